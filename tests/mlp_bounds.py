"""Per-element error bounds for the cost-model kernels against the FP64
reference (test infrastructure).

The kernels store bfloat16 where the reference rounds to bfloat16 and
accumulate in fp32 where the reference sums exactly in float64.  For every
tensor the reference computes, this module derives a first-order bound on
how far an fp32-accumulating implementation of the same steps can be from
it, element by element:

  * a sum of k products (a dot product, a column sum over the batch), in any
    order, in fp32: gamma_k * sum |terms|, gamma_k = k * 2^-24 (the standard
    worst-case bound, independent of the order);
  * an error E already in an operand propagates as E @ |other operand|;
  * a bfloat16 rounding (nearest, ties to even) is monotone, so when the
    rounded values of ref - E and ref + E agree every value in between
    rounds to the same bfloat16 and the stored value carries no error at
    all; otherwise its error is the larger distance to those two;
  * a ReLU mask taken from a stored activation is certain when the interval
    ref +- E lies on one side of zero, and otherwise the masked element may
    be either zero or the unmasked value.

The bound is rigorous (to first order) rather than statistical: it assumes
every rounding whose interval holds a tie goes the wrong way.  It is zero
for most stored activations; on the gradients it is loosest in the first
layer (a few percent of the value at the median, well below 1e-3 in the
later layers), still tight enough that a wrong hidden unit, bias, weight
layout, mask or loss factor exceeds it (the CPU tests plant such mistakes
in the reference and check that they are caught).
"""
from __future__ import annotations

import numpy as np

from oracle import mlp

U32 = 2.0 ** -24
SLACK = 1.25  # first-order bounds: room for the neglected products of errors


def gamma(k):
    return k * U32


def _bf(x):
    return mlp.bf16(x)


def _round_err(ref_pre, e_pre, fn):
    """Bound on |fn(x) - fn(ref_pre)| for |x - ref_pre| <= e_pre, fn monotone
    non-decreasing (bfloat16 rounding, possibly after a ReLU)."""
    lo, hi = fn(ref_pre - e_pre), fn(ref_pre + e_pre)
    mid = fn(ref_pre)
    return np.where(lo == hi, 0.0, np.maximum(np.abs(hi - mid), np.abs(lo - mid)))


def _relu_bf(x):
    return _bf(np.maximum(x, 0.0))


def forward_bounds(params, X):
    """Reference intermediates (bf=True) and the bound of each: returns
    (c, E) with E["H1pre"], E["H1"], E["H2pre"], E["H2"], E["Y"]."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    W1b, W2b, W3b = _bf(W1), _bf(W2), _bf(W3)
    c = mlp.forward(params, X, bf=True)
    E = {}
    # H1pre = Xb @ W1b + b1: 32 products and the bias in fp32 (Xb is exact)
    A = np.abs(c["X"]) @ np.abs(W1b) + np.abs(b1)
    E["H1pre"] = gamma(W1.shape[0] + 1) * A
    E["H1"] = _round_err(c["H1pre"], E["H1pre"], _relu_bf)
    A = np.abs(c["H1"]) @ np.abs(W2b) + np.abs(b2)
    E["H2pre"] = gamma(W2.shape[0] + 1) * A + E["H1"] @ np.abs(W2b)
    E["H2"] = _round_err(c["H2pre"], E["H2pre"], _relu_bf)
    A = np.abs(c["H2"]) @ np.abs(W3b) + np.abs(b3)
    E["Y"] = gamma(W3.shape[0] + 1) * A + E["H2"] @ np.abs(W3b)
    return c, E


def _mask_bound(pre_ref, e_pre, d_ref, e_d):
    """Bound of a gradient masked by (stored activation > 0), given the
    activation's pre-ReLU reference and bound and the unmasked gradient's
    reference and bound."""
    on = _relu_bf(pre_ref - e_pre) > 0       # certainly active
    off = _relu_bf(pre_ref + e_pre) == 0     # certainly inactive
    return np.where(on, e_d, np.where(off, 0.0, np.abs(d_ref) + e_d))


def grad_bounds(params, X, T):
    """Loss, gradients (W1, b1, W2, b2, W3, b3) and the reference
    intermediates, with the bound of y and of each gradient."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    W2b, W3b = _bf(W2), _bf(W3)
    _, E = forward_bounds(params, X)
    loss, g, c = mlp.loss_grads(params, X, T, bf=True)
    B = X.shape[0]
    size = c["Y"].size
    dY = c["dY"]
    E_dY = (2.0 / size) * E["Y"] + 4 * U32 * np.abs(dY)
    G = {}
    G["b3"] = gamma(B) * np.abs(dY).sum(0) + E_dY.sum(0)
    G["W3"] = gamma(B) * (np.abs(c["H2"]).T @ np.abs(dY)) + np.abs(c["H2"]).T @ E_dY + E["H2"].T @ (np.abs(dY) + E_dY)
    # dH2 = (dY @ W3b^T) masked by H2 > 0
    d2 = dY @ W3b.T
    e2 = gamma(W3.shape[1] + 1) * (np.abs(dY) @ np.abs(W3b).T) + E_dY @ np.abs(W3b).T
    E_dH2 = _mask_bound(c["H2pre"], E["H2pre"], d2, e2)
    G["b2"] = gamma(B) * np.abs(c["dH2"]).sum(0) + E_dH2.sum(0)
    dH2b = _bf(c["dH2"])
    E_dH2b = _round_err(c["dH2"], E_dH2, _bf)
    G["W2"] = gamma(B) * (np.abs(c["H1"]).T @ np.abs(dH2b)) + np.abs(c["H1"]).T @ E_dH2b + \
        E["H1"].T @ (np.abs(dH2b) + E_dH2b)
    d1 = dH2b @ W2b.T
    e1 = gamma(W2.shape[1] + 1) * (np.abs(dH2b) @ np.abs(W2b).T) + E_dH2b @ np.abs(W2b).T
    E_dH1 = _mask_bound(c["H1pre"], E["H1pre"], d1, e1)
    G["b1"] = gamma(B) * np.abs(c["dH1"]).sum(0) + E_dH1.sum(0)
    dH1b = _bf(c["dH1"])
    E_dH1b = _round_err(c["dH1"], E_dH1, _bf)
    G["W1"] = gamma(B) * (np.abs(c["X"]).T @ np.abs(dH1b)) + np.abs(c["X"]).T @ E_dH1b
    diff = c["Y"] - np.asarray(T, np.float64)
    # loss = mean(diff^2): an fp32 sum of `size` squares, diff itself within E_Y
    E_loss = gamma(size + 2) * float(np.mean(diff ** 2)) + 2.0 * float(np.mean(np.abs(diff) * E["Y"])) + \
        float(np.mean(E["Y"] ** 2))
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    return loss, g, c, {"Y": E["Y"], "loss": E_loss, "grads": [G[k] for k in names]}


def adam_bounds(p0, g_ref, E_g, lr, b1=0.9, b2=0.999, eps=1e-8):
    """First Adam step from zero moments: the reference update and the bound
    of an fp32 update computed from a gradient within E_g of g_ref.  The
    step is -lr g / (|g| + eps); where the gradient's sign is uncertain
    (|g| <= E_g) only |step| <= lr is known."""
    p0, g, Eg = (np.asarray(a, np.float64) for a in (p0, g_ref, E_g))
    step = -lr * g / (np.abs(g) + eps)
    certain = np.abs(g) > Eg
    gap = np.maximum(np.abs(g) - Eg, 0.0) + eps
    e_step = np.where(certain, lr * eps * Eg / gap ** 2, 2 * lr)
    rel = 2.0 ** -19  # fp32 arithmetic of the update and of the bias corrections
    e_p = e_step + rel * (np.abs(p0) + lr)
    m = (1 - b1) * g
    v = (1 - b2) * g * g
    e_m = (1 - b1) * Eg + rel * np.abs(m)
    e_v = (1 - b2) * (2 * np.abs(g) * Eg + Eg * Eg) + rel * np.abs(v)
    return {"p": p0 + step, "m": m, "v": v, "Ep": e_p, "Em": e_m, "Ev": e_v}


def within(got, ref, bound, floor=0.0):
    """Element-wise |got - ref| <= SLACK * bound + floor: (ok, worst ratio,
    index of the worst element)."""
    got, ref, bound = (np.asarray(a, np.float64) for a in (got, ref, bound))
    err = np.abs(got - ref)
    lim = SLACK * bound + floor
    ratio = np.where(lim > 0, err / np.where(lim > 0, lim, 1.0), np.where(err > 0, np.inf, 0.0))
    k = int(np.argmax(ratio)) if ratio.size else 0
    worst = float(ratio.reshape(-1)[k]) if ratio.size else 0.0
    return worst <= 1.0, worst, np.unravel_index(k, ratio.shape) if ratio.size else None
