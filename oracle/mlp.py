"""FP64 reference of the learned cost model -- TEST INFRASTRUCTURE.

A 32 -> 256 -> 256 -> 2 ReLU network predicting natural-log durations for
the two worker kinds, trained with MSE and Adam.  ``bf=True`` rounds
weights, activations and activation gradients to bfloat16 (round to nearest
even) at exactly the points where the HIP kernels store bfloat16, and keeps
everything else in float64; ``bf=False`` is the exact float64 network, which
the tests check against central finite differences.

Parameter order (packed): W1 [32,256], b1 [256], W2 [256,256], b2 [256],
W3 [256,2], b3 [2].
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through float32; float64 out."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def forward(params, X, bf=True):
    r = bf16 if bf else _id
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    Xb = r(X)
    H1pre = Xb @ r(W1) + b1
    H1 = r(np.maximum(H1pre, 0.0))
    H2pre = H1 @ r(W2) + b2
    H2 = r(np.maximum(H2pre, 0.0))
    Y = H2 @ r(W3) + b3
    return {"X": Xb, "H1pre": H1pre, "H1": H1, "H2pre": H2pre, "H2": H2, "Y": Y}


def loss_grads(params, X, T, bf=True):
    """MSE over all B x 2 outputs and its gradients (same order as params)."""
    r = bf16 if bf else _id
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    c = forward(params, X, bf)
    B = X.shape[0]
    diff = c["Y"] - np.asarray(T, np.float64)
    loss = float(np.mean(diff ** 2))
    dY = diff * (2.0 / diff.size)
    dW3 = c["H2"].T @ dY
    db3 = dY.sum(0)
    dH2 = (dY @ r(W3).T) * (c["H2"] > 0)
    db2 = dH2.sum(0)
    dH2b = r(dH2)
    dW2 = c["H1"].T @ dH2b
    dH1 = (dH2b @ r(W2).T) * (c["H1"] > 0)
    db1 = dH1.sum(0)
    dH1b = r(dH1)
    dW1 = c["X"].T @ dH1b
    c["dY"], c["dH2"], c["dH1"] = dY, dH2, dH1
    return loss, [dW1, db1, dW2, db2, dW3, db3], c


def adam(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015) with bias correction; returns new
    (params, m, v).  step counts from 1."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** step)
        vh = vv / (1 - b2 ** step)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def train(params, X, T, batch=1024, epochs=1, lr=1e-3, bf=True):
    """Minibatch training in order: `epochs` passes over the rows of X, T in
    consecutive minibatches of `batch` rows (a last partial minibatch is not
    used), one Adam step per minibatch on the float64 master parameters, the
    network evaluated with bfloat16 stores when `bf`.  Returns (params, steps)."""
    p = [np.asarray(q, np.float64).copy() for q in params]
    m = [np.zeros_like(q) for q in p]
    v = [np.zeros_like(q) for q in p]
    step = 0
    n = X.shape[0]
    for _ in range(epochs):
        for i in range(0, n - batch + 1, batch):
            _, g, _ = loss_grads(p, X[i:i + batch], T[i:i + batch], bf)
            step += 1
            p, m, v = adam(p, g, m, v, step, lr=lr)
    return p, step


def ticks_from_log(y):
    """Integer estimates clamp(rint(exp(y)), 1, 2^20), ties to even."""
    return np.clip(np.rint(np.exp(np.asarray(y, np.float64))), 1, 1 << 20).astype(np.int32)


def pack(params):
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in params])


def unpack(flat, shapes):
    out, off = [], 0
    for s in shapes:
        cnt = int(np.prod(s))
        out.append(np.asarray(flat[off:off + cnt]).reshape(s))
        off += cnt
    return out
