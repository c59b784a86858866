"""Pins of the FP64 cost-model reference (no GPU)."""
import numpy as np
import pytest

from oracle import mlp
from paper_2404_03226_amd import synth


def small_params(seed=3, scale=1.0):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) * scale * (0.3 if len(s) == 2 else 0.1) for s in synth.MLP_SHAPES]


def test_bf16_matches_library_conversion():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0, 65504.0])])
    ref = torch.tensor(x, dtype=torch.float32).bfloat16().double().numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_exact_gradients_match_central_differences():
    p = small_params()
    rng = np.random.default_rng(1)
    X = rng.random((6, 32))
    T = rng.standard_normal((6, 2))
    _, grads, _ = mlp.loss_grads(p, X, T, bf=False)
    flat = mlp.pack(p)
    g = mlp.pack(grads)
    idx = rng.choice(flat.size, 300, replace=False)
    idx = np.concatenate([idx, [flat.size - 1, flat.size - 2, 8192, 8192 + 255]])
    h = 1e-6
    for i in idx:
        a, b = flat.copy(), flat.copy()
        a[i] += h
        b[i] -= h
        la = mlp.loss_grads(mlp.unpack(a, synth.MLP_SHAPES), X, T, bf=False)[0]
        lb = mlp.loss_grads(mlp.unpack(b, synth.MLP_SHAPES), X, T, bf=False)[0]
        fd = (la - lb) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_linear_regime_is_a_product_of_matrices():
    # every pre-activation positive -> ReLU is the identity
    rng = np.random.default_rng(2)
    p = [np.abs(q) + (0.01 if q.ndim == 2 else 0.1) for q in small_params(4)]
    X = rng.random((5, 32)) + 0.1
    y = mlp.forward(p, X, bf=False)["Y"]
    W1, b1, W2, b2, W3, b3 = p
    assert np.allclose(y, ((X @ W1 + b1) @ W2 + b2) @ W3 + b3, rtol=1e-12)
    # all weights zero -> the output bias
    z = [np.zeros_like(q) for q in p]
    z[5] = np.array([0.5, -2.0])
    assert np.allclose(mlp.forward(z, X, bf=False)["Y"], np.tile([0.5, -2.0], (5, 1)))


def test_first_adam_step_moves_by_lr_against_the_gradient():
    p = small_params(5)
    g = [np.random.default_rng(6).standard_normal(q.shape) for q in p]
    zeros = [np.zeros_like(q) for q in p]
    newp, m, v = mlp.adam(p, g, zeros, zeros, 1, lr=1e-3)
    for a, b, gg in zip(p, newp, g):
        # bias-corrected first moment / sqrt(second) = sign(g) on step 1
        # (the eps term bounds the deviation by lr * eps / |g|)
        assert np.all(np.abs((b - a) + 1e-3 * np.sign(gg)) <= 1e-3 * 1e-8 / np.abs(gg) + 1e-15)


def test_relu_gradient_is_zero_where_inactive():
    p = small_params(7)
    rng = np.random.default_rng(8)
    X = rng.random((16, 32))
    T = rng.standard_normal((16, 2))
    _, grads, c = mlp.loss_grads(p, X, T, bf=False)
    assert np.all(c["dH1"][c["H1pre"] <= 0] == 0)
    assert np.all(c["dH2"][c["H2pre"] <= 0] == 0)


def test_ticks_from_log_rounds_half_to_even_and_clamps():
    y = np.log(np.array([0.2, 2.5, 3.5, 1e9, 7.0]))
    assert mlp.ticks_from_log(y).tolist() == [1, 2, 4, 1 << 20, 7]


def test_records_generator_shapes_and_noise():
    rec = synth.cfg5_records(n=50000)
    assert rec["x"].shape == (50000, 32) and rec["ticks"].shape == (50000, 2)
    assert np.all(rec["x"][np.arange(50000), rec["types"]] == 1.0)
    # lognormal noise sigma 0.2 around a smooth function: residual of the
    # per-type mean in log space is bounded well below the between-type spread
    lt = np.log(rec["ticks"].astype(np.float64))
    for t in range(4):
        s = lt[rec["types"] == t]
        assert 0.15 < s.std(axis=0).min() < 1.0


# ---------------------------------------------------------------------------
# The element-wise bounds the GPU tests use (tests/mlp_bounds.py): sound for
# an fp32-accumulating implementation, tight enough to catch planted
# mistakes.

def _f32_forward_backward(params, X, T):
    """The kernels' arithmetic on the CPU: bfloat16 stores at the reference's
    rounding points, every product and sum in float32 (numpy's own summation
    order, not the kernels')."""
    bf = lambda a: mlp.bf16(a).astype(np.float32)
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float32) for p in params]
    W1b, W2b, W3b = bf(W1), bf(W2), bf(W3)
    Xb = bf(X)
    H1 = bf(np.maximum(Xb @ W1b + b1, 0))
    H2 = bf(np.maximum(H1 @ W2b + b2, 0))
    Y = H2 @ W3b + b3
    T32 = np.asarray(T, np.float32)
    dY = (Y - T32) * np.float32(2.0 / Y.size)
    dW3 = H2.T @ dY
    db3 = dY.sum(0)
    dH2 = (dY @ W3b.T) * (H2 > 0)
    db2 = dH2.sum(0)
    dH2b = bf(dH2)
    dW2 = H1.T @ dH2b
    dH1 = (dH2b @ W2b.T) * (H1 > 0)
    db1 = dH1.sum(0)
    dW1 = Xb.T @ bf(dH1)
    return Y, [dW1, db1, dW2, db2, dW3, db3]


def _bounds_data(B=512, seed=21):
    rng = np.random.default_rng(seed)
    p = synth.mlp_init()
    for i in (1, 3, 5):
        p[i] = rng.normal(0.0, 0.1, p[i].shape).astype(np.float32)
    rec = synth.cfg5_records(n=4096)
    X = rec["x"][:B]
    T = np.log(rec["ticks"][:B].astype(np.float64)).astype(np.float32)
    return p, X, T


def test_bounds_hold_for_an_fp32_implementation():
    import mlp_bounds as mb
    p, X, T = _bounds_data()
    Y, grads = _f32_forward_backward(p, X, T)
    loss, g, c, E = mb.grad_bounds(p, X, T)
    ok, worst, at = mb.within(Y, c["Y"], E["Y"])
    assert ok, ("Y", worst, at)
    for name, a, b, e in zip(("W1", "b1", "W2", "b2", "W3", "b3"), grads, g, E["grads"]):
        ok, worst, at = mb.within(a, b, e)
        assert ok, (name, worst, at)
    # and the bounds are small: most stored activations carry no error, and
    # a gradient's bound is far below its own size
    _, Ef = mb.forward_bounds(p, X)
    assert np.mean(Ef["H1"] == 0) > 0.98 and np.mean(Ef["H2"] == 0) > 0.8
    # (the bound assumes every uncertain rounding flips the same way, so it
    # is loosest on the first layer's gradients, a few percent at the median)
    for b, e in zip(g, E["grads"]):
        assert np.median(e / np.maximum(np.abs(b), 1e-30)) < 5e-2


@pytest.mark.parametrize("mistake", ["drop_b2_unit", "w2_transposed", "w3_column_swap", "relu_on_output",
                                     "dh1_mask_from_h2", "dh1_mask_dropped", "mse_grad_halved"])
def test_bounds_catch_planted_mistakes(mistake):
    """Plausible one-line mistakes, planted in a copy of the reference
    arithmetic on the CPU, land outside the bound of some tensor."""
    import mlp_bounds as mb
    p, X, T = _bounds_data(B=256, seed=22)
    loss, g, c, E = mb.grad_bounds(p, X, T)
    bf = mlp.bf16
    W1, b1, W2, b2, W3, b3 = [np.asarray(q, np.float64) for q in p]
    q2 = b2.copy()
    W2u = bf(W2)
    W3u = bf(W3)
    if mistake == "drop_b2_unit":
        q2[17] = 0.0
    if mistake == "w2_transposed":
        W2u = W2u.T
    if mistake == "w3_column_swap":
        W3u = W3u[:, ::-1]
    Xb = bf(X)
    H1 = bf(np.maximum(Xb @ bf(W1) + b1, 0))
    H2 = bf(np.maximum(H1 @ W2u + q2, 0))
    Y = H2 @ W3u + b3
    if mistake == "relu_on_output":
        Y = np.maximum(Y, 0)
    dY = (Y - T) * ((1.0 if mistake == "mse_grad_halved" else 2.0) / Y.size)
    dH2 = (dY @ W3u.T) * (H2 > 0)
    dH2b = bf(dH2)
    dH1 = dH2b @ W2u.T
    if mistake != "dh1_mask_dropped":
        dH1 = dH1 * ((H2 if mistake == "dh1_mask_from_h2" else H1) > 0)
    db1 = dH1.sum(0)
    got = {"Y": Y, "b1": db1, "W1": Xb.T @ bf(dH1), "b2": dH2.sum(0), "W2": H1.T @ dH2b, "W3": H2.T @ dY}
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    caught = not mb.within(got["Y"], c["Y"], E["Y"])[0]
    for name in ("W1", "b1", "W2", "b2", "W3"):
        caught |= not mb.within(got[name], g[names.index(name)], E["grads"][names.index(name)])[0]
    assert caught, mistake


def test_adam_bounds_hold_and_catch_a_sign_flip():
    import mlp_bounds as mb
    p, X, T = _bounds_data(B=256, seed=23)
    loss, g, c, E = mb.grad_bounds(p, X, T)
    _, grads32 = _f32_forward_backward(p, X, T)
    flat_p, flat_g, flat_e = mlp.pack(p), mlp.pack(g), mlp.pack(E["grads"])
    g32 = mlp.pack(grads32).astype(np.float32)
    lr = 1e-3
    A = mb.adam_bounds(flat_p, flat_g, flat_e, lr)
    # the fp32 update from the fp32 gradient
    p32 = flat_p.astype(np.float32)
    m = np.float32(1 - np.float32(0.9)) * g32
    v = np.float32(1 - np.float32(0.999)) * g32 * g32
    bc1, bc2 = np.float32(1 - np.float32(0.9)), np.float32(1 - np.float32(0.999))
    newp = p32 - np.float32(lr) * (m / bc1) / (np.sqrt(v / bc2) + np.float32(1e-8))
    for got, ref, e in ((newp, A["p"], A["Ep"]), (m, A["m"], A["Em"]), (v, A["v"], A["Ev"])):
        ok, worst, at = mb.within(got, ref, e)
        assert ok, (worst, at)
    # a step along the gradient instead of against it is caught
    flip = p32 + np.float32(lr) * (m / bc1) / (np.sqrt(v / bc2) + np.float32(1e-8))
    assert not mb.within(flip, A["p"], A["Ep"])[0]


def test_reference_network_gains_over_the_table():
    """The method with learned estimates (the reference network trained on
    simulator records) against the per-type average table (Section 4.3's
    average execution times): lower validation error, and schedules of the
    sampled batch DAGs, all run with the true durations, closer to the
    true-estimate makespan on most DAGs."""
    import oracle
    import learned
    from paper_2404_03226_amd import costmodel
    rec, params, steps, table = learned.trained()
    assert steps == learned.EPOCHS * (rec["n_train"] // 1024)
    ntr = rec["n_train"]
    T = np.log(rec["ticks"][ntr:].astype(np.float64))
    y = mlp.forward(params, rec["x"][ntr:], bf=True)["Y"]
    mse_mlp = float(np.mean((y - T) ** 2))
    mse_tab = float(np.mean((np.log(table[rec["types"][ntr:]].astype(np.float64)) - T) ** 2))
    assert mse_mlp < 0.8 * mse_tab
    ws, b, x, ticks, est = learned.sample()
    ms = {}
    for name in ("true", "plain", "learned"):
        b.dur, b.est = ticks, est[name]
        ms[name] = oracle.schedule_batch(b)["makespan"]
    gaps = costmodel.makespan_gaps(ms["true"], ms["plain"], ms["learned"])
    print(gaps)
    assert gaps["paired_gain"] > 0.01 and gaps["frac_improved"] > 0.75
