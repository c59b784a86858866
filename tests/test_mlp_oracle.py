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
