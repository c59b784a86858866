"""HIP cost-model kernels against the FP64 reference with bf16 rounding.

Every floating-point output is compared element by element against the
reference within the per-element bound of tests/mlp_bounds.py (the fp32
accumulation bound of each sum, propagated through the bfloat16 stores and
ReLU masks); integer estimates are compared exactly wherever the kernel's
own exp(y) is not within 1e-3 relative of a rounding tie.
"""
import numpy as np
import pytest

import mlp_bounds as mb
from oracle import mlp
from paper_2404_03226_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def insp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_03226_amd import inspirit
    inspirit.load()
    return inspirit


def close(got, ref, bound, what):
    ok, worst, at = mb.within(got, ref, bound)
    print(f"  {what}: worst |err| / bound = {worst:.3g}", flush=True)
    assert ok, f"{what}: element {at} off by {worst:.3g} x its bound"


def check_y(y, p, X):
    c, E = mb.forward_bounds(p, X)
    close(y, c["Y"], E["Y"], "y")


def batch(n, seed=0):
    rec = synth.cfg5_records(n=max(n, 2048))
    X = rec["x"][:n]
    T = np.log(rec["ticks"][:n].astype(np.float64)).astype(np.float32)
    return X, T


@pytest.mark.parametrize("B", [32, 96, 1024])
def test_forward_backward_match_reference(insp, B):
    import torch
    print("[case] mlp grads", B, flush=True)
    p = synth.mlp_init()
    X, T = batch(B)
    m = insp.Mlp(p)
    g, y, loss = m.grads(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    ref_loss, ref_g, c, E = mb.grad_bounds(p, X, T)
    close(y.cpu().numpy(), c["Y"], E["Y"], "y")
    close(np.array([loss.item()]), np.array([ref_loss]), np.array([E["loss"]]), "loss")
    gg = mlp.unpack(g.cpu().numpy(), synth.MLP_SHAPES)
    for name, a, b, e in zip(("W1", "b1", "W2", "b2", "W3", "b3"), gg, ref_g, E["grads"]):
        close(a, b, e, "d" + name)
    m.free()


def test_adam_step_matches_reference(insp):
    import torch
    print("[case] mlp adam", flush=True)
    p = synth.mlp_init()
    X, T = batch(256)
    m = insp.Mlp(p)
    m.train_step(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), lr=1e-3)
    torch.cuda.synchronize()
    newp, am, av, step = m.state()
    _, g, _, E = mb.grad_bounds(p, X, T)
    zeros = [np.zeros_like(q, dtype=np.float64) for q in p]
    ref_p, ref_m, ref_v = mlp.adam([q.astype(np.float64) for q in p], g, zeros, zeros, 1)
    A = mb.adam_bounds(mlp.pack(p), mlp.pack(g), mlp.pack(E["grads"]), 1e-3)
    # the bound module's closed form of the first step is the reference's
    assert np.allclose(A["p"], mlp.pack(ref_p), rtol=0, atol=1e-12)
    assert np.allclose(A["m"], mlp.pack(ref_m), rtol=1e-12) and np.allclose(A["v"], mlp.pack(ref_v), rtol=1e-12)
    assert step == 1
    close(newp, A["p"], A["Ep"], "params")
    close(am, A["m"], A["Em"], "first moment")
    close(av, A["v"], A["Ev"], "second moment")
    m.free()


def test_predict_matches_reference_and_rounds(insp):
    import torch
    print("[case] mlp predict", flush=True)
    p = synth.mlp_init()
    rec = synth.cfg5_records(n=70000)  # spans two chunks of the predict path plus a tail
    X = rec["x"][:70001 - 2]
    m = insp.Mlp(p)
    y, est = m.predict(torch.from_numpy(X).cuda())
    y, est = y.cpu().numpy(), est.cpu().numpy()
    check_y(y, p, X)
    # integer decision taken from the kernel's own y in the same precision
    e = np.exp(y.astype(np.float32))
    ok = np.abs(e - np.floor(e) - 0.5) > 1e-3 * np.maximum(e, 1.0)
    want = np.clip(np.rint(e), 1, 1 << 20).astype(np.int32)
    assert np.array_equal(est[ok], want[ok])
    m.free()


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65])
def test_predict_small_and_empty(insp, n):
    """Fewer rows than one 64-row tile, exactly one, one plus a row, and none:
    most persistent blocks get no tile; every row against the FP64 reference."""
    import torch
    print(f"[case] mlp predict n={n}", flush=True)
    rng = np.random.default_rng(13)
    p = synth.mlp_init()
    for i in (1, 3, 5):
        p[i] = rng.normal(0.0, 0.1, p[i].shape).astype(np.float32)
    X, _ = batch(max(n, 1))
    X = X[:n]
    m = insp.Mlp(p)
    y, est = m.predict(torch.from_numpy(np.ascontiguousarray(X)).cuda())
    assert y.shape == (n, 2) and est.shape == (n, 2)
    if n == 1:
        # features at a 4-byte offset are refused, not read misaligned
        buf = torch.zeros(33, dtype=torch.float32, device="cuda")
        with pytest.raises(insp.InspError, match="aligned"):
            m.predict(buf[1:].view(1, 32))
    if n:
        y, est = y.cpu().numpy(), est.cpu().numpy()
        check_y(y, p, X)
        e = np.exp(y.astype(np.float32))
        ok = np.abs(e - np.floor(e) - 0.5) > 1e-3 * np.maximum(e, 1.0)
        assert np.array_equal(est[ok], np.clip(np.rint(e), 1, 1 << 20).astype(np.int32)[ok])
    m.free()


def test_predict_full_batch_sampled(insp):
    """Prediction at the size the benchmark times (one row per task of the
    4096-DAG batch: 17,723,451 rows, so a ragged last tile) in the same
    launch, with nonzero biases; sampled rows, the first tile and the tail
    against the FP64 reference, estimates by the same rounding rule."""
    import torch
    n = 17_723_451
    print(f"[case] mlp predict full batch n={n}", flush=True)
    rng = np.random.default_rng(11)
    X = synth.cost_features(5, 7, rng.integers(0, 4, n).astype(np.int32))
    p = synth.mlp_init()
    for i in (1, 3, 5):
        p[i] = rng.normal(0.0, 0.1, p[i].shape).astype(np.float32)
    m = insp.Mlp(p)
    y, est = m.predict(torch.from_numpy(X).cuda())
    idx = np.unique(np.concatenate([rng.integers(0, n, 4000), np.arange(64), np.arange(n - 100, n)]))
    sel = torch.from_numpy(idx).cuda()
    y, est = y[sel].cpu().numpy(), est[sel].cpu().numpy()
    check_y(y, p, X[idx])
    e = np.exp(y.astype(np.float32))
    ok = np.abs(e - np.floor(e) - 0.5) > 1e-3 * np.maximum(e, 1.0)
    want = np.clip(np.rint(e), 1, 1 << 20).astype(np.int32)
    assert np.array_equal(est[ok], want[ok])
    m.free()


def test_training_beats_the_per_type_table(insp):
    import torch
    print("[case] mlp training", flush=True)
    rec = synth.cfg5_records(n=200_000)
    ntr = rec["n_train"]
    X = torch.from_numpy(rec["x"]).cuda()
    LT = torch.from_numpy(np.log(rec["ticks"].astype(np.float64)).astype(np.float32)).cuda()
    m = insp.Mlp(synth.mlp_init())
    B = 1024
    for ep in range(3):
        for i in range(0, ntr - B + 1, B):
            m.train_step(X[i:i + B], LT[i:i + B], lr=1e-3)
    torch.cuda.synchronize()
    y, _ = m.predict(X[ntr:])
    val = LT[ntr:].cpu().numpy()
    mse_mlp = float(np.mean((y.cpu().numpy() - val) ** 2))
    tab = synth.plain_table(rec["types"][:ntr], rec["ticks"][:ntr])
    mse_tab = float(np.mean((np.log(tab[rec["types"][ntr:]].astype(np.float64)) - val) ** 2))
    print("val mse mlp", mse_mlp, "table", mse_tab, flush=True)
    assert mse_mlp < mse_tab
    m.free()


@pytest.mark.parametrize("n,bsz,epochs", [(4096 + 100, 256, 3), (1024, 64, 1), (96, 32, 2)])
def test_graph_training_matches_eager_steps(insp, n, bsz, epochs):
    """insp_mlp_train against a loop of insp_mlp_train_step over the same
    minibatches: parameters, Adam moments, step count and the last loss are
    bit-identical.  Later calls with another batch (a new capture) and with
    the same arguments (the kept graph, a fresh step table) continue from the
    first; n < batch and epochs == 0 do nothing."""
    import torch
    print(f"[case] mlp graph training n={n} batch={bsz} epochs={epochs}", flush=True)
    X, T = batch(n)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    a = insp.Mlp(synth.mlp_init())
    b = insp.Mlp(synth.mlp_init())
    la = torch.zeros(1, dtype=torch.float32, device="cuda")
    lb = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    for bs, ep in ((bsz, epochs), (32, 1), (32, 1)):
        for _ in range(ep):
            for i in range(0, n - bs + 1, bs):
                a.train_step(Xd[i:i + bs], Td[i:i + bs], loss=la)
        b.train(Xd, Td, batch=bs, epochs=ep, loss=lb)
    b.train(Xd[:16], Td[:16], batch=32, epochs=4, loss=lb)  # no full minibatch
    b.train(Xd, Td, batch=32, epochs=0, loss=lb)
    torch.cuda.synchronize()
    sa, sb = a.state(), b.state()
    for u, v in zip(sa[:3], sb[:3]):
        assert np.array_equal(u, v)
    assert sa[3] == sb[3] == epochs * (n // bsz) + 2 * (n // 32)
    assert la.item() == lb.item()
    with pytest.raises(insp.InspError):
        b.train(Xd, Td, batch=48)
    with pytest.raises(insp.InspError, match="2\\^28"):
        b.train(Xd[:32], Td[:32], batch=32, epochs=2 ** 28 + 1)
    assert b.state()[3] == sb[3]
    a.free()
    b.free()


def test_checkpoint_resume_is_bit_identical(insp):
    import torch
    print("[case] mlp resume", flush=True)
    X, T = batch(4096)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    a = insp.Mlp(synth.mlp_init())
    for i in range(2):
        a.train_step(Xd[i * 1024:(i + 1) * 1024], Td[i * 1024:(i + 1) * 1024])
    torch.cuda.synchronize()
    snap = a.state()
    b = insp.Mlp(synth.mlp_init())
    b.load_state(*snap)
    for mdl in (a, b):
        for i in range(2, 4):
            mdl.train_step(Xd[i * 1024:(i + 1) * 1024], Td[i * 1024:(i + 1) * 1024])
    torch.cuda.synchronize()
    pa, pb = a.state()[0], b.state()[0]
    assert np.array_equal(pa, pb)


def test_learned_estimates_schedules_and_gain(insp):
    """The cost-model evaluation on 32 DAGs of the 4096-DAG batch.  (a) The
    scheduler given the reference network's integer estimates, the per-type
    table and the true ticks (every run advancing with the true ticks)
    matches the oracle bit for bit.  (b) The network trained on the GPU by
    the library's own forward, backward and Adam kernels, from the same
    initial parameters and minibatches as the reference, gains over the
    table: lower validation error and, with its estimates, schedules closer
    to the true-estimate makespans on most DAGs."""
    import torch
    import learned
    import oracle
    from paper_2404_03226_amd import costmodel
    print("[case] learned estimates: schedules and gain", flush=True)
    rec, _, steps, table = learned.trained()
    ws, b, x, ticks, est = learned.sample()
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    dag, dur, _ = insp.batch_to_device(b)
    dur = torch.from_numpy(np.ascontiguousarray(ticks, np.int32)).cuda()
    ms = {}
    for name in ("true", "plain", "learned"):
        e = torch.from_numpy(np.ascontiguousarray(est[name], np.int32)).cuda()
        o = insp.schedule_batch(dag, workers, dur, e)
        insp.sync_status(dag)
        b.dur, b.est = ticks, est[name]
        r = oracle.schedule_batch(b)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop", "makespan"):
            assert np.array_equal(o[k].cpu().numpy()[: len(r[k])], r[k]), (name, k)
        ms[name] = r["makespan"]
    ref_gaps = costmodel.makespan_gaps(ms["true"], ms["plain"], ms["learned"])
    # (b) GPU training and inference
    ntr = rec["n_train"]
    X = torch.from_numpy(rec["x"]).cuda()
    LT = torch.from_numpy(np.log(rec["ticks"].astype(np.float64)).astype(np.float32)).cuda()
    m = insp.Mlp(synth.mlp_init())
    m.train(X[:ntr], LT[:ntr], batch=1024, epochs=learned.EPOCHS, lr=learned.LR)
    assert m.state()[3] == steps
    y, _ = m.predict(X[ntr:])
    val = LT[ntr:].cpu().numpy()
    mse_mlp = float(np.mean((y.cpu().numpy() - val) ** 2))
    mse_tab = float(np.mean((np.log(table[rec["types"][ntr:]].astype(np.float64)) - val) ** 2))
    _, est_gpu = m.predict(torch.from_numpy(x).cuda(), want_y=False)
    gms = costmodel.evaluate(dag, workers, b.type, ticks, est_gpu, table)
    gaps = costmodel.makespan_gaps(gms["true"], gms["plain"], gms["learned"])
    print("  reference network:", ref_gaps, flush=True)
    print("  GPU-trained network:", gaps, "val mse", mse_mlp, "table", mse_tab, flush=True)
    assert np.array_equal(gms["true"], ms["true"]) and np.array_equal(gms["plain"], ms["plain"])
    assert mse_mlp < 0.8 * mse_tab
    assert gaps["paired_gain"] > 0.01 and gaps["frac_improved"] > 0.75
    m.free()
    dag.free()
