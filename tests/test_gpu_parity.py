"""Parity of the HIP path with the CPU oracle (bit-exact: all integer work).

Every test prints the case it is about to run, so a failing GPU step can be
named from the log.
"""
import json
import os
from types import SimpleNamespace as NS

import numpy as np
import pytest

import oracle
from paper_2404_03226_amd import synth
from invariants import check_schedule

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def insp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_03226_amd import inspirit
    inspirit.load()
    return inspirit


def say(*a):
    print("[case]", *a, flush=True)


def run_gpu(insp, w, policy="inspirit", trace=False, **kw):
    dag, dur, est = insp.to_device(w)
    prm = insp.params(policy=policy, **kw)
    o = insp.schedule(dag, 0, (w.n_cpu, w.n_gpu), dur, est, prm, trace=trace)
    insp.sync_status(dag)
    n = w.n
    res = {k: o[k][:n].cpu().numpy() for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop")}
    res["makespan"] = int(o["makespan"].item())
    res["n_events"] = int(o["n_events"].item())
    if trace:
        res["trace"] = insp.trace_records(o["trace"], res["n_events"])
    dag.free()
    return res


def assert_same(gpu, ref, what=""):
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
        a, b = np.asarray(gpu[k]), np.asarray(ref[k])
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{what} {k} differs at {bad[:10]} gpu={a[bad[:5]]} ref={b[bad[:5]]}")
    assert gpu["makespan"] == ref["makespan"], what


def test_w2_fig1_analogue_on_gpu(insp):
    g = json.load(open(os.path.join(GOLD, "w2_schedule.json")))
    w = NS(n=5, row_ptr=np.array(g["row_ptr"], np.int32), col=np.array(g["col"], np.int32),
           dur=np.ones((5, 2), np.int32), est=np.ones((5, 2), np.int32), n_cpu=2, n_gpu=0, m=2)
    for pol in ("fifo", "inspirit"):
        say("w2", pol)
        r = run_gpu(insp, w, pol, trace=True)
        assert r["worker"].tolist() == g[pol]["worker"]
        assert r["start"].tolist() == g[pol]["start"]
        assert r["makespan"] == g[pol]["makespan"]
    assert r["trace"]["mode"].tolist() == g["inspirit"]["trace_mode"]
    assert r["trace"]["cnt"].tolist() == g["inspirit"]["trace_cnt"]


def test_w1_attributes_on_gpu(insp):
    import torch
    g = json.load(open(os.path.join(GOLD, "w1_attributes.json")))
    w = NS(n=5, row_ptr=np.array(g["row_ptr"], np.int32), col=np.array(g["col"], np.int32), m=5,
           dur=np.array(g["est"], np.int32), est=np.array(g["est"], np.int32))
    say("w1")
    dag, dur, est = insp.to_device(w)
    ia, ie, U = insp.attributes(dag, 0, est, (0, 1))
    assert ia.cpu().tolist() == g["ia"] and ie.cpu().tolist() == g["ie_auto"] and U[0] == g["unit_time_auto"]
    rem = torch.tensor(g["rem_after_task1"], dtype=torch.int32, device="cuda")
    _, ie5, U5 = insp.attributes(dag, 0, est, (0, 1), unit_time=5, rem=rem)
    assert U5[0] == 5
    assert [ie5.cpu().tolist()[v] for v in g["unfinished_after_task1"]] == \
        [g["ie_after_task1_u5"][v] for v in g["unfinished_after_task1"]]


@pytest.mark.parametrize("seed", range(6))
def test_attributes_match_oracle(insp, seed):
    import torch
    w = synth.cfg3(select=[seed * 97])[0] if seed < 4 else (synth.cfg1() if seed == 4 else synth.cfg2(nb=16))
    say("attributes", w.name)
    dag, dur, est = insp.to_device(w)
    for n_gpu in (0, 4):
        for U in (0, 37, 256):
            ia, ie, Ug = insp.attributes(dag, 0, est, (16, n_gpu), unit_time=U)
            rp, col = oracle.canon(w.n, w.row_ptr, w.col)
            ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, n_gpu, unit_time=U)
            assert Ug[0] == rU
            assert np.array_equal(ia.cpu().numpy(), ria) and np.array_equal(ie.cpu().numpy(), rie)
    # at an arbitrary remaining in-degree (half the tasks finished)
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    finished = synth.Stream(seed, 99).uniform(np.arange(w.n)) < 0.3
    src = np.repeat(np.arange(w.n), np.diff(rp))
    rem = np.bincount(col[~finished[src]], minlength=w.n).astype(np.int32)
    ia, ie, Ug = insp.attributes(dag, 0, est, (16, 4), unit_time=0,
                                 rem=torch.from_numpy(rem).cuda())
    ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, 4, rem=rem)
    assert Ug[0] == rU and np.array_equal(ie.cpu().numpy(), rie)
    dag.free()


def _stars(seed, n_stars, k):
    """n_stars out-stars of k leaves each (every leaf's only predecessor is
    its hub, so every successor has rem == 1) with ticks spread over
    U{1..2000}: the ladder's U lands inside the hubs' spans of tau(v) + tau(s)
    and splits their rows."""
    st = synth.Stream(seed, 2)
    n = n_stars * (k + 1)
    rp = np.zeros(n + 1, np.int32)
    col = []
    for h in range(n_stars):
        base = h * (k + 1)
        col += list(range(base + 1, base + k + 1))
        rp[base + 1:] += k
    col = np.array(col, np.int32)
    d = st.randint(np.arange(2 * n), 1, 2001).astype(np.int32).reshape(n, 2)
    return NS(n=n, row_ptr=rp, col=col, dur=d, est=d.copy(), n_cpu=4, n_gpu=2, m=int(col.size),
              type=np.zeros(n, np.int32), name=f"stars-{n_stars}x{k}")


def test_attributes_rows_split_by_u(insp):
    """Rows whose tau(v) + tau(s) span straddles the ladder's U: IE from a
    count of the row's successors, not from its pass-A summary; rows of 63 or
    more ready successors, whose 16-bit decision word sends them to that
    count whatever their span."""
    for seed, (n_stars, k) in enumerate([(1, 40), (30, 12), (200, 3), (3, 63), (2, 150), (40, 62)]):
        w = _stars(seed, n_stars, k)
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, w.n_gpu)
        hubs = np.arange(0, w.n, k + 1)
        split = int(((rie[hubs] > 0) & (rie[hubs] < ria[hubs])).sum())
        say("attributes split rows", w.name, "U", rU, "split hubs", split)
        assert split > 0
        dag, dur, est = insp.to_device(w)
        ia, ie, Ug = insp.attributes(dag, 0, est, (w.n_cpu, w.n_gpu))
        assert Ug[0] == rU
        assert np.array_equal(ia.cpu().numpy(), ria) and np.array_equal(ie.cpu().numpy(), rie)
        # the same DAG scheduled: the records' IE at pop come from the same pass
        prm = insp.params()
        o = insp.schedule(dag, 0, (w.n_cpu, w.n_gpu), dur, est, prm)
        insp.sync_status(dag)
        r = oracle.schedule(w)
        assert np.array_equal(o["start"][:w.n].cpu().numpy(), r["start"])
        assert np.array_equal(o["ie_at_pop"][:w.n].cpu().numpy(), r["ie_at_pop"])
        dag.free()


def _hub_dag(seed, n, hubs):
    """A DAG of n tasks whose first rows have the given out-degrees (hub rows
    cut into pieces by the grid-wide attribute pass, straddling piece
    boundaries) and every other row 0-6 later targets; ticks U{1..500}."""
    st = synth.Stream(seed, 1)
    rows = []
    for v in range(n):
        d = hubs[v] if v < len(hubs) else int(st.randint(np.array([v]), 0, 6)[0])
        d = min(d, n - 1 - v)
        t = v + 1 + np.sort(synth.Stream(seed, 2 + v).u64(np.arange(3 * d + 8)) % max(n - 1 - v, 1))
        t = np.unique(t)[:d].astype(np.int32)
        rows.append(t)
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(t) for t in rows])
    col = np.concatenate(rows).astype(np.int32)
    est = (synth.Stream(seed, 3).u64(np.arange(2 * n)) % 500 + 1).astype(np.int32).reshape(n, 2)
    return NS(n=n, row_ptr=rp, col=col, dur=est.copy(), est=est, n_cpu=6, n_gpu=2, m=len(col),
              type=np.zeros(n, np.int32), name=f"hubs-{n}")


@pytest.mark.parametrize("hi", [32767, 32768])
def test_per_dag_pass_at_the_16_bit_word_limit(insp, hi):
    """The per-DAG kernel keeps 16-bit task words in LDS when every tau is
    below 2^15 ticks and looks them up from the inputs otherwise: taus just
    below and at that limit, sums of two taus around the explicit U, both
    work-group sizes, the ladder U, a given rem, and a schedule, against the
    oracle."""
    import torch
    for sel in (1, 0):  # 1,529 and 5,477 tasks: 256- and 1024-thread work-groups
        w = synth.cfg3(select=[sel])[0]
        st = synth.Stream(sel, 5)
        est = (hi - st.randint(np.arange(2 * w.n), 0, 40)).astype(np.int32).reshape(w.n, 2)
        est[0] = hi
        w = synth.Workload(w.name, w.n, w.row_ptr, w.col, w.type, est.copy(), est, w.n_cpu, w.n_gpu)
        say("16-bit word limit", w.name, w.n, hi)
        dag, dur, est_d = insp.to_device(w)
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        for n_gpu in (0, 4):
            for U in (0, 2 * hi - 40, 2 * hi - 20, 2 * hi - 1):
                ia, ie, Ug = insp.attributes(dag, 0, est_d, (16, n_gpu), unit_time=U)
                ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, n_gpu, unit_time=U)
                assert Ug[0] == rU, (sel, n_gpu, U)
                assert np.array_equal(ia.cpu().numpy(), ria) and np.array_equal(ie.cpu().numpy(), rie), (sel, n_gpu, U)
        finished = st.uniform(np.arange(w.n)) < 0.3
        src = np.repeat(np.arange(w.n), np.diff(rp))
        rem = np.bincount(col[~finished[src]], minlength=w.n).astype(np.int32)
        ia, ie, Ug = insp.attributes(dag, 0, est_d, (16, 4), unit_time=0, rem=torch.from_numpy(rem).cuda())
        ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, 4, rem=rem)
        assert Ug[0] == rU and np.array_equal(ie.cpu().numpy(), rie)
        dag.free()
        assert_same(run_gpu(insp, w), oracle.schedule(w, variant=oracle.HEAP), w.name)


@pytest.mark.parametrize("case", ["hubs", "powerlaw"])
def test_grid_attribute_pass_with_hub_rows(insp, case):
    # DAGs of at least 32,768 tasks take the grid-wide attribute pass, where
    # rows of more than 64 successors get a wave each
    import torch
    if case == "hubs":
        w = _hub_dag(7, 40000, [4180, 65, 256, 257, 64, 512, 513, 1, 0, 300] + [70] * 60 + [2000])
    else:
        w = synth.cfg4(n=60000)
    say("grid attributes", w.name, w.n, w.m)
    dag, dur, est = insp.to_device(w)
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    for n_gpu in (0, 2):
        for U in (0, 100, 1 << 20):
            ia, ie, Ug = insp.attributes(dag, 0, est, (6, n_gpu), unit_time=U)
            ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, n_gpu, unit_time=U)
            assert Ug[0] == rU, (n_gpu, U)
            assert np.array_equal(ia.cpu().numpy(), ria) and np.array_equal(ie.cpu().numpy(), rie), (n_gpu, U)
    finished = synth.Stream(11, 99).uniform(np.arange(w.n)) < 0.4
    src = np.repeat(np.arange(w.n), np.diff(rp))
    rem = np.bincount(col[~finished[src]], minlength=w.n).astype(np.int32)
    ia, ie, Ug = insp.attributes(dag, 0, est, (6, 2), unit_time=0, rem=torch.from_numpy(rem).cuda())
    ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, 2, rem=rem)
    assert Ug[0] == rU and np.array_equal(ie.cpu().numpy(), rie)
    # the schedule reads the records the grid pass writes
    r = oracle.schedule(w, variant=oracle.HEAP)
    g = run_gpu(insp, w)
    assert_same(g, r, w.name)
    dag.free()


@pytest.mark.parametrize("hi", [126, 127, 32767, 32768])
def test_grid_pass_at_the_word_limits(insp, hi):
    """The grid pass gathers 8-bit task words when no tau of the DAG exceeds
    126 ticks and 16-bit ones (a saturated entry read from the 32-bit word)
    otherwise: taus just below and at both limits, hub rows and rows cut into
    pieces, sums of two taus around the explicit U, the ladder U and a
    schedule, against the oracle."""
    w = _hub_dag(5, 33000, [1500, 70, 600, 3000])
    est = (hi - synth.Stream(hi, 6).randint(np.arange(2 * w.n), 0, 40)).astype(np.int32).reshape(w.n, 2)
    est[0] = hi
    w = NS(**{**vars(w), "est": est, "dur": est.copy()})
    say("grid word limit", w.n, hi)
    dag, dur, est_d = insp.to_device(w)
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    for n_gpu in (0, 2):
        for U in (0, 2 * hi - 20, 2 * hi - 1):
            ia, ie, Ug = insp.attributes(dag, 0, est_d, (6, n_gpu), unit_time=U)
            ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, n_gpu, unit_time=U)
            assert Ug[0] == rU, (n_gpu, U)
            assert np.array_equal(ia.cpu().numpy(), ria) and np.array_equal(ie.cpu().numpy(), rie), (n_gpu, U)
    dag.free()
    assert_same(run_gpu(insp, w), oracle.schedule(w, variant=oracle.HEAP), f"hubs {hi}")


def test_attribute_paths_in_one_batch(insp):
    # small DAGs (one work-group each) beside a large one (the whole grid) and
    # an empty one, in one call: attributes of every DAG and every schedule
    ws = synth.cfg3(select=[3, 700, 2048]) + [_hub_dag(9, 33000, [3000, 100, 65])] + [_empty()] + \
        synth.cfg3(select=[4095])
    b = synth.concat(ws)
    say("mixed attribute paths", [w.n for w in ws])
    dag, dur, est = insp.batch_to_device(b)
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    ia, ie, U = insp.attributes(dag, insp.ALL_DAGS, est, workers)
    ia, ie = ia.cpu().numpy(), ie.cpu().numpy()
    for k, w in enumerate(ws):
        a, z = int(b.task_off[k]), int(b.task_off[k + 1])
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, w.n_gpu)
        assert np.array_equal(ia[a:z], ria) and np.array_equal(ie[a:z], rie) and U[k] == rU, k
    o = insp.schedule_batch(dag, workers, dur, est)
    insp.sync_status(dag)
    r = oracle.schedule_batch(b)
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop", "makespan"):
        assert np.array_equal(o[k].cpu().numpy()[:len(r[k])], r[k]), k
    dag.free()


@pytest.mark.parametrize("policy", ["inspirit", "fifo", "ability", "efi", "heft"])
def test_random_small_dags(insp, policy):
    for i in range(40):
        n = 1 + (i * 7) % 90
        w = synth.random_dag(11, i, n, 0.03 + (i % 6) * 0.04, n_cpu=1 + i % 4, n_gpu=i % 3, dur_hi=30,
                             est_equal=(i % 4 != 0))
        say("random", policy, i, n)
        g = run_gpu(insp, w, policy)
        r = oracle.schedule(w, policy=policy)
        assert_same(g, r, f"random {i}")
        check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"])


def _long_tasks(n, n_cpu, n_gpu, edges, seed):
    """n tasks of 2^19..2^20 ticks on a small machine: once every worker has
    64 such tasks queued, each expected termination time exceeds 2^26 ticks
    and the one-wave loop picks the push worker with its 64-bit argmin."""
    st = synth.Stream(seed, 5)
    src, dst = [], []
    for k in range(edges):
        a, b = sorted(int(x) for x in st.randint(np.array([2 * k, 2 * k + 1]), 0, n - 1))
        if a != b:
            src.append(a)
            dst.append(b)
    order = np.lexsort((dst, src))
    src, dst = np.asarray(src, np.int64)[order], np.asarray(dst, np.int32)[order]
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    lo = 1 << 19
    dur = (lo + st.randint(np.arange(10_000, 10_000 + 2 * n), 0, lo)).reshape(n, 2).astype(np.int32)
    est = (lo + st.randint(np.arange(20_000, 20_000 + 2 * n), 0, lo)).reshape(n, 2).astype(np.int32)
    return synth.Workload(f"long{seed}", n, rp, dst, np.zeros(n, np.int32), dur, est, n_cpu, n_gpu)


@pytest.mark.parametrize("case", [(300, 2, 1, 0), (400, 3, 1, 60), (260, 1, 1, 20)])
def test_push_argmin_beyond_32_bit_costs(insp, case):
    """Expected termination times above 2^26 ticks on every worker take the
    push's 64-bit worker argmin (the 32-bit key holds (cost - t) << 6 only
    below that): single DAG and batch, against the oracle."""
    n, nc, ng, edges = case
    w = _long_tasks(n, nc, ng, edges, seed=n)
    say("push argmin 64-bit", case)
    for policy in ("inspirit", "fifo"):
        g = run_gpu(insp, w, policy)
        r = oracle.schedule(w, policy=policy, variant=oracle.HEAP)
        assert_same(g, r, f"long {case} {policy}")
        check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"])
    # queues reach 64 tasks per worker, so the wide costs really occur
    assert n > 64 * (nc + ng) + 8
    b = synth.concat([w, _long_tasks(n // 2, nc, ng, edges // 2, seed=n + 1)])
    dag, dur, est = insp.batch_to_device(b)
    o = insp.schedule_batch(dag, [(nc, ng), (nc, ng)], dur, est)
    insp.sync_status(dag)
    rb = oracle.schedule_batch(b)
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop", "makespan"):
        assert np.array_equal(o[k].cpu().numpy()[: len(rb[k])], rb[k]), k
    dag.free()


def test_unit_tasks_many_simultaneous_completions(insp):
    # equal durations make many completions coincide: exercises the merge
    for i in range(12):
        w = synth.random_dag(13, i, 150, 0.04, n_cpu=6, n_gpu=3, dur_lo=2, dur_hi=2)
        say("unit", i)
        assert_same(run_gpu(insp, w), oracle.schedule(w), f"unit {i}")


@pytest.mark.parametrize("policy", ["inspirit", "fifo"])
def test_cfg1_layered(insp, policy):
    w = synth.cfg1()
    say("cfg1", policy)
    g = run_gpu(insp, w, policy, trace=True)
    r = oracle.schedule(w, policy=policy, trace=True)
    assert_same(g, r, "cfg1")
    assert g["n_events"] == r["n_events"]
    for f in ("t", "nready", "mode", "cnt", "peak", "pushed", "popped"):
        assert np.array_equal(g["trace"][f], r["trace"][f]), f


def test_cfg2_cholesky(insp):
    w = synth.cfg2()
    say("cfg2")
    g = run_gpu(insp, w)
    r = oracle.schedule(w, variant=oracle.HEAP)
    assert_same(g, r, "cfg2")
    check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"])


@pytest.mark.parametrize("policy", ["inspirit", "fifo"])
def test_lu_tiled(insp, policy):
    w = synth.lu_workload(nb=24)
    say("lu", policy)
    g = run_gpu(insp, w, policy)
    r = oracle.schedule(w, policy=policy, variant=oracle.HEAP)
    assert_same(g, r, "lu")
    check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"])


def test_explicit_parameters(insp):
    w = synth.cfg1()
    kw = dict(unit_time=100, s_inc=2, s_dec=3, dec_step=5, c=1, k_num=3, k_den=40)
    say("params")
    assert_same(run_gpu(insp, w, **kw), oracle.schedule(w, **kw), "params")


def test_batch_small_matches_oracle(insp):
    ws = synth.cfg3(select=list(range(0, 4096, 256)))
    b = synth.concat(ws)
    say("batch16")
    dag, dur, est = insp.batch_to_device(b)
    o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est)
    insp.sync_status(dag)
    r = oracle.schedule_batch(b)
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
        assert np.array_equal(o[k].cpu().numpy(), r[k]), k
    assert np.array_equal(o["makespan"].cpu().numpy(), r["makespan"])
    # tuning must not change results
    for key in ("waves=1,grid=1", "waves=1,grid=3", "waves=1,grid=64", "grid=3,lds_slots=2,lds_keys=40",
                "grid=64,lds_slots=0,lds_keys=8", "grid=5,lds_blocks=4,lds_slots=1,lds_keys=3"):
        o2 = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est, tune_key=key)
        insp.sync_status(dag)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(o2[k].cpu().numpy(), r[k]), (key, k)
    dag.free()


@pytest.mark.skip(reason="several simulating waves per work-group (tune key waves=2..4) faulted the GPU in one "
                         "run with no cause found by reading the code; the launch shape was taken out and waves=1 "
                         "is the only accepted value")
def test_several_simulating_waves_per_work_group(insp):
    ws = synth.cfg3(select=list(range(0, 4096, 256)))
    b = synth.concat(ws)
    say("waves per work-group")
    dag, dur, est = insp.batch_to_device(b)
    r = oracle.schedule_batch(b)
    for key in ("waves=2,grid=3", "waves=3,grid=2", "waves=4,grid=1", "waves=4,grid=256,lds_slots=0"):
        o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est, tune_key=key)
        insp.sync_status(dag)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(o[k].cpu().numpy(), r[k]), (key, k)
    dag.free()


def test_error_codes_through_abi(insp):
    import torch
    say("errors")
    rp = torch.tensor([0, 1, 2, 3], dtype=torch.int32, device="cuda")
    col = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(insp.InspError) as e:
        insp.build_dag([0, 3], [0, 3], rp, col)
    assert e.value.code == insp.E_CYCLE
    col = torch.tensor([1, 2, 7], dtype=torch.int32, device="cuda")
    with pytest.raises(insp.InspError) as e:
        insp.build_dag([0, 3], [0, 3], rp, col)
    assert e.value.code == insp.E_INVAL
    col = torch.tensor([1, 1, 2], dtype=torch.int32, device="cuda")
    with pytest.raises(insp.InspError) as e:
        insp.build_dag([0, 3], [0, 3], rp, col)
    assert e.value.code == insp.E_INVAL
    # duplicates merge; a hang is reported when max_events is too small
    rp = torch.tensor([0, 2, 3, 3], dtype=torch.int32, device="cuda")
    col = torch.tensor([2, 2, 2], dtype=torch.int32, device="cuda")
    dag = insp.build_dag([0, 3], [0, 3], rp, col)
    assert dag.m == [2]
    d = torch.ones((3, 2), dtype=torch.int32, device="cuda")
    insp.schedule(dag, 0, (1, 0), d, d, insp.params(max_events=1))
    with pytest.raises(insp.InspError) as e:
        insp.sync_status(dag)
    assert e.value.code == insp.E_HANG
    bad = d.clone()
    bad[1, 0] = 0
    with pytest.raises(insp.InspError) as e:
        insp.attributes(dag, 0, bad, (1, 0))
    assert e.value.code == insp.E_RANGE
    with pytest.raises(insp.InspError) as e:
        insp.schedule(dag, 0, (0, 0), d, d)
    assert e.value.code == insp.E_RANGE
    dag.free()


def _wide_rows_dag(n, lengths, seed, backward=False):
    """A DAG whose first rows have the given lengths (targets drawn with
    repeats, in random order, from later ids -- or from any other id when
    `backward`, ids then relabelled so that the graph stays acyclic), the
    other rows 0..3 later targets."""
    st = synth.Stream(seed, 9)
    rows = []
    k = 0
    for v in range(n):
        d = lengths[v] if v < len(lengths) else int(st.randint(np.array([k]), 0, 3)[0])
        k += 1
        lo = v + 1
        if lo >= n or d == 0:
            rows.append(np.zeros(0, np.int64))
            continue
        t = st.randint(np.arange(k, k + d), lo, n - 1)
        k += d
        rows.append(t)
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    col = np.concatenate(rows).astype(np.int32) if rp[-1] else np.zeros(0, np.int32)
    if backward:
        # relabel ids by a permutation: edges then point both ways, no cycle
        perm = np.argsort(st.uniform(np.arange(10 ** 7, 10 ** 7 + n)))
        inv = np.empty(n, np.int64)
        inv[perm] = np.arange(n)
        new_rows = [None] * n
        for v in range(n):
            new_rows[inv[v]] = inv[col[rp[v]:rp[v + 1]]]
        rp = np.concatenate([[0], np.cumsum([len(r) for r in new_rows])]).astype(np.int32)
        col = np.concatenate(new_rows).astype(np.int32)
    ty = np.zeros(n, np.int32)
    dur = (1 + st.randint(np.arange(3 * 10 ** 7, 3 * 10 ** 7 + 2 * n), 0, 50)).reshape(n, 2).astype(np.int32)
    return synth.Workload(f"wide{seed}", n, rp, col, ty, dur, dur.copy(), 6, 2)


@pytest.mark.parametrize("backward", [False, True])
def test_build_rows_of_every_length(insp, backward):
    """Canonical rows (sorted, repeats merged) whatever sorts them: rows of
    up to 16 targets in registers, up to 1,024 by one wave, up to 16,384 by a
    work-group, longer ones through a bitmap -- each length at and past its
    limit, with repeated targets, and with ids relabelled so that edges point
    both ways (the Kahn check).  Out-degrees against the oracle's canonical
    CSR, schedules against the oracle."""
    import torch
    lengths = [0, 1, 16, 17, 1024, 1025, 16384, 16385, 40000, 3, 200]
    w = _wide_rows_dag(60000, lengths, seed=41 + backward, backward=backward)
    say("build rows", backward, w.m)
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    dag, dur, est = insp.to_device(w)
    assert dag.m == [len(col)]
    ia, ie, U = insp.attributes(dag, 0, est, (w.n_cpu, w.n_gpu))
    ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, w.n_gpu)
    assert np.array_equal(ia.cpu().numpy(), np.diff(rp)) and np.array_equal(ie.cpu().numpy(), rie) and U[0] == rU
    dag.free()
    g = run_gpu(insp, w)
    assert_same(g, oracle.schedule(w, variant=oracle.HEAP), "wide rows")


@pytest.mark.parametrize("where", [1, 5, 7, 8])
def test_build_rejects_bad_targets_in_long_rows(insp, where):
    """A self loop or an id out of range in a row of each sorting path is
    refused (E_INVAL); a back edge closing a cycle through a long row is
    E_CYCLE."""
    import torch
    lengths = [0, 1, 16, 17, 1024, 1025, 16384, 16385, 40000]
    w = _wide_rows_dag(50000, lengths, seed=43)
    say("build bad target", where)
    a = int(w.row_ptr[where])
    for bad, code in ((where, insp.E_INVAL), (w.n + 3, insp.E_INVAL), (-1, insp.E_INVAL), (0, insp.E_CYCLE)):
        col = w.col.copy()
        col[a + (int(w.row_ptr[where + 1]) - a) // 2] = bad
        if code == insp.E_CYCLE:
            # where -> 0 closes a cycle only if 0 reaches `where`: add 0 -> where
            rows = [list(col[w.row_ptr[v]:w.row_ptr[v + 1]]) for v in range(w.n)]
            rows[0] = [where]
            rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
            col = np.concatenate([np.asarray(r, np.int32) for r in rows])
        else:
            rp = w.row_ptr
        with pytest.raises(insp.InspError) as e:
            insp.build_dag([0, w.n], [0, len(col)], torch.from_numpy(np.asarray(rp, np.int32)).cuda(),
                           torch.from_numpy(np.asarray(col, np.int32)).cuda())
        assert e.value.code == code, (bad, e.value)


def test_failures_are_kept_until_reported(insp):
    """A schedule's device-side failure survives later schedule and
    attribute calls on the handle until insp_sync_status reports it, and is
    cleared once reported."""
    import torch
    say("sticky status")
    ws = [synth.random_dag(31, i, 40, 0.1, n_cpu=2, n_gpu=1) for i in range(3)]
    b = synth.concat(ws)
    dag, dur, est = insp.batch_to_device(b)
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    insp.schedule(dag, 1, workers[1], dur[int(b.task_off[1]):], est[int(b.task_off[1]):], insp.params(max_events=3))
    insp.schedule(dag, 0, workers[0], dur, est)                 # a later good schedule
    insp.attributes(dag, insp.ALL_DAGS, est, workers)            # an attribute-only call
    insp.schedule_batch(dag, workers, dur, est)                  # and a good batch
    with pytest.raises(insp.InspError) as e:
        insp.sync_status(dag)
    assert e.value.code == insp.E_HANG and "DAG 1" in str(e.value)
    insp.sync_status(dag)  # reported once, then cleared
    insp.schedule_batch(dag, workers, dur, est, insp.params(max_events=5))
    with pytest.raises(insp.InspError) as e:
        insp.sync_status(dag)
    assert e.value.code == insp.E_HANG
    insp.sync_status(dag)
    dag.free()


def test_failing_calls_leave_outputs_untouched(insp):
    """Every call that returns a non-OK status writes no output: attribute
    and transitive attribute calls with an estimate out of range (the other
    DAGs' outputs included) and argument errors of the schedule calls; a
    schedule whose DAG fails on the device leaves that DAG's outputs alone
    and sets its makespan to -1."""
    import torch
    say("outputs untouched")
    ws = [synth.random_dag(32, i, 50, 0.1, n_cpu=2, n_gpu=1) for i in range(3)]
    b = synth.concat(ws)
    dag, dur, est = insp.batch_to_device(b)
    N = int(b.task_off[-1])
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    bad = est.clone()
    bad[int(b.task_off[2]) + 3, 1] = (1 << 20) + 1
    lib = insp.load()
    P = insp.C.c_void_p
    ia = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    ie = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    U = np.full(3, -7, np.int32)
    lp = np.full(3, -7, np.int64)
    rc = lib.insp_attributes(dag.handle, insp.ALL_DAGS, P(bad.data_ptr()), insp._workers(workers, 3), 0, None,
                             P(ia.data_ptr()), P(ie.data_ptr()), U.ctypes.data_as(P), insp._stream(None))
    assert rc == insp.E_RANGE
    rc = lib.insp_transitive_attributes(dag.handle, insp.ALL_DAGS, P(bad.data_ptr()), insp._workers(workers, 3), 0,
                                        P(ia.data_ptr()), P(ie.data_ptr()), U.ctypes.data_as(P),
                                        lp.ctypes.data_as(P), insp._stream(None))
    assert rc == insp.E_RANGE
    torch.cuda.synchronize()
    assert (ia == -7).all() and (ie == -7).all() and (U == -7).all() and (lp == -7).all()
    # a schedule call rejected on its arguments
    o = {k: torch.full((N,), -7, dtype=t, device="cuda") for k, t in
         (("worker", torch.int32), ("start", torch.int64), ("finish", torch.int64), ("ie_at_pop", torch.int32),
          ("mode_at_pop", torch.int8))}
    o["makespan"] = torch.full((3,), -7, dtype=torch.int64, device="cuda")
    with pytest.raises(insp.InspError) as e:
        insp.schedule_batch(dag, workers, dur, est, tune_key="waves=2", out=o)
    assert e.value.code == insp.E_INVAL
    with pytest.raises(insp.InspError) as e:
        insp.schedule_batch(dag, workers, dur, est, insp.params(policy=9), out=o)
    assert e.value.code == insp.E_INVAL
    torch.cuda.synchronize()
    assert all((o[k] == -7).all() for k in o)
    # a DAG failing on the device: its outputs stay, the others are written
    insp.schedule_batch(dag, workers, dur, bad, out=o)
    with pytest.raises(insp.InspError) as e:
        insp.sync_status(dag)
    assert e.value.code == insp.E_RANGE
    ms = o["makespan"].cpu().numpy()
    assert ms[2] == -1 and ms[0] > 0 and ms[1] > 0
    a2, z2 = int(b.task_off[2]), int(b.task_off[3])
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
        assert (o[k][a2:z2] == -7).all(), k
    r = oracle.schedule_batch(synth.concat(ws[:2]))
    assert np.array_equal(o["start"][:a2].cpu().numpy(), r["start"])
    dag.free()


def test_allocation_failures_return_nomem_and_leave_state_usable(insp):
    """Injected device allocation failures (insp_test_fail_alloc): the call
    returns E_NOMEM, and the handle or model keeps working -- in particular a
    cost model whose buffers failed to grow still computes what a fresh
    model computes."""
    import torch
    say("nomem")
    w = synth.random_dag(33, 0, 60, 0.08, n_cpu=2, n_gpu=1)
    for k in range(4):
        insp.test_fail_alloc(k)
        try:
            with pytest.raises(insp.InspError) as e:
                insp.to_device(w)
            assert e.value.code == insp.E_NOMEM
        finally:
            insp.test_fail_alloc(-1)
    dag, dur, est = insp.to_device(w)
    insp.test_fail_alloc(1)
    try:
        with pytest.raises(insp.InspError) as e:
            insp.schedule(dag, 0, (w.n_cpu, w.n_gpu), dur, est)
        assert e.value.code == insp.E_NOMEM
    finally:
        insp.test_fail_alloc(-1)
    g = run_gpu(insp, w)
    assert_same(g, oracle.schedule(w), "after nomem")
    dag.free()
    # the cost model: reserve for 64 rows, then fail to grow to 2048
    from paper_2404_03226_amd import synth as sy
    rec = sy.cfg5_records(n=4096)
    X = torch.from_numpy(rec["x"][:2048]).cuda()
    T = torch.from_numpy(np.log(rec["ticks"][:2048].astype(np.float64)).astype(np.float32)).cuda()
    a, ref = insp.Mlp(sy.mlp_init()), insp.Mlp(sy.mlp_init())
    a.grads(X[:64], T[:64])
    for k in range(8):
        insp.test_fail_alloc(k)
        try:
            with pytest.raises(insp.InspError) as e:
                a.grads(X, T)
            assert e.value.code == insp.E_NOMEM
        finally:
            insp.test_fail_alloc(-1)
    for B in (64, 2048):
        ga, ya, la = a.grads(X[:B], T[:B])
        gr, yr, lr_ = ref.grads(X[:B], T[:B])
        assert torch.equal(ga, gr) and torch.equal(ya, yr) and torch.equal(la, lr_)
    a.train(X, T, batch=64, epochs=1)
    ref.train(X, T, batch=64, epochs=1)
    assert np.array_equal(a.state()[0], ref.state()[0])
    a.free()
    ref.free()


def test_batch_graph_replays_match_eager(insp):
    # the batch step captured in a HIP graph, replayed several times with the
    # program's own eager work and synchronisations in between
    import torch
    ws = synth.cfg3(select=list(range(7, 4096, 512)))
    b = synth.concat(ws)
    say("graph", len(ws))
    dag, dur, est = insp.batch_to_device(b)
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    N = int(b.task_off[-1])
    eager = insp.schedule_batch(dag, workers, dur, est)
    torch.cuda.synchronize()
    ref = {k: v.cpu().clone() for k, v in eager.items()}
    out = insp._outputs(N, dur.device)
    out["makespan"] = torch.empty(len(ws), dtype=torch.int64, device=dur.device)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        insp.schedule_batch(dag, workers, dur, est, out=out)   # warm: workspace exists
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        insp.schedule_batch(dag, workers, dur, est, out=out)
    for rep in range(4):
        for k in out:
            out[k].zero_()
        junk = insp.schedule_batch(dag, workers, dur, est)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop", "makespan"):
            assert torch.equal(out[k].cpu(), ref[k]), (rep, k)
        del junk
    r = oracle.schedule_batch(b)
    assert np.array_equal(ref["makespan"].numpy(), r["makespan"])
    dag.free()


def _wide(n, seed):
    # two layers: the first half is ready at once, so queues grow to
    # thousands of entries per worker (block lists and block maxima spill
    # out of LDS)
    from paper_2404_03226_amd.synth import layered_dag, Stream
    rp, col = layered_dag(seed, 0, n, 2, 1, 3)
    st = Stream(seed, 5)
    dur = st.randint(np.arange(2 * n).reshape(n, 2), 1, 40).astype(np.int32)
    return NS(n=n, row_ptr=rp, col=col, dur=dur, est=dur.copy(), n_cpu=2, n_gpu=1, m=int(col.size),
              type=np.zeros(n, np.int32), name=f"wide-{n}")


def _hubs(seed):
    # hub tasks whose successors each have exactly two hub predecessors: one
    # completion leaves hundreds of successors with one unfinished predecessor
    rng = np.random.default_rng(seed)
    H, S = 8, 600
    n = H + S
    edges = []
    for s in range(S):
        a, b = rng.choice(H, 2, replace=False)
        edges += [(a, H + s), (b, H + s)]
    edges.sort()
    rp = np.zeros(n + 1, np.int64)
    for a, _ in edges:
        rp[a + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    col = np.array([b for _, b in edges], np.int32)
    dur = rng.integers(1, 30, (n, 2)).astype(np.int32)
    return NS(n=n, row_ptr=rp, col=col, dur=dur, est=dur.copy(), n_cpu=3, n_gpu=2, m=len(edges), name="hubs",
              type=np.zeros(n, np.int32))


def test_queue_spill_paths_single(insp):
    for seed in (1, 2):
        w = _wide(12000, seed)
        say("wide single", seed)
        assert_same(run_gpu(insp, w), oracle.schedule(w, variant=oracle.HEAP), "wide")


def _wide_keys(n, hub_deg, seed):
    # layered DAG plus one hub task: the largest out-degree needs 8 bits and
    # the push order 17, so 32-bit queue keys do not fit and the general loop
    # (64-bit keys) runs even though the machine has few workers
    from paper_2404_03226_amd.synth import layered_dag, Stream
    rp, col = layered_dag(seed, 0, n, 40, 1, 4)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    hub_t = np.unique(Stream(seed, 6).randint(np.arange(hub_deg), n // 40, n - 1).astype(np.int64))
    src = np.concatenate([src, np.zeros(hub_t.size, np.int64)])
    dst = np.concatenate([col.astype(np.int64), hub_t])
    key = np.unique(src * n + dst)
    src, dst = key // n, key % n
    rp2 = np.zeros(n + 1, np.int32)
    np.add.at(rp2, src + 1, 1)
    rp2 = np.cumsum(rp2).astype(np.int32)
    dur = Stream(seed, 5).randint(np.arange(2 * n).reshape(n, 2), 1, 50).astype(np.int32)
    return NS(n=n, row_ptr=rp2, col=dst.astype(np.int32), dur=dur, est=dur.copy(), n_cpu=6, n_gpu=2,
              m=int(dst.size), type=np.zeros(n, np.int32), name=f"widekeys-{n}")


def test_keys_wider_than_32_bits(insp):
    w = _wide_keys(70000, 200, 3)
    assert int(np.diff(w.row_ptr).max()) >= 128 and w.n - 1 >= 1 << 16
    for pol in ("inspirit", "fifo"):
        say("wide keys", pol)
        assert_same(run_gpu(insp, w, pol), oracle.schedule(w, policy=pol, variant=oracle.HEAP), f"wide keys {pol}")
    # and inside a batch beside DAGs that fit
    ws = [w] + synth.cfg3(select=[7, 70])
    b = synth.concat(ws)
    dag, dur, est = insp.batch_to_device(b)
    o = insp.schedule_batch(dag, [(x.n_cpu, x.n_gpu) for x in ws], dur, est)
    insp.sync_status(dag)
    r = oracle.schedule_batch(b)
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
        assert np.array_equal(o[k].cpu().numpy(), r[k]), k
    dag.free()


def test_queue_spill_paths_batch_small_lds(insp):
    ws = [_wide(6000 + 1000 * i, 10 + i) for i in range(3)] + [_hubs(3)] + synth.cfg3(select=[4, 44])
    b = synth.concat(ws)
    say("spill batch")
    dag, dur, est = insp.batch_to_device(b)
    r = oracle.schedule_batch(b)
    for key in ("waves=1,grid=6,lds_blocks=4,lds_slots=3", "waves=1,grid=2,lds_blocks=0,lds_slots=0",
                "waves=1,grid=3,lds_blocks=64,lds_slots=40", "grid=4,lds_blocks=8,lds_slots=2,lds_keys=50",
                "grid=3,lds_blocks=0,lds_slots=0,lds_keys=12"):
        o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est, tune_key=key)
        insp.sync_status(dag)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(o[k].cpu().numpy(), r[k]), (key, k)
    dag.free()


def test_many_candidates_per_event(insp):
    for seed in range(3):
        w = _hubs(seed)
        say("hubs", seed)
        for pol in ("inspirit", "efi"):
            assert_same(run_gpu(insp, w, pol), oracle.schedule(w, policy=pol), f"hubs {seed} {pol}")


# ------------------------------------------------- id order, machine size, HEFT

def _permuted(w, seed):
    # the same DAG with its task ids shuffled: edges point both ways, so the
    # id order is no topological order
    rng = np.random.default_rng(seed)
    p = rng.permutation(w.n)  # new id of task v
    src = np.repeat(np.arange(w.n), np.diff(np.asarray(w.row_ptr, np.int64)))
    ns, nd = p[src], p[np.asarray(w.col, np.int64)]
    o = np.lexsort((nd, ns))
    ns, nd = ns[o], nd[o]
    rp = np.zeros(w.n + 1, np.int64)
    np.add.at(rp, ns + 1, 1)
    inv = np.argsort(p)  # task at each new id
    return NS(n=w.n, row_ptr=np.cumsum(rp).astype(np.int32), col=nd.astype(np.int32),
              dur=np.asarray(w.dur, np.int32).reshape(w.n, 2)[inv], est=np.asarray(w.est, np.int32).reshape(w.n, 2)[inv],
              n_cpu=w.n_cpu, n_gpu=w.n_gpu, m=int(nd.size), type=np.zeros(w.n, np.int32), name="permuted")


def _backward_edges(w):
    src = np.repeat(np.arange(w.n), np.diff(np.asarray(w.row_ptr, np.int64)))
    return int((np.asarray(w.col) < src).sum())


@pytest.mark.parametrize("policy", ["inspirit", "fifo", "heft"])
def test_permuted_task_ids(insp, policy):
    bases = [synth.lu_workload(nb=10),
             synth.random_dag(41, 0, 300, 0.02, n_cpu=3, n_gpu=2, dur_hi=40, est_equal=False)]
    for i, base in enumerate(bases):
        w = _permuted(base, 7 + i)
        assert _backward_edges(w) > 0
        say("permuted", policy, i, w.n)
        g = run_gpu(insp, w, policy)
        assert_same(g, oracle.schedule(w, policy=policy, variant=oracle.HEAP), f"permuted {i}")
        check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"])


@pytest.mark.parametrize("machine", [(70, 30), (200, 100), (1000, 24)])
def test_many_workers(insp, machine):
    # more than 64 workers: two and sixteen workers per lane
    n_cpu, n_gpu = machine
    w = synth.random_dag(43, n_cpu, 2500, 0.003, n_cpu=n_cpu, n_gpu=n_gpu, dur_hi=60, est_equal=False)
    for policy in ("inspirit", "fifo", "heft"):
        say("workers", machine, policy)
        g = run_gpu(insp, w, policy)
        assert_same(g, oracle.schedule(w, policy=policy, variant=oracle.HEAP), f"workers {machine} {policy}")
        check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"])
    say("workers", machine, "transitive")
    g = run_gpu(insp, w, "inspirit", attr_mode="transitive")
    assert_same(g, oracle.schedule(w, variant=oracle.HEAP, attr_mode="transitive"), f"workers {machine} transitive")


def test_w8_heft_on_gpu(insp):
    with open(os.path.join(GOLD, "w8_heft.json")) as f:
        g8 = json.load(f)["w8"]
    n = g8["n"]
    w = NS(n=n, row_ptr=np.asarray(g8["row_ptr"], np.int32), col=np.asarray(g8["col"], np.int32),
           dur=np.asarray(g8["dur"], np.int32), est=np.asarray(g8["dur"], np.int32), n_cpu=g8["n_cpu"],
           n_gpu=g8["n_gpu"], m=len(g8["col"]), type=np.zeros(n, np.int32), name="w8")
    say("w8 heft")
    g = run_gpu(insp, w, "heft")
    assert g["start"].tolist() == g8["heft"]["start"] and g["worker"].tolist() == g8["heft"]["worker"]
    assert g["makespan"] == g8["heft"]["makespan"]
    assert set(g["mode_at_pop"].tolist()) == {g8["heft"]["mode_at_pop"]}


@pytest.mark.parametrize("policy", ["heft"])
def test_lu_and_cholesky_heft(insp, policy):
    for w in (synth.lu_workload(nb=24), synth.cfg2()):
        say("heft", w.name)
        g = run_gpu(insp, w, policy)
        assert_same(g, oracle.schedule(w, policy=policy, variant=oracle.HEAP), w.name)


def test_heft_batch(insp):
    ws = synth.cfg3(select=list(range(3, 4096, 300))) + [_permuted(synth.lu_workload(nb=8), 5), _hubs(4)]
    b = synth.concat(ws)
    say("heft batch", len(ws))
    dag, dur, est = insp.batch_to_device(b)
    r = oracle.schedule_batch(b, policy="heft")
    for key in (None, "waves=1,grid=2", "waves=1,grid=5,lds_blocks=0,lds_slots=0"):
        o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est, insp.params(policy="heft"),
                                tune_key=key)
        insp.sync_status(dag)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(o[k].cpu().numpy(), r[k]), (key, k)
        assert np.array_equal(o["makespan"].cpu().numpy(), r["makespan"]), key
    # the same handle under another policy afterwards is unaffected
    o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est)
    insp.sync_status(dag)
    assert np.array_equal(o["start"].cpu().numpy(), oracle.schedule_batch(b)["start"])
    dag.free()


def _chain(n, tick, n_cpu):
    rp = np.minimum(np.arange(n + 1), n - 1).astype(np.int32)
    rp[0] = 0
    return NS(n=n, row_ptr=rp, col=np.arange(1, n, dtype=np.int32), dur=np.full((n, 2), tick, np.int32),
              est=np.full((n, 2), tick, np.int32), n_cpu=n_cpu, n_gpu=0, m=n - 1, type=np.zeros(n, np.int32),
              name=f"chain-{n}")


def test_heft_rank_limit(insp):
    # a chain at the largest tick on 1024 workers: the source's rank is
    # n * 1024 * 2^20, which reaches 2^42 at n = 4096
    say("heft rank limit")
    w = _chain(4095, 1 << 20, 1024)
    g = run_gpu(insp, w, "heft")
    assert g["makespan"] == 4095 << 20 and g["start"].tolist() == [v << 20 for v in range(4095)]
    with pytest.raises(insp.InspError) as e:
        run_gpu(insp, _chain(4096, 1 << 20, 1024), "heft")
    assert e.value.code == insp.E_RANGE


# ------------------------------------------------------- transitive attributes

def _trans_pair(insp, w, unit_time=0):
    dag, dur, est = insp.to_device(w)
    ia, ie, U, lp = insp.transitive_attributes(dag, 0, est, (w.n_cpu, w.n_gpu), unit_time=unit_time)
    dag.free()
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    ref = oracle.transitive(w.n, rp, col, w.est, w.n_gpu, unit_time=unit_time)
    return (ia.cpu().numpy(), ie.cpu().numpy(), int(U[0]), int(lp[0])), ref


def _assert_trans(got, ref, what):
    for k, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(np.asarray(a), np.asarray(b)), (what, ("ia", "ie", "U", "longest")[k])


def _from_gold(g, n_cpu=1):
    n = g["n"]
    est = np.asarray(g["est"], np.int32)
    return NS(n=n, row_ptr=np.asarray(g["row_ptr"], np.int32), col=np.asarray(g["col"], np.int32), dur=est,
              est=est, n_cpu=n_cpu, n_gpu=g["n_gpu"], m=len(g["col"]), type=np.zeros(n, np.int32), name="gold")


def test_transitive_fixtures_on_gpu(insp):
    with open(os.path.join(GOLD, "w9_transitive.json")) as f:
        g = json.load(f)
    say("transitive fixtures")
    w9 = _from_gold(g["w9"])
    got, _ = _trans_pair(insp, w9, unit_time=7)
    assert got[0].tolist() == g["w9"]["ia_t"] and got[1].tolist() == g["w9"]["ie_t_u7"] and got[3] == 11
    got, _ = _trans_pair(insp, w9)
    assert got[2] == g["w9"]["unit_time_auto"] and got[1].tolist() == g["w9"]["ie_t_auto"]
    for key in ("w10_tie", "w10_top"):
        got, _ = _trans_pair(insp, _from_gold(g[key]))
        assert got[2] == g[key]["unit_time_auto"] and got[1].tolist() == g[key]["ie_t_auto"], key
    # Section 4.3: the source of a fully connected DAG scores every task
    N = 40
    rp = np.array([0] + list(np.cumsum([N - 1 - i for i in range(N)])), np.int32)
    col = np.array([j for i in range(N) for j in range(i + 1, N)], np.int32)
    wc = NS(n=N, row_ptr=rp, col=col, dur=np.ones((N, 2), np.int32), est=np.ones((N, 2), np.int32), n_cpu=2,
            n_gpu=1, m=int(col.size), type=np.zeros(N, np.int32), name="complete")
    got, ref = _trans_pair(insp, wc)
    assert got[0][0] == N
    _assert_trans(got, ref, "complete")


def test_transitive_random_match_oracle(insp):
    for i in range(24):
        n = 1 + (i * 37) % 700
        w = synth.random_dag(61, i, n, 4.0 / max(n, 4), n_cpu=2, n_gpu=i % 2, dur_hi=40, est_equal=(i % 3 == 0))
        if i % 4 == 3:
            w = _permuted(w, i)
        for U in (0, 1 + (i * 13) % 90):
            say("transitive random", i, n, U)
            got, ref = _trans_pair(insp, w, unit_time=U)
            _assert_trans(got, ref, f"random {i} U={U}")


def test_transitive_batch_match_oracle(insp):
    # all DAGs of a batch in one call, the largest of the layered batch included
    sel = [0, 3, 700, 1500]
    pool = synth.cfg3(select=list(range(0, 4096, 97)))
    big = max(pool, key=lambda w: w.n)
    ws = synth.cfg3(select=sel) + [big, _permuted(synth.lu_workload(nb=8), 3)]
    b = synth.concat(ws)
    say("transitive batch", [w.n for w in ws])
    dag, dur, est = insp.batch_to_device(b)
    ia, ie, U, lp = insp.transitive_attributes(dag, insp.ALL_DAGS, est, [(w.n_cpu, w.n_gpu) for w in ws])
    ia, ie = ia.cpu().numpy(), ie.cpu().numpy()
    dag.free()
    for k, w in enumerate(ws):
        a, z = int(b.task_off[k]), int(b.task_off[k + 1])
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        ria, rie, rU, rcp = oracle.transitive(w.n, rp, col, w.est, w.n_gpu)
        assert np.array_equal(ia[a:z], ria) and np.array_equal(ie[a:z], rie), k
        assert U[k] == rU and lp[k] == rcp, k


@pytest.mark.parametrize("policy", ["inspirit", "ability", "efi", "fifo", "heft"])
def test_transitive_schedule_match_oracle(insp, policy):
    for i in range(16):
        n = 2 + (i * 29) % 300
        w = synth.random_dag(62, i, n, 3.0 / max(n, 3), n_cpu=1 + i % 4, n_gpu=i % 3, dur_hi=30,
                             est_equal=(i % 2 == 0))
        say("transitive schedule", policy, i, n)
        kw = dict(attr_mode="transitive", unit_time=0 if i % 2 else 25)
        g = run_gpu(insp, w, policy, **kw)
        assert_same(g, oracle.schedule(w, policy=policy, variant=oracle.HEAP, **kw), f"trans {policy} {i}")
        check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"])


def test_transitive_schedule_batch(insp):
    ws = synth.cfg3(select=list(range(5, 4096, 400))) + [_hubs(6)]
    b = synth.concat(ws)
    say("transitive schedule batch", len(ws))
    dag, dur, est = insp.batch_to_device(b)
    prm = insp.params(attr_mode="transitive")
    o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est, prm)
    insp.sync_status(dag)
    r = oracle.schedule_batch(b, attr_mode="transitive")
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
        assert np.array_equal(o[k].cpu().numpy(), r[k]), k
    assert np.array_equal(o["makespan"].cpu().numpy(), r["makespan"])
    # the direct attributes afterwards on the same handle are unaffected
    o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est)
    insp.sync_status(dag)
    assert np.array_equal(o["start"].cpu().numpy(), oracle.schedule_batch(b)["start"])
    dag.free()


def test_transitive_range_errors(insp):
    say("transitive range")
    # longest path 1100 * 2^20 ticks >= 2^30
    w = _chain(1100, 1 << 20, 2)
    dag, dur, est = insp.to_device(w)
    with pytest.raises(insp.InspError) as e:
        insp.transitive_attributes(dag, 0, est, (2, 0))
    assert e.value.code == insp.E_RANGE
    insp.schedule(dag, 0, (2, 0), dur, est, insp.params(attr_mode="transitive"))
    with pytest.raises(insp.InspError) as e:
        insp.sync_status(dag)
    assert e.value.code == insp.E_RANGE
    dag.free()
    # 1023 such tasks stay below
    w = _chain(1023, 1 << 20, 2)
    got, ref = _trans_pair(insp, w)
    _assert_trans(got, ref, "chain 1023")
    # more tasks than the transitive pass takes
    w = _chain(insp.MAX_TRANSITIVE_TASKS + 1, 1, 1)
    dag, dur, est = insp.to_device(w)
    with pytest.raises(insp.InspError) as e:
        insp.transitive_attributes(dag, 0, est, (1, 0))
    assert e.value.code == insp.E_RANGE
    dag.free()


# ------------------------------------------------------------------ data model

def _kib(w, seed, hi=64):
    return synth.Stream(seed, 9).randint(np.arange(w.n), 0, hi).astype(np.int32)


def run_gpu_data(insp, w, policy, data_bw, **kw):
    import torch
    dag, dur, est = insp.to_device(w)
    insp.set_task_data(dag, torch.from_numpy(np.ascontiguousarray(w.data_kib, np.int32)).cuda())
    o = insp.schedule(dag, 0, (w.n_cpu, w.n_gpu), dur, est, insp.params(policy=policy, data_bw=data_bw, **kw))
    insp.sync_status(dag)
    res = {k: o[k][:w.n].cpu().numpy() for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop")}
    res["makespan"] = int(o["makespan"].item())
    dag.free()
    return res


def test_data_fixtures_on_gpu(insp):
    with open(os.path.join(GOLD, "w11_data.json")) as f:
        g = json.load(f)
    say("data fixtures")
    for key, pol, fx in (("w11", "locality", "locality"), ("w11", "efi", "efi"), ("w12", "fifo", "fifo")):
        x = g[key]
        d = np.asarray(x["dur"], np.int32)
        w = NS(n=x["n"], row_ptr=np.asarray(x["row_ptr"], np.int32), col=np.asarray(x["col"], np.int32), dur=d,
               est=d, n_cpu=x["n_cpu"], n_gpu=x["n_gpu"], m=len(x["col"]), type=np.zeros(x["n"], np.int32),
               data_kib=np.asarray(x["data_kib"], np.int32), name=key)
        r = run_gpu_data(insp, w, pol, x["data_bw"], unit_time=x.get("unit_time", 0))
        for f in ("worker", "start", "finish"):
            assert r[f].tolist() == x[fx][f], (key, pol, f)
        assert r["makespan"] == x[fx]["makespan"], (key, pol)


@pytest.mark.parametrize("policy", ["inspirit", "locality", "fifo", "efi", "heft"])
def test_data_model_random_match_oracle(insp, policy):
    for i in range(14):
        n = 3 + (i * 41) % 400
        w = synth.random_dag(81, i, n, 3.0 / max(n, 3), n_cpu=1 + i % 4, n_gpu=1 + i % 3, dur_hi=40,
                             est_equal=(i % 2 == 0))
        if i % 5 == 4:
            w = _permuted(w, i)
        w.data_kib = _kib(w, i, hi=40 + 30 * (i % 3))
        bw = 256 * (1 + i % 4)
        kw = dict(attr_mode="transitive") if i % 7 == 3 else {}
        say("data random", policy, i, n, bw, kw)
        g = run_gpu_data(insp, w, policy, bw, **kw)
        r = oracle.schedule(w, policy=policy, variant=oracle.HEAP, data_bw=bw, **kw)
        assert_same(g, r, f"data {policy} {i}")
        check_schedule(w, g["worker"], g["start"], g["finish"], g["makespan"], non_idling=False)


def test_data_model_cholesky_and_many_workers(insp):
    w = synth.cfg2()
    w.data_kib = np.full(w.n, 3600, np.int32)  # a 960 x 960 fp32 tile
    for pol in ("inspirit", "locality"):
        say("data cholesky", pol)
        g = run_gpu_data(insp, w, pol, 1 << 20)
        assert_same(g, oracle.schedule(w, policy=pol, variant=oracle.HEAP, data_bw=1 << 20), f"cholesky {pol}")
    for n_cpu, n_gpu in ((70, 30), (200, 100)):
        w = synth.random_dag(82, n_cpu, 1500, 0.004, n_cpu=n_cpu, n_gpu=n_gpu, dur_hi=60, est_equal=False)
        w.data_kib = _kib(w, n_cpu, hi=100)
        for pol in ("inspirit", "locality"):
            say("data workers", n_cpu, n_gpu, pol)
            g = run_gpu_data(insp, w, pol, 512)
            assert_same(g, oracle.schedule(w, policy=pol, variant=oracle.HEAP, data_bw=512), f"workers {pol}")


def test_data_model_batch(insp):
    import torch
    ws = synth.cfg3(select=list(range(11, 4096, 500))) + [_hubs(8)]
    b = synth.concat(ws)
    b.data_kib = np.concatenate([_kib(w, k, hi=80) for k, w in enumerate(ws)])
    say("data batch", len(ws))
    dag, dur, est = insp.batch_to_device(b)
    insp.set_task_data(dag, torch.from_numpy(b.data_kib).cuda())
    for pol in ("inspirit", "locality"):
        r = oracle.schedule_batch(b, policy=pol, data_bw=700)
        for key in (None, "waves=1,grid=3,lds_blocks=0,lds_slots=0"):
            o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est,
                                    insp.params(policy=pol, data_bw=700), tune_key=key)
            insp.sync_status(dag)
            for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
                assert np.array_equal(o[k].cpu().numpy(), r[k]), (pol, key, k)
    # without the data model the same handle schedules as before
    o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est)
    insp.sync_status(dag)
    assert np.array_equal(o["start"].cpu().numpy(), oracle.schedule_batch(b)["start"])
    dag.free()


def test_data_model_errors(insp):
    import torch
    say("data errors")
    w = synth.random_dag(83, 0, 20, 0.3, n_cpu=1, n_gpu=1)
    dag, dur, est = insp.to_device(w)
    with pytest.raises(insp.InspError) as e:
        insp.schedule(dag, 0, (1, 1), dur, est, insp.params(data_bw=100))
    assert e.value.code == insp.E_INVAL  # no sizes attached
    bad = torch.zeros(w.n, dtype=torch.int32, device="cuda")
    bad[3] = -1
    with pytest.raises(insp.InspError) as e:
        insp.set_task_data(dag, bad)
    assert e.value.code == insp.E_RANGE
    dag.free()
    # three inputs, one on each memory node (the CPU's, then each GPU's): any
    # worker moves two of them, 2 (2^19 + 1) ticks > 2^20
    d = np.array([[1, 100], [100, 1], [100, 1], [1, 1]], np.int32)
    w = NS(n=4, row_ptr=np.array([0, 1, 2, 3, 3], np.int32), col=np.array([3, 3, 3], np.int32), dur=d, est=d,
           n_cpu=1, n_gpu=2, m=3, type=np.zeros(4, np.int32), data_kib=np.array([(1 << 19) + 1] * 3 + [0], np.int32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.schedule(w, data_bw=1024, policy="fifo")
    assert e.value.code == oracle.E_RANGE
    dag, dur, est = insp.to_device(w)
    insp.set_task_data(dag, torch.from_numpy(w.data_kib).cuda())
    insp.schedule(dag, 0, (1, 2), dur, est, insp.params(policy="fifo", data_bw=1024))
    with pytest.raises(insp.InspError) as e:
        insp.sync_status(dag)
    assert e.value.code == insp.E_RANGE
    insp.set_task_data(dag, None)
    dag.free()


# ------------------------------------------------------------------ edge cases

def _empty(n_cpu=2, n_gpu=1):
    return NS(n=0, row_ptr=np.zeros(1, np.int32), col=np.zeros(0, np.int32), dur=np.zeros((0, 2), np.int32),
              est=np.zeros((0, 2), np.int32), n_cpu=n_cpu, n_gpu=n_gpu, m=0, type=np.zeros(0, np.int32),
              name="empty")


def _single(tick, n_cpu=1, n_gpu=1):
    d = np.array([[tick, tick + 1]], np.int32)
    return NS(n=1, row_ptr=np.zeros(2, np.int32), col=np.zeros(0, np.int32), dur=d, est=d, n_cpu=n_cpu,
              n_gpu=n_gpu, m=0, type=np.zeros(1, np.int32), name="single")


def test_batch_with_empty_and_single_task_dags(insp):
    import torch
    ws = [_empty(), _single(5)] + synth.cfg3(select=[9, 90]) + [_empty(1, 0), _single(3, 2, 0),
                                                               synth.lu_workload(nb=5), _empty()]
    b = synth.concat(ws)
    b.data_kib = np.concatenate([np.full(w.n, 7 + k, np.int32) for k, w in enumerate(ws)])
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    dag, dur, est = insp.batch_to_device(b)
    insp.set_task_data(dag, torch.from_numpy(b.data_kib).cuda())
    for pol, kw in (("inspirit", {}), ("fifo", {}), ("heft", {}), ("inspirit", {"attr_mode": "transitive"}),
                    ("locality", {"data_bw": 300}), ("inspirit", {"data_bw": 300})):
        r = oracle.schedule_batch(b, policy=pol, **kw)
        for key in (None, "grid=2,lds_slots=0", "grid=3,lds_slots=1,lds_keys=24"):
            say("edge batch", pol, kw, key)
            o = insp.schedule_batch(dag, workers, dur, est, insp.params(policy=pol, **kw), tune_key=key)
            insp.sync_status(dag)
            for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
                assert np.array_equal(o[k].cpu().numpy(), r[k]), (pol, kw, key, k)
            ms = o["makespan"].cpu().numpy()
            assert np.array_equal(ms, r["makespan"]) and ms[0] == 0 and ms[-1] == 0, (pol, kw, key)
    ia, ie, U, lp = insp.transitive_attributes(dag, insp.ALL_DAGS, est, workers)
    ia, ie = ia.cpu().numpy(), ie.cpu().numpy()
    for k, w in enumerate(ws):
        a, z = int(b.task_off[k]), int(b.task_off[k + 1])
        if w.n == 0:
            assert U[k] == 1 and lp[k] == 0, k
            continue
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        ria, rie, rU, rcp = oracle.transitive(w.n, rp, col, w.est, w.n_gpu)
        assert np.array_equal(ia[a:z], ria) and np.array_equal(ie[a:z], rie) and U[k] == rU and lp[k] == rcp, k
    ia, ie, U = insp.attributes(dag, insp.ALL_DAGS, est, workers)
    ia, ie = ia.cpu().numpy(), ie.cpu().numpy()
    for k, w in enumerate(ws):
        a, z = int(b.task_off[k]), int(b.task_off[k + 1])
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, w.n_gpu)
        assert np.array_equal(ia[a:z], ria) and np.array_equal(ie[a:z], rie) and U[k] == rU, k
    dag.free()


def test_batch_trace_matches_oracle(insp):
    """Per-DAG event traces of one batch call: every record of every DAG
    against the oracle's trace of that DAG alone, under the one-wave loop's
    policies, HEFT, transitive attributes and the data model."""
    import torch
    ws = [_empty(), _single(5)] + synth.cfg3(select=[9, 90, 700, 2048]) + [_hubs(8), synth.lu_workload(nb=5),
                                                                             _empty(1, 0)]
    for k, w in enumerate(ws):
        w.data_kib = np.full(w.n, 7 + k, np.int32) if w.n else np.zeros(0, np.int32)
    b = synth.concat(ws)
    b.data_kib = np.concatenate([w.data_kib for w in ws])
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    dag, dur, est = insp.batch_to_device(b)
    insp.set_task_data(dag, torch.from_numpy(b.data_kib).cuda())
    cases = (("inspirit", {}, None), ("fifo", {}, None), ("efi", {}, "waves=1,grid=3,lds_blocks=0,lds_slots=0"),
             ("heft", {}, None), ("inspirit", {"attr_mode": "transitive"}, None),
             ("inspirit", {"data_bw": 300}, None), ("locality", {"data_bw": 300}, "waves=1,grid=2"))
    for pol, kw, key in cases:
        say("batch trace", pol, kw, key)
        o = insp.schedule_batch(dag, workers, dur, est, insp.params(policy=pol, **kw), tune_key=key, trace=True)
        insp.sync_status(dag)
        r = oracle.schedule_batch(b, policy=pol, **kw)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(o[k].cpu().numpy(), r[k]), (pol, kw, k)
        nev = o["n_events"].cpu().numpy()
        for k, w in enumerate(ws):
            if w.n == 0:
                assert nev[k] == 0, (pol, kw, k)
                continue
            ref = oracle.schedule(w, policy=pol, variant=oracle.HEAP, trace=True, **kw)
            assert nev[k] == ref["n_events"] and nev[k] <= w.n + 1, (pol, kw, k)
            g = insp.batch_trace_records(dag, o, k)
            for f in ("t", "nready", "mode", "cnt", "peak", "pushed", "popped"):
                assert np.array_equal(g[f], ref["trace"][f]), (pol, kw, k, f)
    # the trace arrays are required
    lib = insp.load()
    P = insp.C.c_void_p
    n, B = int(b.task_off[-1]), len(ws)
    o = insp._outputs(n, dur.device)
    ms = torch.empty(B, dtype=torch.int64, device=dur.device)
    prm = insp.params()
    rc = lib.insp_schedule_batch_trace(dag.handle, insp._workers(workers, B), P(dur.data_ptr()), P(est.data_ptr()),
                                       insp.C.byref(prm), P(o["worker"].data_ptr()), P(o["start"].data_ptr()),
                                       P(o["finish"].data_ptr()), P(ms.data_ptr()), None, None, None, None, None,
                                       None)
    assert rc == insp.E_INVAL
    dag.free()


def test_single_empty_dag(insp):
    import torch
    say("single empty dag")
    w = _empty()
    dag = insp.build_dag([0, 0], [0, 0], torch.zeros(1, dtype=torch.int32, device="cuda"),
                         torch.zeros(1, dtype=torch.int32, device="cuda"))
    d = torch.zeros((1, 2), dtype=torch.int32, device="cuda")
    for pol, kw in (("inspirit", {}), ("heft", {}), ("inspirit", {"attr_mode": "transitive"})):
        o = insp.schedule(dag, 0, (w.n_cpu, w.n_gpu), d, d, insp.params(policy=pol, **kw))
        insp.sync_status(dag)
        assert int(o["makespan"].item()) == 0
    ia, ie, U, lp = insp.transitive_attributes(dag, 0, d, (2, 1))
    assert U[0] == 1 and lp[0] == 0
    dag.free()


def test_data_model_long_queues(insp):
    # layered DAGs of thousands of tasks moving 960 x 960 fp32 tiles: queues
    # span several blocks and pops move entries between blocks, which must
    # carry their inputs' arrival bounds along
    ws = synth.cfg3(select=[0, 2])
    b = synth.concat(ws)
    b.data_kib = np.full(int(b.task_off[-1]), 3600, np.int32)
    say("data long queues", [w.n for w in ws])
    dag, dur, est = insp.batch_to_device(b)
    insp.set_task_data(dag, torch_tensor(b.data_kib))
    for pol in ("locality", "inspirit"):
        o = insp.schedule_batch(dag, [(w.n_cpu, w.n_gpu) for w in ws], dur, est,
                                insp.params(policy=pol, data_bw=61440))
        insp.sync_status(dag)
        r = oracle.schedule_batch(b, policy=pol, data_bw=61440)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(o[k].cpu().numpy(), r[k]), (pol, k)
    dag.free()


def torch_tensor(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# --------------------------------------------------------- full-size workloads

def test_full_batch_4096(insp):
    # the 4096-DAG batch at full size: every schedule (default and tuned
    # launch shapes) and the full attribute pass of every DAG
    ws = synth.cfg3()
    b = synth.concat(ws)
    say("full batch", len(ws), int(b.task_off[-1]))
    dag, dur, est = insp.batch_to_device(b)
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    r = oracle.schedule_batch(b, threads=16)
    for key in (None, "waves=1,grid=2048,lds_blocks=256,lds_slots=24"):
        o = insp.schedule_batch(dag, workers, dur, est, tune_key=key)
        insp.sync_status(dag)
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(o[k].cpu().numpy(), r[k]), (key, k)
        assert np.array_equal(o["makespan"].cpu().numpy(), r["makespan"]), key
    ia, ie, U = insp.attributes(dag, insp.ALL_DAGS, est, workers)
    ia, ie = ia.cpu().numpy(), ie.cpu().numpy()
    for k, w in enumerate(ws):
        a, z = int(b.task_off[k]), int(b.task_off[k + 1])
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, w.n_gpu)
        assert np.array_equal(ia[a:z], ria) and np.array_equal(ie[a:z], rie) and U[k] == rU, k
    dag.free()


def test_full_powerlaw_2m(insp):
    # the single 2M-task power-law DAG (72 workers: the 64-bit loop): the full
    # schedule and the full attribute recompute
    w = synth.cfg4()
    say("powerlaw 2M", w.n, w.m)
    dag, dur, est = insp.to_device(w)
    o = insp.schedule(dag, 0, (w.n_cpu, w.n_gpu), dur, est, insp.params())
    insp.sync_status(dag)
    r = oracle.schedule(w, variant=oracle.HEAP)
    for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
        assert np.array_equal(o[k][:w.n].cpu().numpy(), r[k]), k
    assert int(o["makespan"].item()) == r["makespan"]
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    ia, ie, U = insp.attributes(dag, 0, est, (w.n_cpu, w.n_gpu))
    ria, rie, rU = oracle.attributes(w.n, rp, col, w.est, w.n_gpu)
    assert np.array_equal(ia.cpu().numpy(), ria) and np.array_equal(ie.cpu().numpy(), rie) and U[0] == rU
    dag.free()


@pytest.mark.parametrize("mode", ["heft", "transitive", "data", "locality"])
def test_graph_replays_every_mode(insp, mode):
    # the batch step of each policy, attribute reading and data model captured
    # in a HIP graph (after a warm call, which builds the per-handle state),
    # replayed with eager work on the same handle and synchronisations between
    import torch
    ws = synth.cfg3(select=list(range(13, 4096, 600))) + [_hubs(9)]
    b = synth.concat(ws)
    b.data_kib = np.concatenate([_kib(w, k, hi=90) for k, w in enumerate(ws)])
    kw = {"heft": dict(policy="heft"), "transitive": dict(attr_mode="transitive"),
          "data": dict(data_bw=600), "locality": dict(policy="locality", data_bw=600)}[mode]
    say("graph mode", mode, len(ws))
    dag, dur, est = insp.batch_to_device(b)
    insp.set_task_data(dag, torch_tensor(b.data_kib))
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    prm = insp.params(**kw)
    N = int(b.task_off[-1])
    r = oracle.schedule_batch(b, **kw)
    out = insp._outputs(N, dur.device)
    out["makespan"] = torch.empty(len(ws), dtype=torch.int64, device=dur.device)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        insp.schedule_batch(dag, workers, dur, est, prm, out=out)  # warm
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        insp.schedule_batch(dag, workers, dur, est, prm, out=out)
    for rep in range(3):
        for k in out:
            out[k].zero_()
        junk = insp.schedule_batch(dag, workers, dur, est, prm)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(out[k].cpu().numpy(), r[k]), (mode, rep, k)
        assert np.array_equal(out["makespan"].cpu().numpy(), r["makespan"]), (mode, rep)
        del junk
    insp.sync_status(dag)
    dag.free()


@pytest.mark.parametrize("mode", ["inspirit", "fifo", "heft", "transitive", "data", "locality"])
def test_library_graph_replays(insp, mode):
    # the batch step captured by the library itself (insp_batch_graph_create):
    # every replay, with eager work and synchronisations between, matches the
    # oracle; the outputs are cleared before each replay
    import torch
    ws = synth.cfg3(select=list(range(29, 4096, 700))) + [_hubs(5)]
    b = synth.concat(ws)
    b.data_kib = np.concatenate([_kib(w, k, hi=90) for k, w in enumerate(ws)])
    kw = {"inspirit": {}, "fifo": dict(policy="fifo"), "heft": dict(policy="heft"),
          "transitive": dict(attr_mode="transitive"), "data": dict(data_bw=600),
          "locality": dict(policy="locality", data_bw=600)}[mode]
    say("library graph", mode, len(ws))
    dag, dur, est = insp.batch_to_device(b)
    insp.set_task_data(dag, torch_tensor(b.data_kib))
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    r = oracle.schedule_batch(b, **kw)
    g = insp.BatchGraph(dag, workers, dur, est, insp.params(**kw))
    out = g.out
    for rep in range(3):
        for k in out:
            out[k].zero_()
        junk = insp.schedule_batch(dag, workers, dur, est, insp.params(policy="ability"))  # eager work
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(out[k].cpu().numpy(), r[k]), (mode, rep, k)
        assert np.array_equal(out["makespan"].cpu().numpy(), r["makespan"]), (mode, rep)
        del junk
    insp.sync_status(dag)
    g.free()
    dag.free()


def test_library_graph_replays_with_large_dags(insp):
    # two DAGs above the per-DAG kernel's limit in one batch, one whose taus
    # fit the grid pass's 8-bit words and one that needs the 16-bit ones,
    # beside small DAGs: the library-owned graph of the step, replayed with
    # eager work between, matches the oracle every time
    import torch
    narrow = _hub_dag(21, 33000, [1500, 70, 600, 3000])
    narrow = NS(**{**vars(narrow), "est": (narrow.est % 120 + 1).astype(np.int32)})
    narrow.dur = narrow.est.copy()
    wide = _hub_dag(22, 34000, [2100, 90, 5000])
    ws = synth.cfg3(select=[5, 1200]) + [narrow, wide] + synth.cfg3(select=[77])
    b = synth.concat(ws)
    say("library graph, large DAGs", [w.n for w in ws])
    dag, dur, est = insp.batch_to_device(b)
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    r = oracle.schedule_batch(b)
    g = insp.BatchGraph(dag, workers, dur, est, insp.params())
    out = g.out
    for rep in range(3):
        for k in out:
            out[k].zero_()
        junk = insp.schedule_batch(dag, workers, dur, est, insp.params(policy="efi"))  # eager work
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop"):
            assert np.array_equal(out[k].cpu().numpy(), r[k]), (rep, k)
        assert np.array_equal(out["makespan"].cpu().numpy(), r["makespan"]), rep
        del junk
    insp.sync_status(dag)
    g.free()
    dag.free()


def test_library_graph_argument_errors(insp):
    import torch
    say("library graph errors")
    ws = synth.cfg3(select=[3])
    b = synth.concat(ws)
    dag, dur, est = insp.batch_to_device(b)
    with pytest.raises(insp.InspError) as e:
        insp.BatchGraph(dag, [(0, 0)], dur, est)
    assert e.value.code == insp.E_RANGE
    lib = insp.load()
    assert lib.insp_batch_graph_launch(None, None) == insp.E_INVAL
    lib.insp_batch_graph_free(None)
    dag.free()
