"""The allocation-free batch call (insp_schedule_batch_noalloc) against
insp_schedule_batch and the oracle: bit-exact on consecutive calls of
different sizes, allocating no device memory, and refusing what it does not
serve.

Every test prints the case it is about to run, so a failing GPU step can be
named from the log.
"""
from types import SimpleNamespace as NS

import numpy as np
import pytest

import oracle
from paper_2404_03226_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("worker", "start", "finish", "ie_at_pop", "mode_at_pop", "makespan")


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


def batch(select):
    ws = synth.cfg3(select=select)
    return ws, synth.concat(ws)


def host(o, n):
    r = {k: o[k][:n].cpu().numpy().copy() for k in KEYS if k != "makespan"}
    r["makespan"] = o["makespan"].cpu().numpy().copy()
    return r


def same(a, b, what):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), f"{what}: {k} differs"


def run_both(insp, ws, b, policy="inspirit", tune_key=None):
    dag, dur, est = insp.batch_to_device(b)
    wk = [(w.n_cpu, w.n_gpu) for w in ws]
    prm = insp.params(policy=policy)
    n = int(b.task_off[-1])
    ref = host(insp.schedule_batch(dag, wk, dur, est, prm, tune_key=tune_key), n)
    insp.sync_status(dag)
    got = host(insp.schedule_batch_noalloc(dag, wk, dur, est, prm, tune_key=tune_key), n)
    insp.sync_status(dag)
    return dag, dur, est, wk, ref, got


def test_two_calls_in_a_row_second_smaller(insp):
    # a larger batch, then a smaller one on another handle: the second call
    # reuses the array the first one filled
    sizes = []
    for sel, what in ((list(range(0, 4096, 128)), "32 DAGs"), (list(range(7, 4096, 512)), "8 DAGs")):
        ws, b = batch(sel)
        say("noalloc batch", what, int(b.task_off[-1]), "tasks")
        dag, dur, est, wk, ref, got = run_both(insp, ws, b)
        same(got, ref, what)
        same(got, oracle.schedule_batch(b), what + " vs oracle")
        sizes.append(int(b.task_off[-1]))
        dag.free()
    assert sizes[1] < sizes[0]


def test_repeat_and_interleave_with_the_allocating_call(insp):
    ws, b = batch(list(range(3, 4096, 200)))
    say("noalloc repeat", int(b.task_off[-1]), "tasks")
    dag, dur, est, wk, ref, got = run_both(insp, ws, b)
    same(got, ref, "first")
    n = int(b.task_off[-1])
    for i in range(3):
        o = host(insp.schedule_batch_noalloc(dag, wk, dur, est), n)
        insp.sync_status(dag)
        same(o, ref, f"repeat {i}")
    # another handle in between: the tables are uploaded again
    ws2, b2 = batch([5, 9])
    dag2, dur2, est2, wk2, ref2, got2 = run_both(insp, ws2, b2)
    same(got2, ref2, "interleaved handle")
    o = host(insp.schedule_batch_noalloc(dag, wk, dur, est), n)
    insp.sync_status(dag)
    same(o, ref, "after the other handle")
    dag.free()
    dag2.free()


@pytest.mark.parametrize("policy", ["fifo", "ability", "efi"])
def test_policies(insp, policy):
    ws, b = batch(list(range(11, 4096, 409)))
    say("noalloc policy", policy)
    dag, dur, est, wk, ref, got = run_both(insp, ws, b, policy=policy)
    same(got, ref, policy)
    dag.free()


def test_launch_shapes(insp):
    ws, b = batch(list(range(1, 4096, 300)))
    for key in ("grid=1", "grid=3,lds_blocks=4,lds_slots=0", "grid=64,lds_slots=24", "grid=7,lds_slots=3,lds_keys=30"):
        say("noalloc tune", key)
        dag, dur, est, wk, ref, got = run_both(insp, ws, b, tune_key=key)
        same(got, ref, key)
        dag.free()


def test_allocates_no_device_memory(insp):
    import torch
    ws, b = batch(list(range(2, 4096, 256)))
    say("noalloc no allocation")
    dag, dur, est = insp.batch_to_device(b)
    wk = [(w.n_cpu, w.n_gpu) for w in ws]
    n = int(b.task_off[-1])
    out = insp._outputs(n, dur.device)
    out["makespan"] = torch.empty(len(ws), dtype=torch.int64, device=dur.device)
    ref = host(insp.schedule_batch(dag, wk, dur, est), n)
    insp.sync_status(dag)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    # every device allocation the library attempts from here on fails
    insp.test_fail_alloc(0)
    try:
        insp.schedule_batch_noalloc(dag, wk, dur, est, out=out)
        insp.sync_status(dag)
    finally:
        insp.test_fail_alloc(-1)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    same(host(out, n), ref, "preallocated outputs")
    dag.free()


def test_single_dag_empty_and_single_task_dags(insp):
    empty = NS(n=0, row_ptr=np.zeros(1, np.int32), col=np.zeros(0, np.int32), dur=np.zeros((0, 2), np.int32),
               est=np.zeros((0, 2), np.int32), n_cpu=2, n_gpu=1, m=0, type=np.zeros(0, np.int32), name="empty")
    d = np.array([[4, 5]], np.int32)
    single = NS(n=1, row_ptr=np.zeros(2, np.int32), col=np.zeros(0, np.int32), dur=d, est=d, n_cpu=1, n_gpu=1,
                m=0, type=np.zeros(1, np.int32), name="single")
    ws = [synth.cfg1(), empty, single]
    b = synth.concat(ws)
    say("noalloc layered-1k, an empty DAG and a one-task DAG")
    dag, dur, est, wk, ref, got = run_both(insp, ws, b)
    same(got, ref, "layered-1k + empty")
    dag.free()


def test_refusals(insp):
    import torch
    ws, b = batch([0, 1])
    say("noalloc refusals")
    dag, dur, est = insp.batch_to_device(b)
    wk = [(w.n_cpu, w.n_gpu) for w in ws]
    for kw in ({"policy": "heft"}, {"policy": "locality"}, {"attr_mode": "transitive"}):
        with pytest.raises(insp.InspError) as e:
            insp.schedule_batch_noalloc(dag, wk, dur, est, insp.params(**kw))
        assert e.value.code == insp.E_INVAL, kw
    with pytest.raises(insp.InspError) as e:
        insp.schedule_batch_noalloc(dag, wk, dur, est, tune_key="waves=2")
    assert e.value.code == insp.E_INVAL
    dag.free()
    # a batch larger than the static array: refused before any device work
    n = 1_000_000
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda").clamp_(max=n - 1)
    col = torch.arange(1, n, dtype=torch.int32, device="cuda")
    big = insp.build_dag([0, n], [0, n - 1], rp, col)
    d = torch.ones((n, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(insp.InspError) as e:
        insp.schedule_batch_noalloc(big, [(4, 1)], d, d)
    assert e.value.code == insp.E_RANGE
    assert "scratch" in str(e.value)
    big.free()
