"""Benchmark: tasks scheduled per second on the 4096-DAG batch (one MI355X).

A step is one pass of the whole hot path over the batch: the attribute pass
(IA, IE, unit-time ladder) and the persistent simulation of every DAG, from
inputs already resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch|large|cholesky|lu|layered]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tasks scheduled/s on 4096-DAG batch, bit-exact makespan; learned vs plain gap"
# Data model preset: every task leaves one 960 x 960 fp32 tile (the paper's
# Cholesky block); with a GPU GEMM tile at 25 ticks (~60 us), a tick is ~2.4
# us, and a ~25 GB/s host link moves a tile in ~150 us = 60 ticks.
TILE_KIB = 3600
TILE_BW = 61440
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # dense bf16 MFMA
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_batch4096.txt")
SIM_SOURCES = [os.path.join(ROOT, "paper_2404_03226_amd", "csrc", f) for f in ("sim.hip", "common.hpp", "internal.hpp")]
# Algorithmic bytes of the simulation kernel (the dependency release,
# frontier, push, pop and outputs): 76 B per task and 24 B per edge -- per
# edge the successor id (4), the dependency word read and write (8 + 8) and
# a tau gather (4); per task the row pointers (8), compaction (4), est (8),
# queue entry (12), pop key read (12), outputs (20), the IE update of the
# sole remaining predecessor with its tau (12).
SIM_BYTES_PER_TASK = 76
SIM_BYTES_PER_EDGE = 24
# The attribute pass as its definition reads it (standalone call): CSR
# 4(n+1) + 4m, rem 4n, tau 4n, ia/ie out 8n per DAG.
ATTR_BYTES = lambda n, m, b: 20 * n + 4 * m + 4 * b
# The attribute pass inside a schedule step: row pointers 4(n+1), successors
# 4m, the dependency word 8n (in-degree and the record's word), the estimate
# rows 8n (tau and the range check), and the 32-byte simulation record
# written per task in place of ia/ie.
ATTR_SCHED_BYTES = lambda n, m, b: 4 * (n + b) + 4 * m + 8 * n + 8 * n + 32 * n
# Unpacking the schedules: a 16-byte record read, worker/start/finish/IE/mode
# written (4 + 8 + 8 + 4 + 1 bytes) per task.
REC_BYTES_PER_TASK = 16 + 25


def host_info():
    """Host cores and CPU model (the CPU baseline's machine)."""
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": avail, "cpu_count": os.cpu_count(), "cpu_model": model}


def events_per_dag(finish, task_off):
    """Events of each DAG's simulation: one at t = 0 and one per distinct
    completion time (ticks are >= 1, so every finish time is positive)."""
    B = len(task_off) - 1
    dag = np.repeat(np.arange(B, dtype=np.int64), np.diff(task_off))
    keys = np.unique(dag << 42 | finish.astype(np.int64))
    ev = np.bincount((keys >> 42).astype(np.int64), minlength=B)
    return ev + (np.diff(task_off) > 0)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def sources_sha256():
    h = hashlib.sha256()
    for f in SIM_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the simulation kernel from the committed
    rocprofv3 counter summary, or None when the kernel's sources changed
    since the counters were taken."""
    try:
        for line in open(TRAFFIC_FILE):
            if line.startswith("# bench: "):
                kv = dict(x.split("=", 1) for x in line[len("# bench: "):].split())
                if kv.get("sources_sha256") == sources_sha256():
                    return int(kv["traffic_bytes"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def copy_calibration():
    """A plain device copy of 256 MiB, three times: the counters' reading of
    known traffic (FETCH_SIZE / WRITE_SIZE scale factors)."""
    import torch
    x = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 256 << 20, "copies": 3}), flush=True)


def nready_profile(rec, bins=24):
    """Nready over simulated time: per time bin, the mean and maximum of the
    observed ready count, the share of events under each pop rule, and the
    pushes and pops (the per-event trace the kernel records)."""
    t = rec["t"].astype(np.float64)
    edges = np.linspace(0.0, max(t.max(), 1.0), bins + 1)
    idx = np.clip(np.searchsorted(edges, t, side="right") - 1, 0, bins - 1)
    out = []
    for b in range(bins):
        m = idx == b
        if not m.any():
            continue
        mode = rec["mode"][m]
        out.append({"t0": int(edges[b]), "events": int(m.sum()),
                    "nready_mean": round(float(rec["nready"][m].mean()), 1), "nready_max": int(rec["nready"][m].max()),
                    "ability": round(float(np.mean(mode == 0)), 3), "efficiency": round(float(np.mean(mode == 1)), 3),
                    "efficiency_local": round(float(np.mean(mode == 2)), 3),
                    "pushed": int(rec["pushed"][m].sum()), "popped": int(rec["popped"][m].sum())})
    return out


def workload(name, nb=40):
    from paper_2404_03226_amd import synth
    if name == "batch":
        ws = synth.cfg3()
        desc = ("batch of 4096 layered DAGs, sizes log-uniform in [200, 20000] tasks, 2-8 later-layer targets "
                "per task, 4 types, 16 CPU + 4 GPU simulated workers each (seed 3)")
    elif name == "large":
        ws = [synth.cfg4()]
        desc = "one power-law DAG, 2,000,000 tasks, out-degree ~ d^-2.1 on [1, 4180], 64 CPU + 8 GPU (seed 4)"
    elif name == "cholesky":
        ws = [synth.cfg2(nb=nb)]
        desc = f"tiled Cholesky {nb}x{nb} ({ws[0].n:,} tasks), 24 CPU + 4 GPU, +-10% duration jitter (seed 2)"
    elif name == "lu":
        ws = [synth.lu_workload(nb=nb)]
        desc = f"tiled LU {nb}x{nb} without pivoting ({ws[0].n:,} tasks), 24 CPU + 4 GPU, +-10% duration jitter (seed 6)"
    else:
        ws = [synth.cfg1()]
        desc = "one layered DAG, 1,000 tasks in 20 layers, 8 CPU + 2 GPU (seed 1)"
    return ws, desc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["batch", "large", "cholesky", "lu", "layered"])
    ap.add_argument("--policy", default="inspirit")
    ap.add_argument("--tune", default=None, help="launch shape, e.g. waves=1,grid=2048")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-cost-model gap")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default launch shape")
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true", help="only run the counter calibration copy")
    ap.add_argument("--no-graph", action="store_true", help="skip timing hipGraph replays of the step")
    ap.add_argument("--nb", type=int, default=40, help="tiles per side for the cholesky and lu workloads")
    ap.add_argument("--compare-policies", action="store_true",
                    help="makespans under each pop rule against the plain DMDA (FIFO) baseline, checked against the oracle")
    ap.add_argument("--trace", action="store_true",
                    help="single DAG: record the per-event trace, check it against the oracle's, report Nready over time")
    ap.add_argument("--transitive", action="store_true",
                    help="also time the transitive attribute pass and the schedule ordered by it (sampled check)")
    ap.add_argument("--data", action="store_true",
                    help="data model: every task leaves one 960x960 fp32 tile, moved at 60 KiB per tick")
    ap.add_argument("--attr-only", action="store_true",
                    help="only time the standalone attribute pass (warm and cold) on the workload")
    ap.add_argument("--print-sources-sha256", action="store_true")
    args = ap.parse_args()
    if args.print_sources_sha256:
        print(sources_sha256())
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle
    from paper_2404_03226_amd import inspirit, synth

    t0 = time.time()
    ws, desc = workload(args.workload, args.nb)
    b = synth.concat(ws)
    N, M = int(b.task_off[-1]), int(b.edge_off[-1])
    log(f"workload {args.workload}: {len(ws)} DAGs, {N} tasks, {M} edges (generated in {time.time() - t0:.1f}s)")
    torch.cuda.set_device(0)
    dag, dur, est = inspirit.batch_to_device(b)
    workers = [(w.n_cpu, w.n_gpu) for w in ws]
    data_bw = TILE_BW if args.data else 0
    if args.data:
        b.data_kib = np.full(N, TILE_KIB, np.int32)
        inspirit.set_task_data(dag, torch.from_numpy(b.data_kib).to(dur.device))
    if args.attr_only:
        a = attr_measure(dag, workers, b, est, steps=max(args.steps, 1), warmup=max(args.warmup, 1))
        print(json.dumps({"metric": "attribute pass, ms per call", "workload": desc, "tasks": N, "edges": M,
                          "attributes": a}), flush=True)
        dag.free()
        return
    prm = inspirit.params(policy=args.policy, data_bw=data_bw)
    out = inspirit._outputs(N, dur.device)
    out["makespan"] = torch.empty(len(ws), dtype=torch.int64, device=dur.device)
    stream = torch.cuda.current_stream()

    tune_key = args.tune
    if tune_key is None and not args.no_tune and len(ws) > 1:
        from paper_2404_03226_amd import autotune
        tune_key = autotune.tune(dag, workers, dur, est, prm, out, verbose=False)
        log(f"autotuned launch: {tune_key}")

    def step():
        inspirit.schedule_batch(dag, workers, dur, est, prm, tune_key=tune_key, out=out)

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    inspirit.sync_status(dag)
    torch.cuda.synchronize()
    inspirit.profile_enable(2)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    inspirit.sync_status(dag)
    ms = ev0.elapsed_time(ev1) / args.steps
    kern = {}
    for k in ("pass_attr", "attr_dag", "attr_pack", "attr_a", "attr_sel", "attr_b", "sim", "rec"):
        tot, cnt = inspirit.profile_read(k)
        if cnt:
            kern[k] = {"avg_ms": tot / cnt, "launches": cnt // args.steps if cnt >= args.steps else cnt}
    inspirit.profile_enable(False)
    log(f"timed {args.steps} steps: {ms:.3f} ms/step; kernels {kern}")

    B = len(ws)
    for k, nbytes in (("sim", SIM_BYTES_PER_TASK * N + SIM_BYTES_PER_EDGE * M),
                      ("pass_attr", ATTR_SCHED_BYTES(N, M, B)), ("rec", REC_BYTES_PER_TASK * N)):
        if k in kern:
            kern[k]["algorithmic_bytes"] = nbytes
            kern[k]["achieved_GBs"] = round(nbytes / (kern[k]["avg_ms"] * 1e-3) / 1e9, 2)
            kern[k]["frac_hbm_peak"] = round(kern[k]["achieved_GBs"] / HBM_PEAK_GBS, 5)
    if "pass_attr" in kern:
        kern["pass_attr"]["note"] = ("the whole attribute pass as one unit (every launch and the gaps between them); "
                                     "bytes: row pointers, successors, dependency words, estimate rows and the "
                                     "32-byte simulation records it writes")
    dom = "sim"
    roof = {"bound": "hbm", "kernel": dom, "achieved": kern[dom]["achieved_GBs"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kern[dom]["frac_hbm_peak"],
            "traffic": measured_traffic(),
            "bytes_per_launch": kern[dom]["algorithmic_bytes"],
            "note": "76 B per task + 24 B per edge; the simulation is latency-bound along each DAG's chain of "
                    "dependent events, not HBM-bound (see events)"}

    graph = None
    if not args.no_graph and args.workload == "batch":
        # the same step as a HIP graph the library captures and owns
        lg = inspirit.BatchGraph(dag, workers, dur, est, prm, tune_key=tune_key, out=out)
        for i in range(args.warmup):
            lg.launch()
        torch.cuda.synchronize()
        ev0.record(stream)
        for i in range(args.steps):
            lg.launch()
        ev1.record(stream)
        torch.cuda.synchronize()
        gms = ev0.elapsed_time(ev1) / args.steps
        graph = {"ms_per_step": round(gms, 4), "tasks_per_s": round(N / (gms * 1e-3), 1), "replays": args.steps,
                 "capture": "insp_batch_graph_create (library-owned)"}
        log(f"hipGraph replays: {gms:.3f} ms/step")
        inspirit.sync_status(dag)
        lg.free()

    res = {k: out[k][:N].cpu().numpy() for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop")}
    res["makespan"] = out["makespan"].cpu().numpy()
    digest = hashlib.sha256(b"".join(res[k].tobytes() for k in ("worker", "start", "finish", "makespan")))

    # events of every DAG's simulation, from its completion times
    ev = events_per_dag(res["finish"], b.task_off)
    big = int(np.argmax(np.diff(b.task_off)))
    sim_s = kern["sim"]["avg_ms"] * 1e-3
    events = {"largest_dag": {"tasks": int(b.task_off[big + 1] - b.task_off[big]), "events": int(ev[big]),
                              "us_per_event": round(sim_s * 1e6 / max(int(ev[big]), 1), 3)},
              "total": int(ev.sum()), "events_per_s": round(float(ev.sum()) / sim_s, 1),
              "note": "per-event latency of the largest DAG's chain, which bounds the batch"}
    log(f"events: {events}")

    cpu = None
    bit_exact = None
    host = host_info()
    # the oracle on this host's cores, capped at the 16 cores a GPU's share
    # of the box has
    # (the oracle takes one DAG per thread: a single DAG uses one)
    threads = max(1, min(host["nproc"], 16, len(ws)))
    if not args.no_cpu_baseline or not args.no_verify:
        runs = 10 if not args.no_cpu_baseline else 1
        walls = []
        for i in range(runs):
            t1 = time.time()
            ref = oracle.schedule_batch(b, policy=args.policy, variant=oracle.HEAP, threads=threads,
                                        data_bw=data_bw)
            walls.append(time.time() - t1)
        wall = float(np.mean(walls[3:])) if runs == 10 else walls[0]
        log(f"oracle: {wall:.3f}s per run on {threads} threads ({runs} runs)")
        if not args.no_verify:
            bit_exact = bool(all(np.array_equal(res[k], ref[k]) for k in
                                 ("worker", "start", "finish", "ie_at_pop", "mode_at_pop", "makespan")))
        if not args.no_cpu_baseline:
            cpu = {"value": round(N / wall, 1), "unit": "tasks/s", "cores": threads, "kind": "oracle",
                   "sample": f"the whole workload ({len(ws)} DAGs, {N} tasks), heap-variant C oracle, one DAG "
                             f"per thread; 10 runs, the first 3 discarded, the mean of 7",
                   "host": host}

    line = {
        "metric": METRIC if args.workload == "batch" else f"tasks scheduled/s, {args.workload} workload, bit-exact",
        "value": round(N / (ms * 1e-3), 1),
        "unit": "tasks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": desc, "n_dags": len(ws), "tasks": N, "edges": M, "policy": args.policy,
                   "launch": tune_key or "default",
                   "data_model": (f"{TILE_KIB} KiB per task, {TILE_BW} B/tick" if args.data else None)},
        "bit_exact": bit_exact,
        "schedule_sha256": digest.hexdigest(),
        "roofline": roof,
        "events": events,
        "kernels": kern,
        "cpu_baseline": cpu,
        "graph_replay": graph,
        "nready_trace": None,
        "policies_vs_dmda": None,
        "learned_gap": None,
        "transitive": None,
        "attributes": attr_measure(dag, workers, b, est),
    }
    if args.compare_policies:
        line["policies_vs_dmda"] = compare_policies(dag, workers, b, dur, est, threads, data_bw)
    if args.trace and len(ws) == 1:
        w = ws[0]
        o = inspirit.schedule(dag, 0, (w.n_cpu, w.n_gpu), dur, est, prm, trace=True)
        inspirit.sync_status(dag)
        nev = int(o["n_events"].item())
        rec = inspirit.trace_records(o["trace"], nev)
        if args.data:
            w.data_kib = b.data_kib
        ref = oracle.schedule(w, policy=args.policy, variant=oracle.HEAP, trace=True, data_bw=data_bw)["trace"]
        same = bool(len(ref) == nev and all(np.array_equal(rec[f], ref[f]) for f in ref.dtype.names))
        line["nready_trace"] = {"events": nev, "bit_exact": same, "profile": nready_profile(rec)}
    if args.transitive:
        line["transitive"] = transitive_measure(dag, workers, ws, b, dur, est, args.steps, args.warmup, tune_key)
    if args.workload == "batch" and not args.no_learned:
        line["learned_gap"] = learned_gap(dag, workers, b, ws, args.epochs)
    print(json.dumps(line), flush=True)
    dag.free()


def attr_measure(dag, workers, b, est, steps=7, warmup=3):
    """The standalone attribute call (IA, IE and U of every DAG) timed by
    itself, warm and cold (a 1 GiB device fill between calls evicts the
    caches), as the library's attribute pass event brackets it."""
    import torch
    from paper_2404_03226_amd import inspirit
    N, M, B = int(b.task_off[-1]), int(b.edge_off[-1]), len(workers)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=est.device)
    out = {}
    for mode in ("warm", "cold"):
        for _ in range(warmup):
            inspirit.attributes(dag, inspirit.ALL_DAGS, est, workers)
        inspirit.profile_enable(2)
        for _ in range(steps):
            if mode == "cold":
                flush.fill_(1)
            inspirit.attributes(dag, inspirit.ALL_DAGS, est, workers)
        tot, cnt = inspirit.profile_read("pass_attr")
        inspirit.profile_enable(False)
        ms = tot / max(cnt, 1)
        nbytes = ATTR_BYTES(N, M, B)
        out[mode] = {"ms": round(ms, 4), "algorithmic_bytes": nbytes,
                     "achieved_GBs": round(nbytes / (ms * 1e-3) / 1e9, 2),
                     "frac_hbm_peak": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
    del flush
    out["note"] = "insp_attributes over every DAG; bytes 20n + 4m + 4 per DAG (CSR, rem, tau, ia/ie)"
    log(f"attributes: {out}")
    return out


def transitive_measure(dag, workers, ws, b, dur, est, steps, warmup, tune_key):
    """Time the transitive attribute pass over every DAG (and the schedule
    whose queues it orders), check a sample of DAGs against the oracle, and
    time the oracle on that sample."""
    import torch
    import oracle
    from paper_2404_03226_amd import inspirit
    N = int(b.task_off[-1])
    for _ in range(max(warmup, 1)):
        ia, ie, U, lp = inspirit.transitive_attributes(dag, inspirit.ALL_DAGS, est, workers)
    inspirit.profile_enable(2)
    t0 = time.time()
    for _ in range(steps):
        ia, ie, U, lp = inspirit.transitive_attributes(dag, inspirit.ALL_DAGS, est, workers)
    wall = (time.time() - t0) / steps
    tot, cnt = inspirit.profile_read("trans")
    inspirit.profile_enable(False)
    k_ms = tot / max(cnt, 1)
    ia_h, ie_h = ia.cpu().numpy(), ie.cpu().numpy()
    pairs = int(ia_h.astype(np.int64).sum())
    # the schedule ordered by the transitive attributes
    prm = inspirit.params(attr_mode="transitive")
    out = inspirit._outputs(N, dur.device)
    out["makespan"] = torch.empty(len(ws), dtype=torch.int64, device=dur.device)
    for _ in range(max(warmup, 1)):
        inspirit.schedule_batch(dag, workers, dur, est, prm, tune_key=tune_key, out=out)
    inspirit.sync_status(dag)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    inspirit.profile_enable(2)
    ev0.record(stream)
    for _ in range(steps):
        inspirit.schedule_batch(dag, workers, dur, est, prm, tune_key=tune_key, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    sim_tot, sim_cnt = inspirit.profile_read("sim")
    inspirit.profile_enable(False)
    inspirit.sync_status(dag)
    sched_ms = ev0.elapsed_time(ev1) / steps
    # sampled check: every 64th DAG and the largest, attributes and schedules
    big = int(np.argmax([w.n for w in ws]))
    sample = sorted(set(range(0, len(ws), 64)) | {big})
    res = {k: out[k].cpu().numpy() for k in ("worker", "start", "finish", "ie_at_pop", "mode_at_pop", "makespan")}
    exact, t_cpu, n_cpu_tasks = True, 0.0, 0
    for k in sample:
        w = ws[k]
        a, z = int(b.task_off[k]), int(b.task_off[k + 1])
        rp, col = oracle.canon(w.n, w.row_ptr, w.col)
        t1 = time.time()
        ria, rie, rU, rcp = oracle.transitive(w.n, rp, col, w.est, w.n_gpu)
        t_cpu += time.time() - t1
        n_cpu_tasks += w.n
        exact &= bool(np.array_equal(ia_h[a:z], ria) and np.array_equal(ie_h[a:z], rie) and U[k] == rU
                      and lp[k] == rcp)
        r = oracle.schedule(w, variant=oracle.HEAP, attr_mode="transitive")
        exact &= bool(all(np.array_equal(res[f][a:z], r[f]) for f in ("worker", "start", "finish", "ie_at_pop",
                                                                        "mode_at_pop")))
        exact &= int(res["makespan"][k]) == r["makespan"]
    # k_trans: per descendant pair one LDS read and one clear, and one LDS
    # atomicMax per edge out of it; edges approximated by the mean out-degree
    lds_ops = pairs * (2.0 + b.edge_off[-1] / max(N, 1))
    lds_peak = 256 * 32 * 2.4e9  # CUs x LDS banks x clock
    t = {"attr_ms_per_call": round(wall * 1e3, 3), "k_trans_avg_ms": round(k_ms, 3),
         "tasks_per_s": round(N / wall, 1), "descendant_pairs": pairs,
         "pairs_per_s": round(pairs / (k_ms * 1e-3), 1),
         "lds_roofline": {"bound": "lds", "achieved": round(lds_ops / (k_ms * 1e-3) / 1e12, 3),
                          "peak": round(lds_peak / 1e12, 2), "unit": "Tops/s",
                          "frac": round(lds_ops / (k_ms * 1e-3) / lds_peak, 4),
                          "note": "LDS operations estimated from the mean out-degree"},
         "schedule_ms_per_step": round(sched_ms, 3), "schedule_tasks_per_s": round(N / (sched_ms * 1e-3), 1),
         "schedule_sim_ms": round(sim_tot / max(sim_cnt, 1), 3),
         "sample_bit_exact": exact, "sample": f"{len(sample)} DAGs ({n_cpu_tasks} tasks): every 64th and the largest",
         "cpu_baseline": {"value": round(n_cpu_tasks / t_cpu, 1), "unit": "tasks/s", "cores": 1, "kind": "oracle",
                          "sample": "the sampled DAGs' transitive attributes, C oracle, one thread"}}
    log(f"transitive: {t}")
    return t


def compare_policies(dag, workers, b, dur, est, threads, data_bw=0):
    """Per-DAG makespan under each pop rule, and under the HEFT upward-rank
    list baseline, relative to the plain DMDA push with FIFO queues (the
    method's baseline): speedup = M_dmda / M_policy.  Every makespan is
    checked against the oracle's."""
    import oracle
    from paper_2404_03226_amd import inspirit
    ms, exact = {}, True
    pols = ("fifo", "inspirit", "ability", "efi", "heft") + (("locality",) if data_bw else ())
    for pol in pols:
        o = inspirit.schedule_batch(dag, workers, dur, est, inspirit.params(policy=pol, data_bw=data_bw))
        inspirit.sync_status(dag)
        ms[pol] = o["makespan"].cpu().numpy().astype(np.float64)
        ref = oracle.schedule_batch(b, policy=pol, variant=oracle.HEAP, threads=threads, data_bw=data_bw)["makespan"]
        exact = exact and bool(np.array_equal(ms[pol], ref))
    out = {"makespans_bit_exact": exact}
    for pol in pols[1:]:
        sp = ms["fifo"] / ms[pol]
        out[pol] = {"geo_mean_speedup": round(float(np.exp(np.mean(np.log(sp)))), 4),
                    "max_speedup": round(float(sp.max()), 4), "min_speedup": round(float(sp.min()), 4),
                    "frac_faster": round(float(np.mean(sp > 1)), 4), "frac_slower": round(float(np.mean(sp < 1)), 4)}
    log(f"policies vs DMDA: {out}")
    return out


def learned_gap(dag, workers, b, ws, epochs):
    """Train the device MLP on 1M simulator records, predict per-kind ticks for
    every task of the batch, and compare makespans against true durations for
    est = truth, est = per-type table, est = MLP (all runs advance with truth).
    The three schedules of a sample of DAGs (every 64th and the largest) are
    checked against the oracle given the same integer estimates."""
    import torch
    import oracle
    from types import SimpleNamespace
    from paper_2404_03226_amd import costmodel, inspirit, synth
    t0 = time.time()
    rec = synth.cfg5_records()
    ntr = rec["n_train"]
    x = torch.from_numpy(rec["x"]).cuda()
    lt = torch.from_numpy(np.log(rec["ticks"].astype(np.float64)).astype(np.float32)).cuda()
    mlp = inspirit.Mlp(synth.mlp_init())
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    steps = costmodel.train(mlp, x, lt, ntr, epochs=epochs, log=log)
    ev1.record()
    torch.cuda.synchronize()
    train_ms = ev0.elapsed_time(ev1)
    yv, _ = mlp.predict(x[ntr:])
    val = lt[ntr:].cpu().numpy()
    table = synth.plain_table(rec["types"][:ntr], rec["ticks"][:ntr])
    mse_mlp = float(np.mean((yv.cpu().numpy() - val) ** 2))
    mse_tab = float(np.mean((np.log(table[rec["types"][ntr:]].astype(np.float64)) - val) ** 2))
    del x, lt
    xe = synth.cost_features(5, 7, b.type)
    ticks = synth.cost_truth(5, 7, b.type, xe)
    log(f"cost model: trained {steps} steps in {train_ms / 1e3:.1f}s; eval features ready ({time.time() - t0:.0f}s)")
    xd = torch.from_numpy(xe).cuda()
    _, est_mlp = mlp.predict(xd, want_y=False)  # untimed: allocates the output
    pred_ms = float("inf")
    for _ in range(3):
        ev0.record()
        _, est_mlp = mlp.predict(xd, want_y=False)
        ev1.record()
        torch.cuda.synchronize()
        pred_ms = min(pred_ms, ev0.elapsed_time(ev1))
    del xd
    ms, scheds = costmodel.evaluate(dag, workers, b.type, ticks, est_mlp, table, keep_schedules=True)
    gaps = costmodel.makespan_gaps(ms["true"], ms["plain"], ms["learned"])
    # the sampled oracle check of all three runs
    ests = {"true": ticks, "plain": table[b.type], "learned": est_mlp.cpu().numpy().reshape(-1, 2)}
    big = int(np.argmax([w.n for w in ws]))
    sample = sorted(set(range(0, len(ws), 64)) | {big})
    exact = True
    for k in sample:
        a, z = int(b.task_off[k]), int(b.task_off[k + 1])
        for name, est in ests.items():
            w = SimpleNamespace(n=ws[k].n, row_ptr=ws[k].row_ptr, col=ws[k].col, n_cpu=ws[k].n_cpu,
                                n_gpu=ws[k].n_gpu, dur=np.ascontiguousarray(ticks[a:z]),
                                est=np.ascontiguousarray(est[a:z]))
            r = oracle.schedule(w, variant=oracle.HEAP)
            got = scheds[name]
            exact &= all(np.array_equal(got[f][a:z], r[f]) for f in ("worker", "start", "finish"))
            exact &= int(got["makespan"][k]) == r["makespan"]
    gaps["schedules_bit_exact_sample"] = bool(exact)
    gaps["sample"] = f"{len(sample)} DAGs (every 64th and the largest), each run's schedule against the oracle"
    gaps.update({"val_mse_ln_mlp": mse_mlp, "val_mse_ln_table": mse_tab, "train_steps": steps,
                 "train_s": round(train_ms / 1e3, 2), "predict_ms": round(pred_ms, 2),
                 "predict_tasks_per_s": round(len(b.type) / (pred_ms * 1e-3), 1),
                 "predict_TFLOPs": round(148480 * len(b.type) / (pred_ms * 1e-3) / 1e12, 2),
                 "train_TFLOPs": round(445440 * 1024 * steps / (train_ms * 1e-3) / 1e12, 2)})
    # fractions of MI355X's dense bf16 MFMA peak (2.5 PFLOP/s)
    gaps["predict_frac_bf16_peak"] = round(gaps["predict_TFLOPs"] / BF16_PEAK_TFLOPS, 4)
    gaps["train_frac_bf16_peak"] = round(gaps["train_TFLOPs"] / BF16_PEAK_TFLOPS, 4)
    mlp.free()
    log(f"learned gap: {gaps}")
    return gaps


if __name__ == "__main__":
    main()
