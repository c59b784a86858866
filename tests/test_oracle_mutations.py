"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
the pins catch each one: the pins would not pass a wrong oracle."""
import ctypes as C
import json
import os
import subprocess
from types import SimpleNamespace as NS

import numpy as np
import pytest

import oracle
from paper_2404_03226_amd import synth
from invariants import check_schedule

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
GOLD = os.path.join(os.path.dirname(__file__), "golden")

MUTATIONS = {
    "ie_strict_unit_time": ("if (rem[s] == 1 && tv + tau_of(est, n_gpu, s) <= U) c++;",
                            "if (rem[s] == 1 && tv + tau_of(est, n_gpu, s) < U) c++;"),
    "ie_wrong_remaining": ("if (rem[s] == 1 && tv + tau_of(est, n_gpu, s) <= U) c++;",
                           "if (rem[s] >= 1 && tv + tau_of(est, n_gpu, s) <= U) c++;"),
    "ladder_tie_smaller_u": ("if (score >= bestScore) { bestScore = score; bestU = U; }",
                             "if (score > bestScore) { bestScore = score; bestU = U; }"),
    "ladder_one_rung_short": ("while (((int64_t)1 << J) < 2 * maxtau) J++;",
                              "while (((int64_t)1 << J) < maxtau) J++;"),
    "dmda_tie_highest_worker": ("if (best < 0 || c < bestc) { best = w; bestc = c; bestx = x; }",
                                "if (best < 0 || c <= bestc) { best = w; bestc = c; bestx = x; }"),
    "dmda_ignores_running_task": ("if (run[w] >= 0 && exp_end[w] > t) B = exp_end[w];", ""),
    "dmda_ignores_queue": ("int64_t c = B + qest[w] + est[2 * (int64_t)v + k] + x;",
                           "int64_t c = B + est[2 * (int64_t)v + k] + x;"),
    "tau_cpu_column": ("return est[2 * (int64_t)v + (n_gpu > 0 ? 1 : 0)];", "return est[2 * (int64_t)v];"),
    "ability_order_reversed": ("if (ia_a != ia_b) return ia_a > ia_b;\n        if (ie_a != ie_b) return ie_a > ie_b;\n    } else if (order == 1) {",
                               "if (ia_a != ia_b) return ia_a < ia_b;\n        if (ie_a != ie_b) return ie_a > ie_b;\n    } else if (order == 1) {"),
    "fifo_tie_latest": ("    }\n    return sq_a < sq_b;", "    }\n    return sq_a > sq_b;"),
    "reg_inc_margin_strict": ("if (N >= r->peak - r->dec_step) {", "if (N > r->peak - r->dec_step) {"),
    "reg_slope_flipped": ("if (dt == 0 || dn * r->k_den > r->k_num * dt) r->mode = M_ABILITY;\n            else if (dn * r->k_den < r->k_num * dt) r->mode = M_EFI;",
                          "if (dt == 0 || dn * r->k_den < r->k_num * dt) r->mode = M_ABILITY;\n            else if (dn * r->k_den > r->k_num * dt) r->mode = M_EFI;"),
    "reg_no_decrement_count": ("if (N <= r->peak - r->s_dec * (r->cnt + 1)) r->cnt += 1;", ""),
    "reg_no_window": ("if ((dn < 0 ? -dn : dn) < r->s_inc) return;", ""),
    "reg_starts_efficiency": ("r->mode = M_ABILITY;  /* Section 3", "r->mode = M_EFI;  /* Section 3"),
    "ready_not_sorted": ("qsort(newly, (size_t)n_new, sizeof(int32_t), cmp_i32);", ""),
    "regulate_after_pop": ("int64_t observed = nready;", "int64_t observed = nready - 1;"),
    "rank_no_successor_term": ("(int64_t)n_gpu * est[2 * (int64_t)v + 1] + best;",
                               "(int64_t)n_gpu * est[2 * (int64_t)v + 1];"),
    "rank_gpu_column_dropped": ("(int64_t)n_gpu * est[2 * (int64_t)v + 1] + best;", "best;"),
    "rank_lowest_first": ("if (order == 3 && r_a != r_b) return r_a > r_b;",
                          "if (order == 3 && r_a != r_b) return r_a < r_b;"),
    "rank_tie_latest_push": ("if (order == 3) return sq_a < sq_b;", "if (order == 3) return sq_a > sq_b;"),
    "trans_exclusive_count": ("            members++;\n", "            if (u != v) members++;\n"),
    "trans_shortest_path": ("if (f > EF[s]) EF[s] = f;", "if (EF[s] == 0 || f < EF[s]) EF[s] = f;"),
    "trans_window_strict": ("if (unit_time > 0 && EF[u] <= unit_time) in_u++;",
                            "if (unit_time > 0 && EF[u] < unit_time) in_u++;"),
    "trans_rung_strict": ("if (EF[u] <= ((int64_t)1 << j)) within[", "if (EF[u] < ((int64_t)1 << j)) within["),
    "trans_ladder_short": ("while (((int64_t)1 << J) < cp) J++;", "while (((int64_t)1 << J) < cp / 2) J++;"),
    "trans_ladder_tie_smaller": ("if (score >= bestScore) { bestScore = score; bestJ = j; }",
                                 "if (score > bestScore) { bestScore = score; bestJ = j; }"),
    "trans_source_excluded": ("EF[v] = tau_of(est, n_gpu, v);", "EF[v] = 1;"),
    "data_no_transfer_term": ("int64_t c = B + qest[w] + est[2 * (int64_t)v + k] + x;",
                              "int64_t c = B + qest[w] + est[2 * (int64_t)v + k];"),
    "data_transfer_in_queue": ("            qest[best] += est[2 * (int64_t)v + k];",
                               "            qest[best] += est[2 * (int64_t)v + k] + bestx;"),
    "data_no_wait": ("int64_t s0 = data && arr[v] > t ? arr[v] : t;", "int64_t s0 = t;"),
    "data_locality_ignored": ("const int loc = data && mode == M_EFI_LOC;", "const int loc = 0;"),
    "data_all_host": ("static int node_of(int32_t w, int32_t n_cpu) { return w < n_cpu ? 0 : 1 + (w - n_cpu); }",
                      "static int node_of(int32_t w, int32_t n_cpu) { return w < n_cpu ? 0 : 1; }"),
    "data_home_of_consumer": ("if (home[u] != node) x +=", "if (home[u] == node) x +="),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    d = tmp_path / name
    d.mkdir()
    (d / "o.c").write_text(src.replace(old, new))
    so = d / "lib.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", str(so), str(d / "o.c")])
    return str(so)


def _swap(path):
    saved = oracle._lib
    oracle._lib = None
    real = oracle.build
    oracle.build = lambda force=False: path
    try:
        oracle.lib()
    finally:
        oracle.build = real
    return saved


def pins():
    """The pin suite: returns the names of failed pins."""
    failed = []

    def chk(name, fn):
        try:
            if fn() is False:
                failed.append(name)
        except Exception:
            failed.append(name)

    g1 = json.load(open(os.path.join(GOLD, "w1_attributes.json")))
    chk("w1", lambda: oracle.attributes(g1["n"], g1["row_ptr"], g1["col"], g1["est"], 1)[1].tolist() == g1["ie_auto"]
        and oracle.attributes(g1["n"], g1["row_ptr"], g1["col"], g1["est"], 1)[2] == g1["unit_time_auto"])
    g2 = json.load(open(os.path.join(GOLD, "w2_schedule.json")))
    w2 = NS(n=5, row_ptr=np.array(g2["row_ptr"]), col=np.array(g2["col"]), dur=np.ones((5, 2), np.int32),
            est=np.ones((5, 2), np.int32), n_cpu=2, n_gpu=0)
    for pol in ("fifo", "inspirit"):
        chk("w2" + pol, lambda pol=pol: oracle.schedule(w2, policy=pol)["start"].tolist() == g2[pol]["start"]
            and oracle.schedule(w2, policy=pol)["worker"].tolist() == g2[pol]["worker"])
    chk("w2u", lambda: oracle.schedule(w2)["unit_time"] == g2["unit_time"])
    chk("w1u5", lambda: oracle.attributes(g1["n"], g1["row_ptr"], g1["col"], g1["est"], 1, rem=g1["rem_after_task1"],
                                          unit_time=5)[1].tolist()[2] == g1["ie_after_task1_u5"][2])
    small = json.load(open(os.path.join(GOLD, "w4_w7_small.json")))

    def mk(g):
        dur = np.asarray(g.get("dur", g.get("est")), np.int32)
        est = np.asarray(g.get("est", dur), np.int32)
        return NS(n=g["n"], row_ptr=np.asarray(g["row_ptr"], np.int32), col=np.asarray(g["col"], np.int32),
                  dur=dur, est=est, n_cpu=g.get("n_cpu", 0), n_gpu=g.get("n_gpu", 0))
    for key in ("w4", "w5"):
        g = small[key]
        chk(key, lambda g=g: oracle.schedule(mk(g))["worker"].tolist() == g["worker"]
            and oracle.schedule(mk(g))["start"].tolist() == g["start"])
    g6 = small["w6"]
    chk("w6", lambda: oracle.attributes(g6["n"], g6["row_ptr"], g6["col"], g6["est"], 1)[2] == g6["unit_time"]
        and oracle.attributes(g6["n"], g6["row_ptr"], g6["col"], g6["est"], 1)[1].tolist() == g6["ie"])
    chk("w7", lambda: int(oracle.schedule(mk(small["w7"]))["mode_at_pop"][0]) == small["w7"]["mode_at_pop_first"])
    chk("w2trace", lambda: oracle.schedule(w2, trace=True)["trace"]["nready"].tolist() == g2["inspirit"]["trace_nready"])
    g3 = json.load(open(os.path.join(GOLD, "w3_regulator.json")))
    chk("w3", lambda: oracle.regulate(g3["t"], g3["N"], 4, 10)[0].tolist() == g3["mode"]
        and oracle.regulate(g3["t"], g3["N"], 4, 10)[1].tolist() == g3["cnt"])
    # chain: the fastest kind every time
    n = 10
    rp = np.arange(n + 1, dtype=np.int32).clip(max=n - 1)
    rp[0] = 0
    rp = np.array([0] + [i for i in range(1, n)] + [n - 1], np.int32)
    col = np.arange(1, n, dtype=np.int32)
    dur = synth.Stream(9, 9).randint(np.arange(2 * n).reshape(n, 2), 1, 40).astype(np.int32)
    wc = NS(n=n, row_ptr=rp, col=col, dur=dur, est=dur, n_cpu=2, n_gpu=1)
    chk("chain", lambda: oracle.schedule(wc)["makespan"] == int(dur.min(axis=1).sum()))
    # independent unit tasks
    wi = NS(n=13, row_ptr=np.zeros(14, np.int32), col=np.zeros(0, np.int32), dur=np.ones((13, 2), np.int32),
            est=np.ones((13, 2), np.int32), n_cpu=4, n_gpu=0)
    chk("indep", lambda: oracle.schedule(wi)["makespan"] == 4)
    # HEFT: the single-worker fixture, and the rank-order pop property with
    # ranks recomputed from their definition on mixed machines
    g8 = json.load(open(os.path.join(GOLD, "w8_heft.json")))["w8"]
    w8 = NS(n=g8["n"], row_ptr=np.asarray(g8["row_ptr"], np.int32), col=np.asarray(g8["col"], np.int32),
            dur=np.asarray(g8["dur"], np.int32), est=np.asarray(g8["dur"], np.int32), n_cpu=1, n_gpu=0)
    chk("w8", lambda: oracle.schedule(w8, policy="heft")["start"].tolist() == g8["heft"]["start"])
    for i in range(8):
        w = synth.random_dag(31, i, 12, 0.25, dur_hi=20, n_cpu=1 + i % 2, n_gpu=1, est_equal=(i % 2 == 0))
        chk(f"heft{i}", lambda w=w: _heft_pops_by_rank(w))
    # transitive attributes: the hand-worked fixture at a fixed and at the
    # automatic unit time, and the complete-DAG statement
    g9 = json.load(open(os.path.join(GOLD, "w9_transitive.json")))["w9"]
    chk("w9u7", lambda: oracle.transitive(5, g9["row_ptr"], g9["col"], g9["est"], 1, unit_time=7)[:2][0].tolist()
        == g9["ia_t"] and oracle.transitive(5, g9["row_ptr"], g9["col"], g9["est"], 1, unit_time=7)[1].tolist()
        == g9["ie_t_u7"])
    chk("w9auto", lambda: oracle.transitive(5, g9["row_ptr"], g9["col"], g9["est"], 1)[2] == g9["unit_time_auto"]
        and oracle.transitive(5, g9["row_ptr"], g9["col"], g9["est"], 1)[1].tolist() == g9["ie_t_auto"])
    for key in ("w10_tie", "w10_top"):
        gk = json.load(open(os.path.join(GOLD, "w9_transitive.json")))[key]
        chk(key, lambda gk=gk: oracle.transitive(gk["n"], gk["row_ptr"], gk["col"], gk["est"], 1)[2]
            == gk["unit_time_auto"])
    Nc = 7
    rpc = np.array([0] + [sum(Nc - 1 - i for i in range(k + 1)) for k in range(Nc)], np.int32)
    colc = np.array([j for i in range(Nc) for j in range(i + 1, Nc)], np.int32)
    chk("complete", lambda: int(oracle.transitive(Nc, rpc, colc, np.ones((Nc, 2), np.int32), 1)[0][0]) == Nc)
    for i in range(6):
        w = synth.random_dag(58, i, 14, 0.2, dur_hi=20, n_cpu=1, n_gpu=1, est_equal=False)
        chk(f"tladder{i}", lambda w=w: _transitive_ladder_ok(w))
    # data model: the hand-worked fixtures W11 and W12
    gd = json.load(open(os.path.join(GOLD, "w11_data.json")))
    for key, pol, fx, bw in (("w11", "locality", "locality", 1024), ("w11", "efi", "efi", 1024),
                             ("w12", "fifo", "fifo", 1024)):
        g = gd[key]
        d = np.asarray(g["dur"], np.int32)
        wd = NS(n=g["n"], row_ptr=np.asarray(g["row_ptr"], np.int32), col=np.asarray(g["col"], np.int32), dur=d,
                est=d, n_cpu=g["n_cpu"], n_gpu=g["n_gpu"], data_kib=np.asarray(g["data_kib"], np.int32))
        chk(f"{key}{pol}", lambda wd=wd, pol=pol, g=g, fx=fx, bw=bw: oracle.schedule(
            wd, policy=pol, data_bw=bw, unit_time=g.get("unit_time", 0))["start"].tolist() == g[fx]["start"])
    # two GPUs: an item moves between GPU memories as well
    d2 = np.array([[50, 2], [50, 2], [50, 3]], np.int32)
    w2g = NS(n=3, row_ptr=np.array([0, 0, 1, 1], np.int32), col=np.array([2], np.int32), dur=d2, est=d2, n_cpu=1,
             n_gpu=2, data_kib=np.array([0, 9, 0], np.int32))
    # t=0: task 0 -> GPU worker 1, task 1 -> GPU worker 2 (worker 1 now 2 ticks long); t=2: task 2 reads
    # item 1, which lives on worker 2's memory: 2+3+9 on worker 1 against 2+3 on worker 2 (a tie, won by
    # worker 1, if both GPUs shared one memory)
    chk("twogpu", lambda: oracle.schedule(w2g, policy="fifo", data_bw=1024)["worker"].tolist() == [1, 2, 2])
    # invariants and brute force on small random DAGs
    for i in range(6):
        w = synth.random_dag(77, i, 7, 0.3, dur_hi=6, n_cpu=1, n_gpu=1)
        def inv(w=w):
            r = oracle.schedule(w)
            check_schedule(w, r["worker"], r["start"], r["finish"], r["makespan"])
            return r["makespan"] >= oracle.brute_opt(w)
        chk(f"inv{i}", inv)
    return failed


def _transitive_ladder_ok(w):
    # the automatic U is the best-scoring rung of 2^0 .. 2^J (2^J >= longest
    # path), the larger on a tie, scored with the oracle's fixed-U attributes
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    _, _, U, cp = oracle.transitive(w.n, rp, col, w.est, 1)
    J = 0
    while 2 ** J < cp:
        J += 1
    scores = {}
    for j in range(J + 1):
        ia, ie, _, _ = oracle.transitive(w.n, rp, col, w.est, 1, unit_time=2 ** j)
        scores[2 ** j] = int(((ie > 0) & (ie < ia)).sum())
    best = max(scores.values())
    return U == max(u for u, s in scores.items() if s == best)


def _heft_pops_by_rank(w):
    rp, col = oracle.canon(w.n, w.row_ptr, w.col)
    est = np.asarray(w.est, np.int64).reshape(w.n, 2)
    R = [0] * w.n
    for v in range(w.n - 1, -1, -1):  # random_dag edges run from lower to higher ids
        R[v] = int(w.n_cpu * est[v, 0] + w.n_gpu * est[v, 1]) + max((R[s] for s in col[rp[v]:rp[v + 1]]), default=0)
    r = oracle.schedule(w, policy="heft")
    start, finish, worker = r["start"], r["finish"], r["worker"]
    ready = np.zeros(w.n, np.int64)
    for v in range(w.n):
        for s in col[rp[v]:rp[v + 1]]:
            ready[s] = max(ready[s], finish[v])
    for v in range(w.n):
        waiting = [u for u in range(w.n) if worker[u] == worker[v] and ready[u] <= start[v] <= start[u]]
        if max(R[u] for u in waiting) != R[v] or any(R[u] == R[v] and ready[u] < ready[v] for u in waiting):
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MUTATIONS[name]
    path = _build(tmp_path, name, old, new)
    saved = _swap(path)
    try:
        failed = pins()
    finally:
        oracle._lib = saved
    assert failed, f"no pin caught the planted mistake '{name}'"


def test_unmutated_oracle_passes_every_pin():
    assert pins() == []
