"""Seeded synthetic workloads (task DAGs, duration tables, features).

This module only draws inputs; it holds none of the scheduling method's
arithmetic, and both the CPU oracle and the HIP path consume its arrays.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: value i of a stream whose start state is ``s`` is
``mix(s + (i + 1) * 0x9E3779B97F4A7C15)`` with the published SplitMix64
finaliser ``mix``.  A stream's start state is derived from ``(seed, stream)``
by one more SplitMix64 step, so any DAG of a batch can be regenerated on its
own.

The paper evaluates on layered synthetic DAGs produced by an automatic
generator (Section 4.5, Section 5.2) and on tiled Cholesky (Section 5.3);
neither the generator nor its data set is available, so these recipes stand
in for them with the shapes the evaluation describes.  All durations are
integer ticks.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_U30, _U27, _U31, _U11, _U32 = (np.uint64(k) for k in (30, 27, 31, 11, 32))


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64).copy()
    z ^= z >> _U30
    z *= _M1
    z ^= z >> _U27
    z *= _M2
    z ^= z >> _U31
    return z


class Stream:
    """One counter-based SplitMix64 stream identified by (seed, stream)."""

    def __init__(self, seed: int, stream: int = 0):
        key = np.uint64(((seed & 0xFFFFFFFF) << 32) | (stream & 0xFFFFFFFF))
        with np.errstate(over="ignore"):
            self.state = _mix(np.array([key + _GAMMA], dtype=np.uint64))[0]

    def u64(self, idx) -> np.ndarray:
        idx = np.asarray(idx, dtype=np.uint64)
        with np.errstate(over="ignore"):
            return _mix(self.state + (idx + np.uint64(1)) * _GAMMA)

    def uniform(self, idx) -> np.ndarray:
        """Doubles in [0, 1) from the top 53 bits."""
        return (self.u64(idx) >> _U11).astype(np.float64) * (1.0 / 9007199254740992.0)

    def randint(self, idx, lo, hi) -> np.ndarray:
        """Integers in [lo, hi] (inclusive) by multiply-shift of the top 32 bits."""
        lo = np.asarray(lo, dtype=np.int64)
        span = (np.asarray(hi, dtype=np.int64) - lo + 1).astype(np.uint64)
        top = self.u64(idx) >> _U32
        return lo + ((top * span) >> _U32).astype(np.int64)


# Sub-stream tags inside one DAG's stream space.
_S_DEG, _S_TGT, _S_TYPE, _S_TAB, _S_JIT, _S_FEAT = range(6)


def _sub(seed: int, stream: int, tag: int) -> Stream:
    return Stream(seed, stream * 8 + tag)


@dataclass
class Workload:
    """One DAG plus the machine it is scheduled on.

    ``row_ptr``/``col`` is a CSR of successor lists (local ids), ``type`` the
    task kind, ``dur``/``est`` are ``[n, 2]`` integer ticks with column 0 for
    CPU workers and column 1 for GPU workers.
    """
    name: str
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    type: np.ndarray
    dur: np.ndarray
    est: np.ndarray
    n_cpu: int
    n_gpu: int
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])


def _distinct_targets(st: Stream, lo: np.ndarray, hi: np.ndarray, deg: np.ndarray) -> tuple:
    """For every row r draw ``deg[r]`` distinct ids uniformly from [lo[r], hi[r]).

    Candidate k of row r is ``lo + floor(u * (hi - lo))`` with ``u`` the
    stream value at counter ``(r << 24) + k``; candidates are taken in order
    and repeats are skipped until the row has ``deg[r]`` distinct targets
    (``deg`` is first capped at ``hi - lo``).  Returns (row_ptr, col) with
    each row's targets in draw order.
    """
    nrow = deg.shape[0]
    span = np.maximum(hi - lo, 0).astype(np.int64)
    deg = np.minimum(deg.astype(np.int64), span)

    def cand(rows, k):
        u = st.uniform((rows.astype(np.uint64) << np.uint64(24)) + k.astype(np.uint64))
        return np.minimum(lo[rows] + np.floor(u * span[rows]).astype(np.int64), hi[rows] - 1)

    # Vectorised first round: deg + deg//4 + 4 candidates per row.
    cnt = np.where(deg > 0, deg + deg // 4 + 4, 0)
    first = np.cumsum(cnt) - cnt
    rows = np.repeat(np.arange(nrow, dtype=np.int64), cnt)
    k = np.arange(rows.size, dtype=np.int64) - np.repeat(first, cnt)
    vals = cand(rows, k)
    # Sort by (row, value, draw index) through one packed key; the first
    # draw of every repeated value survives.
    assert nrow < (1 << 23) and int(hi.max(initial=0)) < (1 << 26) and int(cnt.max(initial=0)) < (1 << 14)
    key = np.sort((rows << 40) | (vals << 14) | k)
    srt = first[key >> 40] + (key & 0x3FFF)
    rv = key >> 14
    dup = np.zeros(rows.size, dtype=bool)
    dup[srt[1:]] = rv[1:] == rv[:-1]
    keep = ~dup
    csum = np.cumsum(keep)
    before = np.where(first > 0, csum[np.maximum(first - 1, 0)], 0)
    rank = csum - np.repeat(before, cnt)          # 1-based rank among survivors
    keep &= rank <= np.repeat(deg, cnt)
    got = np.bincount(rows[keep], minlength=nrow)
    lists = None
    short = np.nonzero(got < deg)[0]
    if short.size:
        # Rare rows: continue the same candidate sequence one draw at a time.
        lists = {}
        for r in short.tolist():
            a, b = int(first[r]), int(first[r] + cnt[r])
            taken = vals[a:b][keep[a:b]].tolist()
            seen = set(taken)
            kk = int(cnt[r])
            while len(taken) < deg[r]:
                x = int(cand(np.array([r]), np.array([kk]))[0])
                kk += 1
                if x not in seen:
                    seen.add(x)
                    taken.append(x)
            lists[r] = taken
            keep[a:b] = False
    col_rows, col_vals = rows[keep], vals[keep]
    if lists:
        extra_r = np.concatenate([np.full(len(v), r) for r, v in lists.items()])
        extra_v = np.concatenate([np.array(v, dtype=np.int64) for v in lists.values()])
        col_rows = np.concatenate([col_rows, extra_r])
        col_vals = np.concatenate([col_vals, extra_v])
    order = np.argsort(col_rows, kind="stable")
    row_ptr = np.zeros(nrow + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    return row_ptr.astype(np.int32), col_vals[order].astype(np.int32)


def layered_dag(seed: int, stream: int, n: int, n_layers: int, deg_lo: int, deg_hi: int) -> tuple:
    """Layered DAG: ids in layer-major order, every task except those of the
    last layer draws U{deg_lo..deg_hi} distinct targets uniformly from all
    tasks in later layers."""
    sizes = np.full(n_layers, n // n_layers, dtype=np.int64)
    sizes[: n % n_layers] += 1
    bounds = np.zeros(n_layers + 1, dtype=np.int64)
    np.cumsum(sizes, out=bounds[1:])
    layer = np.repeat(np.arange(n_layers), sizes)
    lo = bounds[np.minimum(layer + 1, n_layers)]
    hi = np.full(n, n, dtype=np.int64)
    deg = _sub(seed, stream, _S_DEG).randint(np.arange(n), deg_lo, deg_hi)
    deg[layer == n_layers - 1] = 0
    return _distinct_targets(_sub(seed, stream, _S_TGT), lo, hi, deg)


def _table(seed: int, stream: int, n_types: int) -> np.ndarray:
    st = _sub(seed, stream, _S_TAB)
    cpu = st.randint(np.arange(n_types) * 2, 50, 500)
    gpu = st.randint(np.arange(n_types) * 2 + 1, 10, 120)
    return np.stack([cpu, gpu], axis=1).astype(np.int32)


def cfg1(seed: int = 1) -> Workload:
    """Single layered DAG: 1,000 tasks in 20 layers of 50, 1-6 targets per
    task, 3 types, 8 CPU + 2 GPU workers, ``dur = est = table[type]``."""
    n = 1000
    row_ptr, col = layered_dag(seed, 0, n, 20, 1, 6)
    ty = _sub(seed, 0, _S_TYPE).randint(np.arange(n), 0, 2).astype(np.int32)
    tab = _table(seed, 0, 3)
    d = tab[ty]
    return Workload("layered-1k", n, row_ptr, col, ty, d.copy(), d.copy(), 8, 2, {"table": tab})


# ---------------------------------------------------------------- Cholesky

CHOL_BASE = np.array([[120, 60], [300, 30], [300, 20], [560, 25]], dtype=np.int32)
"""Per-kernel ticks (rows POTRF, TRSM, SYRK, GEMM; columns CPU, GPU)."""


def cholesky_dag(nb: int) -> tuple:
    """Right-looking tiled Cholesky (lower) in sequential-task-flow order.

    Step k submits POTRF(k), then TRSM(k, i) for i > k, then for each i > k
    SYRK(k, i) followed by GEMM(k, i, j) for k < j < i.  Edges follow the
    read-after-write hazards on tiles: POTRF(k) <- SYRK(k-1, k);
    TRSM(k, i) <- POTRF(k), GEMM(k-1, i, k); SYRK(k, i) <- TRSM(k, i),
    SYRK(k-1, i); GEMM(k, i, j) <- TRSM(k, i), TRSM(k, j), GEMM(k-1, i, j).
    Types: 0 POTRF, 1 TRSM, 2 SYRK, 3 GEMM.
    """
    ids = {}
    types = []

    def add(key, ty):
        ids[key] = len(types)
        types.append(ty)

    for k in range(nb):
        add(("P", k), 0)
        for i in range(k + 1, nb):
            add(("T", k, i), 1)
        for i in range(k + 1, nb):
            add(("S", k, i), 2)
            for j in range(k + 1, i):
                add(("G", k, i, j), 3)
    n = len(types)
    succ = [[] for _ in range(n)]

    def edge(a, b):
        succ[ids[a]].append(ids[b])

    for k in range(nb):
        if k > 0:
            edge(("S", k - 1, k), ("P", k))
        for i in range(k + 1, nb):
            edge(("P", k), ("T", k, i))
            if k > 0:
                edge(("G", k - 1, i, k), ("T", k, i))
        for i in range(k + 1, nb):
            edge(("T", k, i), ("S", k, i))
            if k > 0:
                edge(("S", k - 1, i), ("S", k, i))
            for j in range(k + 1, i):
                edge(("T", k, i), ("G", k, i, j))
                edge(("T", k, j), ("G", k, i, j))
                if k > 0:
                    edge(("G", k - 1, i, j), ("G", k, i, j))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([len(s) for s in succ], out=row_ptr[1:])
    col = np.array([x for s in succ for x in s], dtype=np.int32)
    return row_ptr.astype(np.int32), col, np.array(types, dtype=np.int32)


def cfg2(seed: int = 2, nb: int = 40) -> Workload:
    """Tiled Cholesky, ``nb`` x ``nb`` tiles; ``est = CHOL_BASE[type]`` and
    ``dur = est + U{-floor(est/10)..floor(est/10)}`` per task and kind;
    24 CPU + 4 GPU workers."""
    row_ptr, col, ty = cholesky_dag(nb)
    n = ty.shape[0]
    est = CHOL_BASE[ty].astype(np.int64)
    jit = est // 10
    st = _sub(seed, 0, _S_JIT)
    idx = np.arange(2 * n).reshape(n, 2)
    dur = est + st.randint(idx, -jit, jit)
    return Workload(f"cholesky-{nb}", n, row_ptr, col, ty, dur.astype(np.int32),
                    est.astype(np.int32), 24, 4, {"nb": nb})


LU_BASE = np.array([[240, 90], [300, 30], [560, 25]], dtype=np.int32)
"""Per-kernel ticks (rows GETRF, TRSM, GEMM; columns CPU, GPU).  The paper
prints no kernel times: a proposal in the proportions of CHOL_BASE (GETRF
about twice POTRF's flops, TRSM and GEMM as in Cholesky)."""


def lu_dag(nb: int) -> tuple:
    """Right-looking tiled LU without pivoting in sequential-task-flow order.

    Step k submits GETRF(k), then the row-panel TRSM(k, k, j) for j > k, then
    the column-panel TRSM(k, i, k) for i > k, then GEMM(k, i, j) for i, j > k
    (row-major).  Edges follow the read-after-write hazards on tiles:
    GETRF(k) <- GEMM(k-1, k, k); TRSM(k, k, j) <- GETRF(k), GEMM(k-1, k, j);
    TRSM(k, i, k) <- GETRF(k), GEMM(k-1, i, k);
    GEMM(k, i, j) <- TRSM(k, i, k), TRSM(k, k, j), GEMM(k-1, i, j).
    Types: 0 GETRF, 1 TRSM, 2 GEMM.  nb(nb+1)(2nb+1)/6 tasks.
    """
    ids = {}
    types = []

    def add(key, ty):
        ids[key] = len(types)
        types.append(ty)

    for k in range(nb):
        add(("F", k), 0)
        for j in range(k + 1, nb):
            add(("T", k, k, j), 1)
        for i in range(k + 1, nb):
            add(("T", k, i, k), 1)
        for i in range(k + 1, nb):
            for j in range(k + 1, nb):
                add(("G", k, i, j), 2)
    n = len(types)
    succ = [[] for _ in range(n)]

    def edge(a, b):
        succ[ids[a]].append(ids[b])

    for k in range(nb):
        if k > 0:
            edge(("G", k - 1, k, k), ("F", k))
        for j in range(k + 1, nb):
            edge(("F", k), ("T", k, k, j))
            if k > 0:
                edge(("G", k - 1, k, j), ("T", k, k, j))
        for i in range(k + 1, nb):
            edge(("F", k), ("T", k, i, k))
            if k > 0:
                edge(("G", k - 1, i, k), ("T", k, i, k))
        for i in range(k + 1, nb):
            for j in range(k + 1, nb):
                edge(("T", k, i, k), ("G", k, i, j))
                edge(("T", k, k, j), ("G", k, i, j))
                if k > 0:
                    edge(("G", k - 1, i, j), ("G", k, i, j))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([len(x) for x in succ], out=row_ptr[1:])
    col = np.array([x for row in succ for x in row], dtype=np.int32)
    return row_ptr.astype(np.int32), col, np.array(types, dtype=np.int32)


def lu_workload(seed: int = 6, nb: int = 40) -> Workload:
    """Tiled LU, ``nb`` x ``nb`` tiles; ``est = LU_BASE[type]`` and ``dur = est
    + U{-floor(est/10)..floor(est/10)}`` per task and kind; 24 CPU + 4 GPU."""
    row_ptr, col, ty = lu_dag(nb)
    n = ty.shape[0]
    est = LU_BASE[ty].astype(np.int64)
    jit = est // 10
    st = _sub(seed, 0, _S_JIT)
    idx = np.arange(2 * n).reshape(n, 2)
    dur = est + st.randint(idx, -jit, jit)
    return Workload(f"lu-{nb}", n, row_ptr, col, ty, dur.astype(np.int32), est.astype(np.int32), 24, 4, {"nb": nb})


# ------------------------------------------------------------------ batch

def cfg3_sizes(seed: int = 3, n_dags: int = 4096) -> np.ndarray:
    """DAG sizes, log-uniform over [200, 20000]: floor(exp(ln 200 + u ln 100))."""
    u = Stream(seed, 0xFFFFFF).uniform(np.arange(n_dags))
    return np.floor(np.exp(math.log(200.0) + u * math.log(100.0))).astype(np.int64)


def cfg3_dag(seed: int, b: int, n: int) -> Workload:
    """DAG ``b`` of the batch: max(2, round(20 sqrt(n/1000))) layers, 2-8
    distinct later-layer targets per task, 4 types, per-DAG table with CPU
    U{50..500} and GPU U{10..120} ticks, ``dur = est``, 16 CPU + 4 GPU."""
    n_layers = max(2, int(round(20.0 * math.sqrt(n / 1000.0))))
    row_ptr, col = layered_dag(seed, b + 1, n, n_layers, 2, 8)
    ty = _sub(seed, b + 1, _S_TYPE).randint(np.arange(n), 0, 3).astype(np.int32)
    tab = _table(seed, b + 1, 4)
    d = tab[ty]
    return Workload(f"batch-{b}", n, row_ptr, col, ty, d.copy(), d.copy(), 16, 4,
                    {"table": tab, "layers": n_layers})


def cfg3(seed: int = 3, n_dags: int = 4096, select=None) -> list:
    """The batch (or the DAGs listed in ``select``)."""
    sizes = cfg3_sizes(seed, n_dags)
    idx = range(n_dags) if select is None else select
    return [cfg3_dag(seed, int(b), int(sizes[b])) for b in idx]


# ------------------------------------------------------------------ large

def powerlaw_degrees(st: Stream, n: int, alpha: float, dmax: int) -> np.ndarray:
    d = np.arange(1, dmax + 1, dtype=np.float64)
    cdf = np.cumsum(d ** -alpha)
    cdf /= cdf[-1]
    u = st.uniform(np.arange(n))
    return np.minimum(np.searchsorted(cdf, u, side="right") + 1, dmax).astype(np.int64)


def cfg4(seed: int = 4, n: int = 2_000_000) -> Workload:
    """One large DAG: out-degree pmf proportional to d^-2.1 on [1, 4180]
    (mean 4.000), capped at n-1-v, targets distinct and uniform over the
    later ids; 4 types with a U{50..500}/U{10..120} table; 64 CPU + 8 GPU."""
    deg = powerlaw_degrees(_sub(seed, 0, _S_DEG), n, 2.1, 4180)
    v = np.arange(n, dtype=np.int64)
    row_ptr, col = _distinct_targets(_sub(seed, 0, _S_TGT), v + 1,
                                     np.full(n, n, dtype=np.int64), deg)
    ty = _sub(seed, 0, _S_TYPE).randint(np.arange(n), 0, 3).astype(np.int32)
    tab = _table(seed, 0, 4)
    d = tab[ty]
    return Workload(f"powerlaw-{n}", n, row_ptr, col, ty, d.copy(), d.copy(), 64, 8, {"table": tab})


def random_dag(seed: int, stream: int, n: int, p_edge: float, n_types: int = 3,
               dur_lo: int = 1, dur_hi: int = 9, n_cpu: int = 2, n_gpu: int = 1,
               est_equal: bool = True) -> Workload:
    """Small Erdos-Renyi style DAG for sweeps: edge v->s (v < s) with
    probability ``p_edge``; per-task random durations."""
    st = _sub(seed, stream, _S_TGT)
    iu, ju = np.triu_indices(n, 1)
    keep = st.uniform(np.arange(iu.size)) < p_edge
    src, dst = iu[keep], ju[keep]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    col = dst[np.argsort(src, kind="stable")].astype(np.int32)
    ty = _sub(seed, stream, _S_TYPE).randint(np.arange(n), 0, n_types - 1).astype(np.int32)
    sd = _sub(seed, stream, _S_JIT)
    dur = sd.randint(np.arange(2 * n).reshape(n, 2), dur_lo, dur_hi).astype(np.int32)
    if est_equal:
        est = dur.copy()
    else:
        est = sd.randint(np.arange(2 * n, 4 * n).reshape(n, 2), dur_lo, dur_hi).astype(np.int32)
    return Workload(f"random-{stream}", n, row_ptr.astype(np.int32), col, ty, dur, est, n_cpu, n_gpu)


# ------------------------------------------------------------ concatenation

@dataclass
class Batch:
    """B DAGs concatenated: ``task_off``/``edge_off`` are int64 [B+1];
    ``row_ptr`` holds each DAG's local [n_b+1] row pointer back to back;
    ``col`` holds local successor ids; ``dur``/``est`` are [sum n_b, 2]."""
    task_off: np.ndarray
    edge_off: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    type: np.ndarray
    dur: np.ndarray
    est: np.ndarray
    n_cpu: np.ndarray
    n_gpu: np.ndarray

    @property
    def n_dags(self) -> int:
        return int(self.task_off.shape[0] - 1)


def concat(ws: list) -> Batch:
    ns = np.array([w.n for w in ws], dtype=np.int64)
    ms = np.array([w.m for w in ws], dtype=np.int64)
    task_off = np.zeros(len(ws) + 1, dtype=np.int64)
    edge_off = np.zeros(len(ws) + 1, dtype=np.int64)
    np.cumsum(ns, out=task_off[1:])
    np.cumsum(ms, out=edge_off[1:])
    return Batch(task_off, edge_off,
                 np.concatenate([w.row_ptr for w in ws]).astype(np.int32),
                 np.concatenate([w.col for w in ws]).astype(np.int32),
                 np.concatenate([w.type for w in ws]).astype(np.int32),
                 np.concatenate([w.dur for w in ws]).astype(np.int32),
                 np.concatenate([w.est for w in ws]).astype(np.int32),
                 np.array([w.n_cpu for w in ws], dtype=np.int32),
                 np.array([w.n_gpu for w in ws], dtype=np.int32))


# ------------------------------------------------------- learned cost model

N_FEAT = 32
MLP_SHAPES = ((32, 256), (256,), (256, 256), (256,), (256, 2), (2,))
"""Parameter tensors in packed order: W1, b1, W2, b2, W3, b3 (74,754 floats)."""


def _normal(st: Stream, idx) -> np.ndarray:
    """Standard normals by the Box-Muller transform of two stream values."""
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = 1.0 - st.uniform(idx * np.uint64(2))
    u2 = st.uniform(idx * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def cost_coeffs(seed: int = 5) -> tuple:
    """a_k, b_k ~ N(0, 1/28) for k = CPU, GPU: shape [2, 28] each."""
    st = _sub(seed, 1000, _S_FEAT)
    a = _normal(st, np.arange(56)).reshape(2, 28) / math.sqrt(28.0)
    b = _normal(st, np.arange(56, 112)).reshape(2, 28) / math.sqrt(28.0)
    return a, b


def cost_features(seed: int, stream: int, types: np.ndarray) -> np.ndarray:
    """x in R^32: one-hot of the type (4 dims) and 28 values from U[0, 1)
    (value j of task i at counter 28 i + j; chunks are filled in parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    n = types.shape[0]
    x = np.zeros((n, N_FEAT), dtype=np.float32)
    x[np.arange(n), types] = 1.0
    st = _sub(seed, stream, _S_FEAT)
    step = 1 << 18

    def fill(r0):
        r1 = min(n, r0 + step)
        x[r0:r1, 4:] = st.uniform(np.arange(28 * r0, 28 * r1, dtype=np.uint64)).reshape(r1 - r0, 28)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(0, n, step)))
    return x


def cost_truth(seed: int, stream: int, types: np.ndarray, x: np.ndarray) -> np.ndarray:
    """True ticks [n, 2]: ln d_k = ln base[type][k] + 0.8 tanh(a_k . x[4:] - sum(a_k)/2)
    + 0.2 sin(2 pi b_k . x[4:]) + 0.2 z, z ~ N(0, 1); rounded half-to-even and
    clamped to [1, 2^20].  base is the Cholesky per-kernel table."""
    a, b = cost_coeffs(seed)
    n = types.shape[0]
    xr = x[:, 4:].astype(np.float64)
    z = _normal(_sub(seed, stream, _S_JIT), np.arange(2 * n)).reshape(n, 2)
    lnd = (np.log(CHOL_BASE[types].astype(np.float64)) + 0.8 * np.tanh(xr @ a.T - 0.5 * a.sum(axis=1))
           + 0.2 * np.sin(2.0 * np.pi * (xr @ b.T)) + 0.2 * z)
    return np.clip(np.rint(np.exp(lnd)), 1, 1 << 20).astype(np.int32)


def cfg5_records(seed: int = 5, n: int = 1_000_000):
    """Training records from Cholesky-style task mixes (40 x 40 tiles, repeated
    DAG after DAG): features, types and true ticks; first 90% train, rest
    validation."""
    _, _, ty = cholesky_dag(40)
    types = np.tile(ty, -(-n // ty.size))[:n].astype(np.int32)
    x = cost_features(seed, 0, types)
    ticks = cost_truth(seed, 0, types, x)
    cut = (9 * n) // 10
    return {"x": x, "types": types, "ticks": ticks, "n_train": cut}


def plain_table(types: np.ndarray, ticks: np.ndarray, n_types: int = 4) -> np.ndarray:
    """Per-(type, kind) integer mean of observed ticks (the table fallback)."""
    tab = np.ones((n_types, 2), dtype=np.int32)
    for t in range(n_types):
        sel = types == t
        if sel.any():
            tab[t] = np.maximum(1, np.rint(ticks[sel].mean(axis=0))).astype(np.int32)
    return tab


def mlp_init(seed: int = 5) -> list:
    """He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases (fp32)."""
    st = _sub(seed, 2000, _S_FEAT)
    out, off = [], 0
    for shp in MLP_SHAPES:
        cnt = int(np.prod(shp))
        if len(shp) == 2:
            lim = math.sqrt(6.0 / shp[0])
            w = (st.uniform(np.arange(off, off + cnt)) * 2.0 - 1.0) * lim
        else:
            w = np.zeros(cnt)
        out.append(w.reshape(shp).astype(np.float32))
        off += cnt
    return out


def cfg5_eval(seed: int = 5, n_dags: int = 4096):
    """Evaluation workload: the layered batch's DAG shapes with their types
    read as the four Cholesky kernels; per-task features and true ticks."""
    ws = cfg3(seed=3, n_dags=n_dags)
    b = concat(ws)
    x = cost_features(seed, 7, b.type)
    ticks = cost_truth(seed, 7, b.type, x)
    return ws, b, x, ticks
