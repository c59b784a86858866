"""CPU oracle for the INSPIRIT scheduling hot path -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It wraps ``oracle.c`` (plain C, built with gcc
into ``liboracle.so``) through ctypes and never touches the HIP library.

Parity status of each function (what pins it, besides agreement with the
pure-Python twin in ``pyref.py``):
  attributes  -- pinned: IA figure and complete-DAG statement (Section 4.3),
                 IE limits in U (Section 4.2), brute force on tiny DAGs,
                 hand-worked example W1.
  auto U      -- pinned only by the hand-worked example W1 and by brute force
                 of the ladder's score; the paper gives no selection rule, so
                 against the paper itself its parity is unpinned.
  regulator   -- pinned by the 12-step hand-worked table W3 derived from the
                 Section 4.4 pseudocode; its default parameter values are
                 parity unpinned (the paper prints none).
  schedule    -- pinned by closed forms (chains, independent unit tasks),
                 schedule invariants, brute-force optimal makespans on DAGs of
                 at most 8 tasks, and the Fig. 1 analogue W2.
  heft        -- pinned by the hand-worked fixture W8, the rank-order pop
                 property with ranks recomputed from their definition, and
                 planted mistakes.
  transitive  -- pinned by the complete-DAG statement (Section 4.3: the
                 source scores every task), the U limits of Section 4.2,
                 chain and out-tree closed forms, path enumeration and a
                 reachability-matrix closure on small DAGs, the hand-worked
                 fixture W9, and planted mistakes.  Its unit-time ladder, like
                 the direct one, is pinned only by brute force of the score.
  data model  -- pinned by the hand-worked fixtures W11 (transfer term,
                 arrival wait, locality rule) and W12 (transfers overlap the
                 queue and are not shared), reduction to the plain model when
                 no transfer can cost anything, a start-time bound recomputed
                 from the inputs' homes, and planted mistakes.  The model
                 itself is a reading (the paper gives no formulas), so its
                 parity against the paper is partial.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
# INSP_ORACLE_LIB points the module at another build of oracle.c (the
# sanitizer test's); build() always builds the default one
_LIB = os.environ.get("INSP_ORACLE_LIB") or _DEFAULT_LIB

OK, E_INVAL, E_CYCLE, E_RANGE, E_NOMEM, E_HANG = 0, 1, 2, 3, 4, 6
POLICY = {"inspirit": 0, "fifo": 1, "ability": 2, "efi": 3, "heft": 4, "locality": 5}
MODE_ABILITY, MODE_EFI, MODE_EFI_LOC, MODE_FIFO = 0, 1, 2, 3
PLAIN, HEAP = 0, 1


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, pthreads)."""
    lib = _DEFAULT_LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, lib)
    return lib


ATTR_MODE = {"direct": 0, "transitive": 1}


class Params(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("policy", "unit_time", "s_inc", "s_dec", "dec_step", "c",
                                         "k_num", "k_den", "max_events", "attr_mode", "data_bw")] + \
               [("data_kib", C.c_void_p)]


def params(policy="inspirit", unit_time=0, s_inc=-1, s_dec=-1, dec_step=-1, c=-1, k_num=-1, k_den=-1,
           max_events=0, attr_mode="direct", data_bw=0, data_kib=None) -> Params:
    """data_bw > 0 turns the data model on; data_kib (int32 numpy array, one
    entry per task, kept alive by the caller) gives each task's output KiB."""
    pol = POLICY[policy] if isinstance(policy, str) else int(policy)
    am = ATTR_MODE[attr_mode] if isinstance(attr_mode, str) else int(attr_mode)
    return Params(pol, unit_time, s_inc, s_dec, dec_step, c, k_num, k_den, max_events, am, data_bw,
                  None if data_kib is None else data_kib.ctypes.data)


TRACE_DTYPE = np.dtype([("t", "<i8"), ("nready", "<i4"), ("mode", "<i4"), ("cnt", "<i4"), ("peak", "<i4"),
                        ("pushed", "<i4"), ("popped", "<i4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build() if _LIB == _DEFAULT_LIB else _LIB)
        P = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        _lib.orc_canon.argtypes = [i32, P, P, P, P]
        _lib.orc_attributes.argtypes = [i32, P, P, P, i32, P, i32, P, P, P]
        _lib.orc_transitive.argtypes = [i32, P, P, P, i32, i32, P, P, P, P]
        _lib.orc_regulate_seq.argtypes = [i32, P, P, C.POINTER(Params), i32, i64, P, P, P]
        _lib.orc_schedule.argtypes = [i32, P, P, i32, i32, P, P, C.POINTER(Params), i32, P, P, P, P, P, P, P,
                                      i32, P, P]
        _lib.orc_schedule_batch.argtypes = [i32, P, P, P, P, P, P, P, P, C.POINTER(Params), i32, i32, P, P, P,
                                            P, P, P, P]
        _lib.orc_brute_opt.argtypes = [i32, P, P, i32, i32, P, P]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def canon(n, row_ptr, col):
    row_ptr, col = _i32(row_ptr), _i32(col)
    rp = np.zeros(n + 1, np.int32)
    co = np.zeros(max(int(row_ptr[n]) if n >= 0 else 0, 1), np.int32)
    rc = lib().orc_canon(n, _p(row_ptr), _p(col), _p(rp), _p(co))
    if rc:
        raise OracleError(rc, "canon")
    return rp, co[: rp[n]].copy()


def attributes(n, row_ptr, col, est, n_gpu, rem=None, unit_time=0):
    """(ia, ie, U_used) on a canonical CSR."""
    row_ptr, col, est = _i32(row_ptr), _i32(col), _i32(est).reshape(-1)
    ia = np.zeros(max(n, 1), np.int32)
    ie = np.zeros(max(n, 1), np.int32)
    U = np.zeros(1, np.int32)
    rem = None if rem is None else _i32(rem)
    rc = lib().orc_attributes(n, _p(row_ptr), _p(col), _p(est), n_gpu, _p(rem), unit_time, _p(ia), _p(ie), _p(U))
    if rc:
        raise OracleError(rc, "attributes")
    return ia[:n], ie[:n], int(U[0])


def transitive(n, row_ptr, col, est, n_gpu, unit_time=0):
    """Transitive attributes on a canonical CSR: (ia_t, ie_t, U_used, longest
    path).  See orc_transitive."""
    row_ptr, col, est = _i32(row_ptr), _i32(col), _i32(est).reshape(-1)
    ia = np.zeros(max(n, 1), np.int32)
    ie = np.zeros(max(n, 1), np.int32)
    U = np.zeros(1, np.int32)
    cp = np.zeros(1, np.int64)
    rc = lib().orc_transitive(n, _p(row_ptr), _p(col), _p(est), n_gpu, unit_time, _p(ia), _p(ie), _p(U), _p(cp))
    if rc:
        raise OracleError(rc, "transitive")
    return ia[:n], ie[:n], int(U[0]), int(cp[0])


def regulate(ts, Ns, W, tau_bar, **kw):
    ts = np.ascontiguousarray(ts, dtype=np.int64)
    Ns = _i32(Ns)
    k = len(ts)
    mode, cnt, peak = (np.zeros(k, np.int32) for _ in range(3))
    p = params(**kw)
    lib().orc_regulate_seq(k, _p(ts), _p(Ns), C.byref(p), W, tau_bar, _p(mode), _p(cnt), _p(peak))
    return mode, cnt, peak


def schedule(w, policy="inspirit", variant=PLAIN, trace=False, **kw):
    """Schedule one synth.Workload (or any object with n, row_ptr, col, dur,
    est, n_cpu, n_gpu).  Returns a dict of numpy outputs."""
    n = int(w.n)
    kib = _i32(w.data_kib) if kw.get("data_bw", 0) > 0 else None
    p = params(policy=policy, data_kib=kib, **kw)
    rp, col = _i32(w.row_ptr), _i32(w.col)
    dur, est = _i32(w.dur).reshape(-1), _i32(w.est).reshape(-1)
    N = max(n, 1)
    out = {"worker": np.zeros(N, np.int32), "start": np.zeros(N, np.int64), "finish": np.zeros(N, np.int64),
           "ie_at_pop": np.zeros(N, np.int32), "mode_at_pop": np.zeros(N, np.int8)}
    ms = np.zeros(1, np.int64)
    nev = np.zeros(1, np.int32)
    U = np.zeros(1, np.int32)
    cap = (p.max_events if p.max_events > 0 else n + 1) if trace else 0
    tr = np.zeros(max(cap, 1), TRACE_DTYPE) if trace else None
    rc = lib().orc_schedule(n, _p(rp), _p(col), w.n_cpu, w.n_gpu, _p(dur), _p(est), C.byref(p), variant,
                            _p(out["worker"]), _p(out["start"]), _p(out["finish"]), _p(ms), _p(out["ie_at_pop"]),
                            _p(out["mode_at_pop"]), _p(tr), cap, _p(nev), _p(U))
    if rc:
        raise OracleError(rc, "schedule")
    for k in list(out):
        out[k] = out[k][:n]
    out["makespan"] = int(ms[0])
    out["n_events"] = int(nev[0])
    out["unit_time"] = int(U[0])
    if trace:
        out["trace"] = tr[: min(int(nev[0]), cap)]
    return out


def schedule_batch(batch, policy="inspirit", variant=HEAP, threads=None, **kw):
    """Schedule a synth.Batch on host threads; returns concatenated outputs."""
    kib = _i32(batch.data_kib) if kw.get("data_bw", 0) > 0 else None
    p = params(policy=policy, data_kib=kib, **kw)
    B = batch.n_dags
    ntot = int(batch.task_off[-1])
    N = max(ntot, 1)
    out = {"worker": np.zeros(N, np.int32), "start": np.zeros(N, np.int64), "finish": np.zeros(N, np.int64),
           "ie_at_pop": np.zeros(N, np.int32), "mode_at_pop": np.zeros(N, np.int8)}
    ms = np.zeros(max(B, 1), np.int64)
    st = np.zeros(max(B, 1), np.int32)
    threads = threads or os.cpu_count() or 1
    arrs = [np.ascontiguousarray(batch.task_off, np.int64), np.ascontiguousarray(batch.edge_off, np.int64),
            _i32(batch.row_ptr), _i32(batch.col), _i32(batch.n_cpu), _i32(batch.n_gpu),
            _i32(batch.dur).reshape(-1), _i32(batch.est).reshape(-1)]
    rc = lib().orc_schedule_batch(B, *[_p(a) for a in arrs], C.byref(p), variant, threads, _p(out["worker"]),
                                  _p(out["start"]), _p(out["finish"]), _p(ms), _p(out["ie_at_pop"]),
                                  _p(out["mode_at_pop"]), _p(st))
    if rc:
        raise OracleError(rc, "schedule_batch")
    for k in list(out):
        out[k] = out[k][:ntot]
    out["makespan"] = ms[:B]
    return out


def brute_opt(w) -> int:
    rp, col = canon(w.n, w.row_ptr, w.col)
    dur = _i32(w.dur).reshape(-1)
    opt = np.zeros(1, np.int64)
    rc = lib().orc_brute_opt(w.n, _p(rp), _p(col), w.n_cpu, w.n_gpu, _p(dur), _p(opt))
    if rc:
        raise OracleError(rc, "brute_opt")
    return int(opt[0])
