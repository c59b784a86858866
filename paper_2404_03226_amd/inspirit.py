"""Python binding of libinspirit (ctypes; argument marshalling only).

Every step of the scheduling path runs in the library's HIP kernels; torch
supplies device memory and the stream.  The functions mirror the C ABI in
``include/inspirit.h``: ``build_dag``, ``attributes``, ``schedule``,
``schedule_batch``, ``sync_status``.  A missing or unloadable library raises
``ImportError`` -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# INSP_LIB points the binding at another build of the library (the
# sanitizer test's host-instrumented one)
LIB_PATH = os.environ.get("INSP_LIB") or os.path.join(_HERE, "libinspirit.so")

OK, E_INVAL, E_CYCLE, E_RANGE, E_NOMEM, E_DEVICE, E_HANG = 0, 1, 2, 3, 4, 5, 6
POLICY = {"inspirit": 0, "fifo": 1, "ability": 2, "efi": 3, "heft": 4, "locality": 5}
MODE_ABILITY, MODE_EFI, MODE_EFI_LOC, MODE_FIFO, MODE_RANK = 0, 1, 2, 3, 4
ATTR_MODE = {"direct": 0, "transitive": 1}
MAX_TRANSITIVE_TASKS = 1 << 15
ALL_DAGS = -1

EXPORTS = ("insp_build_dag", "insp_set_task_data", "insp_free_dag", "insp_dag_info", "insp_attributes",
           "insp_transitive_attributes",
           "insp_schedule",
           "insp_schedule_batch", "insp_schedule_batch_trace", "insp_schedule_batch_noalloc", "insp_batch_graph_create",
           "insp_batch_graph_launch", "insp_batch_graph_free", "insp_sync_status", "insp_profile_enable", "insp_profile_read",
           "insp_mlp_create", "insp_mlp_free", "insp_mlp_grads", "insp_mlp_train_step", "insp_mlp_train", "insp_mlp_predict",
           "insp_mlp_state", "insp_last_error", "insp_test_fail_alloc")
MLP_PARAMS = 74754


class InspError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Workers(C.Structure):
    _fields_ = [("n_cpu", C.c_int32), ("n_gpu", C.c_int32)]


class Params(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("policy", "unit_time", "s_inc", "s_dec", "dec_step", "c", "k_num",
                                         "k_den", "max_events", "attr_mode", "data_bw")]


TRACE_DTYPE = np.dtype([("t", "<i8"), ("nready", "<i4"), ("mode", "<i4"), ("cnt", "<i4"), ("peak", "<i4"),
                        ("pushed", "<i4"), ("popped", "<i4")])


def params(policy="inspirit", unit_time=0, s_inc=-1, s_dec=-1, dec_step=-1, c=-1, k_num=-1, k_den=-1,
           max_events=0, attr_mode="direct", data_bw=0) -> Params:
    pol = POLICY[policy] if isinstance(policy, str) else int(policy)
    am = ATTR_MODE[attr_mode] if isinstance(attr_mode, str) else int(attr_mode)
    return Params(pol, unit_time, s_inc, s_dec, dec_step, c, k_num, k_den, max_events, am, data_bw)


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises ImportError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libinspirit.so not built at {path}; run __graft_entry__.build()")
    lib = C.CDLL(path)
    P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.insp_build_dag.argtypes = [i32, P, P, P, P, P, P, C.POINTER(P)]
    lib.insp_set_task_data.argtypes = [P, P, P]
    lib.insp_free_dag.argtypes = [P]
    lib.insp_free_dag.restype = None
    lib.insp_dag_info.argtypes = [P, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]
    lib.insp_attributes.argtypes = [P, i32, P, P, i32, P, P, P, P, P]
    lib.insp_transitive_attributes.argtypes = [P, i32, P, P, i32, P, P, P, P, P]
    lib.insp_schedule.argtypes = [P, i32, P, P, P, C.POINTER(Params), P, P, P, P, P, P, P, P, P]
    lib.insp_schedule_batch.argtypes = [P, P, P, P, C.POINTER(Params), P, P, P, P, P, P, C.c_char_p, P]
    lib.insp_schedule_batch_noalloc.argtypes = lib.insp_schedule_batch.argtypes
    lib.insp_schedule_batch_trace.argtypes = [P, P, P, P, C.POINTER(Params), P, P, P, P, P, P, P, P, C.c_char_p, P]
    lib.insp_batch_graph_create.argtypes = lib.insp_schedule_batch.argtypes + [C.POINTER(P)]
    lib.insp_batch_graph_launch.argtypes = [P, P]
    lib.insp_batch_graph_free.argtypes = [P]
    lib.insp_batch_graph_free.restype = None
    lib.insp_sync_status.argtypes = [P, P]
    lib.insp_profile_enable.argtypes = [C.c_int]
    lib.insp_profile_read.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(i64)]
    lib.insp_mlp_create.argtypes = [P, C.POINTER(P)]
    lib.insp_mlp_free.argtypes = [P]
    lib.insp_mlp_free.restype = None
    lib.insp_mlp_grads.argtypes = [P, P, P, i32, P, P, P, P]
    lib.insp_mlp_train_step.argtypes = [P, P, P, i32, C.c_float, P, P]
    lib.insp_mlp_train.argtypes = [P, P, P, i64, i32, i32, C.c_float, P, P]
    lib.insp_mlp_predict.argtypes = [P, P, i64, P, P, P]
    lib.insp_mlp_state.argtypes = [P, P, P, P, C.POINTER(i64), C.c_int]
    lib.insp_last_error.restype = C.c_char_p
    lib.insp_test_fail_alloc.argtypes = [i64]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise InspError(rc, load().insp_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


_DT = {"i32": "int32", "i64": "int64", "i8": "int8", "f32": "float32"}


def _dev(t, what, dtype, cols=None, rows=None):
    """Device tensor `t` as the library reads it: the named dtype, contiguous
    (a strided view would be read as other rows), on a GPU, with `cols`
    columns (a 2-D [rows, cols] tensor, or a flat one of rows * cols) and at
    least `rows` rows.  Returns its pointer; None passes through."""
    if t is None:
        return None
    import torch
    want = getattr(torch, _DT[dtype])
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != want:
        raise TypeError(f"{what}: expected {want}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if t.device.type != "cuda":
        raise ValueError(f"{what}: tensor must be on the GPU, got {t.device}")
    if cols is not None:
        if t.dim() == 2 and t.shape[1] != cols:
            raise ValueError(f"{what}: expected {cols} columns, got shape {tuple(t.shape)}")
        if t.dim() not in (1, 2) or t.numel() % cols:
            raise ValueError(f"{what}: expected [n, {cols}], got shape {tuple(t.shape)}")
    n = t.numel() // (cols or 1)
    if rows is not None and n < rows:
        raise ValueError(f"{what}: expected at least {rows} rows, got {n}")
    return C.c_void_p(t.data_ptr())


def test_fail_alloc(after: int):
    """Testing hook: the device allocation after `after` more successful ones
    fails with E_NOMEM (-1 turns injection off)."""
    _check(load().insp_test_fail_alloc(int(after)))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Dag:
    """Handle of B canonical DAGs resident on the device."""

    def __init__(self, handle, n_dags):
        self._h = handle
        self.n_dags = n_dags
        tn, te = C.c_int64(), C.c_int64()
        nd = C.c_int32()
        self.n = []
        self.m = []
        for b in range(n_dags):
            _check(load().insp_dag_info(self._h, b, C.byref(tn), C.byref(te), C.byref(nd)))
            self.n.append(tn.value)
            self.m.append(te.value)
        self.task_off = np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            load().insp_free_dag(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_dag(task_off, edge_off, row_ptr, col, type=None, stream=None) -> Dag:
    """task_off/edge_off: host int64 [B+1]; row_ptr/col/type: device int32."""
    task_off = np.ascontiguousarray(task_off, dtype=np.int64)
    edge_off = np.ascontiguousarray(edge_off, dtype=np.int64)
    h = C.c_void_p()
    _check(load().insp_build_dag(len(task_off) - 1, _ptr(task_off), _ptr(edge_off), _ptr(row_ptr), _ptr(col),
                                 _ptr(type), _stream(stream), C.byref(h)))
    return Dag(h, len(task_off) - 1)


def _workers(w, count):
    arr = (Workers * count)()
    if isinstance(w, (tuple, list)) and len(w) == 2 and not isinstance(w[0], (tuple, list)) and count == 1:
        w = [w]
    for i in range(count):
        arr[i].n_cpu, arr[i].n_gpu = int(w[i][0]), int(w[i][1])
    return arr


def attributes(dag: Dag, index, est, workers, unit_time=0, rem=None, stream=None):
    """Returns (ia, ie, unit_time_used) as device tensors and a numpy array."""
    import torch
    count = dag.n_dags if index == ALL_DAGS else 1
    lo = 0 if index == ALL_DAGS else dag.task_off[index]
    hi = dag.task_off[-1] if index == ALL_DAGS else dag.task_off[index + 1]
    n = int(hi - lo)
    ia = torch.empty(max(n, 1), dtype=torch.int32, device=est.device)
    ie = torch.empty(max(n, 1), dtype=torch.int32, device=est.device)
    U = np.zeros(count, np.int32)
    _check(load().insp_attributes(dag.handle, index, _dev(est, "est", "i32", 2, n), _workers(workers, count),
                                  unit_time, _dev(rem, "rem", "i32", 1, n), _ptr(ia), _ptr(ie), _ptr(U),
                                  _stream(stream)))
    return ia[:n], ie[:n], U


def set_task_data(dag: Dag, data_kib, stream=None):
    """Attach per-task output sizes (device int32 tensor, KiB, one per task of
    the handle) for the data model; None detaches them."""
    _check(load().insp_set_task_data(dag.handle, _dev(data_kib, "data_kib", "i32", 1, int(dag.task_off[-1])),
                                     _stream(stream)))


def transitive_attributes(dag: Dag, index, est, workers, unit_time=0, stream=None):
    """Transitive (ia_t, ie_t) as device tensors, and the unit time used and
    the longest path of each selected DAG as numpy arrays."""
    import torch
    count = dag.n_dags if index == ALL_DAGS else 1
    lo = 0 if index == ALL_DAGS else dag.task_off[index]
    hi = dag.task_off[-1] if index == ALL_DAGS else dag.task_off[index + 1]
    n = int(hi - lo)
    ia = torch.empty(max(n, 1), dtype=torch.int32, device=est.device)
    ie = torch.empty(max(n, 1), dtype=torch.int32, device=est.device)
    U = np.zeros(count, np.int32)
    lp = np.zeros(count, np.int64)
    _check(load().insp_transitive_attributes(dag.handle, index, _dev(est, "est", "i32", 2, n),
                                             _workers(workers, count), unit_time, _ptr(ia), _ptr(ie), _ptr(U),
                                             _ptr(lp), _stream(stream)))
    return ia[:n], ie[:n], U, lp


def _outputs(n, device, with_pop=True):
    import torch
    N = max(n, 1)
    out = {"worker": torch.empty(N, dtype=torch.int32, device=device),
           "start": torch.empty(N, dtype=torch.int64, device=device),
           "finish": torch.empty(N, dtype=torch.int64, device=device)}
    if with_pop:
        out["ie_at_pop"] = torch.empty(N, dtype=torch.int32, device=device)
        out["mode_at_pop"] = torch.empty(N, dtype=torch.int8, device=device)
    return out


def schedule(dag: Dag, index, workers, dur, est, prm: Params = None, trace=False, stream=None, out=None):
    """Simulate DAG `index`; returns a dict of device tensors (makespan [1])."""
    import torch
    prm = prm or params()
    n = int(dag.n[index])
    dev = dur.device
    o = out or _outputs(n, dev)
    o["makespan"] = o.get("makespan", torch.empty(1, dtype=torch.int64, device=dev))
    o["n_events"] = o.get("n_events", torch.empty(1, dtype=torch.int32, device=dev))
    tr = None
    if trace:
        cap = prm.max_events if prm.max_events > 0 else n + 1
        tr = torch.zeros(cap * TRACE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        o["trace"] = tr
    _check(load().insp_schedule(dag.handle, index, _workers(workers, 1), _dev(dur, "dur", "i32", 2, n),
                                _dev(est, "est", "i32", 2, n), C.byref(prm),
                                _dev(o["worker"], "worker", "i32", 1, n), _dev(o["start"], "start", "i64", 1, n),
                                _dev(o["finish"], "finish", "i64", 1, n), _dev(o["makespan"], "makespan", "i64", 1, 1),
                                _dev(o.get("ie_at_pop"), "ie_at_pop", "i32", 1, n),
                                _dev(o.get("mode_at_pop"), "mode_at_pop", "i8", 1, n), _ptr(tr),
                                _dev(o["n_events"], "n_events", "i32", 1, 1), _stream(stream)))
    return o


def trace_records(trace_tensor, n_events):
    raw = trace_tensor.cpu().numpy().view(TRACE_DTYPE)
    return raw[:n_events]


def schedule_batch(dag: Dag, workers, dur, est, prm: Params = None, tune_key=None, stream=None, out=None,
                   with_pop=True, trace=False):
    """Simulate all DAGs in one persistent launch; returns device tensors.
    trace=True also returns "trace" (raw records, DAG b's from index
    task_off[b] + b on) and "n_events" [B]; see batch_trace_records."""
    if not trace:
        return _batch(load().insp_schedule_batch, dag, workers, dur, est, prm, tune_key, stream, out, with_pop)
    import torch
    dev = dur.device
    o = out or _outputs(int(dag.task_off[-1]), dev, with_pop)
    n, B = int(dag.task_off[-1]), dag.n_dags
    o["trace"] = o.get("trace", torch.zeros((n + B) * TRACE_DTYPE.itemsize, dtype=torch.uint8, device=dev))
    o["n_events"] = o.get("n_events", torch.zeros(max(B, 1), dtype=torch.int32, device=dev))
    if o["trace"].dtype != torch.uint8 or o["trace"].numel() < (n + B) * TRACE_DTYPE.itemsize:
        raise ValueError(f"trace needs {(n + B) * TRACE_DTYPE.itemsize} bytes (uint8)")
    return _batch(load().insp_schedule_batch_trace, dag, workers, dur, est, prm, tune_key, stream, o, with_pop,
                  extra=(_ptr(o["trace"]), _dev(o["n_events"], "n_events", "i32", 1, B)))


def batch_trace_records(dag: Dag, out, b):
    """DAG b's trace records (numpy, TRACE_DTYPE) from a traced schedule_batch."""
    nev = int(out["n_events"][b].item())
    lo = int(dag.task_off[b]) + b
    cap = int(dag.task_off[b + 1] - dag.task_off[b]) + 1
    raw = out["trace"].cpu().numpy().view(TRACE_DTYPE)
    return raw[lo: lo + min(nev, cap)]


NOALLOC_SCRATCH_BYTES = 64 << 20


def schedule_batch_noalloc(dag: Dag, workers, dur, est, prm: Params = None, tune_key=None, stream=None, out=None,
                           with_pop=True):
    """schedule_batch through the allocation-free entry point (per-call state
    in the library's static scratch array); pass `out` to allocate nothing."""
    return _batch(load().insp_schedule_batch_noalloc, dag, workers, dur, est, prm, tune_key, stream, out, with_pop)


def _batch(fn, dag, workers, dur, est, prm, tune_key, stream, out, with_pop, extra=()):
    import torch
    prm = prm or params()
    dev = dur.device
    o = out or _outputs(int(dag.task_off[-1]), dev, with_pop)
    o["makespan"] = o.get("makespan", torch.empty(dag.n_dags, dtype=torch.int64, device=dev))
    key = tune_key.encode() if isinstance(tune_key, str) else tune_key
    n, B = int(dag.task_off[-1]), dag.n_dags
    _check(fn(dag.handle, _workers(workers, B), _dev(dur, "dur", "i32", 2, n),
              _dev(est, "est", "i32", 2, n), C.byref(prm),
              _dev(o["worker"], "worker", "i32", 1, n), _dev(o["start"], "start", "i64", 1, n),
              _dev(o["finish"], "finish", "i64", 1, n),
              _dev(o["makespan"], "makespan", "i64", 1, B),
              _dev(o.get("ie_at_pop"), "ie_at_pop", "i32", 1, n),
              _dev(o.get("mode_at_pop"), "mode_at_pop", "i8", 1, n), *extra, key, _stream(stream)))
    return o


class BatchGraph:
    """One batch step captured in a HIP graph the library owns; `out` holds
    the device outputs every replay writes."""

    def __init__(self, dag: Dag, workers, dur, est, prm: Params = None, tune_key=None, stream=None, out=None,
                 with_pop=True):
        import torch
        prm = prm or params()
        dev = dur.device
        o = out or _outputs(int(dag.task_off[-1]), dev, with_pop)
        o["makespan"] = o.get("makespan", torch.empty(dag.n_dags, dtype=torch.int64, device=dev))
        key = tune_key.encode() if isinstance(tune_key, str) else tune_key
        n, B = int(dag.task_off[-1]), dag.n_dags
        self._keep = (dag, dur, est, prm, key, C.byref(prm))
        self.out = o
        self.handle = None
        g = C.c_void_p()
        _check(load().insp_batch_graph_create(
            dag.handle, _workers(workers, B), _dev(dur, "dur", "i32", 2, n), _dev(est, "est", "i32", 2, n),
            C.byref(prm), _dev(o["worker"], "worker", "i32", 1, n), _dev(o["start"], "start", "i64", 1, n),
            _dev(o["finish"], "finish", "i64", 1, n), _dev(o["makespan"], "makespan", "i64", 1, B),
            _dev(o.get("ie_at_pop"), "ie_at_pop", "i32", 1, n), _dev(o.get("mode_at_pop"), "mode_at_pop", "i8", 1, n),
            key, _stream(stream), C.byref(g)))
        self.handle = g.value

    def launch(self, stream=None):
        _check(load().insp_batch_graph_launch(self.handle, _stream(stream)))
        return self.out

    def free(self):
        if self.handle:
            load().insp_batch_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sync_status(dag: Dag, stream=None):
    _check(load().insp_sync_status(dag.handle, _stream(stream)))


def profile_enable(on=True):
    """True or 1: time every library scope; 2: only the outermost scope of
    each call (no event records between the kernels it brackets); False/0: off."""
    mode = 1 if on is True else 0 if on is False else int(on)
    _check(load().insp_profile_enable(mode))


def profile_read(kernel=""):
    """(total milliseconds, launches) of the library's kernels named `kernel*`."""
    ms, n = C.c_double(), C.c_int64()
    _check(load().insp_profile_read(kernel.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def to_device(w, device="cuda"):
    """Upload one synth.Workload and build its handle; returns (dag, dur, est)."""
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(w.row_ptr, np.int32)).to(device)
    col = torch.from_numpy(np.ascontiguousarray(w.col, np.int32)).to(device)
    if col.numel() == 0:
        col = torch.zeros(1, dtype=torch.int32, device=device)
    dag = build_dag([0, w.n], [0, w.m], rp, col)
    dur = torch.from_numpy(np.ascontiguousarray(w.dur, np.int32)).to(device)
    est = torch.from_numpy(np.ascontiguousarray(w.est, np.int32)).to(device)
    return dag, dur, est


def batch_to_device(b, device="cuda"):
    """Upload one synth.Batch and build its handle; returns (dag, dur, est)."""
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(b.row_ptr, np.int32)).to(device)
    col = torch.from_numpy(np.ascontiguousarray(b.col, np.int32)).to(device)
    dag = build_dag(b.task_off, b.edge_off, rp, col)
    dur = torch.from_numpy(np.ascontiguousarray(b.dur, np.int32)).to(device)
    est = torch.from_numpy(np.ascontiguousarray(b.est, np.int32)).to(device)
    return dag, dur, est


class Mlp:
    """Learned cost model on the device (see insp_mlp_* in the header)."""

    def __init__(self, params):
        flat = np.ascontiguousarray(np.concatenate([np.asarray(q, np.float32).reshape(-1) for q in params]))
        assert flat.size == MLP_PARAMS
        h = C.c_void_p()
        _check(load().insp_mlp_create(_ptr(flat), C.byref(h)))
        self._h = h

    def free(self):
        if getattr(self, "_h", None):
            load().insp_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def grads(self, x, t, stream=None):
        import torch
        B = x.shape[0]
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        y = torch.empty((B, 2), dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(load().insp_mlp_grads(self._h, _dev(x, "x", "f32", 32, B), _dev(t, "t", "f32", 2, B), B, _ptr(g),
                                     _ptr(y), _ptr(loss), _stream(stream)))
        return g, y, loss

    def train_step(self, x, t, lr=1e-3, loss=None, stream=None):
        B = x.shape[0]
        _check(load().insp_mlp_train_step(self._h, _dev(x, "x", "f32", 32, B), _dev(t, "t", "f32", 2, B), B, lr,
                                          _dev(loss, "loss", "f32", 1, 1), _stream(stream)))

    def train(self, x, t, batch=1024, epochs=1, lr=1e-3, loss=None, stream=None):
        """`epochs` passes over all rows of x, t in minibatches (graph-captured)."""
        n = x.shape[0]
        _check(load().insp_mlp_train(self._h, _dev(x, "x", "f32", 32, n), _dev(t, "t", "f32", 2, n), n, batch,
                                     epochs, lr, _dev(loss, "loss", "f32", 1, 1), _stream(stream)))

    def predict(self, x, want_y=True, stream=None):
        import torch
        n = x.shape[0]
        y = torch.empty((max(n, 1), 2), dtype=torch.float32, device=x.device) if want_y else None
        est = torch.empty((max(n, 1), 2), dtype=torch.int32, device=x.device)
        _check(load().insp_mlp_predict(self._h, _dev(x, "x", "f32", 32, n), n, _ptr(y), _ptr(est),
                                       _stream(stream)))
        return (y[:n] if want_y else None), est[:n]

    def state(self):
        p, m, v = (np.zeros(MLP_PARAMS, np.float32) for _ in range(3))
        step = C.c_int64()
        _check(load().insp_mlp_state(self._h, _ptr(p), _ptr(m), _ptr(v), C.byref(step), 1))
        return p, m, v, step.value

    def load_state(self, p, m, v, step):
        p, m, v = (np.ascontiguousarray(a, np.float32) for a in (p, m, v))
        st = C.c_int64(step)
        _check(load().insp_mlp_state(self._h, _ptr(p), _ptr(m), _ptr(v), C.byref(st), 0))
