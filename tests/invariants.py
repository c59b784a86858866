"""Schedule properties that hold for every correct schedule of this method,
at any size; used on oracle and HIP outputs alike."""
import numpy as np


def check_schedule(w, worker, start, finish, makespan, non_idling=True):
    n = w.n
    rp = np.asarray(w.row_ptr, np.int64)
    col = np.asarray(w.col, np.int64)
    dur = np.asarray(w.dur).reshape(n, 2)
    W = w.n_cpu + w.n_gpu
    worker = np.asarray(worker)
    start = np.asarray(start, np.int64)
    finish = np.asarray(finish, np.int64)
    if n == 0:
        assert makespan == 0
        return
    # every task scheduled exactly once, on a real worker
    assert worker.shape == (n,) and ((worker >= 0) & (worker < W)).all()
    kind = (worker >= w.n_cpu).astype(np.int64)
    # duration
    assert (finish - start == dur[np.arange(n), kind]).all()
    assert (start >= 0).all()
    # precedence
    src = np.repeat(np.arange(n), np.diff(rp))
    assert (start[col] >= finish[src]).all(), "precedence violated"
    assert makespan == finish.max()
    # worker exclusivity
    order = np.lexsort((start, worker))
    ws, ss, fs = worker[order], start[order], finish[order]
    same = ws[1:] == ws[:-1]
    assert (ss[1:][same] >= fs[:-1][same]).all(), "overlap on a worker"
    if not non_idling:
        return
    # a worker is never idle at an event time while a task sits in its queue:
    # [ready(v), start(v)) must be covered by busy intervals of worker(v)
    ready = np.zeros(n, np.int64)
    np.maximum.at(ready, col, finish[src])
    for w_id in np.unique(worker):
        idx = order[ws == w_id]
        s_w, f_w = start[idx], finish[idx]
        for v in idx:
            if start[v] == ready[v]:
                continue
            # busy intervals ending after ready[v] and starting before start[v]
            k = np.searchsorted(s_w, start[v])  # tasks starting before start(v)
            t = ready[v]
            covered = True
            for j in range(k):
                if f_w[j] <= t:
                    continue
                if s_w[j] > t:
                    covered = False
                    break
                t = f_w[j]
                if t >= start[v]:
                    break
            assert covered and t >= start[v], f"worker {w_id} idle while task {v} waited"
