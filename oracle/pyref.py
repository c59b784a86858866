"""Pure-Python twin of the oracle, for tiny DAGs -- TEST INFRASTRUCTURE.

A second, independent transcription of the same definitions (Sections 2,
4.2-4.4 of arXiv 2404.03226, with the readings stated in ``oracle.c``),
written with Python containers and no shared code, so that a slip in one
transcription shows up as a disagreement with the other.  Linear scans
everywhere; only for a few hundred tasks.
"""
from __future__ import annotations

ABILITY, EFI, EFI_LOC, FIFO = 0, 1, 2, 3


def _succ(n, row_ptr, col):
    out = []
    for v in range(n):
        out.append(sorted(set(int(x) for x in col[row_ptr[v]:row_ptr[v + 1]])))
    return out


def tau(est, n_gpu, v):
    return int(est[v][1] if n_gpu > 0 else est[v][0])


def ie_at(succ, est, n_gpu, rem, U, v):
    return sum(1 for s in succ[v] if rem[s] == 1 and tau(est, n_gpu, v) + tau(est, n_gpu, s) <= U)


def pick_unit_time(succ, est, n_gpu, rem):
    n = len(succ)
    mx = max((tau(est, n_gpu, v) for v in range(n)), default=0)
    ladder = [1]
    while ladder[-1] < 2 * mx:
        ladder.append(ladder[-1] * 2)
    best_u, best_s = None, None
    for U in ladder:
        s = sum(1 for v in range(n) if 0 < ie_at(succ, est, n_gpu, rem, U, v) < len(succ[v]))
        if best_s is None or s >= best_s:
            best_u, best_s = U, s
    return best_u


class Regulator:
    def __init__(self, W, tau_bar, s_inc=-1, s_dec=-1, dec_step=-1, c=-1, k_num=-1, k_den=-1):
        d_sdec = max(1, -(-W // 2))
        self.s_inc = s_inc if s_inc > 0 else max(1, -(-W // 4))
        self.s_dec = s_dec if s_dec > 0 else d_sdec
        self.dec_step = dec_step if dec_step > 0 else self.s_dec
        self.c = c if c >= 0 else self.s_dec // 2
        if k_num > 0 and k_den > 0:
            self.k_num, self.k_den = k_num, k_den
        else:
            self.k_num, self.k_den = W, tau_bar
        self.peak = self.prev_n = self.prev_t = self.cnt = 0
        self.mode = ABILITY

    def observe(self, t, N):
        if N > self.peak:
            self.peak = N
        if abs(N - self.prev_n) < self.s_inc:
            return
        dn, dt = N - self.prev_n, t - self.prev_t
        self.prev_n, self.prev_t = N, t
        if N >= self.peak - self.dec_step:
            self.cnt = 0
            if dn >= self.s_inc:
                # slope dn/dt against k_num/k_den; zero elapsed time = steep
                if dt == 0 or dn * self.k_den > self.k_num * dt:
                    self.mode = ABILITY
                elif dn * self.k_den < self.k_num * dt:
                    self.mode = EFI
        else:
            hi = self.peak - self.s_dec * self.cnt
            lo = self.peak - self.s_dec * (self.cnt + 1)
            if N > hi:
                self.mode = ABILITY
            elif N <= lo + self.c:
                self.mode = EFI_LOC
                if N <= lo:
                    self.cnt += 1


def schedule(n, row_ptr, col, n_cpu, n_gpu, dur, est, policy="inspirit", unit_time=0, **reg_kw):
    """Returns dict(worker, start, finish, makespan, ie_at_pop, mode_at_pop, trace)."""
    succ = _succ(n, row_ptr, col)
    dur = [tuple(int(x) for x in r) for r in dur]
    est = [tuple(int(x) for x in r) for r in est]
    W = n_cpu + n_gpu
    kind = [0 if w < n_cpu else 1 for w in range(W)]
    rem = [0] * n
    for v in range(n):
        for s in succ[v]:
            rem[s] += 1
    U = unit_time if unit_time > 0 else pick_unit_time(succ, est, n_gpu, rem)
    ia = [len(succ[v]) for v in range(n)]
    tau_bar = max(1, sum(tau(est, n_gpu, v) for v in range(n)) // n) if n else 1
    reg = Regulator(W, tau_bar, **reg_kw)
    queues = [[] for _ in range(W)]     # (seq, task) in push order
    running = [None] * W                # (task, start)
    res = {"worker": [None] * n, "start": [None] * n, "finish": [None] * n,
           "ie_at_pop": [None] * n, "mode_at_pop": [None] * n, "trace": []}
    t, seqno, done = 0, 0, 0
    ready = sorted(v for v in range(n) if rem[v] == 0)
    if n == 0:
        res["makespan"] = 0
        return res
    while True:
        for v in ready:
            costs = []
            for w in range(W):
                free_at = t
                if running[w] is not None:
                    r, st = running[w]
                    free_at = max(t, st + est[r][kind[w]])
                queued = sum(est[q][kind[w]] for _, q in queues[w])
                costs.append((free_at + queued + est[v][kind[w]], w))
            _, w = min(costs)
            queues[w].append((seqno, v))
            seqno += 1
        nready = sum(len(q) for q in queues)
        if policy == "inspirit":
            reg.observe(t, nready)
            mode = reg.mode
        else:
            mode = {"fifo": FIFO, "ability": ABILITY, "efi": EFI}[policy]
        popped = 0
        for w in range(W):
            if running[w] is not None or not queues[w]:
                continue

            def key(item):
                sq, v = item
                e = ie_at(succ, est, n_gpu, rem, U, v)
                if mode == FIFO:
                    return (-sq,)
                if mode == ABILITY:
                    return (ia[v], e, -sq)
                return (e, ia[v], -sq)

            item = max(queues[w], key=key)
            queues[w].remove(item)
            v = item[1]
            running[w] = (v, t)
            res["worker"][v] = w
            res["start"][v] = t
            res["finish"][v] = t + dur[v][kind[w]]
            res["ie_at_pop"][v] = ie_at(succ, est, n_gpu, rem, U, v)
            res["mode_at_pop"][v] = mode
            popped += 1
        res["trace"].append((t, nready, mode, reg.cnt, reg.peak, len(ready), popped))
        if done == n:
            break
        t = min(res["finish"][r] for r, _ in (x for x in running if x is not None))
        finished = [w for w in range(W) if running[w] is not None and res["finish"][running[w][0]] == t]
        ready = []
        for w in finished:
            v = running[w][0]
            running[w] = None
            done += 1
            for s in succ[v]:
                rem[s] -= 1
                if rem[s] == 0:
                    ready.append(s)
        ready.sort()
    res["makespan"] = t
    res["unit_time"] = U
    return res
