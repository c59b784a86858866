// Event-driven list-scheduling simulation with INSPIRIT priorities.
//
// One wave64 work-group owns one DAG at a time and runs its whole event loop
// (a persistent grid takes DAGs, largest first, from an atomic dispenser).
// Per event time t, in order (Section 2 DMDA push, Section 4.1 per-worker
// queues, Section 4.4 adaptive pop rule):
//   push     newly ready tasks in ascending id, each to the worker with the
//            least expected termination time (free time + queued estimates +
//            own estimate; ties to the lower worker id) -- a wave-wide argmin
//            over packed (cost, worker) keys;
//   regulate Nready = queued tasks; the Section 4.4 state machine picks the
//            pop rule (scalar code);
//   pop      every idle worker takes the best task of its own queue under the
//            rule -- two wave-wide argmax steps over 64-slot blocks;
//   advance  t = earliest finish among running tasks (wave min);
//   release  for each completing task c and edge c -> s, one 64-bit
//            read-modify-write (the wave owns the DAG) subtracts (1 << 43) + c
//            from word[s] = rem << 43 | sum of unfinished predecessor ids.  rem reaching 0 makes s ready; rem
//            reaching 1 leaves exactly one unfinished predecessor
//            u = remaining sum, whose IE grows by one when tau(u) + tau(s)
//            <= U (IE counts successors with rem == 1).  Newly ready ids of
//            one completing task arrive ascending (rows are sorted); several
//            such runs are merged by rank.
//
// Queue entry (two 64-bit words):  k = IA << 42 | IE << 21 | (2^21-1-seq),
//                                  x = task << 42 | dur << 21 | est
// (all fields < 2^21).  Under the ability rule the key is k itself; under the
// efficiency rule IA and IE swap places; FIFO keeps only the seq field.  Keys
// are unique (seq), so a max identifies one entry.  Each block keeps the max
// key of its entries under two rules (ability-or-FIFO, efficiency); IE only
// grows while a task waits, so increments update block maxima with atomicMax
// and a pop rescans only the block it touched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

constexpr uint64_t M21 = (1ull << 21) - 1;
constexpr uint64_t M43 = (1ull << 43) - 1;
constexpr uint64_t BIT63 = 1ull << 63;

#ifdef INSP_PHASE_CLOCKS
// Diagnostic build only: per-DAG core-clock totals of each event phase.
__device__ unsigned long long g_phase_clk[8192 * 32];
#define PCLK(i) do { unsigned long long c_ = clock64(); pc[i] += c_ - pc_last; pc_last = c_; } while (0)
#else
#define PCLK(i) do {} while (0)
#endif

// Sort key of a queue entry under rule `ord`: 0 ability, 1 efficiency,
// 2 FIFO, 3 HEFT (whose entries hold rank << 21 | (2^21-1-seq) instead).
__device__ __forceinline__ uint64_t key_of(uint64_t k, int ord) {
    if (ord == 0 || ord == 3) return k | BIT63;
    if (ord == 1) return ((k >> 21) & M21) << 42 | (k >> 42) << 21 | (k & M21) | BIT63;
    return (k & M21) | BIT63;
}

// Makes the compiler wait for a global load inside the branch that issued it.
// A value read from LDS on one side of a uniform branch and from global memory
// on the other otherwise arrives at the join with a pending global load, and
// every later use waits for all outstanding global accesses -- stores
// included -- even when the LDS side ran.
template <typename T>
__device__ __forceinline__ void settle(const T &x) {
    asm volatile("" ::"v"(x));
}

// The popped task's schedule, written over its dead dependency word and
// push order (see TaskRec): one 16-byte store.
__device__ __forceinline__ void put_record(TaskRec *r, int64_t start, int32_t dur, int32_t w, int32_t ie, int mode) {
    const uint64_t wd = (uint64_t)start | (uint64_t)dur << 42;
    int4 q;
    q.x = (int32_t)(uint32_t)wd;
    q.y = (int32_t)(uint32_t)(wd >> 32);
    q.z = -2 - w;
    q.w = ie | mode << 22;
    *reinterpret_cast<int4 *>(r) = q;
}

struct SimArgs {
    const DagDesc *desc;
    const int32_t *order;
    int32_t count, max_w, sum_cap, policy, lb, slot_cap;
    int32_t key_cap;           // queue blocks whose keys live in LDS (>= slot_cap, whose payload does too)
    const int32_t *col;
    const int32_t *dur, *est;
    int64_t base;
    TaskRec *tr;
    unsigned long long *dep;   // dependency words: remaining in-degree << 43 | sum of unfinished predecessor ids
    int32_t *fbuf;
    SlotPool slots;
    unsigned long long *sums;
    int32_t *paux;
    int64_t freeb_base;
    const int32_t *dag_u, *dag_taubar;
    const int64_t *rank;  // HEFT upward ranks (global task index)
    const int32_t *tia, *tie;  // transitive IA, IE (global task index)
    int32_t attr_mode;
    int32_t data_bw;           // data model: bytes per tick between memory nodes (0 = off)
    const int32_t *dkib;       // data model: output KiB per task (global task index)
    const int32_t *pprp, *ppred;  // predecessor lists (local row pointers as rp, ids as col)
    long long *barr;           // data model: per queue block, the latest input arrival pushed into it
    int32_t *dxc;              // data model: transfer ticks of each task's output (global task index)
    int32_t *stat;
    int32_t *counter;
    int64_t *makespan;
    insp_trace_rec *trace;     // DAG di's events from record (toff - base) + di on: n + 1 slots per DAG
    int32_t *n_events;
    int32_t s_inc, s_dec, dec_step, c, k_num, k_den, max_events;
    int32_t prio_top;          // DAGs dispensed before this one run at raised wave priority
    int32_t scan_max;          // a pop scans every entry of a worker with at most this many blocks (<= kScan)
};

// LDS-resident state of the DAG a work-group is simulating.
constexpr int kPF = 8;    // successors of a running task prefetched into registers at its pop
constexpr int kFC = 256;  // frontier slots in LDS (larger frontiers use global memory)
constexpr int kCC = 128;  // candidate slots in LDS

struct Lds {
    int64_t *fin, *expend, *qest;                    // [MW]
    int32_t *run, *len, *nb, *last, *seg, *rsr, *dgr; // [MW]
    int32_t *blist;                                  // [MW * lb] first block ids of each worker
    unsigned long long *sum;                         // [2 * sum_cap] block max keys
    int32_t *fr0, *fr1;                              // [kFC]
    int32_t *cs, *cu;                                // [kCC]
    int32_t *pre;                                    // [8 * kWave] staged frontier rows
    unsigned long long *sk;                          // [64 * key_cap] keys of the low blocks' entries
    unsigned long long *sx;                          // [64 * slot_cap] payload (task, durations) of the lowest
    int32_t *srs;                                    // [64 * slot_cap] ... and their first edges
    int32_t *fstk;                                   // [sum_cap] free block ids below sum_cap
    uint8_t *stale;                                  // [sum_cap] block maxima to rebuild before use
    int32_t *hs;                                     // [4] DAG index, simulation finished, helper sink
};

__host__ __device__ constexpr size_t lds_bytes(int mw, int sc, int lb, int slc, int slk) {
    return (size_t)mw * (3 * 8 + 7 * 4 + (size_t)lb * 4) + (size_t)sc * (16 + 4 + 1) + kFC * 8 + kCC * 8 +
           8 * 64 * 4 + (size_t)slc * 64 * 12 + (size_t)slk * 64 * 8 + 64 + 32;
}

template <int WPL>
__device__ void sim_dag(const SimArgs &A, int32_t di, const Lds &L) {
    constexpr bool kPrefetch = WPL <= 2;
    constexpr int PW = kPrefetch ? WPL : 1;
    const int lane = lane_id();
    const DagDesc d = A.desc[di];
    const int32_t n = d.n, ncpu = d.n_cpu, W = d.n_cpu + d.n_gpu;
    int32_t status = A.stat[2 * d.id];
    if (n == 0 || status != 0) {
        if (lane == 0) {
            A.makespan[di] = status ? -1 : 0;
            if (A.n_events) A.n_events[di] = 0;
        }
        return;
    }
    const int64_t ub = d.toff - A.base;
    const int32_t *col = A.col + d.eoff;
    TaskRec *tr = A.tr + d.toff;
    unsigned long long *dep = A.dep + d.toff;
    int32_t *fbuf = A.fbuf + 3 * d.toff;      // [0,n) runs, [n,2n) merged, [2n,3n) candidates
    const int2 *est2 = reinterpret_cast<const int2 *>(A.est) + ub;
    const int2 *dur2 = reinterpret_cast<const int2 *>(A.dur) + ub;
    const SlotPool slots = A.slots.at(64 * d.blk_off);
    unsigned long long *sums = A.sums + 2 * d.blk_off;
    int32_t *wblk = A.paux + d.wl_off;
    int32_t *freeb = A.paux + A.freeb_base + d.blk_off;
    const int32_t maxb = d.maxb;
    const int32_t SC = A.sum_cap;
    const int32_t kLB = A.lb;
    const int32_t SLC = A.slot_cap;  // blocks [0, SLC) keep their slots in LDS
    const int32_t U = A.dag_u[d.id];

    // regulator parameters (defaults: the paper names them, prints no values)
    const int32_t s_inc = A.s_inc > 0 ? A.s_inc : max(1, (W + 3) / 4);
    const int32_t s_dec = A.s_dec > 0 ? A.s_dec : max(1, (W + 1) / 2);
    const int32_t dec_step = A.dec_step > 0 ? A.dec_step : s_dec;
    const int32_t cc = A.c >= 0 ? A.c : s_dec / 2;
    const bool kset = A.k_num > 0 && A.k_den > 0;
    const int32_t k_num = kset ? A.k_num : W;
    const int32_t k_den = kset ? A.k_den : A.dag_taubar[d.id];
    const bool heft = A.policy == INSP_POLICY_HEFT;
    const bool tattr = A.attr_mode == INSP_ATTR_TRANSITIVE;
    const bool trans = !heft && tattr;  // keys built from the transitive attributes
    const bool skey = heft || trans;  // keys fixed while queued
    const int64_t *rk = A.rank + d.toff;
    const int32_t *tia = A.tia + d.toff, *tie = A.tie + d.toff;
    // data model: inputs move between memory nodes (host for the CPU
    // workers, one per GPU worker); see the push and the pop below
    const bool data = A.data_bw > 0;
    const int32_t *dkib = A.dkib + d.toff, *prp = A.pprp + d.toff + d.id, *pred = A.ppred + d.eoff;
    long long *barr = A.barr + d.blk_off;
    int32_t *dxc = A.dxc + d.toff;
    // block arrival bounds matter only where the locality rule can be used
    const bool lrule = data && (A.policy == INSP_POLICY_INSPIRIT || A.policy == INSP_POLICY_LOCALITY);
    const int slot0 = A.policy == INSP_POLICY_FIFO ? 2 : heft ? 3 : 0;
    const int32_t max_events = A.max_events > 0 ? A.max_events : n + 1;

    for (int32_t w = lane; w < W; w += kWave) {
        L.run[w] = -1;
        L.len[w] = 0;
        L.nb[w] = 0;
        L.last[w] = -1;
        L.fin[w] = 0;
        L.expend[w] = 0;
        L.qest[w] = 0;
        L.rsr[w] = 0;
        L.dgr[w] = 0;
    }
    for (int32_t i = lane; i < d.nblk; i += kWave) freeb[i] = d.nblk - 1 - i;
    int32_t nfree = d.nblk;
    if (data)  // each output's transfer ticks, once per run (no division at the pushes)
        for (int32_t i = lane; i < n; i += kWave)
            dxc[i] = (int32_t)(((int64_t)1024 * dkib[i] + A.data_bw - 1) / A.data_bw);

    // initial frontier: tasks without predecessors, ascending
    int32_t r = 0;
    for (int32_t i0 = 0; i0 < n; i0 += kWave) {
        int32_t i = i0 + lane;
        bool ok = i < n && (dep[i] >> 43) == 0;
        uint64_t mk = ballot(ok);
        if (ok) {
            int32_t pos = r + lanes_below(mk);
            fbuf[pos] = i;
            if (pos < kFC) L.fr0[pos] = i;
        }
        r += __popcll(mk);
    }
    bool merged = false, staged = false;
    int32_t pf[PW][kPF];
#pragma unroll
    for (int k = 0; k < PW; k++)
#pragma unroll
        for (int j = 0; j < kPF; j++) pf[k][j] = 0;
    wg_fence();
    __builtin_amdgcn_wave_barrier();

    int64_t t = 0, prev_t = 0;
    int32_t nready = 0, events = 0, done = 0, seq = 0;
    int32_t peak = 0, prev_n = 0, cnt = 0;
    int mode = INSP_MODE_ABILITY;
#ifdef INSP_PHASE_CLOCKS
    unsigned long long pc[32] = {0}, pc_last = clock64();
#endif

    for (;;) {
        PCLK(9);
        if (++events > max_events) {
            status |= ST_HANG;
            break;
        }
        // ------------------------------------------------------------ push
        int64_t ld[WPL];
#pragma unroll
        for (int k = 0; k < WPL; k++) {
            int32_t w = lane + k * kWave;
            ld[k] = INT64_MAX / 4;
            if (w < W) {
                int64_t B = t;
                if (L.run[w] >= 0 && L.expend[w] > t) B = L.expend[w];
                ld[k] = B + L.qest[w];
            }
        }
        for (int32_t i0 = 0; i0 < r; i0 += kWave) {
            const int32_t idx = i0 + lane;
            const bool ok = idx < r;
            int32_t v_l = 0;
            int2 e_l = make_int2(1, 1), d_l = make_int2(1, 1);
            int32_t ia_l = 0, ie_l = 0, rs_l = 0;
            uint64_t rk_l = 0;
            if (staged) {
                // rows loaded during the previous candidate round trip
                if (ok) {
                    v_l = L.pre[idx];
                    e_l = make_int2(L.pre[64 + idx], L.pre[128 + idx]);
                    d_l = make_int2(L.pre[192 + idx], L.pre[256 + idx]);
                    ia_l = L.pre[320 + idx];
                    rs_l = L.pre[384 + idx];
                    ie_l = L.pre[448 + idx];
                }
            } else {
                if (ok) {
                    if (r <= kFC) v_l = merged ? L.fr1[idx] : L.fr0[idx];
                    else v_l = merged ? fbuf[n + idx] : fbuf[idx];
                }
                if (ok) {
                    e_l = est2[v_l];
                    d_l = dur2[v_l];
                    ia_l = tr[v_l].ia;
                    rs_l = tr[v_l].rs;
                    ie_l = wg_load(&tr[v_l].iev);
                }
            }
            if (heft && ok) rk_l = (uint64_t)rk[v_l];
            if (trans && ok) {
                ia_l = tia[v_l];
                ie_l = tie[v_l];
            }
            if (ballot(ok && (d_l.x < 1 || d_l.x > INSP_MAX_TICK || d_l.y < 1 || d_l.y > INSP_MAX_TICK)))
                status |= ST_DUR;
            const int32_t cntj = min(kWave, r - i0);
            for (int32_t j = 0; j < cntj; j++) {
                const int32_t v = read_lane(v_l, j);
                const int32_t e0 = read_lane(e_l.x, j), e1 = read_lane(e_l.y, j);
                // DMDA's transfer term: ticks to move the inputs whose home
                // node is not the worker's (an item stays where it was made)
                int64_t xk[WPL];
#pragma unroll
                for (int k = 0; k < WPL; k++) xk[k] = 0;
                if (data) {
                    const int32_t pa = prp[v], pz = prp[v + 1];
                    for (int32_t c0 = pa; c0 < pz; c0 += kWave) {
                        int32_t nu = 0;
                        int64_t cu = 0;
                        if (c0 + lane < pz) {
                            const int32_t u = pred[c0 + lane];
                            const int32_t wu = -2 - tr[u].qpos;  // worker of a finished task
                            nu = wu < ncpu ? 0 : 1 + wu - ncpu;
                            cu = dxc[u];
                        }
                        const int32_t cnt = min(kWave, pz - c0);
                        for (int32_t jj = 0; jj < cnt; jj++) {
                            const int32_t nj = read_lane(nu, jj);
                            const int64_t cj = (int64_t)read_lane64((uint64_t)cu, jj);
#pragma unroll
                            for (int k = 0; k < WPL; k++) {
                                const int32_t w = lane + k * kWave;
                                if ((w < ncpu ? 0 : 1 + w - ncpu) != nj) xk[k] += cj;
                            }
                        }
                    }
                }
                uint64_t best = ~0ull;
#pragma unroll
                for (int k = 0; k < WPL; k++) {
                    int32_t w = lane + k * kWave;
                    if (w < W) {
                        uint64_t cst = (uint64_t)(ld[k] + (w < ncpu ? e0 : e1) + xk[k]);
                        uint64_t key = cst << 11 | (uint64_t)w;
                        best = key < best ? key : best;
                    }
                }
                best = wave_min_u64(best);
                const int32_t ws = (int32_t)(best & 2047);
                const bool gpu = ws >= ncpu;
                int64_t xs = 0;
                if (data) {
                    int64_t mine = 0;
#pragma unroll
                    for (int k = 0; k < WPL; k++)
                        if (lane + k * kWave == ws) mine = xk[k];
                    xs = (int64_t)read_lane64((uint64_t)mine, ws & 63);
                    if (xs > INSP_MAX_TICK) status |= ST_XFER;
                }
                const int32_t ek = gpu ? e1 : e0;
                const int32_t dk = read_lane(gpu ? d_l.y : d_l.x, j);
#pragma unroll
                for (int k = 0; k < WPL; k++)
                    if (lane + k * kWave == ws) ld[k] += ek;
                const int32_t len = L.len[ws];
                const int32_t pos = len & 63;
                int32_t blk;
                if (pos == 0) {
                    nfree--;
                    blk = wg_load(&freeb[nfree]);
                    if (lane == 0) {
                        const int32_t nbw = L.nb[ws];
                        if (nbw < kLB) L.blist[ws * kLB + nbw] = blk;
                        else wblk[(int64_t)ws * maxb + nbw] = blk;
                        L.nb[ws] = nbw + 1;
                        L.last[ws] = blk;
                    }
                } else {
                    blk = L.last[ws];
                }
                const int32_t p = blk * 64 + pos;
                const uint64_t kw =
                    heft ? read_lane64(rk_l, j) << 21 | (M21 - (uint64_t)seq)
                         : (uint64_t)read_lane(ia_l, j) << 42 | (uint64_t)read_lane(ie_l, j) << 21 | (M21 - (uint64_t)seq);
                const uint64_t xw = (uint64_t)v << 42 | (uint64_t)(dk & M21) << 21 | (uint64_t)(ek & M21);
                const int32_t rs = read_lane(rs_l, j);
                if (lane == 0) {
                    if (blk < SLC) {
                        L.sk[p] = kw;
                        L.sx[p] = xw;
                        L.srs[p] = rs;
                    } else {
                        slots.k[p] = kw;
                        slots.x[p] = xw;
                        slots.rs[p] = rs;
                    }
                    tr[v].qpos = p;
                    tr[v].seq = seq;
                    // the dependency word is dead once a task is queued: it
                    // holds the time its inputs arrive (transfers start now)
                    if (data) tr[v].word = (unsigned long long)(t + xs);
                    // never lowered by pops: an upper bound for the block
                    if (lrule) barr[blk] = pos == 0 ? t + xs : max(barr[blk], (long long)(t + xs));
                    const uint64_t a0 = key_of(kw, slot0), a1 = key_of(kw, 1);
                    if (blk < SC) {
                        if (pos == 0) {
                            L.sum[2 * blk] = a0;
                            L.sum[2 * blk + 1] = a1;
                        } else {
                            atomicMax(&L.sum[2 * blk], (unsigned long long)a0);
                            atomicMax(&L.sum[2 * blk + 1], (unsigned long long)a1);
                        }
                    } else if (pos == 0) {
                        sums[2 * blk] = a0;
                        sums[2 * blk + 1] = a1;
                    } else {
                        wg_fetch_max(&sums[2 * blk], (unsigned long long)a0);
                        wg_fetch_max(&sums[2 * blk + 1], (unsigned long long)a1);
                    }
                    L.len[ws] = len + 1;
                    L.qest[ws] += ek;
                }
                seq++;
                nready++;
            }
        }
        PCLK(0);
        wg_fence();
        __builtin_amdgcn_wave_barrier();
        PCLK(1);
        // -------------------------------------------------------- regulate
        const int32_t observed = nready;
        if (A.policy == INSP_POLICY_INSPIRIT) {
            if (nready > peak) peak = nready;
            const int32_t dn = nready - prev_n;
            if ((dn < 0 ? -dn : dn) >= s_inc) {
                const int64_t dt = t - prev_t;
                prev_n = nready;
                prev_t = t;
                if (nready >= peak - dec_step) {
                    cnt = 0;
                    if (dn >= s_inc) {
                        const int64_t lhs = (int64_t)dn * k_den, rhs = (int64_t)k_num * dt;
                        if (dt == 0 || lhs > rhs) mode = INSP_MODE_ABILITY;
                        else if (lhs < rhs) mode = INSP_MODE_EFI;
                    }
                } else if ((int64_t)nready > (int64_t)peak - (int64_t)s_dec * cnt) {
                    mode = INSP_MODE_ABILITY;
                } else if ((int64_t)nready <= (int64_t)peak - (int64_t)s_dec * (cnt + 1) + cc) {
                    mode = INSP_MODE_EFI_LOC;
                    if ((int64_t)nready <= (int64_t)peak - (int64_t)s_dec * (cnt + 1)) cnt++;
                }
            }
        }
        const int pmode = A.policy == INSP_POLICY_FIFO ? INSP_MODE_FIFO
                        : A.policy == INSP_POLICY_ABILITY_ONLY ? INSP_MODE_ABILITY
                        : A.policy == INSP_POLICY_EFI_ONLY ? INSP_MODE_EFI
                        : A.policy == INSP_POLICY_LOCALITY ? INSP_MODE_EFI_LOC
                        : heft ? INSP_MODE_RANK : mode;
        // efficiency with locality: tasks whose inputs have arrived first
        const bool loc = data && pmode == INSP_MODE_EFI_LOC;
        const int ord = heft ? 3 : pmode == INSP_MODE_FIFO ? 2 : pmode == INSP_MODE_ABILITY ? 0 : 1;
        const int slot = ord == 1 ? 1 : 0;
        // ------------------------------------------------------------- pop
        int32_t popped = 0;
        for (int32_t w0 = 0; w0 < W; w0 += kWave) {
            const int32_t wl = w0 + lane;
            uint64_t mask = ballot(wl < W && L.run[wl] < 0 && L.len[wl] > 0);
            while (mask) {
                const int32_t w = w0 + (int32_t)__builtin_ctzll(mask);
                mask &= mask - 1;
                int32_t nb = L.nb[w], len = L.len[w];
                const int32_t last = L.last[w];
                int32_t bb = last;
                bool lsel = false;
                if (loc) {
                    // the arrival times are not in the keys.  A block whose
                    // latest input arrival has passed holds only tasks whose
                    // inputs are in place, so its efficiency maximum stands;
                    // the other blocks are scanned entry by entry
                    uint64_t bestk = 0;
                    int32_t bestb = -1;
                    const int32_t lp = (len - 1) & 63;
                    for (int32_t i0 = 0; i0 < nb; i0 += kWave) {
                        const int32_t i = i0 + lane;
                        uint64_t kk = 0;
                        int32_t b = -1;
                        bool mix = false;
                        if (i < nb) {
                            b = i < kLB ? L.blist[w * kLB + i] : wg_load(&wblk[(int64_t)w * maxb + i]);
                            if ((int64_t)wg_load(&barr[b]) <= t) kk = b < SC ? L.sum[2 * b + 1] : wg_load(&sums[2 * b + 1]);
                            else mix = true;
                        }
                        const uint64_t km = wave_max_u64(kk);
                        if (km > bestk) {
                            bestk = km;
                            bestb = read_lane(b, (int)__builtin_ctzll(ballot(kk == km && i < nb)));
                        }
                        uint64_t mm = ballot(mix);
                        while (mm) {
                            const int32_t bm = read_lane(b, (int)__builtin_ctzll(mm));
                            mm &= mm - 1;
                            uint64_t ke = 0;
                            if (lane < (bm == last ? lp + 1 : 64)) {
                                const uint64_t kv = bm < SLC ? L.sk[bm * 64 + lane] : wg_load(&slots.k[bm * 64 + lane]);
                                const uint64_t xv = bm < SLC ? L.sx[bm * 64 + lane] : wg_load(&slots.x[bm * 64 + lane]);
                                if ((int64_t)wg_load(&tr[(int32_t)(xv >> 42)].word) <= t) ke = key_of(kv, 1);
                            }
                            const uint64_t kme = wave_max_u64(ke);
                            if (kme > bestk) {
                                bestk = kme;
                                bestb = bm;
                            }
                        }
                    }
                    if (bestb >= 0) {
                        bb = bestb;
                        lsel = true;
                    }
                }
                if (!lsel && nb > 1) {
                    uint64_t bk = 0;
                    int32_t bid = -1;
                    for (int32_t i0 = 0; i0 < nb; i0 += kWave) {
                        const int32_t i = i0 + lane;
                        if (i < nb) {
                            const int32_t b = i < kLB ? L.blist[w * kLB + i] : wg_load(&wblk[(int64_t)w * maxb + i]);
                            const uint64_t k = b < SC ? L.sum[2 * b + slot] : wg_load(&sums[2 * b + slot]);
                            if (k > bk) {
                                bk = k;
                                bid = b;
                            }
                        }
                    }
                    const uint64_t km = wave_max_u64(bk);
                    const uint64_t wm = ballot(bk == km && bid >= 0);
                    bb = read_lane(bid, (int)__builtin_ctzll(wm));
                }
                const int32_t lastpos = (len - 1) & 63;
                const int32_t cntb = bb == last ? lastpos + 1 : 64;
                const bool ok = lane < cntb;
                const int32_t eb = bb * 64, el = last * 64;
                const bool okl = last != bb && lane <= lastpos;
                uint64_t kw = 0, xw = 0, kl = 0, xl = 0;
                int32_t rw = 0, rl = 0;
                if (ok) {
                    if (bb < SLC) {
                        kw = L.sk[eb + lane];
                        xw = L.sx[eb + lane];
                        rw = L.srs[eb + lane];
                    } else {
                        kw = wg_load(&slots.k[eb + lane]);
                        xw = wg_load(&slots.x[eb + lane]);
                        rw = wg_load(&slots.rs[eb + lane]);
                    }
                }
                if (okl) {
                    if (last < SLC) {
                        kl = L.sk[el + lane];
                        xl = L.sx[el + lane];
                        rl = L.srs[el + lane];
                    } else {
                        kl = wg_load(&slots.k[el + lane]);
                        xl = wg_load(&slots.x[el + lane]);
                        rl = wg_load(&slots.rs[el + lane]);
                    }
                }
                bool here = true;
                if (lsel && ok) here = (int64_t)wg_load(&tr[(int32_t)(xw >> 42)].word) <= t;
                const uint64_t key = ok && here ? key_of(kw, ord) : 0;
                const uint64_t km = wave_max_u64(key);
                const int win = (int)__builtin_ctzll(ballot(key == km && ok));
                const uint64_t vk = read_lane64(kw, win), vx = read_lane64(xw, win);
                const int32_t vr = read_lane(rw, win);
                const int32_t p = eb + win;
                const int32_t q = el + lastpos;
                const int32_t v = (int32_t)(vx >> 42);
                const int32_t dk = (int32_t)((vx >> 21) & M21), ek = (int32_t)(vx & M21);
                uint64_t mk = 0, mx = 0;
                int32_t mr = 0;
                if (p != q) {
                    if (last == bb) {
                        mk = read_lane64(kw, lastpos);
                        mx = read_lane64(xw, lastpos);
                        mr = read_lane(rw, lastpos);
                    } else {
                        mk = read_lane64(kl, lastpos);
                        mx = read_lane64(xl, lastpos);
                        mr = read_lane(rl, lastpos);
                    }
                    if (lane == 0) {
                        if (bb < SLC) {
                            L.sk[p] = mk;
                            L.sx[p] = mx;
                            L.srs[p] = mr;
                        } else {
                            slots.k[p] = mk;
                            slots.x[p] = mx;
                            slots.rs[p] = mr;
                        }
                        tr[(int32_t)(mx >> 42)].qpos = p;
                        // the moved entry keeps block bb's arrival bound valid
                        if (lrule && last != bb) barr[bb] = max(barr[bb], barr[last]);
                    }
                }
                len--;
                const bool freed = (len & 63) == 0;
                int32_t newlast = last;
                if (freed) {
                    if (lane == 0) freeb[nfree] = last;
                    nfree++;
                    nb--;
                    newlast = nb <= 0 ? -1 : nb - 1 < kLB ? L.blist[w * kLB + nb - 1]
                                                         : wg_load(&wblk[(int64_t)w * maxb + nb - 1]);
                }
                if (!(bb == last && freed)) {
                    // block bb after the removal: the winner's slot holds the
                    // moved entry; if bb is the last block its final slot left
                    const uint64_t nk = (p != q && lane == win) ? mk : kw;
                    const bool valid = ok && !(bb == last && lane == lastpos);
                    const uint64_t s0 = wave_max_u64(valid ? key_of(nk, slot0) : 0);
                    const uint64_t s1 = wave_max_u64(valid ? key_of(nk, 1) : 0);
                    if (lane == 0) {
                        if (bb < SC) {
                            L.sum[2 * bb] = s0;
                            L.sum[2 * bb + 1] = s1;
                        } else {
                            sums[2 * bb] = s0;
                            sums[2 * bb + 1] = s1;
                        }
                    }
                }
                if (last != bb && !freed) {
                    // the last block lost its final entry to bb
                    const bool valid = okl && lane != lastpos;
                    const uint64_t s0 = wave_max_u64(valid ? key_of(kl, slot0) : 0);
                    const uint64_t s1 = wave_max_u64(valid ? key_of(kl, 1) : 0);
                    if (lane == 0) {
                        if (last < SC) {
                            L.sum[2 * last] = s0;
                            L.sum[2 * last + 1] = s1;
                        } else {
                            sums[2 * last] = s0;
                            sums[2 * last + 1] = s1;
                        }
                    }
                }
                // fixed keys carry the rank or the transitive attributes, not
                // the out-degree
                const int32_t deg = skey ? tr[v].ia : (int32_t)(vk >> 42);
                const int32_t iep = tattr ? tie[v] : heft ? wg_load(&tr[v].iev) : (int32_t)((vk >> 21) & M21);
                // a task whose inputs are still moving holds the worker until
                // they arrive
                int64_t s0 = t;
                if (data) s0 = max(t, (int64_t)wg_load(&tr[v].word));
                if (lane == 0) {
                    L.len[w] = len;
                    L.nb[w] = nb;
                    L.last[w] = newlast;
                    L.run[w] = v;
                    L.fin[w] = s0 + dk;
                    L.expend[w] = s0 + ek;
                    L.qest[w] -= ek;
                    L.rsr[w] = vr;
                    L.dgr[w] = deg;
                    put_record(&tr[v], s0, dk, w, iep, pmode);  // running, then done
                }
                if constexpr (kPrefetch) {
                    // the running task's first successors, read now and used
                    // when it completes
                    if (lane == (w & 63)) {
#pragma unroll
                        for (int k = 0; k < PW; k++)
                            if (k == (w >> 6)) {
#pragma unroll
                                for (int j = 0; j < kPF; j++) pf[k][j] = j < deg ? col[vr + j] : 0;
                            }
                    }
                }
                nready--;
                popped++;
            }
        }
        PCLK(2);
        if (A.trace && lane == 0 && events <= max_events) {
            insp_trace_rec rec;
            rec.t = t;
            rec.nready = observed;
            rec.mode = pmode;
            rec.cnt = cnt;
            rec.peak = peak;
            rec.pushed = r;
            rec.popped = popped;
            A.trace[(d.toff - A.base) + di + events - 1] = rec;
        }
        if (done == n) break;
        // --------------------------------------------------------- advance
        uint64_t tm = ~0ull;
        for (int32_t w = lane; w < W; w += kWave)
            if (L.run[w] >= 0 && (uint64_t)L.fin[w] < tm) tm = (uint64_t)L.fin[w];
        tm = wave_min_u64(tm);
        if (tm == ~0ull) {
            status |= ST_HANG;
            break;
        }
        t = (int64_t)tm;
        PCLK(3);
        // --------------------------------------------------------- release
        r = 0;
        int32_t nc = 0, nseg = 0, ndone = 0;
        for (int32_t w0 = 0; w0 < W; w0 += kWave) {
            const int32_t wl = w0 + lane;
            const bool fin_now = wl < W && L.run[wl] >= 0 && L.fin[wl] == t;
            uint64_t mask = ballot(fin_now);
            const int32_t c_l = fin_now ? L.run[wl] : -1;
            if (fin_now) L.run[wl] = -1;
            while (mask) {
                const int l = (int)__builtin_ctzll(mask);
                mask &= mask - 1;
                const int32_t w = w0 + l;
                const int32_t c = read_lane(c_l, l);
                done++;
                ndone++;
                const int32_t deg = L.dgr[w], rs = L.rsr[w];
                const int32_t r0 = r;
                const unsigned long long dec = 0ull - ((1ull << 43) + (unsigned long long)c);
                for (int32_t e0 = 0; e0 < deg; e0 += kWave) {
                    const int32_t e = e0 + lane;
                    const bool ok = e < deg;
                    int32_t s = 0;
                    if constexpr (kPrefetch) {
                        if (e0 == 0) {
#pragma unroll
                            for (int k = 0; k < PW; k++)
                                if (k == (w >> 6)) {
#pragma unroll
                                    for (int j = 0; j < kPF; j++) {
                                        const int32_t y = read_lane(pf[k][j], w & 63);
                                        if (lane == j) s = y;
                                    }
                                }
                        }
                        if (ok && e >= kPF) s = col[rs + e];
                    } else {
                        if (ok) s = col[rs + e];
                    }
                    // one wave owns the DAG's words and a row's successors are
                    // distinct (rows are deduplicated), so a plain
                    // read-modify-write replaces the atomic (a wave's accesses
                    // to one address complete in program order)
                    uint64_t old = 0;
                    if (ok) {
                        old = dep[s];
                        dep[s] = old + dec;
                    }
                    const int32_t nr = (int32_t)(old >> 43) - 1;
                    const bool rdy = ok && nr == 0, cd = ok && nr == 1;
                    const uint64_t m1 = ballot(rdy), m2 = ballot(cd);
                    if (rdy) {
                        const int32_t pos = r + lanes_below(m1);
                        fbuf[pos] = s;
                        if (pos < kFC) L.fr0[pos] = s;
                    }
                    if (cd) {
                        const int32_t pos = nc + lanes_below(m2);
                        if (pos < kCC) {
                            L.cs[pos] = s;
                            L.cu[pos] = (int32_t)((old + dec) & M43);
                        } else {
                            fbuf[2 * n + pos] = s;
                        }
                    }
                    r += __popcll(m1);
                    nc += __popcll(m2);
                }
                if (r > r0) {
                    if (lane == 0) L.seg[nseg] = r;
                    nseg++;
                }
            }
        }
        PCLK(4);
        wg_fence();
        __builtin_amdgcn_wave_barrier();
        PCLK(5);
        // successors left with one unfinished predecessor raise its IE.  The
        // predecessor is named by the atomic's result (rem 1, remaining sum);
        // that result is final unless a later completion of the same event
        // made the successor ready, in which case it is not a candidate.
        const bool single = ndone == 1;
        merged = false;
        staged = false;
        if (nc <= kWave && r <= kFC) {
            // one round trip: candidate records and the next push's frontier rows
            const bool hc = lane < nc;
            const int32_t s = hc ? L.cs[lane] : 0;
            int32_t u = hc ? L.cu[lane] : -1;
            if (hc && !single)
                for (int32_t k = 0; k < r; k++)
                    if (L.fr0[k] == s) {
                        u = -1;
                        break;
                    }
            staged = r <= kWave;
            const bool hf = staged && lane < r;
            const int32_t fv = hf ? L.fr0[lane] : 0;
            int32_t tu = 0, ts = 0, iu = 0, qu = -1, au = 0, sq = 0;
            if (u >= 0) {
                tu = tr[u].tau;
                ts = tr[s].tau;
                iu = wg_load(&tr[u].iev);
                qu = wg_load(&tr[u].qpos);
                au = tr[u].ia;
                sq = wg_load(&tr[u].seq);
            }
            int2 fe = make_int2(1, 1), fd = make_int2(1, 1);
            int32_t fa = 0, frs = 0, fie = 0;
            if (hf) {
                fe = est2[fv];
                fd = dur2[fv];
                fa = tr[fv].ia;
                frs = tr[fv].rs;
                fie = wg_load(&tr[fv].iev);
            }
            const bool cond = u >= 0 && (int64_t)tu + ts <= (int64_t)U;
            // several successors may name the same predecessor: the first lane
            // applies all of its increments
            int32_t mult = 0;
            bool lead = cond;
            for (int32_t j = 0; j < nc; j++) {
                const int32_t uj = read_lane(u, j);
                const int32_t cj = read_lane(cond ? 1 : 0, j);
                if (cj && cond && uj == u) {
                    mult++;
                    if (j < lane) lead = false;
                }
            }
            if (lead) {
                const int32_t nie = iu + mult;
                tr[u].iev = nie;
                if (qu >= 0 && !skey) {
                    const uint64_t nk = (uint64_t)au << 42 | (uint64_t)nie << 21 | (M21 - (uint64_t)sq);
                    const int32_t bk = qu >> 6;
                    if (bk < SLC) L.sk[qu] = nk;
                    else slots.k[qu] = nk;
                    if (bk < SC) {
                        atomicMax(&L.sum[2 * bk], (unsigned long long)key_of(nk, slot0));
                        atomicMax(&L.sum[2 * bk + 1], (unsigned long long)key_of(nk, 1));
                    } else {
                        wg_fetch_max(&sums[2 * bk], (unsigned long long)key_of(nk, slot0));
                        wg_fetch_max(&sums[2 * bk + 1], (unsigned long long)key_of(nk, 1));
                    }
                }
            }
            // a raised predecessor that became ready in this very event: its
            // staged row must carry the new IE
            uint64_t lm = ballot(lead && qu == -1);
            while (lm) {
                const int l = (int)__builtin_ctzll(lm);
                lm &= lm - 1;
                const int32_t uu = read_lane(u, l), kk = read_lane(mult, l);
                const uint64_t fm = ballot(hf && fv == uu);
                if (fm && lane == (int)__builtin_ctzll(fm)) fie += kk;
            }
            int32_t pos = lane;
            if (nseg > 1 && hf) {
                // rank of this entry among the ascending runs of the completions
                int32_t rank = 0, lo = 0;
                for (int32_t g = 0; g < nseg; g++) {
                    const int32_t hi = L.seg[g];
                    if (lane >= lo && lane < hi) {
                        rank += lane - lo;
                    } else {
                        int32_t a = lo, b = hi;
                        while (a < b) {
                            const int32_t mid = (a + b) >> 1;
                            if (L.fr0[mid] < fv) a = mid + 1;
                            else b = mid;
                        }
                        rank += a - lo;
                    }
                    lo = hi;
                }
                pos = rank;
            }
            if (!staged && nseg > 1) {
                // frontier too large to stage: merge ids in LDS, rows loaded at push
                for (int32_t i = lane; i < r; i += kWave) {
                    const int32_t x = L.fr0[i];
                    int32_t rank = 0, lo = 0;
                    for (int32_t g = 0; g < nseg; g++) {
                        const int32_t hi = L.seg[g];
                        if (i >= lo && i < hi) {
                            rank += i - lo;
                        } else {
                            int32_t a = lo, b = hi;
                            while (a < b) {
                                const int32_t mid = (a + b) >> 1;
                                if (L.fr0[mid] < x) a = mid + 1;
                                else b = mid;
                            }
                            rank += a - lo;
                        }
                        lo = hi;
                    }
                    L.fr1[rank] = x;
                }
                merged = true;
            }
            if (hf) {
                L.pre[pos] = fv;
                L.pre[64 + pos] = fe.x;
                L.pre[128 + pos] = fe.y;
                L.pre[192 + pos] = fd.x;
                L.pre[256 + pos] = fd.y;
                L.pre[320 + pos] = fa;
                L.pre[384 + pos] = frs;
                L.pre[448 + pos] = fie;
            }
        } else {
            for (int32_t i0 = 0; i0 < nc; i0 += kWave) {
                const int32_t i = i0 + lane;
                if (i < nc) {
                    const int32_t s = i < kCC ? L.cs[i] : wg_load(&fbuf[2 * n + i]);
                    int32_t u = -1;
                    if (single && i < kCC) {
                        u = L.cu[i];
                    } else {
                        const uint64_t wd = wg_load(&dep[s]);
                        if ((wd >> 43) == 1) u = (int32_t)(wd & M43);
                    }
                    if (u >= 0) {
                        const int32_t tu = tr[u].tau, ts = tr[s].tau;
                        const int32_t pu = wg_load(&tr[u].qpos);
                        if ((int64_t)tu + ts <= (int64_t)U) {
                            wg_fetch_add(&tr[u].iev, 1);
                            if (pu >= 0 && !skey) {
                                const int32_t bk = pu >> 6;
                                const uint64_t nk = (bk < SLC ? (uint64_t)atomicAdd(&L.sk[pu], 1ull << 21)
                                                              : (uint64_t)wg_fetch_add(&slots.k[pu], 1ull << 21)) +
                                                    (1ull << 21);
                                if (bk < SC) {
                                    atomicMax(&L.sum[2 * bk], (unsigned long long)key_of(nk, slot0));
                                    atomicMax(&L.sum[2 * bk + 1], (unsigned long long)key_of(nk, 1));
                                } else {
                                    wg_fetch_max(&sums[2 * bk], (unsigned long long)key_of(nk, slot0));
                                    wg_fetch_max(&sums[2 * bk + 1], (unsigned long long)key_of(nk, 1));
                                }
                            }
                        }
                    }
                }
            }
            wg_fence();
            // several completions: merge their ascending runs by rank
            if (nseg > 1) {
                const bool in_lds = r <= kFC;
                for (int32_t i0 = 0; i0 < r; i0 += kWave) {
                    const int32_t i = i0 + lane;
                    if (i < r) {
                        const int32_t x = in_lds ? L.fr0[i] : fbuf[i];
                        int32_t rank = 0, lo = 0;
                        for (int32_t g = 0; g < nseg; g++) {
                            const int32_t hi = L.seg[g];
                            if (i >= lo && i < hi) {
                                rank += i - lo;
                            } else {
                                int32_t a = lo, b = hi;  // count of run g below x
                                while (a < b) {
                                    const int32_t mid = (a + b) >> 1;
                                    const int32_t y = in_lds ? L.fr0[mid] : fbuf[mid];
                                    if (y < x) a = mid + 1;
                                    else b = mid;
                                }
                                rank += a - lo;
                            }
                            lo = hi;
                        }
                        if (in_lds) L.fr1[rank] = x;
                        else fbuf[n + rank] = x;
                    }
                }
                merged = true;
            }
        }
        PCLK(7);
        wg_fence();
        __builtin_amdgcn_wave_barrier();
        PCLK(8);
    }
#ifdef INSP_PHASE_CLOCKS
    if (lane == 0 && d.id < 8192)
        for (int i = 0; i < 32; i++) g_phase_clk[d.id * 32 + i] = pc[i];
#endif
    if (lane == 0) {
        A.makespan[di] = (status & ST_HANG) ? -1 : t;
        if (A.n_events) A.n_events[di] = events;
        if (status) atomicOr(&A.stat[2 * d.id], status);
        A.stat[2 * d.id + 1] = events;
    }
}

// ---------------------------------------------------------------------------
// Machines of at most 64 workers: lane w holds worker w's state in registers
// (running task, its finish and expected-end times, queue length, block count,
// last block, the running task's row and first successors), so pushes, pops
// and the advance read no memory for it.  Same event order and results as the
// general loop above, with two differences in the queue:
//   - 32-bit keys.  IA and IE take `a` bits each (a = bit length of the DAG's
//     largest out-degree; IE <= IA) and the push order `s` bits (s = bit length
//     of n - 1), under a valid bit.  Each entry keeps both rules' keys,
//       kA = V | IA << (a+s) | IE << s | (2^s-1-seq)   (ability; under the
//                                                        FIFO policy V | (2^s-1-seq))
//       kE = V | IE << (a+s) | IA << s | (2^s-1-seq)   (efficiency),
//     so a pop compares plain words.  A DAG whose keys need more than 32 bits
//     runs the general loop instead.
//   - How a pop finds its maximum: a worker with at most kScan blocks has
//     every lane scan its column of all of the worker's blocks, then one wave
//     max; with more blocks, per-block maxima pick the block first.  Every
//     slot without a live entry holds zero keys (all blocks are zeroed when
//     the DAG starts, and a pop zeroes the slot it empties), so scans read
//     whole blocks unpredicated: valid keys carry the top bit.  Maxima of
//     blocks held in LDS are rebuilt lazily: a pop only marks the blocks it
//     touched stale; pushes and IE increments keep raising them with atomicMax
//     (which a later rebuild overwrites), and a many-block pop rebuilds the
//     stale ones of its worker before comparing.  Maxima kept in global memory
//     (block ids >= sum_cap) are rebuilt at once.
constexpr int kScan = 16;  // the most a launch may scan (tune key "scan=")

// Key layout of one DAG.
struct KeyFmt {
    uint32_t sa, sb;    // shifts of the second and first key fields (s, a + s)
    uint32_t smask;     // 2^s - 1
    uint32_t amask;     // 2^a - 1
    bool fifo;          // kA holds the FIFO key
    __device__ __forceinline__ uint32_t ka(uint32_t ia, uint32_t ie, uint32_t seq) const {
        return 0x80000000u | (fifo ? 0u : ia << sb | ie << sa) | (smask - seq);
    }
    __device__ __forceinline__ uint32_t ke(uint32_t ia, uint32_t ie, uint32_t seq) const {
        return 0x80000000u | ie << sb | ia << sa | (smask - seq);
    }
    // increments of kA and kE when IE grows by one
    __device__ __forceinline__ uint32_t da() const { return fifo ? 0u : 1u << sa; }
    __device__ __forceinline__ uint32_t de() const { return 1u << sb; }
};

// Queue keys of the one-wave loop.  Direct attributes: two 32-bit rule keys
// per entry, kA (ability, or FIFO) and kE (efficiency), each raised in place
// when the task's IE grows.  Fixed keys (HEFT ranks, transitive attributes):
// one 64-bit key per entry in the general loop's format, from which key_of
// derives the rule keys when an entry is read (zero stays zero: an empty slot).
template <bool FIX>
struct Keys {
    using T = typename std::conditional<FIX, unsigned long long, uint32_t>::type;
    T *ka, *ke;  // LDS keys [64 * key_cap]: kA and kE, or (fixed) ka the key itself
    T *mx;       // [2 * sum_cap]: the two rule maxima of each block summarised in LDS
    int o0;      // fixed keys: the rule of maximum 0 (0 ability, 2 FIFO, 3 rank)
    __device__ __forceinline__ T rule(uint64_t raw, int r) const {
        if constexpr (FIX) return raw ? key_of(raw, r ? 1 : o0) : 0ull;
        else return (uint32_t)(raw >> (r ? 32 : 0));
    }
    // rule-r key of the entry in LDS slot p
    __device__ __forceinline__ T lds(int32_t p, int r) const {
        if constexpr (FIX) return rule(ka[p], r);
        else return (r ? ke : ka)[p];
    }
};

__device__ __forceinline__ uint32_t wave_max_k(uint32_t x) { return wave_max_u32f(x); }
__device__ __forceinline__ unsigned long long wave_max_k(unsigned long long x) { return wave_max_u64f(x); }

// Rule-`r` keys of block b, one per lane (zero in empty slots).  b is
// wave-uniform: the choice between LDS and global memory is a scalar branch,
// and the global side waits for its load itself, so the LDS side carries no
// wait for outstanding global accesses.
template <bool FIX>
__device__ __forceinline__ typename Keys<FIX>::T block_keys(const SlotPool &slots, const Keys<FIX> &K, int32_t slc,
                                                            int32_t b, int r) {
    const int lane = lane_id();
    typename Keys<FIX>::T k;
    if (b < slc) {
        k = K.lds(b * 64 + lane, r);
    } else {
        const uint64_t raw = wg_load(&slots.k[b * 64 + lane]);
        settle(raw);
        k = K.rule(raw, r);
    }
    return k;
}

// Best rule-R key in column `lane` of the listed blocks (bits of `m` select
// lanes of `bl`, which hold block ids), four loads in flight at a time;
// FROM_LDS picks where the blocks' slots live.
template <bool FIX, bool FROM_LDS, int R>
__device__ __forceinline__ void scan_columns(const SlotPool &slots, const Keys<FIX> &K, uint64_t m, int32_t bl,
                                             typename Keys<FIX>::T &best, int32_t &bp) {
    const int lane = lane_id();
    const int32_t b_last = read_lane(bl, 63 - (int)__builtin_clzll(m | 1));  // any listed block
    while (m) {
        typename Keys<FIX>::T kk[4];
        int32_t pp[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            int32_t b = b_last;  // padding re-reads a listed block: no effect on the max
            if (m) {
                b = read_lane(bl, (int)__builtin_ctzll(m));
                m &= m - 1;
            }
            pp[u] = b * 64 + lane;
            kk[u] = FROM_LDS ? K.lds(pp[u], R) : K.rule(wg_load(&slots.k[pp[u]]), R);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (kk[u] > best) {
                best = kk[u];
                bp = pp[u];
            }
        }
    }
}

// Rebuild both maxima of block b from its first `cnt` entries (wave-wide).
template <bool FIX>
__device__ __forceinline__ void rebuild_max(const SlotPool &slots, const Keys<FIX> &K, const Lds &L,
                                            unsigned long long *sums, int32_t slc, int32_t sc, int32_t b) {
    const int lane = lane_id();
    const auto s0 = wave_max_k(block_keys<FIX>(slots, K, slc, b, 0));
    const auto s1 = wave_max_k(block_keys<FIX>(slots, K, slc, b, 1));
    if (lane == 0) {
        if (b < sc) {
            K.mx[2 * b] = s0;
            K.mx[2 * b + 1] = s1;
            L.stale[b] = 0;
        } else {
            sums[2 * b] = s0;
            sums[2 * b + 1] = s1;
        }
    }
}

// FIX = false: direct attributes on 32-bit keys; returns false, having changed
// nothing the general loop relies on, when the DAG's keys do not fit.
// FIX = true: fixed 64-bit keys (HEFT ranks or transitive attributes); the
// tasks' direct IE is still kept up to date for the records.
// DATA = true: the data model (A.data_bw > 0), as the general loop runs it: a
// push adds each worker's input transfer ticks to its cost and records the
// task's input arrival time, a pop starts its task when the inputs are in,
// and the efficiency-with-locality rule prefers tasks whose inputs are.
template <bool FIX, bool DATA>
__device__ bool sim_lane(const SimArgs &A, int32_t di, const Lds &L) {
    using KT = typename Keys<FIX>::T;
    const int lane = lane_id();
    const DagDesc d = A.desc[di];
    const int32_t n = d.n, ncpu = d.n_cpu, W = d.n_cpu + d.n_gpu;
    int32_t status = A.stat[2 * d.id];
    if (n == 0 || status != 0) {
        if (lane == 0) {
            A.makespan[di] = status ? -1 : 0;
            if (A.n_events) A.n_events[di] = 0;
        }
        return true;
    }
    const int64_t ub = d.toff - A.base;
    const int32_t *col = A.col + d.eoff;
    TaskRec *tr = A.tr + d.toff;
    unsigned long long *dep = A.dep + d.toff;
    int32_t *fbuf = A.fbuf + 3 * d.toff;      // [0,n) runs, [n,2n) merged, [2n,3n) candidates
    const int2 *est2 = reinterpret_cast<const int2 *>(A.est) + ub;
    const int2 *dur2 = reinterpret_cast<const int2 *>(A.dur) + ub;
    const SlotPool slots = A.slots.at(64 * d.blk_off);
    unsigned long long *sums = A.sums + 2 * d.blk_off;
    int32_t *wblk = A.paux + d.wl_off;
    int32_t *freeb = A.paux + A.freeb_base + d.blk_off;
    const int32_t maxb = d.maxb;
    const int32_t SC = A.sum_cap;
    const int32_t kLB = A.lb;
    const int32_t SLC = A.slot_cap;  // blocks [0, SLC) keep their entries' payload in LDS
    const int32_t SLK = A.key_cap;   // blocks [0, SLK) (SLK >= SLC) keep their keys in LDS

    // initial frontier (tasks without predecessors, ascending) and the
    // largest out-degree, which sizes the key fields
    int32_t r = 0;
    uint32_t mdeg = 0;
    for (int32_t i0 = 0; i0 < n; i0 += kWave) {
        int32_t i = i0 + lane;
        bool ok = false;
        if (i < n) {
            ok = (dep[i] >> 43) == 0;
            mdeg = max(mdeg, (uint32_t)tr[i].ia);
        }
        uint64_t mk = ballot(ok);
        if (ok) {
            int32_t pos = r + lanes_below(mk);
            fbuf[pos] = i;
            if (pos < kFC) L.fr0[pos] = i;
        }
        r += __popcll(mk);
    }
    mdeg = wave_max_u32f(mdeg);
    const uint32_t abits = mdeg == 0 ? 1 : 32 - __clz(mdeg);
    const uint32_t sbits = n <= 1 ? 1 : 32 - __clz(n - 1);
    if (!FIX && 1 + 2 * abits + sbits > 32) return false;
    KeyFmt kf;
    kf.sa = sbits;
    kf.sb = abits + sbits;
    kf.smask = (1u << sbits) - 1;
    kf.amask = (1u << abits) - 1;
    kf.fifo = A.policy == INSP_POLICY_FIFO;
    const bool heft = FIX && A.policy == INSP_POLICY_HEFT;
    const bool tattr = FIX && A.attr_mode == INSP_ATTR_TRANSITIVE;
    const int64_t *rk = A.rank + d.toff;
    const int32_t *tia = A.tia + d.toff, *tie = A.tie + d.toff;
    Keys<FIX> K;
    K.ka = reinterpret_cast<KT *>(L.sk);
    K.ke = FIX ? nullptr : K.ka + 64 * SLK;  // the two 32-bit arrays fill the 64-bit key storage
    K.mx = reinterpret_cast<KT *>(L.sum);
    K.o0 = A.policy == INSP_POLICY_FIFO ? 2 : heft ? 3 : 0;
    const int32_t U = A.dag_u[d.id];
    // data model: inputs move between memory nodes (the host for the CPU
    // workers, one per GPU worker)
    const int32_t *prp = A.pprp + d.toff + d.id, *pred = A.ppred + d.eoff;
    int32_t *dxc = A.dxc + d.toff;
    long long *barr = A.barr + d.blk_off;
    // block arrival bounds matter only where the locality rule can be used
    const bool lrule = DATA && (A.policy == INSP_POLICY_INSPIRIT || A.policy == INSP_POLICY_LOCALITY);
    const int32_t mynode = lane < ncpu ? 0 : 1 + lane - ncpu;  // this lane's worker's memory node
    if constexpr (DATA)  // each output's transfer ticks, once per run (no division at the pushes)
        for (int32_t i = lane; i < n; i += kWave)
            dxc[i] = (int32_t)(((int64_t)1024 * A.dkib[d.toff + i] + A.data_bw - 1) / A.data_bw);

    const int32_t s_inc = A.s_inc > 0 ? A.s_inc : max(1, (W + 3) / 4);
    const int32_t s_dec = A.s_dec > 0 ? A.s_dec : max(1, (W + 1) / 2);
    const int32_t dec_step = A.dec_step > 0 ? A.dec_step : s_dec;
    const int32_t cc = A.c >= 0 ? A.c : s_dec / 2;
    const bool kset = A.k_num > 0 && A.k_den > 0;
    const int32_t k_num = kset ? A.k_num : W;
    const int32_t k_den = kset ? A.k_den : A.dag_taubar[d.id];
    const int32_t max_events = A.max_events > 0 ? A.max_events : n + 1;

    // this lane's worker
    const bool wok = lane < W;
    int32_t run = -1, len = 0, nb = 0, last = -1, rsr = 0, dgr = 0;
    int64_t fin = 0, expend = 0, qest = 0, st0 = 0;  // st0: the running task's start
    int32_t pf[kPF];
#pragma unroll
    for (int j = 0; j < kPF; j++) pf[j] = 0;

    // free block ids, lowest first: a stack in LDS below sum_cap, one in
    // global memory above it
    const int32_t nl = min(d.nblk, SC);
    for (int32_t i = lane; i < nl; i += kWave) L.fstk[i] = nl - 1 - i;
    for (int32_t i = lane; i < d.nblk - nl; i += kWave) freeb[i] = d.nblk - 1 - i;
    int32_t nfl = nl, nfg = d.nblk - nl;
    // every slot starts empty (zero keys)
    for (int32_t b = 0; b < d.nblk; b++) {
        if (b < SLK) {
            K.ka[b * 64 + lane] = 0;
            if constexpr (!FIX) K.ke[b * 64 + lane] = 0;
        } else {
            slots.k[b * 64 + lane] = 0;
        }
    }

    bool merged = false, staged = false;
    wg_fence();

    int64_t t = 0, prev_t = 0;
    int32_t nready = 0, events = 0, done = 0, seq = 0;
    int32_t peak = 0, prev_n = 0, cnt = 0;
    int mode = INSP_MODE_ABILITY;
#ifdef INSP_PHASE_CLOCKS
    unsigned long long pc[32] = {0}, pc_last = clock64();
#endif

    for (;;) {
        PCLK(9);
        if (++events > max_events) {
            status |= ST_HANG;
            break;
        }
        // ------------------------------------------------------------ push
        // this lane's load: free time (now, or the running task's expected
        // end) plus the estimates queued on it
        int64_t ld = 0;
        if (wok) ld = (run >= 0 && expend > t ? expend : t) + qest;
        for (int32_t i0 = 0; i0 < r; i0 += kWave) {
            const int32_t idx = i0 + lane;
            const bool ok = idx < r;
            int32_t v_l = 0;
            int2 e_l = make_int2(1, 1), d_l = make_int2(1, 1);
            int32_t ia_l = 0, ie_l = 0, rs_l = 0;
            if (staged) {
                if (ok) {
                    v_l = L.pre[idx];
                    e_l = make_int2(L.pre[64 + idx], L.pre[128 + idx]);
                    d_l = make_int2(L.pre[192 + idx], L.pre[256 + idx]);
                    ia_l = L.pre[320 + idx];
                    rs_l = L.pre[384 + idx];
                    ie_l = L.pre[448 + idx];
                }
            } else {
                if (ok) {
                    if (r <= kFC) v_l = merged ? L.fr1[idx] : L.fr0[idx];
                    else v_l = merged ? fbuf[n + idx] : fbuf[idx];
                }
                if (ok) {
                    e_l = est2[v_l];
                    d_l = dur2[v_l];
                    const int4 fx = *reinterpret_cast<const int4 *>(&tr[v_l].iev);  // IE, IA, tau, first edge
                    ie_l = fx.x;
                    ia_l = fx.y;
                    rs_l = fx.w;
                    // fixed keys: the rank (low and high words), or the transitive attributes
                    if (heft) {
                        const int64_t rv = rk[v_l];
                        ia_l = (int32_t)(uint32_t)rv;
                        ie_l = (int32_t)(uint32_t)((uint64_t)rv >> 32);
                    } else if (tattr) {
                        ia_l = tia[v_l];
                        ie_l = tie[v_l];
                    }
                }
            }
            if (ballot(ok && (d_l.x < 1 || d_l.x > INSP_MAX_TICK || d_l.y < 1 || d_l.y > INSP_MAX_TICK)))
                status |= ST_DUR;
            PCLK(16);
            const int32_t cntj = min(kWave, r - i0);
            int32_t pq = 0, sqj = 0, wsj = 0;  // lane j: slot, push order and worker of task j
            int64_t xsj = 0;                     // ... and (data model) its input transfer ticks
            for (int32_t j = 0; j < cntj; j++) {
                const int32_t e0 = read_lane(e_l.x, j), e1 = read_lane(e_l.y, j);
                // DMDA's transfer term: ticks to move the inputs whose home
                // node is not this lane's worker's (an item stays where it was made)
                int64_t xk = 0;
                if constexpr (DATA) {
                    const int32_t v = read_lane(v_l, j);
                    const int32_t pa = prp[v], pz = prp[v + 1];
                    for (int32_t c0 = pa; c0 < pz; c0 += kWave) {
                        int32_t nu = 0, cu = 0;
                        if (c0 + lane < pz) {
                            const int32_t u = pred[c0 + lane];
                            const int32_t wu = -2 - tr[u].qpos;  // worker of a finished task
                            nu = wu < ncpu ? 0 : 1 + wu - ncpu;
                            cu = dxc[u];
                        }
                        const int32_t cn = min(kWave, pz - c0);
                        for (int32_t jj = 0; jj < cn; jj++) {
                            const int32_t nj = read_lane(nu, jj), cj = read_lane(cu, jj);
                            if (mynode != nj) xk += cj;
                        }
                    }
                }
                // least expected termination, ties to the lower worker: a
                // 32-bit key (cost - t) << 6 | worker while it fits
                const int64_t rc = ld + (lane < ncpu ? e0 : e1) + xk - t;
                const uint32_t k32 = wok && rc < (1 << 26) ? (uint32_t)rc << 6 | (uint32_t)lane : ~0u;
                const uint32_t m32 = wave_min_u32f(k32);
                int32_t ws;
                if (m32 != ~0u) {
                    ws = (int32_t)(m32 & 63);
                } else {
                    const uint64_t k64 = wok ? (uint64_t)rc << 6 | (uint64_t)lane : ~0ull;
                    ws = (int32_t)(wave_min_u64f(k64) & 63);
                }
                const int32_t ek = ws >= ncpu ? e1 : e0;
                int64_t xs = 0;
                if constexpr (DATA) {
                    xs = (int64_t)read_lane64((uint64_t)xk, ws);
                    if (xs > INSP_MAX_TICK) status |= ST_XFER;
                }
                const int32_t lenw = read_lane(len, ws);
                const int32_t pos = lenw & 63;
                int32_t blk;
                if (pos == 0) {
                    if (nfl > 0) {
                        nfl--;
                        blk = L.fstk[nfl];
                    } else {
                        nfg--;
                        blk = wg_load(&freeb[nfg]);
                        settle(blk);
                    }
                    const int32_t nbw = read_lane(nb, ws);
                    if (lane == 0) {
                        if (nbw < kLB) L.blist[ws * kLB + nbw] = blk;
                        else wblk[(int64_t)ws * maxb + nbw] = blk;
                    }
                    if (lane == ws) {
                        nb = nbw + 1;
                        last = blk;
                    }
                } else {
                    blk = read_lane(last, ws);
                }
                if (lane == ws) {
                    len = lenw + 1;
                    qest += ek;
                    ld += ek;
                }
                if (lane == j) {
                    pq = blk * 64 + pos;
                    sqj = seq;
                    wsj = ws;
                    xsj = xs;
                }
                seq++;
                nready++;
            }
            PCLK(17);
            // the chunk's queue entries, task records and block maxima: lane j
            // writes task j's.  The first entry of a new block sets its maxima,
            // then every entry raises them -- the first one's lane too, so that
            // within each lane the store precedes the atomic on that address
            // and the compiler keeps the stores of some lanes ahead of the
            // atomics of the others.
            const int32_t bq = pq >> 6;
            KT a0 = 0, a1 = 0;
            if (ok) {
                const bool g = wsj >= ncpu;
                const int32_t ekl = g ? e_l.y : e_l.x, dkl = g ? d_l.y : d_l.x;
                uint64_t raw;
                if constexpr (FIX) {
                    // the general loop's key: rank << 21 or IA << 42 | IE << 21, then the push order
                    raw = heft ? ((uint64_t)(uint32_t)ie_l << 32 | (uint32_t)ia_l) << 21 | (M21 - (uint64_t)sqj)
                               : (uint64_t)ia_l << 42 | (uint64_t)ie_l << 21 | (M21 - (uint64_t)sqj);
                    a0 = K.rule(raw, 0);
                    a1 = K.rule(raw, 1);
                } else {
                    a0 = kf.ka((uint32_t)ia_l, (uint32_t)ie_l, (uint32_t)sqj);
                    a1 = kf.ke((uint32_t)ia_l, (uint32_t)ie_l, (uint32_t)sqj);
                    raw = (uint64_t)a1 << 32 | a0;
                }
                const uint64_t xw = (uint64_t)v_l << 42 | (uint64_t)(dkl & M21) << 21 | (uint64_t)(ekl & M21);
                if (bq < SLK) {
                    if constexpr (FIX) {
                        K.ka[pq] = raw;
                    } else {
                        K.ka[pq] = a0;
                        K.ke[pq] = a1;
                    }
                } else {
                    slots.k[pq] = raw;
                }
                if (bq < SLC) {
                    L.sx[pq] = xw;
                    L.srs[pq] = rs_l;
                } else {
                    slots.x[pq] = xw;
                    slots.rs[pq] = rs_l;
                }
                tr[v_l].qpos = pq;
                tr[v_l].seq = sqj;
                // data model: the record's first word holds the time the
                // task's inputs arrive (transfers start now) until its pop
                if constexpr (DATA) tr[v_l].word = (unsigned long long)(t + xsj);
                if ((pq & 63) == 0) {
                    if (bq < SC) {
                        K.mx[2 * bq] = a0;
                        K.mx[2 * bq + 1] = a1;
                        L.stale[bq] = 0;
                    } else {
                        sums[2 * bq] = a0;
                        sums[2 * bq + 1] = a1;
                    }
                    // never lowered by pops: an upper bound for the block
                    if (lrule) barr[bq] = t + xsj;
                }
            }
            if (ok) {
                if (bq < SC) {
                    atomicMax(&K.mx[2 * bq], a0);
                    atomicMax(&K.mx[2 * bq + 1], a1);
                } else {
                    wg_fetch_max(&sums[2 * bq], (unsigned long long)a0);
                    wg_fetch_max(&sums[2 * bq + 1], (unsigned long long)a1);
                }
                if (lrule) wg_fetch_max(reinterpret_cast<unsigned long long *>(&barr[bq]), (unsigned long long)(t + xsj));
            }
        }
        PCLK(0);
        wg_fence();
        PCLK(1);
        // -------------------------------------------------------- regulate
        const int32_t observed = nready;
        if (A.policy == INSP_POLICY_INSPIRIT) {
            if (nready > peak) peak = nready;
            const int32_t dn = nready - prev_n;
            if ((dn < 0 ? -dn : dn) >= s_inc) {
                const int64_t dt = t - prev_t;
                prev_n = nready;
                prev_t = t;
                if (nready >= peak - dec_step) {
                    cnt = 0;
                    if (dn >= s_inc) {
                        const int64_t lhs = (int64_t)dn * k_den, rhs = (int64_t)k_num * dt;
                        if (dt == 0 || lhs > rhs) mode = INSP_MODE_ABILITY;
                        else if (lhs < rhs) mode = INSP_MODE_EFI;
                    }
                } else if ((int64_t)nready > (int64_t)peak - (int64_t)s_dec * cnt) {
                    mode = INSP_MODE_ABILITY;
                } else if ((int64_t)nready <= (int64_t)peak - (int64_t)s_dec * (cnt + 1) + cc) {
                    mode = INSP_MODE_EFI_LOC;
                    if ((int64_t)nready <= (int64_t)peak - (int64_t)s_dec * (cnt + 1)) cnt++;
                }
            }
        }
        const int pmode = A.policy == INSP_POLICY_FIFO ? INSP_MODE_FIFO
                        : A.policy == INSP_POLICY_ABILITY_ONLY ? INSP_MODE_ABILITY
                        : A.policy == INSP_POLICY_EFI_ONLY ? INSP_MODE_EFI
                        : (DATA && A.policy == INSP_POLICY_LOCALITY) ? INSP_MODE_EFI_LOC
                        : heft ? INSP_MODE_RANK : mode;
        const int ord = heft ? 3 : pmode == INSP_MODE_FIFO ? 2 : pmode == INSP_MODE_ABILITY ? 0 : 1;
        const int slot = ord == 1 ? 1 : 0;
        // efficiency with locality under the data model: tasks whose inputs
        // have arrived first
        const bool loc = DATA && pmode == INSP_MODE_EFI_LOC;
        // ------------------------------------------------------------- pop
        int32_t popped = 0;
        bool popnow = false;        // this lane's worker took a task in this event
        int32_t iep = 0;            // ... with this IE
        int32_t mvt = -1, mvp = 0;  // lane k: task moved into the hole of the k-th pop, and where
        uint64_t idle = ballot(wok && run < 0 && len > 0);
        while (idle) {
            const int32_t w = (int32_t)__builtin_ctzll(idle);
            idle &= idle - 1;
            const int32_t nbw = read_lane(nb, w), lenw = read_lane(len, w), lastw = read_lane(last, w);
            const int32_t lastpos = (lenw - 1) & 63;
            int32_t p = 0;
            PCLK(10);
            bool lsel = false;  // the locality rule found a task whose inputs are in place
            if constexpr (DATA) {
                if (loc) {
                    // the arrival times are not in the keys.  A block whose
                    // latest input arrival has passed holds only tasks whose
                    // inputs are in place, so its efficiency maximum stands;
                    // the other blocks are scanned entry by entry
                    KT bestk = 0;
                    int32_t bestb = -1;
                    for (int32_t i0 = 0; i0 < nbw; i0 += kWave) {
                        const int32_t i = i0 + lane;
                        int32_t b = -1;
                        if (i < nbw) {
                            if (i < kLB) {
                                b = L.blist[w * kLB + i];
                            } else {
                                b = wg_load(&wblk[(int64_t)w * maxb + i]);
                                settle(b);
                            }
                        }
                        uint64_t sm = ballot(b >= 0 && b < SC && L.stale[b] != 0);
                        while (sm) {
                            const int l = (int)__builtin_ctzll(sm);
                            sm &= sm - 1;
                            rebuild_max<FIX>(slots, K, L, sums, SLK, SC, read_lane(b, l));
                        }
                        KT kk = 0;
                        bool mix = false;
                        if (b >= 0) {
                            if ((int64_t)wg_load(&barr[b]) <= t) kk = b < SC ? K.mx[2 * b + 1] : (KT)wg_load(&sums[2 * b + 1]);
                            else mix = true;
                        }
                        const KT km = wave_max_k(kk);
                        if (km > bestk) {
                            bestk = km;
                            bestb = read_lane(b, (int)__builtin_ctzll(ballot(kk == km && b >= 0)));
                        }
                        uint64_t mm = ballot(mix);
                        while (mm) {
                            const int32_t bm = read_lane(b, (int)__builtin_ctzll(mm));
                            mm &= mm - 1;
                            KT ke = 0;
                            if (lane < (bm == lastw ? lastpos + 1 : 64)) {
                                const int32_t pe = bm * 64 + lane;
                                const uint64_t xv = bm < SLC ? L.sx[pe] : wg_load(&slots.x[pe]);
                                const KT kr = bm < SLK ? K.lds(pe, 1) : K.rule(wg_load(&slots.k[pe]), 1);
                                if ((int64_t)wg_load(&tr[(int32_t)(xv >> 42)].word) <= t) ke = kr;
                            }
                            const KT kme = wave_max_k(ke);
                            if (kme > bestk) {
                                bestk = kme;
                                bestb = bm;
                            }
                        }
                    }
                    if (bestb >= 0) {
                        // the best entry of that block whose inputs are in place
                        KT key = 0;
                        if (lane < (bestb == lastw ? lastpos + 1 : 64)) {
                            const int32_t pe = bestb * 64 + lane;
                            const uint64_t xv = bestb < SLC ? L.sx[pe] : wg_load(&slots.x[pe]);
                            const KT kr = bestb < SLK ? K.lds(pe, 1) : K.rule(wg_load(&slots.k[pe]), 1);
                            if ((int64_t)wg_load(&tr[(int32_t)(xv >> 42)].word) <= t) key = kr;
                        }
                        const KT km = wave_max_k(key);
                        p = bestb * 64 + (int)__builtin_ctzll(ballot(key == km && key != 0));
                        lsel = true;
                    }
                }
            }
            if (lsel) {
                // chosen by the locality rule
            } else if (nbw <= A.scan_max) {
                // lane l compares entry l of every block of the worker: the
                // blocks held in LDS, then those in global memory (a single
                // block is the last one, known without reading the list)
                // (at most 16 blocks: the list's LDS part holds them all, as its
                // capacity is at least min(16, blocks in the pool))
                int32_t bl = -1;
                if (nbw == 1) bl = lastw;
                else if (lane < nbw) bl = L.blist[w * kLB + lane];
                const uint64_t all = nbw == 1 ? 1ull : ballot(lane < nbw);
                const uint64_t inl = nbw == 1 ? (lastw < SLK ? 1ull : 0ull) : ballot(lane < nbw && bl < SLK);
                KT best = 0;
                int32_t bp = -1;
                if (inl == all) {
                    // every block in LDS: blocks i .. i+3 of the list, the
                    // padding past the list re-reading its last block
                    for (int32_t i = 0; i < nbw; i += 4) {
                        KT kk[4];
                        int32_t pp[4];
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            pp[u] = read_lane(bl, min(i + u, nbw - 1)) * 64 + lane;
                            kk[u] = K.lds(pp[u], slot);
                        }
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            if (kk[u] > best) {
                                best = kk[u];
                                bp = pp[u];
                            }
                        }
                    }
                } else if (slot) {
                    if (inl) scan_columns<FIX, true, 1>(slots, K, inl, bl, best, bp);
                    scan_columns<FIX, false, 1>(slots, K, all & ~inl, bl, best, bp);
                } else {
                    if (inl) scan_columns<FIX, true, 0>(slots, K, inl, bl, best, bp);
                    scan_columns<FIX, false, 0>(slots, K, all & ~inl, bl, best, bp);
                }
                const KT km = wave_max_k(best);
                p = read_lane(bp, (int)__builtin_ctzll(ballot(best == km && bp >= 0)));
            } else {
                // many blocks: rebuild stale maxima, pick the block, scan it
                KT bk = 0;
                int32_t bid = -1;
                for (int32_t i0 = 0; i0 < nbw; i0 += kWave) {
                    const int32_t i = i0 + lane;
                    int32_t b = -1;
                    if (i < nbw) {
                        if (i < kLB) {
                            b = L.blist[w * kLB + i];
                        } else {
                            b = wg_load(&wblk[(int64_t)w * maxb + i]);
                            settle(b);
                        }
                    }
                    bool st = false;
                    if (b >= 0 && b < SC) st = L.stale[b] != 0;
                    uint64_t sm = ballot(st);
                    while (sm) {
                        const int l = (int)__builtin_ctzll(sm);
                        sm &= sm - 1;
                        const int32_t sb = read_lane(b, l);
                        rebuild_max<FIX>(slots, K, L, sums, SLK, SC, sb);
                    }
                    if (b >= 0) {
                        KT k;
                        if (b < SC) {
                            k = K.mx[2 * b + slot];
                        } else {
                            k = (KT)wg_load(&sums[2 * b + slot]);
                            settle(k);
                        }
                        if (k > bk) {
                            bk = k;
                            bid = b;
                        }
                    }
                }
                const KT kmb = wave_max_k(bk);
                const int32_t bb = read_lane(bid, (int)__builtin_ctzll(ballot(bk == kmb && bid >= 0)));
                const int32_t cntb = bb == lastw ? lastpos + 1 : 64;
                const KT key = block_keys<FIX>(slots, K, SLK, bb, slot);
                const KT km = wave_max_k(key);
                p = bb * 64 + (int)__builtin_ctzll(ballot(key == km && lane < cntb));
            }
            PCLK(11);
            // take the entry at p; the worker's final entry q fills the hole
            const int32_t bb = p >> 6;
            const int32_t q = lastw * 64 + lastpos;
            uint32_t ve = 0;
            uint64_t vx, mx = 0, mkr = 0;  // mkr: the moved entry's key word (the two 32-bit keys, or the fixed key)
            int32_t vr, mr = 0;
            if (bb < SLC) {
                vx = L.sx[p];
                vr = L.srs[p];
            } else {
                vx = wg_load(&slots.x[p]);
                vr = wg_load(&slots.rs[p]);
                settle(vx);
                settle(vr);
            }
            if constexpr (!FIX) {
                if (bb < SLK) {
                    ve = K.ke[p];
                } else {
                    ve = (uint32_t)(wg_load(&slots.k[p]) >> 32);
                    settle(ve);
                }
            }
            if (p != q) {
                if (lastw < SLK) {
                    if constexpr (FIX) mkr = K.ka[q];
                    else mkr = (uint64_t)K.ke[q] << 32 | K.ka[q];
                } else {
                    mkr = wg_load(&slots.k[q]);
                    settle(mkr);
                }
                if (lastw < SLC) {
                    mx = L.sx[q];
                    mr = L.srs[q];
                } else {
                    mx = wg_load(&slots.x[q]);
                    mr = wg_load(&slots.rs[q]);
                    settle(mx);
                    settle(mr);
                }
            }
            const int32_t v = (int32_t)(vx >> 42);
            const int32_t dk = (int32_t)((vx >> 21) & M21), ek = (int32_t)(vx & M21);
            // a task whose inputs are still moving holds the worker until they arrive
            int64_t s0 = t;
            if constexpr (DATA) s0 = max(t, (int64_t)wg_load(&tr[v].word));
            // out-degree and the IE to record, from the direct key (fixed keys:
            // read from the task's record once the event's pops are done)
            int32_t deg = 0, iev = 0;
            if constexpr (!FIX) {
                deg = (int32_t)((ve >> kf.sa) & kf.amask);
                iev = (int32_t)((ve >> kf.sb) & kf.amask);
            }
            if (p != q) {
                if (lane == 0) {
                    if (bb < SLK) {
                        if constexpr (FIX) {
                            K.ka[p] = mkr;
                        } else {
                            K.ka[p] = (uint32_t)mkr;
                            K.ke[p] = (uint32_t)(mkr >> 32);
                        }
                    } else {
                        slots.k[p] = mkr;
                    }
                    if (bb < SLC) {
                        L.sx[p] = mx;
                        L.srs[p] = mr;
                    } else {
                        slots.x[p] = mx;
                        slots.rs[p] = mr;
                    }
                    // the moved entry keeps block bb's arrival bound valid
                    if (lrule && lastw != bb) barr[bb] = max(barr[bb], barr[lastw]);
                }
                if (lane == popped) {
                    mvt = (int32_t)(mx >> 42);
                    mvp = p;
                }
            }
            // the worker's final slot is now empty
            if (lane == 0) {
                if (lastw < SLK) {
                    K.ka[q] = 0;
                    if constexpr (!FIX) K.ke[q] = 0;
                } else {
                    slots.k[q] = 0;
                }
            }
            PCLK(12);
            const int32_t nlen = lenw - 1;
            const bool freed = (nlen & 63) == 0;
            int32_t nbn = nbw, newlast = lastw;
            if (freed) {
                if (lane == 0) {
                    if (lastw < SC) L.fstk[nfl] = lastw;
                    else freeb[nfg] = lastw;
                }
                if (lastw < SC) nfl++;
                else nfg++;
                nbn = nbw - 1;
                if (nbn <= 0) {
                    newlast = -1;
                } else if (nbn - 1 < kLB) {
                    newlast = L.blist[w * kLB + nbn - 1];
                } else {
                    newlast = wg_load(&wblk[(int64_t)w * maxb + nbn - 1]);
                    settle(newlast);
                }
            }
            // maxima of the blocks that changed: bb lost the winner (and took
            // the final entry), the last block lost its final entry
            if (!(bb == lastw && freed)) {
                if (bb < SC) {
                    if (lane == 0) L.stale[bb] = 1;
                } else {
                    rebuild_max<FIX>(slots, K, L, sums, SLK, SC, bb);
                }
            }
            if (lastw != bb && !freed) {
                if (lastw < SC) {
                    if (lane == 0) L.stale[lastw] = 1;
                } else {
                    rebuild_max<FIX>(slots, K, L, sums, SLK, SC, lastw);
                }
            }
            PCLK(13);
            if (lane == w) {
                len = nlen;
                nb = nbn;
                last = newlast;
                run = v;
                st0 = s0;
                fin = s0 + dk;
                expend = s0 + ek;
                qest -= ek;
                rsr = vr;
                dgr = deg;
                iep = iev;
                popnow = true;
            }
            nready--;
            popped++;
            PCLK(14);
        }
        // the event's pops write their records with one store (a worker pops
        // at most once per event, so the addresses differ), and prefetch the
        // first successors of the tasks they started
        if constexpr (FIX) {
            // every worker that took a task reads its out-degree and IE at once
            if (popnow) {
                const int4 fx = *reinterpret_cast<const int4 *>(&tr[run].iev);  // IE, IA, tau, first edge
                dgr = fx.y;
                iep = tattr ? tie[run] : fx.x;
            }
        }
        if (popnow) put_record(&tr[run], DATA ? st0 : t, (int32_t)(fin - (DATA ? st0 : t)), lane, iep, pmode);
        if (popnow && dgr > 0) {
            // entries past the row repeat its last successor (never used)
#pragma unroll
            for (int j = 0; j < kPF; j++) pf[j] = col[rsr + min(j, dgr - 1)];
        }
        if (mvt >= 0) tr[mvt].qpos = mvp;
        // the running tasks, for the work-group's prefetching wave
        if (wok) {
            L.run[lane] = run;
            L.fin[lane] = fin;
        }
        PCLK(15);
        PCLK(2);
        if (A.trace && lane == 0 && events <= max_events) {
            insp_trace_rec rec;
            rec.t = t;
            rec.nready = observed;
            rec.mode = pmode;
            rec.cnt = cnt;
            rec.peak = peak;
            rec.pushed = r;
            rec.popped = popped;
            A.trace[(d.toff - A.base) + di + events - 1] = rec;
        }
        if (done == n) break;
        // --------------------------------------------------------- advance
        // every running task ends within 2^20 ticks of t
        const uint32_t dtm = wave_min_u32f(wok && run >= 0 ? (uint32_t)(fin - t) : ~0u);
        if (dtm == ~0u) {
            status |= ST_HANG;
            break;
        }
        t += dtm;
        PCLK(3);
        // --------------------------------------------------------- release
        r = 0;
        int32_t nc = 0, nseg = 0, ndone = 0;
        {
            const bool fin_now = wok && run >= 0 && fin == t;
            uint64_t mask = ballot(fin_now);
            const int32_t c_l = fin_now ? run : -1;
            if (fin_now) run = -1;
            while (mask) {
                const int l = (int)__builtin_ctzll(mask);
                mask &= mask - 1;
                const int32_t c = read_lane(c_l, l);
                done++;
                ndone++;
                const int32_t deg = read_lane(dgr, l), rs = read_lane(rsr, l);
                const int32_t r0 = r;
                const unsigned long long dec = 0ull - ((1ull << 43) + (unsigned long long)c);
                for (int32_t e0 = 0; e0 < deg; e0 += kWave) {
                    const int32_t e = e0 + lane;
                    const bool ok = e < deg;
                    int32_t s = 0;
                    if (e0 == 0) {
#pragma unroll
                        for (int j = 0; j < kPF; j++) {
                            const int32_t y = read_lane(pf[j], l);
                            if (lane == j) s = y;
                        }
                    }
                    if (ok && e >= kPF) s = col[rs + e];
                    PCLK(19);
                    // one wave owns the DAG's words and a row's successors are
                    // distinct (rows are deduplicated), so a plain
                    // read-modify-write replaces the atomic (a wave's accesses
                    // to one address complete in program order)
                    uint64_t old = 0;
                    if (ok) {
                        old = dep[s];
                        dep[s] = old + dec;
                    }
                    const int32_t nr = (int32_t)(old >> 43) - 1;
                    const bool rdy = ok && nr == 0, cd = ok && nr == 1;
                    const uint64_t m1 = ballot(rdy), m2 = ballot(cd);
                    PCLK(20);
                    if (rdy) {
                        const int32_t pos = r + lanes_below(m1);
                        fbuf[pos] = s;
                        if (pos < kFC) L.fr0[pos] = s;
                    }
                    if (cd) {
                        const int32_t pos = nc + lanes_below(m2);
                        if (pos < kCC) {
                            L.cs[pos] = s;
                            L.cu[pos] = (int32_t)((old + dec) & M43);
                        } else {
                            fbuf[2 * n + pos] = s;
                        }
                    }
                    r += __popcll(m1);
                    nc += __popcll(m2);
                }
                if (r > r0) {
                    if (lane == 0) L.seg[nseg] = r;
                    nseg++;
                }
            }
        }
        PCLK(4);
        wg_fence();
        PCLK(5);
        // successors left with one unfinished predecessor raise its IE (as in
        // the general loop)
        const bool single = ndone == 1;
        merged = false;
        staged = false;
        if (nc <= kWave && r <= kFC) {
            const bool hc = lane < nc;
            const int32_t s = hc ? L.cs[lane] : 0;
            int32_t u = hc ? L.cu[lane] : -1;
            staged = r <= kWave;
            const bool hf = staged && lane < r;
            const int32_t fv = hf ? L.fr0[lane] : 0;
            // a candidate made ready by a later completion of this event is none
            if (!single) {
                if (staged) {
                    for (int32_t k = 0; k < r; k++)
                        if (read_lane(fv, k) == s) u = -1;
                } else if (hc) {
                    for (int32_t k = 0; k < r; k++)
                        if (L.fr0[k] == s) {
                            u = -1;
                            break;
                        }
                }
            }
            PCLK(22);
            int32_t tu = 0, ts = 0, iu = 0, qu = -1, au = 0, sq = 0;
            if (u >= 0) {
                // one wave owns the records, so plain vector loads see its stores
                const int2 qs = *reinterpret_cast<const int2 *>(&tr[u].qpos);  // queue slot, push order
                const int4 fx = *reinterpret_cast<const int4 *>(&tr[u].iev);   // IE, IA, tau, first edge
                ts = tr[s].tau;
                qu = qs.x;
                sq = qs.y;
                iu = fx.x;
                au = fx.y;
                tu = fx.z;
            }
            int2 fe = make_int2(1, 1), fd = make_int2(1, 1);
            int32_t fa = 0, frs = 0, fie = 0;
            if (hf) {
                fe = est2[fv];
                fd = dur2[fv];
                const int4 fx = *reinterpret_cast<const int4 *>(&tr[fv].iev);
                fie = fx.x;
                fa = fx.y;
                frs = fx.w;
                // fixed keys: the rank (low and high words), or the transitive attributes
                if (heft) {
                    const int64_t rv = rk[fv];
                    fa = (int32_t)(uint32_t)rv;
                    fie = (int32_t)(uint32_t)((uint64_t)rv >> 32);
                } else if (tattr) {
                    fa = tia[fv];
                    fie = tie[fv];
                }
            }
            const bool cond = u >= 0 && (int64_t)tu + ts <= (int64_t)U;
            PCLK(23);
            int32_t mult = cond ? 1 : 0;
            bool lead = cond;
            if (nc > 1) {
                // several successors may name the same predecessor: the
                // first lane applies all of its increments
                mult = 0;
                for (int32_t j = 0; j < nc; j++) {
                    const int32_t uj = read_lane(u, j);
                    const int32_t cj = read_lane(cond ? 1 : 0, j);
                    if (cj && cond && uj == u) {
                        mult++;
                        if (j < lane) lead = false;
                    }
                }
            }
            if (lead) {
                const int32_t nie = iu + mult;
                tr[u].iev = nie;
                if constexpr (!FIX) {
                    if (qu >= 0) {
                        const uint32_t na = kf.ka((uint32_t)au, (uint32_t)nie, (uint32_t)sq);
                        const uint32_t ne = kf.ke((uint32_t)au, (uint32_t)nie, (uint32_t)sq);
                        const int32_t bk = qu >> 6;
                        if (bk < SLK) {
                            K.ka[qu] = na;
                            K.ke[qu] = ne;
                        } else {
                            slots.k[qu] = (uint64_t)ne << 32 | na;
                        }
                        if (bk < SC) {
                            atomicMax(&K.mx[2 * bk], na);
                            atomicMax(&K.mx[2 * bk + 1], ne);
                        } else {
                            wg_fetch_max(&sums[2 * bk], (unsigned long long)na);
                            wg_fetch_max(&sums[2 * bk + 1], (unsigned long long)ne);
                        }
                    }
                }
            }
            PCLK(24);
            // a raised IE of a task staged for this event's pushes goes into its key
            uint64_t lm = FIX ? 0 : ballot(lead && qu == -1);
            while (lm) {
                const int l = (int)__builtin_ctzll(lm);
                lm &= lm - 1;
                const int32_t uu = read_lane(u, l), kk = read_lane(mult, l);
                const uint64_t fm = ballot(hf && fv == uu);
                if (fm && lane == (int)__builtin_ctzll(fm)) fie += kk;
            }
            int32_t pos = lane;
            if (nseg > 1 && staged) {
                // rank in the merged ascending order (the event's ready ids are
                // distinct): how many of them are smaller
                int32_t rank = 0;
                for (int32_t k = 0; k < r; k++) rank += read_lane(fv, k) < fv ? 1 : 0;
                pos = rank;
            }
            if (!staged && nseg > 1) {
                for (int32_t i = lane; i < r; i += kWave) {
                    const int32_t x = L.fr0[i];
                    int32_t rank = 0, lo = 0;
                    for (int32_t g = 0; g < nseg; g++) {
                        const int32_t hi = L.seg[g];
                        if (i >= lo && i < hi) {
                            rank += i - lo;
                        } else {
                            int32_t a = lo, b = hi;
                            while (a < b) {
                                const int32_t mid = (a + b) >> 1;
                                if (L.fr0[mid] < x) a = mid + 1;
                                else b = mid;
                            }
                            rank += a - lo;
                        }
                        lo = hi;
                    }
                    L.fr1[rank] = x;
                }
                merged = true;
            }
            if (hf) {
                L.pre[pos] = fv;
                L.pre[64 + pos] = fe.x;
                L.pre[128 + pos] = fe.y;
                L.pre[192 + pos] = fd.x;
                L.pre[256 + pos] = fd.y;
                L.pre[320 + pos] = fa;
                L.pre[384 + pos] = frs;
                L.pre[448 + pos] = fie;
            }
        } else {
            for (int32_t i0 = 0; i0 < nc; i0 += kWave) {
                const int32_t i = i0 + lane;
                if (i < nc) {
                    const int32_t s = i < kCC ? L.cs[i] : wg_load(&fbuf[2 * n + i]);
                    int32_t u = -1;
                    if (single && i < kCC) {
                        u = L.cu[i];
                    } else {
                        const uint64_t wd = wg_load(&dep[s]);
                        if ((wd >> 43) == 1) u = (int32_t)(wd & M43);
                    }
                    if (u >= 0) {
                        const int32_t tu = tr[u].tau, ts = tr[s].tau;
                        const int32_t pu = wg_load(&tr[u].qpos);
                        if ((int64_t)tu + ts <= (int64_t)U) {
                            wg_fetch_add(&tr[u].iev, 1);
                            if constexpr (!FIX) {
                                if (pu >= 0) {
                                    const int32_t bk = pu >> 6;
                                    uint32_t na, ne;
                                    if (bk < SLK) {
                                        na = atomicAdd(&K.ka[pu], kf.da()) + kf.da();
                                        ne = atomicAdd(&K.ke[pu], kf.de()) + kf.de();
                                    } else {
                                        const unsigned long long inc = (unsigned long long)kf.de() << 32 | kf.da();
                                        const uint64_t nk = wg_fetch_add(&slots.k[pu], inc) + inc;
                                        na = (uint32_t)nk;
                                        ne = (uint32_t)(nk >> 32);
                                    }
                                    if (bk < SC) {
                                        atomicMax(&K.mx[2 * bk], na);
                                        atomicMax(&K.mx[2 * bk + 1], ne);
                                    } else {
                                        wg_fetch_max(&sums[2 * bk], (unsigned long long)na);
                                        wg_fetch_max(&sums[2 * bk + 1], (unsigned long long)ne);
                                    }
                                }
                            }
                        }
                    }
                }
            }
            wg_fence();
            if (nseg > 1) {
                const bool in_lds = r <= kFC;
                for (int32_t i0 = 0; i0 < r; i0 += kWave) {
                    const int32_t i = i0 + lane;
                    if (i < r) {
                        const int32_t x = in_lds ? L.fr0[i] : fbuf[i];
                        int32_t rank = 0, lo = 0;
                        for (int32_t g = 0; g < nseg; g++) {
                            const int32_t hi = L.seg[g];
                            if (i >= lo && i < hi) {
                                rank += i - lo;
                            } else {
                                int32_t a = lo, b = hi;
                                while (a < b) {
                                    const int32_t mid = (a + b) >> 1;
                                    const int32_t y = in_lds ? L.fr0[mid] : fbuf[mid];
                                    if (y < x) a = mid + 1;
                                    else b = mid;
                                }
                                rank += a - lo;
                            }
                            lo = hi;
                        }
                        if (in_lds) L.fr1[rank] = x;
                        else fbuf[n + rank] = x;
                    }
                }
                merged = true;
            }
        }
        PCLK(7);
        wg_fence();
        PCLK(8);
    }
#ifdef INSP_PHASE_CLOCKS
    if (lane == 0 && d.id < 8192)
        for (int i = 0; i < 32; i++) g_phase_clk[d.id * 32 + i] = pc[i];
#endif
    if (lane == 0) {
        A.makespan[di] = (status & ST_HANG) ? -1 : t;
        if (A.n_events) A.n_events[di] = events;
        if (status) atomicOr(&A.stat[2 * d.id], status);
        A.stat[2 * d.id + 1] = events;
    }
    return true;
}

// The work-group's LDS, carved in the order lds_bytes() counts it.
__device__ __forceinline__ Lds carve_lds(const SimArgs &A) {
    extern __shared__ int64_t lds64[];
    const int32_t MW = A.max_w;
    Lds L;
    L.fin = lds64;
    L.expend = lds64 + MW;
    L.qest = lds64 + 2 * MW;
    L.sum = reinterpret_cast<unsigned long long *>(lds64 + 3 * MW);
    L.sk = L.sum + 2 * A.sum_cap;
    L.sx = L.sk + 64 * A.key_cap;
    int32_t *l32 = reinterpret_cast<int32_t *>(L.sx + 64 * A.slot_cap);
    L.run = l32;
    L.len = l32 + MW;
    L.nb = l32 + 2 * MW;
    L.last = l32 + 3 * MW;
    L.seg = l32 + 4 * MW;
    L.rsr = l32 + 5 * MW;
    L.dgr = l32 + 6 * MW;
    L.blist = l32 + 7 * MW;
    L.fr0 = L.blist + MW * A.lb;
    L.fr1 = L.fr0 + kFC;
    L.cs = L.fr1 + kFC;
    L.cu = L.cs + kCC;
    L.pre = L.cu + kCC;
    L.srs = L.pre + 8 * kWave;
    L.fstk = L.srs + 64 * A.slot_cap;
    L.stale = reinterpret_cast<uint8_t *>(L.fstk + A.sum_cap);
    L.hs = reinterpret_cast<int32_t *>(L.stale + ((A.sum_cap + 15) & ~15));
    return L;
}

// The work-group's second wave, while the first simulates DAG di: it reads
// ahead for the running tasks that finish first -- their successor lists,
// the successors' dependency words, and the records and estimate rows the
// release of those tasks will read (of successors about to become ready,
// and of the remaining predecessor of those about to have one left) -- so
// that the simulating wave finds them in the caches.  It only reads, and it
// stops when the simulating wave marks the DAG finished.
constexpr int kAhead = 4;          // running tasks read ahead for, earliest finish first
constexpr int kAheadEdges = 16;    // successors read per task
constexpr int64_t kHelperSpin = 1ll << 40;

__device__ void read_ahead(const SimArgs &A, int32_t di, const Lds &L) {
    const DagDesc d = A.desc[di];
    const int lane = lane_id();
    const int32_t W = d.n_cpu + d.n_gpu;
    const bool wok = lane < W && W <= kWave && d.n > 0;
    const int64_t ub = d.toff - A.base;
    const int32_t *col = A.col + d.eoff;
    const TaskRec *tr = A.tr + d.toff;
    const unsigned long long *dep = A.dep + d.toff;
    const int2 *est2 = reinterpret_cast<const int2 *>(A.est) + ub;
    const int2 *dur2 = reinterpret_cast<const int2 *>(A.dur) + ub;
    int32_t pref = -1;  // the last task read ahead for this lane's worker
    uint32_t sink = 0;
    for (int64_t it = 0; it < kHelperSpin; it++) {
        if (__hip_atomic_load(&L.hs[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
        const int32_t c = wok ? __hip_atomic_load(&L.run[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : -1;
        const int64_t f = c >= 0 ? __hip_atomic_load(&L.fin[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                                 : INT64_MAX;
        // the kAhead-th earliest finish among the running tasks
        uint64_t thr = 0;
        {
            uint64_t prev = 0;
            bool first = true;
            for (int k = 0; k < kAhead; k++) {
                const uint64_t m = wave_min_u64f(first || (uint64_t)f > prev ? (uint64_t)f : ~0ull);
                if (m == ~0ull) break;
                thr = m;
                prev = m;
                first = false;
            }
        }
        const bool go = c >= 0 && c != pref && c < d.n && (uint64_t)f <= thr;
        if (!ballot(go)) {
            __builtin_amdgcn_s_sleep(4);
            continue;
        }
        if (go) {
            pref = c;
            const int4 fx = *reinterpret_cast<const int4 *>(&tr[c].iev);  // IE, IA, tau, first edge
            const int32_t deg = min(fx.y, kAheadEdges), rs = fx.w;
            int32_t sv[kAheadEdges];
            unsigned long long dw[kAheadEdges];
#pragma unroll
            for (int j = 0; j < kAheadEdges; j++) sv[j] = deg > 0 ? col[rs + min(j, deg - 1)] : c;
#pragma unroll
            for (int j = 0; j < kAheadEdges; j++) dw[j] = dep[sv[j]];
#pragma unroll
            for (int j = 0; j < kAheadEdges; j++) {
                if (j >= deg) break;
                const uint32_t rem = (uint32_t)(dw[j] >> 43);
                if (rem == 1) {
                    const int2 e = est2[sv[j]], u = dur2[sv[j]];
                    const int4 q = *reinterpret_cast<const int4 *>(&tr[sv[j]].iev);
                    const int2 qs = *reinterpret_cast<const int2 *>(&tr[sv[j]].qpos);
                    sink ^= (uint32_t)(e.x ^ u.y ^ q.x ^ qs.x);
                } else if (rem == 2) {
                    const int32_t pu = (int32_t)((dw[j] & ((1ull << 43) - 1)) - (unsigned long long)c);
                    if (pu >= 0 && pu < d.n) {
                        const int4 q = *reinterpret_cast<const int4 *>(&tr[pu].iev);
                        const int2 qs = *reinterpret_cast<const int2 *>(&tr[pu].qpos);
                        sink ^= (uint32_t)(q.x ^ qs.y);
                    }
                    sink ^= (uint32_t)tr[sv[j]].tau;
                }
            }
        }
    }
    L.hs[2] = (int32_t)sink;  // keeps the reads
}

// Event loop a launch runs (one kernel each, so that each gets its own
// register allocation), for machines of at most 64 workers: the one-wave loop
// on direct 32-bit keys (DAGs whose keys do not fit fall back to the general
// loop) or on fixed 64-bit keys (HEFT ranks, transitive attributes), each
// with or without the data model; for larger machines the general loop.
enum SimLoop { kLoopDirect = 0, kLoopFixed = 1, kLoopGeneral = 2, kLoopData = 3, kLoopDataFixed = 4 };

template <int WPL, int LOOP>
__global__ __launch_bounds__(WPL == 1 ? 2 * kWave : kWave) void k_sim(SimArgs A) {
    const Lds L = carve_lds(A);
    const int lane = lane_id();
    // one wave simulates; under the one-wave loop's launch a second wave reads ahead
    const bool helper = WPL == 1 && threadIdx.x >= kWave;
    for (;;) {
        if (threadIdx.x == 0) {
            L.hs[0] = dev_fetch_add(A.counter, 1);
            L.hs[1] = 0;
        }
        if (threadIdx.x < kWave)
            for (int32_t w = lane; w < A.max_w * WPL && w < kWave; w += kWave) L.run[w] = -1;
        __syncthreads();
        const int32_t i = L.hs[0];
        if (i >= A.count) break;
        if (helper) {
            read_ahead(A, A.order[i], L);
        } else {
            // the largest DAGs (dispensed first) set the batch's critical path:
            // their waves win instruction issue over co-resident waves
            if (i < A.prio_top) __builtin_amdgcn_s_setprio(3);
            else __builtin_amdgcn_s_setprio(0);
            if constexpr (WPL == 1 && (LOOP == kLoopDirect || LOOP == kLoopData)) {
                if (!sim_lane<false, LOOP == kLoopData>(A, A.order[i], L)) sim_dag<1>(A, A.order[i], L);
            } else if constexpr (WPL == 1 && (LOOP == kLoopFixed || LOOP == kLoopDataFixed)) {
                sim_lane<true, LOOP == kLoopDataFixed>(A, A.order[i], L);
            } else {
                sim_dag<WPL>(A, A.order[i], L);
            }
            wg_fence();
            if (lane == 0) __hip_atomic_store(&L.hs[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
    }
}

__global__ void k_counter_reset(int32_t *c) {
    if (threadIdx.x < 4) c[threadIdx.x] = 0;
}

// Unpack the schedules the simulation left in the task records into the
// caller's arrays (tasks never popped -- a failed DAG -- are left alone).
__global__ __launch_bounds__(256) void k_records(const TaskRec *tr, int64_t n, int32_t *worker, int64_t *start,
                                                 int64_t *finish, int32_t *ie_at_pop, int8_t *mode_at_pop) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int4 q = *reinterpret_cast<const int4 *>(tr + i);
    if (q.z > -2) return;
    const uint64_t wd = (uint64_t)(uint32_t)q.x | (uint64_t)(uint32_t)q.y << 32;
    const int64_t s = (int64_t)(wd & ((1ull << 42) - 1));
    worker[i] = -2 - q.z;
    start[i] = s;
    finish[i] = s + (int64_t)(wd >> 42);
    if (ie_at_pop) ie_at_pop[i] = q.w & ((1 << 22) - 1);
    if (mode_at_pop) mode_at_pop[i] = (int8_t)(q.w >> 22);
}

int launch_sim(insp_dag *dag, Workspace *ws, const insp_params &p, const int32_t *dur, const int32_t *est,
               int32_t *worker, int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop,
               int8_t *mode_at_pop, insp_trace_rec *trace, int32_t *n_events, int waves, int grid,
               int sum_cap, int slot_cap, int key_cap, hipStream_t st, int prio_top, int scan_max) {
    (void)waves;
    SimArgs A;
    memset(&A, 0, sizeof A);
    A.desc = ws->desc.as<DagDesc>();
    A.order = ws->order.as<int32_t>();
    A.count = ws->count;
    A.max_w = ws->max_w;
    A.col = dag->col.as<int32_t>();
    A.dur = dur;
    A.est = est;
    A.base = ws->base;
    A.tr = ws->tr;
    A.dep = ws->dep;
    A.fbuf = ws->fbuf;
    A.slots = SlotPool::over(ws->slots.p, ws->slots.bytes);
    A.sums = ws->sums.as<unsigned long long>();
    A.paux = ws->paux.as<int32_t>();
    A.freeb_base = ws->total_wl;
    A.dag_u = ws->dag_u;
    A.dag_taubar = ws->dag_taubar;
    A.stat = dag->dag_stat.as<int32_t>();
    A.rank = dag->rank.as<int64_t>();
    A.tia = dag->tia.as<int32_t>();
    A.tie = dag->tie.as<int32_t>();
    A.attr_mode = p.attr_mode;
    A.data_bw = p.data_bw;
    A.dkib = dag->dkib.as<int32_t>();
    A.pprp = dag->pprp.as<int32_t>();
    A.ppred = dag->ppred.as<int32_t>();
    A.barr = ws->barr.as<long long>();
    A.dxc = dag->dxc.as<int32_t>();
    A.counter = ws->counter.as<int32_t>();
    A.makespan = makespan;
    A.trace = trace;
    A.n_events = n_events;
    A.policy = p.policy;
    A.s_inc = p.s_inc;
    A.s_dec = p.s_dec;
    A.dec_step = p.dec_step;
    A.c = p.c;
    A.k_num = p.k_num;
    A.k_den = p.k_den;
    A.max_events = p.max_events;
    A.prio_top = prio_top;
    A.scan_max = scan_max;
    // block maxima in LDS: all of a single DAG's blocks up to 64 KB, or the
    // low block ids of each DAG of a batch
    // LDS: block maxima, block lists and the slots of the low blocks --
    // generous for a single DAG (one work-group owns the CU), a few blocks
    // per DAG for a batch (tunable)
    const bool one = ws->count == 1;
    const int64_t budget = (one ? 140 : 150) * 1024;
    int64_t sc = std::min<int64_t>(ws->max_nblk, one ? 2048 : sum_cap);
    int64_t lb = std::min<int64_t>(ws->max_nblk, one ? 64 : 16);
    // machines of hundreds of workers: shorter LDS block lists, then fewer
    // LDS block maxima, until the per-worker state fits (the rest lives in
    // global memory)
    while (lb > 1 && (int64_t)lds_bytes(ws->max_w, (int)sc, (int)lb, 0, 0) > budget) lb /= 2;
    while (sc > 0 && (int64_t)lds_bytes(ws->max_w, (int)sc, (int)lb, 0, 0) > budget) sc /= 2;
    int64_t slc = slot_cap;
    if (one) slc = (budget - (int64_t)lds_bytes(ws->max_w, (int)sc, (int)lb, 0, 0)) / (64 * 20);
    slc = std::max<int64_t>(0, std::min<int64_t>(ws->max_nblk, slc));
    while (slc > 0 && (int64_t)lds_bytes(ws->max_w, (int)sc, (int)lb, (int)slc, (int)slc) > budget) slc--;
    // keys of further blocks in what LDS is left (a pop's scan reads only keys)
    int64_t slk = std::max<int64_t>(slc, std::min<int64_t>(ws->max_nblk, key_cap));
    while (slk > slc && (int64_t)lds_bytes(ws->max_w, (int)sc, (int)lb, (int)slc, (int)slk) > budget) slk--;
    A.sum_cap = (int32_t)sc;
    A.lb = (int32_t)lb;
    A.slot_cap = (int32_t)slc;
    A.key_cap = (int32_t)slk;
    const size_t lds = lds_bytes(ws->max_w, A.sum_cap, A.lb, A.slot_cap, A.key_cap);
    if (lds > 160 * 1024) return set_error(INSP_E_RANGE, "simulation state of %d workers exceeds LDS", ws->max_w);
    grid = std::max(1, std::min(grid, ws->count));
    hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, st, A.counter);
    {
        ProfScope ps(st, "sim");
        // one-wave loops for machines of at most 64 workers: fixed or direct
        // keys, with or without the data model (the locality policy without
        // it runs on the general loop)
        const bool data = p.data_bw > 0;
        const bool fixed = p.policy == INSP_POLICY_HEFT || p.attr_mode == INSP_ATTR_TRANSITIVE;
        if (ws->max_w <= 64 && !data && p.policy == INSP_POLICY_LOCALITY) {
            if (int rc = set_lds_limit((const void *)&k_sim<1, kLoopGeneral>, lds)) return rc;
            hipLaunchKernelGGL((k_sim<1, kLoopGeneral>), dim3(grid), dim3(2 * kWave), lds, st, A);
        } else if (ws->max_w <= 64) {
            const void *k = data ? (fixed ? (const void *)&k_sim<1, kLoopDataFixed> : (const void *)&k_sim<1, kLoopData>)
                                 : (fixed ? (const void *)&k_sim<1, kLoopFixed> : (const void *)&k_sim<1, kLoopDirect>);
            if (int rc = set_lds_limit(k, lds)) return rc;
            if (data && fixed) hipLaunchKernelGGL((k_sim<1, kLoopDataFixed>), dim3(grid), dim3(2 * kWave), lds, st, A);
            else if (data) hipLaunchKernelGGL((k_sim<1, kLoopData>), dim3(grid), dim3(2 * kWave), lds, st, A);
            else if (fixed) hipLaunchKernelGGL((k_sim<1, kLoopFixed>), dim3(grid), dim3(2 * kWave), lds, st, A);
            else hipLaunchKernelGGL((k_sim<1, kLoopDirect>), dim3(grid), dim3(2 * kWave), lds, st, A);
        } else if (ws->max_w <= 128) {
            if (int rc = set_lds_limit((const void *)&k_sim<2, kLoopGeneral>, lds)) return rc;
            hipLaunchKernelGGL((k_sim<2, kLoopGeneral>), dim3(grid), dim3(64), lds, st, A);
        } else {
            if (int rc = set_lds_limit((const void *)&k_sim<16, kLoopGeneral>, lds)) return rc;
            hipLaunchKernelGGL((k_sim<16, kLoopGeneral>), dim3(grid), dim3(64), lds, st, A);
        }
    }
    INSP_HIP(hipGetLastError());
    if (ws->tasks > 0) {
        ProfScope pr(st, "rec");
        hipLaunchKernelGGL(k_records, dim3((unsigned)((ws->tasks + 255) / 256)), dim3(256), 0, st,
                           ws->tr + ws->base, ws->tasks, worker, start, finish, ie_at_pop, mode_at_pop);
    }
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

}  // namespace insp

using namespace insp;

// Transitive attributes of the range into the handle's arrays, read by the
// simulation as fixed keys.
static int run_sim_transitive(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, hipStream_t st) {
    const int64_t N = std::max<int64_t>(dag->N, 1);
    int rc;
    if ((!dag->tia.p && (rc = dag->tia.alloc(sizeof(int32_t) * N))) ||
        (!dag->tie.p && (rc = dag->tie.alloc(sizeof(int32_t) * N))))
        return rc;
    return run_transitive(dag, ws, est, unit_time, dag->tia.as<int32_t>() + ws->base,
                          dag->tie.as<int32_t>() + ws->base, false, st);
}

static int check_params(const insp_params *p) {
    if (!p) return set_error(INSP_E_INVAL, "null params");
    if (p->attr_mode < 0 || p->attr_mode > INSP_ATTR_TRANSITIVE)
        return set_error(INSP_E_INVAL, "unknown attr_mode %d", p->attr_mode);
    if (p->data_bw < 0) return set_error(INSP_E_INVAL, "negative data_bw");
    if (p->policy < 0 || p->policy > INSP_POLICY_LOCALITY) return set_error(INSP_E_INVAL, "unknown policy %d", p->policy);
    if (p->unit_time < 0 || p->max_events < 0) return set_error(INSP_E_INVAL, "negative unit_time/max_events");
    if (p->k_num > INSP_MAX_TICK || p->k_den > INSP_MAX_TICK) return set_error(INSP_E_RANGE, "k_num/k_den > 2^20");
    return INSP_OK;
}

static int check_workers(const insp_workers *w, int32_t count) {
    for (int32_t i = 0; i < count; i++) {
        if (w[i].n_cpu < 0 || w[i].n_gpu < 0) return set_error(INSP_E_INVAL, "negative worker count");
        int32_t W = w[i].n_cpu + w[i].n_gpu;
        if (W < 1 || W > INSP_MAX_WORKERS) return set_error(INSP_E_RANGE, "worker count %d outside [1, 1024]", W);
    }
    return INSP_OK;
}

// Three work-groups per CU: what the default LDS shape (128 block maxima, 24
// blocks of full entries, keys of 40) leaves room for on machines of up to 20
// workers; larger grids only add work-groups that start when the DAGs are gone.
static int default_grid(int count) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    return std::max(1, std::min(count, cus * 3));
}

extern "C" int insp_schedule(const insp_dag *cdag, int32_t index, const insp_workers *workers, const int32_t *dur,
                             const int32_t *est, const insp_params *params, int32_t *worker, int64_t *start,
                             int64_t *finish, int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop,
                             insp_trace_rec *trace, int32_t *n_events, void *stream) {
    insp_dag *dag = const_cast<insp_dag *>(cdag);
    if (!dag || !workers || !makespan) return set_error(INSP_E_INVAL, "null argument");
    if (index < 0 || index >= dag->B) return set_error(INSP_E_INVAL, "dag index %d out of range", index);
    int rc;
    if ((rc = check_params(params)) || (rc = check_workers(workers, 1))) return rc;
    if (params->data_bw > 0 && !dag->dkib.p) return set_error(INSP_E_INVAL, "data_bw > 0 needs insp_set_task_data");
    const int64_t n = dag->toff[index + 1] - dag->toff[index];
    if (n > 0 && (!dur || !est || !worker || !start || !finish)) return set_error(INSP_E_INVAL, "null array");
    if ((((uintptr_t)dur | (uintptr_t)est) & 7) != 0) return set_error(INSP_E_INVAL, "dur/est rows must be 8-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    INSP_HIP(hipSetDevice(dag->device));
    if ((rc = ensure_state(dag, st))) return rc;
    Workspace *ws;
    if ((rc = get_workspace(dag, index, 1, workers, true, &ws))) return rc;
    if ((rc = run_attributes(dag, ws, est, params->unit_time, nullptr, nullptr, nullptr, true, st))) return rc;
    if (params->policy == INSP_POLICY_HEFT && (rc = run_rank(dag, ws, est, st))) return rc;
    if (params->attr_mode == INSP_ATTR_TRANSITIVE && (rc = run_sim_transitive(dag, ws, est, params->unit_time, st)))
        return rc;
    if (params->data_bw > 0 && (rc = ensure_preds(dag, st))) return rc;
    if (params->data_bw > 0 && !dag->dxc.p && (rc = dag->dxc.alloc(sizeof(int32_t) * std::max<int64_t>(dag->N, 1))))
        return rc;
    return launch_sim(dag, ws, *params, dur, est, worker, start, finish, makespan, ie_at_pop, mode_at_pop, trace,
                      n_events, 1, 1, 4096, 0, 0, st, 0, kScan);
}

static void parse_tune(const char *key, int *waves, int *grid, int *sum_cap, int *slot_cap, int *key_cap, int *prio,
                       int *scan) {
    if (!key) return;
    std::string s(key);
    size_t a = s.find("waves="), b = s.find("grid="), c = s.find("lds_blocks="), d = s.find("lds_slots=");
    size_t e = s.find("prio="), f = s.find("scan="), g = s.find("lds_keys=");
    if (g != std::string::npos) *key_cap = atoi(s.c_str() + g + 9);
    if (e != std::string::npos) *prio = atoi(s.c_str() + e + 5);
    if (f != std::string::npos) *scan = atoi(s.c_str() + f + 5);
    if (a != std::string::npos) *waves = atoi(s.c_str() + a + 6);
    if (b != std::string::npos) *grid = atoi(s.c_str() + b + 5);
    if (c != std::string::npos) *sum_cap = atoi(s.c_str() + c + 11);
    if (d != std::string::npos) *slot_cap = atoi(s.c_str() + d + 10);
}

namespace insp {

int batch_prologue(insp_dag *dag, const insp_workers *workers, const int32_t *dur, const int32_t *est,
                   const insp_params *params, const int32_t *worker, const int64_t *start, const int64_t *finish,
                   const int64_t *makespan, const char *tune_key, BatchLaunch *launch) {
    if (!dag || !workers || !makespan) return set_error(INSP_E_INVAL, "null argument");
    int rc;
    if ((rc = check_params(params)) || (rc = check_workers(workers, dag->B))) return rc;
    if (params->data_bw > 0 && !dag->dkib.p) return set_error(INSP_E_INVAL, "data_bw > 0 needs insp_set_task_data");
    if (dag->N > 0 && (!dur || !est || !worker || !start || !finish)) return set_error(INSP_E_INVAL, "null array");
    if ((((uintptr_t)dur | (uintptr_t)est) & 7) != 0) return set_error(INSP_E_INVAL, "dur/est rows must be 8-byte aligned");
    INSP_HIP(hipSetDevice(dag->device));
    int waves = 1, grid = default_grid(dag->B), sum_cap = 128, slot_cap = 24, key_cap = 40, prio = 0, scan = kScan;
    parse_tune(tune_key, &waves, &grid, &sum_cap, &slot_cap, &key_cap, &prio, &scan);
    if (grid < 1 || sum_cap < 0 || sum_cap > 8192 || slot_cap < 0 || key_cap < 0 || prio < 0 || scan < 0 ||
        scan > kScan || lds_bytes(1, sum_cap, 16, slot_cap, std::max(slot_cap, key_cap)) > 150 * 1024)
        return set_error(INSP_E_INVAL, "bad tune key '%s'", tune_key);
    // one wave simulates one DAG; no other shape is implemented
    if (waves != 1) return set_error(INSP_E_INVAL, "tune key '%s': only waves=1 is supported", tune_key);
    launch->grid = grid;
    launch->sum_cap = sum_cap;
    launch->slot_cap = slot_cap;
    launch->key_cap = key_cap;
    launch->prio = prio;
    launch->scan = scan;
    return INSP_OK;
}

}  // namespace insp

static int schedule_batch(const insp_dag *cdag, const insp_workers *workers, const int32_t *dur, const int32_t *est,
                          const insp_params *params, int32_t *worker, int64_t *start, int64_t *finish,
                          int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop, insp_trace_rec *trace,
                          int32_t *n_events, const char *tune_key, void *stream) {
    insp_dag *dag = const_cast<insp_dag *>(cdag);
    BatchLaunch bl;
    int rc;
    if ((rc = batch_prologue(dag, workers, dur, est, params, worker, start, finish, makespan, tune_key, &bl)))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = ensure_state(dag, st))) return rc;
    Workspace *ws;
    if ((rc = get_workspace(dag, 0, dag->B, workers, true, &ws))) return rc;
    if ((rc = run_attributes(dag, ws, est, params->unit_time, nullptr, nullptr, nullptr, true, st))) return rc;
    if (params->policy == INSP_POLICY_HEFT && (rc = run_rank(dag, ws, est, st))) return rc;
    if (params->attr_mode == INSP_ATTR_TRANSITIVE && (rc = run_sim_transitive(dag, ws, est, params->unit_time, st)))
        return rc;
    if (params->data_bw > 0 && (rc = ensure_preds(dag, st))) return rc;
    if (params->data_bw > 0 && !dag->dxc.p && (rc = dag->dxc.alloc(sizeof(int32_t) * std::max<int64_t>(dag->N, 1))))
        return rc;
    return launch_sim(dag, ws, *params, dur, est, worker, start, finish, makespan, ie_at_pop, mode_at_pop, trace,
                      n_events, 1, bl.grid, bl.sum_cap, bl.slot_cap, bl.key_cap, st, bl.prio, bl.scan);
}

extern "C" int insp_schedule_batch(const insp_dag *cdag, const insp_workers *workers, const int32_t *dur,
                                   const int32_t *est, const insp_params *params, int32_t *worker, int64_t *start,
                                   int64_t *finish, int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop,
                                   const char *tune_key, void *stream) {
    return schedule_batch(cdag, workers, dur, est, params, worker, start, finish, makespan, ie_at_pop, mode_at_pop,
                          nullptr, nullptr, tune_key, stream);
}

extern "C" int insp_schedule_batch_trace(const insp_dag *cdag, const insp_workers *workers, const int32_t *dur,
                                         const int32_t *est, const insp_params *params, int32_t *worker,
                                         int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop,
                                         int8_t *mode_at_pop, insp_trace_rec *trace, int32_t *n_events,
                                         const char *tune_key, void *stream) {
    if (!trace || !n_events) return set_error(INSP_E_INVAL, "insp_schedule_batch_trace: null trace or n_events");
    return schedule_batch(cdag, workers, dur, est, params, worker, start, finish, makespan, ie_at_pop, mode_at_pop,
                          trace, n_events, tune_key, stream);
}

// A batch step captured in a HIP graph owned by the library.
struct insp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

extern "C" void insp_batch_graph_free(insp_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

extern "C" int insp_batch_graph_create(const insp_dag *cdag, const insp_workers *workers, const int32_t *dur,
                                       const int32_t *est, const insp_params *params, int32_t *worker,
                                       int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop,
                                       int8_t *mode_at_pop, const char *tune_key, void *stream, insp_graph **out) {
    if (!out) return set_error(INSP_E_INVAL, "null out");
    *out = nullptr;
    // an eager step first: it builds every buffer made on first use and sets
    // the kernels' attributes, so that the captured step only launches kernels
    int rc = insp_schedule_batch(cdag, workers, dur, est, params, worker, start, finish, makespan, ie_at_pop,
                                 mode_at_pop, tune_key, stream);
    if (rc) return rc;
    INSP_HIP(hipStreamSynchronize((hipStream_t)stream));
    std::unique_ptr<insp_graph> g(new insp_graph());
    g->device = cdag->device;
    hipStream_t cs = nullptr;
    INSP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        prof_suspend(true);
        rc = insp_schedule_batch(cdag, workers, dur, est, params, worker, start, finish, makespan, ie_at_pop,
                                 mode_at_pop, tune_key, cs);
        prof_suspend(false);
        e = hipStreamEndCapture(cs, &g->graph);
    }
    (void)hipStreamDestroy(cs);
    if (rc) return rc;
    if (e != hipSuccess) return set_error(INSP_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    INSP_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    *out = g.release();
    return INSP_OK;
}

extern "C" int insp_batch_graph_launch(insp_graph *g, void *stream) {
    if (!g || !g->exec) return set_error(INSP_E_INVAL, "null graph");
    INSP_HIP(hipSetDevice(g->device));
    INSP_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return INSP_OK;
}

#ifdef INSP_PHASE_CLOCKS
extern "C" int insp_debug_phase_clocks(unsigned long long *host, int count) {
    INSP_HIP(hipMemcpyFromSymbol(host, HIP_SYMBOL(g_phase_clk), sizeof(unsigned long long) * 32 * count));
    return INSP_OK;
}
#endif

extern "C" int insp_sync_status(const insp_dag *cdag, void *stream) {
    if (!cdag) return set_error(INSP_E_INVAL, "null handle");
    insp_dag *dag = const_cast<insp_dag *>(cdag);
    hipStream_t st = (hipStream_t)stream;
    INSP_HIP(hipSetDevice(dag->device));
    INSP_HIP(hipStreamSynchronize(st));
    if (!dag->dag_stat.p) return INSP_OK;
    // the latest schedule's status words and the failures of earlier calls
    // not yet reported; both are cleared once read
    std::vector<int32_t> stat(2 * dag->B), sticky(dag->B);
    INSP_HIP(hipMemcpyAsync(stat.data(), dag->dag_stat.p, sizeof(int32_t) * 2 * dag->B, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipMemcpyAsync(sticky.data(), dag->dag_sticky.p, sizeof(int32_t) * dag->B, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    bool any = false;
    for (int32_t b = 0; b < dag->B; b++) {
        any |= (stat[2 * b] | sticky[b]) != 0;
        stat[2 * b] |= sticky[b];
    }
    if (any) {
        std::vector<int32_t> zero(2 * dag->B, 0);
        for (int32_t b = 0; b < dag->B; b++) zero[2 * b + 1] = stat[2 * b + 1];  // event counts stay
        INSP_HIP(hipMemcpyAsync(dag->dag_stat.p, zero.data(), sizeof(int32_t) * 2 * dag->B, hipMemcpyHostToDevice, st));
        INSP_HIP(hipMemsetAsync(dag->dag_sticky.p, 0, sizeof(int32_t) * dag->B, st));
        INSP_HIP(hipStreamSynchronize(st));
    }
    for (int32_t b = 0; b < dag->B; b++) {
        if (stat[2 * b] & ST_EST) return set_error(INSP_E_RANGE, "estimate outside [1, 2^20] in DAG %d", b);
        if (stat[2 * b] & ST_DUR) return set_error(INSP_E_RANGE, "duration outside [1, 2^20] in DAG %d", b);
        if (stat[2 * b] & ST_RANK) return set_error(INSP_E_RANGE, "HEFT rank of DAG %d reaches 2^42", b);
        if (stat[2 * b] & ST_PATH) return set_error(INSP_E_RANGE, "longest path of DAG %d reaches 2^30 ticks", b);
        if (stat[2 * b] & ST_XFER)
            return set_error(INSP_E_RANGE, "input transfers of a task of DAG %d exceed 2^20 ticks", b);
        if (stat[2 * b] & ST_HANG)
            return set_error(INSP_E_HANG, "DAG %d needed more than max_events events", b);
    }
    return INSP_OK;
}
