// Inspiring ability and efficiency (Sections 4.2 and 4.3 of the paper).
//
//   IA(v) = out-degree of v.
//   IE(v) = #{ s in succ(v) : rem[s] == 1 and tau(v) + tau(s) <= U }, tau the
//           GPU estimate (CPU estimate on machines without GPU workers).
//   U     = given, or the ladder choice: U = 2^j for j = 0..J, 2^J the first
//           power of two >= 2 max tau, maximising #{v : 0 < IE(v) < IA(v)},
//           the larger U on a tie.
//
// A task contributes to the score of rung j exactly when IE(v; 2^j) is
// positive but below IA(v): with x_s = tau(v) + tau(s) over successors with
// rem == 1, IE > 0 iff 2^j >= min x_s, and IE == IA iff every successor has
// rem == 1 and 2^j >= max x_s.  So each task adds +1 at rung ceil(log2 min x)
// and -1 at rung ceil(log2 max x) (or never), a difference histogram whose
// running sum over the rungs is the score.  Pass A scans every successor
// list once for all rungs; pass B scans it again to count IE at the chosen U.
//
// Both passes are edge-parallel over chunks of 64 rows, one wave each: the
// scanned rows' successor lists are laid end to end and every lane takes
// every 64th edge (contiguous successor reads), finding its row by binary
// search over the chunk's offsets in LDS; per-row counts and extremes are
// LDS atomics.  Each task is looked up through one 32-bit word, tau with the
// rem == 1 flag.  Two layouts:
//   - k_attr_dag: one work-group per DAG (DAGs below kGridMin tasks; 1024
//     threads above kMidTasks tasks, 256 below, so that several small DAGs
//     share a CU) with the DAG's task words in LDS: pass A, the choice of U, then
//     pass B while the DAG's rows are still in L2 -- every array crosses HBM
//     once and no lookup leaves the CU.  With the ladder's U = 2^j, pass A
//     also leaves one decision word per row (count and the rungs of its least
//     and largest tau(v) + tau(s)), and pass B takes a row per thread, reading
//     the successors only of rows whose span U splits.
//   - k_attr_pack / k_attr_big_a / k_attr_big_sel / k_attr_big_b: one large
//     DAG over a persistent grid: its task words packed to one array (and a
//     16-bit copy for the gathers), pass A leaving a summary per row (count
//     of rem == 1 successors, least and largest tau(v) + tau(s)) and a
//     partial score per work-group, U from the partial scores, then pass B
//     deciding IE from the summary for every row whose count U does not
//     split.  Rows with more than kHubDeg successors (listed once per handle,
//     largest first) get a wave each, or one per kPiece successors when
//     longer than kPieceMin; the select kernel combines the pieces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

__device__ __forceinline__ int ceil_log2(int32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

// Make a wave's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T dev_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void dev_store(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t wave_sum_i32(int32_t x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

struct AttrArgs {
    const DagDesc *desc;
    const int32_t *sorder;      // per-DAG pass: desc indices, largest DAG first
    const int4 *hub;            // grid pass: hub rows of the large DAGs (row, piece, pieces, first piece slot)
    int32_t *pslot;             // grid pass: per-piece partial results of rows cut into pieces (4 ints each)
    const int4 *lrow;           // grid pass: the rows cut into pieces (row, 0, pieces, first piece slot)
    int32_t *part;              // grid pass: per-block partial results [kBigGrid][32]
    uint32_t *pkg;              // grid pass: task words of the large DAG (by row)
    unsigned long long *summ;   // grid pass: each row's pass-A summary
    uint32_t *srow;             // per-DAG pass, ladder U: each row's pass-A decision word, 16 bits (global task index;
                                // scratch the simulation reuses later)
    int32_t first;              // DAG id of desc[0]
    const int32_t *rp, *col;
    const unsigned long long *word0;
    const int32_t *est, *rem;   // user arrays, indexed relative to `base`
    int64_t base;
    int64_t tasks;
    int32_t count;
    int32_t unit_time;
    int32_t *maxtau;  // per DAG: a large DAG's largest tau when above kTau8, else 0
    int32_t *score, *u, *taubar, *done;
    int32_t *stat;    // this call's status words (stride 2)
    int32_t *sticky;  // schedule calls: failures of earlier calls kept for insp_sync_status (nullable)
    int32_t *anybad;  // [1]: some DAG of the call has an estimate out of range
    unsigned long long *tausum;
};

struct AttrOut {
    int32_t *ia_out, *ie_out;   // user arrays (nullable), relative to base
    int sim_init;
    TaskRec *tr;
    unsigned long long *dep;    // the simulation's dependency words
};

// Status words, per-DAG accumulators and the defaults (U for an empty DAG).
__global__ void k_attr_clear(AttrArgs a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *a.anybad = 0;
    if (i >= a.count) return;
    int32_t id = a.desc[i].id;
    a.done[id] = 0;
    a.maxtau[id] = 0;
    a.u[id] = a.unit_time > 0 ? a.unit_time : 1;
    a.taubar[id] = 1;
    // a schedule call keeps the previous call's failures until they are
    // reported: they move to the sticky word before the status restarts
    if (a.sticky) a.sticky[id] |= a.stat[2 * id];
    a.stat[2 * id] = 0;
}

// DAG index (into desc) of the task at offset t from base.
__device__ int32_t dag_of(const AttrArgs &a, int64_t t) {
    int32_t lo = 0, hi = a.count - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (a.desc[mid].toff - a.base <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Attribute-only calls validate every estimate first: a failing call writes
// no output at all.
__global__ __launch_bounds__(256) void k_est_check(AttrArgs a) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < a.tasks; t += (int64_t)gridDim.x * 256) {
        const int2 e = reinterpret_cast<const int2 *>(a.est)[t];
        if (e.x < 1 || e.x > INSP_MAX_TICK || e.y < 1 || e.y > INSP_MAX_TICK) {
            atomicOr(&a.stat[2 * a.desc[dag_of(a, t)].id], ST_EST);
            *a.anybad = 1;
        }
    }
}

// U and the regulator's mean tau of one DAG from its score histogram.
__device__ void select_unit(const AttrArgs &a, int32_t id, int32_t n, int32_t mt, unsigned long long ts,
                            const int32_t *score) {
    int J = 0;
    while (((int64_t)1 << J) < 2 * (int64_t)mt) J++;
    int32_t run = 0, best = -1, bj = 0;
    for (int j = 0; j <= J; j++) {
        run += score[j];
        if (run >= best) {
            best = run;
            bj = j;
        }
    }
    a.u[id] = a.unit_time > 0 ? a.unit_time : (1 << bj);
    long long tb = n > 0 ? (long long)(ts / (unsigned long long)n) : 1;
    a.taubar[id] = (int32_t)(tb < 1 ? 1 : tb);
}

// Per-task word of both passes: tau | (rem == 1) << 31.
constexpr uint32_t kRem1 = 1u << 31;

// A row's pass-A summary (grid pass): successors with rem == 1, and the
// minimum and maximum of tau(v) + tau(s) over them, less one (each < 2^21).
__device__ __forceinline__ unsigned long long pack_summary(int32_t cnt1, int32_t lo, int32_t hi) {
    if (cnt1 <= 0) return 0ull;
    return (unsigned long long)cnt1 | (unsigned long long)(lo - 1) << 21 | (unsigned long long)(hi - 1) << 42;
}
__device__ __forceinline__ void unpack_summary(unsigned long long w, int32_t &cnt1, int32_t &lo, int32_t &hi) {
    cnt1 = (int32_t)(w & 0x1FFFFF);
    lo = (int32_t)(w >> 21 & 0x1FFFFF) + 1;
    hi = (int32_t)(w >> 42 & 0x1FFFFF) + 1;
}

// A row's pass-A result for a U that is a power of two, 2^j: the count of
// successors with rem == 1 (< 2^22) and the rungs ceil(log2) of the least and
// largest tau(v) + tau(s) over them (each <= 22).  Since x <= 2^j exactly when
// ceil(log2 x) <= j, IE at U = 2^j is the count when the largest rung is <= j,
// zero when the least is > j, and needs the row's successors only otherwise.
// Kept in 16 bits: the count in bits 0..5, the rungs in 6..10 and 11..15; a
// count of 63 or more is stored as 63 with rungs 0 and 31, which sends the row
// to the rescan at every U of the ladder.
__device__ __forceinline__ uint16_t decision_word(int32_t cnt1, int32_t lo, int32_t hi) {
    if (cnt1 <= 0) return 0;
    if (cnt1 >= 63) return (uint16_t)(63u | 31u << 11);
    return (uint16_t)((uint32_t)cnt1 | (uint32_t)ceil_log2(lo) << 6 | (uint32_t)ceil_log2(hi) << 11);
}

// The task word from the inputs: rem (given, or the in-degree in the high
// word of word0) and the estimate row; `bad` flags an estimate out of range.
template <bool HAS_REM>
__device__ __forceinline__ uint32_t task_word(const AttrArgs &a, const DagDesc &d, int32_t v, bool &bad) {
    const int64_t ub = d.toff - a.base;
    const int2 e = reinterpret_cast<const int2 *>(a.est)[ub + v];
    const int32_t rm = HAS_REM ? a.rem[ub + v]
                               : (int32_t)(reinterpret_cast<const uint32_t *>(a.word0 + d.toff)[2 * v + 1] >> 11);
    bad = e.x < 1 || e.x > INSP_MAX_TICK || e.y < 1 || e.y > INSP_MAX_TICK;
    return (uint32_t)(d.n_gpu > 0 ? e.y : e.x) | (rm == 1 ? kRem1 : 0u);
}

// One wave's scratch for a chunk of 64 rows.
struct ChunkLds {
    int32_t pre[kWave + 1];  // exclusive prefix of the scanned rows' out-degrees
    int32_t e0[kWave];       // first edge of each row (DAG-local)
    int32_t tau[kWave];
    int32_t cnt[kWave], lo[kWave], hi[kWave];
};

constexpr int kWin = 8;  // 64-edge windows whose loads are issued together

// A wave's walk over 64-row chunks c0, c0 + stride, ...: each step returns
// the first edge and out-degree of row c0 + lane of the current chunk and
// starts the next chunk's row-offset reads, so that they are in flight while
// the current chunk is scanned.
struct RowPrefetch {
    const int32_t *r;
    int32_t n, c0, stride, e0, e1;
    __device__ RowPrefetch(const int32_t *r_, int32_t n_, int32_t c0_, int32_t stride_)
        : r(r_), n(n_), c0(c0_), stride(stride_) {
        load();
    }
    __device__ void load() {
        const int32_t vv = min(c0 + lane_id(), n - 1);
        e0 = r[max(vv, 0)];
        e1 = r[max(vv, 0) + 1];
    }
    __device__ void next(int32_t &first, int32_t &deg) {
        first = e0;
        deg = c0 + lane_id() < n ? e1 - e0 : 0;
        c0 += stride;
        if (c0 < n) load();
    }
};

// Edge-parallel scan of one wave's chunk: the scanned rows' successor lists
// laid end to end, every 64th edge per lane.  A lane finds the row of its
// edge by binary search over the prefix in LDS; successor reads are
// contiguous within rows; the task words come from `pk` (LDS or global).
// Indices are clamped so every load of a window group is unconditional.
// Pass A returns per row the count of rem == 1 successors and the extremes
// of tau(v) + tau(s) over them; pass B the count with tau(v) + tau(s) <= U.
template <bool PASS_B, typename PK>
__device__ __forceinline__ void chunk_scan(const int32_t *c, int32_t e0, int32_t sdeg, int32_t tau, int64_t U,
                                           PK pk, ChunkLds &L, int32_t &cnt, int32_t &lo, int32_t &hi) {
    const int lane = lane_id();
    const int32_t inc = wave_incl_scan(sdeg);
    const int32_t total = read_lane(inc, kWave - 1);
    L.pre[lane] = inc - sdeg;
    if (lane == kWave - 1) L.pre[kWave] = total;
    L.e0[lane] = e0;
    L.tau[lane] = tau;
    L.cnt[lane] = 0;
    L.lo[lane] = INT_MAX;
    L.hi[lane] = 0;
    wave_sync();
    for (int32_t k0 = 0; k0 < total; k0 += kWave * kWin) {
        int32_t q[kWin], sv[kWin];
        uint32_t pv[kWin];
#pragma unroll
        for (int u = 0; u < kWin; u++) {
            const int32_t k = min(k0 + u * kWave + lane, total - 1);
            int32_t r = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) r += L.pre[r + step] <= k ? step : 0;
            q[u] = r;
            sv[u] = c[L.e0[r] + (k - L.pre[r])];
        }
#pragma unroll
        for (int u = 0; u < kWin; u++) pv[u] = pk(sv[u]);
#pragma unroll
        for (int u = 0; u < kWin; u++) {
            if (k0 + u * kWave + lane < total && (pv[u] & kRem1)) {
                const int32_t x = L.tau[q[u]] + (int32_t)(pv[u] & ~kRem1);
                if (PASS_B) {
                    if ((int64_t)x <= U) atomicAdd(&L.cnt[q[u]], 1);
                } else {
                    atomicAdd(&L.cnt[q[u]], 1);
                    atomicMin(&L.lo[q[u]], x);
                    atomicMax(&L.hi[q[u]], x);
                }
            }
        }
    }
    wave_sync();
    cnt = L.cnt[lane];
    lo = L.lo[lane];
    hi = L.hi[lane];
    wave_sync();  // the next chunk rewrites L
}

// Score contribution of a row: +1 at the first rung where IE > 0, -1 at the
// first rung where IE == IA (kRungs - 1: never).
__device__ __forceinline__ void add_rungs(int32_t *hist, int32_t cnt1, int32_t lo, int32_t hi, int32_t deg) {
    if (cnt1 <= 0) return;
    const int jlo = ceil_log2(lo), jhi = cnt1 == deg ? ceil_log2(hi) : kRungs - 1;
    if (jlo < jhi) {
        atomicAdd(&hist[jlo], 1);
        atomicAdd(&hist[jhi], -1);
    }
}

// The outputs of one row: IA/IE for an attribute call, else the simulation
// record and dependency word (w0, the row's initial word) -- or an
// "unscheduled" record when the DAG's estimates failed.
__device__ __forceinline__ void write_row_w(const AttrArgs &a, const AttrOut &o, const DagDesc &d, int32_t v,
                                            int32_t e0, int32_t deg, int32_t tau, int32_t ie, unsigned long long w0,
                                            bool failed = false, bool put_dep = true) {
    const int64_t ub = d.toff - a.base;
    if (o.sim_init) {
        const int64_t t = d.toff + v;
        TaskRec rec;
        if (failed) {
            memset(&rec, 0, sizeof rec);
            rec.qpos = -1;
        } else {
            if (put_dep) o.dep[t] = w0;
            rec.word = 0;
            rec.iev = ie;
            rec.qpos = -1;
            rec.ia = deg;
            rec.tau = tau;
            rec.rs = e0;
            rec.seq = 0;
        }
        o.tr[t] = rec;
    } else if (!failed) {
        if (o.ia_out) o.ia_out[ub + v] = deg;
        if (o.ie_out) o.ie_out[ub + v] = ie;
    }
}
__device__ __forceinline__ void write_row(const AttrArgs &a, const AttrOut &o, const DagDesc &d, int32_t v,
                                          int32_t e0, int32_t deg, int32_t tau, int32_t ie, bool failed,
                                          bool put_dep = true) {
    const unsigned long long w0 = o.sim_init && !failed && put_dep ? a.word0[d.toff + v] : 0ull;
    write_row_w(a, o, d, v, e0, deg, tau, ie, w0, failed, put_dep);
}

// Whether the call writes nothing for DAG d: a schedule skips a DAG whose
// estimates failed, an attribute call writes nothing when any DAG failed.
__device__ __forceinline__ bool dag_failed(const AttrArgs &a, const AttrOut &o, const DagDesc &d) {
    return o.sim_init ? (dev_load(&a.stat[2 * d.id]) & ST_EST) != 0 : dev_load(a.anybad) != 0;
}

// Reduce a per-wave max, sum and flag over a work-group (slots per wave).
struct WaveSlots {
    uint32_t wmax[16];
    unsigned long long wsum[16];
    int32_t bad;
};

constexpr int kDagThreads = 1024;  // work-group of a DAG of more than kMidTasks tasks
constexpr int kMidThreads = 256;   // ... of the others: several such DAGs share a CU
constexpr int kMidTasks = 4096;

// One wave's scratch in the per-DAG kernel.
struct DagLds {
    int32_t pre[kWave + 1];  // exclusive prefix of the chunk's out-degrees
    int32_t cnt[kWave], lo[kWave], hi[kWave];
};

// One wave's share of a pass over a small DAG whose task words are in LDS:
// chunks c0, c0 + stride, ... of 64 rows.  Every row is scanned, so a
// chunk's successors are the contiguous edge range from its first row's
// offset; the next chunk's row offsets and first kWin * 64 successors are
// read while the current chunk is worked on.  Per row, `done` receives
// (row, first edge, out-degree, count, least, largest) as chunk_scan defines
// them.
template <bool PASS_B, typename PK, typename Done>
__device__ __forceinline__ void dag_pass(const int32_t *r, const int32_t *c, int32_t n, PK pks, int32_t c0,
                                         int32_t stride, int64_t U, DagLds &L, Done done) {
    const int lane = lane_id();
    if (c0 >= n) return;
    // the current chunk: row offsets, degrees, prefix, first successors
    int32_t v = c0 + lane;
    int32_t e0 = r[min(v, n - 1)], e1 = r[min(v, n - 1) + 1];
    int32_t deg = v < n ? e1 - e0 : 0;
    int32_t inc = wave_incl_scan(deg);
    int32_t total = read_lane(inc, kWave - 1), E0 = read_lane(e0, 0);
    int32_t sv[kWin];
#pragma unroll
    for (int u = 0; u < kWin; u++) sv[u] = total > 0 ? c[E0 + min(u * kWave + lane, total - 1)] : 0;
    int32_t nv = c0 + stride + lane;
    int32_t ne0 = 0, ne1 = 0;
    if (c0 + stride < n) {
        ne0 = r[min(nv, n - 1)];
        ne1 = r[min(nv, n - 1) + 1];
    }
    for (;;) {
        L.pre[lane] = inc - deg;
        if (lane == kWave - 1) L.pre[kWave] = total;
        L.cnt[lane] = 0;
        L.lo[lane] = INT_MAX;
        L.hi[lane] = 0;
        wave_sync();
        // start the next chunk: its prefix and first successors
        const bool more = c0 + stride < n;
        int32_t ndeg = 0, ninc = 0, ntotal = 0, nE0 = 0, nsv[kWin];
        if (more) {
            ndeg = nv < n ? ne1 - ne0 : 0;
            ninc = wave_incl_scan(ndeg);
            ntotal = read_lane(ninc, kWave - 1);
            nE0 = read_lane(ne0, 0);
#pragma unroll
            for (int u = 0; u < kWin; u++) nsv[u] = ntotal > 0 ? c[nE0 + min(u * kWave + lane, ntotal - 1)] : 0;
        }
        // the current chunk's successors
        for (int32_t k0 = 0; k0 < total; k0 += kWave * kWin) {
            if (k0 > 0) {
#pragma unroll
                for (int u = 0; u < kWin; u++) sv[u] = c[E0 + min(k0 + u * kWave + lane, total - 1)];
            }
#pragma unroll
            for (int u = 0; u < kWin; u++) {
                const int32_t k = min(k0 + u * kWave + lane, total - 1);
                int32_t q = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1) q += L.pre[q + step] <= k ? step : 0;
                const uint32_t pv = pks(sv[u]);
                if (k0 + u * kWave + lane < total && (pv & kRem1)) {
                    const int32_t x = (int32_t)(pks(c0 + q) & ~kRem1) + (int32_t)(pv & ~kRem1);
                    if (PASS_B) {
                        if ((int64_t)x <= U) atomicAdd(&L.cnt[q], 1);
                    } else {
                        atomicAdd(&L.cnt[q], 1);
                        atomicMin(&L.lo[q], x);
                        atomicMax(&L.hi[q], x);
                    }
                }
            }
        }
        wave_sync();
        done(v, e0, deg, L.cnt[lane], L.lo[lane], L.hi[lane]);
        wave_sync();
        if (!more) break;
        c0 += stride;
        v = nv;
        e0 = ne0;
        deg = ndeg;
        inc = ninc;
        total = ntotal;
        E0 = nE0;
#pragma unroll
        for (int u = 0; u < kWin; u++) sv[u] = nsv[u];
        nv = c0 + stride + lane;
        if (c0 + stride < n) {
            ne0 = r[min(nv, n - 1)];
            ne1 = r[min(nv, n - 1) + 1];
        }
    }
}

// 16-bit copy of a task word for the per-DAG kernel's LDS: tau (saturated at
// 2^15 - 1) in bits 0..14, rem == 1 in bit 15.  It is exact, and used, only
// for DAGs whose largest tau is below 2^15 ticks.
constexpr uint32_t kTau16 = 0x7FFF;
__device__ __forceinline__ uint16_t word16(uint32_t w) {
    return (uint16_t)(min(w & ~kRem1, kTau16) | ((w & kRem1) ? 0x8000u : 0u));
}
__device__ __forceinline__ uint32_t word32(uint32_t h) { return (h & kTau16) | (h & 0x8000u) << 16; }

// The grid pass keeps narrow copies of the large DAG's task words beside the
// 32-bit ones, in the decision-word scratch of its own rows (4 bytes per row,
// which only the per-DAG kernel uses): 16 bits at byte 0 and 8 bits (tau
// saturated at kTau8, rem == 1 in bit 7) at byte 2n.  When no tau of the DAG
// exceeds kTau8 the gathers of both passes read the 8-bit copy (a 2 MB array
// for 2M tasks, which the L2 holds), otherwise the 16-bit one, a saturated
// entry sending the lookup to the 32-bit word.
constexpr uint32_t kTau8 = 0x7E;
__device__ __forceinline__ uint8_t word8(uint32_t w) {
    return (uint8_t)(min(w & ~kRem1, kTau8 + 1) | ((w & kRem1) ? 0x80u : 0u));
}
__device__ __forceinline__ uint16_t *pk16_of(const AttrArgs &a, const DagDesc &d) {
    return reinterpret_cast<uint16_t *>(a.srow + d.toff);
}
__device__ __forceinline__ uint8_t *pk8_of(const AttrArgs &a, const DagDesc &d) {
    return reinterpret_cast<uint8_t *>(a.srow + d.toff) + 2 * (int64_t)d.n;
}
struct GridWords {
    const uint32_t *pkg;
    const uint16_t *p16;
    __device__ uint32_t operator()(int32_t s) const {
        const uint32_t h = p16[s];
        return (h & kTau16) == kTau16 ? pkg[s] : word32(h);
    }
};
struct GridBytes {
    const uint8_t *p8;
    __device__ uint32_t operator()(int32_t s) const {
        const uint32_t h = p8[s];
        return (h & 0x7Fu) | (h & 0x80u) << 24;
    }
};

// Pass A, the choice of U and pass B of one DAG in the per-DAG kernel, with
// the task words looked up through pk (LDS or the inputs).
// SIM: a schedule call whose pack phase has already copied the dependency
// words (an attribute-only call keeps the general path).
template <bool SIM, int TPB, typename PK>
__device__ __forceinline__ void dag_passes(const AttrArgs &a, const AttrOut &o, const DagDesc &d, PK pk,
                                           DagLds *dl, WaveSlots &ws, int32_t *hist) {
    constexpr int kDagThreads = TPB, kDagWaves = TPB / kWave;
    const int tid = threadIdx.x, wv = tid / kWave;
    const int32_t *r = a.rp + d.toff + d.id;
    const int32_t *c = a.col + d.eoff;
    const bool ability = a.unit_time == 0;
    uint16_t *srow = reinterpret_cast<uint16_t *>(a.srow) + d.toff;
    dag_pass<false>(r, c, d.n, pk, wv * kWave, kDagThreads, 0, dl[wv],
                    [&](int32_t v, int32_t, int32_t deg, int32_t cnt, int32_t lo, int32_t hi) {
                        if (v < d.n && ability) {
                            add_rungs(hist, cnt, lo, hi, deg);
                            srow[v] = decision_word(cnt, lo, hi);
                        }
                    });
    __syncthreads();
    if (tid == 0) {
        uint32_t m = 0;
        unsigned long long sm = 0;
        for (int w = 0; w < kDagWaves; w++) {
            m = max(m, ws.wmax[w]);
            sm += ws.wsum[w];
        }
        select_unit(a, d.id, d.n, (int32_t)m, sm, hist);
        if (ws.bad) {
            atomicOr(&a.stat[2 * d.id], ST_EST);
            *a.anybad = 1;
        }
    }
    __syncthreads();
    if (o.sim_init && ws.bad != 0) {
        for (int32_t v = tid; v < d.n; v += kDagThreads) write_row(a, o, d, v, 0, 0, 0, 0, true);
        return;
    }
    const int32_t U = a.u[d.id];
    if (ability) {
        // U = 2^j from the ladder: a row per thread, IE from its decision
        // word; a row that U splits counts its successors itself.  Each
        // thread loads kRB rows' words before it uses any of them.
        constexpr int kRB = 4;
        const int j = __builtin_ctz((uint32_t)U);
        for (int32_t v0 = tid; v0 < d.n; v0 += kRB * kDagThreads) {
            uint32_t sw[kRB];
            int32_t e0[kRB], e1[kRB];
            unsigned long long w0[kRB];
#pragma unroll
            for (int k = 0; k < kRB; k++) {
                const int32_t vv = min(v0 + k * kDagThreads, d.n - 1);
                sw[k] = srow[vv];
                e0[k] = r[vv];
                e1[k] = r[vv + 1];
                w0[k] = !SIM && o.sim_init ? a.word0[d.toff + vv] : 0ull;
            }
#pragma unroll
            for (int k = 0; k < kRB; k++) {
                const int32_t v = v0 + k * kDagThreads;
                if (v >= d.n) break;
                const uint32_t w = sw[k];
                const int32_t tv = (int32_t)(pk(v) & ~kRem1);
                const int32_t cnt = (int32_t)(w & 63), jl = (int32_t)(w >> 6 & 31), jh = (int32_t)(w >> 11 & 31);
                int32_t ie = 0;
                if (cnt > 0 && jh <= j) {
                    ie = cnt;
                } else if (cnt > 0 && jl <= j) {
                    for (int32_t e = e0[k]; e < e1[k]; e++) {
                        const uint32_t pv = pk(c[e]);
                        if ((pv & kRem1) && (int64_t)tv + (int32_t)(pv & ~kRem1) <= (int64_t)U) ie++;
                    }
                }
                write_row_w(a, o, d, v, e0[k], e1[k] - e0[k], tv, ie, w0[k], false, !SIM);
            }
        }
        return;
    }
    dag_pass<true>(r, c, d.n, pk, wv * kWave, kDagThreads, U, dl[wv],
                   [&](int32_t v, int32_t e0, int32_t deg, int32_t cnt, int32_t, int32_t) {
                       if (v < d.n) write_row(a, o, d, v, e0, deg, (int32_t)(pk(v) & ~kRem1), cnt, false, !SIM);
                   });
}

// One work-group per DAG: the DAG's task words in LDS, both passes and the
// choice of U.  The words take 16 bits each and the kernel at most 64 VGPRs,
// so that two work-groups of the largest DAGs (eight of the smaller ones)
// share a CU; a DAG with a tau of 2^15 ticks or more looks its task words up
// from the inputs instead.  The DAGs taken are sorder[first + blockIdx.x];
// dynamic LDS: 2 bytes per task of the largest of them.
template <bool HAS_REM, bool SIM, int TPB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(8))) void k_attr_dag(AttrArgs a, AttrOut oin,
                                                                                         int32_t first) {
    constexpr int kDagThreads = TPB, kDagWaves = TPB / kWave;
    const AttrOut &o = oin;
    extern __shared__ uint16_t pks16[];
    __shared__ DagLds dl[kDagWaves];
    __shared__ WaveSlots ws;
    __shared__ int32_t hist[kRungs];
    const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
    const DagDesc d = a.desc[a.sorder[first + blockIdx.x]];
    if (!o.sim_init && dev_load(a.anybad)) return;  // validated before: the call fails
    if (tid < kRungs) hist[tid] = 0;
    if (tid == 0) ws.bad = 0;
    uint32_t tmax = 0;
    unsigned long long tsum = 0;
    bool bad = false;
    constexpr int kTW = 4;  // task words loaded per thread at a time
    for (int32_t v0 = tid; v0 < d.n; v0 += kTW * kDagThreads) {
        uint32_t w[kTW];
        bool b[kTW];
        unsigned long long w0[kTW];
        if constexpr (!HAS_REM && SIM) {
            // a schedule call: each dependency word read whole, its in-degree
            // the task's rem, and copied to the simulation's array here, so
            // that pass B need not read it again
#pragma unroll
            for (int k = 0; k < kTW; k++) {
                const int32_t vv = min(v0 + k * kDagThreads, d.n - 1);
                w0[k] = a.word0[d.toff + vv];
                const int2 e = reinterpret_cast<const int2 *>(a.est)[d.toff - a.base + vv];
                b[k] = e.x < 1 || e.x > INSP_MAX_TICK || e.y < 1 || e.y > INSP_MAX_TICK;
                w[k] = (uint32_t)(d.n_gpu > 0 ? e.y : e.x) | ((w0[k] >> 43) == 1 ? kRem1 : 0u);
            }
#pragma unroll
            for (int k = 0; k < kTW; k++)
                if (v0 + k * kDagThreads < d.n) o.dep[d.toff + v0 + k * kDagThreads] = w0[k];
        } else {
#pragma unroll
            for (int k = 0; k < kTW; k++) w[k] = task_word<HAS_REM>(a, d, min(v0 + k * kDagThreads, d.n - 1), b[k]);
        }
#pragma unroll
        for (int k = 0; k < kTW; k++) {
            if (v0 + k * kDagThreads >= d.n) continue;
            pks16[v0 + k * kDagThreads] = word16(w[k]);
            bad |= b[k];
            tmax = max(tmax, w[k] & ~kRem1);
            tsum += w[k] & ~kRem1;
        }
    }
    tmax = wave_max_u32(tmax);
    tsum = wave_sum_u64(tsum);
    if (ballot(bad) && lane == 0) ws.bad = 1;
    if (lane == 0) {
        ws.wmax[wv] = tmax;
        ws.wsum[wv] = tsum;
    }
    __syncthreads();
    uint32_t m = 0;
    for (int w = 0; w < kDagWaves; w++) m = max(m, ws.wmax[w]);
    if (m <= kTau16) {
        dag_passes<SIM, TPB>(a, o, d, [&](int32_t s) { return word32(pks16[s]); }, dl, ws, hist);
    } else {
        dag_passes<SIM, TPB>(a, o, d,
                        [&](int32_t s) {
                            bool b;
                            return task_word<HAS_REM>(a, d, s, b);
                        },
                        dl, ws, hist);
    }
}

// ---- grid pass over one large DAG -------------------------------------

constexpr int kBigThreads = 256;
constexpr int kBigWaves = kBigThreads / kWave;

// Task words of the DAG into pkg, and each block's max and sum of tau and
// estimate check into its partial slot.
template <bool HAS_REM>
__global__ __launch_bounds__(kBigThreads) void k_attr_pack(AttrArgs a, int32_t di) {
    __shared__ WaveSlots ws;
    const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
    const DagDesc d = a.desc[di];
    if (tid == 0) ws.bad = 0;
    __syncthreads();
    // partial slots past the grid read as zero in the select kernel
    for (int32_t i = gridDim.x + blockIdx.x; i < kBigGrid; i += gridDim.x)
        if (tid < 32) a.part[32 * (int64_t)i + tid] = 0;
    uint32_t tmax = 0;
    unsigned long long tsum = 0;
    bool bad = false;
    for (int32_t v = blockIdx.x * kBigThreads + tid; v < d.n; v += gridDim.x * kBigThreads) {
        bool b;
        const uint32_t w = task_word<HAS_REM>(a, d, v, b);
        a.pkg[v] = w;
        pk16_of(a, d)[v] = word16(w);
        pk8_of(a, d)[v] = word8(w);
        bad |= b;
        tmax = max(tmax, w & ~kRem1);
        tsum += w & ~kRem1;
    }
    tmax = wave_max_u32(tmax);
    tsum = wave_sum_u64(tsum);
    if (ballot(bad) && lane == 0) ws.bad = 1;
    if (lane == 0) {
        ws.wmax[wv] = tmax;
        ws.wsum[wv] = tsum;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t m = 0;
        unsigned long long sm = 0;
        for (int w = 0; w < kBigWaves; w++) {
            m = max(m, ws.wmax[w]);
            sm += ws.wsum[w];
        }
        if (m > kTau8 && dev_load(&a.maxtau[d.id]) < (int32_t)m) atomicMax(&a.maxtau[d.id], (int32_t)m);
        int32_t *slot = a.part + 32 * blockIdx.x;
        slot[24] = (int32_t)m;
        slot[25] = (int32_t)(uint32_t)sm;
        slot[26] = (int32_t)(uint32_t)(sm >> 32);
        slot[27] = ws.bad;
    }
}

// A hub row (more than kHubDeg successors), one wave: the row's successors
// kWin * 64 at a time.  Pass A: count of rem == 1 successors and the
// extremes of tau(v) + tau(s); pass B: the count within U.
template <bool PASS_B, typename PK>
__device__ void scan_hub(const AttrArgs &a, const DagDesc &d, PK pk, int32_t e0, int32_t e1, int32_t tv, int64_t U,
                         int32_t *cnt, int32_t *lo, int32_t *hi) {
    const int lane = lane_id();
    const int32_t *c = a.col + d.eoff;
    int32_t n1 = 0;
    uint32_t mn = INT_MAX, mx = 0;
    for (int32_t b = e0; b < e1; b += kWave * kWin) {
        int32_t sv[kWin];
        uint32_t pv[kWin];
#pragma unroll
        for (int u = 0; u < kWin; u++) sv[u] = c[min(b + u * kWave + lane, e1 - 1)];
#pragma unroll
        for (int u = 0; u < kWin; u++) pv[u] = pk(sv[u]);
#pragma unroll
        for (int u = 0; u < kWin; u++) {
            const int32_t x = tv + (int32_t)(pv[u] & ~kRem1);
            const bool take = b + u * kWave + lane < e1 && (pv[u] & kRem1);
            if (PASS_B) {
                n1 += take && (int64_t)x <= U;
            } else {
                n1 += take;
                mn = take ? min(mn, (uint32_t)x) : mn;
                mx = take ? max(mx, (uint32_t)x) : mx;
            }
        }
    }
    *cnt = wave_sum_i32(n1);
    if (!PASS_B) {
        *lo = (int32_t)wave_min_u32f(mn);
        *hi = (int32_t)wave_max_u32f(mx);
    }
}

// Pass A: each wave takes 64-row chunks (hub rows left out), then hub rows
// (largest first), in grid stride, and leaves each row's summary in `summ`;
// the block's score histogram goes to `hist`.  Task words through pk.
template <typename PK>
__device__ __forceinline__ void big_pass_a(const AttrArgs &a, const DagDesc &d, PK pk, ChunkLds *cl, int32_t *hist) {
    const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
    const int32_t nw = gridDim.x * kBigWaves, w0 = blockIdx.x * kBigWaves + wv;
    const int32_t skip = d.nhub > 0 ? kHubDeg : INT_MAX;
    const int32_t *r = a.rp + d.toff + d.id;
    const int32_t *c = a.col + d.eoff;
    const uint32_t *pkg = a.pkg;
    for (int32_t p = w0; p < d.nhub; p += nw) {
        const int4 h = a.hub[d.hub0 + p];  // row, piece, pieces, first piece slot
        const int32_t v = h.x, e0 = r[v], e1 = r[v + 1];
        const int32_t pe0 = e0 + h.y * kPiece, pe1 = h.z > 1 ? min(e1, pe0 + kPiece) : e1;
        int32_t cnt, lo, hi;
        scan_hub<false>(a, d, pk, pe0, pe1, (int32_t)(pkg[v] & ~kRem1), 0, &cnt, &lo, &hi);
        if (lane == 0) {
            if (h.z > 1) {
                // one piece of a long row: combined by the select kernel
                int32_t *ps = a.pslot + 4 * (int64_t)(h.w + h.y);
                ps[0] = cnt;
                ps[1] = lo;
                ps[2] = hi;
            } else {
                a.summ[v] = pack_summary(cnt, lo, hi);
                if (a.unit_time == 0) add_rungs(hist, cnt, lo, hi, e1 - e0);
            }
        }
    }
    RowPrefetch rf(r, d.n, w0 * kWave, nw * kWave);
    for (int32_t c0 = w0 * kWave; c0 < d.n; c0 += nw * kWave) {
        const int32_t v = c0 + lane, vv = min(v, d.n - 1);
        int32_t e0, deg;
        rf.next(e0, deg);
        const int32_t tau = (int32_t)(pkg[vv] & ~kRem1);
        const bool scanned = deg <= skip;
        int32_t cnt, lo, hi;
        chunk_scan<false>(c, e0, scanned ? deg : 0, tau, 0, pk, cl[wv], cnt, lo, hi);
        if (v < d.n && scanned) {
            a.summ[v] = pack_summary(cnt, lo, hi);
            if (a.unit_time == 0) add_rungs(hist, cnt, lo, hi, deg);
        }
    }
}

// Pass A over the grid; each block leaves its score histogram in its
// partial slot.
__global__ __launch_bounds__(kBigThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_attr_big_a(AttrArgs a,
                                                                                                  int32_t di) {
    __shared__ ChunkLds cl[kBigWaves];
    __shared__ int32_t hist[kRungs];
    const int tid = threadIdx.x;
    const DagDesc d = a.desc[di];
    if (tid < kRungs) hist[tid] = 0;
    __syncthreads();
    if (dev_load(&a.maxtau[d.id]) == 0) big_pass_a(a, d, GridBytes{pk8_of(a, d)}, cl, hist);
    else big_pass_a(a, d, GridWords{a.pkg, pk16_of(a, d)}, cl, hist);
    __syncthreads();
    if (tid < kRungs) a.part[32 * blockIdx.x + tid] = hist[tid];
}

constexpr int kSelThreads = 1024;

// The large DAG's U (one work-group): the rows cut into pieces combined into
// their summaries and score contributions, then every block's partial slot.
__global__ __launch_bounds__(kSelThreads) void k_attr_big_sel(AttrArgs a, int32_t di) {
    __shared__ WaveSlots ws;
    __shared__ int32_t hist[kRungs];
    const int tid = threadIdx.x;
    const DagDesc d = a.desc[di];
    if (tid < kRungs) hist[tid] = 0;
    if (tid == 0) ws.bad = 0;
    __syncthreads();
    // every block's partial slot (rungs 0..23, then max tau, the tau sum's
    // low and high words, the estimate flag), read along the slots: thread
    // (g, j) combines word j of slots 64g .. 64g + 63 (all kBigGrid rows;
    // the pack kernel zeroes those past the grid).  The first long row's
    // descriptor is loaded with them, so that both wait for one round trip.
    constexpr int kGroups = kSelThreads / 32, kU = kBigGrid / kGroups;
    __shared__ long long colsum[kGroups][32];
    int4 h0 = make_int4(0, 0, 0, 0);
    if (tid < d.nlong) h0 = a.lrow[d.long0 + tid];  // row, 0, pieces, first slot
    {
        const int j = tid & 31, g = tid >> 5;
        const uint32_t o = (uint32_t)(32 * g * kU + j);  // 32-bit offsets from the uniform base
        int32_t x[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) x[u] = a.part[o + 32u * u];
        // 32-bit arithmetic (a sum of 32-bit words as the sums of their halves)
        long long acc = 0;
        if (j == 25 || j == 26) {
            uint32_t lo16 = 0, hi16 = 0;
#pragma unroll
            for (int u = 0; u < kU; u++) {
                lo16 += (uint32_t)x[u] & 0xFFFFu;
                hi16 += (uint32_t)x[u] >> 16;
            }
            acc = (long long)lo16 + ((long long)hi16 << 16);
        } else if (j == 24) {
            uint32_t mx = 0;
#pragma unroll
            for (int u = 0; u < kU; u++) mx = max(mx, (uint32_t)x[u]);
            acc = mx;
        } else if (j == 27) {
            int32_t any = 0;
#pragma unroll
            for (int u = 0; u < kU; u++) any |= x[u];
            acc = any != 0;
        } else {
            int32_t t = 0;
#pragma unroll
            for (int u = 0; u < kU; u++) t += x[u];
            acc = t;
        }
        colsum[g][j] = acc;
    }
    const int32_t *r = a.rp + d.toff + d.id;
    for (int32_t p = tid; p < d.nlong; p += kSelThreads) {
        const int4 h = p == tid ? h0 : a.lrow[d.long0 + p];
        const int32_t deg = r[h.x + 1] - r[h.x];
        int32_t c1 = 0, lo = INT_MAX, hi = 0;
        // the pieces' partials kPL at a time (every row of up to 8,192
        // successors in one round), their loads issued together
        constexpr int kPL = 16;
        for (int32_t k0 = 0; k0 < h.z; k0 += kPL) {
            int4 y[kPL];
#pragma unroll
            for (int k = 0; k < kPL; k++) y[k] = reinterpret_cast<const int4 *>(a.pslot)[h.w + min(k0 + k, h.z - 1)];
#pragma unroll
            for (int k = 0; k < kPL; k++) {
                if (k0 + k < h.z && y[k].x > 0) {
                    c1 += y[k].x;
                    lo = min(lo, y[k].y);
                    hi = max(hi, y[k].z);
                }
            }
        }
        a.summ[h.x] = pack_summary(c1, lo, hi);
        if (a.unit_time == 0) add_rungs(hist, c1, lo, hi, deg);
    }
    __syncthreads();
    if (tid < 28) {
        long long t = 0;
        for (int g = 0; g < kGroups; g++) t = tid == 24 ? max(t, colsum[g][tid]) : t + colsum[g][tid];
        if (tid < kRungs) atomicAdd(&hist[tid], (int32_t)t);
        else if (tid == 24) ws.wmax[0] = (uint32_t)t;
        else if (tid == 25) ws.wsum[0] = (unsigned long long)t;
        else if (tid == 26) ws.wsum[1] = (unsigned long long)t;
        else if (t) ws.bad = 1;
    }
    __syncthreads();
    if (tid == 0) {
        const uint32_t mm = ws.wmax[0];
        const unsigned long long ss = ws.wsum[0] + (ws.wsum[1] << 32);
        select_unit(a, d.id, d.n, (int32_t)mm, ss, hist);
        if (ws.bad) {
            atomicOr(&a.stat[2 * d.id], ST_EST);
            *a.anybad = 1;
        }
    }
}

// Pass B: IE at the chosen U from each row's summary -- 0 below the least
// sum, every rem == 1 successor at or above the largest -- rescanning only
// the rows in between (a chunk scan limited to them; a hub row by its wave).
__global__ __launch_bounds__(kBigThreads) void k_attr_big_b(AttrArgs a, AttrOut o, int32_t di) {
    __shared__ ChunkLds cl[kBigWaves];
    const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
    const DagDesc d = a.desc[di];
    const int32_t nw = gridDim.x * kBigWaves, w0 = blockIdx.x * kBigWaves + wv;
    const bool failed = dag_failed(a, o, d);
    const int64_t U = a.u[d.id];
    const int32_t skip = d.nhub > 0 ? kHubDeg : INT_MAX;
    const int32_t *r = a.rp + d.toff + d.id;
    const int32_t *c = a.col + d.eoff;
    const uint32_t *pkg = a.pkg;
    const GridWords pk{pkg, pk16_of(a, d)};
    for (int32_t p = w0; p < d.nhub; p += nw) {
        const int4 h = a.hub[d.hub0 + p];
        if (h.y != 0) continue;  // a row's first piece writes it
        const int32_t v = h.x, e0 = r[v], e1 = r[v + 1];
        const int32_t tau = (int32_t)(pkg[v] & ~kRem1);
        int32_t c1, lo, hi;
        unpack_summary(a.summ[v], c1, lo, hi);
        int32_t ie = c1 == 0 || U < lo ? 0 : c1;
        if (!failed && c1 > 0 && lo <= U && U < hi) {
            int32_t l2, h2;
            scan_hub<true>(a, d, pk, e0, e1, tau, U, &ie, &l2, &h2);
        }
        if (lane == 0) write_row(a, o, d, v, e0, e1 - e0, tau, ie, failed);
    }
    for (int32_t c0 = w0 * kWave; c0 < d.n; c0 += nw * kWave) {
        const int32_t v = c0 + lane, vv = min(v, d.n - 1);
        if (failed) {
            if (v < d.n) write_row(a, o, d, v, 0, 0, 0, 0, true);
            continue;
        }
        const int32_t e0 = r[vv], deg = v < d.n ? r[vv + 1] - e0 : 0;
        const int32_t tau = (int32_t)(pkg[vv] & ~kRem1);
        int32_t c1, lo, hi;
        unpack_summary(a.summ[vv], c1, lo, hi);
        const bool between = v < d.n && c1 > 0 && lo <= U && U < hi;
        const bool hub = deg > skip;
        int32_t ie = c1 == 0 || U < lo ? 0 : c1;
        if (ballot(between && !hub)) {
            int32_t cnt, l2, h2;
            chunk_scan<true>(c, e0, between && !hub ? deg : 0, tau, U, pk, cl[wv], cnt, l2, h2);
            if (between) ie = cnt;
        }
        if (v < d.n && !hub) write_row(a, o, d, v, e0, deg, tau, ie, false);
    }
}

static AttrArgs make_args(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, const int32_t *rem) {
    AttrArgs a;
    a.desc = ws->desc.as<DagDesc>();
    a.sorder = ws->sorder.as<int32_t>();
    a.hub = dag->hub.as<int4>();
    a.pslot = dag->pslot.as<int32_t>();
    a.lrow = dag->lrow.as<int4>();
    a.part = ws->apart;
    a.pkg = ws->apkg;
    a.summ = ws->asumm;
    a.srow = reinterpret_cast<uint32_t *>(ws->fbuf);
    a.first = ws->first;
    a.rp = dag->rp.as<int32_t>();
    a.col = dag->col.as<int32_t>();
    a.word0 = dag->word0.as<unsigned long long>();
    a.est = est;
    a.rem = rem;
    a.base = ws->base;
    a.tasks = ws->tasks;
    a.count = ws->count;
    a.unit_time = unit_time;
    a.maxtau = ws->dag_maxtau;
    a.score = ws->dag_score;
    a.u = ws->dag_u;
    a.taubar = ws->dag_taubar;
    a.done = ws->dag_done;
    a.stat = dag->dag_stat.as<int32_t>();
    a.sticky = dag->dag_sticky.as<int32_t>();
    a.anybad = ws->counter.as<int32_t>() + 3;
    a.tausum = ws->dag_tausum;
    return a;
}

static int big_grid(int32_t n, int32_t nhub) {
    const int64_t waves = (n + kWave - 1) / kWave + nhub;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kBigGrid, (waves + kBigWaves - 1) / kBigWaves));
}

// The per-DAG kernel for a call's mode: DAGs above kMidTasks (first in
// sorder) with 1024 threads, the others with 256.
template <bool HAS_REM, bool SIM>
static int launch_attr_dag(const AttrArgs &a, const AttrOut &o, int32_t n_big, int32_t n_mid, size_t lds_big,
                           size_t lds_mid, hipStream_t st) {
    if (n_big > 0) {
        if (int rc = set_lds_limit((const void *)&k_attr_dag<HAS_REM, SIM, kDagThreads>, lds_big)) return rc;
        hipLaunchKernelGGL((k_attr_dag<HAS_REM, SIM, kDagThreads>), dim3(n_big), dim3(kDagThreads), lds_big, st, a, o,
                           0);
    }
    if (n_mid > 0)
        hipLaunchKernelGGL((k_attr_dag<HAS_REM, SIM, kMidThreads>), dim3(n_mid), dim3(kMidThreads), lds_mid, st, a, o,
                           n_big);
    return INSP_OK;
}

int run_attributes(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, const int32_t *rem,
                   int32_t *ia_out, int32_t *ie_out, bool sim_init, hipStream_t st) {
    if (rem && sim_init) return set_error(INSP_E_INVAL, "a schedule starts from the initial in-degrees");
    AttrArgs a = make_args(dag, ws, est, unit_time, rem);
    if (!sim_init) {
        // an attribute-only call has status words of its own: it neither
        // clears nor reports a schedule's pending failures
        a.stat = dag->dag_astat.as<int32_t>();
        a.sticky = nullptr;
    }
    AttrOut o;
    o.ia_out = ia_out;
    o.ie_out = ie_out;
    o.sim_init = sim_init ? 1 : 0;
    o.tr = ws->tr;
    o.dep = ws->dep;
    ProfScope whole(st, "pass_attr");
    {
        ProfScope ps(st, "attr_clear");
        hipLaunchKernelGGL(k_attr_clear, dim3((ws->count + 255) / 256), dim3(256), 0, st, a);
    }
    if (!sim_init && ws->n_small > 0) {
        // the per-DAG kernel writes as it goes: estimates are checked first
        ProfScope ps(st, "attr_check");
        const int64_t blocks = std::min<int64_t>((ws->tasks + 255) / 256, 4096);
        hipLaunchKernelGGL(k_est_check, dim3((unsigned)blocks), dim3(256), 0, st, a);
    }
    if (ws->n_small > 0) {
        ProfScope ps(st, "attr_dag");
        // the DAGs above kMidTasks (first in sorder) get 1024 threads each,
        // the others 256, so that several of them share a CU
        int32_t n_big = 0;
        while (n_big < ws->n_small && ws->h_desc[ws->h_sorder[n_big]].n > kMidTasks) n_big++;
        const int32_t n_mid = ws->n_small - n_big;
        const size_t lds_big = 4 * (((size_t)std::max(ws->max_small, 1) + 1) / 2);
        const size_t lds_mid = 4 * (((size_t)std::max(n_mid > 0 ? ws->h_desc[ws->h_sorder[n_big]].n : 1, 1) + 1) / 2);
        int rc = rem        ? launch_attr_dag<true, false>(a, o, n_big, n_mid, lds_big, lds_mid, st)
                 : sim_init ? launch_attr_dag<false, true>(a, o, n_big, n_mid, lds_big, lds_mid, st)
                            : launch_attr_dag<false, false>(a, o, n_big, n_mid, lds_big, lds_mid, st);
        if (rc) return rc;
    }
    for (int32_t di : ws->h_large) {
        const DagDesc &d = ws->h_desc[di];
        const int gb = big_grid(d.n, d.nhub);
        {
            ProfScope ps(st, "attr_pack");
            if (rem) hipLaunchKernelGGL(k_attr_pack<true>, dim3(gb), dim3(kBigThreads), 0, st, a, di);
            else hipLaunchKernelGGL(k_attr_pack<false>, dim3(gb), dim3(kBigThreads), 0, st, a, di);
        }
        {
            ProfScope ps(st, "attr_a");
            hipLaunchKernelGGL(k_attr_big_a, dim3(gb), dim3(kBigThreads), 0, st, a, di);
        }
        {
            ProfScope ps(st, "attr_sel");
            hipLaunchKernelGGL(k_attr_big_sel, dim3(1), dim3(kSelThreads), 0, st, a, di);
        }
        {
            ProfScope ps(st, "attr_b");
            hipLaunchKernelGGL(k_attr_big_b, dim3(gb), dim3(kBigThreads), 0, st, a, o, di);
        }
    }
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

int alloc_status(insp_dag *dag) {
    int rc;
    if ((rc = dag->dag_stat.alloc(8 * dag->B)) || (rc = dag->dag_astat.alloc(8 * dag->B)) ||
        (rc = dag->dag_sticky.alloc(4 * dag->B)))
        return rc;
    INSP_HIP(hipMemset(dag->dag_stat.p, 0, 8 * dag->B));
    INSP_HIP(hipMemset(dag->dag_astat.p, 0, 8 * dag->B));
    INSP_HIP(hipMemset(dag->dag_sticky.p, 0, 4 * dag->B));
    return INSP_OK;
}

int32_t large_rows(const insp_dag *dag) {
    int32_t m = 0;
    for (int32_t b = 0; b < dag->B; b++) {
        const int64_t n = dag->toff[b + 1] - dag->toff[b];
        if (n >= kGridMin) m = std::max<int32_t>(m, (int32_t)n);
    }
    return m;
}

int ensure_state(insp_dag *dag, hipStream_t st) {
    (void)st;
    if (dag->tr.p) return INSP_OK;
    const int64_t N = std::max<int64_t>(dag->N, 1);
    int rc;
    if ((rc = dag->tr.alloc(sizeof(TaskRec) * N)) || (rc = dag->dep.alloc(8 * N)) || (rc = dag->fbuf.alloc(12 * N)) ||
        (rc = dag->dag_u.alloc(4 * dag->B)) ||
        (rc = dag->dag_taubar.alloc(4 * dag->B)) || (rc = dag->dag_maxtau.alloc(4 * dag->B)) ||
        (rc = dag->dag_tausum.alloc(8 * dag->B)) || (rc = dag->dag_score.alloc(4 * kRungs * dag->B)) ||
        (rc = dag->dag_done.alloc(4 * dag->B)) || (rc = dag->apart.alloc(4 * 32 * kBigGrid)) ||
        (rc = dag->apkg.alloc(4 * (size_t)large_rows(dag))) || (rc = dag->asumm.alloc(8 * (size_t)large_rows(dag)))) {
        dag->tr.release();
        return rc;
    }
    return INSP_OK;
}

// Queue pool of one DAG: every worker's queue is a list of 64-slot blocks;
// at any time sum over workers of ceil(len/64) <= n/64 + W blocks are in use.
static void pool_shape(int32_t n, int32_t W, int32_t *nblk, int32_t *maxb) {
    *nblk = (n + 63) / 64 + W;
    *maxb = (n + 63) / 64 + 1;
}

int64_t workspace_shape(const insp_dag *dag, int32_t first, int32_t count, const insp_workers *workers,
                        bool per_dag, Workspace *w, std::vector<DagDesc> *desc) {
    w->count = count;
    w->first = first;
    w->base = dag->toff[first];
    w->tasks = dag->toff[first + count] - dag->toff[first];
    desc->assign(count, DagDesc());
    w->h_order.clear();
    w->h_sorder.clear();
    w->h_large.clear();
    w->max_small = 0;
    int64_t boff = 0, wloff = 0;
    for (int32_t i = 0; i < count; i++) {
        const insp_workers &wk = workers[per_dag ? i : 0];
        int32_t b = first + i;
        DagDesc &d = (*desc)[i];
        memset(&d, 0, sizeof d);
        d.id = b;
        d.toff = dag->toff[b];
        d.eoff = dag->eoff[b];
        d.n = (int32_t)(dag->toff[b + 1] - dag->toff[b]);
        d.m = (int32_t)(dag->eoff[b + 1] - dag->eoff[b]);
        d.n_cpu = wk.n_cpu;
        d.n_gpu = wk.n_gpu;
        pool_shape(d.n, wk.n_cpu + wk.n_gpu, &d.nblk, &d.maxb);
        d.blk_off = boff;
        d.wl_off = wloff;
        d.path = d.n >= kGridMin ? 1 : 0;
        d.hub0 = dag->hub0.empty() ? 0 : dag->hub0[b];
        d.nhub = dag->nhub.empty() ? 0 : dag->nhub[b];
        d.long0 = dag->long0.empty() ? 0 : dag->long0[b];
        d.nlong = dag->nlong.empty() ? 0 : dag->nlong[b];
        boff += d.nblk;
        wloff += (int64_t)(wk.n_cpu + wk.n_gpu) * d.maxb;
        w->max_w = std::max(w->max_w, wk.n_cpu + wk.n_gpu);
        w->max_nblk = std::max<int64_t>(w->max_nblk, d.nblk);
        if (d.path) w->h_large.push_back(i);
        else w->max_small = std::max(w->max_small, d.n);
    }
    w->h_desc = *desc;
    // simulation and per-DAG attribute order: largest DAGs first
    for (int32_t b : dag->order)
        if (b >= first && b < first + count) {
            w->h_order.push_back(b - first);
            if (dag->toff[b + 1] - dag->toff[b] > 0 && !(*desc)[b - first].path) w->h_sorder.push_back(b - first);
        }
    w->n_small = (int32_t)w->h_sorder.size();
    w->total_wl = wloff;
    return boff;
}

int get_workspace(insp_dag *dag, int32_t first, int32_t count, const insp_workers *workers, bool per_dag,
                  Workspace **out) {
    std::string key = std::to_string(first) + ":" + std::to_string(count);
    for (int32_t i = 0; i < (per_dag ? count : 1); i++)
        key += ":" + std::to_string(workers[i].n_cpu) + "," + std::to_string(workers[i].n_gpu);
    auto it = dag->ws.find(key);
    Workspace *w = nullptr;
    if (it != dag->ws.end()) {
        w = it->second.get();
    } else {
        std::unique_ptr<Workspace> nw(new Workspace());
        std::vector<DagDesc> desc;
        const int64_t boff = workspace_shape(dag, first, count, workers, per_dag, nw.get(), &desc);
        int rc;
        if ((rc = nw->desc.alloc(sizeof(DagDesc) * count)) ||
            (rc = nw->order.alloc(sizeof(int32_t) * count)) || (rc = nw->sorder.alloc(sizeof(int32_t) * count)) ||
            (rc = nw->slots.alloc(sizeof(Slot) * 64 * (size_t)boff)) ||
            (rc = nw->sums.alloc(16 * (size_t)boff)) || (rc = nw->paux.alloc(4 * (size_t)(nw->total_wl + boff))) ||
            (rc = nw->barr.alloc(8 * (size_t)boff)) ||
            (rc = nw->counter.alloc(16)))
            return rc;
        INSP_HIP(hipMemcpy(nw->desc.p, desc.data(), sizeof(DagDesc) * count, hipMemcpyHostToDevice));
        INSP_HIP(hipMemcpy(nw->order.p, nw->h_order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice));
        if (nw->n_small > 0)
            INSP_HIP(hipMemcpy(nw->sorder.p, nw->h_sorder.data(), sizeof(int32_t) * nw->n_small,
                               hipMemcpyHostToDevice));
        w = nw.get();
        dag->ws[key] = std::move(nw);
    }
    // the handle's per-call state (ensure_state has run)
    w->tr = dag->tr.as<TaskRec>();
    w->dep = dag->dep.as<unsigned long long>();
    w->fbuf = dag->fbuf.as<int32_t>();
    w->dag_u = dag->dag_u.as<int32_t>();
    w->dag_taubar = dag->dag_taubar.as<int32_t>();
    w->dag_maxtau = dag->dag_maxtau.as<int32_t>();
    w->dag_score = dag->dag_score.as<int32_t>();
    w->dag_tausum = dag->dag_tausum.as<unsigned long long>();
    w->dag_done = dag->dag_done.as<int32_t>();
    w->apart = dag->apart.as<int32_t>();
    w->apkg = dag->apkg.as<uint32_t>();
    w->asumm = dag->asumm.as<unsigned long long>();
    *out = w;
    return INSP_OK;
}

}  // namespace insp

using namespace insp;

static int check_workers(const insp_workers *w, int32_t count) {
    for (int32_t i = 0; i < count; i++) {
        if (w[i].n_cpu < 0 || w[i].n_gpu < 0) return set_error(INSP_E_INVAL, "negative worker count");
        int32_t W = w[i].n_cpu + w[i].n_gpu;
        if (W < 1 || W > INSP_MAX_WORKERS) return set_error(INSP_E_RANGE, "worker count %d outside [1, 1024]", W);
    }
    return INSP_OK;
}

extern "C" int insp_attributes(const insp_dag *cdag, int32_t index, const int32_t *est, const insp_workers *workers,
                               int32_t unit_time, const int32_t *rem, int32_t *ia, int32_t *ie,
                               int32_t *unit_time_used, void *stream) {
    insp_dag *dag = const_cast<insp_dag *>(cdag);
    if (!dag || !workers || !unit_time_used) return set_error(INSP_E_INVAL, "null argument");
    if (index != INSP_ALL_DAGS && (index < 0 || index >= dag->B))
        return set_error(INSP_E_INVAL, "dag index %d out of range", index);
    if (unit_time < 0) return set_error(INSP_E_INVAL, "negative unit_time");
    const int32_t first = index == INSP_ALL_DAGS ? 0 : index;
    const int32_t count = index == INSP_ALL_DAGS ? dag->B : 1;
    int rc = check_workers(workers, count);
    if (rc) return rc;
    const int64_t n = dag->toff[first + count] - dag->toff[first];
    if (n > 0 && (!est || !ia || !ie)) return set_error(INSP_E_INVAL, "null est/ia/ie");
    if (((uintptr_t)est & 7) != 0) return set_error(INSP_E_INVAL, "est rows must be 8-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    INSP_HIP(hipSetDevice(dag->device));
    if ((rc = ensure_state(dag, st))) return rc;
    Workspace *ws;
    if ((rc = get_workspace(dag, first, count, workers, true, &ws))) return rc;
    if ((rc = run_attributes(dag, ws, est, unit_time, rem, ia, ie, false, st))) return rc;
    std::vector<int32_t> stat(2 * dag->B), uu(count);
    INSP_HIP(hipMemcpyAsync(uu.data(), ws->dag_u + first, sizeof(int32_t) * count,
                            hipMemcpyDeviceToHost, st));
    INSP_HIP(hipMemcpyAsync(stat.data(), dag->dag_astat.p, sizeof(int32_t) * 2 * dag->B, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    for (int32_t i = first; i < first + count; i++)
        if (stat[2 * i] & ST_EST) return set_error(INSP_E_RANGE, "estimate outside [1, 2^20] in DAG %d", i);
    for (int32_t i = 0; i < count; i++) unit_time_used[i] = uu[i];
    return INSP_OK;
}
