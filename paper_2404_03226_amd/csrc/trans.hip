// Transitive reading of the inspiring attributes (Section 4.3: the source of
// a fully connected DAG scores the number of its tasks; Section 4.2: with a
// large unit time IE converges to IA; Section 7: IE looks at a time window
// after the task), computed on the whole graph:
//   D(v)       = v and every task reachable from v,
//   IA_T(v)    = |D(v)|,
//   EF_v(d)    = the longest tau-weighted path from v to d, both ends
//                included (d's earliest finish with v starting at 0 and
//                unlimited workers),
//   IE_T(v; U) = #{d in D(v) : EF_v(d) <= U}.
//
// One work-group per source v runs the forward pass over D(v): EF lives in
// LDS indexed by the task's position in the DAG's Kahn-level order, so the
// descendants of a level sit at later positions and one barrier per level
// orders the pass.  A member pushes EF + tau(s) into each successor with an
// LDS atomicMax and clears its own slot, so the array is zero again for the
// next source.  The pass stops at the first level beyond the last position
// reached.  Each source leaves IA_T, and either its count within an explicit
// U or its cumulative counts per ladder rung 2^j; a per-DAG pass then scores
// the rungs and picks U.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

constexpr int kTT = 512;                 // threads per work-group
constexpr int kTW = kTT / kWave;
constexpr uint32_t kPathCap = 1u << 30;  // paths saturate here (out of range)
constexpr int kChunk = 4;                // sources taken per counter fetch

struct TransArgs {
    const DagDesc *desc;
    int32_t count;
    int64_t base, items;
    const int32_t *topo, *lvl, *nlev, *plev, *pcol;
    int32_t *ptau;
    int2 *pedge;              // per edge: target position and its tau (this call's estimates)
    const int2 *prow;
    int32_t maxn;             // largest DAG of the launch (LDS entries)
    int32_t clear_status;
    const int32_t *est;
    int32_t unit_time;
    int32_t *ia, *ie;         // outputs by task, relative to base
    int32_t *cum;             // [items][kTRungs]: members with EF <= 2^j (automatic U)
    unsigned int *longest;    // [count]: longest path of each DAG
    int32_t *counter;
    int32_t *stat;
};

// Workspace DAG holding item `item` (its tasks are items toff - base ...).
__device__ __forceinline__ int32_t desc_of(const DagDesc *desc, int32_t count, int64_t base, int64_t item) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (desc[mid].toff - base <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int32_t dag_of_off(const int64_t *off, int32_t B, int64_t x) {
    int32_t lo = 0, hi = B - 1;  // last b with off[b] <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Per handle: positions in level order.

// Position of every task, its row, and its level.
__global__ __launch_bounds__(256) void k_positions(int32_t B, const int64_t *toff, const int32_t *rp,
                                                    const int32_t *topo, const int32_t *lvl, const int32_t *nlev,
                                                    int32_t *ppos, int2 *prow, int32_t *plev) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= toff[B]) return;
    const int32_t b = dag_of_off(toff, B, t);
    const int64_t t0 = toff[b];
    const int32_t i = (int32_t)(t - t0);
    const int32_t v = topo[t];
    const int32_t *r = rp + t0 + b;
    ppos[t0 + v] = i;
    prow[t] = make_int2(r[v], r[v + 1]);
    const int32_t *ls = lvl + t0 + b;
    int32_t lo = 0, hi = nlev[b] - 1;  // last level starting at or before i
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (ls[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    plev[t] = lo;
}

// Position of every edge's target.
__global__ __launch_bounds__(256) void k_edge_positions(int32_t B, const int64_t *toff, const int64_t *eoff,
                                                         const int32_t *col, const int32_t *ppos, int32_t *pcol) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= eoff[B]) return;
    const int32_t b = dag_of_off(eoff, B, e);
    pcol[e] = ppos[toff[b] + col[e]];
}

// ---------------------------------------------------------------------------
// Per call.

// tau by position (the GPU estimate when the machine has GPU workers, else
// the CPU one); estimates outside [1, 2^20] flag the DAG.
__global__ __launch_bounds__(256) void k_position_tau(TransArgs A) {
    const int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (item >= A.items) return;
    const int32_t d = desc_of(A.desc, A.count, A.base, item);
    const DagDesc D = A.desc[d];
    const int64_t u0 = D.toff - A.base;
    const int32_t i = (int32_t)(item - u0);
    const int32_t v = A.topo[D.toff + i];
    const int2 e = reinterpret_cast<const int2 *>(A.est)[u0 + v];
    if (e.x < 1 || e.x > INSP_MAX_TICK || e.y < 1 || e.y > INSP_MAX_TICK) atomicOr(&A.stat[2 * D.id], ST_EST);
    // clamped, so that paths stay in 32 bits even for a DAG already flagged
    A.ptau[D.toff + i] = min(max(D.n_gpu > 0 ? e.y : e.x, 1), INSP_MAX_TICK);
}

// Target position and tau of every edge of the launch's DAGs, packed so that
// the pass reads one 8-byte word per edge.
__global__ __launch_bounds__(256) void k_edge_tau(TransArgs A, int64_t e0, int64_t e1) {
    const int64_t e = e0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= e1) return;
    int32_t lo = 0, hi = A.count - 1;  // last DAG whose edges start at or before e
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (A.desc[mid].eoff <= e) lo = mid;
        else hi = mid - 1;
    }
    const int32_t s = A.pcol[e];
    A.pedge[e] = make_int2(s, A.ptau[A.desc[lo].toff + s]);
}

__global__ void k_trans_clear(TransArgs A) {
    const int32_t d = blockIdx.x * 256 + threadIdx.x;
    if (d < A.count) {
        A.longest[d] = 0;
        if (A.clear_status) A.stat[2 * A.desc[d].id] = 0;
    }
    if (d == 0) *A.counter = 0;
}

template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T x, T *part, Op op) {
    for (int o = 32; o > 0; o >>= 1) x = op(x, (T)__shfl_xor(x, o));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    T r = part[0];
#pragma unroll
    for (int w = 1; w < kTW; w++) r = op(r, part[w]);
    __syncthreads();
    return r;
}

// One source per work-group at a time; sources come from a counter, each
// DAG's in position order (the largest descendant sets first).
__global__ __launch_bounds__(kTT) void k_trans(TransArgs A) {
    extern __shared__ uint32_t EF[];
    __shared__ int64_t s_item;
    __shared__ int32_t s_hi;
    __shared__ int32_t s_hist[kTRungs];
    __shared__ uint32_t s_part[kTW];
    const int tid = threadIdx.x;
    const bool automatic = A.unit_time == 0;
    const uint32_t ut = (uint32_t)A.unit_time;
    for (int32_t p = tid; p < A.maxn; p += kTT) EF[p] = 0;
    // sources come kChunk at a time; the DAG of the previous source is kept
    // (consecutive sources mostly share it), so the descriptor search runs
    // once per DAG change
    int64_t item = 0, chunk_end = 0;
    int32_t d = -1;
    DagDesc D;
    D.toff = 0;
    D.n = 0;
    for (;;) {
        if (item >= chunk_end) {
            if (tid == 0) s_item = dev_fetch_add(A.counter, kChunk);
            __syncthreads();
            item = s_item;
            chunk_end = item + kChunk;
        }
        if (tid < kTRungs) s_hist[tid] = 0;
        __syncthreads();
        if (item >= A.items) break;
        if (d < 0 || item < D.toff - A.base || item >= D.toff - A.base + D.n) {
            d = desc_of(A.desc, A.count, A.base, item);
            D = A.desc[d];
        }
        const int64_t u0 = D.toff - A.base, t0 = D.toff;
        const int32_t i = (int32_t)(item - u0);
        const int32_t *ls = A.lvl + t0 + D.id;
        const int32_t nl = A.nlev[D.id];
        const int32_t L0 = A.plev[t0 + i];
        const int2 *pedge = A.pedge + D.eoff;
        const int32_t *ptau = A.ptau + t0;
        const int2 *prow = A.prow + t0;
        if (tid == 0) {
            EF[i] = (uint32_t)ptau[i];
            s_hi = i;
        }
        __syncthreads();
        uint32_t members = 0, within = 0, mx = 0;
        for (int32_t L = L0; L < nl; L++) {
            const int32_t a = L == L0 ? i : ls[L], z = L == L0 ? i + 1 : ls[L + 1];
            // every thread reads s_hi before any may raise it: a thread that
            // goes on has a <= s_hi, and raises only happen past that point
            if (a > s_hi) break;
            int32_t myhi = 0;
            for (int32_t p = a + tid; p < z; p += kTT) {
                const uint32_t ef = EF[p];
                if (ef == 0) continue;  // not reachable from the source
                const int2 row = prow[p];
                EF[p] = 0;
                members++;
                mx = max(mx, ef);
                if (automatic) {
                    const int b = ef <= 1 ? 0 : 32 - __clz(ef - 1);  // smallest j with ef <= 2^j
                    atomicAdd(&s_hist[b], 1);
                } else {
                    within += ef <= ut ? 1u : 0u;
                }
                for (int32_t e = row.x; e < row.y; e++) {
                    const int2 st = pedge[e];
                    const uint32_t f = min(ef + (uint32_t)st.y, kPathCap);
                    atomicMax(&EF[st.x], f);
                    myhi = max(myhi, st.x);
                }
            }
            for (int o = 32; o > 0; o >>= 1) myhi = max(myhi, __shfl_xor(myhi, o));
            if ((tid & 63) == 0) atomicMax(&s_hi, myhi);
            __syncthreads();
        }
        members = block_reduce(members, s_part, [](uint32_t x, uint32_t y) { return x + y; });
        mx = block_reduce(mx, s_part, [](uint32_t x, uint32_t y) { return max(x, y); });
        if (!automatic) within = block_reduce(within, s_part, [](uint32_t x, uint32_t y) { return x + y; });
        const int32_t v = A.topo[t0 + i];
        if (tid == 0) {
            A.ia[u0 + v] = (int32_t)members;
            if (!automatic) A.ie[u0 + v] = (int32_t)within;
            atomicMax(&A.longest[d], mx);
        }
        if (automatic && tid < kTRungs) {
            int32_t c = 0;
            for (int j = 0; j <= tid; j++) c += s_hist[j];
            A.cum[(u0 + v) * kTRungs + tid] = c;
        }
        __syncthreads();
        item++;
    }
}

// Per DAG: the range check on the longest path, and with an automatic U the
// ladder U = 2^j, j = 0..J (2^J the first power of two at least the longest
// path), scored by #{v : 0 < IE_T < IA_T}, the larger U on a tie.
__global__ __launch_bounds__(kTT) void k_trans_select(TransArgs A, int32_t *u_out) {
    __shared__ uint32_t s_part[kTW];
    __shared__ int32_t s_best;
    const int tid = threadIdx.x;
    const DagDesc D = A.desc[blockIdx.x];
    const int64_t u0 = D.toff - A.base;
    const uint32_t cp = A.longest[blockIdx.x];
    if (cp >= kPathCap) {
        if (tid == 0) {
            atomicOr(&A.stat[2 * D.id], ST_PATH);
            u_out[blockIdx.x] = 0;
        }
        return;
    }
    if (A.unit_time > 0 || D.n == 0) {
        if (tid == 0) u_out[blockIdx.x] = A.unit_time > 0 ? A.unit_time : 1;
        return;
    }
    int J = 0;
    while ((1u << J) < cp) J++;
    int32_t best = 0;
    uint32_t best_score = 0;
    for (int j = 0; j <= J; j++) {
        uint32_t sc = 0;
        for (int32_t v = tid; v < D.n; v += kTT) {
            const int32_t c = A.cum[(u0 + v) * kTRungs + j];
            sc += (c > 0 && c < A.ia[u0 + v]) ? 1u : 0u;
        }
        sc = block_reduce(sc, s_part, [](uint32_t x, uint32_t y) { return x + y; });
        if (j == 0 || sc >= best_score) {
            best_score = sc;
            best = j;
        }
    }
    if (tid == 0) {
        s_best = best;
        u_out[blockIdx.x] = 1 << best;
    }
    __syncthreads();
    for (int32_t v = tid; v < D.n; v += kTT) A.ie[u0 + v] = A.cum[(u0 + v) * kTRungs + s_best];
}

// Positions, level of each position and edge targets by position, built once.
static int ensure_positions(insp_dag *dag, hipStream_t st) {
    int rc;
    if ((rc = ensure_levels(dag, st))) return rc;
    if (dag->pcol.p) return INSP_OK;
    const int64_t N = std::max<int64_t>(dag->N, 1), M = std::max<int64_t>(dag->M, 1);
    DevBuf ppos, pcol;
    if ((rc = ppos.alloc(sizeof(int32_t) * N)) || (rc = dag->prow.alloc(sizeof(int2) * N)) ||
        (rc = dag->plev.alloc(sizeof(int32_t) * N)) || (rc = pcol.alloc(sizeof(int32_t) * M)))
        return rc;
    if (dag->N > 0)
        hipLaunchKernelGGL(k_positions, dim3((unsigned)((dag->N + 255) / 256)), dim3(256), 0, st, dag->B,
                           dag->d_toff.as<int64_t>(), dag->rp.as<int32_t>(), dag->topo.as<int32_t>(),
                           dag->lvl.as<int32_t>(), dag->nlev.as<int32_t>(), ppos.as<int32_t>(), dag->prow.as<int2>(),
                           dag->plev.as<int32_t>());
    if (dag->M > 0)
        hipLaunchKernelGGL(k_edge_positions, dim3((unsigned)((dag->M + 255) / 256)), dim3(256), 0, st, dag->B,
                           dag->d_toff.as<int64_t>(), dag->d_eoff.as<int64_t>(), dag->col.as<int32_t>(),
                           ppos.as<int32_t>(), pcol.as<int32_t>());
    INSP_HIP(hipGetLastError());
    INSP_HIP(hipStreamSynchronize(st));  // before ppos is freed
    std::swap(dag->pcol.p, pcol.p);
    std::swap(dag->pcol.bytes, pcol.bytes);
    return INSP_OK;
}

int run_transitive(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, int32_t *ia, int32_t *ie,
                   bool clear_status, hipStream_t st) {
    int rc;
    int32_t maxn = 0;
    for (int32_t i = 0; i < ws->count; i++) {
        const int32_t b = ws->first + i;
        maxn = std::max<int32_t>(maxn, (int32_t)(dag->toff[b + 1] - dag->toff[b]));
    }
    if (maxn > INSP_MAX_TRANSITIVE_TASKS)
        return set_error(INSP_E_RANGE, "transitive attributes need DAGs of at most %d tasks (got %d)",
                         INSP_MAX_TRANSITIVE_TASKS, maxn);
    if ((rc = ensure_positions(dag, st))) return rc;
    const int64_t N = std::max<int64_t>(dag->N, 1);
    if (!dag->ptau.p && (rc = dag->ptau.alloc(sizeof(int32_t) * N))) return rc;
    if (!dag->pedge.p && (rc = dag->pedge.alloc(sizeof(int2) * std::max<int64_t>(dag->M, 1)))) return rc;
    if (unit_time == 0 && dag->tcum.bytes < sizeof(int32_t) * kTRungs * (size_t)std::max<int64_t>(ws->tasks, 1) &&
        (rc = dag->tcum.alloc(sizeof(int32_t) * kTRungs * (size_t)std::max<int64_t>(ws->tasks, 1))))
        return rc;
    if (ws->tlong.bytes < sizeof(uint32_t) * (size_t)std::max(ws->count, 1) + 16 &&
        (rc = ws->tlong.alloc(sizeof(uint32_t) * (size_t)std::max(ws->count, 1) + 16)))
        return rc;
    if (ws->tu.bytes < sizeof(int32_t) * (size_t)std::max(ws->count, 1) &&
        (rc = ws->tu.alloc(sizeof(int32_t) * (size_t)std::max(ws->count, 1))))
        return rc;
    TransArgs A;
    A.desc = ws->desc.as<DagDesc>();
    A.count = ws->count;
    A.base = ws->base;
    A.items = ws->tasks;
    A.topo = dag->topo.as<int32_t>();
    A.lvl = dag->lvl.as<int32_t>();
    A.nlev = dag->nlev.as<int32_t>();
    A.plev = dag->plev.as<int32_t>();
    A.pcol = dag->pcol.as<int32_t>();
    A.ptau = dag->ptau.as<int32_t>();
    A.pedge = dag->pedge.as<int2>();
    A.prow = dag->prow.as<int2>();
    A.est = est;
    A.maxn = maxn;
    A.clear_status = clear_status ? 1 : 0;
    A.unit_time = unit_time;
    A.ia = ia;
    A.ie = ie;
    A.cum = unit_time == 0 ? dag->tcum.as<int32_t>() : nullptr;
    A.longest = ws->tlong.as<unsigned int>();
    A.counter = reinterpret_cast<int32_t *>(ws->tlong.as<unsigned int>() + ws->count);
    // a standalone call has status words of its own (it neither clears nor
    // reports a schedule's pending failures)
    A.stat = clear_status ? dag->dag_astat.as<int32_t>() : dag->dag_stat.as<int32_t>();
    hipLaunchKernelGGL(k_trans_clear, dim3((unsigned)((ws->count + 255) / 256)), dim3(256), 0, st, A);
    if (ws->tasks > 0) {
        hipLaunchKernelGGL(k_position_tau, dim3((unsigned)((ws->tasks + 255) / 256)), dim3(256), 0, st, A);
        const int64_t e0 = dag->eoff[ws->first], e1 = dag->eoff[ws->first + ws->count];
        if (e1 > e0)
            hipLaunchKernelGGL(k_edge_tau, dim3((unsigned)((e1 - e0 + 255) / 256)), dim3(256), 0, st, A, e0, e1);
        const size_t lds = sizeof(uint32_t) * (size_t)std::max(maxn, 1);
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        }
        const int per_cu = std::max<int>(1, std::min<int>(8, (int)((160 * 1024) / (lds + 1024))));
        const int grid = (int)std::min<int64_t>(ws->tasks, (int64_t)cus * per_cu);
        if ((rc = set_lds_limit((const void *)&k_trans, lds))) return rc;
        ProfScope ps(st, "trans");
        hipLaunchKernelGGL(k_trans, dim3(grid), dim3(kTT), lds, st, A);
    }
    hipLaunchKernelGGL(k_trans_select, dim3((unsigned)std::max(ws->count, 1)), dim3(kTT), 0, st, A,
                       ws->tu.as<int32_t>());
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

}  // namespace insp

using namespace insp;

extern "C" int insp_transitive_attributes(const insp_dag *cdag, int32_t dag_index, const int32_t *est,
                                          const insp_workers *workers, int32_t unit_time, int32_t *ia, int32_t *ie,
                                          int32_t *unit_time_used, int64_t *longest_path, void *stream) {
    insp_dag *dag = const_cast<insp_dag *>(cdag);
    if (!dag || !workers || !unit_time_used) return set_error(INSP_E_INVAL, "null argument");
    if (unit_time < 0) return set_error(INSP_E_INVAL, "negative unit_time");
    if (dag_index != INSP_ALL_DAGS && (dag_index < 0 || dag_index >= dag->B))
        return set_error(INSP_E_INVAL, "dag index %d out of range", dag_index);
    const int32_t first = dag_index == INSP_ALL_DAGS ? 0 : dag_index;
    const int32_t count = dag_index == INSP_ALL_DAGS ? dag->B : 1;
    const int64_t n = dag->toff[first + count] - dag->toff[first];
    if (n > 0 && (!est || !ia || !ie)) return set_error(INSP_E_INVAL, "null est/ia/ie");
    hipStream_t st = (hipStream_t)stream;
    INSP_HIP(hipSetDevice(dag->device));
    int rc;
    if ((rc = ensure_state(dag, st))) return rc;
    Workspace *ws;
    if ((rc = get_workspace(dag, first, count, workers, true, &ws))) return rc;
    // computed into the handle's arrays and copied out once the call is known
    // to succeed, so that a failing call leaves ia and ie untouched
    const int64_t NN = std::max<int64_t>(dag->N, 1);
    if ((!dag->tia.p && (rc = dag->tia.alloc(sizeof(int32_t) * NN))) ||
        (!dag->tie.p && (rc = dag->tie.alloc(sizeof(int32_t) * NN))))
        return rc;
    int32_t *tia = dag->tia.as<int32_t>() + ws->base, *tie = dag->tie.as<int32_t>() + ws->base;
    if ((rc = run_transitive(dag, ws, est, unit_time, tia, tie, true, st))) return rc;
    std::vector<int32_t> stat(2 * dag->B);
    std::vector<uint32_t> lp(count);
    std::vector<int32_t> uu(count);
    INSP_HIP(hipMemcpyAsync(uu.data(), ws->tu.p, sizeof(int32_t) * count, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipMemcpyAsync(lp.data(), ws->tlong.p, sizeof(uint32_t) * count, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipMemcpyAsync(stat.data(), dag->dag_astat.p, sizeof(int32_t) * 2 * dag->B, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    for (int32_t i = first; i < first + count; i++) {
        if (stat[2 * i] & ST_EST) return set_error(INSP_E_RANGE, "estimate outside [1, 2^20] in DAG %d", i);
        if (stat[2 * i] & ST_PATH) return set_error(INSP_E_RANGE, "longest path of DAG %d reaches 2^30 ticks", i);
    }
    if (n > 0) {
        INSP_HIP(hipMemcpyAsync(ia, tia, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
        INSP_HIP(hipMemcpyAsync(ie, tie, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
        INSP_HIP(hipStreamSynchronize(st));
    }
    for (int32_t i = 0; i < count; i++) unit_time_used[i] = uu[i];
    if (longest_path)
        for (int32_t i = 0; i < count; i++) longest_path[i] = lp[i];
    return INSP_OK;
}
