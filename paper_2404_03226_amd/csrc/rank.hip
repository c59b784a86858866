// HEFT upward rank (Topcuoglu, Hariri and Wu 2002), the priority of the HEFT
// list-scheduling baseline the paper compares against (Section 6).  With no
// communication costs (no data model):
//   rank(v) = mean estimate of v over the machine's workers
//             + the largest rank of v's successors,
// kept multiplied by the worker count W so that it stays an integer (the
// order is unchanged):
//   R(v) = n_cpu est_cpu(v) + n_gpu est_gpu(v) + max over successors R(s).
//
// R needs every successor first.  The Kahn levels of a DAG (level 0: no
// predecessors; a task sits one level above its last predecessor) put every
// edge from a lower level to a higher one, so one work-group per DAG walks
// the levels from the last to the first and computes a whole level in
// parallel.  The levels depend only on the graph: they are built once per
// handle; the ranks depend on the estimates and the machine and are
// recomputed by every HEFT call.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

constexpr int kRankThreads = 256;

// Kahn levels of one DAG per work-group.  topo receives the DAG's tasks level
// by level (any order inside a level); lvl[l] is the first position of level
// l in topo and lvl[nlev] = n.
__global__ __launch_bounds__(kRankThreads) void k_levels(const int64_t *toff, const int64_t *eoff, const int32_t *rp,
                                                          const int32_t *col, const unsigned long long *word0,
                                                          int32_t *indeg, int32_t *topo, int32_t *lvl,
                                                          int32_t *nlev) {
    const int32_t b = blockIdx.x;
    const int64_t t0 = toff[b];
    const int32_t n = (int32_t)(toff[b + 1] - t0);
    const int32_t *r = rp + t0 + b;
    const int32_t *c = col + eoff[b];
    int32_t *deg = indeg + t0;
    int32_t *q = topo + t0;
    int32_t *ls = lvl + t0 + b;
    __shared__ int32_t tail;
    if (threadIdx.x == 0) tail = 0;
    __syncthreads();
    for (int32_t v = threadIdx.x; v < n; v += kRankThreads) {
        deg[v] = (int32_t)(word0[t0 + v] >> 43);
        if (deg[v] == 0) q[atomicAdd(&tail, 1)] = v;
    }
    __syncthreads();
    int32_t head = 0, L = 0;
    for (;;) {
        const int32_t end = tail;
        __syncthreads();  // every thread has read tail before the level appends
        if (head == end) break;
        if (threadIdx.x == 0) ls[L] = head;
        L++;
        for (int32_t i = head + threadIdx.x; i < end; i += kRankThreads) {
            const int32_t v = q[i];
            for (int32_t e = r[v]; e < r[v + 1]; e++)
                if (atomicSub(&deg[c[e]], 1) == 1) q[atomicAdd(&tail, 1)] = c[e];
        }
        head = end;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ls[L] = head;
        nlev[b] = L;
    }
}

// Upward ranks of one DAG per work-group, last level first.  A rank at or
// above 2^42 does not fit the simulation's queue key: the DAG is flagged.
__global__ __launch_bounds__(kRankThreads) void k_rank(const DagDesc *desc, const int32_t *topo, const int32_t *lvl,
                                                        const int32_t *nlev, const int32_t *rp, const int32_t *col,
                                                        const int32_t *est, int64_t base, int64_t *rank,
                                                        int32_t *stat) {
    const DagDesc d = desc[blockIdx.x];
    if (d.n == 0) return;
    const int32_t *q = topo + d.toff;
    const int32_t *ls = lvl + d.toff + d.id;
    const int32_t *r = rp + d.toff + d.id;
    const int32_t *c = col + d.eoff;
    const int2 *e2 = reinterpret_cast<const int2 *>(est) + (d.toff - base);
    int64_t *R = rank + d.toff;
    bool wide = false;
    for (int32_t L = nlev[d.id] - 1; L >= 0; L--) {
        const int32_t z = ls[L + 1];
        for (int32_t i = ls[L] + threadIdx.x; i < z; i += kRankThreads) {
            const int32_t v = q[i];
            int64_t best = 0;
            for (int32_t e = r[v]; e < r[v + 1]; e++) best = max(best, R[c[e]]);
            const int2 x = e2[v];
            const int64_t rv = (int64_t)d.n_cpu * x.x + (int64_t)d.n_gpu * x.y + best;
            R[v] = rv;
            wide |= rv >= (1ll << kRankBits);
        }
        __syncthreads();  // the level's ranks are visible to the level below
    }
    if (wide) atomicOr(&stat[2 * d.id], ST_RANK);
}

// Levels of every DAG of the handle, built on the first HEFT call.
int ensure_levels(insp_dag *dag, hipStream_t st) {
    if (dag->nlev.p) return INSP_OK;
    const int64_t N = std::max<int64_t>(dag->N, 1);
    DevBuf indeg, nlev;
    int rc;
    if ((rc = dag->topo.alloc(sizeof(int32_t) * N)) || (rc = dag->lvl.alloc(sizeof(int32_t) * (N + dag->B))) ||
        (rc = indeg.alloc(sizeof(int32_t) * N)) || (rc = nlev.alloc(sizeof(int32_t) * dag->B)))
        return rc;
    hipLaunchKernelGGL(k_levels, dim3((unsigned)dag->B), dim3(kRankThreads), 0, st, dag->d_toff.as<int64_t>(),
                       dag->d_eoff.as<int64_t>(), dag->rp.as<int32_t>(), dag->col.as<int32_t>(),
                       dag->word0.as<unsigned long long>(), indeg.as<int32_t>(), dag->topo.as<int32_t>(),
                       dag->lvl.as<int32_t>(), nlev.as<int32_t>());
    INSP_HIP(hipGetLastError());
    INSP_HIP(hipStreamSynchronize(st));  // before indeg is freed
    std::swap(dag->nlev.p, nlev.p);
    std::swap(dag->nlev.bytes, nlev.bytes);
    return INSP_OK;
}

int run_rank(insp_dag *dag, Workspace *ws, const int32_t *est, hipStream_t st) {
    int rc;
    if ((rc = ensure_levels(dag, st))) return rc;
    if (!dag->rank.p && (rc = dag->rank.alloc(sizeof(int64_t) * std::max<int64_t>(dag->N, 1)))) return rc;
    if (ws->count > 0) {
        ProfScope ps(st, "rank");
        hipLaunchKernelGGL(k_rank, dim3((unsigned)ws->count), dim3(kRankThreads), 0, st, ws->desc.as<DagDesc>(),
                           dag->topo.as<int32_t>(), dag->lvl.as<int32_t>(), dag->nlev.as<int32_t>(),
                           dag->rp.as<int32_t>(), dag->col.as<int32_t>(), est, ws->base, dag->rank.as<int64_t>(),
                           dag->dag_stat.as<int32_t>());
    }
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

}  // namespace insp
