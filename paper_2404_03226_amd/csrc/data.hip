// Data model support: per-task output sizes on the handle, and predecessor
// lists (a task's inputs are its predecessors' outputs), built once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

__device__ __forceinline__ int32_t dag_of_task(const int64_t *toff, int32_t B, int64_t t) {
    int32_t lo = 0, hi = B - 1;  // last b with toff[b] <= t
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (toff[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// In-degree of every task, from the build's initial dependency words.
__global__ __launch_bounds__(256) void k_indeg(int64_t N, const unsigned long long *word0, int64_t *indeg) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < N) indeg[t] = (int64_t)(word0[t] >> 43);
}

// Local predecessor row pointers (same layout as the successor rows: DAG b's
// n_b + 1 entries start at task_off[b] + b).
__global__ __launch_bounds__(256) void k_pred_rows(int32_t B, const int64_t *toff, const int64_t *eoff,
                                                    const int64_t *excl, const int64_t *indeg, int32_t *pprp) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= toff[B]) return;
    const int32_t b = dag_of_task(toff, B, t);
    const int64_t i = t - toff[b];
    pprp[toff[b] + b + i] = (int32_t)(excl[t] - eoff[b]);
    if (t == toff[b + 1] - 1) pprp[toff[b] + b + i + 1] = (int32_t)(excl[t] + indeg[t] - eoff[b]);
}

// Scatter every edge u -> s into s's predecessor row (any order in a row).
__global__ __launch_bounds__(256) void k_pred_fill(int32_t B, const int64_t *toff, const int64_t *eoff,
                                                    const int32_t *rp, const int32_t *col, const int64_t *excl,
                                                    int32_t *fill, int32_t *ppred) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= toff[B]) return;
    const int32_t b = dag_of_task(toff, B, t);
    const int32_t u = (int32_t)(t - toff[b]);
    const int32_t *r = rp + toff[b] + b;
    const int32_t *c = col + eoff[b];
    for (int32_t e = r[u]; e < r[u + 1]; e++) {
        const int64_t s = toff[b] + c[e];
        ppred[excl[s] + atomicAdd(&fill[s], 1)] = u;
    }
}

__global__ __launch_bounds__(256) void k_check_kib(int64_t N, const int32_t *kib, int32_t *bad) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < N && (kib[t] < 0 || kib[t] > INSP_MAX_TICK)) atomicOr(bad, 1);
}

int ensure_preds(insp_dag *dag, hipStream_t st) {
    if (dag->ppred.p) return INSP_OK;
    const int64_t N = std::max<int64_t>(dag->N, 1), M = std::max<int64_t>(dag->M, 1);
    DevBuf indeg, excl, fill, ppred;
    int rc;
    if ((rc = indeg.alloc(sizeof(int64_t) * N)) || (rc = excl.alloc(sizeof(int64_t) * (N + 1))) ||
        (rc = fill.alloc(sizeof(int32_t) * N)) || (rc = dag->pprp.alloc(sizeof(int32_t) * (N + dag->B))) ||
        (rc = ppred.alloc(sizeof(int32_t) * M)))
        return rc;
    INSP_HIP(hipMemsetAsync(fill.p, 0, sizeof(int32_t) * N, st));
    INSP_HIP(hipMemsetAsync(dag->pprp.p, 0, sizeof(int32_t) * (N + dag->B), st));  // empty DAGs: {0}
    if (dag->N > 0) {
        const unsigned g = (unsigned)((dag->N + 255) / 256);
        hipLaunchKernelGGL(k_indeg, dim3(g), dim3(256), 0, st, dag->N, dag->word0.as<unsigned long long>(),
                           indeg.as<int64_t>());
        if ((rc = exclusive_scan(indeg.as<int64_t>(), dag->N, excl.as<int64_t>(), st))) return rc;
        hipLaunchKernelGGL(k_pred_rows, dim3(g), dim3(256), 0, st, dag->B, dag->d_toff.as<int64_t>(),
                           dag->d_eoff.as<int64_t>(), excl.as<int64_t>(), indeg.as<int64_t>(), dag->pprp.as<int32_t>());
        hipLaunchKernelGGL(k_pred_fill, dim3(g), dim3(256), 0, st, dag->B, dag->d_toff.as<int64_t>(),
                           dag->d_eoff.as<int64_t>(), dag->rp.as<int32_t>(), dag->col.as<int32_t>(),
                           excl.as<int64_t>(), fill.as<int32_t>(), ppred.as<int32_t>());
    }
    INSP_HIP(hipGetLastError());
    INSP_HIP(hipStreamSynchronize(st));  // before the scratch is freed
    std::swap(dag->ppred.p, ppred.p);
    std::swap(dag->ppred.bytes, ppred.bytes);
    return INSP_OK;
}

}  // namespace insp

using namespace insp;

extern "C" int insp_set_task_data(insp_dag *dag, const int32_t *data_kib, void *stream) {
    if (!dag) return set_error(INSP_E_INVAL, "null handle");
    hipStream_t st = (hipStream_t)stream;
    INSP_HIP(hipSetDevice(dag->device));
    if (!data_kib) {
        INSP_HIP(hipStreamSynchronize(st));
        dag->dkib.release();
        return INSP_OK;
    }
    const int64_t N = std::max<int64_t>(dag->N, 1);
    DevBuf bad, kib;
    int rc;
    if ((rc = bad.alloc(sizeof(int32_t))) || (rc = kib.alloc(sizeof(int32_t) * N))) return rc;
    INSP_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), st));
    if (dag->N > 0) {
        INSP_HIP(hipMemcpyAsync(kib.p, data_kib, sizeof(int32_t) * dag->N, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_check_kib, dim3((unsigned)((dag->N + 255) / 256)), dim3(256), 0, st, dag->N,
                           kib.as<int32_t>(), bad.as<int32_t>());
    }
    INSP_HIP(hipGetLastError());
    int32_t h_bad = 0;
    INSP_HIP(hipMemcpyAsync(&h_bad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    if (h_bad) return set_error(INSP_E_RANGE, "data size outside [0, 2^20] KiB");
    std::swap(dag->dkib.p, kib.p);
    std::swap(dag->dkib.bytes, kib.bytes);
    return INSP_OK;
}
