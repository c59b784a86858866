// DAG build: validation and canonicalisation of user CSR graphs on the
// device, the initial in-degree / predecessor-sum words used by the
// simulation, and the cycle check (Kahn traversal from the tasks with zero
// in-degree, as in Section 4.3 of the paper).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int set_lds_limit(const void *kernel, size_t bytes) {
    if (bytes <= 65536) return INSP_OK;
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> done;
    int dev = 0;
    INSP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    size_t &cur = done[{kernel, dev}];
    if (bytes <= cur) return INSP_OK;
    INSP_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    cur = bytes;
    return INSP_OK;
}

// Allocation-failure injection (insp_test_fail_alloc): the number of device
// allocations still allowed to succeed, or -1 for no injection.
static std::atomic<int64_t> g_fail_after{-1};

int DevBuf::alloc(size_t nbytes) {
    release();
    if (nbytes == 0) nbytes = 16;
    for (int64_t k = g_fail_after.load(); k >= 0;) {
        if (k == 0) {
            g_fail_after.store(-1);
            return set_error(INSP_E_NOMEM, "hipMalloc(%zu) failed: injected allocation failure", nbytes);
        }
        if (g_fail_after.compare_exchange_weak(k, k - 1)) break;
    }
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        p = nullptr;
        return set_error(INSP_E_NOMEM, "hipMalloc(%zu) failed: %s", nbytes, hipGetErrorString(e));
    }
    bytes = nbytes;
    return INSP_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

// Bits of a packed (row, target) sort key: targets are DAG-local ids < 2^21.
constexpr int kColBits = 21;
enum { ERR_ROWPTR = 1, ERR_COL = 2, ERR_SELF = 4 };

__device__ __forceinline__ int32_t dag_of(const int64_t *toff, int32_t B, int64_t v) {
    int32_t lo = 0, hi = B - 1;  // last b with toff[b] <= v
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (toff[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One thread per task: check the row pointer and the row's targets, and emit
// one packed key per edge.
__global__ void k_rows(int32_t B, const int64_t *toff, const int64_t *eoff, const int32_t *rp, const int32_t *col,
                       uint64_t *keys, int32_t *err) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= toff[B]) return;
    int32_t b = dag_of(toff, B, v);
    int64_t lv = v - toff[b];
    int32_t n = (int32_t)(toff[b + 1] - toff[b]);
    int64_t m = eoff[b + 1] - eoff[b];
    const int32_t *r = rp + toff[b] + b;
    int32_t a = r[lv], z = r[lv + 1];
    int bad = 0;
    if (lv == 0 && a != 0) bad |= ERR_ROWPTR;
    if (lv == n - 1 && z != m) bad |= ERR_ROWPTR;
    if (z < a || a < 0 || z > m) bad |= ERR_ROWPTR;
    if (!bad) {
        for (int32_t e = a; e < z; e++) {
            int32_t s = col[eoff[b] + e];
            if (s < 0 || s >= n) bad |= ERR_COL;
            else if (s == lv) bad |= ERR_SELF;
            keys[eoff[b] + e] = ((uint64_t)v << kColBits) | (uint32_t)(s & ((1 << kColBits) - 1));
        }
    }
    if (bad) atomicOr(err, bad);
}

// After sorting: flag the first copy of every (row, target) pair.
__global__ void k_unique(int64_t M, const uint64_t *keys, int32_t *flag) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= M) return;
    flag[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

// Scatter unique edges, count canonical out-degrees, and accumulate the
// in-degree and predecessor-id sum of each target.
__global__ void k_scatter(int64_t M, const uint64_t *keys, const int32_t *flag, const int32_t *pos,
                          const int64_t *toff, int32_t B, int32_t *col_out, int32_t *outdeg,
                          unsigned long long *word0, int32_t *backward) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= M || !flag[e]) return;
    uint64_t k = keys[e];
    int64_t v = (int64_t)(k >> kColBits);
    int32_t s = (int32_t)(k & ((1 << kColBits) - 1));
    int32_t b = dag_of(toff, B, v);
    int32_t lv = (int32_t)(v - toff[b]);
    col_out[pos[e]] = s;
    atomicAdd(&outdeg[v], 1);
    // word0 = in-degree << 43 | sum of predecessor ids (fits: ids < 2^21)
    atomicAdd(&word0[toff[b] + s], (1ull << 43) + (unsigned long long)lv);
    if (s < lv) atomicOr(backward, 1 << 0), atomicOr(&backward[1 + (b >> 5)], 1 << (b & 31));
}

// Local row pointers from the global exclusive scan of out-degrees.
__global__ void k_rowptr(int32_t B, const int64_t *toff, const int64_t *excl, const int32_t *outdeg,
                         const int64_t *eoff_c, int32_t *rp_out) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= toff[B]) return;
    int32_t b = dag_of(toff, B, v);
    int64_t lv = v - toff[b];
    rp_out[toff[b] + b + lv] = (int32_t)(excl[v] - eoff_c[b]);
    if (lv == toff[b + 1] - toff[b] - 1) rp_out[toff[b] + b + lv + 1] = (int32_t)(excl[v] + outdeg[v] - eoff_c[b]);
}

// Kahn traversal of one DAG per work-group (used only when some edge points
// from a higher id to a lower one, where id order proves nothing).
__global__ void k_kahn(const int32_t *dags, const int64_t *toff, const int64_t *eoff, const int32_t *rp,
                       const int32_t *col, const unsigned long long *word0, int32_t *indeg, int32_t *queue,
                       int32_t *visited_out) {
    int32_t b = dags[blockIdx.x];
    int64_t t0 = toff[b];
    int32_t n = (int32_t)(toff[b + 1] - t0);
    const int32_t *r = rp + t0 + b;
    const int32_t *c = col + eoff[b];
    int32_t *deg = indeg + t0;
    int32_t *q = queue + t0;
    __shared__ int32_t tail;
    if (threadIdx.x == 0) tail = 0;
    __syncthreads();
    for (int32_t v = threadIdx.x; v < n; v += blockDim.x) {
        deg[v] = (int32_t)(word0[t0 + v] >> 43);
        if (deg[v] == 0) q[atomicAdd(&tail, 1)] = v;
    }
    __syncthreads();
    int32_t head = 0;
    for (;;) {
        int32_t end = tail;
        __syncthreads();
        if (head == end) break;
        for (int32_t i = head + threadIdx.x; i < end; i += blockDim.x) {
            int32_t v = q[i];
            for (int32_t e = r[v]; e < r[v + 1]; e++)
                if (atomicSub(&deg[c[e]], 1) == 1) q[atomicAdd(&tail, 1)] = c[e];
        }
        head = end;
        __syncthreads();
    }
    if (threadIdx.x == 0) visited_out[blockIdx.x] = tail;
}

static inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace insp

using namespace insp;

extern "C" const char *insp_last_error(void) { return g_last_error.c_str(); }

extern "C" int insp_test_fail_alloc(int64_t after) {
    if (after < -1) return set_error(INSP_E_INVAL, "insp_test_fail_alloc: after must be >= -1");
    g_fail_after.store(after);
    return INSP_OK;
}

extern "C" void insp_free_dag(insp_dag *dag) { delete dag; }

extern "C" int insp_dag_info(const insp_dag *dag, int32_t index, int64_t *n_tasks, int64_t *n_edges,
                             int32_t *n_dags) {
    if (!dag) return set_error(INSP_E_INVAL, "null handle");
    if (n_dags) *n_dags = dag->B;
    if (index < 0 || index >= dag->B) return set_error(INSP_E_INVAL, "dag index %d out of [0, %d)", index, dag->B);
    if (n_tasks) *n_tasks = dag->toff[index + 1] - dag->toff[index];
    if (n_edges) *n_edges = dag->eoff[index + 1] - dag->eoff[index];
    return INSP_OK;
}

namespace {

struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    int get(T **out, size_t count) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16));
        if (e != hipSuccess)
            return set_error(INSP_E_NOMEM, "hipMalloc(%zu) failed: %s", count * sizeof(T), hipGetErrorString(e));
        ptrs.push_back(p);
        *out = static_cast<T *>(p);
        return INSP_OK;
    }
};

}  // namespace

extern "C" int insp_build_dag(int32_t n_dags, const int64_t *task_off, const int64_t *edge_off,
                              const int32_t *row_ptr, const int32_t *col, const int32_t *type, void *stream_,
                              insp_dag **out) {
    if (!out) return set_error(INSP_E_INVAL, "out is null");
    *out = nullptr;
    if (n_dags < 1 || !task_off || !edge_off) return set_error(INSP_E_INVAL, "need n_dags >= 1 and offsets");
    if (task_off[0] != 0 || edge_off[0] != 0) return set_error(INSP_E_INVAL, "offsets must start at 0");
    for (int32_t b = 0; b < n_dags; b++) {
        int64_t n = task_off[b + 1] - task_off[b], m = edge_off[b + 1] - edge_off[b];
        if (n < 0 || m < 0) return set_error(INSP_E_INVAL, "offsets of DAG %d decrease", b);
        if (n > INSP_MAX_TASKS) return set_error(INSP_E_RANGE, "DAG %d has %lld tasks (max 2^21)", b, (long long)n);
        if (m >= ((int64_t)1 << 31)) return set_error(INSP_E_RANGE, "DAG %d has too many edges", b);
        if (n == 0 && m != 0) return set_error(INSP_E_INVAL, "DAG %d has edges but no tasks", b);
    }
    const int64_t N = task_off[n_dags], M = edge_off[n_dags];
    if (N > 0 && (!row_ptr || (M > 0 && !col))) return set_error(INSP_E_INVAL, "null row_ptr/col");
    hipStream_t st = (hipStream_t)stream_;

    std::unique_ptr<insp_dag> d(new insp_dag());
    d->B = n_dags;
    INSP_HIP(hipGetDevice(&d->device));
    d->N = N;
    d->toff.assign(task_off, task_off + n_dags + 1);
    int rc;
    if ((rc = d->d_toff.alloc(sizeof(int64_t) * (n_dags + 1)))) return rc;
    INSP_HIP(hipMemcpyAsync(d->d_toff.p, task_off, sizeof(int64_t) * (n_dags + 1), hipMemcpyHostToDevice, st));
    Scratch s;
    int64_t *d_eoff_in;
    if ((rc = s.get(&d_eoff_in, n_dags + 1))) return rc;
    INSP_HIP(hipMemcpyAsync(d_eoff_in, edge_off, sizeof(int64_t) * (n_dags + 1), hipMemcpyHostToDevice, st));

    uint64_t *keys, *keys_sorted;
    int32_t *err, *flag, *pos, *outdeg, *backward;
    int64_t *excl;
    const int nbw = 1 + (n_dags + 31) / 32;
    if ((rc = s.get(&keys, M)) || (rc = s.get(&keys_sorted, M)) || (rc = s.get(&err, 1)) ||
        (rc = s.get(&flag, M)) || (rc = s.get(&pos, M + 1)) || (rc = s.get(&outdeg, N)) ||
        (rc = s.get(&backward, nbw)) || (rc = s.get(&excl, N + 1)))
        return rc;
    INSP_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), st));
    INSP_HIP(hipMemsetAsync(backward, 0, sizeof(int32_t) * nbw, st));
    INSP_HIP(hipMemsetAsync(outdeg, 0, sizeof(int32_t) * std::max<int64_t>(N, 1), st));
    if ((rc = d->word0.alloc(sizeof(uint64_t) * N))) return rc;
    INSP_HIP(hipMemsetAsync(d->word0.p, 0, sizeof(uint64_t) * std::max<int64_t>(N, 1), st));

    if (N > 0)
        hipLaunchKernelGGL(k_rows, dim3(grid_for(N, 256)), dim3(256), 0, st, n_dags, d->d_toff.as<int64_t>(),
                           d_eoff_in, row_ptr, col, keys, err);
    INSP_HIP(hipGetLastError());
    int32_t h_err = 0;
    INSP_HIP(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    if (h_err & ERR_ROWPTR) return set_error(INSP_E_INVAL, "row_ptr is not a valid CSR row pointer");
    if (h_err & ERR_COL) return set_error(INSP_E_INVAL, "successor id out of range");
    if (h_err & ERR_SELF) return set_error(INSP_E_INVAL, "self loop");

    // Sort packed (global row, local target) keys: rows become contiguous
    // and ascending, targets ascending inside a row, repeats adjacent.
    int end_bit = kColBits;
    while (end_bit < 64 && (((uint64_t)std::max<int64_t>(N, 1)) >> (end_bit - kColBits)) != 0) end_bit++;
    size_t tmp_bytes = 0;
    if (M > 0) {
        INSP_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_bytes, keys, keys_sorted, (int)M, 0, end_bit, st));
        uint8_t *tmp;
        if ((rc = s.get(&tmp, tmp_bytes))) return rc;
        INSP_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, keys, keys_sorted, (int)M, 0, end_bit, st));
        hipLaunchKernelGGL(k_unique, dim3(grid_for(M, 256)), dim3(256), 0, st, M, keys_sorted, flag);
        size_t t2 = 0;
        INSP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, t2, flag, pos, (int)M, st));
        uint8_t *tmp2;
        if ((rc = s.get(&tmp2, t2))) return rc;
        INSP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp2, t2, flag, pos, (int)M, st));
    }
    int32_t h_last[2] = {0, 0};
    if (M > 0) {
        INSP_HIP(hipMemcpyAsync(&h_last[0], pos + M - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        INSP_HIP(hipMemcpyAsync(&h_last[1], flag + M - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
    INSP_HIP(hipStreamSynchronize(st));
    const int64_t Mc = M > 0 ? (int64_t)h_last[0] + h_last[1] : 0;
    d->M = Mc;
    if ((rc = d->col.alloc(sizeof(int32_t) * Mc))) return rc;
    if (M > 0)
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(M, 256)), dim3(256), 0, st, M, keys_sorted, flag, pos,
                           d->d_toff.as<int64_t>(), n_dags, d->col.as<int32_t>(), outdeg,
                           d->word0.as<unsigned long long>(), backward);
    INSP_HIP(hipGetLastError());

    // Canonical row pointers: global exclusive scan of out-degrees, made
    // local by subtracting each DAG's first canonical edge.
    std::vector<int32_t> h_outdeg(N);
    if (N > 0) INSP_HIP(hipMemcpyAsync(h_outdeg.data(), outdeg, sizeof(int32_t) * N, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    std::vector<int64_t> h_excl(N + 1, 0);
    for (int64_t v = 0; v < N; v++) h_excl[v + 1] = h_excl[v] + h_outdeg[v];
    d->eoff.resize(n_dags + 1);
    for (int32_t b = 0; b <= n_dags; b++) d->eoff[b] = h_excl[task_off[b]];
    if ((rc = d->d_eoff.alloc(sizeof(int64_t) * (n_dags + 1)))) return rc;
    INSP_HIP(hipMemcpyAsync(d->d_eoff.p, d->eoff.data(), sizeof(int64_t) * (n_dags + 1), hipMemcpyHostToDevice, st));
    INSP_HIP(hipMemcpyAsync(excl, h_excl.data(), sizeof(int64_t) * (N + 1), hipMemcpyHostToDevice, st));
    if ((rc = d->rp.alloc(sizeof(int32_t) * (N + n_dags)))) return rc;
    INSP_HIP(hipMemsetAsync(d->rp.p, 0, sizeof(int32_t) * (N + n_dags), st));  // empty DAGs: rp = {0}
    if (N > 0)
        hipLaunchKernelGGL(k_rowptr, dim3(grid_for(N, 256)), dim3(256), 0, st, n_dags, d->d_toff.as<int64_t>(),
                           excl, outdeg, d->d_eoff.as<int64_t>(), d->rp.as<int32_t>());
    INSP_HIP(hipGetLastError());

    // Cycle check: with every edge pointing to a higher id the id order is a
    // topological order; otherwise run Kahn's traversal on the DAGs concerned.
    std::vector<int32_t> h_back(nbw);
    INSP_HIP(hipMemcpyAsync(h_back.data(), backward, sizeof(int32_t) * nbw, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    if (h_back[0]) {
        std::vector<int32_t> todo;
        for (int32_t b = 0; b < n_dags; b++)
            if (h_back[1 + (b >> 5)] >> (b & 31) & 1) todo.push_back(b);
        int32_t *d_todo, *indeg, *queue, *visited;
        if ((rc = s.get(&d_todo, todo.size())) || (rc = s.get(&indeg, N)) || (rc = s.get(&queue, N)) ||
            (rc = s.get(&visited, todo.size())))
            return rc;
        INSP_HIP(hipMemcpyAsync(d_todo, todo.data(), sizeof(int32_t) * todo.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_kahn, dim3((unsigned)todo.size()), dim3(256), 0, st, d_todo, d->d_toff.as<int64_t>(),
                           d->d_eoff.as<int64_t>(), d->rp.as<int32_t>(), d->col.as<int32_t>(),
                           d->word0.as<unsigned long long>(), indeg, queue, visited);
        INSP_HIP(hipGetLastError());
        std::vector<int32_t> h_vis(todo.size());
        INSP_HIP(hipMemcpyAsync(h_vis.data(), visited, sizeof(int32_t) * todo.size(), hipMemcpyDeviceToHost, st));
        INSP_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < todo.size(); i++) {
            int32_t b = todo[i];
            if (h_vis[i] != task_off[b + 1] - task_off[b])
                return set_error(INSP_E_CYCLE, "DAG %d has a dependency cycle", b);
        }
    }
    if (type && N > 0) {
        if ((rc = d->type.alloc(sizeof(int32_t) * N))) return rc;
        INSP_HIP(hipMemcpyAsync(d->type.p, type, sizeof(int32_t) * N, hipMemcpyDeviceToDevice, st));
    }
    // Largest DAGs first: they set the batch's critical path.
    d->order.resize(n_dags);
    std::iota(d->order.begin(), d->order.end(), 0);
    std::stable_sort(d->order.begin(), d->order.end(), [&](int32_t a, int32_t b) {
        int64_t wa = (d->toff[a + 1] - d->toff[a]) + (d->eoff[a + 1] - d->eoff[a]);
        int64_t wb = (d->toff[b + 1] - d->toff[b]) + (d->eoff[b + 1] - d->eoff[b]);
        return wa > wb;
    });
    INSP_HIP(hipStreamSynchronize(st));
    *out = d.release();
    return INSP_OK;
}
