// DAG build: validation and canonicalisation of user CSR graphs on the
// device, the initial in-degree / predecessor-sum words used by the
// simulation, and the cycle check (Kahn traversal from the tasks with zero
// in-degree, as in Section 4.3 of the paper).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
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
    if (p && own) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    own = true;
}

enum { ERR_ROWPTR = 1, ERR_COL = 2, ERR_SELF = 4 };

// Canonical rows are built where the input rows lie: each row is sorted and
// its repeats dropped into a scratch copy at the row's own input offset, its
// canonical length counted; an exclusive scan of those lengths places the
// canonical rows, and a last pass moves them there.  Rows are sorted by
// whoever fits them: a thread in registers (up to kSmallRow entries), one
// wave in LDS (kWaveRow), a 256-thread work-group in LDS (kBlockRow), and
// above that a work-group marks the row's targets in a bitmap of the DAG's
// tasks and reads them back in order (targets are distinct task ids).
constexpr int kSmallRow = 16;
constexpr int kWaveRow = 1024;
constexpr int kBlockRow = 16384;
constexpr int kHugeSlots = 16;  // work-groups (and bitmaps) for rows above kBlockRow
constexpr int32_t kPad = 0x7fffffff;

__device__ __forceinline__ int32_t dag_of(const int64_t *toff, int32_t B, int64_t v) {
    int32_t lo = 0, hi = B - 1;  // last b with toff[b] <= v
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (toff[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct RowArgs {
    int32_t B;
    const int64_t *toff, *eoff;  // task offsets, input edge offsets
    const int32_t *rp, *col;     // the caller's CSR
    int32_t *tmp;                // [M] sorted, deduplicated rows at their input offsets
    int32_t *outdeg;             // [N] canonical row lengths
    int32_t *err;
    int32_t *nwide;              // rows longer than kSmallRow ...
    int64_t *wide;               // ... listed here
    uint32_t *bits;              // [kHugeSlots][bit_words] bitmaps for the longest rows
    int64_t bit_words;
};

// Row v of the global task order: its DAG, local id, task count and input
// row [a, z) (local edge indices).
struct Row {
    int32_t b, lv, n, a, z;
};

__device__ __forceinline__ Row row_of(const RowArgs &A, int64_t v) {
    Row r;
    r.b = dag_of(A.toff, A.B, v);
    r.lv = (int32_t)(v - A.toff[r.b]);
    r.n = (int32_t)(A.toff[r.b + 1] - A.toff[r.b]);
    const int32_t *p = A.rp + A.toff[r.b] + r.b;
    r.a = p[r.lv];
    r.z = p[r.lv + 1];
    return r;
}

__device__ __forceinline__ int check_target(int32_t s, int32_t n, int32_t lv) {
    return (s < 0 || s >= n) ? ERR_COL : (s == lv ? ERR_SELF : 0);
}

// Bitonic sorting network over a register array (all indices fold to
// constants once the loops are unrolled).
template <int P>
__device__ __forceinline__ void sort_registers(int32_t (&x)[P]) {
#pragma unroll
    for (int k = 2; k <= P; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < P; i++) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t lo = min(x[i], x[l]), hi = max(x[i], x[l]);
                    const bool up = (i & k) == 0;
                    x[i] = up ? lo : hi;
                    x[l] = up ? hi : lo;
                }
            }
}

// One thread per task: validate the row pointer and, for short rows, the
// targets; sort and deduplicate short rows in registers; list the others.
__global__ __launch_bounds__(256) void k_rows(RowArgs A) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= A.toff[A.B]) return;
    const Row r = row_of(A, v);
    const int64_t m = A.eoff[r.b + 1] - A.eoff[r.b];
    int bad = 0;
    if (r.lv == 0 && r.a != 0) bad |= ERR_ROWPTR;
    if (r.lv == r.n - 1 && r.z != m) bad |= ERR_ROWPTR;
    if (r.z < r.a || r.a < 0 || r.z > m) bad |= ERR_ROWPTR;
    if (bad) {
        atomicOr(A.err, bad);
        A.outdeg[v] = 0;
        return;
    }
    const int32_t deg = r.z - r.a;
    if (deg > kSmallRow) {
        A.wide[atomicAdd(A.nwide, 1)] = v;
        return;
    }
    const int32_t *src = A.col + A.eoff[r.b] + r.a;
    int32_t *dst = A.tmp + A.eoff[r.b] + r.a;
    int32_t x[kSmallRow];
#pragma unroll
    for (int i = 0; i < kSmallRow; i++) {
        x[i] = i < deg ? src[i] : kPad;
        if (i < deg) bad |= check_target(x[i], r.n, r.lv);
    }
    sort_registers<kSmallRow>(x);
    int32_t cnt = 0, prev = -1;
#pragma unroll
    for (int i = 0; i < kSmallRow; i++) {
        if (i < deg && x[i] != prev) {
            dst[cnt++] = x[i];
            prev = x[i];
        }
    }
    A.outdeg[v] = cnt;
    if (bad) atomicOr(A.err, bad);
}

// Bitonic sort of buf[0, P) in LDS by the work-group, then write the distinct
// values of its first `deg` entries in order to dst; returns their count.
template <int THREADS>
__device__ int32_t sort_unique_lds(int32_t *buf, int32_t P, int32_t deg, int32_t *dst, int32_t *wcnt) {
    const int tid = threadIdx.x;
    for (int32_t k = 2; k <= P; k <<= 1)
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            for (int32_t i = tid; i < P; i += THREADS) {
                const int32_t l = i ^ j;
                if (l > i) {
                    const int32_t a = buf[i], c = buf[l];
                    const bool up = (i & k) == 0;
                    if (up ? a > c : a < c) {
                        buf[i] = c;
                        buf[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    int32_t base = 0;
    const int wv = tid / kWave;
    for (int32_t i0 = 0; i0 < deg; i0 += THREADS) {
        const int32_t i = i0 + tid;
        const bool first = i < deg && (i == 0 || buf[i] != buf[i - 1]);
        const uint64_t mk = ballot(first);
        if ((tid & (kWave - 1)) == 0) wcnt[wv] = __popcll(mk);
        __syncthreads();
        int32_t off = base, tot = 0;
        for (int w = 0; w < THREADS / kWave; w++) {
            if (w < wv) off += wcnt[w];
            tot += wcnt[w];
        }
        if (first) dst[off + lanes_below(mk)] = buf[i];
        base += tot;
        __syncthreads();
    }
    return base;
}

// Rows of kSmallRow < deg <= LIMIT: one work-group of THREADS per listed row
// (listed rows of other lengths are left to the other kernels).
template <int THREADS, int LIMIT, int LOWER>
__global__ __launch_bounds__(THREADS) void k_rows_lds(RowArgs A) {
    __shared__ int32_t buf[LIMIT];
    __shared__ int32_t wcnt[THREADS / kWave];
    const int64_t v = A.wide[blockIdx.x];
    const Row r = row_of(A, v);
    const int32_t deg = r.z - r.a;
    if (deg <= LOWER || deg > LIMIT) return;
    const int32_t *src = A.col + A.eoff[r.b] + r.a;
    int32_t P = 32;
    while (P < deg) P <<= 1;
    int bad = 0;
    for (int32_t i = threadIdx.x; i < P; i += THREADS) {
        const int32_t s = i < deg ? src[i] : kPad;
        if (i < deg) bad |= check_target(s, r.n, r.lv);
        buf[i] = s;
    }
    if (bad) atomicOr(A.err, bad);
    __syncthreads();
    const int32_t cnt = sort_unique_lds<THREADS>(buf, P, deg, A.tmp + A.eoff[r.b] + r.a, wcnt);
    if (threadIdx.x == 0) A.outdeg[v] = cnt;
}

// Rows above kBlockRow: mark the targets in a bitmap of the DAG's tasks and
// read them back in ascending order (a repeated target marks the same bit).
__global__ __launch_bounds__(256) void k_rows_huge(RowArgs A, int32_t nlisted) {
    __shared__ int64_t part[256 / kWave];
    uint32_t *bm = A.bits + (int64_t)blockIdx.x * A.bit_words;
    const int tid = threadIdx.x;
    for (int32_t k = blockIdx.x; k < nlisted; k += gridDim.x) {
        const int64_t v = A.wide[k];
        const Row r = row_of(A, v);
        const int32_t deg = r.z - r.a;
        if (deg <= kBlockRow) continue;  // uniform over the work-group
        const int32_t words = (r.n + 31) / 32;
        for (int32_t w = tid; w < words; w += 256) bm[w] = 0;
        __threadfence();
        __syncthreads();
        const int32_t *src = A.col + A.eoff[r.b] + r.a;
        int bad = 0;
        for (int32_t i = tid; i < deg; i += 256) {
            const int32_t s = src[i];
            const int e = check_target(s, r.n, r.lv);
            bad |= e;
            if (!(e & ERR_COL)) atomicOr(&bm[s >> 5], 1u << (s & 31));
        }
        if (bad) atomicOr(A.err, bad);
        __threadfence();
        __syncthreads();
        // each thread reads back a contiguous run of words
        const int32_t per = (words + 255) / 256, w0 = min(words, tid * per), w1 = min(words, w0 + per);
        int64_t c = 0;
        for (int32_t w = w0; w < w1; w++)
            c += __popc(__hip_atomic_load(&bm[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        // block-wide exclusive scan of the counts
        const int lane = tid & (kWave - 1), wv = tid / kWave;
        int64_t inc = c;
        for (int o = 1; o < kWave; o <<= 1) {
            const int64_t y = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += y;
        }
        if (lane == kWave - 1) part[wv] = inc;
        __syncthreads();
        int64_t pos = inc - c, tot = 0;
        for (int w = 0; w < 256 / kWave; w++) {
            if (w < wv) pos += part[w];
            tot += part[w];
        }
        int32_t *dst = A.tmp + A.eoff[r.b] + r.a;
        for (int32_t w = w0; w < w1; w++) {
            uint32_t x = __hip_atomic_load(&bm[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (x) {
                dst[pos++] = w * 32 + (int32_t)__builtin_ctz(x);
                x &= x - 1;
            }
        }
        if (tid == 0) A.outdeg[v] = (int32_t)tot;
        __syncthreads();  // part and the bitmap are reused by the next row
    }
}

struct PlaceArgs {
    int32_t B;
    const int64_t *toff, *eoff;   // task offsets, input edge offsets
    const int32_t *rp;            // the caller's row pointers
    const int32_t *tmp, *outdeg;
    const int64_t *excl;          // [N + 1] exclusive scan of outdeg: global canonical row starts
    int32_t *col_out, *rp_out;
    unsigned long long *word0;
    int32_t *backward;            // [1 + ceil(B / 32)]: any edge to a lower id, per DAG bits
};

// Move row v's canonical targets to their place and account the edges in
// the targets' dependency words (in-degree << 43 | sum of predecessor ids).
__device__ __forceinline__ void place_edge(const PlaceArgs &A, int32_t b, int32_t lv, int32_t s, int64_t to,
                                           bool &back) {
    A.col_out[to] = s;
    atomicAdd(&A.word0[A.toff[b] + s], (1ull << 43) + (unsigned long long)lv);
    back |= s < lv;
}

// One thread per task: the canonical row pointer, and the row itself when
// it is short.
__global__ __launch_bounds__(256) void k_place(PlaceArgs A) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= A.toff[A.B]) return;
    const int32_t b = dag_of(A.toff, A.B, v);
    const int32_t lv = (int32_t)(v - A.toff[b]);
    const int32_t n = (int32_t)(A.toff[b + 1] - A.toff[b]);
    const int64_t e0 = A.excl[A.toff[b]];  // the DAG's first canonical edge
    const int64_t at = A.excl[v];
    const int32_t cnt = A.outdeg[v];
    A.rp_out[A.toff[b] + b + lv] = (int32_t)(at - e0);
    if (lv == n - 1) A.rp_out[A.toff[b] + b + n] = (int32_t)(at + cnt - e0);
    const int32_t *p = A.rp + A.toff[b] + b;
    if (p[lv + 1] - p[lv] > kSmallRow) return;  // a listed row: k_place_wide
    const int32_t *src = A.tmp + A.eoff[b] + p[lv];
    bool back = false;
    for (int32_t i = 0; i < cnt; i++) place_edge(A, b, lv, src[i], at + i, back);
    if (back) atomicOr(A.backward, 1), atomicOr(&A.backward[1 + (b >> 5)], 1 << (b & 31));
}

// One wave per listed (long) row.
__global__ __launch_bounds__(64) void k_place_wide(PlaceArgs A, const int64_t *wide) {
    const int64_t v = wide[blockIdx.x];
    const int32_t b = dag_of(A.toff, A.B, v);
    const int32_t lv = (int32_t)(v - A.toff[b]);
    const int32_t *p = A.rp + A.toff[b] + b;
    const int32_t *src = A.tmp + A.eoff[b] + p[lv];
    const int64_t at = A.excl[v];
    const int32_t cnt = A.outdeg[v];
    bool back = false;
    for (int32_t i = threadIdx.x; i < cnt; i += 64) place_edge(A, b, lv, src[i], at + i, back);
    if (ballot(back) && threadIdx.x == 0)
        atomicOr(A.backward, 1), atomicOr(&A.backward[1 + (b >> 5)], 1 << (b & 31));
}

// Each DAG's first canonical edge (and the total after the last DAG).
__global__ void k_dag_edges(int32_t B, const int64_t *toff, const int64_t *excl, int64_t *eoff_c) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b <= B) eoff_c[b] = excl[toff[b]];
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

// Hub rows of the large DAGs: rows with more than kHubDeg successors get a
// wave each in the grid-wide attribute pass, the longest first.
__global__ void k_hub_count(const int32_t *r, int32_t n, int32_t *cnt) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    cnt[v] = r[v + 1] - r[v] > kHubDeg ? 1 : 0;
}

__global__ void k_hub_fill(const int32_t *r, int32_t n, const int64_t *off, int32_t *rows, int32_t *degs) {
    const int32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= n || off[v + 1] == off[v]) return;
    rows[off[v]] = v;
    degs[off[v]] = r[v + 1] - r[v];
}

int build_hubs(insp_dag *dag, hipStream_t st) {
    const int32_t B = dag->B;
    dag->hub0.assign(B, 0);
    dag->nhub.assign(B, 0);
    dag->long0.assign(B, 0);
    dag->nlong.assign(B, 0);
    const int32_t max_n = large_rows(dag);
    if (max_n == 0) return INSP_OK;
    DevBuf cnt, off, rows, degs;
    int rc;
    if ((rc = cnt.alloc(sizeof(int32_t) * max_n)) || (rc = off.alloc(sizeof(int64_t) * (max_n + 1))) ||
        (rc = rows.alloc(sizeof(int32_t) * max_n)) || (rc = degs.alloc(sizeof(int32_t) * max_n)))
        return rc;
    const int32_t *rp = dag->rp.as<int32_t>();
    std::vector<int4> all;
    for (int32_t b = 0; b < B; b++) {
        const int32_t n = (int32_t)(dag->toff[b + 1] - dag->toff[b]);
        dag->hub0[b] = (int32_t)all.size();
        if (n < kGridMin) continue;
        const int32_t *r = rp + dag->toff[b] + b;
        hipLaunchKernelGGL(k_hub_count, dim3((n + 255) / 256), dim3(256), 0, st, r, n, cnt.as<int32_t>());
        if ((rc = exclusive_scan(cnt.as<int32_t>(), n, off.as<int64_t>(), st))) return rc;
        hipLaunchKernelGGL(k_hub_fill, dim3((n + 255) / 256), dim3(256), 0, st, r, n, off.as<int64_t>(),
                           rows.as<int32_t>(), degs.as<int32_t>());
        int64_t h = 0;
        INSP_HIP(hipMemcpyAsync(&h, off.as<int64_t>() + n, sizeof h, hipMemcpyDeviceToHost, st));
        INSP_HIP(hipStreamSynchronize(st));
        std::vector<int32_t> hr(h), hd(h);
        if (h > 0) {
            INSP_HIP(hipMemcpyAsync(hr.data(), rows.p, sizeof(int32_t) * h, hipMemcpyDeviceToHost, st));
            INSP_HIP(hipMemcpyAsync(hd.data(), degs.p, sizeof(int32_t) * h, hipMemcpyDeviceToHost, st));
            INSP_HIP(hipStreamSynchronize(st));
        }
        // entries: whole rows, or the pieces of rows longer than kPieceMin;
        // the longest work first
        std::vector<int4> ent;
        for (int64_t i = 0; i < h; i++) {
            const int32_t np = hd[i] > kPieceMin ? (hd[i] + kPiece - 1) / kPiece : 1;
            for (int32_t k = 0; k < np; k++) ent.push_back(make_int4(hr[i], k, np, 0));
        }
        std::stable_sort(ent.begin(), ent.end(), [&](const int4 &x, const int4 &y) {
            auto len = [&](const int4 &e) {
                const int32_t dg = hd[std::lower_bound(hr.begin(), hr.end(), e.x) - hr.begin()];
                return e.z > 1 ? std::min(kPiece, dg - e.y * kPiece) : dg;
            };
            return len(x) > len(y);
        });
        dag->nhub[b] = (int32_t)ent.size();
        all.insert(all.end(), ent.begin(), ent.end());
    }
    // piece slots: each long row's pieces get consecutive slots
    {
        std::map<std::pair<int32_t, int32_t>, int32_t> first;  // (DAG, row) -> first slot
        int32_t next = 0;
        std::vector<int4> lr;
        for (int32_t b = 0, i = 0; b < B; b++) {
            dag->long0[b] = (int32_t)lr.size();
            for (int32_t k = 0; k < dag->nhub[b]; k++, i++) {
                int4 &e = all[i];
                if (e.z <= 1) continue;
                auto key = std::make_pair(b, e.x);
                auto it = first.find(key);
                if (it == first.end()) {
                    it = first.emplace(key, next).first;
                    lr.push_back(make_int4(e.x, 0, e.z, next));
                    next += e.z;
                }
                e.w = it->second;
            }
            dag->nlong[b] = (int32_t)lr.size() - dag->long0[b];
        }
        if (next > 0 && (rc = dag->pslot.alloc(sizeof(int32_t) * 4 * (size_t)next))) return rc;
        if (!lr.empty()) {
            if ((rc = dag->lrow.alloc(sizeof(int4) * lr.size()))) return rc;
            INSP_HIP(hipMemcpyAsync(dag->lrow.p, lr.data(), sizeof(int4) * lr.size(), hipMemcpyHostToDevice, st));
            INSP_HIP(hipStreamSynchronize(st));
        }
    }
    if (!all.empty()) {
        if ((rc = dag->hub.alloc(sizeof(int4) * all.size()))) return rc;
        INSP_HIP(hipMemcpyAsync(dag->hub.p, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice, st));
    }
    INSP_HIP(hipGetLastError());
    INSP_HIP(hipStreamSynchronize(st));
    return INSP_OK;
}

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

extern "C" int insp_build_dag(int32_t n_dags, const int64_t *task_off, const int64_t *edge_off,
                              const int32_t *row_ptr, const int32_t *col, const int32_t *type, void *stream_,
                              insp_dag **out) {
    if (!out) return set_error(INSP_E_INVAL, "out is null");
    *out = nullptr;
    if (n_dags < 1 || !task_off || !edge_off) return set_error(INSP_E_INVAL, "need n_dags >= 1 and offsets");
    if (task_off[0] != 0 || edge_off[0] != 0) return set_error(INSP_E_INVAL, "offsets must start at 0");
    int32_t max_n = 0;
    for (int32_t b = 0; b < n_dags; b++) {
        int64_t n = task_off[b + 1] - task_off[b], m = edge_off[b + 1] - edge_off[b];
        if (n < 0 || m < 0) return set_error(INSP_E_INVAL, "offsets of DAG %d decrease", b);
        if (n > INSP_MAX_TASKS) return set_error(INSP_E_RANGE, "DAG %d has %lld tasks (max 2^21)", b, (long long)n);
        if (m >= ((int64_t)1 << 31)) return set_error(INSP_E_RANGE, "DAG %d has too many edges", b);
        if (n == 0 && m != 0) return set_error(INSP_E_INVAL, "DAG %d has edges but no tasks", b);
        max_n = std::max<int32_t>(max_n, (int32_t)n);
    }
    const int64_t N = task_off[n_dags], M = edge_off[n_dags];
    if (N > 0 && (!row_ptr || (M > 0 && !col))) return set_error(INSP_E_INVAL, "null row_ptr/col");
    hipStream_t st = (hipStream_t)stream_;

    std::unique_ptr<insp_dag> d(new insp_dag());
    static std::atomic<uint64_t> next_serial{1};
    d->serial = next_serial.fetch_add(1);
    d->B = n_dags;
    INSP_HIP(hipGetDevice(&d->device));
    d->N = N;
    d->toff.assign(task_off, task_off + n_dags + 1);
    int rc;
    const int nbw = 1 + (n_dags + 31) / 32;
    DevBuf eoff_in, tmp, outdeg, excl, err, nwide, wide, backward, eoff_c;
    if ((rc = d->d_toff.alloc(sizeof(int64_t) * (n_dags + 1))) || (rc = eoff_in.alloc(sizeof(int64_t) * (n_dags + 1))) ||
        (rc = tmp.alloc(sizeof(int32_t) * M)) || (rc = outdeg.alloc(sizeof(int32_t) * N)) ||
        (rc = excl.alloc(sizeof(int64_t) * (N + 1))) || (rc = err.alloc(sizeof(int32_t))) ||
        (rc = nwide.alloc(sizeof(int32_t))) || (rc = wide.alloc(sizeof(int64_t) * N)) ||
        (rc = backward.alloc(sizeof(int32_t) * nbw)) || (rc = eoff_c.alloc(sizeof(int64_t) * (n_dags + 1))))
        return rc;
    INSP_HIP(hipMemcpyAsync(d->d_toff.p, task_off, sizeof(int64_t) * (n_dags + 1), hipMemcpyHostToDevice, st));
    INSP_HIP(hipMemcpyAsync(eoff_in.p, edge_off, sizeof(int64_t) * (n_dags + 1), hipMemcpyHostToDevice, st));
    INSP_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), st));
    INSP_HIP(hipMemsetAsync(nwide.p, 0, sizeof(int32_t), st));
    INSP_HIP(hipMemsetAsync(backward.p, 0, sizeof(int32_t) * nbw, st));

    // Sort and deduplicate every row where it lies; validate the CSR.
    RowArgs ra;
    ra.B = n_dags;
    ra.toff = d->d_toff.as<int64_t>();
    ra.eoff = eoff_in.as<int64_t>();
    ra.rp = row_ptr;
    ra.col = col;
    ra.tmp = tmp.as<int32_t>();
    ra.outdeg = outdeg.as<int32_t>();
    ra.err = err.as<int32_t>();
    ra.nwide = nwide.as<int32_t>();
    ra.wide = wide.as<int64_t>();
    ra.bits = nullptr;
    ra.bit_words = 0;
    if (N > 0) hipLaunchKernelGGL(k_rows, dim3(grid_for(N, 256)), dim3(256), 0, st, ra);
    INSP_HIP(hipGetLastError());
    int32_t h_err = 0, h_wide = 0;
    INSP_HIP(hipMemcpyAsync(&h_err, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    INSP_HIP(hipMemcpyAsync(&h_wide, nwide.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    if (!(h_err & ERR_ROWPTR) && h_wide > 0) {
        // the listed rows: a wave each up to kWaveRow entries, a work-group
        // each up to kBlockRow, bitmaps above (each kernel skips the others' rows)
        hipLaunchKernelGGL((k_rows_lds<64, kWaveRow, kSmallRow>), dim3((unsigned)h_wide), dim3(64), 0, st, ra);
        hipLaunchKernelGGL((k_rows_lds<256, kBlockRow, kWaveRow>), dim3((unsigned)h_wide), dim3(256), 0, st, ra);
        DevBuf bits;
        ra.bit_words = (max_n + 31) / 32;
        if ((rc = bits.alloc(sizeof(uint32_t) * ra.bit_words * kHugeSlots))) return rc;
        ra.bits = bits.as<uint32_t>();
        hipLaunchKernelGGL(k_rows_huge, dim3((unsigned)std::min(h_wide, kHugeSlots)), dim3(256), 0, st, ra, h_wide);
        INSP_HIP(hipGetLastError());
        INSP_HIP(hipMemcpyAsync(&h_err, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        INSP_HIP(hipStreamSynchronize(st));  // before the bitmaps are released
    }
    if (h_err & ERR_ROWPTR) return set_error(INSP_E_INVAL, "row_ptr is not a valid CSR row pointer");
    if (h_err & ERR_COL) return set_error(INSP_E_INVAL, "successor id out of range");
    if (h_err & ERR_SELF) return set_error(INSP_E_INVAL, "self loop");

    // Place the canonical rows: an exclusive scan of their lengths gives the
    // global row starts; DAG b's local row pointers subtract its first edge.
    if ((rc = exclusive_scan(outdeg.as<int32_t>(), N, excl.as<int64_t>(), st))) return rc;
    hipLaunchKernelGGL(k_dag_edges, dim3(grid_for(n_dags + 1, 256)), dim3(256), 0, st, n_dags,
                       d->d_toff.as<int64_t>(), excl.as<int64_t>(), eoff_c.as<int64_t>());
    INSP_HIP(hipGetLastError());
    d->eoff.resize(n_dags + 1);
    INSP_HIP(hipMemcpyAsync(d->eoff.data(), eoff_c.p, sizeof(int64_t) * (n_dags + 1), hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    const int64_t Mc = d->eoff[n_dags];
    d->M = Mc;
    if ((rc = d->col.alloc(sizeof(int32_t) * Mc)) || (rc = d->rp.alloc(sizeof(int32_t) * (N + n_dags))) ||
        (rc = d->word0.alloc(sizeof(uint64_t) * N)) || (rc = d->d_eoff.alloc(sizeof(int64_t) * (n_dags + 1))))
        return rc;
    INSP_HIP(hipMemcpyAsync(d->d_eoff.p, eoff_c.p, sizeof(int64_t) * (n_dags + 1), hipMemcpyDeviceToDevice, st));
    INSP_HIP(hipMemsetAsync(d->rp.p, 0, sizeof(int32_t) * (N + n_dags), st));  // empty DAGs: rp = {0}
    INSP_HIP(hipMemsetAsync(d->word0.p, 0, sizeof(uint64_t) * std::max<int64_t>(N, 1), st));
    PlaceArgs pa;
    pa.B = n_dags;
    pa.toff = d->d_toff.as<int64_t>();
    pa.eoff = eoff_in.as<int64_t>();
    pa.rp = row_ptr;
    pa.tmp = tmp.as<int32_t>();
    pa.outdeg = outdeg.as<int32_t>();
    pa.excl = excl.as<int64_t>();
    pa.col_out = d->col.as<int32_t>();
    pa.rp_out = d->rp.as<int32_t>();
    pa.word0 = d->word0.as<unsigned long long>();
    pa.backward = backward.as<int32_t>();
    if (N > 0) hipLaunchKernelGGL(k_place, dim3(grid_for(N, 256)), dim3(256), 0, st, pa);
    if (h_wide > 0)
        hipLaunchKernelGGL(k_place_wide, dim3((unsigned)h_wide), dim3(64), 0, st, pa, (const int64_t *)wide.as<int64_t>());
    INSP_HIP(hipGetLastError());

    // Cycle check: with every edge pointing to a higher id the id order is a
    // topological order; otherwise run Kahn's traversal on the DAGs concerned.
    std::vector<int32_t> h_back(nbw);
    INSP_HIP(hipMemcpyAsync(h_back.data(), backward.p, sizeof(int32_t) * nbw, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    if (h_back[0]) {
        std::vector<int32_t> todo;
        for (int32_t b = 0; b < n_dags; b++)
            if (h_back[1 + (b >> 5)] >> (b & 31) & 1) todo.push_back(b);
        DevBuf d_todo, indeg, queue, visited;
        if ((rc = d_todo.alloc(sizeof(int32_t) * todo.size())) || (rc = indeg.alloc(sizeof(int32_t) * N)) ||
            (rc = queue.alloc(sizeof(int32_t) * N)) || (rc = visited.alloc(sizeof(int32_t) * todo.size())))
            return rc;
        INSP_HIP(hipMemcpyAsync(d_todo.p, todo.data(), sizeof(int32_t) * todo.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_kahn, dim3((unsigned)todo.size()), dim3(256), 0, st, d_todo.as<int32_t>(),
                           d->d_toff.as<int64_t>(), d->d_eoff.as<int64_t>(), d->rp.as<int32_t>(), d->col.as<int32_t>(),
                           d->word0.as<unsigned long long>(), indeg.as<int32_t>(), queue.as<int32_t>(),
                           visited.as<int32_t>());
        INSP_HIP(hipGetLastError());
        std::vector<int32_t> h_vis(todo.size());
        INSP_HIP(hipMemcpyAsync(h_vis.data(), visited.p, sizeof(int32_t) * todo.size(), hipMemcpyDeviceToHost, st));
        INSP_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < todo.size(); i++) {
            int32_t b = todo[i];
            if (h_vis[i] != task_off[b + 1] - task_off[b])
                return set_error(INSP_E_CYCLE, "DAG %d has a dependency cycle", b);
        }
    }
    if ((rc = alloc_status(d.get())) || (rc = build_hubs(d.get(), st))) return rc;
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
