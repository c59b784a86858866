// Exclusive prefix sums over device arrays (row pointers of the canonical
// CSR and of the predecessor lists): reduce per tile, scan the tile sums
// (recursively), then scan each tile from its offset.  Tiles of 2048 values
// are staged through LDS so that global reads and writes stay coalesced
// while each thread scans 8 consecutive values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = kScanThreads * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the block total
// through `total`.  `part` holds one slot per wave.
__device__ __forceinline__ int64_t block_exclusive(int64_t x, int64_t *part, int64_t &total) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    int64_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) part[wv] = inc;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; w++) {
        if (w < wv) before += part[w];
        tot += part[w];
    }
    __syncthreads();  // part may be reused by the caller
    total = tot;
    return before + inc - x;
}

// Stage tile `t` of `in` (converted to int64) into LDS.
template <typename T>
__device__ __forceinline__ void stage_tile(const T *in, int64_t n, int64_t t, int64_t *buf) {
    const int64_t base = t * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        const int64_t i = base + j * kScanThreads + threadIdx.x;
        buf[j * kScanThreads + threadIdx.x] = i < n ? (int64_t)in[i] : 0;
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const T *in, int64_t n, int64_t *sums) {
    __shared__ int64_t buf[kScanTile];
    __shared__ int64_t part[kScanThreads / kWave];
    stage_tile(in, n, blockIdx.x, buf);
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) s += buf[threadIdx.x * kScanItems + j];
    int64_t total;
    (void)block_exclusive(s, part, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// out[i] = offs[tile] + sum of in[tile start .. i); with `last` also
// out[n] = the grand total.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const T *in, int64_t n, const int64_t *offs,
                                                            int64_t *out, int last) {
    __shared__ int64_t buf[kScanTile];
    __shared__ int64_t part[kScanThreads / kWave];
    stage_tile(in, n, blockIdx.x, buf);
    int64_t v[kScanItems], s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        v[j] = buf[threadIdx.x * kScanItems + j];
        s += v[j];
    }
    int64_t total;
    int64_t run = block_exclusive(s, part, total) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        buf[threadIdx.x * kScanItems + j] = run;
        run += v[j];
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        const int64_t i = base + j * kScanThreads + threadIdx.x;
        if (i < n) out[i] = buf[j * kScanThreads + threadIdx.x];
    }
    if (last && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) out[n] = run;
}

template <typename T>
static int scan_rec(const T *in, int64_t n, int64_t *out, int last, hipStream_t st) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles <= 1) {
        hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kScanThreads), 0, st, in, n, (const int64_t *)nullptr, out,
                           last);
        INSP_HIP(hipGetLastError());
        return INSP_OK;
    }
    DevBuf sums, offs;
    int rc;
    if ((rc = sums.alloc(sizeof(int64_t) * tiles)) || (rc = offs.alloc(sizeof(int64_t) * (tiles + 1)))) return rc;
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, n, sums.as<int64_t>());
    INSP_HIP(hipGetLastError());
    if ((rc = scan_rec<int64_t>(sums.as<int64_t>(), tiles, offs.as<int64_t>(), 0, st))) return rc;
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, n,
                       (const int64_t *)offs.as<int64_t>(), out, last);
    INSP_HIP(hipGetLastError());
    // the temporaries are released on return: wait for the kernels using them
    INSP_HIP(hipStreamSynchronize(st));
    return INSP_OK;
}

int exclusive_scan(const int32_t *in, int64_t n, int64_t *out, hipStream_t st) {
    if (n <= 0) {
        INSP_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), st));
        return INSP_OK;
    }
    return scan_rec<int32_t>(in, n, out, 1, st);
}

int exclusive_scan(const int64_t *in, int64_t n, int64_t *out, hipStream_t st) {
    if (n <= 0) {
        INSP_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), st));
        return INSP_OK;
    }
    return scan_rec<int64_t>(in, n, out, 1, st);
}

}  // namespace insp
