// Device helpers shared by the gfx950 kernels: wave64 reductions built on
// DPP lane moves, ballot-based compaction, and work-group-scope atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace insp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int32_t uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int32_t read_lane(int32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ uint64_t read_lane64(uint64_t x, int l) {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// DPP move of a 32-bit value; lanes whose source is out of row or masked
// keep their own value, which is harmless for idempotent max/min.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
    uint32_t lo = dpp32<CTRL, ROW_MASK>((uint32_t)x);
    uint32_t hi = dpp32<CTRL, ROW_MASK>((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Full-wave max / min of a 64-bit key (all 64 lanes must be active).  Quad
// swaps, half-row and row mirrors reduce each 16-lane row; row_bcast15 and
// row_bcast31 fold the rows into lane 63, which is then broadcast.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
    uint64_t y;
    y = dpp64<0xB1>(x); x = x > y ? x : y;          // quad_perm [1,0,3,2]
    y = dpp64<0x4E>(x); x = x > y ? x : y;          // quad_perm [2,3,0,1]
    y = dpp64<0x141>(x); x = x > y ? x : y;         // row_half_mirror
    y = dpp64<0x140>(x); x = x > y ? x : y;         // row_mirror
    y = dpp64<0x142, 0xA>(x); x = x > y ? x : y;    // row_bcast15
    y = dpp64<0x143, 0xC>(x); x = x > y ? x : y;    // row_bcast31
    return read_lane64(x, 63);
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
    uint64_t y;
    y = dpp64<0xB1>(x); x = x < y ? x : y;
    y = dpp64<0x4E>(x); x = x < y ? x : y;
    y = dpp64<0x141>(x); x = x < y ? x : y;
    y = dpp64<0x140>(x); x = x < y ? x : y;
    y = dpp64<0x142, 0xA>(x); x = x < y ? x : y;
    y = dpp64<0x143, 0xC>(x); x = x < y ? x : y;
    return read_lane64(x, 63);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    uint32_t y;
    y = dpp32<0xB1>(x); x = x > y ? x : y;
    y = dpp32<0x4E>(x); x = x > y ? x : y;
    y = dpp32<0x141>(x); x = x > y ? x : y;
    y = dpp32<0x140>(x); x = x > y ? x : y;
    y = dpp32<0x142, 0xA>(x); x = x > y ? x : y;
    y = dpp32<0x143, 0xC>(x); x = x > y ? x : y;
    return __builtin_amdgcn_readlane(x, 63);
}
// DPP move whose masked-off or out-of-row lanes read `ident`: with the
// operation's identity there the compiler folds the move into the max/min
// itself (one v_max_u32_dpp per step instead of a move, a compare and a
// select).  Only lane 63's result is used, which every step keeps exact.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_id(uint32_t x, uint32_t ident) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)x, CTRL, ROW_MASK, 0xF, false);
}
__device__ __forceinline__ uint32_t wave_max_u32f(uint32_t x) {
    x = max(x, dpp_id<0xB1>(x, 0u));
    x = max(x, dpp_id<0x4E>(x, 0u));
    x = max(x, dpp_id<0x141>(x, 0u));
    x = max(x, dpp_id<0x140>(x, 0u));
    x = max(x, dpp_id<0x142, 0xA>(x, 0u));
    x = max(x, dpp_id<0x143, 0xC>(x, 0u));
    return __builtin_amdgcn_readlane(x, 63);
}
__device__ __forceinline__ uint32_t wave_min_u32f(uint32_t x) {
    x = min(x, dpp_id<0xB1>(x, ~0u));
    x = min(x, dpp_id<0x4E>(x, ~0u));
    x = min(x, dpp_id<0x141>(x, ~0u));
    x = min(x, dpp_id<0x140>(x, ~0u));
    x = min(x, dpp_id<0x142, 0xA>(x, ~0u));
    x = min(x, dpp_id<0x143, 0xC>(x, ~0u));
    return __builtin_amdgcn_readlane(x, 63);
}
// 64-bit max as two 32-bit passes: the high words, then the low words of
// the lanes that hold the maximal high word.
__device__ __forceinline__ uint64_t wave_max_u64f(uint64_t x) {
    const uint32_t hi = wave_max_u32f((uint32_t)(x >> 32));
    const uint32_t lo = wave_max_u32f((uint32_t)(x >> 32) == hi ? (uint32_t)x : 0u);
    return (uint64_t)hi << 32 | lo;
}
__device__ __forceinline__ uint64_t wave_min_u64f(uint64_t x) {
    const uint32_t hi = wave_min_u32f((uint32_t)(x >> 32));
    const uint32_t lo = wave_min_u32f((uint32_t)(x >> 32) == hi ? (uint32_t)x : ~0u);
    return (uint64_t)hi << 32 | lo;
}

// Wave sum of a 64-bit value via row shifts (non-idempotent, so the DPP
// moves use bound_ctrl and a zero identity).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp32_zero(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, true);
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
    // shuffle-xor tree; sums are rare (once per DAG), so clarity over speed
    for (int off = 32; off >= 1; off >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)x, off, 64), hi = __shfl_xor((uint32_t)(x >> 32), off, 64);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Inclusive prefix sum over the wave (Hillis-Steele within each 16-lane row
// by row shifts, then the row totals carried by row broadcasts).  All 64
// lanes must be active.
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
    uint32_t v = (uint32_t)x;
    v += dpp32_zero<0x111>(v);        // row_shr:1
    v += dpp32_zero<0x112>(v);        // row_shr:2
    v += dpp32_zero<0x114>(v);        // row_shr:4
    v += dpp32_zero<0x118>(v);        // row_shr:8
    v += dpp32_zero<0x142, 0xA>(v);   // row_bcast15 into rows 1 and 3
    v += dpp32_zero<0x143, 0xC>(v);   // row_bcast31 into rows 2 and 3
    return (int32_t)v;
}

// Work-group-scope atomics: every per-DAG array is touched by exactly one
// work-group during a simulation, so L2-resident atomics at work-group scope
// are sufficient and avoid device-scope coherence traffic.
template <typename T>
__device__ __forceinline__ T wg_fetch_add(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T wg_fetch_max(T *p, T v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T wg_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wg_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

template <typename T>
__device__ __forceinline__ T dev_fetch_add(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace insp
