// Small device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace useries {

// x (any image) -> uint32 fraction of the cell edge, rounded to nearest;
// 2^32 wraps to 0.
__device__ __forceinline__ uint32_t to_fixed(double x, double inv_L) {
    double f = x * inv_L;
    f -= floor(f);
    const double t = f * 4294967296.0 + 0.5;
    return (uint32_t)(uint64_t)t;
}

// index of the slab [k/n, (k+1)/n) of the edge that holds fraction u
__device__ __forceinline__ int cell_coord(uint32_t u, int n) {
    return (int)(((uint64_t)u * (uint64_t)n) >> 32);
}

// fraction u on a grid of n points: integer index and fractional offset in [0,1)
__device__ __forceinline__ void grid_coord(uint32_t u, int n, int* gi, float* f) {
    const uint64_t p = (uint64_t)u * (uint64_t)n;
    *gi = (int)(p >> 32);
    *f = (float)(uint32_t)(p & 0xffffffffull) * 2.3283064365386963e-10f;   // 2^-32
}

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// v mod n for -n <= v < 2n (no integer division)
__device__ __forceinline__ int wrap1(int v, int n) {
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

// floor(v / d) for v >= 0, d >= 1 and v < 2^20, from a float reciprocal
// within 1 ulp (the hardware reciprocal, or a division): (v + 1/2)/d lies at
// least 1/(2d) from an integer, and the float error of the product, below
// (v/d) 2^-21, is smaller than that
__device__ __forceinline__ int small_div(int v, float inv_d) {
    return (int)(((float)v + 0.5f) * inv_d);
}

// number of set bits of m in the lanes below this one
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Order LDS traffic between the lanes of one wavefront (the LDS of a
// wavefront-private region needs no block barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work item of block i of a launch of xcd_blocks(nb) blocks.  Consecutive
// blocks go to the 8 XCDs in turn, so this gives each XCD a contiguous range
// of items: neighbouring items (nearby clusters or bricks) then share that
// XCD's L2.  Items >= nb are padding.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_blocks(int nb) { return (nb + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_item(int i, int nb) {
    return (i % kXcds) * (xcd_blocks(nb) / kXcds) + i / kXcds;
}

// DPP lane moves within 16-lane rows (no LDS round trip).  CTRL: 0xB1 and
// 0x4E swap neighbours and pairs within quads (quad_perm [1,0,3,2], [2,3,0,1]),
// 0x141 mirrors each half row (lane i <- 7 - i), 0x140 mirrors the row
// (i <- 15 - i), 0x128 rotates the row by 8 (i <- i xor 8).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                  CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// inclusive prefix sum over the 64 lanes by DPP: a doubling scan within each
// 16-lane row (shifts 1, 2, 4, 8; lanes shifted in from outside the row add
// 0), then the last lane of row 0 added to row 1 and of row 2 to row 3
// (row_bcast:15), then lane 31 added to rows 2 and 3 (row_bcast:31)
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_add_in(int v) {
    return v + __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}
__device__ __forceinline__ int wave_incl_scan(int v) {
    v = dpp_add_in<0x111, 0xF>(v);   // row_shr:1
    v = dpp_add_in<0x112, 0xF>(v);   // row_shr:2
    v = dpp_add_in<0x114, 0xF>(v);   // row_shr:4
    v = dpp_add_in<0x118, 0xF>(v);   // row_shr:8
    v = dpp_add_in<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    return dpp_add_in<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
}

// sum over each group of 8 lanes (lanes 8g .. 8g + 7), every lane of the group
// receiving it, in a fixed order
__device__ __forceinline__ float sum8(float v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    return v + dpp_move<0x141>(v);
}

// sum over each 16-lane row, every lane of the row receiving it
__device__ __forceinline__ float row_sum16(float v) {
    v = sum8(v);
    return v + dpp_move<0x140>(v);
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = dpp_move<CTRL>((int)(uint32_t)u), hi = dpp_move<CTRL>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double read_lane(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// sum over the 64 lanes of a wavefront (all lanes active), in a fixed order:
// each 16-lane row by DPP moves, then the four row sums in order; every lane
// gets the result
__device__ __forceinline__ double wave_sum_d(double v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

}  // namespace useries

namespace useries {

// Batched launches: index i of the batch entry whose work-item range
// [off[i], off[i + 1]) holds item w (off is non-decreasing, off[0] = 0).
__device__ __forceinline__ int batch_find(const int* __restrict__ off, int nbox, int w) {
    int lo = 0, hi = nbox;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= w) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace useries

namespace useries {

// Grid-stride loop of a batched launch over the work items of kernel k:
// f(i, item) runs the one-box body for batch entry i and its local item.
// The block barrier between items lets a body reuse its LDS.
template <class Table, class F>
__device__ __forceinline__ void batch_for(const Table* __restrict__ tab, int k, F&& f) {
    const int nbox = tab->nbox;
    const int* off = tab->off[k];
    const int total = off[nbox];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int i = batch_find(off, nbox, w);
        f(i, w - off[i]);
        __syncthreads();
    }
}

}  // namespace useries
