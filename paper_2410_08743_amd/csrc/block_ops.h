// block_ops.h -- wavefront (64 lanes) and block reductions and scans used by
// the gfx950 kernels.  Lane exchange goes through __shfl_* (ds_bpermute /
// DPP); block-level steps go through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsp {

constexpr int kWave = 64;

// Wave-wide vote on a lane predicate, straight from the compare's lane mask
// (no round trip of the predicate through a vector register).
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Inclusive scan across the wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive scan over a block of NT threads; returns the block total in *total.
// `scratch` must hold NT / 64 elements of T.
template <typename T, int NT>
__device__ __forceinline__ T block_exclusive_scan(T v, T *scratch, T *total) {
    static_assert(NT % kWave == 0, "block must be whole wavefronts");
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) scratch[w] = inc;
    __syncthreads();
    T wave_off = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
        const T s = scratch[k];
        if (k < w) wave_off += s;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return wave_off + inc - v;
}

template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T *scratch) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    T sum = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) sum += scratch[k];
    __syncthreads();
    return sum;
}

}  // namespace gsp

namespace gsp {

// DPP controls (gfx9 encoding) for row-local (16-lane) butterflies.
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

// x + x[permuted lane]; every permutation used here reads a lane inside the
// row, so bound_ctrl (zero for out-of-range sources) never applies and lets
// the compiler fold the move into the add (v_add_f32_dpp).
template <int CTRL>
__device__ __forceinline__ float dpp_add(float x) {
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Sum over the 16 lanes of each row; every lane of the row receives it.
__device__ __forceinline__ float row_sum16(float x) {
    x = dpp_add<kDppQuadXor1>(x);
    x = dpp_add<kDppQuadXor2>(x);
    x = dpp_add<kDppRowHalfMirror>(x);
    return dpp_add<kDppRowMirror>(x);
}

// (a, b) -> lanes 0-31: a[l] + a[l + 32]; lanes 32-63: b[l - 32] + b[l]
// (gfx950 v_permlane32_swap exchanges rows 2-3 of a with rows 0-1 of b).
__device__ __forceinline__ float pair_sum32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// (a, b) -> rows [a0 + a1, b0 + b1, a2 + a3, b2 + b3] (rows of 16 lanes;
// v_permlane16_swap exchanges the odd rows of a with the even rows of b).
__device__ __forceinline__ float pair_sum16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The first two levels of a reduce-scatter of nine values over the wave: a
// 32-lane and a 16-lane swap halve the data at each step, leaving each value
// as 16 partial sums (of the four lanes l, l + 16, l + 32, l + 48 of column
// l) in one 16-lane row:
//   a rows 0..3 = v0, v2, v1, v3;  b rows 0..3 = v4, v6, v5, v7;  c row 0 = v8.
__device__ __forceinline__ void wave_sum9_rows(const float v[9], float &a, float &b, float &c) {
    const float w0 = pair_sum32(v[0], v[1]);
    const float w1 = pair_sum32(v[2], v[3]);
    const float w2 = pair_sum32(v[4], v[5]);
    const float w3 = pair_sum32(v[6], v[7]);
    const float w4 = pair_sum32(v[8], v[8]);
    a = pair_sum16(w0, w1);
    b = pair_sum16(w2, w3);
    c = pair_sum16(w4, w4);
}

// The same for eight values: a rows 0..3 = v0, v2, v1, v3; b rows 0..3 =
// v4, v6, v5, v7.
__device__ __forceinline__ void wave_sum8_rows(const float v[8], float &a, float &b) {
    a = pair_sum16(pair_sum32(v[0], v[1]), pair_sum32(v[2], v[3]));
    b = pair_sum16(pair_sum32(v[4], v[5]), pair_sum32(v[6], v[7]));
}

// Row of the 16-lane row partials that hold value k (register k >> 2 for
// k < 8, register 2 for k = 8).
__host__ __device__ constexpr int sum9_row(int k) {
    return k == 8 ? 0 : ((k & 3) == 1 ? 2 : ((k & 3) == 2 ? 1 : (k & 3)));
}

}  // namespace gsp
