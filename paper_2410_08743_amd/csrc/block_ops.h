// block_ops.h -- wavefront (64 lanes) and block reductions and scans used by
// the gfx950 kernels.  Lane exchange goes through __shfl_* (ds_bpermute /
// DPP); block-level steps go through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsp {

constexpr int kWave = 64;

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
