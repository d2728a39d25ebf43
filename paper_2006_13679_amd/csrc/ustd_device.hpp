// ustd_device.hpp -- device-side helpers for the gfx950 kernels (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ustd {

constexpr int kWave = 64;

// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of two 32x32->64 multiplies whose
// halves are mixed with the odd counter words and the key, the key advancing by the
// Weyl increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // full 32x32 -> 64-bit products: one v_mad_u64_u32 each instead of a low and a high multiply
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    }
    return c;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

// inclusive prefix sum across the 64 lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (l >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Block-wide inclusive scan of one int per thread; *total receives the block sum.
// `sh` must hold at least blockDim.x / 64 + 1 ints.  Contains two barriers.
__device__ __forceinline__ int block_incl_scan(int v, int *total, int *sh) {
    const int l = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    int incl = wave_incl_scan(v);
    if (l == kWave - 1) sh[w] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        const int s = sh[i];
        off += (i < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return incl + off;
}

// Block-wide sum of doubles in a fixed order (deterministic for a fixed blockDim).
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int l = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    v = wave_sum(v);
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += sh[i];
    __syncthreads();
    return s;
}

// Block-wide sum of one value per thread in a fixed order (deterministic for a fixed blockDim);
// `sh` holds at least blockDim.x / 64 values.  Contains two barriers.
template <typename T>
__device__ __forceinline__ T block_sum_t(T v, T *sh) {
    const int l = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    v = wave_sum(v);
    if (l == 0) sh[w] = v;
    __syncthreads();
    T s = (T)0;
    for (int i = 0; i < nw; ++i) s += sh[i];
    __syncthreads();
    return s;
}

}  // namespace ustd
