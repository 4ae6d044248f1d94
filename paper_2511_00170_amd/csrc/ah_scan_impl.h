// Device-wide scans used by the pair, extract, pack and scan stages.
#pragma once

#include "ah_internal.h"

template <typename T>
__device__ __forceinline__ T ah_block_excl_sum(T v, T *lds_waves, T &total) {
    T incl = ah_wave_incl_sum(v);
    const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 63) lds_waves[w] = incl;
    __syncthreads();
    T before = 0, tot = 0;
    for (uint32_t i = 0; i < nw; i++) {
        T x = lds_waves[i];
        if (i < w) before += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return before + incl - v;
}

__device__ __forceinline__ uint64_t ah_scan_count(const uint64_t *d_n, uint64_t cap) {
    uint64_t n = *d_n;
    return n < cap ? n : cap;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) ah_scan_reduce_kernel(const TI *in, const uint64_t *d_n, uint64_t cap,
                                                             TO *partials) {
    __shared__ TO lds[4];
    const uint64_t n = ah_scan_count(d_n, cap);
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = blockIdx.x * chunk;
    const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    TO s = 0;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) s += (TO)in[i];
    TO tot;
    ah_block_excl_sum<TO>(s, lds, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <typename TO>
__global__ void __launch_bounds__(1024) ah_scan_partials_kernel(TO *partials, uint32_t np, TO *d_total) {
    __shared__ TO lds[16];
    TO v = threadIdx.x < np ? partials[threadIdx.x] : 0;
    TO tot;
    TO ex = ah_block_excl_sum<TO>(v, lds, tot);
    if (threadIdx.x < np) partials[threadIdx.x] = ex;
    if (threadIdx.x == 0 && d_total) *d_total = tot;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) ah_scan_down_kernel(const TI *in, TO *out, const uint64_t *d_n, uint64_t cap,
                                                           const TO *partials) {
    __shared__ TO lds[4];
    const uint64_t n = ah_scan_count(d_n, cap);
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = blockIdx.x * chunk;
    const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    TO carry = partials[blockIdx.x];
    for (uint64_t t0 = b0; t0 < b1; t0 += 4 * blockDim.x) {
        TO v[4];
        TO s = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            uint64_t i = t0 + 4 * threadIdx.x + j;
            v[j] = i < b1 ? (TO)in[i] : (TO)0;
            s += v[j];
        }
        TO tot;
        TO ex = ah_block_excl_sum<TO>(s, lds, tot) + carry;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            uint64_t i = t0 + 4 * threadIdx.x + j;
            if (i < b1) out[i] = ex;
            ex += v[j];
        }
        carry += tot;
    }
}

template <typename TI, typename TO>
ah_status ah_exclusive_scan(const TI *d_in, TO *d_out, const uint64_t *d_n, uint64_t cap, TO *d_total,
                            TO *d_partials, hipStream_t s) {
    hipLaunchKernelGGL((ah_scan_reduce_kernel<TI, TO>), dim3(AH_SCAN_BLOCKS), dim3(256), 0, s, d_in, d_n, cap,
                       d_partials);
    hipLaunchKernelGGL((ah_scan_partials_kernel<TO>), dim3(1), dim3(1024), 0, s, d_partials,
                       (uint32_t)AH_SCAN_BLOCKS, d_total);
    hipLaunchKernelGGL((ah_scan_down_kernel<TI, TO>), dim3(AH_SCAN_BLOCKS), dim3(256), 0, s, d_in, d_out, d_n, cap,
                       (const TO *)d_partials);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
