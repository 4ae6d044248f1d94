// Routing of a shared scan's hits to the requests of a serving batch.
//
// One thread per hit: it counts the requests that take the hit, the wave
// reserves room for all its copies with one atomic, and each thread writes
// its copies with the request's own pair slot.
#include <hip/hip_runtime.h>

#include "ah.h"
#include "ah_dev.h"
#include "ah_internal.h"

__global__ void __launch_bounds__(256) ah_route_kernel(const uint32_t *hits, const uint64_t *d_n_hits, uint64_t hit_cap,
                                                      uint32_t n_seqs, const uint64_t *seq_req, const uint16_t *vpair,
                                                      const uint8_t *kmax, uint32_t n_req, uint32_t n_pool,
                                                      uint32_t *out, uint64_t out_cap, uint64_t *n_out) {
    const uint64_t n = *d_n_hits < hit_cap ? *d_n_hits : hit_cap;
    const uint64_t req_bits = n_req >= 64 ? ~0ull : ((1ull << n_req) - 1);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of iterations (the wave-wide
    // reservation below needs all 64 lanes)
    const uint64_t first = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t wave0 = first - ah_lane();
    for (uint64_t base = wave0; base < n; base += stride) {
        const uint64_t i = base + ah_lane();
        uint32_t w0 = 0, w1 = 0, w2 = 0;
        uint64_t take = 0;
        if (i < n) {
            w0 = hits[3 * i];
            w1 = hits[3 * i + 1];
            w2 = hits[3 * i + 2];
            const uint32_t seq = w0, q = w2 & 0xFFFFu, mm = w2 >> 24;
            uint64_t m = (seq < n_seqs && q < n_pool) ? (seq_req[seq] & req_bits) : 0;
            while (m) {
                const uint32_t r = (uint32_t)__builtin_ctzll(m);
                m &= m - 1;
                if (vpair[(uint64_t)r * n_pool + q] != 0xFFFFu && mm <= kmax[r]) take |= 1ull << r;
            }
        }
        const uint64_t cnt = (uint64_t)__popcll(take);
        const uint64_t incl = ah_wave_incl_sum<uint64_t>(cnt);
        const uint64_t total = __shfl(incl, 63, 64);
        uint64_t at = 0;
        if (ah_lane() == 63 && total) at = atomicAdd((unsigned long long *)n_out, (unsigned long long)total);
        at = __shfl(at, 63, 64) + incl - cnt;
        const uint32_t q = w2 & 0xFFFFu;
        while (take) {
            const uint32_t r = (uint32_t)__builtin_ctzll(take);
            take &= take - 1;
            if (at < out_cap) {
                out[3 * at] = w0;
                out[3 * at + 1] = w1;
                out[3 * at + 2] = (w2 & 0xFFFF0000u) | vpair[(uint64_t)r * n_pool + q];
            }
            at++;
        }
    }
}

extern "C" ah_status ah_route_hits(const ah_hit *d_hits, const uint64_t *d_n_hits, uint64_t hit_cap, uint32_t n_seqs,
                                   const uint64_t *d_seq_req, const uint16_t *d_vpair, const uint8_t *d_kmax,
                                   uint32_t n_req, uint32_t n_pool, ah_hit *d_out, uint64_t out_cap,
                                   uint64_t *d_n_out, void *stream) {
    if (!d_n_hits || !d_n_out || (hit_cap && !d_hits) || (out_cap && !d_out)) return AH_E_ARG;
    if (n_req > 64 || n_pool > 0xFFFFu) return AH_E_LIMIT;
    if (n_req && (!d_seq_req || !d_vpair || !d_kmax)) return AH_E_ARG;
    hipStream_t s = ah_stream(stream);
    ah_fill<uint64_t>(d_n_out, 0ull, 1, s);
    if (!hit_cap || !n_req) return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
    uint64_t wgs = (hit_cap + 255) / 256;
    if (wgs > 4096) wgs = 4096;
    hipLaunchKernelGGL(ah_route_kernel, dim3((unsigned)wgs), dim3(256), 0, s, (const uint32_t *)d_hits, d_n_hits,
                       hit_cap, n_seqs, d_seq_req, d_vpair, d_kmax, n_req, n_pool, (uint32_t *)d_out, out_cap, d_n_out);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
