// Amplicon calling (Supplementary, "Amplicon calling and orientation").
//
// Sites are encoded as 64-bit keys whose integer order is the site order
// (sequence, pair, start, end, plus before minus, forward before reverse):
//   key = seq | pair | start | (L - 1) | sense | primer   (most to least significant)
// with end = start + L.  The keys are sorted with an LSD radix sort (8-bit
// digits, stable wave-level ranking by ballot), after which a plus site pairs
// with exactly the minus sites that follow it up to the next plus site.  So
// every minus site t has at most one partner -- the nearest plus site before
// it in the same (sequence, pair) -- and the amplicons are found by one flat
// pass over the sorted keys, compacted with a prefix sum in key order.
#include "ah_internal.h"
#include "ah_scan_impl.h"

#define RS_G 1024  // wave chunks per radix pass (256 workgroups x 4 waves)

struct KeyLayout {
    int pos_bits, pair_bits, seq_bits;
    uint64_t pos_mask, pair_mask;
};

__device__ __forceinline__ uint32_t key_primer(uint64_t k) { return (uint32_t)(k & 1); }
__device__ __forceinline__ uint32_t key_sense(uint64_t k) { return (uint32_t)((k >> 1) & 1); }
__device__ __forceinline__ uint32_t key_len(uint64_t k) { return (uint32_t)((k >> 2) & 31) + 1; }

__global__ void ah_pair_keys_kernel(const uint32_t *hits, const uint64_t *d_n, uint64_t cap, const DPair *pairs,
                                    KeyLayout kl, uint64_t *keys) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t seq = hits[3 * i], pos = hits[3 * i + 1], w = hits[3 * i + 2];
        const uint32_t pair = w & 0xFFFFu, kind = (w >> 16) & 0xFFu;
        const uint32_t primer = kind & 1u, sense = (kind >> 1) & 1u;
        const uint32_t L = primer ? pairs[pair].Lr : pairs[pair].Lf;
        keys[i] = ((uint64_t)seq << (kl.pair_bits + kl.pos_bits + 7)) | ((uint64_t)pair << (kl.pos_bits + 7)) |
                  ((uint64_t)pos << 7) | ((uint64_t)(L - 1) << 2) | ((uint64_t)sense << 1) | primer;
    }
}

__global__ void __launch_bounds__(256) ah_rs_hist_kernel(const uint64_t *keys, const uint64_t *d_n, uint64_t cap,
                                                         int shift, uint32_t *hist) {
    __shared__ uint32_t h_all[4][256];
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t *h = h_all[wv];
    for (uint32_t d = lane; d < 256; d += 64) h[d] = 0;
    ah_wave_sync();
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const uint64_t chunk = (n + RS_G - 1) / RS_G;
    const uint64_t c = blockIdx.x * 4 + wv;
    const uint64_t b0 = c * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    for (uint64_t i = b0 + lane; i < b1; i += 64) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    ah_wave_sync();
    for (uint32_t d = lane; d < 256; d += 64) hist[(uint64_t)d * RS_G + c] = h[d];
}

__global__ void __launch_bounds__(256) ah_rs_scatter_kernel(const uint64_t *in, uint64_t *out, const uint64_t *d_n,
                                                            uint64_t cap, int shift, const uint32_t *hoff) {
    __shared__ uint32_t run_all[4][256];
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t *run = run_all[wv];
    const uint64_t c = blockIdx.x * 4 + wv;
    for (uint32_t d = lane; d < 256; d += 64) run[d] = hoff[(uint64_t)d * RS_G + c];
    ah_wave_sync();
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const uint64_t chunk = (n + RS_G - 1) / RS_G;
    const uint64_t b0 = c * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    uint64_t nxt = (b0 + lane < b1) ? in[b0 + lane] : 0;
    for (uint64_t i0 = b0; i0 < b1; i0 += 64) {
        const uint64_t i = i0 + lane;
        const bool valid = i < b1;
        const uint64_t key = nxt;
        nxt = (i + 64 < b1) ? in[i + 64] : 0;  // prefetch the next step
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const bool on = (d >> bit) & 1u;
            const uint64_t b = __ballot(on);
            peers &= on ? b : ~b;
        }
        const uint32_t rank = ah_mbcnt(peers);
        const uint32_t base = valid ? run[d] : 0;
        ah_wave_sync();
        if (valid && rank == 0) run[d] = base + (uint32_t)__popcll(peers);
        ah_wave_sync();
        if (valid) out[base + rank] = key;
    }
}

// For every minus site: find the nearest plus site before it in the same
// (sequence, pair); emit when the length window and orientation allow.
__global__ void ah_pair_flag_kernel(const uint64_t *keys, const uint64_t *d_n, uint64_t cap, const DPair *pairs,
                                    KeyLayout kl, uint32_t orient_mask, uint32_t *flag, uint32_t *partner) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const int seg_shift = 7 + kl.pos_bits;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t kt = keys[i];
        uint32_t f = 0, part = 0;
        if (key_sense(kt) == 1) {
            const uint64_t seg = kt >> seg_shift;
            const uint32_t pair = (uint32_t)(seg & kl.pair_mask);
            const uint32_t tpos = (uint32_t)((kt >> 7) & kl.pos_mask);
            const uint64_t tend = (uint64_t)tpos + key_len(kt);
            const uint32_t mn = pairs[pair].min_len, mx = pairs[pair].max_len;
            const uint64_t lo_start = tend > mx ? tend - mx : 0;
            for (uint64_t j = i; j-- > 0;) {
                const uint64_t kj = keys[j];
                if ((kj >> seg_shift) != seg) break;
                const uint64_t pj = (kj >> 7) & kl.pos_mask;
                if (pj < lo_start) break;  // any partner from here on is too far
                if (key_sense(kj) == 0) {
                    const uint64_t len = tend - pj;
                    const uint32_t lp = key_primer(kj), rp = key_primer(kt);
                    const uint32_t o = (lp == 0 && rp == 1) ? 0u : (lp == 1 && rp == 0) ? 1u : (lp == 0) ? 2u : 3u;
                    if (len >= mn && len <= mx && ((orient_mask >> o) & 1u)) {
                        f = 1;
                        part = (uint32_t)j;
                    }
                    break;
                }
            }
        }
        flag[i] = f;
        partner[i] = part;
    }
}

__global__ void ah_pair_write_kernel(const uint64_t *keys, const uint64_t *d_n, uint64_t cap, KeyLayout kl,
                                     const uint32_t *flag, const uint32_t *partner, const uint32_t *offs,
                                     uint32_t *amps, uint64_t amp_cap) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (!flag[i]) continue;
        const uint64_t o = offs[i];
        if (o >= amp_cap) continue;
        const uint64_t kt = keys[i], ka = keys[partner[i]];
        const uint32_t seq = (uint32_t)(kt >> (7 + kl.pos_bits + kl.pair_bits));
        const uint32_t pair = (uint32_t)((kt >> (7 + kl.pos_bits)) & kl.pair_mask);
        const uint32_t tpos = (uint32_t)((kt >> 7) & kl.pos_mask);
        const uint32_t apos = (uint32_t)((ka >> 7) & kl.pos_mask);
        const uint32_t lp = key_primer(ka), rp = key_primer(kt);
        const uint32_t orient = (lp == 0 && rp == 1) ? 0u : (lp == 1 && rp == 0) ? 1u : (lp == 0) ? 2u : 3u;
        uint32_t *r = amps + 4 * o;
        r[0] = seq;
        r[1] = apos;
        r[2] = tpos + key_len(kt);
        r[3] = pair | (orient << 16);
    }
}

__global__ void ah_copy_count_kernel(const uint32_t *total, uint64_t *dst) { *dst = *total; }

static KeyLayout key_layout(const ah_store *st, ah_primer_set ps, int *total_bits) {
    KeyLayout kl;
    kl.pos_bits = ah_bits_for((uint64_t)st->max_len + 1);
    kl.pair_bits = ah_bits_for(ps->n_pairs);
    kl.seq_bits = ah_bits_for(st->n_seqs);
    kl.pos_mask = kl.pos_bits >= 64 ? ~0ull : ((1ull << kl.pos_bits) - 1);
    kl.pair_mask = kl.pair_bits >= 64 ? ~0ull : ((1ull << kl.pair_bits) - 1);
    *total_bits = kl.pos_bits + kl.pair_bits + kl.seq_bits + 7;
    return kl;
}

struct PairWs {
    uint64_t *keysA, *keysB;
    uint32_t *hist, *flag, *partner, *offs, *partials32;
    uint32_t *total;
    uint64_t bytes;
};

static PairWs pair_ws(void *base, uint64_t cap) {
    PairWs w;
    char *p = (char *)base;
    uint64_t o = 0;
    auto take = [&](uint64_t n) {
        char *r = p ? p + o : nullptr;
        o += ah_align_up(n, 256);
        return r;
    };
    w.keysA = (uint64_t *)take(8 * cap);
    w.keysB = (uint64_t *)take(8 * cap);
    w.hist = (uint32_t *)take(4ull * 256 * RS_G);
    w.flag = (uint32_t *)take(4 * cap);
    w.partner = (uint32_t *)take(4 * cap);
    w.offs = (uint32_t *)take(4 * cap);
    w.partials32 = (uint32_t *)take(4 * AH_SCAN_BLOCKS);
    w.total = (uint32_t *)take(16);
    w.bytes = o;
    return w;
}

extern "C" ah_status ah_pair_ws_size(const ah_store *st, ah_primer_set ps, uint64_t hit_cap, uint64_t *bytes) {
    if (!st || !ps || !bytes) return AH_E_ARG;
    *bytes = pair_ws(nullptr, hit_cap ? hit_cap : 1).bytes;
    return AH_OK;
}

extern "C" ah_status ah_pair_amplicons(const ah_store *st, ah_primer_set ps, const ah_hit *d_hits,
                                       const uint64_t *d_n_hits, uint64_t hit_cap, uint32_t orient_mask,
                                       ah_amp *d_amps, uint64_t amp_cap, uint64_t *d_n_amps, void *d_ws,
                                       uint64_t ws_bytes, void *stream) {
    if (!st || !ps || !d_n_hits || !d_n_amps || (hit_cap && !d_hits) || (amp_cap && !d_amps)) return AH_E_ARG;
    if (hit_cap >= (1ull << 32)) return AH_E_LIMIT;
    int bits = 0;
    KeyLayout kl = key_layout(st, ps, &bits);
    if (bits > 64) return AH_E_LIMIT;
    const uint64_t cap = hit_cap ? hit_cap : 1;
    PairWs w = pair_ws(d_ws, cap);
    if (!d_ws || ws_bytes < w.bytes) return AH_E_WORKSPACE;
    hipStream_t s = ah_stream(stream);
    hipLaunchKernelGGL(ah_pair_keys_kernel, dim3(1024), dim3(256), 0, s, (const uint32_t *)d_hits, d_n_hits, hit_cap,
                       (const DPair *)ps->d_pairs, kl, w.keysA);
    uint64_t *src = w.keysA, *dst = w.keysB;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        hipLaunchKernelGGL(ah_rs_hist_kernel, dim3(RS_G / 4), dim3(256), 0, s, (const uint64_t *)src, d_n_hits,
                           hit_cap, 8 * p, w.hist);
        // counts in place -> exclusive offsets (256 * RS_G entries)
        hipLaunchKernelGGL(ah_set_kernel<uint64_t>, dim3(1), dim3(1), 0, s, (uint64_t *)(w.total + 2),
                           (uint64_t)256 * RS_G);
        ah_status e = ah_exclusive_scan<uint32_t, uint32_t>(w.hist, w.hist, (const uint64_t *)(w.total + 2), ~0ull,
                                                            nullptr, w.partials32, s);
        if (e) return e;
        hipLaunchKernelGGL(ah_rs_scatter_kernel, dim3(RS_G / 4), dim3(256), 0, s, (const uint64_t *)src, dst,
                           d_n_hits, hit_cap, 8 * p, (const uint32_t *)w.hist);
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    hipLaunchKernelGGL(ah_pair_flag_kernel, dim3(1024), dim3(256), 0, s, (const uint64_t *)src, d_n_hits, hit_cap,
                       (const DPair *)ps->d_pairs, kl, orient_mask, w.flag, w.partner);
    ah_status e = ah_exclusive_scan<uint32_t, uint32_t>(w.flag, w.offs, d_n_hits, hit_cap, w.total, w.partials32, s);
    if (e) return e;
    hipLaunchKernelGGL(ah_copy_count_kernel, dim3(1), dim3(1), 0, s, (const uint32_t *)w.total, d_n_amps);
    hipLaunchKernelGGL(ah_pair_write_kernel, dim3(1024), dim3(256), 0, s, (const uint64_t *)src, d_n_hits, hit_cap,
                       kl, (const uint32_t *)w.flag, (const uint32_t *)w.partner, (const uint32_t *)w.offs,
                       (uint32_t *)d_amps, amp_cap);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
