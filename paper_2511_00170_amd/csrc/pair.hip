// Amplicon calling (Supplementary, "Amplicon calling and orientation").
//
// Sites never pair across sequences, so the work is done per sequence:
//   1. count the hits of every sequence, scan the counts (bucket offsets) and
//      scatter the hits into per-sequence buckets as 64-bit keys whose
//      integer order is the site order within a sequence
//        key = pair | start | (L - 1) | sense | primer   (most to least significant)
//      with end = start + L;
//   2. every bucket is sorted -- by one wave in registers up to 64 keys,
//      else by a workgroup in LDS (bitonic) when it fits, else with a radix
//      sort in global memory -- and, in the sorted
//      order, gives every minus site its only possible partner: the nearest
//      plus site before it in the same pair (a plus site stops the walk);
//      the pairs inside the length window and the orientation mask are
//      ranked in key order;
//   3. the per-sequence amplicon counts are scanned and every amplicon is
//      written at its sequence's offset plus its rank (canonical order).
// Seven launches, whatever the number of hits; no workgroup waits on another.
#include "ah_internal.h"
#include "ah_scan_impl.h"

#define PAIR_WG 256
#define PAIR_LDS_KEYS 1024  // buckets up to this size are sorted in LDS (16.6 KB: 8 workgroups per CU)
#define PAIR_NO_AMP 0xFFFFFFFFu

struct KeyLayout {
    int pos_bits, pair_bits, key_bits;
    uint64_t pos_mask, pair_mask;
};

__device__ __forceinline__ uint32_t key_primer(uint64_t k) { return (uint32_t)(k & 1); }
__device__ __forceinline__ uint32_t key_sense(uint64_t k) { return (uint32_t)((k >> 1) & 1); }
__device__ __forceinline__ uint32_t key_len(uint64_t k) { return (uint32_t)((k >> 2) & 31) + 1; }

__device__ __forceinline__ uint32_t orient_of(uint32_t up_primer, uint32_t down_primer) {
    // (upstream, downstream) = (F, R) FR, (R, F) RF, (F, F) FF, (R, R) RR
    return (up_primer == 0 && down_primer == 1) ? 0u : (up_primer == 1 && down_primer == 0) ? 1u
                                                                                               : (up_primer == 0 ? 2u : 3u);
}

// Hits of a sequence mostly arrive together (the scan writes each wave's
// hits as one run), and with many hits per sequence per-hit atomics on one
// counter serialise.  So a wave first groups its lanes by sequence (one pass
// per distinct sequence, lane reads and ballots only), then the first lane of
// every group adds the group's size with one atomic -- all groups in a single
// instruction -- and the others take their share by rank.  Whole waves: hits
// [b, b + 64) per wave and step.
struct SeqGroup {
    int lead;       // first lane of this lane's group
    uint32_t rank;  // position in the group
    uint32_t size;  // lanes in the group
};

__device__ __forceinline__ SeqGroup group_by_seq(uint32_t s, bool valid) {
    SeqGroup g{(int)ah_lane(), 0u, 0u};
    bool todo = valid;
    for (uint64_t act = __ballot(todo); act; act = __ballot(todo)) {
        const int first = (int)__ffsll((unsigned long long)act) - 1;
        const uint32_t ls = __builtin_amdgcn_readlane(s, first);
        const bool mine = todo && s == ls;
        const uint64_t grp = __ballot(mine);
        if (mine) {
            g.lead = first;
            g.rank = ah_mbcnt(grp);
            g.size = (uint32_t)__popcll(grp);
        }
        todo = todo && !mine;
    }
    return g;
}

// 1. hits per sequence
__global__ void ah_pair_count_kernel(const uint32_t *hits, const uint64_t *d_n, uint64_t cap, uint32_t n_seqs,
                                     uint64_t *cnt) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const uint32_t lane = ah_lane();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t b = wave * 64; b < n; b += n_waves * 64) {
        const uint64_t i = b + lane;
        const uint32_t s = i < n ? hits[3 * i] : 0xFFFFFFFFu;
        const bool valid = s < n_seqs;
        const SeqGroup g = group_by_seq(s, valid);
        if (valid && g.rank == 0) atomicAdd((unsigned long long *)&cnt[s], (unsigned long long)g.size);
    }
}

// Hits into their sequence's bucket (in any order within it): the counts run
// down to zero as the slots are taken; a group of c lanes takes the c slots
// below the count its first lane found.
__global__ void ah_pair_scatter_kernel(const uint32_t *hits, const uint64_t *d_n, uint64_t cap, uint32_t n_seqs,
                                       const DPair *pairs, KeyLayout kl, const uint64_t *boff, uint64_t *cnt,
                                       uint64_t *keys) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const uint32_t lane = ah_lane();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t b = wave * 64; b < n; b += n_waves * 64) {
        const uint64_t i = b + lane;
        uint32_t s = 0xFFFFFFFFu, pos = 0, w = 0;
        if (i < n) {
            s = hits[3 * i];
            pos = hits[3 * i + 1];
            w = hits[3 * i + 2];
        }
        const bool valid = s < n_seqs;
        const SeqGroup g = group_by_seq(s, valid);
        unsigned long long old = 0;
        if (valid && g.rank == 0)
            old = atomicAdd((unsigned long long *)&cnt[s], (unsigned long long)(-(int64_t)g.size));
        old = __shfl(old, g.lead, 64);
        if (valid) {
            const uint32_t pair = w & 0xFFFFu, kind = (w >> 16) & 0xFFu;
            const uint32_t primer = kind & 1u, sense = (kind >> 1) & 1u;
            const uint32_t L = primer ? pairs[pair].Lr : pairs[pair].Lf;
            keys[boff[s] + old - 1 - g.rank] = ((uint64_t)pair << (kl.pos_bits + 7)) | ((uint64_t)pos << 7) |
                                               ((uint64_t)(L - 1) << 2) | ((uint64_t)sense << 1) | primer;
        }
    }
}

// The partner of the minus site k[i] in the sorted bucket k[0..m): index of
// the nearest plus site before it in the same pair, if the amplicon they span
// is inside the pair's window and its orientation is asked for; else -1.
__device__ __forceinline__ int64_t partner_of(const uint64_t *k, uint64_t i, const DPair *pairs, KeyLayout kl,
                                              uint32_t orient_mask) {
    const uint64_t kt = k[i];
    if (key_sense(kt) != 1) return -1;
    const uint64_t seg = kt >> (7 + kl.pos_bits);
    const uint32_t pair = (uint32_t)(seg & kl.pair_mask);
    const uint64_t tend = ((kt >> 7) & kl.pos_mask) + key_len(kt);
    const uint32_t mn = pairs[pair].min_len, mx = pairs[pair].max_len;
    const uint64_t lo_start = tend > mx ? tend - mx : 0;
    for (uint64_t j = i; j-- > 0;) {
        const uint64_t kj = k[j];
        if ((kj >> (7 + kl.pos_bits)) != seg) return -1;
        const uint64_t pj = (kj >> 7) & kl.pos_mask;
        if (pj < lo_start) return -1;  // any partner from here on is too far
        if (key_sense(kj) == 0) {
            const uint64_t len = tend - pj;
            const uint32_t o = orient_of(key_primer(kj), key_primer(kt));
            return (len >= mn && len <= mx && ((orient_mask >> o) & 1u)) ? (int64_t)j : -1;
        }
    }
    return -1;
}

// Ranks the amplicons of a sorted bucket (k[0..m), LDS or global) in key
// order: rank[i] = their index among the bucket's amplicons for every minus
// site with a partner (part[i] = that partner), PAIR_NO_AMP otherwise.
// Returns the bucket's amplicon count.  Whole workgroup.
__device__ uint32_t rank_amplicons(const uint64_t *k, uint64_t m, const DPair *pairs, KeyLayout kl,
                                   uint32_t orient_mask, uint32_t *rank, uint32_t *part, uint32_t *lds16) {
    // contiguous chunk per thread so the ranks follow key order
    const uint64_t per = (m + PAIR_WG - 1) / PAIR_WG;
    const uint64_t i0 = (uint64_t)threadIdx.x * per, i1 = i0 + per < m ? i0 + per : m;
    uint32_t mine = 0;
    for (uint64_t i = i0; i < i1; i++) {
        const int64_t p = partner_of(k, i, pairs, kl, orient_mask);
        rank[i] = p >= 0 ? 1u : 0u;
        part[i] = p >= 0 ? (uint32_t)p : 0u;
        mine += p >= 0 ? 1u : 0u;
    }
    uint32_t total;
    uint32_t r = ah_block_excl_sum<uint32_t>(mine, lds16, total);
    for (uint64_t i = i0; i < i1; i++) {
        const uint32_t f = rank[i];
        rank[i] = f ? r : PAIR_NO_AMP;
        r += f;
    }
    return total;
}

// Stable LSD radix sort (8-bit digits) of a[0..m) by one workgroup, through
// b[0..m); the result ends in a.  For buckets too large for LDS.
__device__ void bucket_radix_sort(uint64_t *a, uint64_t *b, uint64_t m, int key_bits, uint32_t (*h)[256],
                                  uint32_t *lds16) {
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t chunk = (m + 3) / 4;  // one contiguous chunk per wave keeps the sort stable
    const uint64_t c0 = wv * chunk, c1 = c0 + chunk < m ? c0 + chunk : m;
    uint64_t *src = a, *dst = b;
    for (int sh = 0; sh < key_bits; sh += 8) {
        for (uint32_t d = threadIdx.x; d < 4 * 256; d += PAIR_WG) h[d >> 8][d & 255] = 0;
        __syncthreads();
        for (uint64_t i = c0 + lane; i < c1; i += 64) atomicAdd(&h[wv][(src[i] >> sh) & 255u], 1u);
        __syncthreads();
        // offsets: digit-major, then wave (chunk) order
        const uint32_t d = threadIdx.x;  // PAIR_WG == 256: one digit per thread
        const uint32_t c[4] = {h[0][d], h[1][d], h[2][d], h[3][d]};
        uint32_t tot;
        const uint32_t base = ah_block_excl_sum<uint32_t>(c[0] + c[1] + c[2] + c[3], lds16, tot);
        h[0][d] = base;
        h[1][d] = base + c[0];
        h[2][d] = base + c[0] + c[1];
        h[3][d] = base + c[0] + c[1] + c[2];
        __syncthreads();
        uint32_t *run = h[wv];
        for (uint64_t r0 = c0; r0 < c1; r0 += 64) {
            const uint64_t i = r0 + lane;
            const bool valid = i < c1;
            const uint64_t key = valid ? src[i] : 0;
            const uint32_t dg = (uint32_t)(key >> sh) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; bit++) {
                const bool on = (dg >> bit) & 1u;
                const uint64_t bb = __ballot(on);
                peers &= on ? bb : ~bb;
            }
            const uint32_t rk = ah_mbcnt(peers);
            const uint32_t at = valid ? run[dg] : 0;
            ah_wave_sync();
            if (valid && rk == 0) run[dg] = at + (uint32_t)__popcll(peers);
            ah_wave_sync();
            if (valid) dst[at + rk] = key;
        }
        __syncthreads();
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != a)
        for (uint64_t i = threadIdx.x; i < m; i += PAIR_WG) a[i] = src[i];
    __syncthreads();
}

// A bucket of at most 64 keys, by one wave: bitonic sort across the lanes
// (one key per lane, compare-exchange through lane shuffles, no barrier),
// then pairing and ranking over a per-wave LDS copy of the sorted keys.
__device__ __forceinline__ void wave_bucket(uint64_t *keys, uint64_t base, uint32_t m, const DPair *pairs,
                                            KeyLayout kl, uint32_t orient_mask, uint32_t *rank, uint32_t *part,
                                            uint64_t *acnt_s, uint64_t *swk) {
    const uint32_t lane = ah_lane();
    uint64_t v = lane < m ? keys[base + lane] : ~0ull;
#pragma unroll
    for (uint32_t len = 2; len <= 64; len <<= 1) {
#pragma unroll
        for (uint32_t st = len >> 1; st > 0; st >>= 1) {
            const uint64_t o = __shfl_xor(v, (int)st, 64);
            const bool keep_min = ((lane & st) == 0) == ((lane & len) == 0);  // lower lane of an ascending run
            v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
        }
    }
    ah_wave_sync();
    swk[lane] = v;
    ah_wave_sync();
    const int64_t p = lane < m ? partner_of(swk, lane, pairs, kl, orient_mask) : -1;
    const uint64_t bal = __ballot(p >= 0);
    if (lane < m) {
        keys[base + lane] = v;
        rank[base + lane] = p >= 0 ? ah_mbcnt(bal) : PAIR_NO_AMP;
        part[base + lane] = p >= 0 ? (uint32_t)p : 0u;
    }
    if (lane == 0) *acnt_s = (uint64_t)__popcll(bal);
}

// 2. sort every bucket, pair, rank: one workgroup per sequence; a bucket of
// at most 64 keys is done by its first wave alone (no barrier), a larger one
// by the whole workgroup (in LDS up to PAIR_LDS_KEYS, else in global memory).
// Bounded to 64 VGPRs (no spill) so that, with 16.6 KB of LDS, eight
// workgroups fit on a CU: 2048 sequences in one round.
__global__ void __launch_bounds__(PAIR_WG, 8) ah_pair_bucket_kernel(uint64_t *keys, uint64_t *scratch,
                                                                 const uint64_t *boff, uint32_t n_seqs,
                                                                 const DPair *pairs, KeyLayout kl,
                                                                 uint32_t orient_mask, uint32_t *rank,
                                                                 uint32_t *part, uint64_t *acnt) {
    __shared__ uint64_t sk[PAIR_LDS_KEYS];
    __shared__ uint32_t srank[PAIR_LDS_KEYS], spart[PAIR_LDS_KEYS];
    // the radix path's digit counts reuse srank (that path ranks in global memory)
    static_assert(PAIR_LDS_KEYS >= 4 * 256, "digit counts fit in srank");
    uint32_t(*h)[256] = (uint32_t(*)[256])srank;
    __shared__ uint32_t lds16[16];
    __shared__ uint64_t swk[64];
    for (uint32_t s = blockIdx.x; s < n_seqs; s += gridDim.x) {
        // every thread reads the same bounds: the branch is the workgroup's
        const uint64_t base = boff[s], m = boff[s + 1] - base;
        if (m <= 64) {
            if (threadIdx.x < 64) wave_bucket(keys, base, (uint32_t)m, pairs, kl, orient_mask, rank, part,
                                              &acnt[s], swk);
            continue;
        }
        uint32_t total = 0;
        if (m <= PAIR_LDS_KEYS) {
            uint32_t P = 1;
            while (P < m) P <<= 1;
            for (uint32_t i = threadIdx.x; i < P; i += PAIR_WG) sk[i] = i < m ? keys[base + i] : ~0ull;
            __syncthreads();
            // bitonic sort of sk[0..P)
            for (uint32_t len = 2; len <= P; len <<= 1) {
                for (uint32_t st = len >> 1; st > 0; st >>= 1) {
                    for (uint32_t i = threadIdx.x; i < P; i += PAIR_WG) {
                        const uint32_t j = i ^ st;
                        if (j > i) {
                            const bool up = (i & len) == 0;
                            const uint64_t x = sk[i], y = sk[j];
                            if ((x > y) == up) {
                                sk[i] = y;
                                sk[j] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            total = rank_amplicons(sk, m, pairs, kl, orient_mask, srank, spart, lds16);
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < m; i += PAIR_WG) {
                keys[base + i] = sk[i];
                rank[base + i] = srank[i];
                part[base + i] = spart[i];
            }
        } else {
            bucket_radix_sort(keys + base, scratch + base, m, kl.key_bits, h, lds16);
            total = rank_amplicons(keys + base, m, pairs, kl, orient_mask, rank + base, part + base, lds16);
        }
        if (threadIdx.x == 0) acnt[s] = total;
        __syncthreads();
    }
}

// 3. write every amplicon at its sequence's offset plus its rank
__global__ void __launch_bounds__(PAIR_WG) ah_pair_write_kernel(const uint64_t *keys, const uint64_t *boff,
                                                                const uint64_t *aoff, uint32_t n_seqs, KeyLayout kl,
                                                                const uint32_t *rank, const uint32_t *part,
                                                                uint32_t *amps, uint64_t amp_cap,
                                                                uint64_t *d_n_amps) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *d_n_amps = aoff[n_seqs];
    for (uint32_t s = blockIdx.x; s < n_seqs; s += gridDim.x) {
        const uint64_t base = boff[s], m = boff[s + 1] - base, a0 = aoff[s];
        for (uint64_t i = threadIdx.x; i < m; i += PAIR_WG) {
            const uint32_t r = rank[base + i];
            if (r == PAIR_NO_AMP || a0 + r >= amp_cap) continue;
            const uint64_t kt = keys[base + i], ka = keys[base + part[base + i]];
            const uint32_t pair = (uint32_t)((kt >> (7 + kl.pos_bits)) & kl.pair_mask);
            uint32_t *o = amps + 4 * (a0 + r);
            o[0] = s;
            o[1] = (uint32_t)((ka >> 7) & kl.pos_mask);
            o[2] = (uint32_t)((kt >> 7) & kl.pos_mask) + key_len(kt);
            o[3] = pair | (orient_of(key_primer(ka), key_primer(kt)) << 16);
        }
    }
}

static KeyLayout key_layout(const ah_store *st, ah_primer_set ps) {
    KeyLayout kl;
    kl.pos_bits = ah_bits_for((uint64_t)st->max_len + 1);
    kl.pair_bits = ah_bits_for(ps->n_pairs);
    kl.key_bits = kl.pos_bits + kl.pair_bits + 7;
    kl.pos_mask = kl.pos_bits >= 64 ? ~0ull : ((1ull << kl.pos_bits) - 1);
    kl.pair_mask = kl.pair_bits >= 64 ? ~0ull : ((1ull << kl.pair_bits) - 1);
    return kl;
}

struct PairWs {
    uint64_t *keys, *scratch, *cnt, *boff, *aoff;
    uint32_t *rank, *part;
    uint64_t bytes;
};

static PairWs pair_ws(void *base, uint64_t cap, uint32_t n_seqs) {
    PairWs w;
    char *p = (char *)base;
    uint64_t o = 0;
    auto take = [&](uint64_t n) {
        char *r = p ? p + o : nullptr;
        o += ah_align_up(n, 256);
        return r;
    };
    w.keys = (uint64_t *)take(8 * cap);
    w.scratch = (uint64_t *)take(8 * cap);
    w.rank = (uint32_t *)take(4 * cap);
    w.part = (uint32_t *)take(4 * cap);
    w.cnt = (uint64_t *)take(8ull * (n_seqs + 1));
    w.boff = (uint64_t *)take(8ull * (n_seqs + 1));
    w.aoff = (uint64_t *)take(8ull * (n_seqs + 1));
    w.bytes = o;
    return w;
}

extern "C" ah_status ah_pair_ws_size(const ah_store *st, ah_primer_set ps, uint64_t hit_cap, uint64_t *bytes) {
    if (!st || !ps || !bytes) return AH_E_ARG;
    *bytes = pair_ws(nullptr, hit_cap ? hit_cap : 1, st->n_seqs).bytes;
    return AH_OK;
}

extern "C" ah_status ah_pair_amplicons(const ah_store *st, ah_primer_set ps, const ah_hit *d_hits,
                                       const uint64_t *d_n_hits, uint64_t hit_cap, uint32_t orient_mask,
                                       ah_amp *d_amps, uint64_t amp_cap, uint64_t *d_n_amps, void *d_ws,
                                       uint64_t ws_bytes, void *stream) {
    if (!st || !ps || !d_n_hits || !d_n_amps || (hit_cap && !d_hits) || (amp_cap && !d_amps)) return AH_E_ARG;
    if (hit_cap >= (1ull << 32)) return AH_E_LIMIT;
    const KeyLayout kl = key_layout(st, ps);
    if (kl.key_bits > 64) return AH_E_LIMIT;
    const uint64_t cap = hit_cap ? hit_cap : 1;
    const uint32_t ns = st->n_seqs;
    PairWs w = pair_ws(d_ws, cap, ns);
    if (!d_ws || ws_bytes < w.bytes) return AH_E_WORKSPACE;
    hipStream_t s = ah_stream(stream);
    const DPair *pairs = (const DPair *)ps->d_pairs;
    ah_fill<uint64_t>(w.cnt, 0ull, (uint64_t)ns + 1, s);
    hipLaunchKernelGGL(ah_pair_count_kernel, dim3(1024), dim3(256), 0, s, (const uint32_t *)d_hits, d_n_hits, hit_cap,
                       ns, w.cnt);
    ah_scan_small_u64(w.cnt, w.boff, ns, s);  // boff[ns] = hits in buckets
    hipLaunchKernelGGL(ah_pair_scatter_kernel, dim3(1024), dim3(256), 0, s, (const uint32_t *)d_hits, d_n_hits,
                       hit_cap, ns, pairs, kl, (const uint64_t *)w.boff, w.cnt, w.keys);
    const unsigned grid = ns < 8192u ? (ns ? ns : 1u) : 8192u;
    hipLaunchKernelGGL(ah_pair_bucket_kernel, dim3(grid), dim3(PAIR_WG), 0, s, w.keys, w.scratch,
                       (const uint64_t *)w.boff, ns, pairs, kl, orient_mask, w.rank, w.part, w.cnt);
    ah_scan_small_u64(w.cnt, w.aoff, ns, s);  // aoff[ns] = amplicons
    hipLaunchKernelGGL(ah_pair_write_kernel, dim3(grid), dim3(PAIR_WG), 0, s, (const uint64_t *)w.keys,
                       (const uint64_t *)w.boff, (const uint64_t *)w.aoff, ns, kl, (const uint32_t *)w.rank,
                       (const uint32_t *)w.part, (uint32_t *)d_amps, amp_cap, d_n_amps);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
