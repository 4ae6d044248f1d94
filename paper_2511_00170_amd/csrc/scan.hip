// Primer scan over the 2-bit store (Supplementary, "Primer matching and clamp
// logic"): a window is a hit when every 3'-clamp position matches exactly and
// the number of substitutions is at most k.
//
// Layout of the work: a wave owns a tile of 64 blocks (4096 bases) of one
// sequence, lane i owns block i and reads it with one 128-bit load.  For its
// 64 positions the lane forms bit-vectors over positions ("position q matches
// IUPAC set m at offset i") with funnel shifts of the two bit planes and a
// 2-input select per set, and ANDs them over the first W clamp positions of
// each oriented pattern (a pre-filter: a window whose clamp fails is never a
// hit).  Surviving window starts are compacted into an LDS queue with a wave
// prefix sum, and each queued candidate is then verified exactly: the whole
// window is compared with the pattern's per-base masks, the clamp is checked
// in full, N bases are folded in and the substitutions counted.  Hits are
// appended with one atomic per wave and verification round.
#include "ah_internal.h"
#include "ah_scan_impl.h"

struct ScanArgs {
    ah_store st;
    const DPat *pats;
    uint32_t n_groups;        // pattern groups of 4 (one primer pair each)
    const uint32_t *list;     // sequence list (nullptr: identity)
    uint32_t n_list;
    const uint64_t *tile_pref;  // [n_list + 1] first tile of each listed sequence
    uint32_t *hits;           // ah_hit records as 3 words each
    uint64_t hit_cap;
    uint64_t *n_hits;
};

// bit q of the result: base at position q is in the IUPAC set `m` (bit b = base b).
__device__ __forceinline__ uint32_t set_match(uint32_t h, uint32_t l, uint32_t m) {
    const uint32_t sa = (m & 1u) ? 0xFFFFFFFFu : 0u;
    const uint32_t sc = (m & 2u) ? 0xFFFFFFFFu : 0u;
    const uint32_t sg = (m & 4u) ? 0xFFFFFFFFu : 0u;
    const uint32_t st = (m & 8u) ? 0xFFFFFFFFu : 0u;
    const uint32_t low = (l & sc) | (~l & sa);   // h == 0: C if l else A
    const uint32_t high = (l & st) | (~l & sg);  // h == 1: T if l else G
    return (h & high) | (~h & low);
}

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

struct TileCtx {
    uint32_t seq;
    uint32_t len;
    int64_t pos0;     // sequence position of the tile's first base
    uint64_t gblk0;   // store block of the tile's first base
    bool has_n;
};

// Verify queued candidates [0, qn) and append hits.
__device__ void verify_queue(const ScanArgs &a, const TileCtx &t, const uint32_t *sH, const uint32_t *sL,
                             const uint32_t *sQ, uint32_t qn) {
    const uint32_t lane = ah_lane();
    for (uint32_t base = 0; base < qn; base += 64) {
        const uint32_t e = base + lane;
        bool ok = false;
        uint32_t pos = 0, pk = 0, mm = 0;
        if (e < qn) {
            const uint32_t ent = sQ[e];
            const uint32_t X = ent >> 13, ql = ent & 0x1FFFu;
            const DPat &P = a.pats[X];
            const uint4 p0 = *(const uint4 *)&P.P[0];
            const uint4 p1 = *(const uint4 *)&P.clampmask;
            const uint32_t L = p1.z & 0xFFu, k = (p1.z >> 8) & 0xFFu, shift = p1.z >> 24;
            const int32_t pl = (int32_t)ql - (int32_t)shift;  // window start, tile-relative
            const int64_t gpos = t.pos0 + pl;
            if (gpos >= 0 && gpos + (int64_t)L <= (int64_t)t.len) {
                const uint32_t idx = (uint32_t)(pl + 32);
                const uint32_t w = idx >> 5, off = idx & 31u;
                const uint32_t hW = funnel(sH[w + 1], sH[w], off);
                const uint32_t lW = funnel(sL[w + 1], sL[w], off);
                uint32_t nW = 0;
                if (t.has_n) {
                    const uint64_t gp = t.gblk0 * 64 + (uint64_t)((int64_t)pl);
                    const uint64_t ba = gp >> 6, bb = (gp + L - 1) >> 6;
                    const uint32_t o = (uint32_t)(gp & 63);
                    uint64_t m = ah_block_nmask(a.st, ba) >> o;
                    if (bb != ba && o) m |= ah_block_nmask(a.st, bb) << (64 - o);
                    nW = (uint32_t)m;
                }
                const uint32_t lo = (lW & p0.y) | (~lW & p0.x);   // C : A
                const uint32_t hi = (lW & p0.w) | (~lW & p0.z);   // T : G
                const uint32_t matched = ((hW & hi) | (~hW & lo)) & ~nW & p1.y;
                mm = __popc(p1.y & ~matched);
                ok = ((matched & p1.x) == p1.x) && mm <= k;
                pos = (uint32_t)gpos;
                pk = p1.w;
            }
        }
        const uint64_t bal = __ballot(ok);
        if (bal) {
            uint64_t hbase = 0;
            if (lane == 0) hbase = atomicAdd((unsigned long long *)a.n_hits, (unsigned long long)__popcll(bal));
            hbase = __shfl(hbase, 0);
            if (ok) {
                const uint64_t h = hbase + ah_mbcnt(bal);
                if (h < a.hit_cap) {
                    uint32_t *r = a.hits + 3 * h;
                    r[0] = t.seq;
                    r[1] = pos;
                    r[2] = pk | (mm << 24);
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) ah_scan_kernel(ScanArgs a) {
    __shared__ uint32_t sH_all[4][2 * AH_TILE_BLOCKS + 2];
    __shared__ uint32_t sL_all[4][2 * AH_TILE_BLOCKS + 2];
    __shared__ uint32_t sQ_all[4][AH_QCAP];
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t *sH = sH_all[wv], *sL = sL_all[wv], *sQ = sQ_all[wv];
    const uint64_t total = a.tile_pref[a.n_list];
    const uint64_t nwaves = (uint64_t)gridDim.x * 4;
    // XCD-aware order: consecutive workgroups land on different XCDs, so give
    // each XCD a contiguous run of tiles.
    const uint32_t nwg = gridDim.x, xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    const uint32_t per = nwg / 8;
    const uint32_t wg = (nwg % 8 == 0) ? xcd * per + slot : blockIdx.x;
    const uint4 *blocks = (const uint4 *)a.st.d_blocks;

    for (uint64_t tile = (uint64_t)wg * 4 + wv; tile < total; tile += nwaves) {
        // sequence of this tile
        uint32_t lo = 0, hi = a.n_list;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.tile_pref[mid] <= tile) lo = mid;
            else hi = mid;
        }
        const uint32_t s = a.list ? a.list[lo] : lo;
        const uint32_t len = a.st.d_seq_len[s];
        const uint64_t nblk = ((uint64_t)len + 63) / 64;
        const uint64_t rel0 = (tile - a.tile_pref[lo]) * AH_TILE_BLOCKS;
        const uint64_t nb64 = nblk - rel0 < AH_TILE_BLOCKS ? nblk - rel0 : AH_TILE_BLOCKS;
        const uint32_t nb = (uint32_t)nb64;
        const uint64_t gb0 = a.st.d_seq_block0[s] + rel0;
        TileCtx t;
        t.seq = s;
        t.len = len;
        t.pos0 = (int64_t)(rel0 * 64);
        t.gblk0 = gb0;

        uint4 blk = make_uint4(0, 0, 0, 0);
        if (lane < nb) blk = blocks[gb0 + lane];
        uint32_t nxt_h = 0, nxt_l = 0, prv_h = 0, prv_l = 0;
        bool nflag = false;
        if (lane < nb) nflag = (a.st.d_nbits[(gb0 + lane) >> 5] >> ((gb0 + lane) & 31)) & 1u;
        if (lane == 63 && nb == AH_TILE_BLOCKS && rel0 + nb < nblk) {
            const uint4 nx = blocks[gb0 + nb];
            nxt_h = nx.x;
            nxt_l = nx.y;
            nflag = nflag || ((a.st.d_nbits[(gb0 + nb) >> 5] >> ((gb0 + nb) & 31)) & 1u);
        }
        if (lane == 0 && rel0 > 0) {
            const uint4 pv = blocks[gb0 - 1];
            prv_h = pv.z;
            prv_l = pv.w;
            nflag = nflag || ((a.st.d_nbits[(gb0 - 1) >> 5] >> ((gb0 - 1) & 31)) & 1u);
        }
        t.has_n = __ballot(nflag) != 0;
        const uint32_t h0 = blk.x, l0 = blk.y, h1 = blk.z, l1 = blk.w;
        uint32_t nh0 = __shfl_down(h0, 1, 64), nl0 = __shfl_down(l0, 1, 64);
        if (lane == 63) {
            nh0 = nxt_h;
            nl0 = nxt_l;
        }
        // tile words for verification: index 0 = the 32 bases before the tile
        sH[1 + 2 * lane] = h0;
        sH[2 + 2 * lane] = h1;
        sL[1 + 2 * lane] = l0;
        sL[2 + 2 * lane] = l1;
        if (lane == 0) {
            sH[0] = prv_h;
            sL[0] = prv_l;
        }
        if (lane == 63) {
            sH[2 * AH_TILE_BLOCKS + 1] = nxt_h;
            sL[2 * AH_TILE_BLOCKS + 1] = nxt_l;
        }
        // clamp sites q of this lane that lie inside the sequence
        const int64_t q0 = t.pos0 + 64 * (int64_t)lane;
        const int64_t rem = (int64_t)len - q0;
        const uint32_t valid0 = rem >= 32 ? 0xFFFFFFFFu : (rem <= 0 ? 0u : ((1u << rem) - 1u));
        const uint32_t valid1 = rem >= 64 ? 0xFFFFFFFFu : (rem <= 32 ? 0u : ((1u << (rem - 32)) - 1u));
        // shifted planes: bit q of S*[i][w] = plane bit of base q + i
        uint32_t Sh[AH_WMAX][2], Sl[AH_WMAX][2];
#pragma unroll
        for (int i = 0; i < AH_WMAX; i++) {
            Sh[i][0] = funnel(h1, h0, i);
            Sh[i][1] = funnel(nh0, h1, i);
            Sl[i][0] = funnel(l1, l0, i);
            Sl[i][1] = funnel(nl0, l1, i);
        }
        ah_wave_sync();
        uint32_t qn = 0;
        for (uint32_t g = 0; g < a.n_groups; g++) {
            uint32_t C[8];
#pragma unroll
            for (int x = 0; x < 4; x++) {
                const DPat &P = a.pats[4 * g + x];
                const uint32_t W = (P.meta >> 16) & 0xFFu;
                uint32_t c0 = valid0, c1 = valid1;
#pragma unroll
                for (int i = 0; i < AH_WMAX; i++) {
                    if ((uint32_t)i < W) {
                        const uint32_t m = P.fcode[i];
                        c0 &= set_match(Sh[i][0], Sl[i][0], m);
                        c1 &= set_match(Sh[i][1], Sl[i][1], m);
                    }
                }
                C[2 * x] = c0;
                C[2 * x + 1] = c1;
            }
            uint32_t cnt = 0;
#pragma unroll
            for (int w = 0; w < 8; w++) cnt += __popc(C[w]);
            if (__ballot(cnt != 0) == 0) continue;
            uint32_t incl = ah_wave_incl_sum<uint32_t>(cnt);
            const uint32_t tot = __shfl(incl, 63);
            if (qn + tot > AH_QCAP) {
                ah_wave_sync();
                verify_queue(a, t, sH, sL, sQ, qn);
                ah_wave_sync();
                qn = 0;
            }
            if (tot <= AH_QCAP) {
                uint32_t o = qn + incl - cnt;
#pragma unroll
                for (int w = 0; w < 8; w++) {
                    uint32_t c = C[w];
                    const uint32_t tag = ((4 * g + (uint32_t)(w >> 1)) << 13) | (64 * lane + 32 * (uint32_t)(w & 1));
                    while (c) {
                        const uint32_t b = __ffs(c) - 1;
                        c &= c - 1;
                        sQ[o++] = tag + b;
                    }
                }
                qn += tot;
            } else {
                // hit-dense tile: drain the candidates in rounds of at most
                // AH_QCAP / 64 per lane
                uint32_t left = cnt;
                while (__ballot(left != 0)) {
                    const uint32_t take = left < AH_QCAP / 64 ? left : AH_QCAP / 64;
                    const uint32_t inc2 = ah_wave_incl_sum<uint32_t>(take);
                    const uint32_t tot2 = __shfl(inc2, 63);
                    uint32_t o = inc2 - take, done = 0;
#pragma unroll
                    for (int w = 0; w < 8; w++) {
                        const uint32_t tag = ((4 * g + (uint32_t)(w >> 1)) << 13) | (64 * lane + 32 * (uint32_t)(w & 1));
                        while (C[w] && done < take) {
                            const uint32_t b = __ffs(C[w]) - 1;
                            C[w] &= C[w] - 1;
                            sQ[o++] = tag + b;
                            done++;
                        }
                    }
                    left -= take;
                    ah_wave_sync();
                    verify_queue(a, t, sH, sL, sQ, tot2);
                    ah_wave_sync();
                }
            }
        }
        if (qn) {
            ah_wave_sync();
            verify_queue(a, t, sH, sL, sQ, qn);
        }
        ah_wave_sync();
    }
}

__global__ void ah_tile_count_kernel(ah_store st, const uint32_t *list, uint32_t n, uint64_t *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t s = list ? list[i] : i;
        // an index outside the store contributes no tiles
        const uint64_t nblk = s < st.n_seqs ? ((uint64_t)st.d_seq_len[s] + 63) / 64 : 0;
        out[i] = (nblk + AH_TILE_BLOCKS - 1) / AH_TILE_BLOCKS;
    }
}

__global__ void __launch_bounds__(1024) ah_scan_small_u64_kernel(const uint64_t *in, uint64_t *out, uint64_t n) {
    __shared__ uint64_t lds[16];
    uint64_t carry = 0;
    for (uint64_t t0 = 0; t0 < n; t0 += blockDim.x) {
        const uint64_t i = t0 + threadIdx.x;
        const uint64_t v = i < n ? in[i] : 0;
        uint64_t tot;
        const uint64_t ex = ah_block_excl_sum<uint64_t>(v, lds, tot);
        if (i < n) out[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

void ah_scan_small_u64(const uint64_t *d_in, uint64_t *d_out, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(ah_scan_small_u64_kernel, dim3(1), dim3(1024), 0, s, d_in, d_out, n);
}

extern "C" ah_status ah_scan_ws_size(const ah_store *st, uint32_t n_list, uint64_t *bytes) {
    if (!st || !bytes) return AH_E_ARG;
    *bytes = ah_align_up(8ull * n_list, 256) + ah_align_up(8ull * (n_list + 1), 256);
    return AH_OK;
}

static int g_scan_grid = 0;

extern "C" ah_status ah_scan_primers(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset,
                                     uint32_t n_subset, ah_hit *d_hits, uint64_t hit_cap, uint64_t *d_n_hits,
                                     void *d_ws, uint64_t ws_bytes, void *stream) {
    if (!st || !ps || !d_n_hits || (hit_cap && !d_hits)) return AH_E_ARG;
    if (!st->d_blocks || !st->d_seq_block0 || !st->d_seq_len || !st->d_nbits) return AH_E_ARG;
    const uint32_t n_list = d_seq_subset ? n_subset : st->n_seqs;
    uint64_t need = 0;
    ah_scan_ws_size(st, n_list, &need);
    if (!d_ws || ws_bytes < need) return AH_E_WORKSPACE;
    if (ps->n_pats >= (1u << 19)) return AH_E_LIMIT;
    hipStream_t s = ah_stream(stream);
    uint64_t *cnt = (uint64_t *)d_ws;
    uint64_t *pref = (uint64_t *)((char *)d_ws + ah_align_up(8ull * n_list, 256));
    ah_fill<uint64_t>(d_n_hits, 0ull, 1, s);
    if (n_list) {
        hipLaunchKernelGGL(ah_tile_count_kernel, dim3(256), dim3(256), 0, s, *st, d_seq_subset, n_list, cnt);
    }
    ah_scan_small_u64(cnt, pref, n_list, s);
    if (!g_scan_grid) {
        // persistent grid: exactly the workgroups that can be resident at once
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ah_scan_kernel, 256, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        g_scan_grid = cus * per_cu;
    }
    ScanArgs a;
    a.st = *st;
    a.pats = ps->d_pats;
    a.n_groups = ps->n_pairs;
    a.list = d_seq_subset;
    a.n_list = n_list;
    a.tile_pref = pref;
    a.hits = (uint32_t *)d_hits;
    a.hit_cap = hit_cap;
    a.n_hits = d_n_hits;
    if (n_list) hipLaunchKernelGGL(ah_scan_kernel, dim3(g_scan_grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
