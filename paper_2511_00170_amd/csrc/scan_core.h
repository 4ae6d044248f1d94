// Primer scan kernel body (Supplementary, "Primer matching and clamp logic":
// per-base IUPAC masks, reverse-complement masks, substitutions counted with
// bit operations, exact 3' clamp).  Included by scan.hip for the generic
// kernel and compiled by hipRTC, with constant pattern codes, for kernels
// specialised to one primer set.
//
// Work layout.  A tile is 64 blocks (4096 bases) of one sequence; a wave owns
// a contiguous run of tiles and walks it in order, prefetching the next
// tile's blocks while it works on the current one (lane i owns block i and
// reads it with one 128-bit load).  For its 64 clamp sites q a lane builds
// bit-vectors "base q+i is in IUPAC set m" from funnel shifts of the two bit
// planes and ANDs them over the first W clamp positions of each oriented
// pattern -- a window that fails this pre-filter can never be a hit.
// Surviving (pattern, q) pairs are compacted into an LDS queue with a wave
// prefix sum; each queued candidate is verified exactly (full window against
// the pattern's per-base masks, full clamp, N bases, substitution count) and
// hits are appended with one atomic per wave and verification round.
#pragma once

#include "ah_dev.h"

#define AH_LDS_PATS 256  // pattern records staged in LDS for verification

struct ScanArgs {
    ah_store st;
    const DPat *pats;
    uint32_t n_pats;
    uint32_t n_groups;           // pattern groups of 4 (one primer pair each)
    const uint32_t *list;        // listed sequences (nullptr: every sequence)
    uint32_t n_list;
    const uint64_t *tile_pref;   // [n_list + 1] first tile of each listed sequence
    uint32_t *hits;              // ah_hit records, 3 words each
    uint64_t hit_cap;
    uint64_t *n_hits;
};

__device__ __forceinline__ uint32_t ah_funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// acc AND (bit q: base q is in IUPAC set M), M a compile-time set (bit b = base b)
template <uint32_t M>
__device__ __forceinline__ uint32_t ah_and_set(uint32_t acc, uint32_t h, uint32_t l) {
    constexpr uint32_t sa = (M & 1u) ? 0xFFFFFFFFu : 0u, sc = (M & 2u) ? 0xFFFFFFFFu : 0u;
    constexpr uint32_t sg = (M & 4u) ? 0xFFFFFFFFu : 0u, st = (M & 8u) ? 0xFFFFFFFFu : 0u;
    const uint32_t low = (l & sc) | (~l & sa);   // h = 0: C if l else A
    const uint32_t high = (l & st) | (~l & sg);  // h = 1: T if l else G
    return acc & ((h & high) | (~h & low));
}

struct TileCtx {
    uint32_t seq;
    uint32_t len;
    int64_t pos0;    // sequence position of the tile's first base
    uint64_t gblk0;  // store block of the tile's first base
    bool has_n;
};

// Sequence cursor over the tile list of one wave.
struct SeqCursor {
    uint32_t i;        // list index
    uint32_t seq;
    uint32_t len;
    uint64_t nblk;
    uint64_t blk0;
    uint64_t tp0, tp1; // tile_pref[i], tile_pref[i + 1]

    __device__ void load(const ScanArgs &a) {
        seq = a.list ? a.list[i] : i;
        len = a.st.d_seq_len[seq];
        nblk = ((uint64_t)len + 63) / 64;
        blk0 = a.st.d_seq_block0[seq];
        tp0 = a.tile_pref[i];
        tp1 = a.tile_pref[i + 1];
    }
    __device__ void init(const ScanArgs &a, uint64_t t) {
        uint32_t lo = 0, hi = a.n_list;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.tile_pref[mid] <= t) lo = mid;
            else hi = mid;
        }
        i = lo;
        load(a);
    }
    __device__ void advance(const ScanArgs &a, uint64_t t) {
        while (t >= tp1) {
            i++;
            load(a);
        }
    }
};

// Everything one tile needs from global memory, loaded one tile ahead.
struct TileLoad {
    uint4 blk;        // this lane's block
    uint32_t nbw;     // N-bitmap word of this lane's block (bit already extracted)
    uint32_t halo_h;  // lane 0: upper half of the previous block; lane 63: lower half of the next block
    uint32_t halo_l;
    uint32_t halo_n;  // N flag of that halo block
    uint32_t nb;      // blocks in the tile
    uint64_t rel0;    // first block of the tile within its sequence
};

__device__ __forceinline__ void tile_issue(const ScanArgs &a, const SeqCursor &c, uint64_t t, TileLoad &L) {
    const uint32_t lane = ah_lane();
    const uint4 *blocks = (const uint4 *)a.st.d_blocks;
    L.rel0 = (t - c.tp0) * AH_TILE_BLOCKS;
    const uint64_t left = c.nblk - L.rel0;
    L.nb = (uint32_t)(left < AH_TILE_BLOCKS ? left : AH_TILE_BLOCKS);
    const uint64_t gb0 = c.blk0 + L.rel0;
    L.blk = make_uint4(0, 0, 0, 0);
    L.nbw = 0;
    L.halo_h = L.halo_l = L.halo_n = 0;
    if (lane < L.nb) {
        L.blk = blocks[gb0 + lane];
        L.nbw = (a.st.d_nbits[(gb0 + lane) >> 5] >> ((gb0 + lane) & 31)) & 1u;
    }
    if (lane == 0 && L.rel0 > 0) {
        const uint4 pv = blocks[gb0 - 1];
        L.halo_h = pv.z;
        L.halo_l = pv.w;
        L.halo_n = (a.st.d_nbits[(gb0 - 1) >> 5] >> ((gb0 - 1) & 31)) & 1u;
    }
    if (lane == 63 && L.nb == AH_TILE_BLOCKS && L.rel0 + AH_TILE_BLOCKS < c.nblk) {
        const uint4 nx = blocks[gb0 + AH_TILE_BLOCKS];
        L.halo_h = nx.x;
        L.halo_l = nx.y;
        L.halo_n = (a.st.d_nbits[(gb0 + AH_TILE_BLOCKS) >> 5] >> ((gb0 + AH_TILE_BLOCKS) & 31)) & 1u;
    }
}

// Verify queued candidates [0, qn) and append hits.
__device__ void ah_verify_queue(const ScanArgs &a, const TileCtx &t, const uint32_t *sH, const uint32_t *sL,
                                const uint32_t *sQ, uint32_t qn, const DPat *sPat) {
    const uint32_t lane = ah_lane();
    for (uint32_t base = 0; base < qn; base += 64) {
        const uint32_t e = base + lane;
        bool ok = false;
        uint32_t pos = 0, pk = 0, mm = 0;
        if (e < qn) {
            const uint32_t ent = sQ[e];
            const uint32_t X = ent >> 13, ql = ent & 0x1FFFu;
            const DPat *P = X < AH_LDS_PATS ? &sPat[X] : &a.pats[X];
            const uint4 p0 = *(const uint4 *)&P->P[0];
            const uint4 p1 = *(const uint4 *)&P->clampmask;
            const uint32_t L = p1.z & 0xFFu, k = (p1.z >> 8) & 0xFFu, shift = p1.z >> 24;
            const int32_t pl = (int32_t)ql - (int32_t)shift;  // window start, tile-relative
            const int64_t gpos = t.pos0 + pl;
            if (gpos >= 0 && gpos + (int64_t)L <= (int64_t)t.len) {
                const uint32_t idx = (uint32_t)(pl + 32);
                const uint32_t w = idx >> 5, off = idx & 31u;
                const uint32_t hW = ah_funnel(sH[w + 1], sH[w], off);
                const uint32_t lW = ah_funnel(sL[w + 1], sL[w], off);
                uint32_t nW = 0;
                if (t.has_n) {
                    const uint64_t gp = t.gblk0 * 64 + (uint64_t)((int64_t)pl);
                    const uint64_t ba = gp >> 6, bb = (gp + L - 1) >> 6;
                    const uint32_t o = (uint32_t)(gp & 63);
                    uint64_t m = ah_block_nmask(a.st, ba) >> o;
                    if (bb != ba && o) m |= ah_block_nmask(a.st, bb) << (64 - o);
                    nW = (uint32_t)m;
                }
                const uint32_t lo = (lW & p0.y) | (~lW & p0.x);  // C : A
                const uint32_t hi = (lW & p0.w) | (~lW & p0.z);  // T : G
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

// Push the candidate words C[8] (pattern x of group g: words 2x, 2x+1) into
// the wave queue, verifying whenever it would overflow.
__device__ __forceinline__ void ah_push_group(const ScanArgs &a, const TileCtx &t, uint32_t g, uint32_t (&C)[8],
                                              const uint32_t *sH, const uint32_t *sL, uint32_t *sQ, uint32_t &qn,
                                              const DPat *sPat) {
    const uint32_t lane = ah_lane();
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < 8; w++) cnt += __popc(C[w]);
    if (__ballot(cnt != 0) == 0) return;
    const uint32_t incl = ah_wave_incl_sum<uint32_t>(cnt);
    const uint32_t tot = __shfl(incl, 63);
    if (qn + tot > AH_QCAP) {
        ah_wave_sync();
        ah_verify_queue(a, t, sH, sL, sQ, qn, sPat);
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
        // hit-dense tile: drain in rounds of at most AH_QCAP / 64 per lane
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
            ah_verify_queue(a, t, sH, sL, sQ, tot2, sPat);
            ah_wave_sync();
        }
    }
}

// The kernel body.  Filter F provides
//   F::groups(a)  number of pattern groups,
//   f.filter(g, Sh, Sl, v0, v1, C)  candidate words of group g.
template <class F>
__device__ __forceinline__ void ah_scan_body(const ScanArgs &a, F &f, DPat *sPat, uint32_t (*sH_all)[2 * AH_TILE_BLOCKS + 2],
                                             uint32_t (*sL_all)[2 * AH_TILE_BLOCKS + 2], uint32_t (*sQ_all)[AH_QCAP]) {
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t *sH = sH_all[wv], *sL = sL_all[wv], *sQ = sQ_all[wv];
    const uint64_t total = a.tile_pref[a.n_list];
    // XCD-aware numbering: workgroup i runs on XCD i % 8, so give each XCD a
    // contiguous share of the tiles.
    const uint32_t nwg = gridDim.x;
    const uint32_t wg = (nwg % 8 == 0) ? (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8 : blockIdx.x;
    const uint64_t nw = (uint64_t)nwg * 4, gw = (uint64_t)wg * 4 + wv;
    const uint64_t per = (total + nw - 1) / nw;
    uint64_t t = gw * per;
    const uint64_t tend = t + per < total ? t + per : total;
    if (t >= tend) return;

    SeqCursor cur;
    cur.init(a, t);
    TileLoad L;
    tile_issue(a, cur, t, L);
    const uint32_t groups = f.groups(a);

    for (; t < tend; t++) {
        // issue the next tile's loads before working on this one
        SeqCursor nc = cur;
        TileLoad NL;
        const bool has_next = t + 1 < tend;
        if (has_next) {
            nc.advance(a, t + 1);
            tile_issue(a, nc, t + 1, NL);
        }

        TileCtx tc;
        tc.seq = cur.seq;
        tc.len = cur.len;
        tc.pos0 = (int64_t)(L.rel0 * 64);
        tc.gblk0 = cur.blk0 + L.rel0;
        tc.has_n = __ballot(L.nbw | L.halo_n) != 0;

        const uint32_t h0 = L.blk.x, l0 = L.blk.y, h1 = L.blk.z, l1 = L.blk.w;
        uint32_t nh0 = __shfl_down(h0, 1, 64), nl0 = __shfl_down(l0, 1, 64);
        if (lane == 63) {
            nh0 = L.halo_h;
            nl0 = L.halo_l;
        }
        sH[1 + 2 * lane] = h0;
        sH[2 + 2 * lane] = h1;
        sL[1 + 2 * lane] = l0;
        sL[2 + 2 * lane] = l1;
        if (lane == 0) {
            sH[0] = L.halo_h;
            sL[0] = L.halo_l;
        }
        if (lane == 63) {
            sH[2 * AH_TILE_BLOCKS + 1] = L.halo_h;
            sL[2 * AH_TILE_BLOCKS + 1] = L.halo_l;
        }
        // clamp sites of this lane inside the sequence
        const int64_t rem = (int64_t)tc.len - (tc.pos0 + 64 * (int64_t)lane);
        const uint32_t v0 = rem >= 32 ? 0xFFFFFFFFu : (rem <= 0 ? 0u : ((1u << rem) - 1u));
        const uint32_t v1 = rem >= 64 ? 0xFFFFFFFFu : (rem <= 32 ? 0u : ((1u << (rem - 32)) - 1u));
        // bit q of S*[i][w]: plane bit of base q + i (w selects bases 0-31 / 32-63)
        uint32_t Sh[AH_WMAX][2], Sl[AH_WMAX][2];
#pragma unroll
        for (int i = 0; i < AH_WMAX; i++) {
            Sh[i][0] = ah_funnel(h1, h0, i);
            Sh[i][1] = ah_funnel(nh0, h1, i);
            Sl[i][0] = ah_funnel(l1, l0, i);
            Sl[i][1] = ah_funnel(nl0, l1, i);
        }
        ah_wave_sync();
        uint32_t qn = 0;
        for (uint32_t g = 0; g < groups; g++) {
            uint32_t C[8];
            f.filter(g, Sh, Sl, v0, v1, C);
            ah_push_group(a, tc, g, C, sH, sL, sQ, qn, sPat);
        }
        if (qn) {
            ah_wave_sync();
            ah_verify_queue(a, tc, sH, sL, sQ, qn, sPat);
        }
        ah_wave_sync();
        cur = nc;
        L = NL;
    }
}

// Stage the first AH_LDS_PATS pattern records in LDS (all threads of the block).
__device__ __forceinline__ void ah_stage_patterns(const ScanArgs &a, DPat *sPat) {
    const uint32_t n = a.n_pats < AH_LDS_PATS ? a.n_pats : AH_LDS_PATS;
    const uint4 *src = (const uint4 *)a.pats;
    uint4 *dst = (uint4 *)sPat;
    for (uint32_t i = threadIdx.x; i < n * 3; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}
