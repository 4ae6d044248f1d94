// Primer scan kernel body (Supplementary, "Primer matching and clamp logic":
// per-base IUPAC masks, reverse-complement masks, substitutions counted with
// bit operations, exact 3' clamp).  Included by scan.hip for the generic
// kernel and compiled by hipRTC, with constant pattern codes, for kernels
// specialised to one primer set.
//
// Work layout.  A tile is 64 x AH_BPL blocks of one sequence (64 bases each);
// a wave owns a contiguous run of tiles and walks it in order, prefetching
// the next tile's blocks while it works on the current one (lane i owns
// blocks AH_BPL*i .. AH_BPL*i + AH_BPL-1, read with 128-bit loads).  The
// lane's blocks are filtered one after the other (a "half" of a two-block
// tile), so a larger tile shares the per-tile work -- its loads, context and
// sequence walk -- without holding more planes in registers.  For its
// clamp sites q a lane builds bit-vectors "base q+i is in IUPAC set m" from
// funnel shifts of the two bit planes and ANDs them over the filter
// positions of each oriented pattern -- a window that fails this pre-filter
// can never be a hit.  A lane whose candidate mask for a pattern is non-zero
// appends (mask, pattern, lane, tile) to a per-wave LDS queue -- one ballot
// per pattern gives the slots, no prefix sums.  The queue spans several
// tiles and is verified in full-wave rounds against the tiles' words kept in
// LDS: the full clamp, N bases and the substitution count.  Hits go to a
// small per-wave LDS buffer (an LDS atomic each) that is written out with
// one device atomic per batch: a device atomic whose result is needed waits
// for every earlier vector memory operation of the wave, including the next
// tile's prefetch, so one per hit would stall hit-dense scans.
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
    const uint64_t *gmask;       // [n_list] groups to scan per listed sequence (nullptr: all)
    uint32_t *hits;              // ah_hit records, 3 words each
    uint64_t hit_cap;
    uint64_t *n_hits;
};

// Lane i receives lane i+1's value (lane 63: 0) / lane i-1's (lane 0: 0):
// DPP whole-wave shifts, plain vector moves instead of an LDS permute.
__device__ __forceinline__ uint32_t ah_from_next_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);  // wave_shl:1
}
__device__ __forceinline__ uint32_t ah_from_prev_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, false);  // wave_shr:1
}

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

// One block of a lane (64 positions) in both planes with its neighbours:
// word 0 = the 32 positions before it, words 1..AH_HW = the block's own,
// word AH_HW+1 = the 32 positions after it.
#define AH_HW 2  // words per plane of one block
struct AhBase {
    uint32_t h[AH_HW + 2];
    uint32_t l[AH_HW + 2];
};

// Word Wd (positions 32*Wd .. 32*Wd+31 of the lane) of a plane shifted by D
// positions (bit q = base q + D), -31 <= D <= 31: one funnel shift, none for D = 0.
template <int D, int Wd>
__device__ __forceinline__ uint32_t ah_shw(const uint32_t (&x)[AH_HW + 2]) {
    static_assert(D > -32 && D < 32, "shift out of range");
    if constexpr (D == 0) return x[Wd + 1];
    else if constexpr (D > 0) return ah_funnel(x[Wd + 2], x[Wd + 1], D);
    else return ah_funnel(x[Wd + 1], x[Wd], 32 + D);
}

// acc AND (bit q: base q + D is in IUPAC set M), from the base words
template <uint32_t M, int D, int Wd>
__device__ __forceinline__ uint32_t ah_and_at(uint32_t acc, const AhBase &b) {
    return ah_and_set<M>(acc, ah_shw<D, Wd>(b.h), ah_shw<D, Wd>(b.l));
}

// Per-tile context kept for deferred verification.
struct TileCtx {
    uint64_t gbase;  // store position (block index * 64) of the tile's first base
    uint32_t seq;
    int32_t lo;      // lowest tile-relative window start: -min(pos0, 32)
    int32_t room;    // bases from the tile start to the sequence end (capped at 2^20)
    uint32_t pos0;   // sequence position of the tile's first base
    uint32_t has_n;
    // past the sequence's first 32 bases, room for the longest window after
    // the tile's last base, no N: every window of the tile lies inside its
    // sequence and is N-free
    uint32_t plain;
};

#ifndef AH_QCAP
#define AH_QCAP 319                       // queue entries per wave: < 64 left over + 4 x 64 of one group (one spare follows)
#endif
#ifndef AH_NCTX
// tiles whose candidates may wait in the queue (<= 4); with two-block tiles
// one (its context then stays in scalar registers; a second tile's ring
// words and context would cost a workgroup per CU)
#define AH_NCTX (AH_BPL == 1 ? 2 : 1)
#endif
#ifndef AH_HCAP
#define AH_HCAP 48                        // hits buffered per wave (LDS) before one atomic reserves their room
#endif
#define AH_TW (2 * AH_TILE_BLOCKS + 2)    // {h, l} ring words of a tile (+ one word each side)
#define AH_QW (AH_HW + 1)                 // queue entry: one block's candidate words + tag
// N-bitmap words covering the tile's blocks and one block on each side
#define AH_NBW ((AH_TILE_BLOCKS + 2 + 31) / 32 + 1)

__device__ __forceinline__ uint32_t ah_uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t ah_uni64(uint64_t x) {
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32) |
           __builtin_amdgcn_readfirstlane((uint32_t)x);
}

// Sequence cursor over the tile list of one wave (wave-uniform values).
// Tiles are counted from a first tile t0 in 32 bits (the walk covers at most
// 2^31 tiles from it), so the per-tile walk needs no 64-bit compares.
struct SeqCursor {
    uint32_t i;        // list index
    uint32_t seq;
    uint32_t len;
    uint32_t nblk;
    uint64_t blk0;
    uint64_t t0;       // the walk's first tile
    uint32_t d;        // tile_pref[i] - t0 (mod 2^32): tile r is the sequence's tile r - d
    uint32_t r1;       // tile_pref[i + 1] - t0, capped at 2^32 - 1: the first tile past the sequence
    uint64_t gm;       // groups scanned on this sequence (bit g)

    __device__ void load(const ScanArgs &a) {
        seq = ah_uni(a.list ? a.list[i] : i);
        gm = a.gmask ? ah_uni64(a.gmask[i]) : ~0ull;
        // a listed index outside the store has no tiles (the tile table gives
        // it none) and its per-sequence entries are never read
        const bool in_store = seq < a.st.n_seqs;
        len = in_store ? ah_uni(a.st.d_seq_len[seq]) : 0u;
        nblk = (len + 63u) / 64u;
        blk0 = in_store ? ah_uni64(a.st.d_seq_block0[seq]) : 0ull;
        const uint64_t tp0 = ah_uni64(a.tile_pref[i]), tp1 = ah_uni64(a.tile_pref[i + 1]);
        d = (uint32_t)(tp0 - t0);
        r1 = tp1 - t0 < 0xFFFFFFFFull ? (uint32_t)(tp1 - t0) : 0xFFFFFFFFu;  // tp1 > t0 once loaded
    }
    // the sequence holding tile t, which becomes the walk's first
    __device__ void init(const ScanArgs &a, uint64_t t) {
        t0 = t;
        uint32_t lo = 0, hi = a.n_list;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ah_uni64(a.tile_pref[mid]) <= t) lo = mid;
            else hi = mid;
        }
        i = lo;
        load(a);
    }
    // move to the sequence holding tile r (r >= the current one's first)
    __device__ void advance(const ScanArgs &a, uint32_t r) {
        while (r >= r1) {
            i++;
            load(a);
        }
    }
};

// What one tile needs from global memory, issued one tile ahead.  The loads
// are unconditional (addresses clamped into the sequence) so they stay in
// flight until the next iteration uses them.
struct TileLoad {
    uint4 blk[AH_BPL];  // this lane's blocks (lanes past the end repeat the last one)
    uint4 hal;       // lane 0: the block before the tile; lane 63: the block after it
    uint32_t nbw;    // lanes 0..AH_NBW-1: the N-bitmap words around the tile
    uint32_t nb;     // blocks in the tile (uniform)
    uint32_t rel0;   // first block of the tile within its sequence (uniform)
    uint64_t gb0;    // store block of the tile's first block (uniform)
};

__device__ __forceinline__ void tile_issue(const ScanArgs &a, const SeqCursor &c, uint32_t r, TileLoad &L) {
    const uint32_t lane = ah_lane();
    L.rel0 = (r - c.d) * AH_TILE_BLOCKS;
    const uint32_t left = c.nblk - L.rel0;
    L.nb = left < AH_TILE_BLOCKS ? left : AH_TILE_BLOCKS;
    L.gb0 = c.blk0 + L.rel0;
    // Addresses are a uniform base plus a 32-bit per-lane byte offset (one
    // vector op per load).  The base is the block before the tile (its
    // address is formed but only read when that block is in the sequence):
    // block j of the tile is at offset 1 + j, lane 0's halo is block 0 when
    // the tile has a predecessor, lane 63's halo the block after the tile.
    const uint64_t base = (uint64_t)a.st.d_blocks + 16u * (uint64_t)L.gb0 - 16u;
#pragma unroll
    for (int b = 0; b < AH_BPL; b++) {
        uint32_t own = AH_BPL * lane + b;
        own = min(own, L.nb - 1);  // one v_min: L.nb >= 1
        L.blk[b] = ah_ldg<uint4>(base + 16u * (own + 1));
    }
    uint32_t o_hal = min((uint32_t)(AH_BPL * lane), L.nb - 1) + 1;
    if (lane == 0 && L.rel0 != 0) o_hal = 0;
    if (lane == 63 && L.rel0 + AH_TILE_BLOCKS < c.nblk) o_hal = AH_TILE_BLOCKS + 1;
    L.hal = ah_ldg<uint4>(base + 16u * o_hal);
    // N-bitmap words from wb = max(gb0/32, 1) - 1 cover blocks gb0-1 ..
    // gb0+AH_TILE_BLOCKS.  A nonzero word means the tile may touch an N -- a
    // superset, which only costs exact per-block lookups in verification.
    const uint64_t q = L.gb0 >> 5;
    const uint64_t wb = q - (q != 0 ? 1u : 0u);  // max(q, 1) - 1, with scalar compares
    const uint64_t nw = (a.st.n_blocks + 31) >> 5;
    const uint32_t room = (uint32_t)(nw - 1 - wb);  // words after wb
    uint32_t wi = lane < AH_NBW - 1 ? lane : AH_NBW - 1;
    wi = wi < room ? wi : room;
    L.nbw = ah_ldg<uint32_t>((uint64_t)a.st.d_nbits + 4u * (uint64_t)wb + 4u * wi);
}

typedef __attribute__((address_space(3))) uint32_t ah_lds_u32;

// Queue entry `slot` through an LDS-qualified pointer: its address is formed
// in 32 bits (through the generic array type it is a 64-bit multiply-add).
__device__ __forceinline__ ah_lds_u32 *ah_qe(const uint32_t (*sQ)[AH_QW], uint32_t slot) {
    return (ah_lds_u32 *)&sQ[0][0] + __umul24(slot, (uint32_t)AH_QW);
}

// A wave's hit buffer in LDS: records and the count of hits accepted since
// the last write-out (those past AH_HCAP went to global memory directly).
struct HitBuf {
    uint32_t (*rec)[3];
    uint32_t *n;
};

// Append the buffered records to the hit array: one atomic reserves their
// room, the lanes copy them (consecutive records, coalesced).  Wave-wide.
__device__ __forceinline__ void ah_hits_out(const ScanArgs &a, const HitBuf &hb) {
    ah_wave_sync();
    const uint32_t cnt = ah_uni(*hb.n);
    const uint32_t n = cnt < AH_HCAP ? cnt : AH_HCAP;
    if (n) {
        uint64_t base = 0;
        if (ah_lane() == 0) base = atomicAdd((unsigned long long *)a.n_hits, (unsigned long long)n);
        base = ah_uni64(base);
        for (uint32_t i = ah_lane(); i < n; i += 64) {
            if (base + i < a.hit_cap) {
                uint32_t *r = a.hits + 3 * (base + i);
                r[0] = hb.rec[i][0];
                r[1] = hb.rec[i][1];
                r[2] = hb.rec[i][2];
            }
        }
        ah_wave_sync();
        if (ah_lane() == 0) *hb.n = 0u;
        ah_wave_sync();
    }
}

// Block i of the lane's loaded blocks by selection, not by indexing: where the
// block loop stays rolled (many pattern groups make its body too large to
// unroll), an indexed register array would be kept in scratch memory.
static_assert(AH_BPL == 1 || AH_BPL == 2, "one or two blocks per lane");
__device__ __forceinline__ uint4 ah_blk_at(const TileLoad &L, int i) {
    return (AH_BPL == 1 || i == 0) ? L.blk[0] : L.blk[AH_BPL - 1];
}

// Any N in the tile's blocks or its halo blocks (wave-uniform, conservative).
__device__ __forceinline__ bool tile_has_n(const TileLoad &L) { return __ballot(L.nbw != 0) != 0; }

template <bool kLdsOnly>
__device__ __forceinline__ void ah_pattern_record(const ScanArgs &a, const DPat *sPat, uint32_t n_lds, uint32_t X,
                                                  uint4 &p0, uint4 &p1) {
    // With every record in LDS no global load is issued here: a global load
    // in the verification path would have to wait for the next tile's
    // prefetch as well (the vector memory counter is in order).
    if (kLdsOnly || X < n_lds) {
        p0 = ah_lds<uint4>(&sPat[X].P[0]);
        p1 = ah_lds<uint4>(&sPat[X].clampmask);
    } else {
        p0 = ah_ldg<uint4>(&a.pats[X].P[0]);
        p1 = ah_ldg<uint4>(&a.pats[X].clampmask);
    }
}

// Test one candidate window (start pl, tile-relative) against its pattern
// record and buffer it as a hit: hW/lW = the window's plane words, nW = its
// N positions.
__device__ __forceinline__ void ah_window_hit(const ScanArgs &a, const HitBuf &hb, const TileCtx &c, const uint4 &p0,
                                              const uint4 &p1, uint32_t k, int32_t pl, uint32_t hW, uint32_t lW,
                                              uint32_t nW) {
    const uint32_t lo = (lW & p0.y) | (~lW & p0.x);  // C : A
    const uint32_t hi = (lW & p0.w) | (~lW & p0.z);  // T : G
    const uint32_t matched = ((hW & hi) | (~hW & lo)) & ~nW & p1.y;
    const uint32_t nmm = __popc(p1.y & ~matched);
    if ((matched & p1.x) == p1.x && nmm <= k) {
        const uint32_t pos = (uint32_t)((int64_t)c.pos0 + pl), w2 = p1.w | (nmm << 24);
        const uint32_t slot = atomicAdd(hb.n, 1u);  // LDS
        if (slot < AH_HCAP) {
            // through an LDS-qualified pointer: a generic one becomes
            // a FLAT store, which makes every later wait a full drain
            ah_lds_u32 *r = (ah_lds_u32 *)&hb.rec[slot][0];
            r[0] = c.seq;
            r[1] = pos;
            r[2] = w2;
        } else {  // buffer full: straight to the hit array
            const uint64_t h = atomicAdd((unsigned long long *)a.n_hits, 1ull);
            if (h < a.hit_cap) {
                uint32_t *r = a.hits + 3 * h;
                r[0] = c.seq;
                r[1] = pos;
                r[2] = w2;
            }
        }
    }
}

// Verify queued entries [e0, e1) (at most 64).  Entry = {candidate words
// 0..AH_HW-1 (bit q of word w: clamp site 32w+q of one block of the lane),
// X << 9 | block << 8 | ctx << 6 | lane}; windows are read from the tile
// words kept in LDS (sW[ctx][word] = {h, l}).  A round of at most 32 (16)
// entries gives each entry 2 (4) lanes, each taking a contiguous share of
// its candidate bits: the round lasts as long as its busiest lane's bit
// walk, and most entries hold one or two bits.
template <bool kLdsOnly>
__device__ void ah_verify_round(const ScanArgs &a, const DPat *sPat, uint32_t n_lds, const TileCtx *sCtx,
                                const TileCtx &rctx, const uint32_t (*sQ)[AH_QW], uint32_t e0, uint32_t e1,
                                const uint2 (*sW)[AH_TW], const HitBuf &hb) {
    const uint32_t n = e1 - e0;  // wave-uniform
    const uint32_t lg = n <= 16u ? 2u : (n <= 32u ? 1u : 0u);
    const uint32_t lane = ah_lane();
    const uint32_t e = e0 + (lane >> lg);
    if (e >= e1) return;
    const ah_lds_u32 *qe = ah_qe(sQ, e);
    uint64_t mm64 = ((uint64_t)qe[1] << 32) | qe[0];
    if (lg) {
        const uint32_t part = 64u >> lg, sub = lane & ((1u << lg) - 1u);
        mm64 &= (~0ull >> (64u - part)) << (part * sub);
    }
    const uint32_t tag = qe[AH_HW];
    const uint32_t X = tag >> 9, blk = (tag >> 8) & 1u, ci = (tag >> 6) & 3u, ln = tag & 63u;
    // with one tile in the ring its context is wave-uniform (scalar registers)
    const TileCtx c = AH_NCTX == 1 ? rctx : sCtx[ci];
    uint4 p0, p1;
    ah_pattern_record<kLdsOnly>(a, sPat, n_lds, X, p0, p1);
    const uint32_t L = p1.z & 0xFFu, k = (p1.z >> 8) & 0xFFu, shift = p1.z >> 24;
    const uint2 *W = sW[ci];
    // window start of bit 0 (tile-relative; shift <= 31, so >= -31)
    const int32_t lane0 = (int32_t)(64 * (AH_BPL * ln + blk)) - (int32_t)shift;
    // a plain tile (wave-uniform with one tile in the ring): the walk needs
    // no bounds or N tests
    if (AH_NCTX == 1 && c.plain) {
        const uint32_t r0 = (uint32_t)(lane0 + 32);  // ring position of bit 0's window
        while (mm64) {
            const uint32_t bit = (uint32_t)__ffsll((unsigned long long)mm64) - 1;
            mm64 &= mm64 - 1;
            const uint32_t idx = r0 + bit;
            const uint2 u = W[idx >> 5], v = W[(idx >> 5) + 1];
            ah_window_hit(a, hb, c, p0, p1, k, (int32_t)idx - 32, ah_funnel(v.x, u.x, idx & 31u),
                          ah_funnel(v.y, u.y, idx & 31u), 0u);
        }
        return;
    }
    // window starts (tile-relative) allowed by the sequence bounds
    const int32_t lo_ok = c.lo;
    const int32_t hi_ok = c.room - (int32_t)L;
    while (mm64) {
        const uint32_t bit = (uint32_t)__ffsll((unsigned long long)mm64) - 1;
        mm64 &= mm64 - 1;
        const int32_t pl = lane0 + (int32_t)bit;  // window start, tile-relative
        if (pl < lo_ok || pl > hi_ok) continue;
        const uint32_t idx = (uint32_t)(pl + 32);
        const uint32_t w = idx >> 5, off = idx & 31u;
        const uint2 u = W[w], v = W[w + 1];
        uint32_t nW = 0;
        if (c.has_n) {
            const uint64_t gp = c.gbase + (uint64_t)(int64_t)pl;
            const uint64_t ba = gp >> 6, bb = (gp + L - 1) >> 6;
            const uint32_t o = (uint32_t)(gp & 63);
            uint64_t nm = ah_block_nmask(a.st, ba) >> o;
            if (bb != ba && o) nm |= ah_block_nmask(a.st, bb) << (64 - o);
            nW = (uint32_t)nm;
        }
        ah_window_hit(a, hb, c, p0, p1, k, pl, ah_funnel(v.x, u.x, off), ah_funnel(v.y, u.y, off), nW);
    }
}

// Verify whole rounds of 64 queued entries; with drain, also the remainder.
// Entries left over move to the front of the queue.
template <bool kLdsOnly>
__device__ __forceinline__ void ah_flush(const ScanArgs &a, const DPat *sPat, uint32_t n_lds, const TileCtx *sCtx,
                                         const TileCtx &rctx,
                                         uint32_t (*sQ)[AH_QW], uint32_t &qn, const uint2 (*sW)[AH_TW],
                                         const HitBuf &hb, bool drain) {
    ah_wave_sync();
    uint32_t e0 = 0;
    for (; e0 + 64 <= qn; e0 += 64) ah_verify_round<kLdsOnly>(a, sPat, n_lds, sCtx, rctx, sQ, e0, e0 + 64, sW, hb);
    if (drain) {
        if (e0 < qn) ah_verify_round<kLdsOnly>(a, sPat, n_lds, sCtx, rctx, sQ, e0, qn, sW, hb);
        qn = 0u;
    } else if (e0 > 0) {
        const uint32_t rest = qn - e0;  // < 64
        const uint32_t lane = ah_lane();
        uint32_t v[AH_QW];
        if (lane < rest) {
#pragma unroll
            for (int j = 0; j < AH_QW; j++) v[j] = ah_qe(sQ, e0 + lane)[j];
        }
        ah_wave_sync();
        if (lane < rest) {
#pragma unroll
            for (int j = 0; j < AH_QW; j++) ah_qe(sQ, lane)[j] = v[j];
        }
        qn = ah_uni(rest);
    }
    ah_wave_sync();
}

// One tile, its blocks already loaded into L: record its context and words
// for deferred verification, filter every pattern group, queue candidates,
// and verify full rounds of queued candidates.
template <bool kLdsOnly, class F>
__device__ __forceinline__ void ah_tile(const ScanArgs &a, F &f, const DPat *sPat, uint32_t n_lds, TileCtx *sCtx,
                                        TileCtx &rctx, uint32_t (*sQ)[AH_QW], uint2 (*sW)[AH_TW],
                                        const HitBuf &hb, const TileLoad &L, const SeqCursor &cur, uint32_t groups,
                                        uint32_t &qn, uint32_t &nctx) {
    const uint32_t lane = ah_lane();
    if (nctx == AH_NCTX) {  // every context slot is referenced: verify all
        ah_flush<kLdsOnly>(a, sPat, n_lds, sCtx, rctx, sQ, qn, sW, hb, true);
        nctx = 0;
    }
    // buffered hits so far, read here and tested after the filter
    const uint32_t hits_buffered = ah_lds<uint32_t>(hb.n);
    const uint32_t ci = nctx;
    nctx = ah_uni(nctx + 1);
    TileCtx c;  // wave-uniform
    c.gbase = L.gb0 * 64;
    c.seq = cur.seq;
    c.pos0 = L.rel0 * 64;
    c.lo = -(int32_t)(c.pos0 < 32u ? c.pos0 : 32u);
    const uint32_t rest = cur.len - c.pos0;
    c.room = (int32_t)(rest < (1u << 20) ? rest : (1u << 20));
    c.has_n = tile_has_n(L);
    c.plain = c.lo == -32 && c.room >= 64 * AH_TILE_BLOCKS + 32 && !c.has_n;
    if (AH_NCTX == 1) rctx = c;
    else if (lane == 0) sCtx[ci] = c;
    // the tile's words for deferred verification: [0] the 32 positions
    // before the tile, then every lane's blocks in order, then the 32 after
    uint2 *W = sW[ci];
    // the lane after's first words (lane 63: the block after the tile)
    uint32_t nxh = ah_from_next_lane(L.blk[0].x), nxl = ah_from_next_lane(L.blk[0].y);
    if (lane == 63) {
        nxh = L.hal.x;
        nxl = L.hal.y;
    }
    // the halo words without a branch: lane 0 the word before the tile, lane
    // 63 the word after it; every other lane writes its own first word,
    // which its block writes below then overwrite (one wave's LDS writes
    // land in order)
    W[lane == 0 ? 0 : (lane == 63 ? AH_TW - 1 : 1 + AH_NW * lane)] =
        lane == 0 ? make_uint2(L.hal.z, L.hal.w) : make_uint2(nxh, nxl);
#pragma unroll
    for (int b = 0; b < AH_BPL; b++) {
        W[1 + AH_NW * lane + 2 * b] = make_uint2(L.blk[b].x, L.blk[b].y);
        W[2 + AH_NW * lane + 2 * b] = make_uint2(L.blk[b].z, L.blk[b].w);
    }
#pragma unroll
    for (int blk = 0; blk < AH_BPL; blk++) {
        // the block's words and their neighbours
        AhBase B;
        const uint4 cb = ah_blk_at(L, blk);
        B.h[1] = cb.x;
        B.l[1] = cb.y;
        B.h[2] = cb.z;
        B.l[2] = cb.w;
        const uint4 nb = ah_blk_at(L, blk + 1 < AH_BPL ? blk + 1 : 0);
        B.h[3] = blk + 1 < AH_BPL ? nb.x : nxh;
        B.l[3] = blk + 1 < AH_BPL ? nb.y : nxl;
        B.h[0] = B.l[0] = 0u;
        if (F::kUsesBase) {
            // the 32 positions before (lane 0's first block: the block before
            // the tile; at a sequence start they are another sequence's or
            // padding, which only windows that verification rejects can see)
            if (blk > 0) {
                const uint4 pb = ah_blk_at(L, blk > 0 ? blk - 1 : 0);
                B.h[0] = pb.z;
                B.l[0] = pb.w;
            } else {
                B.h[0] = ah_from_prev_lane(L.blk[AH_BPL - 1].z);
                B.l[0] = ah_from_prev_lane(L.blk[AH_BPL - 1].w);
                if (lane == 0) {
                    B.h[0] = L.hal.z;
                    B.l[0] = L.hal.w;
                }
            }
        }
        // Lanes past the sequence end hold repeated blocks; their candidates
        // are windows past the end, which verification rejects, so no lane
        // mask.  bit q of S*[i][w]: plane bit of base 32w + q + i of the
        // block; only the F::kW offsets the filter reads are formed
        uint32_t Sh[AH_WMAX][AH_HW], Sl[AH_WMAX][AH_HW];
#pragma unroll
        for (int i = 0; i < F::kW; i++) {
#pragma unroll
            for (int w = 0; w < AH_HW; w++) {
                Sh[i][w] = ah_funnel(B.h[w + 2], B.h[w + 1], i);
                Sl[i][w] = ah_funnel(B.l[w + 2], B.l[w + 1], i);
            }
        }
        // kHalves = 2: the plus-strand patterns of every group (x = 0, 1),
        // then the minus-strand ones (x = 2, 3), each pass with the filter's
        // own shifted planes for that strand, shared by all groups
        constexpr int kX = 4 / F::kHalves;  // patterns per group and pass
        constexpr int kG = F::kGroupStep;   // groups per filter call
        for (int half = 0; half < F::kHalves; half++) {
            f.block(B, half);
            for (uint32_t g0 = 0; g0 < groups; g0 += kG) {
                // groups asked for on this sequence (all past the first 64)
                const uint32_t req =
                    g0 < 64 ? (uint32_t)(cur.gm >> g0) & ((1u << kG) - 1u) : (1u << kG) - 1u;
                if (!req) continue;
                // Mark the shifted planes as redefined in every iteration (an
                // empty asm, no instruction): otherwise, with compile-time
                // codes, the compiler hoists every group's set tests out of
                // this loop as invariants and runs out of registers once there
                // are many groups.
                if (F::kHoistGuard) {
#pragma unroll
                    for (int i = 0; i < F::kW; i++)
#pragma unroll
                        for (int w = 0; w < AH_HW; w++) asm volatile("" : "+v"(Sh[i][w]), "+v"(Sl[i][w]));
                    if (F::kUsesBase) {
#pragma unroll
                        for (int w = 0; w < AH_HW + 2; w++) asm volatile("" : "+v"(B.h[w]), "+v"(B.l[w]));
                    }
                    f.guard();
                }
                // C[(kX * gi + xi) * AH_HW + w]: clamp sites of word w, group
                // g0 + gi, pattern kX * half + xi
                uint32_t C[kG * kX * AH_HW];
                f.filter(g0, half, B, Sh, Sl, C);
                if (F::kSkipEmpty) {  // many groups: most have no candidate in a block
                    uint32_t any = 0;
#pragma unroll
                    for (int j = 0; j < kG * kX * AH_HW; j++) any |= C[j];
                    if (__ballot(any != 0) == 0) continue;
                }
#pragma unroll
                for (int gi = 0; gi < kG; gi++) {
                    if (!((req >> gi) & 1u)) continue;
                    const uint32_t g = g0 + (uint32_t)gi;
                    // room for this group's entries (at most kX x 64); a
                    // non-draining flush leaves fewer than 64
                    if (qn > AH_QCAP - 64 * kX) ah_flush<kLdsOnly>(a, sPat, n_lds, sCtx, rctx, sQ, qn, sW, hb, false);
#pragma unroll
                    for (int xi = 0; xi < kX; xi++) {
                        uint32_t nzw = 0;
#pragma unroll
                        for (int w = 0; w < AH_HW; w++) nzw |= C[(kX * gi + xi) * AH_HW + w];
                        const bool nz = nzw != 0;
                        const uint64_t bal = __ballot(nz);
                        // With all four patterns in one pass every lane writes,
                        // without a branch, lanes without candidates all to the
                        // one spare entry past the queue (fewer scalar
                        // instructions, 2% faster); in the many-pair kernel only
                        // the lanes with candidates write (the same time with 15%
                        // fewer VALU instructions).
                        const uint32_t x = (uint32_t)(kX * half + xi);
                        // (the lane count is taken outside the select: it is a
                        // cross-lane operation, which a select would turn into a
                        // masked branch)
                        const uint32_t m = F::kHalves == 1 ? ah_mbcnt(bal) : 0u;
                        if (F::kHalves == 1 || nz) {
                            // entry qn + (lane count): the wave-uniform start
                            // plus one 24-bit multiply-add per lane
                            ah_lds_u32 *qe = F::kHalves == 1
                                                 ? (nz ? ah_qe(sQ, qn) + __umul24(m, (uint32_t)AH_QW)
                                                       : ah_qe(sQ, AH_QCAP))
                                                 : ah_qe(sQ, qn) + __umul24(ah_mbcnt(bal), (uint32_t)AH_QW);
#pragma unroll
                            for (int w = 0; w < AH_HW; w++) qe[w] = C[(kX * gi + xi) * AH_HW + w];
                            qe[AH_HW] = ((4 * g + x) << 9) | ((uint32_t)blk << 8) | (ci << 6) | lane;
                        }
                        qn = ah_uni(qn + (uint32_t)__popcll(bal));  // keeps the queue count in a scalar register
                    }
                }
            }
        }
    }
    if (qn >= 64) ah_flush<kLdsOnly>(a, sPat, n_lds, sCtx, rctx, sQ, qn, sW, hb, false);
    if (ah_uni(hits_buffered) >= AH_HCAP / 2) ah_hits_out(a, hb);
}

// The kernel body.  Filter F provides
//   f.groups(a)                         number of pattern groups (primer pairs),
//   f.block(B, half), f.guard()         per-block state of pass `half` (shifted
//                                       planes shared by every group) and its
//                                       hoist guard,
//   f.filter(g0, half, B, Sh, Sl, C)    candidate words of groups g0.. in one block
//                                       (C[AH_HW*xi + w]: clamp sites 32w..32w+31
//                                       of the block, pattern 4/kHalves*half + xi);
//                                       a candidate must pass a necessary
//                                       condition of a hit; verification decides.
//   F::kHalves                          passes per block: 1 (all four patterns of
//                                       a group at once) or 2 (plus, then minus),
//   F::kGroupStep                       groups per filter call (C holds kGroupStep
//                                       groups' words, group after group; groups
//                                       past the last give zero words),
//   F::kUsesBase                        whether filter reads the base words B,
//   F::kW                               shifted planes it reads (offsets 0 .. kW-1),
//   F::kHoistGuard                      its codes are compile-time and there are
//                                       several groups (see the group loop),
//   F::kSkipEmpty                       test for a group without candidates first.
// n_lds: pattern records staged in sPat; kLdsOnly: n_lds covers every record.
template <bool kLdsOnly, class F>
__device__ __forceinline__ void ah_scan_body(const ScanArgs &a, F &f, const DPat *sPat, uint32_t n_lds,
                                             TileCtx (*sCtx_all)[AH_NCTX], uint32_t (*sQ_all)[AH_QCAP + 1][AH_QW],
                                             uint2 (*sW_all)[AH_NCTX][AH_TW],
                                             uint32_t (*sH_all)[AH_HCAP][3], uint32_t *sHn_all) {
    // the wave index is uniform across the wave; saying so keeps the tile
    // walk, the cursor and the queue bookkeeping in scalar registers
    const uint32_t wv = ah_uni(threadIdx.x >> 6);
    TileCtx *sCtx = sCtx_all[wv];
    uint32_t(*sQ)[AH_QW] = sQ_all[wv];
    uint2(*sW)[AH_TW] = sW_all[wv];
    const HitBuf hb{sH_all[wv], sHn_all + wv};
    if (ah_lane() == 0) *hb.n = 0u;
    ah_wave_sync();
    const uint64_t total = ah_uni64(a.tile_pref[a.n_list]);
    // XCD-aware numbering: workgroup i runs on XCD i % 8, so give each XCD a
    // contiguous share of the tiles.
    const uint32_t nwg = gridDim.x;
    const uint32_t wg = (nwg % 8 == 0) ? (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8 : blockIdx.x;
    const uint64_t nw = (uint64_t)nwg * 4, gw = (uint64_t)wg * 4 + wv;
    const uint64_t per = (total + nw - 1) / nw;
    const uint64_t t0 = gw * per;
    if (t0 >= total) return;
    const uint64_t tend = t0 + per < total ? t0 + per : total;

    const uint32_t groups = f.groups(a);
    uint32_t qn = 0, nctx = 0;
    TileCtx rctx{};  // the ring tile's context when the ring holds one tile
    // The wave's tiles in segments of at most 2^31 (one segment in practice),
    // each walked with 32-bit tile counts.
    for (uint64_t s0 = t0; s0 < tend; s0 += (1ull << 31)) {
    const uint32_t nt = (uint32_t)(tend - s0 < (1ull << 31) ? tend - s0 : (1ull << 31));
    SeqCursor cur;
    cur.init(a, s0);
    // Two load sets used in turn: the next tile's loads go to the set not being
    // processed, so no register copy (which would wait for them) is needed.
    // The last tile reloads itself, so the loads are unconditional.
    TileLoad A, B;
    tile_issue(a, cur, 0u, A);
    for (uint32_t r = 0;;) {
        uint32_t rn = r + 1 < nt ? r + 1 : r;
        SeqCursor nc = cur;
        nc.advance(a, rn);
        tile_issue(a, nc, rn, B);
        ah_tile<kLdsOnly>(a, f, sPat, n_lds, sCtx, rctx, sQ, sW, hb, A, cur, groups, qn, nctx);
        cur = nc;
        if (++r >= nt) break;
        rn = r + 1 < nt ? r + 1 : r;
        nc = cur;
        nc.advance(a, rn);
        tile_issue(a, nc, rn, A);
        ah_tile<kLdsOnly>(a, f, sPat, n_lds, sCtx, rctx, sQ, sW, hb, B, cur, groups, qn, nctx);
        cur = nc;
        if (++r >= nt) break;
    }
    }
    if (qn) ah_flush<kLdsOnly>(a, sPat, n_lds, sCtx, rctx, sQ, qn, sW, hb, true);
    ah_hits_out(a, hb);
}

// Stage the first n pattern records in LDS (all threads of the block).
__device__ __forceinline__ void ah_stage_patterns(const ScanArgs &a, DPat *sPat, uint32_t cap) {
    const uint32_t n = a.n_pats < cap ? a.n_pats : cap;
    const uint4 *src = (const uint4 *)a.pats;
    uint4 *dst = (uint4 *)sPat;
    for (uint32_t i = threadIdx.x; i < n * 3; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}
