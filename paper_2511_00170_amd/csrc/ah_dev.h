// Device-visible types and helpers of libah.so.  Self-contained so that the
// same text can be compiled by hipcc and, for primer-set specialised scan
// kernels, by hipRTC at run time.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::uint16_t uint16_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::uint64_t uint64_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::int64_t int64_t;
#endif

#include "ah.h"

// Pre-filter width: at most this many clamp positions are tested with
// bit-parallel word operations before a candidate window is verified.
#define AH_WMAX 6
// A scan tile is 64 lanes x AH_BPL blocks of 64 bases.
#ifndef AH_BPL
#define AH_BPL 1                              // 64-base blocks per lane in the scan
#endif
#define AH_NW (2 * AH_BPL)                    // 32-bit words per lane and bit plane
#define AH_TILE_BLOCKS (64 * AH_BPL)
#define AH_TILE_BASES (AH_TILE_BLOCKS * 64)
#define AH_MAXL 32
// Variants per primer the Tm kernel will enumerate.
#define AH_MAX_VARIANTS (1u << 24)
// Entries of each of the two half tables of a primer's variants (the Tm
// kernel builds variant v from two loads instead of a walk over the
// degenerate positions, for up to AH_VARTAB^2 variants).
#define AH_VARTAB 64

// One oriented pattern: pair q, kind (bit0 reverse primer, bit1 minus strand).
struct alignas(16) DPat {
    uint32_t P[4];       // bit j: base A/C/G/T allowed at pattern position j
    uint32_t clampmask;  // positions that must match
    uint32_t lmask;      // bits [0, L)
    uint32_t meta;       // L | k << 8 | W << 16 | shift << 24
    uint32_t pk;         // pair | kind << 16
    uint8_t fcode[8];    // IUPAC sets of the W filter positions, from the clamp site on
    uint32_t pad[2];
};
static_assert(sizeof(DPat) == 48, "DPat layout");

// One primer for Tm variant enumeration.
struct DPrimer {
    uint8_t L;
    uint8_t n_deg;           // degenerate positions
    uint8_t pad[2];
    uint32_t D;              // number of concrete variants (<= AH_MAX_VARIANTS)
    uint64_t base;           // code[j] at bits 2j: the first variant
    uint8_t code[AH_MAXL];   // 2-bit base of each concrete position
    uint8_t deg_pos[AH_MAXL];
    uint8_t deg_n[AH_MAXL];
    uint8_t deg_base[AH_MAXL][4];
    // Variant v = a * rb + b (b indexes the last degenerate positions, which
    // vary fastest) has the codes hi[a] | lo[b]: lo holds the codes of those
    // last positions, hi every other position.  rb = 0: no split with both
    // halves within AH_VARTAB entries; variants are enumerated on the fly.
    uint32_t rb;
    uint32_t ra;
    uint64_t lo[AH_VARTAB];
    uint64_t hi[AH_VARTAB];
};

// Variant v of a degenerate primer as 2-bit codes (base j at bits 2j): v in
// mixed radix over the degenerate positions, the last one varying fastest.
// The host fills the half tables with it; the Tm kernel calls it when the
// primer has no split.
__host__ __device__ inline uint64_t primer_variant(const DPrimer &P, uint64_t base, uint32_t v) {
    uint64_t V = base;
    for (int d = P.n_deg - 1; d >= 0; d--) {
        const uint32_t n = P.deg_n[d];
        uint32_t q, digit;
        if (n == 2) { q = v >> 1; digit = v & 1u; }
        else if (n == 4) { q = v >> 2; digit = v & 3u; }
        else { q = v / 3u; digit = v - 3u * q; }
        v = q;
        const int pos = P.deg_pos[d];
        V = (V & ~(3ull << (2 * pos))) | ((uint64_t)P.deg_base[d][digit] << (2 * pos));
    }
    return V;
}

struct DPair {
    uint32_t min_len, max_len;
    uint8_t Lf, Lr, k, clamp;
    DPrimer prim[2];  // 0 forward, 1 reverse
};

__device__ __forceinline__ uint32_t ah_lane() { return __lane_id(); }

// Letter of 2-bit code c (0..3 = A, C, G, T) from a packed constant: indexing
// a string literal instead is a dependent global load per byte.
__device__ __forceinline__ char ah_letter(uint32_t c) { return (char)((0x54474341u >> (8u * c)) & 0xFFu); }

// Load through a pointer marked global.  A pointer made from an integer is
// generic and compiles to a FLAT load, which also counts against the LDS
// counter: every later wait for an LDS or cross-lane result would then wait
// for that load too, so a load issued one tile ahead would not overlap.
// uint4 goes through a plain vector type (its class type cannot be copied
// out of an address-space-qualified object).
typedef uint32_t ah_v4u __attribute__((ext_vector_type(4)));
template <typename T>
struct AhLoadAs {
    typedef T raw;
    __device__ static T cvt(raw v) { return v; }
};
template <>
struct AhLoadAs<uint4> {
    typedef ah_v4u raw;
    __device__ static uint4 cvt(ah_v4u v) { return make_uint4(v.x, v.y, v.z, v.w); }
};
template <typename T>
__device__ __forceinline__ T ah_ldg(const void *p) {
    return AhLoadAs<T>::cvt(*(const __attribute__((address_space(1))) typename AhLoadAs<T>::raw *)p);
}
template <typename T>
__device__ __forceinline__ T ah_ldg(uint64_t addr) {
    return ah_ldg<T>((const void *)addr);
}
// Load from LDS through a pointer marked local (p must point into LDS).  With
// one load per address space, a choice between an LDS and a global record
// stays two loads instead of being merged into one FLAT load of either.
template <typename T>
__device__ __forceinline__ T ah_lds(const void *p) {
    return AhLoadAs<T>::cvt(*(const __attribute__((address_space(3))) typename AhLoadAs<T>::raw *)p);
}

__device__ __forceinline__ uint32_t ah_mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T ah_wave_incl_sum(T v) {
    const uint32_t lane = ah_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T u = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += u;
    }
    return v;
}

// A wave-local ordering point for LDS written by one lane and read by another.
__device__ __forceinline__ void ah_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// N-side-table lookup: 64-bit mask of N positions of block b (0 if none).
__device__ __forceinline__ uint64_t ah_block_nmask(const ah_store &st, uint64_t b) {
    uint32_t w = st.d_nbits[b >> 5];
    uint32_t bit = 1u << (b & 31);
    if (!(w & bit)) return 0;
    uint64_t r = (uint64_t)st.d_nrank[b >> 5] + __popc(w & (bit - 1));
    return r < st.nmask_cap ? st.d_nmask[r] : ~0ull;
}
