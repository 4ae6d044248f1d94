// Amplicon sequences, primer trimming and flanking barcodes (Supplementary,
// "Primer trimming and barcode extraction", "Amplicon calling and
// orientation": RF amplicons are reverse-complemented; "Headers and
// outputs": matched primer snippets and fb/rb in the header).
//
// Two passes: per-amplicon output sizes -> exclusive scan -> one wavefront
// per amplicon decodes its bases from the 2-bit store and writes them with
// consecutive lanes on consecutive bytes.
#include "ah_internal.h"
#include "ah_scan_impl.h"

struct AmpGeom {
    uint32_t seq, start, end, pair, orient;
    uint32_t Ll, Lr;  // lengths of the upstream and downstream primers
    int lp, rp;       // upstream / downstream primer: 0 forward, 1 reverse
};

__device__ __forceinline__ AmpGeom amp_geom(const uint32_t *amps, uint64_t i, const DPair *pairs) {
    AmpGeom g;
    g.seq = amps[4 * i];
    g.start = amps[4 * i + 1];
    g.end = amps[4 * i + 2];
    g.pair = amps[4 * i + 3] & 0xFFFFu;
    g.orient = (amps[4 * i + 3] >> 16) & 0xFFu;
    g.lp = (g.orient == 0 || g.orient == 2) ? 0 : 1;
    g.rp = (g.orient == 0 || g.orient == 3) ? 1 : 0;
    g.Ll = g.lp ? pairs[g.pair].Lr : pairs[g.pair].Lf;
    g.Lr = g.rp ? pairs[g.pair].Lr : pairs[g.pair].Lf;
    return g;
}

__device__ __forceinline__ void amp_span(const AmpGeom &g, uint32_t trim, uint64_t *a0, uint64_t *a1) {
    if (trim) {
        *a0 = (uint64_t)g.start + g.Ll;
        const uint64_t e = (uint64_t)g.end - g.Lr;
        *a1 = e > *a0 ? e : *a0;
    } else {
        *a0 = g.start;
        *a1 = g.end;
    }
}

// base at position p of sequence with first block b0: 'A','C','G','T' or 'N'
__device__ __forceinline__ char base_at(const ah_store &st, uint64_t b0, uint64_t p, bool rc) {
    const uint64_t b = b0 + (p >> 6);
    const uint32_t bit = (uint32_t)(p & 63);
    const uint32_t *w = st.d_blocks + 4 * b;
    const uint32_t h = bit < 32 ? w[0] : w[2], l = bit < 32 ? w[1] : w[3];
    uint32_t c = (((h >> (bit & 31)) & 1u) << 1) | ((l >> (bit & 31)) & 1u);
    if ((ah_block_nmask(st, b) >> bit) & 1ull) return 'N';
    if (rc) c ^= 3u;
    return ah_letter(c);
}

// Base at sequence position p from blocks staged in LDS (block p/64 at
// sblk[p/64 - cb]): 'A','C','G','T' or 'N', complemented when rc.
__device__ __forceinline__ char staged_base(const uint4 *sblk, const uint64_t *snm, uint64_t cb, uint64_t p, bool rc) {
    const uint32_t k = (uint32_t)((p >> 6) - cb), bit = (uint32_t)(p & 63);
    const uint4 w = sblk[k];
    const uint32_t h = bit < 32 ? w.x : w.z, l = bit < 32 ? w.y : w.w;
    uint32_t c = (((h >> (bit & 31)) & 1u) << 1) | ((l >> (bit & 31)) & 1u);
    if (rc) c ^= 3u;
    return ((snm[k] >> bit) & 1ull) ? 'N' : ah_letter(c);
}

// Stage blocks [cb, ce) (at most 64) of a sequence (first block b0) and their
// N masks in LDS: one block per lane, all loads in flight together.  Whole
// wave; the caller's previous reads of the staging area must be done.
__device__ __forceinline__ void stage_blocks(const ah_store &st, uint64_t b0, uint64_t cb, uint64_t ce, uint4 *sblk,
                                             uint64_t *snm) {
    const uint32_t lane = ah_lane();
    ah_wave_sync();
    if (cb + lane < ce) {
        const uint64_t gb = b0 + cb + lane;
        sblk[lane] = ah_ldg<uint4>(st.d_blocks + 4 * gb);
        snm[lane] = ah_block_nmask(st, gb);
    }
    ah_wave_sync();
}

// Letters of the four sequence positions P .. P+3 (P a multiple of 4, so
// all in one 32-bit word of the staged block), byte i for position P + i,
// complemented when rc, 'N' where the N mask is set.  The 2-bit codes are
// spread into the bytes of a selector (a 24-bit multiply per plane) and one
// byte permute maps each to its letter.
__device__ __forceinline__ uint32_t staged_quad(const uint4 *sblk, const uint64_t *snm, uint64_t cb, uint64_t P,
                                                bool rc) {
    const uint32_t k = (uint32_t)((P >> 6) - cb), bit = (uint32_t)(P & 63), sh = bit & 31u;
    const uint4 w = sblk[k];
    const uint32_t h4 = ((bit < 32 ? w.x : w.z) >> sh) & 15u, l4 = ((bit < 32 ? w.y : w.w) >> sh) & 15u;
    // bit i of a 4-bit group to bit 0 of byte i
    const uint32_t spread_l = (l4 * 0x204081u) & 0x01010101u;
    const uint32_t spread_h = (h4 * 0x204081u) & 0x01010101u;
    uint32_t sel = spread_l | (spread_h << 1);  // byte i: code of position P + i
    if (rc) sel ^= 0x03030303u;
    uint32_t q = __builtin_amdgcn_perm(0u, 0x54474341u, sel);  // bytes 0..3 of "ACGT"
    const uint32_t n4 = (uint32_t)(snm[k] >> bit) & 15u;
    if (n4) {
        const uint32_t nb = ((n4 * 0x204081u) & 0x01010101u) * 0xFFu;
        q = (q & ~nb) | (0x4E4E4E4Eu & nb);
    }
    return q;
}

// Output bytes j in [j0, j1) of the span [a0, a1), forward or (rc) reverse-
// complemented (out[j] = comp(s[a1 - 1 - j])), decoded from blocks staged
// from block cb on.  Whole wave.  The positions they come from are taken in
// aligned groups of four (one per lane, consecutive lanes on consecutive
// groups); the < 4 positions before the first and after the last group go
// one byte per lane.  Nothing is written at or past seq_cap.
__device__ __forceinline__ void write_staged(const uint4 *sblk, const uint64_t *snm, uint64_t cb, uint64_t a0,
                                             uint64_t a1, bool rc, uint64_t j0, uint64_t j1, char *out, uint64_t dst0,
                                             uint64_t seq_cap) {
    if (j1 <= j0) return;
    const uint32_t lane = ah_lane();
    // positions [pl, ph) of the output range, and its whole groups [qa, qb)
    const uint64_t pl = rc ? a1 - j1 : a0 + j0, ph = rc ? a1 - j0 : a0 + j1;
    uint64_t qa = (pl + 3) & ~3ull, qb = ph & ~3ull;
    if (qa > qb) qa = qb = ph;  // no whole group: every position one by one
    auto put = [&](uint64_t p, char c) {
        const uint64_t j = rc ? a1 - 1 - p : p - a0;
        if (dst0 + j < seq_cap) out[dst0 + j] = c;
    };
    if (lane < qa - pl) put(pl + lane, staged_base(sblk, snm, cb, pl + lane, rc));
    if (lane < ph - qb && qb + lane >= qa) put(qb + lane, staged_base(sblk, snm, cb, qb + lane, rc));
    for (uint64_t P = qa + 4u * lane; P < qb; P += 256) {
        const uint32_t q = staged_quad(sblk, snm, cb, P, rc);
#pragma unroll
        for (uint32_t i = 0; i < 4; i++) put(P + i, (char)(q >> (8 * i)));
    }
}

// Bases [a0, a1) of a sequence (first block b0) to out[dst0 ..], for spans
// of any length: staged 64 blocks at a time.  Whole wave.
__device__ __forceinline__ void copy_span(const ah_store &st, uint64_t b0, uint64_t a0, uint64_t a1, bool rc,
                                          char *out, uint64_t dst0, uint64_t seq_cap, uint4 *sblk, uint64_t *snm) {
    if (a1 <= a0) return;
    const uint64_t bs = a0 >> 6, be = ((a1 - 1) >> 6) + 1;  // blocks of the span, sequence-relative
    for (uint64_t cb = bs; cb < be; cb += 64) {
        const uint64_t ce = cb + 64 < be ? cb + 64 : be;
        stage_blocks(st, b0, cb, ce, sblk, snm);
        // the chunk's positions inside the span, and their output indices
        const uint64_t p0 = cb * 64 > a0 ? cb * 64 : a0, p1 = ce * 64 < a1 ? ce * 64 : a1;
        const uint64_t j0 = rc ? a1 - p1 : p0 - a0, j1 = rc ? a1 - p0 : p1 - a0;
        write_staged(sblk, snm, cb, a0, a1, rc, j0, j1, out, dst0, seq_cap);
    }
}

// Output bytes of amplicon i (0 when it did not pass).
__device__ __forceinline__ uint64_t amp_size(const uint32_t *amps, uint64_t i, const DPair *pairs,
                                             const uint8_t *pass, uint32_t trim) {
    if (pass && !pass[i]) return 0;
    const AmpGeom g = amp_geom(amps, i, pairs);
    uint64_t a0, a1;
    amp_span(g, trim, &a0, &a1);
    return a1 - a0;
}

__global__ void ah_extract_size_kernel(const uint32_t *amps, const uint64_t *d_n, uint64_t cap, const DPair *pairs,
                                       const uint8_t *pass, uint32_t trim, uint64_t *size) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        size[i] = amp_size(amps, i, pairs, pass, trim);
}

// Exclusive prefix of the sizes in one workgroup (for up to AH_EXTRACT_ONE_WG
// amplicons), in coalesced rounds of 4 x 1024: seq_off[i], seq_off[n] =
// *n_bytes = total.
#define AH_EXTRACT_ONE_WG 65536u
__global__ void __launch_bounds__(1024) ah_extract_offsets_kernel(const uint64_t *size, const uint64_t *d_n,
                                                                  uint64_t cap, uint64_t *seq_off,
                                                                  uint64_t *n_bytes) {
    __shared__ uint64_t lds[16];
    const uint64_t n = *d_n < cap ? *d_n : cap;
    uint64_t carry = 0;
    for (uint64_t r0 = 0; r0 < n; r0 += 4 * 1024) {
        const uint64_t i0 = r0 + 4 * threadIdx.x;
        uint64_t v[4], loc = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            v[k] = i0 + k < n ? size[i0 + k] : 0;
            loc += v[k];
        }
        uint64_t tot;
        uint64_t o = carry + ah_block_excl_sum<uint64_t>(loc, lds, tot);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (i0 + k < n) seq_off[i0 + k] = o;
            o += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        seq_off[n] = carry;
        *n_bytes = carry;
    }
}

__global__ void ah_extract_tail_kernel(const uint64_t *d_n, uint64_t cap, const uint64_t *total, uint64_t *seq_off,
                                       uint64_t *n_bytes) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    seq_off[n] = *total;
    *n_bytes = *total;
}

__global__ void __launch_bounds__(256) ah_extract_write_kernel(ah_store st, uint32_t *amps, const uint64_t *d_n,
                                                               uint64_t cap, const DPair *pairs, const uint8_t *pass,
                                                               ah_extract_opts o, const uint64_t *seq_off, char *out,
                                                               uint64_t seq_cap, char *fb, char *rb, uint8_t *bc_len,
                                                               char *fpr, char *rpr) {
    __shared__ uint4 s_blk[4][64];
    __shared__ uint64_t s_nm[4][64];
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t i = blockIdx.x * (uint64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); i < n; i += nw) {
        const bool on = !pass || pass[i];
        const AmpGeom g = amp_geom(amps, i, pairs);
        const uint64_t b0 = st.d_seq_block0[g.seq];
        const uint64_t len = st.d_seq_len[g.seq];
        const bool rc = g.orient == 1;
        // barcode spans on the plus strand
        uint64_t f0, f1, r0, r1;
        if (!rc) {
            f0 = g.start >= o.fb_len ? g.start - o.fb_len : 0;
            f1 = g.start;
            r0 = g.end;
            r1 = (uint64_t)g.end + o.rb_len <= len ? (uint64_t)g.end + o.rb_len : len;
        } else {
            f0 = g.end;
            f1 = (uint64_t)g.end + o.fb_len <= len ? (uint64_t)g.end + o.fb_len : len;
            r0 = g.start >= o.rb_len ? g.start - o.rb_len : 0;
            r1 = g.start;
        }
        if (!on) f1 = f0, r1 = r0;
        const uint32_t nf = (uint32_t)(f1 - f0), nr = (uint32_t)(r1 - r0);
        // primer snippets: upstream site as read, downstream site reverse-complemented
        char *left_dst = (g.lp == 0) ? fpr + 32 * i : rpr + 32 * i;
        char *right_dst = (g.rp == 1) ? rpr + 32 * i : fpr + 32 * i;
        if (g.lp == g.rp) {
            left_dst = fpr + 32 * i;
            right_dst = rpr + 32 * i;
        }
        if (lane == 0) {
            bc_len[2 * i] = (uint8_t)nf;
            bc_len[2 * i + 1] = (uint8_t)nr;
            // flags bit 0: a barcode was clipped at a sequence end (the
            // record's last byte; amp_geom above has read the others)
            const bool clipped = on && (nf < o.fb_len || nr < o.rb_len);
            amps[4 * i + 3] = (amps[4 * i + 3] & 0x00FFFFFFu) | ((uint32_t)clipped << 24);
        }
        uint64_t a0, a1;
        amp_span(g, o.trim, &a0, &a1);
        // Everything read lies in [start - barcode, end + barcode): when that
        // window spans at most 64 blocks it is staged once and every byte is
        // decoded from LDS; otherwise per-base loads and chunked staging.
        const uint64_t pl1 = (uint64_t)g.start + g.Ll, pr0 = (uint64_t)g.end - g.Lr;  // primer sites
        uint64_t lo = f0 < r0 ? f0 : r0, hi = f1 > r1 ? f1 : r1;
        lo = lo < g.start ? lo : g.start;
        lo = lo < pr0 ? lo : pr0;
        hi = hi > g.end ? hi : g.end;
        hi = hi > pl1 ? hi : pl1;
        const uint64_t cb = lo >> 6, ce = hi > lo ? ((hi - 1) >> 6) + 1 : cb;
        uint4 *sblk = s_blk[threadIdx.x >> 6];
        uint64_t *snm = s_nm[threadIdx.x >> 6];
        if (on && ce - cb <= 64) {
            stage_blocks(st, b0, cb, ce, sblk, snm);
            for (uint32_t j = lane; j < o.fb_len; j += 64)
                fb[i * o.fb_len + j] = j < nf ? staged_base(sblk, snm, cb, rc ? f1 - 1 - j : f0 + j, rc) : 0;
            for (uint32_t j = lane; j < o.rb_len; j += 64)
                rb[i * o.rb_len + j] = j < nr ? staged_base(sblk, snm, cb, rc ? r1 - 1 - j : r0 + j, rc) : 0;
            if (lane < 32)
                left_dst[lane] = lane < g.Ll ? staged_base(sblk, snm, cb, (uint64_t)g.start + lane, false) : 0;
            else
                right_dst[lane - 32] =
                    lane - 32 < g.Lr ? staged_base(sblk, snm, cb, (uint64_t)g.end - 1 - (lane - 32), true) : 0;
            if (a1 > a0) write_staged(sblk, snm, cb, a0, a1, rc, 0, a1 - a0, out, seq_off[i], seq_cap);
            continue;
        }
        for (uint32_t j = lane; j < o.fb_len; j += 64)
            fb[i * o.fb_len + j] = j < nf ? base_at(st, b0, rc ? f1 - 1 - j : f0 + j, rc) : 0;
        for (uint32_t j = lane; j < o.rb_len; j += 64)
            rb[i * o.rb_len + j] = j < nr ? base_at(st, b0, rc ? r1 - 1 - j : r0 + j, rc) : 0;
        if (lane < 32) {
            left_dst[lane] = (on && lane < g.Ll) ? base_at(st, b0, (uint64_t)g.start + lane, false) : 0;
        } else {
            const uint32_t j = lane - 32;
            right_dst[j] = (on && j < g.Lr) ? base_at(st, b0, (uint64_t)g.end - 1 - j, true) : 0;
        }
        if (!on) continue;
        copy_span(st, b0, a0, a1, rc, out, seq_off[i], seq_cap, sblk, snm);
    }
}

struct ExtractWs {
    uint64_t *size, *partials, *total;
    uint64_t bytes;
};

static ExtractWs extract_ws(void *base, uint64_t cap) {
    ExtractWs w;
    char *p = (char *)base;
    uint64_t o = 0;
    auto take = [&](uint64_t n) {
        char *r = p ? p + o : nullptr;
        o += ah_align_up(n, 256);
        return r;
    };
    w.size = (uint64_t *)take(8 * cap);
    w.partials = (uint64_t *)take(8 * AH_SCAN_BLOCKS);
    w.total = (uint64_t *)take(16);
    w.bytes = o;
    return w;
}

extern "C" ah_status ah_extract_ws_size(uint64_t amp_cap, uint64_t *bytes) {
    if (!bytes) return AH_E_ARG;
    *bytes = extract_ws(nullptr, amp_cap ? amp_cap : 1).bytes;
    return AH_OK;
}

extern "C" ah_status ah_extract(const ah_store *st, ah_primer_set ps, ah_amp *d_amps, const uint64_t *d_n_amps,
                                uint64_t amp_cap, const uint8_t *d_pass, const ah_extract_opts *o, char *d_seq,
                                uint64_t seq_cap, uint64_t *d_seq_off, char *d_fb, char *d_rb, uint8_t *d_bc_len,
                                char *d_fprimer, char *d_rprimer, uint64_t *d_n_bytes, void *d_ws, uint64_t ws_bytes,
                                void *stream) {
    if (!st || !ps || !o || !d_n_amps || !d_n_bytes || !d_seq_off) return AH_E_ARG;
    if (o->fb_len > 255 || o->rb_len > 255) return AH_E_LIMIT;
    if (amp_cap && (!d_amps || !d_bc_len || !d_fprimer || !d_rprimer)) return AH_E_ARG;
    if (amp_cap && ((o->fb_len && !d_fb) || (o->rb_len && !d_rb))) return AH_E_ARG;
    if (seq_cap && !d_seq) return AH_E_ARG;
    ExtractWs w = extract_ws(d_ws, amp_cap ? amp_cap : 1);
    if (!d_ws || ws_bytes < w.bytes) return AH_E_WORKSPACE;
    hipStream_t s = ah_stream(stream);
    hipLaunchKernelGGL(ah_extract_size_kernel, dim3(1024), dim3(256), 0, s, (const uint32_t *)d_amps, d_n_amps,
                       amp_cap, (const DPair *)ps->d_pairs, d_pass, o->trim, w.size);
    if (amp_cap <= AH_EXTRACT_ONE_WG) {  // one launch for the offsets
        hipLaunchKernelGGL(ah_extract_offsets_kernel, dim3(1), dim3(1024), 0, s, (const uint64_t *)w.size, d_n_amps,
                           amp_cap, d_seq_off, d_n_bytes);
    } else {
        ah_status e =
            ah_exclusive_scan<uint64_t, uint64_t>(w.size, d_seq_off, d_n_amps, amp_cap, w.total, w.partials, s);
        if (e) return e;
        hipLaunchKernelGGL(ah_extract_tail_kernel, dim3(1), dim3(1), 0, s, d_n_amps, amp_cap,
                           (const uint64_t *)w.total, d_seq_off, d_n_bytes);
    }
    if (amp_cap) {
        uint64_t wgs = (amp_cap + 3) / 4;  // one wave per amplicon, at most the resident grid
        const uint64_t resident = ah_resident_wgs(ah_extract_write_kernel, 256);
        if (wgs > resident) wgs = resident;
        hipLaunchKernelGGL(ah_extract_write_kernel, dim3((unsigned)wgs), dim3(256), 0, s, *st,
                           (uint32_t *)d_amps, d_n_amps, amp_cap, (const DPair *)ps->d_pairs, d_pass, *o,
                           (const uint64_t *)d_seq_off, d_seq, seq_cap, d_fb, d_rb, d_bc_len, d_fprimer, d_rprimer);
    }
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}

// ---------------------------------------------------------------- qualities
// Quality bytes of each written amplicon (FASTQ input): the qualities of the
// bases ah_extract wrote for it, in the same order -- forward, or reversed
// for RF, whose bases are reverse-complemented (a quality has no
// complement) -- at the same offsets.  One wave per amplicon, consecutive
// lanes on consecutive bytes.
__global__ void __launch_bounds__(256) ah_extract_qual_kernel(const ah_store st, const uint8_t *qual,
                                                              const uint32_t *amps, const uint64_t *d_n, uint64_t cap,
                                                              const DPair *pairs, const uint8_t *pass, uint32_t trim,
                                                              const uint64_t *seq_off, uint8_t *out,
                                                              uint64_t out_cap) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const uint32_t lane = ah_lane();
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t i = blockIdx.x * (uint64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); i < n; i += nw) {
        if (pass && !pass[i]) continue;
        const AmpGeom g = amp_geom(amps, i, pairs);
        uint64_t a0, a1;
        amp_span(g, trim, &a0, &a1);
        const bool rc = g.orient == 1;
        const uint8_t *q = qual + 64 * st.d_seq_block0[g.seq];
        const uint64_t dst = seq_off[i], len = a1 - a0;
        for (uint64_t j = lane; j < len; j += 64) {
            if (dst + j >= out_cap) break;
            out[dst + j] = q[rc ? a1 - 1 - j : a0 + j];
        }
    }
}

extern "C" ah_status ah_extract_qual(const ah_store *st, const uint8_t *d_qual, uint64_t qual_len, ah_primer_set ps,
                                     const ah_amp *d_amps, const uint64_t *d_n_amps, uint64_t amp_cap,
                                     const uint8_t *d_pass, const ah_extract_opts *o, const uint64_t *d_seq_off,
                                     uint8_t *d_out, uint64_t out_cap, void *stream) {
    if (!st || !ps || !o || !d_n_amps || (amp_cap && (!d_amps || !d_seq_off))) return AH_E_ARG;
    if (!d_qual || qual_len < 64 * st->n_blocks || (out_cap && !d_out)) return AH_E_ARG;
    if (!amp_cap) return AH_OK;
    uint64_t wgs = (amp_cap + 3) / 4;  // one wave per amplicon, at most the resident grid
    const uint64_t resident = ah_resident_wgs(ah_extract_qual_kernel, 256);
    if (wgs > resident) wgs = resident;
    hipLaunchKernelGGL(ah_extract_qual_kernel, dim3((unsigned)wgs), dim3(256), 0, ah_stream(stream), *st, d_qual,
                       (const uint32_t *)d_amps, d_n_amps, amp_cap, (const DPair *)ps->d_pairs, d_pass, o->trim,
                       d_seq_off, d_out, out_cap);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
