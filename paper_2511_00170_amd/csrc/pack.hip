// 2-bit packing of FASTA bytes into the bit-plane block store (the paper's
// 2-bit batches: Implementations, AHv2.alpha paragraph).  One wavefront
// handles one 64-base block: lane i reads base i, and three ballots give the
// high-bit plane, the low-bit plane and the N mask of the block.
#include "ah_internal.h"
#include "ah_scan_impl.h"

__device__ __forceinline__ uint32_t base_code(uint8_t c, bool &is_n) {
    // A=00 C=01 G=10 T=11, case-insensitive; anything else is N (stored as A)
    uint8_t u = c & 0xDF;
    is_n = false;
    switch (u) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: is_n = true; return 0;
    }
}

// One wavefront packs one block: lane i codes src[i] when i < use (else A),
// and lane 0 stores the two planes and flags an N block.
__device__ __forceinline__ void pack_block(const uint8_t *src, uint64_t use, uint64_t gb, uint32_t *blocks,
                                           uint32_t *nbits, uint64_t *counters, uint64_t *nlist,
                                           uint64_t nlist_cap) {
    const uint32_t lane = threadIdx.x & 63;
    bool is_n = false;
    uint32_t code = 0;
    if (lane < use) code = base_code(src[lane], is_n);
    const uint64_t hi = __ballot(code >> 1);
    const uint64_t lo = __ballot(code & 1);
    const uint64_t nm = __ballot(is_n);
    if (lane == 0) {
        uint4 w;
        w.x = (uint32_t)hi;
        w.y = (uint32_t)lo;
        w.z = (uint32_t)(hi >> 32);
        w.w = (uint32_t)(lo >> 32);
        ((uint4 *)blocks)[gb] = w;
        if (nm) {
            atomicOr(&nbits[gb >> 5], 1u << (gb & 31));
            unsigned long long k = atomicAdd((unsigned long long *)&counters[0], 1ull);
            if (k < nlist_cap) {
                nlist[2 * k] = gb;
                nlist[2 * k + 1] = nm;
            }
        }
    }
}

__global__ void __launch_bounds__(256) ah_pack_kernel(ah_store st, const uint8_t *ascii, const uint64_t *off,
                                                      uint32_t first, uint32_t n, uint64_t *nlist,
                                                      uint64_t nlist_cap) {
    const uint32_t si = blockIdx.y;
    if (si >= n) return;
    const uint32_t s = first + si;
    const uint64_t len = st.d_seq_len[s];
    const uint64_t alen = off[si + 1] - off[si];
    const uint64_t use = len < alen ? len : alen;
    const uint64_t nblk = (len + 63) / 64;
    const uint64_t b0 = st.d_seq_block0[s];
    const uint8_t *src = ascii + off[si];
    const uint64_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t b = wave; b < nblk; b += nwaves)
        pack_block(src + b * 64, use > b * 64 ? use - b * 64 : 0, b0 + b, st.d_blocks, st.d_nbits, st.d_counters,
                   nlist, nlist_cap);
}

// blockIdx.y = piece; the waves of the row stride over its blocks.
__global__ void __launch_bounds__(256) ah_pack_pieces_kernel(uint32_t *blocks, uint64_t blocks_cap, uint32_t *nbits,
                                                             uint64_t *counters, const uint8_t *ascii,
                                                             const ah_pack_piece *pieces, uint32_t n,
                                                             uint64_t *nlist, uint64_t nlist_cap) {
    const uint32_t pi = blockIdx.y;
    if (pi >= n) return;
    const ah_pack_piece pc = pieces[pi];
    const uint64_t nblk = ((uint64_t)pc.n + 63) / 64;
    const uint64_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t b = wave; b < nblk; b += nwaves) {
        const uint64_t gb = pc.block + b;
        if (gb >= blocks_cap) break;  // wave-uniform
        pack_block(ascii + pc.src + b * 64, (uint64_t)pc.n - b * 64, gb, blocks, nbits, counters, nlist, nlist_cap);
    }
}

__global__ void ah_popc_kernel(const uint32_t *bits, uint32_t *out, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = __popc(bits[i]);
}

__global__ void ah_nmask_scatter_kernel(ah_store st, const uint64_t *nlist, uint64_t nlist_cap) {
    const uint64_t cnt = st.d_counters[0] < nlist_cap ? st.d_counters[0] : nlist_cap;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = nlist[2 * i];
        const uint32_t w = st.d_nbits[b >> 5];
        const uint64_t r = (uint64_t)st.d_nrank[b >> 5] + __popc(w & ((1u << (b & 31)) - 1u));
        if (r < st.nmask_cap) st.d_nmask[r] = nlist[2 * i + 1];
    }
}

static ah_status check_store(const ah_store *st) {
    if (!st || !st->d_blocks || !st->d_seq_block0 || !st->d_seq_len || !st->d_nbits || !st->d_nrank ||
        !st->d_counters)
        return AH_E_ARG;
    if (st->nmask_cap && !st->d_nmask) return AH_E_ARG;
    return AH_OK;
}

extern "C" ah_status ah_pack_begin(const ah_store *st, void *stream) {
    ah_status e = check_store(st);
    if (e) return e;
    hipStream_t s = ah_stream(stream);
    const uint64_t nw = (st->n_blocks + 31) / 32;
    ah_fill<uint32_t>(st->d_nbits, 0u, nw, s);
    ah_fill<uint32_t>(st->d_nrank, 0u, nw, s);
    ah_fill<uint64_t>(st->d_counters, 0ull, AH_STORE_SCRATCH, s);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}

extern "C" ah_status ah_pack(const ah_store *st, const uint8_t *d_ascii, const uint64_t *d_ascii_off,
                             uint32_t first_seq, uint32_t n, uint64_t *d_nlist, uint64_t nlist_cap, void *stream) {
    ah_status e = check_store(st);
    if (e) return e;
    if (!n) return AH_OK;
    if (!d_ascii || !d_ascii_off || (nlist_cap && !d_nlist)) return AH_E_ARG;
    if ((uint64_t)first_seq + n > st->n_seqs) return AH_E_ARG;
    hipStream_t s = ah_stream(stream);
    for (uint32_t c0 = 0; c0 < n; c0 += 65535) {
        uint32_t cn = n - c0 < 65535 ? n - c0 : 65535;
        hipLaunchKernelGGL(ah_pack_kernel, dim3(64, cn), dim3(256), 0, s, *st, d_ascii, d_ascii_off + c0,
                           first_seq + c0, cn, d_nlist, nlist_cap);
    }
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}

extern "C" ah_status ah_pack_pieces(uint32_t *d_blocks, uint64_t blocks_cap, uint32_t *d_nbits, uint64_t *d_counters,
                                    const uint8_t *d_ascii, const ah_pack_piece *d_pieces, uint32_t n_pieces,
                                    uint64_t *d_nlist, uint64_t nlist_cap, void *stream) {
    if (!n_pieces) return AH_OK;
    if (!d_blocks || !d_nbits || !d_counters || !d_ascii || !d_pieces || (nlist_cap && !d_nlist)) return AH_E_ARG;
    hipStream_t s = ah_stream(stream);
    // workgroups per piece: many pieces in one chunk are short ones
    const uint32_t gx = n_pieces <= 256 ? 64 : (n_pieces <= 4096 ? 16 : 4);
    for (uint32_t c0 = 0; c0 < n_pieces; c0 += 65535) {
        const uint32_t cn = n_pieces - c0 < 65535 ? n_pieces - c0 : 65535;
        hipLaunchKernelGGL(ah_pack_pieces_kernel, dim3(gx, cn), dim3(256), 0, s, d_blocks, blocks_cap, d_nbits,
                           d_counters, d_ascii, d_pieces + c0, cn, d_nlist, nlist_cap);
    }
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}

extern "C" ah_status ah_pack_finish(const ah_store *st, const uint64_t *d_nlist, uint64_t nlist_cap, void *stream) {
    ah_status e = check_store(st);
    if (e) return e;
    hipStream_t s = ah_stream(stream);
    const uint64_t nw = (st->n_blocks + 31) / 32;
    // scratch layout in d_counters: [1] = word count, [8..] = scan partials (u32)
    hipLaunchKernelGGL(ah_set_kernel<uint64_t>, dim3(1), dim3(1), 0, s, st->d_counters + 1, nw);
    hipLaunchKernelGGL(ah_popc_kernel, dim3(1024), dim3(256), 0, s, (const uint32_t *)st->d_nbits, st->d_nrank, nw);
    e = ah_exclusive_scan<uint32_t, uint32_t>(st->d_nrank, st->d_nrank, st->d_counters + 1, ~0ull, nullptr,
                                              (uint32_t *)(st->d_counters + 8), s);
    if (e) return e;
    if (d_nlist && nlist_cap)
        hipLaunchKernelGGL(ah_nmask_scatter_kernel, dim3(256), dim3(256), 0, s, *st, d_nlist, nlist_cap);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}

__global__ void ah_unpack_kernel(ah_store st, uint32_t seq, uint64_t start, uint64_t n, uint8_t *out) {
    const uint64_t b0 = st.d_seq_block0[seq];
    const uint64_t len = st.d_seq_len[seq];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = start + i;
        if (p >= len) {  // past the sequence end
            out[i] = 0;
            continue;
        }
        const uint64_t b = b0 + p / 64;
        const uint32_t bit = (uint32_t)(p & 63);
        const uint4 w = ((const uint4 *)st.d_blocks)[b];
        const uint32_t h = bit < 32 ? w.x : w.z, l = bit < 32 ? w.y : w.w;
        const uint32_t c = (((h >> (bit & 31)) & 1u) << 1) | ((l >> (bit & 31)) & 1u);
        const uint64_t nm = ah_block_nmask(st, b);
        out[i] = ((nm >> bit) & 1ull) ? 'N' : ah_letter(c);
    }
}

extern "C" ah_status ah_unpack(const ah_store *st, uint32_t seq, uint64_t start, uint64_t n, uint8_t *d_out,
                               void *stream) {
    ah_status e = check_store(st);
    if (e) return e;
    if (seq >= st->n_seqs || (n && !d_out)) return AH_E_ARG;
    if (!n) return AH_OK;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(ah_unpack_kernel, dim3((unsigned)blocks), dim3(256), 0, ah_stream(stream), *st, seq, start, n,
                       d_out);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
