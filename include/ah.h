/*
 * ah.h -- C ABI of libah.so, an MI355X (gfx950) implementation of the
 * in-silico PCR hot path of AmpliconHunter2 (Howard-Stone & Mandoiu,
 * arXiv 2511.00170): scan 2-bit genomes for IUPAC-degenerate primers with at
 * most k substitutions and an exact 3' clamp, pair the hits into FR/RF/FF/RR
 * amplicons inside a length window, compute the nearest-neighbour melting
 * temperature, trim primers and cut flanking barcodes.
 *
 * Conventions (every entry point):
 *  - Plain C.  `d_` pointers are device memory owned by the caller; `h_`
 *    pointers are host memory.  No entry point allocates device memory except
 *    ah_primers_compile (a one-time set-up call) and none synchronises the
 *    host except ah_fasta_ingest (file input, which also allocates its pinned
 *    host staging buffers), so the others can be captured into a HIP graph.
 *  - `stream` is a hipStream_t (NULL = the null stream); work is enqueued
 *    asynchronously on it.
 *  - Argument errors are returned synchronously and leave outputs untouched.
 *  - Capacity overflow is not an error at call time: a kernel writes at most
 *    `cap` records and always stores the true count in its device counter;
 *    the caller compares after synchronising and re-runs with a larger cap.
 *    Every output is deterministic, so a re-run is exact.
 *  - Coordinates are 0-based, half-open, on the plus strand of the sequence.
 */
#ifndef AH_H
#define AH_H

#ifndef __HIPCC_RTC__
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ah_status;
#define AH_OK 0
#define AH_E_ARG 1       /* null pointer, zero size where one is needed, bad enum */
#define AH_E_ALPHABET 2  /* a primer letter outside the 15 IUPAC codes (U reads as T) */
#define AH_E_LIMIT 3     /* primer length outside 1..32, clamp > length, too many pairs, key too wide */
#define AH_E_HIP 4       /* a HIP runtime call failed */
#define AH_E_WORKSPACE 5 /* workspace smaller than the matching *_ws_size() */
#define AH_E_IO 6        /* a file could not be opened or read */
#define AH_E_FORMAT 7    /* not FASTA: data before the first header, a record of 2^32 or more bases,
                            2^32 or more records */
#define AH_E_SCRATCH 8   /* input larger than the library's fixed scratch array allows */

/* Human-readable name of a status code (static string). */
const char *ah_status_str(ah_status s);
int ah_version(void);

/* ------------------------------------------------------------------------
 * 2-bit genome store (the paper's 2-bit batches: Implementations, AHv2.alpha
 * paragraph; 2-bit files read ~3.93x fewer bytes than FASTA, Results).
 *
 * Every sequence starts on a 64-base block.  Block b holds four 32-bit words
 * {hi[0:32], lo[0:32], hi[32:64], lo[32:64]}: bit i of hi/lo is the high/low
 * bit of base i of the block with A=00, C=01, G=10, T=11 (the complement of a
 * code is code XOR 3).  Bases past a sequence end are stored as A and never
 * read as sequence.  A byte that is not A/C/G/T (either case) is an N: it is
 * stored as A and flagged in a side table -- d_nbits has one bit per block
 * ("this block holds an N"), d_nrank the number of flagged blocks before each
 * 32-block word, d_nmask one 64-bit mask of N positions per flagged block, in
 * block order.  16 bytes per 64 bases = 0.25 B/base in HBM.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t n_seqs;
    uint32_t max_len;        /* longest sequence, bases */
    uint64_t n_blocks;       /* total 64-base blocks */
    uint32_t *d_blocks;      /* [n_blocks][4] */
    uint64_t *d_seq_block0;  /* [n_seqs] first block of each sequence */
    uint32_t *d_seq_len;     /* [n_seqs] length in bases */
    uint32_t *d_nbits;       /* [ceil(n_blocks/32)] */
    uint32_t *d_nrank;       /* [ceil(n_blocks/32)] */
    uint64_t *d_nmask;       /* [nmask_cap] */
    uint64_t nmask_cap;
    uint64_t *d_counters;    /* [AH_STORE_SCRATCH] library scratch; [0] = number of flagged blocks */
} ah_store;

#define AH_STORE_SCRATCH 2048

/* Host: block layout of sequences with the given lengths.  Writes
 * h_seq_block0[n_seqs] and *h_n_blocks.  Lengths must be < 2^32. */
ah_status ah_pack_layout(const uint64_t *h_lens, uint32_t n_seqs, uint64_t *h_seq_block0, uint64_t *h_n_blocks);

/* Clear the N side table and counters of a store before packing into it. */
ah_status ah_pack_begin(const ah_store *st, void *stream);

/* Pack sequences [first_seq, first_seq + n) whose ASCII bytes are at
 * d_ascii + d_ascii_off[i - first_seq] (d_ascii_off has n + 1 entries,
 * relative to d_ascii; the lengths must equal d_seq_len).  Blocks holding an
 * N are also appended as (block, mask) pairs to d_nlist ([2 * nlist_cap]
 * u64; count in st->d_counters[0]).  May be called for several chunks. */
ah_status ah_pack(const ah_store *st, const uint8_t *d_ascii, const uint64_t *d_ascii_off, uint32_t first_seq,
                  uint32_t n, uint64_t *d_nlist, uint64_t nlist_cap, void *stream);

/* After the last ah_pack: build d_nrank and place the N masks in block order.
 * If more blocks were flagged than nlist_cap / nmask_cap allow, the count in
 * st->d_counters[0] says so and the pack must be redone with larger caps. */
ah_status ah_pack_finish(const ah_store *st, const uint64_t *d_nlist, uint64_t nlist_cap, void *stream);

/* One piece of a sequence for ah_pack_pieces. */
typedef struct {
    uint64_t src;      /* offset of the piece's first base in d_ascii */
    uint64_t block;    /* store block that receives that base */
    uint32_t n;        /* bases in the piece */
    uint32_t reserved; /* 0 */
} ah_pack_piece;

/* Pack pieces of sequences whose layout the caller has fixed: piece i's n
 * bases at d_ascii + src go to blocks [block, block + ceil(n / 64)).  Each
 * piece starts on a 64-base boundary of its sequence; only the last piece of
 * a sequence may end inside a block (the rest of that block is stored as A).
 * Blocks at or past blocks_cap are not written, which is not an error.  N
 * blocks are flagged in d_nbits and appended to d_nlist as by ah_pack (count
 * in d_counters[0]); clear d_nbits and d_counters first (ah_pack_begin does).
 * d_pieces is device memory. */
ah_status ah_pack_pieces(uint32_t *d_blocks, uint64_t blocks_cap, uint32_t *d_nbits, uint64_t *d_counters,
                         const uint8_t *d_ascii, const ah_pack_piece *d_pieces, uint32_t n_pieces, uint64_t *d_nlist,
                         uint64_t nlist_cap, void *stream);

/* Decode bases [start, start + n) of sequence `seq` to ASCII (A/C/G/T/N). */
ah_status ah_unpack(const ah_store *st, uint32_t seq, uint64_t start, uint64_t n, uint8_t *d_out, void *stream);

/* ------------------------------------------------------------------------
 * Primer sets (Supplementary, "Primer matching and clamp logic": primers are
 * compiled into per-base IUPAC masks, reverse-complement masks precomputed).
 * Each pair has its own k (substitutions allowed, inclusive), clamp (number
 * of 3'-terminal primer positions that must match exactly; 0 disables it)
 * and amplicon length window [min_len, max_len] (primers included).
 * ---------------------------------------------------------------------- */
typedef struct {
    const char *fwd;  /* 5'->3', IUPAC, 1..32 letters */
    const char *rev;  /* 5'->3', IUPAC, 1..32 letters */
    uint32_t k;
    uint32_t clamp;
    uint32_t min_len;
    uint32_t max_len;
} ah_pair_spec;

typedef struct ah_primer_set_ *ah_primer_set;

/* Validate and compile pairs (at most AH_MAX_PAIRS).  Allocates a small
 * device table (owned by the handle).  Errors: AH_E_ALPHABET, AH_E_LIMIT. */
#define AH_MAX_PAIRS 4096
ah_status ah_primers_compile(const ah_pair_spec *h_pairs, uint32_t n_pairs, ah_primer_set *out);
void ah_primers_free(ah_primer_set ps);
uint32_t ah_primers_count(ah_primer_set ps);

/* As ah_primers_compile, but the device tables go into caller memory d_buf
 * (at least ah_primers_table_bytes(n_pairs) bytes) by an asynchronous copy on
 * `stream`: no allocation, no synchronisation, so a per-batch primer set can
 * be built while other streams run (serving).  The handle does not own
 * d_buf; keep both alive until the work using the set on `stream` is done,
 * then ah_primers_free.  Errors: as ah_primers_compile; AH_E_WORKSPACE when
 * d_buf is too small. */
ah_status ah_primers_compile_into(const ah_pair_spec *h_pairs, uint32_t n_pairs, void *d_buf, uint64_t buf_bytes,
                                  void *stream, ah_primer_set *out);
uint64_t ah_primers_table_bytes(uint32_t n_pairs);

/* Optional set-up step: compile, with hipRTC, a scan kernel whose clamp
 * pre-filter has this primer set's IUPAC codes as compile-time constants
 * (each set test folds into one bit operation) and use it for later
 * ah_scan_primers calls with this set on the current device.  Results are
 * identical to the generic kernel.  Blocks for the compile (about a second);
 * AH_E_HIP if hipRTC or module loading fails (the generic kernel stays). */
ah_status ah_primers_jit(ah_primer_set ps);

/* Select the specialised kernel variant with blocks_per_lane 64-base blocks
 * per lane (1 or 2: a wave's tile, the positions one wave scans per step, is
 * 4096 x blocks_per_lane bases) and an LDS buffer of hit_buffer hit records
 * per wave (2..256), compiling it on first use (variants stay cached with
 * the set).  Every variant finds the same hits; registers, LDS and hence
 * occupancy and speed differ -- the batch autotuner times them.
 * ah_primers_jit selects (2, 48) unless a variant is already selected.
 * Errors: AH_E_ARG (null set, values out of range), AH_E_HIP. */
ah_status ah_primers_jit_variant(ah_primer_set ps, uint32_t blocks_per_lane, uint32_t hit_buffer);

/* Generate and compile (without loading) the specialised scan kernel variant
 * (blocks_per_lane, hit_buffer as in ah_primers_jit_variant) of the primer
 * pairs h_pairs[n_pairs] for the GPU architecture `arch` (e.g. "gfx950");
 * touches no device.  AH_OK when it compiles; AH_E_ARG for a bad variant;
 * the primer errors of ah_primers_compile; AH_E_HIP when hipRTC fails (its
 * log goes to stderr).  For build checks on machines without a GPU. */
ah_status ah_primers_jit_check(const ah_pair_spec *h_pairs, uint32_t n_pairs, const char *arch,
                               uint32_t blocks_per_lane, uint32_t hit_buffer);

/* Switch between the specialised (on != 0, needs ah_primers_jit first) and
 * the generic scan kernel for this set. */
ah_status ah_primers_use_jit(ah_primer_set ps, int32_t on);

/* Launch shape of the persistent scan for this set: wg_per_cu workgroups of
 * 256 lanes per compute unit (0 = as many as can be resident, the default;
 * larger values are clamped to that maximum).  Applies to whichever kernel
 * (specialised or generic) is selected at the next ah_scan_primers call.
 * If max_wg_per_cu is non-null it receives the resident maximum of the
 * currently selected kernel on the current device.  Results do not depend on
 * the shape (every tile is scanned exactly once); only the speed does.
 * Errors: AH_E_ARG (null set, negative value), AH_E_HIP. */
ah_status ah_primers_launch_shape(ah_primer_set ps, int32_t wg_per_cu, int32_t *max_wg_per_cu);

/* ------------------------------------------------------------------------
 * Scan (Supplementary, "Primer matching and clamp logic"; mismatches are
 * substitutions, Results "Primer degeneracy and mismatch tolerance").
 * For each sequence s, pair q, primer P in {F, R}, strand: the pattern is
 * X = P (plus) or X = rc(P) (minus); position p in [0, len - |X|] is a hit
 * iff every clamp position matches -- the last `clamp` positions of X on the
 * plus strand, the first `clamp` positions of X on the minus strand (the
 * primer's 3' end) -- and mm = #{j : s[p+j] not in X[j]} <= k.  An N matches
 * nothing.  Hits are written in arbitrary order.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t seq;   /* store index */
    uint32_t pos;   /* window start on the plus strand */
    uint16_t pair;  /* pair index in the primer set */
    uint8_t kind;   /* bit0: reverse primer; bit1: minus strand (site of rc(primer)) */
    uint8_t mm;     /* substitutions */
} ah_hit;           /* 12 bytes */

/* Workspace bytes for ah_scan_primers over n_list sequences (all: n_seqs). */
ah_status ah_scan_ws_size(const ah_store *st, uint32_t n_list, uint64_t *bytes);

/* d_seq_subset: NULL for every sequence, else n_subset store indices
 * (n_subset may be 0: nothing is scanned; the pointer must still be non-null;
 * an index >= n_seqs is skipped).
 * Writes min(total, hit_cap) hits; *d_n_hits = total (the call resets it). */
ah_status ah_scan_primers(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset, uint32_t n_subset,
                          ah_hit *d_hits, uint64_t hit_cap, uint64_t *d_n_hits, void *d_ws, uint64_t ws_bytes,
                          void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): ah_scan_primers
 * without a workspace argument.  Its workspace is a fixed array inside the
 * library (AH_STATIC_SCRATCH_BYTES per GPU, held until the process ends), so
 * at most AH_STATIC_SCAN_MAX_LIST sequences may be listed (all of the store's
 * when d_seq_subset is NULL); more returns AH_E_SCRATCH before any work.  The
 * call allocates nothing.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (different streams, or host threads)
 * race and give wrong hits -- order them on one stream.  Results are
 * identical to ah_scan_primers.  Errors: as ah_scan_primers, AH_E_SCRATCH. */
#define AH_STATIC_SCAN_MAX_LIST 65536u
#define AH_STATIC_SCRATCH_BYTES ((1u << 20) + 4096u)
ah_status ah_scan_primers_static(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset,
                                 uint32_t n_subset, ah_hit *d_hits, uint64_t hit_cap, uint64_t *d_n_hits,
                                 void *stream);

/* As ah_scan_primers, with the pairs scanned chosen per listed sequence:
 * d_pair_mask[i] (device, one word per listed sequence, i.e. per subset entry
 * or per store sequence when d_seq_subset is NULL) has bit q set when pair q
 * is to be scanned on that sequence.  The hits are exactly those of
 * ah_scan_primers restricted to the (sequence, pair) combinations asked for;
 * a sequence whose word is 0 still costs its loads, so callers leave it out
 * of the subset.  Serving uses this to batch requests that ask for different
 * pairs on different sequences (Supplementary, "Webserver").
 * Errors: as ah_scan_primers; AH_E_LIMIT if the set has more than 64 pairs. */
ah_status ah_scan_primers_masked(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset,
                                 uint32_t n_subset, const uint64_t *d_pair_mask, ah_hit *d_hits, uint64_t hit_cap,
                                 uint64_t *d_n_hits, void *d_ws, uint64_t ws_bytes, void *stream);

/* Route hits of a shared scan to the requests of a serving batch (Discussion;
 * Supplementary, "Webserver").  Hit h = (seq s, pair q, mm) is copied once for
 * every request r < n_req with bit r of d_seq_req[s] set (the request asked
 * for sequence s), d_vpair[r * n_pool + q] != 0xFFFF (it asked for pool pair
 * q) and mm <= d_kmax[r] (its own mismatch bound).  The copy's pair field is
 * d_vpair[r * n_pool + q]: the request's own slot in the primer set that the
 * pair / Tm / extract calls of the batch use.  All arrays are device memory:
 * d_seq_req[n_seqs] (store sequence index -> request bitmap), d_vpair[n_req *
 * n_pool], d_kmax[n_req].  Writes min(total, out_cap) copies in arbitrary
 * order and *d_n_out = total (the call resets it).  n_req <= 64; the first
 * min(*d_n_hits, hit_cap) hits are read.  Errors: AH_E_ARG, AH_E_LIMIT. */
ah_status ah_route_hits(const ah_hit *d_hits, const uint64_t *d_n_hits, uint64_t hit_cap, uint32_t n_seqs,
                        const uint64_t *d_seq_req, const uint16_t *d_vpair, const uint8_t *d_kmax, uint32_t n_req,
                        uint32_t n_pool, ah_hit *d_out, uint64_t out_cap, uint64_t *d_n_out, void *stream);

/* ------------------------------------------------------------------------
 * Pair (Supplementary, "Amplicon calling and orientation").  Per (sequence,
 * pair) the sites are sorted by (start, end, plus before minus, forward
 * before reverse).  A plus site a pairs with every later minus site t before
 * the next plus site when min_len <= t.end - a.start <= max_len and the
 * orientation is requested: FR (a forward, t reverse) = 1, RF = 2, FF = 4,
 * RR = 8 in orient_mask.  Output order: (seq, pair, then the downstream
 * site's sort key), which is deterministic.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t seq;
    uint32_t start;  /* start of the upstream (plus) site */
    uint32_t end;    /* end of the downstream (minus) site */
    uint16_t pair;
    uint8_t orient;  /* 0 FR, 1 RF, 2 FF, 3 RR */
    uint8_t flags;   /* bit 0: a barcode was clipped at a sequence end (set by ah_extract; 0 before) */
} ah_amp;            /* 16 bytes */

#define AH_ORIENT_FR 1u
#define AH_ORIENT_RF 2u
#define AH_ORIENT_FF 4u
#define AH_ORIENT_RR 8u

ah_status ah_pair_ws_size(const ah_store *st, ah_primer_set ps, uint64_t hit_cap, uint64_t *bytes);

/* Reads min(*d_n_hits, hit_cap) hits (d_hits is left unchanged).  Writes
 * min(total, amp_cap) amplicons, *d_n_amps = total. */
ah_status ah_pair_amplicons(const ah_store *st, ah_primer_set ps, const ah_hit *d_hits, const uint64_t *d_n_hits,
                            uint64_t hit_cap, uint32_t orient_mask, ah_amp *d_amps, uint64_t amp_cap,
                            uint64_t *d_n_amps, void *d_ws, uint64_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Nearest-neighbour melting temperature (Implementations, "AHv2": the model
 * of Biopython's Tm_NN, every parameter combination).  Per amplicon, each of
 * its two sites gets the maximum over the concrete variants of its primer of
 * the duplex Tm of (variant 5'->3', genome strand it anneals to); the
 * amplicon Tm is the smaller site Tm; pass = Tm >= threshold_C (or 1 when
 * filter == 0).  FP64.
 * Duplex Tm, in this order: a dangling end (explicit duplexes only;
 * Bommarito et al. 2000) and then a mismatched end pair (terminal-mismatch
 * stack, SantaLucia & Peyret 2001) leave the helix with their terms;
 * initiation from the primer strand as given (its end bases, whether it
 * holds a G or C); the remaining Watson-Crick stacks of the selected set and
 * internal single mismatches (Allawi & SantaLucia 1997/1998, Peyret et al.
 * 1999); the salt term; Tm = 1000 dH / (dS + 1.987 ln C) - 273.15.  A
 * variant with a stack none of the tables covers is skipped; a site with no
 * usable variant has Tm = -inf.
 * nn_table (Watson-Crick set and initiation, numbered as the Tm_NN model
 * numbers its DNA tables): 1 Breslauer et al. 1986, 2 Sugimoto et al. 1996,
 * 3 SantaLucia 1998 unified (= Allawi & SantaLucia 1997), 4 SantaLucia &
 * Hicks 2004; 0 = 3.
 * saltcorr (the corrections the Tm_NN model offers; [Na+eq] = Na + K +
 * Tris/2 + 120 sqrt(Mg - dNTPs) mM, the last term only when Mg > dNTPs
 * (von Ahsen et al. 2001); N and the G+C fraction are the primer strand's):
 *   0 none
 *   1 Tm += 16.6 log10[Na+eq]                    (Schildkraut & Lifson 1965)
 *   2 Tm += 16.6 log10([Na+eq] / (1 + 0.7 [Na+eq]))   (Wetmur 1991)
 *   3 Tm += 12.5 log10[Na+eq]                    (SantaLucia et al. 1996)
 *   4 Tm += 11.7 log10[Na+eq]                    (SantaLucia 1998)
 *   5 dS += 0.368 (N - 1) ln[Na+eq]              (SantaLucia 1998)
 *   6 1/Tm += (4.29 fGC - 3.95) 1e-5 ln[Na+eq] + 9.40e-6 ln^2[Na+eq]
 *                                                (Owczarzy et al. 2004)
 *   7 1/Tm += the Mg2+ model of Owczarzy et al. 2008 (free Mg2+ after dNTP
 *     binding; monovalent ions Na + K + Tris/2; the 2004 formula when
 *     sqrt[Mg2+]/[mon] < 0.22)
 * AH_E_ARG for another nn_table or saltcorr value or a zero concentration
 * under a logarithm.  Strand concentration C = C_high - C_low / 2.
 * ---------------------------------------------------------------------- */
typedef struct {
    double na_mM, k_mM, tris_mM, mg_mM, dntps_mM;
    double dnac1_nM, dnac2_nM;
    double threshold_C;
    int32_t saltcorr;
    int32_t filter;
    /* NULL, or a device array with one threshold (C) per pair of the set that
     * replaces threshold_C for that pair's amplicons (serving batches whose
     * requests ask for different thresholds). */
    const double *d_pair_threshold;
    int32_t nn_table;
    int32_t reserved;  /* 0 */
} ah_tm_params;

/* d_tm[n], d_tm_site[n][2] (upstream, downstream), d_pass[n]; n = min(*d_n_amps, amp_cap). */
ah_status ah_tm_nn(const ah_store *st, ah_primer_set ps, const ah_amp *d_amps, const uint64_t *d_n_amps,
                   uint64_t amp_cap, const ah_tm_params *p, double *d_tm, double *d_tm_site, uint8_t *d_pass,
                   void *stream);

/* Tm of n explicit duplexes.  Row i of d_seq holds the primer strand
 * (5'->3', d_len[i] letters, 2..32) and row i of d_cseq its partner strand
 * written 3'->5' (d_clen[i] letters, 1..64; d_clen NULL = d_len), rows
 * `stride` bytes apart; d_cseq[i][j] faces d_seq[i][j - d_shift[i]]
 * (d_shift NULL = 0, |shift| <= 64).  An end may keep one unpaired base of
 * either strand (a dangling end); further overhang is ignored.  Writes
 * d_tm[i]: NaN when a letter is not ACGT, a stack or dangling end is not
 * tabulated, fewer than two positions face each other, or a length is out
 * of range. */
ah_status ah_tm_duplex(const char *d_seq, const char *d_cseq, const uint32_t *d_len, const uint32_t *d_clen,
                       const int32_t *d_shift, uint32_t n, uint32_t stride, const ah_tm_params *p, double *d_tm,
                       void *stream);

/* ------------------------------------------------------------------------
 * Extract (Supplementary, "Primer trimming and barcode extraction" and
 * "Headers and outputs").  FR/FF/RR amplicons are s[start:end]; RF ones are
 * reverse-complemented (Supplementary, "Amplicon calling and orientation").
 * trim removes both primer sites.  fb = the fb_len bases upstream of the
 * forward site and rb = the rb_len bases downstream of the reverse site (FR,
 * FF, RR); for RF the opposite sides, both reverse-complemented.  Barcodes
 * are clipped at sequence ends (real lengths in d_bc_len[n][2]); ah_extract
 * then sets bit 0 of that amplicon's flags, and clears it otherwise (the
 * flags byte is the only part of d_amps it writes).
 * fprimer/rprimer: the genome bases under the forward/reverse site in that
 * primer's orientation (FF/RR: upstream / downstream site), NUL-padded to 32.
 * Amplicons with d_pass[i] == 0 (d_pass may be NULL) produce nothing.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t trim;
    uint32_t fb_len;  /* <= 255 */
    uint32_t rb_len;  /* <= 255 */
} ah_extract_opts;

ah_status ah_extract_ws_size(uint64_t amp_cap, uint64_t *bytes);

/* d_seq_off has amp_cap + 1 entries; d_fb [n][fb_len], d_rb [n][rb_len],
 * d_fprimer/d_rprimer [n][32]; *d_n_bytes = total sequence bytes (bytes past
 * seq_cap are not written). */
ah_status ah_extract(const ah_store *st, ah_primer_set ps, ah_amp *d_amps, const uint64_t *d_n_amps,
                     uint64_t amp_cap, const uint8_t *d_pass, const ah_extract_opts *o, char *d_seq, uint64_t seq_cap,
                     uint64_t *d_seq_off, char *d_fb, char *d_rb, uint8_t *d_bc_len, char *d_fprimer,
                     char *d_rprimer, uint64_t *d_n_bytes, void *d_ws, uint64_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Measurement helper: read d_buf[0:bytes) once with 128-bit loads (a
 * persistent grid of at most out_n workgroups, each writing one XOR fold to
 * d_out) -- the HBM read bandwidth a plain streaming kernel reaches, the
 * ceiling the scan's bandwidth is compared with.  bytes must be a multiple of
 * 16; d_out holds out_n words.  Errors: AH_E_ARG, AH_E_HIP.
 * ---------------------------------------------------------------------- */
ah_status ah_read_probe(const void *d_buf, uint64_t bytes, uint32_t *d_out, uint32_t out_n, void *stream);

/* ------------------------------------------------------------------------
 * FASTA ingest (Implementations: AHv2 reads FASTA into 2-bit batches of
 * headers, lengths and bases; Discussion: headers kept apart from the bases).
 *
 * A record is a line starting with '>' and the lines up to the next such line
 * or the end of its file; records never span files.  Its identifier is the
 * first white-space-separated word of the header (may be empty), its
 * sequence the bytes of its other lines with ASCII white space (space, tab,
 * LF, VT, FF, CR) removed; bytes other than A/C/G/T (either case) become N in
 * the store.  Only white space may precede a file's first header.
 *
 * ah_fasta_ingest keeps each record's identifier, source file, length and
 * first block (the layout of ah_pack_layout) on the host and streams the
 * bases through pinned staging buffers: while the GPU copies and packs one
 * chunk, the host fills the next.  With one worker (n_threads <= 1, or one
 * file) the files are read once, in order.  With more, up to n_threads host
 * threads index the files in parallel, the layout is fixed in file order and
 * the files are packed in parallel, each worker with its own two staging
 * buffers and its own part of d_ws (so every file is read twice).  With
 * d_blocks == NULL it only builds the record table (no GPU calls; stream and
 * workspace unused).  The call returns when its GPU work has finished.
 *
 * Store arrays (caller-owned device memory, cleared by the call): d_blocks
 * [blocks_cap][4] u32, d_nbits [ceil(blocks_cap / 32)] u32, d_counters
 * [AH_STORE_SCRATCH] u64, d_nlist [nlist_cap][2] u64.  Blocks past
 * blocks_cap and N blocks past nlist_cap are not written; the record table
 * still counts them (ah_fasta_info's n_blocks, d_counters[0]), so the caller
 * can run again with larger arrays.  To finish a store: copy the record
 * table's lengths and first blocks to d_seq_len / d_seq_block0, fill an
 * ah_store with n_blocks from ah_fasta_info, and call ah_pack_finish.
 * Errors: AH_E_ARG (null paths, chunk_bytes outside [4096, 2^30]), AH_E_IO
 * (also: a file changed between the two reads), AH_E_FORMAT, AH_E_WORKSPACE
 * (smaller than one worker's share; a workspace for fewer workers than
 * n_threads limits the workers), AH_E_HIP; *out is set only on success.
 * ---------------------------------------------------------------------- */
typedef struct ah_fasta ah_fasta;  /* record table (host memory, owned by the library) */

/* Device workspace bytes one ingest worker needs for staging chunks of
 * chunk_bytes (ah_fasta_ingest with W workers needs W times this). */
ah_status ah_fasta_ws_size(uint64_t chunk_bytes, uint64_t *bytes);

ah_status ah_fasta_ingest(const char *const *paths, uint32_t n_files, uint32_t *d_blocks, uint64_t blocks_cap,
                          uint32_t *d_nbits, uint64_t *d_counters, uint64_t *d_nlist, uint64_t nlist_cap,
                          uint64_t chunk_bytes, uint32_t n_threads, void *d_ws, uint64_t ws_bytes, void *stream,
                          ah_fasta **out);

/* Totals of the record table. */
ah_status ah_fasta_info(const ah_fasta *f, uint32_t *n_records, uint64_t *n_bases, uint64_t *n_blocks,
                        uint32_t *max_len);

/* Per-record lengths and first blocks ([n_records] each, host arrays). */
ah_status ah_fasta_table(const ah_fasta *f, uint32_t *h_len, uint64_t *h_block0);

/* Record identifiers and sources as the FASTA writer takes them; the pointers
 * stay owned by f and valid until ah_fasta_free. */
typedef struct {
    const char *ids;          /* NUL-terminated identifiers, back to back */
    const uint64_t *id_off;   /* [n_seqs] offset of sequence i's identifier in ids */
    const uint32_t *seq_file; /* [n_seqs] index of sequence i's source file */
    const char *const *files; /* [n_files] source file names (path without directories) */
    uint32_t n_seqs;
    uint32_t n_files;
} ah_fasta_names;

ah_status ah_fasta_names_of(const ah_fasta *f, ah_fasta_names *out);

void ah_fasta_free(ah_fasta *f);

/* ------------------------------------------------------------------------
 * FASTA output (Supplementary, "Headers and outputs"): one record per
 * amplicon, in amplicon order, skipping those with h_pass[i] == 0 (h_pass may
 * be NULL: all).  Header fields in the paper's order:
 *   >ID.source=FILE.coordinates=S-E.Tm=T.orientation=O.fprimer=P.rprimer=Q[.fb=B][.rb=C]
 * ID and FILE from the names of the amplicon's sequence; S-E the amplicon
 * (primer sites included, also when trimmed) as 1-based inclusive
 * coordinates, start + 1 to end; T the Tm with two decimals (correctly
 * rounded), NA when not finite; O one of FR RF FF RR; P/Q the primer
 * snippets (NUL-padded [32] rows); .fb/.rb only when fb_len / rb_len > 0,
 * their text h_bc_len[i][0] / [1] bytes of the [fb_len] / [rb_len] rows.  The
 * amplicon's bytes follow on one line.  The inputs are the host copies of
 * ah_extract's outputs (all host memory).  *h_n_bytes = the text's length;
 * bytes past out_cap are not written.  AH_E_ARG for a sequence index outside
 * the names, an orientation above 3, barcode lengths above the widths, or
 * decreasing sequence offsets.
 * ---------------------------------------------------------------------- */
ah_status ah_fasta_format(const ah_fasta_names *names, uint32_t fb_len, uint32_t rb_len, const ah_amp *h_amps,
                          uint64_t n_amps, const double *h_tm, const uint8_t *h_pass, const char *h_seq,
                          const uint64_t *h_seq_off, const char *h_fb, const char *h_rb, const uint8_t *h_bc_len,
                          const char *h_fprimer, const char *h_rprimer, char *h_out, uint64_t out_cap,
                          uint64_t *h_n_bytes);

/* ------------------------------------------------------------------------
 * FASTQ input and output with quality propagation (Discussion: FASTQ input
 * with qualities carried to the amplicons, for amplicon sequencing data; the
 * Python AHv1.1 reads FASTQ).  A record is four lines: "@" and a header whose
 * first white-space-separated word is the identifier; the bases (bytes
 * '!'..'~'; other than A/C/G/T in either case they read as N); a line
 * starting with "+" (the rest of it ignored); the qualities, one byte in
 * '!'..'~' per base.  Lines end in LF or CR LF; empty lines between records
 * are skipped; anything else is AH_E_FORMAT, as are records of 2^32 or more
 * bases (records wrapped over several lines are not read).
 *
 * ah_fastq_read parses the files on the host into a record table of the
 * FASTA type (ah_fasta_info, ah_fasta_table, ah_fasta_names_of and
 * ah_fasta_free apply; the store layout is ah_pack_layout's) that also keeps
 * the bases and qualities.  ah_fastq_bases gives the bases back to back with
 * [n_records + 1] offsets (host memory owned by the table, valid until
 * ah_fasta_free) for ah_pack.  ah_fastq_qual_layout writes the qualities
 * laid out like the store's bases: record r's base j at byte
 * 64 * block0[r] + j of h_qual (cap >= 64 * n_blocks bytes, else
 * AH_E_LIMIT; every other byte 0).  Errors: AH_E_ARG (also: a table not read
 * from FASTQ), AH_E_IO, AH_E_FORMAT; *out is set only on success.
 * ---------------------------------------------------------------------- */
ah_status ah_fastq_read(const char *const *paths, uint32_t n_files, ah_fasta **out);
ah_status ah_fastq_bases(const ah_fasta *f, const char **h_bases, const uint64_t **h_off);
ah_status ah_fastq_qual_layout(const ah_fasta *f, uint8_t *h_qual, uint64_t cap);

/* Quality bytes of the amplicons ah_extract wrote, from the same amplicons,
 * pass flags, options and offsets (d_seq_off): for each written amplicon the
 * qualities of its bases in the order ah_extract wrote them -- forward, or
 * reversed for RF, whose bases are reverse-complemented -- at d_out +
 * d_seq_off[i].  d_qual: the device copy of ah_fastq_qual_layout's array
 * (qual_len >= 64 * st->n_blocks bytes).  Bytes at or past out_cap are not
 * written.  Asynchronous on stream; allocates nothing; AH_E_ARG for missing
 * arrays or a short d_qual. */
ah_status ah_extract_qual(const ah_store *st, const uint8_t *d_qual, uint64_t qual_len, ah_primer_set ps,
                          const ah_amp *d_amps, const uint64_t *d_n_amps, uint64_t amp_cap, const uint8_t *d_pass,
                          const ah_extract_opts *o, const uint64_t *d_seq_off, uint8_t *d_out, uint64_t out_cap,
                          void *stream);

/* FASTQ output: the records of ah_fasta_format with "@" in place of ">" and,
 * after the bases, a "+" line and the amplicon's qualities (h_qual at the
 * offsets of h_seq).  Same arguments and errors as ah_fasta_format. */
ah_status ah_fastq_format(const ah_fasta_names *names, uint32_t fb_len, uint32_t rb_len, const ah_amp *h_amps,
                          uint64_t n_amps, const double *h_tm, const uint8_t *h_pass, const char *h_seq,
                          const uint64_t *h_seq_off, const char *h_qual, const char *h_fb, const char *h_rb,
                          const uint8_t *h_bc_len, const char *h_fprimer, const char *h_rprimer, char *h_out,
                          uint64_t out_cap, uint64_t *h_n_bytes);

#ifdef __cplusplus
}
#endif

#endif /* AH_H */
