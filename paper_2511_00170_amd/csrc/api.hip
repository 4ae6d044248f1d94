// Host-side entry points of libah.so: status strings, store layout and the
// primer-set compiler (per-base IUPAC masks and reverse-complement masks,
// Supplementary "Primer matching and clamp logic").
#include <string.h>

#include <vector>

#include "ah_internal.h"

extern "C" const char *ah_status_str(ah_status s) {
    switch (s) {
    case AH_OK: return "ok";
    case AH_E_ARG: return "invalid argument";
    case AH_E_ALPHABET: return "primer letter is not an IUPAC nucleotide code";
    case AH_E_LIMIT: return "size limit exceeded (primer length 1..32, clamp <= length, pairs, key width)";
    case AH_E_HIP: return "HIP runtime error";
    case AH_E_WORKSPACE: return "workspace too small";
    case AH_E_IO: return "file could not be opened or read";
    case AH_E_FORMAT: return "not FASTA (data before the first header, record or record count too large)";
    case AH_E_SCRATCH: return "input larger than the library's fixed scratch array allows";
    default: return "unknown status";
    }
}

extern "C" int ah_version(void) { return 1; }

extern "C" ah_status ah_pack_layout(const uint64_t *h_lens, uint32_t n_seqs, uint64_t *h_seq_block0,
                                    uint64_t *h_n_blocks) {
    if ((!h_lens || !h_seq_block0) && n_seqs) return AH_E_ARG;
    if (!h_n_blocks) return AH_E_ARG;
    uint64_t b = 0;
    for (uint32_t i = 0; i < n_seqs; i++) {
        if (h_lens[i] >= (1ull << 32)) return AH_E_LIMIT;
        h_seq_block0[i] = b;
        b += (h_lens[i] + 63) / 64;
    }
    *h_n_blocks = b;
    return AH_OK;
}

// IUPAC nucleotide code -> set of bases, bit b for base b (A=0, C=1, G=2, T=3).
static int iupac_bits(char ch) {
    static const char *names = "ACGTURYSWKMBDHVN";
    static const int sets[16] = {
        1, 2, 4, 8, 8,            // A C G T U
        1 | 4, 2 | 8,             // R (A/G)  Y (C/T)
        2 | 4, 1 | 8,             // S (C/G)  W (A/T)
        4 | 8, 1 | 2,             // K (G/T)  M (A/C)
        14, 13, 11, 7,            // B (not A) D (not C) H (not G) V (not T)
        15};                      // N
    char u = (ch >= 'a' && ch <= 'z') ? (char)(ch - 32) : ch;
    const char *p = u ? strchr(names, u) : nullptr;
    return p ? sets[p - names] : 0;
}

// Complement of a base set: base b <-> 3 - b.
static int comp_bits(int m) {
    int r = 0;
    for (int b = 0; b < 4; b++)
        if (m & (1 << b)) r |= 1 << (3 - b);
    return r;
}

static ah_status parse_primer(const char *s, int *masks, int *L) {
    if (!s) return AH_E_ARG;
    size_t n = strlen(s);
    if (n < 1 || n > AH_MAXL) return AH_E_LIMIT;
    for (size_t j = 0; j < n; j++) {
        masks[j] = iupac_bits(s[j]);
        if (!masks[j]) return AH_E_ALPHABET;
    }
    *L = (int)n;
    return AH_OK;
}

static void make_pattern(const int *X, int L, int k, int clamp, int minus, uint32_t pair, uint32_t kind, DPat *d) {
    memset(d, 0, sizeof(*d));
    for (int j = 0; j < L; j++)
        for (int b = 0; b < 4; b++)
            if (X[j] & (1 << b)) d->P[b] |= 1u << j;
    d->lmask = L == 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
    for (int j = 0; j < clamp; j++) d->clampmask |= 1u << (minus ? j : L - 1 - j);
    int W = clamp < AH_WMAX ? clamp : AH_WMAX;
    // clamp site q = window start + shift; for the plus strand the filter's
    // first position, for W = 0 the last base (q must lie inside the window)
    int shift = minus ? 0 : L - (W > 0 ? W : 1);
    for (int i = 0; i < W; i++) d->fcode[i] = (uint8_t)(minus ? X[i] : X[L - W + i]);
    int kk = k > 255 ? 255 : k;
    d->meta = (uint32_t)L | ((uint32_t)kk << 8) | ((uint32_t)W << 16) | ((uint32_t)shift << 24);
    d->pk = pair | (kind << 16);
}

static void make_primer(const int *m, int L, DPrimer *p) {
    memset(p, 0, sizeof(*p));
    p->L = (uint8_t)L;
    uint64_t D = 1;
    for (int j = 0; j < L; j++) {
        int n = 0, first = -1;
        for (int b = 0; b < 4; b++)
            if (m[j] & (1 << b)) {
                if (first < 0) first = b;
                n++;
            }
        p->code[j] = (uint8_t)first;
        p->base |= (uint64_t)first << (2 * j);
        if (n > 1) {
            int d = p->n_deg++;
            p->deg_pos[d] = (uint8_t)j;
            p->deg_n[d] = (uint8_t)n;
            int c = 0;
            for (int b = 0; b < 4; b++)
                if (m[j] & (1 << b)) p->deg_base[d][c++] = (uint8_t)b;
        }
        D *= (uint64_t)n;
        if (D > AH_MAX_VARIANTS) D = (uint64_t)AH_MAX_VARIANTS + 1;
    }
    p->D = D > AH_MAX_VARIANTS ? 0u : (uint32_t)D;  // 0: too many variants for Tm
    if (!p->D) return;
    // split the degenerate positions: the longest run of last positions with
    // at most AH_VARTAB combinations (b), the rest (a)
    uint32_t rb = 1;
    int d0 = p->n_deg;
    while (d0 > 0 && rb * p->deg_n[d0 - 1] <= AH_VARTAB) rb *= p->deg_n[--d0];
    const uint32_t ra = p->D / rb;
    if (ra > AH_VARTAB) return;
    uint64_t lo_mask = 0;
    for (int d = d0; d < p->n_deg; d++) lo_mask |= 3ull << (2 * p->deg_pos[d]);
    for (uint32_t b = 0; b < rb; b++) p->lo[b] = primer_variant(*p, p->base, b) & lo_mask;
    for (uint32_t a = 0; a < ra; a++) p->hi[a] = primer_variant(*p, p->base, a * rb) & ~lo_mask;
    for (uint32_t v = 0; v < p->D; v++)
        if ((p->hi[v / rb] | p->lo[v % rb]) != primer_variant(*p, p->base, v)) return;  // (cannot happen)
    p->rb = rb;
    p->ra = ra;
}

// Build the primer set's host tables; unless host_only, also its device tables.
ah_status ah_build_primer_set(const ah_pair_spec *h_pairs, uint32_t n_pairs, bool host_only, ah_primer_set *out) {
    if (!out || (!h_pairs && n_pairs)) return AH_E_ARG;
    if (n_pairs == 0) return AH_E_ARG;
    if (n_pairs > AH_MAX_PAIRS) return AH_E_LIMIT;
    std::vector<DPat> pats(4 * (size_t)n_pairs);
    std::vector<DPair> prs(n_pairs);
    uint32_t maxL = 0, maxW = 0, minW = AH_WMAX;
    for (uint32_t q = 0; q < n_pairs; q++) {
        const ah_pair_spec &sp = h_pairs[q];
        int mf[AH_MAXL], mr[AH_MAXL], Lf = 0, Lr = 0;
        ah_status e = parse_primer(sp.fwd, mf, &Lf);
        if (e) return e;
        e = parse_primer(sp.rev, mr, &Lr);
        if (e) return e;
        if ((int)sp.clamp > (Lf < Lr ? Lf : Lr)) return AH_E_LIMIT;
        if (sp.min_len > sp.max_len) return AH_E_ARG;
        int rf[AH_MAXL], rr[AH_MAXL];  // reverse complements
        for (int j = 0; j < Lf; j++) rf[j] = comp_bits(mf[Lf - 1 - j]);
        for (int j = 0; j < Lr; j++) rr[j] = comp_bits(mr[Lr - 1 - j]);
        int k = (int)(sp.k > 255 ? 255 : sp.k), c = (int)sp.clamp;
        make_pattern(mf, Lf, k, c, 0, q, 0, &pats[4 * q + 0]);  // F+
        make_pattern(mr, Lr, k, c, 0, q, 1, &pats[4 * q + 1]);  // R+
        make_pattern(rf, Lf, k, c, 1, q, 2, &pats[4 * q + 2]);  // F-
        make_pattern(rr, Lr, k, c, 1, q, 3, &pats[4 * q + 3]);  // R-
        DPair &P = prs[q];
        memset(&P, 0, sizeof(P));
        P.min_len = sp.min_len;
        P.max_len = sp.max_len;
        P.Lf = (uint8_t)Lf;
        P.Lr = (uint8_t)Lr;
        P.k = (uint8_t)k;
        P.clamp = (uint8_t)c;
        make_primer(mf, Lf, &P.prim[0]);
        make_primer(mr, Lr, &P.prim[1]);
        maxL = (uint32_t)(Lf > (int)maxL ? Lf : maxL);
        maxL = (uint32_t)(Lr > (int)maxL ? Lr : maxL);
        uint32_t W = c < AH_WMAX ? (uint32_t)c : AH_WMAX;
        if (W > maxW) maxW = W;
        if (W < minW) minW = W;
    }
    ah_primer_set ps = new ah_primer_set_();
    ps->n_pairs = n_pairs;
    ps->n_pats = 4 * n_pairs;
    ps->max_L = maxL;
    ps->max_W = maxW;
    ps->min_W = minW;
    ps->h_pats = new DPat[pats.size()];
    memcpy(ps->h_pats, pats.data(), pats.size() * sizeof(DPat));
    ps->h_pairs = new DPair[n_pairs];
    memcpy(ps->h_pairs, prs.data(), prs.size() * sizeof(DPair));
    if (host_only) {
        *out = ps;
        return AH_OK;
    }
    ps->owns_device = 1;
    if (hipGetDevice(&ps->device) != hipSuccess ||
        hipMalloc((void **)&ps->d_pats, pats.size() * sizeof(DPat)) != hipSuccess ||
        hipMalloc((void **)&ps->d_pairs, prs.size() * sizeof(DPair)) != hipSuccess ||
        hipMemcpy(ps->d_pats, pats.data(), pats.size() * sizeof(DPat), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ps->d_pairs, prs.data(), prs.size() * sizeof(DPair), hipMemcpyHostToDevice) != hipSuccess) {
        ah_primers_free(ps);
        return AH_E_HIP;
    }
    *out = ps;
    return AH_OK;
}

extern "C" ah_status ah_primers_compile(const ah_pair_spec *h_pairs, uint32_t n_pairs, ah_primer_set *out) {
    return ah_build_primer_set(h_pairs, n_pairs, false, out);
}

extern "C" uint64_t ah_primers_table_bytes(uint32_t n_pairs) {
    return ah_pat_bytes(n_pairs) + (uint64_t)n_pairs * sizeof(DPair);
}

extern "C" ah_status ah_primers_compile_into(const ah_pair_spec *h_pairs, uint32_t n_pairs, void *d_buf,
                                             uint64_t buf_bytes, void *stream, ah_primer_set *out) {
    if (!out) return AH_E_ARG;
    if (!d_buf || buf_bytes < ah_primers_table_bytes(n_pairs)) return AH_E_WORKSPACE;
    ah_primer_set ps = nullptr;
    ah_status st = ah_build_primer_set(h_pairs, n_pairs, true, &ps);
    if (st != AH_OK) return st;
    hipStream_t s = ah_stream(stream);
    ps->d_pats = (DPat *)d_buf;
    ps->d_pairs = (DPair *)((char *)d_buf + ah_pat_bytes(n_pairs));
    ps->owns_device = 0;
    if (hipGetDevice(&ps->device) != hipSuccess ||
        hipMemcpyAsync(ps->d_pats, ps->h_pats, 4ull * n_pairs * sizeof(DPat), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(ps->d_pairs, ps->h_pairs, (uint64_t)n_pairs * sizeof(DPair), hipMemcpyHostToDevice, s) !=
            hipSuccess) {
        ps->d_pats = nullptr;
        ps->d_pairs = nullptr;
        ah_primers_free(ps);
        return AH_E_HIP;
    }
    *out = ps;
    return AH_OK;
}

extern "C" void ah_primers_free(ah_primer_set ps) {
    if (!ps) return;
    if (ps->owns_device && ps->d_pats) (void)hipFree(ps->d_pats);
    if (ps->owns_device && ps->d_pairs) (void)hipFree(ps->d_pairs);
    ah_jit_free(ps->jit);
    delete[] ps->h_pats;
    delete[] ps->h_pairs;
    delete ps;
}

extern "C" uint32_t ah_primers_count(ah_primer_set ps) { return ps ? ps->n_pairs : 0; }
