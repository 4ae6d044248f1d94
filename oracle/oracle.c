/*
 * Plain CPU oracle for the in-silico PCR hot path of AmpliconHunter2
 * (Howard-Stone & Mandoiu, arXiv 2511.00170).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  The GPU product
 * path never calls it and shares no code, table or header with it.
 *
 * Every function is a direct, slow restatement of what the paper defines:
 *   - primer matching: Supplementary "Primer matching and clamp logic" --
 *     per-base IUPAC masks, reverse-complement masks, substitution-only
 *     mismatch count, exact 3' clamp (defaults k=2, clamp 3 in Results);
 *   - amplicon calling: Supplementary "Amplicon calling and orientation" --
 *     sort sites, pair opposite-sense hits within the length bounds, stop at
 *     the next same-sense site, FR/RF/FF/RR, RF reverse-complemented;
 *   - melting temperature: Implementations, "AHv2" paragraph -- the
 *     nearest-neighbour Tm model of Biopython's Tm_NN (SantaLucia 1998
 *     formulation, parameter tables transcribed below with their sources);
 *   - trimming and barcodes: Supplementary "Primer trimming and barcode
 *     extraction"; header fields: Supplementary "Headers and outputs".
 * Where the paper is silent the readings are named in comments (R-...).
 *
 * Parity unpinned: the numeric values of the terminal-mismatch stacks (only
 * their physical range is checked), of the three tandem G.T stacks, and of
 * all but two dangling-end entries (only a range is checked).
 * Everything else of the Tm model is pinned outside this file: documented
 * Tm values of the Tm_NN model (every salt correction, the Watson-Crick
 * tables, an internal mismatch, dangling ends), the free energies printed
 * beside each Watson-Crick and internal-mismatch table, and duplexes summed
 * by hand (terminal mismatches, initiation, dangling ends).
 *
 * Records exchanged with the Python wrapper (oracle/__init__.py):
 *   hit: 4 x u32 = {seq, pos, pair, kind | mm << 8}
 *        kind bit0 = reverse primer, bit1 = minus strand (site of rc(primer))
 *   amplicon: 5 x u32 = {seq, start, end, pair, orient}  (0-based, half-open)
 *        orient 0=FR 1=RF 2=FF 3=RR
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXL 32

/* ------------------------------------------------------------------ */
/* O1: alphabet                                                         */
/* ------------------------------------------------------------------ */

/* Genome bases: A,C,G,T (any case) -> 0..3; every other byte is N (4).
 * R-N: an N never matches any primer code and cannot satisfy the clamp. */
static int genome_code(uint8_t ch)
{
    switch (ch) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return 4;
    }
}

static const char CODE_CHAR[5] = {'A', 'C', 'G', 'T', 'N'};

/* IUPAC nucleotide codes as sets of bases (bit A=1, C=2, G=4, T=8). */
static int iupac_set(char ch)
{
    switch (ch) {
    case 'A': case 'a': return 1;
    case 'C': case 'c': return 2;
    case 'G': case 'g': return 4;
    case 'T': case 't': case 'U': case 'u': return 8;
    case 'R': case 'r': return 1 | 4;      /* purine      A/G */
    case 'Y': case 'y': return 2 | 8;      /* pyrimidine  C/T */
    case 'S': case 's': return 2 | 4;      /* strong      C/G */
    case 'W': case 'w': return 1 | 8;      /* weak        A/T */
    case 'K': case 'k': return 4 | 8;      /* keto        G/T */
    case 'M': case 'm': return 1 | 2;      /* amino       A/C */
    case 'B': case 'b': return 2 | 4 | 8;  /* not A */
    case 'D': case 'd': return 1 | 4 | 8;  /* not C */
    case 'H': case 'h': return 1 | 2 | 8;  /* not G */
    case 'V': case 'v': return 1 | 2 | 4;  /* not T */
    case 'N': case 'n': return 15;
    default: return 0;
    }
}

/* IUPAC complement letters: A<->T, C<->G, R<->Y, K<->M, B<->V, D<->H; S, W, N self. */
static char iupac_complement(char ch)
{
    switch (ch) {
    case 'A': case 'a': return 'T';
    case 'T': case 't': case 'U': case 'u': return 'A';
    case 'C': case 'c': return 'G';
    case 'G': case 'g': return 'C';
    case 'R': case 'r': return 'Y';
    case 'Y': case 'y': return 'R';
    case 'K': case 'k': return 'M';
    case 'M': case 'm': return 'K';
    case 'B': case 'b': return 'V';
    case 'V': case 'v': return 'B';
    case 'D': case 'd': return 'H';
    case 'H': case 'h': return 'D';
    case 'S': case 's': return 'S';
    case 'W': case 'w': return 'W';
    case 'N': case 'n': return 'N';
    default: return 0;
    }
}

/* Primer string -> per-position masks.  Returns length, or -1 on a bad
 * letter, -2 on a bad length (1..32). */
int or_primer_masks(const char *primer, uint8_t *masks)
{
    int L = (int)strlen(primer);
    if (L < 1 || L > OR_MAXL) return -2;
    for (int j = 0; j < L; j++) {
        int m = iupac_set(primer[j]);
        if (!m) return -1;
        masks[j] = (uint8_t)m;
    }
    return L;
}

/* Reverse complement of a primer, as IUPAC letters (written into out). */
int or_primer_revcomp(const char *primer, char *out)
{
    int L = (int)strlen(primer);
    for (int j = 0; j < L; j++) {
        char c = iupac_complement(primer[L - 1 - j]);
        if (!c) return -1;
        out[j] = c;
    }
    out[L] = 0;
    return L;
}

/* ------------------------------------------------------------------ */
/* O2/O3: scan                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    int L;
    int k;
    int clamp;
    uint8_t mask[4][OR_MAXL]; /* [kind][j], kind: 0=F+, 1=R+, 2=F-, 3=R- */
} or_pair_pat;

static int build_pair(const char *fwd, const char *rev, int k, int clamp, or_pair_pat *pp, int *Lf, int *Lr)
{
    char rc[OR_MAXL + 1];
    int lf = or_primer_masks(fwd, pp->mask[0]);
    int lr = or_primer_masks(rev, pp->mask[1]);
    if (lf < 0 || lr < 0) return -1;
    or_primer_revcomp(fwd, rc);
    or_primer_masks(rc, pp->mask[2]);
    or_primer_revcomp(rev, rc);
    or_primer_masks(rc, pp->mask[3]);
    *Lf = lf;
    *Lr = lr;
    pp->k = k;
    pp->clamp = clamp;
    return 0;
}

typedef struct {
    uint32_t *v;
    uint64_t n, cap;
} vec32;

static void vpush4(vec32 *a, uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3)
{
    if (a->n + 4 > a->cap) {
        a->cap = a->cap ? a->cap * 2 : 1024;
        a->v = (uint32_t *)realloc(a->v, a->cap * sizeof(uint32_t));
    }
    a->v[a->n++] = x0;
    a->v[a->n++] = x1;
    a->v[a->n++] = x2;
    a->v[a->n++] = x3;
}

/* Is the pattern of `kind` (length L, clamp c) a hit at position p of the
 * sequence `codes`?  Definition: every clamp position matches and the number
 * of positions whose genome base is not in the primer code is <= k.  The
 * clamp sits at the primer's 3' end: the last c positions of the primer for a
 * plus-strand site, the first c positions of rc(primer) for a minus-strand
 * site.  Returns mm or -1. */
static int hit_at(const uint8_t *codes, uint64_t p, const uint8_t *mask, int L, int k, int c, int minus)
{
    int mm = 0;
    for (int j = 0; j < L; j++) {
        int b = codes[p + j];
        int match = (b < 4) && (mask[j] & (1 << b));
        if (!match) {
            int in_clamp = minus ? (j < c) : (j >= L - c);
            if (in_clamp) return -1;
            mm++;
            if (mm > k) return -1;
        }
    }
    return mm;
}

typedef struct {
    const uint8_t *ascii;
    const uint64_t *off;
    uint32_t s0, s1;
    const or_pair_pat *pats;
    const int *Lf, *Lr;
    uint32_t n_pairs;
    vec32 out;
} scan_job;

static void *scan_worker(void *arg)
{
    scan_job *jb = (scan_job *)arg;
    uint8_t *codes = NULL;
    uint64_t codes_cap = 0;
    for (uint32_t s = jb->s0; s < jb->s1; s++) {
        uint64_t n = jb->off[s + 1] - jb->off[s];
        if (n > codes_cap) {
            codes_cap = n;
            codes = (uint8_t *)realloc(codes, n ? n : 1);
        }
        for (uint64_t i = 0; i < n; i++) codes[i] = (uint8_t)genome_code(jb->ascii[jb->off[s] + i]);
        for (uint32_t q = 0; q < jb->n_pairs; q++) {
            const or_pair_pat *pp = &jb->pats[q];
            int Ls[4] = {jb->Lf[q], jb->Lr[q], jb->Lf[q], jb->Lr[q]};
            uint64_t pmax = 0;
            int Lmin = Ls[0] < Ls[1] ? Ls[0] : Ls[1];
            if (n < (uint64_t)Lmin) continue;
            pmax = n - (uint64_t)Lmin;
            for (uint64_t p = 0; p <= pmax; p++) {
                for (int kind = 0; kind < 4; kind++) {
                    int L = Ls[kind];
                    if (p + (uint64_t)L > n) continue;
                    int mm = hit_at(codes, p, pp->mask[kind], L, pp->k, pp->clamp, kind >> 1);
                    if (mm >= 0) vpush4(&jb->out, s, (uint32_t)p, q, (uint32_t)kind | ((uint32_t)mm << 8));
                }
            }
        }
    }
    free(codes);
    return NULL;
}

/* Scan all sequences for all pairs.  primers: 2*n_pairs strings (F0,R0,F1,R1..).
 * Writes min(total, cap) hits in the order (seq, pair, pos, kind) and returns
 * the total, or a negative error. */
int64_t or_scan(const uint8_t *ascii, const uint64_t *off, uint32_t n_seqs, const char *const *primers,
                const int *k, const int *clamp, uint32_t n_pairs, uint32_t *out, uint64_t cap, int n_threads)
{
    or_pair_pat *pats = (or_pair_pat *)calloc(n_pairs ? n_pairs : 1, sizeof(or_pair_pat));
    int *Lf = (int *)calloc(n_pairs ? n_pairs : 1, sizeof(int));
    int *Lr = (int *)calloc(n_pairs ? n_pairs : 1, sizeof(int));
    for (uint32_t q = 0; q < n_pairs; q++) {
        if (build_pair(primers[2 * q], primers[2 * q + 1], k[q], clamp[q], &pats[q], &Lf[q], &Lr[q])) {
            free(pats); free(Lf); free(Lr);
            return -1;
        }
        if (clamp[q] < 0 || clamp[q] > (Lf[q] < Lr[q] ? Lf[q] : Lr[q]) || k[q] < 0) {
            free(pats); free(Lf); free(Lr);
            return -2;
        }
    }
    if (n_threads < 1) n_threads = 1;
    if ((uint32_t)n_threads > n_seqs) n_threads = n_seqs ? (int)n_seqs : 1;
    scan_job *jobs = (scan_job *)calloc((size_t)n_threads, sizeof(scan_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    /* contiguous sequence ranges balanced by base count */
    uint64_t total = off[n_seqs] - off[0];
    uint32_t s = 0;
    for (int t = 0; t < n_threads; t++) {
        uint64_t goal = off[0] + (total * (uint64_t)(t + 1)) / (uint64_t)n_threads;
        uint32_t e = s;
        while (e < n_seqs && (off[e + 1] <= goal || e == s)) e++;
        if (t == n_threads - 1) e = n_seqs;
        jobs[t] = (scan_job){ascii, off, s, e, pats, Lf, Lr, n_pairs, {0}};
        s = e;
    }
    for (int t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, scan_worker, &jobs[t]);
    uint64_t n_out = 0;
    for (int t = 0; t < n_threads; t++) {
        pthread_join(th[t], NULL);
        for (uint64_t i = 0; i < jobs[t].out.n; i += 4) {
            if (n_out < cap) memcpy(out + 4 * n_out, jobs[t].out.v + i, 4 * sizeof(uint32_t));
            n_out++;
        }
        free(jobs[t].out.v);
    }
    free(jobs); free(th); free(pats); free(Lf); free(Lr);
    return (int64_t)n_out;
}

/* ------------------------------------------------------------------ */
/* O4/O5: sites and pairing                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t start, end;
    int sense;  /* 0 = plus (points right), 1 = minus (points left) */
    int primer; /* 0 = forward, 1 = reverse */
} or_site;

/* R-sort: sites ordered by (start, end, plus before minus, F before R). */
static int site_cmp(const void *a, const void *b)
{
    const or_site *x = (const or_site *)a, *y = (const or_site *)b;
    if (x->start != y->start) return x->start < y->start ? -1 : 1;
    if (x->end != y->end) return x->end < y->end ? -1 : 1;
    if (x->sense != y->sense) return x->sense < y->sense ? -1 : 1;
    if (x->primer != y->primer) return x->primer < y->primer ? -1 : 1;
    return 0;
}

static int orient_of(int left_primer, int right_primer)
{
    if (left_primer == 0 && right_primer == 1) return 0; /* FR */
    if (left_primer == 1 && right_primer == 0) return 1; /* RF */
    if (left_primer == 0 && right_primer == 0) return 2; /* FF */
    return 3;                                            /* RR */
}

typedef struct {
    uint32_t seq, start, end, pair, orient;
    uint32_t r_start, r_end, r_primer; /* downstream site key, for ordering */
} or_amp_full;

/* Canonical amplicon order: (seq, pair, downstream-site start, end, primer). */
static int amp_cmp(const void *a, const void *b)
{
    const or_amp_full *x = (const or_amp_full *)a, *y = (const or_amp_full *)b;
    if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
    if (x->pair != y->pair) return x->pair < y->pair ? -1 : 1;
    if (x->r_start != y->r_start) return x->r_start < y->r_start ? -1 : 1;
    if (x->r_end != y->r_end) return x->r_end < y->r_end ? -1 : 1;
    if (x->r_primer != y->r_primer) return x->r_primer < y->r_primer ? -1 : 1;
    return 0;
}

typedef struct {
    uint32_t seq, pair;
    uint64_t i;
} sp_t;

static int sp_cmp(const void *a, const void *b)
{
    const sp_t *x = (const sp_t *)a, *y = (const sp_t *)b;
    if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
    if (x->pair != y->pair) return x->pair < y->pair ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

/* Pair hits (any order) into amplicons.  For every plus site a, walk the later
 * sites in sort order; stop at the first plus site; every minus site t met on
 * the way with min <= t.end - a.start <= max and a requested orientation is an
 * amplicon.  Sites of different (sequence, pair) never interact.  Writes
 * min(total, cap) amplicons in canonical order and returns the total. */
int64_t or_pair(const uint32_t *hits, uint64_t n_hits, const int *Lf, const int *Lr, const uint32_t *min_len,
                const uint32_t *max_len, uint32_t n_pairs, uint32_t orient_mask, uint32_t *out, uint64_t cap)
{
    (void)n_pairs;
    or_site *sites = (or_site *)malloc((n_hits ? n_hits : 1) * sizeof(or_site));
    or_amp_full *amps = NULL;
    uint64_t n_amps = 0, amps_cap = 0;

    /* group the hits by (seq, pair) */
    sp_t *sp = (sp_t *)malloc((n_hits ? n_hits : 1) * sizeof(sp_t));
    for (uint64_t i = 0; i < n_hits; i++) { sp[i].seq = hits[4 * i]; sp[i].pair = hits[4 * i + 2]; sp[i].i = i; }
    qsort(sp, n_hits, sizeof(sp_t), sp_cmp);

    uint64_t g0 = 0;
    while (g0 < n_hits) {
        uint64_t g1 = g0;
        while (g1 < n_hits && sp[g1].seq == sp[g0].seq && sp[g1].pair == sp[g0].pair) g1++;
        uint32_t seq = sp[g0].seq, q = sp[g0].pair;
        uint64_t m = g1 - g0;
        for (uint64_t u = 0; u < m; u++) {
            const uint32_t *h = hits + 4 * sp[g0 + u].i;
            int kind = (int)(h[3] & 0xFF);
            int primer = kind & 1, sense = (kind >> 1) & 1;
            int L = primer ? Lr[q] : Lf[q];
            sites[u].start = h[1];
            sites[u].end = h[1] + (uint32_t)L;
            sites[u].sense = sense;
            sites[u].primer = primer;
        }
        qsort(sites, m, sizeof(or_site), site_cmp);
        for (uint64_t a = 0; a < m; a++) {
            if (sites[a].sense != 0) continue;
            for (uint64_t t = a + 1; t < m; t++) {
                if (sites[t].sense == 0) break; /* same-sense site: stop */
                uint64_t len = (uint64_t)sites[t].end - (uint64_t)sites[a].start;
                int o = orient_of(sites[a].primer, sites[t].primer);
                if (len >= min_len[q] && len <= max_len[q] && (orient_mask >> o) & 1) {
                    if (n_amps == amps_cap) {
                        amps_cap = amps_cap ? 2 * amps_cap : 256;
                        amps = (or_amp_full *)realloc(amps, amps_cap * sizeof(or_amp_full));
                    }
                    amps[n_amps++] = (or_amp_full){seq, sites[a].start, sites[t].end, q, (uint32_t)o,
                                                   sites[t].start, sites[t].end, (uint32_t)sites[t].primer};
                }
            }
        }
        g0 = g1;
    }
    qsort(amps, n_amps, sizeof(or_amp_full), amp_cmp);
    for (uint64_t i = 0; i < n_amps && i < cap; i++) {
        out[5 * i + 0] = amps[i].seq;
        out[5 * i + 1] = amps[i].start;
        out[5 * i + 2] = amps[i].end;
        out[5 * i + 3] = amps[i].pair;
        out[5 * i + 4] = amps[i].orient;
    }
    free(sites); free(amps); free(sp);
    return (int64_t)n_amps;
}

/* ------------------------------------------------------------------ */
/* O8: nearest-neighbour melting temperature                            */
/* ------------------------------------------------------------------ */
/*
 * Stack notation "XY/WZ": top strand 5'-XY-3' paired with bottom strand
 * 3'-WZ-5' (X with W, Y with Z).  dH in kcal/mol, dS in cal/(K mol).
 * A stack read from the other strand, "ZW/YX", is the same physical stack;
 * a lookup tries the key as written first, then that reversed reading.
 *
 * Values are the published parameter sets, transcribed into this file.
 */
typedef struct {
    const char *key;
    double dh, ds;
} nn_param;

/* Nearest-neighbour parameter sets for DNA/DNA duplexes that the Tm_NN
 * model offers (selected by number, as it numbers them): Watson-Crick
 * stacks and initiation terms.  Initiation: `init` for every duplex, `at` /
 * `gc` per duplex end by its terminal pair, `one_gc` / `all_at` by whether
 * any G.C pair occurs.  (The model's 5'-terminal T.A penalty is zero in all
 * four sets and is left out.) */
typedef struct {
    nn_param stack[10];
    double init_dh, init_ds;
    double at_dh, at_ds;
    double gc_dh, gc_ds;
    double one_gc_dh, one_gc_ds;
    double all_at_dh, all_at_ds;
} nn_set;

static const nn_set NN_SETS[5] = {
    /* 0: unused (0 selects set 3) */
    {{{"", 0, 0}}, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    /* 1: Breslauer, Frank, Bloecker & Marky (1986) PNAS 83:3746, Table 2;
     *    initiation 5.0 (with a G.C pair) or 6.0 (A.T only) kcal/mol at 25 C,
     *    entropic. */
    {{{"AA/TT", -9.1, -24.0}, {"AT/TA", -8.6, -23.9}, {"TA/AT", -6.0, -16.9}, {"CA/GT", -5.8, -12.9},
      {"GT/CA", -6.5, -17.3}, {"CT/GA", -7.8, -20.8}, {"GA/CT", -5.6, -13.5}, {"CG/GC", -11.9, -27.8},
      {"GC/CG", -11.1, -26.7}, {"GG/CC", -11.0, -26.6}},
     0, 0, 0, 0, 0, 0, 0, -16.8, 0, -20.1},
    /* 2: Sugimoto, Nakano, Yoneyama & Honda (1996) Nucleic Acids Res
     *    24:4501, Table 1; one initiation term per duplex. */
    {{{"AA/TT", -8.0, -21.9}, {"AT/TA", -5.6, -15.2}, {"TA/AT", -6.6, -18.4}, {"CA/GT", -8.2, -21.0},
      {"GT/CA", -9.4, -25.5}, {"CT/GA", -6.6, -16.4}, {"GA/CT", -8.8, -23.5}, {"CG/GC", -11.8, -29.0},
      {"GC/CG", -10.5, -26.4}, {"GG/CC", -10.9, -28.4}},
     0.6, -9.0, 0, 0, 0, 0, 0, 0, 0, 0},
    /* 3 (default): unified parameters, SantaLucia (1998) PNAS 95:1460,
     *    Table 2 (= Allawi & SantaLucia (1997) Biochemistry 36:10581);
     *    initiation per end with a terminal G.C or A.T pair. */
    {{{"AA/TT", -7.9, -22.2}, {"AT/TA", -7.2, -20.4}, {"TA/AT", -7.2, -21.3}, {"CA/GT", -8.5, -22.7},
      {"GT/CA", -8.4, -22.4}, {"CT/GA", -7.8, -21.0}, {"GA/CT", -8.2, -22.2}, {"CG/GC", -10.6, -27.2},
      {"GC/CG", -9.8, -24.4}, {"GG/CC", -8.0, -19.9}},
     0, 0, 2.3, 4.1, 0.1, -2.8, 0, 0, 0, 0},
    /* 4: SantaLucia & Hicks (2004) Annu Rev Biophys Biomol Struct 33:415,
     *    Table 1; one initiation term plus a penalty per terminal A.T pair. */
    {{{"AA/TT", -7.6, -21.3}, {"AT/TA", -7.2, -20.4}, {"TA/AT", -7.2, -21.3}, {"CA/GT", -8.5, -22.7},
      {"GT/CA", -8.4, -22.4}, {"CT/GA", -7.8, -21.0}, {"GA/CT", -8.2, -22.2}, {"CG/GC", -10.6, -27.2},
      {"GC/CG", -9.8, -24.4}, {"GG/CC", -8.0, -19.9}},
     0.2, -5.7, 2.2, 6.9, 0, 0, 0, 0, 0, 0},
};

/* Internal single mismatches (one mismatched pair inside the stack; also
 * the tandem G.T stacks of the first paper):
 *   G.T  Allawi & SantaLucia (1997) Biochemistry 36:10581;
 *   G.A  Allawi & SantaLucia (1998) Biochemistry 37:2170;
 *   C.T  Allawi & SantaLucia (1998) Nucleic Acids Res 26:2694;
 *   A.C  Allawi & SantaLucia (1998) Biochemistry 37:9435;
 *   A.A, C.C, G.G, T.T  Peyret et al. (1999) Biochemistry 38:3468. */
static const nn_param NN_IMM[] = {
    /* G.T */
    {"AG/TT", 1.0, 0.9}, {"AT/TG", -2.5, -8.3}, {"CG/GT", -4.1, -11.7}, {"CT/GG", -2.8, -8.0},
    {"GG/CT", 3.3, 10.4}, {"GG/TT", 5.8, 16.3}, {"GT/CG", -4.4, -12.3}, {"GT/TG", 4.1, 9.5},
    {"TG/AT", -0.1, -1.7}, {"TG/GT", -1.4, -6.2}, {"TT/AG", -1.3, -5.3},
    /* G.A */
    {"AA/TG", -0.6, -2.3}, {"AG/TA", -0.7, -2.3}, {"CA/GG", -0.7, -2.3}, {"CG/GA", -4.0, -13.2},
    {"GA/CG", -0.6, -1.0}, {"GG/CA", 0.5, 3.2}, {"TA/AG", 0.7, 0.7}, {"TG/AA", 3.0, 7.4},
    /* C.T */
    {"AC/TT", 0.7, 0.2}, {"AT/TC", -1.2, -6.2}, {"CC/GT", -0.8, -4.5}, {"CT/GC", -1.5, -6.1},
    {"GC/CT", 2.3, 5.4}, {"GT/CC", 5.2, 13.5}, {"TC/AT", 1.2, 0.7}, {"TT/AC", 1.0, 0.7},
    /* A.C */
    {"AA/TC", 2.3, 4.6}, {"AC/TA", 5.3, 14.6}, {"CA/GC", 1.9, 3.7}, {"CC/GA", 0.6, -0.6},
    {"GA/CC", 5.2, 14.2}, {"GC/CA", -0.7, -3.8}, {"TA/AC", 3.4, 8.0}, {"TC/AA", 7.6, 20.2},
    /* A.A, C.C, G.G, T.T */
    {"AA/TA", 1.2, 1.7}, {"CA/GA", -0.9, -4.2}, {"GA/CA", -2.9, -9.8}, {"TA/AA", 4.7, 12.9},
    {"AC/TC", 0.0, -4.4}, {"CC/GC", -1.5, -7.2}, {"GC/CC", 3.6, 8.9}, {"TC/AC", 6.1, 16.4},
    {"AG/TG", -3.1, -9.5}, {"CG/GG", -4.9, -15.3}, {"GG/CG", -6.0, -15.8}, {"TG/AG", 1.6, 3.6},
    {"AT/TT", -2.7, -10.8}, {"CT/GT", -5.0, -15.8}, {"GT/CT", -2.2, -8.4}, {"TT/AT", 0.2, -1.5},
};

/* Terminal mismatches: the second pair of the stack is the mismatched duplex
 * end, the first a Watson-Crick pair.  The Tm_NN model's DNA table, from
 * SantaLucia & Peyret (2001), patent application WO 01/94611. */
static const nn_param NN_TMM[] = {
    {"AA/TA", -3.1, -7.8}, {"TA/AA", -2.5, -6.3}, {"CA/GA", -4.3, -10.7}, {"GA/CA", -8.0, -22.5},
    {"AC/TC", -0.1, 0.5}, {"TC/AC", -0.7, -1.3}, {"CC/GC", -2.1, -5.1}, {"GC/CC", -3.9, -10.6},
    {"AG/TG", -1.1, -2.1}, {"TG/AG", -1.1, -2.7}, {"CG/GG", -3.8, -9.5}, {"GG/CG", -0.7, -19.2},
    {"AT/TT", -2.4, -6.5}, {"TT/AT", -3.2, -8.9}, {"CT/GT", -6.1, -16.9}, {"GT/CT", -7.4, -21.2},
    {"AA/TC", -1.6, -4.0}, {"AC/TA", -1.8, -3.8}, {"CA/GC", -2.6, -5.9}, {"CC/GA", -2.7, -6.0},
    {"GA/CC", -5.0, -13.8}, {"GC/CA", -3.2, -7.1}, {"TA/AC", -2.3, -5.9}, {"TC/AA", -2.7, -7.0},
    {"AC/TT", -0.9, -1.7}, {"AT/TC", -2.3, -6.3}, {"CC/GT", -3.2, -8.0}, {"CT/GC", -3.9, -10.6},
    {"GC/CT", -4.9, -13.5}, {"GT/CC", -3.0, -7.8}, {"TC/AT", -2.5, -6.3}, {"TT/AC", -0.7, -1.2},
    {"AA/TG", -1.9, -4.4}, {"AG/TA", -2.5, -5.9}, {"CA/GG", -3.9, -9.6}, {"CG/GA", -6.0, -15.5},
    {"GA/CG", -4.3, -11.1}, {"GG/CA", -4.6, -11.4}, {"TA/AG", -2.0, -4.7}, {"TG/AA", -2.4, -5.8},
    {"AG/TT", -3.2, -8.7}, {"AT/TG", -3.5, -9.4}, {"CG/GT", -3.8, -9.0}, {"CT/GG", -6.6, -18.7},
    {"GG/CT", -5.7, -15.9}, {"GT/CG", -5.9, -16.1}, {"TG/AT", -3.9, -10.5}, {"TT/AG", -3.6, -9.8},
};

/* Dangling ends: one unpaired base ('.' opposite it) beside a terminal
 * Watson-Crick pair.  "XY/.Z": top 5'-XY-3' over bottom 3'-.Z-5', X a
 * 5'-dangling base of the top strand; ".X/YZ": top 5'-.X-3' over bottom
 * 3'-YZ-5', Y a 3'-dangling base of the bottom strand.  Bommarito, Peyret &
 * SantaLucia (2000) Nucleic Acids Res 28:1929. */
static const nn_param NN_DE[] = {
    {"AA/.T", 0.2, 2.3}, {"AC/.G", -6.3, -17.1}, {"AG/.C", -3.7, -10.0}, {"AT/.A", -2.9, -7.6},
    {"CA/.T", 0.6, 3.3}, {"CC/.G", -4.4, -12.6}, {"CG/.C", -4.0, -11.9}, {"CT/.A", -4.1, -13.0},
    {"GA/.T", -1.1, -1.6}, {"GC/.G", -5.1, -14.0}, {"GG/.C", -3.9, -10.9}, {"GT/.A", -4.2, -15.0},
    {"TA/.T", -6.9, -20.0}, {"TC/.G", -4.0, -10.9}, {"TG/.C", -4.9, -13.8}, {"TT/.A", -0.2, -0.5},
    {".A/AT", -0.7, -0.8}, {".C/AG", -2.1, -3.9}, {".G/AC", -5.9, -16.5}, {".T/AA", -0.5, -1.1},
    {".A/CT", 4.4, 14.9}, {".C/CG", -0.2, -0.1}, {".G/CC", -2.6, -7.4}, {".T/CA", 4.7, 14.2},
    {".A/GT", -1.6, -3.6}, {".C/GG", -3.9, -11.2}, {".G/GC", -3.2, -10.4}, {".T/GA", -4.1, -13.1},
    {".A/TT", 2.9, 10.4}, {".C/TG", -4.4, -13.1}, {".G/TC", -5.2, -15.0}, {".T/TA", -3.8, -12.6},
};

#define NPAR(t) ((int)(sizeof(t) / sizeof((t)[0])))

/* Find "XY/WZ" in a table as written. */
static const nn_param *nn_exact(const nn_param *tab, int n, const char key[6])
{
    for (int i = 0; i < n; i++)
        if (!strcmp(tab[i].key, key)) return &tab[i];
    return NULL;
}

/* Find "XY/WZ" in a table, first as written, then read from the other strand. */
static const nn_param *nn_find(const nn_param *tab, int n, const char key[6])
{
    char rev[6] = {key[4], key[3], '/', key[1], key[0], 0};
    const nn_param *p = nn_exact(tab, n, key);
    return p ? p : nn_exact(tab, n, rev);
}

static int wc_pair(char top, char bottom)
{
    return (top == 'A' && bottom == 'T') || (top == 'T' && bottom == 'A') || (top == 'C' && bottom == 'G') ||
           (top == 'G' && bottom == 'C');
}

typedef struct {
    double na, k, tris, mg, dntps; /* mM */
    double dnac1, dnac2;           /* nM */
    int saltcorr;
    int nn_table;                  /* 1..4 as in NN_SETS; 0 = 3 */
} or_tm_cond;

/* Monovalent-equivalent concentration in M (von Ahsen et al. 2001 for Mg2+). */
static double mono_equiv_M(const or_tm_cond *c)
{
    double mon = c->na + c->k + c->tris / 2.0;
    if (c->dntps < c->mg) mon += 120.0 * sqrt(c->mg - c->dntps);
    return mon * 1e-3;
}

/*
 * Salt correction of the nearest-neighbour Tm, the seven methods the Tm_NN
 * model offers (Implementations, "AHv2" paragraph: every salt correction
 * method), each written from its paper.  `seq` is the primer strand (length
 * N, G+C fraction fgc).  mon = Na + K + Tris/2 plus, for methods 1-6, the
 * von Ahsen (2001) Mg2+ equivalent 120 sqrt(Mg - dNTPs) when Mg > dNTPs; M.
 *   1 Schildkraut & Lifson 1965   dTm = 16.6 log10(mon)
 *   2 Wetmur 1991                 dTm = 16.6 log10(mon / (1 + 0.7 mon))
 *   3 SantaLucia et al. 1996      dTm = 12.5 log10(mon)
 *   4 SantaLucia 1998             dTm = 11.7 log10(mon)
 *   5 SantaLucia 1998             dS += 0.368 (N - 1) ln(mon)
 *   6 Owczarzy et al. 2004        d(1/Tm) = (4.29 fgc - 3.95) 1e-5 ln(mon) + 9.40e-6 ln(mon)^2
 *   7 Owczarzy et al. 2008        Mg2+ model: free Mg2+ after dNTP binding
 *                                 (Ka = 3e4 /M); ratio R = sqrt(Mg)/mon; R < 0.22:
 *                                 method 6; otherwise d(1/Tm) = 1e-5 [a + b ln Mg
 *                                 + fgc (c + d ln Mg) + (e + f ln Mg + g ln^2 Mg)
 *                                 / (2 (N - 1))], with a, d, g depending on mon
 *                                 when R < 6.
 * *kind: 1 add to Tm (C), 5 add to dS, 6 add to 1/Tm (1/K).  Returns 0, or 2
 * when a logarithm of a zero concentration would be needed.
 */
int or_salt_correction(const or_tm_cond *c, const char *seq, double *corr, int *kind)
{
    int N = (int)strlen(seq), gc = 0;
    for (int j = 0; j < N; j++) gc += (seq[j] == 'G' || seq[j] == 'C' || seq[j] == 'S');
    double fgc = N ? (double)gc / N : 0.0;
    *corr = 0.0;
    *kind = 0;
    if (c->saltcorr == 0) return 0;
    if (c->saltcorr >= 1 && c->saltcorr <= 6) {
        double mon = mono_equiv_M(c);
        if (!(mon > 0.0)) return 2;
        switch (c->saltcorr) {
        case 1: *corr = 16.6 * log10(mon); *kind = 1; break;
        case 2: *corr = 16.6 * log10(mon / (1.0 + 0.7 * mon)); *kind = 1; break;
        case 3: *corr = 12.5 * log10(mon); *kind = 1; break;
        case 4: *corr = 11.7 * log10(mon); *kind = 1; break;
        case 5: *corr = 0.368 * (double)(N - 1) * log(mon); *kind = 5; break;
        default:
            *corr = (4.29 * fgc - 3.95) * 1e-5 * log(mon) + 9.40e-6 * log(mon) * log(mon);
            *kind = 6;
        }
        return 0;
    }
    if (c->saltcorr != 7) return 2;
    double mon = (c->na + c->k + c->tris / 2.0) * 1e-3;
    double mg = c->mg * 1e-3;
    if (c->dntps > 0.0) {
        /* free Mg2+: [Mg][dNTP] / [MgdNTP] = 1 / Ka with both totals conserved */
        double ka = 3e4, dn = c->dntps * 1e-3;
        double bq = ka * dn - ka * mg + 1.0;
        mg = (-bq + sqrt(bq * bq + 4.0 * ka * mg)) / (2.0 * ka);
    }
    *kind = 6;
    double a = 3.92, b = -0.911, cc = 6.26, d = 1.42, e = -48.2, f = 52.5, g = 8.31;
    if (mon > 0.0) {
        double R = sqrt(mg) / mon, lm = log(mon);
        if (R < 0.22) {
            *corr = (4.29 * fgc - 3.95) * 1e-5 * lm + 9.40e-6 * lm * lm;
            return 0;
        }
        if (R < 6.0) {
            a = 3.92 * (0.843 - 0.352 * sqrt(mon) * lm);
            d = 1.42 * (1.279 - 4.03e-3 * lm - 8.03e-3 * lm * lm);
            g = 8.31 * (0.486 - 0.258 * lm + 5.25e-3 * lm * lm * lm);
        }
    }
    if (!(mg > 0.0) || N < 2) return 2;
    double lg = log(mg);
    *corr = (a + b * lg + fgc * (cc + d * lg) + (e + f * lg + g * lg * lg) / (2.0 * (N - 1))) * 1e-5;
    return 0;
}

#define OR_MAXC 64 /* longest partner strand of an explicit duplex */

/*
 * dH and dS (before salt correction) of the duplex of `seq` (5'->3', 2..32
 * letters) with `cseq` (its partner strand written 3'->5', 1..64 letters),
 * cseq[i] facing seq[i - shift] (shift 0 with equal lengths: position j
 * pairs with position j).  `table` selects the Watson-Crick set (NN_SETS).
 * Returns 0 ok, 1 untabulated stack or end or a non-ACGT letter, 2 bad input
 * (fewer than two facing positions).  or_tm_duplex adds the salt term.
 * Steps, in this order (the Tm_NN model; SantaLucia 1998 formulation):
 *  1. align the strands; an end may keep one unpaired base of either strand
 *     (a dangling end), any further overhang is ignored;
 *  2. a dangling end is charged with its dangling-end parameter and leaves
 *     the duplex (left end first, then right end);
 *  3. a mismatched end pair is charged with the terminal-mismatch stack and
 *     leaves the helix (left, then right);
 *  4. initiation from the primer strand as given (R-init: its end bases and
 *     whether it holds a G or C choose the terms, also when an end pair was
 *     removed in steps 2-3, as the Tm_NN model does);
 *  5. the stacks of the remaining pairs in 5'->3' order: Watson-Crick set,
 *     else the internal-mismatch table; a stack in neither is untabulated.
 */
int or_nn_thermo(const char *seq, const char *cseq, int shift, int table, double *dh_out, double *ds_out)
{
    int L = (int)strlen(seq), Lc = (int)strlen(cseq);
    if (L < 2 || L > OR_MAXL || Lc < 1 || Lc > OR_MAXC || shift < -OR_MAXC || shift > OR_MAXC) return 2;
    if (table == 0) table = 3;
    if (table < 1 || table > 4) return 2;
    const nn_set *set = &NN_SETS[table];
    for (int j = 0; j < L; j++)
        if (!strchr("ACGT", seq[j])) return 1;
    for (int j = 0; j < Lc; j++)
        if (!strchr("ACGT", cseq[j])) return 1;

    /* 1. alignment: column i holds top[i] over bot[i], '.' = no base */
    char top[2 * OR_MAXC + 8], bot[2 * OR_MAXC + 8];
    int st = shift > 0 ? shift : 0, sb = shift < 0 ? -shift : 0;
    int n = L + st > Lc + sb ? L + st : Lc + sb;
    for (int i = 0; i < n; i++) {
        top[i] = (i >= st && i < st + L) ? seq[i - st] : '.';
        bot[i] = (i >= sb && i < sb + Lc) ? cseq[i - sb] : '.';
    }
    int facing = 0;
    for (int i = 0; i < n; i++) facing += top[i] != '.' && bot[i] != '.';
    if (facing < 2) return 2;
    int lo = 0, hi = n - 1; /* inclusive column range still in the duplex */
    while ((top[lo] == '.' && top[lo + 1] == '.') || (bot[lo] == '.' && bot[lo + 1] == '.')) lo++;
    while ((top[hi] == '.' && top[hi - 1] == '.') || (bot[hi] == '.' && bot[hi - 1] == '.')) hi--;

    double dh = 0.0, ds = 0.0;
    char key[6];
    key[2] = '/';
    key[5] = 0;
    const nn_param *p;

    /* 2. dangling ends; the right end is read from the partner strand */
    if (top[lo] == '.' || bot[lo] == '.') {
        key[0] = top[lo]; key[1] = top[lo + 1]; key[3] = bot[lo]; key[4] = bot[lo + 1];
        if (!(p = nn_exact(NN_DE, NPAR(NN_DE), key))) return 1;
        dh += p->dh; ds += p->ds; lo++;
    }
    if (top[hi] == '.' || bot[hi] == '.') {
        key[0] = bot[hi]; key[1] = bot[hi - 1]; key[3] = top[hi]; key[4] = top[hi - 1];
        if (!(p = nn_exact(NN_DE, NPAR(NN_DE), key))) return 1;
        dh += p->dh; ds += p->ds; hi--;
    }

    /* 3. terminal mismatches; the left end is read from the partner strand
     * so that the end pair comes second */
    key[0] = bot[lo + 1]; key[1] = bot[lo]; key[3] = top[lo + 1]; key[4] = top[lo];
    if ((p = nn_exact(NN_TMM, NPAR(NN_TMM), key))) { dh += p->dh; ds += p->ds; lo++; }
    if (hi - 1 >= lo) {
        key[0] = top[hi - 1]; key[1] = top[hi]; key[3] = bot[hi - 1]; key[4] = bot[hi];
        if ((p = nn_exact(NN_TMM, NPAR(NN_TMM), key))) { dh += p->dh; ds += p->ds; hi--; }
    }

    /* 4. initiation from the primer strand as given */
    {
        int any_gc = 0;
        for (int j = 0; j < L; j++) any_gc |= seq[j] == 'G' || seq[j] == 'C';
        dh += set->init_dh; ds += set->init_ds;
        if (any_gc) { dh += set->one_gc_dh; ds += set->one_gc_ds; }
        else { dh += set->all_at_dh; ds += set->all_at_ds; }
        char ends[2] = {seq[0], seq[L - 1]};
        for (int e = 0; e < 2; e++) {
            if (ends[e] == 'A' || ends[e] == 'T') { dh += set->at_dh; ds += set->at_ds; }
            else { dh += set->gc_dh; ds += set->gc_ds; }
        }
    }

    /* 5. stacks */
    for (int j = lo; j < hi; j++) {
        key[0] = top[j]; key[1] = top[j + 1]; key[3] = bot[j]; key[4] = bot[j + 1];
        if (wc_pair(top[j], bot[j]) && wc_pair(top[j + 1], bot[j + 1]))
            p = nn_find(set->stack, 10, key);
        else
            p = nn_find(NN_IMM, NPAR(NN_IMM), key);
        if (!p) return 1;
        dh += p->dh;
        ds += p->ds;
    }

    *dh_out = dh;
    *ds_out = ds;
    return 0;
}

/* Tm (degrees C) of the duplex: the salt correction (on the primer strand),
 * then Tm = 1000 dH / (dS + R ln C) - 273.15, R = 1.987, C = C_high -
 * C_low / 2 for two distinct strands (R-selfcomp: never the self-
 * complementary form).  *status = 0 ok, 1 untabulated (returns -inf), 2 bad
 * input. */
double or_tm_duplex(const char *seq, const char *cseq, int shift, const or_tm_cond *cond, int *status)
{
    double dh = 0.0, ds = 0.0;
    *status = or_nn_thermo(seq, cseq, shift, cond->nn_table, &dh, &ds);
    if (*status == 2) return 0.0;
    if (*status == 1) return -INFINITY;

    double corr = 0.0;
    int kind = 0;
    if (or_salt_correction(cond, seq, &corr, &kind)) { *status = 2; return 0.0; }
    if (kind == 5) ds += corr;
    double hiC = cond->dnac1 > cond->dnac2 ? cond->dnac1 : cond->dnac2;
    double loC = cond->dnac1 > cond->dnac2 ? cond->dnac2 : cond->dnac1;
    double C = (hiC - loC / 2.0) * 1e-9;
    double tm = (1000.0 * dh) / (ds + 1.987 * log(C)) - 273.15;
    if (kind == 1) tm += corr;
    if (kind == 6) tm = 1.0 / (1.0 / (tm + 273.15) + corr) - 273.15;
    return tm;
}

/* The partner table: parameter values of one set or table for inspection
 * by the tests (which=0: Watson-Crick set `table`; 1 internal mismatches;
 * 2 terminal mismatches; 3 dangling ends).  Returns the number of entries
 * and copies up to cap keys (6 bytes each) and (dH, dS) pairs. */
int or_nn_table(int which, int table, char *keys, double *vals, int cap)
{
    const nn_param *t;
    int n;
    if (which == 0) {
        if (table == 0) table = 3;
        if (table < 1 || table > 4) return -1;
        t = NN_SETS[table].stack; n = 10;
    } else if (which == 1) { t = NN_IMM; n = NPAR(NN_IMM); }
    else if (which == 2) { t = NN_TMM; n = NPAR(NN_TMM); }
    else if (which == 3) { t = NN_DE; n = NPAR(NN_DE); }
    else return -1;
    for (int i = 0; i < n && i < cap; i++) {
        memcpy(keys + 6 * i, t[i].key, 6);
        vals[2 * i] = t[i].dh;
        vals[2 * i + 1] = t[i].ds;
    }
    return n;
}

/* Initiation terms of a Watson-Crick set: [init, at, gc, one_gc, all_at] x (dH, dS). */
int or_nn_init(int table, double *vals)
{
    if (table == 0) table = 3;
    if (table < 1 || table > 4) return -1;
    const nn_set *s = &NN_SETS[table];
    double v[10] = {s->init_dh, s->init_ds, s->at_dh, s->at_ds, s->gc_dh, s->gc_ds,
                    s->one_gc_dh, s->one_gc_ds, s->all_at_dh, s->all_at_ds};
    memcpy(vals, v, sizeof v);
    return 0;
}

/* The partner strand (3'->5') of a site, from the genome codes.
 * Plus site (the primer reads the plus strand): complement of s[start..end).
 * Minus site (rc(primer) reads the plus strand): reverse of s[start..end). */
static void site_partner(const uint8_t *codes, uint32_t start, int L, int minus, char *cseq)
{
    static const char comp[5] = {'T', 'G', 'C', 'A', 'N'};
    for (int j = 0; j < L; j++) {
        if (!minus) cseq[j] = comp[codes[start + j]];
        else cseq[j] = CODE_CHAR[codes[start + L - 1 - j]];
    }
    cseq[L] = 0;
}

/* Site Tm: the maximum of the duplex Tm over every concrete expansion of the
 * primer (R-variants: best-binding member of the degenerate mixture).
 * Untabulated variants are skipped and counted; with none left the site Tm
 * is -infinity. */
static double site_tm(const char *primer, const char *cseq, const or_tm_cond *cond, uint32_t *skipped)
{
    int L = (int)strlen(primer);
    char sets[OR_MAXL][5];
    int nset[OR_MAXL];
    uint64_t total = 1;
    for (int j = 0; j < L; j++) {
        int m = iupac_set(primer[j]);
        nset[j] = 0;
        for (int b = 0; b < 4; b++)
            if (m & (1 << b)) sets[j][nset[j]++] = CODE_CHAR[b];
        total *= (uint64_t)nset[j];
    }
    double best = -INFINITY;
    char v[OR_MAXL + 1];
    v[L] = 0;
    *skipped = 0;
    for (uint64_t idx = 0; idx < total; idx++) {
        /* mixed-radix digits, last position fastest: lexicographic in ACGT */
        uint64_t r = idx;
        for (int j = L - 1; j >= 0; j--) {
            v[j] = sets[j][r % (uint64_t)nset[j]];
            r /= (uint64_t)nset[j];
        }
        int st;
        double t = or_tm_duplex(v, cseq, 0, cond, &st);
        if (st != 0) { (*skipped)++; continue; }
        if (t > best) best = t;
    }
    return best;
}

typedef struct {
    const uint8_t *ascii;
    const uint64_t *off;
    const char *const *primers;
    const uint32_t *amps;
    uint64_t a0, a1;
    const or_tm_cond *cond;
    double threshold;
    int filter;
    double *tm, *tm_site;
    uint8_t *pass;
    uint32_t *skipped;
} tm_job;

static void *tm_worker(void *arg)
{
    tm_job *jb = (tm_job *)arg;
    uint8_t *codes = NULL;
    uint64_t cap = 0;
    uint32_t cur_seq = 0xFFFFFFFFu;
    char cseq[OR_MAXL + 1];
    for (uint64_t i = jb->a0; i < jb->a1; i++) {
        const uint32_t *a = jb->amps + 5 * i;
        uint32_t s = a[0], start = a[1], end = a[2], q = a[3], o = a[4];
        if (s != cur_seq) {
            uint64_t n = jb->off[s + 1] - jb->off[s];
            if (n > cap) { cap = n; codes = (uint8_t *)realloc(codes, n ? n : 1); }
            for (uint64_t t = 0; t < n; t++) codes[t] = (uint8_t)genome_code(jb->ascii[jb->off[s] + t]);
            cur_seq = s;
        }
        int lp = (o == 0 || o == 2) ? 0 : 1; /* left (plus) site primer */
        int rp = (o == 0 || o == 3) ? 1 : 0; /* right (minus) site primer */
        const char *P1 = jb->primers[2 * q + lp], *P2 = jb->primers[2 * q + rp];
        int L1 = (int)strlen(P1), L2 = (int)strlen(P2);
        site_partner(codes, start, L1, 0, cseq);
        double t1 = site_tm(P1, cseq, jb->cond, &jb->skipped[2 * i]);
        site_partner(codes, end - (uint32_t)L2, L2, 1, cseq);
        double t2 = site_tm(P2, cseq, jb->cond, &jb->skipped[2 * i + 1]);
        double t = t1 < t2 ? t1 : t2; /* R-amplicon: the weaker primer limits */
        jb->tm_site[2 * i] = t1;
        jb->tm_site[2 * i + 1] = t2;
        jb->tm[i] = t;
        jb->pass[i] = jb->filter ? (uint8_t)(t >= jb->threshold) : (uint8_t)1;
    }
    free(codes);
    return NULL;
}

int or_tm_amps(const uint8_t *ascii, const uint64_t *off, const char *const *primers, const uint32_t *amps,
               uint64_t n_amps, const or_tm_cond *cond, double threshold, int filter, double *tm, double *tm_site,
               uint8_t *pass, uint32_t *skipped, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if ((uint64_t)n_threads > n_amps) n_threads = n_amps ? (int)n_amps : 1;
    tm_job *jobs = (tm_job *)calloc((size_t)n_threads, sizeof(tm_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; t++) {
        uint64_t a0 = n_amps * (uint64_t)t / (uint64_t)n_threads, a1 = n_amps * (uint64_t)(t + 1) / (uint64_t)n_threads;
        jobs[t] = (tm_job){ascii, off, primers, amps, a0, a1, cond, threshold, filter, tm, tm_site, pass, skipped};
        pthread_create(&th[t], NULL, tm_worker, &jobs[t]);
    }
    for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------------------------------ */
/* O6/O7: amplicon sequence, trimming, barcodes, primer snippets        */
/* ------------------------------------------------------------------ */

static char comp_char(char c)
{
    switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return 'N';
    }
}

/* s[a..b) of the normalised sequence, reverse-complemented if rc, into out */
static uint64_t put_span(const uint8_t *ascii, uint64_t base, uint64_t a, uint64_t b, int rc, char *out)
{
    uint64_t n = b > a ? b - a : 0;
    for (uint64_t i = 0; i < n; i++) {
        char c = rc ? comp_char(CODE_CHAR[genome_code(ascii[base + b - 1 - i])])
                    : CODE_CHAR[genome_code(ascii[base + a + i])];
        out[i] = c;
    }
    return n;
}

/*
 * Extract per amplicon (skipped -- empty, zero barcode lengths -- when pass
 * is given and pass[i] == 0):
 *   FR/FF/RR: sequence s[start:end]; trimmed s[start+Lleft : end-Lright];
 *             fb = s[start-fb : start], rb = s[end : end+rb];
 *   RF:       the reverse complement of the same spans; fb = rc(s[end : end+fb]),
 *             rb = rc(s[start-rb : start]).
 * Barcodes are clipped at the sequence ends (R-clip), real lengths in bc_len;
 * flags[i] = 1 when a clipped barcode is shorter than asked for, else 0.
 * fprimer / rprimer: the genome bases under the forward / reverse primer's
 * site, read 5'->3' in that primer's orientation (FF/RR: upstream site ->
 * fprimer, downstream site -> rprimer), NUL-padded to 32 bytes.
 * Sequences are concatenated; seq_off has n+1 entries.  Returns total bytes
 * (writes only while within seq_cap).
 */
int64_t or_extract(const uint8_t *ascii, const uint64_t *off, const char *const *primers, const uint32_t *amps,
                   uint64_t n_amps, const uint8_t *pass, int trim, int fb_len, int rb_len, char *seq_out,
                   uint64_t seq_cap, uint64_t *seq_off, char *fb, char *rb, uint8_t *bc_len, char *fpr, char *rpr,
                   uint8_t *flags)
{
    uint64_t pos = 0;
    char tmp_buf[OR_MAXL];
    for (uint64_t i = 0; i < n_amps; i++) {
        const uint32_t *a = amps + 5 * i;
        uint32_t s = a[0], start = a[1], end = a[2], q = a[3], o = a[4];
        uint64_t base = off[s], n = off[s + 1] - off[s];
        seq_off[i] = pos;
        memset(fpr + 32 * i, 0, 32);
        memset(rpr + 32 * i, 0, 32);
        if (fb_len) memset(fb + (uint64_t)fb_len * i, 0, (size_t)fb_len);
        if (rb_len) memset(rb + (uint64_t)rb_len * i, 0, (size_t)rb_len);
        bc_len[2 * i] = bc_len[2 * i + 1] = 0;
        flags[i] = 0;
        if (pass && !pass[i]) continue;
        int lp = (o == 0 || o == 2) ? 0 : 1;
        int rp = (o == 0 || o == 3) ? 1 : 0;
        uint32_t Ll = (uint32_t)strlen(primers[2 * q + lp]), Lr = (uint32_t)strlen(primers[2 * q + rp]);
        int rc = (o == 1);
        uint64_t a0 = start, a1 = end;
        if (trim) { a0 = start + Ll; a1 = end - Lr; if (a1 < a0) a1 = a0; }
        uint64_t len = a1 - a0;
        if (pos + len <= seq_cap) put_span(ascii, base, a0, a1, rc, seq_out + pos);
        pos += len;
        /* barcodes */
        uint64_t f0, f1, r0, r1;
        if (!rc) {
            f0 = start >= (uint32_t)fb_len ? start - (uint32_t)fb_len : 0; f1 = start;
            r0 = end; r1 = end + (uint64_t)rb_len <= n ? end + (uint64_t)rb_len : n;
        } else {
            f0 = end; f1 = end + (uint64_t)fb_len <= n ? end + (uint64_t)fb_len : n;
            r0 = start >= (uint32_t)rb_len ? start - (uint32_t)rb_len : 0; r1 = start;
        }
        bc_len[2 * i] = (uint8_t)put_span(ascii, base, f0, f1, rc, fb + (uint64_t)fb_len * i);
        bc_len[2 * i + 1] = (uint8_t)put_span(ascii, base, r0, r1, rc, rb + (uint64_t)rb_len * i);
        flags[i] = (bc_len[2 * i] < fb_len || bc_len[2 * i + 1] < rb_len) ? 1 : 0;
        /* primer snippets: left site is plus (read as is), right site is minus (rc) */
        char *left_dst = (lp == 0) ? fpr + 32 * i : rpr + 32 * i;
        char *right_dst = (rp == 1) ? rpr + 32 * i : fpr + 32 * i;
        if (lp == rp) { left_dst = fpr + 32 * i; right_dst = rpr + 32 * i; }
        put_span(ascii, base, start, start + Ll, 0, tmp_buf);
        memcpy(left_dst, tmp_buf, Ll);
        put_span(ascii, base, end - Lr, end, 1, tmp_buf);
        memcpy(right_dst, tmp_buf, Lr);
    }
    seq_off[n_amps] = pos;
    return (int64_t)pos;
}

int or_version(void) { return 1; }
