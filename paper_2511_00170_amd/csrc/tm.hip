// Nearest-neighbour melting temperature in FP64 (Implementations, "AHv2": a
// C re-implementation of Biopython's Tm_NN; Results, "Primer degeneracy and
// mismatch tolerance": Tm is computed for every primer variant).
//
// A wavefront owns one primer site; its lanes stride over the concrete
// variants of the degenerate primer, each lane evaluating the duplex of one
// variant with the genome strand the primer anneals to, and the wave reduces
// the maximum.  Stack parameters live in LDS as 256-entry tables indexed by
// (top dinucleotide, bottom dinucleotide).
#include <math.h>

#include "ah_internal.h"

// ---------------------------------------------------------------- tables
// Stack "XY/WZ": top strand 5'-XY-3' over bottom strand 3'-WZ-5'.
// dH kcal/mol, dS cal/(K mol).
struct NNRow {
    char x, y, w, z;
    double dh, ds;
};

// Watson-Crick nearest neighbours of the Tm_NN model's DNA parameter sets,
// numbered as it numbers them (3 is the default):
// 1 Breslauer, Frank, Bloecker & Marky (1986) PNAS 83:3746, Table 2.
static constexpr NNRow kWatsonCrick1[] = {
    {'A', 'A', 'T', 'T', -9.1, -24.0}, {'A', 'T', 'T', 'A', -8.6, -23.9}, {'T', 'A', 'A', 'T', -6.0, -16.9},
    {'C', 'A', 'G', 'T', -5.8, -12.9}, {'G', 'T', 'C', 'A', -6.5, -17.3}, {'C', 'T', 'G', 'A', -7.8, -20.8},
    {'G', 'A', 'C', 'T', -5.6, -13.5}, {'C', 'G', 'G', 'C', -11.9, -27.8}, {'G', 'C', 'C', 'G', -11.1, -26.7},
    {'G', 'G', 'C', 'C', -11.0, -26.6},
};
// 2 Sugimoto, Nakano, Yoneyama & Honda (1996) Nucleic Acids Res 24:4501, Table 1.
static constexpr NNRow kWatsonCrick2[] = {
    {'A', 'A', 'T', 'T', -8.0, -21.9}, {'A', 'T', 'T', 'A', -5.6, -15.2}, {'T', 'A', 'A', 'T', -6.6, -18.4},
    {'C', 'A', 'G', 'T', -8.2, -21.0}, {'G', 'T', 'C', 'A', -9.4, -25.5}, {'C', 'T', 'G', 'A', -6.6, -16.4},
    {'G', 'A', 'C', 'T', -8.8, -23.5}, {'C', 'G', 'G', 'C', -11.8, -29.0}, {'G', 'C', 'C', 'G', -10.5, -26.4},
    {'G', 'G', 'C', 'C', -10.9, -28.4},
};
// 3 SantaLucia (1998) PNAS 95:1460, Table 2 (unified parameters).
static constexpr NNRow kWatsonCrick3[] = {
    {'A', 'A', 'T', 'T', -7.9, -22.2}, {'A', 'T', 'T', 'A', -7.2, -20.4}, {'T', 'A', 'A', 'T', -7.2, -21.3},
    {'C', 'A', 'G', 'T', -8.5, -22.7}, {'G', 'T', 'C', 'A', -8.4, -22.4}, {'C', 'T', 'G', 'A', -7.8, -21.0},
    {'G', 'A', 'C', 'T', -8.2, -22.2}, {'C', 'G', 'G', 'C', -10.6, -27.2}, {'G', 'C', 'C', 'G', -9.8, -24.4},
    {'G', 'G', 'C', 'C', -8.0, -19.9},
};
// 4 SantaLucia & Hicks (2004) Annu Rev Biophys Biomol Struct 33:415, Table 1.
static constexpr NNRow kWatsonCrick4[] = {
    {'A', 'A', 'T', 'T', -7.6, -21.3}, {'A', 'T', 'T', 'A', -7.2, -20.4}, {'T', 'A', 'A', 'T', -7.2, -21.3},
    {'C', 'A', 'G', 'T', -8.5, -22.7}, {'G', 'T', 'C', 'A', -8.4, -22.4}, {'C', 'T', 'G', 'A', -7.8, -21.0},
    {'G', 'A', 'C', 'T', -8.2, -22.2}, {'C', 'G', 'G', 'C', -10.6, -27.2}, {'G', 'C', 'C', 'G', -9.8, -24.4},
    {'G', 'G', 'C', 'C', -8.0, -19.9},
};

// Initiation terms of each set (dH, dS): every duplex; per duplex end with a
// terminal A.T / G.C pair; a duplex holding at least one G.C pair / none.
// (The model's 5'-terminal T.A penalty is zero in all four sets.)
struct NNInit {
    double init_dh, init_ds, at_dh, at_ds, gc_dh, gc_ds, one_gc_dh, one_gc_ds, all_at_dh, all_at_ds;
};
static constexpr NNInit kInit[5] = {
    {0, 0, 2.3, 4.1, 0.1, -2.8, 0, 0, 0, 0},     // 0 = 3
    {0, 0, 0, 0, 0, 0, 0, -16.8, 0, -20.1},      // Breslauer 1986: 5.0 / 6.0 kcal/mol at 25 C, entropic
    {0.6, -9.0, 0, 0, 0, 0, 0, 0, 0, 0},         // Sugimoto 1996
    {0, 0, 2.3, 4.1, 0.1, -2.8, 0, 0, 0, 0},     // SantaLucia 1998
    {0.2, -5.7, 2.2, 6.9, 0, 0, 0, 0, 0, 0},     // SantaLucia & Hicks 2004
};

// Single internal mismatches (and tandem G.T), one mismatch type per row:
// G.T Allawi & SantaLucia 1997; G.A Allawi & SantaLucia 1998 (Biochemistry
// 37:2170); C.T Allawi & SantaLucia 1998 (NAR 26:2694); A.C Allawi &
// SantaLucia 1998 (Biochemistry 37:9435); A.A C.C G.G T.T Peyret et al. 1999.
static constexpr NNRow kInternalMismatch[] = {
    // G.T
    {'A', 'G', 'T', 'T', 1.0, 0.9}, {'A', 'T', 'T', 'G', -2.5, -8.3}, {'C', 'G', 'G', 'T', -4.1, -11.7},
    {'C', 'T', 'G', 'G', -2.8, -8.0}, {'G', 'G', 'C', 'T', 3.3, 10.4}, {'G', 'G', 'T', 'T', 5.8, 16.3},
    {'G', 'T', 'C', 'G', -4.4, -12.3}, {'G', 'T', 'T', 'G', 4.1, 9.5}, {'T', 'G', 'A', 'T', -0.1, -1.7},
    {'T', 'G', 'G', 'T', -1.4, -6.2}, {'T', 'T', 'A', 'G', -1.3, -5.3},
    // G.A
    {'A', 'A', 'T', 'G', -0.6, -2.3}, {'A', 'G', 'T', 'A', -0.7, -2.3}, {'C', 'A', 'G', 'G', -0.7, -2.3},
    {'C', 'G', 'G', 'A', -4.0, -13.2}, {'G', 'A', 'C', 'G', -0.6, -1.0}, {'G', 'G', 'C', 'A', 0.5, 3.2},
    {'T', 'A', 'A', 'G', 0.7, 0.7}, {'T', 'G', 'A', 'A', 3.0, 7.4},
    // C.T
    {'A', 'C', 'T', 'T', 0.7, 0.2}, {'A', 'T', 'T', 'C', -1.2, -6.2}, {'C', 'C', 'G', 'T', -0.8, -4.5},
    {'C', 'T', 'G', 'C', -1.5, -6.1}, {'G', 'C', 'C', 'T', 2.3, 5.4}, {'G', 'T', 'C', 'C', 5.2, 13.5},
    {'T', 'C', 'A', 'T', 1.2, 0.7}, {'T', 'T', 'A', 'C', 1.0, 0.7},
    // A.C
    {'A', 'A', 'T', 'C', 2.3, 4.6}, {'A', 'C', 'T', 'A', 5.3, 14.6}, {'C', 'A', 'G', 'C', 1.9, 3.7},
    {'C', 'C', 'G', 'A', 0.6, -0.6}, {'G', 'A', 'C', 'C', 5.2, 14.2}, {'G', 'C', 'C', 'A', -0.7, -3.8},
    {'T', 'A', 'A', 'C', 3.4, 8.0}, {'T', 'C', 'A', 'A', 7.6, 20.2},
    // A.A, C.C, G.G, T.T
    {'A', 'A', 'T', 'A', 1.2, 1.7}, {'C', 'A', 'G', 'A', -0.9, -4.2}, {'G', 'A', 'C', 'A', -2.9, -9.8},
    {'T', 'A', 'A', 'A', 4.7, 12.9}, {'A', 'C', 'T', 'C', 0.0, -4.4}, {'C', 'C', 'G', 'C', -1.5, -7.2},
    {'G', 'C', 'C', 'C', 3.6, 8.9}, {'T', 'C', 'A', 'C', 6.1, 16.4}, {'A', 'G', 'T', 'G', -3.1, -9.5},
    {'C', 'G', 'G', 'G', -4.9, -15.3}, {'G', 'G', 'C', 'G', -6.0, -15.8}, {'T', 'G', 'A', 'G', 1.6, 3.6},
    {'A', 'T', 'T', 'T', -2.7, -10.8}, {'C', 'T', 'G', 'T', -5.0, -15.8}, {'G', 'T', 'C', 'T', -2.2, -8.4},
    {'T', 'T', 'A', 'T', 0.2, -1.5},
};

// Terminal mismatches: a Watson-Crick pair, then the mismatched duplex end.
// The Tm_NN model's DNA table, from SantaLucia & Peyret (2001), patent
// application WO 01/94611.
static constexpr NNRow kTerminalMismatch[] = {
    {'A', 'A', 'T', 'A', -3.1, -7.8}, {'T', 'A', 'A', 'A', -2.5, -6.3}, {'C', 'A', 'G', 'A', -4.3, -10.7},
    {'G', 'A', 'C', 'A', -8.0, -22.5}, {'A', 'C', 'T', 'C', -0.1, 0.5}, {'T', 'C', 'A', 'C', -0.7, -1.3},
    {'C', 'C', 'G', 'C', -2.1, -5.1}, {'G', 'C', 'C', 'C', -3.9, -10.6}, {'A', 'G', 'T', 'G', -1.1, -2.1},
    {'T', 'G', 'A', 'G', -1.1, -2.7}, {'C', 'G', 'G', 'G', -3.8, -9.5}, {'G', 'G', 'C', 'G', -0.7, -19.2},
    {'A', 'T', 'T', 'T', -2.4, -6.5}, {'T', 'T', 'A', 'T', -3.2, -8.9}, {'C', 'T', 'G', 'T', -6.1, -16.9},
    {'G', 'T', 'C', 'T', -7.4, -21.2}, {'A', 'A', 'T', 'C', -1.6, -4.0}, {'A', 'C', 'T', 'A', -1.8, -3.8},
    {'C', 'A', 'G', 'C', -2.6, -5.9}, {'C', 'C', 'G', 'A', -2.7, -6.0}, {'G', 'A', 'C', 'C', -5.0, -13.8},
    {'G', 'C', 'C', 'A', -3.2, -7.1}, {'T', 'A', 'A', 'C', -2.3, -5.9}, {'T', 'C', 'A', 'A', -2.7, -7.0},
    {'A', 'C', 'T', 'T', -0.9, -1.7}, {'A', 'T', 'T', 'C', -2.3, -6.3}, {'C', 'C', 'G', 'T', -3.2, -8.0},
    {'C', 'T', 'G', 'C', -3.9, -10.6}, {'G', 'C', 'C', 'T', -4.9, -13.5}, {'G', 'T', 'C', 'C', -3.0, -7.8},
    {'T', 'C', 'A', 'T', -2.5, -6.3}, {'T', 'T', 'A', 'C', -0.7, -1.2}, {'A', 'A', 'T', 'G', -1.9, -4.4},
    {'A', 'G', 'T', 'A', -2.5, -5.9}, {'C', 'A', 'G', 'G', -3.9, -9.6}, {'C', 'G', 'G', 'A', -6.0, -15.5},
    {'G', 'A', 'C', 'G', -4.3, -11.1}, {'G', 'G', 'C', 'A', -4.6, -11.4}, {'T', 'A', 'A', 'G', -2.0, -4.7},
    {'T', 'G', 'A', 'A', -2.4, -5.8}, {'A', 'G', 'T', 'T', -3.2, -8.7}, {'A', 'T', 'T', 'G', -3.5, -9.4},
    {'C', 'G', 'G', 'T', -3.8, -9.0}, {'C', 'T', 'G', 'G', -6.6, -18.7}, {'G', 'G', 'C', 'T', -5.7, -15.9},
    {'G', 'T', 'C', 'G', -5.9, -16.1}, {'T', 'G', 'A', 'T', -3.9, -10.5}, {'T', 'T', 'A', 'G', -3.6, -9.8},
};

// Dangling ends, Bommarito, Peyret & SantaLucia (2000) NAR 28:1929: one
// unpaired base beside a terminal Watson-Crick pair x.w.  Row {d, x, w}: the
// dangling base d and the pair.  kDangleTop5: a 5'-dangling base of the
// strand written on top (5'-dx-3' over 3'-.w-5'); kDangleBottom3: a
// 3'-dangling base of the bottom strand (5'-.x-3' over 3'-dw-5').
struct DERow {
    char d, x, w;
    double dh, ds;
};
static constexpr DERow kDangleTop5[] = {
    {'A', 'A', 'T', 0.2, 2.3}, {'A', 'C', 'G', -6.3, -17.1}, {'A', 'G', 'C', -3.7, -10.0}, {'A', 'T', 'A', -2.9, -7.6},
    {'C', 'A', 'T', 0.6, 3.3}, {'C', 'C', 'G', -4.4, -12.6}, {'C', 'G', 'C', -4.0, -11.9}, {'C', 'T', 'A', -4.1, -13.0},
    {'G', 'A', 'T', -1.1, -1.6}, {'G', 'C', 'G', -5.1, -14.0}, {'G', 'G', 'C', -3.9, -10.9}, {'G', 'T', 'A', -4.2, -15.0},
    {'T', 'A', 'T', -6.9, -20.0}, {'T', 'C', 'G', -4.0, -10.9}, {'T', 'G', 'C', -4.9, -13.8}, {'T', 'T', 'A', -0.2, -0.5},
};
static constexpr DERow kDangleBottom3[] = {
    {'A', 'A', 'T', -0.7, -0.8}, {'A', 'C', 'G', -2.1, -3.9}, {'A', 'G', 'C', -5.9, -16.5}, {'A', 'T', 'A', -0.5, -1.1},
    {'C', 'A', 'T', 4.4, 14.9}, {'C', 'C', 'G', -0.2, -0.1}, {'C', 'G', 'C', -2.6, -7.4}, {'C', 'T', 'A', 4.7, 14.2},
    {'G', 'A', 'T', -1.6, -3.6}, {'G', 'C', 'G', -3.9, -11.2}, {'G', 'G', 'C', -3.2, -10.4}, {'G', 'T', 'A', -4.1, -13.1},
    {'T', 'A', 'T', 2.9, 10.4}, {'T', 'C', 'G', -4.4, -13.1}, {'T', 'G', 'C', -5.2, -15.0}, {'T', 'T', 'A', -3.8, -12.6},
};

struct NNTable {
    double dh[256];
    double ds[256];
    uint32_t ok[8];  // bit i: entry i tabulated
};

constexpr int base_of(char c) { return c == 'A' ? 0 : c == 'C' ? 1 : c == 'G' ? 2 : 3; }
// index: top pair of bases (x, y) in the low nibble, bottom (w, z) in the high nibble
constexpr int nn_index(int x, int y, int w, int z) { return (x | (y << 2)) | ((w | (z << 2)) << 4); }

template <size_t N>
constexpr void put_rows(NNTable &t, const NNRow (&rows)[N], bool reversed) {
    for (size_t r = 0; r < N; r++) {
        const NNRow &e = rows[r];
        int i = reversed ? nn_index(base_of(e.z), base_of(e.w), base_of(e.y), base_of(e.x))
                         : nn_index(base_of(e.x), base_of(e.y), base_of(e.w), base_of(e.z));
        if (t.ok[i >> 5] & (1u << (i & 31))) continue;  // a stack as written wins over a reversed reading
        t.dh[i] = e.dh;
        t.ds[i] = e.ds;
        t.ok[i >> 5] |= 1u << (i & 31);
    }
}

template <size_t N>
constexpr NNTable make_stack_table(const NNRow (&wc)[N]) {
    NNTable t{};
    put_rows(t, wc, false);
    put_rows(t, kInternalMismatch, false);
    put_rows(t, wc, true);
    put_rows(t, kInternalMismatch, true);
    return t;
}

constexpr NNTable make_terminal_table() {
    NNTable t{};
    put_rows(t, kTerminalMismatch, false);
    return t;
}

// Dangling-end index: kind (0 = 5'-dangling base of the top strand, 1 =
// 3'-dangling base of the bottom strand), dangling base, pair top base, pair
// bottom base.
constexpr int de_index(int kind, int d, int x, int w) { return (kind << 6) | (d << 4) | (x << 2) | w; }

template <size_t N>
constexpr void put_dangles(NNTable &t, const DERow (&rows)[N], int kind) {
    for (size_t r = 0; r < N; r++) {
        const int i = de_index(kind, base_of(rows[r].d), base_of(rows[r].x), base_of(rows[r].w));
        t.dh[i] = rows[r].dh;
        t.ds[i] = rows[r].ds;
        t.ok[i >> 5] |= 1u << (i & 31);
    }
}

constexpr NNTable make_dangle_table() {
    NNTable t{};
    put_dangles(t, kDangleTop5, 0);
    put_dangles(t, kDangleBottom3, 1);
    return t;
}

// Stack tables (Watson-Crick set + internal mismatches) by set number (0 = 3).
__constant__ NNTable g_stack[5] = {make_stack_table(kWatsonCrick3), make_stack_table(kWatsonCrick1),
                                   make_stack_table(kWatsonCrick2), make_stack_table(kWatsonCrick3),
                                   make_stack_table(kWatsonCrick4)};
__constant__ NNTable g_term = make_terminal_table();
__constant__ NNTable g_dangle = make_dangle_table();
__constant__ NNInit g_init[5] = {kInit[0], kInit[1], kInit[2], kInit[3], kInit[4]};

// Salt terms (the seven corrections of the Tm_NN model, each from its
// paper): 1-4 add a constant to Tm; 5 adds 0.368 (N-1) ln(mon) to dS;
// 6 (Owczarzy 2004) and 7 (Owczarzy 2008, Mg2+) add a term depending on the
// G+C fraction and length of the primer strand to 1/Tm.
struct TmConst {
    int saltcorr;
    int mg_model;     // method 7: 1 = Mg2+ formula, 0 = monovalent formula of method 6
    int table;        // Watson-Crick set, 1..4
    int filter;
    double ln_mon;    // ln of the monovalent-equivalent concentration (M; methods 5, 6, 7-monovalent)
    double dtm;       // methods 1-4: added to Tm
    // method 7 Mg2+ formula 1e-5 [m7a + fgc m7b + m7d / (2 (N - 1))] with
    // m7a = a + b ln Mg, m7b = c + d ln Mg, m7d = e + f ln Mg + g ln^2 Mg
    // (each folded on the host in the operation order of the full formula)
    double m7a, m7b, m7d;
    double rlnc;      // R ln C, C = C_high - C_low / 2 (M)
    double threshold;
};

// Watson-Crick set of the parameters: 0 selects the default 3; -1 if invalid.
__host__ __device__ inline int tm_table(const ah_tm_params &p) {
    return p.nn_table == 0 ? 3 : (p.nn_table >= 1 && p.nn_table <= 4 ? p.nn_table : -1);
}

// Everything here also runs on the host (ah_tm_nn checks the conditions).
__host__ __device__ inline int tm_salt_setup(const ah_tm_params &p, TmConst *k) {
    double mon = p.na_mM + p.k_mM + p.tris_mM / 2.0;
    if (p.dntps_mM < p.mg_mM) mon += 120.0 * sqrt(p.mg_mM - p.dntps_mM);  // von Ahsen et al. 2001
    mon = mon * 1e-3;
    k->saltcorr = p.saltcorr;
    k->ln_mon = 0.0;
    k->dtm = 0.0;
    k->mg_model = 0;
    k->m7a = k->m7b = k->m7d = 0.0;
    if (p.saltcorr == 0) return 0;
    if (p.saltcorr >= 1 && p.saltcorr <= 6) {
        if (!(mon > 0.0)) return 1;
        k->ln_mon = log(mon);
        if (p.saltcorr == 1) k->dtm = 16.6 * log10(mon);                       // Schildkraut & Lifson 1965
        if (p.saltcorr == 2) k->dtm = 16.6 * log10(mon / (1.0 + 0.7 * mon));   // Wetmur 1991
        if (p.saltcorr == 3) k->dtm = 12.5 * log10(mon);                       // SantaLucia et al. 1996
        if (p.saltcorr == 4) k->dtm = 11.7 * log10(mon);                       // SantaLucia 1998
        return 0;
    }
    if (p.saltcorr != 7) return 1;
    // Owczarzy et al. 2008: monovalent ions without the Mg2+ equivalent, free
    // Mg2+ after dNTP binding (association constant 3e4 /M)
    const double mon7 = (p.na_mM + p.k_mM + p.tris_mM / 2.0) * 1e-3;
    double mg = p.mg_mM * 1e-3;
    if (p.dntps_mM > 0.0) {
        const double ka = 3e4, dn = p.dntps_mM * 1e-3;
        const double bq = ka * dn - ka * mg + 1.0;
        mg = (-bq + sqrt(bq * bq + 4.0 * ka * mg)) / (2.0 * ka);
    }
    double a = 3.92, d = 1.42, g = 8.31;
    if (mon7 > 0.0) {
        const double R = sqrt(mg) / mon7, lm = log(mon7);
        if (R < 0.22) {  // monovalent ions dominate: the 2004 formula
            k->ln_mon = lm;
            return 0;
        }
        if (R < 6.0) {
            a = 3.92 * (0.843 - 0.352 * sqrt(mon7) * lm);
            d = 1.42 * (1.279 - 4.03e-3 * lm - 8.03e-3 * lm * lm);
            g = 8.31 * (0.486 - 0.258 * lm + 5.25e-3 * lm * lm * lm);
        }
    }
    if (!(mg > 0.0)) return 1;
    k->mg_model = 1;
    const double b = -0.911, c = 6.26, e = -48.2, f = 52.5, lg = log(mg);
    k->m7a = a + b * lg;
    k->m7b = c + d * lg;
    k->m7d = e + f * lg + g * lg * lg;
    return 0;
}

// Computed once on the host and passed to the kernels by value: the
// constants then sit in scalar registers instead of a dozen FP64 values per
// lane, and no lane evaluates the logarithms.
__host__ __device__ inline TmConst tm_const(const ah_tm_params &p) {
    TmConst k;
    (void)tm_salt_setup(p, &k);
    const double hiC = p.dnac1_nM > p.dnac2_nM ? p.dnac1_nM : p.dnac2_nM;
    const double loC = p.dnac1_nM > p.dnac2_nM ? p.dnac2_nM : p.dnac1_nM;
    const double C = (hiC - loC / 2.0) * 1e-9;
    k.rlnc = 1.987 * log(C);
    k.threshold = p.threshold_C;
    k.filter = p.filter;
    k.table = tm_table(p) < 0 ? 3 : tm_table(p);
    return k;
}

// The parameter checks of both Tm entry points (host, before any launch).
static bool tm_params_ok(const ah_tm_params &p) {
    TmConst k;
    return tm_table(p) > 0 && tm_salt_setup(p, &k) == 0;  // a zero concentration under a logarithm fails
}

__device__ __forceinline__ bool tab_ok(const uint32_t *ok, int i) { return (ok[i >> 5] >> (i & 31)) & 1u; }

// The tables as the constant-memory records (values and validity bits).
struct ConstTables {
    int set;  // Watson-Crick set
    __device__ bool stack(int i, double &dh, double &ds) const {
        dh = g_stack[set].dh[i];
        ds = g_stack[set].ds[i];
        return tab_ok(g_stack[set].ok, i);
    }
    __device__ bool term(int i, double &dh, double &ds) const {
        dh = g_term.dh[i];
        ds = g_term.ds[i];
        return tab_ok(g_term.ok, i);
    }
};

// The stack and terminal-mismatch tables staged in LDS as (dH, dS) pairs,
// NaN where not tabulated: one 16-byte read per step instead of two values
// and a validity word.
struct LdsTables {
    const double2 *st, *tt;
    __device__ bool stack(int i, double &dh, double &ds) const {
        const double2 e = st[i];
        dh = e.x;
        ds = e.y;
        return e.x == e.x;
    }
    __device__ bool term(int i, double &dh, double &ds) const {
        const double2 e = tt[i];
        dh = e.x;
        ds = e.y;
        return e.x == e.x;
    }
};

// Entries 256..271 of the staged stack table: (0, 0), read by a step outside
// the helix (entry 256 + the variant's dinucleotide: the address needs no
// select per variant).
#define AH_ZERO_ENTRY 256
#define AH_STACK_ENTRIES (256 + 16)

__device__ void stage_tables(double2 *st, double2 *tt, int set) {
    const NNTable &S = g_stack[set];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) {
        st[i] = tab_ok(S.ok, i) ? make_double2(S.dh[i], S.ds[i]) : make_double2(NAN, NAN);
        tt[i] = tab_ok(g_term.ok, i) ? make_double2(g_term.dh[i], g_term.ds[i]) : make_double2(NAN, NAN);
    }
    if (threadIdx.x < AH_STACK_ENTRIES - 256) st[AH_ZERO_ENTRY + threadIdx.x] = make_double2(0.0, 0.0);
    __syncthreads();
}

// What the initiation and salt terms read of the primer strand as given
// (reading R-init: its end bases and G+C content, also when an end pair left
// the helix): 2-bit codes of its first and last base, its length and G+C count.
struct PrimerEnds {
    int e0, e1, L, gc;
};

__device__ __forceinline__ int gc_count(uint64_t V, int L) {
    // codes 1 (C) and 2 (G) have differing bits
    const uint64_t lmask = L >= 32 ? ~0ull : ((1ull << (2 * L)) - 1);
    return __popcll((V ^ (V >> 1)) & 0x5555555555555555ull & lmask);
}

// The salt term and Tm = 1000 dH / (dS + R ln C) - 273.15 from the summed
// dH and dS (salt method 5 adds to dS first; 1-4 add to Tm; 6 and 7 add to
// 1/Tm).
__device__ __forceinline__ double tm_of_sums(double dh, double ds, const PrimerEnds &P, const TmConst &k) {
    const int L = P.L;
    if (k.saltcorr == 5) ds += 0.368 * (double)(L - 1) * k.ln_mon;
    double tm = (1000.0 * dh) / (ds + k.rlnc) - 273.15;
    if (k.saltcorr >= 1 && k.saltcorr <= 4) tm += k.dtm;
    if (k.saltcorr >= 6) {
        const double fgc = (double)P.gc / (double)L;
        double corr;
        if (k.mg_model)
            corr = (k.m7a + fgc * k.m7b + k.m7d / (2.0 * (L - 1))) * 1e-5;
        else
            corr = (4.29 * fgc - 3.95) * 1e-5 * k.ln_mon + 9.40e-6 * k.ln_mon * k.ln_mon;
        tm = 1.0 / (1.0 / (tm + 273.15) + corr) - 273.15;
    }
    return tm;
}

// Steps after the dangling ends, on the helix of n facing pairs V / C (2-bit
// codes, pair j at bits 2j; C is the partner strand read 3'->5' against V),
// accumulating into dh / ds: a mismatched end pair is charged with the
// terminal-mismatch stack and leaves the helix (left end, then right);
// initiation from the primer strand P; the remaining stacks from 5' to 3';
// the salt term; Tm = 1000 dH / (dS + R ln C) - 273.15.  The order of the
// floating-point additions is fixed.  Returns false if a stack is not
// tabulated.
template <class Tab>
__device__ bool helix_tm(uint64_t V, uint64_t C, int n, double dh, double ds, const PrimerEnds &P, const Tab &tab,
                         const TmConst &k, double *out) {
    auto bb = [](uint64_t X, int j) { return (int)((X >> (2 * j)) & 3u); };
    int lo = 0, hi = n - 1;
    {
        // left end read from the partner strand, so the end pair comes second
        const int i = nn_index(bb(C, 1), bb(C, 0), bb(V, 1), bb(V, 0));
        double a, b;
        if (tab.term(i, a, b)) {
            dh += a;
            ds += b;
            lo = 1;
        }
    }
    if (hi - 1 >= lo) {
        const int i = nn_index(bb(V, hi - 1), bb(V, hi), bb(C, hi - 1), bb(C, hi));
        double a, b;
        if (tab.term(i, a, b)) {
            dh += a;
            ds += b;
            hi -= 1;
        }
    }
    {
        const NNInit &I = g_init[k.table];
        dh += I.init_dh;
        ds += I.init_ds;
        if (P.gc) { dh += I.one_gc_dh; ds += I.one_gc_ds; }
        else { dh += I.all_at_dh; ds += I.all_at_ds; }
        if (P.e0 == 0 || P.e0 == 3) { dh += I.at_dh; ds += I.at_ds; }
        else { dh += I.gc_dh; ds += I.gc_ds; }
        if (P.e1 == 0 || P.e1 == 3) { dh += I.at_dh; ds += I.at_ds; }
        else { dh += I.gc_dh; ds += I.gc_ds; }
    }
    for (int j = lo; j < hi; j++) {
        const int i = nn_index(bb(V, j), bb(V, j + 1), bb(C, j), bb(C, j + 1));
        double a, b;
        if (!tab.stack(i, a, b)) return false;
        dh += a;
        ds += b;
    }
    *out = tm_of_sums(dh, ds, P, k);
    return true;
}

// Duplex Tm of primer variant V (L bases) with its partner C of equal length
// and no dangling ends: the helix is the whole duplex.
template <class Tab>
__device__ __forceinline__ bool duplex_tm(uint64_t V, uint64_t C, int L, const Tab &tab, const TmConst &k,
                                          double *out) {
    if (L < 2) return false;
    const PrimerEnds P{(int)(V & 3u), (int)((V >> (2 * (L - 1))) & 3u), L, gc_count(V, L)};
    return helix_tm(V, C, L, 0.0, 0.0, P, tab, k, out);
}

// ---------------------------------------------------------------- sites
// The initiation terms of the selected set, read once per kernel (uniform,
// scalar registers).
struct InitTerms {
    double dh0, ds0, gc_dh, gc_ds, at0_dh, at0_ds, end_at_dh, end_at_ds, end_gc_dh, end_gc_ds;
    __device__ explicit InitTerms(int set) {
        const NNInit &I = g_init[set];
        dh0 = I.init_dh, ds0 = I.init_ds;
        gc_dh = I.one_gc_dh, gc_ds = I.one_gc_ds, at0_dh = I.all_at_dh, at0_ds = I.all_at_ds;
        end_at_dh = I.at_dh, end_at_ds = I.at_ds, end_gc_dh = I.gc_dh, end_gc_ds = I.gc_ds;
    }
};

// Byte offset in a staged table of the entry nn_index(V_j, V_j+1, C_j, C_j+1).
__device__ __forceinline__ uint32_t stack_off(uint64_t V, uint64_t C, int j) {
    return (((uint32_t)(V >> (2 * j)) & 15u) << 4) | (((uint32_t)(C >> (2 * j)) & 15u) << 8);
}

__device__ __forceinline__ double2 lds_at(const double2 *t, uint32_t off) {
    return *(const double2 *)((const char *)t + off);
}

// Tm of variant V (L >= 3 bases) on the site whose partner strand, read
// 3'->5' against it, is C: the additions of helix_tm over the whole duplex,
// in the same order -- terminal mismatch at the left end, then the right
// end; initiation; stacks j = lo .. hi - 1 from 5' to 3'; salt -- with the
// stack loop unrolled over fixed positions, in groups of four up to the
// wave's longest site (lw, wave-uniform).  A step outside the helix reads a
// zero entry: the first and the last step when an end pair left the helix,
// and steps j >= L - 2 of a shorter site in the wave (the partner part of
// the address then points into the zero block).  Adding +0.0 leaves a sum
// unchanged, since the sums start at +0.0 and a sum of two numbers is -0.0
// only when both are.  An untabulated stack reads NaN, which carries to the
// end, where the variant is dropped (helix_tm leaves its loop there instead).
__device__ __forceinline__ bool site_variant_tm(uint64_t V, uint64_t C, int L, int lw, const double2 *st,
                                                const double2 *tt, const InitTerms &I, const TmConst &k,
                                                double *out) {
    double dh = 0.0, ds = 0.0;
    // left end, read from the partner strand: nn_index(C_1, C_0, V_1, V_0)
    const uint32_t il = (uint32_t)(((C >> 2) & 3u) | ((C & 3u) << 2) | (((V >> 2) & 3u) << 4) | ((V & 3u) << 6));
    const double2 tl = tt[il];
    const bool left_out = tl.x == tl.x;
    if (left_out) {
        dh += tl.x;
        ds += tl.y;
    }
    // right end: nn_index(V_L-2, V_L-1, C_L-2, C_L-1)
    const uint32_t last = stack_off(V, C, L - 2);
    const double2 tr = lds_at(tt, last);
    const bool right_out = tr.x == tr.x;
    if (right_out) {
        dh += tr.x;
        ds += tr.y;
    }
    const int gc = gc_count(V, L);
    const int e0 = (int)(V & 3u), e1 = (int)((V >> (2 * (L - 1))) & 3u);
    dh += I.dh0;
    ds += I.ds0;
    dh += gc ? I.gc_dh : I.at0_dh;
    ds += gc ? I.gc_ds : I.at0_ds;
    const bool at0 = e0 == 0 || e0 == 3, at1 = e1 == 0 || e1 == 3;
    dh += at0 ? I.end_at_dh : I.end_gc_dh;
    ds += at0 ? I.end_at_ds : I.end_gc_ds;
    dh += at1 ? I.end_at_dh : I.end_gc_dh;
    ds += at1 ? I.end_at_ds : I.end_gc_ds;
    const uint32_t zero = 16u * AH_ZERO_ENTRY;
    double2 e = lds_at(st, left_out ? zero : stack_off(V, C, 0));
    dh += e.x;
    ds += e.y;
#pragma unroll
    for (int g = 0; g < (AH_MAXL - 3 + 3) / 4; g++) {
        if (1 + 4 * g >= lw - 2) break;  // uniform
        double2 E[4];  // the group's four reads first, then its additions in order
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int j = 1 + 4 * g + t;
            if (j < AH_MAXL - 2) {
                const uint32_t cp = j < L - 2 ? (((uint32_t)(C >> (2 * j)) & 15u) << 8) : zero;
                E[t] = lds_at(st, (((uint32_t)(V >> (2 * j)) & 15u) << 4) | cp);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (1 + 4 * g + t < AH_MAXL - 2) {
                dh += E[t].x;
                ds += E[t].y;
            }
        }
    }
    e = lds_at(st, right_out ? zero : last);
    dh += e.x;
    ds += e.y;
    if (!(dh == dh)) return false;
    *out = tm_of_sums(dh, ds, PrimerEnds{e0, e1, L, gc}, k);
    return true;
}

__device__ __forceinline__ uint64_t spread_bits(uint32_t v) {
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// 2-bit codes of bases [p, p + L) of the store (global base index p, L <= 32),
// base j at bits 2j; *has_n reports an N inside the window.
__device__ uint64_t load_site(const ah_store &st, uint64_t p, int L, bool *has_n) {
    const uint4 *blocks = (const uint4 *)st.d_blocks;
    const uint64_t gb = p >> 6;
    const uint32_t o = (uint32_t)(p & 63);
    const uint4 A = blocks[gb];
    uint32_t hW, lW;
    if (o < 32) {
        hW = __builtin_amdgcn_alignbit(A.z, A.x, o);
        lW = __builtin_amdgcn_alignbit(A.w, A.y, o);
    } else {
        uint32_t bh = 0, bl = 0;
        if (o - 32 + (uint32_t)L > 32 && gb + 1 < st.n_blocks) {
            const uint4 B = blocks[gb + 1];
            bh = B.x;
            bl = B.y;
        }
        hW = __builtin_amdgcn_alignbit(bh, A.z, o - 32);
        lW = __builtin_amdgcn_alignbit(bl, A.w, o - 32);
    }
    const uint64_t lmask = L == 32 ? ~0ull : ((1ull << (2 * L)) - 1);
    uint64_t nm = ah_block_nmask(st, gb) >> o;
    if (o + (uint32_t)L > 64 && o) nm |= ah_block_nmask(st, gb + 1) << (64 - o);
    *has_n = (nm & ((1ull << L) - 1)) != 0;
    return (spread_bits(lW) | (spread_bits(hW) << 1)) & lmask;
}

// reverse the order of the L 2-bit groups
__device__ __forceinline__ uint64_t reverse_codes(uint64_t G, int L) {
    uint64_t r = __builtin_bitreverse64(G);
    r = ((r >> 1) & 0x5555555555555555ull) | ((r & 0x5555555555555555ull) << 1);
    return r >> (64 - 2 * L);
}

__device__ __forceinline__ uint64_t primer_base_codes(const DPrimer &P) { return P.base; }

// Sites packed lps lanes apart (lps = the set's largest variant count rounded
// up to a power of two, at most 64): a wave evaluates 64 / lps sites at once,
// each lane a variant, and max-reduces within its site's lanes.  With
// lps <= 32 the two sites of an amplicon (2a, 2a + 1) sit in one wave, lps
// lanes apart, so the wave also takes their minimum and the pass flag
// (tm != nullptr); otherwise a finish kernel does.
// Bounded to six waves per SIMD (80 VGPRs, two spilled): latency-bound, it
// gains more from the sixth wave than the spills cost (seven: 72, eleven
// spilled, slower).
__global__ void __launch_bounds__(256, 4) ah_tm_site_kernel(ah_store st, const DPair *pairs, const uint32_t *amps,
                                                         const uint64_t *d_n, uint64_t cap, TmConst k,
                                                         uint32_t lps, double *tm_site, const double *pair_thr,
                                                         double *tm, uint8_t *pass) {
    __shared__ double2 sst[AH_STACK_ENTRIES], stt[256];
    stage_tables(sst, stt, k.table);
    const LdsTables nn{sst, stt};
    const InitTerms init(k.table);
    const uint64_t n = *d_n < cap ? *d_n : cap;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t per_wave = 64u / lps, sub = lane / lps, vl = lane % lps;
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t w0 = (blockIdx.x * (uint64_t)(blockDim.x >> 6) + (threadIdx.x >> 6)) * per_wave; w0 < 2 * n;
         w0 += nw * per_wave) {
        const uint64_t w = w0 + sub;  // this lane's site
        const bool live = w < 2 * n;
        const uint64_t a = live ? w >> 1 : 0;
        const int side = (int)(w & 1);
        const uint32_t seq = amps[4 * a], start = amps[4 * a + 1], end = amps[4 * a + 2], meta = amps[4 * a + 3];
        const uint32_t pair = meta & 0xFFFFu, orient = (meta >> 16) & 0xFFu;
        // upstream site: forward primer for FR/FF; downstream: reverse primer for FR/RR
        const int pr = side == 0 ? ((orient == 0 || orient == 2) ? 0 : 1) : ((orient == 0 || orient == 3) ? 1 : 0);
        const DPrimer &P = pairs[pair].prim[pr];
        const int L = P.L;
        const uint64_t s0 = st.d_seq_block0[seq] * 64;
        const uint64_t ws = side == 0 ? (uint64_t)start : (uint64_t)end - (uint64_t)L;
        bool has_n = false;
        const uint64_t G = load_site(st, s0 + ws, L, &has_n);
        // partner strand 3'->5' against the primer: complement of the plus
        // strand for an upstream (plus) site, the plus strand reversed for a
        // downstream (minus) site
        const uint64_t lm = L == 32 ? ~0ull : ((1ull << (2 * L)) - 1);
        const uint64_t Cc = side == 0 ? (G ^ (0xFFFFFFFFFFFFFFFFull & lm)) : reverse_codes(G, L);
        double best = -INFINITY;
        int lw = live && !has_n && P.D ? L : 0;
        for (int d = 32; d >= 1; d >>= 1) {
            const int o = __shfl_xor(lw, d, 64);
            lw = o > lw ? o : lw;
        }
        lw = __builtin_amdgcn_readfirstlane(lw);
        if (live && !has_n && P.D) {
            if (P.rb && L >= 3) {
                // variant v = a * rb + b: both halves advance by lps per step
                // (the loop bound lw: the wave's longest such site)
                const uint32_t rb = P.rb, ia = lps / rb, ib = lps - ia * rb;
                uint32_t a = vl / rb, b = vl - (vl / rb) * rb;
                for (uint32_t v = vl; v < P.D; v += lps) {
                    double t;
                    if (site_variant_tm(P.hi[a] | P.lo[b], Cc, L, lw, sst, stt, init, k, &t))
                        best = t > best ? t : best;
                    a += ia;
                    b += ib;
                    if (b >= rb) {
                        b -= rb;
                        a += 1;
                    }
                }
            } else {
                const uint64_t base = primer_base_codes(P);
                for (uint32_t v = vl; v < P.D; v += lps) {
                    double t;
                    if (duplex_tm(primer_variant(P, base, v), Cc, L, nn, k, &t))
                        best = t > best ? t : best;
                }
            }
        }
        for (uint32_t d = lps >> 1; d >= 1; d >>= 1) {  // within the site's lanes
            const double o = __shfl_xor(best, (int)d, 64);
            best = o > best ? o : best;
        }
        if (live && vl == 0) tm_site[2 * a + side] = best;
        if (tm) {
            const double other = __shfl_xor(best, (int)lps, 64);  // the amplicon's other site
            if (live && vl == 0 && side == 0) {
                const double t = best < other ? best : other;  // the weaker primer limits the amplicon
                const double thr = pair_thr ? pair_thr[pair] : k.threshold;
                tm[a] = t;
                pass[a] = k.filter ? (uint8_t)(t >= thr) : (uint8_t)1;
            }
        }
    }
}

__global__ void ah_tm_finish_kernel(const double *tm_site, const ah_amp *amps, const uint64_t *d_n, uint64_t cap,
                                    ah_tm_params prm, double *tm, uint8_t *pass) {
    const uint64_t n = *d_n < cap ? *d_n : cap;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const double t1 = tm_site[2 * i], t2 = tm_site[2 * i + 1];
        const double t = t1 < t2 ? t1 : t2;  // the weaker primer limits the amplicon
        const double thr = prm.d_pair_threshold ? prm.d_pair_threshold[amps[i].pair] : prm.threshold_C;
        tm[i] = t;
        pass[i] = prm.filter ? (uint8_t)(t >= thr) : (uint8_t)1;
    }
}

extern "C" ah_status ah_tm_nn(const ah_store *st, ah_primer_set ps, const ah_amp *d_amps, const uint64_t *d_n_amps,
                              uint64_t amp_cap, const ah_tm_params *p, double *d_tm, double *d_tm_site,
                              uint8_t *d_pass, void *stream) {
    if (!st || !ps || !p || !d_n_amps || (amp_cap && (!d_amps || !d_tm || !d_tm_site || !d_pass))) return AH_E_ARG;
    if (!tm_params_ok(*p)) return AH_E_ARG;  // unknown set or method, or a zero concentration under a logarithm
    uint32_t maxD = 1;
    for (uint32_t q = 0; q < ps->n_pairs; q++) {
        if (!ps->h_pairs[q].prim[0].D || !ps->h_pairs[q].prim[1].D) return AH_E_LIMIT;
        for (int r = 0; r < 2; r++) maxD = ps->h_pairs[q].prim[r].D > maxD ? ps->h_pairs[q].prim[r].D : maxD;
    }
    uint32_t lps = 1;  // lanes per site: a power of two covering the largest variant count, at most 64
    while (lps < maxD && lps < 64) lps <<= 1;
    if (!amp_cap) return AH_OK;
    hipStream_t s = ah_stream(stream);
    // 64 / lps sites per wave over a persistent grid: every workgroup stages
    // the NN tables in LDS once, so no more workgroups than can be resident
    uint64_t wgs = (2 * amp_cap + 4 * (64 / lps) - 1) / (4 * (64 / lps));
    const uint64_t resident = ah_resident_wgs(ah_tm_site_kernel, 256);
    if (wgs > resident) wgs = resident;
    const bool fused = lps <= 32;  // both sites of an amplicon in one wave
    hipLaunchKernelGGL(ah_tm_site_kernel, dim3((unsigned)wgs), dim3(256), 0, s, *st, (const DPair *)ps->d_pairs,
                       (const uint32_t *)d_amps, d_n_amps, amp_cap, tm_const(*p), lps, d_tm_site,
                       p->d_pair_threshold, fused ? d_tm : nullptr, d_pass);
    if (!fused)
        hipLaunchKernelGGL(ah_tm_finish_kernel, dim3(256), dim3(256), 0, s, (const double *)d_tm_site, d_amps,
                           d_n_amps, amp_cap, *p, d_tm, d_pass);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}

// ---------------------------------------------------------------- explicit duplexes
__device__ __forceinline__ int letter_code(char c) {
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

// Tm of one explicit duplex: primer s[0..L) 5'->3', partner c[0..Lc)
// written 3'->5', c[i] facing s[i - shift].  In a common column frame the
// primer occupies [st, st + L) and the partner [sb, sb + Lc); the positions
// facing each other are [f0, f1).  An end where one strand runs past the
// other keeps one unpaired base next to the helix (a dangling end; further
// overhang is dropped), charged with its dangling-end term -- left end
// first, then the right end read from the partner strand.  The helix is
// columns [f0, f1).  NaN if a letter is not ACGT or a stack or end is not
// tabulated; the caller has checked the lengths and that f1 - f0 >= 2.
__device__ double explicit_duplex_tm(const char *s, int L, const char *c, int Lc, int shift, const TmConst &k) {
    const int st = shift > 0 ? shift : 0, sb = shift < 0 ? -shift : 0;
    const int f0 = st > sb ? st : sb, f1 = st + L < sb + Lc ? st + L : sb + Lc;
    uint64_t S = 0, C = 0;  // the primer, and the partner positions facing the helix [f0, f1)
    for (int j = 0; j < L; j++) {
        const int b = letter_code(s[j]);
        if (b < 0) return NAN;
        S |= (uint64_t)b << (2 * j);
    }
    for (int j = 0; j < Lc; j++) {
        const int b = letter_code(c[j]);
        if (b < 0) return NAN;
        const int col = j + sb;
        if (col >= f0 && col < f1) C |= (uint64_t)b << (2 * (col - f0));
    }
    const int n = f1 - f0;
    const uint64_t V = S >> (2 * (f0 - st));  // primer bases of the helix columns
    double dh = 0.0, ds = 0.0;
    if (f0 > 0) {
        // left end: the strand that starts first keeps its base at column f0 - 1
        const int top0 = (int)(V & 3u), bot0 = (int)(C & 3u);
        const int i = st > sb ? de_index(1, letter_code(c[f0 - 1 - sb]), top0, bot0)   // partner's 3' base
                              : de_index(0, letter_code(s[f0 - 1 - st]), top0, bot0);  // primer's 5' base
        if (!tab_ok(g_dangle.ok, i)) return NAN;
        dh += g_dangle.dh[i];
        ds += g_dangle.ds[i];
    }
    if (st + L != sb + Lc) {
        // right end, read from the partner strand: the primer's 3' base, or
        // the partner's 5' base, at column f1
        const int topn = (int)((V >> (2 * (n - 1))) & 3u), botn = (int)((C >> (2 * (n - 1))) & 3u);
        const int i = st + L > sb + Lc ? de_index(1, letter_code(s[f1 - st]), botn, topn)
                                       : de_index(0, letter_code(c[f1 - sb]), botn, topn);
        if (!tab_ok(g_dangle.ok, i)) return NAN;
        dh += g_dangle.dh[i];
        ds += g_dangle.ds[i];
    }
    const PrimerEnds P{(int)(S & 3u), (int)((S >> (2 * (L - 1))) & 3u), L, gc_count(S, L)};
    double t;
    if (!helix_tm(V, C, n, dh, ds, P, ConstTables{k.table}, k, &t)) return NAN;
    return t;
}

__global__ void ah_tm_duplex_kernel(const char *seq, const char *cseq, const uint32_t *len, const uint32_t *clen,
                                    const int32_t *shift, uint32_t n, uint32_t stride, TmConst k, double *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int L = (int)len[i];
        const int Lc = clen ? (int)clen[i] : L;
        const int sh = shift ? shift[i] : 0;
        const int st = sh > 0 ? sh : 0, sb = sh < 0 ? -sh : 0;
        // facing positions: columns where both strands have a base
        const int f0 = st > sb ? st : sb, f1 = (st + L < sb + Lc ? st + L : sb + Lc);
        const bool ok = L >= 2 && L <= 32 && Lc >= 1 && Lc <= 64 && (uint32_t)L <= stride &&
                        (uint32_t)Lc <= stride && sh >= -64 && sh <= 64 && f1 - f0 >= 2;
        out[i] = ok ? explicit_duplex_tm(seq + (uint64_t)i * stride, L, cseq + (uint64_t)i * stride, Lc, sh, k) : NAN;
    }
}

extern "C" ah_status ah_tm_duplex(const char *d_seq, const char *d_cseq, const uint32_t *d_len,
                                  const uint32_t *d_clen, const int32_t *d_shift, uint32_t n, uint32_t stride,
                                  const ah_tm_params *p, double *d_tm, void *stream) {
    if (!p || (n && (!d_seq || !d_cseq || !d_len || !d_tm))) return AH_E_ARG;
    if (!tm_params_ok(*p)) return AH_E_ARG;  // unknown set or method, or a zero concentration under a logarithm
    if (!n) return AH_OK;
    unsigned blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(ah_tm_duplex_kernel, dim3(blocks), dim3(256), 0, ah_stream(stream), d_seq, d_cseq, d_len,
                       d_clen, d_shift, n, stride, tm_const(*p), d_tm);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
