// Primer scan entry points (Supplementary, "Primer matching and clamp
// logic").  The kernel body is in scan_core.h.  Two filters drive it:
//  - the generic kernel reads each pattern's clamp codes at run time and
//    dispatches every IUPAC set to a one-instruction match with a uniform
//    (scalar) branch;
//  - ah_primers_jit() compiles, with hipRTC, a kernel whose clamp codes are
//    compile-time constants, so each set test folds into the running AND.
// Both share the exact per-candidate verification, so they produce the same
// hits.
#include <hip/hiprtc.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "ah_internal.h"
#include "ah_scan_impl.h"
#include "scan_core.h"

// hipRTC needs the text of the headers the kernel body includes; the build
// embeds them here.
#include "jit_headers.inc"

// ---------------------------------------------------------------- generic filter
// Clamp codes are read at run time.  Per filter offset the four one-hot
// planes (base q+i is A / C / G / T) are formed once and shared by the four
// patterns of the group; a pattern's set test is the OR of the planes its
// IUPAC code allows, selected with scalar all-ones/all-zero masks.
__device__ __forceinline__ uint32_t ah_pick(uint32_t eA, uint32_t eC, uint32_t eG, uint32_t eT, uint32_t m) {
    const uint32_t sa = (m & 1u) ? 0xFFFFFFFFu : 0u, sc = (m & 2u) ? 0xFFFFFFFFu : 0u;
    const uint32_t sg = (m & 4u) ? 0xFFFFFFFFu : 0u, st = (m & 8u) ? 0xFFFFFFFFu : 0u;
    return (eA & sa) | (eC & sc) | (eG & sg) | (eT & st);
}

struct GenericFilter {
    const DPat *sPat;
    const DPat *gPat;
    uint32_t n_lds;
    __device__ uint32_t groups(const ScanArgs &a) const { return a.n_groups; }
    static constexpr bool kUsesBase = false;
    static constexpr int kW = AH_WMAX;
    static constexpr bool kHoistGuard = false;  // codes are read at run time
    static constexpr bool kSkipEmpty = true;
    static constexpr int kHalves = 1;
    static constexpr int kGroupStep = 1;
    __device__ __forceinline__ void block(const AhBase &, int) {}
    __device__ __forceinline__ void guard() {}
    __device__ __forceinline__ void filter(uint32_t g, int, const AhBase &, const uint32_t (&Sh)[AH_WMAX][AH_HW],
                                           const uint32_t (&Sl)[AH_WMAX][AH_HW], uint32_t (&C)[4 * AH_HW]) const {
        uint32_t fc[4][2], W = 0;
#pragma unroll
        for (int x = 0; x < 4; x++) {
            const uint32_t X = 4 * g + (uint32_t)x;
            uint32_t meta, f0, f1;
            if (X < n_lds) {
                meta = ah_lds<uint32_t>(&sPat[X].meta);
                f0 = ah_lds<uint32_t>(&sPat[X].fcode[0]);
                f1 = ah_lds<uint32_t>(&sPat[X].fcode[4]);
            } else {
                meta = ah_ldg<uint32_t>(&gPat[X].meta);
                f0 = ah_ldg<uint32_t>(&gPat[X].fcode[0]);
                f1 = ah_ldg<uint32_t>(&gPat[X].fcode[4]);
            }
            meta = __builtin_amdgcn_readfirstlane(meta);
            f0 = __builtin_amdgcn_readfirstlane(f0);
            f1 = __builtin_amdgcn_readfirstlane(f1);
            // positions past a pattern's own W read as N (every base matches)
            const uint32_t wx = (meta >> 16) & 0xFFu;
            const uint64_t all = ((uint64_t)f1 << 32) | f0;
            const uint64_t keep = wx >= 8 ? ~0ull : ((1ull << (8 * wx)) - 1);
            const uint64_t codes = (all & keep) | (0x0F0F0F0F0F0F0F0Full & ~keep);
            fc[x][0] = (uint32_t)codes;
            fc[x][1] = (uint32_t)(codes >> 32);
            W = wx > W ? wx : W;
#pragma unroll
            for (int w = 0; w < AH_HW; w++) C[AH_HW * x + w] = 0xFFFFFFFFu;
        }
#pragma unroll
        for (int i = 0; i < AH_WMAX; i++) {
            if ((uint32_t)i >= W) break;
#pragma unroll
            for (int w = 0; w < AH_HW; w++) {
                const uint32_t h = Sh[i][w], l = Sl[i][w];
                const uint32_t aa = ~(h | l), cc = ~h & l, gg = h & ~l, tt = h & l;
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    const uint32_t m = ((i < 4 ? fc[x][0] >> (8 * i) : fc[x][1] >> (8 * (i - 4)))) & 0xFu;
                    C[AH_HW * x + w] &= ah_pick(aa, cc, gg, tt, m);
                }
            }
        }
    }
};

// kLdsOnly: every pattern record fits in LDS (at most AH_LDS_PATS patterns).
template <bool kLdsOnly>
__global__ void __launch_bounds__(256) ah_scan_kernel(ScanArgs a) {
    __shared__ DPat sPat[AH_LDS_PATS];
    __shared__ TileCtx sCtx[4][AH_NCTX];
    __shared__ uint32_t sQ[4][AH_QCAP + 1][AH_QW];
    __shared__ uint2 sW[4][AH_NCTX][AH_TW];
    __shared__ uint32_t sH[4][AH_HCAP][3];
    __shared__ uint32_t sHn[4];
    ah_stage_patterns(a, sPat, AH_LDS_PATS);
    const uint32_t n_lds = a.n_pats < AH_LDS_PATS ? a.n_pats : AH_LDS_PATS;
    GenericFilter f{sPat, a.pats, n_lds};
    ah_scan_body<kLdsOnly>(a, f, sPat, n_lds, sCtx, sQ, sW, sH, sHn);
}

// ---------------------------------------------------------------- tile table
__global__ void ah_tile_count_kernel(ah_store st, const uint32_t *list, uint32_t n, uint32_t tile_blocks,
                                     uint64_t *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t s = list ? list[i] : i;
        // an index outside the store contributes no tiles
        const uint64_t nblk = s < st.n_seqs ? ((uint64_t)st.d_seq_len[s] + 63) / 64 : 0;
        out[i] = (nblk + tile_blocks - 1) / tile_blocks;
    }
}

// Tiles per listed sequence and their exclusive prefix in one workgroup (for
// up to AH_TILE_PREF_ONE_WG sequences, one contiguous chunk per thread); also
// clears the hit counter.
#define AH_TILE_PREF_ONE_WG 16384u
__device__ __forceinline__ uint64_t tiles_of(const ah_store &st, const uint32_t *list, uint64_t i,
                                             uint32_t tile_blocks) {
    const uint32_t s = list ? list[i] : (uint32_t)i;
    const uint64_t nblk = s < st.n_seqs ? ((uint64_t)st.d_seq_len[s] + 63) / 64 : 0;
    return (nblk + tile_blocks - 1) / tile_blocks;
}

__global__ void __launch_bounds__(1024) ah_tile_pref_kernel(ah_store st, const uint32_t *list, uint32_t n,
                                                            uint32_t tile_blocks, uint64_t *pref, uint64_t *n_hits) {
    __shared__ uint64_t lds[16];
    if (threadIdx.x == 0) *n_hits = 0;
    const uint64_t per = ((uint64_t)n + blockDim.x - 1) / blockDim.x;
    const uint64_t i0 = threadIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    uint64_t loc = 0;
    for (uint64_t i = i0; i < i1; i++) loc += tiles_of(st, list, i, tile_blocks);
    uint64_t tot;
    uint64_t o = ah_block_excl_sum<uint64_t>(loc, lds, tot);
    for (uint64_t i = i0; i < i1; i++) {
        pref[i] = o;
        o += tiles_of(st, list, i, tile_blocks);
    }
    if (threadIdx.x == 0) pref[n] = tot;
}

__global__ void __launch_bounds__(1024) ah_scan_small_u64_kernel(const uint64_t *in, uint64_t *out, uint64_t n) {
    __shared__ uint64_t lds[16];
    const uint64_t per = (n + blockDim.x - 1) / blockDim.x;  // one contiguous chunk per thread
    const uint64_t i0 = threadIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    uint64_t loc = 0;
    for (uint64_t i = i0; i < i1; i++) loc += in[i];
    uint64_t tot;
    uint64_t o = ah_block_excl_sum<uint64_t>(loc, lds, tot);
    for (uint64_t i = i0; i < i1; i++) {
        const uint64_t v = in[i];
        out[i] = o;
        o += v;
    }
    if (threadIdx.x == 0) out[n] = tot;
}

void ah_scan_small_u64(const uint64_t *d_in, uint64_t *d_out, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(ah_scan_small_u64_kernel, dim3(1), dim3(1024), 0, s, d_in, d_out, n);
}

extern "C" ah_status ah_scan_ws_size(const ah_store *st, uint32_t n_list, uint64_t *bytes) {
    if (!st || !bytes) return AH_E_ARG;
    *bytes = ah_align_up(8ull * n_list, 256) + ah_align_up(8ull * (n_list + 1), 256);
    return AH_OK;
}

// ---------------------------------------------------------------- JIT
struct AhJit {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int per_cu = 0;  // resident workgroups per CU
    int device = -1;
    uint32_t bpl = 1;   // 64-base blocks per lane (a wave's tile: 64 x bpl blocks)
    uint32_t hcap = 0;  // LDS hit buffer records per wave
};

// Every compiled variant of a primer set's specialised kernel; one is active.
struct AhJitSet {
    std::vector<AhJit *> v;
    AhJit *active = nullptr;
};

#define AH_JIT_DEFAULT_BPL 2u
#define AH_JIT_DEFAULT_HCAP 48u

// ---------------------------------------------------------------- filter plan
// The clamp positions alone let through about prod(|set|/4) of all windows;
// with a small clamp and many patterns, verifying those candidates dominates.
// A hit has at most k mismatches outside the clamp, so of k+1 disjoint
// groups of non-clamp positions at least one matches exactly (pigeonhole):
// "clamp exact AND some group exact" is still a necessary condition.  Groups
// take the non-clamp positions nearest the clamp (same offsets for the two
// patterns of a strand, so their shifted planes are shared), round-robin.
// The group size s (0 = clamp only) minimises an estimate of vector
// instructions per 4096-base tile: tests and shifts against candidates
// verified (3.5 instructions each, fitted on a 64-pair set: 2.25, 3.5, 5 and 8
// gave 37.6, 37.3, 37.6 and 37.7 ms per scan).  In a set of many pairs
// the shifted planes of each strand are formed once per block for all of
// them (offsets within [-kSharedReach, kSharedReach + AH_WMAX)), so a
// position costs its two tests only.
struct FiltPos {
    int d;           // offset from the clamp site
    unsigned code;   // IUPAC set (bit b = base b)
};
struct FiltPlan {
    std::vector<FiltPos> groups[AH_MAXL];
    int n_groups = 0;
};

static unsigned pat_code(const DPat &P, int j) {
    unsigned m = 0;
    for (int b = 0; b < 4; b++)
        if ((P.P[b] >> j) & 1u) m |= 1u << b;
    return m;
}

static double set_frac(unsigned m) { return __builtin_popcount(m) / 4.0; }

#define AH_SHARED_REACH 12

static FiltPlan plan_filter(const DPat &P, bool shared) {
    FiltPlan best;
    const int L = (int)(P.meta & 0xFFu), k = (int)((P.meta >> 8) & 0xFFu), W = (int)((P.meta >> 16) & 0xFFu);
    const int shift = (int)(P.meta >> 24);
    const bool minus = ((P.pk >> 16) & 2u) != 0;
    if (k + 1 > AH_MAXL) return best;
    double p_clamp = 1.0;
    for (int i = 0; i < W; i++) p_clamp *= set_frac(P.fcode[i]);
    // non-clamp positions (N codes excluded: they match everything), nearest
    // to the clamp first
    std::vector<FiltPos> near;
    if (minus) {
        for (int j = 0; j < L; j++)
            if (!((P.clampmask >> j) & 1u) && pat_code(P, j) != 15u) near.push_back({j - shift, pat_code(P, j)});
    } else {
        for (int j = L - 1; j >= 0; j--)
            if (!((P.clampmask >> j) & 1u) && pat_code(P, j) != 15u) near.push_back({j - shift, pat_code(P, j)});
    }
    const double kVerify = 3.5, kTile = 4096.0;
    double best_cost = 2.0 * W + kTile * p_clamp * kVerify + 6.0;
    for (int sz = 1; sz <= 4; sz++) {
        const int need = sz * (k + 1);
        if (need > (int)near.size()) break;
        FiltPlan plan;
        plan.n_groups = k + 1;
        bool ok = true;
        double p_any = 0.0;
        for (int g = 0; g <= k; g++) {
            double pg = 1.0;
            for (int t = 0; t < sz; t++) {
                const FiltPos &fp = near[g + t * (k + 1)];
                if (fp.d <= -32 || fp.d >= 32) ok = false;
                if (shared && (fp.d < -AH_SHARED_REACH || fp.d >= AH_SHARED_REACH + AH_WMAX)) ok = false;
                plan.groups[g].push_back(fp);
                pg *= set_frac(fp.code);
            }
            p_any += pg;
        }
        if (!ok) break;
        if (p_any > 1.0) p_any = 1.0;
        // tests: 2 words per position; shifts: 4 funnel shifts per position,
        // shared by the two patterns of a strand (by every pattern of the
        // strand when shared); one OR per group and word
        const double per_pos = shared ? 2.0 : 4.0;
        const double cost = 2.0 * W + 2.0 * (k + 1) + per_pos * need + kTile * p_clamp * p_any * kVerify + 6.0;
        if (cost < best_cost) {
            best_cost = cost;
            best = plan;
        }
    }
    return best;
}

// Set tests of one pigeonhole group, word `word`: from the filter's own
// shifted planes (offsets 0..kW-1), the shared planes of the pass (`offs`,
// when not null), or shifts of the base words.
static std::string set_test_chain(std::string acc, const std::vector<FiltPos> &pos, int word, int kW,
                                  const std::vector<int> *offs) {
    const std::string Ws = std::to_string(word);
    for (const FiltPos &fp : pos) {
        const std::string M = std::to_string(fp.code) + "u";
        if (fp.d >= 0 && fp.d < kW) {
            const std::string I = std::to_string(fp.d);
            acc = "ah_and_set<" + M + ">(" + acc + ", Sh[" + I + "][" + Ws + "], Sl[" + I + "][" + Ws + "])";
        } else if (offs) {
            const int i = (int)(std::find(offs->begin(), offs->end(), fp.d) - offs->begin());
            const std::string I = std::to_string(i);
            acc = "ah_and_set<" + M + ">(" + acc + ", Ph[" + I + "][" + Ws + "], Pl[" + I + "][" + Ws + "])";
        } else {
            acc = "ah_and_at<" + M + ", " + std::to_string(fp.d) + ", " + Ws + ">(" + acc + ", B)";
        }
    }
    return acc;
}

// Kernel source specialised to a primer set: the codes of every oriented
// pattern's filter positions become template constants of the set tests.
static std::string jit_source(const ah_primer_set_ *ps, uint32_t bpl, uint32_t hcap) {
    std::string s;
    const int nw = AH_HW;  // words per plane of the block the filter sees
    const int kW = ps->max_W > 0 ? ps->max_W : 1;
    // many pairs: each strand's shifted planes formed once per block
    const bool shared = ps->n_pairs > 1;
    std::vector<FiltPlan> plans(ps->n_pats);
    bool any_groups = false;
    std::vector<int> offs[2];  // shared offsets of the plus (x = 0, 1) and minus (x = 2, 3) patterns
    for (uint32_t X = 0; X < ps->n_pats; X++) {
        plans[X] = plan_filter(ps->h_pats[X], shared);
        any_groups = any_groups || plans[X].n_groups > 0;
        for (int q = 0; q < plans[X].n_groups; q++)
            for (const FiltPos &fp : plans[X].groups[q]) {
                std::vector<int> &o = offs[(X & 3u) >> 1];
                if ((fp.d < 0 || fp.d >= kW) && std::find(o.begin(), o.end(), fp.d) == o.end()) o.push_back(fp.d);
            }
    }
    const bool halves = shared && any_groups;
    const size_t n_sh = std::max(offs[0].size(), offs[1].size());
    s += "#define AH_BPL " + std::to_string(bpl) + "\n";
    s += "#define AH_HCAP " + std::to_string(hcap) + "\n";
    s += "#include \"scan_core.h\"\n";
    s += std::string("#define AH_JIT_USES_BASE ") + (any_groups ? "true" : "false") + "\n";
    s += "struct JitFilter {\n";
    s += "  static constexpr bool kUsesBase = AH_JIT_USES_BASE;\n";
    s += "  static constexpr int kW = " + std::to_string(kW) + ";\n";
    s += std::string("  static constexpr bool kHoistGuard = ") + (ps->n_pairs > 1 ? "true" : "false") + ";\n";
    s += std::string("  static constexpr bool kSkipEmpty = ") + (ps->n_pairs > 1 ? "true" : "false") + ";\n";
    // with shared planes, four groups per filter call: one dispatch on the
    // group index per four groups
    const uint32_t gstep = halves ? 4u : 1u;
    s += std::string("  static constexpr int kHalves = ") + (halves ? "2" : "1") + ";\n";
    s += "  static constexpr int kGroupStep = " + std::to_string(gstep) + ";\n";
    // the shared planes of the current pass: Ph/Pl[i][w] = word w of the
    // plane shifted by the pass's i-th offset
    s += "  static constexpr int kNP = " + std::to_string(halves && n_sh ? n_sh : 1) + ";\n";
    s += "  uint32_t Ph[kNP][AH_HW], Pl[kNP][AH_HW];\n";
    s += "  __device__ __forceinline__ void block(const AhBase &B, int half) {\n";
    if (halves) {
        for (int h = 0; h < 2; h++) {
            s += std::string(h ? "    else {\n" : "    if (half == 0) {\n");
            for (size_t i = 0; i < offs[h].size(); i++)
                for (int w = 0; w < nw; w++) {
                    const std::string tgt = "[" + std::to_string(i) + "][" + std::to_string(w) + "]";
                    const std::string tp = "<" + std::to_string(offs[h][i]) + ", " + std::to_string(w) + ">";
                    s += "      Ph" + tgt + " = ah_shw" + tp + "(B.h);\n";
                    s += "      Pl" + tgt + " = ah_shw" + tp + "(B.l);\n";
                }
            s += "    }\n";
        }
    }
    s += "  }\n";
    s += "  __device__ __forceinline__ void guard() {\n";
    if (halves && n_sh)
        s += "#pragma unroll\n    for (int i = 0; i < kNP; i++)\n#pragma unroll\n"
             "      for (int w = 0; w < AH_HW; w++) asm volatile(\"\" : \"+v\"(Ph[i][w]), \"+v\"(Pl[i][w]));\n";
    s += "  }\n";
    s += "  __device__ uint32_t groups(const ScanArgs &) const { return " + std::to_string(ps->n_pairs) + "u; }\n";
    s += "  __device__ __forceinline__ void filter(uint32_t g, int half, const AhBase &B, "
         "const uint32_t (&Sh)[AH_WMAX][AH_HW], const uint32_t (&Sl)[AH_WMAX][AH_HW], "
         "uint32_t (&C)[kGroupStep * 4 / kHalves * AH_HW]) const {\n";
    s += "    switch (g) {\n";
    for (uint32_t g0 = 0; g0 < ps->n_pairs; g0 += gstep) {
        s += "    case " + std::to_string(g0) + "u: {\n";
        for (int h = 0; h < (halves ? 2 : 1); h++) {
            if (halves) s += std::string(h ? "      } else {\n" : "      if (half == 0) {\n");
            const int x0 = halves ? 2 * h : 0, nx = halves ? 2 : 4;
            for (uint32_t gi = 0; gi < gstep; gi++)
            for (int xi = 0; xi < nx; xi++) {
                const uint32_t g = g0 + gi;
                const int slot = (int)(gi * nx + xi) * nw;  // first word of (group, pattern) in C
                if (g >= ps->n_pairs) {
                    for (int w = 0; w < nw; w++) s += "      C[" + std::to_string(slot + w) + "] = 0u;\n";
                    continue;
                }
                const int x = x0 + xi;
                const DPat &P = ps->h_pats[4 * g + x];
                const uint32_t W = (P.meta >> 16) & 0xFFu;
                const FiltPlan &plan = plans[4 * g + x];
                for (int w = 0; w < nw; w++) {
                    const std::string Ws = std::to_string(w);
                    std::string c = "0xFFFFFFFFu";
                    for (uint32_t i = 0; i < W; i++) {
                        const unsigned m = P.fcode[i];
                        if (m == 15) continue;  // N matches every base
                        const std::string I = std::to_string(i), M = std::to_string(m);
                        c = "ah_and_set<" + M + "u>(" + c + ", Sh[" + I + "][" + Ws + "], Sl[" + I + "][" + Ws + "])";
                    }
                    if (plan.n_groups) {
                        std::string any;
                        for (int q = 0; q < plan.n_groups; q++)
                            any += (q ? " | " : "") +
                                   set_test_chain("0xFFFFFFFFu", plan.groups[q], w, kW, halves ? &offs[h] : nullptr);
                        c = "(" + c + ") & (" + any + ")";
                    }
                    s += "      C[" + std::to_string(slot + w) + "] = " + c + ";\n";
                }
            }
        }
        if (halves) s += "      }\n";
        s += "      break; }\n";
    }
    s += "    default: for (int w = 0; w < kGroupStep * 4 / kHalves * AH_HW; w++) C[w] = 0u;\n";
    s += "    }\n  }\n};\n";
    const uint32_t n_lds = ps->n_pats < AH_LDS_PATS ? ps->n_pats : AH_LDS_PATS;
    s += "#define AH_JIT_LDS_PATS " + std::to_string(n_lds) + "u\n";
    s += std::string("#define AH_JIT_LDS_ONLY ") + (ps->n_pats <= AH_LDS_PATS ? "true" : "false") + "\n";
    // two-block tiles for a few pairs: bound the registers to six waves per
    // SIMD (80 VGPRs, no spills), the count the LDS allows; with shared
    // strand planes, to three (168 VGPRs), so that both tile sizes keep three
    // workgroups per CU
    const std::string bounds = (bpl == 2 && ps->n_pairs <= 4) ? "__launch_bounds__(256, 6)"
                               : halves                       ? "__launch_bounds__(256, 3)"
                                                              : "__launch_bounds__(256)";
    s += "extern \"C\" __global__ void " + bounds + " ah_scan_jit(ScanArgs a) {\n"
         "  __shared__ DPat sPat[AH_JIT_LDS_PATS];\n"
         "  __shared__ TileCtx sCtx[4][AH_NCTX];\n"
         "  __shared__ uint32_t sQ[4][AH_QCAP + 1][AH_QW];\n"
         "  __shared__ uint2 sW[4][AH_NCTX][AH_TW];\n"
         "  __shared__ uint32_t sH[4][AH_HCAP][3];\n"
         "  __shared__ uint32_t sHn[4];\n"
         "  ah_stage_patterns(a, sPat, AH_JIT_LDS_PATS);\n"
         "  JitFilter f;\n"
         "  ah_scan_body<AH_JIT_LDS_ONLY>(a, f, sPat, AH_JIT_LDS_PATS, sCtx, sQ, sW, sH, sHn);\n"
         "}\n";
    return s;
}

static int device_cus(int dev) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    return cus;
}

// Compile the specialised kernel for `arch` (e.g. "gfx950"); code object in *code.
static bool jit_variant_ok(uint32_t bpl, uint32_t hcap) { return (bpl == 1 || bpl == 2) && hcap >= 2 && hcap <= 256; }

static ah_status jit_compile(const ah_primer_set_ *ps, const std::string &arch, uint32_t bpl, uint32_t hcap,
                             std::vector<char> *code) {
    const std::string src = jit_source(ps, bpl, hcap);
    // AH_JIT_DUMP=<path>: also write the generated source there (inspection)
    if (const char *dump = getenv("AH_JIT_DUMP")) {
        if (FILE *f = fopen(dump, "w")) {
            fwrite(src.data(), 1, src.size(), f);
            fclose(f);
        }
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "ah_scan_jit.hip", AH_JIT_NHEADERS, kJitHeaderText,
                            kJitHeaderNames) != HIPRTC_SUCCESS)
        return AH_E_HIP;
    const std::string arch_opt = "--offload-arch=" + arch;
    // no packed-FP32 instructions, as for the library itself
    const char *opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    if (hiprtcCompileProgram(prog, 8, opts) != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::vector<char> log(n + 1, 0);
        hiprtcGetProgramLog(prog, log.data());
        fprintf(stderr, "ah_primers_jit: hipRTC failed:\n%s\n", log.data());
        hiprtcDestroyProgram(&prog);
        return AH_E_HIP;
    }
    size_t code_n = 0;
    hiprtcGetCodeSize(prog, &code_n);
    code->assign(code_n, 0);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return AH_OK;
}

extern "C" ah_status ah_primers_jit_check(const ah_pair_spec *h_pairs, uint32_t n_pairs, const char *arch,
                                          uint32_t blocks_per_lane, uint32_t hit_buffer) {
    if (!arch || !*arch || !jit_variant_ok(blocks_per_lane, hit_buffer)) return AH_E_ARG;
    ah_primer_set ps = nullptr;
    ah_status st = ah_build_primer_set(h_pairs, n_pairs, true, &ps);
    if (st != AH_OK) return st;
    std::vector<char> code;
    st = jit_compile(ps, arch, blocks_per_lane, hit_buffer, &code);
    ah_primers_free(ps);
    return st;
}

extern "C" ah_status ah_primers_jit_variant(ah_primer_set ps, uint32_t blocks_per_lane, uint32_t hit_buffer) {
    if (!ps || !jit_variant_ok(blocks_per_lane, hit_buffer)) return AH_E_ARG;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess) return AH_E_HIP;
    AhJitSet *set = (AhJitSet *)ps->jit;
    if (set) {
        for (AhJit *j : set->v) {
            if (j->device == dev && j->bpl == blocks_per_lane && j->hcap == hit_buffer) {
                set->active = j;
                ps->use_jit = 1;
                return AH_OK;
            }
        }
    }
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return AH_E_HIP;
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');  // drop feature suffixes such as ":sramecc+:xnack-"
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::vector<char> code;
    const ah_status st = jit_compile(ps, arch, blocks_per_lane, hit_buffer, &code);
    if (st != AH_OK) return st;
    AhJit *j = new AhJit();
    if (hipModuleLoadData(&j->mod, code.data()) != hipSuccess ||
        hipModuleGetFunction(&j->fn, j->mod, "ah_scan_jit") != hipSuccess) {
        if (j->mod) (void)hipModuleUnload(j->mod);
        delete j;
        return AH_E_HIP;
    }
    int per_cu = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, j->fn, 256, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    j->per_cu = per_cu;
    j->device = dev;
    j->bpl = blocks_per_lane;
    j->hcap = hit_buffer;
    if (!set) {
        set = new AhJitSet();
        ps->jit = set;
    }
    set->v.push_back(j);
    set->active = j;
    ps->use_jit = 1;
    return AH_OK;
}

extern "C" ah_status ah_primers_jit(ah_primer_set ps) {
    if (!ps) return AH_E_ARG;
    const AhJitSet *set = (const AhJitSet *)ps->jit;
    if (set && set->active) {
        ps->use_jit = 1;
        return AH_OK;
    }
    return ah_primers_jit_variant(ps, AH_JIT_DEFAULT_BPL, AH_JIT_DEFAULT_HCAP);
}

extern "C" ah_status ah_primers_use_jit(ah_primer_set ps, int32_t on) {
    if (!ps) return AH_E_ARG;
    if (on && !(ps->jit && ((const AhJitSet *)ps->jit)->active)) return AH_E_ARG;
    ps->use_jit = on ? 1 : 0;
    return AH_OK;
}

void ah_jit_free(void *jit) {
    AhJitSet *set = (AhJitSet *)jit;
    if (!set) return;
    for (AhJit *j : set->v) {
        if (j->mod) (void)hipModuleUnload(j->mod);
        delete j;
    }
    delete set;
}

// Resident workgroups per CU of the generic kernel (same on every gfx950 device).
static int generic_per_cu() {
    static int per_cu = 0;
    if (!per_cu) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, ah_scan_kernel<false>, 256, 0) != hipSuccess || v <= 0)
            v = 1;
        per_cu = v;
    }
    return per_cu;
}

// The active specialised variant if it is in use on this device, else null.
static const AhJit *jit_active(ah_primer_set ps, int dev) {
    const AhJitSet *set = (const AhJitSet *)ps->jit;
    const AhJit *j = set ? set->active : nullptr;
    return j && ps->use_jit && j->device == dev ? j : nullptr;
}

extern "C" ah_status ah_primers_launch_shape(ah_primer_set ps, int32_t wg_per_cu, int32_t *max_wg_per_cu) {
    if (!ps || wg_per_cu < 0) return AH_E_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AH_E_HIP;
    ps->wg_per_cu = wg_per_cu;
    const AhJit *j = jit_active(ps, dev);
    if (max_wg_per_cu) *max_wg_per_cu = j ? j->per_cu : generic_per_cu();
    return AH_OK;
}

// ---------------------------------------------------------------- entry point

static ah_status scan_launch(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset, uint32_t n_subset,
                             const uint64_t *d_pair_mask, ah_hit *d_hits, uint64_t hit_cap, uint64_t *d_n_hits,
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
    int dev = 0;
    (void)hipGetDevice(&dev);
    const AhJit *jk = jit_active(ps, dev);
    // tiles of the kernel that will run (a specialised variant may use larger ones)
    const uint32_t tile_blocks = jk ? 64u * jk->bpl : (uint32_t)AH_TILE_BLOCKS;
    if (n_list && n_list <= AH_TILE_PREF_ONE_WG) {  // counts, prefix and the cleared counter in one launch
        hipLaunchKernelGGL(ah_tile_pref_kernel, dim3(1), dim3(1024), 0, s, *st, d_seq_subset, n_list, tile_blocks,
                           pref, d_n_hits);
    } else {
        ah_fill<uint64_t>(d_n_hits, 0ull, 1, s);
        if (!n_list) return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
        hipLaunchKernelGGL(ah_tile_count_kernel, dim3(256), dim3(256), 0, s, *st, d_seq_subset, n_list, tile_blocks,
                           cnt);
        ah_scan_small_u64(cnt, pref, n_list, s);
    }
    ScanArgs a;
    a.st = *st;
    a.pats = ps->d_pats;
    a.n_pats = ps->n_pats;
    a.n_groups = ps->n_pairs;
    a.list = d_seq_subset;
    a.n_list = n_list;
    a.tile_pref = pref;
    a.gmask = d_pair_mask;
    a.hits = (uint32_t *)d_hits;
    a.hit_cap = hit_cap;
    a.n_hits = d_n_hits;
    // persistent grid: the workgroups that can be resident at once (or fewer, as set)
    int per_cu = jk ? jk->per_cu : generic_per_cu();
    if (ps->wg_per_cu > 0 && ps->wg_per_cu < per_cu) per_cu = ps->wg_per_cu;
    const unsigned grid = (unsigned)(device_cus(dev) * per_cu);
    if (jk) {
        void *args[] = {&a};
        if (hipModuleLaunchKernel(jk->fn, grid, 1, 1, 256, 1, 1, 0, s, args, nullptr) != hipSuccess)
            return AH_E_HIP;
        return AH_OK;
    }
    if (ps->n_pats <= AH_LDS_PATS)
        hipLaunchKernelGGL(ah_scan_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(ah_scan_kernel<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}

extern "C" ah_status ah_scan_primers(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset,
                                     uint32_t n_subset, ah_hit *d_hits, uint64_t hit_cap, uint64_t *d_n_hits,
                                     void *d_ws, uint64_t ws_bytes, void *stream) {
    return scan_launch(st, ps, d_seq_subset, n_subset, nullptr, d_hits, hit_cap, d_n_hits, d_ws, ws_bytes, stream);
}

extern "C" ah_status ah_scan_primers_masked(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset,
                                            uint32_t n_subset, const uint64_t *d_pair_mask, ah_hit *d_hits,
                                            uint64_t hit_cap, uint64_t *d_n_hits, void *d_ws, uint64_t ws_bytes,
                                            void *stream) {
    if (!ps || !d_pair_mask) return AH_E_ARG;
    if (ps->n_pairs > 64) return AH_E_LIMIT;
    return scan_launch(st, ps, d_seq_subset, n_subset, d_pair_mask, d_hits, hit_cap, d_n_hits, d_ws, ws_bytes,
                       stream);
}

// ---------------------------------------------------------------- no-allocation variant
// For callers that cannot allocate device memory (code under graph capture,
// serving loops, hosts that forbid hipMalloc): the scan's workspace -- the
// tile count and first tile of every listed sequence -- lives in a fixed
// array of the library instead of a caller buffer.  Each GPU holds its own
// copy until the process ends.
static __device__ __align__(256) uint8_t scratch[AH_STATIC_SCRATCH_BYTES];

// Device address of `scratch` per device, looked up once with that device
// current (the host-side name of the array is not a device address).
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[AH_MAX_DEVICES];

static ah_status static_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= AH_MAX_DEVICES) return AH_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return AH_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AH_OK;
}

extern "C" ah_status ah_scan_primers_static(const ah_store *st, ah_primer_set ps, const uint32_t *d_seq_subset,
                                            uint32_t n_subset, ah_hit *d_hits, uint64_t hit_cap,
                                            uint64_t *d_n_hits, void *stream) {
    if (!st) return AH_E_ARG;
    const uint32_t n_list = d_seq_subset ? n_subset : st->n_seqs;
    if (n_list > AH_STATIC_SCAN_MAX_LIST) return AH_E_SCRATCH;
    uint64_t need = 0;
    ah_scan_ws_size(st, n_list, &need);
    if (need > sizeof(scratch)) return AH_E_SCRATCH;
    void *ws = nullptr;
    const ah_status e = static_scratch(&ws);
    if (e) return e;
    // every workspace word the scan reads is written by the same call first
    // (tile counts, then their prefix), so nothing needs clearing
    return scan_launch(st, ps, d_seq_subset, n_subset, nullptr, d_hits, hit_cap, d_n_hits, ws, sizeof(scratch),
                       stream);
}
