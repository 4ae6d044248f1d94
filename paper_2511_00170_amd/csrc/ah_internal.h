// Internal declarations shared by the HIP translation units of libah.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ah_dev.h"

struct ah_primer_set_ {
    uint32_t n_pairs;
    uint32_t n_pats;
    uint32_t max_L;
    uint32_t max_W;
    uint32_t min_W;
    DPat *d_pats;
    DPair *d_pairs;
    DPair *h_pairs;
    DPat *h_pats;
    int device;
    void *jit;    // primer-set specialised scan kernel (ah_primers_jit), or null
    int use_jit;
    int wg_per_cu;  // persistent scan workgroups per CU (0 = resident maximum)
    int owns_device; // d_pats / d_pairs were allocated by the library
};

void ah_jit_free(void *jit);
// Host tables of a primer set; with host_only no device memory is touched
// (such a set may only be inspected or freed).
ah_status ah_build_primer_set(const ah_pair_spec *h_pairs, uint32_t n_pairs, bool host_only, ah_primer_set *out);

// ---------------------------------------------------------------- helpers
#define AH_CHECK_HIP(x)                         \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return AH_E_HIP;  \
    } while (0)

static inline hipStream_t ah_stream(void *s) { return (hipStream_t)s; }

#define AH_MAX_DEVICES 64  // per-device state of the library (device ordinals 0..63)

// Compute units of the current device (256 on MI355X if the query fails).
static inline uint32_t ah_device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return (uint32_t)cus;
}

// Workgroups of `kernel` (block threads, no dynamic LDS) resident at once on
// the current device: the grid of a grid-stride kernel beyond this only adds
// dispatch work (its extra waves find nothing to do).
template <typename K>
static inline uint32_t ah_resident_wgs(K kernel, int block) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    return (uint32_t)per_cu * ah_device_cus();
}

static inline uint64_t ah_align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }
// Device table layout inside one buffer: patterns first, then pair records.
static inline uint64_t ah_pat_bytes(uint32_t n_pairs) { return ah_align_up(4ull * n_pairs * sizeof(DPat), 256); }

static inline int ah_bits_for(uint64_t n) {  // bits to represent values 0..n-1
    int b = 0;
    while (b < 64 && (n > (1ull << b))) b++;
    return b;
}

// Fill kernel (graph-safe replacement for memset).
template <typename T>
__global__ void ah_fill_kernel(T *p, T v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
__global__ void ah_set_kernel(T *p, T v) { *p = v; }

template <typename T>
static inline void ah_fill(T *p, T v, uint64_t n, hipStream_t s) {
    if (!n) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(ah_fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

// Device-wide exclusive scan in three launches (block reduce, scan of the
// block sums in one workgroup, block-local scans with carry-in).  The element
// count is read on the device from *d_n (clamped to cap) so the sequence can
// be captured in a graph.  *d_total (optional) receives the sum.
#define AH_SCAN_BLOCKS 1024
template <typename TI, typename TO>
ah_status ah_exclusive_scan(const TI *d_in, TO *d_out, const uint64_t *d_n, uint64_t cap, TO *d_total,
                            TO *d_partials /*[AH_SCAN_BLOCKS]*/, hipStream_t s);

// Single-workgroup exclusive scan of n (host-known) u64 values; writes n+1
// outputs (the last one is the total).
void ah_scan_small_u64(const uint64_t *d_in, uint64_t *d_out, uint64_t n, hipStream_t s);

