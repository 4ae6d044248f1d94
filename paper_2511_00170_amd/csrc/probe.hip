// Read-only stream over a device buffer: the HBM read bandwidth a plain
// reading kernel reaches, the ceiling the scan's bandwidth is compared with.
// 128-bit loads, four in flight per lane, a persistent grid; the words are
// XOR-folded into one value per workgroup so the loads cannot be dropped.
#include <hip/hip_runtime.h>

#include "ah.h"
#include "ah_internal.h"

__global__ void __launch_bounds__(256) ah_read_probe_kernel(const uint4 *p, uint64_t n, uint32_t *out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n; i += stride) {
        const uint4 a = p[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    __shared__ uint32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

extern "C" ah_status ah_read_probe(const void *d_buf, uint64_t bytes, uint32_t *d_out, uint32_t out_n,
                                   void *stream) {
    if (!d_buf || !d_out || !out_n || bytes % 16) return AH_E_ARG;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return AH_E_HIP;
    uint32_t grid = (uint32_t)cus * 8u;
    if (grid > out_n) grid = out_n;
    hipLaunchKernelGGL(ah_read_probe_kernel, dim3(grid), dim3(256), 0, ah_stream(stream), (const uint4 *)d_buf,
                       bytes / 16, d_out);
    return hipGetLastError() == hipSuccess ? AH_OK : AH_E_HIP;
}
