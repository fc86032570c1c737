// probe.hip -- streaming kernels that measure what the memory system delivers
// (read-only, copy, and reads with 1/24 as many bytes written back in runs),
// so that the pixel kernels can be compared with an achievable ceiling and
// the HBM traffic counters can be scaled against a copy of known size.
#include "../../include/obg.h"
#include "internal.h"

namespace obg {

// Each lane reads 48 contiguous bytes per step (the pixel kernels' pattern).
template <int WRITE>
__global__ __launch_bounds__(512) void probe_kernel(const uint4 *__restrict__ in, uint16_t *__restrict__ out,
                                                    int64_t n_items, int span, uint32_t *__restrict__ sink) {
    __shared__ uint16_t stage[1024];
    uint32_t acc = 0;
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t base = item * span;
        for (int g = threadIdx.x; g < span; g += blockDim.x) {
            const uint4 *q = in + 3 * (base + g);
            const uint4 a = q[0], b = q[1], c = q[2];
            const uint32_t x = a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w;
            if (WRITE) stage[g] = (uint16_t)x;
            acc ^= x;
        }
        if (WRITE) {
            __syncthreads();
            const uint2 *s2 = reinterpret_cast<const uint2 *>(stage);
            uint2 *o2 = reinterpret_cast<uint2 *>(out + base);
            for (int i = threadIdx.x; i < span / 4; i += blockDim.x) o2[i] = s2[i];
            __syncthreads();
        }
    }
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ in, uint4 *__restrict__ out, int64_t n16) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

}  // namespace obg

using namespace obg;

extern "C" int obg_probe(int kind, const void *src, void *dst, int64_t bytes, uint32_t *sink,
                         int32_t grid, hipStream_t stream) {
    if (!src || bytes <= 0 || (uintptr_t)src % 16 || (dst && (uintptr_t)dst % 16)) return OBG_EINVAL;
    if (kind == OBG_PROBE_COPY) {
        if (!dst || bytes % 16) return OBG_EINVAL;
        hipLaunchKernelGGL(copy_kernel, dim3(4096), dim3(256), 0, stream, (const uint4 *)src, (uint4 *)dst,
                           bytes / 16);
        return hipGetLastError() == hipSuccess ? OBG_OK : OBG_EHIP;
    }
    if (kind != OBG_PROBE_READ && kind != OBG_PROBE_READ_WRITE) return OBG_EINVAL;
    if (!sink || grid < 1 || grid > 65536) return OBG_EINVAL;
    const int span = 832;   // groups per item: the classify default
    const int64_t n_items = bytes / (48 * (int64_t)span);
    if (n_items < 1) return OBG_EINVAL;
    if (kind == OBG_PROBE_READ_WRITE) {
        if (!dst) return OBG_EINVAL;
        hipLaunchKernelGGL(probe_kernel<1>, dim3(grid), dim3(512), 0, stream, (const uint4 *)src, (uint16_t *)dst,
                           n_items, span, sink);
    } else {
        hipLaunchKernelGGL(probe_kernel<0>, dim3(grid), dim3(512), 0, stream, (const uint4 *)src, (uint16_t *)dst,
                           n_items, span, sink);
    }
    return hipGetLastError() == hipSuccess ? OBG_OK : OBG_EHIP;
}
