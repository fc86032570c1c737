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

// Shaped probe: `INFL` groups loaded per lane before any is used, items of
// `span` groups dealt round-robin; with WRITE each item's 16-bit group words
// are staged in LDS and written as one run after the item.
template <int WRITE, int BLOCK, int INFL>
__global__ __launch_bounds__(BLOCK) void probe_shaped_kernel(const uint4 *__restrict__ in, uint16_t *__restrict__ out,
                                                             int64_t n_items, int span, uint32_t *__restrict__ sink) {
    __shared__ uint16_t stage[WRITE ? 4096 : 4];
    uint32_t acc = 0;
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t base = item * span;
        for (int g0 = threadIdx.x; g0 < span; g0 += INFL * BLOCK) {
            uint4 v[INFL][3];
#pragma unroll
            for (int k = 0; k < INFL; ++k) {
                const int g = g0 + k * BLOCK;
                if (g < span) {
                    const uint4 *q = in + 3 * (base + g);
                    v[k][0] = q[0];
                    v[k][1] = q[1];
                    v[k][2] = q[2];
                }
            }
#pragma unroll
            for (int k = 0; k < INFL; ++k) {
                const int g = g0 + k * BLOCK;
                if (g < span) {
                    const uint32_t x = v[k][0].x ^ v[k][0].y ^ v[k][0].z ^ v[k][0].w ^ v[k][1].x ^ v[k][1].y ^
                                       v[k][1].z ^ v[k][1].w ^ v[k][2].x ^ v[k][2].y ^ v[k][2].z ^ v[k][2].w;
                    if (WRITE) stage[g] = (uint16_t)x;
                    acc ^= x;
                }
            }
        }
        if (WRITE) {
            __syncthreads();
            const uint2 *s2 = reinterpret_cast<const uint2 *>(stage);
            uint2 *o2 = reinterpret_cast<uint2 *>(out + base);
            for (int i = threadIdx.x; i < span / 4; i += BLOCK) o2[i] = s2[i];
            __syncthreads();
        }
    }
    sink[blockIdx.x * BLOCK + threadIdx.x] = acc;
}

// Phased read+write probe: every workgroup reads `phase_items` items (their
// group words staged in LDS), all workgroups meet at a grid-wide counter, then
// every workgroup writes its staged runs, so that reads and writes of the whole
// chip are separated in time.  The wait at the counter is bounded: a
// workgroup that has waited `spin_limit` sleeps goes on without it, so the
// kernel always ends (the bytes written do not depend on the separation).
// Launched cooperatively (every workgroup resident).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void probe_phase_kernel(const uint4 *__restrict__ in, uint16_t *__restrict__ out,
                                                            int64_t n_items, int span, int phase_items,
                                                            uint32_t *__restrict__ sink, uint32_t *counter,
                                                            int spin_limit) {
    extern __shared__ uint16_t pstage[];
    uint32_t acc = 0;
    const int64_t per_round = (int64_t)gridDim.x * phase_items;
    const int64_t rounds = (n_items + per_round - 1) / per_round;
    for (int64_t r = 0; r < rounds; ++r) {
        for (int j = 0; j < phase_items; ++j) {
            const int64_t item = r * per_round + (int64_t)j * gridDim.x + blockIdx.x;
            if (item >= n_items) break;
            const int64_t base = item * span;
            for (int g = threadIdx.x; g < span; g += BLOCK) {
                const uint4 *q = in + 3 * (base + g);
                const uint4 a = q[0], b = q[1], c = q[2];
                const uint32_t x = a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w;
                pstage[j * span + g] = (uint16_t)x;
                acc ^= x;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(counter, 1u);
            const uint32_t target = (uint32_t)((r + 1) * gridDim.x);
            for (int it = 0; it < spin_limit; ++it) {
                if (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __syncthreads();
        for (int j = 0; j < phase_items; ++j) {
            const int64_t item = r * per_round + (int64_t)j * gridDim.x + blockIdx.x;
            if (item >= n_items) break;
            const uint2 *s2 = reinterpret_cast<const uint2 *>(pstage + j * span);
            uint2 *o2 = reinterpret_cast<uint2 *>(out + item * span);
            for (int i = threadIdx.x; i < span / 4; i += BLOCK) o2[i] = s2[i];
        }
        __syncthreads();
    }
    sink[blockIdx.x * BLOCK + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ in, uint4 *__restrict__ out, int64_t n16) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

}  // namespace obg

using namespace obg;

namespace {

template <int WRITE, int BLOCK>
hipError_t launch_shaped(int inflight, int grid, const uint4 *in, uint16_t *out, int64_t n_items, int span,
                         uint32_t *sink, hipStream_t st) {
    switch (inflight) {
        case 1: hipLaunchKernelGGL((probe_shaped_kernel<WRITE, BLOCK, 1>), dim3(grid), dim3(BLOCK), 0, st, in, out, n_items, span, sink); break;
        case 2: hipLaunchKernelGGL((probe_shaped_kernel<WRITE, BLOCK, 2>), dim3(grid), dim3(BLOCK), 0, st, in, out, n_items, span, sink); break;
        default: hipLaunchKernelGGL((probe_shaped_kernel<WRITE, BLOCK, 4>), dim3(grid), dim3(BLOCK), 0, st, in, out, n_items, span, sink); break;
    }
    return hipGetLastError();
}

template <int BLOCK>
hipError_t launch_phased(int grid, const uint4 *in, uint16_t *out, int64_t n_items, int span, int phase_items,
                         uint32_t *sink, uint32_t *counter, hipStream_t st) {
    int spin = 1 << 20;
    void *args[] = {(void *)&in, (void *)&out, (void *)&n_items, (void *)&span, (void *)&phase_items,
                    (void *)&sink, (void *)&counter, (void *)&spin};
    const size_t lds = (size_t)phase_items * span * 2;
    hipError_t e = hipFuncSetAttribute((const void *)probe_phase_kernel<BLOCK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel((const void *)probe_phase_kernel<BLOCK>, dim3(grid), dim3(BLOCK), args, lds, st);
}

}  // namespace

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

extern "C" int obg_probe_shaped(const obg_probe_shape *sh, const void *src, void *dst, int64_t bytes, uint32_t *sink,
                                hipStream_t stream) {
    if (!sh || !src || !sink || bytes <= 0 || (uintptr_t)src % 16 || (dst && (uintptr_t)dst % 16)) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    const bool write = sh->kind == OBG_PROBE_READ_WRITE;
    if (!write && sh->kind != OBG_PROBE_READ) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    if (write && !dst) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    if (sh->grid < 1 || sh->grid > 65536) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    if (sh->block != 256 && sh->block != 512 && sh->block != 1024) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    if (sh->inflight != 1 && sh->inflight != 2 && sh->inflight != 4) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    if (sh->span < 4 || sh->span > 4096 || sh->span % 4) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    if (sh->phase_items < 0 || (sh->phase_items > 0 && (!write || (int64_t)sh->phase_items * sh->span * 2 > 65536)))
        return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    const int64_t n_items = bytes / (48 * (int64_t)sh->span);
    if (n_items < 1) return set_error(OBG_EINVAL, "probe shape or buffers rejected");
    const uint4 *in = (const uint4 *)src;
    uint16_t *out = (uint16_t *)dst;
    hipError_t e;
    if (sh->phase_items > 0) {
        uint32_t *counter = sink + (int64_t)sh->grid * sh->block;
        e = hipMemsetAsync(counter, 0, sizeof(uint32_t), stream);
        if (e == hipSuccess) {
            if (sh->block == 256) e = launch_phased<256>(sh->grid, in, out, n_items, sh->span, sh->phase_items, sink, counter, stream);
            else if (sh->block == 512) e = launch_phased<512>(sh->grid, in, out, n_items, sh->span, sh->phase_items, sink, counter, stream);
            else e = launch_phased<1024>(sh->grid, in, out, n_items, sh->span, sh->phase_items, sink, counter, stream);
        }
    } else if (write) {
        if (sh->block == 256) e = launch_shaped<1, 256>(sh->inflight, sh->grid, in, out, n_items, sh->span, sink, stream);
        else if (sh->block == 512) e = launch_shaped<1, 512>(sh->inflight, sh->grid, in, out, n_items, sh->span, sink, stream);
        else e = launch_shaped<1, 1024>(sh->inflight, sh->grid, in, out, n_items, sh->span, sink, stream);
    } else {
        if (sh->block == 256) e = launch_shaped<0, 256>(sh->inflight, sh->grid, in, out, n_items, sh->span, sink, stream);
        else if (sh->block == 512) e = launch_shaped<0, 512>(sh->inflight, sh->grid, in, out, n_items, sh->span, sink, stream);
        else e = launch_shaped<0, 1024>(sh->inflight, sh->grid, in, out, n_items, sh->span, sink, stream);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(OBG_EHIP, hipGetErrorString(e));
    }
    return OBG_OK;
}
