// device.h -- layouts and per-pixel helpers of the gfx950 kernels.
//
// Two index orders of the 8^d depth-d octree nodes are used:
//
//   path key K  (exported): the child indices c_0..c_{d-1} of Algorithm 1 as
//               base-8 digits, c_0 most significant, c_i = 4r_i + 2g_i + b_i
//               with r_i = bit 7-i of R.  In bits: bit 3m+2 of K is bit m of
//               R' = R >> (8-d), bit 3m+1 is bit m of G', bit 3m is bit m of B'.
//   concat J    (LDS only):  J = R' << 2d | G' << d | B'.
//
// J is what a pixel's bytes give with three bit-field extracts and two
// shift-or operations; K would need a bit interleave per pixel.  Both orders
// hold the same set (the map between them is a fixed permutation of the 3d
// index bits), so bitsets are converted when they enter or leave LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace obg {

__host__ __device__ constexpr int leaf_count(int d) { return 1 << (3 * d); }
__host__ __device__ constexpr int leaf_words(int d) { return d >= 2 ? (1 << (3 * d - 5)) : 1; }

// K -> J and J -> K; both are permutations of the index bits.
__host__ __device__ constexpr uint32_t concat_from_key(uint32_t k, int d) {
    uint32_t j = 0;
    for (int m = 0; m < d; ++m) {
        j |= ((k >> (3 * m + 2)) & 1u) << (2 * d + m);
        j |= ((k >> (3 * m + 1)) & 1u) << (d + m);
        j |= ((k >> (3 * m)) & 1u) << m;
    }
    return j;
}

__host__ __device__ constexpr uint32_t key_from_concat(uint32_t j, int d) {
    uint32_t k = 0;
    for (int m = 0; m < d; ++m) {
        k |= ((j >> (2 * d + m)) & 1u) << (3 * m + 2);
        k |= ((j >> (d + m)) & 1u) << (3 * m + 1);
        k |= ((j >> m) & 1u) << (3 * m);
    }
    return k;
}

// Exact unsigned division by a runtime-invariant divisor with one high
// multiply (Granlund & Montgomery, PLDI 1994, unsigned case, N = 32).
struct FastDiv {
    uint32_t m, s1, s2, d;
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f{};
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;                       // l = ceil(log2 d)
    f.m = (uint32_t)(((((1ull << l) - d) << 32) / d) + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    f.d = d;
    return f;
}

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
    uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Concat index of pixel p (0..15) of a 16-pixel group held as 12 dwords.
template <int D>
__device__ __forceinline__ uint32_t concat_index(const uint32_t (&u)[12], int p) {
    constexpr int S = 8 - D;
    const int br = 3 * p, bg = 3 * p + 1, bb = 3 * p + 2;
    const uint32_t R = __builtin_amdgcn_ubfe(u[br >> 2], (br & 3) * 8 + S, D);
    const uint32_t G = __builtin_amdgcn_ubfe(u[bg >> 2], (bg & 3) * 8 + S, D);
    const uint32_t B = __builtin_amdgcn_ubfe(u[bb >> 2], (bb & 3) * 8 + S, D);
    return (R << (2 * D)) | (G << D) | B;
}

// Path key of one pixel from its bytes (generic kernels).
__device__ __forceinline__ uint32_t path_key(uint32_t r, uint32_t g, uint32_t b, int d) {
    uint32_t k = 0;
    for (int i = 0; i < d; ++i) {
        const int bit = 7 - i;
        k = (k << 3) | (((r >> bit) & 1u) << 2) | (((g >> bit) & 1u) << 1) | ((b >> bit) & 1u);
    }
    return k;
}

}  // namespace obg
