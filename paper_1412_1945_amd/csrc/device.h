// device.h -- layouts and per-pixel helpers of the gfx950 kernels.
//
// Two index orders of the 8^d depth-d octree nodes are used:
//
//   path key K  (exported): the child indices c_0..c_{d-1} of Algorithm 1 as
//               base-8 digits, c_0 most significant, c_i = 4r_i + 2g_i + b_i
//               with r_i = bit 7-i of R.  In bits: bit 3m+2 of K is bit m of
//               R' = R >> (8-d), bit 3m+1 is bit m of G', bit 3m is bit m of B'.
//   LDS index L (on chip): bit (L & 31) of 32-bit LDS word (L >> 5), in one
//               of two orders:
//     LAY_COMPACT  L = R' << 2d | G' << d | B'            (8^d bits)
//     LAY_WIDE     L = G' << 13 | R' << 5 | B'   (d <= 5; a sparse table)
//               The wide order follows the bytes of a pixel: the LDS byte
//               address 4 * (G' << 8 | R') is the R,G byte pair of the pixel
//               shifted and masked in one go, and B' is the bit.
//
// L comes from a pixel's bytes with a few shifts and masks; K would need a
// bit interleave per pixel.  The map between K and L permutes index bits
// (with zero gaps in the wide order), so bitsets are converted when they
// enter or leave LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace obg {

enum { LAY_COMPACT = 0, LAY_WIDE = 1 };

__host__ __device__ constexpr int leaf_count(int d) { return 1 << (3 * d); }
__host__ __device__ constexpr int leaf_words(int d) { return d >= 2 ? (1 << (3 * d - 5)) : 1; }

// 32-bit LDS words of one tree in an LDS order
__host__ __device__ constexpr int lds_words(int d, int lay) {
    return lay == LAY_WIDE ? ((((1 << d) - 1) << 8) | ((1 << d) - 1)) + 1
                           : (d >= 2 ? (1 << (3 * d - 5)) : 1);
}

__host__ __device__ constexpr uint32_t lds_from_key(uint32_t k, int d, int lay) {
    uint32_t r = 0, g = 0, b = 0;
    for (int m = 0; m < d; ++m) {
        r |= ((k >> (3 * m + 2)) & 1u) << m;
        g |= ((k >> (3 * m + 1)) & 1u) << m;
        b |= ((k >> (3 * m)) & 1u) << m;
    }
    return lay == LAY_WIDE ? ((g << 13) | (r << 5) | b) : ((((r << d) | g) << d) | b);
}

__host__ __device__ constexpr uint32_t key_from_lds(uint32_t l, int d, int lay) {
    const uint32_t msk = (1u << d) - 1u;
    const uint32_t b = l & msk;
    const uint32_t r = lay == LAY_WIDE ? (l >> 5) & msk : (l >> (2 * d)) & msk;
    const uint32_t g = lay == LAY_WIDE ? (l >> 13) & msk : (l >> d) & msk;
    uint32_t k = 0;
    for (int m = 0; m < d; ++m) {
        k |= ((r >> m) & 1u) << (3 * m + 2);
        k |= ((g >> m) & 1u) << (3 * m + 1);
        k |= ((b >> m) & 1u) << (3 * m);
    }
    return k;
}

// Whole key words <-> LDS words (d >= 2).  The 32 keys of key word kw vary in
// key bits 0..4 = B'0, G'0, R'0, B'1, G'1.  In both LDS orders B'0 and B'1 are
// LDS index bits 0 and 1, so for each of the 8 values q of (G'0, R'0, G'1) the
// four keys that differ in B'0, B'1 are one aligned nibble of one LDS word.
// That nibble sits at LDS index lds_from_key(32 kw) | nib_lds(q) (the two
// parts have disjoint bits), and its bits (B'1 B'0 = 0..3) are the key-word
// bits nib_key(q) + {0, 1, 8, 9}.
template <int D, int LAY>
__host__ __device__ constexpr uint32_t nib_lds(int q) {
    return lds_from_key((uint32_t)(((q >> 2) << 4) | (((q >> 1) & 1) << 2) | ((q & 1) << 1)), D, LAY);
}
__host__ __device__ constexpr int nib_key(int q) { return 2 * (q & 1) + 4 * ((q >> 1) & 1) + 16 * (q >> 2); }
__host__ __device__ inline uint32_t nib_spread(uint32_t n) { return (n & 3u) | ((n & 0xCu) << 6); }
__host__ __device__ inline uint32_t nib_pick(uint32_t w, int off) {
    return ((w >> off) & 3u) | (((w >> (off + 8)) & 3u) << 2);
}

// Dual tables (the fused classify + occupancy pass): one table holds both
// bitsets of a tree in word pairs, word 2w the merged leaf set's word w and
// word 2w + 1 the frame's occupancy word w, so that one 8-byte LDS read gives
// a pixel both bits.

// Key word kw of one tree's LDS table (gather of 8 nibbles); DUAL: the
// occupancy words of a dual table.  lbase = lds_from_key(32 kw).
template <int D, int LAY, bool DUAL = false>
__host__ __device__ inline uint32_t key_word_from_table_at(const uint32_t *tab, uint32_t lbase) {
    static_assert(D >= 2, "a key word holds at least 32 keys from d = 2 on");
    uint32_t out = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t nl = nib_lds<D, LAY>(q);
        const uint32_t w = (lbase >> 5) + (nl >> 5);
        const uint32_t n = (tab[DUAL ? 2 * w + 1 : w] >> ((lbase & 31u) + (nl & 31u))) & 0xFu;
        out |= nib_spread(n) << nib_key(q);
    }
    return out;
}
template <int D, int LAY, bool DUAL = false>
__host__ __device__ inline uint32_t key_word_from_table(const uint32_t *tab, uint32_t kw) {
    return key_word_from_table_at<D, LAY, DUAL>(tab, lds_from_key(kw << 5, D, LAY));
}

// Key word kw with bits `bits` into one tree's LDS table: or_into(word, mask)
// is called for each non-empty nibble (8 at most); DUAL: into the leaf words
// of a dual table.
template <int D, int LAY, bool DUAL = false, typename OrInto>
__host__ __device__ inline void key_word_to_table_at(uint32_t bits, uint32_t lbase, OrInto or_into) {
    static_assert(D >= 2, "a key word holds at least 32 keys from d = 2 on");
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t n = nib_pick(bits, nib_key(q));
        const uint32_t nl = nib_lds<D, LAY>(q);
        const uint32_t w = (lbase >> 5) + (nl >> 5);
        if (n) or_into(DUAL ? 2 * w : w, n << ((lbase & 31u) + (nl & 31u)));
    }
}
template <int D, int LAY, bool DUAL = false, typename OrInto>
__host__ __device__ inline void key_word_to_table(uint32_t bits, uint32_t kw, OrInto or_into) {
    key_word_to_table_at<D, LAY, DUAL>(bits, lds_from_key(kw << 5, D, LAY), or_into);
}

// d = 4 in the compact order, four key words at once: the key words kw0 +
// {0, 2, 16, 18} (kw0 with bits 1 and 4 clear) differ only in B'2 and B'3,
// which are bits 2 and 3 of an LDS bit index, so they come from the same four
// LDS words (G'1 and R'0 vary: word offsets 0, 1, 8, 9).  Each of those words
// holds, for key word j (j = B'2 + 2 B'3), the nibble of G'0 = 0 at bit 4j and
// that of G'0 = 1 at bit 16 + 4j.  DUAL: the occupancy words of a dual table.
template <bool DUAL = false>
__host__ __device__ inline void key_quad_from_table_d4(const uint32_t *tab, uint32_t kw0, uint32_t (&out)[4]) {
    const uint32_t w0 = lds_from_key(kw0 << 5, 4, LAY_COMPACT) >> 5;
    uint32_t wd[4];   // index G'1 + 2 R'0
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint32_t w = w0 + (uint32_t)(m & 1) + 8u * (uint32_t)(m >> 1);
        wd[m] = tab[DUAL ? 2 * w + 1 : w];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int g0 = 0; g0 < 2; ++g0)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t n = (wd[m] >> (16 * g0 + 4 * j)) & 0xFu;
                out[j] |= nib_spread(n) << (16 * (m & 1) + 4 * (m >> 1) + 2 * g0);
            }
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

// LDS byte address (within one tree's table) and bit of pixel p (0..15) of a
// 16-pixel group held as 12 dwords.  Only the low 5 bits of `bit` count.
template <int D, int LAY>
__device__ __forceinline__ void lds_pos(const uint32_t (&u)[12], int p, uint32_t &addr, uint32_t &bit) {
    constexpr int S = 8 - D;
    const int br = 3 * p, bb = 3 * p + 2;
    if (LAY == LAY_WIDE) {
        static_assert(LAY != LAY_WIDE || D <= 5, "wide order needs d <= 5");
        // R byte then G byte, shifted so that R' lands at bit 2 and G' at bit 10
        const int k = br >> 2, o = br & 3;
        uint32_t rg;
        if (o < 3)
            rg = u[k] >> (8 * o + 6 - D);
        else
            rg = __builtin_amdgcn_alignbit(u[k + 1], u[k], 30 - D);
        constexpr uint32_t M = (((1u << D) - 1u) << 2) | (((1u << D) - 1u) << 10);
        addr = rg & M;
        bit = (D == 5) ? (u[bb >> 2] >> ((bb & 3) * 8 + S))
                       : __builtin_amdgcn_ubfe(u[bb >> 2], (bb & 3) * 8 + S, D);
    } else {
        const int bg = 3 * p + 1;
        const uint32_t R = __builtin_amdgcn_ubfe(u[br >> 2], (br & 3) * 8 + S, D);
        const uint32_t G = __builtin_amdgcn_ubfe(u[bg >> 2], (bg & 3) * 8 + S, D);
        const uint32_t B = __builtin_amdgcn_ubfe(u[bb >> 2], (bb & 3) * 8 + S, D);
        const uint32_t l = (((R << D) | G) << D) | B;
        addr = (l >> 5) << 2;
        bit = l;
    }
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
