// strip_core.h -- per-group device code shared by the strip kernels (one
// stream per launch) and the batch kernels (many streams per launch).
#pragma once

#include "internal.h"

namespace obg {

// ---------------------------------------------------------------------------
// LDS <-> HBM bitset conversion (key order in HBM, LDS order on chip)

// lds_from_key(32 kw) for the key words a thread visits in the conversion
// loops below (i = tid, tid + nt, ...; kw = i mod KW).  KW and nt are powers of
// two, so either every kw of a thread is tid mod KW (nt a multiple of KW) or
// kw = tid + u with u a multiple of nt, the same in every lane: the map of
// disjoint bit sets is the OR of their maps, the lane's part is computed once
// and the uniform part in scalar registers.
template <int D, int PAD>
struct KeyWordBase {
    uint32_t lane;    // lds_from_key(32 (tid mod KW))
    int tmod;
    __device__ __forceinline__ KeyWordBase(int tid, int kwords)
        : lane(lds_from_key((uint32_t)(tid % kwords) << 5, D, PAD)), tmod(tid % kwords) {}
    __device__ __forceinline__ uint32_t operator()(int kw) const {
        const uint32_t u = (uint32_t)__builtin_amdgcn_readfirstlane(kw - tmod);
        return lane | lds_from_key(u << 5, D, PAD);
    }
};

// The bits of one key-order word kw are keys 32*kw + b; their LDS indices are
// lds_from_key(32*kw) | lds_from_key(b) because the map permutes index bits.
// From d = 2 on a key word moves as eight nibbles (device.h).
// native: the bitsets in HBM are already in the LDS order (the serving
// runtime's own rings and leaf sets): compact tables copy words as they are,
// wide tables at d = 5 copy word n = G'<<5 | R' to LDS word G'<<8 | R'.
template <int D, int PAD>
__device__ __forceinline__ constexpr bool native_order_ok() { return PAD == LAY_COMPACT || D == 5; }
template <int D, int PAD>
__device__ __forceinline__ int native_word(int n) {
    return PAD == LAY_COMPACT ? n : (((n >> 5) << 8) | (n & 31));
}

template <int D, int PAD, bool DUAL = false>
__device__ __forceinline__ void leaf_to_lds(const uint32_t *__restrict__ leaf, uint32_t *lds,
                                            int n_tiles, int tid, int nt, bool native = false) {
    constexpr int KW = leaf_words(D);
    constexpr int LW = lds_words(D, PAD) * (DUAL ? 2 : 1);   // table words per tile
    constexpr int LC = leaf_count(D);
    constexpr int NB = LC < 32 ? LC : 32;
    const uint32_t valid = LC < 32 ? (1u << (LC & 31)) - 1u : 0xFFFFFFFFu;
    if (native_order_ok<D, PAD>() && native) {
        static_assert(PAD != LAY_COMPACT || lds_words(D, PAD) == KW, "compact tables are key-sized");
        for (int i = tid; i < n_tiles * KW; i += nt) {
            const int c = i / KW;
            const uint32_t w = leaf[i] & valid;
            const int l = c * LW + (DUAL ? 2 : 1) * native_word<D, PAD>(i - c * KW);
            if (DUAL) {
                lds[l] = w;
                lds[l + 1] = 0;
            } else {
                lds[l] = w;
            }
        }
        __syncthreads();
        return;
    }
    for (int i = tid; i < n_tiles * LW; i += nt) lds[i] = 0;
    __syncthreads();
    const KeyWordBase<D, PAD> kbase(tid, KW);
    for (int i = tid; i < n_tiles * KW; i += nt) {
        const int c = i / KW;
        const int kw = i - c * KW;
        uint32_t bits = leaf[i] & valid;
        uint32_t *tile = lds + c * LW;
        if constexpr (D >= 2) {
            // eight nibbles per key word
            const uint32_t lbase = kbase(kw);
            if (bits) key_word_to_table_at<D, PAD, DUAL>(bits, lbase, [&](uint32_t w, uint32_t m) { atomicOr(&tile[w], m); });
        } else {
            if (bits == 0) continue;
            const uint32_t lbase = lds_from_key((uint32_t)kw << 5, D, PAD);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if ((bits >> b) & 1u) {
                    const uint32_t l = lbase | lds_from_key((uint32_t)b, D, PAD);
                    atomicOr(&tile[DUAL ? 2 * (l >> 5) : (l >> 5)], 1u << (l & 31));
                }
            }
        }
    }
    __syncthreads();
}

// Dual tables: clear the occupancy words (the odd ones), keep the leaf words.
__device__ __forceinline__ void clear_dual_occ(uint32_t *lds, int words, int tid, int nt) {
    for (int i = 2 * tid + 1; i < words; i += 2 * nt) lds[i] = 0;
}

// store: every output word belongs to this workgroup alone (one work item per
// segment), so it is written as is; otherwise set bits are OR-ed into words
// other workgroups also write.
template <int D, int PAD, bool DUAL = false>
__device__ __forceinline__ void occ_from_lds(const uint32_t *lds, uint32_t *__restrict__ occ,
                                             int n_tiles, int tid, int nt, bool store = false,
                                             bool native = false) {
    constexpr int KW = leaf_words(D);
    constexpr int LW = lds_words(D, PAD) * (DUAL ? 2 : 1);
    constexpr int LC = leaf_count(D);
    constexpr int NB = LC < 32 ? LC : 32;
    if (native_order_ok<D, PAD>() && native) {
        for (int i = tid; i < n_tiles * KW; i += nt) {
            const int c = i / KW;
            const int l = c * LW + (DUAL ? 2 : 1) * native_word<D, PAD>(i - c * KW);
            const uint32_t w = lds[DUAL ? l + 1 : l];
            if (store)
                occ[i] = w;
            else if (w)
                atomicOr(&occ[i], w);
        }
        return;
    }
    if constexpr (D == 4 && PAD == LAY_COMPACT) {
        // four key words per lane from one read of the four LDS words they
        // share (the region tables: 128 key words per tile)
        constexpr int QW = KW / 4;
        for (int i = tid; i < n_tiles * QW; i += nt) {
            const int c = i / QW;
            const uint32_t q = (uint32_t)(i - c * QW);
            const uint32_t kw0 = (q & 1u) | ((q & 6u) << 1) | ((q & 0x18u) << 2);
            uint32_t out[4];
            key_quad_from_table_d4<DUAL>(lds + c * LW, kw0, out);
            uint32_t *o = occ + (int64_t)c * KW + kw0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int at = 2 * (j & 1) + 16 * (j >> 1);
                if (store)
                    o[at] = out[j];
                else if (out[j])
                    atomicOr(&o[at], out[j]);
            }
        }
        return;
    }
    const KeyWordBase<D, PAD> kbase(tid, KW);
    for (int i = tid; i < n_tiles * KW; i += nt) {
        const int c = i / KW;
        const int kw = i - c * KW;
        const uint32_t *tile = lds + c * LW;
        uint32_t out = 0;
        if constexpr (D >= 2) {
            out = key_word_from_table_at<D, PAD, DUAL>(tile, kbase(kw));
        } else {
            const uint32_t lbase = lds_from_key((uint32_t)kw << 5, D, PAD);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const uint32_t l = lbase | lds_from_key((uint32_t)b, D, PAD);
                out |= ((tile[DUAL ? 2 * (l >> 5) + 1 : (l >> 5)] >> (l & 31)) & 1u) << b;
            }
        }
        if (store)
            occ[i] = out;
        else if (out)
            atomicOr(&occ[i], out);
    }
}

// ---------------------------------------------------------------------------
// Per-group work
//
// Frames are read through a buffer resource per (frame, strip): offsets are
// 32-bit and a read past the end of the frame returns zeros instead of
// faulting, so the partial group at the end of a row and the padding groups
// that only write zero mask bits need no separate load path.

typedef __attribute__((ext_vector_type(4))) unsigned int v4u;
typedef __attribute__((ext_vector_type(2))) unsigned int v2u;



__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// The part of a strip that a work item walks.  With several regions per
// strip, a strip may be cut into chunks of whole region columns, so that a
// workgroup holds the tables of fewer regions and one frame still gives many
// work items; group g of a chunk is row g / cw, column gx0 + g % cw.
struct Chunk {
    FastDiv div;      // divides by cw
    uint32_t cw;      // groups per row of the chunk (a multiple of 4)
    uint32_t gx0;     // the chunk's first group column (a multiple of 4)
    int32_t c0;       // the chunk's first region column
    int32_t tiles;    // region columns in the chunk
};

// Issue the three 16-byte loads of group g (16 pixels = 48 bytes).
template <bool REGION>
__device__ __forceinline__ void fetch_group(__amdgpu_buffer_rsrc_t rs, const StripArgs &a, const Chunk &ch,
                                            int g, uint32_t (&u)[12], uint32_t &yr, uint32_t &gx) {
    if (REGION) {
        yr = fdiv((uint32_t)g, ch.div);
        gx = (uint32_t)g - yr * ch.cw + ch.gx0;
    } else {
        yr = fdiv((uint32_t)g, a.div_gpr);
        gx = (uint32_t)g - yr * (uint32_t)a.gpr;
    }
    const uint32_t off = yr * (uint32_t)a.row_pitch + 48u * gx;
    const v4u v0 = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    const v4u v1 = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0));
    const v4u v2 = __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 32, 0, 0));
    u[0] = v0.x; u[1] = v0.y; u[2] = v0.z; u[3] = v0.w;
    u[4] = v1.x; u[5] = v1.y; u[6] = v1.z; u[7] = v1.w;
    u[8] = v2.x; u[9] = v2.y; u[10] = v2.z; u[11] = v2.w;
}

template <int D, int MODE, int PAD, bool GUARD>
__device__ __forceinline__ uint32_t group_pixels(const uint32_t (&u)[12], int nvalid,
                                                 const uint32_t *leaf_tile, uint32_t *occ_tile,
                                                 uint32_t *__restrict__ cnt, bool occ_test) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr bool OCC = (MODE & MODE_OCC) != 0;
    constexpr bool CNT = (MODE & MODE_COUNTS) != 0;
    uint32_t present = 0;
    if constexpr (MASK && OCC && !CNT) {
        // dual table (leaf_tile == occ_tile): one 8-byte read gives the
        // pixel's leaf word and occupancy word; the occupancy bit is set with
        // an atomic OR only where the word lacks it (the look is free here,
        // so occ_test does not apply)
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            uint32_t addr, bit;
            lds_pos<D, PAD>(u, p, addr, bit);
            const uint2 v = *reinterpret_cast<const uint2 *>(reinterpret_cast<const char *>(occ_tile) + 2 * addr);
            const uint32_t m = 1u << (bit & 31);
            present |= ((v.x >> (bit & 31)) & 1u) << p;
            if ((!GUARD || p < nvalid) && !(v.y & m))
                atomicOr(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(occ_tile) + 2 * addr + 4), m);
        }
        return present;
    }
    uint32_t run_l = 0xFFFFFFFFu, run_n = 0;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        uint32_t addr, bit;
        lds_pos<D, PAD>(u, p, addr, bit);
        // mask bits of pixels past the row end are cleared by the caller
        if (MASK) {
            const uint32_t w = *reinterpret_cast<const uint32_t *>(
                reinterpret_cast<const char *>(leaf_tile) + addr);
            present |= ((w >> (bit & 31)) & 1u) << p;
        }
        if ((OCC || CNT) && (!GUARD || p < nvalid)) {
            if (OCC) {
                uint32_t *w = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(occ_tile) + addr);
                if (!occ_test || !((*w >> (bit & 31)) & 1u)) atomicOr(w, 1u << (bit & 31));
            }
            if (CNT) {
                const uint32_t l = (addr << 3) | (bit & 31);
                if (l == run_l) {
                    ++run_n;
                } else {
                    if (run_n) atomicAdd(&cnt[key_from_lds(run_l, D, PAD)], run_n);
                    run_l = l;
                    run_n = 1;
                }
            }
        }
    }
    if (CNT && run_n) atomicAdd(&cnt[key_from_lds(run_l, D, PAD)], run_n);
    return present;
}

template <int D, int MODE, int PAD, bool REGION>
__device__ __forceinline__ void consume_group(const StripArgs &a, const Chunk &ch, __amdgpu_buffer_rsrc_t ms,
                                              const uint32_t (&u)[12], uint32_t yr, uint32_t gx,
                                              const uint32_t *leaf_lds, uint32_t *occ_lds,
                                              uint32_t *__restrict__ cbase, uint16_t *stage, int gl) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr bool CNT = (MODE & MODE_COUNTS) != 0;
    constexpr int LW = lds_words(D, PAD);
    constexpr int LC = leaf_count(D);
    int nv = a.width - (int)gx * 16;
    nv = nv < 0 ? 0 : (nv > 16 ? 16 : nv);
    int c = 0;
    if (REGION) {
        c = (int)fdiv(gx, a.div_tile) - ch.c0;
        c = c < ch.tiles ? c : ch.tiles - 1;        // padding groups: result discarded
    }
    // fused passes keep one dual table per tile (leaf_lds == occ_lds)
    constexpr int TW = ((MODE & MODE_MASK) && (MODE & MODE_OCC) && !CNT) ? 2 * LW : LW;
    const uint32_t *leaf_tile = leaf_lds + c * TW;
    uint32_t *occ_tile = occ_lds + c * TW;
    uint32_t *cnt = CNT ? cbase + (int64_t)c * LC : nullptr;
    uint32_t present;
    if (nv == 16)
        present = group_pixels<D, MODE, PAD, false>(u, 16, leaf_tile, occ_tile, cnt, a.occ_test != 0);
    else
        present = group_pixels<D, MODE, PAD, true>(u, nv, leaf_tile, occ_tile, cnt, a.occ_test != 0);
    if (MASK) {
        // Four consecutive lanes hold the four 16-pixel groups of one 64-pixel
        // mask word (work spans and rows are multiples of 4 groups): gather
        // them with quad permutes and let the first lane of the quad write the
        // whole aligned 64-bit word.
        const uint32_t valid = 0xFFFFu >> (16 - nv);
        const uint32_t m16 = ~present & valid;
        if (stage) {
            // the item's mask bytes are written out together at its end
            stage[gl] = (uint16_t)m16;
            return;
        }
        const uint32_t n1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m16, 0x39, 0xF, 0xF, false);
        const uint32_t n2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m16, 0x4E, 0xF, 0xF, false);
        const uint32_t n3 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m16, 0x93, 0xF, 0xF, false);
        if ((threadIdx.x & 3) == 0) {
            const uint32_t off = yr * (uint32_t)a.mask_row_words * 8u + 2u * gx;
            const uint32_t lo = m16 | (n1 << 16), hi = n2 | (n3 << 16);
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, make_uint2(lo, hi)), ms, off, 0, 0);
        }
    }
}

// The groups [gb, ge) of one (frame, strip): two groups in flight per lane
// (the next group's loads are issued before the current one is worked on);
// with `stage`, the span's mask is gathered in LDS and written as one run.
// Without regions `ch` is not read (the strip is whole rows).
template <int D, int MODE, int PAD, bool REGION, int BLOCK>
__device__ __forceinline__ void span_loop(const StripArgs &a, __amdgpu_buffer_rsrc_t rs,
                                          __amdgpu_buffer_rsrc_t ms, int gb, int ge,
                                          const uint32_t *leaf_lds, uint32_t *occ_lds,
                                          uint32_t *__restrict__ cbase, uint16_t *stage,
                                          const Chunk &ch = Chunk{}) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    const int tid = threadIdx.x;
    uint32_t ua[12], ub[12], ya = 0, xa = 0, yb = 0, xb = 0;
    int g = gb + tid;
    if (g < ge) fetch_group<REGION>(rs, a, ch, g, ua, ya, xa);
    for (; g < ge; g += 2 * BLOCK) {
        const int g1 = g + BLOCK;
        if (g1 < ge) fetch_group<REGION>(rs, a, ch, g1, ub, yb, xb);
        consume_group<D, MODE, PAD, REGION>(a, ch, ms, ua, ya, xa, leaf_lds, occ_lds, cbase, stage, g - gb);
        const int g2 = g + 2 * BLOCK;
        if (g2 < ge) fetch_group<REGION>(rs, a, ch, g2, ua, ya, xa);
        if (g1 < ge)
            consume_group<D, MODE, PAD, REGION>(a, ch, ms, ub, yb, xb, leaf_lds, occ_lds, cbase, stage, g1 - gb);
    }
    if (MASK && stage) {
        // group g's 16 mask bits are bytes 2g, 2g+1 of the strip's mask, so
        // the span's mask is one contiguous run: write it in 8-byte words
        __syncthreads();
        const int n8 = (ge - gb) >> 2;
        const uint2 *src = reinterpret_cast<const uint2 *>(stage);
        for (int i = tid; i < n8; i += BLOCK)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, src[i]), ms,
                                                  2u * (uint32_t)gb + 8u * (uint32_t)i, 0, 0);
        __syncthreads();
    }
}

// Algorithm 2 in closed form, 32 keys to a word: per key, the number of the
// window's trees that hold it, in bit-sliced counters (plane b holds bit b of
// the 32 counts), compared bit-sliced with kmin.  With group > 1 the window's
// trees are taken in groups of `group` consecutive slots (the last may be
// shorter) and each group counts once, as the OR of its trees (the tree of a
// group of frames, Section 3); n_trees is the window length in slots.
constexpr int kMergeWaves = 4;      // waves of a merge workgroup: 64 words x 4 parts of the window
constexpr int kMergeBlock = 64 * kMergeWaves;
constexpr int64_t kMergeWholeWords = 1 << 19;   // merges of at least this many words: one thread per word

// Add into c the trees (or groups) j = j0, j0 + step, ... of the window for
// word i.  Sixteen loads per round, independent and in flight together.
__device__ __forceinline__ void merge_count(uint32_t (&c)[16], const uint32_t *__restrict__ ring, int ring_len,
                                            int first, int n_trees, int64_t slot_words, int64_t i, uint32_t valid,
                                            int planes, int group, int j0, int step) {
    const int n_groups = (n_trees + group - 1) / group;
    for (int j = j0; j < n_groups; j += 16 * step) {
        uint32_t x[16];
        if (group == 1) {
            // straight-line loads: none waits for another
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int t = j + k * step;
                int sl = first + t;
                if (sl >= ring_len) sl -= ring_len;
                x[k] = t < n_trees ? ring[(int64_t)sl * slot_words + i] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] &= valid;
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                x[k] = 0;
                const int jj = j + k * step;
                if (jj < n_groups) {
                    const int tb = jj * group, te = min(tb + group, n_trees);
                    for (int t = tb; t < te; ++t) {
                        int sl = first + t;
                        if (sl >= ring_len) sl -= ring_len;
                        x[k] |= ring[(int64_t)sl * slot_words + i];
                    }
                    x[k] &= valid;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            uint32_t carry = x[k];
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                if (b < planes) {
                    const uint32_t tmp = c[b] & carry;
                    c[b] ^= carry;
                    carry = tmp;
                }
            }
        }
    }
}

// Words of one merge by a workgroup of kMergeBlock threads (the call is
// workgroup-uniform).  SPLIT = 4: words w0 .. w0+63; wave q counts the
// window's trees j = q, q + 4, ... for the 64 words, the four partial counts
// meet in LDS (`part`, 3 x 16 x 64 words) and the first wave adds them
// bit-sliced, compares with kmin and writes leaf[w0 .. w0+63] (words below
// `words` only).  SPLIT = 1: words w0 .. w0+255, one thread per word over the
// whole window (large merges: enough words to fill the chip without
// splitting the window, and no partial counts to meet).
template <int SPLIT = kMergeWaves>
__device__ __forceinline__ void merge_block(const uint32_t *__restrict__ ring, int ring_len, int first, int n_trees,
                                            int64_t slot_words, int64_t words, int64_t w0, int valid_bits,
                                            uint32_t kmin, int planes, int empty, int group,
                                            uint32_t *__restrict__ leaf, uint32_t *part) {
    static_assert(SPLIT == 1 || SPLIT == kMergeWaves, "a window is counted whole or in four parts");
    const int lane = threadIdx.x & 63, q = SPLIT == 1 ? 0 : (int)(threadIdx.x >> 6);
    const int64_t i = w0 + (SPLIT == 1 ? (int64_t)threadIdx.x : (int64_t)lane);
    const uint32_t valid = valid_bits >= 32 ? 0xFFFFFFFFu : ((1u << valid_bits) - 1u);
    if (empty) {
        if (q == 0 && i < words) leaf[i] = 0;
        return;
    }
    uint32_t c[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) c[b] = 0;
    if (i < words) merge_count(c, ring, ring_len, first, n_trees, slot_words, i, valid, planes, group, q, SPLIT);
    if (SPLIT > 1) {
        if (q > 0) {
#pragma unroll
            for (int b = 0; b < 16; ++b)
                if (b < planes) part[((q - 1) * 16 + b) * 64 + lane] = c[b];
        }
        __syncthreads();
        if (q != 0) return;
    }
#pragma unroll
    for (int r = 0; r < SPLIT - 1; ++r) {
        // c += part r, bit-sliced ripple carry (the sum of all counts fits in
        // `planes` bits: it is at most the window's number of trees, or of
        // groups)
        uint32_t carry = 0;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            if (b < planes) {
                const uint32_t x = part[(r * 16 + b) * 64 + lane], y = c[b];
                c[b] = x ^ y ^ carry;
                carry = (x & y) | (carry & (x ^ y));
            }
        }
    }
    uint32_t ge = 0, eq = 0xFFFFFFFFu;
#pragma unroll
    for (int b = 15; b >= 0; --b) {
        if ((kmin >> b) & 1u) {
            eq &= c[b];
        } else {
            ge |= eq & c[b];
            eq &= ~c[b];
        }
    }
    ge |= eq;
    if (i < words) leaf[i] = ge & valid;
}

}  // namespace obg
