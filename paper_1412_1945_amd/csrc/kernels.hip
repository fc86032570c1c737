// kernels.hip -- gfx950 kernels of octree background modelling.
//
// strip_kernel  one pass over 16-pixel groups (48 contiguous bytes = three
//               16-byte loads per lane).  Per pixel: three bit-field extracts
//               give the top d bits of R, G, B (the depth-d node of the
//               pixel's octree path, Algorithm 1 with the pruning of
//               Section 2), two shift-ors give its LDS index, then
//                 MASK   test the bit in the merged leaf set (Algorithm 3),
//                        16 results per lane packed into one 16-bit store;
//                 OCC    set the bit in this frame's LDS occupancy bitset
//                        (test first, atomic OR only when unset); the bitset
//                        is OR-ed into HBM once per (frame, strip) segment;
//                 COUNTS add the pixel to the key's counter (runs of equal
//                        keys inside a lane are added with one atomic).
// generic_kernel per-pixel fallback for d = 7, 8 and region widths that are
//               not a multiple of 16 pixels; bitsets stay in HBM/L2.
// merge_kernel  per 32 keys: bit-sliced counters of the window's bitsets and
//               a bit-sliced compare against the frame-count threshold
//               (Algorithm 2 in closed form).
#include "internal.h"

namespace obg {

// ---------------------------------------------------------------------------
// LDS <-> HBM bitset conversion (key order in HBM, LDS order on chip)

// The bits of one key-order word kw are keys 32*kw + b; their LDS indices are
// lds_from_key(32*kw) | lds_from_key(b) because the map permutes index bits.
template <int D, int PAD>
__device__ __forceinline__ void leaf_to_lds(const uint32_t *__restrict__ leaf, uint32_t *lds,
                                            int n_tiles, int tid, int nt) {
    constexpr int KW = leaf_words(D);
    constexpr int LW = lds_words(D, PAD);
    constexpr int LC = leaf_count(D);
    constexpr int NB = LC < 32 ? LC : 32;
    for (int i = tid; i < n_tiles * LW; i += nt) lds[i] = 0;
    __syncthreads();
    for (int i = tid; i < n_tiles * KW; i += nt) {
        const int c = i / KW;
        const int kw = i - c * KW;
        uint32_t bits = leaf[i];
        if (LC < 32) bits &= (1u << (LC & 31)) - 1u;
        if (bits == 0) continue;
        const uint32_t lbase = lds_from_key((uint32_t)kw << 5, D, PAD);
        uint32_t *tile = lds + c * LW;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if ((bits >> b) & 1u) {
                const uint32_t l = lbase | lds_from_key((uint32_t)b, D, PAD);
                atomicOr(&tile[l >> 5], 1u << (l & 31));
            }
        }
    }
    __syncthreads();
}

template <int D, int PAD>
__device__ __forceinline__ void occ_from_lds(const uint32_t *lds, uint32_t *__restrict__ occ,
                                             int n_tiles, int tid, int nt) {
    constexpr int KW = leaf_words(D);
    constexpr int LW = lds_words(D, PAD);
    constexpr int LC = leaf_count(D);
    constexpr int NB = LC < 32 ? LC : 32;
    for (int i = tid; i < n_tiles * KW; i += nt) {
        const int c = i / KW;
        const int kw = i - c * KW;
        const uint32_t lbase = lds_from_key((uint32_t)kw << 5, D, PAD);
        const uint32_t *tile = lds + c * LW;
        uint32_t out = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint32_t l = lbase | lds_from_key((uint32_t)b, D, PAD);
            out |= ((tile[l >> 5] >> (l & 31)) & 1u) << b;
        }
        if (out) atomicOr(&occ[i], out);
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

constexpr int kStageGroups = 1024;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// Issue the three 16-byte loads of group g (16 pixels = 48 bytes).
__device__ __forceinline__ void fetch_group(__amdgpu_buffer_rsrc_t rs, const StripArgs &a, int g,
                                            uint32_t (&u)[12], uint32_t &yr, uint32_t &gx) {
    yr = fdiv((uint32_t)g, a.div_gpr);
    gx = (uint32_t)g - yr * (uint32_t)a.gpr;
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
                                                 uint32_t *__restrict__ cnt) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr bool OCC = (MODE & MODE_OCC) != 0;
    constexpr bool CNT = (MODE & MODE_COUNTS) != 0;
    uint32_t present = 0;
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
            if (OCC) atomicOr(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(occ_tile) + addr),
                              1u << (bit & 31));
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
__device__ __forceinline__ void consume_group(const StripArgs &a, __amdgpu_buffer_rsrc_t ms,
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
        c = (int)fdiv(gx, a.div_tile);
        c = c < a.reg_cols ? c : a.reg_cols - 1;     // padding groups: result discarded
    }
    const uint32_t *leaf_tile = leaf_lds + c * LW;
    uint32_t *occ_tile = occ_lds + c * LW;
    uint32_t *cnt = CNT ? cbase + (int64_t)c * LC : nullptr;
    uint32_t present;
    if (nv == 16)
        present = group_pixels<D, MODE, PAD, false>(u, 16, leaf_tile, occ_tile, cnt);
    else
        present = group_pixels<D, MODE, PAD, true>(u, nv, leaf_tile, occ_tile, cnt);
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

template <int D, int MODE, int BLOCK, int PAD, bool REGION>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu((MODE == MODE_MASK && D == 5) ? 8 : 1))) void strip_kernel(StripArgs a) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr bool OCC = (MODE & MODE_OCC) != 0;
    constexpr bool CNT = (MODE & MODE_COUNTS) != 0;
    constexpr int KW = leaf_words(D);
    constexpr int LW = lds_words(D, PAD);
    constexpr int LC = leaf_count(D);
    // one tree per strip: fixed-size tables (their LDS addresses are known
    // when the kernel is compiled); several: tables sized at launch
    extern __shared__ uint32_t dyn_lds[];
    __shared__ uint32_t st_leaf[(!REGION && MASK) ? LW : 1];
    __shared__ uint32_t st_occ[(!REGION && OCC) ? LW : 1];
    // mask staging: one work item's 16-bit group masks (spans <= kStageGroups)
    __shared__ uint16_t st_mask[MASK ? kStageGroups : 4];
    uint16_t *stage = (MASK && a.stage_mask) ? st_mask : nullptr;
    const int tid = threadIdx.x;
    const int tiles = REGION ? a.reg_cols : 1;
    uint32_t *leaf_lds = REGION ? dyn_lds : st_leaf;
    uint32_t *occ_lds = REGION ? dyn_lds + (MASK ? tiles * LW : 0) : st_occ;

    // work items: a contiguous range per workgroup, or interleaved so that
    // the items in flight at any moment are neighbours in memory
    int i0, i1, istep;
    if (a.interleave) {
        i0 = blockIdx.x;
        i1 = a.n_items;
        istep = gridDim.x;
    } else {
        i0 = (int)((int64_t)a.n_items * blockIdx.x / gridDim.x);
        i1 = (int)((int64_t)a.n_items * (blockIdx.x + 1) / gridDim.x);
        istep = 1;
    }
    int cur_s = -1, cur_f = -1;
    for (int it = i0; it < i1; it += istep) {
        const int sf = it / a.spans;
        const int t = it - sf * a.spans;
        const int s = sf / a.n_frames;
        const int f = sf - s * a.n_frames;
        const bool new_seg = (s != cur_s) || (f != cur_f);
        if (OCC && new_seg && cur_f >= 0) {
            __syncthreads();
            occ_from_lds<D, PAD>(occ_lds,
                                 a.occ + ((int64_t)cur_f * a.n_regions + (int64_t)cur_s * tiles) * KW,
                                 tiles, tid, BLOCK);
        }
        if (MASK && s != cur_s) {
            __syncthreads();
            leaf_to_lds<D, PAD>(a.leaf + (int64_t)s * tiles * KW, leaf_lds, tiles, tid, BLOCK);
        }
        if (OCC && new_seg) {
            __syncthreads();
            for (int i = tid; i < tiles * LW; i += BLOCK) occ_lds[i] = 0;
            __syncthreads();
        }
        cur_s = s;
        cur_f = f;

        const int row0 = s * a.strip_rows;
        const int rows = min(a.strip_rows, a.height - row0);
        const int gcount = rows * a.gpr;
        const int gb = t * a.span;
        const int ge = min(gb + a.span, gcount);
        const int64_t strip_off = (int64_t)row0 * a.row_pitch;
        const __amdgpu_buffer_rsrc_t rs =
            make_rsrc(a.rgb + (int64_t)f * a.frame_pitch + strip_off, (uint32_t)(a.frame_pitch - strip_off));
        __amdgpu_buffer_rsrc_t ms = make_rsrc(nullptr, 0);
        if (MASK)
            ms = make_rsrc(a.mask + ((int64_t)f * a.height + row0) * a.mask_row_words,
                           (uint32_t)rows * (uint32_t)a.mask_row_words * 8u);
        uint32_t *cbase = CNT ? a.counts + ((int64_t)f * a.n_regions + (int64_t)s * tiles) * LC
                              : nullptr;
        // two groups in flight per lane: the loads of the next group are
        // issued before the current one is worked on
        uint32_t ua[12], ub[12], ya = 0, xa = 0, yb = 0, xb = 0;
        int g = gb + tid;
        if (g < ge) fetch_group(rs, a, g, ua, ya, xa);
        for (; g < ge; g += 2 * BLOCK) {
            const int g1 = g + BLOCK;
            if (g1 < ge) fetch_group(rs, a, g1, ub, yb, xb);
            consume_group<D, MODE, PAD, REGION>(a, ms, ua, ya, xa, leaf_lds, occ_lds, cbase, stage, g - gb);
            const int g2 = g + 2 * BLOCK;
            if (g2 < ge) fetch_group(rs, a, g2, ua, ya, xa);
            if (g1 < ge)
                consume_group<D, MODE, PAD, REGION>(a, ms, ub, yb, xb, leaf_lds, occ_lds, cbase, stage, g1 - gb);
        }
        if (MASK && a.stage_mask) {
            // group g's 16 mask bits are bytes 2g, 2g+1 of the strip's mask,
            // so the item's mask is one contiguous run: write it in 8-byte words
            __syncthreads();
            const int n8 = (ge - gb) >> 2;
            const uint2 *src = reinterpret_cast<const uint2 *>(st_mask);
            for (int i = tid; i < n8; i += BLOCK)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, src[i]), ms,
                                                      2u * (uint32_t)gb + 8u * (uint32_t)i, 0, 0);
            __syncthreads();
        }
    }
    if (OCC && cur_f >= 0) {
        __syncthreads();
        occ_from_lds<D, PAD>(occ_lds,
                             a.occ + ((int64_t)cur_f * a.n_regions + (int64_t)cur_s * tiles) * KW,
                             tiles, tid, BLOCK);
    }
}

// ---------------------------------------------------------------------------
// Generic per-pixel kernel: one thread per 64-pixel mask word.

__global__ __launch_bounds__(256) void generic_kernel(GenericArgs a, int mode) {
    const int words = leaf_words(a.depth);
    const int64_t lc = (int64_t)leaf_count(a.depth);
    const int64_t total = (int64_t)a.n_frames * a.height * a.mask_row_words;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t fy = t / a.mask_row_words;
        const int wx = (int)(t - fy * a.mask_row_words);
        const int f = (int)(fy / a.height);
        const int y = (int)(fy - (int64_t)f * a.height);
        const uint8_t *row = a.rgb + (int64_t)f * a.frame_pitch + (int64_t)y * a.row_pitch;
        const int ry = a.region_h ? y / a.region_h : 0;
        uint64_t m = 0;
        const int xe = min(a.width, (wx + 1) * 64);
        for (int x = wx * 64; x < xe; ++x) {
            const uint32_t k = path_key(row[3 * x], row[3 * x + 1], row[3 * x + 2], a.depth);
            const int reg = a.region_w ? ry * a.reg_cols + x / a.region_w : 0;
            if (mode & MODE_MASK) {
                const uint32_t w = a.leaf[(int64_t)reg * words + (k >> 5)];
                if (((w >> (k & 31)) & 1u) == 0) m |= 1ull << (x & 63);
            }
            if (mode & MODE_OCC) {
                uint32_t *w = &a.occ[((int64_t)f * a.n_regions + reg) * words + (k >> 5)];
                const uint32_t bit = 1u << (k & 31);
                if ((__atomic_load_n(w, __ATOMIC_RELAXED) & bit) == 0) atomicOr(w, bit);
            }
            if (mode & MODE_COUNTS) atomicAdd(&a.counts[((int64_t)f * a.n_regions + reg) * lc + k], 1u);
        }
        if (mode & MODE_MASK) a.mask[t] = m;
    }
}

// ---------------------------------------------------------------------------
// Merge: bit-sliced frame counts, one thread per 32 keys.

__global__ __launch_bounds__(256) void merge_kernel(MergeArgs a) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.slot_words) return;
    const uint32_t valid = a.valid_bits_last >= 32 ? 0xFFFFFFFFu : ((1u << a.valid_bits_last) - 1u);
    if (a.empty) {
        a.leaf[i] = 0;
        return;
    }
    uint32_t c[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) c[b] = 0;
    // eight window slots per round: their loads are independent and in flight together
    int slot = a.first;
    for (int t0 = 0; t0 < a.n_trees; t0 += 8) {
        uint32_t x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            x[k] = 0;
            if (t0 + k < a.n_trees) {
                int sl = slot + k;
                if (sl >= a.ring_len) sl -= a.ring_len;
                x[k] = a.occ_ring[(int64_t)sl * a.slot_words + i] & valid;
            }
        }
        slot += 8;
        while (slot >= a.ring_len) slot -= a.ring_len;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            uint32_t carry = x[k];
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                if (b < a.planes) {
                    const uint32_t tmp = c[b] & carry;
                    c[b] ^= carry;
                    carry = tmp;
                }
            }
        }
    }
    // bit-sliced count >= kmin
    uint32_t ge = 0, eq = 0xFFFFFFFFu;
#pragma unroll
    for (int b = 15; b >= 0; --b) {
        if ((a.kmin >> b) & 1u) {
            eq &= c[b];
        } else {
            ge |= eq & c[b];
            eq &= ~c[b];
        }
    }
    ge |= eq;
    a.leaf[i] = ge & valid;
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers

template <int D, int LAY, bool REGION>
static hipError_t launch_variant(int mode, int block, const StripArgs &a, int grid, size_t lds,
                                 hipStream_t st) {
    switch (mode) {
        case MODE_MASK:
            if (block == 512)
                hipLaunchKernelGGL((strip_kernel<D, MODE_MASK, 512, LAY, REGION>), dim3(grid), dim3(512), lds, st, a);
            else
                hipLaunchKernelGGL((strip_kernel<D, MODE_MASK, 256, LAY, REGION>), dim3(grid), dim3(256), lds, st, a);
            break;
        case MODE_OCC:
            if (block == 1024)
                hipLaunchKernelGGL((strip_kernel<D, MODE_OCC, 1024, LAY, REGION>), dim3(grid), dim3(1024), lds, st, a);
            else
                hipLaunchKernelGGL((strip_kernel<D, MODE_OCC, 256, LAY, REGION>), dim3(grid), dim3(256), lds, st, a);
            break;
        case MODE_MASK | MODE_OCC:
            hipLaunchKernelGGL((strip_kernel<D, MODE_MASK | MODE_OCC, 256, LAY, REGION>), dim3(grid), dim3(256), lds, st, a);
            break;
        case MODE_OCC | MODE_COUNTS:
            hipLaunchKernelGGL((strip_kernel<D, MODE_OCC | MODE_COUNTS, 256, LAY, REGION>), dim3(grid), dim3(256), lds, st, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int D>
static hipError_t launch_strip_d(int mode, int block, int lay, bool region, const StripArgs &a,
                                 int grid, size_t lds, hipStream_t st) {
    if (lay == LAY_WIDE) {
        if (D > 5) return hipErrorInvalidValue;
        if (region) return launch_variant<D, (D <= 5 ? LAY_WIDE : LAY_COMPACT), true>(mode, block, a, grid, lds, st);
        return launch_variant<D, (D <= 5 ? LAY_WIDE : LAY_COMPACT), false>(mode, block, a, grid, lds, st);
    }
    if (region) return launch_variant<D, LAY_COMPACT, true>(mode, block, a, grid, lds, st);
    return launch_variant<D, LAY_COMPACT, false>(mode, block, a, grid, lds, st);
}

size_t strip_lds_bytes(int depth, int mode, int reg_cols, int lay) {
    if (depth < 1 || depth > 8 || (lay == LAY_WIDE && depth > 5)) return 0;
    const size_t words = (size_t)reg_cols * (size_t)lds_words(depth, lay);
    return words * 4 * (((mode & MODE_MASK) ? 1 : 0) + ((mode & MODE_OCC) ? 1 : 0));
}

// Every pointer a mode writes or reads must be set; a launch with a missing
// one is refused instead of faulting on the device.
static bool strip_pointers_ok(int mode, const StripArgs &a) {
    if (!a.rgb) return false;
    if ((mode & MODE_MASK) && (!a.leaf || !a.mask)) return false;
    if ((mode & MODE_OCC) && !a.occ) return false;
    if ((mode & MODE_COUNTS) && !a.counts) return false;
    return true;
}

hipError_t launch_strip(int depth, int mode, const StripArgs &a, int grid, int block, int pad,
                        bool region, size_t lds_bytes, hipStream_t stream) {
    if (!strip_pointers_ok(mode, a) || grid < 1) return hipErrorInvalidValue;
    if (a.frame_pitch > 0x7FFFFFFFLL) return hipErrorInvalidValue;
    if (!region && a.reg_cols != 1) return hipErrorInvalidValue;
    switch (depth) {
        case 1: return launch_strip_d<1>(mode, block, pad, region, a, grid, lds_bytes, stream);
        case 2: return launch_strip_d<2>(mode, block, pad, region, a, grid, lds_bytes, stream);
        case 3: return launch_strip_d<3>(mode, block, pad, region, a, grid, lds_bytes, stream);
        case 4: return launch_strip_d<4>(mode, block, pad, region, a, grid, lds_bytes, stream);
        case 5: return launch_strip_d<5>(mode, block, pad, region, a, grid, lds_bytes, stream);
        case 6: return launch_strip_d<6>(mode, block, pad, region, a, grid, lds_bytes, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_generic(int mode, const GenericArgs &a, hipStream_t stream) {
    if (!a.rgb || ((mode & MODE_MASK) && (!a.leaf || !a.mask)) || ((mode & MODE_OCC) && !a.occ) ||
        ((mode & MODE_COUNTS) && !a.counts))
        return hipErrorInvalidValue;
    const int64_t total = (int64_t)a.n_frames * a.height * a.mask_row_words;
    if (total == 0) return hipSuccess;
    const int block = 256;
    const int64_t want = (total + block - 1) / block;
    const int grid = (int)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(generic_kernel, dim3(grid), dim3(block), 0, stream, a, mode);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs &a, hipStream_t stream) {
    if (!a.occ_ring || !a.leaf || a.ring_len < 1 || a.first < 0 || a.first >= a.ring_len)
        return hipErrorInvalidValue;
    if (a.slot_words == 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (a.slot_words + block - 1) / block;
    hipLaunchKernelGGL(merge_kernel, dim3((unsigned)grid), dim3(block), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    if (!p || n < 0) return hipErrorInvalidValue;
    const int block = 256;
    const int64_t want = (n + block - 1) / block;
    const int grid = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid), dim3(block), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // namespace obg
