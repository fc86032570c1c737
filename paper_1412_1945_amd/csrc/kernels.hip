// kernels.hip -- gfx950 kernels of octree background modelling.
//
// strip_kernel  one pass over 16-pixel groups (48 contiguous bytes = three
//               16-byte buffer loads per lane, the next group's loads issued
//               before the current group is worked on).  Per pixel: a shift
//               and mask of the R,G bytes (or three bit-field extracts) give
//               the pixel's depth-d octree node (Algorithm 1 with the pruning
//               of Section 2) as an LDS address and bit, then
//                 MASK   test the bit in the merged leaf set (Algorithm 3);
//                        the 16 results of a lane form 16 mask bits, gathered
//                        per work item in LDS and written as one run;
//                 OCC    set the bit in this frame's LDS occupancy bitset with
//                        an LDS atomic OR; the bitset is OR-ed into HBM once
//                        per (frame, strip) segment of a workgroup;
//                 COUNTS add the pixel to the key's counter (runs of equal
//                        keys inside a lane are added with one atomic).
// generic_kernel per-pixel fallback for d = 7, 8 and region widths that are
//               not a multiple of 16 pixels; bitsets stay in HBM/L2.
// merge_kernel  per 32 keys: bit-sliced counters of the window's bitsets and
//               a bit-sliced compare against the frame-count threshold
//               (Algorithm 2 in closed form); 64 words to a workgroup, its
//               four waves count a quarter of the window each.
#include <algorithm>

#include "strip_core.h"

namespace obg {

// Trees of frame f: from the frame list, or at a fixed pitch.
template <bool LIST>
__device__ __forceinline__ uint32_t *frame_occ(const StripArgs &a, int f, int kw) {
    return LIST ? a.occ_list[f] : a.occ + (int64_t)f * a.n_regions * kw;
}

// LIST: frames, masks and trees through the per-frame pointer arrays (a
// separate instance, so the other kernels keep their registers)
template <int D, int MODE, int BLOCK, int PAD, bool REGION, bool LIST = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(
    (MODE == MODE_MASK && D == 5) ? (BLOCK == 512 ? 8 : 4) : ((MODE == (MODE_MASK | MODE_OCC) && BLOCK == 512) ? 4 : 1)))) void
strip_kernel(StripArgs a) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr bool OCC = (MODE & MODE_OCC) != 0;
    constexpr bool CNT = (MODE & MODE_COUNTS) != 0;
    constexpr int KW = leaf_words(D);
    constexpr int LW = lds_words(D, PAD);
    constexpr int LC = leaf_count(D);
    // the fused pass keeps one dual table per tile (leaf and occupancy words
    // in pairs): one 8-byte LDS read per pixel gives both
    constexpr bool DUAL = MASK && OCC && !CNT;
    // one tree per strip: fixed-size tables (their LDS addresses are known
    // when the kernel is compiled); several: tables sized at launch
    extern __shared__ uint32_t dyn_lds[];
    __shared__ uint32_t st_leaf[(!REGION && MASK) ? (DUAL ? 2 * LW : LW) : 1];
    __shared__ uint32_t st_occ[(!REGION && OCC && !DUAL) ? LW : 1];
    // mask staging: one work item's 16-bit group masks (spans <= kStageGroups,
    // kMaxStageGroups for the fused pass without regions)
    __shared__ uint16_t st_mask[MASK ? ((DUAL && !REGION) ? kMaxStageGroups : kStageGroups) : 4];
    uint16_t *stage = (MASK && a.stage_mask) ? st_mask : nullptr;
    const int tid = threadIdx.x;
    // LDS tables of one strip: a chunk of at most chunk_cols regions
    const int max_tiles = REGION ? a.chunk_cols : 1;
    uint32_t *leaf_lds = REGION ? dyn_lds : st_leaf;
    uint32_t *occ_lds = DUAL ? leaf_lds : (REGION ? dyn_lds + (MASK ? max_tiles * LW : 0) : st_occ);
    const bool store = a.occ_store != 0;
    // bitsets kept in the compact LDS order (frame lists of the serving runtime)
    const bool native = LIST && PAD == LAY_COMPACT && a.native != 0;

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
    // the segment (frame, strip) whose occupancy the LDS table holds: its
    // frame, strip, first region and number of regions
    int cur_s = -1, cur_f = -1, cur_tiles = 1;
    int64_t cur_reg0 = 0;
    for (int it = i0; it < i1; it += istep) {
        const int sf = it / a.spans;
        const int t = it - sf * a.spans;
        const int s = sf / a.n_frames;
        const int f = sf - s * a.n_frames;
        // strip s = (row of regions rr, chunk k)
        int rr = s;
        Chunk ch{};
        if (REGION) {
            rr = s / a.n_chunks;
            const int k = s - rr * a.n_chunks;
            const bool last = k == a.n_chunks - 1;
            ch.div = last ? a.div_cgpr_last : a.div_cgpr;
            ch.cw = (uint32_t)(last ? a.cgpr_last : a.cgpr);
            ch.gx0 = (uint32_t)k * (uint32_t)a.cgpr;
            ch.c0 = k * a.chunk_cols;
            ch.tiles = min(a.chunk_cols, a.reg_cols - ch.c0);
        }
        const int tiles = REGION ? ch.tiles : 1;
        const int64_t reg0 = REGION ? (int64_t)rr * a.reg_cols + ch.c0 : (int64_t)s;
        const bool new_seg = (s != cur_s) || (f != cur_f);
        if (OCC && new_seg && cur_f >= 0) {
            __syncthreads();
            occ_from_lds<D, PAD, DUAL>(occ_lds, frame_occ<LIST>(a, cur_f, KW) + cur_reg0 * KW, cur_tiles, tid, BLOCK,
                                       store, native);
        }
        if (MASK && s != cur_s) {
            // (a dual table is cleared whole here, occupancy bits included)
            __syncthreads();
            leaf_to_lds<D, PAD, DUAL>(a.leaf + reg0 * KW, leaf_lds, tiles, tid, BLOCK, native);
        } else if (DUAL && new_seg) {
            __syncthreads();
            clear_dual_occ(occ_lds, tiles * 2 * LW, tid, BLOCK);
            __syncthreads();
        }
        if (OCC && !DUAL && new_seg) {
            __syncthreads();
            for (int i = tid; i < tiles * LW; i += BLOCK) occ_lds[i] = 0;
            __syncthreads();
        }
        cur_s = s;
        cur_f = f;
        cur_tiles = tiles;
        cur_reg0 = reg0;

        const int row0 = rr * a.strip_rows;
        const int rows = min(a.strip_rows, a.height - row0);
        const int gcount = rows * (REGION ? (int)ch.cw : a.gpr);
        const int gb = t * a.span;
        const int ge = min(gb + a.span, gcount);
        const int64_t strip_off = (int64_t)row0 * a.row_pitch;
        const uint8_t *frame = LIST ? a.rgb_list[f] : a.rgb + (int64_t)f * a.frame_pitch;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(frame + strip_off, (uint32_t)(a.frame_pitch - strip_off));
        __amdgpu_buffer_rsrc_t ms = make_rsrc(nullptr, 0);
        if (MASK) {
            uint64_t *fm = LIST ? a.mask_list[f] : a.mask + (int64_t)f * a.height * a.mask_row_words;
            ms = make_rsrc(fm + (int64_t)row0 * a.mask_row_words, (uint32_t)rows * (uint32_t)a.mask_row_words * 8u);
        }
        uint32_t *cbase = CNT ? a.counts + ((int64_t)f * a.n_regions + reg0) * LC : nullptr;
        span_loop<D, MODE, PAD, REGION, BLOCK>(a, rs, ms, gb, ge, leaf_lds, occ_lds, cbase, stage, ch);
    }
    if (OCC && cur_f >= 0) {
        __syncthreads();
        occ_from_lds<D, PAD, DUAL>(occ_lds, frame_occ<LIST>(a, cur_f, KW) + cur_reg0 * KW, cur_tiles, tid, BLOCK,
                                   store, native);
    }
}

// ---------------------------------------------------------------------------
// Redraw (Section 2): a pixel's colour in its frame's pruned tree is its depth-d
// node, whose colour is the node's path bits with the remaining bits zero; the
// frame's own tree holds every pixel's node, so the redraw keeps the top
// `depth` bits of every byte.  One lane per 16 pixels (48 bytes); blockIdx.y
// walks the frames.
__global__ __launch_bounds__(256) void quantize_kernel(QuantArgs a, uint32_t keep, int frame0) {
    const int f = frame0 + (int)blockIdx.y;
    if (f >= a.n_frames) return;
    const int gpr = (a.width + 15) / 16;
    const uint32_t groups = (uint32_t)a.height * (uint32_t)gpr;
    const uint8_t *src = a.rgb + (int64_t)f * a.frame_pitch;
    uint8_t *dst = a.out + (int64_t)f * a.frame_pitch;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += gridDim.x * blockDim.x) {
        const uint32_t y = g / (uint32_t)gpr;
        const uint32_t gx = g - y * (uint32_t)gpr;
        const int64_t off = (int64_t)y * a.row_pitch + 48 * (int64_t)gx;
        const int nv = min(16, a.width - 16 * (int)gx);
        if (nv == 16) {
            const uint4 *s4 = reinterpret_cast<const uint4 *>(src + off);
            uint4 *d4 = reinterpret_cast<uint4 *>(dst + off);
            uint4 v0 = s4[0], v1 = s4[1], v2 = s4[2];
            v0.x &= keep; v0.y &= keep; v0.z &= keep; v0.w &= keep;
            v1.x &= keep; v1.y &= keep; v1.z &= keep; v1.w &= keep;
            v2.x &= keep; v2.y &= keep; v2.z &= keep; v2.w &= keep;
            d4[0] = v0;
            d4[1] = v1;
            d4[2] = v2;
        } else {
            // the row's last, partial group: only its pixels' bytes
            for (int b = 0; b < 3 * nv; ++b) dst[off + b] = src[off + b] & (uint8_t)keep;
        }
    }
}

hipError_t launch_quantize(const QuantArgs &a, hipStream_t stream) {
    if (!a.rgb || !a.out || a.depth < 1 || a.depth > 8 || a.width < 1 || a.height < 1 || a.n_frames < 0)
        return hipErrorInvalidValue;
    if (a.n_frames == 0) return hipSuccess;
    const uint32_t byte = (0xFFu << (8 - a.depth)) & 0xFFu;
    const uint32_t keep = byte * 0x01010101u;
    const int64_t groups = (int64_t)a.height * ((a.width + 15) / 16);
    if (groups > 0xFFFFFFFFLL) return hipErrorInvalidValue;
    int gx = (int)std::min<int64_t>((groups + 255) / 256, 2048);
    for (int f0 = 0; f0 < a.n_frames; f0 += 65535) {
        const int nf = std::min(65535, a.n_frames - f0);
        hipLaunchKernelGGL(quantize_kernel, dim3(gx, nf), dim3(256), 0, stream, a, keep, f0);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scoring against ground truth (Section 5's counts): popcounts of mask and
// truth words, bits past the row's width ignored; per-wave sums, one atomic
// add per wave and counter.
__global__ __launch_bounds__(256) void score_kernel(const uint64_t *__restrict__ mask, const uint64_t *__restrict__ truth,
                                                    int64_t n_words, int32_t row_words, int32_t width,
                                                    unsigned long long *__restrict__ counts) {
    const uint64_t last = (width & 63) ? ((1ull << (width & 63)) - 1ull) : ~0ull;
    unsigned long long tp = 0, fp = 0, fn = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t valid = (i % row_words == row_words - 1) ? last : ~0ull;
        const uint64_t m = mask[i] & valid, t = truth[i] & valid;
        tp += __popcll(m & t);
        fp += __popcll(m & ~t);
        fn += __popcll(~m & t);
    }
    for (int off = 32; off > 0; off >>= 1) {
        tp += __shfl_xor(tp, off);
        fp += __shfl_xor(fp, off);
        fn += __shfl_xor(fn, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counts[0], tp);
        atomicAdd(&counts[1], fp);
        atomicAdd(&counts[2], fn);
    }
}

hipError_t launch_score(const uint64_t *mask, const uint64_t *truth, int64_t rows, int32_t row_words,
                        int32_t width, unsigned long long *counts, hipStream_t stream) {
    if (!mask || !truth || !counts || rows < 0 || row_words < 1 || width < 1 || width > 64 * row_words)
        return hipErrorInvalidValue;
    const int64_t n_words = rows * row_words;
    if (n_words == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n_words + 255) / 256, 4096);
    hipLaunchKernelGGL(score_kernel, dim3(grid), dim3(256), 0, stream, mask, truth, n_words, row_words, width, counts);
    return hipGetLastError();
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

template <int SPLIT>
__global__ __launch_bounds__(kMergeBlock) void merge_kernel(MergeArgs a) {
    __shared__ uint32_t part[SPLIT > 1 ? (SPLIT - 1) * 16 * 64 : 1];
    merge_block<SPLIT>(a.occ_ring, a.ring_len, a.first, a.n_trees, a.slot_words, a.slot_words,
                       blockIdx.x * (int64_t)(kMergeBlock / SPLIT), a.valid_bits_last, a.kmin, a.planes, a.empty,
                       a.group, a.leaf, part);
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers

// Dynamic LDS above 64 KiB (region tables on gfx950) has to be allowed per kernel.
template <typename K>
static hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

#define OBG_LAUNCH(K, BLK)                                                  \
    do {                                                                    \
        const hipError_t e_ = allow_lds(K, lds);                            \
        if (e_ != hipSuccess) return e_;                                    \
        hipLaunchKernelGGL(K, dim3(grid), dim3(BLK), lds, st, a);           \
    } while (0)

template <int D, int LAY, bool REGION>
static hipError_t launch_variant(int mode, int block, const StripArgs &a, int grid, size_t lds,
                                 hipStream_t st) {
    if (a.rgb_list) {
        // frame lists: region passes that build occupancy
        if (!REGION || !a.occ_list || (mode != MODE_OCC && mode != (MODE_MASK | MODE_OCC)))
            return hipErrorInvalidValue;
        if (mode == MODE_OCC) {
            if (block == 1024)
                OBG_LAUNCH((strip_kernel<D, MODE_OCC, 1024, LAY, true, true>), 1024);
            else
                OBG_LAUNCH((strip_kernel<D, MODE_OCC, 256, LAY, true, true>), 256);
        } else {
            if (!a.mask_list) return hipErrorInvalidValue;
            if (block == 512)
                OBG_LAUNCH((strip_kernel<D, MODE_MASK | MODE_OCC, 512, LAY, true, true>), 512);
            else
                OBG_LAUNCH((strip_kernel<D, MODE_MASK | MODE_OCC, 256, LAY, true, true>), 256);
        }
        return hipGetLastError();
    }
    switch (mode) {
        case MODE_MASK:
            if (block == 512)
                OBG_LAUNCH((strip_kernel<D, MODE_MASK, 512, LAY, REGION>), 512);
            else
                OBG_LAUNCH((strip_kernel<D, MODE_MASK, 256, LAY, REGION>), 256);
            break;
        case MODE_OCC:
            if (block == 1024)
                OBG_LAUNCH((strip_kernel<D, MODE_OCC, 1024, LAY, REGION>), 1024);
            else
                OBG_LAUNCH((strip_kernel<D, MODE_OCC, 256, LAY, REGION>), 256);
            break;
        case MODE_MASK | MODE_OCC:
            if (block == 512)
                OBG_LAUNCH((strip_kernel<D, MODE_MASK | MODE_OCC, 512, LAY, REGION>), 512);
            else
                OBG_LAUNCH((strip_kernel<D, MODE_MASK | MODE_OCC, 256, LAY, REGION>), 256);
            break;
        case MODE_OCC | MODE_COUNTS:
            OBG_LAUNCH((strip_kernel<D, MODE_OCC | MODE_COUNTS, 256, LAY, REGION>), 256);
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
    if (!a.rgb && !a.rgb_list) return false;
    if ((mode & MODE_MASK) && (!a.leaf || (!a.mask && !a.mask_list))) return false;
    if ((mode & MODE_OCC) && !a.occ && !a.occ_list) return false;
    if ((a.rgb_list || a.occ_list || a.mask_list) && (mode & MODE_COUNTS)) return false;
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
    if (!a.occ_ring || !a.leaf || a.ring_len < 1 || a.first < 0 || a.first >= a.ring_len || a.group < 1 ||
        a.n_trees < 1 || a.n_trees > a.ring_len)
        return hipErrorInvalidValue;
    if (a.slot_words == 0) return hipSuccess;
    // small merges are latency: four waves share each word's window; large
    // ones (regions: 8160 trees of 128 words at 4K) fill the chip with one
    // thread per word (measured at 1.04 M words: 56 against 140 us)
    if (a.slot_words >= kMergeWholeWords) {
        const int64_t grid = (a.slot_words + kMergeBlock - 1) / kMergeBlock;
        hipLaunchKernelGGL(merge_kernel<1>, dim3((unsigned)grid), dim3(kMergeBlock), 0, stream, a);
    } else {
        const int64_t grid = (a.slot_words + 63) / 64;
        hipLaunchKernelGGL(merge_kernel<kMergeWaves>, dim3((unsigned)grid), dim3(kMergeBlock), 0, stream, a);
    }
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
