// internal.h -- launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/obg.h"
#include "device.h"

namespace obg {

// One pass over frames in 16-pixel groups, strip by strip.  A strip is one
// row of regions (the whole frame without regions); its tiles' bitsets live
// in LDS while the strip is processed.
struct StripArgs {
    const uint8_t *rgb;
    int64_t frame_pitch, row_pitch;
    int32_t width, height, n_frames;
    int32_t gpr;              // 16-pixel groups per row: 4 * ceil(width / 64)
    int32_t strip_rows;       // rows per strip (region_h, or height)
    int32_t n_strips;         // region rows x chunks
    int32_t reg_cols;         // regions per row of regions (1 without regions)
    int32_t n_regions;
    FastDiv div_gpr;          // group-in-strip -> row-in-strip
    FastDiv div_tile;         // group-in-row -> region column (region_w / 16 groups)
    // chunks of a row of regions (regions only; one chunk = the whole row):
    // chunk k holds region columns k*chunk_cols .. and group columns
    // k*cgpr .. (the last chunk runs to the end of the row, cgpr_last groups)
    int32_t n_chunks, chunk_cols, cgpr, cgpr_last;
    FastDiv div_cgpr, div_cgpr_last;
    int32_t span;             // groups per work item
    int32_t spans;            // work items per (strip, frame)
    int32_t n_items;          // n_strips * n_frames * spans
    int32_t interleave;       // 1: item i goes to workgroup i % grid; 0: contiguous ranges
    int32_t stage_mask;       // 1: masks gathered in LDS per item (span <= kStageGroups or kMaxStageGroups)
    int32_t occ_test;         // 1: read an occupancy word first, atomic OR only when the bit is clear
    int32_t occ_store;        // 1: one work item per (frame, strip): occupancy words are stored, not OR-ed
    const uint32_t *leaf;     // [n_regions][words], key order
    uint64_t *mask;           // [n_frames][height][mask_row_words]
    int32_t mask_row_words;
    uint32_t *occ;            // [n_frames][n_regions][words], zeroed and OR-ed into (or stored)
    uint32_t *counts;         // [n_frames][n_regions][8^d], zeroed, added into
    // frame lists (device arrays, or all NULL): frame f's pixels, mask and
    // trees start at rgb_list[f], mask_list[f], occ_list[f] instead of at
    // fixed pitches from rgb, mask and occ
    const uint8_t *const *rgb_list;
    uint64_t *const *mask_list;
    uint32_t *const *occ_list;
    // with frame lists and compact tables: leaf set and trees in HBM are in
    // the compact LDS order instead of key order (copied as they are)
    int32_t native;
};

// Per-pixel fallback for any depth 1..8 and any region size.
struct GenericArgs {
    const uint8_t *rgb;
    int64_t frame_pitch, row_pitch;
    int32_t width, height, n_frames, depth;
    int32_t region_w, region_h, reg_cols, n_regions;
    int32_t mask_row_words;
    const uint32_t *leaf;
    uint64_t *mask;
    uint32_t *occ;
    uint32_t *counts;
};

struct MergeArgs {
    const uint32_t *occ_ring;
    int32_t ring_len, first, n_trees;
    int64_t slot_words;       // n_regions * words
    int32_t words, valid_bits_last;  // bits used in each word (32, or 8^d for d = 1)
    uint32_t kmin;            // keep iff count >= kmin
    int32_t planes;           // counter bit planes: bit length of n_trees
    int32_t empty;            // kmin > n_trees: nothing kept
    uint32_t *leaf;
    int32_t group;            // window slots per counted tree (1 = one tree per frame)
};

enum StripMode { MODE_MASK = 1, MODE_OCC = 2, MODE_COUNTS = 4 };

// Mask staging: a work item of at most this many 16-pixel groups gathers its
// mask in LDS and writes it as one run; the fused pass without regions and
// the served form stage items of up to kMaxStageGroups.
constexpr int kStageGroups = 1024;
constexpr int kMaxStageGroups = 4096;

// Record the calling thread's last error (read by obg_last_error); returns code.
int set_error(int code, const char *msg);
// Current value of launch knob `key` (obg_tune_set), or dflt when unset.
int tune(int key, int dflt);

// lay: LDS order (LAY_WIDE / LAY_COMPACT, see device.h); region: more than
// one region per strip
hipError_t launch_strip(int depth, int mode, const StripArgs &a, int grid, int block, int lay,
                        bool region, size_t lds_bytes, hipStream_t stream);
// LDS bytes one workgroup of the strip kernel needs (0 = order not possible)
size_t strip_lds_bytes(int depth, int mode, int reg_cols, int lay);
// Frames redrawn with their own pruned trees' leaf colours: every channel
// keeps its top `depth` bits.  rgb and out share the geometry; in place is
// allowed (each byte is read and written by the same lane).
struct QuantArgs {
    const uint8_t *rgb;
    uint8_t *out;
    int64_t frame_pitch, row_pitch;
    int32_t width, height, n_frames, depth;
};
hipError_t launch_quantize(const QuantArgs &a, hipStream_t stream);
// Agreement of masks with ground-truth masks (same layout): counts[0] true
// positives, counts[1] false positives, counts[2] false negatives, added to.
hipError_t launch_score(const uint64_t *mask, const uint64_t *truth, int64_t rows, int32_t row_words,
                        int32_t width, unsigned long long *counts, hipStream_t stream);
hipError_t launch_generic(int mode, const GenericArgs &a, hipStream_t stream);
hipError_t launch_merge(const MergeArgs &a, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);

// Frames of one geometry anywhere in device memory (the serving runtime's
// arena blocks): mode MODE_OCC builds each frame's trees, MODE_MASK |
// MODE_OCC also classifies against `leaf`.  The three arrays are device
// arrays of n_frames pointers (mask_list unused without MODE_MASK); each
// frame's trees are written whole (n_regions * words words).  Geometries
// with several regions per row of regions that the LDS kernels take are
// served this way (pixels_list_ok); others are refused.
struct FrameLists {
    const uint8_t *const *rgb;
    uint64_t *const *mask;
    uint32_t *const *occ;
};
bool pixels_list_ok(const obg_geom *g, int mode);
// Both modes take frame lists with compact tables: the geometry's bitsets
// can stay in the compact LDS order (native) from pass to pass.
bool pixels_list_native_ok(const obg_geom *g);
int run_pixels_list(const obg_geom *g, int mode, const FrameLists &l, int32_t n_frames, const uint32_t *leaf,
                    hipStream_t stream, bool native = false);

}  // namespace obg
