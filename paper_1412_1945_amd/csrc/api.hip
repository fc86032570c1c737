// api.hip -- C ABI of libobg.so: argument checks, work split, launches.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/obg.h"
#include "internal.h"

using namespace obg;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// Launch-shape knobs of the pixel kernels (0 = built-in default).
int g_tune[OBG_TUNE_COUNT] = {0};
std::mutex g_tune_mu;

}  // namespace

int obg::tune(int key, int dflt) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune[key] ? g_tune[key] : dflt;
}

int obg::set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}

namespace {

int hip_fail(hipError_t e, const char *what) {
    return fail(OBG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Validated geometry and the sizes derived from it.
struct Geo {
    int32_t width, height, depth, region_w, region_h;
    int64_t row_pitch, frame_pitch;
    int32_t reg_cols, reg_rows, n_regions;
    int32_t words;             // uint32 words per tree
    int32_t mask_row_words;    // uint64 words per mask row
};

int check_geom(const obg_geom *g, Geo *o, bool pixels) {
    if (!g) return fail(OBG_EINVAL, "geometry pointer is NULL");
    if (g->width < 1 || g->height < 1) return fail(OBG_EINVAL, "width and height must be >= 1 (got %d x %d)", g->width, g->height);
    if (g->depth < 1 || g->depth > 8) return fail(OBG_EINVAL, "depth must be in [1, 8] (got %d)", g->depth);
    if (g->region_w < 0 || g->region_h < 0 || ((g->region_w == 0) != (g->region_h == 0)))
        return fail(OBG_EINVAL, "region_w and region_h must both be 0 or both >= 1 (got %d, %d)", g->region_w, g->region_h);
    if (g->width > (1 << 24) || g->height > (1 << 24)) return fail(OBG_EINVAL, "frame side above 2^24");
    o->width = g->width;
    o->height = g->height;
    o->depth = g->depth;
    o->region_w = g->region_w;
    o->region_h = g->region_h;
    o->row_pitch = g->row_pitch;
    o->frame_pitch = g->frame_pitch;
    o->reg_cols = g->region_w ? (g->width + g->region_w - 1) / g->region_w : 1;
    o->reg_rows = g->region_h ? (g->height + g->region_h - 1) / g->region_h : 1;
    if ((int64_t)o->reg_cols * o->reg_rows > (1 << 30)) return fail(OBG_EINVAL, "too many regions");
    o->n_regions = o->reg_cols * o->reg_rows;
    o->words = leaf_words(g->depth);
    o->mask_row_words = (g->width + 63) / 64;
    if (pixels) {
        if (g->frame_pitch > 0x7FFFFFFFLL)
            return fail(OBG_EINVAL, "frame_pitch must be below 2 GiB");
        if (g->row_pitch < 3 * (int64_t)g->width)
            return fail(OBG_EINVAL, "row_pitch %lld < 3*width %lld", (long long)g->row_pitch, 3LL * g->width);
        if (g->frame_pitch < (int64_t)g->height * g->row_pitch)
            return fail(OBG_EINVAL, "frame_pitch %lld < height*row_pitch", (long long)g->frame_pitch);
        if (g->row_pitch % 16 || g->frame_pitch % 16)
            return fail(OBG_EALIGN, "row_pitch and frame_pitch must be multiples of 16 bytes");
    }
    return OBG_OK;
}

int cu_count() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (!cache[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// LDS one workgroup of the strip kernel may hold for its tables: the device's
// per-workgroup limit (160 KiB on gfx950) less room for the kernel's static
// arrays (mask staging).
size_t strip_lds_max() {
    static std::mutex mu;
    static size_t cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    std::lock_guard<std::mutex> lk(mu);
    if (!cache[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || n <= 0)
            n = 64 * 1024;
        size_t lim = (size_t)n;
        if (lim > 160 * 1024) lim = 160 * 1024;
        cache[dev] = lim > 64 * 1024 ? lim - 4 * 1024 : lim;
    }
    return cache[dev];
}

// Does the LDS strip kernel handle this geometry and mode?  Picks the LDS
// order: the wide one when it fits, else the compact one.
constexpr int64_t kOccItemsPerWg = 4;

// Region columns per chunk must cover whole 64-pixel mask words: the
// smallest such number of columns.
int chunk_step(const Geo &g) {
    const int rw16 = g.region_w / 16;
    int gcd = rw16 % 4 == 0 ? 4 : (rw16 % 2 == 0 ? 2 : 1);
    return 4 / gcd;
}

bool strip_ok(const Geo &g, int mode, int *lay) {
    if (g.depth > 6) return false;
    if (g.region_w && (g.region_w % 16) != 0) return false;
    const size_t wide = strip_lds_bytes(g.depth, mode, g.reg_cols, LAY_WIDE);
    // the wide order when its tables fit in 64 KiB (several workgroups per
    // CU); compact tables of many regions may fill the workgroup's whole LDS
    if (wide && wide <= 64 * 1024 && tune(OBG_TUNE_LAYOUT, 1) == 1) {
        *lay = LAY_WIDE;
        return true;
    }
    *lay = LAY_COMPACT;
    if (g.reg_cols == 1) return strip_lds_bytes(g.depth, mode, 1, LAY_COMPACT) <= 64 * 1024;
    // rows of regions are cut into chunks when their tables do not fit: the
    // narrowest chunk has to
    const int narrow = std::min(g.reg_cols, chunk_step(g));
    return strip_lds_bytes(g.depth, mode, narrow, LAY_COMPACT) <= strip_lds_max();
}

// Region columns per chunk of a row of regions: the fewest chunks whose
// tables take at most 64 KiB of LDS (so that two workgroups share a CU) and,
// when the call's rows of regions are fewer than `target` work items, enough
// chunks to give about `target` of them.  Every chunk but the last spans
// chunk_cols columns, a multiple of chunk_step.
int region_chunk_cols(const Geo &g, int mode, int lay, int64_t rows_sf, int64_t target) {
    const int step = chunk_step(g);
    if (g.reg_cols <= step) return g.reg_cols;
    const int max_chunks = g.reg_cols / step;
    int64_t n = 1;
    const size_t row = strip_lds_bytes(g.depth, mode, g.reg_cols, lay);
    const size_t cap = std::min<size_t>(64 * 1024, strip_lds_max());
    if (row > cap) n = (int64_t)((row + cap - 1) / cap);
    if (tune(OBG_TUNE_REGION_CHUNKS, 1) == 1 && rows_sf < target)
        n = std::max<int64_t>(n, (target + rows_sf - 1) / rows_sf);
    n = std::min<int64_t>(n, max_chunks);
    int cols = (int)((g.reg_cols + n - 1) / n);
    cols = (cols + step - 1) / step * step;
    // the chunk must fit the workgroup's LDS (strip_ok guarantees `step` does)
    while (cols > step && strip_lds_bytes(g.depth, mode, cols, lay) > strip_lds_max()) cols -= step;
    return cols >= g.reg_cols ? g.reg_cols : cols;
}

// lists: frames, masks and trees through per-frame pointer arrays (the
// geometry must pass strip_ok; every (frame, strip) is one work item and its
// trees are stored whole); native: with lists, bitsets in the compact order
int run_pixels(const Geo &g, int mode, const uint8_t *rgb, int32_t n_frames, const uint32_t *leaf,
               uint64_t *mask, uint32_t *occ, uint32_t *counts, hipStream_t st, const FrameLists *lists = nullptr,
               bool native = false) {
    hipError_t e;
    const int64_t occ_words = (int64_t)n_frames * g.n_regions * g.words;
    if (mode & MODE_COUNTS) {
        const int64_t n = (int64_t)n_frames * g.n_regions * leaf_count(g.depth);
        if ((e = launch_fill_u32(counts, n, 0u, st)) != hipSuccess) return hip_fail(e, "zero counts");
    }
    int lay = LAY_COMPACT;
    if (!strip_ok(g, mode, &lay)) {
        if (lists) return fail(OBG_EINVAL, "internal: frame lists need the LDS kernels");
        if (mode & MODE_OCC) {
            if ((e = launch_fill_u32(occ, occ_words, 0u, st)) != hipSuccess) return hip_fail(e, "zero occupancy");
        }
        GenericArgs a{};
        a.rgb = rgb;
        a.frame_pitch = g.frame_pitch;
        a.row_pitch = g.row_pitch;
        a.width = g.width;
        a.height = g.height;
        a.n_frames = n_frames;
        a.depth = g.depth;
        a.region_w = g.region_w;
        a.region_h = g.region_h;
        a.reg_cols = g.reg_cols;
        a.n_regions = g.n_regions;
        a.mask_row_words = g.mask_row_words;
        a.leaf = leaf;
        a.mask = mask;
        a.occ = occ;
        a.counts = counts;
        if ((e = launch_generic(mode, a, st)) != hipSuccess) return hip_fail(e, "generic kernel launch");
        return OBG_OK;
    }
    StripArgs a{};
    a.rgb = rgb;
    a.frame_pitch = g.frame_pitch;
    a.row_pitch = g.row_pitch;
    a.width = g.width;
    a.height = g.height;
    a.n_frames = n_frames;
    a.gpr = 4 * g.mask_row_words;
    a.strip_rows = g.region_h ? g.region_h : g.height;
    if (a.strip_rows > g.height) a.strip_rows = g.height;
    a.n_strips = (g.height + a.strip_rows - 1) / a.strip_rows;
    a.reg_cols = g.reg_cols;
    a.n_regions = g.n_regions;
    a.div_gpr = make_fastdiv((uint32_t)a.gpr);
    a.div_tile = make_fastdiv(g.region_w ? (uint32_t)(g.region_w / 16) : (uint32_t)a.gpr);
    const int cus = cu_count();
    // rows of regions cut into chunks of whole region columns
    a.chunk_cols = g.reg_cols;
    a.n_chunks = 1;
    a.cgpr = a.cgpr_last = a.gpr;
    if (g.reg_cols > 1) {
        a.chunk_cols = region_chunk_cols(g, mode, lay, (int64_t)a.n_strips * n_frames, 2LL * cus);
        a.n_chunks = (g.reg_cols + a.chunk_cols - 1) / a.chunk_cols;
        if (a.n_chunks > 1) {
            a.cgpr = a.chunk_cols * (g.region_w / 16);
            a.cgpr_last = a.gpr - (a.n_chunks - 1) * a.cgpr;
            if (a.cgpr % 4 || a.cgpr_last % 4 || a.cgpr_last < 1 || a.cgpr_last > a.cgpr)
                return fail(OBG_EINVAL, "internal: bad region chunk (%d columns)", a.chunk_cols);
        }
        if ((int64_t)a.n_strips * a.n_chunks > 0x7FFFFFFF) return fail(OBG_EINVAL, "too many regions");
        a.n_strips *= a.n_chunks;
    }
    a.div_cgpr = make_fastdiv((uint32_t)a.cgpr);
    a.div_cgpr_last = make_fastdiv((uint32_t)a.cgpr_last);
    const int64_t groups_strip = (int64_t)a.strip_rows * a.cgpr;
    if ((int64_t)a.strip_rows * a.gpr > (1LL << 30)) return fail(OBG_EINVAL, "frame too large");
    const bool occ_only = (mode & MODE_MASK) == 0;
    const int64_t n_sf = (int64_t)a.n_strips * n_frames;
    // with regions, passes that build occupancy take one work item per
    // (frame, chunk) when there are enough of them
    const bool region_items = lists || ((mode & MODE_OCC) && g.reg_cols > 1 && 2 * n_sf >= (int64_t)cus &&
                                        tune(OBG_TUNE_REGION_CHUNKS, 1) == 1);
    // classify: large tables leave room for few workgroups per CU; 512-thread
    // groups keep the CU at its 32 waves with 4 of them.  Small region items
    // (a single 4K frame: about 1000 groups each) run faster in 256-thread
    // groups (measured: 18 vs 27 us per frame for trees, 33 vs 35 us fused)
    const bool small_items = region_items && groups_strip < 2048;
    const int block = occ_only ? tune(OBG_TUNE_TRAIN_BLOCK, small_items ? 256 : 1024)
                               : tune(OBG_TUNE_CLASSIFY_BLOCK, small_items ? 256 : 512);
    if (occ_only && block != 256 && block != 1024) return fail(OBG_EINVAL, "train block size must be 256 or 1024");
    if (!occ_only && block != 256 && block != 512) return fail(OBG_EINVAL, "classify block size must be 256 or 512");
    const size_t lds = strip_lds_bytes(g.depth, mode, a.chunk_cols, lay);
    // workgroups per CU: LDS and the 32 waves of a CU bound it
    int per_cu = lds ? (int)((160 * 1024) / lds) : 32;
    const int wave_cap = 32 / (block / 64);
    if (per_cu > wave_cap) per_cu = wave_cap;
    if (per_cu < 1) per_cu = 1;
    int64_t spans;
    int64_t target;
    bool store = false;
    if (region_items) {
        // one work item per (frame, chunk): enough of them, and each one's
        // occupancy words are written by one workgroup, so they are stored
        // (no zero fill, no atomics)
        target = (int64_t)cus * std::min(per_cu, tune(OBG_TUNE_OCC_WG_PER_CU, block == 1024 ? 2 : 4));
        spans = 1;
        store = true;
    } else if ((mode & MODE_MASK) && (mode & MODE_OCC) && g.reg_cols == 1) {
        // fused classify + occupancy without regions: items of at most
        // kMaxStageGroups groups, whose masks are staged in LDS and written
        // as one run each; a segment's occupancy flush is 1024 words at d = 5
        // against 4096 x 16 pixels (measured on 1000 frames of the 1080p
        // stream: 1.35 ms against 1.44 ms for two whole frames per workgroup
        // with masks written word by word)
        int want = tune(OBG_TUNE_OCC_WG_PER_CU, 4);
        if (want > per_cu) want = per_cu;
        target = (int64_t)cus * want;
        const int64_t fspan = tune(OBG_TUNE_FUSED_SPAN, kMaxStageGroups);
        spans = (groups_strip + fspan - 1) / fspan;
    } else if (mode & MODE_OCC) {
        // each (frame, strip) segment of a workgroup costs one LDS flush:
        // few, large items
        int want = tune(OBG_TUNE_OCC_WG_PER_CU, block == 1024 ? 2 : 4);
        if (want > per_cu) want = per_cu;
        target = (int64_t)cus * want;
        // items per (frame, strip): workgroups take contiguous runs of items,
        // so with n items the busiest one reads ceil(n / target) of them; pick
        // the split whose busiest workgroup reads the least, and among nearly
        // equal ones the fewest items (each segment change costs a flush)
        const int64_t cap = std::max<int64_t>(1, (groups_strip + block - 1) / block);
        const int64_t s0 = std::min<int64_t>(cap, std::max<int64_t>(1, (target + n_sf - 1) / n_sf));
        spans = s0;
        double best = 1e300;
        for (int64_t sp = s0; sp <= std::min<int64_t>(cap, s0 * kOccItemsPerWg); ++sp) {
            const int64_t n = n_sf * sp;
            const double busiest = (double)((n + target - 1) / target) / (double)sp;   // in segments
            if (busiest < best * 0.98) {
                best = busiest;
                spans = sp;
            }
        }
    } else {
        // measured on 1000 frames of the 1080p stream: two 512-thread groups
        // per CU streaming items round-robin give the highest read+write
        // rate; items of 832 groups beat 512 by 3-11 % at d = 3..5 (5.41-5.51
        // vs 4.95-5.23 TB/s), and compact tables (d = 6, regions) prefer 1024
        int want = tune(OBG_TUNE_CLASSIFY_WG_PER_CU, 2);
        if (want > per_cu) want = per_cu;
        target = (int64_t)cus * want;
        const int64_t span_groups = tune(OBG_TUNE_CLASSIFY_SPAN, lay == LAY_COMPACT ? 1024 : 832);
        spans = (groups_strip + span_groups - 1) / span_groups;
    }
    // spans are whole multiples of 4 groups (one 64-pixel mask word)
    const int64_t span = (((groups_strip + spans - 1) / spans) + 3) & ~(int64_t)3;
    const int64_t n_items = n_sf * spans;
    if (n_items > 0x7FFFFFFF) return fail(OBG_EINVAL, "too many work items (n_frames too large for one call)");
    // one tree per strip: the LDS tables never change between items, so
    // items are dealt round-robin and the workgroups stream through
    // neighbouring memory; with several regions per strip a workgroup keeps
    // a contiguous run of items of the same strip
    a.interleave = (g.reg_cols == 1 && a.n_strips == 1 && !(mode & MODE_OCC))
                       ? (tune(OBG_TUNE_INTERLEAVE, 1) == 1)
                       : (tune(OBG_TUNE_INTERLEAVE, 2) == 1);
    // staging writes an item's mask as one run: whole rows only
    const bool fused_plain = (mode & MODE_MASK) && (mode & MODE_OCC) && !(mode & MODE_COUNTS) && g.reg_cols == 1;
    a.stage_mask = ((mode & MODE_MASK) && span <= (fused_plain ? kMaxStageGroups : kStageGroups) && a.n_chunks == 1)
                       ? (tune(OBG_TUNE_MASK_STAGE, 1) == 1)
                       : 0;
    a.occ_store = store ? 1 : 0;
    // reading before the atomic pays when most pixels find their key's bit
    // already set (measured: 1080p trees 25 % faster at d = 3, even at d = 5
    // and 6; 4K trees 14 % faster at d = 5, 15 % at d = 6; with 32x32 regions
    // at 4K, d = 4: 21 % faster in the fused pass, 3 % slower for trees alone)
    const bool read_first = g.reg_cols == 1 || (mode & MODE_MASK);
    a.occ_test = tune(OBG_TUNE_OCC_BLIND, read_first ? 2 : 1) == 2;
    a.span = (int32_t)span;
    a.spans = (int32_t)spans;
    a.n_items = (int32_t)n_items;
    a.leaf = leaf;
    a.mask = mask;
    a.mask_row_words = g.mask_row_words;
    a.occ = occ;
    a.counts = counts;
    if (lists) {
        a.rgb_list = lists->rgb;
        a.mask_list = lists->mask;
        a.occ_list = lists->occ;
        if (native && lay != LAY_COMPACT) return fail(OBG_EINVAL, "internal: native order needs compact tables");
        a.native = native ? 1 : 0;
    }
    if ((mode & MODE_OCC) && !store) {
        if ((e = launch_fill_u32(occ, occ_words, 0u, st)) != hipSuccess) return hip_fail(e, "zero occupancy");
    }
    const int grid = (int)(n_items < target ? n_items : target);
    // one region per strip: the kernel's tables are static, no dynamic LDS
    const size_t dyn_lds = g.reg_cols > 1 ? lds : 0;
    if ((e = launch_strip(g.depth, mode, a, grid, block, lay, g.reg_cols > 1, dyn_lds, st)) != hipSuccess)
        return hip_fail(e, "strip kernel launch");
    return OBG_OK;
}

}  // namespace

bool obg::pixels_list_ok(const obg_geom *g, int mode) {
    Geo o{};
    int lay = 0;
    if (check_geom(g, &o, true) != OBG_OK) return false;
    // the list kernels are the region ones: several regions per row
    if (o.reg_cols < 2) return false;
    return mode == MODE_OCC || mode == (MODE_MASK | MODE_OCC) ? strip_ok(o, mode, &lay) : false;
}

bool obg::pixels_list_native_ok(const obg_geom *g) {
    Geo o{};
    int lay_occ = 0, lay_both = 0;
    if (check_geom(g, &o, true) != OBG_OK || o.reg_cols < 2) return false;
    if (!strip_ok(o, MODE_OCC, &lay_occ) || !strip_ok(o, MODE_MASK | MODE_OCC, &lay_both)) return false;
    return lay_occ == LAY_COMPACT && lay_both == LAY_COMPACT;
}

int obg::run_pixels_list(const obg_geom *g, int mode, const FrameLists &l, int32_t n_frames, const uint32_t *leaf,
                    hipStream_t stream, bool native) {
    Geo o{};
    int rc = check_geom(g, &o, true);
    if (rc != OBG_OK) return rc;
    if (mode != MODE_OCC && mode != (MODE_MASK | MODE_OCC)) return fail(OBG_EINVAL, "internal: frame-list mode");
    if (o.reg_cols < 2) return fail(OBG_EINVAL, "internal: frame lists need several regions per row");
    if (n_frames < 1 || !l.rgb || !l.occ || ((mode & MODE_MASK) && (!l.mask || !leaf)))
        return fail(OBG_EINVAL, "internal: frame lists");
    return run_pixels(o, mode, nullptr, n_frames, leaf, nullptr, nullptr, nullptr, stream, &l, native);
}

extern "C" {

int64_t obg_num_regions(const obg_geom *g) {
    Geo o;
    return check_geom(g, &o, false) == OBG_OK ? o.n_regions : -1;
}

int64_t obg_occ_words(const obg_geom *g) {
    Geo o;
    return check_geom(g, &o, false) == OBG_OK ? (int64_t)o.n_regions * o.words : -1;
}

int64_t obg_mask_words(const obg_geom *g) {
    Geo o;
    return check_geom(g, &o, false) == OBG_OK ? (int64_t)o.height * o.mask_row_words : -1;
}

int obg_train_frame(const obg_geom *g, const uint8_t *rgb, int32_t n_frames, uint32_t *occ,
                    uint32_t *counts, hipStream_t stream) {
    Geo o;
    int rc = check_geom(g, &o, true);
    if (rc) return rc;
    if (n_frames < 0) return fail(OBG_EINVAL, "n_frames < 0");
    if (n_frames == 0) return OBG_OK;
    if (!rgb || !occ) return fail(OBG_EINVAL, "rgb and occ must not be NULL");
    if ((uintptr_t)rgb % 16) return fail(OBG_EALIGN, "rgb must be 16-byte aligned");
    const int mode = MODE_OCC | (counts ? MODE_COUNTS : 0);
    return run_pixels(o, mode, rgb, n_frames, nullptr, nullptr, occ, counts, stream);
}

int obg_merge_groups(const obg_geom *g, const uint32_t *occ_ring, int32_t ring_len, int32_t first,
                     int32_t n_trees, int32_t group, uint32_t thr_num, uint32_t thr_den, uint32_t *leafset,
                     hipStream_t stream) {
    Geo o;
    int rc = check_geom(g, &o, false);
    if (rc) return rc;
    if (!occ_ring || !leafset) return fail(OBG_EINVAL, "occ_ring and leafset must not be NULL");
    if (n_trees < 1) return fail(OBG_EINVAL, "n_trees must be >= 1 (got %d)", n_trees);
    if (n_trees > 65535) return fail(OBG_EINVAL, "n_trees must be <= 65535 (got %d)", n_trees);
    if (ring_len < n_trees) return fail(OBG_EINVAL, "ring_len %d < n_trees %d", ring_len, n_trees);
    if (first < 0 || first >= ring_len) return fail(OBG_EINVAL, "first %d outside [0, ring_len)", first);
    if (group < 1) return fail(OBG_EINVAL, "group must be >= 1 (got %d)", group);
    if (thr_num == 0) return fail(OBG_EINVAL, "thr_num must be >= 1 (a zero threshold keeps paths no tree has)");
    if (thr_den == 0) return fail(OBG_EINVAL, "thr_den must be >= 1");
    const int32_t n_groups = (n_trees + group - 1) / group;
    // smallest count C with C * den >= num * n_groups
    const uint64_t need = (uint64_t)thr_num * (uint64_t)n_groups;
    const uint64_t kmin = (need + thr_den - 1) / thr_den;
    MergeArgs a{};
    a.occ_ring = occ_ring;
    a.ring_len = ring_len;
    a.first = first;
    a.n_trees = n_trees;
    a.group = group;
    a.slot_words = (int64_t)o.n_regions * o.words;
    a.words = o.words;
    a.valid_bits_last = leaf_count(o.depth) < 32 ? leaf_count(o.depth) : 32;
    a.empty = kmin > (uint64_t)n_groups ? 1 : 0;
    a.kmin = a.empty ? 0u : (uint32_t)kmin;
    a.leaf = leafset;
    a.planes = 0;
    while ((1 << a.planes) <= n_groups) ++a.planes;
    hipError_t e = launch_merge(a, stream);
    if (e != hipSuccess) return hip_fail(e, "merge kernel launch");
    return OBG_OK;
}

int obg_merge(const obg_geom *g, const uint32_t *occ_ring, int32_t ring_len, int32_t first,
              int32_t n_trees, uint32_t thr_num, uint32_t thr_den, uint32_t *leafset,
              hipStream_t stream) {
    return obg_merge_groups(g, occ_ring, ring_len, first, n_trees, 1, thr_num, thr_den, leafset, stream);
}

int obg_classify(const obg_geom *g, const uint8_t *rgb, int32_t n_frames, const uint32_t *leafset,
                 uint64_t *mask, uint32_t *occ_out, hipStream_t stream) {
    Geo o;
    int rc = check_geom(g, &o, true);
    if (rc) return rc;
    if (n_frames < 0) return fail(OBG_EINVAL, "n_frames < 0");
    if (n_frames == 0) return OBG_OK;
    if (!rgb || !leafset || !mask) return fail(OBG_EINVAL, "rgb, leafset and mask must not be NULL");
    if ((uintptr_t)rgb % 16) return fail(OBG_EALIGN, "rgb must be 16-byte aligned");
    const int mode = MODE_MASK | (occ_out ? MODE_OCC : 0);
    return run_pixels(o, mode, rgb, n_frames, leafset, mask, occ_out, nullptr, stream);
}

int obg_quantize(const obg_geom *g, const uint8_t *rgb, int32_t n_frames, uint8_t *out, hipStream_t stream) {
    Geo o;
    int rc = check_geom(g, &o, true);
    if (rc) return rc;
    if (n_frames < 0) return fail(OBG_EINVAL, "n_frames < 0");
    if (n_frames == 0) return OBG_OK;
    if (!rgb || !out) return fail(OBG_EINVAL, "rgb and out must not be NULL");
    if ((uintptr_t)rgb % 16 || (uintptr_t)out % 16) return fail(OBG_EALIGN, "rgb and out must be 16-byte aligned");
    const uintptr_t a0 = (uintptr_t)rgb, a1 = a0 + (uintptr_t)n_frames * (uintptr_t)o.frame_pitch;
    const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (uintptr_t)n_frames * (uintptr_t)o.frame_pitch;
    if (a0 != b0 && a0 < b1 && b0 < a1) return fail(OBG_EINVAL, "rgb and out overlap without being the same buffer");
    QuantArgs a{};
    a.rgb = rgb;
    a.out = out;
    a.frame_pitch = o.frame_pitch;
    a.row_pitch = o.row_pitch;
    a.width = o.width;
    a.height = o.height;
    a.n_frames = n_frames;
    a.depth = o.depth;
    hipError_t e = launch_quantize(a, stream);
    if (e != hipSuccess) return hip_fail(e, "quantize kernel launch");
    return OBG_OK;
}

int obg_score(const obg_geom *g, const uint64_t *mask, const uint64_t *truth, int32_t n_frames, uint64_t *counts,
              hipStream_t stream) {
    Geo o;
    int rc = check_geom(g, &o, false);
    if (rc) return rc;
    if (n_frames < 0) return fail(OBG_EINVAL, "n_frames < 0");
    if (!counts) return fail(OBG_EINVAL, "counts must not be NULL");
    if (n_frames > 0 && (!mask || !truth)) return fail(OBG_EINVAL, "mask and truth must not be NULL");
    if ((uintptr_t)mask % 8 || (uintptr_t)truth % 8 || (uintptr_t)counts % 8)
        return fail(OBG_EALIGN, "mask, truth and counts must be 8-byte aligned");
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(counts), 6, 0u, stream);
    if (e == hipSuccess)
        e = launch_score(mask, truth, (int64_t)n_frames * o.height, o.mask_row_words, o.width,
                         reinterpret_cast<unsigned long long *>(counts), stream);
    if (e != hipSuccess) return hip_fail(e, "score kernel launch");
    return OBG_OK;
}

int obg_tune_set(int key, int value) {
    if (key < 0 || key >= OBG_TUNE_COUNT) return fail(OBG_EINVAL, "unknown tuning key %d", key);
    if (value < 0) return fail(OBG_EINVAL, "tuning value must be >= 0");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = value;
    return OBG_OK;
}

int obg_tune_get(int key) {
    if (key < 0 || key >= OBG_TUNE_COUNT) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune[key];
}

const char *obg_last_error(void) { return g_err.c_str(); }

const char *obg_version(void) { return "obg 0.1 gfx950"; }

}  // extern "C"
