// batch.hip -- the batched form: one plan over many streams of uneven
// geometry, depth, training length and threshold, run on work items that the
// caller passes in device memory.
//
// A run has three steps, each one persistent launch over all streams (or one
// per depth present, when the autotuner finds that faster):
//   train     per-frame trees (occupancy bitsets) of every training frame
//             (Algorithm 1 with the pruning of Section 2);
//   merge     the leaf set of every stream from all of its training trees
//             (Algorithm 2, closed form);
//   classify  the foreground mask of every test frame (Algorithm 3).
// The plan fixes each stream's geometry, depth and threshold, and the launch
// shape.  A run's work items (a device array) name the streams that take
// part and give their frames, frame counts and output buffers.  A one-block
// prepare kernel turns the items into the plan's device descriptors: per
// stream its buffers and counts, the first work item of each step, and the
// item total of every launch.  The three steps read everything from those
// descriptors, so they are captured once in a HIP graph at plan creation and
// the same graph serves every run.
//
// Work items of a step are (stream, frame, span of 16-pixel groups); a
// workgroup takes a contiguous run of them (or every grid-th one), so it
// keeps one stream's leaf table in LDS for many items.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/obg.h"
#include "strip_core.h"

namespace obg {

// Largest LDS table of one tree: d = 6 compact (8192 words); d = 5 wide is 7968.
constexpr int kBatchTableWords = 8192;
constexpr int kDepthGroups = 6;           // depths 1..6, one group each at most
constexpr int kPrepareBlock = 1024;
constexpr int kPlanMaxStreams = 8192;     // claims of one run live in LDS
// item totals: [2 * g] train and [2 * g + 1] classify items of depth group g,
// [2 * kDepthGroups (+1)] of all streams
constexpr int kTotals = 2 * kDepthGroups + 2;

struct BatchStreamDev {
    StripArgs a;              // geometry of the stream's frames (one region)
    // fixed by the plan and its launch shape
    int32_t stream;           // plan stream held by this slot (slots are sorted by depth)
    int32_t depth, group;     // depth and index of its depth group
    int32_t groups;           // 16-pixel groups per frame: height * gpr
    int32_t tspans, tspan;    // training frames: items per frame, groups per item
    int32_t cspans, cspan;    // test frames
    FastDiv div_tspans, div_cspans;
    int32_t words, valid_bits;
    uint32_t thr_num, thr_den;
    int32_t max_train, max_test;
    // written by the prepare kernel of each run
    int32_t n_train, n_test;
    const uint8_t *train_rgb, *test_rgb;
    uint32_t *occ, *leaf;
    uint64_t *mask;
    int64_t titem0, citem0;   // the slot's first item in its launch of each step
    uint32_t kmin;
    int32_t planes, empty;
};

struct BatchArgs {
    const BatchStreamDev *streams;   // the launch's first slot
    int32_t n_streams;
    const int64_t *n_items;          // the launch's item count, written by the prepare kernel
    int32_t interleave;
    int32_t stage_mask;
};

// Item `it` belongs to the last slot whose first item is <= it (a slot
// without items has the first item of the next slot, so that slot is never
// the answer).
template <int MODE>
__device__ __forceinline__ int stream_of(const BatchArgs &b, int64_t it) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    int lo = 0, hi = b.n_streams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t first = MASK ? b.streams[mid].citem0 : b.streams[mid].titem0;
        if (first <= it)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// What a work item needs of its stream, read once when a workgroup's items
// reach the stream and kept in registers while they stay on it (items are
// numbered stream by stream, so a workgroup's next item is nearly always in
// the stream of its last one).  Reading the slot again for every item puts a
// chain of dependent loads between the items, which for the classify items of
// one 1080p stream cost about a third of the time.
struct ItemStream {
    StripArgs a;                  // geometry (only the pixel code's fields are kept)
    int64_t first, count;         // the stream's items in this launch: [first, first + count)
    FastDiv div_spans;            // divides by the items per frame
    int32_t spans, span, groups, words;
    int32_t single;               // one item per training frame: its tree is stored whole
    const uint8_t *rgb;
    uint64_t *mask;
    uint32_t *occ;
    const uint32_t *leaf;
};

template <int MODE>
__device__ __forceinline__ ItemStream load_stream(const BatchStreamDev &sd) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    ItemStream c;
    c.a = sd.a;
    c.first = MASK ? sd.citem0 : sd.titem0;
    c.count = MASK ? (int64_t)sd.cspans * sd.n_test : (int64_t)sd.tspans * sd.n_train;
    c.div_spans = MASK ? sd.div_cspans : sd.div_tspans;
    c.spans = MASK ? sd.cspans : sd.tspans;
    c.span = MASK ? sd.cspan : sd.tspan;
    c.groups = sd.groups;
    c.words = sd.words;
    c.single = sd.tspans == 1;
    c.rgb = MASK ? sd.test_rgb : sd.train_rgb;
    c.mask = sd.mask;
    c.occ = sd.occ;
    c.leaf = sd.leaf;
    return c;
}

// Work item `local` of stream cs: the frame and the groups it covers.  A
// training frame that is one item writes its tree with plain stores; frames
// cut into several items OR their words into a zeroed tree.
template <int D, int LAY, int MODE, int BLOCK>
__device__ __forceinline__ void item_body(const BatchArgs &b, const ItemStream &cs, int64_t local,
                                          uint32_t *tab, uint16_t *st_mask, bool new_stream) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr bool OCC = (MODE & MODE_OCC) != 0;
    constexpr int LW = lds_words(D, LAY);
    const int tid = threadIdx.x;
    const StripArgs &a = cs.a;
    int f, t;
    if (local <= 0xFFFFFFFFll) {
        f = (int)fdiv((uint32_t)local, cs.div_spans);
        t = (int)((uint32_t)local - (uint32_t)f * (uint32_t)cs.spans);
    } else {
        f = (int)(local / cs.spans);
        t = (int)(local - (int64_t)f * cs.spans);
    }
    if (MASK && new_stream) {
        __syncthreads();
        leaf_to_lds<D, LAY>(cs.leaf, tab, 1, tid, BLOCK);
    }
    if (OCC) {
        __syncthreads();
        for (int i = tid; i < LW; i += BLOCK) tab[i] = 0;
        __syncthreads();
    }
    const int gb = t * cs.span;
    const int ge = min(gb + cs.span, cs.groups);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(cs.rgb + (int64_t)f * a.frame_pitch, (uint32_t)a.frame_pitch);
    __amdgpu_buffer_rsrc_t ms = make_rsrc(nullptr, 0);
    if (MASK)
        ms = make_rsrc(cs.mask + (int64_t)f * a.height * a.mask_row_words,
                       (uint32_t)a.height * (uint32_t)a.mask_row_words * 8u);
    uint16_t *stage = (MASK && b.stage_mask) ? st_mask : nullptr;
    span_loop<D, MODE, LAY, false, BLOCK>(a, rs, ms, gb, ge, tab, tab, nullptr, stage);
    if (OCC) {
        __syncthreads();
        occ_from_lds<D, LAY>(tab, cs.occ + (int64_t)f * cs.words, 1, tid, BLOCK, cs.single != 0);
    }
}

// The items [i0, i1) (every istep-th) of one launch, the item code of every
// depth reached through `body` (with the stream's depth).
template <int MODE, typename Body>
__device__ __forceinline__ void walk_items(const BatchArgs &b, Body body) {
    const int64_t n_items = *b.n_items;
    int64_t i0, i1, istep;
    if (b.interleave) {
        i0 = blockIdx.x;
        i1 = n_items;
        istep = gridDim.x;
    } else {
        i0 = n_items * blockIdx.x / gridDim.x;
        i1 = n_items * (blockIdx.x + 1) / gridDim.x;
        istep = 1;
    }
    ItemStream cs{};
    const BatchStreamDev *slot = nullptr;
    for (int64_t it = i0; it < i1; it += istep) {
        bool fresh = false;
        if (!slot || it < cs.first || it >= cs.first + cs.count) {
            slot = &b.streams[stream_of<MODE>(b, it)];
            cs = load_stream<MODE>(*slot);
            fresh = true;
        }
        body(cs, *slot, it - cs.first, fresh);
    }
}

// One call per (depth, order) in the one-launch kernel: each depth's code
// gets its own register allocation (all six inlined take 187 VGPRs, two
// waves per SIMD); the price is a call per item that saves 12 VGPRs to the
// stack.  The callee reads the stream's fields from its slot (a copy passed
// to a call would live on the stack).
template <int D, int LAY, int MODE, int BLOCK>
__device__ __attribute__((noinline)) void batch_item(const BatchArgs &b, const BatchStreamDev &sd, int64_t local,
                                                     uint32_t *tab, uint16_t *st_mask, bool new_stream) {
    const ItemStream cs = load_stream<MODE>(sd);
    item_body<D, LAY, MODE, BLOCK>(b, cs, local, tab, st_mask, new_stream);
}

// The streams of one depth (b.streams points at the first of them, items
// numbered from 0 over them): the item code inlined, the LDS table sized for
// the depth.
template <int D, int LAY, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void batch_depth_kernel(BatchArgs b) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    __shared__ uint32_t tab[lds_words(D, LAY)];
    __shared__ uint16_t st_mask[MASK ? kStageGroups : 4];
    walk_items<MODE>(b, [&](const ItemStream &cs, const BatchStreamDev &, int64_t local, bool fresh) {
        item_body<D, LAY, MODE, BLOCK>(b, cs, local, tab, st_mask, fresh);
    });
}

template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void batch_kernel(BatchArgs b) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    __shared__ uint32_t tab[kBatchTableWords];
    __shared__ uint16_t st_mask[MASK ? kStageGroups : 4];
    walk_items<MODE>(b, [&](const ItemStream &, const BatchStreamDev &sd, int64_t local, bool fresh) {
        switch (sd.depth) {
            case 1: batch_item<1, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 2: batch_item<2, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 3: batch_item<3, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 4: batch_item<4, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 5: batch_item<5, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            default: batch_item<6, LAY_COMPACT, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
        }
    });
}

// Merge of every stream that trained in this run: block row y = slot, 64
// words (2048 keys) to a workgroup.
__global__ __launch_bounds__(kMergeBlock) void batch_merge_kernel(const BatchStreamDev *streams) {
    __shared__ uint32_t part[(kMergeWaves - 1) * 16 * 64];
    const BatchStreamDev &sd = streams[blockIdx.y];
    const int64_t w0 = blockIdx.x * (int64_t)64;
    if (sd.n_train < 1 || w0 >= sd.words) return;
    merge_block(sd.occ, sd.n_train, 0, sd.n_train, sd.words, sd.words, w0, sd.valid_bits, sd.kmin, sd.planes,
                sd.empty, 1, sd.leaf, part);
}

// Zero the trees of training frames cut into several items (block row y =
// slot); single-item frames store their trees whole.
__global__ __launch_bounds__(256) void batch_zero_kernel(const BatchStreamDev *streams) {
    const BatchStreamDev &sd = streams[blockIdx.y];
    if (sd.tspans < 2) return;
    const int64_t n = (int64_t)sd.n_train * sd.words;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sd.occ[i] = 0;
}

// ---------------------------------------------------------------------------
// The prepare kernel: one workgroup turns a run's work items into the slots'
// per-run fields and the launches' item counts.

struct PrepareArgs {
    BatchStreamDev *d;
    int32_t n;                 // slots (= plan streams)
    const int32_t *slot_of;    // plan stream -> slot
    int64_t *totals;           // [kTotals]
    int32_t per_depth;         // items numbered per depth group (one launch per depth)
    int32_t n_groups;
};

__device__ __forceinline__ int item_check(const obg_work_item &it, const BatchStreamDev *d, const int32_t *slot_of,
                                          int n) {
    if (it.stream < 0 || it.stream >= n) return OBG_ITEM_BAD_STREAM;
    const BatchStreamDev &s = d[slot_of[it.stream]];
    if (it.n_train < 0 || it.n_train > s.max_train || it.n_test < 0 || it.n_test > s.max_test)
        return OBG_ITEM_BAD_COUNT;
    if (it.n_train == 0 && it.n_test == 0) return OBG_ITEM_OK;
    if (!it.leafset || (it.n_train > 0 && (!it.train_rgb || !it.occ)) || (it.n_test > 0 && (!it.test_rgb || !it.mask)))
        return OBG_ITEM_NULL;
    const uintptr_t a16 = (it.n_train > 0 ? (uintptr_t)it.train_rgb : 0) | (it.n_test > 0 ? (uintptr_t)it.test_rgb : 0);
    const uintptr_t a4 = (uintptr_t)it.leafset | (it.n_train > 0 ? (uintptr_t)it.occ : 0);
    const uintptr_t a8 = it.n_test > 0 ? (uintptr_t)it.mask : 0;
    if ((a16 & 15) || (a4 & 3) || (a8 & 7)) return OBG_ITEM_ALIGN;
    return OBG_ITEM_OK;
}

__global__ __launch_bounds__(kPrepareBlock) void plan_prepare_kernel(PrepareArgs p, obg_work_item *items,
                                                                      int32_t n_items) {
    __shared__ int32_t claim[kPlanMaxStreams];
    __shared__ int64_t sc_t[kPrepareBlock], sc_c[kPrepareBlock];
    __shared__ int64_t g0_t[kDepthGroups + 1], g0_c[kDepthGroups + 1];
    const int tid = threadIdx.x;
    for (int s = tid; s < p.n; s += kPrepareBlock) {
        p.d[s].n_train = 0;
        p.d[s].n_test = 0;
        claim[s] = INT_MAX;
    }
    __syncthreads();
    // each stream is taken by the first item that names it
    for (int i = tid; i < n_items; i += kPrepareBlock) {
        const obg_work_item it = items[i];
        if (item_check(it, p.d, p.slot_of, p.n) == OBG_ITEM_OK) atomicMin(&claim[p.slot_of[it.stream]], i);
    }
    __syncthreads();
    for (int i = tid; i < n_items; i += kPrepareBlock) {
        const obg_work_item it = items[i];
        int st = item_check(it, p.d, p.slot_of, p.n);
        if (st == OBG_ITEM_OK) {
            const int slot = p.slot_of[it.stream];
            if (claim[slot] != i) {
                st = OBG_ITEM_DUPLICATE;
            } else {
                BatchStreamDev &sd = p.d[slot];
                sd.n_train = it.n_train;
                sd.n_test = it.n_test;
                sd.train_rgb = it.train_rgb;
                sd.test_rgb = it.test_rgb;
                sd.occ = it.occ;
                sd.leaf = it.leafset;
                sd.mask = it.mask;
                // keep a key iff count * den >= num * n_train: the smallest such count
                const uint64_t need = (uint64_t)sd.thr_num * (uint64_t)it.n_train;
                const uint64_t kmin = (need + sd.thr_den - 1) / sd.thr_den;
                sd.empty = kmin > (uint64_t)it.n_train ? 1 : 0;
                sd.kmin = sd.empty ? 0u : (uint32_t)kmin;
                int planes = 0;
                while ((1 << planes) <= it.n_train) ++planes;
                sd.planes = planes;
            }
        }
        items[i].status = st;
    }
    __syncthreads();
    // first items: a scan over the slots (each thread a contiguous chunk)
    const int ch = (p.n + kPrepareBlock - 1) / kPrepareBlock;
    const int s0 = min(p.n, tid * ch), s1 = min(p.n, s0 + ch);
    int64_t lt = 0, lc = 0;
    for (int s = s0; s < s1; ++s) {
        lt += (int64_t)p.d[s].tspans * p.d[s].n_train;
        lc += (int64_t)p.d[s].cspans * p.d[s].n_test;
    }
    sc_t[tid] = lt;
    sc_c[tid] = lc;
    __syncthreads();
    for (int off = 1; off < kPrepareBlock; off <<= 1) {
        const int64_t vt = tid >= off ? sc_t[tid - off] : 0;
        const int64_t vc = tid >= off ? sc_c[tid - off] : 0;
        __syncthreads();
        sc_t[tid] += vt;
        sc_c[tid] += vc;
        __syncthreads();
    }
    int64_t rt = sc_t[tid] - lt, rc = sc_c[tid] - lc;
    for (int s = s0; s < s1; ++s) {
        BatchStreamDev &sd = p.d[s];
        sd.titem0 = rt;
        sd.citem0 = rc;
        if (s == 0 || p.d[s - 1].group != sd.group) {
            g0_t[sd.group] = rt;
            g0_c[sd.group] = rc;
        }
        rt += (int64_t)sd.tspans * sd.n_train;
        rc += (int64_t)sd.cspans * sd.n_test;
    }
    if (tid == 0) {
        g0_t[p.n_groups] = sc_t[kPrepareBlock - 1];
        g0_c[p.n_groups] = sc_c[kPrepareBlock - 1];
    }
    __syncthreads();
    if (p.per_depth) {
        for (int s = s0; s < s1; ++s) {
            p.d[s].titem0 -= g0_t[p.d[s].group];
            p.d[s].citem0 -= g0_c[p.d[s].group];
        }
    }
    if (tid < p.n_groups) {
        p.totals[2 * tid] = g0_t[tid + 1] - g0_t[tid];
        p.totals[2 * tid + 1] = g0_c[tid + 1] - g0_c[tid];
    }
    if (tid == 0) {
        p.totals[2 * kDepthGroups] = g0_t[p.n_groups];
        p.totals[2 * kDepthGroups + 1] = g0_c[p.n_groups];
    }
}

// Order-independent checksum of every output word of a run (autotuner
// cross-check).  Each word is mixed with its stream, its kind and its
// position before a non-linear finaliser, so a word written to the wrong
// place (or the wrong stream) changes the sum.
__device__ __forceinline__ unsigned long long check_mix(uint64_t word, uint64_t where) {
    uint64_t x = word ^ (where * 0x9E3779B97F4A7C15ull);
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ __launch_bounds__(256) void batch_checksum_kernel(const BatchStreamDev *streams, unsigned long long *out) {
    const BatchStreamDev &sd = streams[blockIdx.y];
    const int64_t nm = (int64_t)sd.n_test * sd.a.height * sd.a.mask_row_words;
    const int64_t no = (int64_t)sd.n_train * sd.words;
    const int64_t nl = sd.n_train > 0 ? sd.words : 0;
    const uint64_t base = (uint64_t)sd.stream << 42;   // stream; kind in bits 40..41
    unsigned long long h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nm; i += (int64_t)gridDim.x * blockDim.x)
        h += check_mix(sd.mask[i], base + (uint64_t)i);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < no; i += (int64_t)gridDim.x * blockDim.x)
        h += check_mix(sd.occ[i], base + (1ull << 40) + (uint64_t)i);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nl; i += (int64_t)gridDim.x * blockDim.x)
        h += check_mix(sd.leaf[i], base + (2ull << 40) + (uint64_t)i);
    atomicAdd(out, h);
}

// Device memory of the no-allocation run: the slots, the plan-stream -> slot
// map and the launch item counts of at most kNoAllocStreams streams.  Every
// GPU the library runs on holds its own copy until the process ends.
constexpr int kNoAllocStreams = OBG_NOALLOC_MAX_STREAMS;
struct NoAllocLayout {
    BatchStreamDev slots[kNoAllocStreams];
    int32_t slot_of[kNoAllocStreams];
    int64_t totals[kTotals];
};

}  // namespace obg

// The no-allocation run's buffer (host code uses its address from
// hipGetSymbolAddress, never this name).
static __device__ __align__(256) uint64_t scratch[(sizeof(obg::NoAllocLayout) + 7) / 8];

using namespace obg;

namespace {

int bfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

struct Shape {
    int train_block, train_wpc, train_items_per_wg;
    int classify_block, classify_wpc, classify_span;
    int classify_rr;          // 1: classify items dealt round-robin, 0: contiguous runs
    int per_depth;            // 1: one launch per depth and phase, 0: one launch per phase
};

// Classify items of a stream of depth d: the shape's span, twice that with the
// compact table of d = 6 (as in one-stream calls; the 64-stream mix, untuned:
// 22.6-22.8 against 23.0-23.6 ms).  The longest items of a launch decide
// whether its masks are staged, so the one-launch form asks for the span of
// the deepest stream.
constexpr int kCompactDepth = 6;
inline int64_t classify_span_of(const Shape &sh, int d) {
    return (d >= kCompactDepth ? 2 : 1) * (int64_t)sh.classify_span;
}

// Streams of one depth: slots [s0, s1).
struct DepthGroup {
    int depth, s0, s1;
    int64_t max_train_items, max_classify_items;   // when every stream runs its maxima
};

}  // namespace

struct obg_plan {
    int device = 0;
    int n_streams = 0;
    int cus = 256;
    std::vector<BatchStreamDev> h;        // slots, sorted by depth
    std::vector<int32_t> slot_of;         // plan stream -> slot
    std::vector<DepthGroup> groups;
    BatchStreamDev *d = nullptr;
    int32_t *d_slot_of = nullptr;
    int64_t *d_totals = nullptr;
    unsigned long long *d_sum = nullptr;
    int64_t max_train_items = 0, max_classify_items = 0;
    int max_words = 0;
    Shape shape{};
    bool use_graph = false;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double tune_best_ms = 0, tune_default_ms = 0;
    int tune_candidates = 0;
};

namespace {

// Split every stream's frames into work items for the current shape (host
// copies of the slots only).
void split_items(obg_plan *p) {
    int64_t all_groups = 0;
    for (const auto &h : p->h) all_groups += (int64_t)h.groups * h.max_train;
    const int64_t train_wgs = (int64_t)p->cus * p->shape.train_wpc;
    p->max_train_items = p->max_classify_items = 0;
    for (auto &gr : p->groups) {
        // training items: about train_items_per_wg per workgroup of the
        // launch that runs them when every stream trains on its most frames
        // (with one launch per depth, that depth's frames: each launch has
        // the whole grid), whole frames when they are small enough.  Items
        // are dealt to workgroups by count, so they should be of about one
        // size: a frame far larger than the others' items is cut.  At least
        // 4096 groups, and 4 groups per tree word (each item flushes its
        // tree once: at most about 2 % of its pixel bytes)
        int64_t tgroups = all_groups;
        if (p->shape.per_depth) {
            tgroups = 0;
            for (int s = gr.s0; s < gr.s1; ++s) tgroups += (int64_t)p->h[s].groups * p->h[s].max_train;
        }
        int64_t tspan_target = tgroups / std::max<int64_t>(1, train_wgs * p->shape.train_items_per_wg);
        tspan_target = std::max<int64_t>(tspan_target, std::max<int64_t>(4096, 4 * (int64_t)leaf_words(gr.depth)));
        gr.max_train_items = gr.max_classify_items = 0;
        for (int s = gr.s0; s < gr.s1; ++s) {
            BatchStreamDev &h = p->h[s];
            int64_t ts = (std::min<int64_t>(tspan_target, h.groups) + 3) & ~int64_t(3);
            h.tspans = (int32_t)((h.groups + ts - 1) / ts);
            h.tspan = (int32_t)((((h.groups + h.tspans - 1) / h.tspans) + 3) & ~3);
            int64_t cs = (std::min<int64_t>(classify_span_of(p->shape, gr.depth), h.groups) + 3) & ~int64_t(3);
            h.cspans = (int32_t)((h.groups + cs - 1) / cs);
            h.cspan = (int32_t)((((h.groups + h.cspans - 1) / h.cspans) + 3) & ~3);
            h.div_tspans = make_fastdiv((uint32_t)h.tspans);
            h.div_cspans = make_fastdiv((uint32_t)h.cspans);
            gr.max_train_items += (int64_t)h.tspans * h.max_train;
            gr.max_classify_items += (int64_t)h.cspans * h.max_test;
        }
        p->max_train_items += gr.max_train_items;
        p->max_classify_items += gr.max_classify_items;
    }
}

// Split the work for the current shape and upload the slots (their per-run
// fields are the prepare kernel's).
int plan_items(obg_plan *p) {
    split_items(p);
    hipError_t e = hipMemcpy(p->d, p->h.data(), sizeof(BatchStreamDev) * p->h.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bfail(OBG_EHIP, "descriptor upload: %s", hipGetErrorString(e));
    return OBG_OK;
}

template <int D, int LAY>
hipError_t launch_depth(obg_plan *p, int g, bool train, hipStream_t st) {
    const Shape &sh = p->shape;
    const DepthGroup &gr = p->groups[g];
    const BatchStreamDev *d = p->d + gr.s0;
    const int n = gr.s1 - gr.s0;
    if (train) {
        BatchArgs a{d, n, p->d_totals + 2 * g, 0, 0};
        const int grid = (int)std::min<int64_t>(gr.max_train_items, (int64_t)p->cus * sh.train_wpc);
        if (sh.train_block == 1024)
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_OCC, 1024>), dim3(grid), dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_OCC, 256>), dim3(grid), dim3(256), 0, st, a);
    } else {
        BatchArgs a{d, n, p->d_totals + 2 * g + 1, sh.classify_rr, classify_span_of(sh, D) <= kStageGroups ? 1 : 0};
        const int grid = (int)std::min<int64_t>(gr.max_classify_items, (int64_t)p->cus * sh.classify_wpc);
        if (sh.classify_block == 512)
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_MASK, 512>), dim3(grid), dim3(512), 0, st, a);
        else
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_MASK, 256>), dim3(grid), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

// One launch per depth group of the phase (train or classify).
hipError_t enqueue_depths(obg_plan *p, bool train, hipStream_t st) {
    for (int g = 0; g < (int)p->groups.size(); ++g) {
        const DepthGroup &gr = p->groups[g];
        if ((train ? gr.max_train_items : gr.max_classify_items) <= 0) continue;
        hipError_t e;
        switch (gr.depth) {
            case 1: e = launch_depth<1, LAY_WIDE>(p, g, train, st); break;
            case 2: e = launch_depth<2, LAY_WIDE>(p, g, train, st); break;
            case 3: e = launch_depth<3, LAY_WIDE>(p, g, train, st); break;
            case 4: e = launch_depth<4, LAY_WIDE>(p, g, train, st); break;
            case 5: e = launch_depth<5, LAY_WIDE>(p, g, train, st); break;
            default: e = launch_depth<6, LAY_COMPACT>(p, g, train, st); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The three steps of a run (what the graph holds); they read the slots and
// item counts the prepare kernel wrote.
hipError_t enqueue_steps(obg_plan *p, hipStream_t st) {
    const int ny = p->n_streams;
    hipLaunchKernelGGL(batch_zero_kernel, dim3(64, ny), dim3(256), 0, st, (const BatchStreamDev *)p->d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p->shape.per_depth) {
        if ((e = enqueue_depths(p, true, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(batch_merge_kernel, dim3((p->max_words + 63) / 64, ny), dim3(kMergeBlock), 0, st,
                           (const BatchStreamDev *)p->d);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return enqueue_depths(p, false, st);
    }
    if (p->max_train_items > 0) {
        BatchArgs a{p->d, ny, p->d_totals + 2 * kDepthGroups, 0, 0};
        const int grid = (int)std::min<int64_t>(p->max_train_items, (int64_t)p->cus * p->shape.train_wpc);
        if (p->shape.train_block == 1024)
            hipLaunchKernelGGL((batch_kernel<MODE_OCC, 1024>), dim3(grid), dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL((batch_kernel<MODE_OCC, 256>), dim3(grid), dim3(256), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(batch_merge_kernel, dim3((p->max_words + 63) / 64, ny), dim3(kMergeBlock), 0, st,
                       (const BatchStreamDev *)p->d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p->max_classify_items > 0) {
        // round-robin: the items in flight at any moment are neighbours in
        // memory, and items are numbered stream by stream, so a workgroup
        // reloads a leaf table only where its items cross into the next
        // stream; contiguous runs meet each stream's table once
        int deepest = 1;
        for (const DepthGroup &gr : p->groups) deepest = std::max(deepest, gr.depth);
        BatchArgs a{p->d, ny, p->d_totals + 2 * kDepthGroups + 1, p->shape.classify_rr,
                    classify_span_of(p->shape, deepest) <= kStageGroups ? 1 : 0};
        const int grid = (int)std::min<int64_t>(p->max_classify_items, (int64_t)p->cus * p->shape.classify_wpc);
        if (p->shape.classify_block == 512)
            hipLaunchKernelGGL((batch_kernel<MODE_MASK, 512>), dim3(grid), dim3(512), 0, st, a);
        else
            hipLaunchKernelGGL((batch_kernel<MODE_MASK, 256>), dim3(grid), dim3(256), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t enqueue_prepare(obg_plan *p, const obg_work_item *items, int32_t n_items, hipStream_t st) {
    PrepareArgs a{p->d, p->n_streams, p->d_slot_of, p->d_totals, p->shape.per_depth, (int32_t)p->groups.size()};
    hipLaunchKernelGGL(plan_prepare_kernel, dim3(1), dim3(kPrepareBlock), 0, st, a,
                       const_cast<obg_work_item *>(items), n_items);
    return hipGetLastError();
}

void drop_graph(obg_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

int build_graph(obg_plan *p) {
    drop_graph(p);
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(OBG_EHIP, "begin capture: %s", hipGetErrorString(e));
    hipError_t le = enqueue_steps(p, p->cap);
    e = hipStreamEndCapture(p->cap, &p->graph);
    if (le != hipSuccess) return bfail(OBG_EHIP, "launch during capture: %s", hipGetErrorString(le));
    if (e != hipSuccess) return bfail(OBG_EHIP, "end capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(OBG_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    return OBG_OK;
}

int run_once(obg_plan *p, const obg_work_item *items, int32_t n_items, hipStream_t st, bool graph) {
    hipError_t e = enqueue_prepare(p, items, n_items, st);
    if (e == hipSuccess) e = (graph && p->exec) ? hipGraphLaunch(p->exec, st) : enqueue_steps(p, st);
    if (e != hipSuccess) return bfail(OBG_EHIP, "batch launch: %s", hipGetErrorString(e));
    return OBG_OK;
}

int checksum(obg_plan *p, hipStream_t st, unsigned long long *out) {
    hipError_t e = hipMemsetAsync(p->d_sum, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return bfail(OBG_EHIP, "checksum: %s", hipGetErrorString(e));
    hipLaunchKernelGGL(batch_checksum_kernel, dim3(256, p->n_streams), dim3(256), 0, st,
                       (const BatchStreamDev *)p->d, p->d_sum);
    if ((e = hipGetLastError()) != hipSuccess) return bfail(OBG_EHIP, "checksum: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(out, p->d_sum, sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bfail(OBG_EHIP, "checksum: %s", hipGetErrorString(e));
    return OBG_OK;
}

int time_shape(obg_plan *p, const obg_work_item *items, int32_t n_items, hipStream_t st, float *ms) {
    int rc = plan_items(p);
    if (rc) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return bfail(OBG_EHIP, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(OBG_EHIP, "event create");
    }
    rc = run_once(p, items, n_items, st, false);  // warm-up
    float best = 1e30f;
    for (int r = 0; r < 3 && rc == OBG_OK; ++r) {
        (void)hipEventRecord(e0, st);
        rc = run_once(p, items, n_items, st, false);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) rc = bfail(OBG_EHIP, "timing sync");
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        best = std::min(best, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return rc;
}

// Time the candidate shapes on the given work, keep the fastest.  Every
// candidate's outputs must hash to the first shape's.
int autotune(obg_plan *p, const obg_work_item *items, int32_t n_items, hipStream_t st) {
    const Shape base = p->shape;
    float best_ms = 0;
    int rc = time_shape(p, items, n_items, st, &best_ms);
    if (rc) return rc;
    unsigned long long ref = 0;
    if ((rc = checksum(p, st, &ref))) return rc;
    p->tune_default_ms = best_ms;
    Shape best = base;
    int n = 0;
    auto trial = [&](const Shape &s) -> int {
        p->shape = s;
        float ms = 0;
        int r = time_shape(p, items, n_items, st, &ms);
        if (r) return r;
        unsigned long long h = 0;
        if ((r = checksum(p, st, &h))) return r;
        if (h != ref) return bfail(OBG_EHIP, "autotune: shape gives different output (internal error)");
        ++n;
        if (ms < best_ms) {
            best_ms = ms;
            best = s;
        }
        return OBG_OK;
    };
    // one launch per phase or per depth and phase, with the default shape
    {
        Shape s = best;
        s.per_depth = !base.per_depth;
        if ((rc = trial(s))) return rc;
    }
    const int cblocks[] = {256, 512}, cwpcs[] = {1, 2, 4}, cspans[] = {256, 512, 832, 1024, 4096};
    const int tblocks[] = {256, 1024}, twpcs[] = {1, 2, 4}, titems[] = {1, 4, 16};
    for (int cb : cblocks)
        for (int cw : cwpcs)
            for (int cs : cspans)
                for (int rr = 0; rr < 2; ++rr) {
                    if (cb == 512 && cw > 2) continue;   // 32 waves per CU at most
                    Shape s = best;
                    s.classify_block = cb;
                    s.classify_wpc = cw;
                    s.classify_span = cs;
                    s.classify_rr = rr;
                    if ((rc = trial(s))) return rc;
                }
    for (int tb : tblocks)
        for (int tw : twpcs)
            for (int ti : titems) {
                if (tb == 1024 && tw > 2) continue;
                Shape s = best;
                s.train_block = tb;
                s.train_wpc = tw;
                s.train_items_per_wg = ti;
                if ((rc = trial(s))) return rc;
            }
    p->shape = best;
    p->tune_best_ms = best_ms;
    p->tune_candidates = n;
    return plan_items(p);
}

void destroy(obg_plan *p) {
    if (!p) return;
    drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->d) (void)hipFree(p->d);
    if (p->d_slot_of) (void)hipFree(p->d_slot_of);
    if (p->d_totals) (void)hipFree(p->d_totals);
    if (p->d_sum) (void)hipFree(p->d_sum);
    delete p;
}

int check_run_args(const obg_plan *p, const obg_work_item *items, int32_t n_items) {
    if (!p) return bfail(OBG_EINVAL, "plan is NULL");
    if (n_items < 0 || n_items > p->n_streams)
        return bfail(OBG_EINVAL, "n_items must be in [0, n_streams = %d] (got %d)", p->n_streams, n_items);
    if (n_items > 0 && !items) return bfail(OBG_EINVAL, "work items are NULL");
    if ((uintptr_t)items % 8) return bfail(OBG_EALIGN, "work items must be 8-byte aligned");
    return OBG_OK;
}

// Validate the stream descriptions and build the plan's host slots (sorted
// by depth), the plan-stream -> slot map and the depth groups.  Host only.
int describe(const obg_plan_stream *streams, int32_t n_streams, obg_plan *p) {
    p->n_streams = n_streams;
    p->h.clear();
    p->slot_of.clear();
    p->groups.clear();
    p->max_words = 0;
    for (int s = 0; s < n_streams; ++s) {
        const obg_plan_stream &ps = streams[s];
        const obg_geom &g = ps.geom;
        if (g.width < 1 || g.height < 1 || g.depth < 1 || g.depth > 6)
            return bfail(OBG_EINVAL, "stream %d: width, height >= 1 and depth in [1, 6] required", s);
        if (g.region_w || g.region_h) return bfail(OBG_EINVAL, "stream %d: regions are not batched", s);
        if (g.row_pitch < 3LL * g.width || g.frame_pitch < (int64_t)g.height * g.row_pitch ||
            g.frame_pitch > 0x7FFFFFFFLL)
            return bfail(OBG_EINVAL, "stream %d: bad pitches", s);
        if (g.row_pitch % 16 || g.frame_pitch % 16)
            return bfail(OBG_EALIGN, "stream %d: pitches must be multiples of 16 bytes", s);
        if (ps.max_train < 0 || ps.max_train > 65535 || ps.max_test < 0)
            return bfail(OBG_EINVAL, "stream %d: max_train in [0, 65535] and max_test >= 0 required", s);
        if (ps.thr_num == 0 || ps.thr_den == 0) return bfail(OBG_EINVAL, "stream %d: zero threshold", s);
        if ((int64_t)g.height * 4 * ((g.width + 63) / 64) > (1LL << 30))
            return bfail(OBG_EINVAL, "stream %d: frame too large", s);
        BatchStreamDev h{};
        StripArgs &a = h.a;
        a.width = g.width;
        a.height = g.height;
        a.row_pitch = g.row_pitch;
        a.frame_pitch = g.frame_pitch;
        a.gpr = 4 * ((g.width + 63) / 64);
        a.strip_rows = g.height;
        a.n_strips = 1;
        a.reg_cols = 1;
        a.n_regions = 1;
        a.div_gpr = make_fastdiv((uint32_t)a.gpr);
        a.div_tile = make_fastdiv((uint32_t)a.gpr);
        // the batched trees at d = 6 run faster with the plain atomic (1.30
        // against 1.52 ms on the 64-stream mix), the one-stream passes and
        // the served form with a read first
        a.occ_test = tune(OBG_TUNE_OCC_BLIND, g.depth <= 5 ? 2 : 1) == 2;
        a.mask_row_words = (g.width + 63) / 64;
        h.stream = s;
        h.depth = g.depth;
        h.groups = g.height * a.gpr;
        h.words = leaf_words(g.depth);
        h.valid_bits = leaf_count(g.depth) < 32 ? leaf_count(g.depth) : 32;
        h.thr_num = ps.thr_num;
        h.thr_den = ps.thr_den;
        h.max_train = ps.max_train;
        h.max_test = ps.max_test;
        p->max_words = std::max(p->max_words, h.words);
        p->h.push_back(h);
    }
    // slots sorted by depth (outputs are addressed through them, so the
    // order is free): each depth's streams are one contiguous group
    std::stable_sort(p->h.begin(), p->h.end(),
                     [](const BatchStreamDev &x, const BatchStreamDev &y) { return x.depth < y.depth; });
    p->slot_of.assign(n_streams, 0);
    for (int s = 0; s < n_streams; ++s) {
        if (p->groups.empty() || p->groups.back().depth != p->h[s].depth)
            p->groups.push_back(DepthGroup{p->h[s].depth, s, s, 0, 0});
        p->groups.back().s1 = s + 1;
        p->h[s].group = (int32_t)p->groups.size() - 1;
        p->slot_of[p->h[s].stream] = s;
    }
    return OBG_OK;
}

// The launch shape a plan starts from: one launch per depth present and
// phase (faster than one launch per phase on one 1080p stream and on the
// 64-stream mix), training items of about a sixteenth of a workgroup's share
// (the 64-stream mix: 22.1 against 23.3 ms with a quarter).
Shape default_shape() { return Shape{256, 4, 16, 512, 2, 832, 1, tune(OBG_TUNE_BATCH_PER_DEPTH, 2) == 2 ? 1 : 0}; }

// Device address of `scratch` on each device, looked up once per device with
// that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

int scratch_address(int dev, NoAllocLayout **out) {
    if (dev < 0 || dev >= kMaxDevices) return bfail(OBG_EHIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return bfail(OBG_EHIP, "address of the no-allocation buffer: %s", hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = static_cast<NoAllocLayout *>(g_scratch[dev]);
    return OBG_OK;
}

}  // namespace

extern "C" {

int obg_plan_create(const obg_plan_stream *streams, int32_t n_streams, obg_plan **out) {
    if (!out) return bfail(OBG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!streams || n_streams < 1) return bfail(OBG_EINVAL, "need at least one stream");
    if (n_streams > kPlanMaxStreams) return bfail(OBG_EINVAL, "at most %d streams per plan", kPlanMaxStreams);
    obg_plan *p = new obg_plan();
    int rc = describe(streams, n_streams, p);
    if (rc != OBG_OK) {
        destroy(p);
        return rc;
    }
    // every description is valid: only now touch the device
    if (hipGetDevice(&p->device) != hipSuccess) {
        destroy(p);
        return bfail(OBG_EHIP, "no device");
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
        p->cus = cus;
    hipError_t e = hipMalloc(&p->d, sizeof(BatchStreamDev) * n_streams);
    if (e == hipSuccess) e = hipMalloc(&p->d_slot_of, sizeof(int32_t) * n_streams);
    if (e == hipSuccess) e = hipMalloc(&p->d_totals, sizeof(int64_t) * kTotals);
    if (e == hipSuccess) e = hipMalloc(&p->d_sum, sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_slot_of, p->slot_of.data(), sizeof(int32_t) * n_streams, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy(p);
        return bfail(OBG_ENOMEM, "plan allocation: %s", hipGetErrorString(e));
    }
    p->shape = default_shape();
    rc = plan_items(p);
    if (rc == OBG_OK && tune(OBG_TUNE_BATCH_GRAPH, 1) == 1) {
        if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
            rc = bfail(OBG_EHIP, "capture stream");
        else if ((rc = build_graph(p)) == OBG_OK)
            p->use_graph = true;
    }
    if (rc != OBG_OK) {
        destroy(p);
        return rc;
    }
    *out = p;
    return OBG_OK;
}

int obg_plan_tune(obg_plan *p, const obg_work_item *items, int32_t n_items, hipStream_t stream) {
    int rc = check_run_args(p, items, n_items);
    if (rc) return rc;
    if (n_items == 0) return OBG_OK;
    if (hipStreamSynchronize(stream) != hipSuccess) return bfail(OBG_EHIP, "tune: stream sync");
    rc = autotune(p, items, n_items, stream);
    if (rc == OBG_OK && p->use_graph) rc = build_graph(p);
    if (rc == OBG_OK && hipStreamSynchronize(stream) != hipSuccess) rc = bfail(OBG_EHIP, "tune: stream sync");
    if (rc != OBG_OK) p->use_graph = false;
    return rc;
}

int obg_batch_run(obg_plan *p, const obg_work_item *items, int32_t n_items, hipStream_t stream) {
    int rc = check_run_args(p, items, n_items);
    if (rc) return rc;
    if (n_items == 0) return OBG_OK;
    return run_once(p, items, n_items, stream, p->use_graph);
}

int obg_batch_run_noalloc(const obg_plan_stream *streams, int32_t n_streams, const obg_work_item *items,
                          int32_t n_items, hipStream_t stream) {
    if (!streams || n_streams < 1) return bfail(OBG_EINVAL, "need at least one stream");
    if (n_streams > kNoAllocStreams)
        return bfail(OBG_EINVAL, "at most %d streams without allocation (got %d)", kNoAllocStreams, n_streams);
    // host copies of the slots: one per thread, reused from call to call
    thread_local obg_plan p;
    int rc = describe(streams, n_streams, &p);
    if (rc == OBG_OK) rc = check_run_args(&p, items, n_items);
    if (rc != OBG_OK || n_items == 0) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return bfail(OBG_EHIP, "no device");
    NoAllocLayout *buf = nullptr;
    if ((rc = scratch_address(dev, &buf)) != OBG_OK) return rc;
    int cus = 0;
    p.cus = (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
                ? cus
                : 256;
    p.device = dev;
    p.shape = default_shape();
    split_items(&p);
    p.d = buf->slots;
    p.d_slot_of = buf->slot_of;
    p.d_totals = buf->totals;
    // the fixed fields of the slots and the slot map; the prepare kernel
    // writes every per-run field and item count, so nothing is cleared first
    hipError_t e = hipMemcpyAsync(p.d, p.h.data(), sizeof(BatchStreamDev) * n_streams, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p.d_slot_of, p.slot_of.data(), sizeof(int32_t) * n_streams, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) rc = run_once(&p, items, n_items, stream, false);
    else rc = bfail(OBG_EHIP, "descriptor upload: %s", hipGetErrorString(e));
    p.d = nullptr;
    p.d_slot_of = nullptr;
    p.d_totals = nullptr;
    return rc;
}

int obg_plan_info_get(const obg_plan *p, obg_plan_info *out) {
    if (!p || !out) return bfail(OBG_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->n_streams = p->n_streams;
    out->max_train_items = p->max_train_items;
    out->max_classify_items = p->max_classify_items;
    out->train_block = p->shape.train_block;
    out->train_wg_per_cu = p->shape.train_wpc;
    out->train_items_per_wg = p->shape.train_items_per_wg;
    out->classify_block = p->shape.classify_block;
    out->classify_wg_per_cu = p->shape.classify_wpc;
    out->classify_span = p->shape.classify_span;
    out->classify_round_robin = p->shape.classify_rr;
    out->per_depth_launches = p->shape.per_depth;
    out->graph = p->use_graph ? 1 : 0;
    out->tune_candidates = p->tune_candidates;
    out->tune_default_ms = p->tune_default_ms;
    out->tune_best_ms = p->tune_best_ms;
    return OBG_OK;
}

void obg_plan_destroy(obg_plan *p) { destroy(p); }

}  // extern "C"
