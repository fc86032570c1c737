// batch.hip -- many streams of uneven geometry, depth, training length and
// threshold in one persistent launch per step.
//
// A batch has three steps, each one launch over all streams:
//   train     per-frame trees (occupancy bitsets) of every training frame
//             (Algorithm 1 with the pruning of Section 2);
//   merge     the leaf set of every stream from all of its training trees
//             (Algorithm 2, closed form);
//   classify  the foreground mask of every test frame (Algorithm 3).
// Work items are (stream, frame, span of 16-pixel groups); a workgroup takes
// a contiguous run of items, so it keeps one stream's leaf table in LDS for
// many items.  The steps (plus the zeroing of the occupancy outputs) are
// captured once in a HIP graph and replayed by obg_batch_run.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/obg.h"
#include "strip_core.h"

namespace obg {

// Largest LDS table of one tree: d = 6 compact (8192 words); d = 5 wide is 7968.
constexpr int kBatchTableWords = 8192;

struct BatchStreamDev {
    StripArgs a;              // geometry of the stream's frames (one region)
    const uint8_t *train_rgb, *test_rgb;
    uint32_t *occ, *leaf;
    uint64_t *mask;
    int32_t depth;
    int32_t n_train, n_test;
    int32_t groups;           // 16-pixel groups per frame: height * gpr
    int32_t tspans, tspan;    // training frames: items per frame, groups per item
    int32_t cspans, cspan;    // test frames
    int64_t titem0, citem0;   // the stream's first item in each step
    uint32_t kmin;
    int32_t planes, empty, words, valid_bits;
};

struct BatchArgs {
    const BatchStreamDev *streams;
    int32_t n_streams;
    int64_t n_items;
    int32_t interleave;
    int32_t stage_mask;
};

// Item `it` belongs to the last stream whose first item is <= it.  A
// workgroup's next item is nearly always in the stream of its last one
// (`hint`), which is checked first: the search is a chain of dependent loads
// that would cost about as much as streaming a small item.
template <int MODE>
__device__ __forceinline__ int stream_of(const BatchArgs &b, int64_t it, int hint = -1) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    if (hint >= 0) {
        const BatchStreamDev &h = b.streams[hint];
        const int64_t first = MASK ? h.citem0 : h.titem0;
        const int64_t n = MASK ? (int64_t)h.cspans * h.n_test : (int64_t)h.tspans * h.n_train;
        if (it >= first && it < first + n) return hint;
    }
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

// Work item `local` of stream sd: the frame and the groups it covers.
template <int D, int LAY, int MODE, int BLOCK>
__device__ __forceinline__ void item_body(const BatchArgs &b, const BatchStreamDev &sd, int64_t local,
                                          uint32_t *tab, uint16_t *st_mask, bool new_stream) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr bool OCC = (MODE & MODE_OCC) != 0;
    constexpr int LW = lds_words(D, LAY);
    const int tid = threadIdx.x;
    const StripArgs a = sd.a;
    const int spans = MASK ? sd.cspans : sd.tspans;
    const int span = MASK ? sd.cspan : sd.tspan;
    const int f = (int)(local / spans);
    const int t = (int)(local - (int64_t)f * spans);
    if (MASK && new_stream) {
        __syncthreads();
        leaf_to_lds<D, LAY>(sd.leaf, tab, 1, tid, BLOCK);
    }
    if (OCC) {
        __syncthreads();
        for (int i = tid; i < LW; i += BLOCK) tab[i] = 0;
        __syncthreads();
    }
    const int gb = t * span;
    const int ge = min(gb + span, sd.groups);
    const uint8_t *rgb = MASK ? sd.test_rgb : sd.train_rgb;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(rgb + (int64_t)f * a.frame_pitch, (uint32_t)a.frame_pitch);
    __amdgpu_buffer_rsrc_t ms = make_rsrc(nullptr, 0);
    if (MASK)
        ms = make_rsrc(sd.mask + (int64_t)f * a.height * a.mask_row_words,
                       (uint32_t)a.height * (uint32_t)a.mask_row_words * 8u);
    uint16_t *stage = (MASK && b.stage_mask) ? st_mask : nullptr;
    span_loop<D, MODE, LAY, false, BLOCK>(a, rs, ms, gb, ge, tab, tab, nullptr, stage);
    if (OCC) {
        __syncthreads();
        occ_from_lds<D, LAY>(tab, sd.occ + (int64_t)f * sd.words, 1, tid, BLOCK);
    }
}

// One call per (depth, order) in the one-launch kernel: each depth's code
// gets its own register allocation (all six inlined take 187 VGPRs, two
// waves per SIMD); the price is a call per item that saves 12 VGPRs to the
// stack.
template <int D, int LAY, int MODE, int BLOCK>
__device__ __attribute__((noinline)) void batch_item(const BatchArgs &b, const BatchStreamDev &sd, int64_t local,
                                           uint32_t *tab, uint16_t *st_mask, bool new_stream) {
    item_body<D, LAY, MODE, BLOCK>(b, sd, local, tab, st_mask, new_stream);
}

// The streams of one depth (b.streams points at the first of them, items
// numbered from 0 over them): the item code inlined, the LDS table sized for
// the depth.
template <int D, int LAY, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void batch_depth_kernel(BatchArgs b) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    __shared__ uint32_t tab[lds_words(D, LAY)];
    __shared__ uint16_t st_mask[MASK ? kStageGroups : 4];
    int64_t i0, i1, istep;
    if (b.interleave) {
        i0 = blockIdx.x;
        i1 = b.n_items;
        istep = gridDim.x;
    } else {
        i0 = b.n_items * blockIdx.x / gridDim.x;
        i1 = b.n_items * (blockIdx.x + 1) / gridDim.x;
        istep = 1;
    }
    int cur = -1;
    for (int64_t it = i0; it < i1; it += istep) {
        const int s = stream_of<MODE>(b, it, cur);
        const BatchStreamDev &sd = b.streams[s];
        const int64_t local = it - (MASK ? sd.citem0 : sd.titem0);
        item_body<D, LAY, MODE, BLOCK>(b, sd, local, tab, st_mask, s != cur);
        cur = s;
    }
}

template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void batch_kernel(BatchArgs b) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    __shared__ uint32_t tab[kBatchTableWords];
    __shared__ uint16_t st_mask[MASK ? kStageGroups : 4];
    int64_t i0, i1, istep;
    if (b.interleave) {
        i0 = blockIdx.x;
        i1 = b.n_items;
        istep = gridDim.x;
    } else {
        i0 = b.n_items * blockIdx.x / gridDim.x;
        i1 = b.n_items * (blockIdx.x + 1) / gridDim.x;
        istep = 1;
    }
    int cur = -1;
    for (int64_t it = i0; it < i1; it += istep) {
        const int s = stream_of<MODE>(b, it, cur);
        const BatchStreamDev &sd = b.streams[s];
        const int64_t local = it - (MASK ? sd.citem0 : sd.titem0);
        const bool fresh = s != cur;
        switch (sd.depth) {
            case 1: batch_item<1, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 2: batch_item<2, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 3: batch_item<3, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 4: batch_item<4, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            case 5: batch_item<5, LAY_WIDE, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
            default: batch_item<6, LAY_COMPACT, MODE, BLOCK>(b, sd, local, tab, st_mask, fresh); break;
        }
        cur = s;
    }
}

// Merge of every stream: block row y = stream, one thread per 32 keys.
__global__ __launch_bounds__(256) void batch_merge_kernel(const BatchStreamDev *streams) {
    const BatchStreamDev &sd = streams[blockIdx.y];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= sd.words) return;
    sd.leaf[i] = merge_word(sd.occ, sd.n_train, 0, sd.n_train, sd.words, i, sd.valid_bits, sd.kmin,
                            sd.planes, sd.empty);
}

// Zero every stream's occupancy output (block row y = stream).
__global__ __launch_bounds__(256) void batch_zero_kernel(const BatchStreamDev *streams) {
    const BatchStreamDev &sd = streams[blockIdx.y];
    const int64_t n = (int64_t)sd.n_train * sd.words;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sd.occ[i] = 0;
}

// Order-independent checksum of every output word (autotuner cross-check).
// Each word is mixed with its stream, its kind and its position before a
// non-linear finaliser, so a word written to the wrong place (or the wrong
// stream) changes the sum.
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
    const uint64_t base = (uint64_t)blockIdx.y << 42;   // stream; kind in bits 40..41
    unsigned long long h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nm; i += (int64_t)gridDim.x * blockDim.x)
        h += check_mix(sd.mask[i], base + (uint64_t)i);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < no; i += (int64_t)gridDim.x * blockDim.x)
        h += check_mix(sd.occ[i], base + (1ull << 40) + (uint64_t)i);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < sd.words; i += (int64_t)gridDim.x * blockDim.x)
        h += check_mix(sd.leaf[i], base + (2ull << 40) + (uint64_t)i);
    atomicAdd(out, h);
}

}  // namespace obg

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

// Streams of one depth: [s0, s1) of the (depth-sorted) descriptors.
struct DepthGroup {
    int depth, s0, s1;
    int64_t train_items, classify_items;   // with per-depth launches
};

}  // namespace

struct obg_batch {
    int device = 0;
    int n_streams = 0;
    int cus = 256;
    std::vector<obg_stream_desc> desc;
    std::vector<BatchStreamDev> h;        // sorted by depth
    std::vector<DepthGroup> groups;
    BatchStreamDev *d = nullptr;
    unsigned long long *d_sum = nullptr;
    int64_t train_items = 0, classify_items = 0;
    int64_t px_train = 0, px_test = 0;
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

// Split every frame into work items for the current shape and upload the
// descriptors.
int plan_items(obg_batch *b) {
    int64_t tgroups = 0;
    for (const auto &h : b->h) tgroups += (int64_t)h.groups * h.n_train;
    const int64_t train_wgs = (int64_t)b->cus * b->shape.train_wpc;
    // training items: about train_items_per_wg per workgroup, whole frames
    // when they are small enough (one LDS flush per item)
    int64_t tspan_target = tgroups / std::max<int64_t>(1, train_wgs * b->shape.train_items_per_wg);
    tspan_target = std::max<int64_t>(tspan_target, 4096);
    // item numbers run over all streams (one launch per phase) or restart at
    // each depth group (one launch per depth)
    int64_t t0 = 0, c0 = 0, tt = 0, ct = 0;
    for (auto &gr : b->groups) {
        if (b->shape.per_depth) t0 = c0 = 0;
        const int64_t gt = t0, gc = c0;
        for (int s = gr.s0; s < gr.s1; ++s) {
            BatchStreamDev &h = b->h[s];
            int64_t ts = (std::min<int64_t>(tspan_target, h.groups) + 3) & ~int64_t(3);
            h.tspans = (int32_t)((h.groups + ts - 1) / ts);
            h.tspan = (int32_t)((((h.groups + h.tspans - 1) / h.tspans) + 3) & ~3);
            int64_t cs = (std::min<int64_t>(b->shape.classify_span, h.groups) + 3) & ~int64_t(3);
            h.cspans = (int32_t)((h.groups + cs - 1) / cs);
            h.cspan = (int32_t)((((h.groups + h.cspans - 1) / h.cspans) + 3) & ~3);
            h.titem0 = t0;
            h.citem0 = c0;
            t0 += (int64_t)h.tspans * h.n_train;
            c0 += (int64_t)h.cspans * h.n_test;
        }
        gr.train_items = t0 - gt;
        gr.classify_items = c0 - gc;
        tt += gr.train_items;
        ct += gr.classify_items;
    }
    b->train_items = tt;
    b->classify_items = ct;
    hipError_t e = hipMemcpy(b->d, b->h.data(), sizeof(BatchStreamDev) * b->h.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bfail(OBG_EHIP, "descriptor upload: %s", hipGetErrorString(e));
    return OBG_OK;
}

template <int D, int LAY>
hipError_t launch_depth(obg_batch *b, const DepthGroup &gr, bool train, hipStream_t st) {
    const Shape &sh = b->shape;
    const BatchStreamDev *d = b->d + gr.s0;
    const int n = gr.s1 - gr.s0;
    if (train) {
        BatchArgs a{d, n, gr.train_items, 0, 0};
        const int grid = (int)std::min<int64_t>(gr.train_items, (int64_t)b->cus * sh.train_wpc);
        if (sh.train_block == 1024)
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_OCC, 1024>), dim3(grid), dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_OCC, 256>), dim3(grid), dim3(256), 0, st, a);
    } else {
        BatchArgs a{d, n, gr.classify_items, sh.classify_rr, sh.classify_span <= kStageGroups ? 1 : 0};
        const int grid = (int)std::min<int64_t>(gr.classify_items, (int64_t)b->cus * sh.classify_wpc);
        if (sh.classify_block == 512)
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_MASK, 512>), dim3(grid), dim3(512), 0, st, a);
        else
            hipLaunchKernelGGL((batch_depth_kernel<D, LAY, MODE_MASK, 256>), dim3(grid), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

// One launch per depth group of the phase (train or classify).
hipError_t enqueue_depths(obg_batch *b, bool train, hipStream_t st) {
    for (const DepthGroup &gr : b->groups) {
        if ((train ? gr.train_items : gr.classify_items) <= 0) continue;
        hipError_t e;
        switch (gr.depth) {
            case 1: e = launch_depth<1, LAY_WIDE>(b, gr, train, st); break;
            case 2: e = launch_depth<2, LAY_WIDE>(b, gr, train, st); break;
            case 3: e = launch_depth<3, LAY_WIDE>(b, gr, train, st); break;
            case 4: e = launch_depth<4, LAY_WIDE>(b, gr, train, st); break;
            case 5: e = launch_depth<5, LAY_WIDE>(b, gr, train, st); break;
            default: e = launch_depth<6, LAY_COMPACT>(b, gr, train, st); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t enqueue(obg_batch *b, hipStream_t st) {
    const int ny = b->n_streams;
    hipLaunchKernelGGL(batch_zero_kernel, dim3(64, ny), dim3(256), 0, st, (const BatchStreamDev *)b->d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b->shape.per_depth) {
        if ((e = enqueue_depths(b, true, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(batch_merge_kernel, dim3((b->max_words + 255) / 256, ny), dim3(256), 0, st,
                           (const BatchStreamDev *)b->d);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return enqueue_depths(b, false, st);
    }
    if (b->train_items > 0) {
        BatchArgs a{b->d, ny, b->train_items, 0, 0};
        const int grid = (int)std::min<int64_t>(b->train_items, (int64_t)b->cus * b->shape.train_wpc);
        if (b->shape.train_block == 1024)
            hipLaunchKernelGGL((batch_kernel<MODE_OCC, 1024>), dim3(grid), dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL((batch_kernel<MODE_OCC, 256>), dim3(grid), dim3(256), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(batch_merge_kernel, dim3((b->max_words + 255) / 256, ny), dim3(256), 0, st,
                       (const BatchStreamDev *)b->d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (b->classify_items > 0) {
        // round-robin: the items in flight at any moment are neighbours in
        // memory, and items are numbered stream by stream, so a workgroup
        // reloads a leaf table only where its items cross into the next
        // stream; contiguous runs meet each stream's table once
        BatchArgs a{b->d, ny, b->classify_items, b->shape.classify_rr,
                    b->shape.classify_span <= kStageGroups ? 1 : 0};
        const int grid = (int)std::min<int64_t>(b->classify_items, (int64_t)b->cus * b->shape.classify_wpc);
        if (b->shape.classify_block == 512)
            hipLaunchKernelGGL((batch_kernel<MODE_MASK, 512>), dim3(grid), dim3(512), 0, st, a);
        else
            hipLaunchKernelGGL((batch_kernel<MODE_MASK, 256>), dim3(grid), dim3(256), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

void drop_graph(obg_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int build_graph(obg_batch *b) {
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(OBG_EHIP, "begin capture: %s", hipGetErrorString(e));
    hipError_t le = enqueue(b, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess) return bfail(OBG_EHIP, "launch during capture: %s", hipGetErrorString(le));
    if (e != hipSuccess) return bfail(OBG_EHIP, "end capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(OBG_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    return OBG_OK;
}

int run_once(obg_batch *b, hipStream_t st) {
    hipError_t e;
    if (b->use_graph && b->exec)
        e = hipGraphLaunch(b->exec, st);
    else
        e = enqueue(b, st);
    if (e != hipSuccess) return bfail(OBG_EHIP, "batch launch: %s", hipGetErrorString(e));
    return OBG_OK;
}

int checksum(obg_batch *b, hipStream_t st, unsigned long long *out) {
    hipError_t e = hipMemsetAsync(b->d_sum, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return bfail(OBG_EHIP, "checksum: %s", hipGetErrorString(e));
    hipLaunchKernelGGL(batch_checksum_kernel, dim3(256, b->n_streams), dim3(256), 0, st,
                       (const BatchStreamDev *)b->d, b->d_sum);
    if ((e = hipGetLastError()) != hipSuccess) return bfail(OBG_EHIP, "checksum: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(out, b->d_sum, sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bfail(OBG_EHIP, "checksum: %s", hipGetErrorString(e));
    return OBG_OK;
}

int time_shape(obg_batch *b, hipStream_t st, float *ms) {
    int rc = plan_items(b);
    if (rc) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return bfail(OBG_EHIP, "event create");
    rc = run_once(b, st);  // warm-up
    float best = 1e30f;
    for (int r = 0; r < 3 && rc == OBG_OK; ++r) {
        (void)hipEventRecord(e0, st);
        rc = run_once(b, st);
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

int autotune(obg_batch *b, hipStream_t st) {
    const Shape base = b->shape;
    float best_ms = 0;
    int rc = time_shape(b, st, &best_ms);
    if (rc) return rc;
    unsigned long long ref = 0;
    if ((rc = checksum(b, st, &ref))) return rc;
    b->tune_default_ms = best_ms;
    Shape best = base;
    int n = 0;
    // one launch per phase or per depth and phase, with the default shape
    {
        Shape s = best;
        s.per_depth = !base.per_depth;
        b->shape = s;
        float ms = 0;
        if ((rc = time_shape(b, st, &ms))) return rc;
        unsigned long long h = 0;
        if ((rc = checksum(b, st, &h))) return rc;
        if (h != ref) return bfail(OBG_EHIP, "autotune: shape gives different output (internal error)");
        ++n;
        if (ms < best_ms) { best_ms = ms; best = s; }
    }
    const int cblocks[] = {256, 512}, cwpcs[] = {1, 2, 4}, cspans[] = {256, 512, 832, 1024, 4096};
    const int tblocks[] = {256, 1024}, twpcs[] = {1, 2, 4}, titems[] = {1, 4};
    for (int cb : cblocks)
        for (int cw : cwpcs)
            for (int cs : cspans)
                for (int rr = 0; rr < 2; ++rr) {
                    Shape s = best;
                    s.classify_block = cb; s.classify_wpc = cw; s.classify_span = cs; s.classify_rr = rr;
                    if (cb == 512 && cw > 2) continue;   // 32 waves per CU at most
                    b->shape = s;
                    float ms = 0;
                    if ((rc = time_shape(b, st, &ms))) return rc;
                    unsigned long long h = 0;
                    if ((rc = checksum(b, st, &h))) return rc;
                    if (h != ref) return bfail(OBG_EHIP, "autotune: shape gives different output (internal error)");
                    ++n;
                    if (ms < best_ms) { best_ms = ms; best = s; }
                }
    for (int tb : tblocks)
        for (int tw : twpcs)
            for (int ti : titems) {
                Shape s = best;
                s.train_block = tb; s.train_wpc = tw; s.train_items_per_wg = ti;
                if (tb == 1024 && tw > 2) continue;
                b->shape = s;
                float ms = 0;
                if ((rc = time_shape(b, st, &ms))) return rc;
                unsigned long long h = 0;
                if ((rc = checksum(b, st, &h))) return rc;
                if (h != ref) return bfail(OBG_EHIP, "autotune: shape gives different output (internal error)");
                ++n;
                if (ms < best_ms) { best_ms = ms; best = s; }
            }
    b->shape = best;
    b->tune_best_ms = best_ms;
    b->tune_candidates = n;
    return plan_items(b);
}

void destroy(obg_batch *b) {
    if (!b) return;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->d) (void)hipFree(b->d);
    if (b->d_sum) (void)hipFree(b->d_sum);
    delete b;
}

}  // namespace

extern "C" {

int obg_batch_create(const obg_stream_desc *streams, int32_t n_streams, uint32_t flags, hipStream_t stream,
                     obg_batch **out) {
    if (!out) return bfail(OBG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!streams || n_streams < 1) return bfail(OBG_EINVAL, "need at least one stream");
    if (flags & ~(uint32_t)(OBG_BATCH_AUTOTUNE | OBG_BATCH_NO_GRAPH)) return bfail(OBG_EINVAL, "unknown flags");
    obg_batch *b = new obg_batch();
    b->n_streams = n_streams;
    b->desc.assign(streams, streams + n_streams);
    for (int s = 0; s < n_streams; ++s) {
        const obg_stream_desc &sd = streams[s];
        const obg_geom &g = sd.geom;
        if (g.width < 1 || g.height < 1 || g.depth < 1 || g.depth > 6) {
            destroy(b);
            return bfail(OBG_EINVAL, "stream %d: width, height >= 1 and depth in [1, 6] required", s);
        }
        if (g.region_w || g.region_h) { destroy(b); return bfail(OBG_EINVAL, "stream %d: regions are not batched", s); }
        if (g.row_pitch < 3LL * g.width || g.frame_pitch < (int64_t)g.height * g.row_pitch || g.frame_pitch > 0x7FFFFFFFLL) {
            destroy(b);
            return bfail(OBG_EINVAL, "stream %d: bad pitches", s);
        }
        if (g.row_pitch % 16 || g.frame_pitch % 16 || (uintptr_t)sd.train_rgb % 16 || (uintptr_t)sd.test_rgb % 16) {
            destroy(b);
            return bfail(OBG_EALIGN, "stream %d: frames and pitches must be 16-byte aligned", s);
        }
        if (sd.n_train < 1 || sd.n_train > 65535 || sd.n_test < 0) {
            destroy(b);
            return bfail(OBG_EINVAL, "stream %d: n_train in [1, 65535] and n_test >= 0 required", s);
        }
        if (sd.thr_num == 0 || sd.thr_den == 0) { destroy(b); return bfail(OBG_EINVAL, "stream %d: zero threshold", s); }
        if (!sd.train_rgb || !sd.occ || !sd.leafset || (sd.n_test > 0 && (!sd.test_rgb || !sd.mask))) {
            destroy(b);
            return bfail(OBG_EINVAL, "stream %d: NULL buffer", s);
        }
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
        a.occ_test = tune(OBG_TUNE_OCC_BLIND, g.depth <= 5 ? 2 : 1) == 2;
        a.mask_row_words = (g.width + 63) / 64;
        if ((int64_t)g.height * a.gpr > (1LL << 30)) { destroy(b); return bfail(OBG_EINVAL, "stream %d: frame too large", s); }
        h.groups = g.height * a.gpr;
        h.train_rgb = sd.train_rgb;
        h.test_rgb = sd.test_rgb;
        h.occ = sd.occ;
        h.leaf = sd.leafset;
        h.mask = sd.mask;
        h.depth = g.depth;
        h.n_train = sd.n_train;
        h.n_test = sd.n_test;
        h.words = leaf_words(g.depth);
        h.valid_bits = leaf_count(g.depth) < 32 ? leaf_count(g.depth) : 32;
        const uint64_t need = (uint64_t)sd.thr_num * (uint64_t)sd.n_train;
        const uint64_t kmin = (need + sd.thr_den - 1) / sd.thr_den;
        h.empty = kmin > (uint64_t)sd.n_train ? 1 : 0;
        h.kmin = h.empty ? 0u : (uint32_t)kmin;
        h.planes = 0;
        while ((1 << h.planes) <= sd.n_train) ++h.planes;
        b->max_words = std::max(b->max_words, h.words);
        b->px_train += (int64_t)g.width * g.height * sd.n_train;
        b->px_test += (int64_t)g.width * g.height * sd.n_test;
        b->h.push_back(h);
    }
    // descriptors sorted by depth (outputs are addressed through them, so the
    // order is free): each depth's streams are one contiguous group
    std::stable_sort(b->h.begin(), b->h.end(),
                     [](const BatchStreamDev &x, const BatchStreamDev &y) { return x.depth < y.depth; });
    for (int s = 0; s < n_streams; ++s) {
        if (b->groups.empty() || b->groups.back().depth != b->h[s].depth)
            b->groups.push_back(DepthGroup{b->h[s].depth, s, s, 0, 0});
        b->groups.back().s1 = s + 1;
    }
    // every descriptor is valid: only now touch the device
    if (hipGetDevice(&b->device) != hipSuccess) { destroy(b); return bfail(OBG_EHIP, "no device"); }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
        b->cus = cus;
    hipError_t e = hipMalloc(&b->d, sizeof(BatchStreamDev) * n_streams);
    if (e == hipSuccess) e = hipMalloc(&b->d_sum, sizeof(unsigned long long));
    if (e != hipSuccess) { destroy(b); return bfail(OBG_ENOMEM, "descriptor allocation: %s", hipGetErrorString(e)); }
    b->shape = Shape{256, 4, 4, 512, 2, 832, 1, tune(OBG_TUNE_BATCH_PER_DEPTH, 1) == 2 ? 1 : 0};
    int rc = plan_items(b);
    if (rc == OBG_OK && (flags & OBG_BATCH_AUTOTUNE)) rc = autotune(b, stream);
    if (rc == OBG_OK && !(flags & OBG_BATCH_NO_GRAPH)) {
        if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
            rc = bfail(OBG_EHIP, "capture stream");
        else if ((rc = build_graph(b)) == OBG_OK)
            b->use_graph = true;
    }
    if (rc != OBG_OK) {
        destroy(b);
        return rc;
    }
    *out = b;
    return OBG_OK;
}

int obg_batch_run(obg_batch *b, hipStream_t stream) {
    if (!b) return bfail(OBG_EINVAL, "batch is NULL");
    return run_once(b, stream);
}

int obg_batch_info_get(const obg_batch *b, obg_batch_info *out) {
    if (!b || !out) return bfail(OBG_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->n_streams = b->n_streams;
    out->train_items = b->train_items;
    out->classify_items = b->classify_items;
    out->pixels_train = b->px_train;
    out->pixels_test = b->px_test;
    out->train_block = b->shape.train_block;
    out->train_wg_per_cu = b->shape.train_wpc;
    out->train_items_per_wg = b->shape.train_items_per_wg;
    out->classify_block = b->shape.classify_block;
    out->classify_wg_per_cu = b->shape.classify_wpc;
    out->classify_span = b->shape.classify_span;
    out->classify_round_robin = b->shape.classify_rr;
    out->per_depth_launches = b->shape.per_depth;
    out->graph = b->use_graph ? 1 : 0;
    out->tune_candidates = b->tune_candidates;
    out->tune_default_ms = b->tune_default_ms;
    out->tune_best_ms = b->tune_best_ms;
    return OBG_OK;
}

void obg_batch_destroy(obg_batch *b) { destroy(b); }

}  // extern "C"
