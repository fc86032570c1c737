// serve.hip -- continuous batching of camera frames on one GPU.
//
// Frames of many streams arrive at their own times.  The host loop admits
// arrived frames as device memory (a budgeted arena) and batch slots free up,
// forms a batch of frames from many streams, and enqueues it on one of
// several HIP streams, so that batches overlap on the device:
//   ingest    the frames' pixels are written into their buffers (callback);
//   frames    one launch over all frames of the batch: training frames
//             write their occupancy into the stream's ring slot (Algorithm 1
//             with the pruning of Section 2); test frames write their mask
//             and their occupancy in the same pass (Algorithm 3, and the
//             frame's tree for later re-merges);
//   merge     the initial model after the training frames, and every
//             `period` test frames a re-merge over the last `window` ring
//             slots (Algorithm 2; Section 4 names an update of the tree but
//             gives no procedure, this is the reading used here).
// Per stream, the order of frames is kept: a merge is enqueued only when no
// other batch of that stream is in flight, it is the stream's last frame in
// its batch, and no frame of the stream is scheduled while its merge is in
// flight.  Every result is therefore the same whether a stream is served
// alone or in the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <thread>
#include <vector>

#include "../../include/obg.h"
#include "serve_sched.h"
#include "strip_core.h"

namespace obg {

// One frame of a batch.
struct ServeFrameDev {
    StripArgs a;              // geometry (one region)
    const uint8_t *rgb;
    uint32_t *occ;            // ring slot of this frame
    uint32_t *leaf;           // the stream's merged leaf set (test frames)
    uint64_t *mask;           // test frames; NULL for training frames
    int32_t depth, groups, words;
    int32_t native;           // ring slot and leaf set in the LDS order (d = 5, 6)
    int32_t whole;            // one workgroup takes the whole frame: its tree is stored, not ORed
    int64_t g0;               // first group of the frame in the batch's group space
};

// A batch is one space of 16-pixel groups: its frames' groups end to end.
// Workgroup w takes groups [bounds[w], bounds[w+1]), whatever frames they
// fall in; the runs are cut so that they cost about the same (split_by_cost),
// and a cut inside a frame is a multiple of 4 groups from its start, so mask
// words never straddle workgroups.
struct ServeArgs {
    const ServeFrameDev *frames;
    int32_t n_frames;
    const int64_t *bounds;    // [grid + 1]
};

struct MergeJobDev {
    const uint32_t *ring;
    uint32_t *leaf;
    int32_t ring_len, first, n_trees, words, valid_bits;
    uint32_t kmin;
    int32_t planes, empty;
};

constexpr int kServeTableWords = 8192;
constexpr int kServeBlock = 512;

// The frame holding group g: the last frame whose first group is <= g.
__device__ __forceinline__ int frame_of(const ServeArgs &b, int64_t g) {
    int lo = 0, hi = b.n_frames - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.frames[mid].g0 <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Groups [gb, ge) of one frame: its occupancy is built in LDS and ORed into the
// frame's ring slot (stored, when this is the whole frame); test frames also
// get their mask bits from the leaf set, in one dual table (leaf and
// occupancy words in pairs), training frames use an occupancy table in the
// same memory.
template <int D, int LAY, int MODE>
__device__ __attribute__((noinline)) void serve_part(const ServeFrameDev &fd, int gb, int ge, uint32_t *tab,
                                                     uint16_t *stage, bool load_leaf) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr int LW = lds_words(D, LAY);
    const int tid = threadIdx.x;
    const StripArgs a = fd.a;
    __syncthreads();   // the previous part's flush has read the table
    if (MASK) {
        if (load_leaf)
            leaf_to_lds<D, LAY, true>(fd.leaf, tab, 1, tid, kServeBlock, fd.native != 0);
        else
            clear_dual_occ(tab, 2 * LW, tid, kServeBlock);
    } else {
        for (int i = tid; i < LW; i += kServeBlock) tab[i] = 0;
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(fd.rgb, (uint32_t)a.frame_pitch);
    __amdgpu_buffer_rsrc_t ms = make_rsrc(nullptr, 0);
    if (MASK) ms = make_rsrc(fd.mask, (uint32_t)a.height * (uint32_t)a.mask_row_words * 8u);
    if (MASK) {
        // masks gathered in LDS and written in runs of up to kMaxStageGroups
        // groups (frame starts and work splits are multiples of 4 groups, so
        // every run starts on a 64-pixel mask word)
        for (int s0 = gb; s0 < ge; s0 += kMaxStageGroups)
            span_loop<D, MODE, LAY, false, kServeBlock>(a, rs, ms, s0, min(s0 + kMaxStageGroups, ge), tab, tab,
                                                        nullptr, stage);
    } else {
        span_loop<D, MODE, LAY, false, kServeBlock>(a, rs, ms, gb, ge, tab, tab, nullptr, nullptr);
    }
    __syncthreads();
    occ_from_lds<D, LAY, MASK>(tab, fd.occ, 1, tid, kServeBlock, fd.whole != 0, fd.native != 0);
}

template <int MODE>
__device__ __forceinline__ void serve_dispatch(const ServeFrameDev &fd, int gb, int ge, uint32_t *tab,
                                               uint16_t *stage, bool load_leaf) {
    switch (fd.depth) {
        case 1: serve_part<1, LAY_WIDE, MODE>(fd, gb, ge, tab, stage, load_leaf); break;
        case 2: serve_part<2, LAY_WIDE, MODE>(fd, gb, ge, tab, stage, load_leaf); break;
        case 3: serve_part<3, LAY_WIDE, MODE>(fd, gb, ge, tab, stage, load_leaf); break;
        case 4: serve_part<4, LAY_WIDE, MODE>(fd, gb, ge, tab, stage, load_leaf); break;
        case 5: serve_part<5, LAY_WIDE, MODE>(fd, gb, ge, tab, stage, load_leaf); break;
        default: serve_part<6, LAY_COMPACT, MODE>(fd, gb, ge, tab, stage, load_leaf); break;
    }
}

// Training frames (occupancy) and test frames (mask and occupancy) of a batch
// in one launch.
__global__ __launch_bounds__(kServeBlock) __attribute__((amdgpu_waves_per_eu(4))) void serve_kernel(ServeArgs b) {
    __shared__ uint32_t tab[2 * kServeTableWords];
    __shared__ uint16_t stage[kMaxStageGroups];
    int64_t g = b.bounds[blockIdx.x];
    const int64_t gend = b.bounds[blockIdx.x + 1];
    if (g >= gend) return;
    int fi = frame_of(b, g);
    const uint32_t *cur_leaf = nullptr;
    while (g < gend && fi < b.n_frames) {
        const ServeFrameDev &fd = b.frames[fi];
        const int lb = (int)(g - fd.g0);
        const int le = (int)min<int64_t>(gend - fd.g0, (int64_t)fd.groups);
        if (fd.mask) {
            serve_dispatch<MODE_MASK | MODE_OCC>(fd, lb, le, tab, stage, fd.leaf != cur_leaf);
            cur_leaf = fd.leaf;
        } else {
            serve_dispatch<MODE_OCC>(fd, lb, le, tab, nullptr, false);
            cur_leaf = nullptr;   // the table no longer holds a leaf set
        }
        g = fd.g0 + le;
        ++fi;
    }
}

// Zero the ring slots that this batch's frames OR their occupancy into (the
// frames that several workgroups share).
__global__ __launch_bounds__(256) void serve_zero_kernel(const ServeFrameDev *frames) {
    const ServeFrameDev &fd = frames[blockIdx.y];
    if (fd.whole) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < fd.words; i += gridDim.x * blockDim.x) fd.occ[i] = 0;
}

// The batch's due merges: block row y = job, 64 words (2048 keys) to a
// workgroup.
__global__ __launch_bounds__(kMergeBlock) void serve_merge_kernel(const MergeJobDev *jobs) {
    __shared__ uint32_t part[(kMergeWaves - 1) * 16 * 64];
    const MergeJobDev &j = jobs[blockIdx.y];
    const int64_t w0 = blockIdx.x * (int64_t)64;
    if (w0 >= j.words) return;
    merge_block(j.ring, j.ring_len, j.first, j.n_trees, j.words, j.words, w0, j.valid_bits, j.kmin, j.planes,
                j.empty, 1, j.leaf, part);
}

// Per test frame: an order-dependent 64-bit hash of its mask words.
__global__ __launch_bounds__(256) void serve_checksum_kernel(const ServeFrameDev *frames, unsigned long long *out) {
    const ServeFrameDev &fd = frames[blockIdx.y];
    const int64_t n = (int64_t)fd.a.height * fd.a.mask_row_words;
    unsigned long long h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        // each word mixed with its position through a non-linear finaliser,
        // so words moved or bits exchanged between words change the sum
        uint64_t x = fd.mask[i] ^ ((uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        h += x ^ (x >> 31);
    }
    atomicAdd(&out[blockIdx.y], h);
}

}  // namespace obg

using namespace obg;

namespace {

using Clock = std::chrono::steady_clock;

// Geometry and table sizes of one stream, as the kernels see them.
struct StreamDev {
    obg_serve_stream cfg{};
    StripArgs a{};
    int words = 0, valid_bits = 32, groups = 0;
    int n_regions = 1;
    bool region = false;      // one tree per region: the region passes serve it
    bool native = false;      // rings and leaf set kept in the LDS order
    obg_geom geom{};          // for those passes
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr, start = nullptr, k0 = nullptr, k1 = nullptr;
    bool busy = false;
    SchedBatch batch;
    std::vector<double> arrival;   // per frame of the batch: wall seconds after the start
    std::vector<int> order;        // launch order of the batch's frames (indices into batch.frames)
    int n_train_plain = 0;         // order: plain training, plain test, region test, region training
    ServeFrameDev *h_frames = nullptr, *d_frames = nullptr;
    int64_t *h_bounds = nullptr, *d_bounds = nullptr;   // serve_kernel's runs (grid + 1)
    MergeJobDev *h_jobs = nullptr, *d_jobs = nullptr;
    // frame lists of the region frames: pixels, masks, ring slots (maxf each)
    void **h_lists = nullptr, **d_lists = nullptr;
    obg_ingest_item *items = nullptr;
    unsigned long long *h_sum = nullptr, *d_sum = nullptr;
};

int sfail(int code, const char *msg) { return set_error(code, msg); }

// Relative cost of one 16-pixel group in serve_kernel, by depth and by kind
// (training frames build a tree, test frames also classify), and of one
// piece of a frame taken by a workgroup (leaf set into LDS, tree out, the
// pipeline refilled).  Fitted to per-workgroup times over the mixed served
// workload on MI355X (batches of up to 1024 frames): 63 units are about
// 5.0 ns of one workgroup at two workgroups per CU; a piece costs about
// 10 us, some 2000 groups.
int32_t serve_group_cost(int depth, bool test) {
    static const int32_t train[9] = {63, 63, 63, 63, 64, 63, 63, 63, 63};
    static const int32_t test_[9] = {65, 65, 65, 65, 66, 66, 71, 71, 71};
    const int d = depth < 0 ? 0 : (depth > 8 ? 8 : depth);
    return test ? test_[d] : train[d];
}
constexpr int64_t kServePartCost = 130000;

// total length covered by a set of [begin, end] intervals
double union_length(std::vector<std::pair<double, double>> iv) {
    std::sort(iv.begin(), iv.end());
    double total = 0, b = 0, e = -1;
    for (auto &p : iv) {
        if (p.first > e) {
            if (e > b) total += e - b;
            b = p.first;
            e = p.second;
        } else if (p.second > e) {
            e = p.second;
        }
    }
    if (e > b) total += e - b;
    return total;
}

void merge_job(MergeJobDev &j, const StreamDev &sd, const uint32_t *ring, uint32_t *leaf, int ring_len,
               int first, int n) {
    j.ring = ring;
    j.leaf = leaf;
    j.ring_len = ring_len;
    j.first = first;
    j.n_trees = n;
    j.words = sd.words;
    j.valid_bits = sd.valid_bits;
    const uint64_t need = (uint64_t)sd.cfg.thr_num * (uint64_t)n;
    const uint64_t kmin = (need + sd.cfg.thr_den - 1) / sd.cfg.thr_den;
    j.empty = kmin > (uint64_t)n ? 1 : 0;
    j.kmin = j.empty ? 0u : (uint32_t)kmin;
    j.planes = 0;
    while ((1 << j.planes) <= n) ++j.planes;
}

// Checkpoint layout: header, one record per stream, then per stream the leaf
// set and the ring, each padded to 8 bytes.
constexpr uint64_t kStateMagic = 0x3156524553474230ull;   // "0BGSERV1"
struct StateHeader {
    uint64_t magic;
    int32_t n_streams, window;
};
struct StateStream {
    // order: 0 = bitsets in key order, 1 = in the LDS order of the stream's
    // passes (region streams whose passes all run with compact tables; streams
    // without regions at d = 5 and 6)
    int32_t width, height, depth, n_train, region_w, region_h, ring_len, order;
    int64_t next_frame;
    uint64_t tree_bytes;
};
static_assert(sizeof(StateHeader) == 16 && sizeof(StateStream) == 48, "checkpoint layout");

uint64_t pad8(uint64_t b) { return (b + 7) & ~uint64_t(7); }

bool stream_ok(const obg_serve_stream &c) {
    return c.width >= 1 && c.height >= 1 && c.depth >= 1 && c.depth <= 6 && c.n_train >= 1 && c.n_train <= 65535 &&
           c.thr_num != 0 && c.thr_den != 0 && c.region_w >= 0 && c.region_h >= 0 &&
           (c.region_w == 0) == (c.region_h == 0) && c.width <= (1 << 24) && c.height <= (1 << 24);
}

SchedStream sched_stream(const obg_serve_stream &c) {
    const int nreg = c.region_w ? ((c.width + c.region_w - 1) / c.region_w) * ((c.height + c.region_h - 1) / c.region_h) : 1;
    return SchedStream{c.width, c.height, c.depth, c.n_train, nreg};
}

StateStream state_record(const obg_serve_stream &c, int window, int64_t next_frame, bool native = false) {
    StateStream r{};
    r.order = native ? 1 : 0;
    r.width = c.width;
    r.height = c.height;
    r.depth = c.depth;
    r.n_train = c.n_train;
    r.region_w = c.region_w;
    r.region_h = c.region_h;
    r.ring_len = c.n_train > window ? c.n_train : window;
    r.next_frame = next_frame;
    r.tree_bytes = sched_tree_bytes(sched_stream(c));
    return r;
}

}  // namespace

extern "C" int64_t obg_serve_state_bytes(const obg_serve_stream *streams, int32_t n_streams, int32_t remerge_window) {
    if (!streams || n_streams < 1 || remerge_window < 1) return -1;
    uint64_t b = sizeof(StateHeader) + (uint64_t)n_streams * sizeof(StateStream);
    for (int s = 0; s < n_streams; ++s) {
        if (!stream_ok(streams[s])) return -1;
        const StateStream r = state_record(streams[s], remerge_window, 0);
        b += pad8(r.tree_bytes) + pad8((uint64_t)r.ring_len * r.tree_bytes);
    }
    return (int64_t)b;
}

extern "C" int obg_serve_run(const obg_serve_config *cfg, obg_serve_stats *stats) {
    if (!cfg || !stats) return sfail(OBG_EINVAL, "config and stats must not be NULL");
    std::memset(stats, 0, sizeof(*stats));
    const int ns = cfg->n_streams;
    if (ns < 1 || !cfg->streams || !cfg->arrivals || !cfg->n_arrivals) return sfail(OBG_EINVAL, "no streams");
    if (!cfg->ingest) return sfail(OBG_EINVAL, "an ingest callback is required");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 16) return sfail(OBG_EINVAL, "max_inflight must be in [1, 16]");
    if (cfg->max_batch_frames < 1 || cfg->max_batch_frames > 4096) return sfail(OBG_EINVAL, "max_batch_frames must be in [1, 4096]");
    if (cfg->remerge_period < 1 || cfg->remerge_window < 1 || cfg->remerge_window > cfg->remerge_period)
        return sfail(OBG_EINVAL, "need 1 <= remerge_window <= remerge_period");
    if (!(cfg->speed > 0)) return sfail(OBG_EINVAL, "speed must be > 0");
    if (cfg->n_watch > 0 && (!cfg->watch_streams || !cfg->watch_masks)) return sfail(OBG_EINVAL, "watch buffers missing");
    for (int w = 0; w < cfg->n_watch; ++w)
        if (cfg->watch_streams[w] < 0 || cfg->watch_streams[w] >= ns || !cfg->watch_masks[w])
            return sfail(OBG_EINVAL, "bad watched stream");
    if (cfg->checksums && cfg->checksum_stride < 1) return sfail(OBG_EINVAL, "checksum_stride must be >= 1");
    std::vector<StreamDev> D(ns);
    std::vector<SchedStream> sc(ns);
    for (int s = 0; s < ns; ++s) {
        const obg_serve_stream &c = cfg->streams[s];
        if (c.width < 1 || c.height < 1 || c.depth < 1 || c.depth > 6 || c.n_train < 1 || c.n_train > 65535 ||
            c.thr_num == 0 || c.thr_den == 0 || cfg->n_arrivals[s] < 0 || (cfg->n_arrivals[s] && !cfg->arrivals[s]))
            return sfail(OBG_EINVAL, "bad stream description");
        if (c.region_w < 0 || c.region_h < 0 || (c.region_w == 0) != (c.region_h == 0))
            return sfail(OBG_EINVAL, "region_w and region_h must both be 0 or both be >= 1");
        StreamDev &sd = D[s];
        sd.cfg = c;
        sd.region = c.region_w > 0;
        sd.n_regions = sd.region ? ((c.width + c.region_w - 1) / c.region_w) * ((c.height + c.region_h - 1) / c.region_h) : 1;
        sd.geom.width = c.width;
        sd.geom.height = c.height;
        sd.geom.row_pitch = ((3 * (int64_t)c.width + 15) / 16) * 16;
        sd.geom.frame_pitch = sd.geom.row_pitch * c.height;
        sd.geom.depth = c.depth;
        sd.geom.region_w = c.region_w;
        sd.geom.region_h = c.region_h;
        // a stream's rings and leaf set never leave the library: where every
        // pass of the stream keeps its tables in one LDS order they stay in
        // that order, and the flushes and table loads copy words (merges
        // count bit by bit, whatever the order).  Region streams: passes over
        // frame lists with compact tables.  Streams without regions at
        // d = 5 (wide tables, word G'<<5 | R') and d = 6 (compact tables):
        // serve_kernel, where converting the 1024 or 8192 key words of a
        // table at every load and flush costs more than small frames' pixels
        sd.native = sd.region ? pixels_list_native_ok(&sd.geom) : (c.depth == 5 || c.depth == 6);
        StripArgs &a = sd.a;
        a.width = c.width;
        a.height = c.height;
        a.row_pitch = ((3 * (int64_t)c.width + 15) / 16) * 16;
        a.frame_pitch = a.row_pitch * c.height;
        if (a.frame_pitch > 0x7FFFFFFFLL) return sfail(OBG_EINVAL, "frame too large");
        a.gpr = 4 * ((c.width + 63) / 64);
        a.strip_rows = c.height;
        a.n_strips = 1;
        a.reg_cols = 1;
        a.n_regions = 1;
        a.div_gpr = make_fastdiv((uint32_t)a.gpr);
        a.div_tile = make_fastdiv((uint32_t)a.gpr);
        a.occ_test = tune(OBG_TUNE_OCC_BLIND, 2) == 2;
        a.mask_row_words = (c.width + 63) / 64;
        sd.groups = c.height * a.gpr;
        sd.words = leaf_words(c.depth);
        sd.valid_bits = leaf_count(c.depth) < 32 ? leaf_count(c.depth) : 32;
        sc[s] = {c.width, c.height, c.depth, c.n_train, sd.n_regions};
        if (sched_frame_bytes(sc[s]) != (uint64_t)a.frame_pitch ||
            sched_tree_bytes(sc[s]) != (uint64_t)sd.words * 4 * (uint64_t)sd.n_regions)
            return sfail(OBG_EINVAL, "internal size mismatch");
    }

    // a restored state: every record must describe the same stream
    std::vector<int64_t> first(ns, 0);
    if (cfg->state_in) {
        const uint8_t *p = static_cast<const uint8_t *>(cfg->state_in);
        StateHeader h;
        std::memcpy(&h, p, sizeof h);
        if (h.magic != kStateMagic || h.n_streams != ns || h.window != cfg->remerge_window)
            return sfail(OBG_EINVAL, "state_in: not a checkpoint of these streams (header)");
        for (int s = 0; s < ns; ++s) {
            StateStream r;
            std::memcpy(&r, p + sizeof(StateHeader) + (uint64_t)s * sizeof(StateStream), sizeof r);
            StateStream want = state_record(cfg->streams[s], cfg->remerge_window, r.next_frame, D[s].native);
            if (r.order != want.order)
                return sfail(OBG_EINVAL, "state_in: the stream's bitsets were stored in another bit order (a "
                                         "different OBG_TUNE_LAYOUT setting); restore under the setting that wrote it");
            if (std::memcmp(&r, &want, sizeof r) != 0 || r.next_frame < 0 ||
                r.next_frame + cfg->n_arrivals[s] > (int64_t)0x7FFFFFFF)
                return sfail(OBG_EINVAL, "state_in: stream record does not match the stream");
            first[s] = r.next_frame;
        }
    }

    // arrivals in time order (frame numbers continue from a restored state).
    // A stream's frames are served in frame order: a frame that arrives
    // before its predecessor is handed to the scheduler with it (its latency
    // still counts from its own arrival).
    struct Arr { double t; int s, f; };
    std::vector<Arr> arr;
    for (int s = 0; s < ns; ++s) {
        double prev = -std::numeric_limits<double>::infinity();
        for (int f = 0; f < cfg->n_arrivals[s]; ++f) {
            const double t = cfg->arrivals[s][f];
            if (!std::isfinite(t)) return sfail(OBG_EINVAL, "arrival times must be finite");
            prev = t > prev ? t : prev;
            arr.push_back({prev, s, (int)(first[s] + f)});
        }
    }
    std::stable_sort(arr.begin(), arr.end(), [](const Arr &x, const Arr &y) { return x.t < y.t; });

    uint8_t *arena_mem = nullptr;
    if (hipMalloc(&arena_mem, cfg->budget_bytes) != hipSuccess) return sfail(OBG_ENOMEM, "arena allocation failed");
    ServeScheduler sched;
    int rc = OBG_OK;
    {
        const int src = sched.init(sc.data(), ns, cfg->remerge_period, cfg->remerge_window, cfg->max_batch_frames,
                                   arena_mem, cfg->budget_bytes);
        if (src == -1) rc = sfail(OBG_EINVAL, "bad stream description");
        if (src == -2) rc = sfail(OBG_ENOMEM, "budget smaller than the streams' rings and leaf sets");
    }
    if (rc == OBG_OK && !cfg->state_in) {
        // a fresh run starts from empty rings and leaf sets, so that a saved
        // state holds the same bytes however the frames were batched
        for (int s = 0; s < ns && rc == OBG_OK; ++s) {
            const uint64_t tb = sched_tree_bytes(sc[s]);
            if (hipMemset(sched.S[s].leaf, 0, tb) != hipSuccess ||
                hipMemset(sched.S[s].ring, 0, (uint64_t)sched.S[s].ring_len * tb) != hipSuccess)
                rc = sfail(OBG_EHIP, "clearing the rings failed");
        }
        if (rc == OBG_OK && hipDeviceSynchronize() != hipSuccess) rc = sfail(OBG_EHIP, "clearing the rings failed");
    }
    if (rc == OBG_OK && cfg->state_in) {
        // leaf sets and rings into the arena
        const uint8_t *p = static_cast<const uint8_t *>(cfg->state_in) + sizeof(StateHeader) +
                           (uint64_t)ns * sizeof(StateStream);
        for (int s = 0; s < ns && rc == OBG_OK; ++s) {
            const StateStream r = state_record(cfg->streams[s], cfg->remerge_window, 0);
            const uint64_t ring_b = (uint64_t)r.ring_len * r.tree_bytes;
            if (hipMemcpy(sched.S[s].leaf, p, r.tree_bytes, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(sched.S[s].ring, p + pad8(r.tree_bytes), ring_b, hipMemcpyHostToDevice) != hipSuccess)
                rc = sfail(OBG_EHIP, "state_in: copy to the device failed");
            p += pad8(r.tree_bytes) + pad8(ring_b);
        }
    }
    const int maxf = cfg->max_batch_frames;
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) cus = n;
    }
    const int max_grid = 2 * cus;   // serve_kernel: two resident workgroups per CU
    std::vector<int64_t> cut_groups(maxf);
    std::vector<int32_t> cut_weight(maxf);
    std::vector<uint8_t> cut_whole(maxf);
    std::vector<Slot> slots(cfg->max_inflight);
    for (auto &sl : slots) {
        if (rc != OBG_OK) break;
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&sl.done) != hipSuccess || hipEventCreate(&sl.start) != hipSuccess ||
            hipEventCreate(&sl.k0) != hipSuccess || hipEventCreate(&sl.k1) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_frames, sizeof(ServeFrameDev) * maxf, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_frames, sizeof(ServeFrameDev) * maxf) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_bounds, sizeof(int64_t) * (max_grid + 1), hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_bounds, sizeof(int64_t) * (max_grid + 1)) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_jobs, sizeof(MergeJobDev) * ns, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_jobs, sizeof(MergeJobDev) * ns) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_sum, sizeof(unsigned long long) * maxf, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_sum, sizeof(unsigned long long) * maxf) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_lists, sizeof(void *) * 3 * maxf, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_lists, sizeof(void *) * 3 * maxf) != hipSuccess) {
            rc = sfail(OBG_ENOMEM, "slot allocation failed");
            break;
        }
        sl.items = new obg_ingest_item[maxf];
    }
    hipEvent_t t0 = nullptr;
    if (rc == OBG_OK && hipEventCreate(&t0) != hipSuccess) rc = sfail(OBG_EHIP, "event");
    std::vector<double> lat;
    lat.reserve(arr.size());
    std::vector<std::pair<double, double>> busy_iv, path_iv;   // per batch, ms after t0
    size_t next_arr = 0;
    int64_t served = 0, batches = 0, merges = 0, pixels = 0, train_frames = 0, test_frames = 0;
    int64_t train_pixels = 0, test_pixels = 0;
    if (rc == OBG_OK) {
        (void)hipEventRecord(t0, slots[0].st);
        (void)hipEventSynchronize(t0);
    }
    const Clock::time_point start = Clock::now();
    auto wall_now = [&]() { return std::chrono::duration<double>(Clock::now() - start).count(); };
    double idle_since = -1;
    while (rc == OBG_OK) {
        // 1. arrivals up to now (simulated time = wall time * speed)
        const double vt = wall_now() * cfg->speed;
        while (next_arr < arr.size() && arr[next_arr].t <= vt) {
            sched.arrive(arr[next_arr].s, arr[next_arr].f);
            ++next_arr;
        }
        // 2. completed batches
        bool progressed = false;
        for (auto &sl : slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                rc = sfail(OBG_EHIP, "batch failed on the device");
                break;
            }
            float ms = 0, ms_s = 0, ms_k0 = 0, ms_k1 = 0;
            (void)hipEventElapsedTime(&ms, t0, sl.done);
            (void)hipEventElapsedTime(&ms_s, t0, sl.start);
            (void)hipEventElapsedTime(&ms_k0, t0, sl.k0);
            (void)hipEventElapsedTime(&ms_k1, t0, sl.k1);
            busy_iv.push_back({ms_s, ms});
            path_iv.push_back({ms_k0, ms_k1});
            const double done_s = ms * 1e-3;
            for (size_t p = 0; p < sl.order.size(); ++p) {
                const SchedFrame &fr = sl.batch.frames[sl.order[p]];
                const int64_t px = (int64_t)D[fr.stream].cfg.width * D[fr.stream].cfg.height;
                if (fr.test) {
                    lat.push_back((done_s - sl.arrival[p]) * 1e3);
                    // test frames follow the plain training frames in launch order
                    if (cfg->checksums && fr.frame < cfg->checksum_stride)
                        cfg->checksums[(int64_t)fr.stream * cfg->checksum_stride + fr.frame] =
                            sl.h_sum[p - sl.n_train_plain];
                    ++test_frames;
                    test_pixels += px;
                } else {
                    ++train_frames;
                    train_pixels += px;
                }
                pixels += px;
                ++served;
            }
            sched.complete(sl.batch);
            sl.busy = false;
            progressed = true;
        }
        if (rc) break;
        if (next_arr == arr.size() && served == (int64_t)arr.size()) break;
        // 3. a new batch in a free slot
        Slot *free_slot = nullptr;
        for (auto &sl : slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        bool launched = false;
        if (free_slot && sched.form(free_slot->batch)) {
            Slot &sl = *free_slot;
            const std::vector<SchedFrame> &F = sl.batch.frames;
            const int n = (int)F.size();
            // launch order: plain training, plain test, region test, region
            // training frames; test frames are contiguous for the checksums
            sl.order.clear();
            for (int pass = 0; pass < 4; ++pass)
                for (int i = 0; i < n; ++i) {
                    const bool region = D[F[i].stream].region, test = F[i].test;
                    if ((pass == 0 && !region && !test) || (pass == 1 && !region && test) ||
                        (pass == 2 && region && test) || (pass == 3 && region && !test))
                        sl.order.push_back(i);
                }
            int n_plain = 0, nt = 0, n_test_end = 0;
            for (int p = 0; p < n; ++p) {
                const SchedFrame &fr = F[sl.order[p]];
                if (!D[fr.stream].region) ++n_plain;
                if (!D[fr.stream].region && !fr.test) ++nt;
                if (fr.test) n_test_end = p + 1;
            }
            sl.n_train_plain = nt;
            // descriptors; the plain frames' groups are numbered end to end
            int64_t n_groups = 0;
            sl.arrival.resize(n);
            for (int p = 0; p < n; ++p) {
                const SchedFrame &fr = F[sl.order[p]];
                const StreamDev &sd = D[fr.stream];
                uint32_t *ring = reinterpret_cast<uint32_t *>(sched.S[fr.stream].ring);
                ServeFrameDev &fd = sl.h_frames[p];
                fd.a = sd.a;
                fd.rgb = fr.rgb;
                fd.occ = ring + (int64_t)fr.slot * sd.words * sd.n_regions;
                fd.leaf = reinterpret_cast<uint32_t *>(sched.S[fr.stream].leaf);
                fd.mask = fr.mask;
                fd.depth = sd.cfg.depth;
                fd.groups = sd.region ? 0 : sd.groups;
                fd.words = sd.words;
                fd.native = sd.native ? 1 : 0;
                fd.g0 = n_groups;
                n_groups += fd.groups;
                sl.arrival[p] = cfg->arrivals[fr.stream][fr.frame - first[fr.stream]] / cfg->speed;
                sl.items[p].stream = fr.stream;
                sl.items[p].frame = fr.frame;
                sl.items[p].dst = fr.rgb;
                if (p >= n_plain) {
                    sl.h_lists[p - n_plain] = fr.rgb;
                    sl.h_lists[maxf + p - n_plain] = fr.mask;
                    sl.h_lists[2 * maxf + p - n_plain] = fd.occ;
                }
            }
            // serve_kernel's runs, cut by cost; at least kMinChunk groups per
            // workgroup, so that a small batch does not pay for idle ones
            int grid = 0;
            if (n_plain) {
                const int64_t kMinChunk = 2048;
                grid = (int)std::max<int64_t>(1, std::min<int64_t>((n_groups + kMinChunk - 1) / kMinChunk, max_grid));
                for (int p = 0; p < n_plain; ++p) {
                    cut_groups[p] = sl.h_frames[p].groups;
                    cut_weight[p] = serve_group_cost(sl.h_frames[p].depth, sl.h_frames[p].mask != nullptr);
                }
                split_by_cost(cut_groups.data(), cut_weight.data(), n_plain, kServePartCost, grid, sl.h_bounds,
                              cut_whole.data());
            }
            for (int p = 0; p < n; ++p) sl.h_frames[p].whole = p < n_plain ? cut_whole[p] : 0;
            // merges of plain streams in one launch; region streams merge alone
            int n_jobs = 0;
            for (const SchedMerge &m : sl.batch.merges)
                if (!D[m.stream].region)
                    merge_job(sl.h_jobs[n_jobs++], D[m.stream], reinterpret_cast<const uint32_t *>(sched.S[m.stream].ring),
                              reinterpret_cast<uint32_t *>(sched.S[m.stream].leaf), sched.S[m.stream].ring_len, m.first,
                              m.n);
            hipStream_t st = sl.st;
            bool ok = hipEventRecord(sl.start, st) == hipSuccess;
            if (ok) ok = hipMemcpyAsync(sl.d_frames, sl.h_frames, sizeof(ServeFrameDev) * n, hipMemcpyHostToDevice, st) == hipSuccess;
            if (ok && grid)
                ok = hipMemcpyAsync(sl.d_bounds, sl.h_bounds, sizeof(int64_t) * (grid + 1), hipMemcpyHostToDevice, st) ==
                     hipSuccess;
            if (ok && n_jobs)
                ok = hipMemcpyAsync(sl.d_jobs, sl.h_jobs, sizeof(MergeJobDev) * n_jobs, hipMemcpyHostToDevice, st) == hipSuccess;
            if (ok && n > n_plain)
                ok = hipMemcpyAsync(sl.d_lists, sl.h_lists, sizeof(void *) * 3 * maxf, hipMemcpyHostToDevice, st) ==
                     hipSuccess;
            if (ok) ok = cfg->ingest(cfg->ingest_ctx, sl.items, n, st) == 0;
            if (ok) ok = hipEventRecord(sl.k0, st) == hipSuccess;
            if (ok) {
                if (n_plain) {
                    hipLaunchKernelGGL(serve_zero_kernel, dim3(8, n_plain), dim3(256), 0, st,
                                       (const ServeFrameDev *)sl.d_frames);
                    ServeArgs b{sl.d_frames, n_plain, sl.d_bounds};
                    hipLaunchKernelGGL(serve_kernel, dim3((unsigned)grid), dim3(kServeBlock), 0, st, b);
                }
                // frames with regions: one pass per run of a stream's test
                // (or training) frames over their frame lists, trees into the
                // ring slots; geometries the LDS kernels do not take go one
                // frame at a time through the one-stream entry points
                for (int p = n_plain; ok && p < n;) {
                    const SchedFrame &f0 = F[sl.order[p]];
                    int q = p + 1;
                    while (q < n && F[sl.order[q]].stream == f0.stream && F[sl.order[q]].test == f0.test) ++q;
                    const StreamDev &sd = D[f0.stream];
                    const uint32_t *leaf = reinterpret_cast<const uint32_t *>(sched.S[f0.stream].leaf);
                    const int mode = f0.test ? (MODE_MASK | MODE_OCC) : MODE_OCC;
                    if (pixels_list_ok(&sd.geom, mode)) {
                        const int i0 = p - n_plain;
                        FrameLists fl{reinterpret_cast<const uint8_t *const *>(sl.d_lists + i0),
                                      reinterpret_cast<uint64_t *const *>(sl.d_lists + maxf + i0),
                                      reinterpret_cast<uint32_t *const *>(sl.d_lists + 2 * maxf + i0)};
                        ok = run_pixels_list(&sd.geom, mode, fl, q - p, leaf, st, sd.native) == OBG_OK;
                    } else {
                        for (int r = p; ok && r < q; ++r) {
                            const SchedFrame &fr = F[sl.order[r]];
                            uint32_t *slot = reinterpret_cast<uint32_t *>(sched.S[fr.stream].ring) +
                                             (int64_t)fr.slot * sd.words * sd.n_regions;
                            ok = (fr.test ? obg_classify(&sd.geom, fr.rgb, 1, leaf, fr.mask, slot, st)
                                          : obg_train_frame(&sd.geom, fr.rgb, 1, slot, nullptr, st)) == OBG_OK;
                        }
                    }
                    p = q;
                }
                if (ok && n_jobs) {
                    int maxw = 1;
                    for (int i = 0; i < n_jobs; ++i) maxw = std::max(maxw, sl.h_jobs[i].words);
                    hipLaunchKernelGGL(serve_merge_kernel, dim3((maxw + 63) / 64, n_jobs), dim3(kMergeBlock), 0, st,
                                       (const MergeJobDev *)sl.d_jobs);
                }
                for (const SchedMerge &m : sl.batch.merges) {
                    if (!ok || !D[m.stream].region) continue;
                    const StreamDev &sd = D[m.stream];
                    ok = obg_merge(&sd.geom, reinterpret_cast<const uint32_t *>(sched.S[m.stream].ring),
                                   sched.S[m.stream].ring_len, m.first, m.n, sd.cfg.thr_num, sd.cfg.thr_den,
                                   reinterpret_cast<uint32_t *>(sched.S[m.stream].leaf), st) == OBG_OK;
                }
                if (ok) ok = hipEventRecord(sl.k1, st) == hipSuccess;
                const int nc = n_test_end - nt;
                if (ok && nc > 0 && cfg->checksums) {
                    ok = hipMemsetAsync(sl.d_sum, 0, sizeof(unsigned long long) * nc, st) == hipSuccess;
                    hipLaunchKernelGGL(serve_checksum_kernel, dim3(16, nc), dim3(256), 0, st,
                                       (const ServeFrameDev *)(sl.d_frames + nt), sl.d_sum);
                    if (ok)
                        ok = hipMemcpyAsync(sl.h_sum, sl.d_sum, sizeof(unsigned long long) * nc, hipMemcpyDeviceToHost,
                                            st) == hipSuccess;
                }
                for (int w = 0; ok && w < cfg->n_watch; ++w) {
                    const int s = cfg->watch_streams[w];
                    const uint64_t mbytes = sched.S[s].mask_bytes;
                    for (int p = nt; ok && p < n_test_end; ++p) {
                        const SchedFrame &fr = F[sl.order[p]];
                        const int t = fr.frame - D[s].cfg.n_train;
                        if (fr.stream == s && t < cfg->watch_max_frames)
                            ok = hipMemcpyAsync(cfg->watch_masks[w] + (int64_t)t * (int64_t)(mbytes / 8), fr.mask, mbytes,
                                                hipMemcpyDeviceToHost, st) == hipSuccess;
                    }
                }
                if (ok) ok = hipGetLastError() == hipSuccess;
                if (ok) ok = hipEventRecord(sl.done, st) == hipSuccess;
            }
            if (!ok) {
                rc = sfail(OBG_EHIP, "batch launch failed");
                break;
            }
            sl.busy = true;
            ++batches;
            merges += (int64_t)sl.batch.merges.size();
            launched = true;
        }
        if (launched || progressed) idle_since = -1;
        if (!launched && !progressed) {
            bool any_busy = false;
            for (auto &sl : slots) any_busy = any_busy || sl.busy;
            if (!any_busy && sched.any_queued()) {
                // nothing in flight holds arena memory: a refused frame that does
                // not fit now never will
                if (sched.hopeless()) {
                    rc = sfail(OBG_ENOMEM, "budget too small for one frame");
                    break;
                }
                // with nothing in flight every queued frame is admissible; frames
                // that stay queued would mean a scheduling fault: stop, do not spin
                if (idle_since < 0) idle_since = wall_now();
                if (wall_now() - idle_since > 2.0) {
                    rc = sfail(OBG_EHIP, "serving loop stalled with frames queued and nothing in flight");
                    break;
                }
            }
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    const double wall = wall_now();
    for (auto &sl : slots)
        if (sl.st) (void)hipStreamSynchronize(sl.st);
    if (rc == OBG_OK && cfg->state_out) {
        // every batch has completed: the arena holds the final models and rings
        uint8_t *p = static_cast<uint8_t *>(cfg->state_out);
        const StateHeader h{kStateMagic, ns, cfg->remerge_window};
        std::memcpy(p, &h, sizeof h);
        uint8_t *data = p + sizeof(StateHeader) + (uint64_t)ns * sizeof(StateStream);
        for (int s = 0; s < ns && rc == OBG_OK; ++s) {
            const StateStream r =
                state_record(cfg->streams[s], cfg->remerge_window, first[s] + cfg->n_arrivals[s], D[s].native);
            std::memcpy(p + sizeof(StateHeader) + (uint64_t)s * sizeof(StateStream), &r, sizeof r);
            const uint64_t ring_b = (uint64_t)r.ring_len * r.tree_bytes;
            std::memset(data, 0, pad8(r.tree_bytes) + pad8(ring_b));
            if (hipMemcpy(data, sched.S[s].leaf, r.tree_bytes, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(data + pad8(r.tree_bytes), sched.S[s].ring, ring_b, hipMemcpyDeviceToHost) != hipSuccess)
                rc = sfail(OBG_EHIP, "state_out: copy from the device failed");
            data += pad8(r.tree_bytes) + pad8(ring_b);
        }
    }
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) -> double {
        if (lat.empty()) return 0.0;
        size_t i = (size_t)std::ceil(p * lat.size()) - 1;
        if (i >= lat.size()) i = lat.size() - 1;
        return lat[i];
    };
    stats->frames_arrived = (int64_t)arr.size();
    stats->frames_served = served;
    stats->train_frames = train_frames;
    stats->test_frames = test_frames;
    stats->pixels = pixels;
    stats->batches = batches;
    stats->merges = merges;
    stats->admission_waits = sched.admission_waits;
    stats->wall_s = wall;
    stats->lat_p50_ms = pct(0.50);
    stats->lat_p99_ms = pct(0.99);
    stats->lat_max_ms = lat.empty() ? 0.0 : lat.back();
    double sum = 0;
    for (double v : lat) sum += v;
    stats->lat_mean_ms = lat.empty() ? 0.0 : sum / lat.size();
    stats->peak_bytes = (double)sched.arena.peak;
    stats->train_pixels = train_pixels;
    stats->test_pixels = test_pixels;
    stats->busy_s = union_length(busy_iv) * 1e-3;
    stats->path_busy_s = union_length(path_iv) * 1e-3;
    for (auto &sl : slots) {
        if (sl.st) (void)hipStreamDestroy(sl.st);
        for (hipEvent_t ev : {sl.done, sl.start, sl.k0, sl.k1})
            if (ev) (void)hipEventDestroy(ev);
        if (sl.h_frames) (void)hipHostFree(sl.h_frames);
        if (sl.d_frames) (void)hipFree(sl.d_frames);
        if (sl.h_bounds) (void)hipHostFree(sl.h_bounds);
        if (sl.d_bounds) (void)hipFree(sl.d_bounds);
        if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
        if (sl.d_jobs) (void)hipFree(sl.d_jobs);
        if (sl.h_sum) (void)hipHostFree(sl.h_sum);
        if (sl.d_sum) (void)hipFree(sl.d_sum);
        if (sl.h_lists) (void)hipHostFree(sl.h_lists);
        if (sl.d_lists) (void)hipFree(sl.d_lists);
        delete[] sl.items;
    }
    if (t0) (void)hipEventDestroy(t0);
    (void)hipFree(arena_mem);
    return rc;
}
