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
#include <thread>
#include <vector>

#include "../../include/obg.h"
#include "arena.h"
#include "strip_core.h"

namespace obg {

// One frame of a batch.
struct ServeFrameDev {
    StripArgs a;              // geometry (one region)
    const uint8_t *rgb;
    uint32_t *occ;            // ring slot of this frame
    uint32_t *leaf;           // the stream's merged leaf set (test frames)
    uint64_t *mask;           // test frames; NULL for training frames
    int32_t depth, groups, words, pad_;
    int64_t g0;               // first group of the frame in the batch's group space
};

// A batch is one space of 16-pixel groups: its frames' groups end to end.
// Workgroup w takes groups [w*chunk, (w+1)*chunk), whatever frames they fall
// in, so every workgroup has the same number of pixels to read.
struct ServeArgs {
    const ServeFrameDev *frames;
    int32_t n_frames;
    int64_t n_groups;
    int64_t chunk;            // multiple of 4: mask words never straddle workgroups
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
// frame's ring slot; test frames also get their mask bits from the leaf table.
template <int D, int LAY, int MODE>
__device__ __attribute__((noinline)) void serve_part(const ServeFrameDev &fd, int gb, int ge, uint32_t *leaf_tab,
                                                     uint32_t *occ_tab, bool load_leaf) {
    constexpr bool MASK = (MODE & MODE_MASK) != 0;
    constexpr int LW = lds_words(D, LAY);
    const int tid = threadIdx.x;
    const StripArgs a = fd.a;
    if (MASK && load_leaf) leaf_to_lds<D, LAY>(fd.leaf, leaf_tab, 1, tid, kServeBlock);
    __syncthreads();
    for (int i = tid; i < LW; i += kServeBlock) occ_tab[i] = 0;
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(fd.rgb, (uint32_t)a.frame_pitch);
    __amdgpu_buffer_rsrc_t ms = make_rsrc(nullptr, 0);
    if (MASK) ms = make_rsrc(fd.mask, (uint32_t)a.height * (uint32_t)a.mask_row_words * 8u);
    span_loop<D, MODE, LAY, false, kServeBlock>(a, rs, ms, gb, ge, leaf_tab, occ_tab, nullptr, nullptr);
    __syncthreads();
    occ_from_lds<D, LAY>(occ_tab, fd.occ, 1, tid, kServeBlock);
}

template <int MODE>
__device__ __forceinline__ void serve_dispatch(const ServeFrameDev &fd, int gb, int ge, uint32_t *leaf_tab,
                                               uint32_t *occ_tab, bool load_leaf) {
    switch (fd.depth) {
        case 1: serve_part<1, LAY_WIDE, MODE>(fd, gb, ge, leaf_tab, occ_tab, load_leaf); break;
        case 2: serve_part<2, LAY_WIDE, MODE>(fd, gb, ge, leaf_tab, occ_tab, load_leaf); break;
        case 3: serve_part<3, LAY_WIDE, MODE>(fd, gb, ge, leaf_tab, occ_tab, load_leaf); break;
        case 4: serve_part<4, LAY_WIDE, MODE>(fd, gb, ge, leaf_tab, occ_tab, load_leaf); break;
        case 5: serve_part<5, LAY_WIDE, MODE>(fd, gb, ge, leaf_tab, occ_tab, load_leaf); break;
        default: serve_part<6, LAY_COMPACT, MODE>(fd, gb, ge, leaf_tab, occ_tab, load_leaf); break;
    }
}

// Training frames (occupancy) and test frames (mask and occupancy) of a batch
// in one launch.
__global__ __launch_bounds__(kServeBlock) __attribute__((amdgpu_waves_per_eu(4))) void serve_kernel(ServeArgs b) {
    __shared__ uint32_t leaf_tab[kServeTableWords];
    __shared__ uint32_t occ_tab[kServeTableWords];
    int64_t g = (int64_t)blockIdx.x * b.chunk;
    const int64_t gend = min(g + b.chunk, b.n_groups);
    if (g >= gend) return;
    int fi = frame_of(b, g);
    const uint32_t *cur_leaf = nullptr;
    while (g < gend && fi < b.n_frames) {
        const ServeFrameDev &fd = b.frames[fi];
        const int lb = (int)(g - fd.g0);
        const int le = (int)min<int64_t>(gend - fd.g0, (int64_t)fd.groups);
        if (fd.mask) {
            serve_dispatch<MODE_MASK | MODE_OCC>(fd, lb, le, leaf_tab, occ_tab, fd.leaf != cur_leaf);
            cur_leaf = fd.leaf;
        } else {
            serve_dispatch<MODE_OCC>(fd, lb, le, leaf_tab, occ_tab, false);
        }
        g = fd.g0 + le;
        ++fi;
    }
}

// Zero the ring slots that this batch's frames OR their occupancy into.
__global__ __launch_bounds__(256) void serve_zero_kernel(const ServeFrameDev *frames) {
    const ServeFrameDev &fd = frames[blockIdx.y];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < fd.words; i += gridDim.x * blockDim.x) fd.occ[i] = 0;
}

__global__ __launch_bounds__(256) void serve_merge_kernel(const MergeJobDev *jobs) {
    const MergeJobDev &j = jobs[blockIdx.y];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= j.words) return;
    j.leaf[i] = merge_word(j.ring, j.ring_len, j.first, j.n_trees, j.words, i, j.valid_bits, j.kmin, j.planes,
                           j.empty);
}

// Per test frame: an order-dependent 64-bit hash of its mask words.
__global__ __launch_bounds__(256) void serve_checksum_kernel(const ServeFrameDev *frames, unsigned long long *out) {
    const ServeFrameDev &fd = frames[blockIdx.y];
    const int64_t n = (int64_t)fd.a.height * fd.a.mask_row_words;
    unsigned long long h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        h += (fd.mask[i] ^ (0x9E3779B97F4A7C15ull * (uint64_t)(i + 1))) * 0xBF58476D1CE4E5B9ull;
    atomicAdd(&out[blockIdx.y], h);
}

}  // namespace obg

using namespace obg;

namespace {

using Clock = std::chrono::steady_clock;

struct StreamState {
    obg_serve_stream cfg;
    StripArgs a{};
    int words = 0, valid_bits = 32, groups = 0, ring_len = 0;
    uint64_t frame_bytes = 0, mask_bytes = 0;
    uint32_t *ring = nullptr, *leaf = nullptr;
    std::deque<int> queued;     // arrived frames waiting for a batch
    int next_frame = 0;         // next frame index to arrive
    int inflight = 0;           // batches holding frames of this stream
    int inflight_frames = 0;    // frames of this stream in those batches
    bool merge_inflight = false;
    bool head_waited = false;   // the first queued frame has already been refused once
};

struct PendingFrame {
    int stream, frame;
    double arrival;             // wall seconds after start
    uint8_t *rgb;               // frame, then (test frames) its mask, in one arena block
    uint64_t *mask;
    bool test;
    uint64_t bytes;             // size of the arena block
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr, start = nullptr, k0 = nullptr, k1 = nullptr;
    bool busy = false;
    std::vector<PendingFrame> frames;
    std::vector<int> merge_streams;
    ServeFrameDev *h_frames = nullptr, *d_frames = nullptr;
    MergeJobDev *h_jobs = nullptr, *d_jobs = nullptr;
    obg_ingest_item *items = nullptr;
    unsigned long long *h_sum = nullptr, *d_sum = nullptr;
};

int sfail(int code, const char *msg) { return set_error(code, msg); }

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

void fill_frame(ServeFrameDev &fd, const StreamState &ss, const uint8_t *rgb, uint32_t *occ, uint64_t *mask) {
    fd.a = ss.a;
    fd.rgb = rgb;
    fd.occ = occ;
    fd.leaf = ss.leaf;
    fd.mask = mask;
    fd.depth = ss.cfg.depth;
    fd.groups = ss.groups;
    fd.words = ss.words;
    fd.pad_ = 0;
}

void merge_job(MergeJobDev &j, const StreamState &ss, int first, int n, uint32_t num, uint32_t den) {
    j.ring = ss.ring;
    j.leaf = ss.leaf;
    j.ring_len = ss.ring_len;
    j.first = first;
    j.n_trees = n;
    j.words = ss.words;
    j.valid_bits = ss.valid_bits;
    const uint64_t need = (uint64_t)num * (uint64_t)n;
    const uint64_t kmin = (need + den - 1) / den;
    j.empty = kmin > (uint64_t)n ? 1 : 0;
    j.kmin = j.empty ? 0u : (uint32_t)kmin;
    j.planes = 0;
    while ((1 << j.planes) <= n) ++j.planes;
}

uint64_t frame_block(const StreamState &ss, bool test) {
    return Arena::round(ss.frame_bytes) + (test ? Arena::round(ss.mask_bytes) : 0);
}

}  // namespace

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
    if (cfg->speed <= 0) return sfail(OBG_EINVAL, "speed must be > 0");
    std::vector<StreamState> S(ns);
    uint64_t state_bytes = 0;
    for (int s = 0; s < ns; ++s) {
        const obg_serve_stream &c = cfg->streams[s];
        if (c.width < 1 || c.height < 1 || c.depth < 1 || c.depth > 6 || c.n_train < 1 || c.n_train > 65535 ||
            c.thr_num == 0 || c.thr_den == 0 || cfg->n_arrivals[s] < 0)
            return sfail(OBG_EINVAL, "bad stream description");
        StreamState &ss = S[s];
        ss.cfg = c;
        StripArgs &a = ss.a;
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
        a.mask_row_words = (c.width + 63) / 64;
        ss.groups = c.height * a.gpr;
        ss.words = leaf_words(c.depth);
        ss.valid_bits = leaf_count(c.depth) < 32 ? leaf_count(c.depth) : 32;
        ss.ring_len = std::max(c.n_train, cfg->remerge_window);
        ss.frame_bytes = (uint64_t)a.frame_pitch;
        ss.mask_bytes = (uint64_t)c.height * a.mask_row_words * 8;
        state_bytes += Arena::round((uint64_t)ss.ring_len * ss.words * 4) + Arena::round((uint64_t)ss.words * 4);
    }
    if (state_bytes >= cfg->budget_bytes) return sfail(OBG_ENOMEM, "budget smaller than the streams' rings and leaf sets");

    // events sorted by arrival time
    struct Arr { double t; int s, f; };
    std::vector<Arr> arr;
    for (int s = 0; s < ns; ++s)
        for (int f = 0; f < cfg->n_arrivals[s]; ++f) arr.push_back({cfg->arrivals[s][f], s, f});
    std::stable_sort(arr.begin(), arr.end(), [](const Arr &x, const Arr &y) { return x.t < y.t; });

    Arena arena;
    uint8_t *arena_mem = nullptr;
    hipError_t e = hipMalloc(&arena_mem, cfg->budget_bytes);
    if (e != hipSuccess) return sfail(OBG_ENOMEM, "arena allocation failed");
    arena.init(arena_mem, cfg->budget_bytes);
    int rc = OBG_OK;
    const int M = cfg->max_inflight;
    std::vector<Slot> slots(M);
    const int maxf = cfg->max_batch_frames;
    for (auto &sl : slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&sl.done) != hipSuccess || hipEventCreate(&sl.start) != hipSuccess ||
            hipEventCreate(&sl.k0) != hipSuccess || hipEventCreate(&sl.k1) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_frames, sizeof(ServeFrameDev) * maxf * 2, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_frames, sizeof(ServeFrameDev) * maxf * 2) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_jobs, sizeof(MergeJobDev) * ns, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_jobs, sizeof(MergeJobDev) * ns) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_sum, sizeof(unsigned long long) * maxf, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.d_sum, sizeof(unsigned long long) * maxf) != hipSuccess) {
            rc = sfail(OBG_ENOMEM, "slot allocation failed");
            break;
        }
        sl.items = new obg_ingest_item[maxf];
    }
    hipEvent_t t0 = nullptr;
    if (rc == OBG_OK && hipEventCreate(&t0) != hipSuccess) rc = sfail(OBG_EHIP, "event");
    // per-stream state in the arena
    for (int s = 0; s < ns && rc == OBG_OK; ++s) {
        StreamState &ss = S[s];
        ss.ring = (uint32_t *)arena.get((uint64_t)ss.ring_len * ss.words * 4);
        ss.leaf = (uint32_t *)arena.get((uint64_t)ss.words * 4);
        if (!ss.ring || !ss.leaf) rc = sfail(OBG_ENOMEM, "budget too small for stream state");
    }
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) cus = n;
    }
    std::vector<double> lat;
    lat.reserve(arr.size());
    std::vector<std::pair<double, double>> busy_iv, path_iv;   // per batch, ms after t0
    size_t next_arr = 0;
    int64_t served = 0, admission_waits = 0, batches = 0, merges = 0, pixels = 0, train_frames = 0, test_frames = 0;
    int64_t train_pixels = 0, test_pixels = 0;
    const Clock::time_point wall0 = Clock::now();
    if (rc == OBG_OK) {
        (void)hipEventRecord(t0, slots[0].st);
        (void)hipEventSynchronize(t0);
    }
    const Clock::time_point start = Clock::now();
    auto wall_now = [&]() { return std::chrono::duration<double>(Clock::now() - start).count(); };
    int rr = 0;         // round-robin start among streams
    double idle_since = -1;
    int waiting = -1;   // stream whose next frame did not fit: it goes first, and
                        // nothing else is admitted until it fits
    while (rc == OBG_OK) {
        // 1. arrivals up to now (simulated time = wall time * speed)
        const double vt = wall_now() * cfg->speed;
        while (next_arr < arr.size() && arr[next_arr].t <= vt) {
            S[arr[next_arr].s].queued.push_back(arr[next_arr].f);
            ++next_arr;
        }
        // 2. completed batches
        bool progressed = false;
        for (auto &sl : slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) { rc = sfail(OBG_EHIP, "batch failed on the device"); break; }
            float ms = 0, ms_s = 0, ms_k0 = 0, ms_k1 = 0;
            (void)hipEventElapsedTime(&ms, t0, sl.done);
            (void)hipEventElapsedTime(&ms_s, t0, sl.start);
            (void)hipEventElapsedTime(&ms_k0, t0, sl.k0);
            (void)hipEventElapsedTime(&ms_k1, t0, sl.k1);
            busy_iv.push_back({ms_s, ms});
            path_iv.push_back({ms_k0, ms_k1});
            const double done_s = ms * 1e-3;
            int ti = 0;
            for (auto &pf : sl.frames) {
                StreamState &ss = S[pf.stream];
                if (pf.test) {
                    lat.push_back((done_s - pf.arrival) * 1e3);
                    if (cfg->checksums && pf.frame < cfg->checksum_stride)
                        cfg->checksums[(int64_t)pf.stream * cfg->checksum_stride + pf.frame] = sl.h_sum[ti];
                    ++ti;
                    ++test_frames;
                    test_pixels += (int64_t)ss.cfg.width * ss.cfg.height;
                } else {
                    ++train_frames;
                    train_pixels += (int64_t)ss.cfg.width * ss.cfg.height;
                }
                pixels += (int64_t)ss.cfg.width * ss.cfg.height;
                arena.put(pf.rgb, pf.bytes);
                ++served;
            }
            for (auto &pf : sl.frames) S[pf.stream].inflight_frames--;
            {
                std::vector<int> seen;
                for (auto &pf : sl.frames)
                    if (std::find(seen.begin(), seen.end(), pf.stream) == seen.end()) {
                        seen.push_back(pf.stream);
                        S[pf.stream].inflight--;
                    }
            }
            for (int s : sl.merge_streams) S[s].merge_inflight = false;
            sl.frames.clear();
            sl.merge_streams.clear();
            sl.busy = false;
            progressed = true;
        }
        if (rc) break;
        if (next_arr == arr.size() && served == (int64_t)arr.size()) break;
        // 3. form a batch in a free slot
        Slot *free_slot = nullptr;
        for (auto &sl : slots)
            if (!sl.busy) { free_slot = &sl; break; }
        bool launched = false;
        if (free_slot) {
            Slot &sl = *free_slot;
            std::vector<PendingFrame> train_list, test_list;
            int n_jobs = 0;
            bool blocked = false;
            // each stream is visited at most once per batch: a stream's frames
            // after one that ends with a merge must not join the same batch
            const int first_stream = waiting >= 0 ? waiting : rr;
            for (int k = 0; k < ns && (int)(train_list.size() + test_list.size()) < maxf && !blocked; ++k) {
                const int s = (first_stream + k) % ns;
                StreamState &ss = S[s];
                const int T = ss.cfg.n_train;
                bool merged_here = false;
                while (!ss.queued.empty() && !ss.merge_inflight && !merged_here &&
                       (int)(train_list.size() + test_list.size()) < maxf) {
                    const int f = ss.queued.front();
                    const bool test = f >= T;
                    // frames that end with a merge wait until the stream has nothing else in flight
                    const int t = f - T;
                    const bool ends_merge = (f == T - 1) || (test && (t + 1) % cfg->remerge_period == 0);
                    if (ends_merge && ss.inflight > 0) break;
                    // ring slots of frames in flight must stay distinct
                    if (ss.inflight_frames + 1 > ss.ring_len / 2) break;
                    // frames that follow a merge in this batch wait for the next batch
                    PendingFrame pf{s, f, 0.0, nullptr, nullptr, test, frame_block(ss, test)};
                    pf.rgb = arena.get(pf.bytes);
                    if (!pf.rgb) {
                        if (!ss.head_waited) ++admission_waits;
                        ss.head_waited = true;
                        waiting = s;
                        blocked = true;
                        break;
                    }
                    ss.head_waited = false;
                    if (waiting == s) waiting = -1;
                    if (test) pf.mask = (uint64_t *)(pf.rgb + Arena::round(ss.frame_bytes));
                    pf.arrival = cfg->arrivals[s][f] / cfg->speed;
                    ss.queued.pop_front();
                    ss.inflight_frames++;
                    (test ? test_list : train_list).push_back(pf);
                    if (ends_merge) {
                        MergeJobDev &j = sl.h_jobs[n_jobs++];
                        if (f == T - 1)
                            merge_job(j, ss, 0, T, ss.cfg.thr_num, ss.cfg.thr_den);
                        else {
                            const int W = cfg->remerge_window;
                            const int first = ((f - W + 1) % ss.ring_len + ss.ring_len) % ss.ring_len;
                            merge_job(j, ss, first, W, ss.cfg.thr_num, ss.cfg.thr_den);
                        }
                        sl.merge_streams.push_back(s);
                        merged_here = true;
                    }
                }
            }
            rr = (rr + 1) % ns;
            const int nt = (int)train_list.size(), nc = (int)test_list.size();
            if (nt + nc > 0) {
                // descriptors: training frames first, then test frames, their
                // groups numbered end to end
                int64_t n_groups = 0;
                for (int i = 0; i < nt + nc; ++i) {
                    const PendingFrame &pf = i < nt ? train_list[i] : test_list[i - nt];
                    StreamState &ss = S[pf.stream];
                    ServeFrameDev &fd = sl.h_frames[i];
                    fill_frame(fd, ss, pf.rgb, ss.ring + (int64_t)(pf.frame % ss.ring_len) * ss.words, pf.mask);
                    fd.g0 = n_groups;
                    n_groups += ss.groups;
                }
                sl.frames.clear();
                for (auto &pf : train_list) sl.frames.push_back(pf);
                for (auto &pf : test_list) sl.frames.push_back(pf);
                std::vector<int> seen;
                for (int i = 0; i < nt + nc; ++i) {
                    sl.items[i].stream = sl.frames[i].stream;
                    sl.items[i].frame = sl.frames[i].frame;
                    sl.items[i].dst = sl.frames[i].rgb;
                    if (std::find(seen.begin(), seen.end(), sl.frames[i].stream) == seen.end()) {
                        seen.push_back(sl.frames[i].stream);
                        S[sl.frames[i].stream].inflight++;
                    }
                }
                for (int s : sl.merge_streams) S[s].merge_inflight = true;
                hipStream_t st = sl.st;
                bool ok = hipEventRecord(sl.start, st) == hipSuccess;
                if (ok) ok = hipMemcpyAsync(sl.d_frames, sl.h_frames, sizeof(ServeFrameDev) * (nt + nc),
                                         hipMemcpyHostToDevice, st) == hipSuccess;
                if (ok && n_jobs)
                    ok = hipMemcpyAsync(sl.d_jobs, sl.h_jobs, sizeof(MergeJobDev) * n_jobs, hipMemcpyHostToDevice, st) == hipSuccess;
                if (ok) ok = cfg->ingest(cfg->ingest_ctx, sl.items, nt + nc, st) == 0;
                if (ok) ok = hipEventRecord(sl.k0, st) == hipSuccess;
                if (ok) {
                    hipLaunchKernelGGL(serve_zero_kernel, dim3(8, nt + nc), dim3(256), 0, st,
                                       (const ServeFrameDev *)sl.d_frames);
                    {
                        // equal runs of groups, at least kMinChunk per workgroup
                        // so that a small batch does not pay for idle workgroups
                        const int64_t kMinChunk = 2048;
                        int64_t grid = std::min<int64_t>((n_groups + kMinChunk - 1) / kMinChunk, (int64_t)cus * 2);
                        grid = std::max<int64_t>(grid, 1);
                        const int64_t chunk = (((n_groups + grid - 1) / grid) + 3) & ~int64_t(3);
                        grid = (n_groups + chunk - 1) / chunk;
                        ServeArgs b{sl.d_frames, nt + nc, n_groups, chunk};
                        hipLaunchKernelGGL(serve_kernel, dim3((unsigned)grid), dim3(kServeBlock), 0, st, b);
                    }
                    if (n_jobs) {
                        int maxw = 1;
                        for (int i = 0; i < n_jobs; ++i) maxw = std::max(maxw, sl.h_jobs[i].words);
                        hipLaunchKernelGGL(serve_merge_kernel, dim3((maxw + 255) / 256, n_jobs), dim3(256), 0, st,
                                           (const MergeJobDev *)sl.d_jobs);
                    }
                    if (ok) ok = hipEventRecord(sl.k1, st) == hipSuccess;
                    if (nc && cfg->checksums) {
                        ok = hipMemsetAsync(sl.d_sum, 0, sizeof(unsigned long long) * nc, st) == hipSuccess;
                        hipLaunchKernelGGL(serve_checksum_kernel, dim3(16, nc), dim3(256), 0, st,
                                           (const ServeFrameDev *)(sl.d_frames + nt), sl.d_sum);
                        if (ok)
                            ok = hipMemcpyAsync(sl.h_sum, sl.d_sum, sizeof(unsigned long long) * nc,
                                                hipMemcpyDeviceToHost, st) == hipSuccess;
                    }
                    for (int w = 0; ok && w < cfg->n_watch; ++w) {
                        const int s = cfg->watch_streams[w];
                        for (auto &pf : test_list)
                            if (pf.stream == s && pf.frame - S[s].cfg.n_train < cfg->watch_max_frames)
                                ok = hipMemcpyAsync(cfg->watch_masks[w] + (int64_t)(pf.frame - S[s].cfg.n_train) *
                                                                              (S[s].mask_bytes / 8),
                                                    pf.mask, S[s].mask_bytes, hipMemcpyDeviceToHost, st) == hipSuccess;
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
                merges += n_jobs;
                launched = true;
            }
        }
        if (launched || progressed) idle_since = -1;
        if (!launched && !progressed) {
            bool any_busy = false;
            for (auto &sl : slots) any_busy = any_busy || sl.busy;
            // nothing in flight holds arena memory: a frame that does not
            // fit now never will
            if (!any_busy && waiting >= 0 && !S[waiting].queued.empty()) {
                const StreamState &ws = S[waiting];
                if (frame_block(ws, ws.queued.front() >= ws.cfg.n_train) > arena.largest()) {
                    rc = sfail(OBG_ENOMEM, "budget too small for one frame");
                    break;
                }
            }
            // with nothing in flight every queued frame is admissible; frames
            // that stay queued would mean a scheduling fault: stop, do not spin
            bool any_queued = false;
            for (auto &ss : S) any_queued = any_queued || !ss.queued.empty();
            if (!any_busy && any_queued) {
                if (idle_since < 0) idle_since = wall_now();
                if (wall_now() - idle_since > 2.0) {
                    rc = sfail(OBG_EHIP, "serving loop stalled with frames queued and nothing in flight");
                    break;
                }
            } else {
                idle_since = -1;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    const double wall = wall_now();
    for (auto &sl : slots)
        if (sl.st) (void)hipStreamSynchronize(sl.st);
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
    stats->admission_waits = admission_waits;
    stats->wall_s = wall;
    stats->lat_p50_ms = pct(0.50);
    stats->lat_p99_ms = pct(0.99);
    stats->lat_max_ms = lat.empty() ? 0.0 : lat.back();
    double sum = 0;
    for (double v : lat) sum += v;
    stats->lat_mean_ms = lat.empty() ? 0.0 : sum / lat.size();
    stats->peak_bytes = (double)arena.peak;
    stats->train_pixels = train_pixels;
    stats->test_pixels = test_pixels;
    stats->busy_s = union_length(busy_iv) * 1e-3;
    stats->path_busy_s = union_length(path_iv) * 1e-3;
    (void)wall0;
    for (auto &sl : slots) {
        if (sl.st) (void)hipStreamDestroy(sl.st);
        for (hipEvent_t ev : {sl.done, sl.start, sl.k0, sl.k1})
            if (ev) (void)hipEventDestroy(ev);
        if (sl.h_frames) (void)hipHostFree(sl.h_frames);
        if (sl.d_frames) (void)hipFree(sl.d_frames);
        if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
        if (sl.d_jobs) (void)hipFree(sl.d_jobs);
        if (sl.h_sum) (void)hipHostFree(sl.h_sum);
        if (sl.d_sum) (void)hipFree(sl.d_sum);
        delete[] sl.items;
    }
    if (t0) (void)hipEventDestroy(t0);
    (void)hipFree(arena.base);
    return rc;
}
