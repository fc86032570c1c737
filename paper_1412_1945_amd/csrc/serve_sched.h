// serve_sched.h -- the serving runtime's scheduler: admission under the
// memory budget, batch formation and the per-stream ordering rules.  Plain
// C++ (no device code), so the rules can be exercised on the CPU with a stand-
// in for the device.
//
// Per stream, frames 0 .. n_train-1 train; after the last one the model is
// the merge of their trees (Algorithm 2).  Frame f >= n_train is test frame
// t = f - n_train; after every `period`-th test frame the model becomes the
// merge of the trees of the last `window` frames, and it is used from the
// next frame on (Section 4 names an update of the tree but gives no
// procedure; this is the reading used here).  Frame f's tree goes to ring
// slot f mod ring_len, ring_len = max(n_train, window).
//
// A batch is executed in this order: the trees (and masks) of all its frames,
// then its merges.  The rules below make every stream's result independent of
// what else is in the batch or in flight:
//   * a frame whose merge is due is admitted only when no other batch holds a
//     frame of its stream, and it is the stream's last frame in its batch;
//   * no frame of a stream is admitted while that stream's merge is in flight;
//   * the frames of a stream in flight span fewer than ring_len frame
//     indices, so their ring slots differ (batches may finish out of order);
//   * a frame that does not fit in the budget makes its stream go first, and
//     nothing else is admitted until it fits (no stream starves).
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <set>
#include <vector>

#include "arena.h"

namespace obg {

struct SchedStream {
    int32_t width, height, depth, n_train;
    int32_t n_regions;          // trees per frame (1 without regions)
};

struct SchedFrame {
    int stream, frame;
    bool test;
    int slot;                   // ring slot of the frame's tree
    uint8_t *rgb;               // arena block: pixels, then (test frames) the mask
    uint64_t *mask;
    uint64_t bytes;             // size of the arena block
};

struct SchedMerge {
    int stream;
    int first, n;               // ring window: slots first .. first+n-1 (mod ring_len)
};

struct SchedBatch {
    std::vector<SchedFrame> frames;     // training frames first, then test frames
    std::vector<SchedMerge> merges;
};

// Bytes of one frame buffer (RGB8 rows padded to 16 bytes) and of its mask.
inline uint64_t sched_frame_bytes(const SchedStream &c) {
    return (uint64_t)((3 * (int64_t)c.width + 15) / 16 * 16) * (uint64_t)c.height;
}
inline uint64_t sched_mask_bytes(const SchedStream &c) {
    return (uint64_t)c.height * (uint64_t)((c.width + 63) / 64) * 8u;
}
// Bytes of one frame's trees (one ring slot): n_regions bitsets.
inline uint64_t sched_tree_bytes(const SchedStream &c) {
    const uint64_t keys = 1ull << (3 * c.depth);
    return (keys < 32 ? 4 : keys / 8) * (uint64_t)(c.n_regions > 0 ? c.n_regions : 1);
}

class ServeScheduler {
  public:
    struct Stream {
        SchedStream cfg{};
        int ring_len = 0;
        uint64_t frame_bytes = 0, mask_bytes = 0;
        uint8_t *ring = nullptr, *leaf = nullptr;
        std::deque<int> queued;     // arrived frames waiting for a batch
        int inflight = 0;           // batches holding frames of this stream
        std::set<int> live;         // frames of this stream in those batches
        bool merge_inflight = false;
        bool head_waited = false;   // the first queued frame was refused once already
    };

    Arena arena;
    std::vector<Stream> S;
    int period = 1, window = 1, max_batch = 1;
    int rr = 0;                     // round-robin start among streams
    int waiting = -1;               // stream whose next frame did not fit
    int64_t admission_waits = 0;

    // 0 on success; -1 bad configuration; -2 the budget does not hold the
    // streams' rings and leaf sets.
    int init(const SchedStream *streams, int n, int period_, int window_, int max_batch_, uint8_t *base,
             uint64_t budget) {
        if (n < 1 || period_ < 1 || window_ < 1 || window_ > period_ || max_batch_ < 1) return -1;
        period = period_;
        window = window_;
        max_batch = max_batch_;
        arena.init(base, budget);
        S.assign(n, Stream());
        for (int s = 0; s < n; ++s) {
            Stream &ss = S[s];
            ss.cfg = streams[s];
            if (ss.cfg.width < 1 || ss.cfg.height < 1 || ss.cfg.depth < 1 || ss.cfg.depth > 8 ||
                ss.cfg.n_train < 1)
                return -1;
            ss.ring_len = ss.cfg.n_train > window ? ss.cfg.n_train : window;
            ss.frame_bytes = sched_frame_bytes(ss.cfg);
            ss.mask_bytes = sched_mask_bytes(ss.cfg);
            const uint64_t tb = sched_tree_bytes(ss.cfg);
            ss.ring = arena.get((uint64_t)ss.ring_len * tb);
            ss.leaf = arena.get(tb);
            if (!ss.ring || !ss.leaf) return -2;
        }
        return 0;
    }

    uint64_t block_bytes(const Stream &ss, bool test) const {
        return Arena::round(ss.frame_bytes) + (test ? Arena::round(ss.mask_bytes) : 0);
    }

    // Frame f of stream s has arrived (frames of a stream arrive in order).
    void arrive(int s, int f) { S[s].queued.push_back(f); }

    bool any_queued() const {
        for (auto &ss : S)
            if (!ss.queued.empty()) return true;
        return false;
    }

    // Form the next batch from the arrived frames; false when nothing can go.
    bool form(SchedBatch &b) {
        b.frames.clear();
        b.merges.clear();
        const int ns = (int)S.size();
        std::vector<SchedFrame> train, test;
        int count = 0;
        bool blocked = false;
        // each stream is visited at most once per batch: its frames after
        // one whose merge is due must not join the same batch
        const int first_stream = waiting >= 0 ? waiting : rr;
        for (int k = 0; k < ns && count < max_batch && !blocked; ++k) {
            const int s = (first_stream + k) % ns;
            Stream &ss = S[s];
            const int T = ss.cfg.n_train;
            bool merged_here = false;
            while (!ss.queued.empty() && !ss.merge_inflight && !merged_here && count < max_batch) {
                const int f = ss.queued.front();
                const bool is_test = f >= T;
                const int t = f - T;
                const bool ends_merge = (f == T - 1) || (is_test && (t + 1) % period == 0);
                if (ends_merge && ss.inflight > 0) break;
                if (!ss.live.empty() && f - *ss.live.begin() >= ss.ring_len) break;
                SchedFrame fr{s, f, is_test, f % ss.ring_len, nullptr, nullptr, block_bytes(ss, is_test)};
                fr.rgb = arena.get(fr.bytes);
                if (!fr.rgb) {
                    if (!ss.head_waited) ++admission_waits;
                    ss.head_waited = true;
                    waiting = s;
                    blocked = true;
                    break;
                }
                ss.head_waited = false;
                if (waiting == s) waiting = -1;
                if (is_test) fr.mask = reinterpret_cast<uint64_t *>(fr.rgb + Arena::round(ss.frame_bytes));
                ss.queued.pop_front();
                ss.live.insert(f);
                ++count;
                (is_test ? test : train).push_back(fr);
                if (ends_merge) {
                    SchedMerge m{s, 0, T};
                    if (f != T - 1) {
                        m.n = window;
                        m.first = ((f - window + 1) % ss.ring_len + ss.ring_len) % ss.ring_len;
                    }
                    b.merges.push_back(m);
                    merged_here = true;
                }
            }
        }
        rr = (rr + 1) % ns;
        if (count == 0) return false;
        b.frames = train;
        b.frames.insert(b.frames.end(), test.begin(), test.end());
        std::vector<int> seen;
        for (auto &fr : b.frames) {
            bool dup = false;
            for (int s : seen) dup = dup || s == fr.stream;
            if (!dup) {
                seen.push_back(fr.stream);
                S[fr.stream].inflight++;
            }
        }
        for (auto &m : b.merges) S[m.stream].merge_inflight = true;
        return true;
    }

    // The batch has finished on the device.
    void complete(const SchedBatch &b) {
        std::vector<int> seen;
        for (auto &fr : b.frames) {
            arena.put(fr.rgb, fr.bytes);
            S[fr.stream].live.erase(fr.frame);
            bool dup = false;
            for (int s : seen) dup = dup || s == fr.stream;
            if (!dup) {
                seen.push_back(fr.stream);
                S[fr.stream].inflight--;
            }
        }
        for (auto &m : b.merges) S[m.stream].merge_inflight = false;
    }

    // With nothing in flight, the refused frame that still does not fit never
    // will: true means the budget cannot hold it.
    bool hopeless() const {
        if (waiting < 0 || S[waiting].queued.empty()) return false;
        const Stream &ws = S[waiting];
        return block_bytes(ws, ws.queued.front() >= ws.cfg.n_train) > arena.largest();
    }
};

// Runs of 16-pixel groups for the `grid` workgroups of one pass over the
// frames of a batch, laid end to end.  Frame f has groups[f] groups (a
// multiple of 4) and costs weight[f] per group, plus part_cost for every
// workgroup that takes a piece of it (loading its leaf set, flushing its
// tree, refilling the pipeline).  Workgroup w takes groups
// [bounds[w], bounds[w+1]) (bounds has grid + 1 entries); the runs cost about
// total / grid each.  A run boundary inside a frame is a multiple of 4 groups
// from the frame's start (whole 64-pixel mask words); one that would leave
// less than half a part's worth of groups on either side moves to the
// frame's edge.  whole[f] = 1 when a single workgroup takes all of frame f.
inline void split_by_cost(const int64_t *groups, const int32_t *weight, int n, int64_t part_cost, int grid,
                          int64_t *bounds, uint8_t *whole) {
    std::vector<double> c0(n + 1, 0.0);
    std::vector<int64_t> g0(n + 1, 0);
    for (int f = 0; f < n; ++f) {
        c0[f + 1] = c0[f] + (double)part_cost + (double)groups[f] * weight[f];
        g0[f + 1] = g0[f] + groups[f];
    }
    bounds[0] = 0;
    bounds[grid] = g0[n];
    int f = 0;
    for (int w = 1; w < grid; ++w) {
        const double t = c0[n] * w / grid;
        while (f < n - 1 && c0[f + 1] <= t) ++f;
        int64_t off = 0;
        if (n > 0) {
            const double into = (t - c0[f] - (double)part_cost) / weight[f];
            off = into <= 0 ? 0 : std::min<int64_t>(groups[f], (int64_t)into) & ~int64_t(3);
            const int64_t snap = part_cost / (2 * (int64_t)weight[f]);
            if (off < snap)
                off = 0;
            else if (groups[f] - off < snap)
                off = groups[f];
        }
        bounds[w] = std::max(bounds[w - 1], g0[f] + off);
    }
    int w = 1;
    for (int q = 0; q < n; ++q) {
        while (w < grid && bounds[w] <= g0[q]) ++w;
        whole[q] = (w >= grid || bounds[w] >= g0[q + 1]) ? 1 : 0;
    }
}

}  // namespace obg
