// Host-side check of the serving scheduler with a stand-in for the device.
//
// Random streams, budgets, batch limits and arrival orders; batches finish in
// a random order.  The stand-in records what each batch reads and writes (ring
// slots and leaf sets of its streams) and checks that no two batches in flight
// touch the same item with at least one of them writing it, so any overlap on
// the device gives the same result.  At completion it applies the batch in its
// execution order (frames, then merges) and checks, per stream, that:
//   * every frame runs exactly once;
//   * every merge reads exactly the trees of its window (frames 0 .. T-1 for
//     the first model, the last `window` frames for a re-merge);
//   * test frame t is classified with model 1 + t / period (model 1 = the
//     merge of the training frames).
// A budget too small for some frame must end in `hopeless()`, never in a
// stall.  Exit status 0 = all checks passed.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "../../paper_1412_1945_amd/csrc/serve_sched.h"

using namespace obg;

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            if (fails++ < 20) printf("FAIL %s line %d (trial %d)\n", #c, __LINE__, trial); \
        }                                                                  \
    } while (0)

static uint64_t rs = 0x2545F4914F6CDD1Dull;
static uint64_t rnd() {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}
static int rint(int lo, int hi) { return lo + (int)(rnd() % (uint64_t)(hi - lo + 1)); }

struct Access {
    int stream, kind, idx;   // kind 0: ring slot idx; kind 1: leaf set
    bool write;
};

static std::vector<Access> accesses(const ServeScheduler &sc, const SchedBatch &b) {
    std::vector<Access> v;
    for (auto &f : b.frames) {
        v.push_back({f.stream, 0, f.slot, true});
        if (f.test) v.push_back({f.stream, 1, 0, false});
    }
    for (auto &m : b.merges) {
        const int R = sc.S[m.stream].ring_len;
        for (int j = 0; j < m.n; ++j) v.push_back({m.stream, 0, (m.first + j) % R, false});
        v.push_back({m.stream, 1, 0, true});
    }
    return v;
}

static bool conflict(const std::vector<Access> &a, const std::vector<Access> &b) {
    for (auto &x : a)
        for (auto &y : b)
            if (x.stream == y.stream && x.kind == y.kind && x.idx == y.idx && (x.write || y.write)) return true;
    return false;
}

// split_by_cost: the runs of serve_kernel's workgroups cover the group space
// in order, cut inside frames only at multiples of 4 groups, flag exactly the
// frames that one run holds whole, and cost at most total / grid plus the
// pieces' overhead and the snapping slack each.
static void check_split() {
    int trial = 0;
    for (trial = 0; trial < 4000; ++trial) {
        const int n = rint(1, 300);
        const int grid = rint(1, 600);
        const int64_t part = rint(0, 3) == 0 ? 0 : (int64_t)rint(1, 200000);
        std::vector<int64_t> groups(n), g0(n + 1, 0);
        std::vector<int32_t> weight(n);
        for (int f = 0; f < n; ++f) {
            const int kind = rint(0, 3);
            groups[f] = 4 * (int64_t)(kind == 0 ? rint(1, 8) : kind == 1 ? rint(1, 2000) : rint(1, 150000));
            weight[f] = rint(60, 80);
            g0[f + 1] = g0[f] + groups[f];
        }
        std::vector<int64_t> b(grid + 1, -1);
        std::vector<uint8_t> whole(n, 7);
        split_by_cost(groups.data(), weight.data(), n, part, grid, b.data(), whole.data());
        CHECK(b[0] == 0 && b[grid] == g0[n]);
        double total = 0;
        int32_t wmax = 0;
        for (int f = 0; f < n; ++f) {
            total += (double)part + (double)groups[f] * weight[f];
            wmax = std::max(wmax, weight[f]);
        }
        for (int w = 0; w < grid; ++w) {
            CHECK(b[w] <= b[w + 1]);
            // a cut inside frame f is 4-aligned from its start
            const int f = (int)(std::upper_bound(g0.begin(), g0.end(), b[w]) - g0.begin()) - 1;
            if (f >= 0 && f < n) CHECK((b[w] - g0[f]) % 4 == 0);
            // cost of the run: groups by weight, one piece overhead per frame touched
            double c = 0;
            for (int q = 0; q < n; ++q) {
                const int64_t lo = std::max(b[w], g0[q]), hi = std::min(b[w + 1], g0[q + 1]);
                if (hi > lo) c += (double)part + (double)(hi - lo) * weight[q];
            }
            CHECK(c <= total / grid + 2.0 * (double)part + 8.0 * wmax + 1.0);
        }
        for (int f = 0; f < n; ++f) {
            bool cut = false;
            for (int w = 1; w < grid; ++w) cut = cut || (b[w] > g0[f] && b[w] < g0[f + 1]);
            CHECK(whole[f] == (cut ? 0 : 1));
        }
    }
}

int main() {
    int trial = 0, hopeless_runs = 0, waits_runs = 0, batches_total = 0;
    for (trial = 0; trial < 3000; ++trial) {
        const int ns = rint(1, 6);
        const int period = rint(1, 12);
        const int window = rint(1, period);
        const int max_batch = rint(1, 12);
        const int max_inflight = rint(1, 4);
        std::vector<SchedStream> cfg(ns);
        std::vector<int> n_frames(ns);
        uint64_t state = 0, largest = 0;
        for (int s = 0; s < ns; ++s) {
            cfg[s] = {rint(1, 200), rint(1, 40), rint(1, 6), rint(1, 12), rint(0, 3) == 0 ? rint(2, 9) : 1};
            n_frames[s] = cfg[s].n_train + rint(0, 40);
            const uint64_t tb = sched_tree_bytes(cfg[s]);
            const int R = std::max(cfg[s].n_train, window);
            state += Arena::round((uint64_t)R * tb) + Arena::round(tb);
            largest = std::max(largest, Arena::round(sched_frame_bytes(cfg[s])) + Arena::round(sched_mask_bytes(cfg[s])));
        }
        // budgets: tight (about one frame), roomy, and (rarely) too small
        uint64_t budget = state;
        const int kind = rint(0, 9);
        if (kind == 0)
            budget += largest - 256;
        else if (kind <= 5)
            budget += largest + (uint64_t)rint(0, 3) * 256;
        else
            budget += largest * (uint64_t)rint(2, 12);
        ServeScheduler sc;
        uint8_t *base = reinterpret_cast<uint8_t *>(uintptr_t(1) << 40);   // never dereferenced
        CHECK(sc.init(cfg.data(), ns, period, window, max_batch, base, budget) == 0);
        // arrival order: per stream increasing, streams interleaved at random
        std::vector<int> order;
        for (int s = 0; s < ns; ++s)
            for (int f = 0; f < n_frames[s]; ++f) order.push_back(s);
        for (size_t i = order.size(); i > 1; --i) std::swap(order[i - 1], order[rnd() % i]);
        std::vector<int> next(ns, 0);
        size_t arrived = 0;
        // stand-in device state
        std::vector<std::vector<int>> ring(ns), used(ns);
        std::vector<std::vector<char>> done(ns);
        std::vector<int> version(ns, 0);
        for (int s = 0; s < ns; ++s) {
            ring[s].assign(sc.S[s].ring_len, -1);
            used[s].assign(n_frames[s], -1);
            done[s].assign(n_frames[s], 0);
        }
        struct InFlight {
            SchedBatch b;
            std::vector<Access> acc;
        };
        std::vector<InFlight> fly;
        size_t executed = 0, total = order.size();
        bool gave_up = false;
        int guard = 0;
        while (executed < total && ++guard < 1000000) {
            // some arrivals
            if (arrived < total && rint(0, 2) == 0) {
                const int k = rint(1, 8);
                for (int i = 0; i < k && arrived < total; ++i, ++arrived) {
                    const int s = order[arrived];
                    sc.arrive(s, next[s]++);
                }
            }
            const bool try_form = (int)fly.size() < max_inflight && rint(0, 1) == 0;
            SchedBatch b;
            if (try_form && sc.form(b)) {
                ++batches_total;
                // batch shape: per stream increasing frames; a merge only after its stream's last frame
                for (auto &m : b.merges) {
                    int last = -1;
                    for (auto &f : b.frames)
                        if (f.stream == m.stream) last = std::max(last, f.frame);
                    CHECK(last >= 0);
                    const int T = cfg[m.stream].n_train;
                    CHECK(last == T - 1 || (last >= T && (last - T + 1) % period == 0));
                }
                InFlight fl{b, accesses(sc, b)};
                for (auto &o : fly) CHECK(!conflict(fl.acc, o.acc));
                fly.push_back(fl);
                continue;
            }
            if (!fly.empty() && (rint(0, 1) == 0 || (int)fly.size() == max_inflight || arrived == total)) {
                const size_t i = rnd() % fly.size();
                const SchedBatch &d = fly[i].b;
                for (auto &f : d.frames) {
                    CHECK(!done[f.stream][f.frame]);
                    done[f.stream][f.frame] = 1;
                    ring[f.stream][f.slot] = f.frame;
                    if (f.test) used[f.stream][f.frame] = version[f.stream];
                    ++executed;
                }
                for (auto &m : d.merges) {
                    int last = -1;
                    for (auto &f : d.frames)
                        if (f.stream == m.stream) last = std::max(last, f.frame);
                    const int T = cfg[m.stream].n_train;
                    const int R = sc.S[m.stream].ring_len;
                    const int n = last == T - 1 ? T : window;
                    CHECK(m.n == n);
                    for (int j = 0; j < m.n; ++j) CHECK(ring[m.stream][(m.first + j) % R] == last - m.n + 1 + j);
                    version[m.stream]++;
                }
                sc.complete(d);
                fly.erase(fly.begin() + i);
                continue;
            }
            if (fly.empty() && arrived == total) {
                // nothing in flight and everything arrived: a batch must form
                // unless the refused frame can never fit
                if (!sc.form(b)) {
                    CHECK(sc.any_queued());
                    CHECK(sc.hopeless());
                    CHECK(kind == 0);
                    gave_up = true;
                    break;
                }
                ++batches_total;
                InFlight fl{b, accesses(sc, b)};
                fly.push_back(fl);
            }
        }
        CHECK(guard < 1000000);
        if (gave_up) {
            ++hopeless_runs;
            continue;
        }
        CHECK(executed == total);
        CHECK(sc.arena.in_use == state);
        if (sc.admission_waits > 0) ++waits_runs;
        for (int s = 0; s < ns; ++s) {
            const int T = cfg[s].n_train;
            for (int f = T; f < n_frames[s]; ++f) CHECK(used[s][f] == 1 + (f - T) / period);
        }
    }
    trial = -1;
    CHECK(hopeless_runs > 0);
    CHECK(waits_runs > 100);
    check_split();
    if (fails) {
        printf("%d checks failed\n", fails);
        return 1;
    }
    printf("scheduler ok: %d batches, %d runs with admission waits, %d runs with a budget below one frame\n",
           batches_total, waits_runs, hopeless_runs);
    return 0;
}
