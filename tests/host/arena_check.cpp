// Host-side check of the serving runtime's budget arena: random requests and
// releases against a byte map; blocks never overlap and stay inside the
// budget, freed memory coalesces, and a quiet arena serves any request up to
// its whole size.  Exit status 0 = all checks passed.
#include <stdio.h>
#include <stdlib.h>
#include <vector>
#include "../../paper_1412_1945_amd/csrc/arena.h"

using obg::Arena;

static int fails = 0;
#define CHECK(c) do { if (!(c)) { if (fails++ < 10) printf("FAIL %s line %d\n", #c, __LINE__); } } while (0)

int main() {
    const uint64_t size = 1 << 22;          // 16384 units of 256 B
    std::vector<int> owner(size / 256, -1);
    uint8_t *base = reinterpret_cast<uint8_t *>(uintptr_t(1) << 40);   // never dereferenced
    Arena a;
    a.init(base, size);
    struct Blk { uint8_t *p; uint64_t bytes; };
    std::vector<Blk> live;
    uint64_t s = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; };
    const uint64_t sizes[] = {100, 256, 1000, 4096, 24576, 65536 + 7, 300000};
    int refused = 0;
    for (int it = 0; it < 200000; ++it) {
        if (live.empty() || rnd() % 100 < 55) {
            const uint64_t b = sizes[rnd() % 7];
            uint8_t *p = a.get(b);
            if (!p) {
                ++refused;
                CHECK(a.largest() < Arena::round(b));
                continue;
            }
            const uint64_t off = (uint64_t)(p - base), n = Arena::round(b);
            CHECK(off % 256 == 0 && off + n <= size);
            for (uint64_t u = off / 256; u < (off + n) / 256; ++u) {
                CHECK(owner[u] == -1);
                owner[u] = it;
            }
            live.push_back({p, b});
        } else {
            const size_t k = rnd() % live.size();
            const uint64_t off = (uint64_t)(live[k].p - base), n = Arena::round(live[k].bytes);
            for (uint64_t u = off / 256; u < (off + n) / 256; ++u) owner[u] = -1;
            a.put(live[k].p, live[k].bytes);
            live[k] = live.back();
            live.pop_back();
        }
        uint64_t used = 0;
        if (it % 997 == 0) {
            for (int o : owner) used += o >= 0 ? 256 : 0;
            CHECK(used == a.in_use);
            // free blocks: disjoint from live memory, never adjacent
            uint64_t prev_end = ~0ull;
            for (auto &f : a.free_) {
                CHECK(f.first != prev_end);
                prev_end = f.first + f.second;
                for (uint64_t u = f.first / 256; u < prev_end / 256; ++u) CHECK(owner[u] == -1);
            }
        }
    }
    CHECK(refused > 0);
    for (auto &b : live) a.put(b.p, b.bytes);
    CHECK(a.in_use == 0);
    CHECK(a.free_.size() == 1 && a.largest() == size);
    CHECK(a.get(size) == base);
    if (fails) {
        printf("%d checks failed\n", fails);
        return 1;
    }
    printf("arena ok (%d refusals)\n", refused);
    return 0;
}
