// Host-side checks of the GPU library's index helpers (compiled for the CPU
// only): exact division by invariant integers and the key <-> LDS-index
// permutation.  Exit status 0 = all checks passed.
#include <stdio.h>
#include <stdlib.h>
#include "../../paper_1412_1945_amd/csrc/device.h"

using namespace obg;

static int fails = 0;
#define CHECK(c) do { if (!(c)) { if (fails++ < 10) printf("FAIL %s line %d\n", #c, __LINE__); } } while (0)

int main() {
    // divisors: groups per row (4*ceil(W/64)), region widths / 16, and more
    const uint32_t ds[] = {1, 2, 3, 4, 5, 7, 8, 12, 20, 60, 120, 240, 255, 256, 257, 1000, 4095,
                           65535, 65536, 65537, 1u << 20, (1u << 24) + 1, 0x7FFFFFFFu};
    for (uint32_t d : ds) {
        FastDiv f = make_fastdiv(d);
        for (uint32_t n = 0; n < 300000; ++n) CHECK(fdiv(n, f) == n / d);
        for (uint64_t n = 0xFFFFFFFFull; n > 0xFFFFFFFFull - 300000; --n)
            CHECK(fdiv((uint32_t)n, f) == (uint32_t)n / d);
        for (uint32_t k = 1; k < 4000; ++k) {
            uint64_t n = (uint64_t)k * d;
            if (n > 0xFFFFFFFFull) break;
            CHECK(fdiv((uint32_t)n, f) == k);
            CHECK(fdiv((uint32_t)(n - 1), f) == k - 1);
        }
    }
    // random
    uint64_t s = 88172645463325252ull;
    for (int i = 0; i < 2000000; ++i) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        uint32_t d = (uint32_t)(s >> 33) % 100000 + 1, n = (uint32_t)s;
        CHECK(fdiv(n, make_fastdiv(d)) == n / d);
    }
    // key <-> concat permutation is a bijection and inverse pair; the key of
    // (R', G', B') is the base-8 path of Algorithm 1
    for (int d = 1; d <= 8; ++d) {
        const uint32_t n = 1u << (3 * d);
        for (uint32_t k = 0; k < n; ++k) {
            uint32_t j = concat_from_key(k, d);
            CHECK(j < n);
            CHECK(key_from_concat(j, d) == k);
            uint32_t R = j >> (2 * d), G = (j >> d) & ((1u << d) - 1), B = j & ((1u << d) - 1);
            uint32_t path = 0;
            for (int i = 0; i < d; ++i) {
                int b = d - 1 - i;
                path = path * 8 + (((R >> b) & 1) << 2) + (((G >> b) & 1) << 1) + ((B >> b) & 1);
            }
            CHECK(path == k);
        }
        // splitting a key into high and low bits splits the permutation too
        for (uint32_t k = 0; k < n; k += 37)
            CHECK(concat_from_key(k, d) == (concat_from_key(k & ~31u, d) | concat_from_key(k & 31u, d)));
    }
    printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
