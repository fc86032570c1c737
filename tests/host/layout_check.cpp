// Host-side checks of the GPU library's index helpers (compiled for the CPU
// only): exact division by invariant integers and the key <-> LDS-index
// permutation.  Exit status 0 = all checks passed.
#include <stdio.h>
#include <stdlib.h>
#include "../../paper_1412_1945_amd/csrc/device.h"

using namespace obg;

static int fails = 0;
#define CHECK(c) do { if (!(c)) { if (fails++ < 10) printf("FAIL %s line %d\n", #c, __LINE__); } } while (0)

// Word-level conversion between key order and an LDS order (eight nibbles per
// key word) against the bit-by-bit definition, on random tables.
template <int D, int LAY>
static void check_words(uint64_t seed) {
    const uint32_t nkeys = 1u << (3 * D), kwords = nkeys / 32, lw = (uint32_t)lds_words(D, LAY);
    uint32_t *key = (uint32_t *)calloc(kwords, 4), *tab = (uint32_t *)calloc(lw, 4),
             *tab2 = (uint32_t *)calloc(lw, 4);
    for (int trial = 0; trial < 3; ++trial) {
        for (uint32_t i = 0; i < kwords; ++i) {
            seed ^= seed << 13; seed ^= seed >> 7; seed ^= seed << 17;
            key[i] = trial == 0 ? (uint32_t)seed : trial == 1 ? (uint32_t)seed & (uint32_t)(seed >> 32) : 0xFFFFFFFFu;
        }
        // definition: bit k of the key bitset is bit lds_from_key(k) of the table
        for (uint32_t i = 0; i < lw; ++i) tab[i] = tab2[i] = 0;
        for (uint32_t k = 0; k < nkeys; ++k)
            if ((key[k >> 5] >> (k & 31)) & 1u) {
                const uint32_t l = lds_from_key(k, D, LAY);
                tab[l >> 5] |= 1u << (l & 31);
            }
        for (uint32_t kw = 0; kw < kwords; ++kw)
            key_word_to_table<D, LAY>(key[kw], kw, [&](uint32_t w, uint32_t m) {
                CHECK(w < lw);
                if (w < lw) tab2[w] |= m;
            });
        for (uint32_t i = 0; i < lw; ++i) CHECK(tab[i] == tab2[i]);
        for (uint32_t kw = 0; kw < kwords; ++kw) CHECK((key_word_from_table<D, LAY>(tab, kw) == key[kw]));
        // dual tables: word 2w the leaf set's word w, word 2w + 1 the
        // occupancy's (the other words filled with noise that each direction
        // must ignore)
        uint32_t *dt = (uint32_t *)calloc(2 * lw, 4), *dt2 = (uint32_t *)calloc(2 * lw, 4);
        for (uint32_t k = 0; k < nkeys; ++k) {
            const uint32_t l = lds_from_key(k, D, LAY);
            seed ^= seed << 13; seed ^= seed >> 7; seed ^= seed << 17;
            if ((key[k >> 5] >> (k & 31)) & 1u) dt[2 * (l >> 5) + 1] |= 1u << (l & 31);   // occupancy
            if (seed & 1) dt[2 * (l >> 5)] |= 1u << (l & 31);                             // leaf noise
        }
        for (uint32_t kw = 0; kw < kwords; ++kw) CHECK((key_word_from_table<D, LAY, true>(dt, kw) == key[kw]));
        for (uint32_t kw = 0; kw < kwords; ++kw)
            key_word_to_table<D, LAY, true>(key[kw], kw, [&](uint32_t w, uint32_t m) {
                CHECK(w < 2 * lw);
                CHECK(w % 2 == 0);
                if (w < 2 * lw) dt2[w] |= m;
            });
        for (uint32_t k = 0; k < nkeys; ++k) {
            const uint32_t l = lds_from_key(k, D, LAY);
            CHECK((((dt2[2 * (l >> 5)] >> (l & 31)) & 1u) == ((key[k >> 5] >> (k & 31)) & 1u)));
        }
        free(dt);
        free(dt2);
    }
    free(key);
    free(tab);
    free(tab2);
}

// d = 4, compact order: the four-word gather equals the one-word gather for
// every quad of key words, plain and dual tables.
static void check_quads(uint64_t seed) {
    const uint32_t lw = (uint32_t)lds_words(4, LAY_COMPACT);
    uint32_t tab[128], dt[256];
    for (int trial = 0; trial < 20; ++trial) {
        for (uint32_t i = 0; i < lw; ++i) {
            seed ^= seed << 13; seed ^= seed >> 7; seed ^= seed << 17;
            tab[i] = trial % 3 == 0 ? (uint32_t)seed : trial % 3 == 1 ? (uint32_t)seed & (uint32_t)(seed >> 32) : 0u;
        }
        for (uint32_t i = 0; i < 2 * lw; ++i) {
            seed ^= seed << 13; seed ^= seed >> 7; seed ^= seed << 17;
            dt[i] = (uint32_t)seed;
        }
        for (uint32_t q = 0; q < 32; ++q) {
            const uint32_t kw0 = (q & 1u) | ((q & 6u) << 1) | ((q & 0x18u) << 2);
            CHECK((kw0 & 0x12u) == 0);
            uint32_t out[4], outd[4];
            key_quad_from_table_d4(tab, kw0, out);
            key_quad_from_table_d4<true>(dt, kw0, outd);
            for (int j = 0; j < 4; ++j) {
                const uint32_t kw = kw0 + 2u * (uint32_t)(j & 1) + 16u * (uint32_t)(j >> 1);
                CHECK(out[j] == (key_word_from_table<4, LAY_COMPACT>(tab, kw)));
                CHECK(outd[j] == (key_word_from_table<4, LAY_COMPACT, true>(dt, kw)));
            }
        }
    }
    // the 32 quads cover the 128 key words once each
    int seen[128] = {0};
    for (uint32_t q = 0; q < 32; ++q) {
        const uint32_t kw0 = (q & 1u) | ((q & 6u) << 1) | ((q & 0x18u) << 2);
        for (int j = 0; j < 4; ++j) ++seen[kw0 + 2 * (j & 1) + 16 * (j >> 1)];
    }
    for (int i = 0; i < 128; ++i) CHECK(seen[i] == 1);
}

int main() {
    check_quads(12345);
    // the conversion loops' split of lds_from_key(32 kw) into a lane part
    // (tid mod KW) and a part common to a wave's lanes (kw - tid mod KW)
    for (int lay = 0; lay < 2; ++lay)
        for (int d = 2; d <= (lay == LAY_WIDE ? 5 : 6); ++d) {
            const int kwords = 1 << (3 * d - 5);
            for (int nt = 256; nt <= 1024; nt *= 2)
                for (int tid = 0; tid < nt; tid += 7)
                    for (int i = tid; i < 4 * kwords; i += nt) {
                        const int kw = i % kwords, t = tid % kwords;
                        const int u = kw - t;
                        CHECK(u >= 0);
                        CHECK(((u & t) == 0));
                        CHECK((lds_from_key((uint32_t)t << 5, d, lay) | lds_from_key((uint32_t)u << 5, d, lay)) ==
                              lds_from_key((uint32_t)kw << 5, d, lay));
                        if (kwords < nt) CHECK(u == 0);
                        if (kwords >= nt) CHECK(u == (i - tid) % kwords);   // the same for every lane of the step
                    }
        }
    check_words<2, LAY_WIDE>(1); check_words<3, LAY_WIDE>(2); check_words<4, LAY_WIDE>(3);
    check_words<5, LAY_WIDE>(4);
    check_words<2, LAY_COMPACT>(5); check_words<3, LAY_COMPACT>(6); check_words<4, LAY_COMPACT>(7);
    check_words<5, LAY_COMPACT>(8); check_words<6, LAY_COMPACT>(9); check_words<7, LAY_COMPACT>(10);
    check_words<8, LAY_COMPACT>(11);

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
    // key <-> LDS index in both LDS orders: inverse pair, injective, inside
    // the table, and the key of (R', G', B') is the base-8 path of Algorithm 1
    for (int lay = 0; lay < 2; ++lay) {
        for (int d = 1; d <= (lay == LAY_WIDE ? 5 : 8); ++d) {
            const uint32_t n = 1u << (3 * d);
            const uint32_t lsize = (uint32_t)lds_words(d, lay) * 32u;
            unsigned char *seen = (unsigned char *)calloc(lsize, 1);
            for (uint32_t k = 0; k < n; ++k) {
                uint32_t l = lds_from_key(k, d, lay);
                CHECK(l < lsize);
                if (l >= lsize) continue;
                CHECK(!seen[l]);
                seen[l] = 1;
                CHECK(key_from_lds(l, d, lay) == k);
                uint32_t R, G, B;
                if (lay == LAY_WIDE) { R = (l >> 5) & ((1u << d) - 1); G = l >> 13; B = l & 31; }
                else { R = l >> (2 * d); G = (l >> d) & ((1u << d) - 1); B = l & ((1u << d) - 1); }
                uint32_t path = 0;
                for (int i = 0; i < d; ++i) {
                    int b = d - 1 - i;
                    path = path * 8 + (((R >> b) & 1) << 2) + (((G >> b) & 1) << 1) + ((B >> b) & 1);
                }
                CHECK(path == k);
            }
            free(seen);
            // splitting a key into high and low bits splits the map too
            for (uint32_t k = 0; k < n; k += 37)
                CHECK(lds_from_key(k, d, lay) == (lds_from_key(k & ~31u, d, lay) | lds_from_key(k & 31u, d, lay)));
        }
    }
    // wide order: the byte address the kernel forms from a pixel's R,G bytes
    // is 4 * (L >> 5), and B' is L & 31
    for (int d = 1; d <= 5; ++d)
        for (uint32_t R = 0; R < 256; R += 3)
            for (uint32_t G = 0; G < 256; G += 5)
                for (uint32_t B = 0; B < 256; B += 7) {
                    const uint32_t s = 8 - d;
                    uint32_t k = 0;
                    for (int i = 0; i < d; ++i) {
                        int b = 7 - i;
                        k = k * 8 + (((R >> b) & 1) << 2) + (((G >> b) & 1) << 1) + ((B >> b) & 1);
                    }
                    const uint32_t l = lds_from_key(k, d, LAY_WIDE);
                    const uint32_t rg = (R | (G << 8)) >> (6 - d);          // R byte below G byte
                    const uint32_t M = (((1u << d) - 1u) << 2) | (((1u << d) - 1u) << 10);
                    CHECK((rg & M) == 4 * (l >> 5));
                    CHECK((B >> s) == (l & 31));
                }
    printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
