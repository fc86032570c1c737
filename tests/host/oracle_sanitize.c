/* The oracle's whole C interface exercised on random small inputs, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).  Besides
 * memory and arithmetic faults it checks cheap facts: a model rebuilt from
 * its own leaf set classifies identically, Check Color of single pixels
 * agrees with the mask, a frame's trees rebuilt from its exported occupancy
 * export the same bits, and a redrawn pixel keeps the top d bits of each
 * channel.  Exit status 0 = no failure.
 */
#include "../../oracle/octree_oracle.c"

#include <stdio.h>

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(void) {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (uint32_t)rs;
}

static int fails = 0;
#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            if (fails++ < 20) printf("FAIL %s line %d (trial %d)\n", #c, __LINE__, trial); \
        }                                                                       \
    } while (0)

int main(void) {
    int trial;
    for (trial = 0; trial < 400; ++trial) {
        const int W = 1 + (int)(rnd() % 40), H = 1 + (int)(rnd() % 20), d = 1 + (int)(rnd() % 8);
        int rw = 0, rh = 0;
        if (rnd() % 3 == 0) {
            rw = 1 + (int)(rnd() % 24);
            rh = 1 + (int)(rnd() % 12);
        }
        const int64_t pitch = 3 * (int64_t)W + (rnd() % 3) * 16;
        const int T = 1 + (int)(rnd() % 6), nf = T + 2;
        const int ncol = 1 + (int)(rnd() % 12);
        uint8_t pal[12][3];
        for (int c = 0; c < ncol; ++c)
            for (int k = 0; k < 3; ++k) pal[c][k] = (uint8_t)rnd();
        uint8_t *frames = (uint8_t *)malloc((size_t)nf * H * pitch);
        for (int64_t i = 0; i < (int64_t)nf * H * pitch; ++i) frames[i] = (uint8_t)rnd();   /* padding too */
        for (int t = 0; t < nf; ++t)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    const int c = (int)(rnd() % ncol);
                    memcpy(frames + ((int64_t)t * H + y) * pitch + 3 * x, pal[c], 3);
                }
        Forest *f = orc_forest_new(W, H, d, rw, rh);
        CHECK(f != NULL);
        if (!f) {
            free(frames);
            continue;
        }
        const int nreg = orc_forest_regions(f);
        const int64_t words = d >= 2 ? (1 << (3 * d - 5)) : 1, keys = 1ll << (3 * d);
        int32_t idx[8];
        for (int t = 0; t < T; ++t) idx[t] = orc_forest_add_frame(f, frames + (int64_t)t * H * pitch, pitch, (trial & 1) ? 8 : d);
        const uint8_t *grp[2] = {frames + (int64_t)T * H * pitch, frames + (int64_t)(T + 1) * H * pitch};
        const int gi = orc_forest_add_group(f, grp, 2, pitch, d);
        CHECK(gi >= 0);
        uint32_t *occ = (uint32_t *)calloc((size_t)nreg * words, 4);
        uint32_t *occ2 = (uint32_t *)calloc((size_t)nreg * words, 4);
        uint32_t *cnt = d <= 5 ? (uint32_t *)calloc((size_t)nreg * keys, 4) : NULL;
        for (int t = 0; t < T; ++t) {
            CHECK(orc_forest_frame_export(f, idx[t], occ, cnt) == 0);
            CHECK(orc_forest_frame_nodes(f, idx[t]) > 0);
            if (cnt) {
                uint64_t total = 0;
                for (int64_t k = 0; k < (int64_t)nreg * keys; ++k) total += cnt[k];
                CHECK(total == (uint64_t)W * H);
            }
            /* trees rebuilt from the occupancy export the same bits (the
             * rebuild walks all 8^d keys: small depths only) */
            if (d <= 6) {
                const int oi = orc_forest_add_occupancy(f, occ);
                CHECK(orc_forest_frame_export(f, oi, occ2, NULL) == 0);
                CHECK(memcmp(occ, occ2, (size_t)nreg * words * 4) == 0);
                orc_forest_drop_frame(f, oi);
            }
        }
        const uint32_t den = 1 + rnd() % 10, num = 1 + rnd() % (den + 2);
        Model *m = orc_merge(f, idx, T, num, den);
        CHECK(m != NULL);
        uint32_t *leaf = (uint32_t *)calloc((size_t)nreg * words, 4);
        int64_t dang = 0;
        CHECK(orc_model_leafset(m, leaf, &dang) == 0);
        const int mw = (W + 63) / 64;
        uint64_t *mask = (uint64_t *)calloc((size_t)H * mw, 8), *mask2 = (uint64_t *)calloc((size_t)H * mw, 8);
        const uint8_t *test = frames + (int64_t)T * H * pitch;
        CHECK(orc_classify(m, test, pitch, mask) == 0);
        Model *m2 = d <= 6 ? orc_model_from_leafset(W, H, d, rw, rh, leaf) : NULL;
        if (m2) {
            CHECK(orc_classify(m2, test, pitch, mask2) == 0);
            CHECK(memcmp(mask, mask2, (size_t)H * mw * 8) == 0);
        }
        for (int k = 0; k < 8; ++k) {
            const int x = (int)(rnd() % W), y = (int)(rnd() % H);
            const uint8_t *p = test + (int64_t)y * pitch + 3 * x;
            const int fg = (int)((mask[(int64_t)y * mw + (x >> 6)] >> (x & 63)) & 1u);
            CHECK(orc_check_pixel(m, x, y, p[0], p[1], p[2]) == !fg);
        }
        uint8_t *out = (uint8_t *)malloc((size_t)H * pitch);
        CHECK(orc_redraw(f, idx[0], frames, pitch, out, pitch) == 0);
        const uint8_t keep = (uint8_t)(0xFFu << (8 - d));
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < 3 * W; ++x) CHECK(out[(int64_t)y * pitch + x] == (frames[(int64_t)y * pitch + x] & keep));
        orc_forest_drop_frame(f, idx[0]);
        CHECK(orc_forest_frame_export(f, idx[0], occ, NULL) != 0);
        free(out);
        free(mask);
        free(mask2);
        free(leaf);
        orc_model_free(m);
        orc_model_free(m2);
        free(occ);
        free(occ2);
        free(cnt);
        orc_forest_free(f);
        free(frames);
    }
    orc_release_pool();
    printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
