/*
 * octree_oracle.c -- plain CPU model of octree background modelling.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the GPU library never links or calls it,
 * and it shares no code, header or table with the GPU library.
 *
 * It follows the paper ("Background Modeling Using Octree Color Quantization",
 * arXiv 1412.1945) step by step with real pointer octrees, node by node:
 *
 *   - store_color   : Algorithm 1 (Store Color).  One node per level, the child
 *                     index at each level taken from one bit of R, G and B,
 *                     most significant bit first.
 *   - prune_copy    : the level-removal pruning of Section 2: nodes below the
 *                     kept depth are dropped, the exposed nodes become leaves.
 *   - merge_into    : Algorithm 2 (Merge Trees), recursive, Section 3.
 *   - check_color   : Algorithm 3 (Check Color), Section 4.
 *   - regions       : one tree per spatial region, Sections 3 and 4.
 *   - add_group     : one tree holding the colours of a group of frames
 *                     (Section 3 allows a tree per frame or per group).
 *   - redraw        : a frame redrawn with its pruned trees' leaf colours
 *                     (the zero-filled path bits, Section 2).
 *
 * Readings of points the paper leaves open (each one is listed with its
 * justification in the design notes of the repository):
 *   R1  The child index printed as the SUM of the three colour bits cannot
 *       address eight children; it is read as the 3-bit concatenation
 *       4*red_bit + 2*green_bit + blue_bit.
 *   R2  Level i (i = 0 for the first level below the root) uses bit 7-i of
 *       each 8-bit channel; "Number of Levels" is the number of levels below
 *       the root, 1..8.
 *   R3  The merge threshold is a fraction num/den and the test
 *       count/numberOfTrees >= threshold is done exactly as
 *       count*den >= num*numberOfTrees in 64-bit integers.
 *   R4  roots[j].child[i] of an absent roots[j] is read as absent.
 *   R5  The merged leaf set is the set of nodes at the kept depth; nodes left
 *       above that depth without children ("dangling") are reported separately
 *       and never make Check Color return true.
 *   R6  A pixel is foreground (mask bit 1) exactly when Check Color is false.
 *   R7  Regions are a row-major grid of region_w x region_h rectangles
 *       covering the frame (the last row/column may be partial); region id =
 *       (y / region_h) * ceil(W / region_w) + x / region_w.
 *
 * Exported layouts (shared with the GPU library only through their written
 * definition, never through code):
 *   key of a depth-d node = its child indices c_0..c_{d-1} read as base-8
 *     digits, first level most significant;
 *   bitset: bit (k & 31) of 32-bit word (k >> 5), per region
 *     ceil(8^d / 32) words, regions back to back;
 *   mask: per row ceil(W / 64) 64-bit words, pixel x at bit (x & 63) of word
 *     (x >> 6), 1 = foreground, bits past the row end 0.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ORC_MUTANT selects one deliberately planted mistake; the test suite builds
 * each mutant separately and checks that its pins reject every one of them.
 * The normal build leaves it at 0. */
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

/* ------------------------------------------------------------------------ */
/* Nodes and a per-tree arena                                               */

typedef struct Node {
    struct Node *child[8];
    uint64_t pixels;   /* pixels stored at this node (leaves), summed on prune */
} Node;

typedef struct Arena {
    Node **blocks;
    size_t nblocks, cap;
    size_t used;       /* nodes used in the last block */
} Arena;

/* One arena holds every tree of a frame (or of a merged model), so that the
 * nodes of thousands of small region trees come from a few large blocks. */
#define ARENA_BLOCK 8192

/* Freed blocks are kept for reuse, so that building frame after frame does
 * not map fresh memory each time (page faults dominate otherwise). */
static pthread_mutex_t pool_mu = PTHREAD_MUTEX_INITIALIZER;
static Node **pool;
static size_t pool_n, pool_cap;

static Node *block_get(void) {
    Node *blk = NULL;
    pthread_mutex_lock(&pool_mu);
    if (pool_n) blk = pool[--pool_n];
    pthread_mutex_unlock(&pool_mu);
    if (blk) {
        memset(blk, 0, ARENA_BLOCK * sizeof(Node));
        return blk;
    }
    blk = (Node *)calloc(ARENA_BLOCK, sizeof(Node));
    if (!blk) abort();
    return blk;
}

static void block_put(Node *blk) {
    pthread_mutex_lock(&pool_mu);
    if (pool_n == pool_cap) {
        size_t nc = pool_cap ? pool_cap * 2 : 256;
        Node **np = (Node **)realloc(pool, nc * sizeof(Node *));
        if (!np) abort();
        pool = np;
        pool_cap = nc;
    }
    pool[pool_n++] = blk;
    pthread_mutex_unlock(&pool_mu);
}

static Node *new_node(Arena *a) {
    if (a->nblocks == 0 || a->used == ARENA_BLOCK) {
        if (a->nblocks == a->cap) {
            size_t nc = a->cap ? a->cap * 2 : 16;
            Node **nb = (Node **)realloc(a->blocks, nc * sizeof(Node *));
            if (!nb) abort();
            a->blocks = nb;
            a->cap = nc;
        }
        a->blocks[a->nblocks++] = block_get();
        a->used = 0;
    }
    return &a->blocks[a->nblocks - 1][a->used++];
}

static void arena_free(Arena *a) {
    for (size_t i = 0; i < a->nblocks; ++i) block_put(a->blocks[i]);
    free(a->blocks);
    memset(a, 0, sizeof(*a));
}

/* Return pooled blocks to the system (after a large run). */
void orc_release_pool(void) {
    pthread_mutex_lock(&pool_mu);
    for (size_t i = 0; i < pool_n; ++i) free(pool[i]);
    pool_n = 0;
    pthread_mutex_unlock(&pool_mu);
}

static size_t arena_nodes(const Arena *a) {
    return a->nblocks ? (a->nblocks - 1) * ARENA_BLOCK + a->used : 0;
}

/* The trees of one frame (or one merged model): a root per region. */
typedef struct Trees {
    Node **roots;
    Arena arena;
} Trees;

/* ------------------------------------------------------------------------ */
/* Algorithm 1: Store Color                                                 */

/* Child index at level i: one bit of each channel, reading R1 and R2. */
static int child_index(uint8_t r, uint8_t g, uint8_t b, int level) {
    int bit = 7 - level;
#if ORC_MUTANT == 1   /* red and green swapped */
    return (((g >> bit) & 1) << 2) | (((r >> bit) & 1) << 1) | ((b >> bit) & 1);
#elif ORC_MUTANT == 2 /* least significant bit first */
    bit = level;
#endif
    return (((r >> bit) & 1) << 2) | (((g >> bit) & 1) << 1) | ((b >> bit) & 1);
}

static void store_color(Node **root, Arena *a, uint8_t r, uint8_t g, uint8_t b, int levels) {
    if (*root == NULL) *root = new_node(a);
    Node *temp = *root;
    for (int i = 0; i < levels; ++i) {
        int index = child_index(r, g, b, i);
        if (temp->child[index] != NULL) {
            temp = temp->child[index];
        } else {
            temp->child[index] = new_node(a);
            temp = temp->child[index];
        }
    }
    temp->pixels += 1;
}

/* ------------------------------------------------------------------------ */
/* Section 2 pruning: drop every level below `depth`.                       */

static uint64_t subtree_pixels(const Node *n) {
    uint64_t s = n->pixels;
    for (int i = 0; i < 8; ++i)
        if (n->child[i]) s += subtree_pixels(n->child[i]);
    return s;
}

/* Copy the top `depth` levels of `src` into a fresh arena; a node at the
 * kept depth keeps the pixel total of the subtree it replaces. */
static Node *prune_copy(const Node *src, int depth, Arena *dst) {
    if (src == NULL) return NULL;
    Node *n = new_node(dst);
    if (depth == 0) {
        n->pixels = subtree_pixels(src);
        return n;
    }
    n->pixels = src->pixels;
    for (int i = 0; i < 8; ++i)
        if (src->child[i]) n->child[i] = prune_copy(src->child[i], depth - 1, dst);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: Merge Trees                                                 */

/* `result` is the node that stands for the common path so far; `roots` are
 * the n input subtrees at the same path (absent ones NULL, reading R4). */
static void merge_into(Node *result, Node **roots, int n, uint32_t num, uint32_t den,
                       int levels_left, Arena *a) {
    if (levels_left == 0) return;
    for (int i = 0; i < 8; ++i) {
        int count = 0;
        for (int j = 0; j < n; ++j)
#if ORC_MUTANT == 4   /* child test dropped */
            if (roots[j] != NULL) count = count + 1;
#else
            if (roots[j] != NULL && roots[j]->child[i] != NULL) count = count + 1;
#endif
        /* count / numberOfTrees >= threshold, exactly (reading R3) */
#if ORC_MUTANT == 3   /* strict comparison */
        if ((uint64_t)count * den > (uint64_t)num * (uint64_t)n)
#elif ORC_MUTANT == 9 /* numberOfTrees off by one */
        if ((uint64_t)count * den >= (uint64_t)num * (uint64_t)(n + 1))
#else
        if ((uint64_t)count * den >= (uint64_t)num * (uint64_t)n)
#endif
            result->child[i] = new_node(a);
    }
    Node **temp_root = (Node **)malloc((size_t)n * sizeof(Node *));
    if (!temp_root) abort();
    for (int i = 0; i < 8; ++i) {
        if (result->child[i] != NULL) {
            for (int j = 0; j < n; ++j)
                temp_root[j] = roots[j] ? roots[j]->child[i] : NULL;
            merge_into(result->child[i], temp_root, n, num, den, levels_left - 1, a);
        }
    }
    free(temp_root);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3: Check Color                                                 */

static int check_color(const Node *root, uint8_t r, uint8_t g, uint8_t b, int levels) {
    if (root == NULL) return 0;
    const Node *temp = root;
#if ORC_MUTANT == 5   /* last level never checked */
    levels = levels - 1;
#endif
    for (int i = 0; i < levels; ++i) {
        int index = child_index(r, g, b, i);
        if (temp->child[index] != NULL)
            temp = temp->child[index];
        else
            return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Walking a tree to the exported layouts                                   */

static void export_leaves(const Node *n, int level, int depth, uint64_t key,
                          uint32_t *occ, uint32_t *counts) {
    if (level == depth) {
        occ[key >> 5] |= 1u << (key & 31);
        if (counts) counts[key] = (uint32_t)n->pixels;
        return;
    }
    for (int i = 0; i < 8; ++i)
        if (n->child[i]) export_leaves(n->child[i], level + 1, depth, key * 8 + (uint64_t)i, occ, counts);
}

/* Dangling node = node above the kept depth with no child (reading R5).
 * Marked in `dang` per level: bit for key k of depth L at offset dang_off(L). */
static uint64_t count_dangling(const Node *n, int level, int depth) {
    if (level == depth) return 0;
    uint64_t c = 0;
    int kids = 0;
    for (int i = 0; i < 8; ++i)
        if (n->child[i]) { kids++; c += count_dangling(n->child[i], level + 1, depth); }
    return c + (kids == 0 ? 1 : 0);
}

/* Key -> representative colour: the key's d bits per channel followed by
 * zeros (the zero-fill colour of Section 2). */
static void key_colour(uint64_t key, int depth, uint8_t *r, uint8_t *g, uint8_t *b) {
    unsigned R = 0, G = 0, B = 0;
    for (int i = 0; i < depth; ++i) {
        unsigned c = (unsigned)((key >> (3 * (depth - 1 - i))) & 7);
        R |= ((c >> 2) & 1u) << (7 - i);
        G |= ((c >> 1) & 1u) << (7 - i);
        B |= (c & 1u) << (7 - i);
    }
    *r = (uint8_t)R; *g = (uint8_t)G; *b = (uint8_t)B;
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                 */

typedef struct Geom {
    int width, height, depth, region_w, region_h;
    int reg_cols, reg_rows;
} Geom;

static int geom_init(Geom *g, int width, int height, int depth, int region_w, int region_h) {
    if (width < 1 || height < 1 || depth < 1 || depth > 8) return -1;
    if ((region_w == 0) != (region_h == 0) || region_w < 0 || region_h < 0) return -1;
    g->width = width; g->height = height; g->depth = depth;
    g->region_w = region_w ? region_w : width;
    g->region_h = region_h ? region_h : height;
    g->reg_cols = (width + g->region_w - 1) / g->region_w;
    g->reg_rows = (height + g->region_h - 1) / g->region_h;
    return 0;
}

static int geom_regions(const Geom *g) { return g->reg_cols * g->reg_rows; }

static int region_of(const Geom *g, int x, int y) {
#if ORC_MUTANT == 6   /* region grid transposed */
    return (x / g->region_w) * g->reg_rows + y / g->region_h;
#endif
    return (y / g->region_h) * g->reg_cols + x / g->region_w;
}

static uint64_t leaf_words(int depth) {
    uint64_t leaves = 1ull << (3 * depth);
    return (leaves + 31) / 32;
}

/* ------------------------------------------------------------------------ */
/* Forest: the pruned per-frame (per-region) trees                          */

typedef struct Forest {
    Geom g;
    int nframes, cap;
    Trees **frames;    /* [frame] -> trees of that frame (NULL if dropped) */
} Forest;

Forest *orc_forest_new(int width, int height, int depth, int region_w, int region_h) {
    Forest *f = (Forest *)calloc(1, sizeof(Forest));
    if (!f) return NULL;
    if (geom_init(&f->g, width, height, depth, region_w, region_h) != 0) { free(f); return NULL; }
    return f;
}

int orc_forest_regions(const Forest *f) { return geom_regions(&f->g); }

static Trees *trees_new(int nreg) {
    Trees *t = (Trees *)calloc(1, sizeof(Trees));
    if (!t) abort();
    t->roots = (Node **)calloc((size_t)nreg, sizeof(Node *));
    if (!t->roots) abort();
    return t;
}

static void trees_free(Trees *t) {
    if (!t) return;
    arena_free(&t->arena);
    free(t->roots);
    free(t);
}

static int forest_append(Forest *f, Trees *t) {
    if (f->nframes == f->cap) {
        int nc = f->cap ? f->cap * 2 : 16;
        Trees **nt = (Trees **)realloc(f->frames, (size_t)nc * sizeof(Trees *));
        if (!nt) abort();
        f->frames = nt;
        f->cap = nc;
    }
    f->frames[f->nframes] = t;
    return f->nframes++;
}

/* Build the trees of a group of frames: Store Color of every pixel of every
 * frame of the group into its region's tree at `store_levels` levels, then
 * prune each tree to the kept depth.  A group of one frame is a frame's tree;
 * Section 3 allows a tree per frame or per group of frames. */
static int add_group(Forest *f, const uint8_t *const *frames, int n, int64_t row_pitch, int store_levels) {
    const Geom *g = &f->g;
    if (store_levels < g->depth || store_levels > 8 || n < 1) return -1;
    int nreg = geom_regions(g);
    Trees *full = trees_new(nreg);
    Trees *pruned = trees_new(nreg);
#if ORC_MUTANT == 10  /* a group's tree built from its first frame only */
    n = 1;
#endif
    for (int j = 0; j < n; ++j) {
        const uint8_t *rgb = frames[j];
        /* one tree per region, built from that region's pixels (Section 3) */
        for (int ry = 0; ry < g->reg_rows; ++ry) {
            for (int rx = 0; rx < g->reg_cols; ++rx) {
                const int y0 = ry * g->region_h, x0 = rx * g->region_w;
                const int y1 = y0 + g->region_h < g->height ? y0 + g->region_h : g->height;
                const int x1 = x0 + g->region_w < g->width ? x0 + g->region_w : g->width;
                for (int y = y0; y < y1; ++y) {
                    const uint8_t *row = rgb + (int64_t)y * row_pitch;
                    for (int x = x0; x < x1; ++x) {
                        const uint8_t *p = row + 3 * x;
                        store_color(&full->roots[region_of(g, x, y)], &full->arena, p[0], p[1], p[2], store_levels);
                    }
                }
            }
        }
    }
    for (int r = 0; r < nreg; ++r) {
#if ORC_MUTANT == 7   /* one level too many removed, then re-grown by the leaf count */
        pruned->roots[r] = prune_copy(full->roots[r], g->depth > 1 ? g->depth - 1 : 1, &pruned->arena);
#else
        pruned->roots[r] = prune_copy(full->roots[r], g->depth, &pruned->arena);
#endif
    }
    trees_free(full);
    return forest_append(f, pruned);
}

/* One frame's trees. */
int orc_forest_add_frame(Forest *f, const uint8_t *rgb, int64_t row_pitch, int store_levels) {
    return add_group(f, &rgb, 1, row_pitch, store_levels);
}

/* The trees of a group of n frames (all with the same row pitch). */
int orc_forest_add_group(Forest *f, const uint8_t *const *frames, int n, int64_t row_pitch, int store_levels) {
    return add_group(f, frames, n, row_pitch, store_levels);
}

/* Build a frame's trees from an occupancy bitset [n_regions][words]: every
 * set key stores its zero-fill colour at `depth` levels. */
int orc_forest_add_occupancy(Forest *f, const uint32_t *occ) {
    const Geom *g = &f->g;
    int nreg = geom_regions(g);
    uint64_t words = leaf_words(g->depth), leaves = 1ull << (3 * g->depth);
    Trees *t = trees_new(nreg);
    for (int r = 0; r < nreg; ++r) {
        const uint32_t *w = occ + (uint64_t)r * words;
        for (uint64_t k = 0; k < leaves; ++k) {
            if ((w[k >> 5] >> (k & 31)) & 1u) {
                uint8_t R, G, B;
                key_colour(k, g->depth, &R, &G, &B);
                store_color(&t->roots[r], &t->arena, R, G, B, g->depth);
            }
        }
    }
    return forest_append(f, t);
}

int orc_forest_frame_export(const Forest *f, int frame, uint32_t *occ, uint32_t *counts) {
    if (frame < 0 || frame >= f->nframes || f->frames[frame] == NULL) return -1;
    const Geom *g = &f->g;
    int nreg = geom_regions(g);
    uint64_t words = leaf_words(g->depth), leaves = 1ull << (3 * g->depth);
    memset(occ, 0, (size_t)(words * nreg) * sizeof(uint32_t));
    if (counts) memset(counts, 0, (size_t)(leaves * nreg) * sizeof(uint32_t));
    for (int r = 0; r < nreg; ++r) {
        const Node *root = f->frames[frame]->roots[r];
        if (root)
            export_leaves(root, 0, g->depth, 0, occ + (uint64_t)r * words,
                          counts ? counts + (uint64_t)r * leaves : NULL);
    }
    return 0;
}

int64_t orc_forest_frame_nodes(const Forest *f, int frame) {
    if (frame < 0 || frame >= f->nframes || f->frames[frame] == NULL) return -1;
    return (int64_t)arena_nodes(&f->frames[frame]->arena);
}

void orc_forest_drop_frame(Forest *f, int frame) {
    if (frame < 0 || frame >= f->nframes || f->frames[frame] == NULL) return;
    trees_free(f->frames[frame]);
    f->frames[frame] = NULL;
}

void orc_forest_free(Forest *f) {
    if (!f) return;
    for (int i = 0; i < f->nframes; ++i) orc_forest_drop_frame(f, i);
    free(f->frames);
    free(f);
}

/* ------------------------------------------------------------------------ */
/* Model: the merged tree of every region                                   */

typedef struct Model {
    Geom g;
    Trees *trees;      /* one merged root per region */
} Model;

/* Merge the trees of the listed frames, region by region (Algorithm 2). */
Model *orc_merge(const Forest *f, const int32_t *frames, int n, uint32_t num, uint32_t den) {
    if (n < 1 || den == 0) return NULL;
    for (int j = 0; j < n; ++j)
        if (frames[j] < 0 || frames[j] >= f->nframes || f->frames[frames[j]] == NULL) return NULL;
    Model *m = (Model *)calloc(1, sizeof(Model));
    if (!m) abort();
    m->g = f->g;
    int nreg = geom_regions(&f->g);
    m->trees = trees_new(nreg);
    Node **roots = (Node **)malloc((size_t)n * sizeof(Node *));
    if (!roots) abort();
    for (int r = 0; r < nreg; ++r) {
        for (int j = 0; j < n; ++j) roots[j] = f->frames[frames[j]]->roots[r];
        m->trees->roots[r] = new_node(&m->trees->arena);
        merge_into(m->trees->roots[r], roots, n, num, den, f->g.depth, &m->trees->arena);
    }
    free(roots);
    return m;
}

/* A model whose trees hold exactly the keys of a leaf bitset [n_regions][words]. */
Model *orc_model_from_leafset(int width, int height, int depth, int region_w, int region_h,
                              const uint32_t *leaf) {
    Model *m = (Model *)calloc(1, sizeof(Model));
    if (!m) abort();
    if (geom_init(&m->g, width, height, depth, region_w, region_h) != 0) { free(m); return NULL; }
    int nreg = geom_regions(&m->g);
    uint64_t words = leaf_words(depth), leaves = 1ull << (3 * depth);
    m->trees = trees_new(nreg);
    for (int r = 0; r < nreg; ++r) {
        const uint32_t *w = leaf + (uint64_t)r * words;
        for (uint64_t k = 0; k < leaves; ++k)
            if ((w[k >> 5] >> (k & 31)) & 1u) {
                uint8_t R, G, B;
                key_colour(k, depth, &R, &G, &B);
                store_color(&m->trees->roots[r], &m->trees->arena, R, G, B, depth);
            }
    }
    return m;
}

int orc_model_leafset(const Model *m, uint32_t *leaf, int64_t *dangling) {
    int nreg = geom_regions(&m->g);
    uint64_t words = leaf_words(m->g.depth);
    memset(leaf, 0, (size_t)(words * nreg) * sizeof(uint32_t));
    int64_t dang = 0;
    for (int r = 0; r < nreg; ++r) {
        const Node *root = m->trees->roots[r];
        if (root) {
            export_leaves(root, 0, m->g.depth, 0, leaf + (uint64_t)r * words, NULL);
            dang += (int64_t)count_dangling(root, 0, m->g.depth);
        }
    }
    if (dangling) *dangling = dang;
    return 0;
}

/* Label every pixel of one frame: mask bit 1 = Check Color false (R6). */
int orc_classify(const Model *m, const uint8_t *rgb, int64_t row_pitch, uint64_t *mask) {
    const Geom *g = &m->g;
    int mw = (g->width + 63) / 64;
    memset(mask, 0, (size_t)mw * (size_t)g->height * sizeof(uint64_t));
    for (int y = 0; y < g->height; ++y) {
        const uint8_t *row = rgb + (int64_t)y * row_pitch;
        uint64_t *mrow = mask + (size_t)y * mw;
        for (int x = 0; x < g->width; ++x) {
            const uint8_t *p = row + 3 * x;
            const Node *root = m->trees->roots[region_of(g, x, y)];
#if ORC_MUTANT == 8   /* polarity inverted */
            if (check_color(root, p[0], p[1], p[2], g->depth))
#else
            if (!check_color(root, p[0], p[1], p[2], g->depth))
#endif
                mrow[x >> 6] |= 1ull << (x & 63);
        }
    }
    return 0;
}

/* Redraw a frame with its own pruned trees (Section 2): each pixel takes the
 * colour of the depth-d node its path reaches, i.e. the node's path bits with
 * the remaining bits zero.  The colour is rebuilt from the child indices met on
 * the walk.  Returns -1 if some pixel's path is missing from its tree. */
int orc_redraw(const Forest *f, int frame, const uint8_t *rgb, int64_t row_pitch, uint8_t *out,
               int64_t out_pitch) {
    const Geom *g = &f->g;
    if (frame < 0 || frame >= f->nframes || !f->frames[frame]) return -1;
    const Trees *t = f->frames[frame];
    for (int y = 0; y < g->height; ++y) {
        const uint8_t *row = rgb + (int64_t)y * row_pitch;
        uint8_t *orow = out + (int64_t)y * out_pitch;
        for (int x = 0; x < g->width; ++x) {
            const uint8_t *p = row + 3 * x;
            const Node *node = t->roots[region_of(g, x, y)];
            if (!node) return -1;
            unsigned R = 0, G = 0, B = 0;
            for (int i = 0; i < g->depth; ++i) {
                const int index = child_index(p[0], p[1], p[2], i);
                if (!node->child[index]) return -1;
                node = node->child[index];
                R |= (unsigned)((index >> 2) & 1) << (7 - i);
                G |= (unsigned)((index >> 1) & 1) << (7 - i);
                B |= (unsigned)(index & 1) << (7 - i);
            }
            orow[3 * x] = (uint8_t)R;
            orow[3 * x + 1] = (uint8_t)G;
            orow[3 * x + 2] = (uint8_t)B;
        }
    }
    return 0;
}

/* Check Color of one pixel (used for sampled checks of very large runs).
 * Returns -1 for a pixel outside the frame. */
int orc_check_pixel(const Model *m, int x, int y, uint8_t r, uint8_t g, uint8_t b) {
    if (x < 0 || y < 0 || x >= m->g.width || y >= m->g.height) return -1;
#if ORC_MUTANT == 11  /* one pixel's check: red and blue arguments exchanged */
    { uint8_t t = r; r = b; b = t; }
#endif
#if ORC_MUTANT == 12  /* one pixel's check: region looked up in the transposed grid */
    const Node *root = m->trees->roots[(x / m->g.region_w) * m->g.reg_rows + y / m->g.region_h];
#else
    const Node *root = m->trees->roots[region_of(&m->g, x, y)];
#endif
    return check_color(root, r, g, b, m->g.depth);
}

void orc_model_free(Model *m) {
    if (!m) return;
    trees_free(m->trees);
    free(m);
}
