/* Breadth-first heightfield octree pools (input generation only; the same
 * pool format and node order as svogen/octree.py's build_tree with the
 * heightfield classifier and the height-band leaf colours of
 * svogen/scenes.py, written in C so that depth-12 terrains of 10^8 nodes
 * build in seconds).
 *
 * Columns: H[x * n + z] (n = 2^K), voxel (x, y, z) solid iff y < H.  A cell
 * at level l (edge s = 2^(K-l)) is FULL when every column under it reaches
 * its top, EMPTY when no column reaches its bottom voxel, else PARTIAL.
 * FULL cells become leaves (word1 = RGBA8), PARTIAL cells interior nodes
 * whose non-empty children follow breadth first; child offsets of 2^24 - 1
 * or more become far pointers.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { EMPTY = 0, FULL = 1, PARTIAL = 2 };
#define FAR 0xFFFFFFull

static const uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;

static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* hash_keys(x, y, z, l, seed, 7) of svogen/hashing.py */
static uint64_t colour_hash(int64_t x, int64_t y, int64_t z, int64_t l, int64_t seed) {
    const int64_t keys[6] = {x, y, z, l, seed, 7};
    uint64_t h = 0x6A09E667F3BCC909ull;
    for (int i = 0; i < 6; ++i) h = splitmix64(h ^ (uint64_t)keys[i]);
    return h;
}

static uint32_t leaf_colour(int K, int l, int64_t x, int64_t y, int64_t z, int64_t seed) {
    static const double bands[5][3] = {{70, 110, 60}, {110, 150, 70}, {150, 130, 90}, {120, 120, 120}, {235, 235, 240}};
    const double s = (double)(1ll << (K - l));
    const double yfrac = ((double)y + 0.5) * s / (double)(1ll << K);
    const double jit = (double)(colour_hash(x, y, z, l, seed) >> 11) * (1.0 / 9007199254740992.0);
    int64_t b = (int64_t)(yfrac * 5.0);
    if (b < 0) b = 0;
    if (b > 4) b = 4;
    uint32_t out = 255u << 24;
    for (int c = 0; c < 3; ++c) {
        double v = bands[b][c] + (jit - 0.5) * 24.0;
        if (v < 0) v = 0;
        if (v > 255) v = 255;
        out |= (uint32_t)(uint64_t)v << (8 * c);
    }
    return out;
}

typedef struct {
    int K;
    int32_t* mn[17];
    int32_t* mx[17];
} Pyr;

static void pyr_free(Pyr* p) {
    for (int l = 0; l <= p->K; ++l) {
        free(p->mn[l]);
        free(p->mx[l]);
    }
}

static int pyr_build(Pyr* p, int K, const int32_t* H) {
    memset(p, 0, sizeof *p);
    p->K = K;
    const int64_t n = 1ll << K;
    p->mn[K] = (int32_t*)malloc(sizeof(int32_t) * n * n);
    p->mx[K] = (int32_t*)malloc(sizeof(int32_t) * n * n);
    if (!p->mn[K] || !p->mx[K]) return -1;
    memcpy(p->mn[K], H, sizeof(int32_t) * n * n);
    memcpy(p->mx[K], H, sizeof(int32_t) * n * n);
    for (int l = K - 1; l >= 0; --l) {
        const int64_t m = 1ll << l, m2 = 2 * m;
        p->mn[l] = (int32_t*)malloc(sizeof(int32_t) * m * m);
        p->mx[l] = (int32_t*)malloc(sizeof(int32_t) * m * m);
        if (!p->mn[l] || !p->mx[l]) return -1;
        for (int64_t x = 0; x < m; ++x)
            for (int64_t z = 0; z < m; ++z) {
                int32_t lo = p->mn[l + 1][(2 * x) * m2 + 2 * z], hi = p->mx[l + 1][(2 * x) * m2 + 2 * z];
                for (int k = 1; k < 4; ++k) {
                    const int64_t i = (2 * x + (k & 1)) * m2 + 2 * z + (k >> 1);
                    if (p->mn[l + 1][i] < lo) lo = p->mn[l + 1][i];
                    if (p->mx[l + 1][i] > hi) hi = p->mx[l + 1][i];
                }
                p->mn[l][x * m + z] = lo;
                p->mx[l][x * m + z] = hi;
            }
    }
    return 0;
}

static inline int classify(const Pyr* p, int l, uint32_t x, uint32_t y, uint32_t z) {
    const int64_t m = 1ll << l, s = 1ll << (p->K - l);
    const int64_t lo = p->mn[l][(int64_t)x * m + z], hi = p->mx[l][(int64_t)x * m + z];
    const int64_t y0 = (int64_t)y * s;
    if (lo >= y0 + s) return FULL;
    if (hi <= y0) return EMPTY;
    return PARTIAL;
}

/* a cell: x | y << 16 | z << 32 | kind << 48 */
static inline uint64_t pack(uint32_t x, uint32_t y, uint32_t z, int k) {
    return (uint64_t)x | ((uint64_t)y << 16) | ((uint64_t)z << 32) | ((uint64_t)k << 48);
}

/* Walk the breadth-first order; count (nodes == NULL) or write the pool.
 * level_count[l] receives the nodes of level l (l = 0..K).  Returns the
 * node count, -1 on bad arguments or allocation failure, -2 when `cap` is
 * too small. */
static int64_t walk(int K, const int32_t* H, int64_t seed, uint64_t* nodes, int64_t cap, int64_t* level_count,
                    uint64_t far_from) {
    if (K < 0 || K > 16 || !H) return -1;
    Pyr p;
    if (pyr_build(&p, K, H)) {
        pyr_free(&p);
        return -1;
    }
    for (int l = 0; l <= K; ++l) level_count[l] = 0;
    int64_t total = 0;
    const int rk = classify(&p, 0, 0, 0, 0);
    if (rk == EMPTY) {
        pyr_free(&p);
        return 0;
    }
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t));
    int64_t ncur = 1;
    if (!cur) {
        pyr_free(&p);
        return -1;
    }
    cur[0] = pack(0, 0, 0, rk);
    int64_t base = 0;
    int64_t rc = 0;
    for (int l = 0; l <= K && ncur > 0; ++l) {
        level_count[l] = ncur;
        const int64_t next_base = base + ncur;
        /* children of this level, in order */
        int64_t nnext = 0, capn = 0;
        uint64_t* next = NULL;
        int64_t running = 0;
        for (int64_t i = 0; i < ncur; ++i) {
            const uint64_t c = cur[i];
            const uint32_t x = (uint32_t)(c & 0xFFFF), y = (uint32_t)((c >> 16) & 0xFFFF), z = (uint32_t)((c >> 32) & 0xFFFF);
            const int k = (int)(c >> 48);
            const int64_t idx = base + i;
            if (k == FULL) {
                if (nodes) {
                    if (idx >= cap) { rc = -2; break; }
                    nodes[idx] = (uint64_t)leaf_colour(K, l, x, y, z, seed) << 32;
                }
                continue;
            }
            if (l == K) { rc = -1; break; }   /* PARTIAL at the voxel level cannot happen */
            uint32_t mask = 0;
            for (int o = 0; o < 8; ++o) {
                const uint32_t cx = 2 * x + (o & 1), cy = 2 * y + ((o >> 1) & 1), cz = 2 * z + ((o >> 2) & 1);
                const int ck = classify(&p, l + 1, cx, cy, cz);
                if (ck == EMPTY) continue;
                mask |= 1u << o;
                if (nnext == capn) {
                    capn = capn ? capn * 2 : 1024;
                    uint64_t* t = (uint64_t*)realloc(next, sizeof(uint64_t) * capn);
                    if (!t) { rc = -1; break; }
                    next = t;
                }
                next[nnext++] = pack(cx, cy, cz, ck);
            }
            if (rc) break;
            const int64_t start = next_base + running;
            running += __builtin_popcount(mask);
            if (nodes) {
                if (idx >= cap) { rc = -2; break; }
                const uint64_t off = (uint64_t)(start - idx);
                if (off >= far_from)
                    nodes[idx] = (uint64_t)mask | (FAR << 8) | ((uint64_t)start << 32);
                else
                    nodes[idx] = (uint64_t)mask | (off << 8);
            }
        }
        free(cur);
        cur = next;
        ncur = nnext;
        base = next_base;
        total = base;
        if (rc) break;
    }
    free(cur);
    pyr_free(&p);
    return rc ? rc : total;
}

int64_t svogen_hf_count(int K, const int32_t* H, int64_t* level_count) {
    return walk(K, H, 0, NULL, 0, level_count, FAR);
}

/* far_from: child offsets of at least this many nodes become far pointers
 * (FAR, i.e. 2^24 - 1, for the pool format; smaller values only for tests) */
int64_t svogen_hf_build(int K, const int32_t* H, int64_t seed, uint64_t* nodes, int64_t cap, int64_t* level_count,
                        int64_t far_from) {
    if (!nodes || far_from < 1 || far_from > (int64_t)FAR) return -1;
    return walk(K, H, seed, nodes, cap, level_count, (uint64_t)far_from);
}
