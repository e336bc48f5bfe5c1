/*
 * svo_oracle.c -- plain FP64 CPU oracle for first-hit ray tracing of sparse
 * voxel octrees whose nodes carry affine transforms.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library.  It shares no code, header,
 * table or helper with the HIP library: it decodes the pool format from its
 * written definition, composes and inverts transforms itself, and traverses
 * every frame by plain recursive descent.
 *
 * What it computes (the plain definition the fast path must reproduce):
 *   - The scene is a set of rigid bodies, each a static octree with its own
 *     time-varying transform (paper Sec. 3, first paragraph).  Here a body is
 *     the subtree below a transformed node ("frame"); frame F0 is the world
 *     tree with every transformed subtree taken out.  A frame's world map is
 *     W_s = W_parent(s) o A_s with A_s the caller's parent-relative forward
 *     3x4 (nested bodies compose; the paper's larger-octree idea, Sec. 5.4).
 *   - Rays are R(t) = o + t d restricted to [tmin, tmax] (Eq. 1).
 *   - The model is never moved; the ray is mapped into each frame instead
 *     (Sec. 3, Fig. 1): o_F = W_F^-1(o), d_F = L_F^-1 d, with the same t in
 *     both frames (Eq. 2).  For a rotation + translation this is Eq. 3:
 *     d' = M_R^-1 d, o' = M_R^-1 M_T^-1 o.  Anisotropic scale enters either
 *     through the same affine inverse or, as Sec. 3.2 proposes, through the
 *     octree extents; oracle_trace_paper_form() takes the latter route.
 *   - Result = the solid leaf (closed box) with the smallest
 *     t = max(t_near, tmin) over all frames such that the box meets the ray
 *     on [tmin, tmax]; ties go to the smallest slot id (world = 0xffffffff,
 *     i.e. last), then the smallest node index.  Normal = the entry face's
 *     outward normal mapped by the inverse transpose, zero when the ray
 *     starts inside the box.
 *
 * Readings where the paper is silent (listed with reasons in the design
 * notes): no clipping of moved content to its static cell (union of rigid
 * bodies); d_F is never renormalised; an axis with d_a = 0 gives the slab
 * (-inf, inf) when lo <= o_a <= hi and the empty set otherwise; a ray with a
 * non-finite component, a zero direction (below 2^-100 in every component)
 * or tmin > tmax misses.
 *
 * Pool format: 64-bit nodes, bits 0..7 child mask (octant i = x|y<<1|z<<2),
 * bits 8..31 relative child offset c24, bits 32..63 word1.  mask == 0: solid
 * leaf.  word1 bit 31 set: transformed node, slot = word1 & 0x7fffffff,
 * children at slot_child[slot].  c24 == 0xffffff: children at word1.
 * Otherwise children at node + c24.  The k-th existing child in octant order
 * is child_start + k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ONONE 0xFFFFFFFFu

typedef struct {
    int slot;              /* -1 for the world frame */
    int parent;            /* index of the enclosing frame, -1 for the world */
    int root_is_leaf;      /* world root stored as a single solid leaf */
    uint32_t root_id;      /* node index of the frame root */
    unsigned mask;         /* child mask of the frame root */
    uint64_t child;        /* child group start of the frame root */
    double lo[3];          /* local root cell corner */
    double size[3];        /* local root cell extents (per axis) */
    double W[3][4];        /* world <- local */
    double Wi[3][4];       /* local <- world */
} oframe;

typedef struct {
    const uint64_t* nodes;
    uint64_t n_nodes;
    int n_frames;
    oframe* fr;
} oscene;

typedef struct {
    double t;
    uint32_t inst, id;
    int frame;
    int axis;            /* entry axis, -1 when the ray starts inside the box */
    double tn_axis[3];   /* per-axis entry t of the hit box (for the margin) */
    double tn, tf;       /* slab interval of the hit box (unclamped) */
    double lo[3], hi[3]; /* the hit box in its frame */
} ohit;

/* ------------------------------------------------------------ node decoding */

static unsigned nd_mask(uint64_t w) { return (unsigned)(w & 0xFFu); }
static uint32_t nd_c24(uint64_t w) { return (uint32_t)((w >> 8) & 0xFFFFFFu); }
static uint32_t nd_w1(uint64_t w) { return (uint32_t)(w >> 32); }
static int nd_is_leaf(uint64_t w) { return nd_mask(w) == 0; }
static int nd_is_xform(uint64_t w) { return nd_mask(w) != 0 && (nd_w1(w) & 0x80000000u) != 0; }

/* child group start of a plain interior node (not transformed) */
static uint64_t nd_child_start(uint64_t idx, uint64_t w)
{
    uint32_t c = nd_c24(w);
    if (c == 0xFFFFFFu) return (uint64_t)nd_w1(w);
    return idx + (uint64_t)c;
}

static int popc8(unsigned v) { int n = 0; while (v) { n += (int)(v & 1u); v >>= 1; } return n; }

/* ------------------------------------------------------------ affine maps */

/* C = A o B for 3x4 affine maps (x -> A(B x)). */
static void aff_compose(const double A[3][4], const double B[3][4], double C[3][4])
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            C[r][c] = A[r][0] * B[0][c] + A[r][1] * B[1][c] + A[r][2] * B[2][c];
        C[r][3] = A[r][0] * B[0][3] + A[r][1] * B[1][3] + A[r][2] * B[2][3] + A[r][3];
    }
}

/* Inverse of an affine map: linear part by Gauss-Jordan elimination with
   partial pivoting, translation = -L^-1 b.  Returns -1 if singular. */
static int aff_invert(const double A[3][4], double Ai[3][4])
{
    double m[3][6];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) { m[r][c] = A[r][c]; m[r][3 + c] = (r == c) ? 1.0 : 0.0; }
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
        if (!(fabs(m[piv][col]) > 0.0)) return -1;
        if (piv != col)
            for (int c = 0; c < 6; ++c) { double t = m[col][c]; m[col][c] = m[piv][c]; m[piv][c] = t; }
        double p = m[col][col];
        for (int c = 0; c < 6; ++c) m[col][c] /= p;
        for (int r = 0; r < 3; ++r) {
            if (r == col) continue;
            double f = m[r][col];
            if (f != 0.0)
                for (int c = 0; c < 6; ++c) m[r][c] -= f * m[col][c];
        }
    }
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) Ai[r][c] = m[r][3 + c];
        Ai[r][3] = -(Ai[r][0] * A[0][3] + Ai[r][1] * A[1][3] + Ai[r][2] * A[2][3]);
    }
    return 0;
}

static void aff_identity(double A[3][4])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) A[r][c] = (r == c) ? 1.0 : 0.0;
}

/* Eq. 2/3 generalised: the ray in frame coordinates, same parameter t. */
static void map_ray(const double Wi[3][4], const double o[3], const double d[3], double of[3], double df[3])
{
    for (int r = 0; r < 3; ++r) {
        of[r] = Wi[r][0] * o[0] + Wi[r][1] * o[1] + Wi[r][2] * o[2] + Wi[r][3];
        df[r] = Wi[r][0] * d[0] + Wi[r][1] * d[1] + Wi[r][2] * d[2];
    }
}

/* ------------------------------------------------------------ slab test */

/* Interval of the line o + t d inside the closed box [lo, hi].  Returns 0 if
   empty on some axis.  tn_axis[a] = per-axis entry (or -inf for d_a = 0),
   *axis = argmax of tn_axis (ties -> smallest axis). */
static int slab(const double o[3], const double d[3], const double lo[3], const double hi[3],
                double* tn, double* tf, double tn_axis[3], int* axis)
{
    double n = -INFINITY, f = INFINITY;
    int ax = 0;
    for (int a = 0; a < 3; ++a) {
        double na, fa;
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] > hi[a]) return 0;
            na = -INFINITY; fa = INFINITY;
        } else {
            double t1 = (lo[a] - o[a]) / d[a];
            double t2 = (hi[a] - o[a]) / d[a];
            na = t1 < t2 ? t1 : t2;
            fa = t1 < t2 ? t2 : t1;
        }
        tn_axis[a] = na;
        if (na > n) { n = na; ax = a; }
        if (fa < f) f = fa;
    }
    *tn = n; *tf = f; *axis = ax;
    return n <= f;
}

/* ------------------------------------------------------------ exact descent */

typedef struct {
    double te, tx, tn, tf, tna[3];
    int oct, axis;
    uint64_t idx;
    double lo[3], hi[3];
} ochild;

static void sort_children(ochild* c, int n)
{
    for (int i = 1; i < n; ++i) {
        ochild k = c[i];
        int j = i - 1;
        while (j >= 0 && (c[j].te > k.te || (c[j].te == k.te && c[j].oct > k.oct))) { c[j + 1] = c[j]; --j; }
        c[j + 1] = k;
    }
}

static void consider(ohit* best, double t, uint32_t inst, uint32_t id, int frame, int axis,
                     const double tna[3], double tn, double tf, const double lo[3], const double hi[3])
{
    int better = t < best->t ||
                 (t == best->t && (inst < best->inst || (inst == best->inst && id < best->id)));
    if (!better) return;
    best->t = t; best->inst = inst; best->id = id; best->frame = frame; best->axis = axis;
    best->tn_axis[0] = tna[0]; best->tn_axis[1] = tna[1]; best->tn_axis[2] = tna[2];
    best->tn = tn; best->tf = tf;
    for (int a = 0; a < 3; ++a) { best->lo[a] = lo[a]; best->hi[a] = hi[a]; }
}

static void hit_box(const oscene* sc, const ohit* best, double lo[3], double hi[3])
{
    (void)sc;
    for (int a = 0; a < 3; ++a) { lo[a] = best->lo[a]; hi[a] = best->hi[a]; }
}

/* Children of one interior node, visited front to back by entry t (the
   top-down order of Revelles-style traversal, Sec. 5 of the paper); a child
   whose entry lies beyond the best hit so far cannot improve it. */
static void descend(const oscene* sc, int f, uint64_t cstart, unsigned mask, const double lo[3],
                    const double size[3], const double of[3], const double df[3], double tmin, double tmax,
                    ohit* best)
{
    ochild ch[8];
    int n = 0;
    for (int i = 0; i < 8; ++i) {
        if (!(mask & (1u << i))) continue;
        ochild c;
        for (int a = 0; a < 3; ++a) {
            int bit = (i >> a) & 1;
            double h = 0.5 * size[a];
            c.lo[a] = bit ? lo[a] + h : lo[a];
            c.hi[a] = bit ? lo[a] + size[a] : lo[a] + h;
        }
        if (!slab(of, df, c.lo, c.hi, &c.tn, &c.tf, c.tna, &c.axis)) continue;
        c.te = c.tn > tmin ? c.tn : tmin;
        c.tx = c.tf < tmax ? c.tf : tmax;
        if (c.te > c.tx) continue;
        c.oct = i;
        c.idx = cstart + (uint64_t)popc8(mask & ((1u << i) - 1u));
        ch[n++] = c;
    }
    sort_children(ch, n);
    uint32_t inst = sc->fr[f].slot < 0 ? ONONE : (uint32_t)sc->fr[f].slot;
    for (int k = 0; k < n; ++k) {
        const ochild* c = &ch[k];
        if (c->te > best->t) break;
        if (c->idx >= sc->n_nodes) continue;
        uint64_t w = sc->nodes[c->idx];
        if (nd_is_xform(w)) continue;          /* belongs to another frame */
        if (nd_is_leaf(w)) {
            consider(best, c->te, inst, (uint32_t)c->idx, f, c->tn >= tmin ? c->axis : -1, c->tna, c->tn, c->tf,
                     c->lo, c->hi);
            continue;
        }
        double csz[3] = {0.5 * size[0], 0.5 * size[1], 0.5 * size[2]};
        descend(sc, f, nd_child_start(c->idx, w), nd_mask(w), c->lo, csz, of, df, tmin, tmax, best);
    }
}

/* ------------------------------------------------------------ node counts */

/* Node records one frame's front-to-back descent reads before it stops: at
   its own first solid leaf (that leaf included) or once the next cell is
   entered beyond `bound`.  Cells are taken in entry order as in descend();
   a transformed child is read (its record says it belongs to another frame)
   and then skipped.  *found is set at the first leaf. */
static void count_descend(const oscene* sc, uint64_t cstart, unsigned mask, const double lo[3],
                          const double size[3], const double of[3], const double df[3], double tmin, double tmax,
                          double bound, int* found, uint32_t* count)
{
    ochild ch[8];
    int n = 0;
    for (int i = 0; i < 8; ++i) {
        if (!(mask & (1u << i))) continue;
        ochild c;
        for (int a = 0; a < 3; ++a) {
            int bit = (i >> a) & 1;
            double h = 0.5 * size[a];
            c.lo[a] = bit ? lo[a] + h : lo[a];
            c.hi[a] = bit ? lo[a] + size[a] : lo[a] + h;
        }
        if (!slab(of, df, c.lo, c.hi, &c.tn, &c.tf, c.tna, &c.axis)) continue;
        c.te = c.tn > tmin ? c.tn : tmin;
        c.tx = c.tf < tmax ? c.tf : tmax;
        if (c.te > c.tx) continue;
        c.oct = i;
        c.idx = cstart + (uint64_t)popc8(mask & ((1u << i) - 1u));
        ch[n++] = c;
    }
    sort_children(ch, n);
    for (int k = 0; k < n && !*found; ++k) {
        const ochild* c = &ch[k];
        if (c->te > bound) return;
        if (c->idx >= sc->n_nodes) continue;
        uint64_t w = sc->nodes[c->idx];
        ++*count;
        if (nd_is_xform(w)) continue;
        if (nd_is_leaf(w)) { *found = 1; return; }
        double csz[3] = {0.5 * size[0], 0.5 * size[1], 0.5 * size[2]};
        count_descend(sc, nd_child_start(c->idx, w), nd_mask(w), c->lo, csz, of, df, tmin, tmax, bound, found, count);
    }
}

/* ------------------------------------------------------------ grazing margin */

typedef struct {
    double g;          /* running minimum of scaled gaps */
    double t_hit;
    int hit_frame;
    uint32_t hit_id;
} omargin;

static double inf_norm(const double v[3])
{
    double m = fabs(v[0]);
    if (fabs(v[1]) > m) m = fabs(v[1]);
    if (fabs(v[2]) > m) m = fabs(v[2]);
    return m;
}

/* Distance, in units of t, between the ray segment o + t d (t in [tmin, tmax])
   and the closed box [lo, hi]: the smallest delta such that the box grown by
   delta on every side (L-infinity) meets the segment, divided by |d|inf.
   Zero when they intersect.  Growing the box by delta moves the per-axis
   entry down by delta/|d_a| and the exit up by delta/|d_a|, so each pair of
   axes (and each of tmin, tmax) gives one lower bound on delta. */
static double seg_box_gap(const double o[3], const double d[3], const double lo[3], const double hi[3],
                          double tmin, double tmax)
{
    double tn[3], tf[3], w[3], delta = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            double e = o[a] < lo[a] ? lo[a] - o[a] : (o[a] > hi[a] ? o[a] - hi[a] : 0.0);
            if (e > delta) delta = e;
            tn[a] = -INFINITY; tf[a] = INFINITY; w[a] = 0.0;
        } else {
            double t1 = (lo[a] - o[a]) / d[a], t2 = (hi[a] - o[a]) / d[a];
            tn[a] = t1 < t2 ? t1 : t2; tf[a] = t1 < t2 ? t2 : t1;
            w[a] = 1.0 / fabs(d[a]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) continue;
        for (int b = 0; b < 3; ++b) {
            if (w[b] == 0.0 || a == b) continue;
            double c = (tn[a] - tf[b]) / (w[a] + w[b]);
            if (c > delta) delta = c;
        }
        if (isfinite(tmax)) { double c = (tn[a] - tmax) / w[a]; if (c > delta) delta = c; }
        { double c = (tmin - tf[a]) / w[a]; if (c > delta) delta = c; }
    }
    return delta / inf_norm(d);
}

/* Depth, in units of t, of the segment inside the closed box: the largest
   delta such that the box shrunk by delta on every side still meets the
   segment, divided by |d|inf.  Zero for a ray that only touches a face, an
   edge or a corner, or runs along a face. */
static double seg_box_depth(const double o[3], const double d[3], const double lo[3], const double hi[3],
                            double tmin, double tmax)
{
    double tn[3], tf[3], w[3], delta = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            double e1 = o[a] - lo[a], e2 = hi[a] - o[a];
            double e = e1 < e2 ? e1 : e2;
            if (e < delta) delta = e;
            w[a] = 0.0;
        } else {
            double t1 = (lo[a] - o[a]) / d[a], t2 = (hi[a] - o[a]) / d[a];
            tn[a] = t1 < t2 ? t1 : t2; tf[a] = t1 < t2 ? t2 : t1;
            w[a] = 1.0 / fabs(d[a]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) continue;
        for (int b = 0; b < 3; ++b) {
            if (w[b] == 0.0) continue;
            double c = (tf[b] - tn[a]) / (w[a] + w[b]);
            if (c < delta) delta = c;
        }
        if (isfinite(tmax)) { double c = (tmax - tn[a]) / w[a]; if (c < delta) delta = c; }
        { double c = (tf[a] - tmin) / w[a]; if (c < delta) delta = c; }
    }
    if (delta < 0.0) delta = 0.0;
    return delta / inf_norm(d);
}

/* Inflated descent: visit cells missed by less than eps (in t) and entered
   no later than eps after the hit; record near misses (g3) and runner-up
   hits (g2), both divided by the frame's coordinate scale S. */
static void descend_margin(const oscene* sc, int f, uint64_t cstart, unsigned mask, const double lo[3],
                           const double size[3], const double of[3], const double df[3], double tmin,
                           double tmax, double eps, double S, omargin* m)
{
    for (int i = 0; i < 8; ++i) {
        if (!(mask & (1u << i))) continue;
        double clo[3], chi[3], tn, tf, tna[3];
        int ax;
        for (int a = 0; a < 3; ++a) {
            int bit = (i >> a) & 1;
            double h = 0.5 * size[a];
            clo[a] = bit ? lo[a] + h : lo[a];
            chi[a] = bit ? lo[a] + size[a] : lo[a] + h;
        }
        double gap = seg_box_gap(of, df, clo, chi, tmin, tmax);
        if (gap > eps) continue;
        double g = eps * inf_norm(df);
        double glo[3] = {clo[0] - g, clo[1] - g, clo[2] - g}, ghi[3] = {chi[0] + g, chi[1] + g, chi[2] + g};
        if (!slab(of, df, glo, ghi, &tn, &tf, tna, &ax)) continue;
        double teg = tn > tmin ? tn : tmin;
        if (teg > m->t_hit + eps) continue;
        uint64_t idx = cstart + (uint64_t)popc8(mask & ((1u << i) - 1u));
        if (idx >= sc->n_nodes) continue;
        uint64_t w = sc->nodes[idx];
        if (nd_is_xform(w)) continue;
        if (nd_is_leaf(w)) {
            if (gap > 0.0) {
                if (gap / S < m->g) m->g = gap / S;
            } else if (!(f == m->hit_frame && (uint32_t)idx == m->hit_id)) {
                if (slab(of, df, clo, chi, &tn, &tf, tna, &ax)) {
                    double te = tn > tmin ? tn : tmin;
                    double g2 = fabs(te - m->t_hit) / S;
                    if (g2 < m->g) m->g = g2;
                }
            }
            continue;
        }
        double csz[3] = {0.5 * size[0], 0.5 * size[1], 0.5 * size[2]};
        descend_margin(sc, f, nd_child_start(idx, w), nd_mask(w), clo, csz, of, df, tmin, tmax, eps, S, m);
    }
}

/* S(F, t) = max(|o_F|inf, |o_F + t d_F|inf, 1) / |d_F|inf: converts a t gap
   into a gap relative to the coordinate magnitudes FP32 rounds against. */
static double frame_scale(const double of[3], const double df[3], double t)
{
    double m = inf_norm(of);
    if (isfinite(t)) {
        double p[3] = {of[0] + t * df[0], of[1] + t * df[1], of[2] + t * df[2]};
        double q = inf_norm(p);
        if (q > m) m = q;
    }
    if (m < 1.0) m = 1.0;
    return m / inf_norm(df);
}

/* ------------------------------------------------------------ one ray */

typedef struct {
    uint32_t id, inst;
    double t, n[3];
    double margin;      /* id margin: gaps that can change which leaf is hit (g1-g4) */
    double margin_n;    /* normal margin: the id margin and the entry-face gaps (g4 at tmin, g5) */
    uint32_t nnode_lo, nnode_hi, nframe_lo, nframe_hi;
} oresult;

/* Node records read per ray, as two bounds that do not depend on the order
   in which an implementation visits frames.  Every frame whose root cell
   the segment [tmin, tmax] meets is a frame entered; its root record counts
   as one read, then its own front-to-back descent is counted (count_descend).
     upper: every such frame, each descended to its own first hit;
     lower: only frames entered no later than the final hit t*, each
            descended to its own first hit or to t*, whichever comes first.
   A front-to-back traversal that bounds each frame by its best hit so far
   (never below t*) reads between the two; with one frame they coincide. */
static void count_nodes(const oscene* sc, const double o[3], const double d[3], double tmin, double tmax,
                        double tstar, oresult* res)
{
    for (int f = 0; f < sc->n_frames; ++f) {
        const oframe* F = &sc->fr[f];
        double of[3], df[3], hi[3], tn, tf, tna[3];
        int ax;
        map_ray(F->Wi, o, d, of, df);
        for (int a = 0; a < 3; ++a) hi[a] = F->lo[a] + F->size[a];
        if (!slab(of, df, F->lo, hi, &tn, &tf, tna, &ax)) continue;
        double te = tn > tmin ? tn : tmin, tx = tf < tmax ? tf : tmax;
        if (te > tx) continue;
        uint32_t up = 1, lo = 1;
        int found = 0;
        if (!F->root_is_leaf) count_descend(sc, F->child, F->mask, F->lo, F->size, of, df, tmin, tmax, INFINITY, &found, &up);
        res->nframe_hi++;
        res->nnode_hi += up;
        if (te > tstar) continue;
        found = 0;
        if (!F->root_is_leaf) count_descend(sc, F->child, F->mask, F->lo, F->size, of, df, tmin, tmax, tstar, &found, &lo);
        res->nframe_lo++;
        res->nnode_lo += lo;
    }
}

static void trace_one(const oscene* sc, const float* ray, int want_margin, int want_counts, double margin_eps,
                      oresult* res)
{
    double o[3] = {ray[0], ray[1], ray[2]}, d[3] = {ray[4], ray[5], ray[6]};
    double tmin = ray[3], tmax = ray[7];
    res->id = ONONE; res->inst = ONONE; res->t = INFINITY;
    res->n[0] = res->n[1] = res->n[2] = 0.0;
    res->margin = INFINITY; res->margin_n = INFINITY;
    res->nnode_lo = res->nnode_hi = res->nframe_lo = res->nframe_hi = 0;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(o[a]) || !isfinite(d[a])) return;
    if (isnan(tmin) || isnan(tmax) || tmin > tmax || tmin == INFINITY) return;
    /* a direction below 2^-100 in every component counts as zero */
    if (fabs(d[0]) < 0x1p-100 && fabs(d[1]) < 0x1p-100 && fabs(d[2]) < 0x1p-100) return;

    ohit best;
    memset(&best, 0, sizeof best);
    best.t = INFINITY; best.inst = ONONE; best.id = ONONE; best.frame = -1; best.axis = -1;

    for (int f = 0; f < sc->n_frames; ++f) {
        const oframe* F = &sc->fr[f];
        double of[3], df[3], hi[3], tn, tf, tna[3];
        int ax;
        map_ray(F->Wi, o, d, of, df);
        for (int a = 0; a < 3; ++a) hi[a] = F->lo[a] + F->size[a];
        if (!slab(of, df, F->lo, hi, &tn, &tf, tna, &ax)) continue;
        double te = tn > tmin ? tn : tmin, tx = tf < tmax ? tf : tmax;
        if (te > tx) continue;
        if (te > best.t) continue;
        uint32_t inst = F->slot < 0 ? ONONE : (uint32_t)F->slot;
        if (F->root_is_leaf) {
            consider(&best, te, inst, F->root_id, f, tn >= tmin ? ax : -1, tna, tn, tf, F->lo, hi);
            continue;
        }
        descend(sc, f, F->child, F->mask, F->lo, F->size, of, df, tmin, tmax, &best);
    }

    if (best.frame >= 0) {
        const oframe* F = &sc->fr[best.frame];
        double of[3], df[3];
        map_ray(F->Wi, o, d, of, df);
        res->id = best.id; res->inst = best.inst; res->t = best.t;
        if (best.axis >= 0) {
            /* outward normal of the entry face, -sgn(d_a) e_a, mapped by the
               inverse transpose: row a of L^-1 */
            double s = df[best.axis] > 0.0 ? -1.0 : 1.0;
            double n0 = s * F->Wi[best.axis][0], n1 = s * F->Wi[best.axis][1], n2 = s * F->Wi[best.axis][2];
            double len = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
            res->n[0] = n0 / len; res->n[1] = n1 / len; res->n[2] = n2 / len;
        }
    }
    if (want_counts) count_nodes(sc, o, d, tmin, tmax, best.t, res);

    if (!want_margin) return;
    omargin m;
    double gn = INFINITY;   /* gaps that only decide the entry face (normal) */
    m.g = INFINITY; m.t_hit = best.t; m.hit_frame = best.frame; m.hit_id = best.id;
    if (best.frame >= 0) {
        const oframe* F = &sc->fr[best.frame];
        double of[3], df[3];
        map_ray(F->Wi, o, d, of, df);
        double S = frame_scale(of, df, best.t);
        /* g1: how far the hit box can shrink before the segment misses it */
        double blo[3], bhi[3];
        hit_box(sc, &best, blo, bhi);
        double g = seg_box_depth(of, df, blo, bhi, tmin, tmax) / S;
        if (g < m.g) m.g = g;
        if (isfinite(tmax)) { g = fabs(tmax - best.t) / S; if (g < m.g) m.g = g; }   /* g4: hit vs tmax */
        /* g4 at tmin: entered through a face or starting inside the box; the
           box, and so the id, is the same either way */
        g = fabs(best.tn - tmin) / S;
        if (g < gn) gn = g;
        if (best.axis >= 0) {                                  /* g5: entry-axis tie */
            double a1 = -INFINITY, a2 = -INFINITY;
            for (int a = 0; a < 3; ++a) {
                double v = best.tn_axis[a];
                if (v > a1) { a2 = a1; a1 = v; } else if (v > a2) a2 = v;
            }
            if (isfinite(a2)) { g = (a1 - a2) / S; if (g < gn) gn = g; }
        }
    }
    for (int f = 0; f < sc->n_frames; ++f) {
        const oframe* F = &sc->fr[f];
        double of[3], df[3], hi[3], tn, tf, tna[3];
        int ax;
        map_ray(F->Wi, o, d, of, df);
        for (int a = 0; a < 3; ++a) hi[a] = F->lo[a] + F->size[a];
        double tstar = best.t;
        if (!isfinite(tstar)) {
            tstar = tmin > 0.0 ? tmin : 0.0;
            if (slab(of, df, F->lo, hi, &tn, &tf, tna, &ax) && isfinite(tf)) {
                double tx = tf < tmax ? tf : tmax;
                if (tx > tstar) tstar = tx;
            }
        }
        double S = frame_scale(of, df, tstar);
        double eps = margin_eps * S;
        if (seg_box_gap(of, df, F->lo, hi, tmin, tmax) > eps) continue;
        if (F->root_is_leaf) {
            double gap = seg_box_gap(of, df, F->lo, hi, tmin, tmax);
            if (gap > 0.0) {
                if (gap / S < m.g) m.g = gap / S;
            } else if (!(f == best.frame && F->root_id == best.id) && slab(of, df, F->lo, hi, &tn, &tf, tna, &ax)) {
                double te = tn > tmin ? tn : tmin;
                double g2 = fabs(te - best.t) / S;
                if (g2 < m.g) m.g = g2;
            }
            continue;
        }
        descend_margin(sc, f, F->child, F->mask, F->lo, F->size, of, df, tmin, tmax, eps, S, &m);
    }
    res->margin = m.g;
    res->margin_n = gn < m.g ? gn : m.g;
}

/* ------------------------------------------------------------ scene setup */

static int collect_frames(const uint64_t* nodes, uint64_t n_nodes, uint32_t root, const double root_min[3],
                          double root_size, uint32_t n_slots, const uint32_t* slot_child,
                          const double* slot_cell, const double* fwd, oscene* sc)
{
    sc->nodes = nodes;
    sc->n_nodes = n_nodes;
    sc->n_frames = 0;
    sc->fr = NULL;
    if (root == ONONE) return 0;  /* empty world */
    if ((uint64_t)root >= n_nodes) return -1;
    sc->fr = (oframe*)calloc((size_t)n_slots + 1, sizeof(oframe));
    int* slot_frame = (int*)malloc(sizeof(int) * ((size_t)n_slots + 1));
    unsigned char* seen = (unsigned char*)calloc((size_t)n_nodes, 1);
    uint64_t cap = 1024, top = 0;
    uint64_t* stk_node = (uint64_t*)malloc(sizeof(uint64_t) * cap);
    int* stk_frame = (int*)malloc(sizeof(int) * cap);
    int rc = 0;
    if (!sc->fr || !slot_frame || !seen || !stk_node || !stk_frame) { rc = -2; goto done; }
    for (uint32_t s = 0; s <= n_slots; ++s) slot_frame[s] = -1;

    oframe* W = &sc->fr[0];
    W->slot = -1; W->parent = -1; W->root_id = root;
    for (int a = 0; a < 3; ++a) { W->lo[a] = root_min[a]; W->size[a] = root_size; }
    aff_identity(W->W); aff_identity(W->Wi);
    uint64_t rw = nodes[root];
    if (nd_is_xform(rw)) { rc = -1; goto done; }
    if (nd_is_leaf(rw)) { W->root_is_leaf = 1; sc->n_frames = 1; goto done; }
    W->mask = nd_mask(rw);
    W->child = nd_child_start(root, rw);
    sc->n_frames = 1;

    /* depth-first walk over child groups: (group start + mask) is pushed as
       the parent node index; each visited node is examined once */
    stk_node[top] = root; stk_frame[top] = 0; ++top;
    seen[root] = 1;
    while (top) {
        --top;
        uint64_t pidx = stk_node[top];
        int pf = stk_frame[top];
        uint64_t pw = nodes[pidx];
        uint64_t cs;
        if (nd_is_xform(pw)) {
            uint32_t s = nd_w1(pw) & 0x7FFFFFFFu;
            cs = slot_child[s];
        } else {
            cs = nd_child_start(pidx, pw);
        }
        int nc = popc8(nd_mask(pw));
        for (int k = 0; k < nc; ++k) {
            uint64_t ci = cs + (uint64_t)k;
            if (ci >= n_nodes) { rc = -1; goto done; }
            if (seen[ci]) continue;
            seen[ci] = 1;
            uint64_t cw = nodes[ci];
            if (nd_is_leaf(cw)) continue;
            int cf = pf;
            if (nd_is_xform(cw)) {
                uint32_t s = nd_w1(cw) & 0x7FFFFFFFu;
                if (s >= n_slots || slot_frame[s] >= 0) { rc = -1; goto done; }
                if ((uint64_t)slot_child[s] >= n_nodes) { rc = -1; goto done; }
                cf = sc->n_frames++;
                slot_frame[s] = cf;
                oframe* F = &sc->fr[cf];
                F->slot = (int)s; F->parent = pf; F->root_id = (uint32_t)ci;
                F->mask = nd_mask(cw); F->child = slot_child[s];
                for (int a = 0; a < 3; ++a) { F->lo[a] = slot_cell[4 * s + a]; F->size[a] = slot_cell[4 * s + 3]; }
                double A[3][4];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 4; ++c) A[r][c] = fwd[12 * s + 4 * r + c];
                aff_compose(sc->fr[pf].W, A, F->W);
                if (aff_invert(F->W, F->Wi) != 0) { rc = -3; goto done; }
            }
            if (top == cap) {
                cap *= 2;
                stk_node = (uint64_t*)realloc(stk_node, sizeof(uint64_t) * cap);
                stk_frame = (int*)realloc(stk_frame, sizeof(int) * cap);
                if (!stk_node || !stk_frame) { rc = -2; goto done; }
            }
            stk_node[top] = ci; stk_frame[top] = cf; ++top;
        }
    }
done:
    free(slot_frame); free(seen); free(stk_node); free(stk_frame);
    return rc;
}

static void free_scene(oscene* sc) { free(sc->fr); sc->fr = NULL; }

typedef struct {
    uint32_t *id, *inst;
    double *t, *n, *margin, *margin_n;
    uint32_t *nnode_lo, *nnode_hi, *nframe_lo, *nframe_hi;
} oouts;

static void run_rays(const oscene* sc, const float* rays, uint64_t n_rays, const oouts* out, double margin_eps,
                     int nthreads)
{
    if (!(margin_eps > 0.0)) margin_eps = 1e-6;
    int want_margin = out->margin != NULL || out->margin_n != NULL;
    int want_counts = out->nnode_lo || out->nnode_hi || out->nframe_lo || out->nframe_hi;
    int64_t n = (int64_t)n_rays;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < n; ++i) {
        oresult r;
        trace_one(sc, rays + 8 * i, want_margin, want_counts, margin_eps, &r);
        if (out->id) out->id[i] = r.id;
        if (out->inst) out->inst[i] = r.inst;
        if (out->t) out->t[i] = r.t;
        if (out->n) { out->n[3 * i] = r.n[0]; out->n[3 * i + 1] = r.n[1]; out->n[3 * i + 2] = r.n[2]; }
        if (out->margin) out->margin[i] = r.margin;
        if (out->margin_n) out->margin_n[i] = r.margin_n;
        if (out->nnode_lo) out->nnode_lo[i] = r.nnode_lo;
        if (out->nnode_hi) out->nnode_hi[i] = r.nnode_hi;
        if (out->nframe_lo) out->nframe_lo[i] = r.nframe_lo;
        if (out->nframe_hi) out->nframe_hi[i] = r.nframe_hi;
    }
}

/* ------------------------------------------------------------ exported */

/* First hits of n_rays rays (each 8 floats: ox oy oz tmin dx dy dz tmax).
   fwd: n_slots x 12 doubles, row-major 3x4 parent-relative forward maps;
   slot_cell: n_slots x 4 doubles (local root cell corner xyz, edge length).
   Any output pointer may be NULL.
   out_margin / out_margin_n: grazing margins, the smallest t gap, relative to
   the frame's coordinate scale, at which a perturbation of the ray could
   change the hit leaf (id margin) or, in addition, its entry face (normal
   margin); only gaps below margin_eps (<= 0 selects 1e-6) are resolved for
   leaves other than the hit one, larger ones read +inf.
   out_nnode_lo / _hi, out_nframe_lo / _hi: node records read and frames
   entered, lower and upper bound (count_nodes).
   Returns 0, -1 malformed pool, -2 out of memory, -3 singular transform. */
int oracle_trace(const uint64_t* nodes, uint64_t n_nodes, uint32_t root, const double* root_min, double root_size,
                 uint32_t n_slots, const uint32_t* slot_child, const double* slot_cell, const double* fwd,
                 const float* rays, uint64_t n_rays, uint32_t* out_id, uint32_t* out_inst, double* out_t,
                 double* out_n, double* out_margin, double* out_margin_n, uint32_t* out_nnode_lo,
                 uint32_t* out_nnode_hi, uint32_t* out_nframe_lo, uint32_t* out_nframe_hi, double margin_eps,
                 int nthreads)
{
    oscene sc;
    int rc = collect_frames(nodes, n_nodes, root, root_min, root_size, n_slots, slot_child, slot_cell, fwd, &sc);
    if (rc != 0) { free_scene(&sc); return rc; }
    oouts out = {out_id, out_inst, out_t, out_n, out_margin, out_margin_n, out_nnode_lo, out_nnode_hi,
                 out_nframe_lo, out_nframe_hi};
    run_rays(&sc, rays, n_rays, &out, margin_eps, nthreads);
    free_scene(&sc);
    return 0;
}

/* Paper form of a single-level scene (Sec. 3.1-3.2): slot s has rotation
   R_s (9 doubles, row-major), positive axis scales S_s (3), pivot c_s (3) and
   translation tau_s (3), i.e. world = R S (x - c) + c + tau.  The ray is only
   rotated and translated (Eq. 3: d' = R^T d, o' = R^T (o - c - tau)); the
   scale goes into the octree's extents, the box S (cell - c).  No matrix is
   inverted and nothing is composed; nested slots are rejected (-1). */
int oracle_trace_paper_form(const uint64_t* nodes, uint64_t n_nodes, uint32_t root, const double* root_min,
                            double root_size, uint32_t n_slots, const uint32_t* slot_child, const double* slot_cell,
                            const double* rot, const double* scale, const double* pivot, const double* tau,
                            const float* rays, uint64_t n_rays, uint32_t* out_id, uint32_t* out_inst,
                            double* out_t, double* out_n, int nthreads)
{
    /* discover frames with identity maps, then overwrite each slot frame */
    double* ident = (double*)calloc((size_t)n_slots * 12 + 12, sizeof(double));
    if (!ident) return -2;
    for (uint32_t s = 0; s < n_slots; ++s) { ident[12 * s] = 1.0; ident[12 * s + 5] = 1.0; ident[12 * s + 10] = 1.0; }
    oscene sc;
    int rc = collect_frames(nodes, n_nodes, root, root_min, root_size, n_slots, slot_child, slot_cell, ident, &sc);
    free(ident);
    if (rc != 0) { free_scene(&sc); return rc; }
    for (int f = 1; f < sc.n_frames; ++f) {
        oframe* F = &sc.fr[f];
        if (F->parent != 0) { free_scene(&sc); return -1; }
        int s = F->slot;
        const double* R = rot + 9 * s;
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = pivot[3 * s + a] + tau[3 * s + a];
        for (int r = 0; r < 3; ++r) {
            /* inverse rotation = transpose (Sec. 3.1) */
            for (int c = 0; c < 3; ++c) F->Wi[r][c] = R[3 * c + r];
            /* inverse translation = negation, applied before the rotation */
            F->Wi[r][3] = -(F->Wi[r][0] * p[0] + F->Wi[r][1] * p[1] + F->Wi[r][2] * p[2]);
        }
        for (int a = 0; a < 3; ++a) {
            double sa = scale[3 * s + a];
            F->lo[a] = sa * (F->lo[a] - pivot[3 * s + a]);
            F->size[a] = sa * F->size[a];
        }
    }
    oouts out = {out_id, out_inst, out_t, out_n, NULL, NULL, NULL, NULL, NULL, NULL};
    run_rays(&sc, rays, n_rays, &out, 0.0, nthreads);
    free_scene(&sc);
    return 0;
}

/* Frame structure as the oracle sees it: for each slot, the enclosing slot
   (0xffffffff = world) or 0xfffffffe if no transformed node references it;
   and the world<-local composed maps (n_slots x 12).  Returns the number of
   frames or a negative error. */
int oracle_frames(const uint64_t* nodes, uint64_t n_nodes, uint32_t root, const double* root_min, double root_size,
                  uint32_t n_slots, const uint32_t* slot_child, const double* slot_cell, const double* fwd,
                  uint32_t* out_parent, double* out_world)
{
    oscene sc;
    int rc = collect_frames(nodes, n_nodes, root, root_min, root_size, n_slots, slot_child, slot_cell, fwd, &sc);
    if (rc != 0) { free_scene(&sc); return rc; }
    for (uint32_t s = 0; s < n_slots; ++s) out_parent[s] = 0xFFFFFFFEu;
    for (int f = 1; f < sc.n_frames; ++f) {
        int s = sc.fr[f].slot, p = sc.fr[f].parent;
        out_parent[s] = p == 0 ? ONONE : (uint32_t)sc.fr[p].slot;
        if (out_world)
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 4; ++c) out_world[12 * s + 4 * r + c] = sc.fr[f].W[r][c];
    }
    int nf = sc.n_frames;
    free_scene(&sc);
    return nf;
}
