/*
 * FP64 CPU oracle of the pseudo-particle front end (paper Sec. III: gravity
 * tree, adaptive tree walk with Eq. (5), node smoothing lengths Eq. (7)-(9)).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark call this; the HIP library shares no code
 * with it.  Plain, slow, obviously correct: recursive tree build over a sorted
 * index list, depth-first walk, brute-force number density, bisection.
 *
 * Readings (the paper is silent or loose on these points):
 *  - Tree: an octree over 63-bit Morton keys (21 bits per axis) of positions
 *    scaled to the box, standing in for the paper's RCB tree (Sec. III-A).
 *    A node holds the particles whose keys share its first L octal digits;
 *    it is a leaf when it holds at most leaf_size particles or L = 21.  Node
 *    position = centre of mass, size s = distance from it to the furthest
 *    member particle (Sec. III-A).  Label = (1 << 3L) | prefix, so an
 *    ancestor k levels up is label >> 3k (the octree form of the label
 *    arithmetic of Sec. III-A).
 *  - Walk (Sec. III-B): r = minimum distance from the node's centre of mass
 *    to the sources.  The node's ball (centre of mass, s) "comes within" a
 *    radius R when r - s < R.  A leaf within r_part is replaced by its
 *    particles; a node within r_part or r_leaf is opened; otherwise a node is
 *    opened when s > theta * r (Eq. (5), strict); a leaf is never opened
 *    except by r_part.
 *  - Smoothing length (Sec. III-C, Eq. (7)-(8)): with N(h) = h^3 n(h) =
 *    (1/pi) sum_b w(|r_a - r_b| / h), the relation h = h_fact n^(-1/3) is
 *    N(h) = h_fact^3.  N is non-decreasing in h (w decreases in q), so the
 *    root is unique where it exists.  The sum runs over the node pseudo-
 *    particles and, in place of particles extracted within r_part, their
 *    leaves (Sec. III-C), the node itself included.  Initial guess Eq. (9),
 *    h0 = h_fact * 2 s (a zero-size node takes its particles' largest SPH
 *    h); the same value is the fallback when no root exists (N(inf) =
 *    n_points / pi <= h_fact^3) or the bracket cannot be found.
 *  - Output order: pseudo-particles in Morton order of their first particle.
 *  - Re-walk (Sec. III-B, after Eq. (6)): an internal node is also opened
 *    when its label is in a given list (nodes that failed the resolution
 *    check) or when its ball comes within a remembered region (centre c,
 *    radius R, smallest descendant size s_min: |com - c| - s < R) while it is
 *    still larger than that descendant (s > s_min).  Leaves are opened by
 *    r_part only.
 *
 * Functions with pins (tests/test_pseudo_pins.py): orp_morton (cube
 * containment), orp_tree (partition, leaf sizes, label arithmetic, brute-force
 * moments), orp_pseudo (mass conservation, theta limits, walk validity,
 * r_part extraction, h residual and monotone bracket), orp_number_sum and
 * orp_solve_h (closed-form root on a symmetric shell).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORP_BITS 21
#define ORP_MAXLEVEL 21

/* ---------------------------------------------------------------- kernel */
/* M4 cubic spline shape w(q) (Sec. III-C), support q < 2 */
static double orp_w(double q)
{
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) {
        const double t = 2.0 - q;
        return 0.25 * t * t * t;
    }
    return 0.0;
}

/* ---------------------------------------------------------------- Morton keys */
static uint32_t orp_axis(double x, double lo, double ext)
{
    const double t = ((x - lo) / ext) * 2097152.0; /* 2^21 */
    if (!(t > 0.0)) return 0;
    if (t >= 2097151.0) return 2097151u;
    return (uint32_t)floor(t);
}

/* 63-bit key: octal digits from the most significant, digit = (x,y,z) bits */
uint64_t orp_morton(const double *p, const double *box)
{
    uint32_t ix = orp_axis(p[0], box[0], box[3] - box[0]);
    uint32_t iy = orp_axis(p[1], box[1], box[4] - box[1]);
    uint32_t iz = orp_axis(p[2], box[2], box[5] - box[2]);
    uint64_t key = 0;
    for (int b = ORP_BITS - 1; b >= 0; b--) {
        key = (key << 3) | ((uint64_t)((ix >> b) & 1u) << 2) | ((uint64_t)((iy >> b) & 1u) << 1) |
              (uint64_t)((iz >> b) & 1u);
    }
    return key;
}

/* ---------------------------------------------------------------- tree */
typedef struct {
    int32_t level;
    int64_t start, end; /* range in the sorted order */
    int64_t parent;
    int64_t child0;     /* first child (children are consecutive), -1 for a leaf */
    int32_t nchild;
    uint64_t label;
    int leaf;
    double mass, com[3], s;
} orp_node;

typedef struct {
    int64_t n;
    const double *xyz, *m, *h;
    uint64_t *key;      /* by particle */
    int64_t *perm;      /* sorted position -> particle */
    orp_node *nodes;
    int64_t n_nodes, cap;
    int leaf_size;
} orp_tree_t;

static const uint64_t *g_sort_key;
static int orp_cmp(const void *a, const void *b)
{
    const int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (g_sort_key[i] != g_sort_key[j]) return g_sort_key[i] < g_sort_key[j] ? -1 : 1;
    return i < j ? -1 : (i > j);
}

static int orp_digit(uint64_t key, int level) /* octal digit that selects the child at `level` (1..21) */
{
    return (int)((key >> (3 * (ORP_BITS - level))) & 7u);
}

static int64_t orp_new_node(orp_tree_t *T)
{
    if (T->n_nodes == T->cap) {
        T->cap = T->cap ? 2 * T->cap : 1024;
        T->nodes = (orp_node *)realloc(T->nodes, sizeof(orp_node) * (size_t)T->cap);
    }
    return T->n_nodes++;
}

/* mass, centre of mass and size of a node straight from its particles */
static void orp_moments(orp_tree_t *T, orp_node *nd)
{
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t k = nd->start; k < nd->end; k++) {
        const int64_t a = T->perm[k];
        M += T->m[a];
        sx += T->m[a] * T->xyz[3 * a];
        sy += T->m[a] * T->xyz[3 * a + 1];
        sz += T->m[a] * T->xyz[3 * a + 2];
    }
    nd->mass = M;
    nd->com[0] = sx / M;
    nd->com[1] = sy / M;
    nd->com[2] = sz / M;
    double s2 = 0.0;
    for (int64_t k = nd->start; k < nd->end; k++) {
        const int64_t a = T->perm[k];
        const double dx = T->xyz[3 * a] - nd->com[0];
        const double dy = T->xyz[3 * a + 1] - nd->com[1];
        const double dz = T->xyz[3 * a + 2] - nd->com[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 > s2) s2 = d2;
    }
    nd->s = sqrt(s2);
}

static void orp_build(orp_tree_t *T, int64_t self, int level, int64_t start, int64_t end, int64_t parent,
                      uint64_t label)
{
    orp_node *nd = &T->nodes[self];
    nd->level = level;
    nd->start = start;
    nd->end = end;
    nd->parent = parent;
    nd->label = label;
    nd->leaf = (end - start <= T->leaf_size) || level == ORP_MAXLEVEL;
    nd->child0 = -1;
    nd->nchild = 0;
    orp_moments(T, nd);
    if (nd->leaf) return;
    /* children: runs of equal digit at level+1, in digit order (keys are sorted) */
    int64_t runs[8][2];
    int nr = 0;
    int64_t k = start;
    while (k < end) {
        const int d = orp_digit(T->key[T->perm[k]], level + 1);
        int64_t e = k;
        while (e < end && orp_digit(T->key[T->perm[e]], level + 1) == d) e++;
        runs[nr][0] = k;
        runs[nr][1] = e;
        nr++;
        k = e;
    }
    const int64_t c0 = T->n_nodes;
    for (int r = 0; r < nr; r++) orp_new_node(T);
    T->nodes[self].child0 = c0;
    T->nodes[self].nchild = nr;
    for (int r = 0; r < nr; r++) {
        const uint64_t d = (uint64_t)orp_digit(T->key[T->perm[runs[r][0]]], level + 1);
        orp_build(T, c0 + r, level + 1, runs[r][0], runs[r][1], self, (label << 3) | d);
    }
}

static void orp_tree_make(orp_tree_t *T, int64_t n, const double *xyz, const double *m, const double *h,
                          const double *box, int leaf_size)
{
    memset(T, 0, sizeof(*T));
    T->n = n;
    T->xyz = xyz;
    T->m = m;
    T->h = h;
    T->leaf_size = leaf_size;
    T->key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    T->perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t a = 0; a < n; a++) {
        T->key[a] = orp_morton(xyz + 3 * a, box);
        T->perm[a] = a;
    }
    g_sort_key = T->key;
    qsort(T->perm, (size_t)n, sizeof(int64_t), orp_cmp);
    if (n == 0) return;
    const int64_t root = orp_new_node(T);
    orp_build(T, root, 0, 0, n, -1, 1u);
}

static void orp_tree_free(orp_tree_t *T)
{
    free(T->key);
    free(T->perm);
    free(T->nodes);
}

/* Count-then-fill export of the tree (preorder).  Returns the node count;
 * arrays are written when cap >= count.  perm (n) is the sorted order. */
int64_t orp_tree(int64_t n, const double *xyz, const double *m, const double *box, int leaf_size, int64_t cap,
                 int32_t *level, int64_t *start, int64_t *end, int64_t *parent, uint64_t *label, int8_t *leaf,
                 double *mass, double *com, double *s, int64_t *perm)
{
    orp_tree_t T;
    orp_tree_make(&T, n, xyz, m, NULL, box, leaf_size);
    const int64_t nn = T.n_nodes;
    if (cap >= nn) {
        for (int64_t i = 0; i < nn; i++) {
            const orp_node *d = &T.nodes[i];
            level[i] = d->level;
            start[i] = d->start;
            end[i] = d->end;
            parent[i] = d->parent;
            label[i] = d->label;
            leaf[i] = (int8_t)d->leaf;
            mass[i] = d->mass;
            com[3 * i] = d->com[0];
            com[3 * i + 1] = d->com[1];
            com[3 * i + 2] = d->com[2];
            s[i] = d->s;
        }
        if (perm) memcpy(perm, T.perm, sizeof(int64_t) * (size_t)n);
    }
    orp_tree_free(&T);
    return nn;
}

/* ---------------------------------------------------------------- walk */
typedef struct {
    const double *src;
    int n_src;
    double theta, r_part, r_leaf;
    int64_t n_open;
    const int64_t *open;   /* labels of nodes to open */
    int64_t n_reg;
    const double *reg;     /* remembered regions: cx, cy, cz, R, s_min */
} orp_walk_par;

enum { ORP_NODE = 0, ORP_PARTICLE = 1 };

typedef struct {
    int64_t n, cap;
    int64_t *node;   /* node id (ORP_NODE) or sorted position (ORP_PARTICLE) */
    int8_t *kind;
} orp_list;

static void orp_push(orp_list *L, int64_t v, int8_t kind)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->node = (int64_t *)realloc(L->node, sizeof(int64_t) * (size_t)L->cap);
        L->kind = (int8_t *)realloc(L->kind, (size_t)L->cap);
    }
    L->node[L->n] = v;
    L->kind[L->n] = kind;
    L->n++;
}

static double orp_rmin(const orp_node *nd, const orp_walk_par *P)
{
    double best = INFINITY;
    for (int k = 0; k < P->n_src; k++) {
        const double dx = nd->com[0] - P->src[3 * k];
        const double dy = nd->com[1] - P->src[3 * k + 1];
        const double dz = nd->com[2] - P->src[3 * k + 2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r < best) best = r;
    }
    return best;
}

/* opening forced by a failed resolution check (label listed) or by a
 * remembered region the node comes within while larger than its s_min */
static int orp_forced(const orp_node *nd, const orp_walk_par *P)
{
    for (int64_t k = 0; k < P->n_open; k++)
        if ((uint64_t)P->open[k] == nd->label) return 1;
    for (int64_t k = 0; k < P->n_reg; k++) {
        const double *g = P->reg + 5 * k;
        const double dx = nd->com[0] - g[0];
        const double dy = nd->com[1] - g[1];
        const double dz = nd->com[2] - g[2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        if (d - nd->s < g[3] && nd->s > g[4]) return 1;
    }
    return 0;
}

/* depth-first walk (Sec. III-B): pseudo list in Morton order; `subs` gets the
 * leaves whose particles were extracted */
static void orp_walk(const orp_tree_t *T, int64_t id, const orp_walk_par *P, orp_list *out, orp_list *subs)
{
    const orp_node *nd = &T->nodes[id];
    const double r = orp_rmin(nd, P);
    const int in_part = r - nd->s < P->r_part;
    const int in_leaf = r - nd->s < P->r_leaf;
    if (nd->leaf) {
        if (in_part) {
            for (int64_t k = nd->start; k < nd->end; k++) orp_push(out, k, ORP_PARTICLE);
            orp_push(subs, id, ORP_NODE);
        } else {
            orp_push(out, id, ORP_NODE);
        }
        return;
    }
    const int open = in_part || in_leaf || nd->s > P->theta * r || orp_forced(nd, P);
    if (!open) {
        orp_push(out, id, ORP_NODE);
        return;
    }
    for (int c = 0; c < nd->nchild; c++) orp_walk(T, nd->child0 + c, P, out, subs);
}

/* ---------------------------------------------------------------- smoothing lengths */
/* N(h) = (1/pi) sum_b w(|x - p_b| / h) over all points, in point order */
double orp_number_sum(int64_t n_pts, const double *pts, const double *x, double h)
{
    double acc = 0.0;
    for (int64_t b = 0; b < n_pts; b++) {
        const double dx = x[0] - pts[3 * b];
        const double dy = x[1] - pts[3 * b + 1];
        const double dz = x[2] - pts[3 * b + 2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        acc += orp_w(r / h);
    }
    return acc / M_PI;
}

/* Unique root of N(h) = h_fact^3 by bracketing from h0 and bisection
 * (Eq. (7)-(8)); *fallback = 1 and h0 returned when there is none. */
double orp_solve_h(int64_t n_pts, const double *pts, const double *x, double h0, double h_fact, int *fallback)
{
    const double target = h_fact * h_fact * h_fact;
    *fallback = 0;
    if (!(h0 > 0.0) || (double)n_pts / M_PI <= target) {
        *fallback = 1;
        return h0;
    }
    double lo, hi = h0;
    int k = 0;
    if (orp_number_sum(n_pts, pts, x, hi) < target) {
        do {
            lo = hi;
            hi = 2.0 * hi;
        } while (orp_number_sum(n_pts, pts, x, hi) < target && ++k < 200);
    } else {
        lo = 0.5 * hi;
        while (orp_number_sum(n_pts, pts, x, lo) >= target && ++k < 200) {
            hi = lo;
            lo = 0.5 * lo;
        }
    }
    if (k >= 200) {
        *fallback = 1;
        return h0;
    }
    /* N(lo) < target <= N(hi) */
    for (int it = 0; it < 400 && hi - lo > 1e-15 * hi; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (orp_number_sum(n_pts, pts, x, mid) < target) lo = mid;
        else hi = mid;
    }
    return hi;
}

/* ---------------------------------------------------------------- the front end */
/*
 * Pseudo-particles of n particles (Sec. III).  Returns the pseudo count; the
 * arrays are filled when cap >= count:
 *   xyz (3), m, h, s (node size, 0 for particles), kind (0 node, 1 particle),
 *   ref (node label, or the particle's index), leaf (1 for a node
 *   pseudo-particle that is a leaf; may be NULL).
 * stats[0..8]: tree nodes, leaves, pseudo nodes, extracted particles,
 * substitute leaves, h fallbacks, max tree level, neighbour points (< 2h)
 * summed over the node pseudo-particles, size of the root node.
 * open (n_open labels) and reg (n_reg regions of 5 doubles) force openings
 * as described in the header; both may be empty.
 * `only` (optional, n_only entries, indices into the pseudo list) limits the
 * h-solve to those pseudo-particles (the rest get h = 0); NULL solves all.
 */
int64_t orp_pseudo2(int64_t n, const double *xyz, const double *m, const double *h, const double *box, int n_src,
                    const double *src, double theta, double r_part, double r_leaf, int leaf_size, double h_fact,
                    int64_t n_open, const int64_t *open, int64_t n_reg, const double *reg, int64_t cap,
                    double *o_xyz, double *o_m, double *o_h, double *o_s, int32_t *o_kind, int64_t *o_ref,
                    int8_t *o_leaf, const int64_t *only, int64_t n_only, double *stats)
{
    orp_tree_t T;
    orp_tree_make(&T, n, xyz, m, h, box, leaf_size);
    orp_list out = {0}, subs = {0};
    orp_walk_par P = {src, n_src, theta, r_part, r_leaf, n_open, open, n_reg, reg};
    if (n > 0) orp_walk(&T, 0, &P, &out, &subs);
    const int64_t np = out.n;
    if (stats) {
        int64_t leaves = 0, maxl = 0, pn = 0, pp = 0;
        for (int64_t i = 0; i < T.n_nodes; i++) {
            leaves += T.nodes[i].leaf;
            if (T.nodes[i].level > maxl) maxl = T.nodes[i].level;
        }
        for (int64_t i = 0; i < np; i++) {
            if (out.kind[i] == ORP_NODE) pn++;
            else pp++;
        }
        stats[0] = (double)T.n_nodes;
        stats[1] = (double)leaves;
        stats[2] = (double)pn;
        stats[3] = (double)pp;
        stats[4] = (double)subs.n;
        stats[5] = 0.0;
        stats[6] = (double)maxl;
        stats[7] = 0.0;
        stats[8] = n > 0 ? T.nodes[0].s : 0.0;
    }
    if (cap >= np) {
        /* points of the h-solve: node pseudo-particles and substitute leaves, by first particle */
        int64_t npts = 0;
        double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)(np + subs.n + 1));
        {
            int64_t i = 0, j = 0;
            while (i < np || j < subs.n) {
                int64_t si = INT64_MAX, sj = INT64_MAX;
                while (i < np && out.kind[i] != ORP_NODE) i++;
                if (i < np) si = T.nodes[out.node[i]].start;
                if (j < subs.n) sj = T.nodes[subs.node[j]].start;
                if (si == INT64_MAX && sj == INT64_MAX) break;
                const orp_node *d = si < sj ? &T.nodes[out.node[i++]] : &T.nodes[subs.node[j++]];
                pts[3 * npts] = d->com[0];
                pts[3 * npts + 1] = d->com[1];
                pts[3 * npts + 2] = d->com[2];
                npts++;
            }
        }
        for (int64_t i = 0; i < np; i++) {
            if (out.kind[i] == ORP_NODE) {
                const orp_node *d = &T.nodes[out.node[i]];
                o_xyz[3 * i] = d->com[0];
                o_xyz[3 * i + 1] = d->com[1];
                o_xyz[3 * i + 2] = d->com[2];
                o_m[i] = d->mass;
                o_s[i] = d->s;
                o_kind[i] = ORP_NODE;
                o_ref[i] = (int64_t)d->label;
                o_h[i] = 0.0;
                if (o_leaf) o_leaf[i] = (int8_t)d->leaf;
            } else {
                const int64_t a = T.perm[out.node[i]];
                o_xyz[3 * i] = xyz[3 * a];
                o_xyz[3 * i + 1] = xyz[3 * a + 1];
                o_xyz[3 * i + 2] = xyz[3 * a + 2];
                o_m[i] = m[a];
                o_s[i] = 0.0;
                o_kind[i] = ORP_PARTICLE;
                o_ref[i] = a;
                o_h[i] = h[a];
                if (o_leaf) o_leaf[i] = 0;
            }
        }
        /* solve */
        const int64_t n_solve = only ? n_only : np;
        int64_t fallbacks = 0;
        double nb_total = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : fallbacks, nb_total)
        for (int64_t t = 0; t < n_solve; t++) {
            const int64_t i = only ? only[t] : t;
            if (i < 0 || i >= np || out.kind[i] != ORP_NODE) continue;
            const orp_node *d = &T.nodes[out.node[i]];
            double h0;
            if (d->s > 0.0) {
                h0 = h_fact * 2.0 * d->s;
            } else {
                h0 = 0.0;
                for (int64_t k = d->start; k < d->end; k++)
                    if (h[T.perm[k]] > h0) h0 = h[T.perm[k]];
            }
            int fb = 0;
            const double hh = orp_solve_h(npts, pts, d->com, h0, h_fact, &fb);
            o_h[i] = hh;
            fallbacks += fb;
            for (int64_t b = 0; b < npts; b++) {
                const double dx = d->com[0] - pts[3 * b];
                const double dy = d->com[1] - pts[3 * b + 1];
                const double dz = d->com[2] - pts[3 * b + 2];
                if (sqrt(dx * dx + dy * dy + dz * dz) < 2.0 * hh) nb_total += 1.0;
            }
        }
        if (stats) {
            stats[5] = (double)fallbacks;
            stats[7] = nb_total;
        }
        free(pts);
    }
    free(out.node);
    free(out.kind);
    free(subs.node);
    free(subs.kind);
    orp_tree_free(&T);
    return np;
}

/* the walk of Sec. III-B without forced openings (stats: 8 entries) */
int64_t orp_pseudo(int64_t n, const double *xyz, const double *m, const double *h, const double *box, int n_src,
                   const double *src, double theta, double r_part, double r_leaf, int leaf_size, double h_fact,
                   int64_t cap, double *o_xyz, double *o_m, double *o_h, double *o_s, int32_t *o_kind,
                   int64_t *o_ref, const int64_t *only, int64_t n_only, double *stats)
{
    double st[9];
    const int64_t np = orp_pseudo2(n, xyz, m, h, box, n_src, src, theta, r_part, r_leaf, leaf_size, h_fact, 0, NULL,
                                   0, NULL, cap, o_xyz, o_m, o_h, o_s, o_kind, o_ref, NULL, only, n_only, st);
    if (stats) memcpy(stats, st, sizeof(double) * 8);
    return np;
}
