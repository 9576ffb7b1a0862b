/*
 * FP64 CPU oracle of the box-clipped Voronoi grid and its Lloyd iterations
 * (paper Sec. II-A: a Voronoi grid whose generating sites are the particle
 * positions, clipped to the simulation box, relaxed by Lloyd iterations).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite and the benchmark's CPU leg
 * call this; the HIP library shares no code with it.  Plain and slow: each
 * cell starts as the box and is cut by the bisector plane of its site and
 * EVERY other site (no neighbour search, no stopping rule), one face polygon
 * at a time (Sutherland-Hodgman), the cut closed by a new face whose points
 * are ordered by angle about its normal.
 *
 * Output, per cell (the library's cell format): faces with outward unit
 * normals n and offsets c (n.x = c), their vertices counter-clockwise seen
 * from outside (each face owns its vertex copies here), the site or box wall
 * across each face (wall w: -1 - w, walls x-, x+, y-, y+, z-, z+), the volume
 * and the centroid.
 *
 * Lloyd iteration (Lloyd 1982, as Sec. II-A applies it): every site moves to
 * the centroid of its cell; the grid is rebuilt.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORV_MAXV 256 /* points per face polygon */
#define ORV_MAXF 256 /* faces per cell */

typedef struct {
    double n[3], c; /* outward normal (unit), n.x = c */
    int64_t nb;
    int nv;
    double v[ORV_MAXV][3];
} orv_face;

typedef struct {
    int nf;
    orv_face f[ORV_MAXF];
} orv_cell;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* the box as six faces, vertices counter-clockwise about the outward normal */
static void box_cell(orv_cell *C, const double *box)
{
    const double lo[3] = {box[0], box[1], box[2]}, hi[3] = {box[3], box[4], box[5]};
    C->nf = 0;
    for (int ax = 0; ax < 3; ax++)
        for (int side = 0; side < 2; side++) {
            orv_face *F = &C->f[C->nf++];
            memset(F->n, 0, sizeof(F->n));
            F->n[ax] = side ? 1.0 : -1.0;
            F->c = side ? hi[ax] : -lo[ax];
            F->nb = -1 - (2 * ax + side);
            const int u = (ax + 1) % 3, w = (ax + 2) % 3;
            /* corners in the (u, w) plane, counter-clockwise about +axis */
            const double cu[4] = {lo[u], hi[u], hi[u], lo[u]}, cw[4] = {lo[w], lo[w], hi[w], hi[w]};
            F->nv = 4;
            for (int k = 0; k < 4; k++) {
                const int kk = side ? k : 3 - k; /* reversed about -axis */
                F->v[k][ax] = side ? hi[ax] : lo[ax];
                F->v[k][u] = cu[kk];
                F->v[k][w] = cw[kk];
            }
        }
}

/* Points within ORV_EPS of a cutting plane count as on it (degenerate sites:
 * lattices, four sites on a sphere); lengths are box units. */
#define ORV_EPS 1e-12

/* keeps the part of the cell with n.x <= c (n unit); the cut face gets nb */
static void clip(orv_cell *C, const double *n, double c, int64_t nb)
{
    double cut[2 * ORV_MAXF * 2][3];
    int ncut = 0;
    int out = 0;
    for (int i = 0; i < C->nf; i++) {
        orv_face *F = &C->f[i];
        double nv[ORV_MAXV][3];
        int k = 0;
        for (int a = 0; a < F->nv; a++) {
            const double *p = F->v[a], *q = F->v[(a + 1) % F->nv];
            double dp = dot3(n, p) - c, dq = dot3(n, q) - c;
            if (fabs(dp) <= ORV_EPS) dp = 0.0;
            if (fabs(dq) <= ORV_EPS) dq = 0.0;
            if (dp <= 0.0) {
                if (k < ORV_MAXV) memcpy(nv[k++], p, sizeof(double) * 3);
            }
            if ((dp < 0.0 && dq > 0.0) || (dp > 0.0 && dq < 0.0)) {
                const double t = dp / (dp - dq);
                double x[3] = {p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1]), p[2] + t * (q[2] - p[2])};
                if (k < ORV_MAXV) memcpy(nv[k++], x, sizeof(x));
                if (ncut < 2 * ORV_MAXF * 2) memcpy(cut[ncut++], x, sizeof(x));
            } else if (dp == 0.0) {
                if (ncut < 2 * ORV_MAXF * 2) memcpy(cut[ncut++], p, sizeof(double) * 3);
            }
        }
        if (k >= 3) {
            orv_face *G = &C->f[out++];
            if (G != F) memcpy(G, F, sizeof(orv_face));
            G->nv = k;
            memcpy(G->v, nv, sizeof(double) * 3 * (size_t)k);
        }
    }
    C->nf = out;
    if (ncut < 3 || C->nf >= ORV_MAXF) return;
    /* the new face: cut points ordered by angle about n (counter-clockwise seen from outside) */
    double cen[3] = {0, 0, 0};
    for (int a = 0; a < ncut; a++)
        for (int d = 0; d < 3; d++) cen[d] += cut[a][d] / ncut;
    double e1[3] = {cut[0][0] - cen[0], cut[0][1] - cen[1], cut[0][2] - cen[2]};
    {
        const double s = dot3(e1, n);
        for (int d = 0; d < 3; d++) e1[d] -= s * n[d];
        const double l = sqrt(dot3(e1, e1));
        for (int d = 0; d < 3; d++) e1[d] /= l;
    }
    double e2[3];
    cross3(n, e1, e2);
    double ang[2 * ORV_MAXF * 2];
    int idx[2 * ORV_MAXF * 2];
    for (int a = 0; a < ncut; a++) {
        const double r[3] = {cut[a][0] - cen[0], cut[a][1] - cen[1], cut[a][2] - cen[2]};
        ang[a] = atan2(dot3(r, e2), dot3(r, e1));
        idx[a] = a;
    }
    for (int a = 1; a < ncut; a++) /* insertion sort by angle */
        for (int b = a; b > 0 && ang[idx[b]] < ang[idx[b - 1]]; b--) {
            const int t = idx[b];
            idx[b] = idx[b - 1];
            idx[b - 1] = t;
        }
    orv_face *G = &C->f[C->nf];
    memcpy(G->n, n, sizeof(double) * 3);
    G->c = c;
    G->nb = nb;
    G->nv = 0;
    /* drop coincident points (a cut through a vertex is found on both of its faces) */
    for (int a = 0; a < ncut && G->nv < ORV_MAXV; a++) {
        const double *p = cut[idx[a]];
        if (G->nv > 0) {
            const double *q = G->v[G->nv - 1];
            const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
            if (dx * dx + dy * dy + dz * dz <= 1e-26) continue;
        }
        memcpy(G->v[G->nv++], p, sizeof(double) * 3);
    }
    if (G->nv >= 2) {
        const double *p = G->v[0], *q = G->v[G->nv - 1];
        const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        if (dx * dx + dy * dy + dz * dz <= 1e-26) G->nv--;
    }
    if (G->nv < 3) return;
    /* a cut that only grazes the cell (through a vertex or along an edge) adds no face */
    double s[3] = {0, 0, 0};
    for (int a = 0; a < G->nv; a++) {
        double x[3];
        cross3(G->v[a], G->v[(a + 1) % G->nv], x);
        for (int d = 0; d < 3; d++) s[d] += x[d];
    }
    if (0.5 * fabs(dot3(s, n)) > ORV_EPS * ORV_EPS) C->nf++;
}

static const double *g_dist;
static int by_dist(const void *a, const void *b)
{
    const double x = g_dist[*(const int64_t *)a], y = g_dist[*(const int64_t *)b];
    return (x > y) - (x < y);
}

/* farthest vertex of the cell from s */
static double max_dist(const orv_cell *C, const double *s)
{
    double m = 0.0;
    for (int i = 0; i < C->nf; i++)
        for (int a = 0; a < C->f[i].nv; a++) {
            const double *v = C->f[i].v[a];
            const double d[3] = {v[0] - s[0], v[1] - s[1], v[2] - s[2]};
            const double r = sqrt(dot3(d, d));
            m = r > m ? r : m;
        }
    return m;
}

/* volume and centroid: tetrahedra (apex a point inside, base a fan of each face) */
static void measure(const orv_cell *C, const double *apex, double *vol, double *cen)
{
    double V = 0.0, M[3] = {0, 0, 0};
    for (int i = 0; i < C->nf; i++) {
        const orv_face *F = &C->f[i];
        for (int a = 1; a + 1 < F->nv; a++) {
            const double *p0 = F->v[0], *p1 = F->v[a], *p2 = F->v[a + 1];
            double u[3], v[3], w[3], x[3];
            for (int d = 0; d < 3; d++) {
                u[d] = p0[d] - apex[d];
                v[d] = p1[d] - apex[d];
                w[d] = p2[d] - apex[d];
            }
            cross3(v, w, x);
            const double t = dot3(u, x) / 6.0;
            V += t;
            for (int d = 0; d < 3; d++) M[d] += t * (apex[d] + p0[d] + p1[d] + p2[d]) / 4.0;
        }
    }
    *vol = V;
    for (int d = 0; d < 3; d++) cen[d] = V > 0.0 ? M[d] / V : apex[d];
}

/*
 * Box-clipped Voronoi cells of n sites, or of the n_sel selected ones (sel
 * non-NULL; outputs then follow the selection order).  A selected cell takes
 * the other sites in order of distance and stops at the first one at least
 * twice as far as its farthest vertex: that site's bisector lies half its
 * distance away, beyond every point of the cell, and so does every farther
 * one's (this keeps sampled cells of large site sets affordable; without a
 * selection every site clips every cell).  Count-then-fill:
 * counts[0..1] = faces, face-vertex slots (= vertices, one copy per face);
 * arrays are written when cap_faces >= faces and cap_verts >= slots:
 *   cell_face_off (cells+1), face_vert_off (faces+1), face_plane (4 faces),
 *   face_nb (faces), verts (3 slots; face_vert is the identity), vol (cells),
 *   centroid (3 cells).
 */
void orv_voronoi_sel(int64_t n, const double *sites, const double *box, const int64_t *sel, int64_t n_sel,
                     int64_t cap_faces, int64_t cap_verts, int64_t *counts, int64_t *cell_face_off,
                     int64_t *face_vert_off, double *face_plane, int64_t *face_nb, double *verts, double *vol,
                     double *centroid)
{
    orv_cell *C = (orv_cell *)malloc(sizeof(orv_cell));
    int64_t nf = 0, ns = 0;
    const int fill = cell_face_off != NULL;
    if (fill) cell_face_off[0] = 0;
    if (fill) face_vert_off[0] = 0;
    const int64_t n_cells = sel ? n_sel : n;
    double *dist = sel ? (double *)malloc(sizeof(double) * (size_t)n) : NULL;
    int64_t *ord = sel ? (int64_t *)malloc(sizeof(int64_t) * (size_t)n) : NULL;
    for (int64_t ci = 0; ci < n_cells; ci++) {
        const int64_t i = sel ? sel[ci] : ci;
        const double *s = sites + 3 * i;
        box_cell(C, box);
        if (sel) {
            for (int64_t j = 0; j < n; j++) {
                const double *t = sites + 3 * j;
                const double d[3] = {t[0] - s[0], t[1] - s[1], t[2] - s[2]};
                dist[j] = sqrt(dot3(d, d));
                ord[j] = j;
            }
            g_dist = dist;
            qsort(ord, (size_t)n, sizeof(int64_t), by_dist);
        }
        for (int64_t jj = 0; jj < n; jj++) {
            const int64_t j = sel ? ord[jj] : jj;
            if (j == i) continue;
            if (sel && dist[j] >= 2.0 * max_dist(C, s)) break;
            const double *t = sites + 3 * j;
            double d[3] = {t[0] - s[0], t[1] - s[1], t[2] - s[2]};
            const double l = sqrt(dot3(d, d));
            if (l == 0.0) continue; /* coincident sites share no bisector */
            const double u[3] = {d[0] / l, d[1] / l, d[2] / l};
            /* points closer to s: u.x <= u.(s + t)/2 */
            const double mid[3] = {0.5 * (s[0] + t[0]), 0.5 * (s[1] + t[1]), 0.5 * (s[2] + t[2])};
            clip(C, u, dot3(u, mid), j);
        }
        if (fill && nf + C->nf <= cap_faces) {
            for (int a = 0; a < C->nf; a++) {
                const orv_face *F = &C->f[a];
                const int64_t q = nf + a;
                face_plane[4 * q] = F->n[0];
                face_plane[4 * q + 1] = F->n[1];
                face_plane[4 * q + 2] = F->n[2];
                face_plane[4 * q + 3] = F->c;
                face_nb[q] = F->nb;
                face_vert_off[q + 1] = face_vert_off[q] + F->nv;
                if (face_vert_off[q] + F->nv <= cap_verts)
                    for (int k = 0; k < F->nv; k++)
                        memcpy(verts + 3 * (face_vert_off[q] + k), F->v[k], sizeof(double) * 3);
            }
            cell_face_off[ci + 1] = nf + C->nf;
            measure(C, s, vol + ci, centroid + 3 * ci);
        }
        nf += C->nf;
        for (int a = 0; a < C->nf; a++) ns += C->f[a].nv;
    }
    counts[0] = nf;
    counts[1] = ns;
    free(C);
    free(dist);
    free(ord);
}

void orv_voronoi(int64_t n, const double *sites, const double *box, int64_t cap_faces, int64_t cap_verts,
                 int64_t *counts, int64_t *cell_face_off, int64_t *face_vert_off, double *face_plane,
                 int64_t *face_nb, double *verts, double *vol, double *centroid)
{
    orv_voronoi_sel(n, sites, box, NULL, 0, cap_faces, cap_verts, counts, cell_face_off, face_vert_off, face_plane,
                    face_nb, verts, vol, centroid);
}
