/*
 * Plain, slow, FP64 CPU oracle for the Exact mapping of SPH particle mass onto
 * box-clipped Voronoi cells.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code, header,
 * table or helper with the HIP library, and the library never calls it.
 *
 * What it computes (paper Sec. II-B, Eq. (1)-(3)):
 *     f_ai  = integral over cell V_i of W(|r - r_a|, h_a) dV
 *     S_a   = sum_i f_ai                 (sum-to-one normalisation, FP64)
 *     M_i   = sum_a m_a f_ai / S_a       (cell mass)
 *     rho_i = M_i / V_i                  (cell density)
 * for every particle/cell pair whose cell meets the support ball |r-r_a| < 2h_a.
 *
 * The integral is evaluated the way Sec. II-B describes it: the cell volume is
 * cut into vertex pyramids with apex at the particle, each characterised by
 * the distance r0 from the particle to a wall plane, the in-plane distance R0
 * from the particle's projection point on the wall to an edge line, and an
 * angle phi at the projection point.  For each pyramid the radial integral of
 * the kernel is done exactly and the angular integral in closed form.  The
 * closed form is derived in this file's comments from Eq. (3) alone (the paper
 * gives no formula); every step is written in the plainest order, with no
 * far-field subtraction, no blocking and no reuse between triangles.
 *
 * Readings of the paper that this file takes (the paper is silent on them):
 *  - W is the M4 cubic spline, normalised to one, support 2h (Sec. III-C
 *    names the M4 kernel, Sec. III-D its 2h support):
 *        W(r,h) = w(r/h) / (pi h^3),
 *        w(q) = 1 - 1.5 q^2 + 0.75 q^3    (0 <= q < 1)
 *             = 0.25 (2 - q)^3            (1 <= q < 2)
 *             = 0                          (q >= 2).
 *  - The signs of the pyramids (particle outside the cell, projection point
 *    outside a wall polygon) follow the signed-cone identity written out in
 *    orc_pair_fraction below.
 *  - A pair exists iff the Euclidean distance from the particle to the closed
 *    cell is strictly below 2h (distance 0 inside the cell).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Radial profiles.                                                          */
/*                                                                           */
/* For a pyramid with apex at the particle (lengths in units of h), the      */
/* kernel mass inside the cone of directions dOmega up to radius s is        */
/* F(s) dOmega with F(s) = int_0^s (w(q)/pi) q^2 dq.  Integrating F over the */
/* solid angle subtended by a base triangle lying in a plane at distance r0, */
/* with dOmega = r0 dA / |b|^3 and |b|^2 = r0^2 + rho^2, s ds = rho drho,     */
/* gives                                                                     */
/*     I = r0 * int dalpha [ G(S(alpha)) - G(r0) ],   G'(s) = F(s)/s^2,      */
/* where S(alpha) is the distance from the apex to the far side of the base  */
/* in the in-plane direction alpha.  For the M4 kernel, pi*F is              */
/*     s^3/3 - 3 s^5/10 + s^6/8                          (s <= 1)            */
/*     -1/60 + 2 s^3/3 - 3 s^4/4 + 3 s^5/10 - s^6/24      (1 <= s <= 2)      */
/*     1/4                                                (s >= 2)           */
/* and pi*G (continuous, G(0) = 0) is                                        */
/*     s^2/6 - 3 s^4/40 + s^5/40                          (s <= 1)           */
/*     1/(60 s) - 1/20 + s^2/3 - s^3/4 + 3 s^4/40 - s^5/120  (1 <= s <= 2)   */
/*     7/20 - 1/(4 s)                                     (s >= 2).          */
/* Each piece is stored as coefficients of s^n for n = -1, 0, 2, 3, 4, 5.    */
/*                                                                           */
/* Profile 1 is the constant W = 1 (no normalisation): F = s^3/3, G = s^2/6. */
/* The integral of W = 1 over a cell is its volume, which pins the geometry. */
/* ------------------------------------------------------------------------ */

enum { ORC_M4 = 0, ORC_UNIT = 1, ORC_TABLE = 2 /* M4 through the table below */ };

static const int NEXP[6] = { -1, 0, 2, 3, 4, 5 };

static const double M4_G_INNER[6] = { 0.0, 0.0, 1.0 / 6.0, 0.0, -3.0 / 40.0, 1.0 / 40.0 };
static const double M4_G_SHELL[6] = { 1.0 / 60.0, -1.0 / 20.0, 1.0 / 3.0, -1.0 / 4.0, 3.0 / 40.0, -1.0 / 120.0 };
static const double M4_G_OUTER[6] = { -1.0 / 4.0, 7.0 / 20.0, 0.0, 0.0, 0.0, 0.0 };
static const double UNIT_G[6] = { 0.0, 0.0, 1.0 / 6.0, 0.0, 0.0, 0.0 };

/* coefficient table of the piece that contains radius s */
static const double *g_piece(int profile, double s)
{
    if (profile == ORC_UNIT) return UNIT_G;
    if (s < 1.0) return M4_G_INNER;
    if (s < 2.0) return M4_G_SHELL;
    return M4_G_OUTER;
}

static double prof_scale(int profile) { return profile == ORC_UNIT ? 1.0 : 1.0 / M_PI; }

/* w(q) of the M4 kernel (dimensionless, W = w / (pi h^3)) */
double orc_w(double q)
{
    if (q < 0) q = -q;
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) { double u = 2.0 - q; return 0.25 * u * u * u; }
    return 0.0;
}

/* F(s) = int_0^s W q^2 dq per unit solid angle (h = 1) */
double orc_F(int profile, double s)
{
    if (profile == ORC_UNIT) return s * s * s / 3.0;
    double s2 = s * s, s3 = s2 * s, s4 = s3 * s, s5 = s4 * s, s6 = s5 * s;
    double pf;
    if (s < 1.0) pf = s3 / 3.0 - 0.3 * s5 + s6 / 8.0;
    else if (s < 2.0) pf = -1.0 / 60.0 + 2.0 * s3 / 3.0 - 0.75 * s4 + 0.3 * s5 - s6 / 24.0;
    else pf = 0.25;
    return pf / M_PI;
}

/* G(s), the antiderivative of F(s)/s^2 with G(0) = 0 */
double orc_G(int profile, double s)
{
    const double *g = g_piece(profile, s);
    double acc = 0.0;
    for (int k = 0; k < 6; k++) {
        if (g[k] == 0.0) continue;
        acc += g[k] * pow(s, (double)NEXP[k]);
    }
    return acc * prof_scale(profile);
}

/* ------------------------------------------------------------------------ */
/* Angular moments P_n(alpha) = int_0^alpha S(x)^n dx,                        */
/* S(x)^2 = r0^2 + R0^2 sec^2 x.  With A = r0^2, B = R0^2, c^2 = A + B,      */
/* t = tan(alpha), S = sqrt(c^2 + B t^2), a = asinh(R0 t / c) and            */
/* lambda = atan(r0 t / S):                                                  */
/*   r0 P_-1 = lambda                                                        */
/*   P_0 = alpha                                                             */
/*   P_2 = A alpha + B t                                                     */
/*   P_3 = (B t S + R0 c^2 a)/2 + A R0 a + r0^3 lambda                        */
/*   P_4 = A^2 alpha + 2 A B t + B^2 (t + t^3/3)                              */
/*   P_5 = B (t S^3/4 + 3 c^2 t S/8) + 3 R0 c^4 a/8 + A P_3                    */
/* (each obtained by differentiating the right-hand side back to S^n).       */
/* out[0] holds r0*P_-1 so that r0 = 0 stays finite.                          */
/* ------------------------------------------------------------------------ */
void orc_moments(double r0, double R0, double alpha, double out[6])
{
    double A = r0 * r0, B = R0 * R0, c2 = A + B, c = sqrt(c2);
    double t = tan(alpha);
    double S = sqrt(c2 + B * t * t);
    double a = (c > 0.0) ? asinh(R0 * t / c) : 0.0;
    double lam = (S > 0.0) ? atan(r0 * t / S) : 0.0;
    double P3 = 0.5 * (B * t * S + R0 * c2 * a) + A * R0 * a + A * r0 * lam;
    out[0] = lam;
    out[1] = alpha;
    out[2] = A * alpha + B * t;
    out[3] = P3;
    out[4] = A * A * alpha + 2.0 * A * B * t + B * B * (t + t * t * t / 3.0);
    out[5] = B * (t * S * S * S / 4.0 + 3.0 * c2 * t * S / 8.0) + 3.0 * R0 * c2 * c2 * a / 8.0 + A * P3;
}

/* ------------------------------------------------------------------------ */
/* Integral of W over the right-angled vertex pyramid with apex p, base the  */
/* right triangle (f, g, v): |pf| = r0 (f = projection of p on the wall),    */
/* |fg| = R0 (g = projection of f on the edge line, right angle at g), v on  */
/* the edge, phi = angle at f between fg and fv (0 <= phi < pi/2).  Units of */
/* h.  The alpha-range [0, phi] is split where S(alpha) crosses the piece     */
/* radii of the profile (s = 1 and s = 2 for M4), at tan(alpha_k) =          */
/* sqrt(k^2 - r0^2 - R0^2) / R0.                                              */
/* ------------------------------------------------------------------------ */
double orc_pyramid(int profile, double r0, double R0, double phi)
{
    if (r0 <= 0.0 || R0 <= 0.0 || phi <= 0.0) return 0.0;
    double c2 = r0 * r0 + R0 * R0;
    double bounds[4];
    int nb = 0;
    bounds[nb++] = 0.0;
    if (profile == ORC_M4) {
        for (int k = 1; k <= 2; k++) {
            double kk = (double)(k * k);
            if (kk > c2) {
                double ak = atan(sqrt(kk - c2) / R0);
                if (ak < phi) bounds[nb++] = ak;
            }
        }
    }
    bounds[nb++] = phi;

    double sum = 0.0;
    for (int s = 0; s + 1 < nb; s++) {
        double lo = bounds[s], hi = bounds[s + 1];
        if (hi <= lo) continue;
        double mid = 0.5 * (lo + hi);
        double tm = tan(mid);
        double Smid = sqrt(c2 + R0 * R0 * tm * tm);
        const double *g = g_piece(profile, Smid);
        double Plo[6], Phi[6];
        orc_moments(r0, R0, lo, Plo);
        orc_moments(r0, R0, hi, Phi);
        /* r0 * sum_n g_n (P_n(hi) - P_n(lo)); the n = -1 moment is stored times r0 */
        double piece = g[0] * (Phi[0] - Plo[0]);
        for (int k = 1; k < 6; k++) piece += r0 * g[k] * (Phi[k] - Plo[k]);
        sum += piece;
    }
    /* minus r0 * phi * G(r0) */
    const double *g0 = g_piece(profile, r0);
    double Gr0 = 0.0;
    for (int k = 0; k < 6; k++) {
        if (g0[k] == 0.0) continue;
        Gr0 += g0[k] * pow(r0, (double)NEXP[k]);
    }
    sum -= r0 * phi * Gr0;
    return sum * prof_scale(profile);
}

/* ------------------------------------------------------------------------ */
/* Cell geometry (CSR):                                                       */
/*   cell_face_off[n_cells+1]  faces of cell i are [off[i], off[i+1])         */
/*   face_vert_off[n_faces+1]  vertex slots of face j                         */
/*   face_vert[]               vertex ids, counter-clockwise seen from the     */
/*                             outside (about the outward normal)             */
/*   face_plane[4*n_faces]     (nx, ny, nz, c): outward unit normal, n.x = c   */
/*   verts[3*n_verts]                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_cells;
    const int64_t *cell_face_off;
    const int64_t *face_vert_off;
    const int32_t *face_vert;
    const double *face_plane;
    const double *verts;
} orc_cells;

static int sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* ------------------------------------------------------------------------ */
/* Tabulated pyramid integral (the variant Sec. II-B describes: the integral  */
/* is pre-computed and interpolated).  Reading (the paper gives no layout):   */
/* I(r0, R0, phi) on a uniform grid of n0 x n1 x n2 nodes over r0 in [0, 2],  */
/* R0 in [0, 2] and phi in [0, pi/2], read by trilinear interpolation.        */
/* Outside the grid the pyramid's mass follows from the solid angle Omega of  */
/* its triangle (elementary): the pyramid holds the kernel mass of its cone,  */
/* Omega / (4 pi), less D, the mass of the cone beyond the wall.  D = 0 for   */
/* r0 >= 2 (the wall lies beyond the support), and for R0 >= 2 D no longer    */
/* depends on R0 (the support's cross-section with the wall, of radius        */
/* sqrt(4 - r0^2) <= 2 about the foot, lies inside the triangle's wedge), so  */
/*   r0 >= 2:  I = Omega / (4 pi)                                             */
/*   R0 > 2:   I = I(r0, 2, phi) + (Omega(r0, R0, phi) - Omega(r0, 2, phi)) / (4 pi). */
/* Node values come from orc_pyramid; the last phi plane is the limit         */
/* phi -> pi/2, taken at pi/2 - 1e-12.                                        */
/* ------------------------------------------------------------------------ */
static const double *g_tab;
static int g_tn0, g_tn1, g_tn2;

static double tab_r0(int i, int n0) { return 2.0 * (double)i / (double)(n0 - 1); }
static double tab_R0(int j, int n1) { return 2.0 * (double)j / (double)(n1 - 1); }
static double tab_phi(int k, int n2)
{
    return k == n2 - 1 ? 0.5 * M_PI - 1e-12 : 0.5 * M_PI * (double)k / (double)(n2 - 1);
}

/* solid angle of the right triangle (legs R0 at the foot, angle phi there) seen
 * from the apex at height r0 > 0: phi - r0 P_-1(phi) = phi - atan(r0 tan(phi) / S) */
double orc_solid_angle(double r0, double R0, double phi)
{
    if (r0 <= 0.0 || R0 <= 0.0 || phi <= 0.0) return 0.0;
    double t = tan(phi);
    double S = sqrt(r0 * r0 + R0 * R0 * (1.0 + t * t));
    return phi - atan(r0 * t / S);
}

/* node values, index (i * n1 + j) * n2 + k */
void orc_table_build(int n0, int n1, int n2, double *tab)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n0; i++)
        for (int j = 0; j < n1; j++)
            for (int k = 0; k < n2; k++)
                tab[((int64_t)i * n1 + j) * n2 + k] =
                    orc_pyramid(ORC_M4, tab_r0(i, n0), tab_R0(j, n1), tab_phi(k, n2));
}

/* the table that ORC_TABLE reads (the caller keeps it alive) */
void orc_table_use(const double *tab, int n0, int n1, int n2)
{
    g_tab = tab;
    g_tn0 = n0;
    g_tn1 = n1;
    g_tn2 = n2;
}

/* grid coordinate x in [0, n - 1] -> lower node and weight */
static void tab_cell(double x, int n, int *i, double *t)
{
    int k = (int)floor(x);
    if (k < 0) k = 0;
    if (k > n - 2) k = n - 2;
    *i = k;
    *t = x - (double)k;
}

static double tab_trilinear(double r0, double R0, double phi)
{
    int i, j, k;
    double a, b, c;
    tab_cell(r0 * (double)(g_tn0 - 1) / 2.0, g_tn0, &i, &a);
    tab_cell(R0 * (double)(g_tn1 - 1) / 2.0, g_tn1, &j, &b);
    tab_cell(phi * (double)(g_tn2 - 1) / (0.5 * M_PI), g_tn2, &k, &c);
    double v = 0.0;
    for (int di = 0; di < 2; di++)
        for (int dj = 0; dj < 2; dj++)
            for (int dk = 0; dk < 2; dk++) {
                double w = (di ? a : 1.0 - a) * (dj ? b : 1.0 - b) * (dk ? c : 1.0 - c);
                v += w * g_tab[((int64_t)(i + di) * g_tn1 + (j + dj)) * g_tn2 + (k + dk)];
            }
    return v;
}

/* the pyramid integral through the table */
double orc_table_interp(double r0, double R0, double phi)
{
    if (r0 <= 0.0 || R0 <= 0.0 || phi <= 0.0) return 0.0;
    if (!(r0 < 2.0)) return orc_solid_angle(r0, R0, phi) / (4.0 * M_PI);
    if (R0 > 2.0)
        return tab_trilinear(r0, 2.0, phi) +
               (orc_solid_angle(r0, R0, phi) - orc_solid_angle(r0, 2.0, phi)) / (4.0 * M_PI);
    return tab_trilinear(r0, R0, phi);
}

/* signed right-triangle term T(l) = sign(l) * I(r0, R0, atan(|l|/R0)) */
static double tri_term(int profile, double r0, double R0, double l)
{
    if (l == 0.0) return 0.0;
    double phi = atan(fabs(l) / R0);
    if (profile == ORC_TABLE) return sgn(l) * orc_table_interp(r0, R0, phi);
    return sgn(l) * orc_pyramid(profile, r0, R0, phi);
}

/*
 * Integral of W over one convex cell for a particle at p with smoothing length h.
 *
 * Signed-cone identity: for any point p and a convex cell with outward unit
 * normals n_j and planes n_j.x = c_j, the cell is the signed sum over faces of
 * the cones from p to each face polygon, with sign sigma_j = sign(c_j - n_j.p)
 * (+1 when p lies on the inner side of the wall).  Each face polygon is the
 * signed sum over its directed edges v_k -> v_{k+1} (counter-clockwise about
 * n_j) of triangles (f, v_k, v_{k+1}), f the foot of p on the wall, with sign
 * sign(rho_k), rho_k = m_k.(f - v_k), m_k = n_j x e_k the in-plane normal of
 * the edge pointing into the polygon.  Each such triangle is split at g, the
 * foot of f on the edge line, into right triangles (f, g, v) whose signed
 * along-edge coordinates are l_a = e.(v_k - g) and l_b = e.(v_{k+1} - g):
 *     triangle(f, v_k, v_{k+1}) = T(l_b) - T(l_a).
 * Hence
 *     f_ai = sum_j sigma_j sum_k sign(rho_k) [T(l_b) - T(l_a)].
 */
double orc_pair_fraction(int profile, const double *p, double h, const orc_cells *C, int64_t cell)
{
    double sum = 0.0;
    for (int64_t j = C->cell_face_off[cell]; j < C->cell_face_off[cell + 1]; j++) {
        const double *pl = C->face_plane + 4 * j;
        double nx = pl[0], ny = pl[1], nz = pl[2], cc = pl[3];
        double d = cc - (nx * p[0] + ny * p[1] + nz * p[2]);
        if (d == 0.0) continue;
        double sigma = (double)sgn(d);
        double r0 = fabs(d) / h;
        double fx = p[0] + d * nx, fy = p[1] + d * ny, fz = p[2] + d * nz;
        int64_t k0 = C->face_vert_off[j], k1 = C->face_vert_off[j + 1];
        int64_t nv = k1 - k0;
        double face_sum = 0.0;
        for (int64_t k = 0; k < nv; k++) {
            const double *va = C->verts + 3 * (int64_t)C->face_vert[k0 + k];
            const double *vb = C->verts + 3 * (int64_t)C->face_vert[k0 + (k + 1) % nv];
            double ex = vb[0] - va[0], ey = vb[1] - va[1], ez = vb[2] - va[2];
            double len = sqrt(ex * ex + ey * ey + ez * ez);
            if (len == 0.0) continue;
            ex /= len; ey /= len; ez /= len;
            /* m = n x e */
            double mx = ny * ez - nz * ey, my = nz * ex - nx * ez, mz = nx * ey - ny * ex;
            double rho = mx * (fx - va[0]) + my * (fy - va[1]) + mz * (fz - va[2]);
            if (rho == 0.0) continue;
            double gx = fx - rho * mx, gy = fy - rho * my, gz = fz - rho * mz;
            double la = ex * (va[0] - gx) + ey * (va[1] - gy) + ez * (va[2] - gz);
            double lb = ex * (vb[0] - gx) + ey * (vb[1] - gy) + ez * (vb[2] - gz);
            double R0 = fabs(rho) / h;
            face_sum += sgn(rho) * (tri_term(profile, r0, R0, lb / h) - tri_term(profile, r0, R0, la / h));
        }
        sum += sigma * face_sum;
    }
    return sum;
}

/* ------------------------------------------------------------------------ */
/* Pair set.  Distance from p to the closed convex cell: 0 if p is on the    */
/* inner side of every wall; otherwise the minimum over walls with p on the  */
/* outer side (d_j < 0) of the distance to that wall polygon.  The distance  */
/* to a polygon is |d_j| when the projection lies inside it (left of every   */
/* directed edge seen from outside), else the least distance to its edge     */
/* segments.  Squared distances only; no fused multiply-add (gcc does not    */
/* contract on the baseline x86-64 target and this file is built without     */
/* -ffast-math), so every operation is an IEEE-rounded add, mul or divide.    */
/* ------------------------------------------------------------------------ */
static double seg_dist2(const double *p, const double *a, const double *b)
{
    double ex = b[0] - a[0], ey = b[1] - a[1], ez = b[2] - a[2];
    double wx = p[0] - a[0], wy = p[1] - a[1], wz = p[2] - a[2];
    double ee = ex * ex + ey * ey + ez * ez;
    double t = 0.0;
    if (ee > 0.0) {
        t = (wx * ex + wy * ey + wz * ez) / ee;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    double qx = wx - t * ex, qy = wy - t * ey, qz = wz - t * ez;
    return qx * qx + qy * qy + qz * qz;
}

double orc_cell_dist2(const double *p, const orc_cells *C, int64_t cell)
{
    int inside = 1;
    double best = INFINITY;
    for (int64_t j = C->cell_face_off[cell]; j < C->cell_face_off[cell + 1]; j++) {
        const double *pl = C->face_plane + 4 * j;
        double d = pl[3] - (pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2]);
        if (!(d < 0.0)) continue;
        inside = 0;
        int64_t k0 = C->face_vert_off[j], k1 = C->face_vert_off[j + 1];
        int64_t nv = k1 - k0;
        int left = 1;
        for (int64_t k = 0; k < nv; k++) {
            const double *a = C->verts + 3 * (int64_t)C->face_vert[k0 + k];
            const double *b = C->verts + 3 * (int64_t)C->face_vert[k0 + (k + 1) % nv];
            double ex = b[0] - a[0], ey = b[1] - a[1], ez = b[2] - a[2];
            double wx = p[0] - a[0], wy = p[1] - a[1], wz = p[2] - a[2];
            double cr = (ey * wz - ez * wy) * pl[0] + (ez * wx - ex * wz) * pl[1] + (ex * wy - ey * wx) * pl[2];
            if (cr < 0.0) { left = 0; break; }
        }
        double dd;
        if (left) {
            dd = d * d;
        } else {
            dd = INFINITY;
            for (int64_t k = 0; k < nv; k++) {
                const double *a = C->verts + 3 * (int64_t)C->face_vert[k0 + k];
                const double *b = C->verts + 3 * (int64_t)C->face_vert[k0 + (k + 1) % nv];
                double e2 = seg_dist2(p, a, b);
                if (e2 < dd) dd = e2;
            }
        }
        if (dd < best) best = dd;
    }
    return inside ? 0.0 : best;
}

/* Pair (a, i) exists iff dist(p_a, cell_i)^2 < (2 h_a)^2. */
static int meets(const double *p, double h, const orc_cells *C, int64_t cell)
{
    double two_h = 2.0 * h;
    return orc_cell_dist2(p, C, cell) < two_h * two_h;
}

/* Brute force over every cell: for small inputs and for tests of the grid. */
int64_t orc_pairs_brute(int64_t n, const double *xyz, const double *h, const orc_cells *C,
                        int32_t *pair_p, int32_t *pair_c, int64_t cap)
{
    int64_t np = 0;
    for (int64_t i = 0; i < C->n_cells; i++)
        for (int64_t a = 0; a < n; a++)
            if (meets(xyz + 3 * a, h[a], C, i)) {
                if (pair_p && np < cap) { pair_p[np] = (int32_t)a; pair_c[np] = (int32_t)i; }
                np++;
            }
    return np;
}

/*
 * Pair set with a plain uniform grid over cell bounding boxes.  Output sorted
 * by cell, then by particle.  Returns the pair count; arrays may be NULL (count
 * only) and are filled up to cap entries.
 */
int64_t orc_pairs(int64_t n, const double *xyz, const double *h, const orc_cells *C,
                  const double *box, int32_t *pair_p, int32_t *pair_c, int64_t cap)
{
    int64_t nc = C->n_cells;
    if (nc == 0 || n == 0) return 0;
    /* bounding boxes */
    double *bb = (double *)malloc(sizeof(double) * 6 * nc);
    for (int64_t i = 0; i < nc; i++) {
        double lo[3] = { INFINITY, INFINITY, INFINITY }, hi[3] = { -INFINITY, -INFINITY, -INFINITY };
        for (int64_t j = C->cell_face_off[i]; j < C->cell_face_off[i + 1]; j++)
            for (int64_t k = C->face_vert_off[j]; k < C->face_vert_off[j + 1]; k++) {
                const double *v = C->verts + 3 * (int64_t)C->face_vert[k];
                for (int d = 0; d < 3; d++) {
                    if (v[d] < lo[d]) lo[d] = v[d];
                    if (v[d] > hi[d]) hi[d] = v[d];
                }
            }
        for (int d = 0; d < 3; d++) { bb[6 * i + d] = lo[d]; bb[6 * i + 3 + d] = hi[d]; }
    }
    int G = (int)ceil(2.0 * cbrt((double)nc));
    if (G < 1) G = 1;
    if (G > 256) G = 256;
    double ext[3], inv[3];
    for (int d = 0; d < 3; d++) {
        ext[d] = box[3 + d] - box[d];
        inv[d] = G / ext[d];
    }
    int64_t nbin = (int64_t)G * G * G;
#define BINRANGE(lo_, hi_, d_, a_, b_)                                   \
    do {                                                                 \
        a_ = (int)floor(((lo_) - box[d_]) * inv[d_]);                    \
        b_ = (int)floor(((hi_) - box[d_]) * inv[d_]);                    \
        if (a_ < 0) a_ = 0;                                              \
        if (b_ > G - 1) b_ = G - 1;                                      \
    } while (0)
    /* bins: CSR of the cells whose bounding box overlaps each bin */
    int64_t *bstart = (int64_t *)calloc(nbin + 1, sizeof(int64_t));
    for (int64_t i = 0; i < nc; i++) {
        int x0, x1, y0, y1, z0, z1;
        BINRANGE(bb[6 * i + 0], bb[6 * i + 3], 0, x0, x1);
        BINRANGE(bb[6 * i + 1], bb[6 * i + 4], 1, y0, y1);
        BINRANGE(bb[6 * i + 2], bb[6 * i + 5], 2, z0, z1);
        for (int z = z0; z <= z1; z++)
            for (int y = y0; y <= y1; y++)
                for (int x = x0; x <= x1; x++) bstart[((int64_t)z * G + y) * G + x + 1]++;
    }
    for (int64_t b = 0; b < nbin; b++) bstart[b + 1] += bstart[b];
    int64_t *blist = (int64_t *)malloc(sizeof(int64_t) * (bstart[nbin] > 0 ? bstart[nbin] : 1));
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * nbin);
        memcpy(fill, bstart, sizeof(int64_t) * nbin);
        for (int64_t i = 0; i < nc; i++) {
            int x0, x1, y0, y1, z0, z1;
            BINRANGE(bb[6 * i + 0], bb[6 * i + 3], 0, x0, x1);
            BINRANGE(bb[6 * i + 1], bb[6 * i + 4], 1, y0, y1);
            BINRANGE(bb[6 * i + 2], bb[6 * i + 5], 2, z0, z1);
            for (int z = z0; z <= z1; z++)
                for (int y = y0; y <= y1; y++)
                    for (int x = x0; x <= x1; x++) blist[fill[((int64_t)z * G + y) * G + x]++] = i;
        }
        free(fill);
    }

    /* per particle: candidate cells (deduplicated, ascending) that meet the ball */
    int64_t *pcount = (int64_t *)calloc(n + 1, sizeof(int64_t));
    int32_t **plist = (int32_t **)calloc(n, sizeof(int32_t *));
#pragma omp parallel
    {
        int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * nc);
        for (int64_t i = 0; i < nc; i++) stamp[i] = -1;
        int64_t tcap = 256;
        int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * tcap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < n; a++) {
            const double *p = xyz + 3 * a;
            double r = 2.0 * h[a];
            int x0, x1, y0, y1, z0, z1;
            BINRANGE(p[0] - r, p[0] + r, 0, x0, x1);
            BINRANGE(p[1] - r, p[1] + r, 1, y0, y1);
            BINRANGE(p[2] - r, p[2] + r, 2, z0, z1);
            int64_t m = 0;
            for (int z = z0; z <= z1; z++)
                for (int y = y0; y <= y1; y++)
                    for (int x = x0; x <= x1; x++) {
                        int64_t b = ((int64_t)z * G + y) * G + x;
                        for (int64_t q = bstart[b]; q < bstart[b + 1]; q++) {
                            int64_t i = blist[q];
                            if (stamp[i] == a) continue;
                            stamp[i] = a;
                            if (!meets(p, h[a], C, i)) continue;
                            if (m == tcap) {
                                tcap *= 2;
                                tmp = (int32_t *)realloc(tmp, sizeof(int32_t) * tcap);
                            }
                            tmp[m++] = (int32_t)i;
                        }
                    }
            /* insertion sort: lists are short */
            for (int64_t u = 1; u < m; u++) {
                int32_t key = tmp[u];
                int64_t v = u - 1;
                while (v >= 0 && tmp[v] > key) { tmp[v + 1] = tmp[v]; v--; }
                tmp[v + 1] = key;
            }
            plist[a] = (int32_t *)malloc(sizeof(int32_t) * (m > 0 ? m : 1));
            memcpy(plist[a], tmp, sizeof(int32_t) * m);
            pcount[a] = m;
        }
        free(tmp);
        free(stamp);
    }
    int64_t total = 0;
    for (int64_t a = 0; a < n; a++) total += pcount[a];
    if (pair_p && pair_c) {
        /* counting sort by cell, stable in particle order */
        int64_t *coff = (int64_t *)calloc(nc + 1, sizeof(int64_t));
        for (int64_t a = 0; a < n; a++)
            for (int64_t u = 0; u < pcount[a]; u++) coff[plist[a][u] + 1]++;
        for (int64_t i = 0; i < nc; i++) coff[i + 1] += coff[i];
        for (int64_t a = 0; a < n; a++)
            for (int64_t u = 0; u < pcount[a]; u++) {
                int64_t slot = coff[plist[a][u]]++;
                if (slot < cap) { pair_p[slot] = (int32_t)a; pair_c[slot] = plist[a][u]; }
            }
        free(coff);
    }
    for (int64_t a = 0; a < n; a++) free(plist[a]);
    free(plist);
    free(pcount);
    free(bstart);
    free(blist);
    free(bb);
#undef BINRANGE
    return total;
}

/*
 * Pairs restricted to selected cells (brute force over particles) or to
 * selected particles (brute force over cells), for sampled checks of large
 * inputs.  Output in selection order, then ascending particle (cell) index.
 * Returns the pair count; arrays may be NULL (count only).
 */
static void cell_box(const orc_cells *C, int64_t i, double *lo, double *hi)
{
    for (int d = 0; d < 3; d++) { lo[d] = INFINITY; hi[d] = -INFINITY; }
    for (int64_t j = C->cell_face_off[i]; j < C->cell_face_off[i + 1]; j++)
        for (int64_t k = C->face_vert_off[j]; k < C->face_vert_off[j + 1]; k++) {
            const double *v = C->verts + 3 * (int64_t)C->face_vert[k];
            for (int d = 0; d < 3; d++) {
                if (v[d] < lo[d]) lo[d] = v[d];
                if (v[d] > hi[d]) hi[d] = v[d];
            }
        }
}

static int box_near(const double *p, double r, const double *lo, const double *hi)
{
    for (int d = 0; d < 3; d++)
        if (p[d] + r < lo[d] || p[d] - r > hi[d]) return 0;
    return 1;
}

int64_t orc_pairs_for_cells(int64_t n, const double *xyz, const double *h, const orc_cells *C, int64_t nsel,
                            const int32_t *sel, int32_t *pair_p, int32_t *pair_c, int64_t cap)
{
    int64_t *cnt = (int64_t *)calloc(nsel + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            for (int64_t t = 0; t < nsel; t++) cnt[t + 1] += cnt[t];
            if (!pair_p) break;
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t t = 0; t < nsel; t++) {
            int64_t i = sel[t];
            double lo[3], hi[3];
            cell_box(C, i, lo, hi);
            int64_t k = pass ? cnt[t] : 0;
            for (int64_t a = 0; a < n; a++) {
                const double *p = xyz + 3 * a;
                if (!box_near(p, 2.0 * h[a], lo, hi)) continue;
                if (!meets(p, h[a], C, i)) continue;
                if (pass && k < cap) { pair_p[k] = (int32_t)a; pair_c[k] = (int32_t)i; }
                k++;
            }
            if (!pass) cnt[t + 1] = k;
        }
    }
    int64_t total = cnt[nsel];
    free(cnt);
    return total;
}

int64_t orc_pairs_for_particles(int64_t n, const double *xyz, const double *h, const orc_cells *C, int64_t nsel,
                                const int32_t *sel, int32_t *pair_p, int32_t *pair_c, int64_t cap)
{
    int64_t nc = C->n_cells;
    double *bb = (double *)malloc(sizeof(double) * 6 * (nc > 0 ? nc : 1));
    for (int64_t i = 0; i < nc; i++) cell_box(C, i, bb + 6 * i, bb + 6 * i + 3);
    int64_t total = 0;
    for (int64_t t = 0; t < nsel; t++) {
        int64_t a = sel[t];
        if (a < 0 || a >= n) continue;
        const double *p = xyz + 3 * a;
        for (int64_t i = 0; i < nc; i++) {
            if (!box_near(p, 2.0 * h[a], bb + 6 * i, bb + 6 * i + 3)) continue;
            if (!meets(p, h[a], C, i)) continue;
            if (pair_p && total < cap) { pair_p[total] = (int32_t)a; pair_c[total] = (int32_t)i; }
            total++;
        }
    }
    free(bb);
    return total;
}

/* f_ai for a list of pairs (any order). */
void orc_pair_fractions(int profile, const double *xyz, const double *h, const orc_cells *C, int64_t npairs,
                        const int32_t *pair_p, const int32_t *pair_c, double *f)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < npairs; q++)
        f[q] = orc_pair_fraction(profile, xyz + 3 * (int64_t)pair_p[q], h[pair_p[q]], C, pair_c[q]);
}

/*
 * Reductions of Eq. (3) with the sum-to-one normalisation:
 *   S_a = sum over pairs of particle a of f,  M_i = sum over pairs of cell i of m_a f / S_a,
 *   rho_i = M_i / V_i.  Plain sequential sums in pair order.
 */
void orc_reduce(int64_t n, const double *m, int64_t n_cells, const double *vol, int64_t npairs,
                const int32_t *pair_p, const int32_t *pair_c, const double *f, double *S, double *M, double *rho)
{
    for (int64_t a = 0; a < n; a++) S[a] = 0.0;
    for (int64_t q = 0; q < npairs; q++) S[pair_p[q]] += f[q];
    for (int64_t i = 0; i < n_cells; i++) M[i] = 0.0;
    for (int64_t q = 0; q < npairs; q++) {
        int32_t a = pair_p[q];
        if (S[a] > 0.0) M[pair_c[q]] += m[a] * (f[q] / S[a]);
    }
    for (int64_t i = 0; i < n_cells; i++) rho[i] = (vol && vol[i] > 0.0) ? M[i] / vol[i] : 0.0;
}

/*
 * Inverse mapping (Sec. II-B, Eq. (4)): a particle value from the cell values
 * weighted by the particle's kernel integrals over the cells, with the same
 * sum-to-one normalisation as the forward mapping,
 *   q_a = (sum over pairs of particle a of q_i f) / S_a,   0 when S_a = 0,
 * so that sum_a m_a q_a = sum_i q_i M_i.  Plain sequential sums in pair order.
 */
void orc_map_back(int64_t n, int64_t npairs, const int32_t *pair_p, const int32_t *pair_c, const double *f,
                  const double *S, const double *q_cell, double *q_part)
{
    for (int64_t a = 0; a < n; a++) q_part[a] = 0.0;
    for (int64_t q = 0; q < npairs; q++) q_part[pair_p[q]] += q_cell[pair_c[q]] * f[q];
    for (int64_t a = 0; a < n; a++) q_part[a] = S[a] > 0.0 ? q_part[a] / S[a] : 0.0;
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Operation count of the direct form above (the flop model of the mapping). */
/* Counted by hand from the statements of orc_moments, orc_pyramid, tri_term */
/* and orc_pair_fraction: every add, subtract, multiply, divide, square root */
/* and elementary function (tan, atan, asinh, pow) counts one; compares,     */
/* sign tests and fabs count zero (the file is built without fused           */
/* multiply-add, so every operation is one IEEE operation).                  */
/*   orc_moments                      61  (5 of them sqrt/tan/asinh/atan)    */
/*   orc_pyramid   3 (c^2) + 4 per breakpoint found (sub, sqrt, div, atan)   */
/*                 + 153 per piece (midpoint 2, tan 1, S 5, two moments 122, */
/*                   the g_0 term 2, five g_n terms 4 each, sum 1)           */
/*                 + 3 per nonzero coefficient of G(r0) (pow, mul, add)       */
/*                 + 4 (r0 phi G(r0), the subtraction, the scale)            */
/*   tri_term      3 (|l|/R0, atan, the sign) + the pyramid (l != 0)         */
/*   edge          29 up to rho (e 3, |e| 6, e/|e| 3, m 9, rho 8); when      */
/*                 rho != 0, 28 more (g 6, l_a 8, l_b 8, R0 1, l/h 2, the    */
/*                 update 3) and its two tri_terms                           */
/*   face          6 (d); when d != 0, 9 more (r0 1, f 6, the update 2) and  */
/*                 its edges                                                 */
/* The walk below follows orc_pair_fraction's control flow (the same skips,  */
/* the same breakpoints and pieces) without the arithmetic of the integrals. */
/* counts[0..6]: faces, edges, triangle terms, pyramids, pieces, moment      */
/* evaluations, flops (all summed over the pairs).                           */
/* ------------------------------------------------------------------------ */
static void count_pyramid(double r0, double R0, double phi, int64_t *cnt)
{
    if (r0 <= 0.0 || R0 <= 0.0 || phi <= 0.0) return;
    double c2 = r0 * r0 + R0 * R0;
    double bounds[4];
    int nb = 0;
    int64_t fl = 3;
    bounds[nb++] = 0.0;
    for (int k = 1; k <= 2; k++) {
        double kk = (double)(k * k);
        if (kk > c2) {
            double ak = atan(sqrt(kk - c2) / R0);
            fl += 4;
            if (ak < phi) bounds[nb++] = ak;
        }
    }
    bounds[nb++] = phi;
    for (int s = 0; s + 1 < nb; s++) {
        if (bounds[s + 1] <= bounds[s]) continue;
        fl += 153;
        cnt[4] += 1;
        cnt[5] += 2;
    }
    const double *g0 = g_piece(ORC_M4, r0);
    for (int k = 0; k < 6; k++)
        if (g0[k] != 0.0) fl += 3;
    fl += 4;
    cnt[3] += 1;
    cnt[6] += fl;
}

static void count_pair(const double *p, double h, const orc_cells *C, int64_t cell, int64_t *cnt)
{
    for (int64_t j = C->cell_face_off[cell]; j < C->cell_face_off[cell + 1]; j++) {
        const double *pl = C->face_plane + 4 * j;
        double nx = pl[0], ny = pl[1], nz = pl[2], cc = pl[3];
        double d = cc - (nx * p[0] + ny * p[1] + nz * p[2]);
        cnt[0] += 1;
        cnt[6] += 6;
        if (d == 0.0) continue;
        cnt[6] += 9;
        double r0 = fabs(d) / h;
        double fx = p[0] + d * nx, fy = p[1] + d * ny, fz = p[2] + d * nz;
        int64_t k0 = C->face_vert_off[j], k1 = C->face_vert_off[j + 1];
        int64_t nv = k1 - k0;
        for (int64_t k = 0; k < nv; k++) {
            const double *va = C->verts + 3 * (int64_t)C->face_vert[k0 + k];
            const double *vb = C->verts + 3 * (int64_t)C->face_vert[k0 + (k + 1) % nv];
            double ex = vb[0] - va[0], ey = vb[1] - va[1], ez = vb[2] - va[2];
            double len = sqrt(ex * ex + ey * ey + ez * ez);
            cnt[1] += 1;
            cnt[6] += 9;
            if (len == 0.0) continue;
            cnt[6] += 20;
            ex /= len; ey /= len; ez /= len;
            double mx = ny * ez - nz * ey, my = nz * ex - nx * ez, mz = nx * ey - ny * ex;
            double rho = mx * (fx - va[0]) + my * (fy - va[1]) + mz * (fz - va[2]);
            if (rho == 0.0) continue;
            cnt[6] += 28;
            double gx = fx - rho * mx, gy = fy - rho * my, gz = fz - rho * mz;
            double la = ex * (va[0] - gx) + ey * (va[1] - gy) + ez * (va[2] - gz);
            double lb = ex * (vb[0] - gx) + ey * (vb[1] - gy) + ez * (vb[2] - gz);
            double R0 = fabs(rho) / h;
            double ls[2] = { lb / h, la / h };
            for (int q = 0; q < 2; q++) {
                if (ls[q] == 0.0) continue;
                cnt[2] += 1;
                cnt[6] += 3;
                count_pyramid(r0, R0, atan(fabs(ls[q]) / R0), cnt);
            }
        }
    }
}

void orc_flop_model(const double *xyz, const double *h, const orc_cells *C, int64_t npairs, const int32_t *pair_p,
                    const int32_t *pair_c, int64_t counts[7])
{
    for (int k = 0; k < 7; k++) counts[k] = 0;
#pragma omp parallel
    {
        int64_t loc[7] = { 0, 0, 0, 0, 0, 0, 0 };
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < npairs; q++)
            count_pair(xyz + 3 * (int64_t)pair_p[q], h[pair_p[q]], C, pair_c[q], loc);
#pragma omp critical
        for (int k = 0; k < 7; k++) counts[k] += loc[k];
    }
}
