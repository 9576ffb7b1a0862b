// Integration of the M4 kernel over each (particle, cell) pair, Sec. II-B.
//
// Far-field-subtracted form.  With lengths in units of h, the kernel mass in
// a cone of directions up to radius s is F(s) per steradian, F(s) -> 1/(4 pi)
// for s >= 2.  Writing F = 1/(4 pi) - F_c splits each vertex-pyramid integral
// into a solid-angle part and a remainder that vanishes beyond the support:
//     I(r0, R0, phi) = Omega/(4 pi) - [ Q(phi) - phi H(r0) ],
//     Q(phi) = r0 int_0^phi G_c(S(alpha)) dalpha,   H(r0) = r0 G_c(r0),
// where G_c' = F_c/s^2, G_c = 0 for s >= 2, and S(alpha) is the distance from
// the particle to the edge line's point at in-plane angle alpha.  Summed with
// the signs of the signed-cone decomposition, the solid-angle parts give the
// winding number of the cell about the particle (1 inside, 0 outside), so
//     f = [p inside] - (1/pi) sum_faces sigma_j { sum_edges sign(rho) [Q(l_b) - Q(l_a)] - pi H(r0) A_j },
// with A_j the signed angle the face's edges subtend at the foot point, and
// the per-edge Q difference taken along the edge (signed coordinate l from
// the foot g of the projection point on the edge line).  Walls with r0 >= 2
// and edges whose line lies beyond 2h contribute nothing to Q; such walls are
// skipped entirely.
//
// pi G_c as polynomials in s (exponents -1, 0, 2, 3, 4, 5):
//   s <= 1:      -1/(4s) + 7/20 - s^2/6 + 3 s^4/40 - s^5/40
//   1 <= s <= 2: -4/(15s) + 2/5 - s^2/3 + s^3/4 - 3 s^4/40 + s^5/120
//              = -(2 - s)^5 (s + 1) / (120 s)
// and the angular moments P_n = int S^n dalpha are evaluated in closed form
// from l (t = l/R0, S = sqrt(c^2 + l^2), c^2 = r0^2 + R0^2):
//   r0 P_-1 = atan2(r0 l, R0 S),  P_0 = atan2(l, R0),  P_2 = r0^2 P_0 + R0 l,
//   P_3 = (R0 l S + R0 c^2 a)/2 + r0^2 R0 a + r0^2 (r0 P_-1),  a = asinh(l/c),
//   P_4 = r0^4 P_0 + 2 r0^2 R0 l + R0^3 l + R0 l^3/3,
//   P_5 = R0 l (S^3/4 + 3 c^2 S/8) + 3 R0 c^4 a/8 + r0^2 P_3.
// The M4 piece radii s = 1, 2 split the edge at l_k = sqrt(k^2 - c^2).
#include <cmath>

#include "em_internal.h"
#include "em_boundary.h"
#include "em_fmath.h"
#include "em_wave.h"

namespace em {

namespace {

__device__ __forceinline__ double f_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float f_log1p(float x) { return log1p_f32(x); }  // x >= 0 in the edge terms
__device__ __forceinline__ double f_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float f_atan2(float y, float x) { return atan2_f32(y, x); }  // y >= 0 in the edge terms
__device__ __forceinline__ double f_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float f_sqrt(float x) { return sqrt_f32(x); }
__device__ __forceinline__ double f_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float f_rcp(float x) { return rcp_f32(x); }

// Work counters of one thread (feed the algorithmic flop model).
struct Work {
    unsigned faces = 0, edges = 0, eterms = 0, moments = 0, quads = 0, angles = 0, qpoints = 0;
};

// pi * H(r0) = pi * r0 * G_c(r0)
template <typename R>
__device__ __forceinline__ R pi_H(R r0)
{
    if (r0 <= R(1)) {
        R r2 = r0 * r0;
        R r3 = r2 * r0;
        return R(0.35) * r0 - R(0.25) - r3 * R(1.0 / 6.0) + R(0.075) * r3 * r2 - R(0.025) * r3 * r3;
    }
    R u = R(2) - r0;
    R u2 = u * u;
    return -(u2 * u2 * u) * (r0 + R(1)) * R(1.0 / 120.0);
}

// pi r0 (G_shell - G_inner)(r0) = (r0 - 1)^5 (2 r0 + 1) / 60 (zero for r0 >= 1, where G_c is the shell polynomial)
template <typename R>
__device__ __forceinline__ R pi_dH(R r0)
{
    if (!(r0 < R(1))) return R(0);
    R u = r0 - R(1);
    R u2 = u * u;
    return u2 * u2 * u * (R(2) * r0 + R(1)) * R(1.0 / 60.0);
}

// angle atan(b/R0) - atan(a/R0) subtended at the foot point by the part [a, b] of the edge line
template <typename R>
__device__ __forceinline__ R seg_angle(R R0, R a, R b, Work &wk)
{
    wk.angles++;
    return f_atan2(R0 * (b - a), R0 * R0 + a * b);
}

// Transcendentals of the closed form at x >= 0 with S = sqrt(c^2 + x^2):
//   a = asinh(x/c), beta = P_0 - r0 P_-1 = atan(x/R0) - atan(r0 x/(R0 S)).
template <typename R>
struct Trans {
    R x, S, a, beta;
};

template <typename R>
__device__ __forceinline__ Trans<R> trans(R r0, R R0, R c2, R c, R x, R S, Work &wk)
{
    wk.moments++;
    Trans<R> t;
    t.x = x;
    t.S = S;
    t.a = f_log1p(x * (R(1) + x * f_rcp(S + c)) * f_rcp(c));
    const R R02 = R0 * R0;
    t.beta = f_atan2(x * R0 * (R02 + x * x), (S + r0) * (R02 * S + r0 * x * x));
    return t;
}

// Closed form of pi r0 int_0^alpha(x) [G_p(S) - G_p(r0)] dalpha for the piece
// polynomial pi G_p = g_-1/s + g_0 + g_2 s^2 + g_3 s^3 + g_4 s^4 + g_5 s^5:
//   -beta H_odd + r0 R0 T,  H_odd = g_-1 + g_3 r0^4 + g_5 r0^6,
//   T = g_2 x + g_3 P3' + g_4 (2 r0^2 x + R0^2 x + x^3/3)
//       + g_5 (x (S^3/4 + 3 c^2 S/8) + 3 c^4 a/8 + r0^2 P3'),
//   P3' = (x S + c^2 a)/2 + r0^2 a.
template <typename R>
__device__ __forceinline__ R core(const Trans<R> &t, R r0, R R0, R A, R c2, R gm1, R g2, R g3, R g4, R g5)
{
    const R x = t.x, S = t.S, a = t.a;
    const R Hodd = gm1 + g3 * A * A + g5 * A * A * A;
    const R P3r = R(0.5) * (x * S + c2 * a) + A * a;
    const R T = g2 * x + g3 * P3r + g4 * (R(2) * A * x + R0 * R0 * x + x * x * x * R(1.0 / 3.0)) +
                g5 * (x * (S * S * S * R(0.25) + R(0.375) * c2 * S) + R(0.375) * c2 * c2 * a + A * P3r);
    return -t.beta * Hodd + r0 * R0 * T;
}

template <typename R>
__device__ __forceinline__ R core_inner(const Trans<R> &t, R r0, R R0, R A, R c2)
{
    return core<R>(t, r0, R0, A, c2, R(-0.25), R(-1.0 / 6.0), R(0), R(0.075), R(-0.025));
}

template <typename R>
__device__ __forceinline__ R core_shell(const Trans<R> &t, R r0, R R0, R A, R c2)
{
    return core<R>(t, r0, R0, A, c2, R(-4.0 / 15.0), R(-1.0 / 3.0), R(0.25), R(-0.075), R(1.0 / 120.0));
}

__constant__ float kGLx[4] = {0.1834346424956498f, 0.5255324099163290f, 0.7966664774136267f, 0.9602898564975363f};
__constant__ float kGLw[4] = {0.3626837833783620f, 0.3137066458778873f, 0.2223810344533745f, 0.1012285362903763f};

__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

// shell piece by Gauss-Legendre:  pi r0 R0 int_a^b D_shell(R0^2 + l^2) dl,  a < b.
// 8 points per sub-interval, sub-intervals at most 0.8 dsing long (dsing: a
// lower bound of the distance from the part to the integrand's branch points
// l = +-ic), so the branch points stay outside the Bernstein ellipse of
// parameter 2.5 + sqrt(7.25) of every sub-interval and the truncation is far
// below the FP32 rounding of the term.
__device__ __forceinline__ float shell_quad(float r0, float R0, float c2, float dsing, float a, float b, Work &wk)
{
    const float V = 2.0f - r0;
    const float V2 = V * V, V4 = V2 * V2, V5 = V4 * V;
    const float rp1 = r0 + 1.0f;
    const float len = b - a;
    int nsub = (int)ceilf(len * rcp32(0.8f * dsing));
    nsub = nsub < 1 ? 1 : (nsub > 8 ? 8 : nsub);
    const float hl = 0.5f * len * rcp_f32((float)nsub);
    float tot = 0.0f;
    for (int k = 0; k < nsub; k++) {
        const float mid = a + (2.0f * (float)k + 1.0f) * hl;
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const float xq = (q & 1) ? -kGLx[q >> 1] : kGLx[q >> 1];
            const float l = mid + hl * xq;
            const float S = sqrt_f32(c2 + l * l);
            const float U = 2.0f - S;
            const float U2 = U * U;
            const float Sig = (((U + V) * U + V2) * U + V2 * V) * U + V4;
            const float num = rp1 * (r0 * Sig + V5) - r0 * U2 * U2 * U;
            acc += kGLw[q >> 1] * num * rcp32(S * (S + r0));
        }
        tot += acc * hl;
    }
    wk.quads += nsub;
    wk.qpoints += 8 * nsub;
    return tot * R0 * (1.0f / 120.0f);
}

__device__ __forceinline__ float shell_quad_t(float r0, float R0, float c2, float dsing, float a, float b, Work &wk)
{
    return shell_quad(r0, R0, c2, dsing, a, b, wk);
}

__device__ __forceinline__ double shell_quad_t(double, double, double, double, double, double, Work &)
{
    return 0.0;
}

// pi [Qt(l_b) - Qt(l_a)] for one directed edge (R0 > 0), lengths in units of h:
// the edge's whole share of pi int (G_c(S) - G_c(r0)) dalpha.  The signed edge
// interval is cut at the support crossings +-l2 and (when c < 1) the inner
// crossings +-l1 into parts beyond the support (-H times their angle), shell
// parts and an inner part (closed forms at their endpoints, odd in l; the
// FP32 path integrates shell parts by quadrature instead), plus the piece
// correction dH times the angle of the shell parts when r0 < 1.
//
// All cases are expressed as one fixed list of tasks - up to 4 angles, 3
// closed-form points (|l_a|, |l_b| clamped, and l1; each point serves both
// piece polynomials with its own weights) and 2 quadrature intervals - so that
// the lanes of a wavefront, which hold different particles, run each task
// type in the same code instead of one branch per geometric case.
template <typename R>
__device__ __forceinline__ R sgnr(R x)
{
    return x > R(0) ? R(1) : (x < R(0) ? R(-1) : R(0));
}

template <typename R>
__device__ __forceinline__ R edge_term(R r0, R R0, R la, R lb, R Ht, R dH, Work &wk)
{
    constexpr bool kQuad = std::is_same<R, float>::value;
    const R A = r0 * r0;
    const R c2 = A + R0 * R0;
    // angle tasks: (a, b, weight)
    R aa0 = la, ab0 = lb, aw0 = R(0), aa1 = R(0), ab1 = R(0), aw1 = R(0);
    R aa2 = R(0), ab2 = R(0), aw2 = R(0), aa3 = R(0), ab3 = R(0), aw3 = R(0);
    // closed-form point weights (inner, shell) at |ca|, |cb| and l1
    R wi0 = R(0), wi1 = R(0), wi2 = R(0), ws0 = R(0), ws1 = R(0), ws2 = R(0);
    // quadrature intervals
    R qa0 = R(0), qb0 = R(0), qa1 = R(0), qb1 = R(0);
    bool q0 = false, q1 = false;
    R l2 = R(0), c = R(1), l1 = R(0), ca = la, cb = lb;
    if (!(c2 < R(4))) {
        aw0 = -Ht;  // the whole edge lies beyond the support
    } else {
        wk.eterms++;
        l2 = f_sqrt(R(4) - c2);
        c = f_sqrt(c2);
        ca = fmin(fmax(la, -l2), l2);
        cb = fmin(fmax(lb, -l2), l2);
        if (la < -l2) {
            aw0 = -Ht;
            ab0 = fmin(lb, -l2);
        }
        if (lb > l2) {
            aa1 = fmax(la, l2);
            ab1 = lb;
            aw1 = -Ht;
        }
        if (c2 >= R(1)) {
            if (cb > ca) {
                if (kQuad) {
                    q0 = true;
                    qa0 = ca;
                    qb0 = cb;
                } else {
                    ws1 += sgnr(cb);
                    ws0 -= sgnr(ca);
                }
                aa2 = ca;
                ab2 = cb;
                aw2 = dH;
            }
        } else {
            l1 = f_sqrt(R(1) - c2);
            // left shell part [max(ca, -l2), min(cb, -l1)]
            if (ca < -l1) {
                const R B = fmin(cb, -l1);
                if (kQuad) {
                    q0 = true;
                    qa0 = ca;
                    qb0 = B;
                } else {
                    ws0 -= sgnr(ca);
                    if (B == cb) ws1 += sgnr(cb);
                    else ws2 -= R(1);  // B = -l1
                }
                aa2 = ca;
                ab2 = B;
                aw2 = dH;
            }
            // right shell part [max(ca, l1), min(cb, l2)]
            if (cb > l1) {
                const R Aq = fmax(ca, l1);
                if (kQuad) {
                    q1 = true;
                    qa1 = Aq;
                    qb1 = cb;
                } else {
                    ws1 += sgnr(cb);
                    if (Aq == ca) ws0 -= sgnr(ca);
                    else ws2 -= R(1);  // A = +l1
                }
                aa3 = Aq;
                ab3 = cb;
                aw3 = dH;
            }
            // inner part [max(ca, -l1), min(cb, l1)]
            const R Ai = fmax(ca, -l1), Bi = fmin(cb, l1);
            if (Bi > Ai) {
                if (Bi == cb) wi1 += sgnr(cb);
                else wi2 += R(1);  // B = +l1
                if (Ai == ca) wi0 -= sgnr(ca);
                else wi2 += R(1);  // A = -l1: -sgn(A) core(l1) = +core(l1)
            }
        }
    }
    R tot = R(0);
    if (aw0 != R(0)) tot += aw0 * seg_angle<R>(R0, aa0, ab0, wk);
    if (aw1 != R(0)) tot += aw1 * seg_angle<R>(R0, aa1, ab1, wk);
    if (aw2 != R(0)) tot += aw2 * seg_angle<R>(R0, aa2, ab2, wk);
    if (aw3 != R(0)) tot += aw3 * seg_angle<R>(R0, aa3, ab3, wk);
    const R x0 = fabs(ca), x1 = fabs(cb);
    if ((wi0 != R(0) || ws0 != R(0)) && x0 > R(0)) {
        const Trans<R> t = trans<R>(r0, R0, c2, c, x0, x0 == l2 ? R(2) : f_sqrt(c2 + x0 * x0), wk);
        tot += wi0 * core_inner<R>(t, r0, R0, A, c2) + ws0 * core_shell<R>(t, r0, R0, A, c2);
    }
    if ((wi1 != R(0) || ws1 != R(0)) && x1 > R(0)) {
        const Trans<R> t = trans<R>(r0, R0, c2, c, x1, x1 == l2 ? R(2) : f_sqrt(c2 + x1 * x1), wk);
        tot += wi1 * core_inner<R>(t, r0, R0, A, c2) + ws1 * core_shell<R>(t, r0, R0, A, c2);
    }
    if (wi2 != R(0) || ws2 != R(0)) {
        const Trans<R> t = trans<R>(r0, R0, c2, c, l1, R(1), wk);
        tot += wi2 * core_inner<R>(t, r0, R0, A, c2) + ws2 * core_shell<R>(t, r0, R0, A, c2);
    }
    if (kQuad) {
        if (q0) tot += shell_quad_t(r0, R0, c2, c2 >= R(1) ? c : R(1), qa0, qb0, wk);
        if (q1) tot += shell_quad_t(r0, R0, c2, R(1), qa1, qb1, wk);
    }
    return tot;
}

constexpr double kInvPi = 0.318309886183790671537767526745;
constexpr float kInvPiF = 0.318309886183790671537767526745f;

// Error estimate of the FP32 terms of a pair in the mixed path: each term
// (an angle times its weight, an inner-part closed form, a Gauss-Legendre
// sub-interval) is taken to carry a relative error of up to 16 units of FP32
// rounding (a few for the inputs rounded from FP64, up to 5 for each
// transcendental, the rest for the arithmetic and the truncation of the
// sub-interval rule), the errors of different terms adding like a random walk:
// err = 16 * 2^-24 * sqrt(sum of squared terms) / pi, in units of f.
constexpr float kTermErr = 16.0f * 5.9604644775390625e-08f;

// Conditioning test of one edge in the mixed path: true for near-degenerate
// triangles that FP32 cannot resolve: the projection point within FP32
// rounding of the edge line, or the wall plane, the edge line's closest
// point or the edge itself within FP32 rounding of a piece radius (s = 1, 2)
// of the kernel, where the FP32 piece assignment is not reliable; also the
// particle within 2^-30 h of the edge line (c^2 < 2^-60), which keeps the FP32
// square roots and reciprocals away from denormal arguments.
__device__ __forceinline__ bool needs_fp64(double r0, double R0, double c2)
{
    const double e = 9.5367431640625e-07;  // 2^-20
    return (R0 * R0 < e * e * c2) || (c2 < 8.673617379884035e-19) || (fabs(r0 - 1.0) < e) ||
           (fabs(c2 - 1.0) < e) || (fabs(c2 - 4.0) < 4.0 * e);
}

// The same test on the FP32 values the terms use (r0, R0 rounded from FP64;
// the FP32 rounding of c^2 is 2^-24 relative, far inside the 2^-20 margins).
__device__ __forceinline__ bool needs_fp64_f32(float r0, float R0, float c2)
{
    const float e = 9.5367431640625e-07f;  // 2^-20
    return (R0 * R0 < 9.094947017729282e-13f * c2) || (c2 < 8.673617379884035e-19f) || (fabsf(r0 - 1.0f) < e) ||
           (fabsf(c2 - 1.0f) < e) || (fabsf(c2 - 4.0f) < 4.0f * e);
}

// Raw f for one pair.  PREC = MAP_FP64 or MAP_MIXED.  Wall distance, foot
// point and edge projections are always FP64; in the mixed path the edge
// terms are FP32 (accumulated in FP64) unless the conditioning test sends the
// edge to the FP64 fixup pass.
template <int PREC>
__device__ __forceinline__ double pair_fraction(double px, double py, double pz, double h, int64_t cell,
                                                const int64_t *__restrict__ cfo, const int64_t *__restrict__ fvo,
                                                const double *__restrict__ plane, const EdgeRec *__restrict__ edges,
                                                Work &wk, uint64_t pair_k, unsigned *fix_count, uint64_t *fix_items,
                                                unsigned fix_cap, float &ev)
{
    using R = typename std::conditional<PREC == MAP_FP64, double, float>::type;
    const double invh = 1.0 / h;
    bool inside = true;
    int n_on = 0;
    double acc = 0.0;
    const int64_t f0 = cfo[cell], f1 = cfo[cell + 1];
    for (int64_t j = f0; j < f1; j++) {
        const double nx = plane[4 * j], ny = plane[4 * j + 1], nz = plane[4 * j + 2], cj = plane[4 * j + 3];
        const double d = cj - (nx * px + ny * py + nz * pz);
        wk.faces++;
        const bool in_j = d >= 0.0;
        inside = inside && in_j;
        n_on += d == 0.0 ? 1 : 0;
        const double r0d = fabs(d) * invh;
        if (!(r0d < 2.0)) continue;
        const R r0 = (R)r0d;
        const R Ht = pi_H<R>(r0);
        const R dH = pi_dH<R>(r0);
        double face = 0.0;
        const int64_t s0 = fvo[j], s1 = fvo[j + 1];
        for (int64_t s = s0; s < s1; s++) {
            const EdgeRec E = edges[s];
            const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
            const double rho = E.mx * wx + E.my * wy + E.mz * wz;
            wk.edges++;
            if (rho == 0.0) continue;
            const double la = -(E.ex * wx + E.ey * wy + E.ez * wz) * invh;
            const double lb = la + E.L * invh;
            const double R0d = fabs(rho) * invh;
            if (PREC == MAP_MIXED && needs_fp64(r0d, R0d, r0d * r0d + R0d * R0d)) {
                const unsigned slot = atomicAdd(fix_count, 1u);
                if (slot < fix_cap) fix_items[slot] = (pair_k << 32) | (uint64_t)(uint32_t)s;
                continue;
            }
            const R t = edge_term<R>(r0, (R)R0d, (R)la, (R)lb, Ht, dH, wk);
            face += (rho > 0.0) ? (double)t : -(double)t;
            if (PREC == MAP_MIXED) ev = fmaf((float)t, (float)t, ev);
        }
        acc += in_j ? face : -face;
    }
    return winding_term(inside, n_on, px, py, pz, cell, cfo, fvo, plane, edges) - acc * kInvPi;
}

// FP64 contribution of one edge to f (the fixup pass): the same terms as one
// iteration of the FP64 edge loop, with its wall's sign.
__device__ double edge_contribution_fp64(double px, double py, double pz, double h, const double *pl,
                                         const EdgeRec &E)
{
    Work wk;
    const double invh = 1.0 / h;
    const double d = pl[3] - (pl[0] * px + pl[1] * py + pl[2] * pz);
    const double r0 = fabs(d) * invh;
    if (!(r0 < 2.0)) return 0.0;
    const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
    const double rho = E.mx * wx + E.my * wy + E.mz * wz;
    if (rho == 0.0) return 0.0;
    const double la = -(E.ex * wx + E.ey * wy + E.ez * wz) * invh;
    const double lb = la + E.L * invh;
    const double t = edge_term<double>(r0, fabs(rho) * invh, la, lb, pi_H<double>(r0), pi_dH<double>(r0), wk);
    const double face = (rho > 0.0) ? t : -t;
    return -(d >= 0.0 ? face : -face) * kInvPi;
}

// wave sums of the work counters, one atomic per counter per wave
__device__ __forceinline__ void flush_work(const Work &wk, unsigned long long *counters)
{
    unsigned long long v[7] = {wk.eterms, wk.faces, wk.edges, wk.moments, wk.quads, wk.angles, wk.qpoints};
#pragma unroll
    for (int q = 0; q < 7; q++)
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(counters + C_EDGE_TERMS, v[0]);
        atomicAdd(counters + C_FACES, v[1]);
        atomicAdd(counters + C_EDGES, v[2]);
        atomicAdd(counters + C_MOMENTS, v[3]);
        atomicAdd(counters + C_QUADS, v[4]);
        atomicAdd(counters + C_ANGLES, v[5]);
        atomicAdd(counters + C_QPOINTS, v[6]);
    }
}

struct FixList {
    unsigned *count;
    uint64_t *items;
    unsigned cap;
    float *err;  // mixed path: per-pair FP32 error estimates (or null)
};

// Appends the fixup item (pair k, slot) when the list has room; the count
// keeps growing past the capacity, which tells the host that items were lost.
__device__ __forceinline__ void push_fix(const FixList &fx, int64_t k, uint32_t slot)
{
    const unsigned i = atomicAdd(fx.count, 1u);
    if (i < fx.cap) fx.items[i] = ((uint64_t)k << 32) | (uint64_t)slot;
}

template <int PREC>
__device__ __forceinline__ double one_pair(int64_t k, const uint32_t *__restrict__ pair_p,
                                           const uint32_t *__restrict__ pair_c, const double *__restrict__ xyz,
                                           const double *__restrict__ h, const int64_t *__restrict__ cfo,
                                           const int64_t *__restrict__ fvo, const double *__restrict__ plane,
                                           const EdgeRec *__restrict__ edges, Work &wk, const FixList &fx)
{
    const int64_t a = pair_p[k];
    const int64_t c = pair_c[k];
    float ev = 0.0f;
    const double v = pair_fraction<PREC>(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], h[a], c, cfo, fvo, plane, edges,
                                         wk, (uint64_t)k, fx.count, fx.items, fx.cap, ev);
    if (PREC == MAP_MIXED && fx.err) fx.err[k] = kTermErr * kInvPiF * sqrt_f32(ev);
    return v;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_integrate_flat(int64_t np, const uint32_t *__restrict__ pair_p,
                                                         const uint32_t *__restrict__ pair_c,
                                                         const double *__restrict__ xyz, const double *__restrict__ h,
                                                         const int64_t *__restrict__ cfo,
                                                         const int64_t *__restrict__ fvo,
                                                         const double *__restrict__ plane,
                                                         const EdgeRec *__restrict__ edges, double *__restrict__ f,
                                                         unsigned long long *counters, FixList fx)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Work wk;
    if (k < np) f[k] = one_pair<PREC>(k, pair_p, pair_c, xyz, h, cfo, fvo, plane, edges, wk, fx);
    flush_work(wk, counters);
}

// Persistent form: each wavefront takes tiles of 64*tile_waves consecutive
// (cell-ordered) pairs from a queue until the pairs run out.
template <int PREC, int WPE>
__global__ void __launch_bounds__(256, WPE) k_integrate_persistent(int64_t np, const uint32_t *__restrict__ pair_p,
                                                               const uint32_t *__restrict__ pair_c,
                                                               const double *__restrict__ xyz,
                                                               const double *__restrict__ h,
                                                               const int64_t *__restrict__ cfo,
                                                               const int64_t *__restrict__ fvo,
                                                               const double *__restrict__ plane,
                                                               const EdgeRec *__restrict__ edges,
                                                               double *__restrict__ f, unsigned long long *counters,
                                                               unsigned *tile_ctr, int tile_waves, FixList fx)
{
    const int lane = threadIdx.x & 63;
    const int64_t tile = 64 * (int64_t)tile_waves;
    const int64_t ntiles = (np + tile - 1) / tile;
    Work wk;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(tile_ctr, 1u);
        t = __shfl(t, 0, 64);
        if ((int64_t)t >= ntiles) break;
        const int64_t base = (int64_t)t * tile;
        for (int w = 0; w < tile_waves; w++) {
            const int64_t k = base + 64 * w + lane;
            if (k < np) f[k] = one_pair<PREC>(k, pair_p, pair_c, xyz, h, cfo, fvo, plane, edges, wk, fx);
        }
    }
    flush_work(wk, counters);
}

// Next tile of a persistent kernel in XCD-aware order, or -1 when none is
// left.  Workgroups are dispatched round-robin over the 8 XCDs, so workgroup
// b runs on XCD b mod 8; each XCD first takes the tiles of its own eighth of
// the (cell-ordered) pair list from its own counter ctr[x], so the tiles that
// share a cell's wall and edge records meet in one L2, then takes what is
// left in the other eighths.  `probe` (0 at the start) persists between
// calls.  Wave-uniform.  A pair's result does not depend on the wavefront
// that computes it.
__device__ __forceinline__ int64_t next_tile_xcd(unsigned *ctr, int64_t ntiles, int &probe, int lane)
{
    const int xcd = (int)(blockIdx.x & 7);
    const int64_t chunk = (ntiles + 7) / 8;
    while (probe < 8) {
        const int y = (xcd + probe) & 7;
        const int64_t lo = (int64_t)y * chunk;
        const int64_t hi = lo + chunk < ntiles ? lo + chunk : ntiles;
        if (lo < hi) {
            unsigned v = 0;
            if (lane == 0) v = atomicAdd(ctr + y, 1u);
            v = __builtin_amdgcn_readfirstlane(v);
            if (lo + (int64_t)v < hi) return lo + (int64_t)v;
        }
        probe++;
    }
    return -1;
}

// ---------------------------------------------------------------- queued tasks (mixed path)
// The edge terms split into independent tasks of three kinds: angles (one
// atan2), closed-form points (one trans + core) and shell quadrature
// sub-intervals (4 Gauss-Legendre points each, see run_quad).  In a wavefront of 64 pairs most
// lanes need only a few of the possible tasks at a given edge, so running
// every kind whenever any lane needs it leaves most lanes idle.  Here each
// lane classifies its edge and pushes its tasks, with their weights and the
// edge's sign, onto per-wavefront stacks in LDS; a stack holding 64 tasks is
// run by the whole wavefront at once, and every result is added to its
// pair's FP64 accumulator (LDS).  Lanes walk their cell's wall slots with one
// wave-uniform counter, so the pushes and runs are in uniform control flow.
constexpr int kQ = 128;  // stack capacity: below 64 pending before a push of at most 64

constexpr int kQA = 64;  // angle stack capacity: run before a push that would overflow it
struct WaveStacks {
    float ang[3][kQA];  // atan2 arguments of the angle (imaginary, real part), weight
    float pnt[4][kQ];   // inner parts: r0, signed R0 (sign = the term's sign), start a, length L
    float qd[4][kQ];    // shell sub-intervals: r0, signed R0, mid, half-length
    uint8_t ang_o[kQA], pnt_o[kQ], qd_o[kQ];  // owner lanes
    double acc[64];
    float ev[64];  // sums of the squared FP32 task values per owner (error estimate)
};

__device__ __forceinline__ void run_angle(WaveStacks &W, int i, Work &wk)
{
    wk.angles++;
    const float v = W.ang[2][i] * atan2_f32(W.ang[0][i], W.ang[1][i]);
    atomicAdd(&W.acc[W.ang_o[i]], (double)v);
    atomicAdd(&W.ev[W.ang_o[i]], v * v);
}

// Closed form of the inner piece (s <= 1) over one edge part [a, a + L],
// a >= -l1, a + L <= l1: the integral along it of pi r0 [G_inner(S) -
// G_inner(r0)] dalpha, that is the difference of the antiderivative
//     -beta H_odd + r0 R0 T
// (see core) between the part's ends, written so that every difference
// between the ends carries the factor L explicitly instead of subtracting
// two nearly equal end values (a part much shorter than h would lose most of
// its digits in FP32 otherwise):
//   beta_b - beta_a      = 2 atan2(R0 L, S_a S_b + a b + c^2 + r0 (S_a + S_b))
//                          (the solid angle of the triangle foot-v_a-v_b);
//   asinh(b/c) - asinh(a/c) = asinh(L (c^2 + S_a S_b - a b) / (c^2 (S_a + S_b)));
//   b S_b - a S_a         = L (S_b + a (a + b) / (S_a + S_b));
//   b S_b^3 - a S_a^3     = L (S_b^3 + a (a + b) (S_a^2 + S_a S_b + S_b^2) / (S_a + S_b));
//   b^3 - a^3             = L (a^2 + a b + b^2);
// S_a S_b +- a b is formed from (S_a S_b)^2 - (a b)^2 = c^2 (a^2 + b^2 + c^2)
// on the side where it would cancel.  L comes from the FP64 edge length when
// the part is the whole edge.
__device__ __forceinline__ void run_seg(WaveStacks &W, int i, Work &wk)
{
    wk.moments++;
    const float r0 = W.pnt[0][i], sR0 = W.pnt[1][i], a = W.pnt[2][i], L = W.pnt[3][i];
    const float R0 = fabsf(sR0), w = sR0 < 0.0f ? -1.0f : 1.0f;
    const float b = a + L;
    const float A = r0 * r0, R02 = R0 * R0, c2 = fmaf(R0, R0, A);
    const float Sa = sqrt_f32(fmaf(a, a, c2)), Sb = sqrt_f32(fmaf(b, b, c2));
    const float ab = a * b, SS = Sa * Sb, Ssum = Sa + Sb;
    const float q = c2 * (fmaf(a, a, fmaf(b, b, c2)));  // (S_a S_b)^2 - (a b)^2
    float sp, sm;                                       // S_a S_b + a b, S_a S_b - a b
    if (ab > 0.0f) {
        sp = SS + ab;
        sm = q * rcp_f32(sp);
    } else {
        sm = SS - ab;
        sp = q * rcp_f32(sm);
    }
    const float rs = rcp_f32(Ssum);
    const float Dbeta = 2.0f * atan2_f32(R0 * L, fmaf(r0, Ssum, sp + c2));
    const float Z = L * (c2 + sm) * rcp_f32(c2 * Ssum);
    const float Da = log1p_f32(fmaf(Z * Z, rcp_f32(1.0f + sqrt_f32(fmaf(Z, Z, 1.0f))), Z));
    const float t = a * (a + b) * rs;
    const float DxS = L * (Sb + t);
    const float DxS3 = L * fmaf(t, Sb * Sb + SS + Sa * Sa, Sb * Sb * Sb);
    const float D3 = L * (fmaf(a, a, ab) + b * b);
    // inner piece: g_-1 = -1/4, g_2 = -1/6, g_3 = 0, g_4 = 3/40, g_5 = -1/40
    const float Hodd = -0.25f - 0.025f * A * A * A;
    const float DP3r = 0.5f * fmaf(c2, Da, DxS) + A * Da;
    const float DT = (-1.0f / 6.0f) * L + 0.075f * fmaf(2.0f * A + R02, L, D3 * (1.0f / 3.0f)) -
                     0.025f * (0.25f * DxS3 + 0.375f * c2 * fmaf(c2, Da, DxS) + A * DP3r);
    const float v = w * fmaf(-Dbeta, Hodd, r0 * R0 * DT);
    atomicAdd(&W.acc[W.pnt_o[i]], (double)v);
    atomicAdd(&W.ev[W.pnt_o[i]], v * v);
}

// 4-point Gauss-Legendre nodes and weights on [-1, 1] (nodes in pairs +-x)
__constant__ float kGL4x[2] = {0.3399810435848563f, 0.8611363115940526f};
__constant__ float kGL4w[2] = {0.6521451548625461f, 0.3478548451374538f};

// One sub-interval of the shell integrand (the integrand of shell_quad) by
// 4-point Gauss-Legendre.  Sub-intervals are at most 0.4 times the distance
// to the integrand's branch points l = +-ic long (and at most 2 - r0), so
// the branch points lie outside the Bernstein ellipse of parameter
// 5 + sqrt(26) of every sub-interval; the Gauss-Legendre error theorem for
// analytic integrands then bounds the truncation by 1e-8 of the pair fraction
// per sub-interval over the whole (r0, c) range (measured: below 3e-10).
__device__ __forceinline__ void run_quad(WaveStacks &W, int i, Work &wk)
{
    const float r0 = W.qd[0][i], sR0 = W.qd[1][i], mid = W.qd[2][i], hl = W.qd[3][i];
    const float c2 = fmaf(sR0, sR0, r0 * r0), w = sR0 * hl * (1.0f / 120.0f);
    // the numerator (r0+1)(r0 Sigma + V^5) - r0 U^5 as a polynomial in U with
    // coefficients a0..a5 (a1..a4 = (r0+1) r0 V^(4-k), a0 = (r0+1)(V^5 + r0 V^4), a5 = -r0)
    const float V = 2.0f - r0;
    const float V2 = V * V, V3 = V2 * V, V4 = V2 * V2;
    const float t = (r0 + 1.0f) * r0;
    const float a0 = (r0 + 1.0f) * fmaf(r0, V4, V4 * V), a1 = t * V3, a2 = t * V2, a3 = t * V;
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const float xq = (q & 1) ? -kGL4x[q >> 1] : kGL4x[q >> 1];
        const float l = fmaf(hl, xq, mid);
        const float S = sqrt_f32(fmaf(l, l, c2));
        const float U = 2.0f - S;
        const float num = fmaf(fmaf(fmaf(fmaf(fmaf(-r0, U, t), U, a3), U, a2), U, a1), U, a0);
        acc = fmaf(kGL4w[q >> 1], num * rcp_f32(S * (S + r0)), acc);
    }
    wk.quads++;
    wk.qpoints += 4;
    const float v = w * acc;
    atomicAdd(&W.acc[W.qd_o[i]], (double)v);
    atomicAdd(&W.ev[W.qd_o[i]], v * v);
}

template <int KIND>
__device__ __forceinline__ void run_one(WaveStacks &W, int i, Work &wk)
{
    if (KIND == 0) run_angle(W, i, wk);
    else if (KIND == 1) run_seg(W, i, wk);
    else run_quad(W, i, wk);
}

// run the top 64 entries when 64 are pending (all = false), or all pending ones
template <int KIND>
__device__ __forceinline__ void run_stack(WaveStacks &W, int &count, int lane, bool all, Work &wk)
{
    if (count >= 64) {
        lds_sync_wave();
        run_one<KIND>(W, count - 64 + lane, wk);
        count -= 64;
        lds_sync_wave();
    }
    if (all && count > 0) {
        lds_sync_wave();
        if (lane < count) run_one<KIND>(W, lane, wk);
        count = 0;
        lds_sync_wave();
    }
}

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// One step of the mixed task batches: this lane's edge (slot s of the current
// wall; live = the lane has a wall within the support and an edge at this
// step) is projected in FP64, classified in FP32 and its tasks are pushed;
// full stacks run as they fill.  Wave-uniform control flow; r0d, r0, Ht, dH
// and fsign describe the lane's current wall.
__device__ __forceinline__ void mixed_edge_step(WaveStacks &W, int lane, Work &wk, int &nA, int &nP, int &nQ, bool live,
                                                const EdgeRec *__restrict__ edges, int32_t s, double px, double py,
                                                double pz, double invh, double r0d, float r0, float Ht, float dH,
                                                float fsign, int64_t k, FixList fx, double &acc_in, float &ev_in)
{
    float R0 = 0.0f, la = 0.0f, lb = 0.0f, Le = 0.0f, sg = 0.0f;
    if (live) {
        const EdgeRec E = edges[s];
        const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
        const double rho = E.mx * wx + E.my * wy + E.mz * wz;
        wk.edges++;
        if (rho == 0.0) {
            live = false;
        } else {
            const double lad = -(E.ex * wx + E.ey * wy + E.ez * wz) * invh;
            const double Ld = E.L * invh;
            const float R0f = (float)(fabs(rho) * invh);
            if (needs_fp64_f32(r0, R0f, fmaf(r0, r0, R0f * R0f))) {
                const unsigned slot = atomicAdd(fx.count, 1u);
                if (slot < fx.cap) fx.items[slot] = ((uint64_t)k << 32) | (uint64_t)(uint32_t)s;
                live = false;
            } else {
                R0 = R0f;
                la = (float)lad;
                lb = (float)(lad + Ld);
                Le = (float)Ld;  // the edge's length from FP64: parts spanning the whole edge keep their digits
                sg = (rho > 0.0 ? 1.0f : -1.0f) * fsign;
            }
        }
    }
    // length of the part [x, y] of the edge: the FP64-derived length when it
    // is the whole edge, else the FP32 difference (a clipped end sits on a
    // kernel sphere, where an end shift changes the integral only to second order)
    auto part_len = [&](float x, float y) { return (x == la && y == lb) ? Le : y - x; };
    // classification (the mixed form of edge_term).  The edge [la, lb] splits
    // into the parts beyond the support (|l| > l2), the shell parts and the
    // inner part (|l| < l1, when c < 1): [la, ca] + [cb, lb] beyond,
    // [ca, ia] + [ib, cb] shell, [ia, ib] inner, every part oriented and
    // possibly empty.  Far edges (c >= 2) are all beyond (l2 = 0).
    const float A = r0 * r0;
    const float c2 = A + R0 * R0;
    const bool near = live && c2 < 4.0f;
    const bool has_inner = near && c2 < 1.0f;
    const float l2 = near ? sqrt_f32(4.0f - c2) : 0.0f;
    const float l1 = has_inner ? sqrt_f32(1.0f - c2) : 0.0f;
    const float c = near && !has_inner ? sqrt_f32(c2) : 1.0f;
    // clamps as medians of three (la <= lb, so min(max(x, lo), hi) is the
    // median of x, lo and hi also when lo > hi: one instruction each)
    const float ca = __builtin_amdgcn_fmed3f(la, -l2, lb);
    const float cb = __builtin_amdgcn_fmed3f(ca, l2, lb);
    const float ia = has_inner ? __builtin_amdgcn_fmed3f(ca, -l1, cb) : cb;
    const float ib = has_inner ? __builtin_amdgcn_fmed3f(ia, l1, cb) : cb;
    if (near) wk.eterms++;
    // angle terms: -H times the beyond parts' angle, dH times the shell
    // parts' angle.  The angle of two parts is the argument of the product of
    // their complex numbers (R0^2 + a b) + i R0 (b - a) (sum below pi).  One
    // angle per lane is taken here; a lane that has both pushes the shell
    // angle as a task.
    const bool has_b = live && (la < ca || cb < lb);
    const bool has_s = near && dH != 0.0f && (ca < ia || ib < cb);
    float zx, zy;
    {
        const float R02 = R0 * R0;
        const bool b = has_b;
        const float a1 = b ? la : ca, b1 = b ? ca : ia, a2 = b ? cb : ib, b2 = b ? lb : cb;
        const float x1 = R02 + a1 * b1, y1 = R0 * part_len(a1, b1), x2 = R02 + a2 * b2, y2 = R0 * part_len(a2, b2);
        zx = x1 * x2 - y1 * y2;
        zy = x1 * y2 + x2 * y1;
    }
    const float w_in = has_b ? -Ht * sg : (has_s ? dH * sg : 0.0f);
    {
        const float v = w_in * atan2_f32(zy, zx);
        acc_in += (double)v;
        ev_in = fmaf(v, v, ev_in);
    }
    wk.angles += (has_b || has_s) ? 1u : 0u;
    {
        const bool want = has_b && has_s;
        const unsigned long long m = __ballot(want);
        if (m != 0) {
            if (nA + __popcll(m) > kQA) run_stack<0>(W, nA, lane, true, wk);
            const int slot = wave_push(want, nA);
            if (want) {
                const float R02 = R0 * R0;
                const float x1 = R02 + ca * ia, y1 = R0 * part_len(ca, ia), x2 = R02 + ib * cb, y2 = R0 * part_len(ib, cb);
                W.ang[0][slot] = x1 * y2 + x2 * y1;
                W.ang[1][slot] = x1 * x2 - y1 * y2;
                W.ang[2][slot] = dH * sg;
                W.ang_o[slot] = (uint8_t)lane;
            }
            run_stack<0>(W, nA, lane, false, wk);
        }
    }
    // inner part [ia, ib]: one closed-form task over the part (run_seg)
    {
        const bool want = has_inner && ib > ia;
        if (__ballot(want) != 0) {
            const int slot = wave_push(want, nP);
            if (want) {
                W.pnt[0][slot] = r0;
                W.pnt[1][slot] = sg < 0.0f ? -R0 : R0;
                W.pnt[2][slot] = ia;
                W.pnt[3][slot] = part_len(ia, ib);
                W.pnt_o[slot] = (uint8_t)lane;
            }
            run_stack<1>(W, nP, lane, false, wk);
        }
    }
    // shell parts by quadrature: [ca, ia] and [ib, cb]
    const bool q0 = near && ia > ca, q1 = near && cb > ib;
    const float qa0 = ca, qb0 = ia, qa1 = ib, qb1 = cb, qd0 = has_inner ? 1.0f : c;
    // both shell parts' sub-intervals in one uniform loop
    int n0 = 0, n1 = 0;
    float hl0 = 0.0f, hl1 = 0.0f;
    // sub-intervals no longer than 0.4 times the distance to the branch points
    // l = +-ic of the integrand, nor than V = 2 - r0: the shell integrand is of
    // order V^4 on the edge, and a sub-interval longer than V would let the
    // polynomial in U = 2 - S grow far beyond that inside the ellipse of
    // analyticity that bounds the Gauss-Legendre error
    const float Vs = 2.0f - r0;
    if (q0) {
        const float len = part_len(qa0, qb0);
        n0 = min(max((int)ceilf(len * rcp_f32(fminf(0.4f * qd0, Vs))), 1), 32);
        hl0 = 0.5f * len * rcp_f32((float)n0);
    }
    if (q1) {
        const float len = part_len(qa1, qb1);
        n1 = min(max((int)ceilf(len * rcp_f32(fminf(0.4f, Vs))), 1), 32);
        hl1 = 0.5f * len * rcp_f32((float)n1);
    }
    const int nq = n0 + n1;
    for (int kk = 0; __ballot(kk < nq) != 0; kk++) {
        const bool want = kk < nq;
        const int slot = wave_push(want, nQ);
        if (want) {
            const bool first = kk < n0;
            const float hl = first ? hl0 : hl1;
            W.qd[0][slot] = r0;
            W.qd[1][slot] = sg < 0.0f ? -R0 : R0;
            W.qd[2][slot] = first ? qa0 + (2.0f * (float)kk + 1.0f) * hl0 : qa1 + (2.0f * (float)(kk - n0) + 1.0f) * hl1;
            W.qd[3][slot] = hl;
            W.qd_o[slot] = (uint8_t)lane;
        }
        run_stack<2>(W, nQ, lane, false, wk);
    }
}

// The job of global tile t of a launch of several jobs (wave-uniform): the
// last job whose first tile is at or before t.
__device__ __forceinline__ int job_of_tile(const JobsArg &A, int64_t t)
{
    int lo = 0, hi = A.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.table[mid].tile_base <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Field of the current job: the kernel argument itself for a one-job launch
// (kept in scalar registers as plain arguments would be), the device table
// entry otherwise.
#define JOB(field) (MULTI ? A.table[jj].field : A.one.field)

// Marker slot of a fixup item that asks for the winding weight of a pair whose
// particle lies on two or more of its cell's wall planes (an edge or a vertex
// of the cell; see em_boundary.h).
constexpr uint32_t kWindingSlot = 0xffffffffu;

template <int WPE, bool MULTI>
__global__ void __launch_bounds__(256, WPE) k_integrate_queued(JobsArg A, unsigned *tile_ctr)
{
    __shared__ WaveStacks stacks[4];
    const int lane = threadIdx.x & 63;
    WaveStacks &W = stacks[threadIdx.x >> 6];
    int probe = 0;
    int cur = MULTI ? -1 : 0;
    Work wk;
    for (;;) {
        const int64_t t = next_tile_xcd(tile_ctr + 16, A.n_tiles, probe, lane);
        if (t < 0) break;
        const int jj = MULTI ? job_of_tile(A, t) : 0;
        if (MULTI && jj != cur) {
            if (cur >= 0) flush_work(wk, A.table[cur].counters);
            wk = Work();
            cur = jj;
        }
        const FixList fx = {JOB(fix_count), JOB(fix_items), JOB(fix_cap), nullptr};
        const EdgeRec *__restrict__ edges = JOB(edges);
        const double *__restrict__ plane = JOB(plane);
        const int64_t *__restrict__ fvo = JOB(fvo);
        const int64_t k = (t - JOB(tile_base)) * 64 + lane;
        const bool active = k < JOB(np);
        double px = 0.0, py = 0.0, pz = 0.0, invh = 1.0;
        int32_t s = 0, s_end = 0, j = 0;
        if (active) {
            const int64_t a = JOB(pair_p)[k];
            const int64_t c = JOB(pair_c)[k];
            px = JOB(xyz)[3 * a];
            py = JOB(xyz)[3 * a + 1];
            pz = JOB(xyz)[3 * a + 2];
            invh = 1.0 / JOB(h)[a];
            const int64_t *__restrict__ cfo = JOB(cfo);
            j = (int32_t)cfo[c] - 1;
            s = (int32_t)fvo[cfo[c]];
            s_end = (int32_t)fvo[cfo[c + 1]];
        }
        W.acc[lane] = 0.0;
        W.ev[lane] = 0.0f;
        int32_t face_end = s;  // first slot past the current wall: the first step opens the cell's first wall
        const int n_steps = wave_max((int)(s_end - s));
        int nA = 0, nP = 0, nQ = 0;
        double acc_in = 0.0;  // this lane's terms taken in place (not as tasks)
        float ev_in = 0.0f;   // the sum of their squares
        bool inside = true;
        int n_on = 0;  // walls whose plane holds the particle
        bool face_ok = false;
        double r0d = 0.0;
        float r0 = 0.0f, Ht = 0.0f, dH = 0.0f, fsign = 1.0f;
        for (int it = 0; it < n_steps; it++, s++) {
            const bool valid = s < s_end;
            if (valid && s == face_end) {
                j++;
                face_end = (int32_t)fvo[j + 1];
                const double d = plane[4 * j + 3] - (plane[4 * j] * px + plane[4 * j + 1] * py + plane[4 * j + 2] * pz);
                wk.faces++;
                const bool in_j = d >= 0.0;
                inside = inside && in_j;
                n_on += d == 0.0 ? 1 : 0;
                fsign = in_j ? 1.0f : -1.0f;
                r0d = fabs(d) * invh;
                face_ok = r0d < 2.0;
                r0 = (float)r0d;
                Ht = pi_H<float>(r0);
                dH = pi_dH<float>(r0);
            }
            mixed_edge_step(W, lane, wk, nA, nP, nQ, valid && face_ok, edges, s, px, py, pz, invh, r0d, r0, Ht, dH,
                            fsign, k, fx, acc_in, ev_in);
        }
        run_stack<0>(W, nA, lane, true, wk);
        run_stack<1>(W, nP, lane, true, wk);
        run_stack<2>(W, nQ, lane, true, wk);
        lds_sync_wave();
        if (active) {
            JOB(f)[k] = (inside ? 1.0 : 0.0) - (W.acc[lane] + acc_in) * kInvPi;
            float *const err = JOB(err);  // null when no estimate is wanted (the autotuner's timing runs)
            if (err) err[k] = kTermErr * kInvPiF * sqrt_f32(ev_in + W.ev[lane]);
            if (inside && n_on >= 2) push_fix(fx, k, kWindingSlot);
        }
        lds_sync_wave();
    }
    if (cur >= 0) flush_work(wk, MULTI ? A.table[cur].counters : A.one.counters);
}

// FP64 form of the task batches: no quadrature (the shell piece keeps its
// closed form), so two task kinds: angles and closed-form points carrying
// both piece weights.
struct WaveStacks64 {
    double ang[4][kQ];  // R0, a, b, weight
    double pnt[8][kQ];  // r0, R0, c2, c, x, S, inner weight, shell weight
    double acc[64];
    uint8_t ang_o[kQ], pnt_o[kQ];  // owner lanes
};

template <int KIND>
__device__ __forceinline__ void run_one64(WaveStacks64 &W, int i, Work &wk)
{
    if (KIND == 0) {
        const double R0 = W.ang[0][i], a = W.ang[1][i], b = W.ang[2][i], w = W.ang[3][i];
        atomicAdd(&W.acc[W.ang_o[i]], w * seg_angle<double>(R0, a, b, wk));
    } else {
        const double r0 = W.pnt[0][i], R0 = W.pnt[1][i], c2 = W.pnt[2][i], c = W.pnt[3][i];
        const double x = W.pnt[4][i], S = W.pnt[5][i], wi = W.pnt[6][i], wsh = W.pnt[7][i];
        const Trans<double> t = trans<double>(r0, R0, c2, c, x, S, wk);
        const double A = r0 * r0;
        atomicAdd(&W.acc[W.pnt_o[i]], wi * core_inner<double>(t, r0, R0, A, c2) + wsh * core_shell<double>(t, r0, R0, A, c2));
    }
}

template <int KIND>
__device__ __forceinline__ void run_stack64(WaveStacks64 &W, int &count, int lane, bool all, Work &wk)
{
    if (count >= 64) {
        lds_sync_wave();
        run_one64<KIND>(W, count - 64 + lane, wk);
        count -= 64;
        lds_sync_wave();
    }
    if (all && count > 0) {
        lds_sync_wave();
        if (lane < count) run_one64<KIND>(W, lane, wk);
        count = 0;
        lds_sync_wave();
    }
}

// WPE: resident wavefronts per SIMD the register budget is cut for (2: no
// spills; 3: the LDS stacks of three workgroups fit a compute unit, at the
// price of a few spilled registers)
template <int WPE, bool MULTI>
__global__ void __launch_bounds__(256, WPE) k_integrate_queued64(JobsArg A, unsigned *tile_ctr)
{
    __shared__ WaveStacks64 stacks[4];
    const int lane = threadIdx.x & 63;
    WaveStacks64 &W = stacks[threadIdx.x >> 6];
    int probe = 0;
    int cur = MULTI ? -1 : 0;
    Work wk;
    for (;;) {
        const int64_t t = next_tile_xcd(tile_ctr + 16, A.n_tiles, probe, lane);
        if (t < 0) break;
        const int jj = MULTI ? job_of_tile(A, t) : 0;
        if (MULTI && jj != cur) {
            if (cur >= 0) flush_work(wk, A.table[cur].counters);
            wk = Work();
            cur = jj;
        }
        const EdgeRec *__restrict__ edges = JOB(edges);
        const double *__restrict__ plane = JOB(plane);
        const int64_t *__restrict__ fvo = JOB(fvo);
        const int64_t k = (t - JOB(tile_base)) * 64 + lane;
        const bool active = k < JOB(np);
        double px = 0.0, py = 0.0, pz = 0.0, invh = 1.0;
        int64_t s = 0, s_end = 0, j = 0;
        if (active) {
            const int64_t a = JOB(pair_p)[k];
            const int64_t c = JOB(pair_c)[k];
            px = JOB(xyz)[3 * a];
            py = JOB(xyz)[3 * a + 1];
            pz = JOB(xyz)[3 * a + 2];
            invh = 1.0 / JOB(h)[a];
            const int64_t *__restrict__ cfo = JOB(cfo);
            j = cfo[c] - 1;
            s = fvo[cfo[c]];
            s_end = fvo[cfo[c + 1]];
        }
        W.acc[lane] = 0.0;
        int64_t face_end = s;
        const int n_steps = wave_max((int)(s_end - s));
        int nA = 0, nP = 0;
        bool inside = true;
        int n_on = 0;  // walls whose plane holds the particle
        bool face_ok = false;
        double r0 = 0.0, Ht = 0.0, dH = 0.0, fsign = 1.0;
        for (int it = 0; it < n_steps; it++, s++) {
            const bool valid = s < s_end;
            if (valid && s == face_end) {
                j++;
                face_end = fvo[j + 1];
                const double d = plane[4 * j + 3] - (plane[4 * j] * px + plane[4 * j + 1] * py + plane[4 * j + 2] * pz);
                wk.faces++;
                const bool in_j = d >= 0.0;
                inside = inside && in_j;
                n_on += d == 0.0 ? 1 : 0;
                fsign = in_j ? 1.0 : -1.0;
                r0 = fabs(d) * invh;
                face_ok = r0 < 2.0;
                Ht = pi_H<double>(r0);
                dH = pi_dH<double>(r0);
            }
            bool live = valid && face_ok;
            double R0 = 0.0, la = 0.0, lb = 0.0, sg = 0.0;
            if (live) {
                const EdgeRec E = edges[s];
                const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
                const double rho = E.mx * wx + E.my * wy + E.mz * wz;
                wk.edges++;
                if (rho == 0.0) {
                    live = false;
                } else {
                    la = -(E.ex * wx + E.ey * wy + E.ez * wz) * invh;
                    lb = la + E.L * invh;
                    R0 = fabs(rho) * invh;
                    sg = (rho > 0.0 ? 1.0 : -1.0) * fsign;
                }
            }
            // classification (the FP64 form of edge_term)
            const double A = r0 * r0;
            const double c2 = A + R0 * R0;
            double aa[4] = {la, 0.0, 0.0, 0.0}, ab[4] = {lb, 0.0, 0.0, 0.0}, aw[4] = {0.0, 0.0, 0.0, 0.0};
            double wi[3] = {0.0, 0.0, 0.0}, wsh[3] = {0.0, 0.0, 0.0};
            double l2 = 0.0, c = 1.0, l1 = 0.0, ca = la, cb = lb;
            if (live) {
                if (!(c2 < 4.0)) {
                    aw[0] = -Ht;
                } else {
                    wk.eterms++;
                    l2 = sqrt(4.0 - c2);
                    c = sqrt(c2);
                    ca = fmin(fmax(la, -l2), l2);
                    cb = fmin(fmax(lb, -l2), l2);
                    if (la < -l2) {
                        aw[0] = -Ht;
                        ab[0] = fmin(lb, -l2);
                    }
                    if (lb > l2) {
                        aa[1] = fmax(la, l2);
                        ab[1] = lb;
                        aw[1] = -Ht;
                    }
                    if (c2 >= 1.0) {
                        if (cb > ca) {
                            wsh[1] += sgnr(cb);
                            wsh[0] -= sgnr(ca);
                            aa[2] = ca;
                            ab[2] = cb;
                            aw[2] = dH;
                        }
                    } else {
                        l1 = sqrt(1.0 - c2);
                        if (ca < -l1) {
                            const double B = fmin(cb, -l1);
                            wsh[0] -= sgnr(ca);
                            if (B == cb) wsh[1] += sgnr(cb);
                            else wsh[2] -= 1.0;
                            aa[2] = ca;
                            ab[2] = B;
                            aw[2] = dH;
                        }
                        if (cb > l1) {
                            const double Aq = fmax(ca, l1);
                            wsh[1] += sgnr(cb);
                            if (Aq == ca) wsh[0] -= sgnr(ca);
                            else wsh[2] -= 1.0;
                            aa[3] = Aq;
                            ab[3] = cb;
                            aw[3] = dH;
                        }
                        const double Ai = fmax(ca, -l1), Bi = fmin(cb, l1);
                        if (Bi > Ai) {
                            if (Bi == cb) wi[1] += sgnr(cb);
                            else wi[2] += 1.0;
                            if (Ai == ca) wi[0] -= sgnr(ca);
                            else wi[2] += 1.0;
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const bool want = live && aw[q] != 0.0;
                const int slot = wave_push(want, nA);
                if (want) {
                    W.ang[0][slot] = R0;
                    W.ang[1][slot] = aa[q];
                    W.ang[2][slot] = ab[q];
                    W.ang[3][slot] = sg * aw[q];
                    W.ang_o[slot] = (uint8_t)lane;
                }
                run_stack64<0>(W, nA, lane, false, wk);
            }
            {
                const double xs[3] = {fabs(ca), fabs(cb), l1};
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    const double x = xs[q];
                    const bool want = live && (wi[q] != 0.0 || wsh[q] != 0.0) && (q == 2 || x > 0.0);
                    const int slot = wave_push(want, nP);
                    if (want) {
                        W.pnt[0][slot] = r0;
                        W.pnt[1][slot] = R0;
                        W.pnt[2][slot] = c2;
                        W.pnt[3][slot] = c;
                        W.pnt[4][slot] = x;
                        W.pnt[5][slot] = q == 2 ? 1.0 : (x == l2 ? 2.0 : sqrt(c2 + x * x));
                        W.pnt[6][slot] = sg * wi[q];
                        W.pnt[7][slot] = sg * wsh[q];
                        W.pnt_o[slot] = (uint8_t)lane;
                    }
                    run_stack64<1>(W, nP, lane, false, wk);
                }
            }
        }
        run_stack64<0>(W, nA, lane, true, wk);
        run_stack64<1>(W, nP, lane, true, wk);
        lds_sync_wave();
        if (active) {
            JOB(f)[k] = (inside ? 1.0 : 0.0) - W.acc[lane] * kInvPi;
            if (inside && n_on >= 2) push_fix(FixList{JOB(fix_count), JOB(fix_items), JOB(fix_cap), nullptr}, k, kWindingSlot);
        }
        lds_sync_wave();
    }
    if (cur >= 0) flush_work(wk, MULTI ? A.table[cur].counters : A.one.counters);
}
#undef JOB

// ---------------------------------------------------------------- cell tiles
// A tile is up to 64 consecutive pairs of one cell (key = cell << 32 | tile
// index within the cell).  A wavefront integrating a tile shares the cell, so
// the cell's walls and edge records are wave-uniform: they are read with
// scalar loads into scalar registers, and the face/edge loops are uniform.
__global__ void k_tile_counts(int64_t n_cells, const int64_t *__restrict__ coff, int64_t *__restrict__ tcnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_cells) tcnt[i] = (coff[i + 1] - coff[i] + 63) / 64;
}

__global__ void k_tile_fill(int64_t n_cells, const int64_t *__restrict__ toff, uint64_t *__restrict__ tiles)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_cells) return;
    for (int64_t u = 0; u < toff[i + 1] - toff[i]; u++) tiles[toff[i] + u] = ((uint64_t)i << 32) | (uint64_t)u;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_integrate_tiles(int64_t n_tiles, const uint64_t *__restrict__ tiles,
                                                          const int64_t *__restrict__ coff,
                                                          const uint32_t *__restrict__ pair_p,
                                                          const double *__restrict__ xyz,
                                                          const double *__restrict__ h,
                                                          const int64_t *__restrict__ cfo,
                                                          const int64_t *__restrict__ fvo,
                                                          const double *__restrict__ plane,
                                                          const EdgeRec *__restrict__ edges, double *__restrict__ f,
                                                          unsigned long long *counters, unsigned *tile_ctr, FixList fx)
{
    using R = typename std::conditional<PREC == MAP_FP64, double, float>::type;
    const int lane = threadIdx.x & 63;
    Work wk;
    for (;;) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(tile_ctr, 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        if ((int64_t)t >= n_tiles) break;
        const uint64_t key = tiles[t];
        const int64_t cell = uniform64((int64_t)(key >> 32));
        const int64_t start = uniform64(coff[cell] + 64 * (int64_t)(key & 0xffffffffu));
        const int64_t end = uniform64(coff[cell + 1]);
        const int64_t k = start + lane;
        const bool active = k < end;
        double px = 0.0, py = 0.0, pz = 0.0, hh = 1.0;
        if (active) {
            const int64_t a = pair_p[k];
            px = xyz[3 * a];
            py = xyz[3 * a + 1];
            pz = xyz[3 * a + 2];
            hh = h[a];
        }
        const double invh = 1.0 / hh;
        bool inside = true;
        int n_on = 0;
        double acc = 0.0;
        float ev = 0.0f;
        const int64_t f0 = uniform64(cfo[cell]), f1 = uniform64(cfo[cell + 1]);
        for (int64_t j = f0; j < f1; j++) {
            const double nx = plane[4 * j], ny = plane[4 * j + 1], nz = plane[4 * j + 2], cj = plane[4 * j + 3];
            const double d = cj - (nx * px + ny * py + nz * pz);
            wk.faces += active;
            const bool in_j = d >= 0.0;
            inside = inside && in_j;
            n_on += d == 0.0 ? 1 : 0;
            const double r0d = fabs(d) * invh;
            const int64_t s0 = uniform64(fvo[j]), s1 = uniform64(fvo[j + 1]);
            if (active && r0d < 2.0) {
                const R r0 = (R)r0d;
                const R Ht = pi_H<R>(r0);
                const R dH = pi_dH<R>(r0);
                double face = 0.0;
                for (int64_t s = s0; s < s1; s++) {
                    const EdgeRec &E = edges[s];
                    const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
                    const double rho = E.mx * wx + E.my * wy + E.mz * wz;
                    wk.edges++;
                    if (rho == 0.0) continue;
                    const double la = -(E.ex * wx + E.ey * wy + E.ez * wz) * invh;
                    const double lb = la + E.L * invh;
                    const double R0d = fabs(rho) * invh;
                    if (PREC == MAP_MIXED && needs_fp64(r0d, R0d, r0d * r0d + R0d * R0d)) {
                        const unsigned slot = atomicAdd(fx.count, 1u);
                        if (slot < fx.cap) fx.items[slot] = ((uint64_t)k << 32) | (uint64_t)(uint32_t)s;
                        continue;
                    }
                    const R tv = edge_term<R>(r0, (R)R0d, (R)la, (R)lb, Ht, dH, wk);
                    face += (rho > 0.0) ? (double)tv : -(double)tv;
                    if (PREC == MAP_MIXED) ev = fmaf((float)tv, (float)tv, ev);
                }
                acc += in_j ? face : -face;
            }
        }
        if (active) {
            f[k] = winding_term(inside, n_on, px, py, pz, cell, cfo, fvo, plane, edges) - acc * kInvPi;
            if (PREC == MAP_MIXED && fx.err) fx.err[k] = kTermErr * kInvPiF * sqrt_f32(ev);
        }
    }
    flush_work(wk, counters);
}

// FP64 values of flagged edges (fixup items, key = pair << 32 | face-vertex slot)
__global__ void k_fixup_values(int64_t n_fix, const uint64_t *__restrict__ keys, const uint32_t *__restrict__ pair_p,
                               const uint32_t *__restrict__ pair_c, const double *__restrict__ xyz,
                               const double *__restrict__ h, const int64_t *__restrict__ cfo,
                               const int64_t *__restrict__ fvo, const double *__restrict__ plane,
                               const EdgeRec *__restrict__ edges, double *__restrict__ vals,
                               unsigned long long *counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_fix) return;
    const uint64_t key = keys[i];
    const int64_t k = (int64_t)(key >> 32);
    const int64_t s = (int64_t)(key & 0xffffffffu);
    const int64_t a = pair_p[k], c = pair_c[k];
    if ((uint32_t)s == kWindingSlot) {
        // the kernel took the winding weight of the particle as 1
        vals[i] = cell_winding(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], c, cfo, fvo, plane, edges) - 1.0;
        atomicAdd(counters + C_WINDING, 1ull);
        return;
    }
    // the face of slot s within the cell
    int64_t lo = cfo[c], hi = cfo[c + 1] - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (fvo[mid] <= s) lo = mid;
        else hi = mid - 1;
    }
    vals[i] = edge_contribution_fp64(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], h[a], plane + 4 * lo, edges[s]);
}

// Adds the (key-sorted) fixup values of each pair, in key order, to f.
__global__ void k_fixup_apply(int64_t n_fix, const uint64_t *__restrict__ keys, const double *__restrict__ vals,
                              double *__restrict__ f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_fix) return;
    const uint64_t k = keys[i] >> 32;
    if (i > 0 && (keys[i - 1] >> 32) == k) return;
    double sum = 0.0;
    for (int64_t j = i; j < n_fix && (keys[j] >> 32) == k; j++) sum += vals[j];
    f[k] += sum;
}

// Node values of the tabulated pyramid integral I(r0, R0, phi) (the variant of
// Sec. II-B that interpolates a pre-computed table): r0 = 2 i / (n0 - 1),
// R0 = 2 j / (n1 - 1), phi = (pi/2) k / (n2 - 1) (the last plane at
// pi/2 - 1e-12), from the FP64 closed form above:
//     I = Omega / (4 pi) - (1/pi) [pi (Q - phi H)](0 .. l),   l = R0 tan(phi),
// with the triangle's solid angle Omega = atan2(l R0 (R0^2 + l^2), (S + r0)(R0^2 S + r0 l^2)).
__global__ void k_table_build(int n0, int n1, int n2, double *__restrict__ tab64, float *__restrict__ tab32)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n0 * n1 * n2;
    if (q >= total) return;
    const int k = (int)(q % n2);
    const int j = (int)((q / n2) % n1);
    const int i = (int)(q / ((int64_t)n1 * n2));
    const double r0 = 2.0 * i / (double)(n0 - 1);
    const double R0 = 2.0 * j / (double)(n1 - 1);
    const double phi = k == n2 - 1 ? 0.5 * M_PI - 1e-12 : 0.5 * M_PI * k / (double)(n2 - 1);
    double I = 0.0;
    if (r0 > 0.0 && R0 > 0.0 && phi > 0.0) {
        const double l = R0 * tan(phi);
        const double S = sqrt(r0 * r0 + R0 * R0 + l * l);
        const double om = atan2(l * R0 * (R0 * R0 + l * l), (S + r0) * (R0 * R0 * S + r0 * l * l));
        Work wk;
        const double e = edge_term<double>(r0, R0, 0.0, l, pi_H<double>(r0), pi_dH<double>(r0), wk);
        I = om * (0.25 * kInvPi) - e * kInvPi;
    }
    tab64[q] = I;
    tab32[q] = (float)I;
}

}  // namespace

// The listed cells' pairs in FP64, to the bit as pair_fraction<MAP_FP64>
// (the per-pair FP64 form): each workgroup takes chunks of 32 of a cell's pairs (kRecBlocks workgroups
// per cell, chunks round-robin), computes every (pair, wall) term of a chunk
// in parallel (the wall's edge loop of pair_fraction), then one thread per
// pair adds its walls in wall order, as pair_fraction does, so the result is
// the FP64 path's to the bit (cells of up to 64 walls; larger ones take one
// thread per pair).  One thread per pair left most of the
// workgroup idle and each thread with all of its pair's edge terms in a row.
constexpr int kRecPairs = 32, kRecBlocks = 4, kRecWalls = 64;

__global__ void __launch_bounds__(256) k_recompute_cells(int64_t n_list, const uint32_t *__restrict__ cells,
                                                         const int64_t *__restrict__ coff,
                                                         const uint32_t *__restrict__ pair_p,
                                                         const double *__restrict__ xyz, const double *__restrict__ h,
                                                         const int64_t *__restrict__ cfo,
                                                         const int64_t *__restrict__ fvo,
                                                         const double *__restrict__ plane,
                                                         const EdgeRec *__restrict__ edges, double *__restrict__ f,
                                                         unsigned long long *counters)
{
    static_assert(kRecPairs * kRecWalls <= 2048, "one chunk's terms in LDS");
    __shared__ double term[kRecPairs * kRecWalls];
    __shared__ uint8_t side[kRecPairs * kRecWalls];  // bit 0: d >= 0, bit 1: d == 0
    const int64_t q = blockIdx.x;
    if (q >= n_list) return;
    const int64_t c = cells[q];
    const int64_t f0 = cfo[c], nw = cfo[c + 1] - f0;
    const int64_t k0 = coff[c], np = coff[c + 1] - k0;
    if (nw > kRecWalls) {  // cells of more walls: one thread per pair
        for (int64_t k = k0 + (int64_t)blockIdx.y * blockDim.x + threadIdx.x; k < k0 + np;
             k += (int64_t)gridDim.y * blockDim.x) {
            const int64_t a = pair_p[k];
            Work wk;
            float ev = 0.0f;
            f[k] = pair_fraction<MAP_FP64>(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], h[a], c, cfo, fvo, plane,
                                           edges, wk, (uint64_t)k, nullptr, nullptr, 0u, ev);
        }
    } else {
        const int W = (int)nw;
        for (int64_t pb = (int64_t)blockIdx.y * kRecPairs; pb < np; pb += (int64_t)gridDim.y * kRecPairs) {
            const int nc = (int)(np - pb < kRecPairs ? np - pb : kRecPairs);
            __syncthreads();  // the previous chunk's sums are done
            for (int it = threadIdx.x; it < nc * W; it += blockDim.x) {
                const int p = it / W, w = it - p * W;
                const int64_t a = pair_p[k0 + pb + p];
                const double px = xyz[3 * a], py = xyz[3 * a + 1], pz = xyz[3 * a + 2];
                const double invh = 1.0 / h[a];
                const int64_t j = f0 + w;
                const double nx = plane[4 * j], ny = plane[4 * j + 1], nz = plane[4 * j + 2], cj = plane[4 * j + 3];
                const double d = cj - (nx * px + ny * py + nz * pz);
                side[it] = (uint8_t)((d >= 0.0 ? 1 : 0) | (d == 0.0 ? 2 : 0));
                const double r0d = fabs(d) * invh;
                double face = 0.0;
                if (r0d < 2.0) {
                    Work wk;
                    const double Ht = pi_H<double>(r0d), dH = pi_dH<double>(r0d);
                    for (int64_t sl = fvo[j]; sl < fvo[j + 1]; sl++) {
                        const EdgeRec E = edges[sl];
                        const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
                        const double rho = E.mx * wx + E.my * wy + E.mz * wz;
                        if (rho == 0.0) continue;
                        const double la = -(E.ex * wx + E.ey * wy + E.ez * wz) * invh;
                        const double lb = la + E.L * invh;
                        const double t = edge_term<double>(r0d, fabs(rho) * invh, la, lb, Ht, dH, wk);
                        face += (rho > 0.0) ? t : -t;
                    }
                }
                term[it] = face;
            }
            __syncthreads();
            for (int p = threadIdx.x; p < nc; p += blockDim.x) {
                const int64_t k = k0 + pb + p, a = pair_p[k];
                bool inside = true;
                int n_on = 0;
                double acc = 0.0;
                for (int w = 0; w < W; w++) {
                    const uint8_t sd = side[p * W + w];
                    const bool in_j = (sd & 1) != 0;
                    inside = inside && in_j;
                    n_on += (sd >> 1) & 1;
                    const double face = term[p * W + w];
                    acc += in_j ? face : -face;
                }
                f[k] = winding_term(inside, n_on, xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], c, cfo, fvo, plane,
                                    edges) -
                       acc * kInvPi;
            }
        }
    }
    if (threadIdx.x == 0 && blockIdx.y == 0) atomicAdd(counters + C_FP64_PAIRS, (unsigned long long)np);
}

void launch_table_build(int n0, int n1, int n2, double *tab64, float *tab32, hipStream_t s)
{
    const int64_t total = (int64_t)n0 * n1 * n2;
    hipLaunchKernelGGL(k_table_build, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n0, n1, n2, tab64,
                       tab32);
    EM_HIP(hipGetLastError());
}

void build_tiles(Workspace &ws, const DevInputs &in, PairSet &ps, hipStream_t s)
{
    const int64_t nc = in.n_cells;
    ps.n_tiles = 0;
    if (nc == 0 || ps.n_pairs == 0) return;
    int64_t *tcnt = ws.get<int64_t>(S_TILE_CNT, (size_t)nc);
    int64_t *toff = ws.get<int64_t>(S_TILE_OFF, (size_t)nc + 1);
    hipLaunchKernelGGL(k_tile_counts, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, nc, ps.coff, tcnt);
    EM_HIP(hipGetLastError());
    scan_counts(ws, tcnt, toff, nc, s);
    int64_t nt = 0;
    EM_HIP(hipMemcpyAsync(&nt, toff + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    stream_sync(s);
    uint64_t *tiles = ws.get<uint64_t>(S_TILES, (size_t)(nt > 0 ? nt : 1));
    hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, nc, (const int64_t *)toff,
                       tiles);
    EM_HIP(hipGetLastError());
    ps.tiles = tiles;
    ps.n_tiles = nt;
}

// The task-batch kernels (distribution 3) over one job (its entry passed by
// value) or several (the table in device memory, h_jobs its host copy): the
// tile space of a launch is the concatenation of the jobs' tiles of 64 pairs.
static void launch_queued(const IntJob *h_jobs, const IntJob *d_jobs, int n_jobs, int precision,
                          const IntegrateTune &tune, unsigned *tile_ctr, bool zero_ctr, hipStream_t s)
{
    EM_CHECK(n_jobs >= 1 && h_jobs, MAP_EINVAL, "integration launch without jobs");
    EM_CHECK(n_jobs == 1 || d_jobs, MAP_EINVAL, "integration launch of several jobs without a device table");
    int64_t tiles = 0;
    for (int i = 0; i < n_jobs; i++) {
        EM_CHECK(h_jobs[i].tile_base == tiles && h_jobs[i].np > 0, MAP_EINVAL,
                 "integration job table: tile bases are not the running tile count");
        tiles += (h_jobs[i].np + 63) / 64;
    }
    JobsArg A;
    A.table = d_jobs;
    A.n = n_jobs;
    A.n_tiles = tiles;
    A.one = h_jobs[0];
    // [16..23] per-XCD tile counters
    if (zero_ctr) fill_zero_bytes(tile_ctr, 24 * sizeof(unsigned), s);
    const int block = 256;
    int64_t g = (int64_t)device_cu_count() * (tune.grid_per_cu > 0 ? tune.grid_per_cu : 8);
    const int64_t need = (tiles + (block / 64) - 1) / (block / 64);
    if (g > need) g = need;
    if (g < 1) g = 1;
    const bool multi = n_jobs > 1;
#define EM_LAUNCH_Q(...) hipLaunchKernelGGL((__VA_ARGS__), dim3((unsigned)g), dim3(block), 0, s, A, tile_ctr)
    if (precision == MAP_FP64 && tune.waves >= 3) {
        if (multi) EM_LAUNCH_Q(k_integrate_queued64<3, true>);
        else EM_LAUNCH_Q(k_integrate_queued64<3, false>);
    } else if (precision == MAP_FP64) {
        if (multi) EM_LAUNCH_Q(k_integrate_queued64<2, true>);
        else EM_LAUNCH_Q(k_integrate_queued64<2, false>);
    } else if (tune.waves >= 6 || tune.waves <= 0) {
        if (multi) EM_LAUNCH_Q(k_integrate_queued<6, true>);
        else EM_LAUNCH_Q(k_integrate_queued<6, false>);
    } else if (tune.waves >= 3) {
        if (multi) EM_LAUNCH_Q(k_integrate_queued<3, true>);
        else EM_LAUNCH_Q(k_integrate_queued<3, false>);
    } else {
        if (multi) EM_LAUNCH_Q(k_integrate_queued<2, true>);
        else EM_LAUNCH_Q(k_integrate_queued<2, false>);
    }
#undef EM_LAUNCH_Q
    EM_HIP(hipGetLastError());
}

void launch_integrate(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, int precision,
                      const IntegrateTune &tune, double *f, float *err, int64_t *counters, uint32_t *tile_ctr,
                      uint64_t *fix_items, int64_t fix_cap, hipStream_t s)
{
    const int64_t np = ps.n_pairs;
    if (np == 0) return;
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(counters);
    FixList fx;
    fx.count = tile_ctr + 1;
    fx.items = fix_items;
    fx.cap = (unsigned)(fix_cap > 0xffffffffLL ? 0xffffffffLL : fix_cap);
    fx.err = precision == MAP_MIXED ? err : nullptr;
    // [0] tile counter, [1] fixup count, [16..23] per-XCD tile counters
    fill_zero_bytes(tile_ctr, 24 * sizeof(unsigned), s);
    const int block = 256;
    if (!tune.persistent) {
        const unsigned g = (unsigned)((np + block - 1) / block);
        if (precision == MAP_FP64)
            hipLaunchKernelGGL(k_integrate_flat<MAP_FP64>, dim3(g), dim3(block), 0, s, np, ps.pair_p, ps.pair_c, in.xyz,
                               in.h, in.cfo, in.fvo, in.plane, edges, f, cnt, fx);
        else
            hipLaunchKernelGGL(k_integrate_flat<MAP_MIXED>, dim3(g), dim3(block), 0, s, np, ps.pair_p, ps.pair_c,
                               in.xyz, in.h, in.cfo, in.fvo, in.plane, edges, f, cnt, fx);
        EM_HIP(hipGetLastError());
        return;
    }
    if (tune.persistent == 3) {
        IntJob J;
        J.np = np;
        J.tile_base = 0;
        J.pair_p = ps.pair_p;
        J.pair_c = ps.pair_c;
        J.xyz = in.xyz;
        J.h = in.h;
        J.cfo = in.cfo;
        J.fvo = in.fvo;
        J.plane = in.plane;
        J.edges = edges;
        J.f = f;
        J.err = fx.err;
        J.counters = cnt;
        J.fix_count = fx.count;
        J.fix_items = fx.items;
        J.fix_cap = fx.cap;
        launch_queued(&J, nullptr, 1, precision, tune, tile_ctr, false, s);
        return;
    }
    if (tune.persistent == 2 && ps.tiles) {
        int64_t g = (int64_t)device_cu_count() * (tune.grid_per_cu > 0 ? tune.grid_per_cu : 8);
        int64_t need = (ps.n_tiles + (block / 64) - 1) / (block / 64);
        if (g > need) g = need;
        if (g < 1) g = 1;
        if (precision == MAP_FP64)
            hipLaunchKernelGGL(k_integrate_tiles<MAP_FP64>, dim3((unsigned)g), dim3(block), 0, s, ps.n_tiles,
                               ps.tiles, ps.coff, ps.pair_p, in.xyz, in.h, in.cfo, in.fvo, in.plane, edges, f, cnt,
                               tile_ctr, fx);
        else
            hipLaunchKernelGGL(k_integrate_tiles<MAP_MIXED>, dim3((unsigned)g), dim3(block), 0, s, ps.n_tiles,
                               ps.tiles, ps.coff, ps.pair_p, in.xyz, in.h, in.cfo, in.fvo, in.plane, edges, f, cnt,
                               tile_ctr, fx);
        EM_HIP(hipGetLastError());
        return;
    }
    const int tw = tune.tile_waves > 0 ? tune.tile_waves : 1;
    int64_t tiles = (np + 64 * tw - 1) / (64 * tw);
    int64_t g = (int64_t)device_cu_count() * (tune.grid_per_cu > 0 ? tune.grid_per_cu : 8);
    int64_t need = (tiles + (block / 64) - 1) / (block / 64);
    if (g > need) g = need;
    if (g < 1) g = 1;
#define EM_LAUNCH_P(P, W)                                                                                         \
    hipLaunchKernelGGL((k_integrate_persistent<P, W>), dim3((unsigned)g), dim3(block), 0, s, np, ps.pair_p,      \
                       ps.pair_c, in.xyz, in.h, in.cfo, in.fvo, in.plane, edges, f, cnt, tile_ctr, tw, fx)
    const int w = tune.waves;
    if (precision == MAP_FP64) {
        if (w >= 4) EM_LAUNCH_P(MAP_FP64, 4);
        else if (w == 3) EM_LAUNCH_P(MAP_FP64, 3);
        else EM_LAUNCH_P(MAP_FP64, 2);
    } else {
        if (w >= 6) EM_LAUNCH_P(MAP_MIXED, 6);
        else if (w == 5) EM_LAUNCH_P(MAP_MIXED, 5);
        else EM_LAUNCH_P(MAP_MIXED, 4);
    }
#undef EM_LAUNCH_P
    EM_HIP(hipGetLastError());
}

void launch_integrate_jobs(const IntJob *h_jobs, const IntJob *d_jobs, int n_jobs, int precision,
                           const IntegrateTune &tune, unsigned *tile_ctr, hipStream_t s)
{
    launch_queued(h_jobs, d_jobs, n_jobs, precision, tune, tile_ctr, true, s);
}

void launch_recompute_cells(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, const uint32_t *cells,
                            int64_t n_cells, double *f, int64_t *counters, hipStream_t s)
{
    if (n_cells <= 0) return;
    hipLaunchKernelGGL(k_recompute_cells, dim3((unsigned)n_cells, kRecBlocks), dim3(256), 0, s, n_cells,
                       cells, ps.coff, ps.pair_p, in.xyz, in.h, in.cfo, in.fvo, in.plane, edges, f,
                       reinterpret_cast<unsigned long long *>(counters));
    EM_HIP(hipGetLastError());
}

void launch_fixup(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, const uint64_t *fix_keys,
                  int64_t n_fix, double *fix_vals, int64_t *counters, hipStream_t s)
{
    if (n_fix <= 0) return;
    hipLaunchKernelGGL(k_fixup_values, dim3((unsigned)((n_fix + 255) / 256)), dim3(256), 0, s, n_fix, fix_keys,
                       ps.pair_p, ps.pair_c, in.xyz, in.h, in.cfo, in.fvo, in.plane, edges, fix_vals,
                       reinterpret_cast<unsigned long long *>(counters));
    EM_HIP(hipGetLastError());
}

void launch_fixup_apply(const uint64_t *keys, const double *vals, int64_t n_fix, double *f, hipStream_t s)
{
    if (n_fix <= 0) return;
    hipLaunchKernelGGL(k_fixup_apply, dim3((unsigned)((n_fix + 255) / 256)), dim3(256), 0, s, n_fix, keys, vals, f);
    EM_HIP(hipGetLastError());
}

}  // namespace em
