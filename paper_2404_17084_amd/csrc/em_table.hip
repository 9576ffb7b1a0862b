// Tabulated variant of the pair integral (Sec. II-B: the vertex-pyramid
// integral pre-computed on a grid and interpolated).
//
// The table holds I(r0, R0, phi) on a uniform n0 x n1 x n2 grid over
// r0, R0 in [0, 2] and phi in [0, pi/2] (FP32 node values of the FP64 closed
// form).  A pair is assembled in the far-field-subtracted form of the closed
// form: with D = Omega / (4 pi) - I, the mass of a pyramid's cone beyond its
// wall,
//     f = [p inside] - sum_walls sigma_j sum_edges sign(rho) [D~(l_b) - D~(l_a)],
//     D~(l) = sign(l) D(r0, R0, atan(|l| / R0)),
// because the solid angles of a cell's pyramids add up to its winding number
// about the particle.  D = 0 for walls with r0 >= 2 (skipped), and for R0 > 2
// D does not depend on R0 (the support's cross-section with the wall lies in
// the triangle's wedge), so it is read at R0 = 2 with the same angle.  Each D
// is one solid angle (FP32, one atan2) less a trilinear read of the table;
// geometry is FP64, sums are FP64.
//
// One thread per pair, cell-major pair order (neighbouring threads share a
// cell, so wall and edge records are read once per wavefront from cache); the
// table stays in L2 (1 MiB at 64^3).
#include <cmath>

#include "em_boundary.h"
#include "em_internal.h"
#include "em_fmath.h"

namespace em {

namespace {

struct TableView {
    const float *__restrict__ t;
    int n0, n1, n2;
    float s0, s1, s2;  // grid coordinates per unit of r0, R0, phi
};

__device__ __forceinline__ void grid_cell(float x, int n, int &i, float &a)
{
    int k = (int)floorf(x);
    k = k < 0 ? 0 : (k > n - 2 ? n - 2 : k);
    i = k;
    a = x - (float)k;
}

__device__ __forceinline__ float table_I(const TableView &T, float r0, float R0, float phi)
{
    int i, j, k;
    float a, b, c;
    grid_cell(r0 * T.s0, T.n0, i, a);
    grid_cell(R0 * T.s1, T.n1, j, b);
    grid_cell(phi * T.s2, T.n2, k, c);
    const float *p = T.t + ((int64_t)i * T.n1 + j) * T.n2 + k;
    const int64_t dj = T.n2, di = (int64_t)T.n1 * T.n2;
    const float v00 = p[0] + c * (p[1] - p[0]);
    const float v01 = p[dj] + c * (p[dj + 1] - p[dj]);
    const float v10 = p[di] + c * (p[di + 1] - p[di]);
    const float v11 = p[di + dj] + c * (p[di + dj + 1] - p[di + dj]);
    const float v0 = v00 + b * (v01 - v00);
    const float v1 = v10 + b * (v11 - v10);
    return v0 + a * (v1 - v0);
}

// D of the right triangle [0, l] (l >= 0) at wall distance r0 < 2
__device__ __forceinline__ float table_D(const TableView &T, float r0, float R0, float l)
{
    if (!(l > 0.0f)) return 0.0f;
    const float phi = atan2_f32(l, R0);
    float Rc = R0, lc = l;
    if (R0 > 2.0f) {  // same angle at R0 = 2
        Rc = 2.0f;
        lc = l * (2.0f * rcp_f32(R0));
    }
    const float R2 = Rc * Rc, l2 = lc * lc;
    const float S = sqrt_f32(r0 * r0 + R2 + l2);
    const float om = atan2_f32(lc * Rc * (R2 + l2), (S + r0) * (R2 * S + r0 * l2));
    return om * 0.0795774715459477f - table_I(T, r0, Rc, phi);
}

__device__ __forceinline__ float table_Dt(const TableView &T, float r0, float R0, float l)
{
    return l < 0.0f ? -table_D(T, r0, R0, -l) : table_D(T, r0, R0, l);
}

__global__ void __launch_bounds__(256) k_integrate_table(int64_t np, const uint32_t *__restrict__ pair_p,
                                                         const uint32_t *__restrict__ pair_c,
                                                         const double *__restrict__ xyz, const double *__restrict__ h,
                                                         const int64_t *__restrict__ cfo,
                                                         const int64_t *__restrict__ fvo,
                                                         const double *__restrict__ plane,
                                                         const EdgeRec *__restrict__ edges, TableView T,
                                                         double *__restrict__ f, unsigned long long *counters)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long n_faces = 0, n_edges = 0, n_terms = 0;
    if (q < np) {
        const int64_t a = pair_p[q], cell = pair_c[q];
        const double px = xyz[3 * a], py = xyz[3 * a + 1], pz = xyz[3 * a + 2];
        const double invh = 1.0 / h[a];
        bool inside = true;
        int n_on = 0;
        double acc = 0.0;
        for (int64_t j = cfo[cell]; j < cfo[cell + 1]; j++) {
            const double nx = plane[4 * j], ny = plane[4 * j + 1], nz = plane[4 * j + 2], cj = plane[4 * j + 3];
            const double d = cj - (nx * px + ny * py + nz * pz);
            n_faces++;
            const bool in_j = d >= 0.0;
            inside = inside && in_j;
            n_on += d == 0.0 ? 1 : 0;
            const double r0d = fabs(d) * invh;
            if (!(r0d < 2.0)) continue;
            const float r0 = (float)r0d;
            double face = 0.0;
            for (int64_t s = fvo[j]; s < fvo[j + 1]; s++) {
                const EdgeRec E = edges[s];
                const double wx = px - E.vx, wy = py - E.vy, wz = pz - E.vz;
                const double rho = E.mx * wx + E.my * wy + E.mz * wz;
                n_edges++;
                if (rho == 0.0) continue;
                const double la = -(E.ex * wx + E.ey * wy + E.ez * wz) * invh;
                const double lb = la + E.L * invh;
                const float R0 = (float)(fabs(rho) * invh);
                const float t = table_Dt(T, r0, R0, (float)lb) - table_Dt(T, r0, R0, (float)la);
                n_terms += 2;
                face += rho > 0.0 ? (double)t : -(double)t;
            }
            acc += in_j ? face : -face;
        }
        f[q] = winding_term(inside, n_on, px, py, pz, cell, cfo, fvo, plane, edges) - acc;
    }
    for (int o = 32; o > 0; o >>= 1) {
        n_faces += __shfl_xor(n_faces, o, 64);
        n_edges += __shfl_xor(n_edges, o, 64);
        n_terms += __shfl_xor(n_terms, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(counters + C_FACES, n_faces);
        atomicAdd(counters + C_EDGES, n_edges);
        atomicAdd(counters + C_EDGE_TERMS, n_terms);
    }
}

}  // namespace

void launch_integrate_table(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, const float *tab, int n0,
                            int n1, int n2, double *f, int64_t *counters, hipStream_t s)
{
    const int64_t np = ps.n_pairs;
    if (np <= 0) return;
    TableView T;
    T.t = tab;
    T.n0 = n0;
    T.n1 = n1;
    T.n2 = n2;
    T.s0 = (float)(n0 - 1) * 0.5f;
    T.s1 = (float)(n1 - 1) * 0.5f;
    T.s2 = (float)((double)(n2 - 1) / (0.5 * M_PI));
    hipLaunchKernelGGL(k_integrate_table, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np, ps.pair_p,
                       ps.pair_c, in.xyz, in.h, in.cfo, in.fvo, in.plane, edges, T, f,
                       reinterpret_cast<unsigned long long *>(counters));
    EM_HIP(hipGetLastError());
}

}  // namespace em
