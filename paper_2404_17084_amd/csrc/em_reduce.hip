// Reductions of Eq. (3): per-particle sums S_a (sum-to-one normalisation),
// per-cell masses M_i = sum_a m_a f_ai / S_a and densities rho_i = M_i / V_i.
// S_a is summed in 2^-52 fixed point with integer atomics (exact, so the
// result does not depend on the order of the additions); the cell sums use one
// wavefront per cell, lanes strided over the segment and a fixed butterfly.
#include <cmath>

#include "em_internal.h"

namespace em {

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// S_a: every pair adds round(f 2^52) to its particle's 64-bit counter (each
// term rounded by at most 2^-53, the sum exact), then the counters become
// doubles in place.
__global__ void k_particle_sum(int64_t np, const uint32_t *__restrict__ pair_p, const double *__restrict__ f,
                               unsigned long long *__restrict__ acc)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const long long q = __double2ll_rn(f[k] * 4503599627370496.0);
    atomicAdd(&acc[pair_p[k]], (unsigned long long)q);
}

__global__ void k_fixed_to_double(int64_t n, double *S)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const long long q = reinterpret_cast<const long long *>(S)[a];
    S[a] = (double)q * 2.220446049250313e-16;
}

// Inverse mapping, one wavefront per particle over its pairs in cell order
// (lanes strided, fixed butterfly): q_a = sum_i q_i f_ai / S_a.
__global__ void k_map_back(int64_t n, const int64_t *__restrict__ poff, const uint32_t *__restrict__ perm,
                           const uint32_t *__restrict__ pair_c, const double *__restrict__ f,
                           const double *__restrict__ S, const double *__restrict__ q_cell, double *__restrict__ q_part)
{
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n) return;
    double v = 0.0;
    for (int64_t q = poff[a] + lane; q < poff[a + 1]; q += 64) {
        const uint32_t k = perm[q];
        v += q_cell[pair_c[k]] * f[k];
    }
    v = wave_sum(v);
    if (lane == 0) q_part[a] = S[a] > 0.0 ? v / S[a] : 0.0;
}

__global__ void k_cell_mass(int64_t nc, const int64_t *coff, const uint32_t *pair_p, const double *f,
                            const double *S, const double *m, const double *vol, double *M, double *rho)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= nc) return;
    double v = 0.0;
    for (int64_t k = coff[i] + lane; k < coff[i + 1]; k += 64) {
        const uint32_t a = pair_p[k];
        const double sa = S[a];
        if (sa > 0.0) v += m[a] * (f[k] / sa);
    }
    v = wave_sum(v);
    if (lane == 0) {
        M[i] = v;
        rho[i] = v / vol[i];
    }
}

// Mixed path, before the normalisation: one wavefront per cell,
// sqrt(sum (m_a err_ai)^2) against tol |sum m_a f_ai| (the cell's estimated
// FP32 error relative to its raw mass; the sum-to-one normalisation divides
// both by S_a, close to one); the cells over the budget are listed.
__global__ void k_cell_check(int64_t nc, const int64_t *coff, const uint32_t *pair_p, const float *err,
                             const double *f, const double *m, double tol, unsigned *count, uint32_t *list,
                             int64_t cap)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= nc) return;
    double v = 0.0, raw = 0.0;
    for (int64_t k = coff[i] + lane; k < coff[i + 1]; k += 64) {
        const double ma = m[pair_p[k]];
        const double e = ma * (double)err[k];
        v += e * e;
        raw += ma * f[k];
    }
    v = wave_sum(v);
    raw = wave_sum(raw);
    if (lane == 0 && sqrt(v) > tol * fabs(raw)) {
        const unsigned q = atomicAdd(count, 1u);
        if ((int64_t)q < cap) list[q] = (uint32_t)i;
    }
}

// Block partials: [0] sum M, [1] max |S-1| over particles whose support lies in
// the box, [2] sum m, [3] 1 if any M is not finite.
constexpr int RB = 256;

__global__ void k_stats_partial(int64_t nc, const double *M, int64_t n, const double *S, const double *xyz,
                                const double *h, const double *m, const double *box, double *part)
{
    __shared__ double sh[4][RB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double sm = 0.0, mx = 0.0, sin = 0.0, bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        sm += M[i];
        if (!isfinite(M[i])) bad = 1.0;
    }
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += stride) {
        sin += m[a];
        const double r = 2.0 * h[a];
        bool interior = true;
        for (int d = 0; d < 3; d++) {
            const double x = xyz[3 * a + d];
            interior = interior && (x - r > box[d]) && (x + r < box[3 + d]);
        }
        if (interior) mx = fmax(mx, fabs(S[a] - 1.0));
    }
    sm = wave_sum(sm);
    sin = wave_sum(sin);
    mx = wave_max(mx);
    bad = wave_max(bad);
    if (lane == 0) {
        sh[0][wave] = sm;
        sh[1][wave] = mx;
        sh[2][wave] = sin;
        sh[3][wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int w = 0; w < RB / 64; w++) {
            a0 += sh[0][w];
            a1 = fmax(a1, sh[1][w]);
            a2 += sh[2][w];
            a3 = fmax(a3, sh[3][w]);
        }
        part[4 * blockIdx.x + 0] = a0;
        part[4 * blockIdx.x + 1] = a1;
        part[4 * blockIdx.x + 2] = a2;
        part[4 * blockIdx.x + 3] = a3;
    }
}

__global__ void k_stats_final(int nb, const double *part, double *red, unsigned *flags)
{
    if (threadIdx.x != 0) return;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int b = 0; b < nb; b++) {
        a0 += part[4 * b + 0];
        a1 = fmax(a1, part[4 * b + 1]);
        a2 += part[4 * b + 2];
        a3 = fmax(a3, part[4 * b + 3]);
    }
    red[0] = a0;
    red[1] = a1;
    red[2] = a2;
    if (a3 > 0.0) atomicOr(flags, F_RESULT_NONFINITE);
}

}  // namespace

void launch_map_back(int64_t n, const int64_t *poff, const uint32_t *perm, const uint32_t *pair_c, const double *f,
                     const double *S, const double *q_cell, double *q_part, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_map_back, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, s, n, poff, perm, pair_c, f,
                       S, q_cell, q_part);
    EM_HIP(hipGetLastError());
}

void launch_cell_check(const DevInputs &in, const PairSet &ps, const float *err, const double *f, double tol,
                       unsigned *count, uint32_t *list, int64_t cap, hipStream_t s)
{
    const int64_t nc = in.n_cells;
    fill_zero_bytes(count, sizeof(unsigned), s);
    if (nc <= 0 || ps.n_pairs <= 0) return;
    hipLaunchKernelGGL(k_cell_check, dim3((unsigned)((nc * 64 + 255) / 256)), dim3(256), 0, s, nc, ps.coff, ps.pair_p,
                       err, f, in.m, tol, count, list, cap);
    EM_HIP(hipGetLastError());
}

void launch_reduce(const DevInputs &in, const PairSet &ps, const double *f, double *S, double *M,
                   double *rho, double *red, unsigned *flags, hipStream_t s)
{
    const int64_t n = in.n, nc = in.n_cells;
    if (n > 0) {
        fill_zero_bytes(S, sizeof(double) * n, s);
        if (ps.n_pairs > 0)
            hipLaunchKernelGGL(k_particle_sum, dim3((unsigned)((ps.n_pairs + 255) / 256)), dim3(256), 0, s,
                               ps.n_pairs, ps.pair_p, f, reinterpret_cast<unsigned long long *>(S));
        hipLaunchKernelGGL(k_fixed_to_double, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, S);
    }
    if (nc > 0)
        hipLaunchKernelGGL(k_cell_mass, dim3((unsigned)((nc * 64 + 255) / 256)), dim3(256), 0, s, nc, ps.coff,
                           ps.pair_p, f, (const double *)S, in.m, in.vol, M, rho);
    EM_HIP(hipGetLastError());
    const int nb = 240;
    // red: [0..3] results, [4..9] the box (written by the caller), [16..] block partials
    double *part = red + 16;
    double *dbox = red + 4;
    hipLaunchKernelGGL(k_stats_partial, dim3(nb), dim3(RB), 0, s, nc, (const double *)M, n, (const double *)S,
                       in.xyz, in.h, in.m, (const double *)dbox, part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, s, nb, (const double *)part, red, flags);
    EM_HIP(hipGetLastError());
}

}  // namespace em
