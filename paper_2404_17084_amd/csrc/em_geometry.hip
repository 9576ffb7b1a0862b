// Input validation and per-cell geometry tables (edge records, bounding boxes,
// volumes).  Geometry is kept in FP64.
#include <cmath>

#include "em_internal.h"
#include "em_wave.h"

namespace em {

// Structure checks: only reads offsets and ids at fixed indices, so malformed
// input cannot make it read out of bounds.
__global__ void k_validate_structure(int64_t n_cells, int64_t n_faces, int64_t n_face_verts, int64_t n_verts,
                                     const int64_t *cfo, const int64_t *fvo, const int32_t *fv, unsigned *flags)
{
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned f = 0;
    for (int64_t i = tid; i <= n_cells; i += stride) {
        int64_t a = cfo[i];
        if (i == 0 && a != 0) f |= F_CFO_BAD;
        if (i == n_cells && a != n_faces) f |= F_CFO_BAD;
        if (i < n_cells) {
            int64_t b = cfo[i + 1];
            if (b - a < 4 || a < 0 || b > n_faces) f |= F_CFO_BAD;
        }
    }
    for (int64_t j = tid; j <= n_faces; j += stride) {
        int64_t a = fvo[j];
        if (j == 0 && a != 0) f |= F_FVO_BAD;
        if (j == n_faces && a != n_face_verts) f |= F_FVO_BAD;
        if (j < n_faces) {
            int64_t b = fvo[j + 1];
            if (a < 0 || b > n_face_verts || b < a) f |= F_FVO_BAD;
            else if (b - a < 3) f |= F_FACE_SMALL;
        }
    }
    for (int64_t s = tid; s < n_face_verts; s += stride) {
        int32_t v = fv[s];
        if (v < 0 || (int64_t)v >= n_verts) f |= F_VID_RANGE;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_validate_values(int64_t n, const double *xyz, const double *m, const double *h, int64_t n_faces,
                                  const double *plane, int64_t n_verts, const double *verts, int64_t n_cells,
                                  const double *vol, unsigned *flags)
{
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned f = 0;
    for (int64_t a = tid; a < n; a += stride) {
        double x = xyz[3 * a], y = xyz[3 * a + 1], z = xyz[3 * a + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) f |= F_PART_NONFINITE;
        double ha = h[a];
        if (!(ha > 0.0) || !isfinite(ha)) f |= F_H_NONPOS;
        double ma = m[a];
        if (!(ma >= 0.0) || !isfinite(ma)) f |= F_M_BAD;
    }
    for (int64_t j = tid; j < n_faces; j += stride) {
        double nx = plane[4 * j], ny = plane[4 * j + 1], nz = plane[4 * j + 2], c = plane[4 * j + 3];
        double nn = nx * nx + ny * ny + nz * nz;
        if (!isfinite(c) || !(fabs(nn - 1.0) <= 1e-10)) f |= F_PLANE_BAD;
    }
    for (int64_t v = tid; v < n_verts; v += stride) {
        if (!isfinite(verts[3 * v]) || !isfinite(verts[3 * v + 1]) || !isfinite(verts[3 * v + 2]))
            f |= F_VERT_NONFINITE;
    }
    if (vol)
        for (int64_t i = tid; i < n_cells; i += stride)
            if (!(vol[i] > 0.0) || !isfinite(vol[i])) f |= F_VOL_BAD;
    if (f) atomicOr(flags, f);
}

void launch_validate(const DevInputs &in, unsigned *flags, hipStream_t s)
{
    int64_t big = in.n_face_verts;
    if (in.n_faces > big) big = in.n_faces;
    if (in.n_cells > big) big = in.n_cells;
    if (in.n > big) big = in.n;
    if (in.n_verts > big) big = in.n_verts;
    int64_t g = (big + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_validate_structure, dim3((unsigned)g), dim3(256), 0, s, in.n_cells, in.n_faces,
                       in.n_face_verts, in.n_verts, in.cfo, in.fvo, in.fv, flags);
    EM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_validate_values, dim3((unsigned)g), dim3(256), 0, s, in.n, in.xyz, in.m, in.h, in.n_faces,
                       in.plane, in.n_verts, in.verts, in.n_cells, in.vol, flags);
    EM_HIP(hipGetLastError());
}

// Directed edges of every face (counter-clockwise about the outward normal
// n) with unit direction e and in-plane inward normal m = n x e, one record
// per slot.  A wavefront takes 64 consecutive faces and gives its lanes
// consecutive slots; a lane finds its slot's face by binary search in the
// wavefront's face offsets (faces have at least 3 slots, checked by the
// structure validation that runs first).  The 64 records of a round are
// staged in LDS and stored as consecutive 16-byte chunks: stored straight
// from the lanes, each store instruction would touch every fifth 16 bytes of
// forty cache lines.
__global__ void __launch_bounds__(256) k_edge_table(int64_t n_faces, const int64_t *fvo, const int32_t *fv,
                                                    const double *plane, const double *verts, EdgeRec *edges)
{
    static_assert(sizeof(EdgeRec) == 80, "records of five 16-byte chunks");
    __shared__ int64_t off[4][65];
    __shared__ float4 stage[4][5 * 64];  // a wavefront's 64 records, written out in whole 16-byte chunks
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t j0 = ((int64_t)blockIdx.x * 4 + w) * 64;
    if (j0 >= n_faces) return;
    const int nf = (int)(n_faces - j0 < 64 ? n_faces - j0 : 64);
    if (lane < nf) off[w][lane] = fvo[j0 + lane];
    if (lane == 0) off[w][nf] = fvo[j0 + nf];
    lds_sync_wave();
    const int64_t s_end = off[w][nf];
    for (int64_t q0 = off[w][0]; q0 < s_end; q0 += 64) {
        const int64_t q = q0 + lane;
        const int cnt = (int)(s_end - q0 < 64 ? s_end - q0 : 64);
        if (q < s_end) {
            int lo = 0, hi = nf - 1;  // face f with off[f] <= q < off[f + 1]
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (off[w][mid] <= q) lo = mid;
                else hi = mid - 1;
            }
            const int64_t j = j0 + lo;
            const int64_t qn = q + 1 == off[w][lo + 1] ? off[w][lo] : q + 1;
            const double *a = verts + 3 * (int64_t)fv[q];
            const double *b = verts + 3 * (int64_t)fv[qn];
            const double nx = plane[4 * j], ny = plane[4 * j + 1], nz = plane[4 * j + 2];
            double ex = b[0] - a[0], ey = b[1] - a[1], ez = b[2] - a[2];
            const double L = sqrt(ex * ex + ey * ey + ez * ez);
            const double inv = L > 0.0 ? 1.0 / L : 0.0;
            ex *= inv;
            ey *= inv;
            ez *= inv;
            EdgeRec &r = *reinterpret_cast<EdgeRec *>(&stage[w][5 * lane]);
            r.vx = a[0];
            r.vy = a[1];
            r.vz = a[2];
            r.L = L;
            r.ex = ex;
            r.ey = ey;
            r.ez = ez;
            r.mx = ny * ez - nz * ey;
            r.my = nz * ex - nx * ez;
            r.mz = nx * ey - ny * ex;
        }
        lds_sync_wave();
        // records q0 .. q0 + cnt - 1 are 5 cnt consecutive chunks: lane k writes chunks k, k + 64, ...
        float4 *dst = reinterpret_cast<float4 *>(edges + q0);
        for (int c = lane; c < 5 * cnt; c += 64) dst[c] = stage[w][c];
        lds_sync_wave();  // the chunks are read before the next records overwrite them
    }
}

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wmin(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wmax(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// One wavefront per cell, lanes over its walls: bounding box, an interior
// point g (the mean of the wall vertices), the volume (when asked), and the
// radii of the balls about g inside the cell (least wall-plane distance) and
// containing it (greatest vertex distance).  Lanes combine in a fixed order.
__global__ void k_cell_boxes(int64_t n_cells, const int64_t *cfo, const int64_t *fvo, const int32_t *fv,
                             const double *plane, const double *verts, double *aabb, double *vol_out)
{
    // one wavefront per cell, lanes over the cell's slots; a lane finds its
    // slot's wall by binary search in the wall offsets
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= n_cells) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double cen[3] = {0.0, 0.0, 0.0};
    double nslot = 0.0, vol = 0.0;
    const int64_t f0 = cfo[i], f1 = cfo[i + 1];
    const int64_t sb = fvo[f0], se = fvo[f1];
    const double *ref = verts + 3 * (int64_t)fv[sb];
    for (int64_t q = sb + lane; q < se; q += 64) {
        int64_t jl = f0, jh = f1 - 1;  // wall j with fvo[j] <= q < fvo[j + 1]
        while (jl < jh) {
            const int64_t mid = (jl + jh + 1) >> 1;
            if (fvo[mid] <= q) jl = mid;
            else jh = mid - 1;
        }
        const int64_t j = jl, s0 = fvo[j], s1 = fvo[j + 1];
        const double *v = verts + 3 * (int64_t)fv[q];
        for (int d = 0; d < 3; d++) {
            lo[d] = fmin(lo[d], v[d]);
            hi[d] = fmax(hi[d], v[d]);
            cen[d] += v[d];
        }
        nslot += 1.0;
        if (q > s0 && q + 1 < s1) {  // triangle (v_0, v_q, v_q+1) of the wall's fan
            const double *v0 = verts + 3 * (int64_t)fv[s0];
            const double *w = verts + 3 * (int64_t)fv[q + 1];
            const double nx = plane[4 * j], ny = plane[4 * j + 1], nz = plane[4 * j + 2], c = plane[4 * j + 3];
            const double ax = v[0] - v0[0], ay = v[1] - v0[1], az = v[2] - v0[2];
            const double bx = w[0] - v0[0], by = w[1] - v0[1], bz = w[2] - v0[2];
            const double t = (ay * bz - az * by) * nx + (az * bx - ax * bz) * ny + (ax * by - ay * bx) * nz;
            const double height = c - (nx * ref[0] + ny * ref[1] + nz * ref[2]);
            vol += height * t / 6.0;
        }
    }
    double g[3];
    const double ns = wsum(nslot);
    for (int d = 0; d < 3; d++) {
        lo[d] = wmin(lo[d]);
        hi[d] = wmax(hi[d]);
        g[d] = wsum(cen[d]) / ns;
    }
    vol = wsum(vol);
    double rin = INFINITY, rc2 = 0.0;
    for (int64_t j = f0 + lane; j < f1; j += 64)
        rin = fmin(rin, plane[4 * j + 3] - (plane[4 * j] * g[0] + plane[4 * j + 1] * g[1] + plane[4 * j + 2] * g[2]));
    for (int64_t q = sb + lane; q < se; q += 64) {
        const double *v = verts + 3 * (int64_t)fv[q];
        const double dx = v[0] - g[0], dy = v[1] - g[1], dz = v[2] - g[2];
        rc2 = fmax(rc2, dx * dx + dy * dy + dz * dz);
    }
    rin = wmin(rin);
    rc2 = wmax(rc2);
    if (lane == 0) {
        for (int d = 0; d < 3; d++) {
            aabb[6 * i + d] = lo[d];
            aabb[6 * i + 3 + d] = hi[d];
            aabb[6 * n_cells + 3 * i + d] = g[d];
        }
        aabb[9 * n_cells + 2 * i] = fmax(rin, 0.0);
        aabb[9 * n_cells + 2 * i + 1] = sqrt(rc2);
        if (vol_out) vol_out[i] = vol;
    }
}

void launch_geometry(const DevInputs &in, EdgeRec *edges, double *aabb, double *vol_out, hipStream_t s)
{
    if (in.n_faces > 0) {
        hipLaunchKernelGGL(k_edge_table, dim3((unsigned)((in.n_faces + 255) / 256)), dim3(256), 0, s, in.n_faces,
                           in.fvo, in.fv, in.plane, in.verts, edges);
        EM_HIP(hipGetLastError());
    }
    if (in.n_cells > 0) {
        hipLaunchKernelGGL(k_cell_boxes, dim3((unsigned)((in.n_cells * 64 + 255) / 256)), dim3(256), 0, s, in.n_cells,
                           in.cfo, in.fvo, in.fv, in.plane, in.verts, aabb, vol_out);
        EM_HIP(hipGetLastError());
    }
}

}  // namespace em
