// Pair search: every (particle a, cell i) whose closed cell lies closer to r_a
// than 2 h_a, ordered by cell and then particle.
//
// The particles, in storage order, are grouped 8 per leaf of an implicit
// complete binary tree of the boxes their supports can reach.  Each cell
// walks the tree without a stack (heap indices) and lists the particles whose
// support comes within its bounding box (candidates), already in cell-major
// order with particles ascending.  Cheap ball and box tests settle most
// candidates, the rest take the exact distance test below (FP32 screening
// with a rounding bound, then the exact IEEE arithmetic near the threshold),
// and a wavefront per cell compacts the pairs.
#include <cmath>

#include "em_internal.h"
#include "em_wave.h"

namespace em {

constexpr int64_t kLeaf = 8;  // particles per leaf of the bounding-volume tree

// Exact distance test.  Squared distance from p to the closed convex cell: 0
// inside; else the least squared distance to a wall polygon that p sees from
// outside (d_j < 0): d_j^2 if p projects inside the polygon, else the least
// squared distance to its edge segments.  Evaluated with plain IEEE adds,
// multiplies and divides in a fixed order, without fused multiply-adds, so
// that the decision dist^2 < (2h)^2 is reproducible on any IEEE machine.
// cell_meets decides dist^2 < r2 with that arithmetic, with two shortcuts
// that cannot change the decision.  (1) The cell lies inside every face's
// half-space, so its distance is at least max_j(-d_j); when that bound
// exceeds sqrt(r2) by a relative margin far above the rounding of the
// polygon distances, the pair is rejected.  (2) The first face or edge
// distance computed below r2 accepts the pair, since the minimum is no
// larger.
template <class G>
__device__ __forceinline__ bool meets_impl(double px, double py, double pz, double r2, const G &g)
{
#pragma clang fp contract(off)
    const int nf = g.n_faces();
    double far = 0.0;
    bool inside = true;
    for (int j = 0; j < nf; j++) {
        const double d = g.pl(j, 3) - (g.pl(j, 0) * px + g.pl(j, 1) * py + g.pl(j, 2) * pz);
        if (d < 0.0) {
            inside = false;
            if (-d > far) far = -d;
        }
    }
    if (inside) return true;
    if (far * far > r2 * (1.0 + 1e-9)) return false;
    for (int j = 0; j < nf; j++) {
        const double n0 = g.pl(j, 0), n1 = g.pl(j, 1), n2 = g.pl(j, 2), c = g.pl(j, 3);
        const double d = c - (n0 * px + n1 * py + n2 * pz);
        if (!(d < 0.0)) continue;
        const int k0 = g.slot0(j), nv = g.slot0(j + 1) - k0;
        bool left = true;
        for (int k = 0; k < nv; k++) {
            const int kb = k0 + (k + 1 == nv ? 0 : k + 1);
            const double ax = g.vx(k0 + k, 0), ay = g.vx(k0 + k, 1), az = g.vx(k0 + k, 2);
            const double ex = g.vx(kb, 0) - ax, ey = g.vx(kb, 1) - ay, ez = g.vx(kb, 2) - az;
            const double wx = px - ax, wy = py - ay, wz = pz - az;
            const double cr = (ey * wz - ez * wy) * n0 + (ez * wx - ex * wz) * n1 + (ex * wy - ey * wx) * n2;
            if (cr < 0.0) {
                left = false;
                break;
            }
        }
        if (left) {
            if (d * d < r2) return true;
            continue;
        }
        for (int k = 0; k < nv; k++) {
            const int kb = k0 + (k + 1 == nv ? 0 : k + 1);
            const double ax = g.vx(k0 + k, 0), ay = g.vx(k0 + k, 1), az = g.vx(k0 + k, 2);
            const double ex = g.vx(kb, 0) - ax, ey = g.vx(kb, 1) - ay, ez = g.vx(kb, 2) - az;
            const double wx = px - ax, wy = py - ay, wz = pz - az;
            const double ee = ex * ex + ey * ey + ez * ez;
            double t = 0.0;
            if (ee > 0.0) {
                t = (wx * ex + wy * ey + wz * ez) / ee;
                if (t < 0.0) t = 0.0;
                if (t > 1.0) t = 1.0;
            }
            const double qx = wx - t * ex, qy = wy - t * ey, qz = wz - t * ez;
            if (qx * qx + qy * qy + qz * qz < r2) return true;
        }
    }
    return false;
}

// One cell's walls read from the global tables (slots relative to the cell's first).
struct CellGlobal {
    const double *plane;  // at the cell's first wall
    const int64_t *fvo;   // at the cell's first wall
    const EdgeRec *edges;  // at the cell's first slot
    int nf;
    __device__ int n_faces() const { return nf; }
    __device__ double pl(int j, int q) const { return plane[4 * j + q]; }
    __device__ int slot0(int j) const { return (int)(fvo[j] - fvo[0]); }
    __device__ double vx(int k, int q) const { return q == 0 ? edges[k].vx : (q == 1 ? edges[k].vy : edges[k].vz); }
};

// One cell staged in LDS by a wavefront for the screened distance test:
// wall planes in FP64 (the exact test's plane pass) and, per slot, the edge
// start vertex relative to the cell centre g, the unit direction, the unit
// in-wall normal (pointing into the wall polygon) and the length, in FP32.
constexpr int kExactMaxFaces = 40, kExactMaxSlots = 160;
struct CellFast {
    double pl_[kExactMaxFaces][4];
    float4 a_[kExactMaxSlots];  // vertex - g (x, y, z), length
    float4 b_[kExactMaxSlots];  // e (x, y, z), m.x
    float2 c_[kExactMaxSlots];  // m.y, m.z
    int so_[kExactMaxFaces + 1];
    int nf;
};

__device__ __noinline__ bool cell_meets(double px, double py, double pz, double r2, int64_t cell,
                                        const int64_t *cfo, const int64_t *fvo, const EdgeRec *edges,
                                        const double *plane)
{
    const int64_t j0 = cfo[cell];
    CellGlobal g{plane + 4 * j0, fvo + j0, edges + fvo[j0], (int)(cfo[cell + 1] - j0)};
    return meets_impl(px, py, pz, r2, g);
}


// Leaves of the implicit tree: heap nodes [NL, 2NL), leaf j holds the cells
// cperm[kLeaf*(j-NL) .. +kLeaf).  Empty leaves get an inverted box.
__global__ void k_leaf_boxes(int64_t n_items, int64_t NL, const uint32_t *perm, const double *aabb, double *nodes)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NL) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t t = kLeaf * j; t < kLeaf * (j + 1) && t < n_items; t++) {
        const double *bb = aabb + 6 * (perm ? (int64_t)perm[t] : t);
        for (int d = 0; d < 3; d++) {
            lo[d] = fmin(lo[d], bb[d]);
            hi[d] = fmax(hi[d], bb[3 + d]);
        }
    }
    double *o = nodes + 6 * (NL + j);
    for (int d = 0; d < 3; d++) {
        o[d] = lo[d];
        o[3 + d] = hi[d];
    }
}

// Box of every point a particle's support can reach: x +- 2h (1 + 1e-8), widened
// by 1e-15 (|x| + 2h) for the rounding of its ends, so that it meets every cell
// box that the candidate test below accepts.
__global__ void k_particle_boxes(int64_t n, const double *__restrict__ xyz, const double *__restrict__ h,
                                 double *__restrict__ pbox)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const double R = 2.0 * h[a] * (1.0 + 1e-8);
    for (int d = 0; d < 3; d++) {
        const double x = xyz[3 * a + d];
        const double pad = 1e-15 * (fabs(x) + R);
        pbox[6 * a + d] = (x - R) - pad;
        pbox[6 * a + 3 + d] = (x + R) + pad;
    }
}

__global__ void k_parent_boxes(int64_t first, int64_t count, double *nodes)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    int64_t i = first + t;
    const double *a = nodes + 6 * (2 * i), *b = nodes + 6 * (2 * i + 1);
    double *o = nodes + 6 * i;
    for (int d = 0; d < 3; d++) {
        o[d] = fmin(a[d], b[d]);
        o[3 + d] = fmax(a[3 + d], b[3 + d]);
    }
}

__device__ __forceinline__ double box_dist2(const double *bb, double px, double py, double pz)
{
    double dx = fmax(fmax(bb[0] - px, px - bb[3]), 0.0);
    double dy = fmax(fmax(bb[1] - py, py - bb[4]), 0.0);
    double dz = fmax(fmax(bb[2] - pz, pz - bb[5]), 0.0);
    return dx * dx + dy * dy + dz * dz;
}

// Candidates of every cell: the particles whose support ball (radius 2h, with
// a relative 1e-9 on its square) comes within the cell's bounding box.  The
// particles form an implicit complete binary tree (heap indices: children 2i,
// 2i+1) over leaves of 8 consecutive particles, each node holding the box of
// its particles' reach boxes.  A wavefront of 64 consecutive cells walks it as
// one packet: it descends into a node when the node's box meets any lane's
// cell box, and at a leaf each lane whose box meets the leaf box tests the
// leaf's particles.  Leaves are visited left to right, so each cell lists its
// particles in ascending order: the candidate list comes out cell-major with
// particles ascending, with no sort.  Particles stored in a spatially coherent
// order (Morton, Hilbert, as SPH codes keep them) give tight boxes; any order
// gives the same candidates.
// The walk also settles what it can without the exact test: accepted when
// the cell's whole bounding box lies within (1 - 1e-6) 2h of the particle, or
// when the ball about the cell's interior point g (radius rin) comes closer
// than (1 - 1e-9) 2h; dropped when the ball about g that contains the cell
// (radius rc) stays (1 + 1e-9) 2h or more away.  The margins exceed the
// rounding of every distance involved, so these decisions are the exact
// test's.  The rest are marked for the exact test.
// MODE 0 counts every cell's kept candidates (kept, marked, accepted) and
// stores the first K of them in buf (particle index, bit 31 = marked); MODE 1
// writes the candidates past the first K of the cells that have more, at
// their final places, with their marks and exact-test list entries.
template <int MODE>
__global__ void k_candidates(int64_t n_cells, const double *__restrict__ aabb, const double *__restrict__ centre,
                             const double *__restrict__ radii, int64_t n, const double *__restrict__ xyz,
                             const double *__restrict__ h, const double *__restrict__ nodes, int64_t NL,
                             int64_t *__restrict__ ccount, int64_t *__restrict__ ncount, int64_t *__restrict__ qcount,
                             const int64_t *__restrict__ coffs, const int64_t *__restrict__ noffs,
                             uint32_t *__restrict__ buf, int K, uint32_t *__restrict__ cand_c,
                             uint32_t *__restrict__ cand_p, uint8_t *__restrict__ flag, uint32_t *__restrict__ list,
                             unsigned *__restrict__ max_count)
{
    const int64_t c = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    bool active = c < n_cells;
    if (MODE == 1 && active) active = ccount[c] > K;
    if (MODE == 1 && __ballot(active) == 0) return;
    double lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    double gx = 0.0, gy = 0.0, gz = 0.0, rin = 0.0, rc = 0.0;
    if (active) {
        lo0 = aabb[6 * c];
        lo1 = aabb[6 * c + 1];
        lo2 = aabb[6 * c + 2];
        hi0 = aabb[6 * c + 3];
        hi1 = aabb[6 * c + 4];
        hi2 = aabb[6 * c + 5];
        gx = centre[3 * c];
        gy = centre[3 * c + 1];
        gz = centre[3 * c + 2];
        rin = radii[2 * c];
        rc = radii[2 * c + 1];
    }
    const double cb[6] = {lo0, lo1, lo2, hi0, hi1, hi2};
    int64_t count = 0, nmark = 0, nacc = 0;
    const int64_t out = (MODE == 1 && active) ? coffs[c] : 0;
    const int64_t nout = (MODE == 1 && active) ? noffs[c] : 0;
    uint32_t *mine = buf + (MODE == 0 ? c * (int64_t)K : 0);
    // The walk is a chain of dependent loads of node boxes (wave-uniform).  A
    // descent loads both children's boxes at once (adjacent in the heap), so
    // that a left child that is a leaf or not entered hands over to its right
    // sibling without a load.
    int64_t i = 1;
    double b[6], sib[6];
    bool have_sib = false;
    for (int d = 0; d < 6; d++) b[d] = nodes[6 + d];
    for (;;) {
        const bool hit = active && b[0] <= hi0 && lo0 <= b[3] && b[1] <= hi1 && lo1 <= b[4] && b[2] <= hi2 &&
                         lo2 <= b[5];
        const bool any = __ballot(hit) != 0;
        if (any && i < NL) {
            i = 2 * i;
            const double *nb = nodes + 6 * i;
            for (int d = 0; d < 6; d++) {
                b[d] = nb[d];
                sib[d] = nb[6 + d];
            }
            have_sib = true;
            continue;
        }
        if (hit) {
            const int64_t t0 = kLeaf * (i - NL);
            for (int64_t t = t0; t < t0 + kLeaf && t < n; t++) {
                const double px = xyz[3 * t], py = xyz[3 * t + 1], pz = xyz[3 * t + 2];
                const double r = 2.0 * h[t];
                const double r2 = r * r;
                if (box_dist2(cb, px, py, pz) > r2 * (1.0 + 1e-9)) continue;
                const double fx = fmax(fabs(lo0 - px), fabs(hi0 - px));
                const double fy = fmax(fabs(lo1 - py), fabs(hi1 - py));
                const double fz = fmax(fabs(lo2 - pz), fabs(hi2 - pz));
                const double dx = gx - px, dy = gy - py, dz = gz - pz;
                const double dg = sqrt(dx * dx + dy * dy + dz * dz);
                const bool ok = fx * fx + fy * fy + fz * fz < r2 * 0.999998 || dg - rin < r * (1.0 - 1e-9);
                if (!ok && dg - rc >= r * (1.0 + 1e-9)) continue;
                if (MODE == 0 && count < K) mine[count] = (uint32_t)t | (ok ? 0u : 0x80000000u);
                if (MODE == 1 && count >= K) {
                    cand_c[out + count] = (uint32_t)c;
                    cand_p[out + count] = (uint32_t)t;
                    flag[out + count] = ok ? 1 : 0;
                    if (!ok) list[nout + nmark] = (uint32_t)(out + count);
                }
                nmark += ok ? 0 : 1;
                nacc += ok ? 1 : 0;
                count++;
            }
        }
        if ((i & 1) == 0 && have_sib) {  // the right sibling, loaded with this node
            i += 1;
            for (int d = 0; d < 6; d++) b[d] = sib[d];
            have_sib = false;
            continue;
        }
        while (i & 1) i >>= 1;
        if (i == 0) break;
        i += 1;
        for (int d = 0; d < 6; d++) b[d] = nodes[6 * i + d];
        have_sib = false;
    }
    if (MODE == 0) {
        if (active) {
            ccount[c] = count;
            ncount[c] = nmark;
            qcount[c] = nacc;
        }
        unsigned m = (unsigned)(count < 0xffffffffLL ? count : 0xffffffffLL);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
        if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(max_count, m);
    }
}

// The first K candidates of every cell from buf to their places in the
// cell-major candidate list, with their marks and exact-test list entries (in
// candidate order), one wavefront per cell.
__global__ void k_cand_gather(int64_t n_cells, int K, const int64_t *__restrict__ ccount,
                              const int64_t *__restrict__ coffs, const int64_t *__restrict__ noffs,
                              const uint32_t *__restrict__ buf, uint32_t *__restrict__ cand_c,
                              uint32_t *__restrict__ cand_p, uint8_t *__restrict__ flag, uint32_t *__restrict__ list)
{
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= n_cells) return;
    const int64_t cnt = ccount[c] < K ? ccount[c] : K;
    const int64_t o = coffs[c];
    int64_t nl = noffs[c];
    for (int64_t k0 = 0; k0 < cnt; k0 += 64) {
        const int64_t k = k0 + lane;
        const bool valid = k < cnt;
        const uint32_t e = valid ? buf[c * K + k] : 0u;
        const bool marked = valid && (e >> 31) != 0;
        const unsigned long long m = __ballot(marked);
        if (valid) {
            cand_c[o + k] = (uint32_t)c;
            cand_p[o + k] = e & 0x7fffffffu;
            flag[o + k] = marked ? 0 : 1;
        }
        if (marked) {
            const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            list[nl + below] = (uint32_t)(o + k);
        }
        nl += __popcll(m);
    }
}

// Pairs per cell: accepted by the walk's tests plus accepted by the exact test.
__global__ void k_pair_counts(int64_t n_cells, const int64_t *__restrict__ qcount, const unsigned *__restrict__ ecount,
                              int64_t *__restrict__ pcount)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n_cells) pcount[c] = qcount[c] + (int64_t)ecount[c];
}

// Accepted candidates of each cell to the cell-major pair list (candidate
// order kept), one wavefront per cell.
__global__ void k_compact(int64_t n_cells, const int64_t *__restrict__ coffs, const int64_t *__restrict__ coff,
                          const uint32_t *__restrict__ cand_p, const uint8_t *__restrict__ flag,
                          uint32_t *__restrict__ pair_c, uint32_t *__restrict__ pair_p)
{
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= n_cells) return;
    const int64_t b = coffs[c], e = coffs[c + 1];
    int64_t o = coff[c];
    for (int64_t k0 = b; k0 < e; k0 += 64) {
        const int64_t k = k0 + lane;
        const bool take = k < e && flag[k] != 0;
        const unsigned long long m = __ballot(take);
        if (take) {
            const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            pair_c[o + below] = (uint32_t)c;
            pair_p[o + below] = cand_p[k];
        }
        o += __popcll(m);
    }
}


__global__ void k_set_u64(unsigned long long *p, unsigned long long v)
{
    if (threadIdx.x == 0) *p = v;
}


// Exact test of the listed candidates, one wavefront per 64 consecutive list
// entries (the list is in cell order).  The wavefront stages each distinct
// cell of its entries in LDS; each lane then (1) runs the exact test's plane
// pass (inside: accept; a wall plane beyond the radius by the relative margin:
// reject), (2) computes the squared distance D to the cell in FP32 about the
// cell centre (least over the walls seen from outside of d^2 when the foot
// point is inside the wall polygon, else of the squared distances to the
// wall's edge segments) and decides when |D - r^2| exceeds a bound on its
// rounding, tol = 1e-6 (r + 2 rc)^2 (every vector involved is shorter than
// r + 2 rc, FP32 rounding of D is below 10 u (r + 2 rc)^2), and (3) runs the
// exact test from the global tables for the rest (D within tol of r^2) and
// for cells too large for the staging area.
__global__ void __launch_bounds__(256) k_exact(int64_t n_need, const uint32_t *__restrict__ list,
                                               const uint32_t *__restrict__ cand_c, const uint32_t *__restrict__ cand_p,
                                               const double *__restrict__ xyz, const double *__restrict__ h,
                                               const int64_t *__restrict__ cfo, const int64_t *__restrict__ fvo,
                                               const EdgeRec *__restrict__ edges, const double *__restrict__ plane,
                                               const double *__restrict__ centre, const double *__restrict__ radii,
                                               uint8_t *__restrict__ flag, unsigned *__restrict__ ecount)
{
#pragma clang fp contract(off)
    __shared__ CellFast stage[4];
    CellFast &L = stage[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = t < n_need;
    int64_t i = 0, c = -1, a = 0;
    double px = 0.0, py = 0.0, pz = 0.0, r2 = 0.0, r = 0.0;
    if (valid) {
        i = list[t];
        c = cand_c[i];
        a = cand_p[i];
        px = xyz[3 * a];
        py = xyz[3 * a + 1];
        pz = xyz[3 * a + 2];
        r = 2.0 * h[a];
        r2 = r * r;
    }
    bool hit = false;
    unsigned long long todo = __ballot(valid);
    while (todo != 0) {
        const int leader = __builtin_ctzll(todo);
        const int64_t cc = (int64_t)__shfl((long long)c, leader, 64);
        const bool mine = valid && c == cc;
        todo &= ~__ballot(mine);
        const int64_t j0 = cfo[cc], nf = cfo[cc + 1] - j0;
        const int64_t s0 = fvo[j0], ns = fvo[j0 + nf] - s0;
        const double gx = centre[3 * cc], gy = centre[3 * cc + 1], gz = centre[3 * cc + 2];
        bool exact = mine;
        if (nf <= kExactMaxFaces && ns <= kExactMaxSlots) {
            lds_sync_wave();
            for (int q = lane; q < 4 * nf; q += 64) L.pl_[q >> 2][q & 3] = plane[4 * j0 + q];
            for (int q = lane; q <= nf; q += 64) L.so_[q] = (int)(fvo[j0 + q] - s0);
            for (int q = lane; q < ns; q += 64) {
                const EdgeRec &E = edges[s0 + q];
                L.a_[q] = make_float4((float)(E.vx - gx), (float)(E.vy - gy), (float)(E.vz - gz), (float)E.L);
                L.b_[q] = make_float4((float)E.ex, (float)E.ey, (float)E.ez, (float)E.mx);
                L.c_[q] = make_float2((float)E.my, (float)E.mz);
            }
            if (lane == 0) L.nf = (int)nf;
            lds_sync_wave();
            if (mine) {
                exact = false;
                // (1) the exact test's plane pass, same arithmetic
                double far = 0.0;
                bool inside = true;
                unsigned long long seen = 0;  // walls seen from outside
                for (int j = 0; j < nf; j++) {
                    const double d = L.pl_[j][3] - (L.pl_[j][0] * px + L.pl_[j][1] * py + L.pl_[j][2] * pz);
                    if (d < 0.0) {
                        inside = false;
                        seen |= 1ull << j;
                        if (-d > far) far = -d;
                    }
                }
                if (inside) {
                    hit = true;
                } else if (!(far * far > r2 * (1.0 + 1e-9))) {
                    // (2) screened distance in FP32 about g
                    const float qx = (float)(px - gx), qy = (float)(py - gy), qz = (float)(pz - gz);
                    float D = INFINITY;
                    for (unsigned long long sm = seen; sm != 0; sm &= sm - 1) {
                        const int j = __builtin_ctzll(sm);
                        const double d = L.pl_[j][3] - (L.pl_[j][0] * px + L.pl_[j][1] * py + L.pl_[j][2] * pz);
                        bool in_poly = true;
                        float Dj = INFINITY;
                        for (int k = L.so_[j]; k < L.so_[j + 1]; k++) {
                            const float4 A = L.a_[k], B = L.b_[k];
                            const float2 C = L.c_[k];
                            const float wx = qx - A.x, wy = qy - A.y, wz = qz - A.z;
                            in_poly = in_poly && fmaf(B.w, wx, fmaf(C.x, wy, C.y * wz)) >= 0.0f;
                            const float sp = fmaf(B.x, wx, fmaf(B.y, wy, B.z * wz));
                            const float tt = fminf(fmaxf(sp, 0.0f), A.w);
                            const float ux = fmaf(-tt, B.x, wx), uy = fmaf(-tt, B.y, wy), uz = fmaf(-tt, B.z, wz);
                            Dj = fminf(Dj, fmaf(ux, ux, fmaf(uy, uy, uz * uz)));
                        }
                        D = fminf(D, in_poly ? (float)(d * d) : Dj);
                    }
                    const double rr = r + 2.0 * radii[2 * cc + 1];
                    const double tol = 1e-6 * rr * rr;
                    if ((double)D < r2 - tol) hit = true;
                    else if (!((double)D > r2 + tol)) exact = true;
                }
            }
        }
        // (3) the exact test from the global tables
        if (exact) hit = cell_meets(px, py, pz, r2, cc, cfo, fvo, edges, plane);
    }
    if (valid) {
        flag[i] = hit ? 1 : 0;
        if (hit) atomicAdd(&ecount[c], 1u);
    }
}


// Segment offsets of sorted keys: off[v] = first i with keys[i] >= v, v = 0..n_seg.
__global__ void k_seg_offsets(int64_t n_items, const uint32_t *__restrict__ keys, int64_t n_seg,
                              int64_t *__restrict__ off)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n_items) return;
    const int64_t prev = i == 0 ? -1 : (int64_t)keys[i - 1];
    const int64_t cur = i == n_items ? n_seg : (int64_t)keys[i];
    for (int64_t v = prev + 1; v <= cur; v++) off[v] = i;
}

void build_particle_view(Workspace &ws, const uint32_t *pair_p, int64_t n_pairs, int64_t n, uint32_t *perm,
                         int64_t *poff, hipStream_t s)
{
    if (n_pairs == 0) {
        fill_zero_bytes(poff, sizeof(int64_t) * (n + 1), s);
        return;
    }
    uint32_t *key = ws.get<uint32_t>(S_KEY2, (size_t)n_pairs);
    EM_HIP(hipMemcpyAsync(key, pair_p, sizeof(uint32_t) * n_pairs, hipMemcpyDeviceToDevice, s));
    fill_iota_u32(perm, n_pairs, s);
    int bits = 1;
    while (bits < 32 && ((uint64_t)(n - 1) >> bits) != 0) bits++;
    radix_sort_u32(ws, key, perm, ws.get<uint32_t>(S_IOTA, (size_t)n_pairs), ws.get<uint32_t>(S_PC_PM, (size_t)n_pairs),
                   n_pairs, bits, s);
    hipLaunchKernelGGL(k_seg_offsets, dim3((unsigned)((n_pairs + 1 + 255) / 256)), dim3(256), 0, s, n_pairs,
                       (const uint32_t *)key, n, poff);
    EM_HIP(hipGetLastError());
}

PairSet build_pairs(Workspace &ws, const DevInputs &in, const double *aabb, const EdgeRec *edges,
                    int64_t *counters, hipStream_t s)
{
    PairSet ps;
    const int64_t n = in.n, nc = in.n_cells;
    int64_t *coff = ws.get<int64_t>(S_COFF, (size_t)nc + 1);
    ps.coff = coff;
    if (n == 0 || nc == 0) {
        fill_zero_bytes(coff, sizeof(int64_t) * (nc + 1), s);
        return ps;
    }
    for (int d = 0; d < 3; d++) {
        const double ext = in.box[3 + d] - in.box[d];
        EM_CHECK(ext > 0.0 && std::isfinite(ext), MAP_EINVAL, "box has non-positive extent");
    }
    // bounding-volume tree over the particles' reach boxes, leaves of 8 particles in storage order
    double *pbox = ws.get<double>(S_PBOX, (size_t)(6 * n));
    hipLaunchKernelGGL(k_particle_boxes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in.xyz, in.h, pbox);
    EM_HIP(hipGetLastError());
    int64_t nleaf = (n + kLeaf - 1) / kLeaf, NL = 1;
    while (NL < nleaf) NL <<= 1;
    double *nodes = ws.get<double>(S_BINOFF_G, (size_t)(12 * NL));
    hipLaunchKernelGGL(k_leaf_boxes, dim3((unsigned)((NL + 255) / 256)), dim3(256), 0, s, n, NL,
                       (const uint32_t *)nullptr, (const double *)pbox, nodes);
    EM_HIP(hipGetLastError());
    for (int64_t first = NL / 2; first >= 1; first /= 2) {
        hipLaunchKernelGGL(k_parent_boxes, dim3((unsigned)((first + 255) / 256)), dim3(256), 0, s, first, first,
                           nodes);
        EM_HIP(hipGetLastError());
    }

    // candidates per cell (tree walk with the cheap tests), cell-major with
    // particles ascending: one walk keeps the first K of each cell's
    // candidates; cells with more walk again
    int64_t *ccount = ws.get<int64_t>(S_PCNT, (size_t)nc);
    int64_t *coffs = ws.get<int64_t>(S_CCNT64, (size_t)(nc + 1));
    int64_t *ncount = ws.get<int64_t>(S_NCNT, (size_t)nc);
    int64_t *noffs = ws.get<int64_t>(S_NOFF, (size_t)(nc + 1));
    int64_t *qcount = ws.get<int64_t>(S_QCNT, (size_t)nc);
    // candidate slots per cell: at most 2^30 in all (4 GiB; 128 per cell at
    // 8.4 million cells), and in arena mode at most a quarter of the free
    // scratch (cells with more candidates walk again)
    const int64_t slot_cap = std::min<int64_t>(int64_t(1) << 30, (int64_t)std::min<size_t>(ws.arena_free() / 16, size_t(1) << 40));
    const int K = (int)std::max<int64_t>(32, std::min<int64_t>(512, slot_cap / nc));
    uint32_t *cbuf = ws.get<uint32_t>(S_CAND_BUF, (size_t)(nc * K));
    unsigned *cmax = ws.get<unsigned>(S_CAND_MAX, 64);
    fill_zero_bytes(cmax, sizeof(unsigned), s);
    const double *centre = aabb + 6 * nc, *radii = aabb + 9 * nc;
    const unsigned pb = 128;
    const unsigned pg = (unsigned)((nc + pb - 1) / pb);
    hipLaunchKernelGGL(k_candidates<0>, dim3(pg), dim3(pb), 0, s, nc, aabb, centre, radii, n, in.xyz, in.h,
                       (const double *)nodes, NL, ccount, ncount, qcount, (const int64_t *)nullptr,
                       (const int64_t *)nullptr, cbuf, K, (uint32_t *)nullptr, (uint32_t *)nullptr, (uint8_t *)nullptr,
                       (uint32_t *)nullptr, cmax);
    EM_HIP(hipGetLastError());
    scan_counts(ws, ccount, coffs, nc, s);
    scan_counts(ws, ncount, noffs, nc, s);
    int64_t ncand = 0, n_need = 0;
    unsigned max_cand = 0;
    EM_HIP(hipMemcpyAsync(&ncand, coffs + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(&n_need, noffs + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(&max_cand, cmax, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    stream_sync(s);
    EM_CHECK(ncand < (int64_t)UINT32_MAX, MAP_ENOMEM, "candidate count exceeds 2^32-1");
    uint32_t *cand_c = ws.get<uint32_t>(S_KEY2, (size_t)(ncand > 0 ? ncand : 1));
    uint32_t *cand_p = ws.get<uint32_t>(S_IOTA, (size_t)(ncand > 0 ? ncand : 1));
    uint8_t *flag = reinterpret_cast<uint8_t *>(ws.get<uint32_t>(S_F_PM, (size_t)(ncand / 4 + 1)));
    uint32_t *list = ws.get<uint32_t>(S_BINLIST, (size_t)(n_need > 0 ? n_need : 1));
    unsigned *ecount = ws.get<unsigned>(S_ECNT, (size_t)nc);
    fill_zero_bytes(ecount, sizeof(unsigned) * nc, s);
    if (ncand > 0) {
        hipLaunchKernelGGL(k_cand_gather, dim3((unsigned)((nc + 3) / 4)), dim3(256), 0, s, nc, K,
                           (const int64_t *)ccount, (const int64_t *)coffs, (const int64_t *)noffs,
                           (const uint32_t *)cbuf, cand_c, cand_p, flag, list);
        EM_HIP(hipGetLastError());
    }
    if ((int64_t)max_cand > K) {
        hipLaunchKernelGGL(k_candidates<1>, dim3(pg), dim3(pb), 0, s, nc, aabb, centre, radii, n, in.xyz, in.h,
                           (const double *)nodes, NL, ccount, ncount, qcount, (const int64_t *)coffs,
                           (const int64_t *)noffs, cbuf, K, cand_c, cand_p, flag, list, cmax);
        EM_HIP(hipGetLastError());
    }
    // the exact test of the marked candidates (listed in candidate order)
    if (n_need > 0) {
        hipLaunchKernelGGL(k_exact, dim3((unsigned)((n_need + 255) / 256)), dim3(256), 0, s, n_need,
                           (const uint32_t *)list, (const uint32_t *)cand_c, (const uint32_t *)cand_p, in.xyz, in.h,
                           in.cfo, in.fvo, edges, in.plane, centre, radii, flag, ecount);
        EM_HIP(hipGetLastError());
    }
    unsigned long long *cand = reinterpret_cast<unsigned long long *>(counters + C_CANDIDATES);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, cand, (unsigned long long)n_need);
    EM_HIP(hipGetLastError());
    // pairs per cell, their offsets, and the cell-major pair list
    int64_t *pcount = ws.get<int64_t>(S_PCNT2, (size_t)nc);
    hipLaunchKernelGGL(k_pair_counts, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, nc,
                       (const int64_t *)qcount, (const unsigned *)ecount, pcount);
    EM_HIP(hipGetLastError());
    scan_counts(ws, pcount, coff, nc, s);
    int64_t np = 0;
    EM_HIP(hipMemcpyAsync(&np, coff + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    stream_sync(s);
    EM_CHECK(np < (int64_t)UINT32_MAX, MAP_ENOMEM, "pair count exceeds 2^32-1");
    ps.n_pairs = np;
    if (np == 0) return ps;
    uint32_t *pair_c = ws.get<uint32_t>(S_PAIR_C, (size_t)np);
    uint32_t *pair_p = ws.get<uint32_t>(S_PAIR_P, (size_t)np);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)((nc + 3) / 4)), dim3(256), 0, s, nc, (const int64_t *)coffs,
                       (const int64_t *)coff, (const uint32_t *)cand_p, (const uint8_t *)flag, pair_c, pair_p);
    EM_HIP(hipGetLastError());
    ps.pair_c = pair_c;
    ps.pair_p = pair_p;
    return ps;
}

}  // namespace em
