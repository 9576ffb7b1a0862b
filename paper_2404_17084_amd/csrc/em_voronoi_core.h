// Box-clipped Voronoi cell of one site (Sec. II-A: the grid whose generating
// sites are the particle positions): the cell representation, the box, the
// site-tree tests and the serial candidate walk, host- and device-callable.
// The construction itself runs one wavefront per cell (em_voronoi.hip).
//
// The cell is held as the dual of a convex polyhedron: a list of planes
// (n.x <= d in coordinates centred on the site, n not normalised) and a list
// of triangles (a, b, c) of plane indices, one per polyhedron vertex (the
// point where the three planes meet), oriented so that det(n_a, n_b, n_c) > 0;
// every dual edge then appears once in each direction.  The cell starts as the
// box (6 planes, 8 triangles) and is cut by bisector planes of other sites:
// the triangles whose vertex lies beyond the plane are removed, and every edge
// (x, y) of a removed triangle whose reverse belongs to a kept triangle gets a
// new triangle (x, y, P).  This is the dual-triangle clipping of Ray, Sokolov,
// Lefebvre and Levy ("Meshless Voronoi on the GPU", ACM Trans. Graph. 2018).  Sites are taken nearest first (a tree of the sites
// sorted by Morton key, leaves of 8), in passes that only consider sites whose
// bisector can still reach the cell's bounding box; once the next site is at
// least twice as far as the farthest vertex, no other site can cut the cell
// (the bisector of a site at distance D lies D/2 from the site).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace em {
namespace vor {

constexpr int kMaxPlanes = 64;   // 6 walls + 58 neighbours
constexpr int kMaxTris = 128;    // vertices (2 faces - 4 for a simple polyhedron)
constexpr int kMaxCand = 64;     // candidate sites taken per pass
constexpr int kLeaf = 8;         // sites per leaf of the site tree
constexpr double kEps = 1e-12;   // a vertex within this distance of a cutting plane is on it

enum : int32_t { ST_OK = 0, ST_PLANES = 1, ST_TRIS = 2, ST_PASSES = 3, ST_FACE = 4 };

struct Plane {
    double nx, ny, nz, d;
};

// A built cell as the extraction pass reads it (device memory, one per site).
struct Cell {
    Plane pl[kMaxPlanes];
    int32_t src[kMaxPlanes];  // site (input index) across the plane, or -1 - wall
    uint32_t tri[kMaxTris];   // a | b << 8 | c << 16
    double vx[kMaxTris], vy[kMaxTris], vz[kMaxTris];
    int32_t np, nt, status, pad;
};

__host__ __device__ inline uint32_t tri_pack(int a, int b, int c)
{
    return (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)c << 16);
}
__host__ __device__ inline int tri_a(uint32_t t) { return (int)(t & 255u); }
__host__ __device__ inline int tri_b(uint32_t t) { return (int)((t >> 8) & 255u); }
__host__ __device__ inline int tri_c(uint32_t t) { return (int)((t >> 16) & 255u); }

// the point where three planes meet
__host__ __device__ inline void meet(const Plane &A, const Plane &B, const Plane &C, double &x, double &y, double &z)
{
    const double bcx = B.ny * C.nz - B.nz * C.ny, bcy = B.nz * C.nx - B.nx * C.nz, bcz = B.nx * C.ny - B.ny * C.nx;
    const double cax = C.ny * A.nz - C.nz * A.ny, cay = C.nz * A.nx - C.nx * A.nz, caz = C.nx * A.ny - C.ny * A.nx;
    const double abx = A.ny * B.nz - A.nz * B.ny, aby = A.nz * B.nx - A.nx * B.nz, abz = A.nx * B.ny - A.ny * B.nx;
    const double det = A.nx * bcx + A.ny * bcy + A.nz * bcz;
    x = (A.d * bcx + B.d * cax + C.d * abx) / det;
    y = (A.d * bcy + B.d * cay + C.d * aby) / det;
    z = (A.d * bcz + B.d * caz + C.d * abz) / det;
}

template <class CellT>
__host__ __device__ inline void set_vertex(CellT &C, int t)
{
    const uint32_t q = C.tri[t];
    meet(C.pl[tri_a(q)], C.pl[tri_b(q)], C.pl[tri_c(q)], C.vx[t], C.vy[t], C.vz[t]);
}

// the box [lo, hi] around site s: planes 0..5 = x-, x+, y-, y+, z-, z+
template <class CellT>
__host__ __device__ inline void init_box(CellT &C, const double *box, double sx, double sy, double sz)
{
    const double s[3] = {sx, sy, sz};
    for (int ax = 0; ax < 3; ax++)
        for (int side = 0; side < 2; side++) {
            Plane &P = C.pl[2 * ax + side];
            P.nx = P.ny = P.nz = 0.0;
            const double sg = side ? 1.0 : -1.0;
            if (ax == 0) P.nx = sg;
            if (ax == 1) P.ny = sg;
            if (ax == 2) P.nz = sg;
            P.d = side ? box[3 + ax] - s[ax] : s[ax] - box[ax];
            C.src[2 * ax + side] = -1 - (2 * ax + side);
        }
    C.np = 6;
    C.nt = 0;
    for (int k = 0; k < 8; k++) {
        const int px = k & 1, py = (k >> 1) & 1, pz = (k >> 2) & 1;
        const int a = px, b = 2 + py, c = 4 + pz;
        // det(n_a, n_b, n_c) = product of the three signs
        const int sgn = (px ? 1 : -1) * (py ? 1 : -1) * (pz ? 1 : -1);
        C.tri[C.nt] = sgn > 0 ? tri_pack(a, b, c) : tri_pack(a, c, b);
        set_vertex(C, C.nt);
        C.nt++;
    }
    C.status = ST_OK;
}

__host__ __device__ inline double box_gap2(const double *bb, double px, double py, double pz)
{
    const double dx = fmax(fmax(bb[0] - px, px - bb[3]), 0.0);
    const double dy = fmax(fmax(bb[1] - py, py - bb[4]), 0.0);
    const double dz = fmax(fmax(bb[2] - pz, pz - bb[5]), 0.0);
    return dx * dx + dy * dy + dz * dz;
}

// Key order of the candidate sites: squared distance, then sorted index.
__host__ __device__ inline bool key_less(double d2, int64_t q, double e2, int64_t r)
{
    return d2 < e2 || (d2 == e2 && q < r);
}

template <class CellT>
__host__ __device__ inline void heap_down(CellT &C, int k, int cnt)
{
    for (;;) {
        const int l = 2 * k + 1, r = l + 1;
        int m = k;
        if (l < cnt && key_less(C.cd2[m], C.cand[m], C.cd2[l], C.cand[l])) m = l;
        if (r < cnt && key_less(C.cd2[m], C.cand[m], C.cd2[r], C.cand[r])) m = r;
        if (m == k) return;
        const double td = C.cd2[k];
        const int32_t tq = C.cand[k];
        C.cd2[k] = C.cd2[m];
        C.cand[k] = C.cand[m];
        C.cd2[m] = td;
        C.cand[m] = tq;
        k = m;
    }
}

// Support of the cell's bounding box [lo, hi] (site-centred) along w:
// max over the box of w.x, the largest reach of any vertex along w.
__host__ __device__ inline double reach(const double *lo, const double *hi, double wx, double wy, double wz)
{
    return fmax(wx * lo[0], wx * hi[0]) + fmax(wy * lo[1], wy * hi[1]) + fmax(wz * lo[2], wz * hi[2]);
}

// The (up to kMaxCand) nearest sorted sites, in key order (|p - s|^2, then
// index), whose key follows (lo2, lo_q) and whose bisector can reach the
// cell's bounding box [blo, bhi] (a site at offset w cuts only if some vertex
// v has w.v > |w|^2 / 2, and w.v is at most the box's reach along w); *more is
// set when further sites qualified.  A tree box is skipped when no offset in
// it can reach (its least |w|^2 / 2 is at least the largest reach over it,
// the reach being separable and convex), or when the list is full and the box
// is farther than its farthest entry.  The list is a max-heap on the key
// during the walk, sorted at the end.  Tree: heap of 2 NL boxes (6 doubles
// each; leaves NL + j hold sites kLeaf j .. kLeaf j + 7).
template <class CellT>
__host__ __device__ inline int collect(CellT &C, const double *ps, int64_t n, const double *bx, int64_t NL,
                                       int64_t self, double sx, double sy, double sz, double lo2, int64_t lo_q,
                                       double hi2, const double *blo, const double *bhi, bool *more, int64_t *stack)
{
    int cnt = 0;
    *more = false;
    // depth-first, nearer child first; the stack (64 entries) holds at most
    // one pending sibling per level
    int sp = 0;
    stack[sp++] = 1;
    while (sp > 0) {
        const int64_t i = stack[--sp];
        const double *b = bx + 6 * i;
        const double g2 = box_gap2(b, sx, sy, sz);
        bool visit = g2 < hi2 && !(cnt == kMaxCand && g2 > C.cd2[0]);
        if (visit) {
            const double ax = b[0] - sx, bxx = b[3] - sx, ay = b[1] - sy, by = b[4] - sy, az = b[2] - sz, bz = b[5] - sz;
            const double gm = fmax(fmax(ax * blo[0], ax * bhi[0]), fmax(bxx * blo[0], bxx * bhi[0])) +
                              fmax(fmax(ay * blo[1], ay * bhi[1]), fmax(by * blo[1], by * bhi[1])) +
                              fmax(fmax(az * blo[2], az * bhi[2]), fmax(bz * blo[2], bz * bhi[2]));
            visit = 0.5 * g2 < gm;
        } else if (cnt == kMaxCand && g2 < hi2) {
            *more = true;  // a box skipped for distance may hold qualifying sites
        }
        if (!visit) continue;
        if (i < NL) {
            const double gl = box_gap2(bx + 6 * (2 * i), sx, sy, sz), gr = box_gap2(bx + 6 * (2 * i + 1), sx, sy, sz);
            if (sp + 2 > 64) {  // cannot happen for trees of fewer than 2^62 leaves
                C.status = ST_PASSES;
                return 0;
            }
            stack[sp++] = gl <= gr ? 2 * i + 1 : 2 * i;  // farther child later
            stack[sp++] = gl <= gr ? 2 * i : 2 * i + 1;
            continue;
        }
        const int64_t j = i - NL;
        for (int64_t q = kLeaf * j; q < kLeaf * (j + 1) && q < n; q++) {
            if (q == self) continue;
            const double dx = ps[3 * q] - sx, dy = ps[3 * q + 1] - sy, dz = ps[3 * q + 2] - sz;
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (!(d2 < hi2) || !key_less(lo2, lo_q, d2, q) || !(0.5 * d2 < reach(blo, bhi, dx, dy, dz))) continue;
            if (cnt < kMaxCand) {  // push, sift up
                int k = cnt++;
                while (k > 0) {
                    const int pa = (k - 1) / 2;
                    if (!key_less(C.cd2[pa], C.cand[pa], d2, q)) break;
                    C.cd2[k] = C.cd2[pa];
                    C.cand[k] = C.cand[pa];
                    k = pa;
                }
                C.cd2[k] = d2;
                C.cand[k] = (int32_t)q;
            } else {
                *more = true;
                if (key_less(d2, q, C.cd2[0], C.cand[0])) {  // replace the farthest kept
                    C.cd2[0] = d2;
                    C.cand[0] = (int32_t)q;
                    heap_down(C, 0, cnt);
                }
            }
        }
    }
    for (int end = cnt - 1; end > 0; end--) {  // heap sort: ascending keys
        const double td = C.cd2[0];
        const int32_t tq = C.cand[0];
        C.cd2[0] = C.cd2[end];
        C.cand[0] = C.cand[end];
        C.cd2[end] = td;
        C.cand[end] = tq;
        heap_down(C, 0, end);
    }
    return cnt;
}

}  // namespace vor
}  // namespace em
