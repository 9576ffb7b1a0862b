// Pseudo-particle front end (Sec. III): gravity tree, adaptive walk, node
// smoothing lengths.
//
// Tree (Sec. III-A).  An octree over 63-bit Morton keys (21 bits per axis,
// octal digits (x, y, z) from the most significant).  Particles are sorted by
// key; dlev[i] is the first level at which particles i-1 and i sit in
// different nodes, so a level-L node is a maximal run of particles of one
// internal level-(L-1) node with no dlev <= L inside.  Levels are built one at
// a time from segment flags and a scan; a node is a leaf when it holds at most
// leaf_size particles or L = 21.  Masses and mass-weighted positions are summed
// bottom-up (leaves over their particles, internal nodes over their children,
// each in Morton order); the size s (distance from the centre of mass to the
// furthest member) is a max over the node's particles, by one thread for
// small nodes and by wavefront chunks with an order-independent max for big
// ones.
//
// Walk (Sec. III-B, Eq. (5)).  Every node's opening decision depends only on
// the node and the sources, so all are taken at once; a node is visible when
// all its ancestors are open.  Visible unopened nodes are pseudo-particles;
// visible leaves opened by r_part give their particles.  Both are compacted
// in Morton order of their first particle by a scan over the sorted
// particles.
//
// Smoothing lengths (Sec. III-C, Eq. (7)-(9)).  The number sum
// N(h) = (1/pi) sum_b w(|x - x_b| / h) runs over the node pseudo-particles and
// the leaves standing in for extracted particles, grouped 8 per box in Morton
// order.  One wavefront per node solves N(h) = h_fact^3 by Newton steps kept
// inside a bisection bracket, stopping once a step no longer moves the
// iterate; each evaluation tests the boxes listed within 2h (64 per step),
// each lane sums its box's points in point order, and the box sums are added
// in box order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "em_internal.h"
#include "em_wave.h"

namespace em {
namespace {

constexpr int kPtLeaf = 8;         // points per leaf of the h-solve tree
constexpr int kMaxLevel = 21;
constexpr int64_t kSmallNode = 64; // nodes up to this size get their s from one thread
constexpr int64_t kChunk = 512;    // particles per wavefront item for bigger nodes

__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

__device__ __forceinline__ uint64_t axis21(double x, double lo, double ext)
{
#pragma clang fp contract(off)
    const double t = ((x - lo) / ext) * 2097152.0;
    if (!(t > 0.0)) return 0;
    if (t >= 2097151.0) return 2097151ULL;
    return (uint64_t)floor(t);
}

struct BoxIn {
    double lo[3], ext[3];
};

__global__ void k_check_particles(int64_t n, const double *__restrict__ xyz, const double *__restrict__ m,
                                  const double *__restrict__ h, unsigned *flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned f = 0;
    if (!isfinite(xyz[3 * i]) || !isfinite(xyz[3 * i + 1]) || !isfinite(xyz[3 * i + 2])) f |= F_PART_NONFINITE;
    if (!(h[i] > 0.0) || !isfinite(h[i])) f |= F_H_NONPOS;
    if (!(m[i] > 0.0) || !isfinite(m[i])) f |= F_M_BAD;
    if (f) atomicOr(flags, f);
}

__global__ void k_keys(int64_t n, const double *__restrict__ xyz, BoxIn B, uint64_t *__restrict__ key,
                       uint32_t *__restrict__ idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t ix = axis21(xyz[3 * i], B.lo[0], B.ext[0]);
    const uint64_t iy = axis21(xyz[3 * i + 1], B.lo[1], B.ext[1]);
    const uint64_t iz = axis21(xyz[3 * i + 2], B.lo[2], B.ext[2]);
    key[i] = (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
    idx[i] = (uint32_t)i;
}

// sorted particles: (x, y, z, m); dlev = first level where i-1 and i differ
__global__ void k_sorted(int64_t n, const uint32_t *__restrict__ perm, const uint64_t *__restrict__ key,
                         const double *__restrict__ xyz, const double *__restrict__ m, double4 *__restrict__ pos,
                         uint8_t *__restrict__ dlev)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = perm[i];
    pos[i] = make_double4(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], m[a]);
    int d = 0;
    if (i > 0) {
        const uint64_t x = key[i - 1] ^ key[i];
        d = x ? (__clzll((long long)x) - 1) / 3 + 1 : kMaxLevel + 1;
    }
    dlev[i] = (uint8_t)d;
}

// Node table (structure of arrays, capacity `cap`).
struct Nodes {
    int32_t *start, *end, *parent, *cb, *ce;
    uint8_t *level, *leaf, *open, *vis;
    uint64_t *label;
    double *msum, *mx, *my, *mz;
    double *com;       // 3 per node
    uint64_t *d2;      // bits of the largest squared member distance
};

__global__ void k_root(int64_t n, int leaf_size, Nodes T, int32_t *__restrict__ cur, int32_t *__restrict__ leaf_of)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool leaf = n <= leaf_size;
    if (i == 0) {
        T.start[0] = 0;
        T.end[0] = (int32_t)n;
        T.parent[0] = -1;
        T.level[0] = 0;
        T.leaf[0] = leaf;
        T.label[0] = 1;
    }
    if (i < n) {
        cur[i] = leaf ? -1 : 0;
        leaf_of[i] = leaf ? 0 : -1;
    }
}

__global__ void k_lv_flags(int64_t n, int L, const int32_t *__restrict__ cur, const uint8_t *__restrict__ dlev,
                           int64_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cur[i];
    flag[i] = (c >= 0 && (i == 0 || cur[i - 1] != c || dlev[i] <= L)) ? 1 : 0;
}

// Level state on the device (so a level needs one host read, at its end):
// lv[0] internal nodes of the level, lv[1] nodes of the level, lv[2] set when
// the node table would overflow (the level's kernels then write nothing),
// lv[3] index of the level's first node.
__global__ void k_lv_init(unsigned *lv)
{
    lv[0] = 0u;
    lv[1] = 0u;
    lv[2] = 0u;
    lv[3] = 1u;
}

__global__ void k_lv_count(int64_t n, const int64_t *__restrict__ off, int32_t cap, unsigned *lv)
{
    const int64_t cnt = off[n];
    lv[0] = 0u;
    lv[1] = (unsigned)cnt;
    if ((int64_t)lv[3] + cnt > (int64_t)cap) lv[2] = 1u;
}

__global__ void k_lv_advance(unsigned *lv)
{
    if (!lv[2]) lv[3] += lv[1];
}

__global__ void k_lv_nodes(int64_t n, int L, const unsigned *__restrict__ lv, const int32_t *__restrict__ cur,
                           const int64_t *__restrict__ flag, const int64_t *__restrict__ off,
                           const uint64_t *__restrict__ key, Nodes T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || lv[2]) return;
    const int32_t c = cur[i];
    if (c < 0) return;
    const int32_t nid = (int32_t)lv[3] + (int32_t)(off[i] + flag[i] - 1);
    if (flag[i]) {
        T.start[nid] = (int32_t)i;
        T.parent[nid] = c;
        T.level[nid] = (uint8_t)L;
        T.label[nid] = (1ULL << (3 * L)) | (key[i] >> (63 - 3 * L));
    }
    if (i + 1 == n || cur[i + 1] != c || flag[i + 1]) T.end[nid] = (int32_t)(i + 1);
}

__global__ void k_lv_leaf(int L, int leaf_size, Nodes T, unsigned *lv)
{
    const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    bool inner = false;
    if (!lv[2] && t < (int32_t)lv[1]) {
        const int32_t i = (int32_t)lv[3] + t;
        const bool leaf = (T.end[i] - T.start[i] <= leaf_size) || L == kMaxLevel;
        T.leaf[i] = leaf;
        inner = !leaf;
    }
    const unsigned long long b = __ballot(inner);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(lv, (unsigned)__popcll(b));
}

__global__ void k_lv_cur(int64_t n, const unsigned *__restrict__ lv, const int64_t *__restrict__ flag,
                         const int64_t *__restrict__ off, const uint8_t *__restrict__ leaf, int32_t *__restrict__ cur,
                         int32_t *__restrict__ leaf_of)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || lv[2] || cur[i] < 0) return;
    const int32_t nid = (int32_t)lv[3] + (int32_t)(off[i] + flag[i] - 1);
    if (leaf[nid]) {
        leaf_of[i] = nid;
        cur[i] = -1;
    } else {
        cur[i] = nid;
    }
}

// children of a node are consecutive in the next level
__global__ void k_children(int32_t n_nodes, Nodes T)
{
    const int32_t c = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c < 1 || c >= n_nodes) return;
    const int32_t p = T.parent[c];
    if (T.parent[c - 1] != p) T.cb[p] = c;
    if (c + 1 == n_nodes || T.parent[c + 1] != p) T.ce[p] = c + 1;
}

// masses and mass-weighted positions of the nodes of one level
__global__ void k_moments(int32_t lo, int32_t hi, const double4 *__restrict__ pos, Nodes T)
{
#pragma clang fp contract(off)
    const int32_t i = lo + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= hi) return;
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    if (T.leaf[i]) {
        for (int32_t k = T.start[i]; k < T.end[i]; k++) {
            const double4 p = pos[k];
            M += p.w;
            sx += p.w * p.x;
            sy += p.w * p.y;
            sz += p.w * p.z;
        }
    } else {
        for (int32_t c = T.cb[i]; c < T.ce[i]; c++) {
            M += T.msum[c];
            sx += T.mx[c];
            sy += T.my[c];
            sz += T.mz[c];
        }
    }
    T.msum[i] = M;
    T.mx[i] = sx;
    T.my[i] = sy;
    T.mz[i] = sz;
    T.com[3 * i] = sx / M;
    T.com[3 * i + 1] = sy / M;
    T.com[3 * i + 2] = sz / M;
}

__device__ __forceinline__ double dist2(double ax, double ay, double az, double bx, double by, double bz)
{
#pragma clang fp contract(off)
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return dx * dx + dy * dy + dz * dz;
}

// s of small nodes (one thread each); big nodes get items
__global__ void k_size_small(int32_t n_nodes, const double4 *__restrict__ pos, Nodes T, int64_t *__restrict__ items)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_nodes) return;
    const int64_t cnt = T.end[i] - T.start[i];
    if (cnt > kSmallNode) {
        items[i] = (cnt + kChunk - 1) / kChunk;
        T.d2[i] = 0;
        return;
    }
    items[i] = 0;
    const double cx = T.com[3 * i], cy = T.com[3 * i + 1], cz = T.com[3 * i + 2];
    double best = 0.0;
    for (int32_t k = T.start[i]; k < T.end[i]; k++) {
        const double4 p = pos[k];
        const double d = dist2(p.x, p.y, p.z, cx, cy, cz);
        if (d > best) best = d;
    }
    T.d2[i] = __double_as_longlong(best);
}

__global__ void k_size_items(int32_t n_nodes, const int64_t *__restrict__ ioff, uint64_t *__restrict__ item)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_nodes) return;
    for (int64_t j = ioff[i]; j < ioff[i + 1]; j++) item[j] = ((uint64_t)i << 32) | (uint64_t)(j - ioff[i]);
}

// one wavefront per item: max squared distance over a chunk, then an atomic max
// on the bit pattern (non-negative doubles order like their bits)
__global__ void k_size_big(int64_t n_items, const uint64_t *__restrict__ item, const double4 *__restrict__ pos,
                           Nodes T)
{
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= n_items) return;
    const uint64_t it = item[w];
    const int32_t i = (int32_t)(it >> 32);
    const int64_t k0 = T.start[i] + (int64_t)(it & 0xffffffffu) * kChunk;
    const int64_t k1 = k0 + kChunk < T.end[i] ? k0 + kChunk : T.end[i];
    const double cx = T.com[3 * i], cy = T.com[3 * i + 1], cz = T.com[3 * i + 2];
    double best = 0.0;
    for (int64_t k = k0 + lane; k < k1; k += 64) {
        const double4 p = pos[k];
        const double d = dist2(p.x, p.y, p.z, cx, cy, cz);
        if (d > best) best = d;
    }
    for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
    if (lane == 0) atomicMax((unsigned long long *)&T.d2[i], (unsigned long long)__double_as_longlong(best));
}

struct Walk {
    double src[3 * 64];
    int n_src;
    double theta, r_part, r_leaf;
    // forced openings (re-walk): sorted labels of nodes that failed the
    // resolution check, and remembered regions (cx, cy, cz, R, s_min)
    const uint64_t *open;
    int64_t n_open;
    const double *reg;
    int64_t n_reg;
};

__device__ __forceinline__ double src_dist(const Walk *W, double x, double y, double z)
{
    double r = INFINITY;
    for (int k = 0; k < W->n_src; k++) {
        const double d = sqrt(dist2(x, y, z, W->src[3 * k], W->src[3 * k + 1], W->src[3 * k + 2]));
        if (d < r) r = d;
    }
    return r;
}

// an internal node opened by a failed check (label listed) or by a region it
// comes within (|com - c| - s < R) while larger than the region's s_min
__device__ __forceinline__ bool forced_open(const Walk *W, uint64_t label, double cx, double cy, double cz, double s)
{
#pragma clang fp contract(off)
    int64_t lo = 0, hi = W->n_open;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (W->open[mid] < label) lo = mid + 1;
        else hi = mid;
    }
    if (lo < W->n_open && W->open[lo] == label) return true;
    for (int64_t k = 0; k < W->n_reg; k++) {
        const double *g = W->reg + 5 * k;
        const double d = sqrt(dist2(cx, cy, cz, g[0], g[1], g[2]));
        if (d - s < g[3] && s > g[4]) return true;
    }
    return false;
}

// opening decision of every node; bit 0: opened, bit 1: leaf opened into particles
__global__ void k_open(int32_t n_nodes, const Walk *__restrict__ W, Nodes T)
{
#pragma clang fp contract(off)
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_nodes) return;
    const double cx = T.com[3 * i], cy = T.com[3 * i + 1], cz = T.com[3 * i + 2];
    const double r = src_dist(W, cx, cy, cz);
    const double s = sqrt(__longlong_as_double((long long)T.d2[i]));
    const bool in_part = r - s < W->r_part;
    const bool in_leaf = r - s < W->r_leaf;
    uint8_t o;
    if (T.leaf[i]) o = in_part ? 3 : 0;
    else o = (in_part || in_leaf || s > W->theta * r || forced_open(W, T.label[i], cx, cy, cz, s)) ? 1 : 0;
    T.open[i] = o;
}

// visible: every ancestor opened
__global__ void k_visible(int32_t n_nodes, Nodes T)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_nodes) return;
    uint8_t v = 1;
    for (int32_t j = T.parent[i]; j >= 0; j = T.parent[j])
        if (!(T.open[j] & 1)) {
            v = 0;
            break;
        }
    T.vis[i] = v;
}

// marks over the sorted particles: output slots (accepted node at its first
// particle, each extracted particle) and h-solve points (accepted nodes and
// substitute leaves, at their first particle); owner = node id, or -1 for a
// particle
__global__ void k_mark(int32_t n_nodes, Nodes T, int64_t *__restrict__ omark, int64_t *__restrict__ pmark,
                       int32_t *__restrict__ owner)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_nodes || !T.vis[i]) return;
    const uint8_t o = T.open[i];
    if (!(o & 1)) {
        omark[T.start[i]] = 1;
        pmark[T.start[i]] = 1;
        owner[T.start[i]] = i;
    } else if (o & 2) {
        for (int32_t k = T.start[i]; k < T.end[i]; k++) {
            omark[k] = 1;
            owner[k] = -1;
        }
        pmark[T.start[i]] = 1;
    }
}

// leaves, accepted nodes, substitute leaves and extracted particles
__global__ void k_walk_stats(int32_t n_nodes, Nodes T, unsigned long long *__restrict__ cnt)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    unsigned long long v[4] = {0, 0, 0, 0};
    if (i < n_nodes) {
        v[0] = T.leaf[i];
        if (T.vis[i]) {
            v[1] = !(T.open[i] & 1);
            if (T.open[i] & 2) {
                v[2] = 1;
                v[3] = (unsigned long long)(T.end[i] - T.start[i]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++)
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; q++)
            if (v[q]) atomicAdd(cnt + q, v[q]);
}

struct PseudoOut {
    double *xyz, *m, *h, *s;
    int32_t *kind;
    int64_t *ref;
    int32_t *node;  // tree node of a node pseudo-particle, -1 for a particle
};

// output records; the points of the h-solve and, for each point that is a
// pseudo node, its output slot (else -1)
__global__ void k_emit(int64_t n, const int64_t *__restrict__ omark, const int64_t *__restrict__ ooff,
                       const int64_t *__restrict__ pmark, const int64_t *__restrict__ poff,
                       const int32_t *__restrict__ owner, const int32_t *__restrict__ leaf_of,
                       const uint32_t *__restrict__ perm, const double *__restrict__ xyz,
                       const double *__restrict__ m, const double *__restrict__ h, Nodes T, PseudoOut O,
                       double4 *__restrict__ pts, int64_t *__restrict__ pt_slot, int32_t *__restrict__ pt_node)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (omark[i]) {
        const int64_t o = ooff[i];
        const int32_t nd = owner[i];
        if (nd >= 0) {
            O.xyz[3 * o] = T.com[3 * nd];
            O.xyz[3 * o + 1] = T.com[3 * nd + 1];
            O.xyz[3 * o + 2] = T.com[3 * nd + 2];
            O.m[o] = T.msum[nd];
            O.h[o] = 0.0;
            O.s[o] = sqrt(__longlong_as_double((long long)T.d2[nd]));
            O.kind[o] = MAP_PSEUDO_NODE;
            O.ref[o] = (int64_t)T.label[nd];
            O.node[o] = nd;
        } else {
            const int64_t a = perm[i];
            O.xyz[3 * o] = xyz[3 * a];
            O.xyz[3 * o + 1] = xyz[3 * a + 1];
            O.xyz[3 * o + 2] = xyz[3 * a + 2];
            O.m[o] = m[a];
            O.h[o] = h[a];
            O.s[o] = 0.0;
            O.kind[o] = MAP_PSEUDO_PARTICLE;
            O.ref[o] = a;
            O.node[o] = -1;
        }
    }
    if (pmark[i]) {
        const int64_t q = poff[i];
        const int32_t nd = omark[i] && owner[i] >= 0 ? owner[i] : leaf_of[i];
        pts[q] = make_double4(T.com[3 * nd], T.com[3 * nd + 1], T.com[3 * nd + 2], 0.0);
        const bool is_node = omark[i] && owner[i] >= 0;
        pt_slot[q] = is_node ? ooff[i] : -1;
        pt_node[q] = nd;
    }
}

// ---------------------------------------------------------------- h-solve
__global__ void k_pt_leaf_boxes(int64_t n_pts, int64_t NL, const double4 *__restrict__ pts, double *__restrict__ bx)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NL) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t t = kPtLeaf * j; t < kPtLeaf * (j + 1) && t < n_pts; t++) {
        const double4 p = pts[t];
        lo[0] = fmin(lo[0], p.x), hi[0] = fmax(hi[0], p.x);
        lo[1] = fmin(lo[1], p.y), hi[1] = fmax(hi[1], p.y);
        lo[2] = fmin(lo[2], p.z), hi[2] = fmax(hi[2], p.z);
    }
    double *o = bx + 6 * (NL + j);
    for (int d = 0; d < 3; d++) {
        o[d] = lo[d];
        o[3 + d] = hi[d];
    }
}

// boxes of the internal nodes [first, 2 first) of the point tree (heap order)
__global__ void k_pt_parent_boxes(int64_t first, double *__restrict__ bx)
{
    const int64_t i = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * first) return;
    const double *a = bx + 6 * (2 * i), *b = bx + 6 * (2 * i + 1);
    double *o = bx + 6 * i;
    for (int d = 0; d < 3; d++) {
        o[d] = fmin(a[d], b[d]);
        o[3 + d] = fmax(a[3 + d], b[3 + d]);
    }
}

__device__ __forceinline__ double box_gap2(const double *bb, double px, double py, double pz)
{
#pragma clang fp contract(off)
    const double dx = fmax(fmax(bb[0] - px, px - bb[3]), 0.0);
    const double dy = fmax(fmax(bb[1] - py, py - bb[4]), 0.0);
    const double dz = fmax(fmax(bb[2] - pz, pz - bb[5]), 0.0);
    return dx * dx + dy * dy + dz * dz;
}

// M4 shape w(q) and q w'(q), q < 2
__device__ __forceinline__ double m4_w(double q)
{
#pragma clang fp contract(off)
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    const double t = 2.0 - q;
    return 0.25 * t * t * t;
}

__device__ __forceinline__ double m4_qdw(double q)
{
    if (q < 1.0) return q * (-3.0 * q + 2.25 * q * q);
    const double t = 2.0 - q;
    return -0.75 * q * t * t;
}

struct NumSum {
    double sum_w, sum_qdw;
    int64_t count;
};

// The terms of one leaf's (up to 8) points, added in point order.
__device__ __forceinline__ NumSum leaf_terms(double px, double py, double pz, double h, int64_t n_pts,
                                            const double4 *__restrict__ pts, int64_t j)
{
#pragma clang fp contract(off)
    NumSum r{0.0, 0.0, 0};
#pragma unroll
    for (int k = 0; k < kPtLeaf; k++) {
        const int64_t t = kPtLeaf * j + k;
        if (t < n_pts) {
            const double4 p = pts[t];
            const double q = sqrt(dist2(px, py, pz, p.x, p.y, p.z)) / h;
            if (q < 2.0) {
                r.sum_w += m4_w(q);
                r.sum_qdw += m4_qdw(q);
                r.count++;
            }
        }
    }
    return r;
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Adds the leaf sums of the lanes in `mask` to r, in lane order.
__device__ __forceinline__ void add_leaf_sums(NumSum &r, const NumSum &mine, unsigned long long mask)
{
#pragma clang fp contract(off)
    while (mask) {
        const int l = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        r.sum_w += readlane_f64(mine.sum_w, l);
        r.sum_qdw += readlane_f64(mine.sum_qdw, l);
        r.count += __builtin_amdgcn_readlane((int)mine.count, l);
    }
}

// One wavefront evaluates the number sum for one node.  Lane l tests leaf
// base+l of the point tree and adds its points' terms in point order; the
// leaves' sums are then added in leaf order.  Leaves beyond the support add
// nothing, so the result does not depend on the launch shape nor on which
// other leaves are scanned (number_sum_list below gives the same bits).
__device__ NumSum number_sum_wave(double px, double py, double pz, double h, int64_t n_pts,
                                  const double4 *__restrict__ pts, const double *__restrict__ bx, int64_t NL,
                                  int64_t nleaf, int lane)
{
    NumSum r{0.0, 0.0, 0};
    const double R2 = 4.0 * h * h * (1.0 + 1e-9);
    for (int64_t base = 0; base < nleaf; base += 64) {
        const int64_t j = base + lane;
        NumSum mine{0.0, 0.0, 0};
        if (j < nleaf && box_gap2(bx + 6 * (NL + j), px, py, pz) <= R2)
            mine = leaf_terms(px, py, pz, h, n_pts, pts, j);
        add_leaf_sums(r, mine, __ballot(mine.count > 0));
    }
    return r;
}

constexpr int kFront = 512;  // nodes per level (and listed leaves) a wavefront keeps in LDS

// Leaves of the point tree whose boxes lie within sqrt(R2) of p, in
// increasing order: a level-by-level descent from the root in which every node
// that passes the box test pushes its two children, in order, to the next
// level.  On return *out points at the leaf indices (in buf0 or buf1, kFront
// entries each, this wavefront's LDS); the count is returned, or -1 when a
// level holds more than kFront nodes.  Wave-uniform control flow.
__device__ int collect_leaves(double px, double py, double pz, double R2, const double *__restrict__ bx, int64_t NL,
                              int lane, int32_t *buf0, int32_t *buf1, int32_t **out)
{
    int32_t *cur = buf0, *nxt = buf1;
    if (lane == 0) cur[0] = 1;
    lds_sync_wave();
    int n = 1;
    for (int64_t width = 1; width < NL; width <<= 1) {
        int m = 0;
        for (int base = 0; base < n; base += 64) {
            const int k = base + lane;
            int32_t node = 0;
            bool hit = false;
            if (k < n) {
                node = cur[k];
                hit = box_gap2(bx + 6 * (int64_t)node, px, py, pz) <= R2;
            }
            int cnt = m / 2;
            const int slot = 2 * wave_push(hit, cnt);
            if (hit && slot + 1 < kFront) {
                nxt[slot] = 2 * node;
                nxt[slot + 1] = 2 * node + 1;
            }
            m = 2 * cnt;
        }
        if (m > kFront) return -1;
        lds_sync_wave();
        int32_t *t = cur;
        cur = nxt;
        nxt = t;
        n = m;
        if (n == 0) break;
    }
    // cur holds nodes of the leaf level (NL + j): keep those whose box passes
    int m = 0;
    for (int base = 0; base < n; base += 64) {
        const int k = base + lane;
        int32_t node = 0;
        bool hit = false;
        if (k < n) {
            node = cur[k];
            hit = box_gap2(bx + 6 * (int64_t)node, px, py, pz) <= R2;
        }
        const int slot = wave_push(hit, m);
        if (hit) nxt[slot] = node - (int32_t)NL;
    }
    lds_sync_wave();
    *out = nxt;
    return m;
}

// The number sum of number_sum_wave restricted to listed leaves (a superset
// of the leaves that meet the ball of radius 2h, in increasing order): the same
// leaf sums are added in the same order, so the result is bitwise the same.
__device__ NumSum number_sum_list(double px, double py, double pz, double h, int64_t n_pts,
                                  const double4 *__restrict__ pts, const double *__restrict__ bx, int64_t NL,
                                  const int32_t *list, int cnt, int lane)
{
    NumSum r{0.0, 0.0, 0};
    const double R2 = 4.0 * h * h * (1.0 + 1e-9);
    for (int base = 0; base < cnt; base += 64) {
        const int i = base + lane;
        NumSum mine{0.0, 0.0, 0};
        if (i < cnt) {
            const int64_t j = list[i];
            if (box_gap2(bx + 6 * (NL + j), px, py, pz) <= R2) mine = leaf_terms(px, py, pz, h, n_pts, pts, j);
        }
        add_leaf_sums(r, mine, __ballot(mine.count > 0));
    }
    return r;
}

// Number sums of one node's solve: the leaves met at the largest h evaluated
// so far are kept and reused for every smaller h; a larger h lists them again;
// when a list does not fit, the sum scans all leaves.
struct LeafCache {
    int32_t *buf0, *buf1, *list;
    int cnt;       // -1: no list
    double h;      // the list holds every leaf within 2 h (1 + 1e-9)
};

__device__ NumSum number_sum_cached(LeafCache &C, double px, double py, double pz, double h, int64_t n_pts,
                                    const double4 *__restrict__ pts, const double *__restrict__ bx, int64_t NL,
                                    int64_t nleaf, int lane)
{
    if (!(C.cnt >= 0 && h <= C.h)) {
        C.cnt = collect_leaves(px, py, pz, 4.0 * h * h * (1.0 + 1e-9), bx, NL, lane, C.buf0, C.buf1, &C.list);
        C.h = h;
    }
    if (C.cnt < 0) return number_sum_wave(px, py, pz, h, n_pts, pts, bx, NL, nleaf, lane);
    return number_sum_list(px, py, pz, h, n_pts, pts, bx, NL, C.list, C.cnt, lane);
}

// One wavefront per point; points that are pseudo nodes solve N(h) = h_fact^3.
// All lanes run the same control flow on the same (wave-uniform) values.
__global__ void __launch_bounds__(256) k_hsolve(int64_t n_pts, const double4 *__restrict__ pts,
                                                const double *__restrict__ bx, int64_t NL, int64_t nleaf,
                                                const int64_t *__restrict__ pt_slot,
                                                const int32_t *__restrict__ pt_node, Nodes T,
                                                const uint32_t *__restrict__ perm, const double *__restrict__ hpart,
                                                double h_fact, double *__restrict__ out_h,
                                                unsigned long long *__restrict__ counters)
{
#pragma clang fp contract(off)
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (t >= n_pts || pt_slot[t] < 0) return;  // wave-uniform
    __shared__ int32_t lds_front[4][2][kFront];
    const int wv = (int)(threadIdx.x >> 6);
    LeafCache LC{lds_front[wv][0], lds_front[wv][1], nullptr, -1, 0.0};
    unsigned long long evals = 0, nb = 0, fb = 0;
    const int32_t nd = pt_node[t];
    const double4 x = pts[t];
    const double s = sqrt(__longlong_as_double((long long)T.d2[nd]));
    double h0;
    if (s > 0.0) {
        h0 = h_fact * 2.0 * s;
    } else {
        h0 = 0.0;
        for (int32_t k = T.start[nd]; k < T.end[nd]; k++) h0 = fmax(h0, hpart[perm[k]]);
    }
    const double target = h_fact * h_fact * h_fact;
    double result = h0;
    bool ok = h0 > 0.0 && (double)n_pts / M_PI > target;
    double lo = 0.0, hi = h0;
    NumSum Nh{};
    if (ok) {
        int k = 0;
        Nh = number_sum_cached(LC, x.x, x.y, x.z, hi, n_pts, pts, bx, NL, nleaf, lane);
        evals++;
        if (Nh.sum_w / M_PI < target) {
            do {
                lo = hi;
                hi = 2.0 * hi;
                Nh = number_sum_cached(LC, x.x, x.y, x.z, hi, n_pts, pts, bx, NL, nleaf, lane);
                evals++;
            } while (Nh.sum_w / M_PI < target && ++k < 200);
        } else {
            lo = 0.5 * hi;
            NumSum Nl = number_sum_cached(LC, x.x, x.y, x.z, lo, n_pts, pts, bx, NL, nleaf, lane);
            evals++;
            while (Nl.sum_w / M_PI >= target && ++k < 200) {
                hi = lo;
                Nh = Nl;
                lo = 0.5 * lo;
                Nl = number_sum_cached(LC, x.x, x.y, x.z, lo, n_pts, pts, bx, NL, nleaf, lane);
                evals++;
            }
        }
        ok = k < 200;
    }
    if (ok) {
        // N(lo) < target <= N(hi); Newton steps kept inside the bracket.  The
        // iterates may approach the root from one side only, so a converged
        // iterate, not the far end of the bracket, is the answer.
        double hc = hi;
        NumSum Nc = Nh;
        result = hi;
        nb = (unsigned long long)Nh.count;
        for (int it = 0; it < 100 && hi - lo > 1e-15 * hi; it++) {
            const double N = Nc.sum_w / M_PI;
            const double dN = -Nc.sum_qdw / (M_PI * hc);
            double hn = dN > 0.0 ? hc - (N - target) / dN : 0.5 * (lo + hi);
            if (dN > 0.0 && fabs(hn - hc) <= 4e-16 * hc) {
                // the Newton step no longer moves the iterate (N(hc) is the
                // target to rounding): hc is the root, whichever side of the
                // bracket it sits on
                result = hc;
                nb = (unsigned long long)Nc.count;
                break;
            }
            if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
            if (hn <= lo || hn >= hi) break;
            const NumSum Nn = number_sum_cached(LC, x.x, x.y, x.z, hn, n_pts, pts, bx, NL, nleaf, lane);
            evals++;
            if (Nn.sum_w / M_PI >= target) {
                hi = hn;
                Nh = Nn;
            } else {
                lo = hn;
            }
            const bool tiny = fabs(hn - hc) <= 4e-16 * hn;
            hc = hn;
            Nc = Nn;
            result = hi;
            nb = (unsigned long long)Nh.count;
            if (tiny) {
                result = hn;
                nb = (unsigned long long)Nn.count;
                break;
            }
        }
    } else {
        fb = 1;
    }
    if (lane == 0) {
        out_h[pt_slot[t]] = result;
        atomicAdd(counters + 0, evals);
        atomicAdd(counters + 1, nb);
        if (fb) atomicAdd(counters + 2, fb);
    }
}

unsigned grid_of(int64_t n, int block = 256)
{
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

template <typename T>
T *carve(char *&p, int64_t count)
{
    T *r = reinterpret_cast<T *>(p);
    p += ((int64_t)sizeof(T) * count + 255) & ~int64_t(255);
    return r;
}

// ---------------------------------------------------------------- resolution check (Eq. (6))
// code 0: passes (or not checked), 1: internal node fails, 2: leaf fails; for
// a failing leaf, need = r - s (its distance to the nearest source less its size)
__global__ void k_check(int64_t n_out, const double *__restrict__ xyz, const double *__restrict__ sz,
                        const int32_t *__restrict__ kind, const int32_t *__restrict__ node,
                        const uint8_t *__restrict__ leaf, const double *__restrict__ f, double K, double s_root,
                        const Walk *__restrict__ W, int32_t *__restrict__ code, double *__restrict__ need)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    int32_t c = 0;
    double nd = -INFINITY;
    if (kind[i] == MAP_PSEUDO_NODE && sz[i] > 0.0) {
        const double lim = (K - s_root / sz[i]) / K;
        if (f[i] < lim) {
            c = leaf[node[i]] ? 2 : 1;
            if (c == 2) nd = src_dist(W, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]) - sz[i];
        }
    }
    code[i] = c;
    need[i] = nd;
}

// One wavefront per remembered region: keep[r] = some pseudo-particle lies
// inside (|x - c| < R) and the smallest neutral fraction inside is below the
// limit of Eq. (6) for a node of size R.
__global__ void k_region_keep(int64_t n_reg, const double *__restrict__ reg, int64_t n_out,
                              const double *__restrict__ xyz, const double *__restrict__ f, double K, double s_root,
                              int32_t *__restrict__ keep)
{
#pragma clang fp contract(off)
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= n_reg) return;  // whole wavefront
    const double *g = reg + 5 * r;
    int any = 0;
    double mn = INFINITY;
    for (int64_t i = lane; i < n_out; i += 64) {
        const double d = sqrt(dist2(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], g[0], g[1], g[2]));
        if (d < g[3]) {
            any = 1;
            mn = fmin(mn, f[i]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        any |= __shfl_xor(any, o, 64);
        mn = fmin(mn, __shfl_xor(mn, o, 64));
    }
    if (lane == 0) {
        const double lim = (K - s_root / g[3]) / K;
        keep[r] = any && !(mn >= lim);
    }
}

__device__ __forceinline__ int label_level(uint64_t label) { return (63 - __clzll((long long)label)) / 3; }

// One wavefront per failed node label: the smallest size among the node
// pseudo-particles that are that node or descend from it (0 if none).
__global__ void k_region_smin(int64_t n_lab, const uint64_t *__restrict__ lab, int64_t n_out,
                              const int32_t *__restrict__ kind, const int64_t *__restrict__ ref,
                              const double *__restrict__ sz, double *__restrict__ smin)
{
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= n_lab) return;  // whole wavefront
    const uint64_t a = lab[w];
    const int la = label_level(a);
    double mn = INFINITY;
    for (int64_t i = lane; i < n_out; i += 64) {
        if (kind[i] != MAP_PSEUDO_NODE) continue;
        const uint64_t b = (uint64_t)ref[i];
        const int lb = label_level(b);
        if (lb >= la && (b >> (3 * (lb - la))) == a) mn = fmin(mn, sz[i]);
    }
    for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
    if (lane == 0) smin[w] = mn < INFINITY ? mn : 0.0;
}

// Tree of one call, kept between its walks.
struct TreeState {
    int32_t n_nodes = 0;
    int max_level = 0;
    Nodes T;
    uint32_t *perm = nullptr;
    int32_t *cur = nullptr, *leaf_of = nullptr;
    int64_t *flag = nullptr, *off = nullptr;
    unsigned *small = nullptr;
};

// Forced openings of a walk (device memory).
struct Forced {
    const uint64_t *open = nullptr;
    int64_t n_open = 0;
    const double *reg = nullptr;
    int64_t n_reg = 0;
};

void check_particles(Workspace &ws, const DevParticles &P, hipStream_t s)
{
    const int64_t n = P.n;
    unsigned *flags = ws.get<unsigned>(S_FLAGS, 4);
    fill_zero_bytes(flags, sizeof(unsigned) * 4, s);
    if (n > 0) {
        hipLaunchKernelGGL(k_check_particles, dim3(grid_of(n)), dim3(256), 0, s, n, P.xyz, P.m, P.h, flags);
        EM_HIP(hipGetLastError());
    }
    unsigned hf = 0;
    EM_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    EM_CHECK(!(hf & F_PART_NONFINITE), MAP_EINVAL, "non-finite particle position");
    EM_CHECK(!(hf & F_H_NONPOS), MAP_EINVAL, "smoothing length h <= 0 or non-finite");
    EM_CHECK(!(hf & F_M_BAD), MAP_EINVAL, "particle mass <= 0 or non-finite");
}

}  // namespace

namespace {

// The octree of n > 0 validated particles (Sec. III-A), kept in TS.
void build_tree(Workspace &ws, const DevParticles &P, const double box[6], int ls, TreeState &TS, hipStream_t s,
                hipEvent_t *ev)
{
    const int64_t n = P.n;
    const int64_t cap64 = n + (int64_t)kMaxLevel * ((n + ls) / (ls + 1)) + 1;
    EM_CHECK(cap64 < (int64_t)INT32_MAX, MAP_EINVAL, "too many particles for this leaf size");
    const int32_t cap = (int32_t)cap64;

    // ---------------------------------------------------------------- tree
    BoxIn B;
    for (int d = 0; d < 3; d++) {
        B.lo[d] = box[d];
        B.ext[d] = box[3 + d] - box[d];
    }
    uint64_t *key = ws.get<uint64_t>(S_PSEUDO0, (size_t)n);
    uint64_t *key2 = ws.get<uint64_t>(S_PSEUDO1, (size_t)n);
    uint32_t *perm = ws.get<uint32_t>(S_PSEUDO2, (size_t)n);
    uint32_t *perm2 = ws.get<uint32_t>(S_PSEUDO3, (size_t)n);
    hipLaunchKernelGGL(k_keys, dim3(grid_of(n)), dim3(256), 0, s, n, P.xyz, B, key, perm);
    EM_HIP(hipGetLastError());
    radix_sort_u64(ws, key, perm, key2, perm2, n, 63, s);
    double4 *pos = ws.get<double4>(S_PSEUDO4, (size_t)n);
    uint8_t *dlev = ws.get<uint8_t>(S_PSEUDO5, (size_t)n);
    hipLaunchKernelGGL(k_sorted, dim3(grid_of(n)), dim3(256), 0, s, n, (const uint32_t *)perm,
                       (const uint64_t *)key, P.xyz, P.m, pos, dlev);
    EM_HIP(hipGetLastError());

    // node table in one allocation
    const size_t node_bytes = (size_t)cap * (5 * 4 + 4 * 1 + 8 + 4 * 8 + 3 * 8 + 8) + 16 * 256;
    char *np = static_cast<char *>(ws.get(S_PSEUDO6, node_bytes));
    Nodes T;
    T.start = carve<int32_t>(np, cap);
    T.end = carve<int32_t>(np, cap);
    T.parent = carve<int32_t>(np, cap);
    T.cb = carve<int32_t>(np, cap);
    T.ce = carve<int32_t>(np, cap);
    T.level = carve<uint8_t>(np, cap);
    T.leaf = carve<uint8_t>(np, cap);
    T.open = carve<uint8_t>(np, cap);
    T.vis = carve<uint8_t>(np, cap);
    T.label = carve<uint64_t>(np, cap);
    T.msum = carve<double>(np, cap);
    T.mx = carve<double>(np, cap);
    T.my = carve<double>(np, cap);
    T.mz = carve<double>(np, cap);
    T.com = carve<double>(np, 3 * (int64_t)cap);
    T.d2 = carve<uint64_t>(np, cap);

    int32_t *cur = ws.get<int32_t>(S_PSEUDO7, (size_t)n);
    int32_t *leaf_of = ws.get<int32_t>(S_PSEUDO8, (size_t)n);
    int64_t *flag = ws.get<int64_t>(S_PSEUDO9, (size_t)n + 1);
    int64_t *off = ws.get<int64_t>(S_PSEUDO10, (size_t)n + 1);
    unsigned *small = ws.get<unsigned>(S_PSEUDO11, 64);  // [0..3] level state, see k_lv_init
    hipLaunchKernelGGL(k_root, dim3(grid_of(n)), dim3(256), 0, s, n, ls, T, cur, leaf_of);
    EM_HIP(hipGetLastError());

    int32_t lvl_off[kMaxLevel + 2];
    lvl_off[0] = 0;
    lvl_off[1] = 1;
    int32_t base = 1;
    int max_level = 0;
    bool inner = n > ls;
    hipLaunchKernelGGL(k_lv_init, dim3(1), dim3(1), 0, s, small);
    EM_HIP(hipGetLastError());
    for (int L = 1; L <= kMaxLevel && inner; L++) {
        hipLaunchKernelGGL(k_lv_flags, dim3(grid_of(n)), dim3(256), 0, s, n, L, (const int32_t *)cur,
                           (const uint8_t *)dlev, flag);
        EM_HIP(hipGetLastError());
        scan_counts(ws, flag, off, n, s);
        hipLaunchKernelGGL(k_lv_count, dim3(1), dim3(1), 0, s, n, (const int64_t *)off, cap, small);
        EM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_lv_nodes, dim3(grid_of(n)), dim3(256), 0, s, n, L, (const unsigned *)small,
                           (const int32_t *)cur, (const int64_t *)flag, (const int64_t *)off, (const uint64_t *)key, T);
        EM_HIP(hipGetLastError());
        // a level has at most n nodes
        hipLaunchKernelGGL(k_lv_leaf, dim3(grid_of(n)), dim3(256), 0, s, L, ls, T, small);
        EM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_lv_cur, dim3(grid_of(n)), dim3(256), 0, s, n, (const unsigned *)small,
                           (const int64_t *)flag, (const int64_t *)off, (const uint8_t *)T.leaf, cur, leaf_of);
        EM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_lv_advance, dim3(1), dim3(1), 0, s, small);
        EM_HIP(hipGetLastError());
        unsigned lv[4] = {0u, 0u, 0u, 0u};
        EM_HIP(hipMemcpyAsync(lv, small, sizeof(lv), hipMemcpyDeviceToHost, s));
        EM_HIP(hipStreamSynchronize(s));
        EM_CHECK(lv[2] == 0u, MAP_EDEVICE, "octree node table overflow");
        base = (int32_t)lv[3];
        lvl_off[L + 1] = base;
        max_level = L;
        inner = lv[0] > 0u;
    }
    const int32_t n_nodes = base;
    hipLaunchKernelGGL(k_children, dim3(grid_of(n_nodes)), dim3(256), 0, s, n_nodes, T);
    EM_HIP(hipGetLastError());
    for (int L = max_level; L >= 0; L--) {
        const int32_t lo = lvl_off[L], hi = lvl_off[L + 1];
        hipLaunchKernelGGL(k_moments, dim3(grid_of(hi - lo)), dim3(256), 0, s, lo, hi, (const double4 *)pos, T);
        EM_HIP(hipGetLastError());
    }
    // sizes
    int64_t *icnt = ws.get<int64_t>(S_PSEUDO12, (size_t)n_nodes + 1);
    int64_t *ioff = ws.get<int64_t>(S_PSEUDO13, (size_t)n_nodes + 1);
    hipLaunchKernelGGL(k_size_small, dim3(grid_of(n_nodes)), dim3(256), 0, s, n_nodes, (const double4 *)pos, T,
                       icnt);
    EM_HIP(hipGetLastError());
    scan_counts(ws, icnt, ioff, n_nodes, s);
    int64_t n_items = 0;
    EM_HIP(hipMemcpyAsync(&n_items, ioff + n_nodes, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    if (n_items > 0) {
        uint64_t *items = ws.get<uint64_t>(S_PSEUDO14, (size_t)n_items);
        hipLaunchKernelGGL(k_size_items, dim3(grid_of(n_nodes)), dim3(256), 0, s, n_nodes, (const int64_t *)ioff,
                           items);
        EM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_size_big, dim3(grid_of(64 * n_items)), dim3(256), 0, s, n_items,
                           (const uint64_t *)items, (const double4 *)pos, T);
        EM_HIP(hipGetLastError());
    }
    if (ev) EM_HIP(hipEventRecord(ev[1], s));
    TS.n_nodes = n_nodes;
    TS.max_level = max_level;
    TS.T = T;
    TS.perm = perm;
    TS.cur = cur;
    TS.leaf_of = leaf_of;
    TS.flag = flag;
    TS.off = off;
    TS.small = small;
}

// One walk over the tree (Sec. III-B) with forced openings F.  Returns the
// pseudo count; when capacity >= it, the set is written to O (workspace
// memory) with node smoothing lengths (Sec. III-C).
int64_t walk_tree(Workspace &ws, const TreeState &TS, const DevParticles &P, const double *src, int n_src,
                  const map_pseudo_params &par, const Forced &F, int64_t capacity, map_pseudo_stats &local,
                  PseudoOut &O, hipStream_t s, hipEvent_t *ev)
{
    const int64_t n = P.n;
    const int32_t n_nodes = TS.n_nodes;
    Nodes T = TS.T;
    const uint32_t *perm = TS.perm;
    int32_t *cur = TS.cur;
    const int32_t *leaf_of = TS.leaf_of;
    int64_t *flag = TS.flag, *off = TS.off;
    unsigned *small = TS.small;
    // ---------------------------------------------------------------- walk
    Walk Wh{};
    for (int k = 0; k < 3 * n_src; k++) Wh.src[k] = src[k];
    Wh.n_src = n_src;
    Wh.theta = par.theta;
    Wh.r_part = par.r_part;
    Wh.r_leaf = par.r_leaf;
    Wh.open = F.open;
    Wh.n_open = F.n_open;
    Wh.reg = F.reg;
    Wh.n_reg = F.n_reg;
    Walk *Wd = reinterpret_cast<Walk *>(ws.get(S_PSEUDO15, sizeof(Walk)));
    EM_HIP(hipMemcpyAsync(Wd, &Wh, sizeof(Walk), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_open, dim3(grid_of(n_nodes)), dim3(256), 0, s, n_nodes, (const Walk *)Wd, T);
    EM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_visible, dim3(grid_of(n_nodes)), dim3(256), 0, s, n_nodes, T);
    EM_HIP(hipGetLastError());
    unsigned long long *wc = reinterpret_cast<unsigned long long *>(small + 32);
    fill_zero_bytes(wc, 4 * sizeof(unsigned long long), s);
    hipLaunchKernelGGL(k_walk_stats, dim3(grid_of(n_nodes)), dim3(256), 0, s, n_nodes, T, wc);
    EM_HIP(hipGetLastError());
    // marks and their scans (reuse the level buffers)
    int64_t *omark = flag;
    int64_t *ooff = off;
    int64_t *pmark = ws.get<int64_t>(S_PCNT, (size_t)n + 1);
    int64_t *poff = ws.get<int64_t>(S_POFF, (size_t)n + 1);
    int32_t *owner = cur;
    fill_zero_bytes(omark, sizeof(int64_t) * n, s);
    fill_zero_bytes(pmark, sizeof(int64_t) * n, s);
    hipLaunchKernelGGL(k_mark, dim3(grid_of(n_nodes)), dim3(256), 0, s, n_nodes, T, omark, pmark, owner);
    EM_HIP(hipGetLastError());
    scan_counts(ws, omark, ooff, n, s);
    scan_counts(ws, pmark, poff, n, s);
    int64_t cnts[2] = {0, 0};
    unsigned long long wcnt[4] = {0, 0, 0, 0};
    EM_HIP(hipMemcpyAsync(&cnts[0], ooff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(&cnts[1], poff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(wcnt, wc, sizeof(wcnt), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    const int64_t n_out = cnts[0], n_pts = cnts[1];
    local.n_tree_nodes = n_nodes;
    local.max_level = TS.max_level;
    local.n_pseudo = n_out;
    local.n_leaves = (int64_t)wcnt[0];
    local.n_pseudo_nodes = (int64_t)wcnt[1];
    local.n_substitute_leaves = (int64_t)wcnt[2];
    local.n_particles = (int64_t)wcnt[3];
    if (capacity < n_out) {
        if (ev) {
            EM_HIP(hipEventRecord(ev[2], s));
            EM_HIP(hipEventRecord(ev[3], s));
        }
        EM_HIP(hipStreamSynchronize(s));
        return n_out;
    }

    double *ob = ws.get<double>(S_PP_PM, (size_t)(6 * n_out + 8));
    O.xyz = ob;
    O.m = ob + 3 * n_out;
    O.h = ob + 4 * n_out;
    O.s = ob + 5 * n_out;
    O.kind = ws.get<int32_t>(S_PC_PM, (size_t)(n_out + 1));
    O.ref = ws.get<int64_t>(S_PAIR_P, (size_t)(n_out + 1));
    O.node = ws.get<int32_t>(S_ADAPT0, (size_t)(n_out + 1));
    double4 *pts = ws.get<double4>(S_PAIR_C, (size_t)(n_pts + 1));
    int64_t *pt_slot = ws.get<int64_t>(S_CCNT64, (size_t)(n_pts + 1));
    int32_t *pt_node = ws.get<int32_t>(S_CCNT, (size_t)(n_pts + 1));
    hipLaunchKernelGGL(k_emit, dim3(grid_of(n)), dim3(256), 0, s, n, (const int64_t *)omark, (const int64_t *)ooff,
                       (const int64_t *)pmark, (const int64_t *)poff, (const int32_t *)owner,
                       (const int32_t *)leaf_of, (const uint32_t *)perm, P.xyz, P.m, P.h, T, O, pts, pt_slot,
                       pt_node);
    EM_HIP(hipGetLastError());
    if (ev) EM_HIP(hipEventRecord(ev[2], s));

    // ---------------------------------------------------------------- h-solve
    unsigned long long *hc = reinterpret_cast<unsigned long long *>(small + 16);
    fill_zero_bytes(hc, 3 * sizeof(unsigned long long), s);
    if (n_pts > 0) {
        const int64_t nleaf = (n_pts + kPtLeaf - 1) / kPtLeaf;
        int64_t NL = 1;
        while (NL < nleaf) NL <<= 1;
        double *bx = ws.get<double>(S_BINOFF_G, (size_t)(12 * NL));
        hipLaunchKernelGGL(k_pt_leaf_boxes, dim3(grid_of(NL)), dim3(256), 0, s, n_pts, NL, (const double4 *)pts,
                           bx);
        EM_HIP(hipGetLastError());
        for (int64_t first = NL / 2; first >= 1; first /= 2) {
            hipLaunchKernelGGL(k_pt_parent_boxes, dim3(grid_of(first)), dim3(256), 0, s, first, bx);
            EM_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_hsolve, dim3(grid_of(64 * n_pts)), dim3(256), 0, s, n_pts, (const double4 *)pts,
                           (const double *)bx, NL, nleaf, (const int64_t *)pt_slot, (const int32_t *)pt_node, T,
                           (const uint32_t *)perm, P.h, par.h_fact_node, O.h, hc);
        EM_HIP(hipGetLastError());
    }
    if (ev) EM_HIP(hipEventRecord(ev[3], s));
    unsigned long long hcnt[3] = {0, 0, 0};
    EM_HIP(hipMemcpyAsync(hcnt, hc, sizeof(hcnt), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    local.n_h_evals = (int64_t)hcnt[0];
    local.n_neighbours = (int64_t)hcnt[1];
    local.n_fallbacks = (int64_t)hcnt[2];
    return n_out;
}

void copy_out_set(const PseudoOut &O, int64_t n_out, const PseudoDest &dest, hipStream_t s)
{
    const hipMemcpyKind kind = dest.mem_kind == MAP_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (n_out > 0) {
        if (dest.xyz) EM_HIP(hipMemcpyAsync(dest.xyz, O.xyz, sizeof(double) * 3 * n_out, kind, s));
        if (dest.m) EM_HIP(hipMemcpyAsync(dest.m, O.m, sizeof(double) * n_out, kind, s));
        if (dest.h) EM_HIP(hipMemcpyAsync(dest.h, O.h, sizeof(double) * n_out, kind, s));
        if (dest.size) EM_HIP(hipMemcpyAsync(dest.size, O.s, sizeof(double) * n_out, kind, s));
        if (dest.kind) EM_HIP(hipMemcpyAsync(dest.kind, O.kind, sizeof(int32_t) * n_out, kind, s));
        if (dest.ref) EM_HIP(hipMemcpyAsync(dest.ref, O.ref, sizeof(int64_t) * n_out, kind, s));
    }
    EM_HIP(hipStreamSynchronize(s));
}

}  // namespace

int64_t run_pseudo(Workspace &ws, const DevParticles &P, const double box[6], const double *src, int n_src,
                   const map_pseudo_params &par, const PseudoDest &dest, map_pseudo_stats *st, hipStream_t s,
                   hipEvent_t *ev)
{
    map_pseudo_stats local{};
    if (ev) EM_HIP(hipEventRecord(ev[0], s));
    check_particles(ws, P, s);
    if (P.n == 0) {
        if (st) *st = local;
        return 0;
    }
    TreeState TS;
    build_tree(ws, P, box, par.leaf_size, TS, s, ev);
    PseudoOut O{};
    const int64_t n_out = walk_tree(ws, TS, P, src, n_src, par, Forced{}, dest.capacity, local, O, s, ev);
    if (dest.capacity >= n_out) copy_out_set(O, n_out, dest, s);
    if (st) *st = local;
    return n_out;
}

int64_t run_pseudo_adaptive(Workspace &ws, const DevParticles &P, const double box[6], const double *src, int n_src,
                            const map_pseudo_params &par0, const map_adapt_params &ap, std::vector<double> &regions,
                            const PseudoDest &dest, map_pseudo_stats *st, map_adapt_stats *ast, hipStream_t s,
                            hipEvent_t *ev)
{
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    map_pseudo_stats local{};
    map_adapt_stats A{};
    map_pseudo_params par = par0;
    const int64_t n_reg_in = (int64_t)regions.size() / 5;
    A.n_regions_in = n_reg_in;
    A.r_part = par.r_part;
    A.r_leaf = par.r_leaf;
    check_particles(ws, P, s);
    if (P.n == 0) {
        // nothing lies inside any region: all are dropped
        A.converged = 1;
        A.n_regions_dropped = n_reg_in;
        regions.clear();
        A.ms_total = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        if (st) *st = local;
        if (ast) *ast = A;
        return 0;
    }
    EM_HIP(hipEventRecord(ev[0], s));
    TreeState TS;
    build_tree(ws, P, box, par.leaf_size, TS, s, ev);
    double s_root = 0.0;
    {
        uint64_t d2 = 0;
        EM_HIP(hipMemcpyAsync(&d2, TS.T.d2, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        EM_HIP(hipStreamSynchronize(s));
        double v;
        std::memcpy(&v, &d2, sizeof(v));
        s_root = std::sqrt(v);
    }
    float ms_tree = 0.f;
    EM_HIP(hipEventElapsedTime(&ms_tree, ev[0], ev[1]));
    A.ms_tree = ms_tree;
    A.s_root = s_root;

    // remembered regions on the device
    double *d_reg = ws.get<double>(S_ADAPT1, (size_t)(5 * n_reg_in + 5));
    if (n_reg_in > 0)
        EM_HIP(hipMemcpyAsync(d_reg, regions.data(), sizeof(double) * 5 * n_reg_in, hipMemcpyHostToDevice, s));
    Walk *Wd = reinterpret_cast<Walk *>(ws.get(S_ADAPT7, sizeof(Walk)));
    {
        Walk Wh{};
        for (int k = 0; k < 3 * n_src; k++) Wh.src[k] = src[k];
        Wh.n_src = n_src;
        EM_HIP(hipMemcpyAsync(Wd, &Wh, sizeof(Walk), hipMemcpyHostToDevice, s));
        EM_HIP(hipStreamSynchronize(s));
    }

    std::vector<uint64_t> opened;     // labels of failed internal nodes (sorted before each walk)
    std::vector<uint64_t> rec_label;  // every failed node, in failure order
    std::vector<double> rec_geom;     // its centre of mass and size (4 per node)
    std::vector<double> hx, hm, hh, hs, hf, hneed;
    std::vector<int32_t> hk, hcode;
    std::vector<int64_t> href;
    PseudoOut O{};
    int64_t n_out = 0;
    double ms_cb = 0.0;
    for (;;) {
        // forced openings of this walk
        std::sort(opened.begin(), opened.end());
        uint64_t *d_open = ws.get<uint64_t>(S_ADAPT2, opened.size() + 1);
        if (!opened.empty())
            EM_HIP(hipMemcpyAsync(d_open, opened.data(), sizeof(uint64_t) * opened.size(), hipMemcpyHostToDevice,
                                  s));
        Forced F;
        F.open = d_open;
        F.n_open = (int64_t)opened.size();
        F.reg = d_reg;
        F.n_reg = n_reg_in;
        local = map_pseudo_stats{};
        n_out = walk_tree(ws, TS, P, src, n_src, par, F, INT64_MAX, local, O, s, nullptr);
        A.n_walks++;
        // the set on the host for the radiative-transfer step
        hx.resize(3 * n_out);
        hm.resize(n_out);
        hh.resize(n_out);
        hs.resize(n_out);
        hk.resize(n_out);
        href.resize(n_out);
        hf.assign(n_out, 0.0);
        EM_HIP(hipMemcpyAsync(hx.data(), O.xyz, sizeof(double) * 3 * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipMemcpyAsync(hm.data(), O.m, sizeof(double) * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipMemcpyAsync(hh.data(), O.h, sizeof(double) * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipMemcpyAsync(hs.data(), O.s, sizeof(double) * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipMemcpyAsync(hk.data(), O.kind, sizeof(int32_t) * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipMemcpyAsync(href.data(), O.ref, sizeof(int64_t) * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipStreamSynchronize(s));
        const auto tc = clk::now();
        const int rc = ap.neutral(ap.user, n_out, hx.data(), hm.data(), hh.data(), hs.data(), hk.data(), hf.data());
        ms_cb += std::chrono::duration<double, std::milli>(clk::now() - tc).count();
        EM_CHECK(rc == 0, MAP_EINVAL, "the neutral-fraction callback returned " + std::to_string(rc));
        for (int64_t i = 0; i < n_out; i++)
            EM_CHECK(std::isfinite(hf[i]), MAP_EINVAL, "non-finite neutral fraction from the callback");
        // the check of Eq. (6)
        double *d_f = ws.get<double>(S_ADAPT3, (size_t)(n_out + 1));
        int32_t *d_code = ws.get<int32_t>(S_ADAPT4, (size_t)(n_out + 1));
        double *d_need = ws.get<double>(S_ADAPT5, (size_t)(n_out + 1));
        hcode.assign(n_out, 0);
        hneed.assign(n_out, 0.0);
        EM_HIP(hipMemcpyAsync(d_f, hf.data(), sizeof(double) * n_out, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_check, dim3(grid_of(n_out)), dim3(256), 0, s, n_out, (const double *)O.xyz,
                           (const double *)O.s, (const int32_t *)O.kind, (const int32_t *)O.node,
                           (const uint8_t *)TS.T.leaf, (const double *)d_f, ap.K, s_root, (const Walk *)Wd, d_code,
                           d_need);
        EM_HIP(hipGetLastError());
        EM_HIP(hipMemcpyAsync(hcode.data(), d_code, sizeof(int32_t) * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipMemcpyAsync(hneed.data(), d_need, sizeof(double) * n_out, hipMemcpyDeviceToHost, s));
        EM_HIP(hipStreamSynchronize(s));
        int64_t n_fail = 0;
        bool leaf_failed = false;
        double need = -INFINITY;
        for (int64_t i = 0; i < n_out; i++) {
            if (!hcode[i]) continue;
            n_fail++;
            rec_label.push_back((uint64_t)href[i]);
            rec_geom.insert(rec_geom.end(), {hx[3 * i], hx[3 * i + 1], hx[3 * i + 2], hs[i]});
            if (hcode[i] == 1) {
                opened.push_back((uint64_t)href[i]);
            } else {
                leaf_failed = true;
                need = std::max(need, hneed[i]);
            }
        }
        A.n_failed += n_fail;
        if (n_fail == 0) {
            A.converged = 1;
            break;
        }
        if (leaf_failed) {
            const double grown = need * (1.0 + 0x1p-30) + 1e-300;
            par.r_leaf = par.r_part > 0.0 ? par.r_leaf * (grown / par.r_part) : std::max(par.r_leaf, grown);
            par.r_part = grown;
            A.n_r_part_growths++;
        }
        if (A.n_walks >= ap.max_walks) break;
    }
    A.r_part = par.r_part;
    A.r_leaf = par.r_leaf;

    // regions: drop the shielded or empty ones, add the failed nodes
    std::vector<double> out_reg;
    if (n_reg_in > 0) {
        int32_t *d_keep = ws.get<int32_t>(S_ADAPT6, (size_t)n_reg_in);
        const double *d_f = ws.get<double>(S_ADAPT3, (size_t)(n_out + 1));
        hipLaunchKernelGGL(k_region_keep, dim3((unsigned)((n_reg_in + 3) / 4)), dim3(256), 0, s, n_reg_in,
                           (const double *)d_reg, n_out, (const double *)O.xyz, d_f, ap.K, s_root, d_keep);
        EM_HIP(hipGetLastError());
        std::vector<int32_t> keep(n_reg_in);
        EM_HIP(hipMemcpyAsync(keep.data(), d_keep, sizeof(int32_t) * n_reg_in, hipMemcpyDeviceToHost, s));
        EM_HIP(hipStreamSynchronize(s));
        for (int64_t r = 0; r < n_reg_in; r++) {
            if (keep[r]) out_reg.insert(out_reg.end(), regions.begin() + 5 * r, regions.begin() + 5 * r + 5);
            else A.n_regions_dropped++;
        }
    }
    const int64_t n_new = (int64_t)rec_label.size();
    if (n_new > 0) {
        uint64_t *d_lab = ws.get<uint64_t>(S_ADAPT2, (size_t)n_new);
        double *d_smin = ws.get<double>(S_ADAPT5, (size_t)n_new);
        EM_HIP(hipMemcpyAsync(d_lab, rec_label.data(), sizeof(uint64_t) * n_new, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_region_smin, dim3((unsigned)((n_new + 3) / 4)), dim3(256), 0, s, n_new,
                           (const uint64_t *)d_lab, n_out, (const int32_t *)O.kind, (const int64_t *)O.ref,
                           (const double *)O.s, d_smin);
        EM_HIP(hipGetLastError());
        std::vector<double> smin(n_new);
        EM_HIP(hipMemcpyAsync(smin.data(), d_smin, sizeof(double) * n_new, hipMemcpyDeviceToHost, s));
        EM_HIP(hipStreamSynchronize(s));
        for (int64_t k = 0; k < n_new; k++)
            out_reg.insert(out_reg.end(),
                           {rec_geom[4 * k], rec_geom[4 * k + 1], rec_geom[4 * k + 2], rec_geom[4 * k + 3], smin[k]});
    }
    EM_CHECK((int64_t)out_reg.size() / 5 <= MAP_MAX_REGIONS, MAP_ENOMEM, "more than MAP_MAX_REGIONS regions");
    if (dest.capacity >= n_out) copy_out_set(O, n_out, dest, s);
    regions.swap(out_reg);
    A.n_regions_out = (int64_t)regions.size() / 5;
    A.ms_callback = ms_cb;
    A.ms_total = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    A.ms_walks = A.ms_total - A.ms_tree - ms_cb;
    if (st) *st = local;
    if (ast) *ast = A;
    return n_out;
}

}  // namespace em
