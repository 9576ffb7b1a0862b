// Box-clipped Voronoi grid of the sites on the device, with Lloyd iterations
// (Sec. II-A: the grid is initialised with its generating sites at the
// particle positions and relaxed by Lloyd iterations).
//
// Sites are sorted by Morton key and grouped 8 per leaf of a box tree (heap
// order, internal boxes bottom-up).  One wavefront builds one cell (the box
// cut by bisector planes, nearest sites first, until no farther site can
// reach it; em_voronoi_core.h) into a per-cell record in device memory;
// its face, face-vertex and vertex counts are scanned into offsets in input
// order, and a second pass writes the cells in the library's cell format
// (faces counter-clockwise about outward unit normals, vertices per cell),
// the site or wall across each face, the volumes and the centroids.  A Lloyd
// step moves every site to its cell's centroid and builds the grid again.
#include <cmath>

#include "em_internal.h"
#include "em_voronoi_core.h"
#include "em_wave.h"

namespace em {

namespace {

__device__ __forceinline__ uint64_t spread3v(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

__device__ __forceinline__ uint64_t axis21v(double x, double lo, double ext)
{
    const double t = ((x - lo) / ext) * 2097152.0;
    if (!(t > 0.0)) return 0;
    if (t >= 2097151.0) return 2097151ULL;
    return (uint64_t)floor(t);
}

struct VBox {
    double lo[3], hi[3];
};

// flags: bit 0 a site outside the box or not finite
__global__ void k_vor_keys(int64_t n, const double *__restrict__ s, VBox B, uint64_t *__restrict__ key,
                           uint32_t *__restrict__ idx, unsigned *flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t k[3];
    bool bad = false;
    for (int d = 0; d < 3; d++) {
        const double x = s[3 * i + d];
        if (!(x >= B.lo[d] && x <= B.hi[d])) bad = true;
        k[d] = axis21v(x, B.lo[d], B.hi[d] - B.lo[d]);
    }
    if (bad) atomicOr(flags, 1u);
    key[i] = (spread3v(k[0]) << 2) | (spread3v(k[1]) << 1) | spread3v(k[2]);
    idx[i] = (uint32_t)i;
}

// sorted positions, input index of each sorted site, rank of each input site;
// flags bit 1: two sites coincide (neighbours in Morton order share the key)
__global__ void k_vor_sorted(int64_t n, const uint32_t *__restrict__ perm, const double *__restrict__ s,
                             double *__restrict__ ps, int32_t *__restrict__ orig, int64_t *__restrict__ rank,
                             unsigned *flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t i = perm[r];
    ps[3 * r] = s[3 * i];
    ps[3 * r + 1] = s[3 * i + 1];
    ps[3 * r + 2] = s[3 * i + 2];
    orig[r] = (int32_t)i;
    rank[i] = r;
    if (r > 0) {
        const int64_t j = perm[r - 1];
        if (s[3 * i] == s[3 * j] && s[3 * i + 1] == s[3 * j + 1] && s[3 * i + 2] == s[3 * j + 2]) atomicOr(flags, 2u);
    }
}

__global__ void k_vor_leaf_boxes(int64_t n, int64_t NL, const double *__restrict__ ps, double *__restrict__ bx)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NL) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t q = vor::kLeaf * j; q < vor::kLeaf * (j + 1) && q < n; q++)
        for (int d = 0; d < 3; d++) {
            lo[d] = fmin(lo[d], ps[3 * q + d]);
            hi[d] = fmax(hi[d], ps[3 * q + d]);
        }
    for (int d = 0; d < 3; d++) {
        bx[6 * (NL + j) + d] = lo[d];
        bx[6 * (NL + j) + 3 + d] = hi[d];
    }
}

__global__ void k_vor_parent_boxes(int64_t first, double *__restrict__ bx)
{
    const int64_t i = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * first) return;
    for (int d = 0; d < 3; d++) {
        bx[6 * i + d] = fmin(bx[6 * (2 * i) + d], bx[6 * (2 * i + 1) + d]);
        bx[6 * i + 3 + d] = fmax(bx[6 * (2 * i) + 3 + d], bx[6 * (2 * i + 1) + 3 + d]);
    }
}

// ---------------------------------------------------------------- one wavefront per cell
// The working cell of each wavefront is in LDS: the lanes own the cell's
// triangles (lane l: triangles l and l + 64), so a cut tests every vertex at
// once, finds the boundary of the removed triangles through a bit set of the
// kept triangles' directed edges (each dual edge is in exactly one triangle,
// so the reverse of a removed triangle's edge is kept exactly when it is in
// no removed triangle), and compacts kept and new triangles with prefix
// counts.  The candidate sites of a pass come from a walk of the site tree by
// the whole wavefront (a node stack in LDS, 64 nodes at a time).  A cell built
// by one lane in private memory instead reads its arrays with a different
// index on every lane, so that each access fetches a cache line per lane.
constexpr int kWCand = 192;   // candidates of one pass (wavefront walk); the serial walk uses the first 64
constexpr int kWStack = 384;  // tree nodes pending in the wavefront walk (with kWCand: 9.7 kB of LDS per cell, 4 cells per SIMD)
static_assert(kWCand >= vor::kMaxCand, "the serial walk's candidate heap lives in the same arrays");

struct WCell {
    vor::Plane pl[vor::kMaxPlanes];
    double vx[vor::kMaxTris], vy[vor::kMaxTris], vz[vor::kMaxTris];
    uint32_t tri[vor::kMaxTris];
    int32_t src[vor::kMaxPlanes];
    double cd2[kWCand];
    int32_t cand[kWCand];
    union {  // (never live at the same time)
        int32_t nodes[kWStack];                                 // the wavefront walk's pending nodes
        int64_t stack[64];                                      // the serial walk's stack
        uint32_t bits[vor::kMaxPlanes * vor::kMaxPlanes / 32];  // a cut's directed edges (x, y) of kept triangles: bit 64 x + y
    };
    int32_t np, nt, status, cnt;
    int32_t more, pad[3];
};

__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_min_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Set lanes of mask m below this lane.
__device__ __forceinline__ int lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// The farthest vertex's squared distance and the vertices' bounding box
// (site-centred) of the wavefront's cell.
__device__ double wbounds(const WCell &W, int nt, int lane, double *blo, double *bhi)
{
    double m = 0.0, lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    for (int t = lane; t < nt; t += 64) {
        const double x = W.vx[t], y = W.vy[t], z = W.vz[t];
        m = fmax(m, x * x + y * y + z * z);
        lx = fmin(lx, x), hx = fmax(hx, x);
        ly = fmin(ly, y), hy = fmax(hy, y);
        lz = fmin(lz, z), hz = fmax(hz, z);
    }
    blo[0] = wave_min_d(lx), blo[1] = wave_min_d(ly), blo[2] = wave_min_d(lz);
    bhi[0] = wave_max_d(hx), bhi[1] = wave_max_d(hy), bhi[2] = wave_max_d(hz);
    return wave_max_d(m);
}

// Sorts the first cnt (<= kWCand) candidates by key (squared distance, then
// index) in LDS: each lane holds up to 4 of them and counts the keys below
// each (keys are distinct: the index breaks ties), reading the list with
// broadcast loads; then writes each at its rank.
__device__ void sort_cands(WCell &W, int cnt, int lane)
{
    if (cnt <= 1) return;
    static_assert(kWCand <= 256, "four candidates per lane");
    double d[4];
    int32_t q[4];
    int rk[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int i = lane + 64 * u;
        d[u] = i < cnt ? W.cd2[i] : INFINITY;
        q[u] = i < cnt ? W.cand[i] : 0x7fffffff;
        rk[u] = 0;
    }
    const int per = (cnt + 63) >> 6;  // wave-uniform
    for (int j = 0; j < cnt; j++) {
        const double e = W.cd2[j];
        const int32_t eq = W.cand[j];
        rk[0] += vor::key_less(e, eq, d[0], q[0]) ? 1 : 0;
        if (per > 1) rk[1] += vor::key_less(e, eq, d[1], q[1]) ? 1 : 0;
        if (per > 2) rk[2] += vor::key_less(e, eq, d[2], q[2]) ? 1 : 0;
        if (per > 3) rk[3] += vor::key_less(e, eq, d[3], q[3]) ? 1 : 0;
    }
    lds_sync_wave();  // every read done before the list is rewritten
#pragma unroll
    for (int u = 0; u < 4; u++)
        if (lane + 64 * u < cnt) {
            W.cd2[rk[u]] = d[u];
            W.cand[rk[u]] = q[u];
        }
    lds_sync_wave();
}

// The candidate sites of one pass with the whole wavefront: pending tree
// nodes sit on a stack in LDS, and each step takes the top 64 (one per lane):
// an internal node pushes those of its children that pass the visit test, a
// leaf tests its sites, with the tests of the serial walk (vor::collect).  The
// walk starts from the (at most 64) nodes of the tree's level 6.  The list of
// candidates holds kWCand: when it fills up, it is sorted and cut to the
// sites nearer than its (kWCand / 2)th, whose distance becomes the walk's radius (as the
// serial walk's heap prunes with its farthest entry), and *more is set.  So
// the result is the nearest sites of the ball whose key follows (lo2, lo_q)
// and whose bisector can reach the box [blo, bhi], sorted by key (squared
// distance, then index), all of them unless *more.  Returns the count, or -1
// when the node stack would overflow or a cut list keeps nothing (the caller
// then takes the serial walk).
__device__ int collect_wave(WCell &W, const double *__restrict__ ps, int64_t n, const double *__restrict__ bx,
                            int64_t NL, int64_t self, double sx, double sy, double sz, double lo2, int64_t lo_q,
                            double hi2, const double *blo, const double *bhi, int lane, bool *more)
{
    double h2 = hi2;
    *more = false;
    auto visit = [&](int64_t node) {
        const double *b = bx + 6 * node;
        const double g2 = vor::box_gap2(b, sx, sy, sz);
        if (!(g2 < h2)) return false;
        const double ax = b[0] - sx, bxx = b[3] - sx, ay = b[1] - sy, by = b[4] - sy, az = b[2] - sz, bz = b[5] - sz;
        const double gm = fmax(fmax(ax * blo[0], ax * bhi[0]), fmax(bxx * blo[0], bxx * bhi[0])) +
                          fmax(fmax(ay * blo[1], ay * bhi[1]), fmax(by * blo[1], by * bhi[1])) +
                          fmax(fmax(az * blo[2], az * bhi[2]), fmax(bz * blo[2], bz * bhi[2]));
        return 0.5 * g2 < gm;
    };
    // level 6 of the tree (or the leaves, for a tree of fewer than 64): nodes
    // first .. 2 first - 1; NL is a power of two
    const int64_t first = NL < 64 ? NL : 64;
    int sp = 0, cnt = 0;
    bool cut = false;  // h2 was lowered: popped nodes are tested again
    {
        const bool v = lane < first && visit(first + lane);
        const int c = wave_push(v, sp);
        if (v) W.nodes[c] = (int32_t)(first + lane);
    }
    lds_sync_wave();
    while (sp > 0) {
        const int k = sp < 64 ? sp : 64;
        sp -= k;
        const int64_t node = lane < k ? (int64_t)W.nodes[sp + lane] : 0;
        lds_sync_wave();  // read before the pushes below overwrite these slots
        const bool act = lane < k && (!cut || visit(node));
        const bool internal = act && node < NL, leaf = act && node >= NL;
        const bool v1 = internal && visit(2 * node), v2 = internal && visit(2 * node + 1);
        const int c1 = wave_push(v1, sp);
        const int c2 = wave_push(v2, sp);
        if (v1 && c1 < kWStack) W.nodes[c1] = (int32_t)(2 * node);
        if (v2 && c2 < kWStack) W.nodes[c2] = (int32_t)(2 * node + 1);
        // a leaf's sites, all loaded before any is pushed
        const int64_t j = leaf ? node - NL : 0;
        double d2[vor::kLeaf];
        bool take[vor::kLeaf];
#pragma unroll
        for (int t = 0; t < vor::kLeaf; t++) {
            const int64_t q = vor::kLeaf * j + t;
            const bool ok = leaf && q < n && q != self;
            const int64_t qq = ok ? q : 0;
            const double dx = ps[3 * qq] - sx, dy = ps[3 * qq + 1] - sy, dz = ps[3 * qq + 2] - sz;
            d2[t] = dx * dx + dy * dy + dz * dz;
            take[t] = ok && vor::key_less(lo2, lo_q, d2[t], q) && 0.5 * d2[t] < vor::reach(blo, bhi, dx, dy, dz);
        }
#pragma unroll
        for (int t = 0; t < vor::kLeaf; t++) {
            if (cnt > kWCand - 64) {
                // full: keep the sites nearer than the (kWCand / 2)th
                lds_sync_wave();
                sort_cands(W, cnt, lane);
                h2 = W.cd2[kWCand / 2 - 1];
                int keep = 0;
                for (int u = lane; u < cnt; u += 64) keep += W.cd2[u] < h2 ? 1 : 0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) keep += __shfl_xor(keep, o, 64);
                cnt = keep;
                *more = true;
                cut = true;
                if (cnt == 0) return -1;  // ties: the serial walk orders them by index
                lds_sync_wave();
            }
            const bool tk = take[t] && d2[t] < h2;
            const int c = wave_push(tk, cnt);
            if (tk) {
                W.cd2[c] = d2[t];
                W.cand[c] = (int32_t)(vor::kLeaf * j + t);
            }
        }
        lds_sync_wave();
        if (sp > kWStack) return -1;
    }
    sort_cands(W, cnt, lane);
    return cnt;
}

// Cut by P (n.x <= d) in wave-uniform control flow; np, nt, status are
// wave-uniform copies of the cell's counts.  Returns true when P removed a vertex.
__device__ bool wclip(WCell &W, int &np, int &nt, int &status, const vor::Plane &P, int32_t src, int lane)
{
    const double nn = sqrt(P.nx * P.nx + P.ny * P.ny + P.nz * P.nz);
    const double tol = vor::kEps * nn;
    const int t0 = lane, t1 = lane + 64;
    const bool h0 = t0 < nt, h1 = t1 < nt;
    uint32_t q0 = 0, q1 = 0;
    double x0 = 0.0, y0 = 0.0, z0 = 0.0, x1 = 0.0, y1 = 0.0, z1 = 0.0;
    if (h0) {
        q0 = W.tri[t0];
        x0 = W.vx[t0];
        y0 = W.vy[t0];
        z0 = W.vz[t0];
    }
    if (h1) {
        q1 = W.tri[t1];
        x1 = W.vx[t1];
        y1 = W.vy[t1];
        z1 = W.vz[t1];
    }
    const bool o0 = h0 && P.nx * x0 + P.ny * y0 + P.nz * z0 - P.d > tol;
    const bool o1 = h1 && P.nx * x1 + P.ny * y1 + P.nz * z1 - P.d > tol;
    const uint64_t m0 = __ballot(o0), m1 = __ballot(o1);
    if ((m0 | m1) == 0) return false;
    if (np >= vor::kMaxPlanes) {
        status = vor::ST_PLANES;
        return false;
    }
    const int p = np;
    if (lane == 0) {
        W.pl[p] = P;
        W.src[p] = src;
    }
    np++;
    // directed edges of the kept triangles
    W.bits[lane] = 0u;
    W.bits[lane + 64] = 0u;
    lds_sync_wave();
    auto mark = [&](uint32_t q) {
        const int a = vor::tri_a(q), b = vor::tri_b(q), c = vor::tri_c(q);
        const int e0 = 64 * a + b, e1 = 64 * b + c, e2 = 64 * c + a;
        atomicOr(&W.bits[e0 >> 5], 1u << (e0 & 31));
        atomicOr(&W.bits[e1 >> 5], 1u << (e1 & 31));
        atomicOr(&W.bits[e2 >> 5], 1u << (e2 & 31));
    };
    if (h0 && !o0) mark(q0);
    if (h1 && !o1) mark(q1);
    lds_sync_wave();
    // new triangles (x, y, p) on the boundary edges (x, y) of the removed
    // ones, in the serial order: by removed triangle, then edge
    uint32_t n0[3], n1[3];
    int c0 = 0, c1 = 0;
    auto boundary = [&](uint32_t q, uint32_t *out, int &c) {
        const int v[3] = {vor::tri_a(q), vor::tri_b(q), vor::tri_c(q)};
        for (int e = 0; e < 3; e++) {
            const int x = v[e], y = v[(e + 1) % 3];
            const int r = 64 * y + x;
            if ((W.bits[r >> 5] >> (r & 31)) & 1u) out[c++] = vor::tri_pack(x, y, p);
        }
    };
    if (o0) boundary(q0, n0, c0);
    if (o1) boundary(q1, n1, c1);
    const uint64_t a0 = __ballot(c0 & 1), b0 = __ballot(c0 & 2), a1 = __ballot(c1 & 1), b1 = __ballot(c1 & 2);
    const int s0 = lanes_below(a0) + 2 * lanes_below(b0), s1 = lanes_below(a1) + 2 * lanes_below(b1);
    const int tot0 = __popcll(a0) + 2 * __popcll(b0), tot1 = __popcll(a1) + 2 * __popcll(b1);
    const uint64_t k0 = __ballot(h0 && !o0), k1 = __ballot(h1 && !o1);
    const int kept = __popcll(k0) + __popcll(k1);
    if (kept + tot0 + tot1 > vor::kMaxTris) {
        status = vor::ST_TRIS;
        return false;
    }
    // every lane holds its triangles in registers: compact in place
    if (h0 && !o0) {
        const int k = lanes_below(k0);
        W.tri[k] = q0;
        W.vx[k] = x0;
        W.vy[k] = y0;
        W.vz[k] = z0;
    }
    if (h1 && !o1) {
        const int k = __popcll(k0) + lanes_below(k1);
        W.tri[k] = q1;
        W.vx[k] = x1;
        W.vy[k] = y1;
        W.vz[k] = z1;
    }
    for (int i = 0; i < c0; i++) {
        const int k = kept + s0 + i;
        const uint32_t q = n0[i];
        W.tri[k] = q;
        vor::meet(W.pl[vor::tri_a(q)], W.pl[vor::tri_b(q)], W.pl[vor::tri_c(q)], W.vx[k], W.vy[k], W.vz[k]);
    }
    for (int i = 0; i < c1; i++) {
        const int k = kept + tot0 + s1 + i;
        const uint32_t q = n1[i];
        W.tri[k] = q;
        vor::meet(W.pl[vor::tri_a(q)], W.pl[vor::tri_b(q)], W.pl[vor::tri_c(q)], W.vx[k], W.vy[k], W.vz[k]);
    }
    nt = kept + tot0 + tot1;
    lds_sync_wave();
    return true;
}

// One wavefront per sorted site: its cell, the cell's record and its face,
// face-vertex slot and vertex counts (stored at the site's input index); flags
// bit 2: a cell needed more planes, vertices or passes than its record holds.
__global__ void __launch_bounds__(128) k_vor_build_wave(int64_t n, const double *__restrict__ ps,
                                                        const int32_t *__restrict__ orig,
                                                        const double *__restrict__ bx, int64_t NL, VBox B,
                                                        vor::Cell *__restrict__ cells, int64_t *__restrict__ nfc,
                                                        int64_t *__restrict__ nsc, int64_t *__restrict__ nvc,
                                                        unsigned *flags)
{
    __shared__ WCell cellbuf[2];
    const int lane = threadIdx.x & 63;
    WCell &W = cellbuf[threadIdx.x >> 6];
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= n) return;  // whole wavefronts
    const double box[6] = {B.lo[0], B.lo[1], B.lo[2], B.hi[0], B.hi[1], B.hi[2]};
    const double sx = ps[3 * r], sy = ps[3 * r + 1], sz = ps[3 * r + 2];
    if (lane == 0) {
        vor::init_box(W, box, sx, sy, sz);
        W.status = vor::ST_OK;
    }
    lds_sync_wave();
    int np = 6, nt = 8, status = vor::ST_OK;
    // The first pass only looks within 0.87 times the diagonal of the site's
    // leaf box (about 110 sites when the leaf's 8 sites fill it: most cells
    // end within it), at least an eighth of the mean spacing (for a leaf of
    // very close sites); later passes look anywhere.  The cell does not depend
    // on this choice (see below).
    const double *lb = bx + 6 * (NL + r / vor::kLeaf);
    const double ex = box[3] - box[0], ey = box[4] - box[1], ez = box[5] - box[2];
    const double mean = cbrt(ex * ey * ez / (double)n);
    double hi2 = 0.75 * ((lb[3] - lb[0]) * (lb[3] - lb[0]) + (lb[4] - lb[1]) * (lb[4] - lb[1]) +
                         (lb[5] - lb[2]) * (lb[5] - lb[2]));
    if (hi2 < mean * mean / 64.0) hi2 = mean * mean / 64.0;
    double lo2 = -1.0;
    int64_t lo_q = -1;
    double blo[3], bhi[3];
    double m2 = wbounds(W, nt, lane, blo, bhi);
    // Passes: the ball first, then everything that can still reach the cell;
    // each pass lists the nearest sites whose key follows the last one taken.
    // The sites are cut in key order, skipping those whose bisector cannot
    // reach the vertices' current bounding box (a pass's own reach filter used
    // the box at its start, which contains the current one), until one is at
    // least twice as far as the farthest vertex: the sequence of cuts, and so
    // the cell, is the same however the passes split it.
    bool done = false;
    int pass = 0;
    for (; pass < 4096 && !done && status == vor::ST_OK; pass++) {
        bool more = false;
        int cnt = collect_wave(W, ps, n, bx, NL, r, sx, sy, sz, lo2, lo_q, hi2, blo, bhi, lane, &more);
        if (cnt < 0) {  // the serial walk, 64 at a time
            if (lane == 0) {
                bool m = false;
                W.cnt = vor::collect(W, ps, n, bx, NL, r, sx, sy, sz, lo2, lo_q, hi2, blo, bhi, &m, W.stack);
                W.more = m ? 1 : 0;
            }
            lds_sync_wave();
            cnt = __builtin_amdgcn_readfirstlane(W.cnt);
            more = __builtin_amdgcn_readfirstlane(W.more) != 0;
            if (__builtin_amdgcn_readfirstlane(W.status) != vor::ST_OK) {
                status = vor::ST_PASSES;
                break;
            }
        }
        for (int it = 0; it < cnt; it++) {
            const double bd = W.cd2[it];
            const int64_t q = W.cand[it];
            if (bd >= 4.0 * m2) {  // this site and every farther one miss the cell
                done = true;
                break;
            }
            lo2 = bd;
            lo_q = q;
            vor::Plane P;
            P.nx = ps[3 * q] - sx;
            P.ny = ps[3 * q + 1] - sy;
            P.nz = ps[3 * q + 2] - sz;
            P.d = 0.5 * (P.nx * P.nx + P.ny * P.ny + P.nz * P.nz);
            if (P.d == 0.0) continue;
            if (!(P.d < vor::reach(blo, bhi, P.nx, P.ny, P.nz))) continue;
            if (wclip(W, np, nt, status, P, orig[q], lane)) m2 = wbounds(W, nt, lane, blo, bhi);
            if (status != vor::ST_OK) break;
        }
        if (done || status != vor::ST_OK) break;
        if (!more) {
            if (hi2 == INFINITY) {
                done = true;
                break;
            }
            hi2 = INFINITY;
        }
        lds_sync_wave();  // the candidate list is rewritten by the next pass
    }
    if (!done && status == vor::ST_OK) status = vor::ST_PASSES;
    // the record for the extraction pass, and the counts
    vor::Cell &G = cells[r];
    if (lane == 0) {
        G.np = np;
        G.nt = nt;
        G.status = status;
    }
    if (lane < np) {
        G.pl[lane] = W.pl[lane];
        G.src[lane] = W.src[lane];
    }
    for (int t = lane; t < nt; t += 64) {
        G.tri[t] = W.tri[t];
        G.vx[t] = W.vx[t];
        G.vy[t] = W.vy[t];
        G.vz[t] = W.vz[t];
    }
    int64_t f = 0, sl = 0;
    if (status == vor::ST_OK) {
        int c = 0;
        if (lane < np)
            for (int t = 0; t < nt; t++) {
                const uint32_t q = W.tri[t];
                c += (vor::tri_a(q) == lane || vor::tri_b(q) == lane || vor::tri_c(q) == lane) ? 1 : 0;
            }
        const bool face = c >= 3;
        f = __popcll(__ballot(face));
        int cs = face ? c : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cs += __shfl_xor(cs, o, 64);
        sl = cs;
    } else if (lane == 0) {
        atomicOr(flags, 4u);
    }
    if (lane == 0) {
        const int64_t i = orig[r];
        nfc[i] = f;
        nsc[i] = sl;
        nvc[i] = status == vor::ST_OK ? nt : 0;
    }
}

struct VorOut {
    int64_t *cfo, *fvo, *fnb;
    int32_t *fv;
    double *plane, *verts, *vol, *cen;
};

// One wavefront per input site writes its cell at the scanned offsets: for
// each plane with at least 3 vertices (lane p: plane p), its vertices in
// order around it, counter-clockwise seen from outside (the triangle (p, a, b)
// is followed by the one holding the directed edge (p, b), found in a table of
// the cell's directed edges; the order is reversed if the polygon's vector
// area points inward), the outward unit normal and offset in box
// coordinates, and the site or wall across it; the cell's vertices (in box
// coordinates), volume and centroid (tetrahedra from the site over face fans,
// summed over the faces of each lane and then across the wavefront).  The
// record is read once into LDS.  flags bit 3: a face's vertices did not close
// into one loop.
struct XCell {
    vor::Plane pl[vor::kMaxPlanes];
    double vx[vor::kMaxTris], vy[vor::kMaxTris], vz[vor::kMaxTris];
    uint32_t tri[vor::kMaxTris];
    int32_t src[vor::kMaxPlanes];
    uint8_t et[vor::kMaxPlanes * vor::kMaxPlanes];  // directed edge (x, y): its triangle at 64 x + y, 0xff: none
    uint8_t ring[vor::kMaxPlanes][64];               // ring[k][p]: the k-th triangle around plane p
};
static_assert(vor::kMaxTris < 255 && vor::kMaxPlanes <= 64, "triangle ids in bytes, one plane per lane");

__global__ void __launch_bounds__(128) k_vor_extract(int64_t n, const double *__restrict__ s,
                                                     const int64_t *__restrict__ rank,
                                                     const vor::Cell *__restrict__ cells,
                                                     const int64_t *__restrict__ foff, const int64_t *__restrict__ soff,
                                                     const int64_t *__restrict__ voff, VorOut O, unsigned *flags)
{
    __shared__ XCell xbuf[2];
    const int lane = threadIdx.x & 63;
    XCell &X = xbuf[threadIdx.x >> 6];
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= n) return;  // whole wavefronts
    const vor::Cell &C = cells[rank[i]];
    if (lane == 0) {
        O.cfo[i] = foff[i];
        if (i == n - 1) O.cfo[n] = foff[n];
    }
    if (C.status != vor::ST_OK) return;
    const int np = C.np, nt = C.nt;
    const double sx = s[3 * i], sy = s[3 * i + 1], sz = s[3 * i + 2];
    const int64_t vbase = voff[i], fbase = foff[i], sbase = soff[i];
    uint32_t *et32 = reinterpret_cast<uint32_t *>(X.et);
    for (int k = lane; k < vor::kMaxPlanes * vor::kMaxPlanes / 4; k += 64) et32[k] = 0xffffffffu;
    if (lane < np) {
        X.pl[lane] = C.pl[lane];
        X.src[lane] = C.src[lane];
    }
    for (int t = lane; t < nt; t += 64) {
        const double x = C.vx[t], y = C.vy[t], z = C.vz[t];
        X.tri[t] = C.tri[t];
        X.vx[t] = x;
        X.vy[t] = y;
        X.vz[t] = z;
        O.verts[3 * (vbase + t)] = x + sx;
        O.verts[3 * (vbase + t) + 1] = y + sy;
        O.verts[3 * (vbase + t) + 2] = z + sz;
    }
    lds_sync_wave();
    for (int t = lane; t < nt; t += 64) {
        const uint32_t q = X.tri[t];
        const int a = vor::tri_a(q), b = vor::tri_b(q), c = vor::tri_c(q);
        X.et[64 * a + b] = (uint8_t)t;
        X.et[64 * b + c] = (uint8_t)t;
        X.et[64 * c + a] = (uint8_t)t;
    }
    lds_sync_wave();
    // the ring of triangles around plane p = lane, from the first that holds it
    const int p = lane;
    int nr = 0, first = -1;
    for (int t = 0; t < nt; t++) {
        const uint32_t q = X.tri[t];
        if (vor::tri_a(q) == p || vor::tri_b(q) == p || vor::tri_c(q) == p) {
            nr++;
            if (first < 0) first = t;
        }
    }
    const bool face = p < np && nr >= 3;
    int len = 0;
    if (face) {
        int t = first;
        while (len < nr && len < vor::kMaxPlanes) {  // (a valid cell has at most np - 1)
            X.ring[len][p] = (uint8_t)t;
            len++;
            const uint32_t q = X.tri[t];
            const int b = vor::tri_a(q) == p ? vor::tri_c(q) : (vor::tri_b(q) == p ? vor::tri_a(q) : vor::tri_b(q));
            const int nx = X.et[64 * p + b];  // the triangle holding the directed edge (p, b)
            if (nx == 0xff || nx == first) break;
            t = nx;
        }
    }
    if (__ballot(face && len != nr) != 0) {
        if (lane == 0) atomicOr(flags, 8u);
        return;
    }
    // face index and first slot: prefix counts over the lanes below
    const uint64_t fm = __ballot(face);
    const int nf = __popcll(fm);
    int incl = face ? len : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    double V = 0.0, M0 = 0.0, M1 = 0.0, M2 = 0.0;
    if (face) {
        const int64_t f = fbase + lanes_below(fm), slot = sbase + incl - len;
        const vor::Plane P = X.pl[p];
        const double nn = sqrt(P.nx * P.nx + P.ny * P.ny + P.nz * P.nz);
        const double ux = P.nx / nn, uy = P.ny / nn, uz = P.nz / nn;
        // vector area about the site (local coordinates)
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int k = 0; k < len; k++) {
            const int a = X.ring[k][p], b = X.ring[k + 1 < len ? k + 1 : 0][p];
            ax += X.vy[a] * X.vz[b] - X.vz[a] * X.vy[b];
            ay += X.vz[a] * X.vx[b] - X.vx[a] * X.vz[b];
            az += X.vx[a] * X.vy[b] - X.vy[a] * X.vx[b];
        }
        const bool rev = ax * ux + ay * uy + az * uz < 0.0;
        auto at = [&](int k) { return (int)X.ring[rev ? len - 1 - k : k][p]; };
        O.fvo[f] = slot;
        for (int k = 0; k < len; k++) O.fv[slot + k] = (int32_t)(vbase + at(k));
        O.plane[4 * f] = ux;
        O.plane[4 * f + 1] = uy;
        O.plane[4 * f + 2] = uz;
        O.plane[4 * f + 3] = P.d / nn + (ux * sx + uy * sy + uz * sz);
        O.fnb[f] = X.src[p];
        // tetrahedra (site, v0, vk, vk+1) in counter-clockwise order
        const int o0 = at(0);
        const double x0 = X.vx[o0], y0 = X.vy[o0], z0 = X.vz[o0];
        for (int k = 1; k + 1 < len; k++) {
            const int o1 = at(k), o2 = at(k + 1);
            const double x1 = X.vx[o1], y1 = X.vy[o1], z1 = X.vz[o1];
            const double x2 = X.vx[o2], y2 = X.vy[o2], z2 = X.vz[o2];
            const double tv = (x0 * (y1 * z2 - z1 * y2) + y0 * (z1 * x2 - x1 * z2) + z0 * (x1 * y2 - y1 * x2)) / 6.0;
            V += tv;
            M0 += tv * (x0 + x1 + x2) / 4.0;
            M1 += tv * (y0 + y1 + y2) / 4.0;
            M2 += tv * (z0 + z1 + z2) / 4.0;
        }
    }
    if (lane == 0) O.fvo[fbase + nf] = sbase + total;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        V += __shfl_xor(V, o, 64);
        M0 += __shfl_xor(M0, o, 64);
        M1 += __shfl_xor(M1, o, 64);
        M2 += __shfl_xor(M2, o, 64);
    }
    if (lane == 0) {
        O.vol[i] = V;
        O.cen[3 * i] = sx + (V > 0.0 ? M0 / V : 0.0);
        O.cen[3 * i + 1] = sy + (V > 0.0 ? M1 / V : 0.0);
        O.cen[3 * i + 2] = sz + (V > 0.0 ? M2 / V : 0.0);
    }
}

// Merging of tightly packed sites: a site is dropped when a site of lower
// input index lies closer than sqrt(d2max) (one thread per sorted site, a walk
// of the site tree that stops at the first such site).
__global__ void k_vor_merge(int64_t n, const double *__restrict__ ps, const int32_t *__restrict__ orig,
                            const double *__restrict__ bx, int64_t NL, double d2max, int64_t *__restrict__ keep)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double sx = ps[3 * r], sy = ps[3 * r + 1], sz = ps[3 * r + 2];
    const int32_t me = orig[r];
    bool found = false;
    int64_t i = 1;
    while (!found) {
        if (vor::box_gap2(bx + 6 * i, sx, sy, sz) < d2max) {
            if (i < NL) {
                i = 2 * i;
                continue;
            }
            const int64_t j = i - NL;
            for (int64_t q = vor::kLeaf * j; q < vor::kLeaf * (j + 1) && q < n && !found; q++) {
                if (orig[q] >= me) continue;
                const double dx = ps[3 * q] - sx, dy = ps[3 * q + 1] - sy, dz = ps[3 * q + 2] - sz;
                if (dx * dx + dy * dy + dz * dz < d2max) found = true;
            }
        }
        while (i & 1) i >>= 1;
        if (i == 0) break;
        i += 1;
    }
    keep[me] = found ? 0 : 1;
}

// the kept sites, in input order
__global__ void k_vor_gather(int64_t n, const double *__restrict__ s, const int64_t *__restrict__ keep,
                             const int64_t *__restrict__ koff, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !keep[i]) return;
    const int64_t k = koff[i];
    out[3 * k] = s[3 * i];
    out[3 * k + 1] = s[3 * i + 1];
    out[3 * k + 2] = s[3 * i + 2];
}

// The cell holding each input point by a walk over the grid's cells: from a
// start cell, move to the face neighbour whose site is nearest the point, as
// long as one is nearer than the current site.  Over the box-clipped Voronoi
// grid this ends at the cell that holds the point (the segment from a site to
// the point leaves the site's cell through a face whose neighbour is nearer;
// the cells fill the box).  A point with a face neighbour at the current
// distance or within a relative 1e-10 of it (a tie, or one that rounding could
// decide: a site tied at an edge or vertex of the cell is tied with a face
// neighbour too), or a walk longer than 4096 steps, is listed for the tree
// walk below instead, which breaks ties by the lower index.  Points take as
// start the cell of the same relative index (the point's own site after Lloyd
// steps; near it for points in a spatially coherent order).
__global__ void __launch_bounds__(128) k_vor_site_walk(int64_t n_in, const double *__restrict__ x, int64_t n,
                                                       const double *__restrict__ sites,
                                                       const int64_t *__restrict__ cfo,
                                                       const int64_t *__restrict__ fnb,
                                                       int64_t *__restrict__ site_cell, int64_t *__restrict__ list,
                                                       unsigned long long *__restrict__ n_list)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_in) return;
    const double px = x[3 * a], py = x[3 * a + 1], pz = x[3 * a + 2];
    auto dist2 = [&](int64_t q) {
        const double dx = sites[3 * q] - px, dy = sites[3 * q + 1] - py, dz = sites[3 * q + 2] - pz;
        return dx * dx + dy * dy + dz * dz;
    };
    int64_t c = n_in == n ? a : (int64_t)((double)a * (double)n / (double)n_in);
    if (c >= n) c = n - 1;
    double d = dist2(c);
    bool settled = false;
    for (int step = 0; step < 4096; step++) {
        int64_t best = -1;
        double bd = d;
        for (int64_t f = cfo[c]; f < cfo[c + 1]; f++) {
            const int64_t q = fnb[f];
            if (q < 0) continue;  // a wall
            const double dq = dist2(q);
            if (dq < bd) {
                bd = dq;
                best = q;
            }
        }
        if (best < 0) {
            settled = true;
            break;
        }
        c = best;
        d = bd;
    }
    bool tie = !settled;
    if (settled)
        for (int64_t f = cfo[c]; f < cfo[c + 1] && !tie; f++) {
            const int64_t q = fnb[f];
            tie = q >= 0 && dist2(q) <= d * (1.0 + 1e-10);
        }
    if (tie) {
        const unsigned long long k = atomicAdd(n_list, 1ull);
        list[k] = a;
    } else {
        site_cell[a] = c;
    }
}

// The cell holding each input point: its nearest site of the grid (ties to
// the lower index), by a walk of the grid's site tree, nearer child first,
// skipping boxes farther than the best so far.  Each thread's stack is a
// column of an LDS array (at most one pending sibling per level: 32 entries
// hold trees of up to 2^30 leaves).
constexpr int kSiteStack = 32;

__global__ void __launch_bounds__(128) k_vor_site_cell(int64_t n_in, const int64_t *__restrict__ list,
                                                       const double *__restrict__ x, int64_t n,
                                                       const double *__restrict__ ps, const int32_t *__restrict__ orig,
                                                       const double *__restrict__ bx, int64_t NL,
                                                       int64_t *__restrict__ site_cell)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_in) return;
    const int64_t a = list ? list[t] : t;  // the listed points, or every point
    const double px = x[3 * a], py = x[3 * a + 1], pz = x[3 * a + 2];
    double best = INFINITY;
    int32_t bi = -1;
    __shared__ int32_t stk[kSiteStack][128];
    int32_t *stack = &stk[0][threadIdx.x];  // entry k at stack[128 k]
    int sp = 0;
    stack[0] = 1;
    sp = 1;
    while (sp > 0) {
        const int64_t i = stack[128 * --sp];
        if (vor::box_gap2(bx + 6 * i, px, py, pz) > best) continue;
        if (i < NL) {
            if (sp + 2 > kSiteStack) break;  // cannot happen below 2^30 leaves
            const double gl = vor::box_gap2(bx + 6 * (2 * i), px, py, pz);
            const double gr = vor::box_gap2(bx + 6 * (2 * i + 1), px, py, pz);
            stack[128 * sp++] = (int32_t)(gl <= gr ? 2 * i + 1 : 2 * i);
            stack[128 * sp++] = (int32_t)(gl <= gr ? 2 * i : 2 * i + 1);
            continue;
        }
        const int64_t j = i - NL;
        for (int64_t q = vor::kLeaf * j; q < vor::kLeaf * (j + 1) && q < n; q++) {
            const double dx = ps[3 * q] - px, dy = ps[3 * q + 1] - py, dz = ps[3 * q + 2] - pz;
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < best || (d2 == best && orig[q] < bi)) {
                best = d2;
                bi = orig[q];
            }
        }
    }
    site_cell[a] = bi;
}

unsigned vgrid(int64_t n, int block) { return (unsigned)((n + block - 1) / block > 0 ? (n + block - 1) / block : 1); }

template <typename T>
T *dev_alloc(T *&p, size_t &cap, size_t count)
{
    if (count > cap || !p) {
        if (p) EM_HIP(hipFree(p));
        p = nullptr;
        EM_HIP(hipMalloc(&p, sizeof(T) * (count > 0 ? count : 1)));
        cap = count;
    }
    return p;
}

struct SiteTree {
    const double *ps;
    const int32_t *orig;
    const int64_t *rank;
    double *bx;
    int64_t NL;
};

// Sites sorted by Morton key (positions, input index of each sorted site,
// rank of each input site) and the box tree over leaves of 8.  Rejects sites
// outside the box or not finite, and (when asked) coinciding sites.
SiteTree site_tree(Workspace &ws, int64_t n, const double *sites, const VBox &B, bool distinct, hipStream_t s)
{
    unsigned *flags = ws.get<unsigned>(S_FLAGS, 4);
    fill_zero_bytes(flags, sizeof(unsigned) * 4, s);
    uint64_t *key = ws.get<uint64_t>(S_VOR0, (size_t)n);
    uint64_t *key2 = ws.get<uint64_t>(S_VOR1, (size_t)n);
    uint32_t *perm = ws.get<uint32_t>(S_VOR2, (size_t)n);
    uint32_t *perm2 = ws.get<uint32_t>(S_VOR3, (size_t)n);
    hipLaunchKernelGGL(k_vor_keys, dim3(vgrid(n, 256)), dim3(256), 0, s, n, sites, B, key, perm, flags);
    EM_HIP(hipGetLastError());
    radix_sort_u64(ws, key, perm, key2, perm2, n, 63, s);
    double *ps = ws.get<double>(S_VOR4, (size_t)(3 * n));
    int32_t *orig = ws.get<int32_t>(S_VOR5, (size_t)n);
    int64_t *rank = ws.get<int64_t>(S_VOR6, (size_t)n);
    hipLaunchKernelGGL(k_vor_sorted, dim3(vgrid(n, 256)), dim3(256), 0, s, n, (const uint32_t *)perm, sites, ps, orig,
                       rank, flags);
    EM_HIP(hipGetLastError());
    unsigned hf = 0;
    EM_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    EM_CHECK(!(hf & 1u), MAP_EINVAL, "a site is not finite or lies outside the box");
    EM_CHECK(!distinct || !(hf & 2u), MAP_EINVAL, "two sites coincide (merge them first)");

    const int64_t nleaf = (n + vor::kLeaf - 1) / vor::kLeaf;
    int64_t NL = 1;
    while (NL < nleaf) NL <<= 1;
    double *bx = ws.get<double>(S_VOR7, (size_t)(12 * NL));
    hipLaunchKernelGGL(k_vor_leaf_boxes, dim3(vgrid(NL, 256)), dim3(256), 0, s, n, NL, (const double *)ps, bx);
    EM_HIP(hipGetLastError());
    for (int64_t first = NL / 2; first >= 1; first /= 2) {
        hipLaunchKernelGGL(k_vor_parent_boxes, dim3(vgrid(first, 256)), dim3(256), 0, s, first, bx);
        EM_HIP(hipGetLastError());
    }
    return SiteTree{ps, orig, rank, bx, NL};
}

}  // namespace

// Builds the grid of n sites (device memory) into V; returns the counts.
void build_voronoi(Workspace &ws, VorGrid &V, int64_t n, const double *sites, const double box[6], hipStream_t s)
{
    VBox B;
    for (int d = 0; d < 3; d++) {
        B.lo[d] = box[d];
        B.hi[d] = box[3 + d];
    }
    const SiteTree T = site_tree(ws, n, sites, B, true, s);
    const double *ps = T.ps;
    const int32_t *orig = T.orig;
    const int64_t *rank = T.rank;
    const double *bx = T.bx;
    const int64_t NL = T.NL;
    unsigned *flags = ws.get<unsigned>(S_FLAGS, 4);
    unsigned hf = 0;
    vor::Cell *cells = reinterpret_cast<vor::Cell *>(ws.get(S_VOR8, sizeof(vor::Cell) * (size_t)n));
    int64_t *nfc = ws.get<int64_t>(S_VOR9, (size_t)n + 1);
    int64_t *nsc = ws.get<int64_t>(S_VOR10, (size_t)n + 1);
    int64_t *nvc = ws.get<int64_t>(S_VOR11, (size_t)n + 1);
    hipLaunchKernelGGL(k_vor_build_wave, dim3(vgrid(64 * n, 128)), dim3(128), 0, s, n, (const double *)ps,
                       (const int32_t *)orig, (const double *)bx, NL, B, cells, nfc, nsc, nvc, flags);
    EM_HIP(hipGetLastError());
    int64_t *foff = ws.get<int64_t>(S_VOR12, (size_t)n + 1);
    int64_t *soff = ws.get<int64_t>(S_VOR13, (size_t)n + 1);
    int64_t *voff = ws.get<int64_t>(S_VOR14, (size_t)n + 1);
    scan_counts(ws, nfc, foff, n, s);
    scan_counts(ws, nsc, soff, n, s);
    scan_counts(ws, nvc, voff, n, s);
    int64_t tot[3] = {0, 0, 0};
    EM_HIP(hipMemcpyAsync(&tot[0], foff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(&tot[1], soff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(&tot[2], voff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    EM_CHECK(!(hf & 4u), MAP_EDEVICE,
             "a Voronoi cell needs more than 64 faces or 128 vertices (or its neighbour search did not settle)");
    EM_CHECK(tot[2] < (int64_t)INT32_MAX, MAP_EINVAL, "too many Voronoi vertices for 32-bit vertex ids");
    V.n_faces = tot[0];
    V.n_slots = tot[1];
    V.n_verts = tot[2];
    VorOut O;
    O.cfo = dev_alloc(V.cfo, V.cap_cells, (size_t)n + 1);
    O.vol = dev_alloc(V.vol, V.cap_vol, (size_t)n);
    O.cen = dev_alloc(V.cen, V.cap_cen, (size_t)(3 * n));
    O.fvo = dev_alloc(V.fvo, V.cap_fvo, (size_t)tot[0] + 1);
    O.fnb = dev_alloc(V.fnb, V.cap_fnb, (size_t)tot[0]);
    O.plane = dev_alloc(V.plane, V.cap_plane, (size_t)(4 * tot[0]));
    O.fv = dev_alloc(V.fv, V.cap_fv, (size_t)tot[1]);
    O.verts = dev_alloc(V.verts, V.cap_verts, (size_t)(3 * tot[2]));
    hipLaunchKernelGGL(k_vor_extract, dim3(vgrid(64 * n, 128)), dim3(128), 0, s, n, sites, (const int64_t *)rank,
                       (const vor::Cell *)cells,
                       (const int64_t *)foff, (const int64_t *)soff, (const int64_t *)voff, O, flags);
    EM_HIP(hipGetLastError());
    EM_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    EM_CHECK(!(hf & 8u), MAP_EDEVICE, "a Voronoi face did not close into one loop");
    V.n = n;
}

// Merging (d > 0): the n_in input sites less those with a lower-index site
// closer than d, in input order, into out (3 n_in doubles); returns the count.
int64_t merge_sites(Workspace &ws, int64_t n_in, const double *in, const double box[6], double d, double *out,
                    hipStream_t s)
{
    VBox B;
    for (int k = 0; k < 3; k++) {
        B.lo[k] = box[k];
        B.hi[k] = box[3 + k];
    }
    const SiteTree T = site_tree(ws, n_in, in, B, false, s);
    int64_t *keep = ws.get<int64_t>(S_VOR9, (size_t)n_in + 1);
    int64_t *koff = ws.get<int64_t>(S_VOR10, (size_t)n_in + 1);
    hipLaunchKernelGGL(k_vor_merge, dim3(vgrid(n_in, 128)), dim3(128), 0, s, n_in, T.ps, T.orig, (const double *)T.bx,
                       T.NL, d * d, keep);
    EM_HIP(hipGetLastError());
    scan_counts(ws, keep, koff, n_in, s);
    int64_t m = 0;
    EM_HIP(hipMemcpyAsync(&m, koff + n_in, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_vor_gather, dim3(vgrid(n_in, 256)), dim3(256), 0, s, n_in, in, (const int64_t *)keep,
                       (const int64_t *)koff, out);
    EM_HIP(hipGetLastError());
    EM_HIP(hipStreamSynchronize(s));
    return m;
}

// The cell of the grid V that holds each of the n_in input points.
void site_cells(Workspace &ws, const VorGrid &V, int64_t n_in, const double *in, const double box[6],
                int64_t *site_cell, hipStream_t s)
{
    VBox B;
    for (int k = 0; k < 3; k++) {
        B.lo[k] = box[k];
        B.hi[k] = box[3 + k];
    }
    // the walk over the cells, then the tree walk for the points it lists
    int64_t *list = ws.get<int64_t>(S_VOR9, (size_t)n_in);
    unsigned long long *n_list = reinterpret_cast<unsigned long long *>(ws.get<int64_t>(S_VOR10, 1));
    fill_zero_bytes(n_list, sizeof(unsigned long long), s);
    hipLaunchKernelGGL(k_vor_site_walk, dim3(vgrid(n_in, 128)), dim3(128), 0, s, n_in, in, V.n,
                       (const double *)V.sites, (const int64_t *)V.cfo, (const int64_t *)V.fnb, site_cell, list,
                       n_list);
    EM_HIP(hipGetLastError());
    unsigned long long n_tree = 0;
    EM_HIP(hipMemcpyAsync(&n_tree, n_list, sizeof(n_tree), hipMemcpyDeviceToHost, s));
    EM_HIP(hipStreamSynchronize(s));
    if (n_tree == 0) return;
    const SiteTree T = site_tree(ws, V.n, V.sites, B, true, s);
    hipLaunchKernelGGL(k_vor_site_cell, dim3(vgrid((int64_t)n_tree, 128)), dim3(128), 0, s, (int64_t)n_tree,
                       (const int64_t *)list, in, V.n, T.ps, T.orig, (const double *)T.bx, T.NL, site_cell);
    EM_HIP(hipGetLastError());
}

void free_voronoi(VorGrid &V)
{
    for (void *p : {(void *)V.cfo, (void *)V.vol, (void *)V.cen, (void *)V.fvo, (void *)V.fnb, (void *)V.plane,
                    (void *)V.fv, (void *)V.verts, (void *)V.sites, (void *)V.input, (void *)V.site_cell})
        if (p) (void)hipFree(p);
    V = VorGrid{};
}

}  // namespace em
