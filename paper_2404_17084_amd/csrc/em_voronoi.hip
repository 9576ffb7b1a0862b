// Box-clipped Voronoi grid of the sites on the device, with Lloyd iterations
// (Sec. II-A: the grid is initialised with its generating sites at the
// particle positions and relaxed by Lloyd iterations).
//
// Sites are sorted by Morton key and grouped 8 per leaf of a box tree (heap
// order, internal boxes bottom-up).  One thread builds one cell
// (em_voronoi_core.h: the box cut by bisector planes, nearest sites first,
// until no farther site can reach it) in a per-cell record in device memory;
// its face, face-vertex and vertex counts are scanned into offsets in input
// order, and a second pass writes the cells in the library's cell format
// (faces counter-clockwise about outward unit normals, vertices per cell),
// the site or wall across each face, the volumes and the centroids.  A Lloyd
// step moves every site to its cell's centroid and builds the grid again.
#include <cmath>

#include "em_internal.h"
#include "em_voronoi_core.h"

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

// one thread per sorted site: build its cell, count faces, face-vertex slots
// and vertices (stored at the site's input index); flags bit 2: a cell needed
// more planes, vertices or passes than its record holds
__global__ void __launch_bounds__(128) k_vor_build(int64_t n, const double *__restrict__ ps,
                                                   const int32_t *__restrict__ orig, const double *__restrict__ bx,
                                                   int64_t NL, VBox B, vor::Cell *__restrict__ cells,
                                                   int64_t *__restrict__ nfc, int64_t *__restrict__ nsc,
                                                   int64_t *__restrict__ nvc, unsigned *flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double box[6] = {B.lo[0], B.lo[1], B.lo[2], B.hi[0], B.hi[1], B.hi[2]};
    // the working cell in private memory (interleaved across the lanes of a
    // wavefront), then its planes and vertices copied to the record
    vor::Cell C;
    vor::build_cell(C, ps, orig, n, bx, NL, box, r);
    vor::Cell &G = cells[r];
    G.np = C.np;
    G.nt = C.nt;
    G.status = C.status;
    for (int p = 0; p < C.np; p++) {
        G.pl[p] = C.pl[p];
        G.src[p] = C.src[p];
    }
    for (int t = 0; t < C.nt; t++) {
        G.tri[t] = C.tri[t];
        G.vx[t] = C.vx[t];
        G.vy[t] = C.vy[t];
        G.vz[t] = C.vz[t];
    }
    int64_t f = 0, sl = 0;
    if (C.status == vor::ST_OK) vor::cell_counts(C, f, sl);
    else atomicOr(flags, 4u);
    const int64_t i = orig[r];
    nfc[i] = f;
    nsc[i] = sl;
    nvc[i] = C.status == vor::ST_OK ? C.nt : 0;
}

struct VorOut {
    int64_t *cfo, *fvo, *fnb;
    int32_t *fv;
    double *plane, *verts, *vol, *cen;
};

// one thread per input site: write its cell at the scanned offsets
__global__ void __launch_bounds__(128) k_vor_extract(int64_t n, const double *__restrict__ s,
                                                     const int64_t *__restrict__ rank, vor::Cell *__restrict__ cells,
                                                     const int64_t *__restrict__ foff, const int64_t *__restrict__ soff,
                                                     const int64_t *__restrict__ voff, VorOut O, unsigned *flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    vor::Cell &C = cells[rank[i]];
    O.cfo[i] = foff[i];
    if (i == n - 1) O.cfo[n] = foff[n];
    if (C.status != vor::ST_OK) return;
    double vol = 0.0;
    vor::extract_cell(C, s[3 * i], s[3 * i + 1], s[3 * i + 2], voff[i], foff[i], soff[i], O.fvo, O.fv, O.plane, O.fnb,
                      O.verts, vol, O.cen + 3 * i);
    if (C.status != vor::ST_OK) atomicOr(flags, 8u);
    O.vol[i] = vol;
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

// The cell holding each input point: its nearest site of the grid (ties to
// the lower index), by a walk of the grid's site tree, nearer child first,
// skipping boxes farther than the best so far.
__global__ void k_vor_site_cell(int64_t n_in, const double *__restrict__ x, int64_t n, const double *__restrict__ ps,
                                const int32_t *__restrict__ orig, const double *__restrict__ bx, int64_t NL,
                                int64_t *__restrict__ site_cell)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_in) return;
    const double px = x[3 * a], py = x[3 * a + 1], pz = x[3 * a + 2];
    double best = INFINITY;
    int32_t bi = -1;
    int64_t stack[64];
    int sp = 0;
    stack[sp++] = 1;
    while (sp > 0) {
        const int64_t i = stack[--sp];
        if (vor::box_gap2(bx + 6 * i, px, py, pz) > best) continue;
        if (i < NL) {
            if (sp + 2 > 64) break;  // cannot happen below 2^62 leaves
            const double gl = vor::box_gap2(bx + 6 * (2 * i), px, py, pz);
            const double gr = vor::box_gap2(bx + 6 * (2 * i + 1), px, py, pz);
            stack[sp++] = gl <= gr ? 2 * i + 1 : 2 * i;
            stack[sp++] = gl <= gr ? 2 * i : 2 * i + 1;
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
    hipLaunchKernelGGL(k_vor_build, dim3(vgrid(n, 128)), dim3(128), 0, s, n, (const double *)ps,
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
    hipLaunchKernelGGL(k_vor_extract, dim3(vgrid(n, 128)), dim3(128), 0, s, n, sites, (const int64_t *)rank, cells,
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
    const SiteTree T = site_tree(ws, V.n, V.sites, B, true, s);
    hipLaunchKernelGGL(k_vor_site_cell, dim3(vgrid(n_in, 128)), dim3(128), 0, s, n_in, in, V.n, T.ps, T.orig,
                       (const double *)T.bx, T.NL, site_cell);
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
