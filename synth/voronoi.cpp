// Box-clipped Voronoi cells of a point set, for the synthetic inputs.
//
// Input generation only: this file holds none of the mapping arithmetic.  The
// cells are the grid of the paper's coupling (Sec. II-A: a Voronoi grid whose
// generating sites are the particle positions, clipped to the simulation box).
//
// Each cell starts as the box and is cut by the bisector plane of its site and
// each candidate neighbour, nearest first.  The caller supplies candidate
// neighbours sorted by distance (a k-nearest-neighbour list); a cell is final
// once the next unused candidate is at least twice as far as the farthest
// cell vertex (no farther site can cut it).  Cells whose candidate list ran
// out before that bound are reported so the caller can retry with a longer
// list.
//
// Output per cell: faces with outward unit normals and planes n.x = c, their
// vertices counter-clockwise seen from outside, vertices shared within the
// cell, the neighbour across each face (-1-w for box wall w), and the volume.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

namespace {

struct V3 {
    double x, y, z;
};

inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

struct Face {
    V3 n;
    double c;
    int64_t nb;
    std::vector<V3> v;
};

struct Cell {
    std::vector<Face> faces;
};

const double kEps = 1e-13;

bool lex_less(V3 a, V3 b)
{
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.z < b.z;
}

// Point where segment a-b crosses the plane; computed from the
// lexicographically smaller end so both faces sharing the edge get the same bits.
V3 cut_point(V3 a, double sa, V3 b, double sb)
{
    if (lex_less(b, a)) {
        std::swap(a, b);
        std::swap(sa, sb);
    }
    double t = sa / (sa - sb);
    return {a.x + t * (b.x - a.x), a.y + t * (b.y - a.y), a.z + t * (b.z - a.z)};
}

bool same(V3 a, V3 b) { return a.x == b.x && a.y == b.y && a.z == b.z; }

// Clip the cell to n.x <= c.  Returns true when the plane removed something.
bool clip(Cell &cell, V3 n, double c, int64_t nb)
{
    bool any_out = false;
    for (const Face &f : cell.faces) {
        for (const V3 &v : f.v)
            if (dot(n, v) - c > kEps) { any_out = true; break; }
        if (any_out) break;
    }
    if (!any_out) return false;

    std::vector<Face> out;
    out.reserve(cell.faces.size() + 1);
    std::vector<V3> cutpts;
    for (const Face &f : cell.faces) {
        size_t m = f.v.size();
        std::vector<double> s(m);
        for (size_t k = 0; k < m; k++) s[k] = dot(n, f.v[k]) - c;
        Face g;
        g.n = f.n;
        g.c = f.c;
        g.nb = f.nb;
        for (size_t k = 0; k < m; k++) {
            V3 a = f.v[k], b = f.v[(k + 1) % m];
            double sa = s[k], sb = s[(k + 1) % m];
            if (sa <= kEps) {
                g.v.push_back(a);
                if (sa >= -kEps) cutpts.push_back(a);
            }
            if ((sa < -kEps && sb > kEps) || (sa > kEps && sb < -kEps)) {
                V3 x = cut_point(a, sa, b, sb);
                g.v.push_back(x);
                cutpts.push_back(x);
            }
        }
        // drop exact consecutive duplicates
        std::vector<V3> w;
        for (const V3 &p : g.v)
            if (w.empty() || !same(w.back(), p)) w.push_back(p);
        while (w.size() > 1 && same(w.front(), w.back())) w.pop_back();
        g.v.swap(w);
        if (g.v.size() >= 3) out.push_back(std::move(g));
    }
    // the new face on the cutting plane
    std::vector<V3> uniq;
    for (const V3 &p : cutpts) {
        bool dup = false;
        for (const V3 &q : uniq)
            if (same(p, q)) { dup = true; break; }
        if (!dup) uniq.push_back(p);
    }
    if (uniq.size() >= 3) {
        V3 cen = {0, 0, 0};
        for (const V3 &p : uniq) { cen.x += p.x; cen.y += p.y; cen.z += p.z; }
        double inv = 1.0 / uniq.size();
        cen = {cen.x * inv, cen.y * inv, cen.z * inv};
        V3 ref = std::fabs(n.x) < 0.9 ? V3{1, 0, 0} : V3{0, 1, 0};
        V3 u = cross(n, ref);
        double ul = std::sqrt(dot(u, u));
        u = {u.x / ul, u.y / ul, u.z / ul};
        V3 w = cross(n, u);
        std::vector<std::pair<double, V3>> ang;
        for (const V3 &p : uniq) {
            V3 d = sub(p, cen);
            ang.push_back({std::atan2(dot(d, w), dot(d, u)), p});
        }
        std::sort(ang.begin(), ang.end(), [](const std::pair<double, V3> &a, const std::pair<double, V3> &b) {
            return a.first < b.first;
        });
        Face g;
        g.n = n;
        g.c = c;
        g.nb = nb;
        for (auto &pr : ang) g.v.push_back(pr.second);
        out.push_back(std::move(g));
    }
    cell.faces.swap(out);
    return true;
}

Cell box_cell(const double *box)
{
    double x0 = box[0], y0 = box[1], z0 = box[2], x1 = box[3], y1 = box[4], z1 = box[5];
    V3 P[8] = {{x0, y0, z0}, {x1, y0, z0}, {x1, y1, z0}, {x0, y1, z0},
               {x0, y0, z1}, {x1, y0, z1}, {x1, y1, z1}, {x0, y1, z1}};
    Cell c;
    // walls: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z; vertices counter-clockwise seen from outside
    c.faces.push_back({{-1, 0, 0}, -x0, -1, {P[0], P[4], P[7], P[3]}});
    c.faces.push_back({{1, 0, 0}, x1, -2, {P[1], P[2], P[6], P[5]}});
    c.faces.push_back({{0, -1, 0}, -y0, -3, {P[0], P[1], P[5], P[4]}});
    c.faces.push_back({{0, 1, 0}, y1, -4, {P[3], P[7], P[6], P[2]}});
    c.faces.push_back({{0, 0, -1}, -z0, -5, {P[0], P[3], P[2], P[1]}});
    c.faces.push_back({{0, 0, 1}, z1, -6, {P[4], P[5], P[6], P[7]}});
    return c;
}

double max_r2(const Cell &c, V3 s)
{
    double r = 0;
    for (const Face &f : c.faces)
        for (const V3 &v : f.v) {
            V3 d = sub(v, s);
            r = std::max(r, dot(d, d));
        }
    return r;
}

struct Built {
    int64_t n = 0;
    std::vector<Cell> cells;
};

}  // namespace

extern "C" {

// Build (or rebuild, for the listed sites) the clipped cells.  nbr holds, for
// each listed site, k candidate neighbour ids sorted by distance (-1 pads).
// fail[t] is set to 1 when the candidates did not reach the security radius.
void *syn_vor_build(void *handle, int64_t n, const double *xyz, const double *box, const int64_t *idx,
                    int64_t n_idx, const int64_t *nbr, int32_t k, int32_t *fail)
{
    Built *B = static_cast<Built *>(handle);
    if (!B) {
        B = new Built;
        B->n = n;
        B->cells.resize(n);
    }
    int64_t cnt = idx ? n_idx : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < cnt; t++) {
        int64_t i = idx ? idx[t] : t;
        V3 s = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
        Cell c = box_cell(box);
        double r2 = max_r2(c, s);
        bool done = false;
        for (int32_t q = 0; q < k; q++) {
            int64_t j = nbr[t * k + q];
            if (j < 0) break;
            if (j == i) continue;
            V3 o = {xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2]};
            V3 d = sub(o, s);
            double dd = dot(d, d);
            if (dd >= 4.0 * r2) { done = true; break; }
            if (dd == 0.0) continue;  // coincident sites: no bisector
            double l = std::sqrt(dd);
            V3 nn = {d.x / l, d.y / l, d.z / l};
            V3 mid = {0.5 * (s.x + o.x), 0.5 * (s.y + o.y), 0.5 * (s.z + o.z)};
            if (clip(c, nn, dot(nn, mid), j)) r2 = max_r2(c, s);
        }
        if (!done) {
            // candidates exhausted: done only if the list was shorter than k (all sites used)
            int32_t used = 0;
            for (int32_t q = 0; q < k; q++) if (nbr[t * k + q] >= 0) used++;
            done = used < k;
        }
        if (fail) fail[t] = done ? 0 : 1;
        B->cells[i] = std::move(c);
    }
    return B;
}

// sizes[0] = faces, sizes[1] = face-vertex slots, sizes[2] = vertices
void syn_vor_sizes(void *handle, int64_t *sizes)
{
    Built *B = static_cast<Built *>(handle);
    int64_t nf = 0, ns = 0, nv = 0;
    for (const Cell &c : B->cells) {
        nf += (int64_t)c.faces.size();
        std::map<std::tuple<double, double, double>, int> seen;
        for (const Face &f : c.faces) {
            ns += (int64_t)f.v.size();
            for (const V3 &v : f.v) seen.emplace(std::make_tuple(v.x, v.y, v.z), 0);
        }
        nv += (int64_t)seen.size();
    }
    sizes[0] = nf;
    sizes[1] = ns;
    sizes[2] = nv;
}

void syn_vor_copy(void *handle, const double *xyz, int64_t *cell_face_off, int64_t *face_vert_off,
                  int32_t *face_vert, double *face_plane, int64_t *face_nb, double *verts, double *cell_volume)
{
    Built *B = static_cast<Built *>(handle);
    int64_t fo = 0, so = 0, vo = 0;
    cell_face_off[0] = 0;
    face_vert_off[0] = 0;
    for (int64_t i = 0; i < B->n; i++) {
        const Cell &c = B->cells[i];
        std::map<std::tuple<double, double, double>, int64_t> id;
        V3 s = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
        double vol = 0.0;
        for (const Face &f : c.faces) {
            face_plane[4 * fo + 0] = f.n.x;
            face_plane[4 * fo + 1] = f.n.y;
            face_plane[4 * fo + 2] = f.n.z;
            face_plane[4 * fo + 3] = f.c;
            face_nb[fo] = f.nb;
            for (const V3 &v : f.v) {
                auto key = std::make_tuple(v.x, v.y, v.z);
                auto it = id.find(key);
                int64_t vid;
                if (it == id.end()) {
                    vid = vo++;
                    id.emplace(key, vid);
                    verts[3 * vid] = v.x;
                    verts[3 * vid + 1] = v.y;
                    verts[3 * vid + 2] = v.z;
                } else {
                    vid = it->second;
                }
                face_vert[so++] = (int32_t)vid;
            }
            // pyramid volume from the site: height * area / 3
            double area2 = 0.0;
            for (size_t k = 1; k + 1 < f.v.size(); k++)
                area2 += dot(cross(sub(f.v[k], f.v[0]), sub(f.v[k + 1], f.v[0])), f.n);
            vol += (f.c - dot(f.n, s)) * 0.5 * area2 / 3.0;
            fo++;
            face_vert_off[fo] = so;
        }
        cell_face_off[i + 1] = fo;
        cell_volume[i] = vol;
    }
}

void syn_vor_free(void *handle) { delete static_cast<Built *>(handle); }

}  // extern "C"
