"""FP64 CPU oracle of the Exact mapping (paper Sec. II-B, Eq. (1)-(3)).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The HIP library never imports,
links or loads anything here, and nothing here uses the library.

The arithmetic lives in ``exact_oracle.c`` (plain C, FP64, no fast-math) and
``pseudo_oracle.c``; this file only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_SRCS = [os.path.join(_HERE, "exact_oracle.c")]
if os.path.exists(os.path.join(_HERE, "pseudo_oracle.c")):
    _SRCS.append(os.path.join(_HERE, "pseudo_oracle.c"))
if os.path.exists(os.path.join(_HERE, "voronoi_oracle.c")):
    _SRCS.append(os.path.join(_HERE, "voronoi_oracle.c"))

M4 = 0
UNIT = 1
TABLE = 2  # M4 through an interpolated table of the pyramid integral (use_table first)


def build_lib(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        os.makedirs(os.path.dirname(_SO), exist_ok=True)
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Cells(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("cell_face_off", ctypes.c_void_p),
                ("face_vert_off", ctypes.c_void_p), ("face_vert", ctypes.c_void_p),
                ("face_plane", ctypes.c_void_p), ("verts", ctypes.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_lib(force=True)
        lib = ctypes.CDLL(_SO)
        d, i64, vp, i = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        lib.orc_w.restype = d
        lib.orc_w.argtypes = [d]
        lib.orc_F.restype = d
        lib.orc_F.argtypes = [i, d]
        lib.orc_G.restype = d
        lib.orc_G.argtypes = [i, d]
        lib.orc_moments.argtypes = [d, d, d, vp]
        lib.orc_pyramid.restype = d
        lib.orc_pyramid.argtypes = [i, d, d, d]
        lib.orc_pair_fraction.restype = d
        lib.orc_pair_fraction.argtypes = [i, vp, d, ctypes.POINTER(_Cells), i64]
        lib.orc_cell_dist2.restype = d
        lib.orc_cell_dist2.argtypes = [vp, ctypes.POINTER(_Cells), i64]
        lib.orc_pairs_brute.restype = i64
        lib.orc_pairs_brute.argtypes = [i64, vp, vp, ctypes.POINTER(_Cells), vp, vp, i64]
        lib.orc_pairs.restype = i64
        lib.orc_pairs.argtypes = [i64, vp, vp, ctypes.POINTER(_Cells), vp, vp, vp, i64]
        for nm in ("orc_pairs_for_cells", "orc_pairs_for_particles"):
            getattr(lib, nm).restype = i64
            getattr(lib, nm).argtypes = [i64, vp, vp, ctypes.POINTER(_Cells), i64, vp, vp, vp, i64]
        lib.orc_pair_fractions.argtypes = [i, vp, vp, ctypes.POINTER(_Cells), i64, vp, vp, vp]
        lib.orc_reduce.argtypes = [i64, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp]
        lib.orc_map_back.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
        lib.orc_num_threads.restype = i
        lib.orc_set_num_threads.argtypes = [i]
        lib.orc_flop_model.argtypes = [vp, vp, ctypes.POINTER(_Cells), i64, vp, vp, vp]
        lib.orc_table_build.argtypes = [i, i, i, vp]
        lib.orc_table_use.argtypes = [vp, i, i, i]
        for nm in ("orc_table_interp", "orc_solid_angle"):
            getattr(lib, nm).restype = d
            getattr(lib, nm).argtypes = [d, d, d]
        if hasattr(lib, "orp_pseudo"):
            u64 = ctypes.c_uint64
            lib.orp_morton.restype = u64
            lib.orp_morton.argtypes = [vp, vp]
            lib.orp_tree.restype = i64
            lib.orp_tree.argtypes = [i64, vp, vp, vp, i, i64] + [vp] * 10
            lib.orp_number_sum.restype = d
            lib.orp_number_sum.argtypes = [i64, vp, vp, d]
            lib.orp_solve_h.restype = d
            lib.orp_solve_h.argtypes = [i64, vp, vp, d, d, ctypes.POINTER(ctypes.c_int)]
            lib.orp_pseudo.restype = i64
            lib.orp_pseudo.argtypes = [i64, vp, vp, vp, vp, i, vp, d, d, d, i, d, i64] + [vp] * 6 + [vp, i64, vp]
            lib.orp_pseudo2.restype = i64
            lib.orp_pseudo2.argtypes = ([i64, vp, vp, vp, vp, i, vp, d, d, d, i, d, i64, vp, i64, vp, i64] +
                                        [vp] * 7 + [vp, i64, vp])
        if hasattr(lib, "orv_voronoi"):
            lib.orv_voronoi.argtypes = [i64, vp, vp, i64, i64] + [vp] * 8
            lib.orv_voronoi_sel.argtypes = [i64, vp, vp, vp, i64, i64, i64] + [vp] * 8
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _Geom:
    """Keeps contiguous copies alive while the C struct points at them."""

    def __init__(self, cells):
        self.cf = np.ascontiguousarray(cells.cell_face_off, dtype=np.int64)
        self.fv = np.ascontiguousarray(cells.face_vert_off, dtype=np.int64)
        self.fvert = np.ascontiguousarray(cells.face_vert, dtype=np.int32)
        self.plane = _f64(cells.face_plane)
        self.verts = _f64(cells.verts)
        self.s = _Cells(self.cf.size - 1, _p(self.cf).value, _p(self.fv).value, _p(self.fvert).value,
                        _p(self.plane).value, _p(self.verts).value)


# ---------------------------------------------------------------- primitives
def w(q: float) -> float:
    return _load().orc_w(q)


def F(s: float, profile: int = M4) -> float:
    return _load().orc_F(profile, s)


def G(s: float, profile: int = M4) -> float:
    return _load().orc_G(profile, s)


def moments(r0: float, R0: float, alpha: float) -> np.ndarray:
    """[r0*P_-1, P_0, P_2, P_3, P_4, P_5] at alpha."""
    out = np.zeros(6)
    _load().orc_moments(r0, R0, alpha, _p(out))
    return out


def pyramid(r0: float, R0: float, phi: float, profile: int = M4) -> float:
    """Integral of W (h = 1) over the right-angled vertex pyramid (r0, R0, phi)."""
    return _load().orc_pyramid(profile, r0, R0, phi)


# ---------------------------------------------------------------- per pair
_TABLE = {}


def table(n0: int = 64, n1: int = 64, n2: int = 64) -> np.ndarray:
    """Node values of the pyramid integral (r0, R0 in [0, 2], phi in [0, pi/2]), shape (n0, n1, n2)."""
    key = (n0, n1, n2)
    if key not in _TABLE:
        t = np.zeros((n0, n1, n2))
        _load().orc_table_build(n0, n1, n2, _p(t))
        _TABLE[key] = t
    return _TABLE[key]


def use_table(n0: int = 64, n1: int = 64, n2: int = 64) -> np.ndarray:
    """Make profile TABLE read the table of this size; returns it."""
    t = table(n0, n1, n2)
    _load().orc_table_use(_p(t), n0, n1, n2)
    return t


def table_interp(r0: float, R0: float, phi: float) -> float:
    """The pyramid integral through the table (trilinear on the grid, solid-angle identities outside)."""
    return _load().orc_table_interp(r0, R0, phi)


def solid_angle(r0: float, R0: float, phi: float) -> float:
    return _load().orc_solid_angle(r0, R0, phi)


def pair_fraction(p, h: float, cells, cell: int, profile: int = M4) -> float:
    g = _Geom(cells)
    pp = _f64(p)
    return _load().orc_pair_fraction(profile, _p(pp), h, ctypes.byref(g.s), cell)


def cell_dist2(p, cells, cell: int) -> float:
    g = _Geom(cells)
    pp = _f64(p)
    return _load().orc_cell_dist2(_p(pp), ctypes.byref(g.s), cell)


def pairs(xyz, h, cells, brute: bool = False):
    """(pair_p, pair_c) int32, sorted by cell then particle."""
    lib = _load()
    g = _Geom(cells)
    xyz = _f64(xyz)
    h = _f64(h)
    n = h.size
    if brute:
        cnt = lib.orc_pairs_brute(n, _p(xyz), _p(h), ctypes.byref(g.s), None, None, 0)
        pp = np.zeros(cnt, np.int32)
        pc = np.zeros(cnt, np.int32)
        lib.orc_pairs_brute(n, _p(xyz), _p(h), ctypes.byref(g.s), _p(pp), _p(pc), cnt)
        order = np.lexsort((pp, pc))
        return pp[order], pc[order]
    box = _f64(cells.box)
    cnt = lib.orc_pairs(n, _p(xyz), _p(h), ctypes.byref(g.s), _p(box), None, None, 0)
    pp = np.zeros(cnt, np.int32)
    pc = np.zeros(cnt, np.int32)
    lib.orc_pairs(n, _p(xyz), _p(h), ctypes.byref(g.s), _p(box), _p(pp), _p(pc), cnt)
    return pp, pc


def _pairs_sel(fn, xyz, h, cells, sel):
    lib = _load()
    g = _Geom(cells)
    xyz = _f64(xyz)
    h = _f64(h)
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    f = getattr(lib, fn)
    cnt = f(h.size, _p(xyz), _p(h), ctypes.byref(g.s), sel.size, _p(sel), None, None, 0)
    pp = np.zeros(cnt, np.int32)
    pc = np.zeros(cnt, np.int32)
    f(h.size, _p(xyz), _p(h), ctypes.byref(g.s), sel.size, _p(sel), _p(pp), _p(pc), cnt)
    return pp, pc


def pairs_for_cells(xyz, h, cells, sel):
    """All pairs of the selected cells (brute force over particles)."""
    return _pairs_sel("orc_pairs_for_cells", xyz, h, cells, sel)


def pairs_for_particles(xyz, h, cells, sel):
    """All pairs of the selected particles (brute force over cells)."""
    return _pairs_sel("orc_pairs_for_particles", xyz, h, cells, sel)


def sampled_cell_mass(particles, cells, sel_cells, profile: int = M4):
    """M_i and rho_i of the selected cells, with S_a of every particle touching them.

    Returns (M, rho, S_of, pairs) where S_of maps particle -> S_a.
    """
    pp, pc = pairs_for_cells(particles.xyz, particles.h, cells, sel_cells)
    parts = np.unique(pp)
    qp, qc = pairs_for_particles(particles.xyz, particles.h, cells, parts)
    fq = pair_fractions(particles.xyz, particles.h, cells, qp, qc, profile)
    S = np.zeros(particles.h.size)
    np.add.at(S, qp, fq)
    f = pair_fractions(particles.xyz, particles.h, cells, pp, pc, profile)
    M = np.zeros(len(sel_cells))
    pos = {int(c): t for t, c in enumerate(sel_cells)}
    for k in range(pp.size):
        a = pp[k]
        if S[a] > 0:
            M[pos[int(pc[k])]] += particles.m[a] * (f[k] / S[a])
    rho = M / np.asarray(cells.cell_volume)[np.asarray(sel_cells)]
    return M, rho, S, (pp, pc, f)


def pair_fractions(xyz, h, cells, pair_p, pair_c, profile: int = M4) -> np.ndarray:
    lib = _load()
    g = _Geom(cells)
    xyz = _f64(xyz)
    h = _f64(h)
    pp = np.ascontiguousarray(pair_p, dtype=np.int32)
    pc = np.ascontiguousarray(pair_c, dtype=np.int32)
    f = np.zeros(pp.size)
    lib.orc_pair_fractions(profile, _p(xyz), _p(h), ctypes.byref(g.s), pp.size, _p(pp), _p(pc), _p(f))
    return f


def reduce(m, cell_volume, n_cells, pair_p, pair_c, f):
    lib = _load()
    m = _f64(m)
    vol = _f64(cell_volume)
    pp = np.ascontiguousarray(pair_p, dtype=np.int32)
    pc = np.ascontiguousarray(pair_c, dtype=np.int32)
    f = _f64(f)
    S = np.zeros(m.size)
    M = np.zeros(n_cells)
    rho = np.zeros(n_cells)
    lib.orc_reduce(m.size, _p(m), n_cells, _p(vol), pp.size, _p(pp), _p(pc), _p(f), _p(S), _p(M), _p(rho))
    return S, M, rho


def map_particles(particles, cells, profile: int = M4):
    """Full Exact mapping: pairs, per-pair fractions, S_a, cell mass and density."""
    pp, pc = pairs(particles.xyz, particles.h, cells)
    f = pair_fractions(particles.xyz, particles.h, cells, pp, pc, profile)
    S, M, rho = reduce(particles.m, cells.cell_volume, cells.n_cells, pp, pc, f)
    return {"pair_p": pp, "pair_c": pc, "f": f, "S": S, "M": M, "rho": rho}


def map_back(q_cell, mapping, n):
    """Inverse mapping, Eq. (4): particle values from cell values with the pair
    weights of ``mapping`` (a ``map_particles`` result) normalised by S_a."""
    pp = np.ascontiguousarray(mapping["pair_p"], dtype=np.int32)
    pc = np.ascontiguousarray(mapping["pair_c"], dtype=np.int32)
    f = _f64(mapping["f"])
    S = _f64(mapping["S"])
    q = _f64(q_cell)
    out = np.zeros(n)
    _load().orc_map_back(n, pp.size, _p(pp), _p(pc), _p(f), _p(S), _p(q), _p(out))
    return out


def flop_model(xyz, h, cells, pair_p, pair_c) -> dict:
    """Operation count of the direct form (orc_pair_fraction) over the given pairs: faces, edges,
    triangle terms, pyramids, pieces, moment evaluations and flops (see orc_flop_model)."""
    lib = _load()
    g = _Geom(cells)
    xyz = _f64(xyz)
    h = _f64(h)
    pp = np.ascontiguousarray(pair_p, dtype=np.int32)
    pc = np.ascontiguousarray(pair_c, dtype=np.int32)
    cnt = np.zeros(7, np.int64)
    lib.orc_flop_model(_p(xyz), _p(h), ctypes.byref(g.s), pp.size, _p(pp), _p(pc), _p(cnt))
    keys = ("faces", "edges", "triangle_terms", "pyramids", "pieces", "moments", "flops")
    return {k: int(v) for k, v in zip(keys, cnt)}


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops."""
    _load().orc_set_num_threads(int(n))


# ---------------------------------------------------------------- pseudo-particle front end (Sec. III)
PSEUDO_NODE = 0
PSEUDO_PARTICLE = 1


def morton(p, box) -> int:
    """63-bit Morton key of one point in the box."""
    pp = _f64(p)
    bb = _f64(box)
    return int(_load().orp_morton(_p(pp), _p(bb)))


def tree(xyz, m, box, leaf_size: int = 8):
    """Octree in preorder: dict of level, start, end, parent, label, leaf, mass, com, s and perm."""
    lib = _load()
    xyz, m, bb = _f64(xyz), _f64(m), _f64(box)
    n = m.size
    args = [n, _p(xyz), _p(m), _p(bb), leaf_size]
    cnt = lib.orp_tree(*args, 0, *([None] * 10))
    out = dict(level=np.zeros(cnt, np.int32), start=np.zeros(cnt, np.int64), end=np.zeros(cnt, np.int64),
               parent=np.zeros(cnt, np.int64), label=np.zeros(cnt, np.uint64), leaf=np.zeros(cnt, np.int8),
               mass=np.zeros(cnt), com=np.zeros((cnt, 3)), s=np.zeros(cnt), perm=np.zeros(n, np.int64))
    lib.orp_tree(*args, cnt, *[_p(out[k]) for k in ("level", "start", "end", "parent", "label", "leaf", "mass",
                                                    "com", "s", "perm")])
    out["leaf"] = out["leaf"].astype(bool)
    return out


def number_sum(pts, x, h: float) -> float:
    """N(h) = (1/pi) sum_b w(|x - p_b| / h) over all points."""
    pts, x = _f64(pts), _f64(x)
    return _load().orp_number_sum(pts.size // 3, _p(pts), _p(x), h)


def solve_h(pts, x, h0: float, h_fact: float = 1.1):
    """Root of N(h) = h_fact^3 (Eq. (7)-(8)); returns (h, fell_back)."""
    pts, x = _f64(pts), _f64(x)
    fb = ctypes.c_int(0)
    h = _load().orp_solve_h(pts.size // 3, _p(pts), _p(x), h0, h_fact, ctypes.byref(fb))
    return h, bool(fb.value)


def pseudo(xyz, m, h, box, sources, theta=0.5, r_part=0.05, r_leaf=0.1, leaf_size=8, h_fact=1.1, only=None,
           open_labels=None, regions=None):
    """Pseudo-particles (Sec. III) in Morton order: dict of xyz, m, h, s, kind, ref, leaf and stats.

    `only` restricts the h-solve to those pseudo indices (others get h = 0 unless they are particles).
    `open_labels` (node labels) and `regions` (rows cx, cy, cz, R, s_min) force openings of the walk
    (re-walk after a failed resolution check, remembered regions; Sec. III-B)."""
    lib = _load()
    xyz, m, h, bb = _f64(xyz), _f64(m), _f64(h), _f64(box)
    src = _f64(sources).reshape(-1, 3)
    n = m.size
    ol = np.ascontiguousarray(np.zeros(0, np.int64) if open_labels is None else open_labels, dtype=np.int64)
    rg = _f64(np.zeros((0, 5)) if regions is None else regions).reshape(-1, 5)
    st = np.zeros(9)
    head = [n, _p(xyz), _p(m), _p(h), _p(bb), src.shape[0], _p(src), theta, r_part, r_leaf, leaf_size, h_fact,
            ol.size, _p(ol), rg.shape[0], _p(rg)]
    cnt = lib.orp_pseudo2(*head, 0, *([None] * 7), None, 0, _p(st))
    out = dict(xyz=np.zeros((cnt, 3)), m=np.zeros(cnt), h=np.zeros(cnt), s=np.zeros(cnt),
               kind=np.zeros(cnt, np.int32), ref=np.zeros(cnt, np.int64), leaf=np.zeros(cnt, np.int8))
    if only is None:
        o, no = None, 0
    else:
        only = np.ascontiguousarray(only, dtype=np.int64)
        o, no = _p(only), only.size
    lib.orp_pseudo2(*head, cnt, *[_p(out[k]) for k in ("xyz", "m", "h", "s", "kind", "ref", "leaf")], o, no,
                    _p(st))
    out["leaf"] = out["leaf"].astype(bool)
    out["stats"] = dict(tree_nodes=int(st[0]), leaves=int(st[1]), pseudo_nodes=int(st[2]),
                        particles=int(st[3]), substitute_leaves=int(st[4]), fallbacks=int(st[5]),
                        max_level=int(st[6]), neighbours=float(st[7]), s_root=float(st[8]))
    return out


# ---------------------------------------------------------------- adaptive re-walk (Sec. III-B, Eq. (6))
def neutral_limit(s, s_root: float, K: float):
    """Eq. (6): f_neu,limit = (1/K) (K - s_root / s_node), written as (K - s_root / s) / K."""
    s = np.asarray(s, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return (K - s_root / s) / K


def resolution_check(P, f_neu, K: float):
    """Nodes under-resolved by Eq. (6): node pseudo-particles with s > 0 and f_neu below the limit.

    Extracted particles are never checked (Sec. III-B); a zero-size node has no limit."""
    f_neu = np.asarray(f_neu, dtype=np.float64)
    node = (P["kind"] == PSEUDO_NODE) & (P["s"] > 0.0)
    fail = np.zeros(P["kind"].size, dtype=bool)
    fail[node] = f_neu[node] < neutral_limit(P["s"][node], P["stats"]["s_root"], K)
    return fail


def _rmin(xyz, sources):
    """Smallest distance from each point to the sources (the walk's r)."""
    src = _f64(sources).reshape(-1, 3)
    r = np.full(xyz.shape[0], np.inf)
    for q in src:
        d = np.sqrt((xyz[:, 0] - q[0]) * (xyz[:, 0] - q[0]) + (xyz[:, 1] - q[1]) * (xyz[:, 1] - q[1]) +
                    (xyz[:, 2] - q[2]) * (xyz[:, 2] - q[2]))
        r = np.minimum(r, d)
    return r


def _level(label: int) -> int:
    return (int(label).bit_length() - 1) // 3


def _descends(label: int, anc: int) -> bool:
    """Whether node `label` is node `anc` or one of its descendants (anc = label >> 3k)."""
    k = _level(label) - _level(anc)
    return k >= 0 and (int(label) >> (3 * k)) == int(anc)


def pseudo_adaptive(xyz, m, h, box, sources, field, theta=0.5, r_part=0.05, r_leaf=0.1, leaf_size=8, h_fact=1.1,
                    K=100.0, regions=None, max_walks=32):
    """Adaptive tree walk of Sec. III-B, driven by a neutral-fraction field.

    field(P) gives the neutral fraction of every pseudo-particle of the set P
    (the radiative-transfer step).  Each walk is checked with Eq. (6); the
    labels of failing internal nodes are opened in the next walk, and when a
    leaf fails r_part grows to the smallest value that extracts every failing
    leaf (times 1 + 2^-30), r_leaf by the same factor (to at least r_part when
    r_part was 0).  Walks repeat until a set passes or max_walks walks ran.
    Remembered regions (rows cx, cy, cz, R, s_min) force openings from the
    first walk; afterwards a region is dropped when no pseudo-particle of the
    final set lies inside it (|x - c| < R) or the smallest neutral fraction
    inside is at least Eq. (6)'s limit for a node of size R (the node it was
    recorded for would now pass), and each node that failed adds the region
    (its centre of mass, its size, the smallest size among the final set's
    node pseudo-particles descending from it, 0 if none).
    Returns the final set (as `pseudo`) with f_neu, walks, converged, r_part,
    r_leaf, failed (labels per walk), regions (rows) and dropped (count)."""
    regions_in = _f64(np.zeros((0, 5)) if regions is None else regions).reshape(-1, 5)
    opened = []
    failed = []          # per walk: labels of failing nodes (pseudo order)
    records = []         # (label, cx, cy, cz, s) of every failing node
    walks, converged = 0, False
    P = f = None
    while walks < max_walks:
        P = pseudo(xyz, m, h, box, sources, theta, r_part, r_leaf, leaf_size, h_fact,
                   open_labels=np.array(opened, np.int64), regions=regions_in)
        walks += 1
        f = np.asarray(field(P), dtype=np.float64)
        fail = resolution_check(P, f, K)
        idx = np.nonzero(fail)[0]
        failed.append([int(P["ref"][i]) for i in idx])
        if idx.size == 0:
            converged = True
            break
        for i in idx:
            records.append((int(P["ref"][i]), *P["xyz"][i], P["s"][i]))
        inner = idx[~P["leaf"][idx]]
        opened.extend(int(P["ref"][i]) for i in inner)
        leaves = idx[P["leaf"][idx]]
        if leaves.size:
            need = float(np.max(_rmin(P["xyz"][leaves], sources) - P["s"][leaves]))
            new = need * (1.0 + 2.0 ** -30) + 1e-300
            r_leaf = r_leaf * (new / r_part) if r_part > 0.0 else max(r_leaf, new)
            r_part = new
    # remembered regions
    s_root = P["stats"]["s_root"]
    keep = []
    for g in regions_in:
        d = np.sqrt((P["xyz"][:, 0] - g[0]) * (P["xyz"][:, 0] - g[0]) + (P["xyz"][:, 1] - g[1]) *
                    (P["xyz"][:, 1] - g[1]) + (P["xyz"][:, 2] - g[2]) * (P["xyz"][:, 2] - g[2]))
        inside = d < g[3]
        if inside.any() and not (f[inside].min() >= float(neutral_limit(g[3], s_root, K))):
            keep.append(g)
    nodes = np.nonzero(P["kind"] == PSEUDO_NODE)[0]
    new_rows = []
    for lab, cx, cy, cz, s in records:
        sizes = [P["s"][i] for i in nodes if _descends(int(P["ref"][i]), lab)]
        new_rows.append((cx, cy, cz, s, min(sizes) if sizes else 0.0))
    out_regions = np.array(keep + new_rows, dtype=np.float64).reshape(-1, 5)
    P = dict(P)
    P.update(f_neu=f, walks=walks, converged=converged, r_part=r_part, r_leaf=r_leaf, failed=failed,
             regions=out_regions, dropped=regions_in.shape[0] - len(keep))
    return P


# ---------------------------------------------------------------- Voronoi grid (Sec. II-A)
def voronoi(sites, box, sel=None):
    """Box-clipped Voronoi cells of the sites (brute force: every site clips every cell).

    Returns a dict with the cell arrays (cell_face_off, face_vert_off, face_vert, face_plane,
    face_nb, verts, cell_volume; every face owns its vertex copies) and the cell centroids;
    with `sel`, only the selected cells, in that order."""
    lib = _load()
    s, bb = _f64(sites).reshape(-1, 3), _f64(box)
    n = s.shape[0]
    if sel is None:
        sp, ns_ = None, 0
        nc = n
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        sp, ns_ = _p(sel), sel.size
        nc = sel.size
    cnt = np.zeros(3, np.int64)
    lib.orv_voronoi_sel(n, _p(s), _p(bb), sp, ns_, 0, 0, _p(cnt), *([None] * 7))
    nf, ns = int(cnt[0]), int(cnt[1])
    out = dict(cell_face_off=np.zeros(nc + 1, np.int64), face_vert_off=np.zeros(nf + 1, np.int64),
               face_plane=np.zeros((nf, 4)), face_nb=np.zeros(nf, np.int64), verts=np.zeros((ns, 3)),
               cell_volume=np.zeros(nc), centroid=np.zeros((nc, 3)))
    lib.orv_voronoi_sel(n, _p(s), _p(bb), sp, ns_, nf, ns, _p(cnt), *[_p(out[k]) for k in (
        "cell_face_off", "face_vert_off", "face_plane", "face_nb", "verts", "cell_volume", "centroid")])
    out["face_vert"] = np.arange(ns, dtype=np.int32)
    return out


def lloyd(sites, box, iterations: int = 5):
    """Lloyd iterations (sites moved to their cells' centroids), then the cells of the final sites."""
    s = _f64(sites).reshape(-1, 3).copy()
    for _ in range(iterations):
        s = voronoi(s, box)["centroid"].copy()
    V = voronoi(s, box)
    V["sites"] = s
    return V


def merge_sites(sites, d: float):
    """Tightly packed sites merged (reading of Sec. II-A's merging of tightly packed cells): site i is
    dropped when a site of lower index lies closer than d.  Returns the indices kept, ascending."""
    s = _f64(sites).reshape(-1, 3)
    keep = np.ones(len(s), dtype=bool)
    for i in range(1, len(s)):
        w = s[:i] - s[i]
        keep[i] = not np.any(w[:, 0] * w[:, 0] + w[:, 1] * w[:, 1] + w[:, 2] * w[:, 2] < d * d)
    return np.nonzero(keep)[0]


def site_cells(points, sites):
    """The cell of the grid of `sites` that holds each point: its nearest site (ties to the lower index)."""
    p, s = _f64(points).reshape(-1, 3), _f64(sites).reshape(-1, 3)
    out = np.zeros(len(p), dtype=np.int64)
    for a in range(len(p)):
        w = s - p[a]
        out[a] = int(np.argmin(w[:, 0] * w[:, 0] + w[:, 1] * w[:, 1] + w[:, 2] * w[:, 2]))
    return out

