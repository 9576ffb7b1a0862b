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

M4 = 0
UNIT = 1


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


def num_threads() -> int:
    return _load().orc_num_threads()


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


def pseudo(xyz, m, h, box, sources, theta=0.5, r_part=0.05, r_leaf=0.1, leaf_size=8, h_fact=1.1, only=None):
    """Pseudo-particles (Sec. III) in Morton order: dict of xyz, m, h, s, kind, ref and stats.

    `only` restricts the h-solve to those pseudo indices (others get h = 0 unless they are particles)."""
    lib = _load()
    xyz, m, h, bb = _f64(xyz), _f64(m), _f64(h), _f64(box)
    src = _f64(sources).reshape(-1, 3)
    n = m.size
    st = np.zeros(8)
    head = [n, _p(xyz), _p(m), _p(h), _p(bb), src.shape[0], _p(src), theta, r_part, r_leaf, leaf_size, h_fact]
    cnt = lib.orp_pseudo(*head, 0, *([None] * 6), None, 0, _p(st))
    out = dict(xyz=np.zeros((cnt, 3)), m=np.zeros(cnt), h=np.zeros(cnt), s=np.zeros(cnt),
               kind=np.zeros(cnt, np.int32), ref=np.zeros(cnt, np.int64))
    if only is None:
        o, no = None, 0
    else:
        only = np.ascontiguousarray(only, dtype=np.int64)
        o, no = _p(only), only.size
    lib.orp_pseudo(*head, cnt, *[_p(out[k]) for k in ("xyz", "m", "h", "s", "kind", "ref")], o, no, _p(st))
    out["stats"] = dict(tree_nodes=int(st[0]), leaves=int(st[1]), pseudo_nodes=int(st[2]),
                        particles=int(st[3]), substitute_leaves=int(st[4]), fallbacks=int(st[5]),
                        max_level=int(st[6]), neighbours=float(st[7]))
    return out
