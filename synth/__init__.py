"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds none of the mapping arithmetic: it draws particle clouds,
assigns smoothing lengths from a neighbour count, and builds the box-clipped
Voronoi cells of the particle positions.  Both the oracle and the HIP library
consume exactly the arrays produced here.

Workloads (stand-ins for the paper's Starbench uniform medium and turbulent
cloud, whose data are not available):

* ``uniform``   -- uniform random positions in the unit box.
* ``clumps``    -- a uniform background plus Gaussian clumps (sigma 0.05 box,
                   peak density contrast 1e4), rejection-sampled into the box.
* ``lognormal`` -- a log-normal density field (sigma_ln_rho = 1.5) whose
                   Gaussian log has a k^-4 power spectrum on a periodic grid;
                   multinomial counts per grid cell, uniform placement inside.

Masses are equal (m = 1/N) as in an SPH code with equal-mass particles.
Particles are returned in Morton (Z-curve) order of their positions, the order
an SPH tree code keeps them in.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "libsynth.so")
_SRC = os.path.join(_HERE, "voronoi.cpp")

BOX = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)


def build_lib(force: bool = True) -> str:
    """Compile the Voronoi clipper (host C++, OpenMP)."""
    if force or not os.path.exists(_SO):
        os.makedirs(os.path.dirname(_SO), exist_ok=True)
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_lib(force=True)
        lib = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.syn_vor_build.restype = vp
        lib.syn_vor_build.argtypes = [vp, i64, vp, vp, vp, i64, vp, i32, vp]
        lib.syn_vor_sizes.argtypes = [vp, vp]
        lib.syn_vor_copy.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.syn_vor_free.argtypes = [vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# data containers
# --------------------------------------------------------------------------
@dataclass
class Particles:
    xyz: np.ndarray  # (n, 3) float64
    m: np.ndarray  # (n,) float64
    h: np.ndarray  # (n,) float64

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


@dataclass
class Cells:
    """Box-clipped convex cells in CSR form.

    cell_face_off[i]:cell_face_off[i+1] are the faces of cell i;
    face_vert_off[j]:face_vert_off[j+1] index face_vert, the vertex ids of face j
    counter-clockwise seen from outside; face_plane[j] = (nx, ny, nz, c) with
    the outward unit normal n and the plane n.x = c; face_nb[j] is the site on
    the other side (-1-w for box wall w).
    """

    cell_face_off: np.ndarray
    face_vert_off: np.ndarray
    face_vert: np.ndarray
    face_plane: np.ndarray
    face_nb: np.ndarray
    verts: np.ndarray
    cell_volume: np.ndarray
    box: tuple = field(default=BOX)

    @property
    def n_cells(self) -> int:
        return int(self.cell_face_off.shape[0] - 1)

    @property
    def n_faces(self) -> int:
        return int(self.face_plane.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    def cell_vertices(self, i: int) -> np.ndarray:
        ids = []
        for j in range(self.cell_face_off[i], self.cell_face_off[i + 1]):
            ids.extend(self.face_vert[self.face_vert_off[j]:self.face_vert_off[j + 1]].tolist())
        return self.verts[sorted(set(ids))]


def cells_subset(cells: Cells, sel) -> Cells:
    """The selected cells alone, in selection order (cell t of the result is cell sel[t]).

    Faces, their vertex lists and planes are gathered; the vertex array is kept
    whole (face_vert still indexes it).  Used to run a pair search over a sample
    of the cells of a large grid.
    """
    sel = np.asarray(sel, dtype=np.int64)
    cfo = np.asarray(cells.cell_face_off, dtype=np.int64)
    fvo = np.asarray(cells.face_vert_off, dtype=np.int64)
    nf = cfo[sel + 1] - cfo[sel]
    new_cfo = np.zeros(sel.size + 1, np.int64)
    np.cumsum(nf, out=new_cfo[1:])
    faces = np.repeat(cfo[sel], nf) + (np.arange(new_cfo[-1]) - np.repeat(new_cfo[:-1], nf))
    nv = fvo[faces + 1] - fvo[faces]
    new_fvo = np.zeros(faces.size + 1, np.int64)
    np.cumsum(nv, out=new_fvo[1:])
    slots = np.repeat(fvo[faces], nv) + (np.arange(new_fvo[-1]) - np.repeat(new_fvo[:-1], nv))
    face_nb = np.asarray(cells.face_nb)[faces] if cells.face_nb is not None else np.zeros(faces.size, np.int64)
    return Cells(new_cfo, new_fvo, np.ascontiguousarray(np.asarray(cells.face_vert)[slots]),
                 np.ascontiguousarray(np.asarray(cells.face_plane)[faces]), np.ascontiguousarray(face_nb),
                 np.asarray(cells.verts), np.ascontiguousarray(np.asarray(cells.cell_volume)[sel]),
                 tuple(cells.box))


def cells_from(obj) -> Cells:
    """A Cells on the host from any object with the same fields (numpy arrays or torch tensors)."""
    def host(a):
        if a is None:
            return None
        return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)

    return Cells(host(obj.cell_face_off), host(obj.face_vert_off), host(obj.face_vert), host(obj.face_plane),
                 host(getattr(obj, "face_nb", None)), host(obj.verts), host(obj.cell_volume), tuple(obj.box))


# --------------------------------------------------------------------------
# positions
# --------------------------------------------------------------------------
def morton_order(xyz: np.ndarray, box=BOX) -> np.ndarray:
    """Permutation sorting points along the 3-D Z-curve (21 bits per axis)."""
    lo = np.asarray(box[:3])
    ext = np.asarray(box[3:]) - lo
    q = np.clip(((xyz - lo) / ext * (1 << 21)).astype(np.int64), 0, (1 << 21) - 1).astype(np.uint64)

    def spread(v):
        v = v & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v

    key = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)) | (spread(q[:, 2]) << np.uint64(2))
    return np.argsort(key, kind="stable")


def uniform_positions(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((n, 3))


def clump_positions(n: int, seed: int, n_clumps: int = 3, sigma: float = 0.05,
                    contrast: float = 1e4) -> np.ndarray:
    """Uniform background plus Gaussian clumps of peak density contrast ``contrast``.

    Background density rho_bg over the unit box; each clump adds
    rho_bg*(contrast-1)*exp(-r^2/(2 sigma^2)), so the mixture weight of a clump is
    (contrast-1)(2 pi)^{3/2} sigma^3 relative to 1 for the background.
    Clump centres are uniform in [0.2, 0.8]^3; samples outside the box are redrawn.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = 0.2 + 0.6 * rng.random((n_clumps, 3))
    wc = (contrast - 1.0) * (2.0 * np.pi) ** 1.5 * sigma ** 3
    w = np.array([1.0] + [wc] * n_clumps)
    w /= w.sum()
    comp = rng.choice(n_clumps + 1, size=n, p=w)
    out = np.empty((n, 3))
    bg = comp == 0
    out[bg] = rng.random((int(bg.sum()), 3))
    for k in range(n_clumps):
        sel = np.nonzero(comp == k + 1)[0]
        todo = sel
        while todo.size:
            pts = centres[k] + sigma * rng.standard_normal((todo.size, 3))
            ok = np.all((pts >= 0.0) & (pts < 1.0), axis=1)
            out[todo[ok]] = pts[ok]
            todo = todo[~ok]
    return out


def lognormal_positions(n: int, seed: int, grid: int = 256, slope: float = -4.0,
                        sigma_ln: float = 1.5) -> np.ndarray:
    """Positions sampled from a log-normal density field.

    g is a unit-variance Gaussian random field on a periodic grid^3 mesh with
    power spectrum P(k) ~ k^slope; ln(rho) = sigma_ln*g - sigma_ln^2/2 (mean
    density one).  Counts per mesh cell are multinomial with probabilities
    rho/sum(rho); positions are uniform inside each mesh cell.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kf = np.fft.fftfreq(grid) * grid
    kr = np.fft.rfftfreq(grid) * grid
    k2 = kf[:, None, None] ** 2 + kf[None, :, None] ** 2 + kr[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)  # sqrt(P(k)) with P ~ k^slope
    noise = rng.standard_normal((grid, grid, grid))
    g = np.fft.irfftn(np.fft.rfftn(noise) * amp, s=(grid, grid, grid), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln ** 2).ravel()
    del g, noise, amp, k2
    p = rho / rho.sum()
    counts = rng.multinomial(n, p)
    cell = np.repeat(np.arange(grid ** 3, dtype=np.int64), counts)
    iz = cell % grid
    iy = (cell // grid) % grid
    ix = cell // (grid * grid)
    base = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    return (base + rng.random((n, 3))) / grid


# --------------------------------------------------------------------------
# smoothing lengths
# --------------------------------------------------------------------------
def neighbour_h(xyz: np.ndarray, n_ngb: int = 58, h_fact: float = 1.2) -> np.ndarray:
    """h = h_fact * (m / rho_local)^(1/3) with a top-hat neighbour density.

    rho_local = n_ngb * m / (4/3 pi r_ngb^3), r_ngb the distance to the n_ngb-th
    nearest other particle, so h = h_fact * (4 pi / (3 n_ngb))^(1/3) * r_ngb
    (h_fact 1.2 with 58 neighbours gives h ~ r_ngb / 2: about 58 particles
    inside 2h).  Within 2h of a box wall fewer particles are found, and h grows.
    """
    from scipy.spatial import cKDTree

    n = xyz.shape[0]
    k = min(n_ngb + 1, n)
    d, _ = cKDTree(xyz).query(xyz, k=k, workers=-1)
    r = d[:, -1] if k > 1 else np.full(n, 0.5)
    return h_fact * (4.0 * np.pi / (3.0 * n_ngb)) ** (1.0 / 3.0) * r


# --------------------------------------------------------------------------
# Voronoi cells
# --------------------------------------------------------------------------
def voronoi_cells(xyz: np.ndarray, box=BOX, k0: int = 48) -> Cells:
    from scipy.spatial import cKDTree

    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    n = xyz.shape[0]
    boxa = np.asarray(box, dtype=np.float64)
    tree = cKDTree(xyz)

    def knn(idx, k):
        kk = min(k, n)
        _, nb = tree.query(xyz[idx], k=kk, workers=-1)
        nb = np.asarray(nb, dtype=np.int64).reshape(len(idx), kk)
        nb[nb >= n] = -1
        return np.ascontiguousarray(nb), kk

    idx = np.arange(n, dtype=np.int64)
    nb, k = knn(idx, k0)
    fail = np.zeros(n, dtype=np.int32)
    handle = lib.syn_vor_build(None, n, _ptr(xyz), _ptr(boxa), None, 0, _ptr(nb), k, _ptr(fail))
    while fail.any():
        todo = np.ascontiguousarray(np.nonzero(fail)[0].astype(np.int64))
        k = min(4 * k, n)
        nb, k = knn(todo, k)
        f2 = np.zeros(todo.size, dtype=np.int32)
        lib.syn_vor_build(handle, n, _ptr(xyz), _ptr(boxa), _ptr(todo), todo.size, _ptr(nb), k, _ptr(f2))
        fail[:] = 0
        fail[todo] = f2
        if k >= n:
            break
    sizes = np.zeros(3, dtype=np.int64)
    lib.syn_vor_sizes(handle, _ptr(sizes))
    nf, ns, nv = (int(s) for s in sizes)
    cf = np.zeros(n + 1, dtype=np.int64)
    fv = np.zeros(nf + 1, dtype=np.int64)
    fvert = np.zeros(ns, dtype=np.int32)
    plane = np.zeros((nf, 4), dtype=np.float64)
    fnb = np.zeros(nf, dtype=np.int64)
    verts = np.zeros((nv, 3), dtype=np.float64)
    vol = np.zeros(n, dtype=np.float64)
    lib.syn_vor_copy(handle, _ptr(xyz), _ptr(cf), _ptr(fv), _ptr(fvert), _ptr(plane), _ptr(fnb),
                     _ptr(verts), _ptr(vol))
    lib.syn_vor_free(handle)
    return Cells(cf, fv, fvert, plane, fnb, verts, vol, tuple(box))


# --------------------------------------------------------------------------
# neutral-fraction field (stand-in for the radiative transfer)
# --------------------------------------------------------------------------
def ionised_spheres(xyz: np.ndarray, centres, radius: float, width: float) -> np.ndarray:
    """Neutral fraction of an H II region around each centre: 0 within `radius`
    of the nearest centre, rising linearly to 1 at `radius + width`.

    Stands in for the neutral fractions a radiative-transfer run would return
    for the pseudo-particles (Sec. III-B); the adaptive walk only needs a
    field that is ionised near the sources and neutral far from them."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    c = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    d = np.full(xyz.shape[0], np.inf)
    for q in c:
        d = np.minimum(d, np.sqrt(((xyz - q) ** 2).sum(axis=1)))
    return np.clip((d - radius) / width, 0.0, 1.0)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def particles(kind: str, n: int, seed: int, **kw) -> Particles:
    if kind == "uniform":
        xyz = uniform_positions(n, seed)
    elif kind == "clumps":
        xyz = clump_positions(n, seed, **kw)
    elif kind == "lognormal":
        xyz = lognormal_positions(n, seed, **kw)
    else:
        raise ValueError(kind)
    xyz = np.ascontiguousarray(xyz[morton_order(xyz)])
    h = neighbour_h(xyz)
    m = np.full(n, 1.0 / n)
    return Particles(xyz, m, h)


def workload(kind: str, n: int, seed: int, **kw):
    """Particles and the box-clipped Voronoi cells of their positions."""
    p = particles(kind, n, seed, **kw)
    return p, voronoi_cells(p.xyz)


# The mapping benchmarks: (kind, n, seed)
UNIFORM_4K = ("uniform", 4096, 1)
CLUMPS_256K = ("clumps", 262144, 2)
LOGNORMAL_2M = ("lognormal", 2097152, 3)
