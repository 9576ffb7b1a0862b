"""Python binding of libexactmap (MI355X Exact mapping of SPH particles onto cells).

Argument marshalling only: every step of the mapping runs in the HIP library.
The functions keep the C ABI's names (``map_init``, ``map_pairs``,
``map_particles``, ...).  Host inputs are numpy arrays; device inputs are torch
CUDA tensors (torch is used only for device memory).  If the built library is
missing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libexactmap.so")

MAP_OK = 0
MAP_EINVAL = -1
MAP_ENOMEM = -2
MAP_EDEVICE = -3
MAP_EBUSY = -4
MAP_ENOTFOUND = -5
MAP_EGEOM = -6
MAP_ENUMERIC = -7
MAP_ENOTSUP = -8
MAP_FP64 = 0
MAP_MIXED = 1
MAP_TABLE = 2
MAP_MEM_HOST = 0
MAP_MEM_DEVICE = 1
JOB_PENDING, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

_ERRNAMES = {v: k for k, v in dict(MAP_EINVAL=-1, MAP_ENOMEM=-2, MAP_EDEVICE=-3, MAP_EBUSY=-4, MAP_ENOTFOUND=-5,
                                   MAP_EGEOM=-6, MAP_ENUMERIC=-7,
                                   MAP_ENOTSUP=-8).items()}

c_i64, c_i32, c_int, c_dbl, c_vp, c_u64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_uint64)


class map_config(ctypes.Structure):
    _fields_ = [("device", c_int), ("precision", c_int), ("hbm_budget_bytes", c_u64), ("max_jobs", c_int),
                ("max_queue", c_int), ("tune_cache_path", ctypes.c_char_p), ("serve_timeout_ms", c_int),
                ("serve_trace", c_int), ("fixup_cap", c_i64), ("cell_tol", c_dbl)]


class map_particles_in(ctypes.Structure):
    _fields_ = [("n", c_i64), ("xyz", c_vp), ("m", c_vp), ("h", c_vp), ("mem_kind", c_int)]


class map_cells_in(ctypes.Structure):
    _fields_ = [("n_cells", c_i64), ("n_faces", c_i64), ("n_face_verts", c_i64), ("n_verts", c_i64),
                ("cell_face_off", c_vp), ("face_vert_off", c_vp), ("face_vert", c_vp), ("face_plane", c_vp),
                ("verts", c_vp), ("cell_volume", c_vp), ("box", c_dbl * 6), ("mem_kind", c_int)]


class map_voronoi_out(ctypes.Structure):
    _fields_ = [("n_cells", c_i64), ("n_faces", c_i64), ("n_face_verts", c_i64), ("n_verts", c_i64),
                ("cells", map_cells_in), ("face_nb", c_vp), ("sites", c_vp), ("centroid", c_vp),
                ("n_sites", c_i64), ("site_cell", c_vp), ("ms", c_dbl)]


class map_stats(ctypes.Structure):
    _fields_ = [("n_pairs", c_i64), ("n_candidates", c_i64), ("n_edge_terms", c_i64), ("n_fixup_terms", c_i64),
                ("n_face_visits", c_i64), ("n_edge_visits", c_i64), ("n_moment_evals", c_i64),
                ("n_quad_intervals", c_i64), ("n_angle_evals", c_i64), ("n_quad_points", c_i64),
                ("n_boundary_pairs", c_i64), ("n_fp64_cells", c_i64), ("n_fp64_pairs", c_i64),
                ("mass_in", c_dbl), ("mass_out", c_dbl), ("max_abs_S_minus_1", c_dbl), ("ms_setup", c_dbl),
                ("ms_pairs", c_dbl), ("ms_integrate", c_dbl), ("ms_fixup", c_dbl), ("ms_reduce", c_dbl),
                ("ms_total", c_dbl), ("ms_queue", c_dbl), ("ms_latency", c_dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class map_out(ctypes.Structure):
    _fields_ = [("cell_mass", c_vp), ("cell_density", c_vp), ("frac_sum_raw", c_vp), ("pair_frac", c_vp),
                ("pair_p", c_vp), ("pair_c", c_vp), ("pair_capacity", c_i64), ("mem_kind", c_int),
                ("stats", ctypes.POINTER(map_stats))]


PSEUDO_NODE, PSEUDO_PARTICLE = 0, 1


class map_pseudo_params(ctypes.Structure):
    _fields_ = [("theta", c_dbl), ("r_part", c_dbl), ("r_leaf", c_dbl), ("leaf_size", c_int), ("h_fact_node", c_dbl)]


class map_pseudo_stats(ctypes.Structure):
    _fields_ = [(k, c_i64) for k in ("n_tree_nodes", "n_leaves", "max_level", "n_pseudo", "n_pseudo_nodes",
                                     "n_particles", "n_substitute_leaves", "n_fallbacks", "n_h_evals",
                                     "n_neighbours")] + \
               [(k, c_dbl) for k in ("ms_tree", "ms_walk", "ms_hsolve", "ms_total")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class map_pseudo_out(ctypes.Structure):
    _fields_ = [("capacity", c_i64), ("xyz", c_vp), ("m", c_vp), ("h", c_vp), ("size", c_vp), ("kind", c_vp),
                ("ref", c_vp), ("mem_kind", c_int), ("n_out", c_i64), ("stats", ctypes.POINTER(map_pseudo_stats))]


# neutral-fraction callback of the adaptive walk (host arrays)
NEUTRAL_FN = ctypes.CFUNCTYPE(c_int, c_vp, c_i64, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl),
                              ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(c_dbl))


class map_adapt_params(ctypes.Structure):
    _fields_ = [("K", c_dbl), ("max_walks", c_int), ("neutral", NEUTRAL_FN), ("user", c_vp)]


class map_adapt_stats(ctypes.Structure):
    _fields_ = [(k, c_i64) for k in ("n_walks", "converged", "n_failed", "n_r_part_growths", "n_regions_in",
                                     "n_regions_dropped", "n_regions_out")] + \
               [(k, c_dbl) for k in ("r_part", "r_leaf", "s_root", "ms_tree", "ms_walks", "ms_callback",
                                     "ms_total")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "map_init": (c_int, [ctypes.POINTER(map_config), ctypes.POINTER(c_vp)]),
    "map_shutdown": (c_int, [c_vp]),
    "map_last_error": (ctypes.c_char_p, [c_vp]),
    "map_set_precision": (c_int, [c_vp, c_int]),
    "map_set_tune": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_int]),
    "map_get_tune": (c_int, [c_vp, c_int, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "map_autotune": (c_int, [c_vp, ctypes.POINTER(map_particles_in), ctypes.POINTER(map_cells_in), c_int, c_vp,
                             c_vp]),
    "map_pairs": (c_int, [c_vp, ctypes.POINTER(map_particles_in), ctypes.POINTER(map_cells_in), c_vp, c_vp, c_vp,
                          c_i64]),
    "map_particles": (c_int, [c_vp, ctypes.POINTER(map_particles_in), ctypes.POINTER(map_cells_in),
                              ctypes.POINTER(map_out)]),
    "map_back": (c_int, [c_vp, c_vp, c_int, c_vp, c_int]),
    "map_particles_noalloc": (c_int, [c_vp, ctypes.POINTER(map_particles_in), ctypes.POINTER(map_cells_in),
                                      ctypes.POINTER(map_out)]),
    "map_submit": (c_int, [c_vp, ctypes.POINTER(map_particles_in), ctypes.POINTER(map_cells_in),
                           ctypes.POINTER(map_out), ctypes.POINTER(c_u64)]),
    "map_poll": (c_int, [c_vp, c_u64, c_i64, ctypes.POINTER(c_int)]),
    "map_pseudo": (c_int, [c_vp, ctypes.POINTER(map_particles_in), ctypes.POINTER(c_dbl * 6), c_vp, c_int,
                           ctypes.POINTER(map_pseudo_params), ctypes.POINTER(map_pseudo_out)]),
    "map_pseudo_adaptive": (c_int, [c_vp, ctypes.POINTER(map_particles_in), ctypes.POINTER(c_dbl * 6), c_vp, c_int,
                                    ctypes.POINTER(map_pseudo_params), ctypes.POINTER(map_adapt_params),
                                    ctypes.POINTER(map_pseudo_out), ctypes.POINTER(map_adapt_stats)]),
    "map_get_regions": (c_int, [c_vp, c_i64, c_vp, ctypes.POINTER(c_i64)]),
    "map_set_table": (c_int, [c_vp, c_int, c_int, c_int]),
    "map_voronoi": (c_int, [c_vp, c_i64, c_vp, c_int, ctypes.POINTER(c_dbl * 6), c_int, c_dbl,
                            ctypes.POINTER(map_voronoi_out)]),
    "map_voronoi_copy": (c_int, [c_vp, c_int] + [c_vp] * 10),
    "map_get_table": (c_int, [c_vp, c_vp]),
    "map_set_regions": (c_int, [c_vp, c_i64, c_vp]),
}


def _runtime_of_torch():
    """Load torch (the plumbing for device memory and streams) before the library.

    torch ships a HIP runtime of its own whose soname equals the system one's;
    when torch is in the process first, the library binds to that same runtime
    and one runtime serves both.  Loading the library first would map the
    system runtime and then torch's as a second one."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def hip_runtimes_mapped():
    """Distinct libamdhip64 files mapped into this process."""
    seen = []
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                path = line.split()[-1] if "/" in line else ""
                if "libamdhip64" in path and path not in seen:
                    seen.append(path)
    except OSError:
        pass
    return seen


def load():
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libexactmap is not built ({LIB_PATH}); run __graft_entry__.build() first")
        _runtime_of_torch()
        lib = ctypes.CDLL(LIB_PATH)
        rts = hip_runtimes_mapped()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes are mapped into this process ({rts}); import torch before "
                               f"anything else that loads a HIP runtime")
        for name, (res, args) in _SIGS.items():
            if hasattr(lib, name):
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
        _lib = lib
    return _lib


def _check(ctx, rc):
    if rc != MAP_OK:
        msg = load().map_last_error(ctx if ctx else None)
        raise MapError(rc, (msg or b"").decode())


# ---------------------------------------------------------------- marshalling
def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        assert x.is_contiguous()
        return x.data_ptr()
    assert isinstance(x, np.ndarray) and x.flags["C_CONTIGUOUS"]
    return x.ctypes.data


def _kind(x):
    return MAP_MEM_DEVICE if (_is_torch(x) and x.is_cuda) else MAP_MEM_HOST


@dataclass
class _Keep:
    """Holds contiguous arrays alive for the duration of a call."""
    items: list


def particles_in(xyz, m, h):
    keep = []

    def prep(a, dt):
        if _is_torch(a):
            a = a.contiguous()
        else:
            a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    xyz, m, h = prep(xyz, np.float64), prep(m, np.float64), prep(h, np.float64)
    n = int(h.shape[0])
    s = map_particles_in(n, _ptr(xyz), _ptr(m), _ptr(h), _kind(xyz))
    return s, _Keep(keep)


def cells_in(cells, device_arrays=None):
    """cells: a synth.Cells (host) or an object with the same fields as torch tensors (device)."""
    keep = []

    def prep(a, dt):
        if a is None:
            return None
        if _is_torch(a):
            a = a.contiguous()
        else:
            a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    cfo = prep(cells.cell_face_off, np.int64)
    fvo = prep(cells.face_vert_off, np.int64)
    fv = prep(cells.face_vert, np.int32)
    plane = prep(cells.face_plane, np.float64)
    verts = prep(cells.verts, np.float64)
    vol = prep(getattr(cells, "cell_volume", None), np.float64)
    box = (c_dbl * 6)(*[float(b) for b in cells.box])
    s = map_cells_in(int(cfo.shape[0]) - 1, int(plane.shape[0]), int(fv.shape[0]), int(verts.shape[0]), _ptr(cfo),
                     _ptr(fvo), _ptr(fv), _ptr(plane), _ptr(verts), _ptr(vol), box, _kind(cfo))
    return s, _Keep(keep)


# ---------------------------------------------------------------- ABI-named wrappers
def map_init(device: int = 0, precision: int = MAP_FP64, hbm_budget_bytes: int = 0, max_jobs: int = 0,
             max_queue: int = 0, tune_cache_path: str | None = None, serve_timeout_ms: int = 0,
             serve_trace: bool = False, fixup_cap: int = 0, cell_tol: float = 0.0):
    lib = load()
    cfg = map_config(device, precision, hbm_budget_bytes, max_jobs, max_queue,
                     tune_cache_path.encode() if tune_cache_path else None, int(serve_timeout_ms),
                     1 if serve_trace else 0, int(fixup_cap), float(cell_tol))
    ctx = c_vp()
    _check(None, lib.map_init(ctypes.byref(cfg), ctypes.byref(ctx)))
    return ctx


def map_shutdown(ctx):
    _check(None, load().map_shutdown(ctx))


def map_last_error(ctx) -> str:
    return (load().map_last_error(ctx) or b"").decode()


def map_set_precision(ctx, precision: int):
    _check(ctx, load().map_set_precision(ctx, precision))


def map_set_table(ctx, n0: int = 64, n1: int = 64, n2: int = 64):
    """Size of the MAP_TABLE table of the pyramid integral (rebuilt on next use)."""
    _check(ctx, load().map_set_table(ctx, int(n0), int(n1), int(n2)))


def map_get_table(ctx, shape):
    """FP64 node values of the table of the given (current) size, as an array of that shape."""
    out = np.zeros(tuple(int(x) for x in shape))
    _check(ctx, load().map_get_table(ctx, _ptr(out)))
    return out


def map_set_tune(ctx, precision, waves=0, tile_waves=1, grid_per_cu=8, persistent=1):
    """Explicit launch shape for one precision; persistent=-1 clears it."""
    _check(ctx, load().map_set_tune(ctx, precision, waves, tile_waves, grid_per_cu, persistent))


def map_get_tune(ctx, precision, n_pairs=1):
    v = [c_int() for _ in range(4)]
    _check(ctx, load().map_get_tune(ctx, precision, n_pairs, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def map_autotune(ctx, xyz, m, h, cells, precision):
    """Times the candidate launch shapes; returns ((waves, tile_waves, grid_per_cu, persistent), ms)."""
    lib = load()
    P, k1 = particles_in(xyz, m, h)
    C, k2 = cells_in(cells)
    best = (c_int * 4)()
    ms = c_dbl()
    _check(ctx, lib.map_autotune(ctx, ctypes.byref(P), ctypes.byref(C), precision, best, ctypes.byref(ms)))
    return tuple(best), ms.value


def map_pairs(ctx, xyz, m, h, cells, want_pairs: bool = True):
    """Exact pair set sorted by (cell, particle): returns (pair_p, pair_c) int32, or the count."""
    lib = load()
    P, k1 = particles_in(xyz, m, h)
    C, k2 = cells_in(cells)
    n = c_i64()
    _check(ctx, lib.map_pairs(ctx, ctypes.byref(P), ctypes.byref(C), ctypes.byref(n), None, None, 0))
    if not want_pairs:
        return int(n.value)
    pp = np.zeros(n.value, np.int32)
    pc = np.zeros(n.value, np.int32)
    _check(ctx, lib.map_pairs(ctx, ctypes.byref(P), ctypes.byref(C), ctypes.byref(n), _ptr(pp), _ptr(pc),
                              pp.size))
    return pp, pc


def map_particles(ctx, xyz, m, h, cells, cell_mass=None, cell_density=None, frac_sum_raw=None, pair_frac=None,
                  pair_p=None, pair_c=None):
    """Synchronous mapping.  Output arrays (numpy or torch CUDA, all of one kind) are
    filled in place when given.  Returns the statistics as a dict."""
    lib = load()
    P, k1 = particles_in(xyz, m, h)
    C, k2 = cells_in(cells)
    st = map_stats()
    outs = [x for x in (cell_mass, cell_density, frac_sum_raw, pair_frac, pair_p, pair_c) if x is not None]
    kind = _kind(outs[0]) if outs else MAP_MEM_HOST
    cap = 0
    for x in (pair_frac, pair_p, pair_c):
        if x is not None:
            cap = int(x.shape[0]) if cap == 0 else min(cap, int(x.shape[0]))
    O = map_out(_ptr(cell_mass), _ptr(cell_density), _ptr(frac_sum_raw), _ptr(pair_frac), _ptr(pair_p),
                _ptr(pair_c), cap, kind, ctypes.pointer(st))
    _last_n.pop(_ctx_key(ctx), None)
    _check(ctx, lib.map_particles(ctx, ctypes.byref(P), ctypes.byref(C), ctypes.byref(O)))
    _last_n[_ctx_key(ctx)] = int(P.n)
    return st.as_dict()


def map_particles_noalloc(ctx, xyz, m, h, cells, cell_mass=None, cell_density=None, frac_sum_raw=None):
    """map_particles with no device allocation (fixed scratch array): inputs and outputs must be
    contiguous torch CUDA float64/int tensors already of the right size.  Returns the statistics."""
    lib = load()
    P, k1 = particles_in(xyz, m, h)
    C, k2 = cells_in(cells)
    st = map_stats()
    outs = [x for x in (cell_mass, cell_density, frac_sum_raw) if x is not None]
    kind = _kind(outs[0]) if outs else MAP_MEM_DEVICE
    O = map_out(_ptr(cell_mass), _ptr(cell_density), _ptr(frac_sum_raw), None, None, None, 0, kind,
                ctypes.pointer(st))
    _check(ctx, lib.map_particles_noalloc(ctx, ctypes.byref(P), ctypes.byref(C), ctypes.byref(O)))
    _last_n.pop(_ctx_key(ctx), None)
    return st.as_dict()


def map_back(ctx, cell_values, out=None):
    """Inverse mapping (Eq. (4)) with the pairs of the context's last map_particles:
    particle values from cell values.  cell_values: numpy or torch CUDA float64;
    out: a preallocated array of the particle count (numpy or torch CUDA), or
    None for a new numpy array (its length is the last mapping's particle count)."""
    lib = load()
    if _is_torch(cell_values):
        q = cell_values.contiguous()
    else:
        q = np.ascontiguousarray(cell_values, dtype=np.float64)
    if out is None:
        n = _last_n.get(_ctx_key(ctx))
        if n is None:
            raise MapError(MAP_EINVAL, "map_back: no mapping of this context to invert")
        out = np.zeros(n)
    _check(ctx, lib.map_back(ctx, _ptr(q), _kind(q), _ptr(out), _kind(out)))
    return out


# particle count of each context's last map_particles call (size of map_back's result)
_last_n = {}


def _ctx_key(ctx):
    return ctx.value if isinstance(ctx, ctypes.c_void_p) else int(ctx)


# Served jobs: references the library may still write to, kept until the job is reported finished.
_SERVED = {}


def map_submit(ctx, xyz, m, h, cells, cell_mass=None, cell_density=None, frac_sum_raw=None):
    """Queue a mapping job (inputs are copied before this returns); returns the job id.

    The output arrays (numpy or torch CUDA, all of one kind) are filled when the
    job completes; they are kept referenced here until map_poll reports it."""
    lib = load()
    P, k1 = particles_in(xyz, m, h)
    C, k2 = cells_in(cells)
    st = map_stats()
    outs = [x for x in (cell_mass, cell_density, frac_sum_raw) if x is not None]
    kind = _kind(outs[0]) if outs else MAP_MEM_HOST
    O = map_out(_ptr(cell_mass), _ptr(cell_density), _ptr(frac_sum_raw), None, None, None, 0, kind,
                ctypes.pointer(st))
    jid = c_u64()
    _check(ctx, lib.map_submit(ctx, ctypes.byref(P), ctypes.byref(C), ctypes.byref(O), ctypes.byref(jid)))
    # outputs, statistics and borrowed device inputs stay referenced until the job has finished
    _SERVED[(ctx.value, jid.value)] = (O, st, outs, k1, k2, xyz, m, h, cells)
    return jid.value


def map_poll(ctx, job_id, timeout_us=-1):
    """Job state (JOB_PENDING/RUNNING/DONE/FAILED) and, once finished, its statistics.

    Raises MapError when the job failed (its error code and message)."""
    state = c_int()
    rc = load().map_poll(ctx, job_id, timeout_us, ctypes.byref(state))
    key = (ctx.value, job_id)
    if state.value in (JOB_DONE, JOB_FAILED) or rc == MAP_ENOTFOUND:
        held = _SERVED.pop(key, None)
        if rc != MAP_OK:
            _check(ctx, rc)
        return state.value, (held[1].as_dict() if held else None)
    _check(ctx, rc)
    return state.value, None


def map_pseudo(ctx, xyz, m, h, box, sources, theta=0.5, r_part=0.05, r_leaf=0.1, leaf_size=8, h_fact_node=1.1,
               out=None, capacity=None):
    """Pseudo-particles of the particles (Sec. III), in Morton order.

    Returns (count, stats) when capacity == 0, else a dict of xyz, m, h, size,
    kind, ref and stats.  `out` may hold preallocated arrays (numpy or torch
    CUDA, all of one kind) under those names with at least `capacity` rows."""
    lib = load()
    P, k1 = particles_in(xyz, m, h)
    bx = (c_dbl * 6)(*[float(b) for b in box])
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.float64).reshape(-1, 3))
    par = map_pseudo_params(float(theta), float(r_part), float(r_leaf), int(leaf_size), float(h_fact_node))
    st = map_pseudo_stats()
    n = int(P.n)
    if capacity is None:
        capacity = max(n, 1) if out is None else int(out["m"].shape[0])
    if out is None and capacity > 0:
        out = dict(xyz=np.zeros((capacity, 3)), m=np.zeros(capacity), h=np.zeros(capacity),
                   size=np.zeros(capacity), kind=np.zeros(capacity, np.int32), ref=np.zeros(capacity, np.int64))
    arrs = [out[k] if out is not None else None for k in ("xyz", "m", "h", "size", "kind", "ref")]
    kind = _kind(arrs[1]) if out is not None else MAP_MEM_HOST
    O = map_pseudo_out(int(capacity), *[_ptr(a) for a in arrs], kind, 0, ctypes.pointer(st))
    _check(ctx, lib.map_pseudo(ctx, ctypes.byref(P), ctypes.byref(bx), _ptr(src), src.shape[0], ctypes.byref(par),
                               ctypes.byref(O)))
    cnt = int(O.n_out)
    if capacity == 0:
        return cnt, st.as_dict()
    res = {k: out[k][:cnt] for k in ("xyz", "m", "h", "size", "kind", "ref")}
    res["stats"] = st.as_dict()
    return res


def map_pseudo_adaptive(ctx, xyz, m, h, box, sources, neutral, K=100.0, max_walks=32, theta=0.5, r_part=0.05,
                        r_leaf=0.1, leaf_size=8, h_fact_node=1.1):
    """Adaptive tree walk (Sec. III-B, Eq. (6)) with the context's remembered regions.

    neutral(P) returns the neutral fraction of each pseudo-particle of the set
    P (a dict of host arrays xyz, m, h, size, kind).  Returns the final set
    (as map_pseudo, host arrays) with "stats" and "adapt" (walks, radii,
    region counts)."""
    lib = load()
    P, k1 = particles_in(xyz, m, h)
    bx = (c_dbl * 6)(*[float(b) for b in box])
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.float64).reshape(-1, 3))
    par = map_pseudo_params(float(theta), float(r_part), float(r_leaf), int(leaf_size), float(h_fact_node))
    raised = []

    def cb(user, n, px, pm, ph, ps, pk, pf):
        try:
            if n > 0:
                S = dict(xyz=np.ctypeslib.as_array(px, (n, 3)), m=np.ctypeslib.as_array(pm, (n,)),
                         h=np.ctypeslib.as_array(ph, (n,)), size=np.ctypeslib.as_array(ps, (n,)),
                         kind=np.ctypeslib.as_array(pk, (n,)))
                np.ctypeslib.as_array(pf, (n,))[:] = np.asarray(neutral(S), dtype=np.float64).reshape(n)
            return 0
        except Exception as e:  # re-raised once the call has returned
            raised.append(e)
            return 1

    fn = NEUTRAL_FN(cb)
    ap = map_adapt_params(float(K), int(max_walks), fn, None)
    n = int(P.n)
    cap = max(n, 1)
    out = dict(xyz=np.zeros((cap, 3)), m=np.zeros(cap), h=np.zeros(cap), size=np.zeros(cap),
               kind=np.zeros(cap, np.int32), ref=np.zeros(cap, np.int64))
    st = map_pseudo_stats()
    ast = map_adapt_stats()
    O = map_pseudo_out(cap, *[_ptr(out[k]) for k in ("xyz", "m", "h", "size", "kind", "ref")], MAP_MEM_HOST, 0,
                       ctypes.pointer(st))
    rc = lib.map_pseudo_adaptive(ctx, ctypes.byref(P), ctypes.byref(bx), _ptr(src), src.shape[0],
                                 ctypes.byref(par), ctypes.byref(ap), ctypes.byref(O), ctypes.byref(ast))
    if raised:
        raise raised[0]
    _check(ctx, rc)
    cnt = int(O.n_out)
    res = {k: out[k][:cnt] for k in ("xyz", "m", "h", "size", "kind", "ref")}
    res["stats"] = st.as_dict()
    res["adapt"] = ast.as_dict()
    return res


class VoronoiCells:
    """Box-clipped Voronoi cells in the library's cell format (numpy or torch CUDA arrays)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    @property
    def n_cells(self) -> int:
        return int(self.cell_face_off.shape[0]) - 1


def map_voronoi_copy(ctx, mem_kind, cell_face_off=None, face_vert_off=None, face_vert=None, face_plane=None,
                     face_nb=None, verts=None, cell_volume=None, centroid=None, sites=None, site_cell=None):
    """Copies the context's last Voronoi grid into the given arrays (None skips one)."""
    arrs = (cell_face_off, face_vert_off, face_vert, face_plane, face_nb, verts, cell_volume, centroid, sites,
            site_cell)
    _check(ctx, load().map_voronoi_copy(ctx, mem_kind, *[_ptr(a) for a in arrs]))


def map_voronoi(ctx, sites, box, lloyd_iters=0, merge_dist=0.0, device=False):
    """Voronoi grid of the sites (Sec. II-A), tightly packed sites merged, after lloyd_iters Lloyd iterations.

    Returns VoronoiCells with cell_face_off, face_vert_off, face_vert, face_plane, verts,
    cell_volume, face_nb, centroid, sites, site_cell, box and ms; host numpy arrays, or torch
    CUDA tensors when device=True."""
    lib = load()
    if _is_torch(sites):
        s = sites.contiguous()
    else:
        s = np.ascontiguousarray(np.asarray(sites, dtype=np.float64).reshape(-1, 3))
    bx = (c_dbl * 6)(*[float(b) for b in box])
    out = map_voronoi_out()
    _check(ctx, lib.map_voronoi(ctx, int(s.shape[0]), _ptr(s), _kind(s), ctypes.byref(bx), int(lloyd_iters),
                                float(merge_dist), ctypes.byref(out)))
    n, nf, ns, nv = int(out.n_cells), int(out.n_faces), int(out.n_face_verts), int(out.n_verts)
    n_in = int(out.n_sites)
    shapes = dict(cell_face_off=((n + 1,), np.int64), face_vert_off=((nf + 1,), np.int64),
                  face_vert=((ns,), np.int32), face_plane=((nf, 4), np.float64), face_nb=((nf,), np.int64),
                  verts=((nv, 3), np.float64), cell_volume=((n,), np.float64), centroid=((n, 3), np.float64),
                  sites=((n, 3), np.float64), site_cell=((n_in,), np.int64))
    if device:
        import torch
        tdt = {np.int64: torch.int64, np.int32: torch.int32, np.float64: torch.float64}
        arr = {k: torch.empty(sh, dtype=tdt[dt], device="cuda") for k, (sh, dt) in shapes.items()}
        kind = MAP_MEM_DEVICE
    else:
        arr = {k: np.zeros(sh, dtype=dt) for k, (sh, dt) in shapes.items()}
        kind = MAP_MEM_HOST
    order = ("cell_face_off", "face_vert_off", "face_vert", "face_plane", "face_nb", "verts", "cell_volume",
             "centroid", "sites", "site_cell")
    map_voronoi_copy(ctx, kind, *[arr[k] for k in order])
    return VoronoiCells(box=tuple(float(b) for b in box), ms=float(out.ms), **arr)


def map_get_regions(ctx):
    """The context's remembered regions, an (n, 5) array of cx, cy, cz, R, s_min."""
    lib = load()
    n = c_i64()
    _check(ctx, lib.map_get_regions(ctx, 0, None, ctypes.byref(n)))
    out = np.zeros((n.value, 5))
    if n.value:
        _check(ctx, lib.map_get_regions(ctx, n.value, _ptr(out), ctypes.byref(n)))
    return out


def map_set_regions(ctx, regions):
    """Replaces the context's remembered regions (rows cx, cy, cz, R, s_min)."""
    r = np.ascontiguousarray(np.asarray(regions, dtype=np.float64).reshape(-1, 5))
    _check(ctx, load().map_set_regions(ctx, r.shape[0], _ptr(r) if r.size else None))


class Mapper:
    """Owns one library context."""

    def __init__(self, device: int = 0, precision: int = MAP_FP64, **kw):
        self.ctx = map_init(device, precision, **kw)

    def close(self):
        if self.ctx:
            map_shutdown(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_precision(self, precision):
        map_set_precision(self.ctx, precision)

    def voronoi(self, sites, box, lloyd_iters=0, merge_dist=0.0, device=False):
        return map_voronoi(self.ctx, sites, box, lloyd_iters, merge_dist, device)

    def set_table(self, n0=64, n1=64, n2=64):
        map_set_table(self.ctx, n0, n1, n2)
        self._table_shape = (n0, n1, n2)

    def table(self):
        return map_get_table(self.ctx, getattr(self, "_table_shape", (64, 64, 64)))

    def back(self, cell_values, out=None):
        """Inverse mapping with the pairs of this mapper's last map()."""
        return map_back(self.ctx, cell_values, out)

    def pseudo(self, particles, box, sources, **kw):
        return map_pseudo(self.ctx, particles.xyz, particles.m, particles.h, box, sources, **kw)

    def pseudo_adaptive(self, particles, box, sources, neutral, **kw):
        return map_pseudo_adaptive(self.ctx, particles.xyz, particles.m, particles.h, box, sources, neutral, **kw)

    @property
    def regions(self):
        return map_get_regions(self.ctx)

    @regions.setter
    def regions(self, value):
        map_set_regions(self.ctx, value)

    def pairs(self, particles, cells):
        return map_pairs(self.ctx, particles.xyz, particles.m, particles.h, cells)

    def map(self, particles, cells, want_pairs=False):
        """Host convenience: returns dict with M, rho, S (and per-pair data if asked)."""
        nc = cells.cell_face_off.shape[0] - 1
        M = np.zeros(nc)
        rho = np.zeros(nc)
        S = np.zeros(particles.h.shape[0])
        res = {}
        if want_pairs:
            npairs = map_pairs(self.ctx, particles.xyz, particles.m, particles.h, cells, want_pairs=False)
            f = np.zeros(npairs)
            pp = np.zeros(npairs, np.int32)
            pc = np.zeros(npairs, np.int32)
            st = map_particles(self.ctx, particles.xyz, particles.m, particles.h, cells, M, rho, S, f, pp, pc)
            res.update(f=f, pair_p=pp, pair_c=pc)
        else:
            st = map_particles(self.ctx, particles.xyz, particles.m, particles.h, cells, M, rho, S)
        res.update(M=M, rho=rho, S=S, stats=st)
        return res
