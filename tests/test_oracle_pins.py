"""Pins of the FP64 oracle against what the mathematics fixes.

Every check here uses something other than the oracle's own formulas: direct
numerical quadrature of the kernel, closed forms of simple solids, exact
geometric identities, or brute-force integration over tiny inputs.  A dropped
term, a wrong sign, a swapped index or a transposed operand anywhere in the
oracle's closed form or its signed assembly fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import ConvexHull

import oracle
import synth
from synth import Cells

PI = math.pi


# ------------------------------------------------------------------ helpers
def w_m4(q):
    """M4 cubic spline shape, written from its definition (Sec. III-C names it)."""
    q = abs(q)
    if q < 1:
        return 1 - 1.5 * q * q + 0.75 * q ** 3
    if q < 2:
        return 0.25 * (2 - q) ** 3
    return 0.0


def F_quad(s):
    """Kernel mass per unit solid angle within radius s, by quadrature (h = 1)."""
    pts = [x for x in (1.0,) if x < s]
    return integrate.quad(lambda q: w_m4(q) * q * q / PI, 0, min(s, 2.0), points=pts or None,
                          epsabs=1e-15, epsrel=1e-14, limit=200)[0]


def pyramid_3d(r0, R0, phi):
    """Integral of W over the right-angled pyramid, straight from the volume integral.

    Points of the pyramid are x = u*b with b = (rho cos a, rho sin a, r0) on the
    base triangle (0 <= a <= phi, 0 <= rho <= R0/cos a) and 0 <= u <= 1; the volume
    element is u^2 r0 rho drho da du.  No radial antiderivative is used.
    """
    def inner(a):
        rmax = R0 / math.cos(a)

        def over_rho(rho):
            b = math.sqrt(rho * rho + r0 * r0)
            brk = [1.0 / b, 2.0 / b]
            pts = [x for x in brk if x < 1.0]
            val = integrate.quad(lambda u: u * u * w_m4(u * b) / PI, 0.0, 1.0, points=pts or None,
                                 epsabs=1e-15, epsrel=1e-13, limit=200)[0]
            return val * r0 * rho
        # breakpoints in rho where b crosses 1 and 2
        pts = [math.sqrt(k * k - r0 * r0) for k in (1.0, 2.0) if k > r0 and math.sqrt(k * k - r0 * r0) < rmax]
        return integrate.quad(over_rho, 0.0, rmax, points=pts or None, epsabs=1e-14, epsrel=1e-12, limit=200)[0]

    pts = [math.atan(math.sqrt(k * k - r0 * r0 - R0 * R0) / R0) for k in (1.0, 2.0)
           if k * k > r0 * r0 + R0 * R0]
    pts = [x for x in pts if x < phi]
    return integrate.quad(inner, 0.0, phi, points=pts or None, epsabs=1e-13, epsrel=1e-11, limit=200)[0]


def half_space(u):
    """Kernel mass beyond a plane at distance u (h = 1), by nested quadrature.

    Phi(u) = int_{z>u} W dV = 2 int_u^2 dz int_z^2 s w(s) ds.
    """
    if u >= 2:
        return 0.0
    inner = lambda z: integrate.quad(lambda s: s * w_m4(s), z, 2.0, points=[1.0] if z < 1 else None,
                                     epsabs=1e-15, epsrel=1e-14)[0]
    return 2.0 * integrate.quad(inner, u, 2.0, points=[1.0] if u < 1 else None, epsabs=1e-15, epsrel=1e-13)[0]


def box_cell(lo, hi):
    """One axis-aligned box as a single cell, faces counter-clockwise from outside."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    P = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], dtype=float)
    faces = [([-1, 0, 0], -x0, [0, 4, 7, 3]), ([1, 0, 0], x1, [1, 2, 6, 5]),
             ([0, -1, 0], -y0, [0, 1, 5, 4]), ([0, 1, 0], y1, [3, 7, 6, 2]),
             ([0, 0, -1], -z0, [0, 3, 2, 1]), ([0, 0, 1], z1, [4, 5, 6, 7])]
    plane = np.array([n + [c] for n, c, _ in faces], dtype=float)
    fv = np.array([0, 4, 8, 12, 16, 20, 24], dtype=np.int64)
    fvert = np.array(sum((v for _, _, v in faces), []), dtype=np.int32)
    vol = float(np.prod(np.subtract(hi, lo)))
    return Cells(np.array([0, 6], dtype=np.int64), fv, fvert, plane, -np.arange(1, 7, dtype=np.int64), P,
                 np.array([vol]), tuple(lo) + tuple(hi))


# ------------------------------------------------------------------ P0: the kernel profile
def test_w_is_the_m4_spline():
    """w(q) is the M4 cubic spline of Sec. III-C up to its normalisation: w(0) = 1, zero from q = 2
    on, value and slope continuous at the piece boundaries q = 1 and 2 (finite differences), a
    cubic on each piece (four samples fix the cubic, others lie on it), and sigma = 1/pi makes it
    integrate to one over 3-D space."""
    assert oracle.w(0.0) == 1.0
    for q in (2.0, 2.5, 7.0):
        assert oracle.w(q) == 0.0
    h = 1e-6
    for q in (1.0, 2.0):
        lo, hi = oracle.w(q - h), oracle.w(q + h)
        assert abs(hi - lo) < 1e-5
        dl = (oracle.w(q - h) - oracle.w(q - 2 * h)) / h
        dr = (oracle.w(q + 2 * h) - oracle.w(q + h)) / h
        assert abs(dl - dr) < 1e-4
    # exactly cubic on each piece: four samples determine the cubic, a fifth lies on it
    for a, b in ((0.05, 0.95), (1.05, 1.95)):
        xs = np.linspace(a, b, 4)
        c = np.polyfit(xs, [oracle.w(x) for x in xs], 3)
        for x in np.linspace(a, b, 9):
            assert oracle.w(x) == pytest.approx(np.polyval(c, x), abs=1e-14)
    total = integrate.quad(lambda q: oracle.w(q) * q * q, 0.0, 2.0, points=[1.0], epsabs=1e-15)[0]
    assert 4.0 * PI * total / PI == pytest.approx(1.0, abs=1e-13)


# ------------------------------------------------------------------ P1: radial profile
@pytest.mark.parametrize("s", [0.1, 0.5, 0.9, 1.0, 1.3, 1.7, 1.99, 2.0, 3.0])
def test_F_is_kernel_mass_per_steradian(s):
    assert oracle.F(s) == pytest.approx(F_quad(s), abs=1e-15, rel=1e-13)


def test_F_total_is_one_over_four_pi():
    assert oracle.F(2.0) * 4 * PI == pytest.approx(1.0, abs=1e-15)
    assert oracle.F(7.0) * 4 * PI == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("s", [0.2, 0.7, 1.2, 1.6, 1.9, 2.5])
def test_G_derivative_is_F_over_s2(s):
    eps = 1e-5
    d = (oracle.G(s + eps) - oracle.G(s - eps)) / (2 * eps)
    assert d == pytest.approx(oracle.F(s) / s ** 2, rel=1e-8)


@pytest.mark.parametrize("s", [1.0, 2.0])
def test_G_and_F_continuous_at_piece_radii(s):
    e = 1e-12
    assert abs(oracle.G(s - e) - oracle.G(s + e)) < 1e-11
    assert abs(oracle.F(s - e) - oracle.F(s + e)) < 1e-11


# ------------------------------------------------------------------ P2: angular moments
@pytest.mark.parametrize("r0,R0,al", [(0.37, 0.81, 1.1), (0.2, 0.3, 1.4), (1.3, 0.4, 0.9), (1e-3, 0.5, 1.2),
                                      (0.4, 1e-3, 1.2), (1.7, 1.1, 0.3)])
def test_moments_match_quadrature(r0, R0, al):
    got = oracle.moments(r0, R0, al)
    for k, n in enumerate([-1, 0, 2, 3, 4, 5]):
        ref = integrate.quad(lambda x: (r0 * r0 + R0 * R0 / math.cos(x) ** 2) ** (n / 2.0), 0, al,
                             epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        if n == -1:
            ref *= r0
        assert got[k] == pytest.approx(ref, rel=2e-13, abs=1e-15), n


# ------------------------------------------------------------------ P3: pyramid vs 3-D integral
@pytest.mark.parametrize("r0,R0,phi", [(0.37, 0.81, 1.1), (0.2, 0.3, 1.4), (1.3, 0.4, 0.9), (0.5, 1.7, 0.6),
                                       (2.5, 0.5, 1.0), (0.05, 0.5, 1.2), (0.4, 0.02, 1.2), (0.9, 0.9, 0.785)])
def test_pyramid_matches_volume_integral(r0, R0, phi):
    ref = pyramid_3d(r0, R0, phi)
    assert oracle.pyramid(r0, R0, phi) == pytest.approx(ref, rel=1e-9, abs=1e-13)


# ------------------------------------------------------------------ P4: constant kernel gives volume
def test_unit_profile_pyramid_is_volume():
    for r0, R0, phi in [(0.3, 0.7, 0.4), (2.0, 1.0, 1.3), (0.01, 3.0, 0.2)]:
        assert oracle.pyramid(r0, R0, phi, oracle.UNIT) == pytest.approx(r0 * R0 * R0 * math.tan(phi) / 6, rel=1e-13)


def test_unit_profile_cell_volume_matches_convex_hull():
    p, c = synth.workload("uniform", 300, 11)
    rng = np.random.default_rng(5)
    for i in rng.choice(c.n_cells, 25, replace=False):
        hull = ConvexHull(c.cell_vertices(int(i))).volume
        # any apex works, inside or outside the cell
        for apex in (p.xyz[i], np.array([0.5, 0.5, 0.5]), np.array([1.7, -0.4, 0.2])):
            v = oracle.pair_fraction(apex, 1.0, c, int(i), profile=oracle.UNIT)
            assert v == pytest.approx(hull, rel=1e-10, abs=1e-15)


# ------------------------------------------------------------------ P5: far pyramids are solid angles
def solid_angle(a, b, c):
    """Van Oosterom-Strackee solid angle of triangle (a, b, c) seen from the origin."""
    la, lb, lc = (np.linalg.norm(x) for x in (a, b, c))
    num = abs(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2 * math.atan2(num, den)


@pytest.mark.parametrize("r0,R0,phi", [(2.0, 0.5, 1.0), (2.5, 0.1, 1.5), (3.0, 4.0, 0.7)])
def test_far_pyramid_is_solid_angle(r0, R0, phi):
    f = np.array([0, 0, r0])
    g = np.array([R0, 0, r0])
    v = np.array([R0, R0 * math.tan(phi), r0])
    ref = solid_angle(f, g, v) / (4 * PI)
    assert oracle.pyramid(r0, R0, phi) == pytest.approx(ref, rel=1e-12)


# ------------------------------------------------------------------ P6: cube about the particle
def test_cube_fractions():
    # 48 right pyramids make a cube of half-side L centred on the particle.
    for L in (2.0, 2.5, 4.0):
        assert 48 * oracle.pyramid(L, L, PI / 4) == pytest.approx(1.0, abs=1e-14)
    # sqrt(2) <= L <= 2: only the six face caps leave the cube; 1.5 gives 1 - 6/768 exactly
    assert 48 * oracle.pyramid(1.5, 1.5, PI / 4) == pytest.approx(127.0 / 128.0, abs=1e-14)
    for L in (1.45, 1.8):
        assert 48 * oracle.pyramid(L, L, PI / 4) == pytest.approx(1 - 6 * half_space(L), abs=1e-13)


def test_cube_cell_assembly():
    # the same through the signed face/edge assembly on an actual cell, particle off-centre
    c = box_cell((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    f = oracle.pair_fraction(np.array([0.5, 0.5, 0.5]), 0.5 / 1.5, c, 0)
    assert f == pytest.approx(127.0 / 128.0, abs=1e-14)


# ------------------------------------------------------------------ P7: one wall
@pytest.mark.parametrize("u", [0.0, 0.3, 0.77, 1.0, 1.5, 1.93])
def test_single_wall_loses_half_space_mass(u):
    h = 0.1
    c = box_cell((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    p = np.array([u * h, 0.5, 0.5]) if u > 0 else np.array([1e-300, 0.5, 0.5])
    f = oracle.pair_fraction(p, h, c, 0)
    assert f == pytest.approx(1.0 - half_space(u), abs=2e-14)


def test_half_space_closed_values():
    assert half_space(0.0) == pytest.approx(0.5, abs=1e-14)
    assert half_space(1.0) == pytest.approx(1.0 / 30.0, abs=1e-14)
    assert half_space(1.5) == pytest.approx(1.0 / 768.0, abs=1e-15)


def test_particle_outside_box_opposite_wall():
    # particle outside the cell, beyond one wall: gets exactly the half-space mass
    h = 0.1
    c = box_cell((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    for u in (0.2, 1.1):
        f = oracle.pair_fraction(np.array([-u * h, 0.5, 0.5]), h, c, 0)
        assert f == pytest.approx(half_space(u), abs=2e-14)


# ------------------------------------------------------------------ P8, P9: partition of unity
def test_partition_of_unity_interior(uniform4k, uniform4k_oracle):
    p, c = uniform4k
    S = uniform4k_oracle["S"]
    inside = np.all((p.xyz - 2 * p.h[:, None] > 0) & (p.xyz + 2 * p.h[:, None] < 1), axis=1)
    assert inside.sum() > 1000
    assert np.abs(S[inside] - 1).max() < 1e-12
    assert np.all(S <= 1 + 1e-12) and np.all(S > 0.1)


def test_single_cell_whole_support():
    c = box_cell((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    assert oracle.pair_fraction(np.array([0.5, 0.5, 0.5]), 0.24, c, 0) == pytest.approx(1.0, abs=1e-14)
    assert oracle.pair_fraction(np.array([0.3, 0.6, 0.45]), 0.1, c, 0) == pytest.approx(1.0, abs=1e-14)


# ------------------------------------------------------------------ P10: brute force on tiny inputs
def _F_table():
    q = np.linspace(0, 2, 200001)
    wq = np.where(q < 1, 1 - 1.5 * q ** 2 + 0.75 * q ** 3, 0.25 * (2 - q) ** 3) * q * q / PI
    cum = np.concatenate([[0], np.cumsum((wq[1:] + wq[:-1]) * 0.5 * (q[1] - q[0]))])
    return q, cum


def ray_fraction(p, h, c, i, n_mu=160, n_az=320, table=None):
    """Integral of W over cell i by ray casting: for each direction the radial
    integral is the tabulated kernel mass between entry and exit distances."""
    q, cum = table
    mu, wmu = np.polynomial.legendre.leggauss(n_mu)
    az = (np.arange(n_az) + 0.5) * 2 * PI / n_az
    MU, AZ = np.meshgrid(mu, az, indexing="ij")
    st = np.sqrt(1 - MU ** 2)
    d = np.stack([st * np.cos(AZ), st * np.sin(AZ), MU], axis=-1).reshape(-1, 3)
    wts = (wmu[:, None] * np.full(n_az, 2 * PI / n_az)[None, :]).reshape(-1)
    t_in = np.zeros(d.shape[0])
    t_out = np.full(d.shape[0], np.inf)
    for j in range(c.cell_face_off[i], c.cell_face_off[i + 1]):
        n = c.face_plane[j, :3]
        cc = c.face_plane[j, 3]
        num = cc - n @ p
        den = d @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            t = num / den
        ent = den < 0
        ext = den > 0
        t_in = np.where(ent, np.maximum(t_in, t), t_in)
        t_out = np.where(ext, np.minimum(t_out, t), t_out)
        par = den == 0
        t_out = np.where(par & (num < 0), -np.inf, t_out)
    ok = t_out > t_in
    Fi = np.interp(np.clip(t_in / h, 0, 2), q, cum)
    Fo = np.interp(np.clip(np.where(np.isfinite(t_out), t_out, 1e9) / h, 0, 2), q, cum)
    return float(np.sum(np.where(ok, Fo - Fi, 0.0) * wts))


def test_brute_force_ray_quadrature_tiny():
    rng = np.random.default_rng(3)
    g = (np.stack(np.meshgrid([0.25, 0.75], [0.25, 0.75], [0.25, 0.75], indexing="ij"), -1).reshape(-1, 3)
         + 0.08 * (rng.random((8, 3)) - 0.5))
    c = synth.voronoi_cells(g)
    h = 0.12 + 0.1 * rng.random(8)
    table = _F_table()
    worst = 0.0
    for a in range(8):
        for i in range(8):
            ref = ray_fraction(g[a], h[a], c, i, table=table)
            got = oracle.pair_fraction(g[a], h[a], c, i)
            worst = max(worst, abs(ref - got))
    assert worst < 3e-5


# ------------------------------------------------------------------ P11: conservation and invariances
def test_mass_conserved(uniform4k, uniform4k_oracle):
    p, c = uniform4k
    assert abs(uniform4k_oracle["M"].sum() - p.m.sum()) < 1e-12


def test_translation_invariance():
    p, c = synth.workload("uniform", 200, 4)
    shift = np.array([0.3, -0.2, 0.1])
    c2 = Cells(c.cell_face_off, c.face_vert_off, c.face_vert,
               np.column_stack([c.face_plane[:, :3], c.face_plane[:, 3] + c.face_plane[:, :3] @ shift]),
               c.face_nb, c.verts + shift, c.cell_volume, tuple(np.add(c.box[:3], shift)) + tuple(np.add(c.box[3:], shift)))
    pp, pc = oracle.pairs(p.xyz, p.h, c)
    f1 = oracle.pair_fractions(p.xyz, p.h, c, pp, pc)
    f2 = oracle.pair_fractions(p.xyz + shift, p.h, c2, pp, pc)
    assert np.abs(f1 - f2).max() < 1e-12


def test_mirror_invariance():
    p, c = synth.workload("uniform", 200, 5)
    plane = c.face_plane.copy()
    plane[:, 3] = plane[:, 3] - plane[:, 0]
    plane[:, 0] = -plane[:, 0]
    verts = c.verts.copy()
    verts[:, 0] = 1 - verts[:, 0]
    fvert = c.face_vert.copy()
    for j in range(c.n_faces):  # mirroring flips orientation: reverse each face's vertex order
        a, b = c.face_vert_off[j], c.face_vert_off[j + 1]
        fvert[a:b] = fvert[a:b][::-1]
    cm = Cells(c.cell_face_off, c.face_vert_off, fvert, plane, c.face_nb, verts, c.cell_volume, c.box)
    xm = p.xyz.copy()
    xm[:, 0] = 1 - xm[:, 0]
    pp, pc = oracle.pairs(p.xyz, p.h, c)
    pp2, pc2 = oracle.pairs(xm, p.h, cm)
    assert np.array_equal(pp, pp2) and np.array_equal(pc, pc2)
    f1 = oracle.pair_fractions(p.xyz, p.h, c, pp, pc)
    f2 = oracle.pair_fractions(xm, p.h, cm, pp, pc)
    assert np.abs(f1 - f2).max() < 1e-12


def test_permutation_invariance():
    p, c = synth.workload("uniform", 300, 6)
    r1 = oracle.map_particles(p, c)
    perm = np.random.default_rng(0).permutation(p.n)
    p2 = synth.Particles(p.xyz[perm], p.m[perm], p.h[perm])
    r2 = oracle.map_particles(p2, c)
    assert np.abs(r1["M"] - r2["M"]).max() < 1e-15
    assert np.abs(r1["S"][perm] - r2["S"]).max() < 1e-15


# ------------------------------------------------------------------ pair set
def test_grid_pairs_equal_brute_force():
    p, c = synth.workload("clumps", 400, 7)
    a = oracle.pairs(p.xyz, p.h, c)
    b = oracle.pairs(p.xyz, p.h, c, brute=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_pair_set_is_support_of_integrand():
    """Non-pairs integrate to zero; pairs well inside the support integrate to > 0."""
    p, c = synth.workload("uniform", 64, 8)
    pp, pc = oracle.pairs(p.xyz, p.h, c)
    inset = set(zip(pp.tolist(), pc.tolist()))
    for a in range(p.n):
        for i in range(c.n_cells):
            f = oracle.pair_fraction(p.xyz[a], p.h[a], c, i)
            d = math.sqrt(oracle.cell_dist2(p.xyz[a], c, i))
            if (a, i) in inset:
                assert d < 2 * p.h[a]
                if d < 1.9 * p.h[a]:
                    assert f > 1e-12
            else:
                assert d >= 2 * p.h[a]
                assert abs(f) < 1e-14


def test_cell_distance_against_sampling():
    """Distance to a cell vs the nearest of many sampled points of its surface."""
    p, c = synth.workload("uniform", 50, 9)
    rng = np.random.default_rng(1)
    i = 17
    # sample the cell surface densely
    pts = []
    for j in range(c.cell_face_off[i], c.cell_face_off[i + 1]):
        ids = c.face_vert[c.face_vert_off[j]:c.face_vert_off[j + 1]]
        V = c.verts[ids]
        for k in range(1, len(V) - 1):
            u = rng.random((4000, 2))
            u = np.where(u.sum(1, keepdims=True) > 1, 1 - u, u)
            pts.append(V[0] + u[:, :1] * (V[k] - V[0]) + u[:, 1:] * (V[k + 1] - V[0]))
    pts = np.concatenate(pts)
    for q in rng.random((20, 3)) * 1.4 - 0.2:
        d_or = math.sqrt(oracle.cell_dist2(q, c, i))
        d_s = np.linalg.norm(pts - q, axis=1).min()
        inside = all(c.face_plane[j, 3] - c.face_plane[j, :3] @ q >= 0
                     for j in range(c.cell_face_off[i], c.cell_face_off[i + 1]))
        if inside:
            assert d_or == 0.0
        else:
            assert d_or <= d_s + 1e-12 and d_s - d_or < 0.02


@pytest.mark.parametrize("h,expected", [(1.0 / 3.0, 10146), (2.0 / 3.0, 9906)])
def test_flop_model_hand_count(h, expected):
    """The operation count of the direct form, on a cube of half-side 1/2 about the particle
    (6 walls, 24 edges, 48 right-triangle pyramids with r0 = R0 = L/h, phi = pi/4), equals the
    count done by hand from the per-statement costs listed in orc_flop_model's comment:
    L/h = 1.5: no breakpoint (c^2 = 4.5), one shell-piece G(r0) (6 terms): pyramid 3 + 153 + 18 + 4;
    L/h = 0.75: the s = 2 breakpoint computed but beyond phi, one piece, inner G(r0) (3 terms):
    pyramid 3 + 4 + 153 + 9 + 4; then 3 per triangle term, 57 + two terms per edge, 15 per wall."""
    c = box_cell([0.0, 0.0, 0.0], [1.0, 1.0, 1.0])
    xyz = np.array([[0.5, 0.5, 0.5]])
    fm = oracle.flop_model(xyz, np.array([h]), c, np.array([0]), np.array([0]))
    assert fm["faces"] == 6 and fm["edges"] == 24 and fm["pyramids"] == 48
    assert fm["flops"] == expected
