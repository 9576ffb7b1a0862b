"""Pins of the oracle's tabulated variant (Sec. II-B: the pyramid integral pre-computed and interpolated).

The table holds the closed-form pyramid integral I(r0, R0, phi) on a uniform
grid over [0, 2] x [0, 2] x [0, pi/2]; between nodes it is trilinear, outside
the grid it follows from the triangle's solid angle.  Checked independently of
the table code: node values equal the closed form; the interpolant is linear
along each axis between nodes (a transposed index would break both); the
interpolation error against the closed form falls at second order when the
grid is refined; the identities outside the grid hold against the closed form
(r0 >= 2 gives exactly the cone's mass Omega / 4 pi, with Omega checked against
the Van Oosterom-Strackee formula; for R0 > 2 the error equals the error at
R0 = 2); and at the cell level the tabulated mapping converges to the closed
form as the grid is refined, within a bound set by the pointwise error.
"""
import math

import numpy as np
import pytest

import oracle
import synth

N = 32


@pytest.fixture
def tab():
    # the oracle reads one table at a time: select this one for every test that uses it
    return oracle.use_table(N, N + 4, N + 8)


def _node(i, j, k, n0, n1, n2):
    phi = math.pi / 2 - 1e-12 if k == n2 - 1 else 0.5 * math.pi * k / (n2 - 1)
    return 2.0 * i / (n0 - 1), 2.0 * j / (n1 - 1), phi


def test_nodes_equal_the_closed_form(tab):
    n0, n1, n2 = tab.shape
    rng = np.random.default_rng(0)
    for _ in range(200):
        i, j, k = rng.integers(0, n0), rng.integers(0, n1), rng.integers(0, n2)
        r0, R0, phi = _node(i, j, k, n0, n1, n2)
        assert tab[i, j, k] == oracle.pyramid(r0, R0, phi)
        if r0 > 0 and R0 > 0 and phi > 0 and r0 < 2.0:
            assert oracle.table_interp(r0, R0, phi) == pytest.approx(tab[i, j, k], rel=1e-11, abs=1e-15)


def test_linear_between_nodes_along_each_axis(tab):
    n0, n1, n2 = tab.shape
    rng = np.random.default_rng(1)
    for _ in range(100):
        i, j, k = rng.integers(1, n0 - 2), rng.integers(1, n1 - 2), rng.integers(1, n2 - 2)
        r0, R0, phi = _node(i, j, k, n0, n1, n2)
        t = rng.uniform(0.1, 0.9)
        dr, dR, dp = 2.0 / (n0 - 1), 2.0 / (n1 - 1), 0.5 * math.pi / (n2 - 1)
        assert oracle.table_interp(r0 + t * dr, R0, phi) == pytest.approx(
            (1 - t) * tab[i, j, k] + t * tab[i + 1, j, k], rel=1e-12, abs=1e-16)
        assert oracle.table_interp(r0, R0 + t * dR, phi) == pytest.approx(
            (1 - t) * tab[i, j, k] + t * tab[i, j + 1, k], rel=1e-12, abs=1e-16)
        assert oracle.table_interp(r0, R0, phi + t * dp) == pytest.approx(
            (1 - t) * tab[i, j, k] + t * tab[i, j, k + 1], rel=1e-12, abs=1e-16)


def test_second_order_convergence():
    rng = np.random.default_rng(2)
    pts = np.column_stack([rng.uniform(0, 2, 3000), rng.uniform(0, 2, 3000), rng.uniform(0, 0.5 * math.pi, 3000)])
    exact = np.array([oracle.pyramid(*q) for q in pts])
    err = []
    for n in (16, 32, 64):
        oracle.use_table(n, n, n)
        err.append(np.mean(np.abs(np.array([oracle.table_interp(*q) for q in pts]) - exact)))
    assert err[1] < err[0] / 3.0 and err[2] < err[1] / 3.0, err


def _vos_triangle(r0, R0, phi):
    """Solid angle of the triangle (foot, foot + R0 e1, foot + R0 e1 + R0 tan(phi) e2) seen from height r0
    (Van Oosterom and Strackee)."""
    a = np.array([0.0, 0.0, -r0])
    b = np.array([R0, 0.0, -r0])
    c = np.array([R0, R0 * math.tan(phi), -r0])
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = abs(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * math.atan2(num, den)


def test_outside_the_grid(tab):
    rng = np.random.default_rng(3)
    for _ in range(200):
        r0, R0, phi = rng.uniform(2.0, 4.0), rng.uniform(0.01, 4.0), rng.uniform(0.01, 1.5)
        om = _vos_triangle(r0, R0, phi)
        assert oracle.solid_angle(r0, R0, phi) == pytest.approx(om, rel=1e-12)
        # beyond the support the pyramid holds the whole cone
        assert oracle.table_interp(r0, R0, phi) == pytest.approx(oracle.pyramid(r0, R0, phi), rel=1e-12)
        assert oracle.pyramid(r0, R0, phi) == pytest.approx(om / (4.0 * math.pi), rel=1e-12)
    for _ in range(200):
        r0, R0, phi = rng.uniform(0.01, 1.99), rng.uniform(2.0, 5.0), rng.uniform(0.01, 1.55)
        e_far = oracle.table_interp(r0, R0, phi) - oracle.pyramid(r0, R0, phi)
        e_edge = oracle.table_interp(r0, 2.0, phi) - oracle.pyramid(r0, 2.0, phi)
        assert e_far == pytest.approx(e_edge, abs=1e-14)


def test_cell_level_converges_to_the_closed_form():
    p, c = synth.workload("uniform", 800, 19)
    ref = oracle.map_particles(p, c)
    interior = np.all((p.xyz > 2 * p.h[:, None]) & (p.xyz < 1 - 2 * p.h[:, None]), axis=1)
    dev = []
    for n in (16, 32, 64):
        oracle.use_table(n, n, n)
        o = oracle.map_particles(p, c, profile=oracle.TABLE)
        assert np.array_equal(o["pair_p"], ref["pair_p"]) and np.array_equal(o["pair_c"], ref["pair_c"])
        # mass is conserved by the normalisation whatever the table
        assert o["M"].sum() == pytest.approx(p.m.sum(), rel=1e-12)
        dev.append((np.abs(o["S"][interior] - 1.0).max(), np.abs(o["f"] - ref["f"]).max()))
    assert dev[1][0] < dev[0][0] / 2 and dev[2][0] < dev[1][0] / 2, dev
    assert dev[1][1] < dev[0][1] / 2 and dev[2][1] < dev[1][1] / 2, dev
    assert dev[2][0] < 2e-3
