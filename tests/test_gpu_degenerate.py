"""Mixed-path parity on the geometry that the right-triangle split of Sec. II-B makes degenerate.

The particles sit exactly on a wall plane (r0 = 0), on an edge line (R0 = 0
for the walls it projects onto), on a vertex, at a wall distance of exactly
h and 2h (r0 at the piece radii 1 and 2 of the M4 kernel), and at a distance
of exactly h and 2h from an edge line (c = 1, 2), all on a lattice of cubes
whose coordinates are exact binary fractions.  Such edges go to the
conditioning test of the mixed path and are recomputed in FP64; a particle on
an edge or a vertex of its cell has its winding weight (the dihedral angle
over 2 pi, the corner's solid angle over 4 pi) recomputed in FP64 in both
paths.  Both paths
are compared with the oracle pair by pair; the mixed path must report FP64
fixups.  A fixup list of capacity 1 sends the mixed mapping down its overflow
branch (every pair recomputed in FP64): the result must then equal the FP64
path bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2404_17084_amd as em

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cube_lattice(n):
    """n^3 cubes of side 1/n filling the unit box (n a power of two: exact coordinates)."""
    g = np.arange(n + 1) / n
    vid = lambda i, j, k: (i * (n + 1) + j) * (n + 1) + k
    verts = np.array([[g[i], g[j], g[k]] for i in range(n + 1) for j in range(n + 1) for k in range(n + 1)])
    cfo, fvo, fv, planes, nb, vols = [0], [0], [], [], [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                faces = [  # vertex ids counter-clockwise seen from outside, outward normal, plane constant
                    ([vid(i, j, k), vid(i, j, k + 1), vid(i, j + 1, k + 1), vid(i, j + 1, k)], (-1, 0, 0), -g[i]),
                    ([vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i + 1, j + 1, k + 1), vid(i + 1, j, k + 1)], (1, 0, 0), g[i + 1]),
                    ([vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j, k + 1), vid(i, j, k + 1)], (0, -1, 0), -g[j]),
                    ([vid(i, j + 1, k), vid(i, j + 1, k + 1), vid(i + 1, j + 1, k + 1), vid(i + 1, j + 1, k)], (0, 1, 0), g[j + 1]),
                    ([vid(i, j, k), vid(i, j + 1, k), vid(i + 1, j + 1, k), vid(i + 1, j, k)], (0, 0, -1), -g[k]),
                    ([vid(i, j, k + 1), vid(i + 1, j, k + 1), vid(i + 1, j + 1, k + 1), vid(i, j + 1, k + 1)], (0, 0, 1), g[k + 1]),
                ]
                for ids, nrm, cst in faces:
                    fv.extend(ids)
                    fvo.append(len(fv))
                    planes.append([nrm[0], nrm[1], nrm[2], cst])
                    nb.append(0)
                cfo.append(len(planes))
                vols.append(1.0 / n ** 3)
    return synth.Cells(np.array(cfo, np.int64), np.array(fvo, np.int64), np.array(fv, np.int32),
                       np.array(planes, np.float64), np.array(nb, np.int64), verts, np.array(vols), synth.BOX)


def degenerate_particles():
    h = 0.0625
    pts = [
        ((0.5, 0.3, 0.35), 0.06),                 # on the wall plane x = 1/2 (r0 = 0)
        ((0.5, 0.5, 0.37), 0.07),                 # on the edge line x = y = 1/2
        ((0.5, 0.5, 0.5), 0.05),                  # on a vertex
        ((0.5 - h, 0.33, 0.41), h),               # wall at exactly h (r0 = 1)
        ((0.5 - 2 * h, 0.31, 0.43), h),           # wall at exactly 2h (r0 = 2)
        ((0.5 - 0.0375, 0.25 + 0.05, 0.62), h),   # edge line x = 1/2, y = 1/4 at h (c = 1)
        ((0.5 - 0.075, 0.25 + 0.1, 0.66), h),     # the same edge line at 2h (c = 2)
        ((0.25 + 1e-9, 0.71, 0.29), 0.08),        # 1e-9 from a wall
        ((0.75 - 1e-9, 0.75 + 1e-9, 0.21), 0.05), # 1e-9 from an edge line
        ((0.6, 0.45, 0.55), 0.09),                # a generic particle
        ((0.125, 0.125, 0.125), 0.1),             # at a cell centre
    ]
    xyz = np.array([p for p, _ in pts], np.float64)
    hh = np.array([q for _, q in pts], np.float64)
    m = np.full(len(pts), 1.0 / len(pts))
    return synth.Particles(xyz, m, hh)


@pytest.fixture(scope="module")
def case():
    c = cube_lattice(4)
    p = degenerate_particles()
    return p, c, oracle.map_particles(p, c)


@pytest.mark.parametrize("prec,pair_tol", [(em.MAP_FP64, 1e-12), (em.MAP_MIXED, 1e-6)])
def test_degenerate_pairs_against_oracle(case, prec, pair_tol):
    p, c, o = case
    say(f"case: degenerate geometry, precision {prec}")
    with em.Mapper(device=0, precision=prec) as mp:
        r = mp.map(p, c, want_pairs=True)
    assert np.array_equal(r["pair_p"], o["pair_p"]) and np.array_equal(r["pair_c"], o["pair_c"])
    df = np.abs(r["f"] - o["f"])
    dS = np.abs(r["S"] - o["S"])
    say(f"  pairs {o['f'].size}, max |df| {df.max():.3e}, max |dS| {dS.max():.3e}, "
        f"fixups {r['stats']['n_fixup_terms']}")
    assert df.max() < pair_tol
    assert dS.max() < pair_tol * 10
    nz = o["M"] > 1e-3 * o["M"].max()
    assert (np.abs(r["M"][nz] - o["M"][nz]) / o["M"][nz]).max() < (1e-10 if prec == em.MAP_FP64 else 1e-5)
    assert abs(r["M"].sum() - p.m.sum()) < 1e-12
    # the particles on an edge line and on a vertex: their winding weight is recomputed
    assert r["stats"]["n_boundary_pairs"] >= 4 + 8
    if prec == em.MAP_MIXED:
        assert r["stats"]["n_fixup_terms"] > 0


def test_each_degenerate_particle_flags_or_matches(case):
    """Per particle: the mixed fractions of each degenerate particle alone agree with the oracle."""
    p, c, _ = case
    with em.Mapper(device=0, precision=em.MAP_MIXED) as mp:
        for a in range(p.n):
            q = synth.Particles(p.xyz[a:a + 1].copy(), np.ones(1), p.h[a:a + 1].copy())
            o = oracle.map_particles(q, c)
            r = mp.map(q, c, want_pairs=True)
            assert np.array_equal(r["pair_c"], o["pair_c"]), a
            assert np.abs(r["f"] - o["f"]).max() < 1e-6, (a, np.abs(r["f"] - o["f"]).max())
            assert abs(r["S"][0] - o["S"][0]) < 1e-6, a


def test_fixup_overflow_branch(case):
    """More flagged edges than the fixup list holds: every pair of the call is recomputed in FP64."""
    p, c, o = case
    say("case: fixup list overflow")
    with em.Mapper(device=0, precision=em.MAP_FP64) as mp:
        ref = mp.map(p, c, want_pairs=True)
    with em.Mapper(device=0, precision=em.MAP_MIXED, fixup_cap=1) as mp:
        r = mp.map(p, c, want_pairs=True)
    assert r["stats"]["n_fixup_terms"] == r["stats"]["n_pairs"]
    assert np.array_equal(r["f"], ref["f"]) and np.array_equal(r["M"], ref["M"])
    assert np.abs(r["f"] - o["f"]).max() < 1e-12
