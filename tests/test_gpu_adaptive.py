"""GPU parity of the adaptive tree walk (Sec. III-B, Eq. (6)) through the C ABI.

Both sides are driven by the same neutral-fraction field (synth's ionised
spheres, the stand-in for the radiative transfer).  The library's walk count,
convergence, failure count and final set must equal the oracle's: kinds, node
labels and particle indices exactly, positions, masses, sizes and smoothing
lengths within the bars of the plain pseudo-particle parity (4 k u, 64 k u for
h, for a node of k particles; u = 2^-53).  The grown radii come from r - s of
the failing leaves, computed from those positions, so they agree to 1e-12
relative; so do the remembered regions (centre of mass, size, smallest
descendant size), whose count must match exactly.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2404_17084_amd as em
from tests.test_gpu_pseudo import _compare

pytestmark = pytest.mark.gpu

BOX = np.array(synth.BOX, dtype=np.float64)
K = 100.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sphere(src, radius=0.15, width=0.05):
    return lambda P: synth.ionised_spheres(P["xyz"], src, radius, width)


def _regions_close(G, O):
    assert G.shape == O.shape, (G.shape, O.shape)
    if G.size:
        assert np.allclose(G, O, rtol=1e-12, atol=1e-15)


def _check_pair(G, O, n):
    a = G["adapt"]
    assert a["n_walks"] == O["walks"] and bool(a["converged"]) == O["converged"]
    assert a["n_failed"] == sum(len(f) for f in O["failed"])
    assert a["r_part"] == pytest.approx(O["r_part"], rel=1e-12)
    assert a["r_leaf"] == pytest.approx(O["r_leaf"], rel=1e-12)
    _compare(G, O, n)


CASES = [
    ("clumps", 12000, 71, [[0.5, 0.5, 0.5]], 0.15),
    ("uniform", 20000, 5, [[0.5, 0.5, 0.5]], 0.15),
    ("lognormal", 40000, 7, [[0.3, 0.4, 0.5], [0.7, 0.6, 0.5]], 0.1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adaptive_matches_oracle_two_steps(case):
    kind, n, seed, src, radius = case
    say(f"case: adaptive walk {kind} n={n} seed={seed} sources={len(src)}")
    p = synth.particles(kind, n, seed)
    field = sphere(src, radius)
    with em.Mapper(device=0) as mp:
        G1 = mp.pseudo_adaptive(p, BOX, src, field, K=K)
        O1 = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, src, field, K=K)
        _check_pair(G1, O1, n)
        assert O1["walks"] >= 2
        _regions_close(mp.regions, O1["regions"])
        # next step: particles moved a little, regions and radii carried over
        rng = np.random.default_rng(seed)
        xyz2 = np.clip(p.xyz + rng.normal(0.0, 1e-4, p.xyz.shape), 0.0, 1.0 - 1e-12)
        p2 = synth.Particles(xyz2, p.m, p.h)
        say(f"  step 2 of {kind}")
        kw = dict(K=K, r_part=G1["adapt"]["r_part"], r_leaf=G1["adapt"]["r_leaf"])
        G2 = mp.pseudo_adaptive(p2, BOX, src, field, **kw)
        O2 = oracle.pseudo_adaptive(xyz2, p.m, p.h, BOX, src, field, regions=O1["regions"], **kw)
        _check_pair(G2, O2, n)
        assert G2["adapt"]["n_regions_in"] == O1["regions"].shape[0]
        assert G2["adapt"]["n_regions_dropped"] == O2["dropped"]
        _regions_close(mp.regions, O2["regions"])
        # shielded: a neutral field drops every region
        say(f"  shielded step of {kind}")
        neutral = lambda P: np.ones(P["m"].size)
        G3 = mp.pseudo_adaptive(p2, BOX, src, neutral, **kw)
        O3 = oracle.pseudo_adaptive(xyz2, p.m, p.h, BOX, src, neutral, regions=O2["regions"], **kw)
        _check_pair(G3, O3, n)
        assert G3["adapt"]["n_regions_out"] == 0 and mp.regions.shape == (0, 5)


def test_failing_leaf_grows_r_part():
    say("case: adaptive walk, a far leaf ionised")
    p = synth.particles("clumps", 12000, 71)
    src = [[0.5, 0.5, 0.5]]
    Q = oracle.pseudo(p.xyz, p.m, p.h, BOX, src)
    leaves = np.nonzero(Q["leaf"] & (Q["s"] > 2.0 * Q["stats"]["s_root"] / K))[0]
    t = leaves[np.argmax(np.sqrt(((Q["xyz"][leaves] - src[0]) ** 2).sum(axis=1)) - Q["s"][leaves])]
    field = sphere([Q["xyz"][t]], radius=1e-3, width=1e-3)
    with em.Mapper(device=0) as mp:
        G = mp.pseudo_adaptive(p, BOX, src, field, K=K)
    O = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, src, field, K=K)
    _check_pair(G, O, p.n)
    assert G["adapt"]["n_r_part_growths"] >= 1


def test_walk_limit_and_neutral_field():
    say("case: adaptive walk, one walk allowed; neutral field")
    p = synth.particles("uniform", 8000, 9)
    src = [[0.5, 0.5, 0.5]]
    with em.Mapper(device=0) as mp:
        G = mp.pseudo_adaptive(p, BOX, src, sphere(src), K=K, max_walks=1)
        O = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, src, sphere(src), K=K, max_walks=1)
        _check_pair(G, O, p.n)
        assert not G["adapt"]["converged"] and G["adapt"]["n_walks"] == 1
        _regions_close(mp.regions, O["regions"])
        mp.regions = np.zeros((0, 5))
        G = mp.pseudo_adaptive(p, BOX, src, lambda P: np.ones(P["m"].size), K=K)
        Q = mp.pseudo(p, BOX, src)
        assert G["adapt"]["n_walks"] == 1 and G["adapt"]["converged"]
        for k in ("kind", "ref", "xyz", "m", "h", "size"):
            assert np.array_equal(G[k], Q[k])


def test_regions_interface_and_errors():
    say("case: adaptive walk, regions and errors")
    p = synth.particles("uniform", 3000, 10)
    src = [[0.5, 0.5, 0.5]]
    with em.Mapper(device=0) as mp:
        rows = np.array([[0.5, 0.5, 0.5, 0.1, 0.01], [0.2, 0.3, 0.4, 0.05, 0.0]])
        mp.regions = rows
        assert np.array_equal(mp.regions, rows)
        for bad in ([[0.5, 0.5, 0.5, 0.0, 0.01]], [[0.5, np.nan, 0.5, 0.1, 0.01]], [[0.5, 0.5, 0.5, 0.1, -1.0]]):
            with pytest.raises(em.MapError) as ei:
                mp.regions = bad
            assert ei.value.code == em.MAP_EINVAL
        assert np.array_equal(mp.regions, rows)
        # the walk with set regions equals the oracle's with the same regions
        G = mp.pseudo_adaptive(p, BOX, src, sphere(src), K=K)
        O = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, src, sphere(src), K=K, regions=rows)
        _check_pair(G, O, p.n)
        _regions_close(mp.regions, O["regions"])
        before = mp.regions
        # a failing callback stops the call and leaves the regions alone
        def broken(P):
            raise ValueError("no radiative transfer today")
        with pytest.raises(ValueError):
            mp.pseudo_adaptive(p, BOX, src, broken, K=K)
        assert np.array_equal(mp.regions, before)
        with pytest.raises(em.MapError) as ei:
            mp.pseudo_adaptive(p, BOX, src, lambda P: np.full(P["m"].size, np.nan), K=K)
        assert ei.value.code == em.MAP_EINVAL
        for kw in (dict(K=0.0), dict(K=np.inf), dict(max_walks=0)):
            with pytest.raises(em.MapError) as ei:
                mp.pseudo_adaptive(p, BOX, src, sphere(src), **{**dict(K=K), **kw})
            assert ei.value.code == em.MAP_EINVAL
        # no particles: nothing lies in any region, so all are dropped
        e = synth.Particles(np.zeros((0, 3)), np.zeros(0), np.zeros(0))
        G = mp.pseudo_adaptive(e, BOX, src, sphere(src), K=K)
        assert G["m"].size == 0 and mp.regions.shape == (0, 5)
