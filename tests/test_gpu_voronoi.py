"""GPU parity of the Voronoi grid (Sec. II-A) and its Lloyd iterations through the C ABI.

Against the brute-force oracle on the same sites: per cell the volume (1e-12
relative; both are sums of a few dozen tetrahedra over vertices computed in
FP64 from different plane triplets, measured ~2e-14), the centroid (1e-13),
and the set of neighbours across the faces (exact); every face is planar,
counter-clockwise about its outward unit normal, and shared faces have equal
areas; the cells feed the FP64 mapping to the same cell masses as the oracle's
cells (1e-10); five Lloyd iterations give the oracle's sites to 1e-12.  At
262,144 clumpy sites, 32 seeded cells and the largest cells and those with
the most faces are checked against the oracle's selected cells, and the whole
grid fills the box.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2404_17084_amd as em

pytestmark = pytest.mark.gpu

BOX = np.array(synth.BOX, dtype=np.float64)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _nb_sets(V, cells):
    cfo, nb = np.asarray(V["cell_face_off"] if isinstance(V, dict) else V.cell_face_off), \
        np.asarray(V["face_nb"] if isinstance(V, dict) else V.face_nb)
    return [sorted(nb[cfo[i]:cfo[i + 1]].tolist()) for i in cells]


def _check_faces(G):
    areas = {}
    cfo = G.cell_face_off
    for i in range(G.n_cells):
        for q in range(cfo[i], cfo[i + 1]):
            P = G.verts[G.face_vert[G.face_vert_off[q]:G.face_vert_off[q + 1]]]
            a = np.zeros(3)
            for k in range(len(P)):
                a += np.cross(P[k], P[(k + 1) % len(P)])
            n = G.face_plane[q, :3]
            assert abs(np.linalg.norm(n) - 1.0) < 1e-14 and np.dot(a, n) > 0
            assert np.abs(P @ n - G.face_plane[q, 3]).max() < 1e-13
            if G.face_nb[q] >= 0:
                areas[(i, int(G.face_nb[q]))] = 0.5 * np.linalg.norm(a)
    for (i, j), a in areas.items():
        assert areas[(j, i)] == pytest.approx(a, rel=1e-9, abs=1e-15)


@pytest.mark.parametrize("kind,n,seed", [("uniform", 300, 1), ("clumps", 700, 81), ("uniform", 2000, 3)])
def test_voronoi_matches_oracle(kind, n, seed):
    say(f"case: voronoi {kind} n={n} seed={seed}")
    s = synth.particles(kind, n, seed).xyz
    with em.Mapper(device=0) as mp:
        G = mp.voronoi(s, BOX)
    O = oracle.voronoi(s, BOX)
    rel = np.abs(G.cell_volume - O["cell_volume"]) / O["cell_volume"]
    say(f"  volume rel max {rel.max():.3e}, centroid max {np.abs(G.centroid - O['centroid']).max():.3e}")
    assert rel.max() < 1e-12
    assert np.abs(G.centroid - O["centroid"]).max() < 1e-13
    assert G.cell_volume.sum() == pytest.approx(1.0, rel=1e-12)
    assert _nb_sets(G, range(n)) == _nb_sets(O, range(n))
    assert np.array_equal(G.sites, s)
    _check_faces(G)


def test_voronoi_cells_feed_the_mapping():
    say("case: voronoi cells in the mapping")
    p = synth.particles("clumps", 1500, 85)
    O = oracle.voronoi(p.xyz, BOX)
    oc = synth.Cells(O["cell_face_off"], O["face_vert_off"], O["face_vert"], O["face_plane"], O["face_nb"],
                     O["verts"], O["cell_volume"], tuple(BOX))
    ref = oracle.map_particles(p, oc)
    with em.Mapper(device=0) as mp:
        G = mp.voronoi(p.xyz, BOX)
        r = mp.map(p, G)
        D = mp.voronoi(p.xyz, BOX, device=True)
        import torch
        dev = torch.device("cuda:0")
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        M = torch.zeros(G.n_cells, dtype=torch.float64, device=dev)
        em.map_particles(mp.ctx, t(p.xyz), t(p.m), t(p.h), D, M)
        Md = M.cpu().numpy()
    rel = (np.abs(r["M"] - ref["M"]) / ref["M"]).max()
    say(f"  cell mass rel max {rel:.3e}")
    assert rel < 1e-10
    assert np.array_equal(Md, r["M"])


def test_lloyd_matches_oracle():
    say("case: voronoi with 5 Lloyd iterations")
    s = synth.particles("clumps", 500, 87).xyz
    with em.Mapper(device=0) as mp:
        G = mp.voronoi(s, BOX, lloyd_iters=5)
    O = oracle.lloyd(s, BOX, 5)
    say(f"  sites max diff {np.abs(G.sites - O['sites']).max():.3e}")
    assert np.abs(G.sites - O["sites"]).max() < 1e-12
    assert (np.abs(G.cell_volume - O["cell_volume"]) / O["cell_volume"]).max() < 1e-11
    assert _nb_sets(G, range(500)) == _nb_sets(O, range(500))


def test_voronoi_full_size_sampled():
    say("case: voronoi clumps 262144, sampled cells")
    p = synth.particles(*synth.CLUMPS_256K)
    with em.Mapper(device=0) as mp:
        G = mp.voronoi(p.xyz, BOX)
    say(f"  built in {G.ms:.2f} ms, {G.face_plane.shape[0] / G.n_cells:.2f} faces per cell")
    assert G.cell_volume.sum() == pytest.approx(1.0, rel=1e-11)
    # 32 seeded cells, and the 16 largest cells and the 16 with the most faces: large cells next to
    # the clumps have the longest candidate walks (the ones that can leave the wavefront walk's node
    # stack for the serial walk)
    nf = np.diff(G.cell_face_off)
    sel = np.unique(np.concatenate([np.random.default_rng(17).choice(p.n, 32, replace=False),
                                    np.argsort(G.cell_volume)[-16:], np.argsort(nf, kind="stable")[-16:]]))
    O = oracle.voronoi(p.xyz, BOX, sel=sel)
    rel = np.abs(G.cell_volume[sel] - O["cell_volume"]) / O["cell_volume"]
    assert rel.max() < 1e-12
    assert _nb_sets(G, sel) == _nb_sets(O, range(len(sel)))
    # shared faces are mutual across the whole grid
    i = np.repeat(np.arange(p.n), np.diff(G.cell_face_off))
    j = G.face_nb
    inner = j >= 0
    fwd = set(zip(i[inner].tolist(), j[inner].tolist()))
    assert all((b, a) in fwd for a, b in fwd)


def test_voronoi_rejects_bad_sites():
    say("case: voronoi errors")
    s = synth.particles("uniform", 200, 5).xyz
    with em.Mapper(device=0) as mp:
        for bad in (np.vstack([s, s[:1]]), np.vstack([s, [[1.5, 0.5, 0.5]]]), np.vstack([s, [[np.nan, 0.5, 0.5]]])):
            with pytest.raises(em.MapError) as ei:
                mp.voronoi(bad, BOX)
            assert ei.value.code == em.MAP_EINVAL
        with pytest.raises(em.MapError):
            mp.voronoi(s, BOX, lloyd_iters=-1)
        G = mp.voronoi(s, BOX)  # the context still works
        assert G.cell_volume.sum() == pytest.approx(1.0, rel=1e-12)


def test_voronoi_edge_cases():
    say("case: voronoi one site, two sites, sites on the walls, a lattice")
    g = (np.arange(4) + 0.5) / 4
    cases = {
        "one": np.array([[0.3, 0.6, 0.2]]),
        "two": np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]]),
        "walls": np.vstack([np.random.default_rng(4).random((200, 3)),
                            [[0.0, 0.5, 0.5], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0], [0.5, 0.0, 0.3]]]),
        "lattice": np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T,
    }
    with em.Mapper(device=0) as mp:
        for name, s in cases.items():
            G = mp.voronoi(s, BOX)
            O = oracle.voronoi(s, BOX)
            assert np.allclose(G.cell_volume, O["cell_volume"], rtol=1e-12, atol=0), name
            assert _nb_sets(G, range(len(s))) == _nb_sets(O, range(len(s))), name
            _check_faces(G)
        G = mp.voronoi(cases["one"], BOX)
        assert G.face_plane.shape[0] == 6 and G.cell_volume[0] == pytest.approx(1.0, rel=1e-15)
        G = mp.voronoi(cases["lattice"], BOX)
        assert np.all(np.diff(G.cell_face_off) == 6) and np.allclose(G.cell_volume, 1 / 64, rtol=1e-13)
        assert np.allclose(G.centroid, cases["lattice"], atol=1e-15)


def test_site_cell_ties():
    """An input point equidistant from two grid sites belongs to the lower index: the walk over the
    cells lists it for the tree walk, which breaks the tie."""
    say("case: voronoi site cells with a tie")
    s = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5], [0.5, 0.5, 0.5], [0.5, 0.25, 0.25]])
    kept = oracle.merge_sites(s, 0.3)
    assert kept.tolist() == [0, 1, 3]  # the midpoint is merged away
    with em.Mapper(device=0) as mp:
        G = mp.voronoi(s, BOX, merge_dist=0.3)
    assert np.array_equal(G.site_cell, oracle.site_cells(s, s[kept]))
    assert G.site_cell[2] == 0


def test_merging_and_site_cells():
    say("case: voronoi with tightly packed sites merged, then Lloyd steps")
    s = synth.particles("clumps", 2000, 91).xyz
    s = np.vstack([s, s[:5]])  # coinciding copies are merged too
    kept = oracle.merge_sites(s, 0.004)
    assert 0 < kept.size < s.shape[0] - 5
    with em.Mapper(device=0) as mp:
        G = mp.voronoi(s, BOX, merge_dist=0.004)
        assert G.n_cells == kept.size and np.array_equal(G.sites, s[kept])
        O = oracle.voronoi(s[kept], BOX)
        assert np.allclose(G.cell_volume, O["cell_volume"], rtol=1e-12, atol=0)
        assert _nb_sets(G, range(kept.size)) == _nb_sets(O, range(kept.size))
        assert np.array_equal(G.site_cell, oracle.site_cells(s, s[kept]))
        # after Lloyd steps the input sites are assigned to the cells of the moved sites
        L = mp.voronoi(s, BOX, lloyd_iters=2, merge_dist=0.004)
        OL = oracle.lloyd(s[kept], BOX, 2)
        assert np.abs(L.sites - OL["sites"]).max() < 1e-12
        assert np.array_equal(L.site_cell, oracle.site_cells(s, OL["sites"]))
        # no merging: every site keeps its own cell
        N = mp.voronoi(s[:2000], BOX)
        assert np.array_equal(N.site_cell, np.arange(2000))
        with pytest.raises(em.MapError):
            mp.voronoi(s, BOX, merge_dist=-1.0)
