"""Pins of the oracle's box-clipped Voronoi grid and Lloyd iterations (paper Sec. II-A).

Checked against what the definition and geometry fix, not against the
oracle's clipping code: volumes add up to the box; a cubic lattice gives its
cubes exactly; every vertex is no farther from its own site than from any
other site and lies on the bisector of the face it belongs to (or on the box
wall); neighbour relations are symmetric with equal shared-face areas; faces
are planar, counter-clockwise about their outward normals and convex; interior
cells match Qhull's Voronoi vertices (scipy); centroids of lattice cubes are
their centres; and each Lloyd step lowers the quantisation energy
sum_i int_{V_i} |x - s_i|^2 dx, estimated independently by nearest-site
assignment of random points.
"""
import numpy as np
import pytest
from scipy.spatial import Voronoi, cKDTree

import oracle
import synth

BOX = np.array(synth.BOX, dtype=np.float64)


@pytest.fixture(scope="module")
def clumpy():
    p = synth.particles("clumps", 700, 81)
    return p.xyz, oracle.voronoi(p.xyz, BOX)


def _faces(V, i):
    for q in range(V["cell_face_off"][i], V["cell_face_off"][i + 1]):
        yield q, V["verts"][V["face_vert_off"][q]:V["face_vert_off"][q + 1]]


def _area_normal(P):
    """Newell's vector area of a polygon (twice the area times the unit normal, halved)."""
    s = np.zeros(3)
    for a in range(len(P)):
        s += np.cross(P[a], P[(a + 1) % len(P)])
    return 0.5 * s


def test_volumes_fill_the_box(clumpy):
    sites, V = clumpy
    assert V["cell_volume"].sum() == pytest.approx(1.0, rel=1e-12)
    assert np.all(V["cell_volume"] > 0)
    u = np.random.default_rng(2).random((300, 3))
    assert oracle.voronoi(u, BOX)["cell_volume"].sum() == pytest.approx(1.0, rel=1e-12)


def test_cubic_lattice_gives_cubes():
    k = 4
    g = (np.arange(k) + 0.5) / k
    sites = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T
    V = oracle.voronoi(sites, BOX)
    assert np.allclose(V["cell_volume"], 1.0 / k ** 3, rtol=1e-12)
    assert np.all(np.diff(V["cell_face_off"]) == 6)
    assert np.all(np.diff(V["face_vert_off"]) == 4)
    assert np.allclose(V["centroid"], sites, atol=1e-14)


def test_vertices_obey_the_definition(clumpy):
    sites, V = clumpy
    tree = cKDTree(sites)
    for i in range(0, len(sites), 7):
        for q, P in _faces(V, i):
            d_own = np.linalg.norm(P - sites[i], axis=1)
            d_near, _ = tree.query(P, k=1)
            assert np.all(d_own <= d_near + 1e-12)  # no site is closer than the cell's own
            nb = V["face_nb"][q]
            if nb >= 0:
                assert np.allclose(np.linalg.norm(P - sites[nb], axis=1), d_own, atol=1e-12)
            else:
                w = -1 - nb
                assert np.allclose(P[:, w // 2], BOX[3 * (w % 2) + w // 2], atol=1e-15)


def test_neighbours_symmetric_and_faces_oriented(clumpy):
    sites, V = clumpy
    area = {}
    for i in range(len(sites)):
        for q, P in _faces(V, i):
            an = _area_normal(P)
            n = V["face_plane"][q, :3]
            assert abs(np.linalg.norm(n) - 1.0) < 1e-14
            assert np.dot(an, n) > 0  # counter-clockwise about the outward normal
            assert np.allclose(P @ n, V["face_plane"][q, 3], atol=1e-13)  # planar, on its plane
            c = P.mean(axis=0)
            for a in range(len(P)):  # convex: every turn is to the left about n
                e1, e2 = P[(a + 1) % len(P)] - P[a], P[(a + 2) % len(P)] - P[(a + 1) % len(P)]
                assert np.dot(np.cross(e1, e2), n) > -1e-14
            assert np.dot(n, c - sites[i]) > 0  # the site is on the inner side
            if V["face_nb"][q] >= 0:
                area[(i, int(V["face_nb"][q]))] = np.linalg.norm(an)
    for (i, j), a in area.items():
        assert (j, i) in area
        assert area[(j, i)] == pytest.approx(a, rel=1e-9, abs=1e-14)


def test_interior_cells_match_qhull(clumpy):
    sites, V = clumpy
    vor = Voronoi(sites)
    checked = 0
    for i in range(len(sites)):
        reg = vor.regions[vor.point_region[i]]
        if not reg or -1 in reg:
            continue
        qv = vor.vertices[reg]
        if np.any(qv < 0.02) or np.any(qv > 0.98):
            continue  # touches or nears the box
        ours = np.concatenate([P for _, P in _faces(V, i)])
        if np.any(V["face_nb"][V["cell_face_off"][i]:V["cell_face_off"][i + 1]] < 0):
            continue
        # every Qhull vertex is one of ours and vice versa (ours repeat per face)
        d1, _ = cKDTree(ours).query(qv)
        d2, _ = cKDTree(qv).query(ours)
        assert d1.max() < 1e-9 and d2.max() < 1e-9
        checked += 1
    assert checked > 50


def _energy(sites, rng):
    x = rng.random((400000, 3))
    d, _ = cKDTree(sites).query(x)
    return float(np.mean(d * d))


def test_lloyd_lowers_the_energy():
    rng = np.random.default_rng(5)
    s = synth.particles("clumps", 300, 83).xyz
    e = [_energy(s, np.random.default_rng(9))]
    for _ in range(5):
        s = oracle.voronoi(s, BOX)["centroid"]
        e.append(_energy(s, np.random.default_rng(9)))
    assert all(b < a for a, b in zip(e, e[1:])), e
    V = oracle.lloyd(synth.particles("clumps", 300, 83).xyz, BOX, 5)
    assert np.allclose(V["sites"], s, atol=1e-15)
    assert V["cell_volume"].sum() == pytest.approx(1.0, rel=1e-12)


def test_selected_cells_with_the_stopping_rule_equal_the_full_build(clumpy):
    """Sampled cells stop at the first site twice as far as the farthest vertex; they must equal the cells
    that every site clipped."""
    sites, V = clumpy
    sel = np.arange(0, len(sites), 3)
    S = oracle.voronoi(sites, BOX, sel=sel)
    assert np.allclose(S["cell_volume"], V["cell_volume"][sel], rtol=1e-13, atol=0)
    assert np.allclose(S["centroid"], V["centroid"][sel], atol=1e-14)
    for t, i in enumerate(sel):
        a = sorted(S["face_nb"][S["cell_face_off"][t]:S["cell_face_off"][t + 1]].tolist())
        b = sorted(V["face_nb"][V["cell_face_off"][i]:V["cell_face_off"][i + 1]].tolist())
        assert a == b


def test_merging_a_chain_of_close_sites():
    """a, b = a + 0.01 x, c = b + 0.01 x with d = 0.015: b is dropped (a is close), so is c (b, although
    dropped, is close and of lower index); a far site stays."""
    s = np.array([[0.5, 0.5, 0.5], [0.51, 0.5, 0.5], [0.52, 0.5, 0.5], [0.1, 0.2, 0.3]])
    assert oracle.merge_sites(s, 0.015).tolist() == [0, 3]
    assert oracle.merge_sites(s, 0.0).tolist() == [0, 1, 2, 3]
    assert oracle.merge_sites(s, 0.02).tolist() == [0, 3]
    assert oracle.merge_sites(np.vstack([s, s[1:2]]), 1e-9).tolist() == [0, 1, 2, 3]  # the copy of b goes


def test_site_cells_hold_their_points():
    sites = synth.particles("clumps", 600, 89).xyz
    kept = oracle.merge_sites(sites, 0.01)
    assert 0 < kept.size < sites.shape[0]
    V = oracle.voronoi(sites[kept], BOX)
    cell = oracle.site_cells(sites, sites[kept])
    assert np.array_equal(cell[kept], np.arange(kept.size))
    for a in range(sites.shape[0]):  # the point lies inside its cell: on the inner side of every face
        f0, f1 = V["cell_face_off"][cell[a]], V["cell_face_off"][cell[a] + 1]
        n, c = V["face_plane"][f0:f1, :3], V["face_plane"][f0:f1, 3]
        assert np.all(n @ sites[a] <= c + 1e-12)
