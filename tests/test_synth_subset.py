"""Host helpers of the sampled checks of large jobs: the cell subset used to
run the oracle's pair search over a sample of the cells."""
import numpy as np

import oracle
import synth


def test_cells_subset_pairs_and_fractions():
    p, c = synth.workload("clumps", 3000, 9)
    sel = np.sort(np.random.default_rng(1).choice(c.n_cells, 200, replace=False))
    sub = synth.cells_subset(c, sel)
    assert sub.n_cells == sel.size
    assert np.array_equal(sub.cell_volume, c.cell_volume[sel])
    # the oracle's grid pair search over the subset finds exactly the brute-force pairs of those cells
    pp, pc = oracle.pairs(p.xyz, p.h, sub)
    qp, qc = oracle.pairs_for_cells(p.xyz, p.h, c, sel)
    a = np.stack([sel[pc], pp], 1)
    b = np.stack([qc, qp], 1)
    a = a[np.lexsort((a[:, 1], a[:, 0]))]
    b = b[np.lexsort((b[:, 1], b[:, 0]))]
    assert np.array_equal(a, b)
    # and the same fractions as over the whole grid
    f1 = oracle.pair_fractions(p.xyz, p.h, sub, pp, pc)
    f2 = oracle.pair_fractions(p.xyz, p.h, c, pp, sel[pc])
    assert np.array_equal(f1, f2)


def test_cells_subset_empty_and_all():
    p, c = synth.workload("uniform", 300, 2)
    e = synth.cells_subset(c, np.zeros(0, np.int64))
    assert e.n_cells == 0 and e.face_plane.shape[0] == 0
    a = synth.cells_subset(c, np.arange(c.n_cells))
    for k in ("cell_face_off", "face_vert_off", "face_vert", "face_plane", "cell_volume"):
        assert np.array_equal(getattr(a, k), getattr(c, k)), k
    h = synth.cells_from(c)
    assert np.array_equal(h.face_vert, c.face_vert) and h.box == tuple(c.box)
