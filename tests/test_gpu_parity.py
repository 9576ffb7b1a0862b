"""Parity of the HIP library with the FP64 oracle, called through the C ABI.

Bars (per the target of the mapping): pair sets identical; all-FP64 path within
1e-10 relative per cell (and 1e-12 absolute per pair fraction); mixed path
within 1e-5 relative per cell; mass conserved to 1e-9 in both.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2404_17084_amd as em

pytestmark = pytest.mark.gpu

FP64_CELL_REL = 1e-10
FP64_PAIR_ABS = 1e-12
MIXED_CELL_REL = 1e-5
MASS_ABS = 1e-9


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mapper():
    m = em.Mapper(device=0)
    yield m
    m.close()


@pytest.fixture(scope="module")
def clumps256k():
    return synth.workload(*synth.CLUMPS_256K)


def _run(mapper, p, c, precision, want_pairs=True):
    mapper.set_precision(precision)
    return mapper.map(p, c, want_pairs=want_pairs)


# ------------------------------------------------------------------ uniform 4096 (full oracle)
def test_pairs_identical_uniform4k(mapper, uniform4k, uniform4k_oracle):
    say("case: pairs uniform 4096")
    p, c = uniform4k
    pp, pc = mapper.pairs(p, c)
    assert np.array_equal(pp, uniform4k_oracle["pair_p"])
    assert np.array_equal(pc, uniform4k_oracle["pair_c"])


def test_fp64_parity_uniform4k(mapper, uniform4k, uniform4k_oracle):
    say("case: FP64 uniform 4096")
    p, c = uniform4k
    r = _run(mapper, p, c, em.MAP_FP64)
    o = uniform4k_oracle
    assert np.array_equal(r["pair_p"], o["pair_p"]) and np.array_equal(r["pair_c"], o["pair_c"])
    assert np.abs(r["f"] - o["f"]).max() < FP64_PAIR_ABS
    assert np.abs(r["S"] - o["S"]).max() < 1e-12
    rel = np.abs(r["M"] - o["M"]) / o["M"]
    assert rel.max() < FP64_CELL_REL, rel.max()
    assert np.abs(r["rho"] - o["rho"]).max() / o["rho"].max() < FP64_CELL_REL
    st = r["stats"]
    assert st["n_pairs"] == o["f"].size
    assert abs(st["mass_out"] - p.m.sum()) < MASS_ABS
    assert abs(r["M"].sum() - p.m.sum()) < 1e-12


def test_mixed_parity_uniform4k(mapper, uniform4k, uniform4k_oracle):
    say("case: mixed uniform 4096")
    p, c = uniform4k
    r = _run(mapper, p, c, em.MAP_MIXED)
    o = uniform4k_oracle
    rel = np.abs(r["M"] - o["M"]) / o["M"]
    say(f"mixed uniform4k: max cell rel err {rel.max():.3e}, max pair abs err {np.abs(r['f'] - o['f']).max():.3e}, "
        f"fixups {r['stats']['n_fixup_terms']}")
    assert rel.max() < MIXED_CELL_REL
    assert abs(r["M"].sum() - p.m.sum()) < MASS_ABS


def test_deterministic_bits(mapper, uniform4k):
    say("case: determinism")
    p, c = uniform4k
    for prec in (em.MAP_FP64, em.MAP_MIXED):
        a = _run(mapper, p, c, prec)
        b = _run(mapper, p, c, prec)
        assert np.array_equal(a["M"], b["M"]) and np.array_equal(a["f"], b["f"]) and np.array_equal(a["S"], b["S"])


def test_fp64_task_batches_uniform4k(mapper, uniform4k, uniform4k_oracle):
    """Distribution 3 in FP64: oracle parity at the FP64 bars, determinism."""
    say("case: FP64 task batches uniform 4096")
    p, c = uniform4k
    em.map_set_tune(mapper.ctx, em.MAP_FP64, persistent=3)
    try:
        a = _run(mapper, p, c, em.MAP_FP64)
        b = _run(mapper, p, c, em.MAP_FP64)
    finally:
        em.map_set_tune(mapper.ctx, em.MAP_FP64, persistent=-1)
    o = uniform4k_oracle
    assert np.abs(a["f"] - o["f"]).max() < FP64_PAIR_ABS
    assert (np.abs(a["M"] - o["M"]) / o["M"]).max() < FP64_CELL_REL
    assert np.array_equal(a["M"], b["M"]) and np.array_equal(a["f"], b["f"])


def test_mixed_task_batches_uniform4k(mapper, uniform4k, uniform4k_oracle):
    """Distribution 3 (edge terms as wavefront task batches): oracle parity, determinism."""
    say("case: mixed task batches uniform 4096")
    p, c = uniform4k
    em.map_set_tune(mapper.ctx, em.MAP_MIXED, persistent=3)
    try:
        a = _run(mapper, p, c, em.MAP_MIXED)
        b = _run(mapper, p, c, em.MAP_MIXED)
    finally:
        em.map_set_tune(mapper.ctx, em.MAP_MIXED, persistent=-1)
    o = uniform4k_oracle
    rel = np.abs(a["M"] - o["M"]) / o["M"]
    say(f"task batches uniform4k: max cell rel err {rel.max():.3e}, max pair abs err "
        f"{np.abs(a['f'] - o['f']).max():.3e}")
    assert rel.max() < MIXED_CELL_REL
    assert abs(a["M"].sum() - p.m.sum()) < MASS_ABS
    assert np.array_equal(a["M"], b["M"]) and np.array_equal(a["f"], b["f"]) and np.array_equal(a["S"], b["S"])


# ------------------------------------------------------------------ ragged and edge cases
def test_ragged_small_clumps(mapper):
    say("case: clumps 1000 ragged")
    p, c = synth.workload("clumps", 1000, 21)
    o = oracle.map_particles(p, c)
    for prec, tol, dist in ((em.MAP_FP64, FP64_CELL_REL, 1), (em.MAP_MIXED, MIXED_CELL_REL, 1),
                            (em.MAP_MIXED, MIXED_CELL_REL, 3), (em.MAP_FP64, FP64_CELL_REL, 3)):
        em.map_set_tune(mapper.ctx, prec, persistent=dist)
        r = _run(mapper, p, c, prec)
        em.map_set_tune(mapper.ctx, prec, persistent=-1)
        assert np.array_equal(r["pair_p"], o["pair_p"]) and np.array_equal(r["pair_c"], o["pair_c"])
        assert (np.abs(r["M"] - o["M"]) / o["M"]).max() < tol


def test_wide_supports(mapper):
    """Particles whose supports cover most cells: more candidate cells than the
    walk keeps per particle in its first pass, so the overflow walk runs."""
    say("case: wide supports (candidate overflow)")
    p, c = synth.workload("uniform", 2048, 25)
    h = p.h.copy()
    h[[3, 700, 1500]] = [0.3, 0.45, 0.6]
    p2 = synth.Particles(p.xyz, p.m, h)
    o = oracle.map_particles(p2, c)
    assert np.bincount(o["pair_p"], minlength=p.n)[[700, 1500]].min() > 512
    for prec, tol in ((em.MAP_FP64, FP64_CELL_REL), (em.MAP_MIXED, MIXED_CELL_REL)):
        r = _run(mapper, p2, c, prec)
        assert np.array_equal(r["pair_p"], o["pair_p"]) and np.array_equal(r["pair_c"], o["pair_c"])
        assert (np.abs(r["M"] - o["M"]) / o["M"]).max() < tol


def test_single_cell_fraction_one(mapper):
    say("case: single cell")
    from tests.test_oracle_pins import box_cell
    c = box_cell((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    p = synth.Particles(np.array([[0.5, 0.5, 0.5]]), np.array([2.0]), np.array([0.2]))
    for prec in (em.MAP_FP64, em.MAP_MIXED):
        r = _run(mapper, p, c, prec)
        assert r["f"].size == 1
        assert abs(r["f"][0] - 1.0) < 1e-14
        assert abs(r["M"][0] - 2.0) < 1e-14


def test_one_wall_half_space(mapper):
    say("case: one wall")
    from tests.test_oracle_pins import box_cell, half_space
    c = box_cell((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    us = np.array([0.3, 0.77, 1.0, 1.5])
    h = 0.1
    xyz = np.column_stack([us * h, np.full(4, 0.5), np.full(4, 0.5)])
    p = synth.Particles(xyz, np.full(4, 0.25), np.full(4, h))
    r = _run(mapper, p, c, em.MAP_FP64)
    ref = np.array([1 - half_space(u) for u in us])
    assert np.abs(r["S"] - ref).max() < 1e-13


def test_particle_on_wall_plane(mapper):
    say("case: particle on a wall plane")
    p, c = synth.workload("uniform", 64, 23)
    # move particle 5 onto a wall plane of its own cell (the face's plane)
    j = c.cell_face_off[5]
    n, cc = c.face_plane[j, :3], c.face_plane[j, 3]
    x = p.xyz.copy()
    x[5] = x[5] + (cc - n @ x[5]) * n
    p2 = synth.Particles(x, p.m, p.h)
    o = oracle.map_particles(p2, c)
    r = _run(mapper, p2, c, em.MAP_FP64)
    assert np.array_equal(r["pair_c"], o["pair_c"])
    assert np.abs(r["f"] - o["f"]).max() < 1e-12


def test_empty_inputs(mapper):
    say("case: empty particles")
    p, c = synth.workload("uniform", 32, 24)
    e = synth.Particles(np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    r = _run(mapper, e, c, em.MAP_FP64, want_pairs=False)
    assert r["stats"]["n_pairs"] == 0 and np.all(r["M"] == 0)


@pytest.mark.parametrize("what", ["h_zero", "nan_pos", "bad_offsets", "vid_range", "small_face", "bad_normal"])
def test_invalid_inputs_rejected(mapper, what):
    say(f"case: invalid input {what}")
    p, c = synth.workload("uniform", 32, 25)
    xyz, m, h = p.xyz.copy(), p.m.copy(), p.h.copy()
    cc = synth.Cells(c.cell_face_off.copy(), c.face_vert_off.copy(), c.face_vert.copy(), c.face_plane.copy(),
                     c.face_nb, c.verts.copy(), c.cell_volume.copy(), c.box)
    expect = em.MAP_EINVAL
    if what == "h_zero":
        h[3] = 0.0
    elif what == "nan_pos":
        xyz[7, 1] = np.nan
    elif what == "bad_offsets":
        cc.cell_face_off[5] = cc.cell_face_off[6] + 1
        expect = em.MAP_EGEOM
    elif what == "vid_range":
        cc.face_vert[10] = c.n_verts + 5
        expect = em.MAP_EGEOM
    elif what == "small_face":
        cc.face_vert_off[3] = cc.face_vert_off[2] + 2
        expect = em.MAP_EGEOM
    elif what == "bad_normal":
        cc.face_plane[4, :3] *= 1.5
        expect = em.MAP_EGEOM
    with pytest.raises(em.MapError) as ei:
        mapper.map(synth.Particles(xyz, m, h), cc)
    assert ei.value.code == expect
    # the context stays usable
    r = mapper.map(p, c)
    assert abs(r["M"].sum() - p.m.sum()) < 1e-12


# ------------------------------------------------------------------ clumps 262144 (sampled oracle)
QUEUED = "mixed-queued"  # mixed path with its edge terms run as wavefront task batches (distribution 3)
QUEUED64 = "fp64-queued"  # the same for the FP64 path


@pytest.fixture(scope="module")
def clumps_gpu(mapper, clumps256k):
    p, c = clumps256k
    out = {}
    for prec in (em.MAP_FP64, em.MAP_MIXED):
        say(f"case: clumps 262144 precision {prec}")
        em.map_set_tune(mapper.ctx, prec, persistent=1)
        out[prec] = _run(mapper, p, c, prec)
    say("case: clumps 262144 mixed, task batches")
    em.map_set_tune(mapper.ctx, em.MAP_MIXED, persistent=3)
    out[QUEUED] = _run(mapper, p, c, em.MAP_MIXED)
    say("case: clumps 262144 FP64, task batches")
    em.map_set_tune(mapper.ctx, em.MAP_FP64, persistent=3)
    out[QUEUED64] = _run(mapper, p, c, em.MAP_FP64)
    for prec in (em.MAP_FP64, em.MAP_MIXED):
        em.map_set_tune(mapper.ctx, prec, persistent=-1)
    return out


def test_clumps_pairs_sampled(clumps256k, clumps_gpu):
    p, c = clumps256k
    r = clumps_gpu[em.MAP_FP64]
    sel = np.sort(np.random.default_rng(7).choice(c.n_cells, 64, replace=False))
    pp, pc = oracle.pairs_for_cells(p.xyz, p.h, c, sel)
    for i in sel:
        gpu = r["pair_p"][r["pair_c"] == i]
        ref = np.sort(pp[pc == i])
        assert np.array_equal(gpu, ref), i
    sp = np.random.default_rng(8).choice(p.n, 64, replace=False)
    qp, qc = oracle.pairs_for_particles(p.xyz, p.h, c, sp)
    counts = np.bincount(r["pair_p"], minlength=p.n)
    assert np.array_equal(counts[sp], np.array([(qp == a).sum() for a in sp]))


@pytest.mark.parametrize("prec,tol", [(em.MAP_FP64, FP64_CELL_REL), (em.MAP_MIXED, MIXED_CELL_REL),
                                      (QUEUED, MIXED_CELL_REL), (QUEUED64, FP64_CELL_REL)])
def test_clumps_cells_sampled(clumps256k, clumps_gpu, prec, tol):
    p, c = clumps256k
    r = clumps_gpu[prec]
    sel = np.sort(np.random.default_rng(9).choice(c.n_cells, 48, replace=False))
    M, rho, S, _ = oracle.sampled_cell_mass(p, c, sel)
    rel = np.abs(r["M"][sel] - M) / M
    say(f"clumps precision {prec}: sampled cell rel err max {rel.max():.3e}")
    assert rel.max() < tol
    assert abs(r["stats"]["mass_out"] - 1.0) < MASS_ABS
    assert abs(r["M"].sum() - 1.0) < MASS_ABS
    interior = np.all((p.xyz - 2 * p.h[:, None] > 0) & (p.xyz + 2 * p.h[:, None] < 1), axis=1)
    assert np.abs(r["S"][interior] - 1).max() < (1e-12 if prec in (em.MAP_FP64, QUEUED64) else 1e-5)
    if prec == QUEUED:  # the two mixed distributions agree to FP32 rounding of the terms
        ref = clumps_gpu[em.MAP_MIXED]
        assert np.array_equal(ref["pair_p"], r["pair_p"]) and np.array_equal(ref["pair_c"], r["pair_c"])
        assert (np.abs(r["M"] - ref["M"]) / ref["M"]).max() < MIXED_CELL_REL
    if prec == QUEUED64:  # the FP64 distributions differ only in the order of FP64 additions
        ref = clumps_gpu[em.MAP_FP64]
        assert np.abs(r["f"] - ref["f"]).max() < FP64_PAIR_ABS
        assert (np.abs(r["M"] - ref["M"]) / ref["M"]).max() < FP64_CELL_REL


def test_autotune_and_cache(tmp_path, uniform4k):
    say("case: autotune and cache")
    p, c = uniform4k
    cache = str(tmp_path / "tune.txt")
    with em.Mapper(device=0, tune_cache_path=cache) as mp:
        mp.set_precision(em.MAP_MIXED)
        ref = mp.map(p, c)
        shape, ms = em.map_autotune(mp.ctx, p.xyz, p.m, p.h, c, em.MAP_MIXED)
        assert ms > 0 and shape[3] in (1, 2, 3)
        r = mp.map(p, c)
        # distributions agree to the FP32 rounding of the terms
        assert (np.abs(r["M"] - ref["M"]) / ref["M"]).max() < MIXED_CELL_REL
    lines = open(cache).read().split()
    assert len(lines) >= 8
    with em.Mapper(device=0, tune_cache_path=cache) as mp2:
        assert em.map_get_tune(mp2.ctx, em.MAP_MIXED, r["stats"]["n_pairs"]) == tuple(shape)


def test_clumps_all_cells_mixed_vs_fp64(clumps256k, clumps_gpu):
    """Every cell of the 262,144-particle workload: the mixed path the benchmark times (task batches)
    against the FP64 path (itself held to the oracle at 1e-10 on sampled cells above), at the mixed
    bar per cell, and every pair fraction within 1e-6."""
    a, b = clumps_gpu[QUEUED], clumps_gpu[QUEUED64]
    assert np.array_equal(a["pair_p"], b["pair_p"]) and np.array_equal(a["pair_c"], b["pair_c"])
    rel = np.abs(a["M"] - b["M"]) / b["M"]
    df = np.abs(a["f"] - b["f"])
    say(f"clumps all cells: mixed vs FP64 max rel {rel.max():.3e} (mean {rel.mean():.3e}), "
        f"max pair |df| {df.max():.3e}, fixups {a['stats']['n_fixup_terms']}")
    assert rel.max() < MIXED_CELL_REL
    assert df.max() < 1e-6
    assert a["stats"]["n_fixup_terms"] > 0


def test_mixed_cell_budget_switches(uniform4k, uniform4k_oracle):
    """The per-cell error budget of the mixed path: a negative budget leaves every pair in FP32; a
    budget no cell can meet sends every pair to the FP64 recomputation, whose values then equal the
    oracle's to the FP64 bar; the default recomputes few cells and meets the mixed bar."""
    say("case: mixed per-cell error budget")
    p, c = uniform4k
    o = uniform4k_oracle
    with em.Mapper(device=0, precision=em.MAP_MIXED, cell_tol=-1.0) as mp:
        raw = mp.map(p, c, want_pairs=True)
    assert raw["stats"]["n_fp64_cells"] == 0 and raw["stats"]["n_fp64_pairs"] == 0
    with em.Mapper(device=0, precision=em.MAP_MIXED, cell_tol=1e-300) as mp:
        allc = mp.map(p, c, want_pairs=True)
    assert allc["stats"]["n_fp64_cells"] == c.n_cells and allc["stats"]["n_fp64_pairs"] == o["f"].size
    assert np.abs(allc["f"] - o["f"]).max() < FP64_PAIR_ABS
    assert (np.abs(allc["M"] - o["M"]) / o["M"]).max() < FP64_CELL_REL
    # the recomputation (pair, wall terms in parallel, walls added in order) is the per-pair FP64 form
    # (distribution 0, one thread per pair) to the bit
    with em.Mapper(device=0, precision=em.MAP_FP64) as mp:
        em.map_set_tune(mp.ctx, em.MAP_FP64, 0, 1, 4, 0)
        flat = mp.map(p, c, want_pairs=True)
    assert np.array_equal(allc["pair_p"], flat["pair_p"]) and np.array_equal(allc["f"], flat["f"])
    with em.Mapper(device=0, precision=em.MAP_MIXED) as mp:
        dflt = mp.map(p, c, want_pairs=True)
    rel_raw = (np.abs(raw["M"] - o["M"]) / o["M"]).max()
    rel = (np.abs(dflt["M"] - o["M"]) / o["M"]).max()
    say(f"  raw mixed max cell rel {rel_raw:.3e}; with the budget {rel:.3e} "
        f"({dflt['stats']['n_fp64_cells']} cells, {dflt['stats']['n_fp64_pairs']} pairs in FP64)")
    assert rel < MIXED_CELL_REL
    assert dflt["stats"]["n_fp64_cells"] < c.n_cells // 10
