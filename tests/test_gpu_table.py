"""GPU parity of the tabulated variant (MAP_TABLE; Sec. II-B's pre-computed pyramid integral).

The library builds its table from its own FP64 closed form; the node values
must equal the oracle's (built from the oracle's closed form) to 1e-13.  The
mapping reads the table in FP32 (node values, trilinear weights, the
triangle's solid angle), so each of a pair's table terms carries an error of a
few FP32 ulps of its size (at most 1/8, ulp 1.5e-8); with up to ~300 terms per
pair the bar against the FP64 tabulated oracle is 2e-5 per pair, and the cell
masses, averages of such fractions normalised by S_a, get 2e-5 relative.
The pair sets are the ordinary ones (identical).  Against the closed form the
variant is an approximation: with the default 64^3 table the interior S_a
deviate from 1 by less than 2e-3 (the oracle's own convergence pin gives the
same order), and total mass is kept by the normalisation.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2404_17084_amd as em

pytestmark = pytest.mark.gpu

PAIR_ABS = 2e-5
CELL_REL = 2e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def uniform4k():
    p, c = synth.workload(*synth.UNIFORM_4K)
    oracle.use_table(64, 64, 64)
    return p, c, oracle.map_particles(p, c, profile=oracle.TABLE)


def test_table_nodes_match_oracle():
    say("case: table node values 32 x 36 x 40")
    with em.Mapper(device=0) as mp:
        mp.set_table(32, 36, 40)
        G = mp.table()
    O = oracle.table(32, 36, 40)
    err = np.abs(G - O).max()
    say(f"  max |node difference| = {err:.3e}")
    assert err < 1e-13


def test_table_mapping_matches_oracle_uniform4k(uniform4k):
    say("case: MAP_TABLE uniform 4096 vs the tabulated oracle")
    p, c, o = uniform4k
    with em.Mapper(device=0, precision=em.MAP_TABLE) as mp:
        r = mp.map(p, c, want_pairs=True)
        r2 = mp.map(p, c, want_pairs=True)
    assert np.array_equal(r["pair_p"], o["pair_p"]) and np.array_equal(r["pair_c"], o["pair_c"])
    df = np.abs(r["f"] - o["f"]).max()
    rel = (np.abs(r["M"] - o["M"]) / o["M"]).max()
    say(f"  pair |df| max {df:.3e}, cell rel max {rel:.3e}")
    assert df < PAIR_ABS and rel < CELL_REL
    assert np.abs(r["S"] - o["S"]).max() < PAIR_ABS * 8
    assert abs(r["M"].sum() - p.m.sum()) < 1e-12
    assert r["stats"]["n_fixup_terms"] == 0
    for k in ("f", "M", "S"):
        assert np.array_equal(r[k], r2[k])  # repeatable bit for bit


def test_table_accuracy_against_closed_form(uniform4k):
    say("case: MAP_TABLE against the FP64 closed form")
    p, c, _ = uniform4k
    with em.Mapper(device=0) as mp:
        ref = mp.map(p, c)
        mp.set_precision(em.MAP_TABLE)
        r = mp.map(p, c)
        mp.set_table(128, 128, 128)
        r128 = mp.map(p, c)
    interior = np.all((p.xyz > 2 * p.h[:, None]) & (p.xyz < 1 - 2 * p.h[:, None]), axis=1)
    d64 = np.abs(r["S"][interior] - 1).max()
    d128 = np.abs(r128["S"][interior] - 1).max()
    c64 = (np.abs(r["M"] - ref["M"]) / ref["M"]).max()
    c128 = (np.abs(r128["M"] - ref["M"]) / ref["M"]).max()
    say(f"  interior |S-1|: 64^3 {d64:.3e}, 128^3 {d128:.3e}; cell rel vs closed form {c64:.3e}, {c128:.3e}")
    assert d64 < 2e-3 and d128 < d64 / 2 and c128 < c64


def test_table_sampled_cells_clumps262144():
    say("case: MAP_TABLE clumps 262144, sampled cells")
    p, c = synth.workload(*synth.CLUMPS_256K)
    with em.Mapper(device=0, precision=em.MAP_TABLE) as mp:
        r = mp.map(p, c)
    oracle.use_table(64, 64, 64)
    sel = np.sort(np.random.default_rng(13).choice(c.n_cells, 32, replace=False))
    M, _, _, _ = oracle.sampled_cell_mass(p, c, sel, profile=oracle.TABLE)
    rel = (np.abs(r["M"][sel] - M) / M).max()
    say(f"  sampled cell rel max {rel:.3e}")
    assert rel < CELL_REL
    assert abs(r["M"].sum() - 1.0) < 1e-9


def test_table_arguments():
    say("case: MAP_TABLE arguments")
    with em.Mapper(device=0) as mp:
        for bad in ((4, 64, 64), (64, 2000, 64), (1024, 1024, 1024)):
            with pytest.raises(em.MapError) as ei:
                mp.set_table(*bad)
            assert ei.value.code == em.MAP_EINVAL
        with pytest.raises(em.MapError):
            mp.set_precision(3)
        with pytest.raises(em.MapError):
            em.map_set_tune(mp.ctx, em.MAP_TABLE, 2, 1, 4, 3)
