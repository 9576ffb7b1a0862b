"""The largest single-GPU job: 8,388,608 particles of the log-normal cloud
(sigma_ln 1.5, P(k) ~ k^-4), box-clipped Voronoi cells of the particles built
on the device, full-resolution mapping in both precisions and the
pseudo-particle variant with four sources (the ~1e7-particle regime of the
paper's timings, Sec. IV-B).

The oracle cannot map the whole job in test time, so it checks seeded samples
against the same device run:
  * the pair set of 0.25 % of the cells (oracle pair search over those cells
    alone) equals the device's pairs of those cells, bit for bit;
  * each of their pair fractions, and each cell's raw sum of m_a f_ai, agrees
    with the oracle (mixed: 1e-5 relative per cell; FP64: 1e-10);
  * their normalised cell masses agree with the oracle's fractions over the
    device's S_a;
  * S_a of 2,000 sampled particles (all their pairs, oracle pair search over
    the whole grid) agrees with the oracle;
  * over all 8.4 million cells, the mixed result agrees with the FP64 result
    within 1e-5 relative, and mass is conserved to 1e-9 in both.
The device grid itself is checked against the oracle's cells on sampled cells
(the largest and most-faceted among them).  The pseudo variant is small enough
for the oracle to map in full.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
import paper_2404_17084_amd as em

pytestmark = pytest.mark.gpu

N_LARGE = 8388608
SEED_LARGE = 5
SOURCES4 = [[0.25, 0.25, 0.25], [0.75, 0.75, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75]]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def large():
    import torch

    t0 = time.perf_counter()
    say(f"case: large job, generating {N_LARGE} log-normal particles (seed {SEED_LARGE})")
    p = synth.particles("lognormal", N_LARGE, SEED_LARGE)
    say(f"  generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    mp = em.Mapper(device=0, precision=em.MAP_MIXED)
    xyz, m, h = t(p.xyz), t(p.m), t(p.h)
    say("case: large job, device Voronoi grid")
    G = em.map_voronoi(mp.ctx, xyz, synth.BOX, 0, device=True)
    torch.cuda.synchronize()
    assert G.n_cells == N_LARGE
    say(f"  {G.n_cells} cells, {int(G.face_plane.shape[0])} walls, {int(G.face_vert.shape[0])} wall-vertex slots, "
        f"{G.ms:.0f} ms")
    yield dict(p=p, mp=mp, xyz=xyz, m=m, h=h, G=G)
    mp.close()


def _map_with_pairs(mp, L, precision):
    import torch

    mp.set_precision(precision)
    dev = L["xyz"].device
    npairs = em.map_pairs(mp.ctx, L["xyz"], L["m"], L["h"], L["G"], want_pairs=False)
    F = torch.empty(npairs, dtype=torch.float64, device=dev)
    PP = torch.empty(npairs, dtype=torch.int32, device=dev)
    PC = torch.empty(npairs, dtype=torch.int32, device=dev)
    M = torch.zeros(L["G"].n_cells, dtype=torch.float64, device=dev)
    S = torch.zeros(L["p"].n, dtype=torch.float64, device=dev)
    st = em.map_particles(mp.ctx, L["xyz"], L["m"], L["h"], L["G"], cell_mass=M, frac_sum_raw=S, pair_frac=F,
                          pair_p=PP, pair_c=PC)
    torch.cuda.synchronize()
    return st, M, S, F, PP, PC


def test_large_full_resolution(large):
    import torch

    L = large
    p, mp = L["p"], L["mp"]
    say("case: large job, mixed mapping with pair outputs")
    st, M, S, F, PP, PC = _map_with_pairs(mp, L, em.MAP_MIXED)
    say(f"  {st['n_pairs']} pairs, integrate {st['ms_integrate']:.1f} ms, total {st['ms_total']:.1f} ms, "
        f"FP64 cells {st['n_fp64_cells']}, fixups {st['n_fixup_terms']}")
    assert st["n_pairs"] > 4e8
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-9 * st["mass_in"]

    # seeded 0.25 % of the cells: pair sets, fractions, raw and normalised cell sums
    rng = np.random.default_rng(2024)
    sel = np.sort(rng.choice(N_LARGE, N_LARGE // 400, replace=False))
    say(f"case: large job, oracle on {sel.size} sampled cells")
    cells = synth.cells_from(L["G"])
    sub = synth.cells_subset(cells, sel)
    op, oc_local = oracle.pairs(p.xyz, p.h, sub)
    oc = sel[oc_local]
    lut = torch.zeros(N_LARGE, dtype=torch.bool, device=PC.device)
    lut[torch.from_numpy(sel).to(PC.device)] = True
    mask = lut[PC.long()]
    gp = PP[mask].cpu().numpy()
    gc = PC[mask].cpu().numpy()
    gf = F[mask].cpu().numpy()
    o_ord = np.lexsort((op, oc))
    assert np.array_equal(gc, oc[o_ord]) and np.array_equal(gp, op[o_ord]), "pair sets differ"
    fo = oracle.pair_fractions(p.xyz, p.h, sub, op, oc_local)[o_ord]
    say(f"  {gp.size} pairs; max |df| {np.abs(gf - fo).max():.3e}")
    assert np.abs(gf - fo).max() <= 1e-5
    raw_g = np.bincount(np.searchsorted(sel, gc), weights=p.m[gp] * gf, minlength=sel.size)
    raw_o = np.bincount(np.searchsorted(sel, gc), weights=p.m[gp] * fo, minlength=sel.size)
    rel = np.abs(raw_g - raw_o) / raw_o
    say(f"  raw cell sums: max rel {rel.max():.3e}")
    assert rel.max() <= 1e-5
    Sg = S.cpu().numpy()
    Mo = np.bincount(np.searchsorted(sel, gc), weights=p.m[gp] * fo / Sg[gp], minlength=sel.size)
    Mg = M.cpu().numpy()[sel]
    relm = np.abs(Mg - Mo) / Mo
    say(f"  normalised cell masses: max rel {relm.max():.3e}")
    assert relm.max() <= 1e-5

    # S_a of sampled particles against the oracle over the whole grid
    psel = np.sort(rng.choice(N_LARGE, 2000, replace=False))
    say(f"case: large job, S_a of {psel.size} sampled particles")
    qp, qc = oracle.pairs(p.xyz[psel], p.h[psel], cells)
    fq = oracle.pair_fractions(p.xyz[psel], p.h[psel], cells, qp, qc)
    So = np.bincount(qp, weights=fq, minlength=psel.size)
    plut = torch.zeros(N_LARGE, dtype=torch.bool, device=PP.device)
    plut[torch.from_numpy(psel).to(PP.device)] = True
    gmask = plut[PP.long()]
    assert int(gmask.sum()) == qp.size, "pair counts of the sampled particles differ"
    dS = np.abs(Sg[psel] - So)
    say(f"  max |dS| {dS.max():.3e}")
    assert dS.max() <= 1e-5

    # FP64 on the same job: the sample at 1e-10, and every cell of the mixed result against it
    say("case: large job, FP64 mapping")
    st64, M64, S64, F64, PP64, PC64 = _map_with_pairs(mp, L, em.MAP_FP64)
    assert st64["n_pairs"] == st["n_pairs"]
    assert torch.equal(PP64, PP) and torch.equal(PC64, PC)
    assert abs(st64["mass_out"] - st64["mass_in"]) <= 1e-9 * st64["mass_in"]
    gf64 = F64[mask].cpu().numpy()
    raw64 = np.bincount(np.searchsorted(sel, gc), weights=p.m[gp] * gf64, minlength=sel.size)
    rel64 = np.abs(raw64 - raw_o) / raw_o
    say(f"  FP64 integrate {st64['ms_integrate']:.1f} ms; sample raw cell sums max rel {rel64.max():.3e}")
    assert rel64.max() <= 1e-10
    M64h = M64.cpu().numpy()
    relall = np.abs(M.cpu().numpy() - M64h) / M64h
    say(f"  mixed vs FP64 over all {N_LARGE} cells: max rel {relall.max():.3e}, mean {relall.mean():.3e}")
    assert relall.max() <= 1e-5
    del F, PP, PC, F64, PP64, PC64
    torch.cuda.empty_cache()


def test_large_voronoi_sampled(large):
    """The device grid of the 8.4 million sites against the oracle's cells on 16 seeded cells, the 8
    largest and the 8 with the most faces (the longest candidate walks: those that can leave the
    wavefront walk for the serial one): volumes to 1e-12 relative, neighbour sets exact."""
    L = large
    cells = synth.cells_from(L["G"])
    nf = np.diff(cells.cell_face_off)
    rng = np.random.default_rng(99)
    sel = np.unique(np.concatenate([rng.choice(N_LARGE, 16, replace=False), np.argsort(cells.cell_volume)[-8:],
                                    np.argsort(nf, kind="stable")[-8:]]))
    say(f"case: large job, device Voronoi cells against the oracle on {sel.size} cells")
    O = oracle.voronoi(L["p"].xyz, synth.BOX, sel=sel)
    rel = np.abs(cells.cell_volume[sel] - O["cell_volume"]) / O["cell_volume"]
    say(f"  volume max rel {rel.max():.3e}")
    assert rel.max() < 1e-12
    for k, c in enumerate(sel):
        dev = set(cells.face_nb[cells.cell_face_off[c]:cells.cell_face_off[c + 1]].tolist())
        orc = set(O["face_nb"][O["cell_face_off"][k]:O["cell_face_off"][k + 1]].tolist())
        assert dev == orc, (int(c), sorted(dev ^ orc))


def test_large_pseudo_variant(large):
    """Four sources, theta 0.5, r_part 0.05, r_leaf 0.1, leaf <= 8: the pseudo set's device Voronoi cells and
    its mixed mapping against the oracle over every cell."""
    import torch

    L = large
    mp = L["mp"]
    say("case: large job, pseudo variant (4 sources)")
    dev = L["xyz"].device
    n = L["p"].n
    out = dict(xyz=torch.zeros((n, 3), dtype=torch.float64, device=dev),
               m=torch.zeros(n, dtype=torch.float64, device=dev), h=torch.zeros(n, dtype=torch.float64, device=dev),
               size=torch.zeros(n, dtype=torch.float64, device=dev),
               kind=torch.zeros(n, dtype=torch.int32, device=dev), ref=torch.zeros(n, dtype=torch.int64, device=dev))
    r = em.map_pseudo(mp.ctx, L["xyz"], L["m"], L["h"], synth.BOX, SOURCES4, theta=0.5, r_part=0.05, r_leaf=0.1,
                      leaf_size=8, out=out)
    host = lambda a: np.ascontiguousarray(a.cpu().numpy())
    q = synth.Particles(host(r["xyz"]), host(r["m"]), host(r["h"]))
    say(f"  {q.n} pseudo-particles ({r['stats']['n_pseudo_nodes']} nodes)")
    assert abs(q.m.sum() - L["p"].m.sum()) <= 1e-12
    del out, r
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    qx, qm, qh = t(q.xyz), t(q.m), t(q.h)
    G = em.map_voronoi(mp.ctx, qx, synth.BOX, 0, device=True)
    mp.set_precision(em.MAP_MIXED)
    M = torch.zeros(G.n_cells, dtype=torch.float64, device=dev)
    st = em.map_particles(mp.ctx, qx, qm, qh, G, cell_mass=M)
    torch.cuda.synchronize()
    say(f"  {st['n_pairs']} pairs, integrate {st['ms_integrate']:.2f} ms")
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-9 * st["mass_in"]
    cells = synth.cells_from(G)
    O = oracle.map_particles(q, cells)
    assert O["pair_p"].size == st["n_pairs"]
    rel = np.abs(M.cpu().numpy() - O["M"]) / O["M"]
    say(f"  all {G.n_cells} cells vs oracle: max rel {rel.max():.3e}")
    assert rel.max() <= 1e-5
