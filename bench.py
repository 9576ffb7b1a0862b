#!/usr/bin/env python
"""Throughput of the Exact mapping on one MI355X: particle-cell pairs mapped per second.

One step = one synchronous ``map_particles`` call on the 262,144-particle clumpy
workload (uniform background plus three Gaussian clumps, sigma 0.05 box,
density contrast 1e4; box-clipped Voronoi cells of the particles): input
validation, geometry tables, pair search, integration of every pair, FP64
fixups, the sum-to-one normalisation and the per-cell reduction.  Inputs are
resident in device memory before the timed region.  The mixed path (FP32
closed-form terms, FP64 geometry and sums) is the headline value; the all-FP64
path is timed beside it.  Further legs: served mapping of 64 jobs with Poisson
arrivals (p50/p99 latency), inverse mapping, tabulated variant, device Voronoi
grid, pseudo-particle front end, the oracle on the host cores, and (on
request) a VALU calibration kernel.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Work counters of the integration kernel (the GPU's own formulation; transcendentals = 1 flop each),
# reported beside the model below for comparison.
FLOP_FACE, FLOP_EDGE, FLOP_ETERM, FLOP_MOMENT, FLOP_QPOINT, FLOP_ANGLE = 7, 19, 8, 66, 31, 6

# HBM bytes per launch of the mixed integration kernel (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy) and
# its measured VALU FLOPs (the SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32/F64 counters, 64 lanes per instruction,
# FMA = 2), valid only for the kernel source they were measured on
# (profiles/traffic_integrate_queued_clumps262144.md, profiles/valu_integrate_queued_clumps262144.md); null
# once the source has changed.
COUNTER_SOURCE = "paper_2404_17084_amd/csrc/em_integrate.hip"
COUNTER_SHA256_PREFIX = "e913931a62f3ef08"
TRAFFIC_BYTES = 2.631e9
VALU_FLOPS_PER_LAUNCH = 5.581e11

PEAK_FP64 = 78.6   # TFLOP/s, MI355X FP64 vector
PEAK_FP32 = 157.3  # TFLOP/s, MI355X FP32 vector (packed)

WORKLOAD = ("clumps-262144: uniform background + 3 Gaussian clumps (sigma 0.05 box, contrast 1e4, seed 2); "
            "h = 1.2 (m/rho)^(1/3) with rho a top-hat density over the 58 nearest neighbours (h = r_58/2, "
            "58 particles within 2h); box-clipped Voronoi cells of the particles")


def counters_valid():
    import hashlib

    if COUNTER_SHA256_PREFIX is None:
        return False
    try:
        with open(os.path.join(ROOT, COUNTER_SOURCE), "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return False
    return digest.startswith(COUNTER_SHA256_PREFIX)


def kernel_work_flops(st) -> float:
    return (FLOP_FACE * st["n_face_visits"] + FLOP_EDGE * st["n_edge_visits"] + FLOP_ETERM * st["n_edge_terms"]
            + FLOP_MOMENT * st["n_moment_evals"] + FLOP_QPOINT * st["n_quad_points"]
            + FLOP_ANGLE * st["n_angle_evals"])


def to_device(p, c):
    import torch

    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    class DevCells:
        pass

    dc = DevCells()
    dc.cell_face_off = t(c.cell_face_off)
    dc.face_vert_off = t(c.face_vert_off)
    dc.face_vert = t(c.face_vert.astype(np.int32))
    dc.face_plane = t(c.face_plane)
    dc.verts = t(c.verts)
    dc.cell_volume = t(c.cell_volume)
    dc.box = c.box
    return t(p.xyz), t(p.m), t(p.h), dc


def oracle_sample(p, c, n_cells, seed=12345):
    import oracle

    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(c.n_cells, n_cells, replace=False))
    return sel, oracle.pairs_for_cells(p.xyz, p.h, c, sel)


def cpu_baseline(p, c, target_s: float = 12.0):
    """The FP64 oracle, untuned, on a seeded sample of cells with all their pairs (pair search and
    closed-form integrals): on all host cores, then on one core for a smaller sample.  Also returns the
    operation count of the oracle's formulas over the larger sample (the flop model of the roofline)."""
    import oracle

    t0 = time.perf_counter()
    sel, (pp, pc) = oracle_sample(p, c, 400)
    oracle.pair_fractions(p.xyz, p.h, c, pp, pc)
    dt = time.perf_counter() - t0
    n_cells = int(min(c.n_cells, max(400, 400 * target_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    sel, (pp, pc) = oracle_sample(p, c, n_cells)
    f = oracle.pair_fractions(p.xyz, p.h, c, pp, pc)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(f))
    cores = oracle.num_threads()
    fm = oracle.flop_model(p.xyz, p.h, c, pp, pc)
    # one core: a sample sized for about 6 s
    oracle.set_num_threads(1)
    try:
        n1 = max(50, int(n_cells * 6.0 / max(dt * cores, 1e-3)))
        t0 = time.perf_counter()
        _, (qp, qc) = oracle_sample(p, c, n1, seed=54321)
        oracle.pair_fractions(p.xyz, p.h, c, qp, qc)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    base = {"value": pp.size / dt, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_cells} of {c.n_cells} cells (seeded), all {pp.size} of their pairs: pair search + "
                      f"closed-form integrals, {dt:.1f} s on {cores} threads",
            "one_core": {"value": qp.size / dt1, "unit": "pairs/s",
                         "sample": f"{n1} cells, {qp.size} pairs, {dt1:.1f} s on 1 thread"}}
    model = {"flops_per_pair": fm["flops"] / max(pp.size, 1), "sample_pairs": int(pp.size),
             "faces_per_pair": fm["faces"] / max(pp.size, 1), "edges_per_pair": fm["edges"] / max(pp.size, 1),
             "pyramids_per_pair": fm["pyramids"] / max(pp.size, 1), "pieces_per_pair": fm["pieces"] / max(pp.size, 1)}
    return base, model


def flop_model_only(p, c, n_cells=6000):
    import oracle

    _, (pp, pc) = oracle_sample(p, c, n_cells)
    fm = oracle.flop_model(p.xyz, p.h, c, pp, pc)
    return {"flops_per_pair": fm["flops"] / max(pp.size, 1), "sample_pairs": int(pp.size),
            "faces_per_pair": fm["faces"] / max(pp.size, 1), "edges_per_pair": fm["edges"] / max(pp.size, 1),
            "pyramids_per_pair": fm["pyramids"] / max(pp.size, 1), "pieces_per_pair": fm["pieces"] / max(pp.size, 1)}


def serve_leg(em, seed_sizes=4, n_jobs=64, budget=32_000_000_000, max_jobs=8, arrival_seeds=5, load=0.7):
    """Served mapping (continuous batching): n_jobs clumpy jobs of log-uniform sizes 1e4-1e6 particles
    (per-job seeds 1000 + j), their Voronoi cells built on the device beforehand; admission by the
    device-memory estimate against a 32 GB budget, mixed precision, device-resident inputs.  First all
    jobs at once (sustained rate), then Poisson arrivals at `load` times that rate for several arrival
    seeds: latency = completion - submission, p50/p99 by nearest rank."""
    import torch
    import synth

    rng = np.random.default_rng(seed_sizes)
    sizes = np.floor(10 ** rng.uniform(4, 6, n_jobs)).astype(int)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    jobs = []
    t_gen = time.perf_counter()
    with em.Mapper(device=0) as gen:
        for j, n in enumerate(sizes):
            p = synth.particles("clumps", int(n), 1000 + j)
            xyz = t(p.xyz)
            G = em.map_voronoi(gen.ctx, xyz, synth.BOX, 0, device=True)
            M = torch.zeros(int(n), dtype=torch.float64, device=dev)
            jobs.append((xyz, t(p.m), t(p.h), G, M, float(p.m.sum())))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    print(f"bench: serving inputs ready ({sizes.sum()} particles in {n_jobs} jobs, {t_gen:.1f} s)", file=sys.stderr,
          flush=True)

    def run(mp, order, arrivals=None):
        ids = []
        t0 = time.perf_counter()
        for k, j in enumerate(order):
            if arrivals is not None:
                wait = t0 + arrivals[k] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            xyz, m, h, G, M, _ = jobs[j]
            ids.append((j, em.map_submit(mp.ctx, xyz, m, h, G, M)))
        stats = []
        for j, jid in ids:
            state, st = em.map_poll(mp.ctx, jid, 120_000_000)
            assert state == em.JOB_DONE
            stats.append((j, st))
        return time.perf_counter() - t0, stats

    with em.Mapper(device=0, precision=em.MAP_MIXED, hbm_budget_bytes=budget, max_jobs=max_jobs) as mp:
        run(mp, list(range(4)))  # warm-up
        wall, stats = run(mp, list(range(n_jobs)))
        pairs = sum(st["n_pairs"] for _, st in stats)
        rate = n_jobs / wall
        mass_err = max(abs(float(jobs[j][4].sum()) - jobs[j][5]) for j, _ in stats)
        lam = load * rate
        lat = []
        open_wall = open_pairs = 0.0
        for s in range(arrival_seeds):
            arr = np.cumsum(np.random.default_rng(100 + s).exponential(1.0 / lam, n_jobs))
            order = list(np.random.default_rng(200 + s).permutation(n_jobs))
            w, st2 = run(mp, order, arr)
            lat.extend(st["ms_latency"] for _, st in st2)
            open_wall += w
            open_pairs += sum(st["n_pairs"] for _, st in st2)
    lat = np.sort(np.array(lat))
    rank = lambda q: float(lat[max(0, int(np.ceil(q * lat.size)) - 1)])
    return {"workload": f"{n_jobs} clumpy jobs, sizes log-uniform 1e4-1e6 (seed {seed_sizes}; {int(sizes.sum())} "
                        f"particles), per-job seeds 1000+j, device-built Voronoi cells, mixed precision, "
                        f"budget {budget / 1e9:.0f} GB, {max_jobs} slots",
            "closed_loop": {"jobs_per_s": rate, "pairs_per_s": pairs / wall, "wall_s": wall, "pairs": pairs,
                            "max_mass_err": mass_err},
            "open_loop": {"arrival_rate_per_s": lam, "load": load, "arrival_seeds": arrival_seeds,
                          "samples": int(lat.size), "p50_ms": rank(0.50), "p99_ms": rank(0.99),
                          "mean_ms": float(lat.mean()), "max_ms": float(lat[-1]),
                          "pairs_per_s": open_pairs / open_wall}}


def pseudo_leg(em, steps: int, warmup: int):
    """The pseudo-particle path: front end on the 2,097,152-particle log-normal cloud (one source at the
    centre, theta 0.5, r_part 0.05, r_leaf 0.1, leaf <= 8), then the mixed mapping of the pseudo set."""
    import torch
    import synth

    print("bench: generating the 2,097,152-particle log-normal cloud", file=sys.stderr, flush=True)
    p = synth.particles(*synth.LOGNORMAL_2M)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    xyz, m, h = t(p.xyz), t(p.m), t(p.h)
    n = p.n
    out = dict(xyz=torch.zeros((n, 3), dtype=torch.float64, device=dev),
               m=torch.zeros(n, dtype=torch.float64, device=dev), h=torch.zeros(n, dtype=torch.float64, device=dev),
               size=torch.zeros(n, dtype=torch.float64, device=dev),
               kind=torch.zeros(n, dtype=torch.int32, device=dev), ref=torch.zeros(n, dtype=torch.int64, device=dev))
    torch.cuda.synchronize()
    src = [[0.5, 0.5, 0.5]]
    par = dict(theta=0.5, r_part=0.05, r_leaf=0.1, leaf_size=8, h_fact_node=1.1)
    mp = em.Mapper(device=0, precision=em.MAP_MIXED)
    for _ in range(warmup):
        em.map_pseudo(mp.ctx, xyz, m, h, synth.BOX, src, out=out, **par)
    torch.cuda.synchronize()
    sts = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = em.map_pseudo(mp.ctx, xyz, m, h, synth.BOX, src, out=out, **par)
        sts.append(r["stats"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = sts[-1]
    adaptive = adaptive_leg(em, mp, xyz, m, h, src, par)
    q = synth.Particles(r["xyz"].cpu().numpy().copy(), r["m"].cpu().numpy().copy(), r["h"].cpu().numpy().copy())
    cells = synth.voronoi_cells(q.xyz)
    qx, qm, qh, qc = to_device(q, cells)
    M = torch.zeros(cells.n_cells, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        em.map_particles(mp.ctx, qx, qm, qh, qc, M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ms = em.map_particles(mp.ctx, qx, qm, qh, qc, M)
    torch.cuda.synchronize()
    dm = (time.perf_counter() - t0) / steps
    mp.close()
    return {"workload": "lognormal-2097152: log-normal density (sigma_ln 1.5, P(k) ~ k^-4, 256^3 mesh, seed 3), "
                        "h from 58 neighbours; one source at the box centre, theta 0.5, r_part 0.05, r_leaf 0.1, "
                        "leaf <= 8, h_fact 1.1",
            "particles": n, "pseudo": st["n_pseudo"], "pseudo_nodes": st["n_pseudo_nodes"],
            "particles_kept": st["n_particles"], "tree_nodes": st["n_tree_nodes"], "max_level": st["max_level"],
            "h_fallbacks": st["n_fallbacks"], "mean_neighbours": st["n_neighbours"] / max(st["n_pseudo_nodes"], 1),
            "ms_front_end": 1e3 * dt, "ms_tree": float(np.mean([s["ms_tree"] for s in sts])),
            "ms_walk": float(np.mean([s["ms_walk"] for s in sts])),
            "ms_hsolve": float(np.mean([s["ms_hsolve"] for s in sts])),
            "particles_per_s_front_end": n / dt,
            "pseudo_pairs": ms["n_pairs"], "ms_map_pseudo": 1e3 * dm, "pairs_per_s_pseudo": ms["n_pairs"] / dm,
            "fp64_cells_pseudo": ms["n_fp64_cells"], "fp64_pairs_pseudo": ms["n_fp64_pairs"],
            "mass_err_pseudo": abs(ms["mass_out"] - ms["mass_in"]), "adaptive": adaptive}


LARGE_N, LARGE_SEED = 8388608, 5
LARGE_SOURCES = [[0.25, 0.25, 0.25], [0.75, 0.75, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75]]


def large_leg(em, steps: int, with_oracle: bool):
    """The largest single-GPU job: 8,388,608 log-normal particles, their device-built Voronoi cells, the
    full-resolution mapping in both precisions (mixed vs FP64 over every cell), the oracle on a seeded 1 % of
    the cells (all their pairs) and on S_a of 8,000 particles, and the pseudo variant with four sources mapped
    in mixed precision and checked by the oracle over every cell."""
    import torch
    import oracle
    import synth

    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    print(f"bench: generating the {LARGE_N:,}-particle log-normal cloud", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    p = synth.particles("lognormal", LARGE_N, LARGE_SEED)
    gen_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    mp = em.Mapper(device=0, precision=em.MAP_MIXED)
    xyz, m, h = t(p.xyz), t(p.m), t(p.h)
    G = em.map_voronoi(mp.ctx, xyz, synth.BOX, 0, device=True)
    torch.cuda.synchronize()
    nc = G.n_cells
    res = {"workload": f"lognormal-{LARGE_N}: log-normal density (sigma_ln 1.5, P(k) ~ k^-4, 256^3 mesh, seed "
                       f"{LARGE_SEED}), h from 58 neighbours; box-clipped Voronoi cells of the particles built on "
                       f"the device; pseudo variant with 4 sources",
           "particles": p.n, "cells": nc, "walls": int(G.face_plane.shape[0]),
           "wall_vertex_slots": int(G.face_vert.shape[0]), "host_generation_s": gen_s, "ms_voronoi": G.ms}
    M = torch.zeros(nc, dtype=torch.float64, device=dev)
    Ms = {}
    for prec, name, k in ((em.MAP_MIXED, "mixed", steps), (em.MAP_FP64, "fp64", 1)):
        mp.set_precision(prec)
        em.map_particles(mp.ctx, xyz, m, h, G, M)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [em.map_particles(mp.ctx, xyz, m, h, G, M) for _ in range(k)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        st = sts[-1]
        Ms[name] = M.cpu().numpy().copy()
        res[name] = {"pairs": st["n_pairs"], "pairs_per_s": st["n_pairs"] / dt, "ms_per_step": 1e3 * dt,
                     "ms_integrate": float(np.mean([x["ms_integrate"] for x in sts])),
                     "stages_ms": {q: float(np.mean([x[q] for x in sts]))
                                   for q in ("ms_setup", "ms_pairs", "ms_integrate", "ms_fixup", "ms_reduce")},
                     "mass_rel_err": abs(st["mass_out"] - st["mass_in"]) / st["mass_in"],
                     "n_fixup_terms": st["n_fixup_terms"], "n_fp64_cells": st["n_fp64_cells"],
                     "n_candidates": st["n_candidates"]}
        print(f"bench: large {name}: {res[name]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    res["device_bytes_in_use"] = int(free0 - torch.cuda.mem_get_info()[0])
    rel = np.abs(Ms["mixed"] - Ms["fp64"]) / Ms["fp64"]
    res["mixed_vs_fp64_max_cell_rel"] = float(rel.max())
    res["mixed_vs_fp64_mean_cell_rel"] = float(rel.mean())
    res["speedup_mixed_vs_fp64"] = res["mixed"]["pairs_per_s"] / res["fp64"]["pairs_per_s"]
    if with_oracle:
        mp.set_precision(em.MAP_MIXED)
        npairs = res["mixed"]["pairs"]
        F = torch.empty(npairs, dtype=torch.float64, device=dev)
        PP = torch.empty(npairs, dtype=torch.int32, device=dev)
        PC = torch.empty(npairs, dtype=torch.int32, device=dev)
        S = torch.zeros(p.n, dtype=torch.float64, device=dev)
        em.map_particles(mp.ctx, xyz, m, h, G, cell_mass=M, frac_sum_raw=S, pair_frac=F, pair_p=PP, pair_c=PC)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rng = np.random.default_rng(2025)
        sel = np.sort(rng.choice(nc, nc // 100, replace=False))
        cells = synth.cells_from(G)
        sub = synth.cells_subset(cells, sel)
        print(f"bench: large oracle sample: pairs of {sel.size} cells", file=sys.stderr, flush=True)
        op, oc_local = oracle.pairs(p.xyz, p.h, sub)
        lut = torch.zeros(nc, dtype=torch.bool, device=dev)
        lut[t(sel)] = True
        mask = lut[PC.long()]
        gp, gc, gf = PP[mask].cpu().numpy(), PC[mask].cpu().numpy(), F[mask].cpu().numpy()
        o_ord = np.lexsort((op, sel[oc_local]))
        same = bool(np.array_equal(gp, op[o_ord]) and np.array_equal(gc, sel[oc_local][o_ord]))
        fo = oracle.pair_fractions(p.xyz, p.h, sub, op, oc_local)[o_ord] if same else None
        ocell = {"cells": int(sel.size), "pairs": int(op.size), "pair_sets_equal": same}
        if same:
            idx = np.searchsorted(sel, gc)
            raw_g = np.bincount(idx, weights=p.m[gp] * gf, minlength=sel.size)
            raw_o = np.bincount(idx, weights=p.m[gp] * fo, minlength=sel.size)
            Sg = S.cpu().numpy()
            Mo = np.bincount(idx, weights=p.m[gp] * fo / Sg[gp], minlength=sel.size)
            ocell.update(max_abs_pair_frac_err=float(np.abs(gf - fo).max()),
                         max_rel_raw_cell_sum=float((np.abs(raw_g - raw_o) / raw_o).max()),
                         max_rel_cell_mass=float((np.abs(M.cpu().numpy()[sel] - Mo) / Mo).max()))
            psel = np.sort(rng.choice(p.n, 8000, replace=False))
            print(f"bench: large oracle sample: S_a of {psel.size} particles", file=sys.stderr, flush=True)
            qp, qc = oracle.pairs(p.xyz[psel], p.h[psel], cells)
            fq = oracle.pair_fractions(p.xyz[psel], p.h[psel], cells, qp, qc)
            So = np.bincount(qp, weights=fq, minlength=psel.size)
            plut = torch.zeros(p.n, dtype=torch.bool, device=dev)
            plut[t(psel)] = True
            ocell["S_sample"] = {"particles": int(psel.size), "pairs": int(qp.size),
                                 "pair_counts_equal": int(plut[PP.long()].sum()) == int(qp.size),
                                 "max_abs_S_err": float(np.abs(Sg[psel] - So).max())}
        ocell["oracle_s"] = time.perf_counter() - t0
        res["oracle_sample"] = ocell
        del F, PP, PC, S, lut, mask
        print(f"bench: large oracle sample: {ocell}", file=sys.stderr, flush=True)
    # pseudo variant
    n = p.n
    out = dict(xyz=torch.zeros((n, 3), dtype=torch.float64, device=dev),
               m=torch.zeros(n, dtype=torch.float64, device=dev), h=torch.zeros(n, dtype=torch.float64, device=dev),
               size=torch.zeros(n, dtype=torch.float64, device=dev),
               kind=torch.zeros(n, dtype=torch.int32, device=dev), ref=torch.zeros(n, dtype=torch.int64, device=dev))
    par = dict(theta=0.5, r_part=0.05, r_leaf=0.1, leaf_size=8, h_fact_node=1.1)
    em.map_pseudo(mp.ctx, xyz, m, h, synth.BOX, LARGE_SOURCES, out=out, **par)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = em.map_pseudo(mp.ctx, xyz, m, h, synth.BOX, LARGE_SOURCES, out=out, **par)
    torch.cuda.synchronize()
    ms_front = 1e3 * (time.perf_counter() - t0)
    qx, qm, qh = r["xyz"].contiguous(), r["m"].contiguous(), r["h"].contiguous()
    Gq = em.map_voronoi(mp.ctx, qx, synth.BOX, 0, device=True)
    mp.set_precision(em.MAP_MIXED)
    Mq = torch.zeros(Gq.n_cells, dtype=torch.float64, device=dev)
    em.map_particles(mp.ctx, qx, qm, qh, Gq, Mq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stq = em.map_particles(mp.ctx, qx, qm, qh, Gq, Mq)
    torch.cuda.synchronize()
    dq = time.perf_counter() - t0
    ps = {"sources": LARGE_SOURCES, "pseudo": int(qm.shape[0]), "pseudo_nodes": r["stats"]["n_pseudo_nodes"],
          "ms_front_end": ms_front, "ms_voronoi": Gq.ms, "pairs": stq["n_pairs"], "ms_map": 1e3 * dq,
          "pairs_per_s": stq["n_pairs"] / dq, "mass_rel_err": abs(stq["mass_out"] - stq["mass_in"]) / stq["mass_in"]}
    if with_oracle:
        print(f"bench: large pseudo variant: oracle over {stq['n_pairs']} pairs", file=sys.stderr, flush=True)
        q = synth.Particles(qx.cpu().numpy(), qm.cpu().numpy(), qh.cpu().numpy())
        O = oracle.map_particles(q, synth.cells_from(Gq))
        ps["oracle_all_cells"] = {"pairs_equal_count": int(O["pair_p"].size) == int(stq["n_pairs"]),
                                  "max_cell_rel": float((np.abs(Mq.cpu().numpy() - O["M"]) / O["M"]).max())}
    res["pseudo_variant"] = ps
    del out, r
    mp.close()
    return res


def adaptive_leg(em, mp, xyz, m, h, src, par):
    """Adaptive walk (Sec. III-B, Eq. (6), K = 100) on the same cloud, driven by an ionised sphere (radius
    0.15, linear rise to neutral over 0.05) standing in for the radiative transfer: a first step from no
    regions, then a second step with the regions and radii it left."""
    import synth
    field = lambda P: synth.ionised_spheres(P["xyz"], src, 0.15, 0.05)
    mp.regions = np.zeros((0, 5))
    em.map_pseudo_adaptive(mp.ctx, xyz, m, h, synth.BOX, src, field, K=100.0, **par)  # warm-up
    mp.regions = np.zeros((0, 5))
    r1 = em.map_pseudo_adaptive(mp.ctx, xyz, m, h, synth.BOX, src, field, K=100.0, **par)
    a1 = r1["adapt"]
    par2 = dict(par, r_part=a1["r_part"], r_leaf=a1["r_leaf"])
    r2 = em.map_pseudo_adaptive(mp.ctx, xyz, m, h, synth.BOX, src, field, K=100.0, **par2)
    a2 = r2["adapt"]
    keys = ("n_walks", "converged", "n_failed", "n_r_part_growths", "n_regions_in", "n_regions_dropped",
            "n_regions_out", "r_part", "r_leaf", "ms_tree", "ms_walks", "ms_callback", "ms_total")
    one = lambda r, a: dict({k: a[k] for k in keys}, pseudo=int(r["m"].size),
                            ms_per_walk=a["ms_walks"] / max(a["n_walks"], 1),
                            last_walk={k: r["stats"][k] for k in ("n_pseudo_nodes", "n_h_evals")})
    return {"field": "ionised sphere r 0.15 + 0.05 ramp at the source; K 100",
            "step1": one(r1, a1), "step2_with_regions": one(r2, a2)}


def table_leg(em, mapper, p, xyz, m, h, dc, M, rho, S, M_fp64, steps, warmup):
    """The tabulated variant (MAP_TABLE) on the same workload at two table sizes: throughput, and its
    error against the FP64 closed form (cell masses, interior S_a)."""
    import torch
    interior = np.all((p.xyz > 2 * p.h[:, None]) & (p.xyz < 1 - 2 * p.h[:, None]), axis=1)
    mapper.set_precision(em.MAP_TABLE)
    out = {}
    for n in (64, 128):
        em.map_set_table(mapper.ctx, n, n, n)
        for _ in range(max(warmup, 1)):  # the first call builds the table
            em.map_particles(mapper.ctx, xyz, m, h, dc, M, rho, S)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            stats.append(em.map_particles(mapper.ctx, xyz, m, h, dc, M, rho, S))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rel = np.abs(M.cpu().numpy() - M_fp64) / np.abs(M_fp64)
        s_dev = np.abs(S.cpu().numpy()[interior] - 1.0)
        out[f"{n}^3"] = {"pairs_per_s": stats[-1]["n_pairs"] / dt, "ms_per_step": 1e3 * dt,
                         "ms_integrate": float(np.mean([s["ms_integrate"] for s in stats])),
                         "cell_rel_err_vs_fp64_max": float(rel.max()), "cell_rel_err_vs_fp64_mean": float(rel.mean()),
                         "interior_abs_S_minus_1_max": float(s_dev.max()),
                         "interior_abs_S_minus_1_mean": float(s_dev.mean())}
    em.map_set_table(mapper.ctx, 64, 64, 64)
    mapper.set_precision(em.MAP_FP64)
    return out


def voronoi_leg(em, mapper, p, xyz, m, h, c, M_fp64, steps, with_oracle):
    """The box-clipped Voronoi grid of the same 262,144 sites on the device (no Lloyd step, then 5), the
    FP64 mapping on those cells against the mapping on the host-generated cells, and the oracle's
    per-cell time on a sample of cells."""
    import torch
    import oracle
    import synth
    sites = torch.from_numpy(np.ascontiguousarray(p.xyz)).to("cuda:0")
    out = {}
    for it in (0, 5):
        em.map_voronoi(mapper.ctx, sites, synth.BOX, it, device=True)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            G = em.map_voronoi(mapper.ctx, sites, synth.BOX, it, device=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[f"lloyd_{it}"] = {"ms": 1e3 * dt, "ms_device": G.ms, "cells_per_s": p.n / dt}
    out["merge_lloyd_5"] = merge_timing(em, mapper.ctx, sites, p.n)
    G = em.map_voronoi(mapper.ctx, sites, synth.BOX, 0, device=True)
    mapper.set_precision(em.MAP_FP64)
    M = torch.zeros(p.n, dtype=torch.float64, device="cuda:0")
    em.map_particles(mapper.ctx, xyz, m, h, G, M)
    rel = np.abs(M.cpu().numpy() - M_fp64) / np.abs(M_fp64)
    out["faces_per_cell"] = float(G.face_plane.shape[0]) / p.n
    out["mapping_on_device_cells_vs_host_cells_max_rel"] = float(rel.max())
    if with_oracle:
        sel = np.arange(0, p.n, p.n // 16)
        t0 = time.perf_counter()
        oracle.voronoi(p.xyz, synth.BOX, sel=sel)
        dt = time.perf_counter() - t0
        out["oracle"] = {"cells_per_s": sel.size / dt, "sample": f"{sel.size} cells (each sorts all sites by "
                         f"distance, then clips nearest first)", "cores": 1}
    return out


def back_leg(em, mapper, p, M, nc, steps):
    """Inverse mapping (Eq. (4)) with the pairs of the last (mixed) mapping: a
    random cell field gathered to the particles, device buffers."""
    import torch

    dev = torch.device("cuda:0")
    q = torch.rand(nc, dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(7))
    out = torch.zeros(p.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    em.map_back(mapper.ctx, q, out)  # builds the particle-major view of the pairs
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(steps):
        em.map_back(mapper.ctx, q, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    mq = float(torch.dot(torch.from_numpy(p.m).to(dev), out))
    mref = float(torch.dot(q, M))
    return {"ms_first_call": 1e3 * first, "ms": 1e3 * dt, "mass_rel_err": abs(mq - mref) / abs(mref)}


def valu_calibration():
    """The calibration kernel (16 independent FP32 FMA chains per lane, 8 workgroups of 256 per CU): its
    FLOP rate is the measured non-packed FP32 vector rate of the device."""
    import ctypes
    from paper_2404_17084_amd import build as hipbuild

    lib = ctypes.CDLL(hipbuild.CALIB_LIB)
    ms = ctypes.c_double()
    fma = ctypes.c_double()
    blocks, iters = 256 * 8, 20000
    rc = lib.em_calib_valu(0, blocks, iters, 5, ctypes.byref(ms), ctypes.byref(fma))
    assert rc == 0, rc
    tf = 2.0 * fma.value / (ms.value * 1e-3) / 1e12
    return {"kernel": "k_valu_fma", "workgroups": blocks, "iterations": iters, "ms_per_launch": ms.value,
            "fma_per_launch": fma.value, "valu_instructions_per_launch": fma.value / 64.0,
            "tflops_fp32_nonpacked": tf, "frac_of_157_3": tf / PEAK_FP32}


def copy_calibration():
    """One plain 1 GiB device-to-device copy: the known byte count that scales the HBM byte counters
    (FETCH_SIZE, WRITE_SIZE) of a profiled run."""
    import torch

    src_t = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst_t = torch.empty_like(src_t)
    torch.cuda.synchronize()
    dst_t.copy_(src_t)
    torch.cuda.synchronize()
    return 1 << 30


def merge_timing(em, ctx, sites, n):
    """The grid with merging and 5 Lloyd steps: sites closer than 1 % of the mean spacing to a site of
    lower index merged (the paper gives no merge criterion)."""
    import torch
    import synth

    d = 0.01 / n ** (1.0 / 3.0)
    em.map_voronoi(ctx, sites, synth.BOX, 5, merge_dist=d, device=True)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = em.map_voronoi(ctx, sites, synth.BOX, 5, merge_dist=d, device=True)
    torch.cuda.synchronize()
    return {"merge_dist": d, "cells": int(G.n_cells), "merged": int(n - G.n_cells),
            "ms": 1e3 * (time.perf_counter() - t0), "ms_device": G.ms}


def voronoi_only(em, args):
    """The device Voronoi grid alone (profiling mode): timings of the 262,144-site build."""
    import torch
    import synth

    p = synth.particles(*synth.CLUMPS_256K)
    sites = torch.from_numpy(np.ascontiguousarray(p.xyz)).to("cuda:0")
    out = {}
    with em.Mapper(device=0) as mp:
        G = em.map_voronoi(mp.ctx, sites, synth.BOX, 0, device=True)  # warm-up
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            G = em.map_voronoi(mp.ctx, sites, synth.BOX, 0, device=True)
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
        out["lloyd_0"] = {"ms": float(np.mean(ms)), "ms_device": G.ms, "faces": int(G.face_plane.shape[0])}
        t0 = time.perf_counter()
        G = em.map_voronoi(mp.ctx, sites, synth.BOX, 5, device=True)
        torch.cuda.synchronize()
        out["lloyd_5"] = {"ms": 1e3 * (time.perf_counter() - t0), "ms_device": G.ms,
                          "faces": int(G.face_plane.shape[0])}
        out["merge_lloyd_5"] = merge_timing(em, mp.ctx, sites, p.n)
    line = {"voronoi_grid": out, "sites": p.n, "steps": args.steps}
    if args.copy_calibration:
        line["copy_calibration_bytes"] = copy_calibration()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-pseudo", action="store_true", help="skip the pseudo-particle leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-mapping leg")
    ap.add_argument("--no-large", action="store_true", help="skip the 8,388,608-particle job")
    ap.add_argument("--oracle-full", action="store_true",
                    help="also run the oracle over the whole 262,144-particle workload (about 80 s on 16 cores) and "
                         "compare every cell of both precisions with it")
    ap.add_argument("--quick", action="store_true",
                    help="only the FP64 and mixed steps of the main workload (for profiling runs)")
    ap.add_argument("--mixed-shape", default=None,
                    help="explicit mixed launch shape 'waves,tile_waves,grid_per_cu,distribution' instead of tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with one plain 1 GiB device-to-device copy (scale for HBM byte counters)")
    ap.add_argument("--valu-calibration", action="store_true",
                    help="run the VALU calibration kernel (scale for the VALU counters; measured FP32 rate)")
    ap.add_argument("--voronoi-only", action="store_true",
                    help="only build the device Voronoi grid of the 262,144 clumpy sites (1 warm-up, then --steps "
                         "builds, then one with 5 Lloyd iterations, then one with merging and 5 Lloyd iterations) "
                         "and print its timings (for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the mapping runs on a single "
              f"MI355X; see the sharding design for several GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2404_17084_amd as em

    em.load()
    if args.voronoi_only:
        voronoi_only(em, args)
        return
    print("bench: generating the 262,144-particle clumpy workload", file=sys.stderr, flush=True)
    p, c = synth.workload(*synth.CLUMPS_256K)
    xyz, m, h, dc = to_device(p, c)
    nc = c.n_cells
    M = torch.zeros(nc, dtype=torch.float64, device="cuda:0")
    rho = torch.zeros_like(M)
    S = torch.zeros(p.n, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()

    mapper = em.Mapper(device=0)
    results = {}
    Ms = {}
    tuned = {}
    for prec, name in ((em.MAP_FP64, "fp64"), (em.MAP_MIXED, "mixed")):
        mapper.set_precision(prec)
        if prec == em.MAP_MIXED and args.mixed_shape:
            w, tw, g, d = (int(v) for v in args.mixed_shape.split(","))
            em.map_set_tune(mapper.ctx, prec, w, tw, g, d)
            tuned[name] = {"waves": w, "tile_waves": tw, "grid_per_cu": g, "distribution": d, "ms_integrate": None}
        elif not args.no_tune and not args.quick:
            shape, ms = em.map_autotune(mapper.ctx, xyz, m, h, dc, prec)
            tuned[name] = {"waves": shape[0], "tile_waves": shape[1], "grid_per_cu": shape[2],
                           "distribution": shape[3], "ms_integrate": ms}
            print(f"bench: autotuned {name}: {tuned[name]}", file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            em.map_particles(mapper.ctx, xyz, m, h, dc, M, rho, S)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            stats.append(em.map_particles(mapper.ctx, xyz, m, h, dc, M, rho, S))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = stats[-1]
        npairs = st["n_pairs"]
        ms_int = float(np.mean([s["ms_integrate"] for s in stats]))
        results[name] = {"pairs_per_s": args.steps * npairs / dt, "ms_per_step": 1e3 * dt / args.steps,
                         "ms_integrate": ms_int, "ms_pairs": float(np.mean([s["ms_pairs"] for s in stats])),
                         "ms_fixup": float(np.mean([s["ms_fixup"] for s in stats])),
                         "ms_reduce": float(np.mean([s["ms_reduce"] for s in stats])),
                         "ms_setup": float(np.mean([s["ms_setup"] for s in stats])),
                         "kernel_work_flops": kernel_work_flops(st),
                         "mass_err": abs(st["mass_out"] - st["mass_in"]),
                         "max_abs_S_minus_1": st["max_abs_S_minus_1"], "n_pairs": npairs,
                         "n_fixup_terms": st["n_fixup_terms"], "n_boundary_pairs": st["n_boundary_pairs"],
                         "n_fp64_cells": st["n_fp64_cells"], "n_fp64_pairs": st["n_fp64_pairs"],
                         "n_moment_evals": st["n_moment_evals"], "n_quad_intervals": st["n_quad_intervals"],
                         "n_quad_points": st["n_quad_points"], "n_angle_evals": st["n_angle_evals"],
                         "n_edge_visits": st["n_edge_visits"], "n_candidates": st["n_candidates"]}
        Ms[name] = M.cpu().numpy().copy()
        print(f"bench: {name}: {results[name]}", file=sys.stderr, flush=True)
    rel = np.abs(Ms["mixed"] - Ms["fp64"]) / np.abs(Ms["fp64"])
    extra = {}
    if args.oracle_full:
        import oracle

        print("bench: the oracle over the whole workload", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        O = oracle.map_particles(p, c)
        dt = time.perf_counter() - t0
        extra["oracle_full"] = {
            "pairs": int(O["pair_p"].size), "pairs_equal_count": int(O["pair_p"].size) == results["mixed"]["n_pairs"],
            "seconds": dt, "pairs_per_s": O["pair_p"].size / dt, "cores": oracle.num_threads(),
            "max_cell_rel_mixed": float((np.abs(Ms["mixed"] - O["M"]) / O["M"]).max()),
            "max_cell_rel_fp64": float((np.abs(Ms["fp64"] - O["M"]) / O["M"]).max()),
            "mass_rel_err_oracle": float(abs(O["M"].sum() - p.m.sum()) / p.m.sum())}
        print(f"bench: oracle over the whole workload: {extra['oracle_full']}", file=sys.stderr, flush=True)
    if not args.quick:
        extra["inverse_mapping"] = back_leg(em, mapper, p, M, nc, args.steps)
        print(f"bench: inverse mapping: {extra['inverse_mapping']}", file=sys.stderr, flush=True)
        extra["tabulated"] = table_leg(em, mapper, p, xyz, m, h, dc, M, rho, S, Ms["fp64"], args.steps, args.warmup)
        print(f"bench: tabulated variant: {extra['tabulated']}", file=sys.stderr, flush=True)
        extra["voronoi_grid"] = voronoi_leg(em, mapper, p, xyz, m, h, c, Ms["fp64"], args.steps,
                                            not args.no_cpu_baseline)
        print(f"bench: voronoi grid: {extra['voronoi_grid']}", file=sys.stderr, flush=True)
    mapper.close()
    if not args.quick and not args.no_serve:
        extra["served"] = serve_leg(em)
        print(f"bench: served: {extra['served']}", file=sys.stderr, flush=True)
    if not args.quick and not args.no_pseudo:
        extra["pseudo_path"] = pseudo_leg(em, args.steps, args.warmup)
        print(f"bench: pseudo path: {extra['pseudo_path']}", file=sys.stderr, flush=True)
    if not args.quick and not args.no_large:
        extra["large_job"] = large_leg(em, 2, not args.no_cpu_baseline)
        print(f"bench: large job: {extra['large_job']}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline and not args.quick:
        print("bench: timing the oracle on a cell sample", file=sys.stderr, flush=True)
        cpu, model = cpu_baseline(p, c)
    else:
        model = flop_model_only(p, c)
    if args.valu_calibration:
        extra["valu_calibration"] = valu_calibration()
        print(f"bench: valu calibration: {extra['valu_calibration']}", file=sys.stderr, flush=True)

    mx, fp = results["mixed"], results["fp64"]
    model_flops = model["flops_per_pair"] * mx["n_pairs"]
    ach = model_flops / (mx["ms_integrate"] * 1e-3) / 1e12
    ach64 = model_flops / (fp["ms_integrate"] * 1e-3) / 1e12
    valid = counters_valid()
    line = {
        "metric": "particle-cell pairs mapped/s (mixed FP32/FP64, <=1e-5 rel err per cell)",
        "value": mx["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 terms, f64 geometry/sums",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "particles": p.n, "cells": nc, "pairs": mx["n_pairs"], "precision": "mixed"},
        "fp64": {"pairs_per_s": fp["pairs_per_s"], "ms_per_step": fp["ms_per_step"],
                 "ms_integrate": fp["ms_integrate"], "model_tflops_integrate": ach64,
                 "roofline_frac": ach64 / PEAK_FP64},
        "speedup_mixed_vs_fp64": mx["pairs_per_s"] / fp["pairs_per_s"],
        "mixed_vs_fp64_max_cell_rel": float(rel.max()),
        "mixed_vs_fp64_mean_cell_rel": float(rel.mean()),
        "mass_err_mixed": mx["mass_err"],
        "mixed_fp64_work": {k: mx[k] for k in ("n_fixup_terms", "n_boundary_pairs", "n_fp64_cells", "n_fp64_pairs")},
        "stages_ms_mixed": {k: mx[k] for k in ("ms_setup", "ms_pairs", "ms_integrate", "ms_fixup", "ms_reduce")},
        "stages_ms_fp64": {k: fp[k] for k in ("ms_setup", "ms_pairs", "ms_integrate", "ms_fixup", "ms_reduce")},
        "flop_model": dict(model, source="static count of the oracle's direct-form formulas (orc_flop_model) "
                                         "over a seeded sample of cells"),
        "kernel_work_tflops_integrate": mx["kernel_work_flops"] / (mx["ms_integrate"] * 1e-3) / 1e12,
        "launch_shape": tuned,
        "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP32, "unit": "TFLOP/s", "frac": ach / PEAK_FP32,
                     "traffic": TRAFFIC_BYTES if valid else None,
                     "measured_valu_tflops": (VALU_FLOPS_PER_LAUNCH / (mx["ms_integrate"] * 1e-3) / 1e12
                                              if valid and VALU_FLOPS_PER_LAUNCH else None)},
    }
    line.update(extra)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    if args.copy_calibration:
        line["copy_calibration_bytes"] = copy_calibration()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
