"""Served mapping (map_submit / map_poll) through the C ABI.

Each served result must match the synchronous path (and hence the oracle) and be
bitwise the same whether the job runs alone or batched with other jobs; admission
must respect the device-memory budget; a failing job must not disturb the others.
"""
import sys

import numpy as np
import pytest

import synth
import paper_2404_17084_amd as em

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.timeout(90),
    pytest.mark.skip(reason="served mapping is switched off (map_submit returns MAP_ENOTSUP): a device run of "
                            "test_served_matches_synchronous stopped making progress and its cause is not found"),
]

POLL_US = 60_000_000  # bounded waits: a stuck job fails the test instead of blocking it


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def jobs():
    specs = [("uniform", 900, 31), ("clumps", 1500, 32), ("uniform", 2500, 33), ("clumps", 700, 34),
             ("clumps", 3000, 35), ("uniform", 1200, 36)]
    return [synth.workload(*s) for s in specs]


def _serve(mp, batch):
    ids = []
    outs = []
    for p, c in batch:
        M = np.zeros(c.n_cells)
        rho = np.zeros(c.n_cells)
        S = np.zeros(p.n)
        ids.append(em.map_submit(mp.ctx, p.xyz, p.m, p.h, c, M, rho, S))
        outs.append((M, rho, S))
    stats = []
    for jid in ids:
        state, st = em.map_poll(mp.ctx, jid, POLL_US)
        assert state == em.JOB_DONE
        stats.append(st)
    return outs, stats


@pytest.mark.parametrize("prec,tol", [(em.MAP_FP64, 1e-12), (em.MAP_MIXED, 1e-5)])
def test_served_matches_synchronous(jobs, prec, tol):
    say(f"case: served vs synchronous, precision {prec}")
    with em.Mapper(device=0, precision=prec, max_jobs=3) as mp:
        outs, stats = _serve(mp, jobs)
        for (p, c), (M, rho, S), st in zip(jobs, outs, stats):
            ref = mp.map(p, c)
            assert (np.abs(M - ref["M"]) / ref["M"]).max() < tol
            assert abs(M.sum() - p.m.sum()) < 1e-9
            assert st["n_pairs"] == ref["stats"]["n_pairs"]
            assert st["ms_latency"] >= st["ms_queue"] >= 0.0


def test_alone_and_in_mix_bitwise(jobs):
    say("case: alone vs in the mix")
    with em.Mapper(device=0, precision=em.MAP_MIXED, max_jobs=4) as mp:
        alone = [_serve(mp, [j])[0][0] for j in jobs]
        mixed, _ = _serve(mp, jobs)
        for a, b in zip(alone, mixed):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_budget_admission_and_enomem(jobs):
    say("case: admission by budget")
    p, c = jobs[4]
    # a budget that holds about one of these jobs at a time
    with em.Mapper(device=0, precision=em.MAP_MIXED, max_jobs=8, hbm_budget_bytes=70_000_000) as mp:
        outs, stats = _serve(mp, jobs)
        assert all(st["ms_latency"] > 0 for st in stats)
        big = synth.workload("uniform", 20000, 37)
        with pytest.raises(em.MapError) as ei:
            em.map_submit(mp.ctx, big[0].xyz, big[0].m, big[0].h, big[1])
        assert ei.value.code == em.MAP_ENOMEM


def test_failed_job_is_isolated(jobs):
    say("case: failure isolation")
    with em.Mapper(device=0, precision=em.MAP_FP64, max_jobs=2) as mp:
        good = []
        for p, c in jobs[:3]:
            M = np.zeros(c.n_cells)
            good.append((em.map_submit(mp.ctx, p.xyz, p.m, p.h, c, M), M, p))
        p, c = jobs[3]
        # a zero cell volume passes the host checks and fails on the device
        vol = c.cell_volume.copy()
        vol[3] = 0.0
        badc = synth.Cells(c.cell_face_off, c.face_vert_off, c.face_vert, c.face_plane, c.face_nb, c.verts, vol, c.box)
        bad = em.map_submit(mp.ctx, p.xyz, p.m, p.h, badc, np.zeros(c.n_cells))
        with pytest.raises(em.MapError) as ei:
            em.map_poll(mp.ctx, bad, POLL_US)
        assert ei.value.code == em.MAP_EGEOM
        for jid, M, pp in good:
            state, _ = em.map_poll(mp.ctx, jid, POLL_US)
            assert state == em.JOB_DONE
            assert abs(M.sum() - pp.m.sum()) < 1e-12
        with pytest.raises(em.MapError) as ei:
            em.map_poll(mp.ctx, bad, 0)
        assert ei.value.code == em.MAP_ENOTFOUND


def test_device_inputs_and_outputs(jobs):
    import torch
    say("case: served device buffers")
    p, c = jobs[2]
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    class DC:
        pass

    dc = DC()
    dc.cell_face_off, dc.face_vert_off = t(c.cell_face_off), t(c.face_vert_off)
    dc.face_vert, dc.face_plane, dc.verts = t(c.face_vert), t(c.face_plane), t(c.verts)
    dc.cell_volume, dc.box = t(c.cell_volume), c.box
    M = torch.zeros(c.n_cells, dtype=torch.float64, device=dev)
    with em.Mapper(device=0, precision=em.MAP_FP64) as mp:
        jid = em.map_submit(mp.ctx, t(p.xyz), t(p.m), t(p.h), dc, M)
        state, _ = em.map_poll(mp.ctx, jid, POLL_US)
        assert state == em.JOB_DONE
        ref = mp.map(p, c)
        assert np.abs(M.cpu().numpy() - ref["M"]).max() < 1e-15
