"""Served mapping (map_submit / map_poll) through the C ABI.

A served job is integrated by the same task-batch kernel as a synchronous
map_particles call with the default launch shape, over a table of the jobs in
the launch, so its results must equal the synchronous ones bit for bit, alone
or in any mix; the synchronous path itself is checked against the oracle in
test_gpu_parity.py, and here once more directly.  Admission must respect the
device-memory budget, a failing job must not disturb the others, device inputs
are borrowed until the job finishes.  Every context runs with a job time limit
and a per-job trace on stderr, and every poll is bounded.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2404_17084_amd as em

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(120)]

POLL_US = 60_000_000  # bounded waits: a stuck job fails the test instead of blocking it
LIMIT_MS = 30_000


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mapper(**kw):
    return em.Mapper(device=0, serve_timeout_ms=LIMIT_MS, serve_trace=True, **kw)


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


@pytest.mark.parametrize("prec,tol", [(em.MAP_FP64, 1e-10), (em.MAP_MIXED, 1e-5)])
def test_served_matches_synchronous_and_oracle(jobs, prec, tol):
    say(f"case: served vs synchronous vs oracle, precision {prec}")
    with mapper(precision=prec, max_jobs=3) as mp:
        outs, stats = _serve(mp, jobs)
        for (p, c), (M, rho, S), st in zip(jobs, outs, stats):
            ref = mp.map(p, c)
            assert np.array_equal(M, ref["M"]) and np.array_equal(rho, ref["rho"]) and np.array_equal(S, ref["S"])
            assert st["n_pairs"] == ref["stats"]["n_pairs"]
            assert st["n_fixup_terms"] == ref["stats"]["n_fixup_terms"]
            assert abs(M.sum() - p.m.sum()) < 1e-9
            assert st["ms_latency"] >= st["ms_queue"] >= 0.0
        # the oracle on two of the jobs
        for k in (1, 2):
            p, c = jobs[k]
            o = oracle.map_particles(p, c)
            assert (np.abs(outs[k][0] - o["M"]) / o["M"]).max() < tol


def test_alone_and_in_mix_bitwise(jobs):
    say("case: alone vs in the mix")
    with mapper(precision=em.MAP_MIXED, max_jobs=4) as mp:
        alone = [_serve(mp, [j])[0][0] for j in jobs]
        mixed, _ = _serve(mp, jobs)
        for a, b in zip(alone, mixed):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_mixed_precisions_in_one_context(jobs):
    say("case: FP64 and mixed jobs interleaved")
    with mapper(precision=em.MAP_FP64, max_jobs=4) as mp:
        ids = []
        for k, (p, c) in enumerate(jobs):
            mp.set_precision(em.MAP_FP64 if k % 2 == 0 else em.MAP_MIXED)
            M = np.zeros(c.n_cells)
            ids.append((em.map_submit(mp.ctx, p.xyz, p.m, p.h, c, M), M, k))
        for jid, M, k in ids:
            state, _ = em.map_poll(mp.ctx, jid, POLL_US)
            assert state == em.JOB_DONE
            mp.set_precision(em.MAP_FP64 if k % 2 == 0 else em.MAP_MIXED)
            assert np.array_equal(M, mp.map(*jobs[k])["M"])


def test_budget_admission_and_enomem(jobs):
    say("case: admission by budget")
    p, c = jobs[4]
    # a budget that holds about one of these jobs at a time
    with mapper(precision=em.MAP_MIXED, max_jobs=8, hbm_budget_bytes=70_000_000) as mp:
        outs, stats = _serve(mp, jobs)
        assert all(st["ms_latency"] > 0 for st in stats)
        for (p, c), (M, _, _) in zip(jobs, outs):
            assert abs(M.sum() - p.m.sum()) < 1e-9
        big = synth.workload("uniform", 20000, 37)
        with pytest.raises(em.MapError) as ei:
            em.map_submit(mp.ctx, big[0].xyz, big[0].m, big[0].h, big[1])
        assert ei.value.code == em.MAP_ENOMEM


def test_failed_job_is_isolated(jobs):
    say("case: failure isolation")
    with mapper(precision=em.MAP_FP64, max_jobs=2) as mp:
        good = []
        for p, c in jobs[:3]:
            M = np.zeros(c.n_cells)
            good.append((em.map_submit(mp.ctx, p.xyz, p.m, p.h, c, M), M, p, c))
        p, c = jobs[3]
        # a zero cell volume passes the host checks and fails on the device
        vol = c.cell_volume.copy()
        vol[3] = 0.0
        badc = synth.Cells(c.cell_face_off, c.face_vert_off, c.face_vert, c.face_plane, c.face_nb, c.verts, vol, c.box)
        bad = em.map_submit(mp.ctx, p.xyz, p.m, p.h, badc, np.zeros(c.n_cells))
        with pytest.raises(em.MapError) as ei:
            em.map_poll(mp.ctx, bad, POLL_US)
        assert ei.value.code == em.MAP_EGEOM
        for jid, M, pp, cc in good:
            state, _ = em.map_poll(mp.ctx, jid, POLL_US)
            assert state == em.JOB_DONE
            assert np.array_equal(M, mp.map(pp, cc)["M"])
        with pytest.raises(em.MapError) as ei:
            em.map_poll(mp.ctx, bad, 0)
        assert ei.value.code == em.MAP_ENOTFOUND


def test_device_inputs_and_outputs(jobs):
    import torch
    say("case: served device buffers")
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    class DC:
        pass

    with mapper(precision=em.MAP_MIXED, max_jobs=3) as mp:
        ids = []
        for p, c in jobs[:4]:
            dc = DC()
            dc.cell_face_off, dc.face_vert_off = t(c.cell_face_off), t(c.face_vert_off)
            dc.face_vert, dc.face_plane, dc.verts = t(c.face_vert), t(c.face_plane), t(c.verts)
            dc.cell_volume, dc.box = t(c.cell_volume), c.box
            M = torch.zeros(c.n_cells, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            ids.append((em.map_submit(mp.ctx, t(p.xyz), t(p.m), t(p.h), dc, M), M, p, c))
        for jid, M, p, c in ids:
            state, _ = em.map_poll(mp.ctx, jid, POLL_US)
            assert state == em.JOB_DONE
            assert np.array_equal(M.cpu().numpy(), mp.map(p, c)["M"])


def test_empty_job_and_zero_timeout_poll(jobs):
    say("case: empty job, zero-timeout poll")
    p, c = jobs[0]
    with mapper(precision=em.MAP_MIXED, max_jobs=2) as mp:
        M = np.zeros(c.n_cells)
        jid = em.map_submit(mp.ctx, p.xyz[:0], p.m[:0], p.h[:0], c, M)
        state, st = em.map_poll(mp.ctx, jid, POLL_US)
        assert state == em.JOB_DONE and st["n_pairs"] == 0 and not M.any()
        jid = em.map_submit(mp.ctx, p.xyz, p.m, p.h, c, M)
        state, _ = em.map_poll(mp.ctx, jid, 0)
        assert state in (em.JOB_PENDING, em.JOB_RUNNING, em.JOB_DONE)
        if state != em.JOB_DONE:
            state, _ = em.map_poll(mp.ctx, jid, POLL_US)
        assert state == em.JOB_DONE
