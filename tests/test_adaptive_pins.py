"""Pins of the oracle's adaptive re-walk (paper Sec. III-B, Eq. (6)) and remembered regions.

Checked without the oracle's own code path: Eq. (6) at its special sizes
(a fully ionised node passes exactly when s <= s_root / K; the root's limit
is 1 - 1/K), the converged set re-tested in the multiplied-out form
f K s >= K s - s_root, mass conservation and the particle partition by cube
containment decoded from labels, a forced opening that changes only the
forced node's subtree, regions that open overlapping nodes down to s_min,
a failing leaf that makes r_part grow until its particles come out, the
smallest descendant size of each new region from the tree's particle ranges,
and the two behaviours the paper names for regions across steps: the next
step needs no re-walk, and shielded (neutral) regions are dropped.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_pseudo_pins import _members

BOX = np.array(synth.BOX, dtype=np.float64)
SRC = [[0.5, 0.5, 0.5]]
K = 100.0


def _sphere(radius=0.15, width=0.05, centres=SRC):
    return lambda P: synth.ionised_spheres(P["xyz"], centres, radius, width)


@pytest.fixture(scope="module")
def cloud():
    return synth.particles("clumps", 12000, 71)


def _fake_set(kind, s, s_root):
    return dict(kind=np.asarray(kind, np.int32), s=np.asarray(s, np.float64), stats=dict(s_root=s_root))


def test_limit_special_sizes():
    s_root = 0.8
    edge = s_root / K
    P = _fake_set([0, 0, 0, 1, 0, 0], [edge * (1 + 1e-9), edge * (1 - 1e-9), edge, 0.0, 0.0, s_root], s_root)
    f = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 1.0 - 1.0 / K - 1e-9])
    fail = oracle.resolution_check(P, f, K)
    # ionised node just above s_root/K fails, at or below passes; particles and
    # zero-size nodes are never checked; the root needs f >= 1 - 1/K
    assert fail.tolist() == [True, False, False, False, False, True]
    f[5] = 1.0 - 1.0 / K + 1e-9
    assert not oracle.resolution_check(P, f, K)[5]
    # a fully neutral node passes at any size
    P = _fake_set([0] * 4, [1e-6, 0.1, 0.8, 5.0], s_root)
    assert not oracle.resolution_check(P, np.ones(4), K).any()


def test_neutral_field_is_the_plain_walk(cloud):
    p = cloud
    R = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, SRC, lambda P: np.ones(P["m"].size), K=K)
    Q = oracle.pseudo(p.xyz, p.m, p.h, BOX, SRC)
    assert R["walks"] == 1 and R["converged"] and R["regions"].shape == (0, 5)
    for k in ("ref", "kind", "m", "s", "h"):
        assert np.array_equal(R[k], Q[k])


def test_converged_set_passes_and_partitions(cloud):
    p = cloud
    R = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, SRC, _sphere(), K=K)
    assert R["converged"] and R["walks"] >= 2
    node = (R["kind"] == oracle.PSEUDO_NODE) & (R["s"] > 0)
    f = synth.ionised_spheres(R["xyz"], SRC, 0.15, 0.05)
    s, sr = R["s"][node], R["stats"]["s_root"]
    assert np.all(f[node] * K * s >= K * s - sr * (1 + 1e-12))
    assert R["m"].sum() == pytest.approx(p.m.sum(), rel=1e-13)
    count = np.zeros(p.n, dtype=np.int64)
    for t in np.nonzero(R["kind"] == oracle.PSEUDO_NODE)[0]:
        count += _members(p.xyz, R["ref"][t])
    count[R["ref"][R["kind"] == oracle.PSEUDO_PARTICLE]] += 1
    assert np.all(count == 1)


def test_forced_label_changes_only_its_subtree(cloud):
    p = cloud
    Q = oracle.pseudo(p.xyz, p.m, p.h, BOX, SRC)
    cand = np.nonzero((Q["kind"] == oracle.PSEUDO_NODE) & ~Q["leaf"])[0]
    x = cand[np.argmax(Q["m"][cand])]
    lab = int(Q["ref"][x])
    R = oracle.pseudo(p.xyz, p.m, p.h, BOX, SRC, open_labels=[lab])
    inside = _members(p.xyz, lab)
    def within(t):  # the pseudo-particle's particles all lie in the forced node's cube
        if R["kind"][t] == oracle.PSEUDO_PARTICLE:
            return bool(inside[R["ref"][t]])
        mem = _members(p.xyz, R["ref"][t])
        return bool(mem.any() and not (mem & ~inside).any())

    sub = np.array([within(t) for t in range(R["m"].size)])
    assert lab not in set(R["ref"][R["kind"] == oracle.PSEUDO_NODE].tolist())
    assert R["m"][sub].sum() == pytest.approx(Q["m"][x], rel=1e-13)
    keep = np.arange(Q["m"].size) != x
    assert np.array_equal(R["ref"][~sub], Q["ref"][keep]) and np.array_equal(R["kind"][~sub], Q["kind"][keep])


def test_region_opens_overlapping_nodes_down_to_s_min(cloud):
    p = cloud
    Q = oracle.pseudo(p.xyz, p.m, p.h, BOX, SRC)
    c, R0, s_min = np.array([0.2, 0.75, 0.3]), 0.12, 0.004
    R = oracle.pseudo(p.xyz, p.m, p.h, BOX, SRC, regions=[[*c, R0, s_min]])
    assert R["m"].size > Q["m"].size
    T = oracle.tree(p.xyz, p.m, BOX)
    leaf_of = dict(zip(T["label"].tolist(), T["leaf"].tolist()))
    for t in np.nonzero(R["kind"] == oracle.PSEUDO_NODE)[0]:
        d = np.sqrt(((R["xyz"][t] - c) ** 2).sum())
        if d - R["s"][t] < R0:  # comes within the region: a leaf or no larger than s_min
            assert leaf_of[int(R["ref"][t])] or R["s"][t] <= s_min
    assert R["m"].sum() == pytest.approx(p.m.sum(), rel=1e-13)


def test_failing_leaf_grows_r_part(cloud):
    p = cloud
    Q = oracle.pseudo(p.xyz, p.m, p.h, BOX, SRC)
    # an accepted leaf big enough to fail when ionised (s > s_root / K), the farthest from the source
    leaves = np.nonzero(Q["leaf"] & (Q["s"] > 2.0 * Q["stats"]["s_root"] / K))[0]
    r = np.sqrt(((Q["xyz"][leaves] - SRC[0]) ** 2).sum(axis=1)) - Q["s"][leaves]
    t = leaves[np.argmax(r)]
    lab, rt = int(Q["ref"][t]), float(r.max())
    field = _sphere(radius=1e-3, width=1e-3, centres=[Q["xyz"][t]])
    R = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, SRC, field, K=K)
    assert R["converged"] and R["walks"] >= 2
    assert R["r_part"] > rt and R["r_leaf"] / R["r_part"] == pytest.approx(0.1 / 0.05, rel=1e-12)
    extracted = set(R["ref"][R["kind"] == oracle.PSEUDO_PARTICLE].tolist())
    assert set(np.nonzero(_members(p.xyz, lab))[0].tolist()) <= extracted
    assert any(lab in f for f in R["failed"])


def test_new_region_sizes_from_the_tree(cloud):
    p = cloud
    R = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, SRC, _sphere(), K=K)
    T = oracle.tree(p.xyz, p.m, BOX)
    by_label = {int(l): i for i, l in enumerate(T["label"].tolist())}
    labels = [l for walk in R["failed"] for l in walk]
    assert R["regions"].shape == (len(labels), 5)
    nodes = [by_label[int(l)] for l in R["ref"][R["kind"] == oracle.PSEUDO_NODE]]
    sizes = R["s"][R["kind"] == oracle.PSEUDO_NODE]
    for row, lab in zip(R["regions"], labels):
        i = by_label[lab]
        assert np.array_equal(row[:3], T["com"][i]) and row[3] == T["s"][i]
        within = [sizes[k] for k, j in enumerate(nodes) if T["start"][i] <= T["start"][j] and T["end"][j] <= T["end"][i]]
        assert row[4] == (min(within) if within else 0.0)


def test_regions_restore_the_next_step_and_shielded_ones_drop(cloud):
    p = cloud
    R1 = oracle.pseudo_adaptive(p.xyz, p.m, p.h, BOX, SRC, _sphere(), K=K)
    assert R1["walks"] >= 2 and R1["regions"].shape[0] > 0
    # the next step (particles moved a little) starts from the remembered regions
    rng = np.random.default_rng(3)
    xyz2 = np.clip(p.xyz + rng.normal(0.0, 1e-4, p.xyz.shape), 0.0, 1.0 - 1e-12)
    R2 = oracle.pseudo_adaptive(xyz2, p.m, p.h, BOX, SRC, _sphere(), K=K, regions=R1["regions"],
                                r_part=R1["r_part"], r_leaf=R1["r_leaf"])
    assert R2["walks"] == 1 and R2["converged"]
    # shielded: the region turned neutral, so every region is dropped
    R3 = oracle.pseudo_adaptive(xyz2, p.m, p.h, BOX, SRC, lambda P: np.ones(P["m"].size), K=K,
                                regions=R1["regions"], r_part=R1["r_part"], r_leaf=R1["r_leaf"])
    assert R3["walks"] == 1 and R3["dropped"] == R1["regions"].shape[0] and R3["regions"].shape == (0, 5)
