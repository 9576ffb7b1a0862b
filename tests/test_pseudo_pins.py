"""Pins of the pseudo-particle oracle (paper Sec. III) against geometry, brute force and closed forms.

Each check recomputes what the paper fixes without the oracle's own code path:
cube containment decoded from node labels (Morton keys and tree), brute-force
masses, centres of mass and sizes (Sec. III-A), the label arithmetic, mass
conservation of the accepted set, the opening rule Eq. (5) evaluated node by
node, r_part extraction, the smoothing-length relation Eq. (7)-(8) by a
vectorised residual, and a closed-form root on a symmetric shell.
"""
import numpy as np
import pytest

import oracle
import synth

BOX = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
HF = 1.1


def _w(q):
    q = np.asarray(q, dtype=np.float64)
    out = np.zeros_like(q)
    a = q < 1.0
    b = (q >= 1.0) & (q < 2.0)
    out[a] = 1.0 - 1.5 * q[a] ** 2 + 0.75 * q[a] ** 3
    out[b] = 0.25 * (2.0 - q[b]) ** 3
    return out


def _decode(label):
    """(level, cube integer coords) of a node label (1 << 3L | octal prefix)."""
    label = int(label)
    L = (label.bit_length() - 1) // 3
    cx = cy = cz = 0
    for k in range(L - 1, -1, -1):
        d = (label >> (3 * k)) & 7
        cx, cy, cz = 2 * cx + (d >> 2 & 1), 2 * cy + (d >> 1 & 1), 2 * cz + (d & 1)
    return L, np.array([cx, cy, cz])


def _members(xyz, label):
    """Boolean mask of the particles inside the node's cube (the cube of level L, index c)."""
    L, c = _decode(label)
    n = 2 ** L
    # same scaling as the keys: floor(x * 2^21) >> (21 - L), via integer coordinates
    ii = np.clip(np.floor(xyz * 2097152.0), 0, 2097151).astype(np.int64) >> (21 - L)
    return np.all(ii == c[None, :], axis=1) & (n > 0)


@pytest.fixture(scope="module")
def clumpy():
    p, _ = synth.workload("clumps", 3000, 41)
    return p


@pytest.fixture(scope="module")
def uniform():
    rng = np.random.default_rng(42)
    xyz = rng.random((2500, 3))
    return xyz, np.full(2500, 1.0 / 2500), np.full(2500, 0.04)


def test_morton_key_orders_octants():
    # the first octal digit is the octant (x, y, z bits), the key is monotone in each axis within a cell row
    k = oracle.morton([0.75, 0.25, 0.75], BOX)
    assert k >> 60 == 0b101
    assert oracle.morton([0.0, 0.0, 0.0], BOX) == 0
    assert oracle.morton([1.0, 1.0, 1.0], BOX) == (1 << 63) - 1
    xs = np.linspace(0.01, 0.99, 50)
    keys = [oracle.morton([x, 0.3, 0.3], BOX) for x in xs]
    assert all(a <= b for a, b in zip(keys, keys[1:]))


@pytest.mark.parametrize("leaf", [1, 4, 8])
def test_tree_partition_and_labels(clumpy, leaf):
    T = oracle.tree(clumpy.xyz, clumpy.m, BOX, leaf)
    n = clumpy.m.size
    assert np.array_equal(np.sort(T["perm"]), np.arange(n))
    cnt = T["end"] - T["start"]
    lv = T["level"]
    # leaves partition the sorted order
    lf = np.flatnonzero(T["leaf"])
    order = lf[np.argsort(T["start"][lf])]
    assert T["start"][order[0]] == 0 and T["end"][order[-1]] == n
    assert np.array_equal(T["start"][order[1:]], T["end"][order[:-1]])
    assert np.all((cnt[lf] <= leaf) | (lv[lf] == 21))
    assert np.all(cnt[~T["leaf"]] > leaf)
    # label arithmetic: ancestor k levels up = label >> 3k = floor(label / 8^k); level from the sentinel
    lab = T["label"].astype(object)
    for i in range(len(lab)):
        assert (int(lab[i]).bit_length() - 1) // 3 == lv[i]
        j, k = i, 0
        while T["parent"][j] >= 0:
            j = T["parent"][j]
            k += 1
            assert int(lab[j]) == int(lab[i]) // 8 ** k
    # children partition their parent's range
    for i in np.flatnonzero(~T["leaf"]):
        ch = np.flatnonzero(T["parent"] == i)
        ch = ch[np.argsort(T["start"][ch])]
        assert T["start"][ch[0]] == T["start"][i] and T["end"][ch[-1]] == T["end"][i]
        assert np.array_equal(T["start"][ch[1:]], T["end"][ch[:-1]])


def test_node_cubes_and_moments_brute_force(clumpy):
    T = oracle.tree(clumpy.xyz, clumpy.m, BOX, 8)
    xyz, m = clumpy.xyz, clumpy.m
    rng = np.random.default_rng(5)
    sel = np.concatenate([[0], rng.choice(len(T["level"]), 120, replace=False)])
    for i in sel:
        mask = _members(xyz, T["label"][i])
        # the node's particles are exactly those in its cube
        got = np.sort(T["perm"][T["start"][i]:T["end"][i]])
        assert np.array_equal(got, np.flatnonzero(mask))
        M = m[mask].sum()
        com = (m[mask, None] * xyz[mask]).sum(0) / M
        s = np.sqrt(((xyz[mask] - com) ** 2).sum(1)).max()
        # sequential vs pairwise summation: |delta| <= n eps sum|terms| (n <= 3000 here)
        tol = 4 * mask.sum() * 2.2e-16
        assert abs(T["mass"][i] - M) <= tol * M
        assert np.abs(T["com"][i] - com).max() <= tol
        assert abs(T["s"][i] - s) <= tol


def _pseudo_sets(P, T, xyz):
    """Particle sets of the pseudo-particles, via cube containment (not the oracle's ranges)."""
    owner = np.full(xyz.shape[0], -1)
    for t in range(P["m"].size):
        if P["kind"][t] == oracle.PSEUDO_NODE:
            mask = _members(xyz, P["ref"][t])
            assert np.all(owner[mask] == -1)
            owner[mask] = t
        else:
            a = P["ref"][t]
            assert owner[a] == -1
            owner[a] = t
    return owner


@pytest.mark.parametrize("theta,r_part,r_leaf", [(0.5, 0.05, 0.1), (0.3, 0.0, 0.2), (0.8, 0.1, 0.1)])
def test_accepted_set_partitions_and_conserves_mass(clumpy, theta, r_part, r_leaf):
    src = np.array([[0.5, 0.5, 0.5], [0.3, 0.6, 0.45]])
    P = oracle.pseudo(clumpy.xyz, clumpy.m, clumpy.h, BOX, src, theta, r_part, r_leaf)
    T = oracle.tree(clumpy.xyz, clumpy.m, BOX, 8)
    owner = _pseudo_sets(P, T, clumpy.xyz)
    assert np.all(owner >= 0)
    tot = clumpy.m.sum()
    assert abs(P["m"].sum() - tot) <= 1e-12 * tot
    # each pseudo mass is the mass of its particles (summation-order rounding only)
    Mb = np.bincount(owner, weights=clumpy.m, minlength=P["m"].size)
    assert np.abs(Mb - P["m"]).max() <= 1e-12
    # Morton order of first particles
    first = np.array([np.flatnonzero(owner == t).min() for t in range(P["m"].size)])
    key = np.array([oracle.morton(clumpy.xyz[a], BOX) for a in first], dtype=np.uint64)
    assert np.all(np.diff(key.astype(np.float64)) >= 0)


def test_theta_limits(uniform):
    xyz, m, h = uniform
    T = oracle.tree(xyz, m, BOX, 8)
    # theta = 0, no radii and the source outside every node's ball: every internal node
    # opens (s > 0 = theta r), no leaf is within r_part, so the pseudo set is the leaves
    P = oracle.pseudo(xyz, m, h, BOX, [[3.0, -2.0, 0.5]], 0.0, 0.0, 0.0)
    assert np.all(P["kind"] == oracle.PSEUDO_NODE)
    assert np.array_equal(np.sort(P["ref"].astype(np.uint64)), np.sort(T["label"][T["leaf"]]))
    # huge theta, source far away: nothing opens
    P = oracle.pseudo(xyz, m, h, BOX, [[10.0, 10.0, 10.0]], 1e9, 0.0, 0.0)
    assert P["m"].size == 1 and P["ref"][0] == 1 and abs(P["m"][0] - m.sum()) < 1e-12


def test_walk_rule_node_by_node(clumpy):
    """Accepted = every ancestor opened and the node not opened, with Eq. (5) and the radii, per node."""
    theta, rp, rl = 0.5, 0.05, 0.12
    src = np.array([[0.45, 0.5, 0.55], [0.7, 0.3, 0.4]])
    T = oracle.tree(clumpy.xyz, clumpy.m, BOX, 8)
    P = oracle.pseudo(clumpy.xyz, clumpy.m, clumpy.h, BOX, src, theta, rp, rl)
    r = np.sqrt(((T["com"][:, None, :] - src[None, :, :]) ** 2).sum(2)).min(1)
    s = T["s"]
    part = r - s < rp
    opened = np.where(T["leaf"], part, part | (r - s < rl) | (s > theta * r))
    vis = np.zeros(len(s), bool)
    for i in np.argsort(T["level"], kind="stable"):
        p = T["parent"][i]
        vis[i] = p < 0 or (vis[p] and opened[p])
    acc = vis & ~opened
    ext = vis & opened & T["leaf"]
    want_nodes = np.sort(T["label"][acc])
    got_nodes = np.sort(P["ref"][P["kind"] == oracle.PSEUDO_NODE].astype(np.uint64))
    assert np.array_equal(want_nodes, got_nodes)
    want_parts = np.sort(np.concatenate([T["perm"][T["start"][i]:T["end"][i]] for i in np.flatnonzero(ext)]))
    got_parts = np.sort(P["ref"][P["kind"] == oracle.PSEUDO_PARTICLE])
    assert np.array_equal(want_parts, got_parts)
    # every particle within r_part of a source is extracted
    d = np.sqrt(((clumpy.xyz[:, None, :] - src[None]) ** 2).sum(2)).min(1)
    assert np.all(np.isin(np.flatnonzero(d < rp), got_parts))
    assert P["stats"]["substitute_leaves"] == int(ext.sum())


def test_h_residual_and_bracket(clumpy):
    theta, rp, rl = 0.5, 0.05, 0.1
    src = np.array([[0.5, 0.5, 0.5]])
    P = oracle.pseudo(clumpy.xyz, clumpy.m, clumpy.h, BOX, src, theta, rp, rl)
    T = oracle.tree(clumpy.xyz, clumpy.m, BOX, 8)
    # points: node pseudo-particles and the leaves standing in for extracted particles
    nodes = P["kind"] == oracle.PSEUDO_NODE
    lab2i = {int(l): i for i, l in enumerate(T["label"])}
    ext_leaf = set()
    inv = np.empty_like(T["perm"])
    inv[T["perm"]] = np.arange(inv.size)
    leaves = np.flatnonzero(T["leaf"])
    leaf_of = np.empty(inv.size, np.int64)
    for i in leaves:
        leaf_of[T["start"][i]:T["end"][i]] = i
    for a in P["ref"][~nodes]:
        ext_leaf.add(int(leaf_of[inv[a]]))
    pts = np.concatenate([P["xyz"][nodes], T["com"][sorted(ext_leaf)]])
    assert P["stats"]["fallbacks"] == 0
    target = HF ** 3
    for t in np.flatnonzero(nodes):
        x, hh = P["xyz"][t], P["h"][t]
        r = np.sqrt(((pts - x) ** 2).sum(1))
        N = _w(r / hh).sum() / np.pi
        assert abs(N - target) <= 1e-12
        assert _w(r / (hh * (1 - 1e-9))).sum() / np.pi < target <= _w(r / (hh * (1 + 1e-9))).sum() / np.pi
        assert lab2i[int(P["ref"][t])] >= 0
    # particles keep their SPH smoothing lengths
    assert np.array_equal(P["h"][~nodes], clumpy.h[P["ref"][~nodes]])


@pytest.mark.parametrize("k,r", [(12, 1.0), (30, 0.37), (6, 2.5)])
def test_h_closed_form_shell(k, r):
    """Self plus k points at distance r: w(r/h) = (pi h_fact^3 - 1)/k, a cubic in q = r/h."""
    rng = np.random.default_rng(k)
    v = rng.normal(size=(k, 3))
    v = r * v / np.linalg.norm(v, axis=1, keepdims=True)
    pts = np.concatenate([[[0.0, 0.0, 0.0]], v]) + 0.5
    c = (np.pi * HF ** 3 - 1.0) / k
    roots = []
    # inner piece 1 - 1.5 q^2 + 0.75 q^3 = c on [0,1); outer 0.25 (2-q)^3 = c on [1,2)
    for q in np.roots([0.75, -1.5, 0.0, 1.0 - c]):
        if abs(q.imag) < 1e-12 and 0.0 <= q.real < 1.0:
            roots.append(q.real)
    qo = 2.0 - (4.0 * c) ** (1.0 / 3.0)
    if 1.0 <= qo < 2.0:
        roots.append(qo)
    assert len(roots) == 1
    h_exact = r / roots[0]
    h, fb = oracle.solve_h(pts, pts[0], 0.3 * h_exact)
    assert not fb
    assert abs(h - h_exact) <= 1e-13 * h_exact
    h2, _ = oracle.solve_h(pts, pts[0], 5.0 * h_exact)
    assert abs(h2 - h_exact) <= 1e-13 * h_exact


def test_h_fallback_without_root():
    pts = np.array([[0.5, 0.5, 0.5], [0.6, 0.5, 0.5], [0.5, 0.7, 0.5], [0.2, 0.2, 0.2]])
    h, fb = oracle.solve_h(pts, pts[0], 0.123)
    assert fb and h == 0.123
