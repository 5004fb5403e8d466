"""Pins for the oracle's tree (Sec. 2.1, "Partitioning the matrix").

Reading: complete binary tree of depth D = ceil(log2(N/m)); each split gives
floor(n/2) points to the left child, the points with the smallest projections
on the principal axis of the node's points (median split, ties by index)."""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _nodes(o):
    for node in range(o.nnodes):
        yield node, int(np.floor(np.log2(node + 1)))


@pytest.mark.parametrize("N,m", [(1, 2), (2, 2), (5, 2), (64, 8), (1000, 64), (4096, 64), (777, 100)])
def test_depth_and_ranges(orc, N, m):
    X = np.random.default_rng(N).uniform(size=(N, 3))
    o = orc.Oracle(X, m, 4, 1.0)
    D = orc.depth(N, m)
    assert m * 2 ** D >= N and (D == 0 or m * 2 ** (D - 1) < N)
    perm = o.build_tree()
    assert np.array_equal(np.sort(perm), np.arange(N))
    for node, lvl in _nodes(o):
        b, e = o.node_range(node)
        n = e - b
        assert n in (N // 2 ** lvl, -(-N // 2 ** lvl))
        if lvl < o.D:
            lb, le = o.node_range(2 * node + 1)
            rb, re = o.node_range(2 * node + 2)
            assert (lb, le, rb, re) == (b, b + n // 2, b + n // 2, e)
        else:
            assert 1 <= n <= m


def _axis_eigh(P):
    mu = P.mean(0)
    C = (P - mu).T @ (P - mu)
    w, V = np.linalg.eigh(C)
    v = V[:, -1]
    k = int(np.argmax(np.abs(v)))
    if v[k] < 0:
        v = -v
    gap = w[-2] / w[-1] if w[-1] > 0 else 1.0
    return mu, v, gap


@pytest.mark.parametrize("N,m,seed", [(48, 4, 0), (64, 8, 1), (600, 16, 2), (3000, 40, 3)])
def test_split_is_principal_axis_median(orc, N, m, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, 3)) * np.array([4.0, 2.0, 1.0]) @ np.linalg.qr(rng.standard_normal((3, 3)))[0]
    o = orc.Oracle(X, m, 4, 1.0)
    perm = o.build_tree()
    checked = 0
    for node, lvl in _nodes(o):
        if lvl >= o.D:
            continue
        b, e = o.node_range(node)
        ids = perm[b:e]
        mu, v, gap = _axis_eigh(X[ids])
        key = (X[ids] - mu) @ v
        order = np.argsort(key, kind="stable")
        nl = (e - b) // 2
        srt = np.sort(key)
        # only nodes whose axis is well determined (power iteration converged,
        # eigh agrees) and whose median is not a near tie are compared
        if gap > 0.6 or (nl < e - b and srt[nl] - srt[nl - 1] < 1e-9 * (1 + abs(srt).max())):
            continue
        checked += 1
        left_set = set(ids[order[:nl]].tolist())
        lb, le = o.node_range(2 * node + 1)
        assert set(perm[lb:le].tolist()) == left_set
    assert checked >= max(1, (o.nnodes // 2) // 3)


def test_brute_force_small(orc):
    # N = 24, m = 3: enumerate each node's keys by brute force and check the
    # left child is exactly the floor(n/2) smallest (key, index) pairs
    rng = np.random.default_rng(11)
    X = rng.standard_normal((24, 2)) * np.array([3.0, 1.0])
    o = orc.Oracle(X, 3, 2, 1.0)
    perm = o.build_tree()
    for node, lvl in _nodes(o):
        if lvl >= o.D:
            continue
        b, e = o.node_range(node)
        ids = perm[b:e]
        mu, v, gap = _axis_eigh(X[ids])
        if gap > 0.6:
            continue
        pairs = sorted(((float((X[i] - mu) @ v), int(i)) for i in ids))
        lb, le = o.node_range(2 * node + 1)
        assert sorted(perm[lb:le].tolist()) == sorted(i for _, i in pairs[: (e - b) // 2])


def test_tree_ties_by_index(orc):
    # all points identical: keys tie everywhere, so the order is by index
    X = np.ones((40, 3))
    o = orc.Oracle(X, 5, 2, 1.0)
    assert np.array_equal(o.build_tree(), np.arange(40))


def test_golden_perm(orc):
    """Regression fixture written by tests/golden/make_golden.py (oracle only)."""
    path = os.path.join(HERE, "golden", "tree_perm_n200_d3.txt")
    data = np.loadtxt(path, dtype=np.int64)
    import synth
    X, _ = synth.small(200, 3, 1, kind="mixture", scale=3.0)
    o = orc.Oracle(X, 10, 4, 1.0)
    assert np.array_equal(o.build_tree(), data)
