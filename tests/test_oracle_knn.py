"""Pins for the oracle's kappa-nearest-neighbour importance sampling (the kappa
of the sampling in Sec. 4, Table "speedup"; reading: a node samples first the
neighbours of its points that lie outside it, ranked by how many of its
points have them as neighbours, then uniform rows).

The neighbours are checked against scipy's k-d tree (an independent exact
search), the recursive node lists against their direct, non-recursive
definition, and the sampler against the uniform sampler it extends."""
import collections

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth


def _tree(orc, X, m, s, nsamp=None, kappa=0, seed=3):
    o = orc.Oracle(X, m, s, 0.7, nsamp=nsamp, seed=seed)
    perm = o.build_tree()
    if kappa:
        o.set_knn(kappa)
    return o, perm


@pytest.mark.parametrize("kappa", [1, 7, 32])
def test_knn_matches_kdtree(orc, kappa):
    X, _ = synth.small(1500, 5, 21, kind="mixture", scale=3.0)
    o, perm = _tree(orc, X, 64, 16, kappa=kappa)
    Y = X[perm]  # points in tree order: positions index Y
    nn = o.knn()
    dist, idx = cKDTree(Y).query(Y, k=kappa + 1)
    for i in range(o.N):
        # the search returns i itself first (distance 0, no duplicates here)
        ref = [j for j in idx[i] if j != i][:kappa]
        if list(nn[i]) != ref:
            # only a reordering among equal distances is allowed
            d_or = np.sum((Y[nn[i]] - Y[i]) ** 2, axis=1)
            d_ref = np.sum((Y[ref] - Y[i]) ** 2, axis=1)
            assert np.allclose(np.sort(d_or), np.sort(d_ref), rtol=1e-13, atol=0)
    # ascending distance along every list
    d = np.sum((Y[nn] - Y[:, None, :]) ** 2, axis=2)
    assert np.all(np.diff(d, axis=1) >= 0)
    assert not np.any(nn == np.arange(o.N)[:, None])


def test_knn_ties_go_to_the_lower_position(orc):
    # every point appears three times: its two copies are at distance 0 and
    # come first, lower position first, then the next nearest
    rng = np.random.default_rng(4)
    base = rng.uniform(size=(200, 3))
    X = np.repeat(base, 3, axis=0)
    o, perm = _tree(orc, X, 32, 8, kappa=4)
    nn = o.knn()
    Y = X[perm]
    for i in range(o.N):
        twins = [j for j in range(o.N) if j != i and np.array_equal(Y[j], Y[i])]
        assert list(nn[i][:2]) == sorted(twins)
        d = np.sum((Y[nn[i]] - Y[i]) ** 2, axis=1)
        for a in range(3):  # equal distances: increasing positions
            if d[a] == d[a + 1]:
                assert nn[i][a] < nn[i][a + 1]


def test_knn_pads_short_lists(orc):
    X, _ = synth.small(6, 2, 3)
    o, _ = _tree(orc, X, 2, 1, kappa=8)
    nn = o.knn()
    assert np.all(nn[:, 5:] == -1) and np.all(nn[:, :5] >= 0)


def _direct_list(nn, b, e):
    """Neighbours of the points [b, e) outside [b, e), weighted by how many
    of those points have them, ranked by weight then position."""
    c = collections.Counter(int(j) for i in range(b, e) for j in nn[i] if j >= 0 and not b <= j < e)
    return sorted(c.items(), key=lambda kv: (-kv[1], kv[0]))


def test_node_lists_equal_their_direct_definition(orc):
    # sample size above every list length: no list is cut, and the merge of
    # the children's lists must equal the direct count over the node's points
    X, _ = synth.small(1200, 3, 8, kind="mixture", scale=2.0)
    o, _ = _tree(orc, X, 40, 4, nsamp=4000, kappa=6)
    nn = o.knn()
    for node in range(1, o.nnodes):
        b, e = o.node_range(node)
        pos, w = o.node_neighbors(node)
        ref = _direct_list(nn, b, e)
        assert [int(p) for p in pos] == [p for p, _ in ref]
        assert [int(x) for x in w] == [x for _, x in ref]


def test_cut_lists_keep_their_invariants(orc):
    X, _ = synth.small(3000, 4, 9, kind="mixture", scale=3.0)
    o, _ = _tree(orc, X, 64, 8, kappa=16)  # sample size 32: lists are cut
    nn = o.knn()
    for node in range(1, o.nnodes):
        b, e = o.node_range(node)
        pos, w = o.node_neighbors(node)
        assert len(pos) <= o.nsamp
        assert np.all((pos < b) | (pos >= e))
        assert len(set(pos.tolist())) == len(pos)
        key = list(zip((-w).tolist(), pos.tolist()))
        assert key == sorted(key)
        full = dict(_direct_list(nn, b, e))
        assert all(full.get(int(p), 0) >= int(x) for p, x in zip(pos, w))
        if node >= (1 << o.D) - 1:  # a leaf's list is the head of its direct ranking
            ref = _direct_list(nn, b, e)[:o.nsamp]
            assert [int(p) for p in pos] == [p for p, _ in ref]


def test_sample_opens_with_the_list(orc):
    X, _ = synth.small(3000, 4, 9, kind="mixture", scale=3.0)
    o, _ = _tree(orc, X, 64, 16, kappa=2)  # short lists: uniform draws fill
    for node in range(1, o.nnodes):
        b, e = o.node_range(node)
        pos, _ = o.node_neighbors(node)
        q = o.node_sample(node)
        assert len(q) == min(o.nsamp, o.N - (e - b))
        assert len(set(q.tolist())) == len(q)
        assert np.all((q < b) | (q >= e))
        if o.N - (e - b) > o.nsamp:
            assert np.array_equal(q[:len(pos)], pos)
            # the fill is the uniform stream with the list's positions rejected
            ref = orc.sample_prefix(o.seed, 0, node, o.N, b, e, o.nsamp, pos)
            assert np.array_equal(q, ref)


def test_empty_prefix_is_the_uniform_sampler(orc):
    X, _ = synth.small(2000, 3, 2)
    o, _ = _tree(orc, X, 64, 16)
    for node in (1, 2, 9, 40):
        b, e = o.node_range(node)
        assert np.array_equal(o.node_sample(node), orc.sample(o.seed, 0, node, o.N, b, e, o.nsamp))
        assert np.array_equal(orc.sample_prefix(o.seed, 0, node, o.N, b, e, o.nsamp, []),
                              orc.sample(o.seed, 0, node, o.N, b, e, o.nsamp))
    # a complement no larger than the sample is taken whole, in order
    q = orc.sample_prefix(1, 0, 1, 100, 0, 40, 64, [70, 50])
    assert np.array_equal(q, np.arange(40, 100))


def test_subtree_sample_agrees_with_the_whole_tree(orc):
    X, _ = synth.small(2500, 4, 13, kind="mixture", scale=3.0)
    o, _ = _tree(orc, X, 64, 16, kappa=8)
    for node in (3, 12, 40):
        pos, w = o.node_neighbors(node)
        p2, w2, q2 = o.subtree_sample(node, 8)
        assert np.array_equal(pos, p2) and np.array_equal(w, w2)
        assert np.array_equal(o.node_sample(node), q2)


@pytest.mark.parametrize("N,d,scale,h", [(2048, 4, 4.0, 0.8), (3000, 3, 3.0, 0.4), (4096, 6, 8.0, 0.6)])
def test_neighbour_sampling_approximates_k_better(orc, N, d, scale, h):
    # the point of the importance sampling: rows near the node carry the
    # large kernel entries that uniform rows miss on clustered data, so the
    # skeletons see them and the approximation of K improves (measured
    # 0.33-0.43 relative Frobenius error with uniform rows, 0.20-0.30 with
    # kappa = 4..32 on these cases)
    X, _ = synth.small(N, d, 5, kind="mixture", scale=scale)
    lam = 0.5
    K = orc.dense_kernel(X, h) + lam * np.eye(N)
    err = {}
    for kappa in (0, 8):
        o = orc.Oracle(X, 64, 16, h, seed=3)
        o.build_tree()
        o.set_knn(kappa)
        o.skeletonize()
        o.factorize(lam)
        err[kappa] = np.linalg.norm(o.dense() - K) / np.linalg.norm(K)
    assert err[8] < 0.8 * err[0]
