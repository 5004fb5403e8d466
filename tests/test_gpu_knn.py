"""GPU parity of the kappa-nearest-neighbour importance sampling (the kappa of
the sampling in Sec. 4, Table "speedup"): the neighbours of every point
(bit-exact indices, ties to the lower position), the ranked neighbour list of
every node (positions and weights), the sampled rows that open with that
list, the skeletons and the solve, against the oracle on the same input; and
at the 1M workload, the neighbours, lists and samples of a subtree the
oracle can afford."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import colrel, skeleton_parity

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ak():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_02324_amd as ak
    ak.load()
    return ak


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


# name: (N, d, m, s, h, kappa, kind, scale); the lists of "wide" (m kappa =
# 8192 entries per leaf) are ranked in the global scratch path, the others in LDS
CASES = {
    "ragged_k8": (3001, 3, 64, 16, 0.5, 8, "uniform", 1.0),
    "mix_k16": (6000, 8, 128, 32, 1.5, 16, "mixture", 3.0),
    "d20_k32": (4000, 20, 64, 24, 3.0, 32, "mixture", 3.0),
    "d40_k8": (2000, 40, 64, 16, 5.0, 8, "mixture", 2.0),
    "wide_k64": (8192, 16, 128, 32, 2.0, 64, "mixture", 4.0),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, ak, orc):
    N, d, m, s, h, kappa, kind, scale = CASES[request.param]
    X, B = synth.small(N, d, 31, nrhs=2, kind=kind, scale=scale)
    say(f"[gpu knn] case {request.param}: N={N} d={d} m={m} s={s} kappa={kappa}")
    o = orc.Oracle(X, m, s, h, seed=17)
    o.build_tree()
    o.set_knn(kappa)
    t = ak.Tree(_cuda(X), m, s, h, seed=17, knn=kappa)
    yield dict(X=X, B=B, o=o, t=t, h=h, kappa=kappa, name=request.param)
    t.close()


def test_neighbours_bit_exact(case):
    o, t = case["o"], case["t"]
    assert np.array_equal(_np(t.perm()), o.perm())
    g, r = t.neighbors().astype(np.int64), o.knn()
    bad = np.nonzero(np.any(g != r, axis=1))[0]
    assert bad.size == 0, (bad[:5], g[bad[:2]], r[bad[:2]])


def test_neighbour_lists_match_oracle(case):
    o, t = case["o"], case["t"]
    pos, w, n = t.neighbor_lists()
    for node in range(1, t.nnodes):
        rp, rw = o.node_neighbors(node)
        assert n[node] == len(rp), node
        assert np.array_equal(pos[node, :n[node]], rp), node
        assert np.array_equal(w[node, :n[node]], rw), node
    assert n[0] == 0


def test_samples_open_with_the_lists(case):
    o, t = case["o"], case["t"]
    t.skeletonize()
    samp = t.samples()
    _, cands = t.skeleton_sizes()
    checked = 0
    for node in range(1, t.nnodes):
        if cands[node] <= t.s:
            continue
        q = o.node_sample(node)
        assert np.array_equal(samp[node, :len(q)], q), node
        checked += 1
    say(f"  samples identical on {checked} nodes")
    assert checked > 0


def test_skeletons_and_solve(case, ak, orc):
    import oracle as orc_mod
    o, t, X, B, h = case["o"], case["t"], case["X"], case["B"], case["h"]
    t.skeletonize()
    o.skeletonize()
    ids, P, sizes = t.export_skeletons()
    rep = skeleton_parity(orc_mod, o, X, h, 17, ids, P, sizes, t.s, t.cmax, sampler=o.node_sample)
    say(f"  skeletons: {rep['identical']}/{rep['compared']} identical, {rep['near_tie']} near-ties")
    assert not rep["failures"], rep["failures"][:5]
    if rep["identical"] == rep["compared"] == t.nnodes - 1:
        lam = 0.5
        f = t.factorize(lam, ak.ASKIT_FP64)
        x = _np(f.solve(_cuda(B)))
        f.close()
        o.factorize(lam)
        err = colrel(x, o.solve(B))
        say(f"  solve vs oracle {err:.2e}")
        assert err < 1e-10


def test_wrong_state_and_uniform_trees(ak):
    import torch
    X, _ = synth.small(2000, 3, 4)
    t = ak.Tree(_cuda(X), 64, 16, 1.0, seed=2)  # knn = 0
    with pytest.raises(ak.AskitError):
        t.neighbors()
    with pytest.raises(ak.AskitError):
        t.neighbor_lists()
    t.close()
    # kappa at least N - 1: every other point is a neighbour, -1 pads
    t = ak.Tree(_cuda(X[:40]), 8, 2, 1.0, seed=2, knn=64)
    nn = t.neighbors()
    assert np.all(nn[:, 39:] == -1) and np.all(nn[:, :39] >= 0)
    assert all(sorted(nn[i, :39].tolist()) == [j for j in range(40) if j != i] for i in range(40))
    t.close()
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def c3knn(ak, orc):
    """The 1M workload with kappa = 32."""
    c = synth.config(3, nrhs=1)
    say("[gpu knn] 1M workload, kappa = 32: GPU tree, neighbours, lists, samples")
    t = ak.Tree(_cuda(c["X"]), c["m"], c["s"], c["h"], n_samples=c["nsamp"], seed=c["seed"], knn=32)
    t.skeletonize()
    o = orc.Oracle(c["X"], c["m"], c["s"], c["h"], nsamp=c["nsamp"], seed=c["seed"])
    o.build_tree()
    yield dict(c=c, t=t, o=o)
    t.close()


def test_c3_subtree_against_oracle(c3knn):
    """A level-10 node (1024 points) and its two leaves: the oracle finds
    the neighbours of those points by brute force over all 2^20 points and
    ranks the subtree's lists; the GPU's neighbours, lists and samples must
    match bit for bit."""
    t, o = c3knn["t"], c3knn["o"]
    assert np.array_equal(_np(t.perm()), o.perm())
    nn = t.neighbors()
    pos, w, n = t.neighbor_lists()
    samp = t.samples()
    _, cands = t.skeleton_sizes()
    node = (1 << 10) - 1 + 357
    b, e = o.node_range(node)
    say(f"  oracle: neighbours of positions [{b}, {e}) over N = {o.N}")
    ref = o.knn_rows(b, e, 32)
    assert np.array_equal(nn[b:e].astype(np.int64), ref)
    for nd in (node, 2 * node + 1, 2 * node + 2):
        rp, rw, rq = o.subtree_sample(nd, 32)
        assert n[nd] == len(rp) and np.array_equal(pos[nd, :n[nd]], rp) and np.array_equal(w[nd, :n[nd]], rw), nd
        if cands[nd] > t.s:
            assert np.array_equal(samp[nd, :len(rq)], rq), nd
        say(f"  node {nd}: list of {len(rp)} (top weight {rw[0] if len(rw) else 0}), sample identical")
