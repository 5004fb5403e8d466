"""GPU edge cases with closed-form answers and limits of the entry points.

- a single leaf (depth 0): the solver is a dense LU of lambda I + K;
- full rank (s >= |C| at every node, R12): Ktilde = K exactly;
- h -> 0: every off-diagonal kernel entry underflows, K = I, x = b / (1 + lambda);
- h -> infinity: K = 1 1^T exactly, Sherman-Morrison closed form;
- the largest leaf and rank the library accepts (m = 512, s = 256), against
  the oracle on the oracle's skeletons;
- arguments at and past the limits."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import colrel, oracle_skeletons

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


def _kexact(X, h):
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / (2.0 * h * h))


def _solve(ak, X, B, m, s, h, lam, prec=None, seed=1):
    t = ak.Tree(_cuda(X), m, s, h, seed=seed)
    t.skeletonize()
    f = t.factorize(lam, ak.ASKIT_FP64 if prec is None else prec)
    x = f.solve(_cuda(B)).cpu().numpy()
    return t, f, x


def test_single_leaf_is_dense_lu(ak):
    X, B = synth.small(100, 3, 21, nrhs=3)
    h, lam = 0.4, 0.3
    t, f, x = _solve(ak, X, B, 128, 16, h, lam)
    assert t.D == 0
    A = _kexact(X, h) + lam * np.eye(100)
    kappa = np.linalg.cond(A)
    say(f"[gpu edge] single leaf: kappa {kappa:.1e}")
    assert colrel(x, np.linalg.solve(A, B)) < 1e-13 * kappa
    xt = f.solve_transpose(_cuda(B)).cpu().numpy()
    assert colrel(xt, np.linalg.solve(A.T, B)) < 1e-13 * kappa
    assert colrel(f.matvec(_cuda(B)).cpu().numpy(), A @ B) < 1e-14
    f.close()
    t.close()


@pytest.mark.parametrize("N,m,s", [(200, 32, 100), (128, 64, 64), (97, 10, 49)])
def test_full_rank_is_exact(ak, N, m, s):
    X, B = synth.small(N, 3, N, nrhs=2)
    h, lam = 0.3, 0.5
    t, f, x = _solve(ak, X, B, m, s, h, lam)
    ranks, cands = t.skeleton_sizes()
    assert np.array_equal(ranks[1:], cands[1:])  # every node keeps its candidates
    A = _kexact(X, h) + lam * np.eye(N)
    kappa = np.linalg.cond(A)
    assert colrel(x, np.linalg.solve(A, B)) < 1e-12 * kappa
    f.close()
    t.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_narrow_bandwidth_identity(ak, mixed):
    X, B = synth.small(500, 3, 4, nrhs=3)
    lam = 0.25
    t, f, x = _solve(ak, X, B, 32, 8, 1e-4, lam, ak.ASKIT_MIXED if mixed else None)
    want = B / (1 + lam)
    err = np.max(np.abs(x - want) / np.abs(want))
    say(f"[gpu edge] K = I ({'mixed' if mixed else 'fp64'}): max relative error {err:.2e}")
    # FP64: two roundings; mixed: FP32 factors refined to the default target
    # relative residual 1e-11 (with K = I the residual is the error)
    assert err <= (1e-11 if mixed else 4.5e-16)
    f.close()
    t.close()


@pytest.mark.parametrize("s", [1, 3])
def test_wide_bandwidth_rank_one(ak, s):
    N, lam = 700, 1.0
    X, B = synth.small(N, 3, 5, nrhs=2)
    t, f, x = _solve(ak, X, B, 40, s, 1e9, lam)
    want = (B - np.ones((N, 1)) * (B.sum(0) / (lam + N))) / lam
    ranks, cands = t.skeleton_sizes()
    # the rank guard keeps one point wherever a node has more than s
    # candidates; a node with |C| <= s keeps them all
    assert np.array_equal(ranks[1:], np.where(cands[1:] > s, 1, cands[1:]))
    # kappa(lambda I + 1 1^T) = (lambda + N) / lambda.  With s = 3 the nodes
    # that keep two identical skeleton points solve Z with duplicated
    # directions; the FP64 oracle itself reaches 1.2e-12 (column-wise) here
    kappa = (lam + N) / lam
    err = colrel(x, want)
    say(f"[gpu edge] K = 1 1^T, s={s}: {err:.2e} (kappa {kappa:.0f})")
    assert err < 1e-14 * kappa
    f.close()
    t.close()


def test_largest_leaf_and_rank(ak, orc):
    """m = 512 and s = 256 (2s = 512, the largest reduced system), d = 16,
    N = 4096 (depth 3): FP64 solve on the oracle's skeletons vs the oracle."""
    X, B = synth.small(4096, 16, 77, nrhs=4, kind="mixture", scale=4.0)
    h, lam = 2.0, 0.5
    o = orc.Oracle(X, 512, 256, h, seed=9)
    o.build_tree()
    o.skeletonize()
    o.factorize(lam)
    t = ak.Tree(_cuda(X), 512, 256, h, seed=9)
    assert np.array_equal(t.perm().cpu().numpy(), o.perm())
    t.import_skeletons(*oracle_skeletons(o, t.s, t.cmax))
    f = t.factorize(lam, ak.ASKIT_FP64)
    x = f.solve(_cuda(B)).cpu().numpy()
    err = colrel(x, o.solve(B))
    say(f"[gpu edge] m=512 s=256: vs oracle {err:.2e}")
    assert err < 1e-10
    f.close()
    t.close()


def test_limits(ak):
    import torch
    X1 = _cuda(np.zeros((1, 2)))
    t = ak.Tree(X1, 2, 1, 1.0)  # one point: a single leaf
    t.skeletonize()
    f = t.factorize(0.5, ak.ASKIT_FP64)
    x = f.solve(_cuda(np.array([[3.0]]))).cpu().numpy()
    assert abs(x[0, 0] - 2.0) < 1e-15  # (lambda + k(x, x)) x = 3
    f.close()
    t.close()
    X64 = _cuda(np.random.default_rng(0).uniform(size=(300, 64)))
    t = ak.Tree(X64, 64, 8, 4.0)  # d = 64 is the largest dimension
    t.skeletonize()
    t.close()
    with pytest.raises(RuntimeError):
        ak.Tree(_cuda(np.zeros((300, 65))), 64, 8, 1.0)
    ak.Tree(X64, 513, 8, 1.0).close()  # m > 512 is fine: the one leaf holds 300
    with pytest.raises(RuntimeError):
        ak.Tree(_cuda(np.zeros((1100, 2))), 600, 8, 1.0)  # leaves of 550 > 512
    with pytest.raises(RuntimeError):
        ak.Tree(X64, 64, 257, 1.0)  # 2s larger than 512
    with pytest.raises(RuntimeError):
        ak.Tree(X64, 64, 8, 1.0, n_samples=5000)
    t = ak.Tree(X64, 64, 8, 4.0)
    t.skeletonize()
    with pytest.raises(RuntimeError):
        t.factorize(-1.0, ak.ASKIT_FP64)
    f = t.factorize(0.1, ak.ASKIT_FP64)
    with pytest.raises((RuntimeError, ValueError)):
        f.solve(torch.empty((300, 0), dtype=torch.float64, device="cuda"))
    f.close()
    t.close()
