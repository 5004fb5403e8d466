"""askit_skeletonize_factorize: skeletonization and factorization pipelined
over two streams give the results of the two separate calls bit for bit
(skeletons, solves in FP64 and mixed precision, matvecs), and leave the tree
in the state the separate calls leave it."""
import sys

import numpy as np
import pytest

import synth

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


# (N, d, m, s, h, lambda, split levels): several heights, ragged leaves,
# nodes with |C| <= s next to QR'd ones, both QR launch shapes
CASES = {
    "mixture-d8": (20000, 8, 128, 64, 1.0, 0.1, 0),
    "uniform-d3-oneWG": (9001, 3, 64, 32, 0.5, 1.0, -1),
    "mixture-d16-wide": (40000, 16, 256, 128, 2.0, 0.01, 0),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mixed", [False, True])
def test_fused_matches_separate_calls(ak, name, mixed):
    N, d, m, s, h, lam, split = CASES[name]
    say(f"[gpu fused] {name} N={N} d={d} m={m} s={s} mixed={mixed}")
    X, B = synth.small(N, d, 31, nrhs=3, kind="mixture" if "mixture" in name else "uniform",
                       scale=4.0 if "mixture" in name else 1.0)
    prec = ak.ASKIT_MIXED if mixed else ak.ASKIT_FP64
    Xd, Bd = _cuda(X), _cuda(B)
    out = []
    for fused in (False, True):
        t = ak.Tree(Xd, m, s, h, seed=5, qr_split_levels=split)
        if fused:
            f = t.skeletonize_factorize(lam, prec)
        else:
            t.skeletonize()
            f = t.factorize(lam, prec)
        sk = t.export_skeletons()
        x = _np(f.solve(Bd))
        xt = _np(f.solve_transpose(Bd))
        y = _np(f.matvec(Bd))
        ratio = f.pivot_ratio()
        out.append((sk, x, xt, y, ratio))
        f.close()
        # the tree is skeletonized afterwards: a second factorization works
        f2 = t.factorize(2 * lam, prec)
        out[-1] += (_np(f2.solve(Bd)),)
        f2.close()
        t.close()
    a, b = out
    for u, v in zip(a[0], b[0]):
        assert np.array_equal(u, v)
    for k in range(1, 4):
        assert np.array_equal(a[k], b[k]), k
    assert a[4] == b[4]
    assert np.array_equal(a[5], b[5])


def test_fused_rejects_live_factors(ak):
    X, _ = synth.small(3000, 3, 2)
    t = ak.Tree(_cuda(X), 64, 16, 0.5)
    f = t.skeletonize_factorize(0.5)
    with pytest.raises(RuntimeError):
        t.skeletonize_factorize(0.5)
    with pytest.raises(RuntimeError):
        t.skeletonize()
    f.close()
    g = t.skeletonize_factorize(0.5)  # allowed again once the factor is gone
    g.close()
    t.close()
    t = ak.Tree(_cuda(X), 64, 16, 0.5)
    with pytest.raises(RuntimeError):
        t.skeletonize_factorize(-1.0)
    with pytest.raises(RuntimeError):
        t.skeletonize_factorize(0.5, 7)
    t.close()
