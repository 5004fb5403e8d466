"""The factorization's launch shapes (level-batched execution, Sec. 2.2's
level schedule): a tuned tree factorizes to the same solution up to the
rounding of the regrouped split sums, through both entry points, in FP64
and in mixed precision; tile widths and the LU split over launches change
no result."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import colrel

pytestmark = pytest.mark.gpu


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


def test_tuned_factorization_matches(ak):
    X, B = synth.small(20000, 8, 41, nrhs=3, kind="mixture", scale=4.0)
    lam = 0.5
    print(f"[gpu tune] N=20000 m=256 s=128", file=sys.stderr, flush=True)
    t = ak.Tree(_cuda(X), 256, 128, 1.5, seed=4)
    t.skeletonize()
    Bd = _cuda(B)
    f = t.factorize(lam, ak.ASKIT_FP64)
    x0 = f.solve(Bd).cpu().numpy()
    r0 = float((np.linalg.norm(B - f.matvec(_cuda(x0)).cpu().numpy(), axis=0) / np.linalg.norm(B, axis=0)).max())
    f.close()
    table = t.tune(lam)
    assert table and len(table) == t.D
    for h, (ktc, kkc, gtc) in table.items():
        assert ktc in (64, 128, 256) and gtc in (64, 128, 256) and kkc in (2048, 4096, 8192), (h, table)
    f = t.factorize(lam, ak.ASKIT_FP64)
    x1 = f.solve(Bd).cpu().numpy()
    r1 = float((np.linalg.norm(B - f.matvec(_cuda(x1)).cpu().numpy(), axis=0) / np.linalg.norm(B, axis=0)).max())
    f.close()
    # a different split chunk regroups the partial sums of the Z blocks: the
    # two solutions are two FP64 orderings of the same algebra, as close as
    # the recursion's amplification of rounding allows (measured 1.4e-10
    # here, with residuals of 2.0e-9 and 2.9e-9)
    print(f"  tuned {table}; solutions differ by {colrel(x1, x0):.1e}, residuals {r0:.1e} {r1:.1e}",
          file=sys.stderr, flush=True)
    assert colrel(x1, x0) < 1e-8
    assert r1 < 10 * max(r0, 1e-12)
    # the pipelined call on the tuned tree gives the separate calls' factors
    f = t.skeletonize_factorize(lam, ak.ASKIT_FP64)
    x2 = f.solve(Bd).cpu().numpy()
    f.close()
    assert np.array_equal(x2, x1)
    # mixed precision keeps tiles of at most 128 columns
    f = t.factorize(lam, ak.ASKIT_MIXED)
    f.set_refinement(50, 1e-11)
    x3 = f.solve(Bd).cpu().numpy()
    f.close()
    assert colrel(x3, x0) < 1e-8
    t.close()


@pytest.mark.parametrize("d", [8, 20])
def test_tile_width_changes_no_result(ak, d):
    """Every tile width sums the same products in the same order: 64-, 128-
    and 256-column tiles (two 128-column wave groups sharing the generated
    kernel tile; row points in registers for d <= 16, in LDS above) give the
    same factors bit for bit, through both entry points; a table with sizes
    the kernels do not have is refused."""
    X, B = synth.small(12000, d, 43, nrhs=2, kind="mixture", scale=4.0)
    lam = 0.5
    print(f"[gpu tune] tile widths, N=12000 d={d} m=128 s=128", file=sys.stderr, flush=True)
    t = ak.Tree(_cuda(X), 128, 128, 2.0, seed=5)
    t.skeletonize()
    Bd = _cuda(B)
    xs = {}
    for w in (64, 128, 256):
        t.set_tiling({h: (w, 4096, w) for h in range(1, t.D + 1)})
        f = t.factorize(lam, ak.ASKIT_FP64)
        xs[w] = f.solve(Bd).cpu().numpy()
        f.close()
        assert t.stats()["tune"]["1"] == [w, 4096, w]
    assert np.array_equal(xs[64], xs[128]) and np.array_equal(xs[128], xs[256])
    f = t.skeletonize_factorize(lam, ak.ASKIT_FP64)  # still the 256-column tiles
    assert np.array_equal(f.solve(Bd).cpu().numpy(), xs[256])
    f.close()
    t.set_tiling(None)
    f = t.factorize(lam, ak.ASKIT_FP64)
    assert np.array_equal(f.solve(Bd).cpu().numpy(), xs[128])  # built-in: 128 columns, 4096-point chunks
    f.close()
    with pytest.raises(ak.AskitError):
        t.set_tiling({h: (96, 4096, 64) for h in range(1, t.D + 1)})
    with pytest.raises(ak.AskitError):
        t.set_tiling({h: (64, 1000, 64) for h in range(1, t.D + 1)})
    t.close()


@pytest.mark.parametrize("lam", [0.5, 0.0])
def test_lu_split_changes_no_result(ak, lam):
    """The LU with partial pivoting split over launches (a 32-column panel
    per launch over the batch, the trailing update in 64 x 64 tiles) gives
    the factors of the one-workgroup LU bit for bit: reduced systems Z of up
    to 2s = 320 rows (split from 257 rows by default), and with lambda = 0
    the leaf blocks (up to 256 rows, factored with pivoting) too when every
    batch is split; through both entry points."""
    X, B = synth.small(12000, 8, 47, nrhs=2, kind="mixture", scale=4.0)
    print(f"[gpu tune] LU split, N=12000 d=8 m=256 s=160 lambda={lam}", file=sys.stderr, flush=True)
    t = ak.Tree(_cuda(X), 256, 160, 2.0, seed=5)
    t.skeletonize()
    r = t.skeleton_sizes()[0]
    zmax = max(int(r[2 * i + 1] + r[2 * i + 2]) for i in range((len(r) - 1) // 2))
    assert zmax > 256  # the default splits the upper heights
    Bd = _cuda(B)
    xs, ratios = {}, {}
    for n in (512, 256, 0):
        t.set_lu_split(n)
        f = t.factorize(lam, ak.ASKIT_FP64)
        xs[n] = f.solve(Bd).cpu().numpy()
        ratios[n] = f.pivot_ratio()
        f.close()
    assert np.array_equal(xs[512], xs[256], equal_nan=True) and np.array_equal(xs[512], xs[0], equal_nan=True)
    assert ratios[512] == ratios[256] == ratios[0]
    if lam > 0:
        assert np.all(np.isfinite(xs[0]))
    t.set_lu_split(0)
    f = t.skeletonize_factorize(lam, ak.ASKIT_FP64)
    assert np.array_equal(f.solve(Bd).cpu().numpy(), xs[512], equal_nan=True)
    f.close()
    with pytest.raises(ak.AskitError):
        t.set_lu_split(-1)
    t.close()
