"""Device block cache: a factorization that reuses the blocks released by
the one before gives the same result bit for bit, and
askit_release_cached_memory frees what the cache holds (then nothing)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ak():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1701_02324_amd as ak
    ak.load()
    return ak


@pytest.mark.parametrize("mixed", [False, True])
def test_cached_blocks_reused(ak, mixed):
    import torch
    # 256 leaves of ~235 points: the leaf LU arena (~146 MB) is above the
    # cache threshold of 64 MiB
    N, d, m, s = 60000, 4, 256, 64
    print(f"[gpu cache] N={N} d={d} m={m} s={s} mixed={mixed}", file=sys.stderr, flush=True)
    X, B = synth.small(N, d, 17, nrhs=2, kind="mixture", scale=4.0)
    Xd = torch.as_tensor(X, device="cuda")
    Bd = torch.as_tensor(B, device="cuda")
    prec = ak.ASKIT_MIXED if mixed else ak.ASKIT_FP64
    ak.askit_release_cached_memory()
    t = ak.Tree(Xd, m, s, 1.0, seed=3)
    t.skeletonize()
    xs = []
    for rep in range(3):
        f = t.factorize(0.1, prec)
        xs.append(f.solve(Bd).cpu().numpy())
        f.close()
    t.close()
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    freed = ak.askit_release_cached_memory()
    assert freed >= 64 << 20
    assert ak.askit_release_cached_memory() == 0
