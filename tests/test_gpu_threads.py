"""Calls on different handles made from two threads at once (each thread on
its own stream) give the results of the same calls made one after the
other, bit for bit: the pipelined skeletonize + factorize, and the solve."""
import sys
import threading

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


# (N, d, m, s, h, lambda)
CASES = [(20000, 8, 128, 64, 1.0, 0.1), (12000, 4, 64, 32, 0.5, 1.0)]


def _run(ak, idx, out):
    import torch
    try:
        N, d, m, s, h, lam = CASES[idx]
        X, B = synth.small(N, d, 40 + idx, nrhs=2, kind="mixture", scale=4.0)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            Xd = torch.as_tensor(X, device="cuda")
            Bd = torch.as_tensor(B, device="cuda")
            t = ak.Tree(Xd, m, s, h, seed=9)
            f = t.skeletonize_factorize(lam, ak.ASKIT_MIXED)
            x = f.solve(Bd)
            st.synchronize()
            out[idx] = (t.export_skeletons(), x.cpu().numpy())
            f.close()
            t.close()
    except Exception as e:  # re-raised by the test
        out[idx] = e


def test_two_threads_match_sequential(ak):
    print(f"[gpu threads] cases {CASES}", file=sys.stderr, flush=True)
    seq, par = [None] * len(CASES), [None] * len(CASES)
    for i in range(len(CASES)):
        _run(ak, i, seq)
    threads = [threading.Thread(target=_run, args=(ak, i, par)) for i in range(len(CASES))]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
        assert not th.is_alive()
    for i in range(len(CASES)):
        for r in (seq[i], par[i]):
            if isinstance(r, Exception):
                raise r
        (sk_a, x_a), (sk_b, x_b) = seq[i], par[i]
        for u, v in zip(sk_a, sk_b):
            assert np.array_equal(u, v)
        assert np.array_equal(x_a, x_b)
