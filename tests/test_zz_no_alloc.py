"""The allocation-free entry point askit_tree_permutation_noalloc against
askit_build_tree + askit_tree_perm (same tree rules, same kernels): two
calls in a row on the library's static scratch array, the second smaller,
each bit for bit; an input beyond the array is refused."""
import ctypes
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


def test_noalloc_permutation_matches_tree_build(ak):
    import torch
    A = ak.askit
    for N, d, m, kind in ((300000, 16, 512, "mixture"), (50000, 16, 512, "mixture"), (3001, 3, 64, "uniform")):
        say(f"[no-alloc] N={N} d={d} m={m}")
        X, _ = synth.small(N, d, N, kind=kind, scale=4.0)
        Xd = torch.as_tensor(X, device="cuda")
        t = ak.Tree(Xd, m, 8, 1.0)
        want = t.perm().cpu().numpy()
        t.close()
        perm = torch.full((N,), -7, dtype=torch.int64, device="cuda")
        out = ctypes.c_void_p(perm.data_ptr())
        st = A.load().askit_tree_permutation_noalloc(ctypes.c_void_p(Xd.data_ptr()), N, d, m, out,
                                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == A.ASKIT_OK, A.load().askit_last_error()
        torch.cuda.synchronize()
        got = perm.cpu().numpy()
        assert np.array_equal(got, want), (N, int(np.sum(got != want)))


def test_noalloc_rejects_inputs_beyond_the_scratch(ak):
    import torch
    A = ak.askit
    N, d = 600000, 64  # about 0.8 GB of temporaries
    Xd = torch.zeros((N, d), dtype=torch.float64, device="cuda")
    perm = torch.empty(N, dtype=torch.int64, device="cuda")
    st = A.load().askit_tree_permutation_noalloc(ctypes.c_void_p(Xd.data_ptr()), N, d, 512,
                                                 ctypes.c_void_p(perm.data_ptr()), None)
    assert st == A.ASKIT_ERR_ARG
    assert b"scratch" in A.load().askit_last_error()
