"""The C ABI library: loads, exports every declared entry point, validates
arguments on the host (no compute call is made without a GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "askit.h")).read()
    return sorted(set(re.findall(r"\b(askit_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1701_02324_amd.askit as A
    if not os.path.exists(A.LIB_PATH):
        pytest.fail("libaskit.so not built (python -m paper_1701_02324_amd.build)")
    return A.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_1701_02324_amd.askit as A
    assert sorted(A.EXPORTED) == _declared()


def test_argument_validation_without_gpu(lib):
    import paper_1701_02324_amd.askit as A
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    bad = [
        (0, 3, A.Options(64, 8, 0, 0, 0, 0, 1.0)),      # N < 1
        (100, 0, A.Options(64, 8, 0, 0, 0, 0, 1.0)),    # d < 1
        (100, 65, A.Options(64, 8, 0, 0, 0, 0, 1.0)),   # d > 64
        (100, 3, A.Options(1, 8, 0, 0, 0, 0, 1.0)),     # m < 2
        (100, 3, A.Options(64, 0, 0, 0, 0, 0, 1.0)),    # s < 1
        (100, 3, A.Options(64, 8, 0, 0, 0, 0, 0.0)),    # h <= 0
        (100, 3, A.Options(64, 8, 0, 0, 0, 0, float("nan"))),
        (5000, 3, A.Options(1024, 8, 0, 0, 0, 0, 1.0)),  # leaf blocks above 512
        (100, 3, A.Options(64, 300, 0, 0, 0, 0, 1.0)),  # 2 s above 512
        (100, 3, A.Options(64, 8, 0, 0, 0, 0, 1.0, -1e-3)),  # tol < 0
        (100, 3, A.Options(64, 8, 0, 0, 0, 0, 1.0, 1.0)),    # tol >= 1
        (100, 3, A.Options(64, 8, 0, 0, 0, 0, 1.0, 0.0, -1)),  # knn < 0
        (100, 3, A.Options(64, 8, 0, 0, 0, 0, 1.0, 0.0, 65)),  # knn > 64
        (100, 40, A.Options(64, 8, 0, 0, 0, 0, 1.0, 0.0, 33)),  # knn > 32 for d > 32
        (40_000_000, 3, A.Options(512, 8, 0, 0, 0, 0, 1.0, 0.0, 64)),  # knn N >= 2^31
    ]
    for N, d, opt in bad:
        st = lib.askit_build_tree(fake, N, d, ctypes.byref(opt), None, ctypes.byref(out))
        assert st == A.ASKIT_ERR_ARG, (N, d)
        assert lib.askit_last_error().decode()
    assert lib.askit_build_tree(None, 10, 3, ctypes.byref(A.Options(4, 2, 0, 0, 0, 0, 1.0)), None,
                                ctypes.byref(out)) == A.ASKIT_ERR_ARG
    # NULL handles
    assert lib.askit_tree_knn(None, fake) == A.ASKIT_ERR_ARG
    assert lib.askit_tune_factorization(None, 1.0, None) == A.ASKIT_ERR_ARG
    assert lib.askit_tree_set_tiling(None, None, 0) == A.ASKIT_ERR_ARG
    assert lib.askit_tree_set_lu_split(None, 256) == A.ASKIT_ERR_ARG
    assert lib.askit_tree_neighbor_lists(None, fake, fake, fake) == A.ASKIT_ERR_ARG
    assert lib.askit_skeletonize(None, None) == A.ASKIT_ERR_ARG
    assert lib.askit_factorize(None, 1.0, 0, None, ctypes.byref(out)) == A.ASKIT_ERR_ARG
    assert lib.askit_solve(None, fake, 10, 1, fake, 10, None) == A.ASKIT_ERR_ARG
    assert lib.askit_solve_transpose(None, fake, 10, 1, fake, 10, None) == A.ASKIT_ERR_ARG
    assert lib.askit_matvec(None, 0, fake, 10, 1, fake, 10, None) == A.ASKIT_ERR_ARG
    lib.askit_tree_destroy(None)
    lib.askit_factor_destroy(None)
