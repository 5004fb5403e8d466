"""ctypes binding of libaskit (include/askit.h): argument marshalling only.

Every arithmetic step runs in the HIP kernels of the library; this module
passes device pointers of torch tensors and the current HIP stream.  The
function names match the C entry points.  Importing it without a built
library, or calling it without a GPU, raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime first, so the library binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaskit.so")

ASKIT_OK, ASKIT_ERR_ARG, ASKIT_ERR_ALLOC, ASKIT_ERR_HIP, ASKIT_ERR_STATE, ASKIT_ERR_SINGULAR, ASKIT_WARN_ILLCOND = range(7)
ASKIT_FP64, ASKIT_MIXED = 0, 1

EXPORTED = [
    "askit_build_tree", "askit_tree_depth", "askit_tree_perm", "askit_skeletonize", "askit_skeletons_export",
    "askit_skeletons_import", "askit_factorize", "askit_solve", "askit_solve_transpose", "askit_matvec",
    "askit_set_refinement", "askit_last_solve_info", "askit_factor_pivot_ratio", "askit_get_stats",
    "askit_last_error", "askit_tree_destroy", "askit_factor_destroy", "askit_profile_enable",
    "askit_profile_report", "askit_tree_set_bandwidth", "askit_adjoint_scalars", "askit_skeletonize_batched",
    "askit_batch_create", "askit_batch_factorize", "askit_batch_check", "askit_batch_solve", "askit_batch_factor",
    "askit_batch_destroy", "askit_skeletonize_factorize", "askit_release_cached_memory",
    "askit_factorize_batched", "askit_tree_qr_rows", "askit_tree_samples", "askit_tree_permutation_noalloc",
    "askit_factorize_hybrid", "askit_tree_knn", "askit_tree_neighbor_lists", "askit_tune_factorization",
    "askit_tree_set_tiling",
    "askit_tree_set_lu_split",
]


class AskitError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"askit status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("rank", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("qr_split_levels", ctypes.c_int32), ("seed", ctypes.c_uint64), ("problem", ctypes.c_int64),
                ("h", ctypes.c_double), ("tol", ctypes.c_double), ("knn", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("initial_residual", ctypes.c_double), ("residual", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def load(path: str = LIB_PATH):
    """Load libaskit.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1701_02324_amd.build`")
    L = ctypes.CDLL(path)
    L.askit_last_error.restype = ctypes.c_char_p
    L.askit_build_tree.argtypes = [_vp, _i64, _i32, ctypes.POINTER(Options), _vp, ctypes.POINTER(_vp)]
    L.askit_tree_depth.argtypes = [_vp, ctypes.POINTER(_i32)]
    L.askit_tree_perm.argtypes = [_vp, _vp]
    L.askit_tree_qr_rows.argtypes = [_vp, _vp]
    L.askit_tree_samples.argtypes = [_vp, _vp]
    L.askit_tree_knn.argtypes = [_vp, _vp]
    L.askit_tune_factorization.argtypes = [_vp, ctypes.c_double, _vp]
    L.askit_tree_set_tiling.argtypes = [_vp, _vp, _i32]
    L.askit_tree_set_lu_split.argtypes = [_vp, _i32]
    L.askit_tree_neighbor_lists.argtypes = [_vp, _vp, _vp, _vp]
    L.askit_tree_permutation_noalloc.argtypes = [_vp, _i64, _i32, _i32, _vp, _vp]
    L.askit_skeletonize.argtypes = [_vp, _vp]
    L.askit_skeletons_export.argtypes = [_vp, _vp, _vp, _vp]
    L.askit_skeletons_import.argtypes = [_vp, _vp, _vp, _vp]
    L.askit_factorize.argtypes = [_vp, ctypes.c_double, _i32, _vp, ctypes.POINTER(_vp)]
    L.askit_skeletonize_factorize.argtypes = [_vp, ctypes.c_double, _i32, _vp, ctypes.POINTER(_vp)]
    L.askit_factorize_hybrid.argtypes = [_vp, ctypes.c_double, _i32, _vp, ctypes.POINTER(_vp)]
    for f in ("askit_solve", "askit_solve_transpose"):
        getattr(L, f).argtypes = [_vp, _vp, _i64, _i32, _vp, _i64, _vp]
    L.askit_matvec.argtypes = [_vp, _i32, _vp, _i64, _i32, _vp, _i64, _vp]
    L.askit_set_refinement.argtypes = [_vp, _i32, ctypes.c_double]
    L.askit_last_solve_info.argtypes = [_vp, ctypes.POINTER(SolveInfo)]
    L.askit_factor_pivot_ratio.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32)]
    L.askit_get_stats.argtypes = [_vp, _vp, ctypes.c_char_p, ctypes.c_size_t]
    L.askit_tree_set_bandwidth.argtypes = [_vp, ctypes.c_double]
    L.askit_adjoint_scalars.argtypes = [_vp, _vp, _vp, _i64, _i32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), _vp]
    L.askit_skeletonize_batched.argtypes = [ctypes.POINTER(_vp), _i32, _vp]
    L.askit_batch_create.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(ctypes.c_double), _i32, _i32,
                                     ctypes.POINTER(_vp)]
    L.askit_batch_factorize.argtypes = [_vp, _vp]
    L.askit_factorize_batched.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(ctypes.c_double), _i32, _i32,
                                          _vp, ctypes.POINTER(_vp)]
    L.askit_batch_check.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32), _vp]
    L.askit_batch_solve.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]
    L.askit_batch_factor.argtypes = [_vp, _i32, ctypes.POINTER(_vp)]
    L.askit_batch_destroy.argtypes = [_vp]
    L.askit_profile_enable.argtypes = [_i32]
    L.askit_profile_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.askit_tree_destroy.argtypes = [_vp]
    L.askit_factor_destroy.argtypes = [_vp]
    for name in EXPORTED:
        if name not in ("askit_last_error", "askit_tree_destroy", "askit_factor_destroy", "askit_batch_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st, allow_warn=False):
    if st == ASKIT_OK or (allow_warn and st == ASKIT_WARN_ILLCOND):
        return st
    raise AskitError(st, load().askit_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev64(x, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    return x.to(torch.float64)


def _colmajor(B):
    """N x nrhs (or N) tensor -> (column-major storage tensor of shape nrhs x N, was_vector)."""
    vec = B.dim() == 1
    B2 = B[:, None] if vec else B
    return B2.t().contiguous(), vec


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def askit_build_tree(X, leaf_size, rank, h, n_samples=0, seed=0, problem=0, stream=None, qr_split_levels=0,
                     tol=0.0, knn=0):
    X = _dev64(X, "X").contiguous()
    N, d = X.shape
    opt = Options(int(leaf_size), int(rank), int(n_samples), int(qr_split_levels), int(seed) & 0xFFFFFFFFFFFFFFFF,
                  int(problem), float(h), float(tol), int(knn), 0)
    out = _vp()
    _check(load().askit_build_tree(_vp(X.data_ptr()), N, d, ctypes.byref(opt), _stream(stream), ctypes.byref(out)))
    return out


def askit_tree_depth(tree):
    D = _i32()
    _check(load().askit_tree_depth(tree, ctypes.byref(D)))
    return D.value


def askit_tree_perm(tree, N, device="cuda"):
    p = torch.empty(N, dtype=torch.int64, device=device)
    _check(load().askit_tree_perm(tree, _vp(p.data_ptr())))
    return p


def askit_tree_permutation_noalloc(X, leaf_size, perm=None, stream=None):
    """Tree permutation without any device allocation by the library (the
    output buffer `perm`, int64 N on the device, may be passed in)."""
    X = _dev64(X, "X")
    if not X.is_contiguous():
        raise ValueError("X must be contiguous")
    N, d = X.shape
    if perm is None:
        perm = torch.empty(N, dtype=torch.int64, device=X.device)
    _check(load().askit_tree_permutation_noalloc(_vp(X.data_ptr()), N, d, int(leaf_size), _vp(perm.data_ptr()),
                                                 _stream(stream)))
    return perm


def askit_tree_qr_rows(tree, nnodes):
    """Rows each node's pivoted QR factored (numpy int32 per heap node)."""
    import numpy as np
    rows = np.zeros(nnodes, dtype=np.int32)
    _check(load().askit_tree_qr_rows(tree, rows.ctypes.data))
    return rows


def askit_tree_samples(tree, nnodes, nsamp):
    """Sampled rows of each node (numpy int32, nnodes x nsamp, tree positions)."""
    import numpy as np
    out = np.zeros(nnodes * nsamp, dtype=np.int32)
    _check(load().askit_tree_samples(tree, out.ctypes.data))
    return out.reshape(nnodes, nsamp)


def askit_tree_knn(tree, N, kappa):
    """The kappa nearest tree positions of every tree position (numpy int32, N x kappa)."""
    import numpy as np
    out = np.zeros(N * kappa, dtype=np.int32)
    _check(load().askit_tree_knn(tree, out.ctypes.data))
    return out.reshape(N, kappa)


def askit_tree_neighbor_lists(tree, nnodes, nsamp):
    """(positions, weights, lengths) of every node's ranked neighbour list."""
    import numpy as np
    pos = np.zeros(nnodes * nsamp, dtype=np.int32)
    w = np.zeros(nnodes * nsamp, dtype=np.int32)
    n = np.zeros(nnodes, dtype=np.int32)
    _check(load().askit_tree_neighbor_lists(tree, pos.ctypes.data, w.ctypes.data, n.ctypes.data))
    return pos.reshape(nnodes, nsamp), w.reshape(nnodes, nsamp), n


def askit_tune_factorization(tree, lam, stream=None):
    _check(load().askit_tune_factorization(tree, float(lam), _stream(stream)))


def askit_skeletonize(tree, stream=None):
    _check(load().askit_skeletonize(tree, _stream(stream)))


def askit_skeletons_export(tree, nnodes, rank, cmax, sizes_only=False):
    """(ids, P, sizes); with sizes_only, ids and P are None and only the
    per-node (s_alpha, |C|) pairs are fetched."""
    import numpy as np
    sizes = np.zeros(2 * nnodes, dtype=np.int32)
    if sizes_only:
        _check(load().askit_skeletons_export(tree, None, None, sizes.ctypes.data))
        return None, None, sizes
    ids = np.zeros(nnodes * rank, dtype=np.int32)
    P = np.zeros(nnodes * rank * cmax, dtype=np.float64)
    _check(load().askit_skeletons_export(tree, ids.ctypes.data, P.ctypes.data, sizes.ctypes.data))
    return ids, P, sizes


def askit_skeletons_import(tree, ids, P, sizes):
    import numpy as np
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    P = np.ascontiguousarray(P, dtype=np.float64)
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    _check(load().askit_skeletons_import(tree, ids.ctypes.data, P.ctypes.data, sizes.ctypes.data))


def askit_factorize(tree, lam, precision=ASKIT_FP64, stream=None):
    out = _vp()
    st = load().askit_factorize(tree, float(lam), int(precision), _stream(stream), ctypes.byref(out))
    _check(st, allow_warn=True)
    return out, st


def askit_skeletonize_factorize(tree, lam, precision=ASKIT_FP64, stream=None):
    out = _vp()
    st = load().askit_skeletonize_factorize(tree, float(lam), int(precision), _stream(stream), ctypes.byref(out))
    _check(st, allow_warn=True)
    return out, st


def askit_factorize_hybrid(tree, lam, level, stream=None):
    out = _vp()
    st = load().askit_factorize_hybrid(tree, float(lam), int(level), _stream(stream), ctypes.byref(out))
    _check(st, allow_warn=True)
    return out, st


def _apply(fn, factor, B, stream, *pre):
    B = _dev64(B, "B")
    Bc, vec = _colmajor(B)
    nrhs, N = Bc.shape
    Xc = torch.empty_like(Bc)
    _check(fn(factor, *pre, _vp(Bc.data_ptr()), N, nrhs, _vp(Xc.data_ptr()), N, _stream(stream)))
    X = Xc.t()
    return X[:, 0] if vec else X


def askit_solve(factor, B, stream=None):
    return _apply(load().askit_solve, factor, B, stream)


def askit_solve_transpose(factor, B, stream=None):
    return _apply(load().askit_solve_transpose, factor, B, stream)


def askit_matvec(factor, X, which=0, stream=None):
    return _apply(load().askit_matvec, factor, X, stream, int(which))


def askit_tree_set_bandwidth(tree, h):
    _check(load().askit_tree_set_bandwidth(tree, float(h)))


def askit_adjoint_scalars(factor, X, Z, stream=None):
    """(dlambda, dh) = (-sum z.x, -sum z.(dKtilde/dh x)) for N x nrhs tensors X, Z."""
    Xc, _ = _colmajor(_dev64(X, "X"))
    Zc, _ = _colmajor(_dev64(Z, "Z"))
    nrhs, N = Xc.shape
    a = ctypes.c_double()
    b = ctypes.c_double()
    _check(load().askit_adjoint_scalars(factor, _vp(Xc.data_ptr()), _vp(Zc.data_ptr()), N, nrhs, ctypes.byref(a),
                                        ctypes.byref(b), _stream(stream)))
    return a.value, b.value


def askit_set_refinement(factor, max_refine, refine_tol):
    _check(load().askit_set_refinement(factor, int(max_refine), float(refine_tol)))


def askit_last_solve_info(factor):
    info = SolveInfo()
    _check(load().askit_last_solve_info(factor, ctypes.byref(info)))
    return dict(iterations=info.iterations, converged=bool(info.converged),
                initial_residual=info.initial_residual, residual=info.residual)


def askit_factor_pivot_ratio(factor):
    r = ctypes.c_double()
    n = _i32()
    _check(load().askit_factor_pivot_ratio(factor, ctypes.byref(r), ctypes.byref(n)))
    return r.value, n.value


def askit_get_stats(tree=None, factor=None):
    import json
    buf = ctypes.create_string_buffer(2048)
    _check(load().askit_get_stats(tree, factor, buf, 2048))
    return json.loads(buf.value.decode())


def askit_profile_enable(on=True, per_height=False, timeline=False):
    """Per-kernel HIP-event timing; per_height keeps totals per tree height,
    timeline also every launch's start and end."""
    _check(load().askit_profile_enable((3 if timeline else 2 if per_height else 1) if on else 0))


def askit_profile_report():
    """{"phase:kernel": (total_ms, launches)} since profiling was enabled."""
    import json
    cap = 1 << 16
    while True:
        buf = ctypes.create_string_buffer(cap)
        st = load().askit_profile_report(buf, cap)
        if st != ASKIT_ERR_ARG or cap >= 1 << 28:
            break
        cap *= 8
    _check(st)
    d = json.loads(buf.value.decode())
    return {k: (v if k == "@timeline" else tuple(v)) for k, v in d.items()}


def askit_release_cached_memory():
    """Frees the library's cache of released device blocks; returns the bytes freed."""
    n = ctypes.c_uint64(0)
    _check(load().askit_release_cached_memory(ctypes.byref(n)))
    return int(n.value)


def askit_tree_destroy(tree):
    if tree:
        load().askit_tree_destroy(tree)


def askit_factor_destroy(factor):
    if factor:
        load().askit_factor_destroy(factor)


# ---------------------------------------------------------------------------
# convenience objects (own their handles)
# ---------------------------------------------------------------------------

class Tree:
    """Tree + skeletons of one problem (points X on the GPU, FP64)."""

    def __init__(self, X, leaf_size, rank, h, n_samples=0, seed=0, problem=0, stream=None, qr_split_levels=0,
                 tol=0.0, knn=0):
        self.N, self.d = X.shape
        self.m, self.s, self.h = int(leaf_size), int(rank), float(h)
        self.nsamp = int(n_samples) or 4 * self.s
        self.tol = float(tol)
        self.knn = int(knn)
        self.handle = askit_build_tree(X, leaf_size, rank, h, n_samples, seed, problem, stream, qr_split_levels,
                                       tol, knn)
        self.D = askit_tree_depth(self.handle)
        self.nnodes = (2 << self.D) - 1
        self.mmax = -(-self.N // (1 << self.D))
        self.cmax = max(self.mmax, 2 * self.s)
        self.device = X.device

    def perm(self):
        return askit_tree_perm(self.handle, self.N, self.device)

    def skeletonize(self, stream=None):
        askit_skeletonize(self.handle, stream)
        return self

    def export_skeletons(self):
        return askit_skeletons_export(self.handle, self.nnodes, self.s, self.cmax)

    def skeleton_sizes(self):
        """(ranks s_alpha, candidate counts |C|) per heap node (root: 0, 0)."""
        sizes = askit_skeletons_export(self.handle, self.nnodes, self.s, self.cmax, sizes_only=True)[2]
        return sizes[0::2].copy(), sizes[1::2].copy()

    def samples(self):
        """Sampled rows of each node's ID (nnodes x n_samples tree positions)."""
        return askit_tree_samples(self.handle, self.nnodes, self.nsamp)

    def neighbors(self):
        """kappa nearest tree positions of every tree position (knn > 0)."""
        return askit_tree_knn(self.handle, self.N, self.knn)

    def neighbor_lists(self):
        """(positions, weights, lengths) of the nodes' ranked neighbour lists (knn > 0)."""
        return askit_tree_neighbor_lists(self.handle, self.nnodes, self.nsamp)

    def qr_rows(self):
        """Rows of the sampled block each node's QR factored (0: no QR)."""
        return askit_tree_qr_rows(self.handle, self.nnodes)

    def import_skeletons(self, ids, P, sizes):
        askit_skeletons_import(self.handle, ids, P, sizes)

    def factorize(self, lam, precision=ASKIT_FP64, stream=None):
        return Factor(self, lam, precision, stream)

    def tune(self, lam, stream=None):
        """Time the factorization's level products in each tile configuration
        and keep the fastest per tree height (askit_tune_factorization)."""
        askit_tune_factorization(self.handle, lam, stream)
        return self.stats().get("tune")

    def set_tiling(self, table):
        """Fix the factorization's tiles per height: {h: (kmm columns, kmm
        chunk, gmm columns)} for h = 1 .. D (the form of tune()'s result),
        or None for the built-in choice (askit_tree_set_tiling)."""
        if table is None:
            _check(load().askit_tree_set_tiling(self.handle, None, 0))
            return
        flat = []
        for h in range(1, self.D + 1):
            flat.extend(int(v) for v in (table[h] if h in table else table[str(h)]))
        arr = (ctypes.c_int32 * len(flat))(*flat)
        _check(load().askit_tree_set_tiling(self.handle, ctypes.cast(arr, _vp), len(table)))

    def set_lu_split(self, n):
        """LU batches whose largest matrix has more than n rows run panel by
        panel over launches (askit_tree_set_lu_split; default 256, 512 never
        splits, 0 always)."""
        _check(load().askit_tree_set_lu_split(self.handle, int(n)))

    def skeletonize_factorize(self, lam, precision=ASKIT_FP64, stream=None):
        """skeletonize() then factorize(), pipelined over two streams."""
        return Factor(self, lam, precision, stream, fused=True)

    def factorize_hybrid(self, lam, level, stream=None):
        """Level-restricted factorization; solve() then runs the hybrid solver."""
        return Factor(self, lam, ASKIT_FP64, stream, level=level)

    def set_bandwidth(self, h):
        """Bandwidth of subsequent factorizations (skeletons frozen)."""
        askit_tree_set_bandwidth(self.handle, h)
        self.hfac = float(h)

    def stats(self):
        return askit_get_stats(self.handle, None)

    def close(self):
        askit_tree_destroy(getattr(self, "handle", None))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factor:
    """Factorization of lambda I + Ktilde on a skeletonized tree."""

    def __init__(self, tree, lam, precision=ASKIT_FP64, stream=None, fused=False, level=0):
        self.tree = tree
        self.lam = float(lam)
        self.precision = precision
        self.level = int(level)
        if level:
            self.handle, self.status = askit_factorize_hybrid(tree.handle, lam, level, stream)
        else:
            make = askit_skeletonize_factorize if fused else askit_factorize
            self.handle, self.status = make(tree.handle, lam, precision, stream)

    def solve(self, B, stream=None):
        return askit_solve(self.handle, B, stream)

    def solve_transpose(self, B, stream=None):
        return askit_solve_transpose(self.handle, B, stream)

    def matvec(self, X, which=0, stream=None):
        return askit_matvec(self.handle, X, which, stream)

    def set_refinement(self, max_refine, tol):
        askit_set_refinement(self.handle, max_refine, tol)

    def adjoint_scalars(self, X, Z, stream=None):
        return askit_adjoint_scalars(self.handle, X, Z, stream)

    def info(self):
        return askit_last_solve_info(self.handle)

    def pivot_ratio(self):
        return askit_factor_pivot_ratio(self.handle)

    def stats(self):
        return askit_get_stats(self.tree.handle, self.handle)

    def close(self):
        askit_factor_destroy(getattr(self, "handle", None))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batches of independent problems
# ---------------------------------------------------------------------------

def askit_skeletonize_batched(trees, stream=None):
    arr = (_vp * len(trees))(*[t.handle for t in trees])
    _check(load().askit_skeletonize_batched(arr, len(trees), _stream(stream)))


def askit_batch_create(trees, lambdas, precision=ASKIT_FP64, nrhs=1):
    arr = (_vp * len(trees))(*[t.handle for t in trees])
    lam = (ctypes.c_double * len(trees))(*[float(x) for x in lambdas])
    out = _vp()
    _check(load().askit_batch_create(arr, len(trees), lam, int(precision), int(nrhs), ctypes.byref(out)))
    return out


def askit_batch_factorize(batch, stream=None):
    _check(load().askit_batch_factorize(batch, _stream(stream)))


def askit_factorize_batched(trees, lambdas, precision=ASKIT_FP64, nrhs=1, stream=None):
    """Batch of the trees with its factorization graph launched once on `stream`."""
    arr = (_vp * len(trees))(*[t.handle for t in trees])
    lam = (ctypes.c_double * len(trees))(*[float(x) for x in lambdas])
    out = _vp()
    _check(load().askit_factorize_batched(arr, len(trees), lam, int(precision), int(nrhs), _stream(stream),
                                          ctypes.byref(out)))
    return out


def askit_batch_check(batch, stream=None):
    r = ctypes.c_double()
    p = _i32()
    _check(load().askit_batch_check(batch, ctypes.byref(r), ctypes.byref(p), _stream(stream)))
    return r.value, p.value


def askit_batch_solve(batch, Bs, stream=None):
    """Bs: list of N_i x nrhs CUDA tensors -> list of solutions."""
    cols = [_colmajor(_dev64(B, "B"))[0] for B in Bs]
    outs = [torch.empty_like(c) for c in cols]
    pb = (_vp * len(cols))(*[c.data_ptr() for c in cols])
    px = (_vp * len(cols))(*[o.data_ptr() for o in outs])
    _check(load().askit_batch_solve(batch, pb, px, _stream(stream)))
    return [o.t() for o in outs]


def askit_batch_factor(batch, i):
    f = _vp()
    _check(load().askit_batch_factor(batch, int(i), ctypes.byref(f)))
    return f


def askit_batch_destroy(batch):
    if batch:
        load().askit_batch_destroy(batch)


class Batch:
    """Independent problems factorized and solved together (one launch per
    kernel and tree height, replayed from hipGraphs)."""

    def __init__(self, trees, lambdas, precision=ASKIT_FP64, nrhs=1, factorize=False, stream=None):
        self.trees = list(trees)
        if factorize:
            self.handle = askit_factorize_batched(self.trees, lambdas, precision, nrhs, stream)
        else:
            self.handle = askit_batch_create(self.trees, lambdas, precision, nrhs)
        self.nrhs = nrhs

    def factorize(self, stream=None):
        askit_batch_factorize(self.handle, stream)

    def check(self, stream=None):
        return askit_batch_check(self.handle, stream)

    def solve(self, Bs, stream=None):
        return askit_batch_solve(self.handle, Bs, stream)

    def factor_handle(self, i):
        return askit_batch_factor(self.handle, i)

    def close(self):
        askit_batch_destroy(getattr(self, "handle", None))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
