"""Reference oracle for the N log N hierarchical kernel solver (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It wraps the plain-C FP64 library ``libaskit_oracle.so``
(built from ``askit_oracle.c`` by :func:`build`) with ctypes and numpy; it never
touches the GPU library and shares no code with it.

Paper: Yu, March & Biros, "An N log N Parallel Fast Direct Solver for Kernel
Matrices", arXiv:1701.02324.  Section, equation and algorithm numbers below
refer to that paper.

Every function here follows a passage of the paper; the pins that hold each one
to the paper and to the mathematics live in ``tests/test_oracle_*.py``.
Parity status per function: every function is pinned (see those tests).
How close the hierarchical approximation is to the exact kernel is a
property of the method's inputs, not of an oracle function; it is measured
and reported, not gated.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "askit_oracle.c")
_LIB = os.path.join(_HERE, "libaskit_oracle.so")

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_new.restype = ctypes.c_void_p
        L.orc_new.argtypes = [_dp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_uint64, _i64, ctypes.c_double]
        L.orc_free.argtypes = [ctypes.c_void_p]
        for f in ("orc_build_tree", "orc_skeletonize"):
            getattr(L, f).argtypes = [ctypes.c_void_p]
            getattr(L, f).restype = ctypes.c_int
        L.orc_get_depth.argtypes = [ctypes.c_void_p]
        L.orc_set_h.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_set_tol.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_set_level.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_reduced_ratio.argtypes = [ctypes.c_void_p]
        L.orc_reduced_ratio.restype = ctypes.c_double
        L.orc_reduced_order.argtypes = [ctypes.c_void_p]
        L.orc_reduced_order.restype = _i64
        L.orc_get_perm.argtypes = [ctypes.c_void_p, _lp]
        L.orc_node_range.argtypes = [ctypes.c_void_p, _i64, _lp, _lp]
        L.orc_skel_info.argtypes = [ctypes.c_void_p, _i64, _ip, _ip, _ip]
        L.orc_skel_get.argtypes = [ctypes.c_void_p, _i64, _lp, _dp]
        L.orc_skel_set.argtypes = [ctypes.c_void_p, _i64, ctypes.c_int, _lp, _dp]
        L.orc_factorize.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        L.orc_get_phat.argtypes = [ctypes.c_void_p, _i64, _dp]
        L.orc_block_size.argtypes = [ctypes.c_void_p, _i64]
        L.orc_get_lu.argtypes = [ctypes.c_void_p, _i64, _dp, _ip]
        L.orc_pivratio.argtypes = [ctypes.c_void_p, _i64]
        L.orc_pivratio.restype = ctypes.c_double
        for f in ("orc_solve", "orc_solve_t"):
            getattr(L, f).argtypes = [ctypes.c_void_p, _dp, _i64, ctypes.c_int, _dp, _i64]
            getattr(L, f).restype = ctypes.c_int
        L.orc_matvec.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _i64, ctypes.c_int, _dp, _i64]
        L.orc_dense.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.orc_kernel.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_double]
        L.orc_kernel.restype = ctypes.c_double
        L.orc_kernel_matrix.argtypes = [_dp, ctypes.c_int, ctypes.c_double, _lp, _i64, _lp, _i64, _dp]
        L.orc_qrcp.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, _ip]
        L.orc_qrcp_tol.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip, _dp, _dp,
                                   _ip]
        L.orc_lu.argtypes = [_dp, ctypes.c_int, _ip]
        L.orc_lu.restype = ctypes.c_double
        L.orc_lu_solve.argtypes = [_dp, _ip, ctypes.c_int, _dp, ctypes.c_int]
        L.orc_lu_solve_t.argtypes = [_dp, _ip, ctypes.c_int, _dp, ctypes.c_int]
        L.orc_splitmix64.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_node_seed.argtypes = [ctypes.c_uint64, _i64, _i64]
        L.orc_node_seed.restype = ctypes.c_uint64
        L.orc_sample.argtypes = [ctypes.c_uint64, _i64, _i64, _i64, _i64, _i64, ctypes.c_int, _lp]
        L.orc_sample.restype = _i64
        L.orc_sample_prefix.argtypes = [ctypes.c_uint64, _i64, _i64, _i64, _i64, _i64, ctypes.c_int, _lp, _i64,
                                        _lp]
        L.orc_sample_prefix.restype = _i64
        L.orc_set_knn.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_knn.restype = ctypes.c_int
        L.orc_get_knn.argtypes = [ctypes.c_void_p, _lp]
        L.orc_node_nbr.argtypes = [ctypes.c_void_p, _i64, _lp, _lp]
        L.orc_node_nbr.restype = _i64
        L.orc_knn_rows.argtypes = [ctypes.c_void_p, _i64, _i64, ctypes.c_int, _lp]
        L.orc_subtree_sample.argtypes = [ctypes.c_void_p, _i64, ctypes.c_int, _lp, _lp, _lp, _lp]
        L.orc_subtree_sample.restype = _i64
        L.orc_node_sample.argtypes = [ctypes.c_void_p, _i64, _lp]
        L.orc_node_sample.restype = _i64
        L.orc_depth.argtypes = [_i64, ctypes.c_int]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _l(a):
    return a.ctypes.data_as(_lp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# Stand-alone building blocks
# ----------------------------------------------------------------------------

def kernel(x, y, h):
    """Gaussian kernel of eq. (1) between two points."""
    x = _f64c(x); y = _f64c(y)
    return lib().orc_kernel(_d(x), _d(y), x.size, h)


def kernel_matrix(X, h, I, J):
    """K(X_I, X_J) by eq. (1), direct differences."""
    X = _f64c(X)
    I = np.ascontiguousarray(I, dtype=np.int64); J = np.ascontiguousarray(J, dtype=np.int64)
    out = np.empty((I.size, J.size))
    lib().orc_kernel_matrix(_d(X), X.shape[1], h, _l(I), I.size, _l(J), J.size, _d(out))
    return out


def qrcp(M, steps, tau=0.0):
    """Column-pivoted Householder QR used for the ID of eq. (4), stopped after
    `steps` steps, at the rank guard, or (tau > 0) at the first |R_jj| <
    tau |R_00| (adaptive rank, Sec. 2.1).

    Returns (rank, piv, Rdiag, T, R, truncated) with T = R11^{-1} R12 and R the
    upper-trapezoidal factor (rank x cols, columns in pivot order)."""
    M = np.asarray(M, dtype=np.float64)
    rows, cols = M.shape
    A = np.asfortranarray(M).copy(order="F")
    piv = np.zeros(cols, dtype=np.int32)
    rd = np.zeros(max(cols, 1))
    T = np.zeros(max(steps, 1) * max(cols, 1))
    tr = np.zeros(1, dtype=np.int32)
    buf = A.ravel(order="F")
    rank = lib().orc_qrcp_tol(_d(buf), rows, cols, steps, float(tau), _i(piv), _d(rd), _d(T), _i(tr))
    A = buf.reshape((rows, cols), order="F")
    R = np.triu(A[:rank, :])
    Tm = T[: rank * (cols - rank)].reshape(rank, cols - rank)
    return rank, piv.astype(np.int64), rd[:rank].copy(), Tm, R, bool(tr[0])


def lu(A):
    """Partial-pivoting LU (GETRF reading): returns (LU, piv, min|Uii|/max|Uii|)."""
    A = _f64c(A).copy()
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    ratio = lib().orc_lu(_d(A), n, _i(piv))
    return A, piv, ratio


def lu_solve(LU, piv, B, trans=False):
    LU = _f64c(LU); piv = np.ascontiguousarray(piv, dtype=np.int32)
    B = _f64c(B).copy()
    vec = B.ndim == 1
    if vec:
        B = B[:, None].copy()
    f = lib().orc_lu_solve_t if trans else lib().orc_lu_solve
    f(_d(LU), _i(piv), LU.shape[0], _d(B), B.shape[1])
    return B[:, 0] if vec else B


def splitmix64_stream(state, n):
    """n successive SplitMix64 outputs starting from the given state."""
    st = ctypes.c_uint64(state)
    return [lib().orc_splitmix64(ctypes.byref(st)) for _ in range(n)]


def node_seed(seed, problem, node):
    return lib().orc_node_seed(seed, problem, node)


def sample(seed, problem, node, N, b, e, nsamp):
    """Sampled complement rows S' of node [b,e) (positions in tree order)."""
    q = np.zeros(max(nsamp, 1), dtype=np.int64)
    k = lib().orc_sample(seed, problem, node, N, b, e, nsamp, _l(q))
    return q[:k].copy()


def sample_prefix(seed, problem, node, N, b, e, nsamp, pre):
    """S' of node [b,e) opened by the positions pre (distinct, outside the
    node), filled by uniform draws."""
    pre = np.ascontiguousarray(pre, dtype=np.int64)
    q = np.zeros(max(nsamp, 1), dtype=np.int64)
    k = lib().orc_sample_prefix(seed, problem, node, N, b, e, nsamp, _l(pre), pre.size, _l(q))
    return q[:k].copy()


def depth(N, m):
    return lib().orc_depth(N, m)


def num_threads():
    return lib().orc_num_threads()


# ----------------------------------------------------------------------------
# The whole method on one problem
# ----------------------------------------------------------------------------

class Oracle:
    """Tree, skeletons, factorization and solves of one problem, in FP64.

    Steps: build_tree (Sec. 2.1 partitioning) -> skeletonize (Alg. 1) ->
    factorize (Alg. 2) -> solve (Alg. 3); plus the transpose solve, the
    hierarchical matvec and the dense assembly of lambda I + Ktilde."""

    def __init__(self, X, m, s, h, nsamp=None, seed=0, problem=0, tol=0.0):
        X = _f64c(X)
        if X.ndim != 2:
            raise ValueError("X must be N x d")
        self.X = X
        self.N, self.d = X.shape
        self.m, self.s, self.h = int(m), int(s), float(h)
        self.nsamp = int(nsamp) if nsamp else 4 * self.s
        self.seed, self.problem = int(seed), int(problem)
        self._h = lib().orc_new(_d(X), self.N, self.d, self.m, self.s, self.nsamp,
                                ctypes.c_uint64(self.seed & 0xFFFFFFFFFFFFFFFF), self.problem, self.h)
        if not self._h:
            raise ValueError("invalid oracle arguments")
        self.tol = float(tol)
        if lib().orc_set_tol(self._h, self.tol):
            raise ValueError("tol must be in [0, 1)")
        self.D = lib().orc_get_depth(self._h)
        self.lam = None
        self.kappa = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def set_h(self, h):
        """New bandwidth with the same tree and skeletons (drops the factorization)."""
        if lib().orc_set_h(self._h, float(h)):
            raise ValueError("h must be positive")
        self.h = float(h)

    # tree ------------------------------------------------------------------
    def build_tree(self):
        lib().orc_build_tree(self._h)
        return self.perm()

    def perm(self):
        p = np.zeros(self.N, dtype=np.int64)
        lib().orc_get_perm(self._h, _l(p))
        return p

    def node_range(self, node):
        b = ctypes.c_int64(); e = ctypes.c_int64()
        lib().orc_node_range(self._h, node, ctypes.byref(b), ctypes.byref(e))
        return b.value, e.value

    @property
    def nnodes(self):
        return (2 << self.D) - 1

    # kappa-nearest-neighbour sampling --------------------------------------------
    def set_knn(self, kappa):
        """Neighbours of every point and the ranked neighbour list of every
        node; the next skeletonize() samples each node's list first, then
        uniform rows.  kappa = 0: uniform rows only."""
        rc = lib().orc_set_knn(self._h, int(kappa))
        if rc:
            raise ValueError(f"set_knn failed ({rc})")
        self.kappa = int(kappa)

    def knn(self):
        """N x kappa nearest positions of every position (tree order), -1 padded."""
        out = np.zeros((self.N, self.kappa), dtype=np.int64)
        lib().orc_get_knn(self._h, _l(out))
        return out

    def knn_rows(self, b, e, kappa):
        """Neighbours of the positions [b, e) only (brute force against all N)."""
        out = np.zeros((e - b, kappa), dtype=np.int64)
        lib().orc_knn_rows(self._h, b, e, int(kappa), _l(out))
        return out

    def node_neighbors(self, node):
        """(positions, weights) of a node's ranked neighbour list."""
        pos = np.zeros(self.nsamp, dtype=np.int64); w = np.zeros(self.nsamp, dtype=np.int64)
        n = lib().orc_node_nbr(self._h, node, _l(pos), _l(w))
        return pos[:n].copy(), w[:n].copy()

    def node_sample(self, node):
        """The sampled rows S' the next skeletonize() uses for a node."""
        q = np.zeros(self.nsamp, dtype=np.int64)
        k = lib().orc_node_sample(self._h, node, _l(q))
        return q[:k].copy()

    def subtree_sample(self, node, kappa):
        """(list positions, list weights, S') of a node computed from its
        subtree alone: the same as set_knn(kappa) + node_neighbors/node_sample
        at the cost of n_node x N distances."""
        pos = np.zeros(self.nsamp, dtype=np.int64); w = np.zeros(self.nsamp, dtype=np.int64)
        q = np.zeros(self.nsamp, dtype=np.int64); nl = np.zeros(1, dtype=np.int64)
        k = lib().orc_subtree_sample(self._h, node, int(kappa), _l(pos), _l(w), _l(nl), _l(q))
        n = int(nl[0])
        return pos[:n].copy(), w[:n].copy(), q[:k].copy()

    # skeletons ---------------------------------------------------------------
    def skeletonize(self):
        rc = lib().orc_skeletonize(self._h)
        if rc:
            raise RuntimeError(f"oracle skeletonize failed ({rc})")

    def skel_info(self, node):
        a = ctypes.c_int(); b = ctypes.c_int(); c = ctypes.c_int()
        lib().orc_skel_info(self._h, node, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, bool(c.value)

    def skeleton(self, node):
        """(skeleton positions, P_{alpha~ C} as s_alpha x |C|, truncated flag)."""
        sr, nc, tr = self.skel_info(node)
        pos = np.zeros(sr, dtype=np.int64)
        P = np.zeros((sr, nc))
        lib().orc_skel_get(self._h, node, _l(pos), _d(P))
        return pos, P, tr

    def set_skeleton(self, node, pos, P):
        pos = np.ascontiguousarray(pos, dtype=np.int64); P = _f64c(P)
        rc = lib().orc_skel_set(self._h, node, pos.size, _l(pos), _d(P))
        if rc:
            raise ValueError("bad skeleton")

    def candidates(self, node):
        """Candidate positions C of a node: its points (leaf) or [l~ r~]."""
        lvl = int(np.floor(np.log2(node + 1)))
        if lvl == self.D:
            b, e = self.node_range(node)
            return np.arange(b, e, dtype=np.int64)
        return np.concatenate([self.skeleton(2 * node + 1)[0], self.skeleton(2 * node + 2)[0]])

    # level restriction (hybrid solver, Sec. 2.3) ------------------------------
    def set_level(self, L):
        """Frontier at level L (0: the full method).  Above it nothing is
        compressed; factorize() then factors the frontier's subtrees and the
        reduced system I + V W, solve() runs HybridSolve, matvec() and
        dense() apply that matrix."""
        if lib().orc_set_level(self._h, int(L)):
            raise ValueError("level must be in [0, D]")
        self.level = int(L)

    def reduced_system(self):
        """(order of I + V W, its pivot ratio) after a factorization with a level restriction."""
        return lib().orc_reduced_order(self._h), lib().orc_reduced_ratio(self._h)

    # factorization -----------------------------------------------------------
    def factorize(self, lam, variant=0):
        """variant 0: eq. (10) through Solve(alpha, W P_c, false) (Alg. 2);
        1: full subtree solve (N log^2 N scheme); 2: push-through W Z^{-1} P_c."""
        rc = lib().orc_factorize(self._h, float(lam), int(variant))
        if rc:
            raise RuntimeError(f"oracle factorize failed ({rc})")
        self.lam = float(lam)

    def phat(self, node):
        b, e = self.node_range(node)
        sr = self.skel_info(node)[0]
        out = np.zeros((e - b, sr))
        lib().orc_get_phat(self._h, node, _d(out))
        return out

    def block_lu(self, node):
        n = lib().orc_block_size(self._h, node)
        out = np.zeros((n, n)); piv = np.zeros(n, dtype=np.int32)
        lib().orc_get_lu(self._h, node, _d(out), _i(piv))
        return out, piv

    def pivratio(self, node):
        return lib().orc_pivratio(self._h, node)

    def _cols(self, B):
        B = np.asarray(B, dtype=np.float64)
        vec = B.ndim == 1
        Bf = np.asfortranarray(B[:, None] if vec else B)
        return Bf, vec

    def _apply(self, fn, B, *extra):
        Bf, vec = self._cols(B)
        N, nrhs = Bf.shape
        out = np.zeros((N, nrhs), order="F")
        rc = fn(self._h, *extra, _d(Bf), N, nrhs, _d(out), N)
        if rc:
            raise RuntimeError(f"oracle call failed ({rc})")
        return out[:, 0] if vec else np.ascontiguousarray(out)

    def solve(self, B):
        """(lambda I + Ktilde)^{-1} B (Alg. 3), B in original point order."""
        return self._apply(lib().orc_solve, B)

    def solve_t(self, B):
        """(lambda I + Ktilde)^{-T} B."""
        return self._apply(lib().orc_solve_t, B)

    def matvec(self, B, which=0):
        """(lambda I + Ktilde) B (which=0) or dKtilde/dh B (which=1)."""
        return self._apply(lib().orc_matvec, B, int(which))

    def dense(self, which=0):
        A = np.zeros((self.N, self.N))
        rc = lib().orc_dense(self._h, int(which), _d(A))
        if rc:
            raise RuntimeError("dense assembly needs skeletons")
        return A

    def gradient(self, B, Y):
        """Adjoint gradient of L = sum_j ||x_j - y_j||^2 with x = A^{-1} b,
        A = lambda I + Ktilde:  z = A^{-T} 2(x - y);  dL/db = z;
        dL/dlambda = -sum z.x;  dL/dh = -sum z.(dKtilde/dh x)."""
        x = self.solve(B)
        z = self.solve_t(2.0 * (x - np.asarray(Y, dtype=np.float64)))
        dlam = -float(np.sum(z * x))
        dh = -float(np.sum(z * self.matvec(x, which=1)))
        loss = float(np.sum((x - Y) ** 2))
        return loss, x, z, dlam, dh


def dense_kernel(X, h):
    """The exact kernel matrix K of eq. (1) (small N only)."""
    X = _f64c(X)
    idx = np.arange(X.shape[0], dtype=np.int64)
    return kernel_matrix(X, h, idx, idx)
