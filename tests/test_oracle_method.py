"""Pins for the oracle's skeletonization, factorization and solves.

The hierarchical approximation Ktilde depends on the tree, the samples and the
pivots, so the factorization is pinned against (a) dense LU of the explicitly
assembled lambda I + Ktilde, (b) special cases where Ktilde is known in closed
form (full rank, h -> 0, h -> infinity), (c) exact identities of the ID, and
(d) the paper's statement that the N log^2 N and N log N schemes build the
same factorization up to roundoff (Sec. 2.2; experiments of Table "speedup")."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth


def _kexact(X, h):
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / (2.0 * h * h))


def _build(orc, X, m, s, h, lam=None, nsamp=None, seed=1, variant=0):
    o = orc.Oracle(X, m, s, h, nsamp=nsamp, seed=seed)
    o.build_tree()
    o.skeletonize()
    if lam is not None:
        o.factorize(lam, variant)
    return o


@pytest.fixture(scope="module")
def c1(orc):
    c = synth.config(1)
    o = _build(orc, c["X"], c["m"], c["s"], c["h"], c["lam"], seed=c["seed"])
    return c, o, o.dense()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --- (a) the factorization inverts the assembled Ktilde ----------------------

def test_solve_inverts_dense_c1(c1):
    c, o, A = c1
    x = o.solve(c["B"])
    assert _rel(x, np.linalg.solve(A, c["B"])) < 1e-10
    assert _rel(x, sla.lu_solve(sla.lu_factor(A), c["B"])) < 1e-10


def test_transpose_solve_dense_c1(c1):
    c, o, A = c1
    g = np.random.default_rng(0).standard_normal((c["X"].shape[0], 2))
    assert _rel(o.solve_t(g), np.linalg.solve(A.T, g)) < 1e-10


def test_matvec_matches_dense_c1(c1):
    c, o, A = c1
    v = np.random.default_rng(1).standard_normal((c["X"].shape[0], 3))
    assert _rel(o.matvec(v), A @ v) < 1e-13


def test_residual_machine_precision_c1(c1):
    # relative residual of eq. (15); the paper prints 5e-12 .. 1e-13 for direct solves
    c, o, A = c1
    x = o.solve(c["B"])
    assert np.linalg.norm(c["B"] - o.matvec(x)) / np.linalg.norm(c["B"]) < 1e-11


def test_ktilde_is_nonsymmetric_c1(c1):
    # with the left-projection form of eq. (6) Ktilde need not be symmetric
    _, _, A = c1
    assert np.abs(A - A.T).max() > 1e-8


def test_skeleton_rows_exact(c1):
    # rows of the skeleton points of l are reproduced exactly in Ktilde_{l r}
    c, o, A = c1
    X, h = c["X"], c["h"]
    perm = o.perm()
    for node in range(0, (1 << o.D) - 1, 5):
        for child, other in ((2 * node + 1, 2 * node + 2), (2 * node + 2, 2 * node + 1)):
            sk = perm[o.skeleton(child)[0]]
            b, e = o.node_range(other)
            cols = perm[b:e]
            d2 = ((X[sk][:, None, :] - X[cols][None, :, :]) ** 2).sum(-1)
            np.testing.assert_allclose(A[np.ix_(sk, cols)], np.exp(-d2 / (2 * h * h)), rtol=0, atol=1e-12)


def test_dense_block_structure_c1(c1):
    # diagonal leaf blocks are exact lambda I + K
    c, o, A = c1
    K = _kexact(c["X"], c["h"])
    perm = o.perm()
    leaf0 = (1 << o.D) - 1
    for leaf in range(leaf0, 2 * leaf0 + 1, 7):
        b, e = o.node_range(leaf)
        ids = perm[b:e]
        np.testing.assert_allclose(A[np.ix_(ids, ids)], K[np.ix_(ids, ids)] + c["lam"] * np.eye(e - b),
                                   rtol=0, atol=1e-14)


@pytest.mark.parametrize("N,d,m,s,h,lam", [(1500, 4, 48, 20, 0.8, 0.05), (2048, 8, 128, 64, 1.5, 0.1)])
def test_solve_inverts_dense_mixture(orc, N, d, m, s, h, lam):
    X, B = synth.small(N, d, N, nrhs=4, kind="mixture", scale=3.0)
    o = _build(orc, X, m, s, h, lam, seed=5)
    A = o.dense()
    assert _rel(o.solve(B), np.linalg.solve(A, B)) < 1e-10
    assert _rel(o.solve_t(B), np.linalg.solve(A.T, B)) < 1e-10


# --- (b) closed forms -------------------------------------------------------

@pytest.mark.parametrize("N,m", [(200, 32), (256, 64), (97, 10)])
def test_full_rank_is_exact(orc, N, m):
    # s >= N/2: every skeleton is its whole candidate set, P = I, Ktilde = K
    X, B = synth.small(N, 3, N, nrhs=2)
    h, lam = 0.3, 0.5
    o = _build(orc, X, m, (N + 1) // 2, h, lam)
    K = _kexact(X, h) + lam * np.eye(N)
    np.testing.assert_allclose(o.dense(), K, rtol=0, atol=1e-15)
    kappa = np.linalg.cond(K)
    assert _rel(o.solve(B), np.linalg.solve(K, B)) < 1e-12 * kappa


def test_two_leaves_full_rank_s_equals_m(orc):
    X, B = synth.small(128, 2, 3, nrhs=1)
    o = _build(orc, X, 64, 64, 0.2, 0.3)
    K = _kexact(X, 0.2) + 0.3 * np.eye(128)
    assert _rel(o.solve(B), np.linalg.solve(K, B)) < 1e-12 * np.linalg.cond(K)


def test_narrow_bandwidth_identity(orc):
    # h so small that every off-diagonal exp underflows: K = I, x = b / (1 + lambda)
    X, B = synth.small(500, 3, 4, nrhs=3)
    lam = 0.25
    o = _build(orc, X, 32, 8, 1e-4, lam)
    x = o.solve(B)
    assert np.array_equal(o.dense(), (1 + lam) * np.eye(500))
    assert np.max(np.abs(x - B / (1 + lam)) / np.abs(B / (1 + lam))) <= 4.5e-16


@pytest.mark.parametrize("s", [1, 3])
def test_wide_bandwidth_rank_one(orc, s):
    # h = 1e9 in the unit cube: K = 1 1^T exactly; Sherman-Morrison closed form
    N, lam = 700, 1.0
    X, B = synth.small(N, 3, 5, nrhs=2)
    o = _build(orc, X, 40, s, 1e9, lam)
    x = o.solve(B)
    want = (B - np.ones((N, 1)) * (B.sum(0) / (lam + N))) / lam
    assert _rel(x, want) < 1e-12
    if s > 1:
        # the rank guard keeps one skeleton point wherever there are more than
        # s candidates; a parent of two rank-1 children has |C| = 2 <= s and
        # keeps both (P = I)
        for n in range(1, o.nnodes):
            sr, nc, tr = o.skel_info(n)
            assert (sr, tr) == ((1, True) if nc > s else (nc, False))


# --- (c) the ID error bounds the error against the true K -------------------

def test_one_level_error_equals_id_residuals(orc):
    # D = 1 and every complement row sampled: Ktilde - K has exactly the two
    # off-diagonal ID residuals, whose norms are ||R22|| of LAPACK's QRCP of
    # K_{r l} and K_{l r}
    N, m, s, h = 160, 80, 12, 0.35
    X, _ = synth.small(N, 3, 9)
    o = _build(orc, X, m, s, h, nsamp=N)
    perm = o.perm()
    K = _kexact(X, h)
    err2 = np.linalg.norm(o.dense() - K) ** 2
    want = 0.0
    for child, other in ((1, 2), (2, 1)):
        b, e = o.node_range(child)
        ob, oe = o.node_range(other)
        M = K[np.ix_(perm[ob:oe], perm[b:e])]
        R = sla.qr(M, pivoting=True, mode="r")[0]
        want += np.linalg.norm(R[s:, s:]) ** 2
    assert abs(err2 - want) <= 1e-10 * np.linalg.norm(K) ** 2


def test_approximation_improves_with_rank(orc):
    # reported, not a closed form: ||K - Ktilde|| / ||K|| at small N
    X, _ = synth.small(1024, 3, 10, kind="mixture", scale=2.0)
    K = _kexact(X, 0.7)
    errs = []
    for s in (4, 16, 48):
        o = _build(orc, X, 64, s, 0.7)
        errs.append(np.linalg.norm(o.dense() - K) / np.linalg.norm(K))
    assert errs[0] > errs[1] > errs[2]


# --- (d) same factorization by the three telescoping forms ------------------

@pytest.mark.parametrize("N,d,m,s,h", [(2048, 3, 64, 32, 0.5), (3000, 6, 100, 40, 1.2)])
def test_telescoping_variants_agree(orc, N, d, m, s, h):
    X, B = synth.small(N, d, N + 1, kind="mixture", scale=2.0)
    lam = 0.2
    outs = []
    for v in (0, 1, 2):
        o = _build(orc, X, m, s, h, lam, seed=3, variant=v)
        outs.append((o, [o.phat(n) for n in range(1, o.nnodes)], o.solve(B)))
    for o, ph, x in outs[1:]:
        for a, b in zip(ph, outs[0][1]):
            assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))
        assert _rel(x, outs[0][2]) < 1e-12


# --- adjoint identity and gradients ---------------------------------------------

def test_adjoint_identity(c1):
    c, o, _ = c1
    rng = np.random.default_rng(2)
    b = rng.standard_normal(c["X"].shape[0]); g = rng.standard_normal(c["X"].shape[0])
    lhs = np.dot(o.solve(b), g)
    rhs = np.dot(b, o.solve_t(g))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-14


def test_gradients_match_finite_differences(orc):
    N, m, s = 1200, 64, 24
    X, B = synth.small(N, 4, 21, nrhs=2, kind="mixture", scale=2.0)
    Y = np.random.default_rng(5).standard_normal(B.shape)
    h, lam = 1.1, 0.5
    o = _build(orc, X, m, s, h, lam)
    loss, x, z, dlam, dh = o.gradient(B, Y)

    def L(bb=B, ll=lam, hh=h):
        o.set_h(hh)
        o.factorize(ll)
        return float(np.sum((o.solve(bb) - Y) ** 2))

    eps = 1e-5
    dirb = np.random.default_rng(6).standard_normal(B.shape)
    fd_b = (L(bb=B + eps * dirb) - L(bb=B - eps * dirb)) / (2 * eps)
    fd_l = (L(ll=lam + eps) - L(ll=lam - eps)) / (2 * eps)
    fd_h = (L(hh=h + eps) - L(hh=h - eps)) / (2 * eps)
    assert abs(fd_b - np.sum(z * dirb)) <= 1e-6 * abs(fd_b)
    assert abs(fd_l - dlam) <= 1e-6 * abs(fd_l)
    assert abs(fd_h - dh) <= 1e-6 * abs(fd_h)


def test_gradient_dense_route(orc):
    # dense oracle: A(h) assembled explicitly (frozen skeletons) and solved by
    # LAPACK; its FD derivative in h and its analytic lambda-derivative
    N, m, s = 800, 50, 20
    X, B = synth.small(N, 3, 22, nrhs=1)
    Y = np.random.default_rng(7).standard_normal(B.shape)
    h, lam = 0.6, 0.1
    o = _build(orc, X, m, s, h, lam)
    loss, x, z, dlam, dh = o.gradient(B, Y)

    def Ld(hh):
        o.set_h(hh)
        A = o.dense()
        return float(np.sum((np.linalg.solve(A, B) - Y) ** 2)), A

    (lp, _), (lm, _) = Ld(h + 1e-5), Ld(h - 1e-5)
    l0, A = Ld(h)
    xd = np.linalg.solve(A, B)
    zd = np.linalg.solve(A.T, 2 * (xd - Y))
    assert abs(l0 - loss) <= 1e-9 * loss
    assert abs(-np.sum(zd * xd) - dlam) <= 1e-9 * abs(dlam)
    assert abs((lp - lm) / 2e-5 - dh) <= 1e-6 * abs(dh)
    # dense dKtilde/dh against the matvec form
    o.factorize(lam)
    assert _rel(o.matvec(x, which=1), o.dense(1) @ x) < 1e-13


# --- stability detection (Sec. 3, "Stability") ------------------------------

def test_instability_is_detected(orc):
    # wide bandwidth and tiny lambda: the leaf blocks lambda I + K_aa are
    # numerically singular and the pivot ratio flags it
    X, _ = synth.small(512, 3, 30)
    o = _build(orc, X, 64, 8, 50.0, 1e-13)
    leaf0 = (1 << o.D) - 1
    assert min(o.pivratio(n) for n in range(leaf0, o.nnodes)) < 1e-12
    o2 = _build(orc, X, 64, 8, 0.3, 1.0)
    assert min(o2.pivratio(n) for n in range(o2.nnodes)) > 1e-6


# --- level restriction and the hybrid solver (Sec. 2.3) ---------------------

def _hybrid_case(orc):
    X, B = synth.small(2000, 3, 7, nrhs=3, kind="mixture", scale=2.0)
    o = orc.Oracle(X, 64, 24, 0.6, seed=3)
    o.build_tree()
    o.skeletonize()
    return o, B, 0.3


def test_hybrid_level_one_is_the_full_method(orc):
    # the root has no skeleton, so a frontier at level 1 leaves the matrix of
    # the full method unchanged (only the root's Z changes hands: from a
    # direct node step to the reduced system I + V W of order s_l + s_r)
    o, B, lam = _hybrid_case(orc)
    o.factorize(lam)
    x0, A0, y0 = o.solve(B), o.dense(), o.matvec(B)
    o.set_level(1)
    o.factorize(lam)
    assert np.array_equal(o.dense(), A0)
    assert np.array_equal(o.matvec(B), y0)
    assert _rel(o.solve(B), x0) < 1e-13


@pytest.mark.parametrize("L", [2, 3, 5])
def test_hybrid_solve_inverts_the_restricted_matrix(orc, L):
    # HybridSolve against LAPACK on the assembled level-restricted
    # lambda I + Ktilde; the reduced system has order sum_a s_a <= 2^L s
    o, B, lam = _hybrid_case(orc)
    o.set_level(L)
    o.factorize(lam)
    A = o.dense()
    xd = sla.solve(A, B)
    assert _rel(o.solve(B), xd) < 1e-11
    assert _rel(o.matvec(B), A @ B) < 1e-13
    M, ratio = o.reduced_system()
    ranks = [o.skel_info(n)[0] for n in range((1 << L) - 1, (2 << L) - 1)]
    assert M == sum(ranks) <= (1 << L) * 24
    assert ratio > 1e-6
    # nothing is compressed above the frontier: the blocks between two
    # frontier nodes are P_{a a~} K_{a~ b}, one skeleton deep, so a frontier
    # lower in the tree approximates K less and less (no error is added above)
    K = orc.dense_kernel(o.X, o.h) + lam * np.eye(o.N)
    errs = []
    for LL in (1, L):
        o.set_level(LL)
        errs.append(np.linalg.norm(o.dense() - K))
    assert errs[1] <= errs[0] * (1 + 1e-12)


def test_hybrid_has_no_transpose_solve(orc):
    o, B, lam = _hybrid_case(orc)
    o.set_level(2)
    o.factorize(lam)
    with pytest.raises(RuntimeError):
        o.solve_t(B)
