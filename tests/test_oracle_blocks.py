"""Pins for the oracle's building blocks (kernel, sampler, QRCP-ID, LU).

Each test checks the oracle against something other than itself: closed
forms, published generator outputs, LAPACK through scipy, or brute force."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))


# --- Gaussian kernel, eq. (1) ------------------------------------------------

def test_kernel_closed_forms(orc):
    x = np.array([0.3, -1.0, 2.0])
    assert orc.kernel(x, x, 0.7) == 1.0
    # |x - y| = h  ->  exp(-1/2)
    y = x + np.array([0.0, 0.0, 0.7])
    assert abs(orc.kernel(x, y, 0.7) - np.exp(-0.5)) < 1e-15
    # 3-4-5 triangle, h = 5: exp(-25 / 50)
    assert abs(orc.kernel([0.0, 0.0], [3.0, 4.0], 5.0) - np.exp(-0.5)) < 1e-15
    # the two regimes named after eq. (1): h -> 0 gives I, h -> inf gives 1 1^T
    assert orc.kernel([0.0], [1.0], 1e-3) == 0.0
    assert orc.kernel([0.0, 0.0, 0.0], [1.0, 1.0, 1.0], 1e9) == 1.0


def test_kernel_matrix_symmetric_psd(orc):
    rng = np.random.default_rng(1)
    X = rng.uniform(size=(60, 4))
    K = orc.dense_kernel(X, 0.4)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(K) == 1.0)
    assert np.linalg.eigvalsh(K).min() > -1e-12


# --- SplitMix64 and the sampler (reading: uniform rows outside the node) -----

def test_splitmix64_published_outputs(orc):
    with open(os.path.join(HERE, "golden", "splitmix64_seed0.txt")) as f:
        want = [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
    assert orc.splitmix64_stream(0, len(want)) == want


def test_sample_full_complement_when_small(orc):
    q = orc.sample(5, 0, 3, 100, 20, 40, 200)
    assert list(q) == list(range(0, 20)) + list(range(40, 100))


@pytest.mark.parametrize("N,b,e,ns", [(1000, 0, 100, 64), (1000, 900, 1000, 256), (5000, 1234, 1300, 900),
                                      (300, 100, 199, 200)])
def test_sample_invariants(orc, N, b, e, ns):
    q = orc.sample(123, 2, 7, N, b, e, ns)
    assert q.size == min(ns, N - (e - b))
    assert len(set(q.tolist())) == q.size
    assert np.all((q < b) | (q >= e)) and np.all((q >= 0) & (q < N))


def test_sample_first_draw_maps_to_position(orc):
    # first draw r = floor(u c / 2^64) of the node's stream, then q = r or r + n
    N, b, e, seed, prob, node = 10_000, 4000, 4500, 99, 3, 12
    st = orc.node_seed(seed, prob, node)
    # the node's state is output number k = node + 1 + prob 2^32 of SplitMix64(seed)
    k = node + 1 + (prob << 32)
    assert st == orc.splitmix64_stream((seed + (k - 1) * 0x9E3779B97F4A7C15) % (1 << 64), 1)[0]
    assert orc.node_seed(seed, 0, 4) == orc.splitmix64_stream(seed, 5)[4]
    u = orc.splitmix64_stream(st, 1)[0]
    c = N - (e - b)
    r = (u * c) >> 64
    q0 = r if r < b else r + (e - b)
    assert orc.sample(seed, prob, node, N, b, e, 50)[0] == q0


def test_sample_is_uniform(orc):
    # pooled over many nodes, every complement position is hit equally often
    N, b, e, ns = 200, 50, 100, 30
    counts = np.zeros(N)
    for node in range(4000):
        counts[orc.sample(7, 0, node, N, b, e, ns)] += 1
    comp = np.r_[0:b, e:N]
    assert np.all(counts[b:e] == 0)
    expect = 4000 * ns / comp.size
    chi2 = np.sum((counts[comp] - expect) ** 2 / expect)
    # chi-square with 149 dof: mean 149, sd ~17; 5 sd margin
    assert chi2 < 149 + 5 * 17.3


# --- QRCP interpolative decomposition, eq. (4) -------------------------------

def _kernel_block(rng, rows, cols, h):
    Y = rng.uniform(size=(rows, 3)); Xc = rng.uniform(size=(cols, 3))
    d2 = ((Y[:, None, :] - Xc[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / (2 * h * h))


@pytest.mark.parametrize("rows,cols,steps", [(40, 30, 10), (128, 64, 32), (50, 80, 20), (20, 20, 20)])
def test_qrcp_matches_lapack(orc, rows, cols, steps):
    rng = np.random.default_rng(rows * cols)
    M = rng.standard_normal((rows, cols))
    rank, piv, rd, T, R, tr = orc.qrcp(M, steps)
    Q2, R2, P2 = sla.qr(M, pivoting=True, mode="economic")
    assert rank == min(steps, rows, cols) and not tr
    assert list(piv[:rank]) == list(P2[:rank])
    np.testing.assert_allclose(np.abs(rd), np.abs(np.diag(R2)[:rank]), rtol=1e-12)
    np.testing.assert_allclose(np.abs(R[:rank, :rank]), np.abs(R2[:rank, :rank]), rtol=1e-10, atol=1e-12)


def test_qrcp_id_residual_identity(orc):
    # ||M - M[:, skel] P||_F = ||R22||_F  (R22 = trailing block of LAPACK's R)
    rng = np.random.default_rng(3)
    M = _kernel_block(rng, 120, 60, 0.5)
    k = 15
    rank, piv, rd, T, R, tr = orc.qrcp(M, k)
    P = np.zeros((k, 60))
    P[np.arange(k), piv[:k]] = 1.0
    P[:, piv[k:]] = T
    err = np.linalg.norm(M - M[:, piv[:k]] @ P)
    Q2, R2, P2 = sla.qr(M, pivoting=True, mode="economic")
    assert list(P2[:k]) == list(piv[:k])
    r22 = np.linalg.norm(R2[k:, k:])
    assert abs(err - r22) <= 1e-10 * np.linalg.norm(M)
    # T against an independent triangular solve on LAPACK's R
    # (the columns of T follow the trailing pivot order, which is compared by
    # original column index)
    T2 = sla.solve_triangular(R2[:k, :k], R2[:k, k:])
    mine = np.zeros((k, 60)); mine[:, piv[k:]] = T
    lap = np.zeros((k, 60)); lap[:, P2[k:]] = T2
    np.testing.assert_allclose(mine, lap, rtol=1e-8, atol=1e-10)


def test_qrcp_rank_guard(orc):
    rng = np.random.default_rng(4)
    B = rng.standard_normal((30, 3))
    M = B @ rng.standard_normal((3, 12))      # exact rank 3
    rank, piv, rd, T, R, tr = orc.qrcp(M, 8)
    assert rank == 3 and tr
    P = np.zeros((3, 12)); P[np.arange(3), piv[:3]] = 1.0; P[:, piv[3:]] = T
    assert np.linalg.norm(M - M[:, piv[:3]] @ P) < 1e-12 * np.linalg.norm(M)
    # zero matrix: one skeleton column, zero coefficients
    rank, piv, rd, T, R, tr = orc.qrcp(np.zeros((10, 6)), 4)
    assert rank == 1 and piv[0] == 0 and np.all(T == 0)


@pytest.mark.parametrize("tau", [1e-1, 1e-3, 1e-5, 1e-8])
def test_qrcp_adaptive_rank_matches_lapack_diagonal(orc, tau):
    # Sec. 2.1: the rank is the smallest s with sigma_{s+1} / sigma_1 < tau,
    # the singular values estimated by the diagonal of the pivoted QR; the
    # diagonal is LAPACK's (geqp3 through scipy) on a kernel block whose
    # spectrum decays smoothly
    rng = np.random.default_rng(11)
    M = _kernel_block(rng, 200, 90, 0.45)
    Q2, R2, P2 = sla.qr(M, pivoting=True, mode="economic")
    dg = np.abs(np.diag(R2))
    want = int(np.argmax(dg < tau * dg[0])) if np.any(dg < tau * dg[0]) else min(M.shape)
    rank, piv, rd, T, R, tr = orc.qrcp(M, 80, tau)
    assert rank == min(want, 80)
    assert tr == (rank < 80)
    assert list(piv[:rank]) == list(P2[:rank])
    # the ID error is that of the truncated QR: ||M - M_skel P||_2 <= ||R22||_F;
    # and with column pivoting every column of R22 is at most |R_ss| long, so
    # sigma_{s+1}(M) <= ||R22||_2 <= sqrt(n - s) |R_ss|
    P = np.zeros((rank, 90)); P[np.arange(rank), piv[:rank]] = 1.0; P[:, piv[rank:]] = T
    err = np.linalg.norm(M - M[:, piv[:rank]] @ P, 2)
    assert err <= np.linalg.norm(R2[rank:, rank:]) * (1 + 1e-8) + 1e-13 * np.linalg.norm(M)
    sv = np.linalg.svd(M, compute_uv=False)
    if rank < 80:
        assert sv[rank] <= np.sqrt(90 - rank) * dg[rank] * (1 + 1e-8)


def test_qrcp_adaptive_rank_zero_keeps_fixed_rank(orc):
    rng = np.random.default_rng(12)
    M = rng.standard_normal((50, 30))
    a = orc.qrcp(M, 20)
    b = orc.qrcp(M, 20, 0.0)
    assert a[0] == b[0] == 20
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])


def test_qrcp_ties_lowest_column(orc):
    # identical columns: the first pivot is the lowest position among maxima
    M = np.ones((6, 5)); M[:, 3] *= 2.0; M[:, 1] *= 2.0
    rank, piv, *_ = orc.qrcp(M, 1)
    assert piv[0] == 1


# --- LU (GETRF reading) ---------------------------------------------------------

@pytest.mark.parametrize("n", [1, 7, 64, 130])
def test_lu_matches_lapack(orc, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    LU, piv, ratio = orc.lu(A)
    LU2, piv2 = sla.lu_factor(A)
    assert np.array_equal(piv, piv2)
    np.testing.assert_allclose(LU, LU2, rtol=1e-11, atol=1e-12)
    b = rng.standard_normal((n, 3))
    np.testing.assert_allclose(orc.lu_solve(LU, piv, b), np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(orc.lu_solve(LU, piv, b, trans=True), np.linalg.solve(A.T, b), rtol=1e-9,
                               atol=1e-10)
    d = np.abs(np.diag(LU))
    assert ratio == d.min() / d.max()


def test_lu_ties_lowest_row(orc):
    A = np.array([[1.0, 2.0], [-1.0, 5.0]])
    LU, piv, _ = orc.lu(A)
    assert piv[0] == 0
