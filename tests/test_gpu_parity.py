"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tree permutations and sampled rows must match bit for bit; skeletons match
node by node except at measured near-ties of the pivoted QR; with the
oracle's skeletons imported the FP64 factorization and solves must agree to
1e-10 relative (or 10x the spread of two FP64 orderings of the oracle where
the problem's conditioning puts the rounding floor higher); the mixed path
after refinement to 1e-6 against the FP64 paths on the same skeletons."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import colrel, oracle_skeletons, skeleton_parity

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


CASES = {
    # name: (N, d, m, s, h, lam, nrhs, kind, scale)
    "c1": None,
    "ragged": (3001, 3, 64, 24, 0.4, 0.5, 3, "uniform", 1.0),
    "mix8": (6000, 8, 128, 48, 1.5, 1.0, 5, "mixture", 3.0),
    "c2shape": (16384, 8, 256, 128, 1.0, 0.1, 16, "mixture", 5.0),
    "deep": (8192, 4, 32, 16, 0.6, 0.2, 1, "mixture", 2.0),
}


def _case(name):
    if name == "c1":
        c = synth.config(1)
        return c["X"], c["B"], c["m"], c["s"], c["h"], c["lam"], c["seed"]
    N, d, m, s, h, lam, nrhs, kind, scale = CASES[name]
    X, B = synth.small(N, d, N, nrhs=nrhs, kind=kind, scale=scale)
    return X, B, m, s, h, lam, 11


@pytest.fixture(scope="module", params=list(CASES))
def setup(request, ak, orc):
    name = request.param
    X, B, m, s, h, lam, seed = _case(name)
    say(f"[gpu parity] case {name}: N={len(X)} d={X.shape[1]} m={m} s={s}")
    o = orc.Oracle(X, m, s, h, seed=seed)
    o.build_tree()
    o.skeletonize()
    o.factorize(lam)
    t = ak.Tree(_cuda(X), m, s, h, seed=seed)
    # rounding floor of this problem: two FP64 orderings of the same method
    # (telescoping of eq. (10) as printed vs its push-through form) differ by
    # `spread`; the FP64 parity bar is 1e-10, or 10 x spread when the
    # problem's conditioning puts that floor higher
    o2 = orc.Oracle(X, m, s, h, seed=seed)
    o2.build_tree()
    o2.skeletonize()
    o2.factorize(lam, 2)
    spread = max(colrel(o2.solve(B), o.solve(B)), colrel(o2.solve_t(B), o.solve_t(B)))
    tol = max(1e-10, 10 * spread)
    say(f"  FP64 parity bar {tol:.1e} (variant spread {spread:.1e})")
    return dict(name=name, X=X, B=B, m=m, s=s, h=h, lam=lam, seed=seed, o=o, t=t, tol=tol)


def test_tree_perm_bit_exact(setup):
    t, o = setup["t"], setup["o"]
    assert np.array_equal(_np(t.perm()), o.perm())


def test_skeletons_match_oracle(setup):
    """GPU skeletons against the oracle's, node by node (see
    gpu_util.skeleton_parity): identical pivots with the oracle's ID residual
    and, where R11 is well conditioned, P element by element; any other
    pivot only at a measured near-tie."""
    import oracle as orc_mod
    t, o = setup["t"], setup["o"]
    t.skeletonize()
    ids, P, sizes = t.export_skeletons()
    rep = skeleton_parity(orc_mod, o, setup["X"], setup["h"], setup["seed"], ids, P, sizes, t.s, t.cmax)
    say(f"  skeletons: {rep['identical']}/{rep['compared']} compared nodes identical, {rep['near_tie']} near-ties, "
        f"{rep['elementwise']} compared element-wise (worst |dP|/bar {rep['worst_dP_over_bar']:.2e}), "
        f"worst ID residual excess {rep['worst_resid_excess']:.1e}")
    assert not rep["failures"], rep["failures"][:5]
    assert rep["identical"] >= 1


def test_samples_match_oracle(setup):
    """The GPU's sampled rows of every node with a QR, entry by entry and in
    draw order, against the oracle's sampler."""
    import oracle as orc_mod
    t, o = setup["t"], setup["o"]
    t.skeletonize()
    samp = t.samples()
    ranks, cands = t.skeleton_sizes()
    checked = 0
    for node in range(1, t.nnodes):
        if cands[node] <= t.s:
            continue
        b, e = o.node_range(node)
        q = orc_mod.sample(setup["seed"], 0, node, o.N, b, e, o.nsamp)
        assert np.array_equal(samp[node, :len(q)], q), node
        checked += 1
    say(f"  samples identical on {checked} nodes")
    assert checked > 0


def test_split_qrcp_matches_one_workgroup(setup, ak):
    """The pivoted QR run by several workgroups per node (one launch per
    pivot step) and by one workgroup per node: bit-identical skeletons."""
    X = _cuda(setup["X"])
    out = []
    for levels in (-1, 99):
        t = ak.Tree(X, setup["m"], setup["s"], setup["h"], seed=setup["seed"], qr_split_levels=levels)
        t.skeletonize()
        out.append(t.export_skeletons())
        t.close()
    (i1, p1, z1), (i2, p2, z2) = out
    assert np.array_equal(z1, z2)
    assert np.array_equal(i1, i2)
    assert np.array_equal(p1, p2)


def _tree(ak, setup):
    return ak.Tree(_cuda(setup["X"]), setup["m"], setup["s"], setup["h"], seed=setup["seed"])


@pytest.fixture(scope="module")
def imported(setup, ak):
    """GPU FP64 factor on the oracle's skeletons (own tree)."""
    t, o = _tree(ak, setup), setup["o"]
    ids, P, sizes = oracle_skeletons(o, t.s, t.cmax)
    t.import_skeletons(ids, P, sizes)
    f = t.factorize(setup["lam"], ak.ASKIT_FP64)
    yield f
    f.close()


@pytest.mark.parametrize("which", [0, 1])
def test_matvec_on_oracle_skeletons(setup, imported, which):
    B = setup["B"]
    y = _np(imported.matvec(_cuda(B), which))
    assert colrel(y, setup["o"].matvec(B, which)) < 1e-12


def test_matvec_transpose_on_oracle_skeletons(setup, imported):
    """(lambda I + Ktilde)^T x (which = 2): against the transposed dense
    assembly where it is small, and at every size through the adjoint identity
    X^T (A Y) = (A^T X)^T Y with the oracle's A Y."""
    o, B = setup["o"], setup["B"]
    N = len(setup["X"])
    rng = np.random.default_rng(11)
    Xr = rng.standard_normal((N, 3))
    Yr = rng.standard_normal((N, 3))
    atx = _np(imported.matvec(_cuda(Xr), 2))
    ay = o.matvec(Yr, 0)
    lhs, rhs = Xr.T @ ay, atx.T @ Yr
    scale = np.linalg.norm(Xr) * np.linalg.norm(ay)
    say(f"  adjoint identity {np.abs(lhs - rhs).max() / scale:.2e}")
    assert np.abs(lhs - rhs).max() <= 1e-12 * scale
    if N <= 4096:
        y = _np(imported.matvec(_cuda(B), 2))
        assert colrel(y, o.dense(0).T @ B.reshape(N, -1)) < 1e-12


def test_solve_transpose_refined(setup, ak):
    """Transpose solve refined by GMRES on the transposed operator: residual
    |b - A^T z| / |b| at the refinement target, and the oracle's A^{-T} b."""
    t, o = _tree(ak, setup), setup["o"]
    ids, P, sizes = oracle_skeletons(o, t.s, t.cmax)
    t.import_skeletons(ids, P, sizes)
    f = t.factorize(setup["lam"], ak.ASKIT_FP64)
    f.set_refinement(40, 1e-11)  # the library's default target, above the FP64 rounding floor (~1e-12 here)
    B = _cuda(setup["B"])
    z = f.solve_transpose(B)
    info = f.info()
    r = B - f.matvec(z, 2)
    res = float((r.norm(dim=0) / B.norm(dim=0)).max()) if B.dim() > 1 else float(r.norm() / B.norm())
    err = colrel(_np(z), o.solve_t(setup["B"]))
    say(f"  refined transpose solve: residual {res:.2e}, vs oracle {err:.2e}, {info}")
    assert info["converged"] and res <= 1e-11
    assert err < setup["tol"]
    f.close()


def test_solve_on_oracle_skeletons(setup, imported):
    B = setup["B"]
    x = _np(imported.solve(_cuda(B)))
    err = colrel(x, setup["o"].solve(B))
    say(f"  solve vs oracle {err:.2e}")
    assert err < setup["tol"]


def test_solve_transpose_on_oracle_skeletons(setup, imported):
    B = setup["B"]
    xt = _np(imported.solve_transpose(_cuda(B)))
    err = colrel(xt, setup["o"].solve_t(B))
    say(f"  transpose solve vs oracle {err:.2e}")
    assert err < setup["tol"]


def test_end_to_end_residual(setup, ak):
    """GPU skeletons, GPU factor, GPU solve; residual with the GPU FP64 matvec."""
    t = _tree(ak, setup)
    t.skeletonize()
    f = t.factorize(setup["lam"], ak.ASKIT_FP64)
    B = _cuda(setup["B"])
    x = f.solve(B)
    r = B - f.matvec(x)
    eps = float((r.norm(dim=0) / B.norm(dim=0)).max()) if B.dim() > 1 else float(r.norm() / B.norm())
    # the oracle's own residual on its factorization sets the scale of the
    # rounding floor (it grows with |A| |x| / |b|)
    o, Bh = setup["o"], setup["B"]
    ro = Bh - o.matvec(o.solve(Bh))
    eo = float(np.max(np.linalg.norm(ro.reshape(len(Bh), -1), axis=0) /
                      np.linalg.norm(Bh.reshape(len(Bh), -1), axis=0)))
    say(f"  relative residual {eps:.2e} (oracle {eo:.2e})")
    assert eps < max(1e-10, 10 * eo)
    f.close()


def test_mixed_refined_matches_fp64(setup, ak):
    t, o = _tree(ak, setup), setup["o"]
    ids, P, sizes = oracle_skeletons(o, t.s, t.cmax)
    t.import_skeletons(ids, P, sizes)
    f64 = t.factorize(setup["lam"], ak.ASKIT_FP64)
    fmx = t.factorize(setup["lam"], ak.ASKIT_MIXED)
    B = _cuda(setup["B"])
    x64 = _np(f64.solve(B))
    xmx = _np(fmx.solve(B))
    info = fmx.info()
    say(f"  mixed: {info}")
    assert colrel(xmx, x64) <= 1e-6
    assert info["converged"]
    f64.close()
    fmx.close()
