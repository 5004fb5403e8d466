"""Batched execution: many independent problems of uneven size factorized and
solved with one launch per kernel and tree height, replayed from hipGraphs.
Each problem is checked against its own oracle (1e-10 on the oracle's
skeletons) and against the unbatched GPU path (identical skeletons)."""
import sys

import numpy as np
import pytest

import synth
from gpu_util import colrel, oracle_skeletons

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


def _problems(count=7, nmin=300, nmax=3000):
    """Shapes of the batched workload (log-uniform sizes, 4-cluster mixtures in
    8-D, h ~ U[0.5, 2], lambda ~ 10^U[-1, 0]), scaled down: m = 32, s = 16."""
    probs = synth.batched_problems(count=count, nrhs=3, nmin=nmin, nmax=nmax)
    for p in probs:
        p["m"], p["s"], p["nsamp"] = 32, 16, 64
        p["lam"] = max(p["lam"], 0.1)  # keep every problem well conditioned at this size
    return probs


def test_batched_matches_oracle_and_unbatched(ak, orc):
    import torch
    probs = _problems()
    say(f"[gpu batch] {len(probs)} problems, N = {[len(p['X']) for p in probs]}")
    trees = [ak.Tree(torch.as_tensor(p["X"], device="cuda"), p["m"], p["s"], p["h"], n_samples=p["nsamp"],
                     seed=p["seed"], problem=p["problem"]) for p in probs]
    ak.askit_skeletonize_batched(trees)
    # unbatched skeletons must be identical (same per-node kernels)
    for p, t in zip(probs, trees):
        t2 = ak.Tree(torch.as_tensor(p["X"], device="cuda"), p["m"], p["s"], p["h"], n_samples=p["nsamp"],
                     seed=p["seed"], problem=p["problem"])
        t2.skeletonize()
        a, b = t.export_skeletons(), t2.export_skeletons()
        assert all(np.array_equal(x, y) for x, y in zip(a, b))  # root slots included: both -1
        t2.close()
    # oracle skeletons imported so that the factorization can be compared at 1e-10
    oracles = []
    for p, t in zip(probs, trees):
        o = orc.Oracle(p["X"], p["m"], p["s"], p["h"], nsamp=p["nsamp"], seed=p["seed"], problem=p["problem"])
        o.build_tree()
        o.skeletonize()
        o.factorize(p["lam"])
        t.import_skeletons(*oracle_skeletons(o, t.s, t.cmax))
        oracles.append(o)
    batch = ak.Batch(trees, [p["lam"] for p in probs], ak.ASKIT_FP64, nrhs=3)
    for rep in range(2):  # replay both graphs twice, with host work in between
        batch.factorize()
        xs = batch.solve([torch.as_tensor(p["B"], device="cuda") for p in probs])
        torch.cuda.synchronize()
        for p, o, x in zip(probs, oracles, xs):
            err = colrel(x.cpu().numpy(), o.solve(p["B"]))
            assert err < 1e-10, (rep, len(p["X"]), err)
        ratio, _ = batch.check()
        assert ratio > 1e-12
    # the batched factors are ordinary factors for the other entry points
    f0 = batch.factor_handle(0)
    xt = ak.askit_solve_transpose(f0, torch.as_tensor(probs[0]["B"], device="cuda")).cpu().numpy()
    assert colrel(xt, oracles[0].solve_t(probs[0]["B"])) < 1e-10
    batch.close()
    for t in trees:
        t.close()


def test_batched_mixed_precision(ak):
    """Mixed-precision batch factors.  Both factorizations invert the same
    Ktilde and amplify their rounding through the same reduced systems, so
    the unrefined mixed solve's backward error (relative residual against the
    FP64 operator) is held to 16 x 2^29 (the FP32 / FP64 unit-roundoff ratio)
    times the FP64 solve's; its forward error scales with each problem's
    condition number and is only reported.  Refined against the FP64 operator
    (GMRES-IR on the batch's own factor handles): within 1e-6 of the FP64
    solution."""
    import torch
    probs = _problems(count=4)
    trees = [ak.Tree(torch.as_tensor(p["X"], device="cuda"), p["m"], p["s"], p["h"], n_samples=p["nsamp"],
                     seed=p["seed"], problem=p["problem"]) for p in probs]
    ak.askit_skeletonize_batched(trees)
    b64 = ak.Batch(trees, [p["lam"] for p in probs], ak.ASKIT_FP64, nrhs=3)
    b32 = ak.Batch(trees, [p["lam"] for p in probs], ak.ASKIT_MIXED, nrhs=3)
    b64.factorize()
    b32.factorize()
    Bs = [torch.as_tensor(p["B"], device="cuda") for p in probs]
    x64 = b64.solve(Bs)
    x32 = b32.solve(Bs)
    for i, (a, b) in enumerate(zip(x32, x64)):
        err = colrel(a.cpu().numpy(), b.cpu().numpy())
        op = b64.factor_handle(i)
        rel = lambda x: float(((ak.askit_matvec(op, x) - Bs[i]).norm(dim=0) / Bs[i].norm(dim=0)).max())
        bwd, bwd64 = rel(a), rel(b)
        xr = ak.askit_solve(b32.factor_handle(i), Bs[i])
        info = ak.askit_last_solve_info(b32.factor_handle(i))
        errr = colrel(xr.cpu().numpy(), b.cpu().numpy())
        say(f"  problem {i}: unrefined backward {bwd:.1e} (FP64 {bwd64:.1e}) forward {err:.1e}, refined {errr:.1e} "
            f"({info['iterations']} iterations)")
        assert bwd <= 16 * 2.0 ** 29 * max(bwd64, 2.0 ** -52), (i, bwd, bwd64)
        assert errr <= 1e-6
    b64.close()
    b32.close()


def test_batched_lu_split_graph_replays(ak):
    """The LU with partial pivoting split over launches inside the batch's
    captured graph: reduced systems of up to 320 rows (s = 160), a batch
    with every LU split over launches against one with none; three replays
    of each graph, with eager work between them, give the same solutions bit
    for bit, and the two batches agree bit for bit."""
    import torch
    probs = synth.batched_problems(count=4, nrhs=3, nmin=2000, nmax=6000)
    for p in probs:
        p["m"], p["s"], p["nsamp"] = 128, 160, 320
        p["lam"] = max(p["lam"], 0.1)
    say(f"[gpu batch] LU split in the graph, N = {[len(p['X']) for p in probs]}")
    trees = [ak.Tree(torch.as_tensor(p["X"], device="cuda"), p["m"], p["s"], p["h"], n_samples=p["nsamp"],
                     seed=p["seed"], problem=p["problem"]) for p in probs]
    ak.askit_skeletonize_batched(trees)
    zmax = 0
    for t in trees:
        r = t.skeleton_sizes()[0]
        zmax = max([zmax] + [int(r[2 * i + 1] + r[2 * i + 2]) for i in range((len(r) - 1) // 2)])
    assert zmax > 256
    Bs = [torch.as_tensor(p["B"], device="cuda") for p in probs]
    out = {}
    for n in (512, 0):
        for t in trees:
            t.set_lu_split(n)
        batch = ak.Batch(trees, [p["lam"] for p in probs], ak.ASKIT_FP64, nrhs=3)
        runs = []
        for rep in range(3):
            batch.factorize()
            runs.append([x.cpu().numpy() for x in batch.solve(Bs)])
            torch.cuda.synchronize()
            assert torch.randn(4096, device="cuda").abs().sum().item() > 0  # eager work between replays
        for rep in (1, 2):
            assert all(np.array_equal(a, b) for a, b in zip(runs[0], runs[rep])), (n, rep)
        assert all(np.all(np.isfinite(x)) for x in runs[0])
        ratio, _ = batch.check()
        assert ratio > 1e-12
        out[n] = runs[0]
        batch.close()
    assert all(np.array_equal(a, b) for a, b in zip(out[512], out[0]))
    for t in trees:
        t.close()
