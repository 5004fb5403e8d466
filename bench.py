#!/usr/bin/env python3
"""Benchmark of the hierarchical kernel solver on one MI355X.

Workload (the paper's N log N scaling shape, m = 512, s = 256, on a synthetic
Gaussian mixture in place of its datasets): N = 1,048,576 points in 16-D, 32
clusters with centres ~ U[-10,10]^16 and sigma ~ U[0.5,2]; h = 2, lambda = 0.01,
64 right-hand sides ~ N(0,1).

One step = skeletonize (sampled ID, FP64 QRCP) + factorize (mixed precision:
FP32 kernel blocks and level products, FP64 LUs), as the one pipelined call
askit_skeletonize_factorize, + solve of the 64 right-hand sides with iterative
refinement against the FP64 operator.  Inputs are resident in HBM before the
timed region; the tree is built once, outside it.

Printed: one JSON line.  value = factor time (skeletonize + factorize) of the
mixed path in seconds; the same step through the two separate calls, solves/s,
the plain FP64 path (timed once after the steps), the mixed-vs-FP64 relative
error, the roofline of the dominant kernel (per-kernel HIP-event timings) and
the oracle CPU baseline are included.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N=1M d=16 s=256: factor time (s), solves/s; mixed vs FP64 at rel err≤1e-6"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def node_sizes(N, D):
    """Points per heap node of the complete tree (left child gets floor(n/2))."""
    n = np.zeros((2 << D) - 1, dtype=np.int64)
    n[0] = N
    for i in range((1 << D) - 1):
        n[2 * i + 1] = n[i] // 2
        n[2 * i + 2] = n[i] - n[i] // 2
    return n


def algorithmic_counts(N, d, m, s, D, nsamp, nrhs, ranks=None, split_levels=6):
    """Algorithmic flops and bytes of each kernel family in one step, from the
    tree's actual skeleton ranks s_a (ranks[i] for heap node i; full rank s
    when None).  These are the counts the method needs, not what the kernels
    execute:
      skel:k_qrcp         pivot step j of an r x c sampled block: 6 (r-j)(c-j-1)
                          flops (reflector dot 2 + axpy 2 + column norm 2 per
                          trailing element), s_a steps, then T = R11^-1 R12:
                          s_a^2 (c - s_a); nothing when c <= s (P = I).
                          Nodes at tree levels <= split_levels count for the
                          split form (skel:k_qrcp_split), the rest for k_qrcp
      skel:k_sample_block 3d + 1 flops per sampled kernel entry (difference,
                          fma, exp counted as one), nodes with c > s only, at
                          the split levels; skel:k_sample_rownorm the same at
                          the other levels (it forms the entries and their
                          row sums, k_qrcp regenerates the kept rows)
      factor:k_lu_nopiv   (2/3) m^3 per leaf LU (no row exchanges)
      factor:k_lu         (2/3) n^3 per Z LU (n = s_l + s_r, partial pivoting)
      factor:k_lusolve    2 n^2 s_a (leaf Phat, internal Z^-1 P_c below the root)
      factor:k_kmm        2 s_l n_r s_r + 2 s_r n_l s_l per internal node (eq. (8))
      factor:k_gmm        2 (n_l s_l + n_r s_r) s_a per internal non-root node
                          (telescoping, eq. (10))
      solve:k_lusolve     LU factors read once (8 n^2 bytes) + right-hand sides
                          read and written (16 n nrhs bytes) per node
      solve:k_kmm         2 (s_l n_r + s_r n_l) nrhs per internal node
    """
    nn = (2 << D) - 1
    sz = node_sizes(N, D)
    r = np.full(nn, s, dtype=np.int64) if ranks is None else np.asarray(ranks, dtype=np.int64)
    first_leaf = (1 << D) - 1
    c = {k: 0.0 for k in ("qr", "qr1", "qrs", "samp", "samp1", "samps", "lu", "lu_leaf", "lu_z", "fsolve", "zblk",
                          "tele", "sbytes", "sflops", "skmm")}
    for i in range(nn):
        n = float(sz[i])
        leaf = i >= first_leaf
        if i > 0:
            cols = n if leaf else float(r[2 * i + 1] + r[2 * i + 2])
            if cols > s:
                rows = float(min(nsamp, N - n))
                k = int(r[i])
                w = sum(6.0 * (rows - j) * (cols - j - 1) for j in range(k)) + k * k * (cols - k)
                c["qr"] += w
                split_node = int(np.log2(i + 1)) <= split_levels
                c["qrs" if split_node else "qr1"] += w
                c["samp"] += rows * cols * (3.0 * d + 1)
                c["samps" if split_node else "samp1"] += rows * cols * (3.0 * d + 1)
        nlu = n if leaf else float(r[2 * i + 1] + r[2 * i + 2])
        c["lu"] += (2.0 / 3.0) * nlu ** 3
        c["lu_leaf" if leaf else "lu_z"] += (2.0 / 3.0) * nlu ** 3
        if i > 0:
            c["fsolve"] += 2.0 * nlu * nlu * r[i]
        c["sflops"] += 2.0 * nlu * nlu * nrhs
        c["sbytes"] += 8.0 * nlu * nlu + 16.0 * nlu * nrhs
        if not leaf:
            l, rr = 2 * i + 1, 2 * i + 2
            sl, sr, nl, nr = float(r[l]), float(r[rr]), float(sz[l]), float(sz[rr])
            c["zblk"] += 2.0 * sl * nr * sr + 2.0 * sr * nl * sl
            c["skmm"] += 2.0 * (sl * nr + sr * nl) * nrhs
            if i > 0:
                c["tele"] += 2.0 * (nl * sl + nr * sr) * r[i]
    return c


# Kernel families reported against their roofline: (profile key, count key,
# bound, peak key, unit).  FP64 vector and FP64 MFMA share one peak on MI355X;
# the mixed path's products run FP32 MFMA.
ROOF_TABLE = [
    # (profile key, count key, bound, peak, unit, launches of one pass: a
    # function of the depth, or None when the count varies with the ranks --
    # then the measured launches of the timed steps are used)
    ("skel:k_qrcp", "qr1", "alu", "fp64", "TFLOP/s", None),
    ("skel:k_qrcp_split", "qrs", "alu", "fp64", "TFLOP/s", None),
    ("skel:k_sample_rownorm", "samp1", "alu", "fp64", "TFLOP/s", None),
    ("skel:k_sample_block", "samps", "alu", "fp64", "TFLOP/s", None),
    ("factor:k_lu_nopiv", "lu_leaf", "mfma", "fp64", "TFLOP/s", lambda D: 1),
    ("factor:k_lu", "lu_z", "alu", "fp64", "TFLOP/s", lambda D: D),
    ("factor:k_lusolve", "fsolve", "mfma", "fp64", "TFLOP/s", lambda D: D),
    ("factor:k_kmm", "zblk", "mfma", "fp32", "TFLOP/s", None),
    ("factor:k_gmm", "tele", "mfma", "fp32", "TFLOP/s", None),
    ("solve:k_lusolve", "sbytes", "hbm", None, "GB/s", lambda D: D + 1),
    ("solve:k_kmm", "skmm", "mfma", "fp32", "TFLOP/s", lambda D: D),
]

# HBM bytes per launch of single kernels, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, averaged over the launches of one step),
# scaled by what the same counters read for a plain 1 GiB read + 1 GiB write
# (torch.neg).  Valid only for the kernel source they were taken on (sha256 of
# its files) and for this workload; otherwise "traffic" is null.
TRAFFIC = {
    "factor:k_lu_nopiv": {
        "source": ["k_lu.hip", "askit_dev.h"],
        "src_sha256": "5b2819c17ec7374da3c112dc76273c139a7c74eda652d6d610105d445e3491d1",
        "workload": (1048576, 16, 512, 256, 1024),
        "bytes_per_launch": 32444892314.45556,
    },
    "skel:k_qrcp": {
        "source": ["k_skel.hip", "askit_dev.h"],
        "src_sha256": "88879bf3a579a06c7f1a8c9956337b093968cc75e018ff72d89e06d08f387dfd",
        "workload": (1048576, 16, 512, 256, 1024),
        "bytes_per_launch": 3819166883.375679,
    },
}


def kernel_source_sha(names):
    """sha256 over the kernel's source files (a file name or a list), in order."""
    import hashlib
    h = hashlib.sha256()
    for name in [names] if isinstance(names, str) else names:
        with open(os.path.join(ROOT, "paper_1701_02324_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def roofline_of(key, cnt_key, bound, peak_key, unit, nlaunch, prof, cnt, D, steps):
    """Algorithmic work of one pass of the kernel family divided over the
    launches one pass makes (one per tree level); the solve plan runs once per
    operator application, so the measured launch count may be a multiple."""
    if key not in prof:
        return None
    ms, launches = prof[key]
    per_launch_ms = ms / launches
    work_per_launch = cnt[cnt_key] / (nlaunch(D) if nlaunch else launches / steps)
    if unit == "GB/s":
        achieved = work_per_launch / (per_launch_ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
    else:
        achieved = work_per_launch / (per_launch_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[peak_key]
    return dict(kernel=key, bound=bound, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak,
                traffic=None, avg_launch_ms=per_launch_ms, launches=launches,
                work_per_launch=work_per_launch)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-sample", type=int, default=262144, help="points in the oracle's sample problem")
    ap.add_argument("--max-refine", type=int, default=10, help="GMRES-IR operator applications (mixed path)")
    ap.add_argument("--no-stable-check", action="store_true",
                    help="skip the mixed-vs-FP64 check on the N=65536 d=8 mixture (lambda=0.1)")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip the extra step through the two separate calls")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the timings of the other forms (batched problems, gradient, transpose solve)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB elementwise copy (reference for the HBM byte counters)")
    ap.add_argument("--tol", type=float, default=1e-11, help="target relative residual of the refined solves")
    ap.add_argument("--qr-split-levels", type=int, default=0,
                    help="tree levels factored by the split pivoted QR (0: library default, -1: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1701_02324_amd as ak
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    c = synth.config(3, N=args.N, nrhs=args.nrhs)
    N, d = c["X"].shape
    m, s, h, lam, nsamp = c["m"], c["s"], c["h"], c["lam"], c["nsamp"]
    log(f"[bench] workload N={N} d={d} m={m} s={s} h={h} lambda={lam} nrhs={args.nrhs}")
    X = torch.as_tensor(c["X"], device=dev)
    B = torch.as_tensor(c["B"], device=dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    tree = ak.Tree(X, m, s, h, n_samples=nsamp, seed=c["seed"], qr_split_levels=args.qr_split_levels)
    torch.cuda.synchronize()
    t_tree = time.perf_counter() - t0
    log(f"[bench] tree built in {t_tree:.3f} s (depth {tree.D})")

    def step(prec, keep=False, fused=True):
        # fused: askit_skeletonize_factorize (the two phases pipelined over
        # two streams); else the two separate calls
        torch.cuda.synchronize()
        a = time.perf_counter()
        if fused:
            f = tree.skeletonize_factorize(lam, prec)
            b = None
        else:
            tree.skeletonize()
            torch.cuda.synchronize()
            b = time.perf_counter()
            f = tree.factorize(lam, prec)
        if prec == ak.ASKIT_MIXED:
            f.set_refinement(args.max_refine, args.tol)
        torch.cuda.synchronize()
        cc = time.perf_counter()
        x = f.solve(B)
        torch.cuda.synchronize()
        e = time.perf_counter()
        info = f.info() if prec == ak.ASKIT_MIXED else None
        if info is not None:
            info["min_pivot_ratio"] = f.pivot_ratio()[0]
        out = dict(total=cc - a, skel=None if b is None else b - a, factor=None if b is None else cc - b,
                   solve=e - cc, info=info)
        if keep:
            return out, f, x
        f.close()
        del x
        return out, None, None

    for w in range(args.warmup):
        r, _, _ = step(ak.ASKIT_MIXED)
        log(f"[bench] warmup {w}: skeletonize+factorize {r['total']:.3f} s solve {r['solve']:.3f} s")

    ak.askit_profile_enable(True)
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    runs = []
    fmx = xmx = None
    for k in range(args.steps):
        r, f, x = step(ak.ASKIT_MIXED, keep=(k == args.steps - 1))
        runs.append(r)
        if f is not None:
            fmx, xmx = f, x
        log(f"[bench] step {k}: skeletonize+factorize {r['total']:.3f} s solve {r['solve']:.3f} s "
            f"refine {r['info']}")
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    prof = ak.askit_profile_report()
    ak.askit_profile_enable(False)
    # the stored mixed factors applied once (no refinement): 64 right-hand
    # sides, and one right-hand side (latency)
    fmx.set_refinement(0, args.tol)
    direct = {}
    for name, Bx in (("nrhs", B), ("one_rhs", B[:, :1].contiguous())):
        fmx.solve(Bx)
        torch.cuda.synchronize()
        a = time.perf_counter()
        fmx.solve(Bx)
        torch.cuda.synchronize()
        direct[name] = time.perf_counter() - a
    fmx.close()
    ms_step = 1e3 * (T1 - T0) / args.steps
    t_total = float(np.mean([r["total"] for r in runs]))
    t_sol = float(np.mean([r["solve"] for r in runs]))
    info = runs[-1]["info"]
    # the same step through the two separate calls (no overlap), once
    two_call = None
    if not args.no_separate:
        r2, _, _ = step(ak.ASKIT_MIXED, fused=False)
        two_call = dict(skeletonize_s=r2["skel"], factorize_s=r2["factor"], total_s=r2["total"])
        log(f"[bench] separate calls: skeletonize {r2['skel']:.3f} s factorize {r2['factor']:.3f} s")

    res = {}
    if not args.no_fp64:
        # one untimed FP64 pass first (its first allocations), like the
        # warm-up of the timed mixed steps
        tree.skeletonize_factorize(lam, ak.ASKIT_FP64).close()
        torch.cuda.synchronize()
        # factorization alone (the skeletons of the pass above), then the
        # pipelined call; each reuses the device blocks of the one before
        a = time.perf_counter()
        f64 = tree.factorize(lam, ak.ASKIT_FP64)
        torch.cuda.synchronize()
        t_f64_only = time.perf_counter() - a
        f64.close()
        a = time.perf_counter()
        f64 = tree.skeletonize_factorize(lam, ak.ASKIT_FP64)
        torch.cuda.synchronize()
        b = time.perf_counter()
        x64 = f64.solve(B)
        torch.cuda.synchronize()
        e = time.perf_counter()
        r64 = B - f64.matvec(x64)
        eps64 = float((r64.norm(dim=0) / B.norm(dim=0)).max())
        # the FP64 path refined against the same FP64 operator (GMRES-IR with
        # the FP64 factors) is the reference the mixed result is compared with
        f64.set_refinement(50, args.tol)
        g0 = time.perf_counter()
        xref = f64.solve(B)
        torch.cuda.synchronize()
        g1 = time.perf_counter()
        info64 = f64.info()
        info64["min_pivot_ratio"] = f64.pivot_ratio()[0]
        err = float(((xmx - xref).norm(dim=0) / xref.norm(dim=0)).max())
        err_direct = float(((xmx - x64).norm(dim=0) / x64.norm(dim=0)).max())
        res = dict(fp64_factor_s=b - a, fp64_factorize_only_s=t_f64_only, fp64_solve_s=e - b,
                   fp64_solves_per_s=args.nrhs / (e - b), fp64_residual=eps64,
                   fp64_refined_solve_s=g1 - g0, fp64_refinement=info64,
                   mixed_vs_fp64_rel_err=err, mixed_vs_fp64_direct_rel_err=err_direct,
                   speedup_factor_mixed_over_fp64=(b - a) / t_total,
                   speedup_factorize_only=t_f64_only / two_call["factorize_s"] if two_call else None)
        log(f"[bench] fp64: skeletonize+factorize {b - a:.3f} s (factorize alone {t_f64_only:.3f} s) solve "
            f"{e - b:.3f} s (residual {eps64:.2e}); refined "
            f"{g1 - g0:.3f} s {info64}; mixed vs fp64 refined {err:.2e}, vs fp64 direct {err_direct:.2e}")
        f64.close()
        del x64, r64, xref

    # roofline of every reported kernel family; the dominant one (largest
    # total time in the timed steps) is the headline
    ranks, cands = tree.skeleton_sizes()
    # the library's default split levels in the pipelined call (the timed
    # steps): those with fewer than 1024 nodes
    split = {0: min(tree.D - 1, 9), -1: 0}.get(args.qr_split_levels, args.qr_split_levels)
    cnt = algorithmic_counts(N, d, m, s, tree.D, nsamp, args.nrhs, ranks, split)
    rank_levels = {}
    for lvl in range(1, tree.D + 1):
        rl = ranks[(1 << lvl) - 1:(2 << lvl) - 1]
        rank_levels[lvl] = [int(rl.min()), round(float(rl.mean()), 1), int(rl.max())]
    rooflines = {}
    for key, ck, bound, pk, unit, nl in ROOF_TABLE:
        r = roofline_of(key, ck, bound, pk, unit, nl, prof, cnt, tree.D, args.steps)
        if r is not None:
            rooflines[key] = r
    # the headline is the kernel that dominates the metric's value (the
    # skeletonize + factorize time)
    top = sorted(prof.items(), key=lambda kv: -kv[1][0])
    # (single kernels only: the split QR family is a sequence of launches)
    dom = next((k for k, _ in top if k in rooflines and k.split(":")[0] in ("skel", "factor")
                and k != "skel:k_qrcp_split"), None)
    roof = dict(rooflines[dom]) if dom else None
    tr = TRAFFIC.get(dom) if dom else None
    if roof is not None and tr is not None and tr["src_sha256"] == kernel_source_sha(tr["source"]) \
            and tr["workload"] == (N, d, m, s, nsamp):
        roof["traffic"] = tr["bytes_per_launch"]

    forms = None
    if not args.no_forms:
        forms = forms_timings(ak, torch, dev, tree, lam, B)
    stable = None
    if not args.no_stable_check:
        stable = stable_config_check(ak, torch, dev, args.tol)
    if args.calibrate_copy:
        x = torch.empty(1 << 27, dtype=torch.float64, device=dev).uniform_()
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 3 x (1 GiB read + 1 GiB write), torch.neg")
        del x, y

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(c, args.cpu_sample, args.nrhs)

    out = {
        "metric": METRIC, "value": t_total, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"gaussian-mixture N={N} d={d} m={m} s={s} h={h} lambda={lam} nrhs={args.nrhs}",
                   "N": N, "d": d, "leaf_size": m, "rank": s, "n_samples": nsamp, "nrhs": args.nrhs,
                   "precision": "mixed"},
        "skeletonize_factorize_s": t_total, "separate_calls": two_call, "solve_s": t_sol, "solves_per_s": args.nrhs / t_sol,
        "direct_solve_s": direct["nrhs"], "direct_solves_per_s": args.nrhs / direct["nrhs"],
        "one_rhs_direct_solve_s": direct["one_rhs"],
        "refinement": info, "tree_s": t_tree,
        **res,
        "skeleton_ranks_min_mean_max": rank_levels,
        "roofline": roof,
        "rooflines": rooflines,
        "mixed_on_stable_config": stable,
        "forms": forms,
        "cpu_baseline": cpu,
        "kernels_ms": {k: [round(v[0] / args.steps, 3), v[1] // args.steps] for k, v in top[:12]},
    }
    print(json.dumps(out))


def _timed(torch, fn, reps=1):
    fn()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - a) / reps, out


def forms_timings(ak, torch, dev, tree, lam, B):
    """Timings of the forms beside the plain solve, each on its own workload:
    the FP64 transpose solve and hierarchical matvecs of the 1M workload
    (64 right-hand sides); one adjoint gradient (forward solve, transpose
    solve, derivative matvec) on the differentiation workload (N = 262,144,
    d = 8, h = 1, lambda = 0.05, m = 256, s = 128, 4 right-hand sides); and the
    batched workload: 256 independent problems with N log-uniform in
    [2048, 32768], d = 8, m = 128, s = 64, 8 right-hand sides each,
    skeletonized together, then factorized and solved by hipGraph replays."""
    import synth
    out = {}
    f = tree.factorize(lam, ak.ASKIT_FP64)
    out["fp64_solve_transpose_s"], _ = _timed(torch, lambda: f.solve_transpose(B))
    out["fp64_matvec_s"], _ = _timed(torch, lambda: f.matvec(B, 0))
    out["fp64_matvec_transpose_s"], _ = _timed(torch, lambda: f.matvec(B, 2))
    out["fp64_matvec_dh_s"], _ = _timed(torch, lambda: f.matvec(B, 1))
    f.close()
    # adjoint gradient
    c = synth.config(5)
    t5 = ak.Tree(torch.as_tensor(c["X"], device=dev), c["m"], c["s"], c["h"], seed=c["seed"])
    t5.skeletonize()
    B5 = torch.as_tensor(c["B"], device=dev)
    Y5 = torch.as_tensor(c["Y"], device=dev)

    def grad():
        b = B5.clone().requires_grad_(True)
        lt = torch.tensor(c["lam"], dtype=torch.float64, requires_grad=True)
        ht = torch.tensor(c["h"], dtype=torch.float64, requires_grad=True)
        x = ak.kernel_solve(b, lt, ht, t5)
        ((x - Y5) ** 2).sum().backward()
        return float(lt.grad)
    out["gradient_n262144_s"], _ = _timed(torch, grad)
    t5.close()
    # batched problems
    probs = synth.batched_problems()
    trees = [ak.Tree(torch.as_tensor(p["X"], device=dev), p["m"], p["s"], p["h"], n_samples=p["nsamp"],
                     seed=p["seed"], problem=p["problem"]) for p in probs]
    torch.cuda.synchronize()
    a = time.perf_counter()
    ak.askit_skeletonize_batched(trees)
    torch.cuda.synchronize()
    t_skel = time.perf_counter() - a
    a = time.perf_counter()
    batch = ak.Batch(trees, [p["lam"] for p in probs], ak.ASKIT_FP64, nrhs=8)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - a
    Bs = [torch.as_tensor(p["B"], device=dev) for p in probs]
    t_fac, _ = _timed(torch, batch.factorize, reps=3)
    t_sol, _ = _timed(torch, lambda: batch.solve(Bs), reps=3)
    ratio, worst = batch.check()
    out["batched"] = {"problems": len(probs), "points": int(sum(len(p["X"]) for p in probs)),
                      "skeletonize_s": t_skel, "plan_and_capture_s": t_create, "factorize_graph_s": t_fac,
                      "solve_graph_s": t_sol, "factorizations_per_s": len(probs) / t_fac,
                      "min_pivot_ratio": ratio}
    log(f"[bench] forms: {out}")
    batch.close()
    for t in trees:
        t.close()
    return out


def stable_config_check(ak, torch, dev, tol):
    """Mixed vs FP64 where the recursion is stable: N = 65,536 points of an
    8-cluster mixture in 8-D (centres ~ U[-5,5]^8, sigma = 1), h = 1, lambda = 0.1,
    m = 256, s = 128, 16 right-hand sides."""
    import synth
    c = synth.config(2)
    X = torch.as_tensor(c["X"], device=dev)
    B = torch.as_tensor(c["B"], device=dev)
    t = ak.Tree(X, c["m"], c["s"], c["h"], n_samples=c["nsamp"], seed=c["seed"])
    t.skeletonize()
    out = {"workload": "gaussian-mixture N=65536 d=8 m=256 s=128 h=1 lambda=0.1 nrhs=16"}
    res = {}
    for name, prec in (("fp64", ak.ASKIT_FP64), ("mixed", ak.ASKIT_MIXED)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        f = t.factorize(c["lam"], prec)
        torch.cuda.synchronize()
        b = time.perf_counter()
        f.set_refinement(50, tol)
        x = f.solve(B)
        torch.cuda.synchronize()
        e = time.perf_counter()
        res[name] = (x, f.info())
        out[f"{name}_factorize_s"] = b - a
        out[f"{name}_refined_solve_s"] = e - b
        out[f"{name}_refinement"] = f.info()
        f.close()
    x64, xm = res["fp64"][0], res["mixed"][0]
    out["mixed_vs_fp64_rel_err"] = float(((xm - x64).norm(dim=0) / x64.norm(dim=0)).max())
    log(f"[bench] stable config: mixed vs fp64 {out['mixed_vs_fp64_rel_err']:.2e}, "
        f"mixed refinement {out['mixed_refinement']}")
    t.close()
    return out


def cpu_baseline(c, n_sample, nrhs):
    """The oracle (plain C, OpenMP) on a bounded sample of the same workload:
    the first n_sample points of the mixture with the same d, m, s, h, lambda;
    factor time (skeletonize + factorize) scaled to N by the N log(N/m) work
    model of the method (Sec. 3, "Work")."""
    import oracle
    X = c["X"][:n_sample]
    Bs = c["B"][:n_sample]
    m, s = c["m"], c["s"]
    o = oracle.Oracle(X, m, s, c["h"], nsamp=c["nsamp"], seed=c["seed"])
    o.build_tree()
    log(f"[bench] cpu baseline: oracle on {n_sample} points, {oracle.num_threads()} threads")
    a = time.perf_counter()
    o.skeletonize()
    b = time.perf_counter()
    o.factorize(c["lam"])
    e = time.perf_counter()
    o.solve(Bs)
    g = time.perf_counter()
    N = c["X"].shape[0]
    Dn = max(1, int(np.ceil(np.log2(n_sample / m))))
    DN = max(1, int(np.ceil(np.log2(N / m))))
    scale = (N * DN) / (n_sample * Dn)
    t_fac = (e - a) * scale
    log(f"[bench] cpu baseline: skel {b - a:.2f} s factor {e - b:.2f} s solve {g - e:.2f} s (sample)")
    return {"value": t_fac, "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {n_sample} points of the workload (depth {Dn}); skeletonize+factorize "
                      f"{e - a:.2f} s measured, scaled by N log(N/m) to N={N} (depth {DN})",
            "sample_solve_s": g - e}


if __name__ == "__main__":
    main()
