#!/usr/bin/env python3
"""Benchmark of the hierarchical kernel solver on one MI355X.

Workload (the paper's N log N scaling shape, m = 512, s = 256, on a synthetic
Gaussian mixture in place of its datasets): N = 1,048,576 points in 16-D, 32
clusters with centres ~ U[-10,10]^16 and sigma ~ U[0.5,2]; h = 2, lambda = 0.01,
64 right-hand sides ~ N(0,1).

One step = skeletonize (sampled ID, FP64 pivoted QR) + factorize (FP64), as
the one pipelined call askit_skeletonize_factorize, + the direct solve of the
64 right-hand sides.  Inputs are resident in HBM before the timed region; the
tree is built once, outside it.

value = the factor time (skeletonize + factorize) of the FP64 path in seconds,
the paper's precision.  The mixed path (FP32 kernel blocks and level products,
FP64 LUs) is timed the same way and reported beside it with its accuracy gate
(relative error to the refined FP64 solution <= 1e-6 with converged
refinement); it is the headline only if that gate holds.

Before the timed steps the tree's level-product tiles are autotuned once
(askit_tune_factorization; --no-tune keeps the built-in choice); the tuning
time is reported, not timed.  The timed steps run without per-launch events.  Per-kernel times come from a
separate pass of the same steps with HIP events around every launch
(askit_profile_enable), and give the rooflines.  The oracle (plain C, OpenMP)
is the CPU baseline, timed on the whole workload (about 50 s on 16 cores);
with --cpu-check it also checks the GPU's tree, skeletons and FP64 solution.
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
MIXED_GATE = 1e-6


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


def algorithmic_counts(N, d, m, s, D, nsamp, nrhs, ranks, qrows, split_levels, fp64=True):
    """Algorithmic flops and bytes of each kernel of one step, from the tree's
    actual skeleton ranks s_a (ranks[i] for heap node i) and the rows each
    node's pivoted QR factored (qrows[i], numerically zero sampled rows
    dropped).  These are the counts the method needs, not what the kernels
    execute:
      skel:k_qrcp          nodes at levels > split_levels with c > s candidate
                           columns and r factored rows: pivot step j reads and
                           writes the trailing block once, 16 (r-j)(c-j-1)
                           bytes in FP64 (the block does not fit on chip, so
                           the unblocked Householder QR streams it every step;
                           its flops, 6 (r-j)(c-j-1), are 0.375 per byte), s_a
                           steps; plus the r c generated entries written once
      skel:k_qs_step       the pivot steps of the nodes at levels 1..split_levels
                           (bytes as above)
      skel:k_qs_finish     T = R11^-1 R12: s_a^2 (c - s_a) flops
      skel:k_sample_rownorm (3d+1) flops per sampled kernel entry (difference,
                           fma, exp counted as one), nsamp' x c per node, one-
                           workgroup levels; skel:k_sample_block the same at
                           the split levels
      factor:k_lu_nopiv    (2/3) n^3 per leaf LU
      factor:k_lu          (2/3) n^3 per Z LU (n = s_l + s_r)
      factor:k_lusolve     2 n^2 s_a (leaf Phat, internal Z^-1 P_c)
      factor:k_kmm         2 s_l n_r s_r + 2 s_r n_l s_l per internal node (eq. (8))
      factor:k_gmm         2 (n_l s_l + n_r s_r) s_a per internal non-root node
                           (telescoping, eq. (10))
      solve:k_lusolve      LU factors read once (8 n^2 bytes) + right-hand
                           sides read and written (2 w n nrhs bytes, w = 8 in
                           FP64) per node
      solve:k_kmm          2 (s_l n_r + s_r n_l) nrhs per internal node
      solve:k_gmm          2 (n_l s_l + n_r s_r) nrhs per internal node
    """
    nn = (2 << D) - 1
    sz = node_sizes(N, D)
    r = np.asarray(ranks, dtype=np.int64)
    qr = np.asarray(qrows, dtype=np.int64)
    first_leaf = (1 << D) - 1
    keys = ("skel:k_qrcp", "skel:k_qs_step", "skel:k_qs_finish", "skel:k_sample_rownorm",
            "skel:k_sample_block", "factor:k_lu_nopiv", "factor:k_lu", "factor:k_lusolve", "factor:k_kmm",
            "factor:k_gmm", "solve:k_lusolve", "solve:k_kmm", "solve:k_gmm")
    c = {k: 0.0 for k in keys}
    w = 8.0 if fp64 else 4.0
    for i in range(nn):
        n = float(sz[i])
        leaf = i >= first_leaf
        lvl = int(np.log2(i + 1))
        if i > 0:
            cols = n if leaf else float(r[2 * i + 1] + r[2 * i + 2])
            if cols > s:
                rows_s = float(min(nsamp, N - n))
                rows = float(qr[i])
                k = int(r[i])
                steps = sum(16.0 * (rows - j) * (cols - j - 1) for j in range(k))
                tsolve = k * k * (cols - k)
                samp = rows_s * cols * (3.0 * d + 1)
                if lvl <= split_levels:
                    c["skel:k_qs_step"] += steps
                    c["skel:k_qs_finish"] += tsolve
                    c["skel:k_sample_block"] += samp
                else:
                    c["skel:k_qrcp"] += steps + 8.0 * rows * cols
                    c["skel:k_sample_rownorm"] += samp
        nlu = n if leaf else float(r[2 * i + 1] + r[2 * i + 2])
        c["factor:k_lu_nopiv" if leaf else "factor:k_lu"] += (2.0 / 3.0) * nlu ** 3
        if i > 0:
            c["factor:k_lusolve"] += 2.0 * nlu * nlu * r[i]
        c["solve:k_lusolve"] += 8.0 * nlu * nlu + 2.0 * w * nlu * nrhs
        if not leaf:
            l, rr = 2 * i + 1, 2 * i + 2
            sl, sr, nl, nr = float(r[l]), float(r[rr]), float(sz[l]), float(sz[rr])
            c["factor:k_kmm"] += 2.0 * sl * nr * sr + 2.0 * sr * nl * sl
            c["solve:k_kmm"] += 2.0 * (sl * nr + sr * nl) * nrhs
            c["solve:k_gmm"] += 2.0 * (nl * sl + nr * sr) * nrhs
            if i > 0:
                c["factor:k_gmm"] += 2.0 * (nl * sl + nr * sr) * r[i]
    return c


# Kernels reported against their roofline: key -> (bound, peak key, unit).
# FP64 vector and FP64 MFMA share one peak on MI355X (78.6 TFLOP/s); the
# products of the mixed path would run FP32 MFMA, the timed FP64 path does not.
ROOF_KIND = {
    "skel:k_qrcp": ("hbm", None, "GB/s"),
    "skel:k_qs_step": ("hbm", None, "GB/s"),
    "skel:k_qs_finish": ("alu", "fp64", "TFLOP/s"),
    "skel:k_sample_rownorm": ("alu", "fp64", "TFLOP/s"),
    "skel:k_sample_block": ("alu", "fp64", "TFLOP/s"),
    "factor:k_lu_nopiv": ("mfma", "fp64", "TFLOP/s"),
    "factor:k_lu": ("mfma", "fp64", "TFLOP/s"),
    "factor:k_lusolve": ("mfma", "fp64", "TFLOP/s"),
    "factor:k_kmm": ("mfma", "fp64", "TFLOP/s"),
    "factor:k_gmm": ("mfma", "fp64", "TFLOP/s"),
    "solve:k_lusolve": ("hbm", None, "GB/s"),
    "solve:k_kmm": ("mfma", "fp64", "TFLOP/s"),
    "solve:k_gmm": ("mfma", "fp64", "TFLOP/s"),
}

# HBM bytes per launch of single kernels, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, averaged over the launches of one step),
# scaled by what the same counters read for a plain 1 GiB read + 1 GiB write
# (torch.neg).  Valid only for the kernel source they were taken on (sha256 of
# its files) and for this workload; otherwise "traffic" is null.
TRAFFIC = {
    "skel:k_qs_step": {
        "source": ["k_skel.hip", "askit_dev.h"],
        "src_sha256": "2ee4b4dd202670b7a795b1ebadde224b6563daf510b0b3dd40f37f9e1cadeeac",
        "workload": (1048576, 16, 512, 256, 1024),
        "bytes_per_launch": (2341.1 * 2.0 + 3744.1) * 1024.0,
    },
    "skel:k_qrcp": {
        "source": ["k_skel.hip", "askit_dev.h"],
        "src_sha256": "2ee4b4dd202670b7a795b1ebadde224b6563daf510b0b3dd40f37f9e1cadeeac",
        "workload": (1048576, 16, 512, 256, 1024),
        "bytes_per_launch": (1041292.5 * 2.0 + 1642088.7) * 1024.0,
    },
    "factor:k_lu_nopiv": {
        "source": ["k_lu.hip", "askit_dev.h"],
        "src_sha256": "f6104c39adc9229c98bea4e249a3bc3daf7ab6903b1648d6d8ac8d035d3d29de",
        "workload": (1048576, 16, 512, 256, 1024),
        "bytes_per_launch": (7562807.0 * 2.0 + 16138858.1) * 1024.0,
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


def rooflines_of(prof, cnt, steps):
    """Per kernel: algorithmic work of one step over its launches in one step,
    divided by its average launch duration (HIP events on its stream)."""
    out = {}
    for key, (bound, pk, unit) in ROOF_KIND.items():
        if key not in prof or cnt.get(key, 0.0) <= 0.0:
            continue
        ms, launches = prof[key]
        per_step = launches / steps
        per_launch_ms = ms / launches
        work = cnt[key] / per_step
        if unit == "GB/s":
            achieved, peak = work / (per_launch_ms * 1e-3) / 1e9, HBM_PEAK_GBS
        else:
            achieved, peak = work / (per_launch_ms * 1e-3) / 1e12, PEAK_TFLOPS[pk]
        out[key] = dict(kernel=key, bound=bound, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak,
                        traffic=None, avg_launch_ms=per_launch_ms, launches_per_step=per_step,
                        work_per_launch=work, step_ms=ms / steps)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision steps")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-check", action="store_true",
                    help="after the oracle's timed run on the whole workload, check the GPU's tree, skeletons and "
                         "FP64 solution against it (about two minutes more on 16 cores)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="time the oracle on the first CPU_SAMPLE points only, scaled by N log(N/m) (0: the "
                         "whole workload)")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel profiled pass")
    ap.add_argument("--max-refine", type=int, default=60, help="GMRES-IR operator applications (mixed path)")
    ap.add_argument("--no-stable-check", action="store_true",
                    help="skip the mixed-vs-FP64 check on the N=65536 d=8 mixture (lambda=0.1)")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip the extra step through the two separate calls")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the timings of the other forms (batched problems, gradient, transpose solve)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB elementwise copy (reference for the HBM byte counters)")
    ap.add_argument("--tol", type=float, default=1e-11, help="target relative residual of the refined solves")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in tile choices (skip askit_tune_factorization before the timed steps)")
    ap.add_argument("--qr-split-levels", type=int, default=0,
                    help="tree levels factored by the split pivoted QR (0: library default, -1: none)")
    ap.add_argument("--cpu-rhs", type=int, default=4, help="right-hand sides the oracle solves in its check")
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
    # tile autotuning of the factorization's level products, once, outside
    # the timed steps (it needs skeletons: one skeletonization first)
    tune = None
    if not args.no_tune:
        tree.skeletonize()
        torch.cuda.synchronize()
        a = time.perf_counter()
        table = tree.tune(lam)
        torch.cuda.synchronize()
        tune = {"seconds": time.perf_counter() - a, "kmm_columns_chunk_gmm_columns_by_height": table}
        log(f"[bench] tuned tiles in {tune['seconds']:.2f} s: {table}")

    def step(prec, keep=False, fused=True, refine=0):
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
        f.set_refinement(refine, args.tol)
        torch.cuda.synchronize()
        cc = time.perf_counter()
        x = f.solve(B)
        torch.cuda.synchronize()
        e = time.perf_counter()
        out = dict(total=cc - a, skel=None if b is None else b - a, factor=None if b is None else cc - b,
                   solve=e - cc, info=f.info() if refine else None)
        if keep:
            return out, f, x
        f.close()
        del x
        return out, None, None

    def timed_steps(prec, label, refine=0):
        for w in range(args.warmup):
            r, _, _ = step(prec, refine=refine)
            log(f"[bench] {label} warmup {w}: skeletonize+factorize {r['total']:.4f} s solve {r['solve']:.4f} s")
        torch.cuda.synchronize()
        T0 = time.perf_counter()
        runs, fk, xk = [], None, None
        for k in range(args.steps):
            r, f, x = step(prec, keep=(k == args.steps - 1), refine=refine)
            runs.append(r)
            if f is not None:
                fk, xk = f, x
            log(f"[bench] {label} step {k}: skeletonize+factorize {r['total']:.4f} s solve {r['solve']:.4f} s"
                + (f" refine {r['info']}" if r["info"] else ""))
        torch.cuda.synchronize()
        T1 = time.perf_counter()
        return runs, fk, xk, T1 - T0

    # --- the FP64 path: the headline ------------------------------------------
    runs64, f64, x64, wall64 = timed_steps(ak.ASKIT_FP64, "fp64")
    t_fac64 = float(np.mean([r["total"] for r in runs64]))
    t_sol64 = float(np.mean([r["solve"] for r in runs64]))
    pr64 = f64.pivot_ratio()
    r64 = B - f64.matvec(x64)
    eps64 = float((r64.norm(dim=0) / B.norm(dim=0)).max())
    del r64
    f64.set_refinement(0, args.tol)
    Bone = B[:, :1].contiguous()
    f64.solve(Bone)
    torch.cuda.synchronize()
    a = time.perf_counter()
    f64.solve(Bone)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - a
    # the FP64 factors refined against the same FP64 operator (GMRES-IR): the
    # reference solution of the mixed path
    f64.set_refinement(50, args.tol)
    a = time.perf_counter()
    xref = f64.solve(B)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - a
    info64 = f64.info()
    log(f"[bench] fp64: skeletonize+factorize {t_fac64:.4f} s, solve {t_sol64:.4f} s, direct residual "
        f"{eps64:.2e}, refined {t_ref:.3f} s {info64}, min pivot ratio {pr64[0]:.2e}")
    ranks, cands = tree.skeleton_sizes()
    qrows = tree.qr_rows()
    ids64, P64, sizes64 = tree.export_skeletons() if args.cpu_check else (None, None, None)
    f64.close()

    # --- per-kernel times: the same FP64 steps again, every launch between
    # HIP events on its stream
    prof = {}
    if not args.no_profile:
        ak.askit_profile_enable(True)
        for k in range(args.steps):
            step(ak.ASKIT_FP64)
        torch.cuda.synchronize()
        prof = ak.askit_profile_report()
        ak.askit_profile_enable(False)
        log("[bench] profiled pass done")

    # --- the mixed path --------------------------------------------------------
    mixed = None
    if not args.no_mixed:
        runsm, fm, _, _ = timed_steps(ak.ASKIT_MIXED, "mixed")
        t_facm = float(np.mean([r["total"] for r in runsm]))
        t_solm = float(np.mean([r["solve"] for r in runsm]))
        fm.set_refinement(args.max_refine, args.tol)
        a = time.perf_counter()
        xm = fm.solve(B)
        torch.cuda.synchronize()
        t_refm = time.perf_counter() - a
        infom = fm.info()
        err = float(((xm - xref).norm(dim=0) / xref.norm(dim=0)).max())
        gate = bool(err <= MIXED_GATE and infom["converged"])
        mixed = dict(skeletonize_factorize_s=t_facm, direct_solve_s=t_solm, refined_solve_s=t_refm,
                     refinement=infom, rel_err_vs_fp64_refined=err, gate=f"rel err <= {MIXED_GATE:g}, converged",
                     gate_pass=gate, speedup_factor_over_fp64=t_fac64 / t_facm,
                     min_pivot_ratio=fm.pivot_ratio()[0])
        log(f"[bench] mixed: skeletonize+factorize {t_facm:.4f} s ({t_fac64 / t_facm:.2f}x fp64), refined "
            f"{t_refm:.3f} s {infom}, vs fp64 {err:.2e}: gate {'pass' if gate else 'FAIL'}")
        fm.close()
        del xm

    two_call = None
    if not args.no_separate:
        r2, _, _ = step(ak.ASKIT_FP64, fused=False)
        two_call = dict(skeletonize_s=r2["skel"], factorize_s=r2["factor"], total_s=r2["total"])
        log(f"[bench] fp64 separate calls: skeletonize {r2['skel']:.4f} s factorize {r2['factor']:.4f} s")

    # --- rooflines of the FP64 step ----------------------------------------------
    split = {0: min(tree.D - 1, 9), -1: 0}.get(args.qr_split_levels, args.qr_split_levels)
    cnt = algorithmic_counts(N, d, m, s, tree.D, nsamp, args.nrhs, ranks, qrows, split)
    rank_levels = {}
    for lvl in range(1, tree.D + 1):
        rl = ranks[(1 << lvl) - 1:(2 << lvl) - 1]
        ql = qrows[(1 << lvl) - 1:(2 << lvl) - 1]
        ql = ql[ql > 0]
        rank_levels[lvl] = dict(rank=[int(rl.min()), round(float(rl.mean()), 1), int(rl.max())],
                                qr_rows_mean=round(float(ql.mean()), 1) if ql.size else 0.0)
    rooflines = rooflines_of(prof, cnt, args.steps) if prof else {}
    # the headline roofline is the kernel with the largest time in the step
    top = sorted(((k, v) for k, v in prof.items() if k != "@timeline"), key=lambda kv: -kv[1][0])
    dom = next((k for k, _ in top if k in rooflines), None)
    for key, r in rooflines.items():
        tr = TRAFFIC.get(key)
        if tr is not None and tr["src_sha256"] == kernel_source_sha(tr["source"]) \
                and tr["workload"] == (N, d, m, s, nsamp):
            r["traffic"] = tr["bytes_per_launch"]
    roof = dict(rooflines[dom]) if dom else None

    forms = None
    if not args.no_forms:
        forms = forms_timings(ak, torch, dev, tree, lam, B)
        forms["knn_sampling"] = knn_sampling_form(ak, torch, dev, c, X, B, tree, lam)
    stable = None
    if not args.no_stable_check:
        stable = stable_config_check(ak, torch, dev, args.tol)
    if args.calibrate_copy:
        xc = torch.empty(1 << 27, dtype=torch.float64, device=dev).uniform_()
        yc = torch.empty_like(xc)
        for _ in range(3):
            torch.neg(xc, out=yc)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 3 x (1 GiB read + 1 GiB write), torch.neg")
        del xc, yc

    cpu = None
    batched_sample = forms.pop("_batched_sample", None) if forms else None
    if args.cpu_sample:
        cpu = cpu_baseline(c, args.cpu_sample)
    elif not args.no_cpu:
        cpu = cpu_full_check(c, tree, ids64, P64, sizes64, x64, xref, args.cpu_rhs, args.cpu_check)
    if cpu is not None and batched_sample:
        cpu["batched_check"] = cpu_batched_check(batched_sample)

    out = {
        "metric": METRIC, "value": t_fac64, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall64 / args.steps, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"gaussian-mixture N={N} d={d} m={m} s={s} h={h} lambda={lam} nrhs={args.nrhs}",
                   "N": N, "d": d, "leaf_size": m, "rank": s, "n_samples": nsamp, "nrhs": args.nrhs,
                   "precision": "fp64"},
        "skeletonize_factorize_s": t_fac64, "separate_calls": two_call, "tile_tuning": tune,
        "solve_s": t_sol64, "solves_per_s": args.nrhs / t_sol64, "one_rhs_solve_s": t_one,
        "fp64_direct_residual": eps64, "fp64_refined_solve_s": t_ref, "fp64_refinement": info64,
        "fp64_min_pivot_ratio": pr64[0], "tree_s": t_tree,
        "mixed": mixed,
        "skeleton_ranks_by_level": rank_levels,
        "roofline": roof,
        "rooflines": rooflines,
        "mixed_on_stable_config": stable,
        "forms": forms,
        "cpu_baseline": cpu,
        "kernels_ms_per_step": {k: [round(v[0] / args.steps, 3), round(v[1] / args.steps, 1)] for k, v in top[:16]},
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


def knn_sampling_form(ak, torch, dev, c, X, B, tree, lam, kappa=32, rows=64):
    """kappa-nearest-neighbour importance sampling on the 1M workload (kappa =
    32) beside the headline's uniform rows: the neighbour search and list
    ranking (part of the tree build), one FP64 pipelined skeletonize +
    factorize, the ranks, the 4-RHS direct residual, and the approximation
    error |Ktilde u - K u| / |K u| on 64 random rows (u ~ N(0,1), K u summed
    exactly with torch) for both samplings.  k_knn is reported against the
    FP64 vector peak on the points it actually compared (3 d flops per
    pair: difference and fma), and against the brute-force pair count."""
    N, d = X.shape
    h, m, s, nsamp, seed = c["h"], c["m"], c["s"], c["nsamp"], c["seed"]
    gen = torch.Generator().manual_seed(5)
    ridx = torch.randperm(N, generator=gen)[:rows].to(dev)
    u = B[:, :1].contiguous()
    Xr = X[ridx]
    Ku = torch.zeros(rows, 1, dtype=torch.float64, device=dev)
    for j0 in range(0, N, 1 << 16):
        d2 = torch.cdist(Xr, X[j0:j0 + (1 << 16)], compute_mode="donot_use_mm_for_euclid_dist") ** 2
        Ku += torch.exp(-d2 / (2.0 * h * h)) @ u[j0:j0 + (1 << 16)]

    def eps(f):
        kt = f.matvec(u)[ridx] - lam * u[ridx]
        return float((kt - Ku).norm() / Ku.norm())

    ak.askit_profile_enable(True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    tk = ak.Tree(X, m, s, h, n_samples=nsamp, seed=seed, knn=kappa)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - a
    prof = ak.askit_profile_report()
    ak.askit_profile_enable(False)
    st = tk.stats()
    f = tk.skeletonize_factorize(lam)
    f.close()
    torch.cuda.synchronize()
    a = time.perf_counter()
    f = tk.skeletonize_factorize(lam)
    torch.cuda.synchronize()
    t_sf = time.perf_counter() - a
    ranks, _ = tk.skeleton_sizes()
    _, _, nlen = tk.neighbor_lists()
    B4 = B[:, :4].contiguous()
    res = float(((B4 - f.matvec(f.solve(B4))).norm(dim=0) / B4.norm(dim=0)).max())
    e_knn = eps(f)
    f.close()
    fu = tree.factorize(lam, ak.ASKIT_FP64)
    e_uni = eps(fu)
    fu.close()
    ranks_u, _ = tree.skeleton_sizes()
    tk.close()
    lv = lambda r: [round(float(r[(1 << l) - 1:(2 << l) - 1].mean()), 1) for l in range(1, len(r).bit_length())]
    knn_ms = prof.get("tree:k_knn", (0.0, 1))[0]
    pairs = float(st["knn_wave_points"]) * 64.0
    out = {
        "kappa": kappa, "tree_build_s": t_build, "neighbour_search_and_lists_s": st["knn_ms"] / 1e3,
        "kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if k.startswith("tree:k_knn") or
                       k.startswith("tree:k_nbr")},
        "k_knn_roofline": {"bound": "alu", "pairs_compared": pairs, "achieved": 3.0 * d * pairs / (knn_ms * 1e-3) / 1e12,
                           "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                           "brute_force_pairs": float(N) * (N - 1),
                           "brute_force_equivalent_tflops": 3.0 * d * N * (N - 1.0) / (knn_ms * 1e-3) / 1e12},
        "mean_list_length_by_level": lv(nlen.astype(np.float64)),
        "skeletonize_factorize_s": t_sf, "direct_residual_4rhs": res,
        "mean_rank_by_level": {"knn": lv(ranks.astype(np.float64)), "uniform": lv(ranks_u.astype(np.float64))},
        "approx_error_64_rows": {"knn": e_knn, "uniform": e_uni},
    }
    r = out["k_knn_roofline"]
    r["frac"] = r["achieved"] / r["peak"]
    log(f"[bench] knn sampling: {out}")
    return out


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
    # hybrid solver (level restriction, Sec. 2.3) on the same tree, 4
    # right-hand sides: level 1 keeps the matrix of the direct method (the
    # root's reduced system solved by GMRES instead of its LU), level 3
    # leaves the top three levels uncompressed
    B4 = B[:, :4].contiguous()
    x4 = f.solve(B4)
    out["fp64_direct_residual_4rhs"] = float(((B4 - f.matvec(x4)).norm(dim=0) / B4.norm(dim=0)).max())
    f.close()
    ranks, _ = tree.skeleton_sizes()
    hyb = {}
    for L in (1, 3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        fh = tree.factorize_hybrid(lam, L)
        torch.cuda.synchronize()
        b = time.perf_counter()
        xh = fh.solve(B4)
        torch.cuda.synchronize()
        e = time.perf_counter()
        info = fh.info()
        res = float(((B4 - fh.matvec(xh)).norm(dim=0) / B4.norm(dim=0)).max())
        hyb[f"level_{L}"] = {"factorize_s": b - a, "solve_s": e - b, "gmres": info, "residual": res,
                             "reduced_order": int(ranks[(1 << L) - 1:(2 << L) - 1].sum())}
        log(f"[bench] hybrid level {L}: factorize {b - a:.3f} s solve {e - b:.3f} s {info} residual {res:.2e}")
        fh.close()
    out["hybrid_4rhs"] = hyb
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
    # solutions of eight problems spread over the batch, for the oracle
    # comparison of the CPU leg
    xs = batch.solve(Bs)
    torch.cuda.synchronize()
    pick = list(range(0, len(probs), len(probs) // 8))[:8]
    out["_batched_sample"] = [(probs[i], xs[i].cpu().numpy(), trees[i].export_skeletons(), trees[i].cmax)
                              for i in pick]
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
    out["gate_pass"] = bool(out["mixed_vs_fp64_rel_err"] <= MIXED_GATE and out["mixed_refinement"]["converged"])
    log(f"[bench] stable config: mixed vs fp64 {out['mixed_vs_fp64_rel_err']:.2e}, "
        f"mixed refinement {out['mixed_refinement']}")
    t.close()
    return out


def cpu_baseline(c, n_sample):
    """The oracle (plain C, OpenMP over the nodes of a level) on a bounded
    sample of the workload: the first n_sample points of the mixture with the
    same d, m, s, h, lambda and sample count; its skeletonize + factorize time
    is scaled to N by the method's N log(N/m) work (Sec. 3, "Work").  The
    default run times the whole workload instead."""
    import oracle
    X = c["X"][:n_sample]
    m, s = c["m"], c["s"]
    o = oracle.Oracle(X, m, s, c["h"], nsamp=c["nsamp"], seed=c["seed"])
    o.build_tree()
    nth = oracle.num_threads()
    log(f"[bench] cpu baseline: oracle on {n_sample} points, {nth} threads")
    a = time.perf_counter()
    o.skeletonize()
    b = time.perf_counter()
    o.factorize(c["lam"])
    e = time.perf_counter()
    N = c["X"].shape[0]
    Dn = max(1, int(np.ceil(np.log2(n_sample / m))))
    DN = max(1, int(np.ceil(np.log2(N / m))))
    scale = (N * DN) / (n_sample * Dn)
    log(f"[bench] cpu baseline: skeletonize {b - a:.2f} s factorize {e - b:.2f} s (sample)")
    return {"value": (e - a) * scale, "unit": "s", "cores": nth, "kind": "oracle",
            "sample": f"first {n_sample} points of the workload (depth {Dn}): skeletonize+factorize "
                      f"{e - a:.2f} s measured, scaled by N log(N/m) to N={N} (depth {DN})"}


def cpu_full_check(c, tree, ids, P, sizes, x64, xref, nrhs_check, check):
    """The oracle (plain C, OpenMP over the nodes of a level) on the whole
    workload: its skeletonize + factorize time is the CPU baseline.  With
    `check` it then compares the GPU's results: the tree permutation bit for
    bit, the skeletons node by node (pivots identical), and, factored on the
    GPU's own skeletons, the GPU's FP64 direct and refined solutions of the
    first nrhs_check right-hand sides against the oracle's solution and
    operator."""
    import oracle
    X, B = c["X"], c["B"]
    N = X.shape[0]
    m, s = c["m"], c["s"]
    nth = oracle.num_threads()
    log(f"[bench] cpu baseline: oracle on the whole workload (N={N}), {nth} threads")
    o = oracle.Oracle(X, m, s, c["h"], nsamp=c["nsamp"], seed=c["seed"])
    a = time.perf_counter()
    perm = o.build_tree()
    b = time.perf_counter()
    o.skeletonize()
    e = time.perf_counter()
    o.factorize(c["lam"])
    g = time.perf_counter()
    log(f"[bench] cpu baseline: tree {b - a:.1f} s, skeletonize {e - b:.1f} s, factorize {g - e:.1f} s")
    out = {"value": g - b, "unit": "s", "cores": nth, "kind": "oracle",
           "sample": f"the whole workload (N={N}); skeletonize {e - b:.2f} s + factorize {g - e:.2f} s",
           "tree_s": b - a}
    if not check:
        return out
    check = {"perm_bit_exact": bool(np.array_equal(perm, tree.perm().cpu().numpy()))}
    # skeletons: identical pivot lists per node (internal nodes are compared
    # only where both children agree, since their candidates differ otherwise)
    nn = tree.nnodes
    same = np.zeros(nn, dtype=bool)
    comparable = 0
    for node in range(nn - 1, 0, -1):
        leaf = node >= (1 << tree.D) - 1
        if not leaf and not (same[2 * node + 1] and same[2 * node + 2]):
            continue
        comparable += 1
        pos, _, _ = o.skeleton(node)
        sr = int(sizes[2 * node])
        same[node] = sr == len(pos) and np.array_equal(ids[node * s: node * s + sr], pos)
    check["skeleton_nodes_identical"] = int(same.sum())
    check["skeleton_nodes_compared"] = comparable
    check["skeleton_nodes"] = nn - 1
    # factor on the GPU's skeletons and compare solutions
    cm = tree.cmax
    for node in range(1, nn):
        sr, nc = int(sizes[2 * node]), int(sizes[2 * node + 1])
        o.set_skeleton(node, ids[node * s: node * s + sr],
                       P[node * s * cm: node * s * cm + sr * nc].reshape(sr, nc))
    o.factorize(c["lam"])
    k = nrhs_check
    Bk = B[:, :k]
    xo = o.solve(Bk)
    xg = x64[:, :k].cpu().numpy()
    xr = xref[:, :k].cpu().numpy()
    nb = np.linalg.norm(Bk, axis=0)

    def rel(u, v):
        return float((np.linalg.norm(u - v, axis=0) / np.linalg.norm(v, axis=0)).max())

    check["gpu_fp64_direct_vs_oracle_direct"] = rel(xg, xo)
    check["oracle_direct_residual"] = float((np.linalg.norm(Bk - o.matvec(xo), axis=0) / nb).max())
    check["gpu_fp64_direct_residual_oracle_operator"] = float((np.linalg.norm(Bk - o.matvec(xg), axis=0) / nb).max())
    check["gpu_fp64_refined_residual_oracle_operator"] = float((np.linalg.norm(Bk - o.matvec(xr), axis=0) / nb).max())
    check["gpu_fp64_refined_vs_oracle_direct"] = rel(xr, xo)
    check["rhs_checked"] = k
    out["check"] = check
    log(f"[bench] cpu check: {check}")
    return out


def cpu_batched_check(sample):
    """The batched workload against the oracle, problem by problem (the
    structure of the full check of the 1M workload):
      - skeletons: the oracle's own skeletonization against the GPU's batched
        one, node by node (identical pivot lists; internal nodes compared
        where both children agree);
      - solve: the oracle factored on the GPU's skeletons (the same operator
        lambda I + Ktilde) against the GPU's batched FP64 solution (hipGraph
        replay), 8 right-hand sides, and the GPU solution's residual under
        the oracle's operator;
      - own skeletons: the two solutions each on its own skeletons, for
        information (where the skeletons differ, so do the operators)."""
    import oracle
    rows = []
    a = time.perf_counter()
    for p, xg, (ids, P, sizes), cmax in sample:
        s = p["s"]
        o = oracle.Oracle(p["X"], p["m"], s, p["h"], nsamp=p["nsamp"], seed=p["seed"], problem=p["problem"])
        o.build_tree()
        o.skeletonize()
        o.factorize(p["lam"])
        B = p["B"]
        x_own = o.solve(B)
        nn = o.nnodes
        same = np.zeros(nn, dtype=bool)
        compared = 0
        for node in range(nn - 1, 0, -1):
            leaf = node >= (1 << o.D) - 1
            if not leaf and not (same[2 * node + 1] and same[2 * node + 2]):
                continue
            compared += 1
            pos, _, _ = o.skeleton(node)
            sr = int(sizes[2 * node])
            same[node] = sr == len(pos) and np.array_equal(ids[node * s: node * s + sr], pos)
        for node in range(1, nn):
            sr, nc = int(sizes[2 * node]), int(sizes[2 * node + 1])
            o.set_skeleton(node, ids[node * s: node * s + sr],
                           P[node * s * cmax: node * s * cmax + sr * nc].reshape(sr, nc))
        o.factorize(p["lam"])
        xo = o.solve(B)
        nb = np.linalg.norm(B, axis=0)
        rel = lambda u, v: float((np.linalg.norm(u - v, axis=0) / np.linalg.norm(v, axis=0)).max())
        rows.append({"problem": p["problem"], "N": len(p["X"]), "lambda": p["lam"], "h": p["h"],
                     "skeleton_nodes_identical": int(same.sum()), "skeleton_nodes_compared": compared,
                     "skeleton_nodes": nn - 1,
                     "gpu_vs_oracle_same_skeletons": rel(xg, xo),
                     "gpu_residual_oracle_operator": float((np.linalg.norm(B - o.matvec(xg), axis=0) / nb).max()),
                     "oracle_residual": float((np.linalg.norm(B - o.matvec(xo), axis=0) / nb).max()),
                     "gpu_vs_oracle_own_skeletons": rel(xg, x_own)})
    out = {"problems": rows, "seconds": time.perf_counter() - a,
           "max_gpu_vs_oracle_same_skeletons": max(r["gpu_vs_oracle_same_skeletons"] for r in rows),
           "max_gpu_residual_oracle_operator": max(r["gpu_residual_oracle_operator"] for r in rows)}
    log(f"[bench] batched check: GPU vs oracle on the same skeletons max {out['max_gpu_vs_oracle_same_skeletons']:.2e}, "
        f"GPU residual under the oracle's operator max {out['max_gpu_residual_oracle_operator']:.2e}; skeleton nodes "
        f"identical {[r['skeleton_nodes_identical'] for r in rows]} of {[r['skeleton_nodes'] for r in rows]}")
    return out


if __name__ == "__main__":
    main()
