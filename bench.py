#!/usr/bin/env python3
"""Benchmark of the FP64 RBT + GENP solve on one MI355X.

One step = the whole method on one system: coefficient draw, the fused
two-sided transform A~ = U^T A V, b~ = U^T b, elimination without pivoting,
the two triangular solves, x = V x~, then the Eq. 7 backward error and FP64
refinement steps until it is <= 10 n eps (the usual outcome is zero or one
step). Inputs (A ~ N(0,1), b ~ N(0,1), seeds 42 / 64) are resident in HBM
before the timed region. Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 20000] [--nrhs 1]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solve TFLOP/s (2/3·n³) RBT+GENP vs GEPP at n=20000; backward error; GB/s"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0

# HBM bytes per launch of a benchmark's dominant kernel, from rocprofv3 counter
# runs (FETCH_SIZE x 2 + WRITE_SIZE x 1 in KiB, scaled by a plain copy of known
# size): valid only while the kernel's source is the one the counters were taken
# with, and for the configuration they were taken on.
KERNEL_TRAFFIC = {
    "fp64": {"source": "paper_2312_09376_amd/csrc/k_gemm.hip",
             "sha256": "cd064f89968f0e242177948f6fad7a7d0a8deea95567454ad17bee080fbabd6a",
             "config": {"n": 20000, "nrhs": 1, "depth": 2, "outer_nb": 2048},
             "bytes_per_launch": (2 * 3752645.5 + 957781.3) * 1024},
    "bf16": {"source": "paper_2312_09376_amd/csrc/k_hgemm.hip",
             "sha256": "a2e326c4190c3373b06045510896c621b5b597abc03e3147a85aefe0e7c2de42",
             "config": {"n": 32768, "nrhs": 1, "depth": 2, "outer_nb": 2048, "matrix": "dominant"},
             # k_hgemm plus its two operand conversions (the timed trailing stage)
             "bytes_per_launch": ((2 * 1811397.4 + 1448020.9) + (2 * 65548.8 + 109875.7)
                                  + (2 * 65561.2 + 65536.0)) * 1024},
    # (re-hashed after a change to the BF16 panel-update launcher only; the
    # FP32 trailing kernel the counters cover is unchanged)
    "fp32": {"source": "paper_2312_09376_amd/csrc/k_sgemm.hip",
             "sha256": "e0d176a1042a66d7e65237b7e4d0f0b3e0e86603bf87ca1447bb13bee746c02d",
             "config": {"n": 32768, "nrhs": 1, "depth": 2, "outer_nb": 2048, "matrix": "dominant"},
             "bytes_per_launch": (2 * 4755728.4 + 1354453.7) * 1024},
    "batched_fp32": {"source": "paper_2312_09376_amd/csrc/k_batched.hip",
                     "sha256": "7e5d2b3d29a20b2468be1b6161cc084487143fdd8f6bf71a4c5aabd6ae2384d9",
                     "config": {"batch": 2048, "depth": 2, "matrix": "randn"},
                     "bytes_per_launch": (2 * 172929152.5 + 95883867.0) * 1024},
}


def stage_breakdown(rbt, step, steps):
    """Per-stage milliseconds per step from `steps` extra steps with every
    stage timed. Each timed scope records two events on the stream (a few
    microseconds of device time apiece), so the measured steps time only the
    kernels the benchmark line reports and the breakdown comes from here."""
    import torch
    if steps <= 0:
        return {}
    torch.cuda.synchronize()
    rbt.timing_read()
    rbt.timing_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    rbt.timing_enable(False)
    return {s_: round(v[0] / steps, 3) for s_, v in rbt.timing_read().items()}


def trailing_shapes(n, W, remainder=True):
    """(rc, w) of every trailing update of the blocked elimination: rc rows
    and columns remain right of a panel of width w. The first panel also takes
    the n mod 128 columns (not with BF16 updates: remainder=False)."""
    k0, w = 0, min(n, W + (n % 128 if remainder else 0))
    out = []
    while n - k0 - w > 0:
        out.append((n - k0 - w, w))
        k0 += w
        w = min(n - k0, W)
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--depth", type=int, default=2)
    ap.add_argument("--seed", type=int, default=2023)
    ap.add_argument("--max-iter", type=int, default=10)
    ap.add_argument("--no-gepp", action="store_true", help="skip the GEPP comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--stage-steps", type=int, default=2,
                    help="extra steps after the measured ones with every stage timed, for the "
                         "stage breakdown (the measured steps time only the reported kernels)")
    ap.add_argument("--cpu-panels", type=int, default=4,
                    help="oracle sample: panels (of 256 columns) of the benchmarked elimination")
    ap.add_argument("--lookahead", type=int, default=-1, help="0/1 (-1: library default)")
    ap.add_argument("--panel-split", type=int, default=-1,
                    help="order inside a panel: 0 block by block, 1 recursive halves "
                         "(-1: library default)")
    ap.add_argument("--outer-nb", type=int, default=0,
                    help="panel width of the elimination (multiple of 128; 0 = library default)")
    ap.add_argument("--mode", choices=["solve", "mixed", "batched", "backward", "copy", "small"],
                    default="solve",
                    help="solve: the FP64 step (default); mixed: FP32/BF16 elimination with FP64 "
                         "refinement; copy: a plain FP64 matrix copy through the transform kernel "
                         "at depth 0 (reference point for HBM byte counters); small: the "
                         "n = 1000 / 1001 / 1003 FP64 solves beside the single-threaded oracle")
    ap.add_argument("--prec", choices=["fp32", "bf16", "fp64"], default="fp32",
                    help="mixed / batched / backward modes (fp64: backward mode only)")
    ap.add_argument("--solver", choices=["classic", "gmres"], default="classic", help="mixed mode")
    ap.add_argument("--guarded", action="store_true",
                    help="mixed mode: fall back to FP64 factors when the low-precision "
                         "refinement cannot reach tol (max-iter is then its budget)")
    ap.add_argument("--max-iter64", type=int, default=10, help="guarded mixed mode: FP64 budget")
    ap.add_argument("--batch", type=int, default=2048, help="batched mode: number of systems")
    ap.add_argument("--streams", type=int, default=16,
                    help="backward mode: host threads, one stream each, over which the "
                         "independent systems are dealt")
    ap.add_argument("--batch-n", type=int, default=0,
                    help="batched mode: all systems of this order (0: n ~ U{37..1500})")
    ap.add_argument("--batch-nrhs", type=int, default=0,
                    help="batched mode: all systems with this many right-hand sides (0: U{1..16})")
    ap.add_argument("--batch-tile-cols2-min-n", type=int, default=-1,
                    help="batched mode: systems with n >= this take two 64-column tiles per "
                         "trailing-update round, smaller ones one (-1: tuned)")
    ap.add_argument("--batch-wgs", type=int, default=0,
                    help="batched mode: persistent workgroups per CU (0: tuned)")
    ap.add_argument("--tol-scale", type=float, default=10.0,
                    help="batched mode: refine to tol-scale * n * eps per system (0: max_iter steps)")
    ap.add_argument("--matrix", choices=["randn", "logcond", "dominant", "hostile", "orthog"],
                    default="randn",
                    help="solve / mixed modes: N(0,1); Q1 diag(10^-6 .. 1) Q2^T with Haar Q1, Q2 "
                         "(cond 1e6); I + 0.3 N(0,1)/sqrt(n); N(0,1) with the leading 8 x 8 block "
                         "scaled by 1e-12 (solve mode); the orthog matrix (solve mode, guarded)")
    ap.add_argument("--guarded-solve", action="store_true",
                    help="solve mode: rbt_solve_guarded (FP64 RBT, then partial pivoting if "
                         "refinement cannot reach tol)")
    return ap.parse_args()


def copy_mode(args):
    """Depth-0 transform = plain out-of-place copy of an n x n FP64 matrix
    (8 n^2 bytes read, 8 n^2 bytes written per launch)."""
    import torch
    from paper_2312_09376_amd import rbt, workloads
    n = args.n
    A = workloads.device_randn(n, n, workloads.MATRIX_SEED)
    out = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        rbt.transform2(A, None, None, 0, out=out)
    torch.cuda.synchronize()
    rbt.timing_read()
    rbt.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rbt.transform2(A, None, None, 0, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rbt.timing_enable(False)
    ms, cnt, nbytes = rbt.timing_read()["transform2"]
    gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    ms_step = (t1 - t0) * 1e3 / args.steps
    print(json.dumps({
        "metric": "FP64 matrix copy GB/s (reference point for HBM byte counters)",
        "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"copy of an n x n FP64 matrix, n={n}", "n": n,
                   "bytes_per_launch": 16 * n * n},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None},
        "cpu_baseline": None}), flush=True)


def measured_traffic(key, **config):
    import hashlib
    t = KERNEL_TRAFFIC.get(key)
    if t is None:
        return None
    try:
        with open(os.path.join(ROOT, t["source"]), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if digest != t["sha256"] or any(config.get(k) != v for k, v in t["config"].items()):
        return None
    return t["bytes_per_launch"]


def mixed_mode(args):
    """One step = rbt_solve_mixed: transform to FP32, elimination with FP32 or
    BF16 updates, FP64 refinement to 10 n eps (or max_iter)."""
    import torch
    from paper_2312_09376_amd import rbt, workloads

    n, k, d = args.n, args.nrhs, args.depth
    tol = 10.0 * n * 2.0 ** -52
    prec = rbt.RBT_FP32 if args.prec == "fp32" else rbt.RBT_BF16
    solver = rbt.RBT_IR_CLASSIC if args.solver == "classic" else rbt.RBT_IR_GMRES
    if args.matrix == "randn":
        A = workloads.device_randn(n, n, workloads.MATRIX_SEED)
    elif args.matrix == "logcond":
        A = workloads.device_logcond(n, workloads.MATRIX_SEED)
    else:
        A = workloads.device_randn(n, n, workloads.MATRIX_SEED) * (0.3 / math.sqrt(n))
        A.diagonal().add_(1.0)
    B = workloads.device_randn(n, k, workloads.RHS_SEED)
    LU = torch.empty_strided((n, n), (1, n), dtype=torch.float32, device="cuda")
    LU64 = (torch.empty_strided((n, n), (1, n), dtype=torch.float64, device="cuda")
            if args.guarded else None)
    X = torch.empty_strided((n, k), (1, n), dtype=torch.float64, device="cuda")
    work = rbt._workspace(n, k, d, A.device, prec)
    torch.cuda.synchronize()

    def step():
        if args.guarded:
            X_, _, _, it_, be_, info_, path_, _ = rbt.solve_mixed_guarded(
                A, B, d, args.seed, prec=prec, solver=solver, tol=tol, max_iter=args.max_iter,
                max_iter64=args.max_iter64, LU=LU, LU64=LU64, X=X, work=work)
            return X_, None, (it_, path_), be_, info_, None
        return rbt.solve_mixed(A, B, d, args.seed, prec=prec, solver=solver, tol=tol,
                               max_iter=args.max_iter, LU=LU, X=X, work=work)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rbt.timing_read()
    rbt.timing_enable(True, stages=("trailing",))
    iters = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, it, be, info, _ = step()
        iters.append(it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rbt.timing_enable(False)
    stages = rbt.timing_read()
    tr_ms, tr_cnt, tr_work = stages["trailing"]
    # A guarded step that falls back to FP64 factors adds the FP64 trailing
    # updates of that factorization to the stage. The low-precision
    # factorization runs in every step, so one solve without the fallback,
    # timed alone, separates the two kernels.
    fb_steps = sum(1 for i in iters if int(i[1].item()) != 0) if args.guarded else 0
    lp_ms, lp_cnt, lp_work = tr_ms, tr_cnt, tr_work
    if fb_steps:
        rbt.timing_enable(True, stages=("trailing",))
        rbt.solve_mixed(A, B, d, args.seed, prec=prec, solver=solver, tol=tol, max_iter=1,
                        LU=LU, X=X, work=work)
        torch.cuda.synchronize()
        rbt.timing_enable(False)
        one_ms, one_cnt, one_work = rbt.timing_read()["trailing"]
        lp_ms, lp_cnt, lp_work = (one_ms * args.steps, one_cnt * args.steps,
                                  one_work * args.steps)
    breakdown = stage_breakdown(rbt, step, args.stage_steps)  # also restores X
    ms_step = (t1 - t0) * 1e3 / args.steps
    flops = (2.0 / 3.0) * n ** 3
    berr = float(be.item())
    peak = PEAK_FP32_MFMA_TFLOPS if args.prec == "fp32" else PEAK_BF16_MFMA_TFLOPS
    gemm_tflops = lp_work / (lp_ms * 1e-3) / 1e12 if lp_ms > 0 else 0.0
    W = rbt.get_option(rbt._lib.RBT_OPT_OUTER_NB)
    # BF16 updates run the staged k_hgemm (the trailing stage then also holds
    # its two operand conversions)
    staged = (args.prec == "bf16" and rbt.get_option(rbt._lib.RBT_OPT_BF16_STAGED) == 1)
    tr_bytes = sum(8.0 * rc * rc + 8.0 * rc * w for rc, w in
                   trailing_shapes(n, W, args.prec != "bf16")) * args.steps
    low_roofline = {
        "bound": "mfma",
        "kernel": ("trailing-update GEMM (k_hgemm and its operand staging, BF16 MFMA)"
                   if staged else f"trailing-update GEMM (k_sgemm, {args.prec.upper()} MFMA)"),
        "achieved": round(gemm_tflops, 3), "peak": peak, "unit": "TFLOP/s",
        "frac": round(gemm_tflops / peak, 4),
        "traffic": measured_traffic("bf16" if staged else args.prec, n=n, nrhs=k, depth=d,
                                    outer_nb=W, matrix=args.matrix),
        "algorithmic_bytes_per_launch": tr_bytes / max(lp_cnt, 1),
        "launches": lp_cnt, "avg_launch_ms": round(lp_ms / max(lp_cnt, 1), 4),
        "flops_per_launch": lp_work / max(lp_cnt, 1)}
    roofline, other = low_roofline, None
    if fb_steps:
        f_ms, f_cnt, f_work = tr_ms - lp_ms, tr_cnt - lp_cnt, tr_work - lp_work
        f_tflops = f_work / (f_ms * 1e-3) / 1e12 if f_ms > 0 else 0.0
        f_bytes = sum(16.0 * rc * rc + 16.0 * rc * w for rc, w in
                      trailing_shapes(n, W, True)) * fb_steps
        fp64_roofline = {
            "bound": "mfma", "kernel": "FP64 fallback trailing-update GEMM (k_dgemm, FP64 MFMA)",
            "achieved": round(f_tflops, 3), "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": round(f_tflops / PEAK_FP64_MFMA_TFLOPS, 4),
            "traffic": measured_traffic("fp64", n=n, nrhs=k, depth=d, outer_nb=W),
            "algorithmic_bytes_per_launch": f_bytes / max(f_cnt, 1),
            "launches": f_cnt, "avg_launch_ms": round(f_ms / max(f_cnt, 1), 4),
            "flops_per_launch": f_work / max(f_cnt, 1)}
        # the roofline line is the kernel with more time in the step
        if f_ms > lp_ms:
            roofline, other = fp64_roofline, low_roofline
        else:
            other = fp64_roofline
    out = {
        "metric": f"mixed-precision solve TFLOP/s (2/3·n³, FP64-accurate result), "
                  f"{args.prec.upper()} elimination + FP64 {args.solver} refinement",
        "value": round(flops / (ms_step * 1e-3) / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"RBT+GENP {args.prec.upper()} elimination, FP64 {args.solver} "
                               f"refinement to berr<=10*n*eps, n={n}, nrhs={k}, depth {d}, "
                               f"A={args.matrix} seed 42, b~N(0,1) seed 64",
                   "n": n, "nrhs": k, "depth": d, "outer_nb": W, "matrix": args.matrix,
                   "lookahead": rbt.get_option(rbt._lib.RBT_OPT_LOOKAHEAD),
                   "panel_split": rbt.get_option(rbt._lib.RBT_OPT_PANEL_SPLIT)},
        "roofline": roofline,
        "berr": berr, "berr_tol": tol, "converged": berr <= tol,
        "stages_ms_per_step": breakdown,
        "cpu_baseline": None,
    }
    if other is not None:
        out["roofline_other_kernel"] = other
    if args.guarded:
        out["config"]["guarded"] = True
        out["ir_steps"] = [[int(v) for v in i[0].cpu()] for i in iters]  # [low prec, FP64]
        out["fp64_fallback"] = [int(i[1].item()) for i in iters]  # path: 0, 1 RBT64, 2 GEPP
        out["info"] = [int(v) for v in info.cpu()]
    else:
        out["ir_steps"] = [int(i.item()) for i in iters]
        out["info"] = int(info.item())
    if not args.no_gepp:
        out["gepp"] = gepp_comparator(A, B, flops, ms_step, X=X)
    print(json.dumps(out), flush=True)


def gepp_comparator(A, B, flops, ms_step, reps=2, X=None):
    """FP64 partial-pivoting solve of the same system on the same GPU (torch ->
    rocSOLVER getrf/getrs) and its Eq. 7 backward error; with X (this
    library's solution), also max|X - X_gepp| / max|X_gepp|."""
    import torch
    from paper_2312_09376_amd import rbt
    Xg = torch.linalg.solve(A, B)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(reps):
        Xg = torch.linalg.solve(A, B)
    torch.cuda.synchronize()
    g_ms = (time.perf_counter() - g0) * 1e3 / reps
    gb = float(rbt.backward_error(A, Xg.t().contiguous().t(), B).item())
    out = {"solver": "torch.linalg.solve FP64 (partial pivoting)", "ms": round(g_ms, 3),
           "TFLOP/s": round(flops / (g_ms * 1e-3) / 1e12, 4), "berr": gb,
           "speedup_rbt": round(g_ms / ms_step, 3)}
    if X is not None:
        out["rel_diff_to_rbt_x"] = float(((X - Xg).abs().max() / Xg.abs().max()).item())
    return out


def batched_mode(args):
    """One step = one graph replay of rbt_solve_batched over the whole batch:
    `batch` systems with n ~ U{37..1500}, nrhs ~ U{1..16} (size seed 7),
    A_s ~ N(0,1) (seed 42 + s), B_s ~ N(0,1) (seed 64 + s); FP32 (or BF16
    update) elimination and FP64 refinement to 10 n_s eps per system."""
    import numpy as np
    import torch
    from paper_2312_09376_amd import rbt, workloads
    ns, ks = workloads.batch_sizes(count=args.batch)
    if args.batch_n:
        ns = np.full(args.batch, args.batch_n, dtype=np.int64)
    if args.batch_nrhs:
        ks = np.full(args.batch, args.batch_nrhs, dtype=np.int64)
    tol = -args.tol_scale
    prec = rbt.RBT_FP32 if args.prec == "fp32" else rbt.RBT_BF16
    d = args.depth
    As, Bs = [], []
    for s_, (n, k) in enumerate(zip(ns, ks)):
        if args.matrix == "dominant":
            A = workloads.device_randn(int(n), int(n), workloads.MATRIX_SEED + s_) * (0.3 / math.sqrt(n))
            A.diagonal().add_(1.0)
        else:
            A = workloads.device_randn(int(n), int(n), workloads.MATRIX_SEED + s_)
        As.append(A)
        Bs.append(workloads.device_randn(int(n), int(k), workloads.RHS_SEED + s_))
    # an explicit shape overrides the tuned table
    tuned = args.batch_tile_cols2_min_n < 0 and not args.batch_wgs
    if args.batch_tile_cols2_min_n >= 0:
        rbt.set_option(rbt._lib.RBT_OPT_BATCH_TILE_COLS2_MIN_N, args.batch_tile_cols2_min_n)
    if args.batch_wgs:
        rbt.set_option(rbt._lib.RBT_OPT_BATCH_WGS_PER_CU, args.batch_wgs)
    plan = rbt.batched_plan(ns, ks, d, prec)
    bargs = rbt.BatchArgs(plan, As, Bs)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        rbt.solve_batched_launch(plan, bargs, seed=args.seed, tol=tol, max_iter=args.max_iter,
                                 tuned=tuned)
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rbt.solve_batched_launch(plan, bargs, seed=args.seed, tol=tol, max_iter=args.max_iter,
                                 tuned=tuned)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_gpu = ev0.elapsed_time(ev1) / args.steps
    flops = float(np.sum((2.0 / 3.0) * ns.astype(np.float64) ** 3))
    iters = bargs.iters.cpu().numpy()
    berr = bargs.berr.cpu().numpy()
    info = bargs.info.cpu().numpy()
    path = bargs.path.cpu().numpy()
    tols = max(args.tol_scale, 10.0) * ns * 2.0 ** -52
    converged = int(np.sum(berr <= tols))
    peak = PEAK_FP32_MFMA_TFLOPS if args.prec == "fp32" else PEAK_BF16_MFMA_TFLOPS
    achieved = flops / (ms_gpu * 1e-3) / 1e12
    out = {
        "metric": "batched solve TFLOP/s (sum of 2/3 n^3 over the batch) and systems/s",
        "value": round(flops / (ms_step * 1e-3) / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"{args.batch} systems, "
                               + (f"n={args.batch_n}, " if args.batch_n else "n~U{37..1500}, ")
                               + (f"nrhs={args.batch_nrhs}, " if args.batch_nrhs else "nrhs~U{1..16} (seed 7), ")
                               + f"A={args.matrix} (seed 42+s), depth {d}, {args.prec.upper()} "
                               f"elimination + FP64 refinement to 10 n eps, one persistent "
                               f"launch replayed from a HIP graph",
                   "batch": args.batch, "depth": d, "matrix": args.matrix,
                   "sum_n2": int(np.sum(ns.astype(np.int64) ** 2)), "flops": flops,
                   "tile_cols2_min_n": rbt.get_option(rbt._lib.RBT_OPT_BATCH_TILE_COLS2_MIN_N),
                   "wgs_per_cu": rbt.get_option(rbt._lib.RBT_OPT_BATCH_WGS_PER_CU)},
        "systems_per_s": round(args.batch / (ms_step * 1e-3), 1),
        "roofline": {"bound": "mfma", "kernel": "k_batched (persistent, whole method per system)",
                     "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": (measured_traffic("batched_fp32", batch=args.batch, depth=d,
                                                  matrix=args.matrix)
                                 if args.prec == "fp32" and not args.batch_n and not args.batch_nrhs
                                 else None),
                     "avg_launch_ms": round(ms_gpu, 4), "flops_per_launch": flops},
        "converged": converged, "max_iters": int(iters.max()), "mean_iters": float(iters.mean()),
        "max_berr_over_tol": float(np.max(berr / tols)), "zero_pivots": int(np.sum(info != 0)),
        "fp64_fallbacks": int(np.sum(path != 0)),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def backward_mode(args):
    """One step = forward solve + adjoint (dA and dB for dL/dX = G) of each of
    `batch` systems: A_s = N(0,1)/sqrt(n) + I (seed 42 + s), B_s, G_s ~ N(0,1)
    (n x nrhs). fp64: FP64 solve with refinement and the FP64 adjoint;
    fp32/bf16: low-precision factors with FP64 GMRES refinement forward and
    FP64 refinement of the adjoint solve. The systems are independent: they
    are dealt round-robin to `--streams` host threads, each with its own
    stream, factors and workspace (the elimination of one system at these
    sizes is a chain of latency-bound launches that fills a fraction of the
    GPU)."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2312_09376_amd import rbt, workloads
    n, k, d = args.n, args.nrhs, args.depth
    nb = args.batch
    tol = 10.0 * n * 2.0 ** -52
    As = []
    for s_ in range(nb):
        A = workloads.device_randn(n, n, workloads.MATRIX_SEED + s_) / math.sqrt(n)
        A.diagonal().add_(1.0)
        As.append(A)
    Bs = [workloads.device_randn(n, k, workloads.RHS_SEED + s_) for s_ in range(nb)]
    Gs = [workloads.device_randn(n, k, 1000 + s_) for s_ in range(nb)]
    fp64 = args.prec == "fp64"
    prec = {"fp32": rbt.RBT_FP32, "bf16": rbt.RBT_BF16, "fp64": rbt.RBT_FP64}[args.prec]
    S = max(1, min(args.streams, nb))
    streams = [torch.cuda.Stream() for _ in range(S)]  # default priority
    bufs = []
    for _ in range(S):
        LU = torch.empty_strided((n, n), (1, n), dtype=torch.float64 if fp64 else torch.float32,
                                 device="cuda")
        X = torch.empty_strided((n, k), (1, n), dtype=torch.float64, device="cuda")
        bufs.append((LU, X, rbt._workspace(n, k, d, As[0].device, prec)))
    torch.cuda.synchronize()
    errs = []  # (forward berr, adjoint berr or None) tensors, read after the timing

    def part(t_, stride=S):
        LU, X, work = bufs[t_]
        out = []
        with torch.cuda.stream(streams[t_]):
            for i_ in range(t_, nb, stride):
                A, B, G = As[i_], Bs[i_], Gs[i_]
                if fp64:
                    _, _, _, be, _, _ = rbt.solve_refine(A, B, d, args.seed, tol=tol,
                                                         max_iter=args.max_iter, LU=LU, X=X,
                                                         work=work)
                    dA, dB = rbt.solve_backward(LU, X, G, d, args.seed, work=work)
                    bb = None
                else:
                    _, _, _, be, _, _ = rbt.solve_mixed(A, B, d, args.seed, prec=prec,
                                                        solver=rbt.RBT_IR_GMRES, tol=tol,
                                                        max_iter=args.max_iter, LU=LU, X=X,
                                                        work=work)
                    dA, dB, _, bb = rbt.solve_backward_mixed(LU, A, X, G, d, args.seed, tol=tol,
                                                             max_iter=args.max_iter, work=work)
                out.append((be, bb))
        return out

    pool = ThreadPoolExecutor(max_workers=S)

    def step():
        for out in pool.map(part, range(S)):
            errs.extend(out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rbt.timing_read()
    rbt.timing_enable(True, stages=("outer",))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    rbt.timing_enable(False)
    stages = rbt.timing_read()
    if S > 1:
        # in the timed steps the dA launches share the GPU with the other
        # streams' work; the kernel's own rate is timed in one pass over the
        # systems on one stream
        rbt.timing_enable(True, stages=("outer",))
        errs.extend(part(0, 1))
        torch.cuda.synchronize()
        rbt.timing_enable(False)
        stages = rbt.timing_read()
    breakdown = stage_breakdown(rbt, step, args.stage_steps)
    worst = {"fwd": max(float(e[0].item()) for e in errs),
             "bwd": max((float(e[1].item()) for e in errs if e[1] is not None), default=0.0)}
    flops = nb * (2.0 / 3.0) * n ** 3
    o_ms, o_cnt, o_bytes = stages["outer"]
    o_gbs = o_bytes / (o_ms * 1e-3) / 1e9 if o_ms > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": "k_neg_outer (dA = -Lambda X^T, a pure write)",
                "achieved": round(o_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(o_gbs / PEAK_HBM_GBS, 4), "traffic": None,
                "algorithmic_bytes_per_launch": 8.0 * n * n, "launches": o_cnt,
                "avg_launch_ms": round(o_ms / max(o_cnt, 1), 4),
                "timed": "in the timed steps" if S == 1 else "one pass on one stream"}
    # FP64 partial pivoting on the same GPU: factor, solve, adjoint solve
    # with the same factors and the outer product, per system
    gepp = None
    if not args.no_gepp:
        def gepp_part(t_):
            with torch.cuda.stream(streams[t_]):
                for i_ in range(t_, nb, S):
                    A, B, G = As[i_], Bs[i_], Gs[i_]
                    LUp, piv = torch.linalg.lu_factor(A)
                    Xp = torch.linalg.lu_solve(LUp, piv, B)
                    lam = torch.linalg.lu_solve(LUp, piv, G, adjoint=True)
                    dAp = -(lam @ Xp.t())
            return Xp, lam, dAp

        def gepp_step():  # the same streams and threads as the solves
            return list(pool.map(gepp_part, range(S)))[(nb - 1) % S]
        gepp_step()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        Xp, lam, _ = gepp_step()
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - g0) * 1e3
        gb = float(rbt.backward_error(As[-1], Xp.t().contiguous().t(), Bs[-1]).item())
        gepp = {"solver": "torch.linalg.lu_factor / lu_solve FP64 (partial pivoting), forward "
                          "and adjoint solves + dA", "ms": round(g_ms, 3),
                "berr_forward_last": gb, "speedup_rbt": round(g_ms / ms_step, 3)}
    out = {
        "metric": "solve + adjoint (dA, dB) throughput, TFLOP/s of the forward eliminations",
        "value": round(flops / (ms_step * 1e-3) / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"{nb} systems, n={n}, nrhs={k}, depth {d}, A=N(0,1)/sqrt(n)+I "
                               f"(seed 42+s), forward {args.prec.upper()} solve to 10 n eps + "
                               f"adjoint with dA", "batch": nb, "n": n, "nrhs": k, "depth": d,
                   "streams": S},
        "systems_per_s": round(nb / (ms_step * 1e-3), 2),
        "max_forward_berr": worst["fwd"], "max_adjoint_berr": worst["bwd"] if not fp64 else None,
        "berr_tol": tol, "roofline": roofline, "gepp": gepp,
        "stages_ms_per_step": breakdown,
        "cpu_baseline": None,
    }
    if S > 1:
        out["stages_note"] = "stage times are summed over the concurrent streams"
    print(json.dumps(out), flush=True)


def step_statistics(seconds):
    """Mean and 99 % confidence half-width (Student t) of per-step times, ms."""
    ms = [1e3 * x for x in seconds]
    k = len(ms)
    mean = sum(ms) / k
    if k < 2:
        return {"mean_ms": round(mean, 3), "ci99_ms": None, "n": k}
    from scipy import stats
    sd = math.sqrt(sum((x - mean) ** 2 for x in ms) / (k - 1))
    half = float(stats.t.ppf(0.995, k - 1)) * sd / math.sqrt(k)
    return {"mean_ms": round(mean, 3), "ci99_ms": round(half, 3), "n": k,
            "min_ms": round(min(ms), 3), "max_ms": round(max(ms), 3)}


def cpu_baseline(n, nrhs, depth, seed, panels=4, nb=256):
    """The oracle, as it stands, on the host cores, on a bounded sample of the
    benchmarked solve: the oracle's blocked elimination over the first
    `panels` panels (width nb) of the benchmarked n x n matrix (same seed).
    The elimination is 2/3 n^3 of the solve's flops and its cost does not
    depend on the values, so the sample takes the matrix as generated (the
    oracle's O(n^2) transform alone takes about a minute at n = 20000). The
    rate is the elimination flops of those panels over their time."""
    import numpy as np
    from oracle import solve as osolve
    from paper_2312_09376_amd import workloads
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    A = workloads.randn_matrix(n, seed=workloads.MATRIX_SEED)
    t0 = time.perf_counter()
    osolve.genp_blocked(A, nb=nb, max_panels=panels)
    t = time.perf_counter() - t0
    flops = 0.0
    for j in range(min(panels, (n + nb - 1) // nb)):
        k0 = j * nb
        w = min(nb, n - k0)
        r = n - k0 - w  # rows and columns after the panel
        flops += sum(2.0 * (n - k - 1) * (k0 + w - k - 1) for k in range(k0, k0 + w))  # in panel
        flops += w * (w - 1) * r  # U12
        flops += 2.0 * r * r * w  # Schur complement
    return {"value": round(flops / t / 1e12, 6), "unit": "TFLOP/s", "cores": int(threads),
            "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"the oracle's blocked elimination (nb={nb}) of the benchmarked n={n} "
                      f"matrix (same seed) over its first {panels} panels: {flops / 1e9:.1f} "
                      f"GFLOP in {t:.2f} s on {threads} BLAS threads of {os.cpu_count()} host "
                      f"CPUs (depth {depth}, nrhs {nrhs} solve; its O(n^2) transform, solves and "
                      f"refinement are not in the sample)"}


def oracle_small(n, depth, seed):
    """The oracle's unblocked elimination (plain right-looking, one BLAS
    thread) on the n x n N(0,1) system: seconds and its backward error."""
    import numpy as np
    from oracle import coeffs, solve as osolve
    from paper_2312_09376_amd import workloads
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(limits=1, user_api="blas")
    except Exception:
        import contextlib
        ctx = contextlib.nullcontext()
    A = workloads.randn_matrix(n, seed=workloads.MATRIX_SEED)
    B = workloads.randn(n, 1, seed=workloads.RHS_SEED)
    with ctx:
        t0 = time.perf_counter()
        U, V = coeffs.generate(n, depth, seed)
        X, LU, _ = osolve.rbt_solve(A, B, U, V, depth, nb=0)
        t = time.perf_counter() - t0
    return t, osolve.backward_error(A, X, B), A, B


def small_mode(args):
    """The n = 1000 / 1001 / 1003 workload (A, b ~ N(0,1), depth 2, FP64): the
    GPU solve with refinement to 10 n eps, timed over `steps` solves, beside
    the single-threaded oracle's unrefined solve."""
    import torch
    from paper_2312_09376_amd import rbt, workloads
    cells = []
    for n in (1000, 1001, 1003):
        t_o, be_o, A_h, B_h = oracle_small(n, args.depth, args.seed)
        A = torch.from_numpy(A_h.T.copy()).cuda().t()  # the oracle's bytes, column-major
        B = torch.from_numpy(B_h.T.copy()).cuda().t()
        tol = 10.0 * n * 2.0 ** -52
        LU = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device="cuda")
        X = torch.empty_strided((n, 1), (1, n), dtype=torch.float64, device="cuda")
        work = rbt._workspace(n, 1, args.depth, A.device)
        for _ in range(max(args.warmup, 1)):
            rbt.solve_refine(A, B, args.depth, args.seed, tol=tol, LU=LU, X=X, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, _, it, be, info, _ = rbt.solve_refine(A, B, args.depth, args.seed, tol=tol, LU=LU,
                                                     X=X, work=work)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        cells.append({"n": n, "gpu_ms": round(ms, 4),
                      "gpu_TFLOP/s": round((2.0 / 3.0) * n ** 3 / (ms * 1e-3) / 1e12, 4),
                      "gpu_berr": float(be.item()), "gpu_ir_steps": int(it.item()),
                      "oracle_s_1_thread": round(t_o, 3), "oracle_berr_unrefined": be_o,
                      "speedup": round(t_o * 1e3 / ms, 1)})
    print(json.dumps({
        "metric": "FP64 RBT+GENP solve time at n = 1000 / 1001 / 1003 (GPU, refined to 10 n eps) "
                  "and the single-threaded CPU oracle (seconds)",
        "value": cells[0]["gpu_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": cells[0]["gpu_ms"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "n=1000/1001/1003, A,b~N(0,1) seeds 42/64, depth 2, FP64"},
        "cells": cells, "roofline": None, "cpu_baseline": None}), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the single-system solve runs on one GPU and is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2312_09376_amd import rbt, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    # elimination options, for every mode that factors
    if args.outer_nb:
        rbt.set_option(rbt._lib.RBT_OPT_OUTER_NB, args.outer_nb)
    if args.lookahead >= 0:
        rbt.set_option(rbt._lib.RBT_OPT_LOOKAHEAD, args.lookahead)
    if args.panel_split >= 0:
        rbt.set_option(rbt._lib.RBT_OPT_PANEL_SPLIT, args.panel_split)
    if args.mode == "copy":
        copy_mode(args)
        return
    if args.mode == "mixed":
        mixed_mode(args)
        return
    if args.mode == "batched":
        batched_mode(args)
        return
    if args.mode == "backward":
        backward_mode(args)
        return
    if args.mode == "small":
        small_mode(args)
        return

    n, k, d = args.n, args.nrhs, args.depth
    tol = 10.0 * n * 2.0 ** -52

    if args.matrix == "hostile":
        A = workloads.device_hostile(n)
    elif args.matrix == "orthog":
        A = torch.from_numpy(workloads.orthog(n).T.copy()).cuda().t()
    elif args.matrix == "logcond":
        A = workloads.device_logcond(n, workloads.MATRIX_SEED)
    elif args.matrix == "dominant":
        A = workloads.device_randn(n, n, workloads.MATRIX_SEED) * (0.3 / math.sqrt(n))
        A.diagonal().add_(1.0)
    else:
        A = workloads.device_randn(n, n, workloads.MATRIX_SEED)
    B = workloads.device_randn(n, k, workloads.RHS_SEED)
    LU = torch.empty_strided((n, n), (1, n), dtype=torch.float64, device="cuda")
    X = torch.empty_strided((n, k), (1, n), dtype=torch.float64, device="cuda")
    work = rbt._workspace(n, k, d, A.device)
    torch.cuda.synchronize()
    paths = []

    def step():
        if args.guarded_solve:
            X_, LU_, it_, be_, info_, path_, w_ = rbt.solve_guarded(
                A, B, d, args.seed, tol=tol, max_iter=args.max_iter, LU=LU, X=X, work=work)
            paths.append(path_)
            return X_, LU_, it_[:1], be_, info_[:1], w_
        return rbt.solve_refine(A, B, d, args.seed, tol=tol, max_iter=args.max_iter, LU=LU, X=X,
                                work=work)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    rbt.timing_read()          # discard anything recorded so far
    # the measured steps time only the kernels this line reports (the
    # trailing update and the transform); the stage breakdown comes from
    # extra steps afterwards
    rbt.timing_enable(True, stages=("trailing", "transform2", "pivoted"))
    iters = []
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, it, be, info, _ = step()   # ends with a stream synchronization
        marks.append(time.perf_counter())
        iters.append(it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rbt.timing_enable(False)
    stages = rbt.timing_read()
    paths_measured = list(paths)
    breakdown = stage_breakdown(rbt, step, args.stage_steps)

    ms_step = (t1 - t0) * 1e3 / args.steps
    flops = (2.0 / 3.0) * n ** 3
    value = flops / (ms_step * 1e-3) / 1e12
    step_stats = step_statistics([b - a for a, b in zip([t0] + marks[:-1], marks)])
    berr = float(be.item())
    ir_steps = [int(i.item()) for i in iters]
    info_v = int(info.item())

    tr_ms, tr_cnt, tr_work = stages["trailing"]
    # algorithmic bytes of a trailing update: read + write A22 (16 rc^2) and
    # read L21, U12 (16 rc w); with flops 2 rc^2 w this is 8/w + 8/rc per flop
    W = rbt.get_option(rbt._lib.RBT_OPT_OUTER_NB)
    tr_bytes = sum(16.0 * rc * rc + 16.0 * rc * w for rc, w in trailing_shapes(n, W)) * args.steps
    gemm_avg_ms = tr_ms / max(tr_cnt, 1)
    gemm_tflops = tr_work / (tr_ms * 1e-3) / 1e12 if tr_ms > 0 else 0.0
    k1_ms, k1_cnt, k1_bytes = stages["transform2"]
    k1_gbs = k1_bytes / (k1_ms * 1e-3) / 1e9 if k1_ms > 0 else 0.0

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"RBT+GENP FP64 solve, n={n}, nrhs={k}, depth {d}, "
                               + ("A~N(0,1) seed 42" if args.matrix == "randn" else
                                  f"A={args.matrix} (seed 42)")
                               + ", b~N(0,1) seed 64, FP64 refinement to berr<=10*n*eps"
                               + (", partial-pivoting fallback" if args.guarded_solve else ""),
                   "n": n, "nrhs": k, "depth": d, "matrix": args.matrix,
                   "outer_nb": rbt.get_option(rbt._lib.RBT_OPT_OUTER_NB),
                   "lookahead": rbt.get_option(rbt._lib.RBT_OPT_LOOKAHEAD),
                   "panel_split": rbt.get_option(rbt._lib.RBT_OPT_PANEL_SPLIT)},
        "roofline": {"bound": "mfma", "kernel": "trailing-update GEMM (k_dgemm, FP64 MFMA)",
                     "achieved": round(gemm_tflops, 3), "peak": PEAK_FP64_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(gemm_tflops / PEAK_FP64_MFMA_TFLOPS, 4),
                     "traffic": measured_traffic("fp64", n=n, nrhs=k, depth=d,
                                                 outer_nb=rbt.get_option(rbt._lib.RBT_OPT_OUTER_NB)),
                     "traffic_unit": "bytes per launch (HBM read + write, counter runs)",
                     "algorithmic_bytes_per_launch": tr_bytes / max(tr_cnt, 1),
                     "launches": tr_cnt,
                     "avg_launch_ms": round(gemm_avg_ms, 4),
                     "flops_per_launch": tr_work / max(tr_cnt, 1)},
        "berr": berr,
        "berr_tol": tol,
        "ir_steps": ir_steps,
        "info": info_v,
        "transform2": {"GB/s": round(k1_gbs, 1), "frac_hbm": round(k1_gbs / PEAK_HBM_GBS, 4),
                       "avg_ms": round(k1_ms / max(k1_cnt, 1), 4),
                       "bytes_per_launch": k1_bytes / max(k1_cnt, 1)},
        "stages_ms_per_step": breakdown,
        "step_ms": step_stats,
    }
    if args.guarded_solve:
        out["paths"] = [int(p_.item()) for p_ in paths_measured[-args.steps:]]
        if stages["pivoted"][1]:
            out["pivoted_ms_per_step"] = round(stages["pivoted"][0] / args.steps, 3)

    if not args.no_gepp:
        # FP64 partial-pivoting LU solve on the same GPU (torch -> rocSOLVER)
        Xg = torch.linalg.solve(A, B)
        torch.cuda.synchronize()
        reps = 2
        g0 = time.perf_counter()
        for _ in range(reps):
            Xg = torch.linalg.solve(A, B)
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - g0) * 1e3 / reps
        gb = float(rbt.backward_error(A, Xg.t().contiguous().t(), B).item())
        out["gepp"] = {"solver": "torch.linalg.solve FP64 (partial pivoting)",
                       "ms": round(g_ms, 3), "TFLOP/s": round(flops / (g_ms * 1e-3) / 1e12, 4),
                       "berr": gb, "speedup_rbt": round(g_ms / ms_step, 3)}
        del Xg
        # this library's own partial-pivoting factorization and solve (the
        # Sec. 5 fallback's re-solve), one run
        LUg = A.clone()
        Xo = B.clone()
        torch.cuda.synchronize()
        o0 = time.perf_counter()
        _, ipiv, _ = rbt.gepp(LUg, work=work)
        rbt.gepp_solve(LUg, ipiv, Xo, work=work)
        torch.cuda.synchronize()
        o_ms = (time.perf_counter() - o0) * 1e3
        ob = float(rbt.backward_error(A, Xo, B).item())
        out["gepp_own"] = {"solver": "rbt_gepp + rbt_gepp_solve (this library, FP64)",
                           "ms": round(o_ms, 3), "TFLOP/s": round(flops / (o_ms * 1e-3) / 1e12, 4),
                           "berr": ob}
        del LUg, Xo

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, k, d, args.seed, panels=args.cpu_panels)
    else:
        out["cpu_baseline"] = None

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
