"""Autotuner for the batched solver's tile shape and launch shape.

rbt_solve_batched has two schedule parameters (library options):
  RBT_OPT_BATCH_TILE_COLS2_MIN_N  systems with n >= this take two 64-column
                                  tiles per round of the low-precision
                                  trailing update, smaller ones one: the
                                  tile shape per n-bucket,
  RBT_OPT_BATCH_WGS_PER_CU        persistent workgroups per compute unit (1
                                  or 2).
Neither changes any system's arithmetic, so every candidate must reproduce
the first candidate's solutions, iteration counts and backward errors bit for
bit; a candidate that does not is rejected. The candidate thresholds are the
bounds of the n-buckets (BUCKETS; 0: two tiles for all, NEVER: one for all).
Among the accepted candidates the fastest (median of graph replays of one
launch over the whole batch) wins.

    python -m paper_2312_09376_amd.tune [--batch 2048] [--prec fp32 bf16]

times every candidate on the GPU for a batch of the requested shape and
writes the winners to tuned_batched.json beside this file. BatchPlan reads
that table and solve_batched_launch applies the entry of the plan's
precision before each launch (without a table the library's defaults hold:
one tile per round for every system, two workgroups per compute unit)."""
import argparse
import json
import math
import os
import statistics

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_batched.json")
NEVER = 2 ** 63 - 1  # threshold above every n: one tile per round for all systems
BUCKETS = (0, 256, 512, 768, 1024, 1280, NEVER)
CANDIDATES = [{"tile_cols2_min_n": t, "wgs_per_cu": w} for t in BUCKETS for w in (1, 2)]
PRECS = ("fp32", "bf16")


def select(results):
    """The fastest accepted candidate. results: dicts with tile_cols2_min_n,
    wgs_per_cu, ms and ok. Ties go to the higher threshold (fewer systems
    with the two-tile round, which holds more registers), then to more
    workgroups. Raises ValueError when no candidate was accepted."""
    ok = [r for r in results if r["ok"] and math.isfinite(r["ms"])]
    if not ok:
        raise ValueError("no candidate reproduced the reference outputs")
    return min(ok, key=lambda r: (r["ms"], -r["tile_cols2_min_n"], -r["wgs_per_cu"]))


def load_table(path=TABLE):
    """{prec: {"tile_cols2_min_n": t, "wgs_per_cu": w}} from the table, or {}
    if there is none."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    out = {}
    for prec, e in data.get("batched", {}).items():
        t, w = int(e["tile_cols2_min_n"]), int(e["wgs_per_cu"])
        if prec not in PRECS or t < 0 or t > NEVER or w not in (1, 2):
            raise ValueError(f"invalid entry in {path}: {prec}: {e}")
        out[prec] = {"tile_cols2_min_n": t, "wgs_per_cu": w}
    return out


def _inputs(ns, ks, matrix):
    from . import workloads
    As, Bs = [], []
    for s, (n, k) in enumerate(zip(ns, ks)):
        A = workloads.device_randn(int(n), int(n), workloads.MATRIX_SEED + s)
        if matrix == "dominant":
            A = A * (0.3 / math.sqrt(int(n)))
            A.diagonal().add_(1.0)
        As.append(A)
        Bs.append(workloads.device_randn(int(n), int(k), workloads.RHS_SEED + s))
    return As, Bs


def time_candidates(prec, ns, ks, matrix="randn", reps=3, seed=2023, max_iter=10,
                    candidates=CANDIDATES, log=print):
    """Time each candidate (graph replays of one launch over the batch) and
    check its outputs against the first candidate's. Returns the result
    dicts (tile_cols2_min_n, wgs_per_cu, ms, ok)."""
    import torch
    from . import rbt
    p = rbt.RBT_FP32 if prec == "fp32" else rbt.RBT_BF16
    As, Bs = _inputs(ns, ks, matrix)
    plan = rbt.batched_plan(ns, ks, 2, p)
    saved = (rbt.get_option(rbt._lib.RBT_OPT_BATCH_TILE_COLS2_MIN_N),
             rbt.get_option(rbt._lib.RBT_OPT_BATCH_WGS_PER_CU))
    ref = None
    results = []
    try:
        for c in candidates:
            rbt.set_option(rbt._lib.RBT_OPT_BATCH_TILE_COLS2_MIN_N, c["tile_cols2_min_n"])
            rbt.set_option(rbt._lib.RBT_OPT_BATCH_WGS_PER_CU, c["wgs_per_cu"])
            args = rbt.BatchArgs(plan, As, Bs)
            stream = torch.cuda.Stream()
            stream.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(stream):
                rbt.solve_batched_launch(plan, args, seed=seed, max_iter=max_iter, tuned=False)
            torch.cuda.current_stream().wait_stream(stream)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                rbt.solve_batched_launch(plan, args, seed=seed, max_iter=max_iter, tuned=False)
            times = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                graph.replay()
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            out = ([x.cpu() for x in args.Xs], args.iters.cpu(), args.berr.cpu(), args.info.cpu())
            if ref is None:
                ref = out
                ok = True
            else:
                ok = (all(torch.equal(a, b) for a, b in zip(out[0], ref[0]))
                      and all(torch.equal(a, b) for a, b in zip(out[1:], ref[1:])))
            r = dict(c, ms=statistics.median(times), ok=bool(ok))
            log(f"  {prec} tile_cols2_min_n={c['tile_cols2_min_n']} wgs_per_cu={c['wgs_per_cu']}: "
                f"{r['ms']:.3f} ms{'' if ok else ' (outputs differ: rejected)'}")
            results.append(r)
            del graph
    finally:
        rbt.set_option(rbt._lib.RBT_OPT_BATCH_TILE_COLS2_MIN_N, saved[0])
        rbt.set_option(rbt._lib.RBT_OPT_BATCH_WGS_PER_CU, saved[1])
    return results


def main(argv=None):
    import torch
    from . import workloads
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--prec", nargs="+", choices=PRECS, default=list(PRECS))
    ap.add_argument("--matrix", choices=["randn", "dominant"], default="randn")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--max-iter", type=int, default=10, help="refinement cap (as the benchmark)")
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner times kernels: it needs a GPU")
    ns, ks = workloads.batch_sizes(count=a.batch)
    table = {"device": torch.cuda.get_device_name(0),
             "workload": f"{a.batch} systems, n~U{{37..1500}}, nrhs~U{{1..16}} (seed 7), "
                         f"A={a.matrix}, depth 2, max_iter {a.max_iter}",
             "batched": {}}
    for prec in a.prec:
        res = time_candidates(prec, ns, ks, a.matrix, a.reps, max_iter=a.max_iter)
        best = select(res)
        table["batched"][prec] = {"tile_cols2_min_n": best["tile_cols2_min_n"],
                                  "wgs_per_cu": best["wgs_per_cu"], "ms": round(best["ms"], 3),
                                  "candidates": res}
        print(f"{prec}: tile_cols2_min_n={best['tile_cols2_min_n']} wgs_per_cu={best['wgs_per_cu']} "
              f"({best['ms']:.3f} ms)", flush=True)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(f"wrote {a.out}")


if __name__ == "__main__":
    main()
