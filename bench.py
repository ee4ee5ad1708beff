"""Benchmark: multigrid-preconditioned CG on the 1024^2 cubic B-spline immersed
Poisson problem (unit square minus 200 seeded discs, manufactured solution,
6-level V(2,2)), on one MI355X.

A step is one full PCG solve from x0 = 0 to a relative residual of 1e-8 (every
V-cycle level, smoother, transfer, coarsest solve and CG update runs inside
it).  Inputs (operator hierarchy, right-hand side) are resident in HBM before
the timed region starts.  `value` = fine DOFs x PCG iterations / wall time of
the timed solves (each iteration applies one V-cycle and the CG updates).

Prints one JSON line (see the keys at the end of main()).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V-cycle MDOF/s + PCG time to 1e-8 rel. residual, plain FP64 vs mixed/learned"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes_per_row(K, value_bytes, vec_bytes=8):
    # lattice-ELL residual y = b - A x: K values, row lattice index (4 B),
    # x once, b once, y once (vectors FP64)
    return K * value_bytes + 4 + 3 * vec_bytes


def cpu_baseline(seconds_budget=20.0):
    """The oracle (plain FP64 NumPy/SciPy) on a bounded sample of the same
    workload: the same 200-disc geometry and cubic V(2,2) hierarchy at 128^2
    (4 levels, coarsest 16^2); throughput in the same unit (DOFs x PCG
    iterations / solve seconds)."""
    import numpy as np
    import workloads as W
    from oracle import problem as P
    w = W.c2(n=128, levels=4)
    t0 = time.time()
    op = P.build(w)
    t_setup = time.time() - t0
    t0 = time.time()
    x, it, _ = op.solve(tol=1e-8)
    t_solve = time.time() - t0
    n = op.A.shape[0]
    try:
        import threadpoolctl
        threads = max(i["num_threads"] for i in threadpoolctl.threadpool_info()) if threadpoolctl.threadpool_info() else 1
    except Exception:
        threads = 1
    return {"value": n * it / t_solve / 1e6, "unit": "MDOF/s", "cores": 1,
            "cores_available": len(os.sched_getaffinity(0)), "blas_threads": threads, "kind": "oracle",
            "sample": f"oracle PCG solve to 1e-8 on the same 200-disc cubic V(2,2) workload at 128^2 "
                      f"({n} DOFs, 4 levels, {it} iterations, solve {t_solve:.2f} s, setup {t_setup:.1f} s); "
                      f"scipy sparse products are single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_1903_10977_amd import generator as GN
    from paper_1903_10977_amd import solver as S

    assert torch.cuda.is_available(), "bench needs a GPU"
    levels = int(round(math.log2(args.n // 32))) + 1
    w = W.c2(n=args.n, levels=levels)
    t0 = time.time()
    g = GN.generate(w)
    log(f"generated {w.name}: fine DOFs {g.fine.n}, nnz {g.fine.A.nnz}, {time.time() - t0:.1f} s")
    b = torch.tensor(g.b, device="cuda:0")
    n = g.fine.n
    K = (2 * w.degree + 1) ** w.dim

    def make(prec, timing=0, graph=1):
        o = S.default_options(nu_pre=w.nu, nu_post=w.nu, precision=prec, timing=timing,
                              use_graph=0 if (args.no_graph or timing) else graph, max_iter=1000)
        t = time.time()
        sol = S.Solver(0).setup(g, o).factor()
        log(f"setup+factor precision={prec} {time.time() - t:.2f} s")
        return sol

    prec = S.MIXED if args.precision == "mixed" else S.FP64
    sol = make(prec)
    x = torch.zeros_like(b)
    for _ in range(args.warmup):
        x.zero_()
        sol.pcg(b, x, rtol=1e-8)
    torch.cuda.synchronize()
    iters = 0
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        info = sol.pcg(b, x, rtol=1e-8)
        iters += info.iterations
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    value = n * iters / dt / 1e6
    log(f"timed: {args.steps} solves, {iters} iterations, {ms_step:.2f} ms/solve, {value:.1f} MDOF/s")

    # dominant kernel: the finest-level lattice-ELL residual, timed with HIP
    # events on the library stream during the same solves (eager launches)
    solt = make(prec, timing=1)
    solt.kernel_time(reset=True)
    xt = torch.zeros_like(b)
    for _ in range(args.steps):
        xt.zero_()
        solt.pcg(b, xt, rtol=1e-8)
    ms, cnt = solt.kernel_time()
    avg_ms = ms / max(cnt, 1)
    vb = 4 if prec == S.MIXED else 8
    bytes_launch = n * spmv_bytes_per_row(K, vb)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    log(f"fine residual kernel: {cnt} launches, avg {avg_ms * 1e3:.1f} us, {achieved:.0f} GB/s")
    solt.close()

    # accuracy against the manufactured discretization: true residual
    xs = x.cpu().numpy()
    res = float(np.linalg.norm(g.b - g.fine.A @ xs) / np.linalg.norm(g.b))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        cpu = cpu_baseline()
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "MDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == S.FP64 else "f32-operators/f64-cg", "data": "synthetic",
        "config": {"workload": f"2D Poisson, cubic B-splines, {args.n}^2, unit square minus 200 seeded discs "
                               f"(r ~ U[0.01,0.04]), manufactured sin(2 pi x) sin(2 pi y), {levels}-level V(2,2), "
                               f"PCG to 1e-8 from x0 = 0", "fine_dofs": n, "precision": args.precision,
                   "iterations_per_solve": iters / args.steps, "pcg_time_s": round(ms_step / 1e3, 5),
                   "true_rel_res": res},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_ell_residual (finest level)", "bytes_per_launch": bytes_launch,
                     "avg_launch_us": round(avg_ms * 1e3, 2)},
        "cpu_baseline": cpu,
    }
    sol.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
