"""Benchmark: multigrid-preconditioned CG on the 1024^2 cubic B-spline immersed
Poisson problem (unit square minus 200 seeded discs, manufactured solution,
6-level V(2,2)), on one MI355X.

A step is one full PCG solve from x0 = 0 to a relative residual of 1e-8 (every
V-cycle level, smoother, transfer, coarsest solve and CG update runs inside
it).  Inputs (operator hierarchy, right-hand side) are resident in HBM before
the timed region starts.  `value` = fine DOFs x PCG iterations / wall time of
the timed solves of the headline form (each iteration applies one V-cycle and
the CG updates); the plain FP64 form is timed in the same run and reported in
`config`.

The dominant kernel is the finest level's fused residual + trivial-row
smoothing step; its duration is measured with HIP events on the library stream
during a second pass of the same solves (each timed step launches the kernel
TIMED_REPS times back to back between its two events, which spreads the events'
own overhead; the step only reads x_a and r, so the repeats change nothing),
and its algorithmic bytes come from the level's storage statistics (compressed
rows read only vectors).

Prints one JSON line.
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
# launches of the timed kernel per event pair (spreads the event packets' overhead)
TIMED_REPS = 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def smooth_step_bytes(st):
    """Algorithmic bytes of one launch of the fused residual + trivial-row
    smoothing step on a level: per row row_lat (4) + meta (4) + c (8) + r (8)
    + x_a (8, each entry once) + x_b (8); rows of general blocks also store
    their residual (8); stored rows read K values."""
    return (st["n"] * 40 + st["general_rows"] * 8
            + st["stored_rows"] * st["stencil"] * st["value_bytes"])


def cpu_baseline():
    """The oracle (plain FP64 NumPy/SciPy) on a bounded sample of the same
    workload: the same 200-disc geometry and cubic V(2,2) hierarchy at 128^2
    (4 levels, coarsest 16^2); throughput in the same unit (DOFs x PCG
    iterations / solve seconds)."""
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
    return {"value": round(n * it / t_solve / 1e6, 4), "unit": "MDOF/s", "cores": 1,
            "cores_available": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"oracle PCG solve to 1e-8 on the same 200-disc cubic V(2,2) workload at 128^2 "
                      f"({n} DOFs, 4 levels, {it} iterations, solve {t_solve:.2f} s, setup {t_setup:.1f} s); "
                      f"scipy sparse products and the per-block Python loops run on one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed",
                    help="headline form (the other form is timed too)")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-autotune", action="store_true",
                    help="general-row smoother with 4 lanes per row on every level instead of the measured choice")
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="c2: 1024^2 cubic discs (headline); c3: 128^3 quadratic gyroid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the mixed+learned form")
    ap.add_argument("--nrhs", type=int, default=16, help="columns of the multi-right-hand-side form (1: skip)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-problem form")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for FETCH_SIZE/WRITE_SIZE scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU: --gpus must be 1 (sharding across GPUs is designed, not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_1903_10977_amd import generator as GN
    from paper_1903_10977_amd import profiling as PR
    from paper_1903_10977_amd import solver as S

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.workload == "c3":
        # 3D gyroid, quadratic B-splines, 128^3, 4 levels, V(1,1); no multi-column or batched forms
        w = W.c3(n=args.n if args.n != 1024 else 128)
        levels = w.levels
        args.nrhs, args.no_batched = 1, True
    else:
        levels = int(round(math.log2(args.n // 32))) + 1
        w = W.c2(n=args.n, levels=levels)
    t0 = time.time()
    g = GN.generate(w, with_mass=args.nrhs > 1)
    log(f"generated {w.name}: fine DOFs {g.fine.n}, nnz {g.fine.A.nnz}, {time.time() - t0:.1f} s")
    b = torch.tensor(g.b, device="cuda:0")
    n = g.fine.n

    def make(prec, timing=0, learned=None, block_gemm=0):
        o = S.default_options(nu_pre=w.nu, nu_post=w.nu, precision=prec, timing=timing,
                              use_graph=0 if (args.no_graph or timing) else 1, max_iter=2000,
                              use_learned=int(learned is not None), autotune=int(not args.no_autotune),
                              block_gemm=block_gemm)
        t = time.time()
        sol = S.Solver(0).setup(g, o)
        if learned is not None:
            sol.load_mlp(learned)
        sol.factor()
        lanes = [sol.level_stats(l)["general_lanes"] for l in range(1, len(g.levels))]
        log(f"setup+factor precision={prec} {time.time() - t:.2f} s (general-row lanes per level {lanes})")
        return sol

    def timed(sol):
        x = torch.zeros_like(b)
        for _ in range(args.warmup):
            x.zero_()
            sol.pcg(b, x, rtol=1e-8)
        torch.cuda.synchronize()
        iters = 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x.zero_()
            info = sol.pcg(b, x, rtol=1e-8)
            iters += info.iterations
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return x, iters, dt

    head = S.MIXED if args.precision == "mixed" else S.FP64
    other = S.FP64 if head == S.MIXED else S.MIXED
    results = {}
    for prec in (other, head):
        sol = make(prec)
        x, iters, dt = timed(sol)
        res = float(np.linalg.norm(g.b - g.fine.A @ x.cpu().numpy()) / np.linalg.norm(g.b))
        results[prec] = dict(iters=iters, dt=dt, ms=1e3 * dt / args.steps, mdofs=n * iters / dt / 1e6,
                             true_rel_res=res, x=x)
        log(f"precision={prec}: {args.steps} solves, {iters} iterations, {1e3 * dt / args.steps:.2f} ms/solve, "
            f"{n * iters / dt / 1e6:.1f} MDOF/s, true rel. residual {res:.2e}")
        sol.close()
    # mixed + learned per-block damping (the committed network), same solves
    learned = None
    if not args.no_learned:
        from paper_1903_10977_amd import learn as LN
        model = LN.MODEL_DEFAULT + ("_gyroid3d" if args.workload == "c3" else "")
        sol = make(S.MIXED, learned=LN.load_params(model))
        status = [sol.weights(l)[1] for l in range(1, len(g.levels))]
        x, iters, dt = timed(sol)
        res = float(np.linalg.norm(g.b - g.fine.A @ x.cpu().numpy()) / np.linalg.norm(g.b))
        learned = dict(iters=iters, ms=1e3 * dt / args.steps, mdofs=n * iters / dt / 1e6, true_rel_res=res,
                       level_status=status)
        log(f"mixed+learned: {args.steps} solves, {iters} iterations, {learned['ms']:.2f} ms/solve, "
            f"level status {status} (1 = network weights kept), true rel. residual {res:.2e}")
        sol.close()
    # several right-hand sides with the same matrix: the 16-column form
    multi = None
    if args.nrhs > 1:
        rng = np.random.Generator(np.random.PCG64(1000))
        M = g.M
        U = rng.standard_normal((args.nrhs, n))
        Bm = torch.tensor(np.stack([M @ u for u in U]), device="cuda:0")  # load vectors of random L2 data
        Bm[0] = b
        # general Schwarz blocks: 0 assembled FP64 CSR product, 1 FP64 patch
        # GEMMs on the matrix cores, 2 BF16 patch GEMMs with FP32 accumulation
        forms = {}
        for mode, label in ((0, "csr_fp64"), (1, "mfma_fp64"), (2, "mfma_bf16")):
            sol = make(head, block_gemm=mode)
            Xm = torch.zeros_like(Bm)
            sol.pcg_multi(Bm, Xm, rtol=1e-8)  # warm-up (graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tot_it = 0
            for _ in range(args.steps):
                Xm.zero_()
                infos = sol.pcg_multi(Bm, Xm, rtol=1e-8)
                tot_it += sum(i.iterations for i in infos)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            worst = max(i.true_rel_res for i in infos)
            forms[label] = {"ms_per_solve": round(1e3 * dt / args.steps, 3), "mdofs": round(n * tot_it / dt / 1e6, 1),
                            "iterations_per_column": [i.iterations for i in infos], "worst_true_rel_res": worst,
                            "patch_gemm_levels": [sol.level_stats(l)["patch_gemm"] for l in range(1, len(g.levels))]}
            log(f"{args.nrhs} right-hand sides ({label}): {forms[label]['ms_per_solve']:.2f} ms per solve, "
                f"{forms[label]['mdofs']} MDOF/s (DOF x iterations summed over columns), worst true rel. residual "
                f"{worst:.2e}")
            sol.close()
        multi = {"nrhs": args.nrhs, **{k: v for k, v in forms["csr_fp64"].items() if k != "patch_gemm_levels"},
                 "general_blocks": forms,
                 "rhs": "column 0: the workload's load vector; others: load vectors M u of random normal u"}
    # batched: 64 independent problems (n in {64..512}^2, p in {1,2,3}), 16
    # right-hand sides each, one context and stream per problem, 16 host threads
    batched = None
    if not args.no_batched:
        from paper_1903_10977_amd import batch as BT
        # the configuration's form: general blocks as BF16 patch GEMMs (FP32
        # accumulation) on the matrix cores; the assembled CSR product beside it
        batched = BT.run_batch(64, 16, workers=16, steps=2, precision=head, block_gemm=2)
        batched["csr_fp64"] = BT.run_batch(64, 16, workers=16, steps=2, precision=head, block_gemm=0)
    hr = results[head]
    ms_step = hr["ms"]
    value = hr["mdofs"]
    # the two forms' solutions agree (L2 on the coefficients is dominated by
    # near-null cut modes; report the relative residual of each instead)

    # dominant kernel: the finest level's fused residual + trivial smoothing
    # step, timed with HIP events on the library stream during the same solves
    solt = make(head, timing=TIMED_REPS)
    stats = solt.level_stats(len(g.levels) - 1)
    solt.kernel_time(reset=True)
    xt = torch.zeros_like(b)
    for _ in range(args.steps):
        xt.zero_()
        solt.pcg(b, xt, rtol=1e-8)
    ms, cnt = solt.kernel_time()
    avg_ms = ms / max(cnt, 1)
    bytes_launch = smooth_step_bytes(stats)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    log(f"fine smoothing-step kernel: {cnt} launches, avg {avg_ms * 1e3:.1f} us, {bytes_launch / 1e6:.1f} MB, "
        f"{achieved:.0f} GB/s; stats {stats}")
    solt.close()

    if args.copy_calibration_mib > 0:
        # a plain device copy of known size for the counter scaling: one
        # elementwise kernel reading M MiB and writing M MiB
        m = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.rand(m, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 elementwise copies of {args.copy_calibration_mib} MiB")
        del src, dst

    # measured HBM traffic of the same kernel (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    # copy-calibrated), valid only while the kernel sources are unchanged
    traffic = None
    if args.n == 1024 and args.workload == "c2":
        form = "mixed" if head == S.MIXED else "fp64"
        traffic = PR.read_traffic(os.path.join(ROOT, "profiles", f"traffic_k_residual_smooth_1024_discs_{form}.txt"))

    cpu = None
    if not args.no_cpu_baseline and args.workload == "c2":
        log("timing the oracle on the host (bounded sample)")
        cpu = cpu_baseline()
    names = {S.FP64: "fp64", S.MIXED: "mixed"}
    forms = {names[p]: {"ms_per_solve": round(r["ms"], 3), "mdofs": round(r["mdofs"], 1),
                        "iterations_per_solve": r["iters"] / args.steps, "true_rel_res": r["true_rel_res"]}
             for p, r in results.items()}
    if learned is not None:
        forms["mixed+learned"] = {"ms_per_solve": round(learned["ms"], 3), "mdofs": round(learned["mdofs"], 1),
                                  "iterations_per_solve": learned["iters"] / args.steps,
                                  "true_rel_res": learned["true_rel_res"],
                                  "levels_with_network_weights": learned["level_status"]}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "MDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if head == S.FP64 else "f32-vcycle-operators/f64",
        "data": "synthetic",
        "config": {"workload": (f"2D Poisson, cubic B-splines, {args.n}^2, unit square minus 200 seeded discs "
                                f"(r ~ U[0.01,0.04]), manufactured sin(2 pi x) sin(2 pi y), {levels}-level V(2,2), "
                                f"PCG to 1e-8 from x0 = 0") if args.workload == "c2" else
                               (f"3D Poisson, quadratic B-splines, {w.n}^3 gyroid {{g < 0.3}} (two periods, seeded "
                                f"phase), f = 1, u = 0 on the box, {levels}-level V(1,1), PCG to 1e-8 from x0 = 0"),
                   "fine_dofs": n, "headline_form": names[head],
                   "pcg_time_s": round(ms_step / 1e3, 5), "forms": forms,
                   "speedup_mixed_vs_fp64": round(results[S.FP64]["ms"] / results[S.MIXED]["ms"], 3),
                   "multi_rhs": multi, "batched": batched},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_residual_smooth (finest level)", "bytes_per_launch": int(bytes_launch),
                     "avg_launch_us": round(avg_ms * 1e3, 2), "launches_per_event_pair": TIMED_REPS},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
