"""Benchmark: multigrid-preconditioned CG on the 3D immersed Poisson problem
(quadratic B-splines, 128^3 gyroid, 1.48M DOFs, 4-level V(1,1)) on one MI355X,
with the 2D 1024^2 cubic 200-disc problem (6-level V(2,2)), 3D linear
elasticity on the 80^3 apple with a bite (667k DOFs), a locally refined problem
with truncated hierarchical B-splines (58k DOFs, general sparse levels),
several right-hand sides and the 64-problem batch beside it.

Metric (both parts are reported for every form):
* V-cycle MDOF/s = fine DOFs / median time of one V-cycle (imsmg_vcycle as
  one captured graph, HIP events around each of --vcycles cycles after warm-up);
* PCG time to 1e-8 = wall time of one imsmg_pcg_solve from x0 = 0 until the
  true relative residual ||b - A x|| / ||b|| <= 1e-8 (rechecked on the host).
A timed step is one FP64 PCG solve of the workload (every level, smoother,
transfer, coarsest solve and CG update runs inside it); `value` is the FP64
V-cycle MDOF/s, `ms_per_step` the FP64 PCG time.  The other forms (FP32
V-cycle operators, multiplicative Schwarz, the damping network) are timed in
the same run and reported in `config`.  Inputs (operator hierarchy, right-hand
side) are resident in HBM before the timed region starts.

Roofline of the dominant kernel (the finest level's fused residual +
one-function-block smoothing step, FP64): its duration is measured with HIP
events on the library stream during a second pass of the same solves (each
timed step launches the kernel TIMED_REPS times back to back between its two
events; the step only reads x_a and r, so the repeats change nothing), its
algorithmic bytes come from the level's storage statistics.

Prints one JSON line.
"""
import argparse
import dataclasses
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
    """Algorithmic bytes of one launch of the fused residual + one-function
    block smoothing step on a level: per row row_lat (4) + meta (4) + c (8) +
    r (8) + x_a (8, each entry once) + x_b (8); rows of larger blocks also
    store their residual (8); stored rows read K values."""
    return (st["n"] * 40 + st["general_rows"] * 8
            + st["stored_rows"] * st["stencil"] * st["value_bytes"])


def csr_smooth_step_bytes(st, nnz):
    """Algorithmic bytes of one launch of the CSR residual + smoothing step
    (general sparse level, FP64 values): per row the row pointer (4), meta
    (4), c (8), r (8), x_a (8, each entry once), x_b (8); rows of larger
    blocks also store their residual (8); per stored entry its column (4)
    and value (8)."""
    return st["n"] * 40 + st["general_rows"] * 8 + nnz * (4 + st["value_bytes"])


def device_copy_gbs(torch, mib=1024, reps=10):
    """Read + write bandwidth of torch's device-to-device copy of `mib` MiB."""
    cb = (mib << 20) // 8
    src = torch.ones(cb, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 2 * 8 * cb * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def cpu_baseline(budget_s=25.0):
    """The oracle (plain FP64 NumPy/SciPy) on bounded samples: the gyroid
    workload at 16^3 (3 levels; the headline's geometry, basis and cycle at a
    size the oracle finishes), its V-cycle time (median of 5) in the metric's
    unit and its PCG solve; C1 (the 32^2 disc configuration, whole) and the
    200-disc cubic V(2,2) workload at 128^2 when the budget allows."""
    import numpy as np
    import workloads as W
    from oracle import problem as P
    out = {}

    def sample(name, w):
        t0 = time.time()
        op = P.build(w)
        t_setup = time.time() - t0
        r = op.b
        ts = []
        for _ in range(5):
            t0 = time.time()
            op.vcycle.apply(r)
            ts.append(time.time() - t0)
        t0 = time.time()
        _, it, _ = op.solve(tol=1e-8)
        t_solve = time.time() - t0
        n = op.A.shape[0]
        out[name] = {"dofs": n, "levels": w.levels, "vcycle_ms": round(1e3 * float(np.median(ts)), 2),
                     "vcycle_mdofs": round(n / float(np.median(ts)) / 1e6, 5), "pcg_s": round(t_solve, 3),
                     "iterations": it, "setup_s": round(t_setup, 2)}
        log(f"oracle {name}: {out[name]}")

    t_all = time.time()
    sample("gyroid-16^3", W.c3(n=16, levels=3))
    sample("C1", W.c1())
    if time.time() - t_all < budget_s:
        sample("discs-cubic-128^2", W.c2(n=128, levels=4))
    head = out["gyroid-16^3"]
    return {"value": head["vcycle_mdofs"], "unit": "MDOF/s", "cores": 1,
            "cores_available": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": ("oracle V-cycle (median of 5) on the quadratic gyroid workload at 16^3 "
                       f"({head['dofs']} DOFs, 3 levels); also its PCG solve and the C1 and 128^2 cubic-disc "
                       "samples in `samples`; scipy sparse products and the per-block Python loops run on one "
                       "thread"),
            "samples": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--vcycles", type=int, default=50, help="timed V-cycles per form (median)")
    ap.add_argument("--workload", choices=["c3", "c2"], default="c3",
                    help="c3: 128^3 quadratic gyroid (headline); c2: 1024^2 cubic discs")
    ap.add_argument("--n", type=int, default=0, help="elements per axis (0: the workload's own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the mixed+learned form")
    ap.add_argument("--no-second", action="store_true", help="skip the second workload (c2 beside c3)")
    ap.add_argument("--no-elasticity", action="store_true", help="skip the 3D elasticity workload (apple 80^3)")
    ap.add_argument("--elasticity-n", type=int, default=80, help="elements per axis of the elasticity workload")
    ap.add_argument("--elasticity-forms", default="", help="comma list to restrict the elasticity forms")
    ap.add_argument("--no-thb", action="store_true", help="skip the locally refined (THB) workload")
    ap.add_argument("--nrhs", type=int, default=16, help="columns of the multi-right-hand-side form (1: skip)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-problem form")
    ap.add_argument("--forms", default="", help="comma list to restrict the timed forms")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for FETCH_SIZE/WRITE_SIZE scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: --gpus must be 1 "
                                   "(sharding across GPUs is designed, not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_1903_10977_amd import generator as GN
    from paper_1903_10977_amd import profiling as PR
    from paper_1903_10977_amd import solver as S

    assert torch.cuda.is_available(), "bench needs a GPU"

    def workload(kind):
        if kind == "c3":
            return W.c3(n=args.n or 128)
        n = args.n or 1024
        return W.c2(n=n, levels=int(round(math.log2(n // 32))) + 1)

    def make(g, w, prec, smoother="as", timing=0, learned=None, block_gemm=0):
        wl = dataclasses.replace(w, smoother=smoother)  # coarse_smoother: carried by w
        o = S.default_options(nu_pre=w.nu, nu_post=w.nu, precision=prec, timing=timing,
                              use_graph=0 if timing else 1, max_iter=2000, use_learned=int(learned is not None),
                              autotune=1, block_gemm=block_gemm, **S.smoother_options(wl))
        t = time.time()
        sol = S.Solver(0).setup(g, o)
        if learned is not None:
            sol.load_mlp(learned)
        sol.factor()
        log(f"{w.name} setup+factor precision={prec} smoother={smoother}: {time.time() - t:.2f} s")
        return sol

    def run_forms(w, g, forms, steps, warmup):
        b = torch.tensor(g.b, device="cuda:0")
        n = g.fine.n
        res = {}
        for label, (prec, smoother, learned, coarse) in forms.items():
            gg = GN.with_coarse_diagonal(g, coarse) if coarse else g
            wl = dataclasses.replace(w, coarse_smoother=coarse) if coarse else w
            sol = make(gg, wl, prec, smoother, learned=learned)
            x = torch.zeros_like(b)
            for _ in range(warmup):
                x.zero_()
                sol.pcg(b, x, rtol=1e-8)
            torch.cuda.synchronize()
            iters = 0
            t0 = time.perf_counter()
            for _ in range(steps):
                x.zero_()
                info = sol.pcg(b, x, rtol=1e-8)
                iters += info.iterations
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            true_res = float(np.linalg.norm(g.b - g.fine.A @ x.cpu().numpy()) / np.linalg.norm(g.b))
            vmed, vmean = sol.vcycle_time(b, reps=args.vcycles)
            entry = {"pcg_ms": round(1e3 * dt / steps, 3), "iterations": iters / steps, "setup_ms": round(info.setup_ms, 1),
                     "factor_ms": round(info.factor_ms, 1),
                     "true_rel_res": true_res, "vcycle_ms_median": round(vmed, 4), "vcycle_ms_mean": round(vmean, 4),
                     "vcycle_mdofs": round(n / (vmed * 1e-3) / 1e6, 1),
                     "mdofs_x_iterations_per_s": round(n * iters / dt / 1e6, 1)}
            if learned is not None:
                entry["learned_status_per_level"] = [sol.weights(l)[1] for l in range(1, len(g.levels))]
            res[label] = entry
            log(f"{w.name} {label}: {entry}")
            if true_res > 1.01e-8:
                raise RuntimeError(f"{label}: true relative residual {true_res:.2e} above 1e-8")
            sol.close()
        return res

    want = set(args.forms.split(",")) if args.forms else None

    def pick(forms):
        return {k: v for k, v in forms.items() if want is None or k in want}

    # ---------------------------------------------------------------- headline
    w = workload(args.workload)
    t0 = time.time()
    g = GN.generate(w, with_mass=(args.workload == "c2" and args.nrhs > 1))
    log(f"generated {w.name}: fine DOFs {g.fine.n}, nnz {g.fine.A.nnz}, {time.time() - t0:.1f} s")
    n = g.fine.n
    # (precision, finest-level smoother, damping network, coarse-level diagonal smoother)
    forms = {"fp64": (S.FP64, "as", None, None), "mixed": (S.MIXED, "as", None, None),
             "ms-fp64": (S.FP64, "ms", None, None), "ms-mixed": (S.MIXED, "ms", None, None),
             "ms+jacobi-fp64": (S.FP64, "ms", None, "jacobi"), "ms+jacobi-mixed": (S.MIXED, "ms", None, "jacobi"),
             "ms+gs-mixed": (S.MIXED, "ms", None, "gs")}
    if not args.no_learned:
        from paper_1903_10977_amd import learn as LN
        model = LN.MODEL_DEFAULT + ("_gyroid3d" if w.dim == 3 else "")
        forms["mixed+learned"] = (S.MIXED, "as", LN.load_params(model), None)
    head = run_forms(w, g, pick(forms) if want else forms, args.steps, args.warmup)
    if "fp64" not in head:
        head.update(run_forms(w, g, {"fp64": forms["fp64"]}, args.steps, args.warmup))
    hf = head["fp64"]

    # multigrid as a standalone solver (x <- x + B (b - A x)), from zero and
    # from a full-multigrid start, with the multiplicative cycle and Jacobi
    # on the coarser levels (the additive cycle contracts slowly on its own)
    mg_forms = {}
    if want is None or "mg-solver" in want:
        gj = GN.with_coarse_diagonal(g, "jacobi")
        wj = dataclasses.replace(w, coarse_smoother="jacobi")
        solm = make(gj, wj, S.FP64, "ms")
        bm = torch.tensor(g.b, device="cuda:0")
        for label, fmg in (("ms+jacobi-fp64", False), ("fmg+ms+jacobi-fp64", True)):
            xm = torch.zeros_like(bm)
            for _ in range(args.warmup):
                xm.zero_()
                solm.mg_solve(bm, xm, rtol=1e-8, max_cycles=2000, fmg=fmg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                xm.zero_()
                im = solm.mg_solve(bm, xm, rtol=1e-8, max_cycles=2000, fmg=fmg)
            torch.cuda.synchronize()
            dtm = (time.perf_counter() - t0) / args.steps
            res_m = float(np.linalg.norm(g.b - g.fine.A @ xm.cpu().numpy()) / np.linalg.norm(g.b))
            mg_forms[label] = {"ms_per_solve": round(1e3 * dtm, 3), "cycles": im.iterations, "true_rel_res": res_m}
            log(f"{w.name} multigrid solver {label}: {mg_forms[label]}")
        solm.close()
        del gj

    # dominant kernel: the finest level's fused residual + smoothing step,
    # FP64, timed with HIP events on the library stream during the same solves
    solt = make(g, w, S.FP64, timing=TIMED_REPS)
    stats = solt.level_stats(len(g.levels) - 1)
    solt.kernel_time(reset=True)
    b = torch.tensor(g.b, device="cuda:0")
    xt = torch.zeros_like(b)
    for _ in range(max(1, min(args.steps, 3))):
        xt.zero_()
        solt.pcg(b, xt, rtol=1e-8)
    ms, cnt = solt.kernel_time()
    avg_ms = ms / max(cnt, 1)
    bytes_launch = smooth_step_bytes(stats)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    log(f"fine smoothing-step kernel: {cnt} launches, avg {avg_ms * 1e3:.1f} us, {bytes_launch / 1e6:.1f} MB, "
        f"{achieved:.0f} GB/s; stats {stats}")
    solt.close()
    # what a plain streaming kernel gets from HBM on this device: torch's
    # device-to-device copy of 1 GiB (read + write), timed with events on
    # torch's stream (where the copy runs); left out of counter runs, whose
    # calibration copy must be the only large elementwise kernel
    copy_gbs = None
    if args.copy_calibration_mib <= 0:
        copy_gbs = device_copy_gbs(torch)
        log(f"device copy of 1 GiB: {copy_gbs:.0f} GB/s (read + write)")
    tag = "128cube_gyroid" if (args.workload == "c3" and w.n == 128) else (
        "1024_discs" if (args.workload == "c2" and w.n == 1024) else None)
    traffic = None
    if tag:
        traffic = PR.read_traffic(os.path.join(ROOT, "profiles", f"traffic_k_residual_smooth_{tag}_fp64.txt"))

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
    del g

    # ------------------------------------------------ the second workload (2D)
    second = None
    if args.workload == "c3" and not args.no_second:
        w2 = workload("c2")
        t0 = time.time()
        g2 = GN.generate(w2, with_mass=args.nrhs > 1)
        log(f"generated {w2.name}: fine DOFs {g2.fine.n}, {time.time() - t0:.1f} s")
        forms2 = {"fp64": (S.FP64, "as", None, None), "mixed": (S.MIXED, "as", None, None),
                  "ms-fp64": (S.FP64, "ms", None, None), "ms+jacobi-fp64": (S.FP64, "ms", None, "jacobi"),
                  "ms+jacobi-mixed": (S.MIXED, "ms", None, "jacobi")}
        second = {"workload": (f"2D Poisson, cubic B-splines, {w2.n}^2, unit square minus 200 seeded discs, "
                               f"manufactured sin(2 pi x) sin(2 pi y), {w2.levels}-level V(2,2)"),
                  "fine_dofs": g2.fine.n, "forms": run_forms(w2, g2, pick(forms2) if want else forms2,
                                                            args.steps, args.warmup)}
        mw, mg = w2, g2
    elif args.workload == "c2":
        mw, mg = w, GN.generate(w, with_mass=True) if args.nrhs > 1 else None
    else:
        mw = mg = None

    # ------------------------------------ linear elasticity (vector problem)
    elastic = None
    if not args.no_elasticity and (want is None or "elasticity" in want):
        we = W.apple(n=args.elasticity_n, levels=4)
        t0 = time.time()
        ge = GN.generate(we)
        log(f"generated {we.name}: fine DOFs {ge.fine.n} (3 components), nnz {ge.fine.A.nnz}, "
            f"{time.time() - t0:.1f} s")
        # FP32 operators with the multiplicative smoother do not reach 1e-8 here: the colour
        # residuals feed cut blocks whose inverses amplify FP32 rounding by up to 1e16
        forms_e = {"fp64": (S.FP64, "as", None, None), "mixed": (S.MIXED, "as", None, None),
                   "ms-fp64": (S.FP64, "ms", None, None), "ms+jacobi-fp64": (S.FP64, "ms", None, "jacobi")}
        if args.elasticity_forms:
            forms_e = {k: v for k, v in forms_e.items() if k in args.elasticity_forms.split(",")}
        elastic = {"workload": (f"3D linear elasticity, quadratic B-splines, {we.n}^3 apple with a bite in "
                                f"(-2,2)^3, lambda = mu = 1e3, gravity, penalty Dirichlet (2/h) on the bite, "
                                f"{we.levels}-level V(1,1), additive or multiplicative Schwarz with "
                                f"per-component blocks"),
                   "fine_dofs": ge.fine.n, "generate_s": round(time.time() - t0, 1),
                   "forms": run_forms(we, ge, forms_e, min(args.steps, 3), min(args.warmup, 1))}
        del ge

    # -------------------- truncated hierarchical B-splines (general sparse levels)
    thb = None
    if not args.no_thb and (want is None or "thb" in want):
        from paper_1903_10977_amd import thb as TB
        wt = W.thb_256()
        t0 = time.time()
        gt = TB.generate(wt)
        gen_s = time.time() - t0
        log(f"generated {wt.name}: fine DOFs {gt.fine.n}, nnz {gt.fine.A.nnz}, levels "
            f"{[lv.n for lv in gt.levels]}, {gen_s:.1f} s")
        forms_t = {"fp64": (S.FP64, "as", None, None), "mixed": (S.MIXED, "as", None, None),
                   "ms-fp64": (S.FP64, "ms", None, None)}
        res_t = run_forms(wt, gt, forms_t, args.steps, args.warmup)
        gj = TB.with_coarse_diagonal(gt)
        res_t.update(run_forms(gj.workload, gj, {"as+jacobi-fp64": (S.FP64, "as", None, None)},
                               args.steps, args.warmup))
        gs = TB.with_coarse_diagonal(gt, "gs")
        res_t.update(run_forms(gs.workload, gs, {"ms+gs-fp64": (S.FP64, "ms", None, None)},
                               args.steps, args.warmup))
        del gs
        # the finest level's CSR residual + smoothing step, FP64, HIP events
        solk = make(gt, wt, S.FP64, timing=TIMED_REPS)
        stk = solk.level_stats(len(gt.levels) - 1)
        solk.kernel_time(reset=True)
        bt = torch.tensor(gt.b, device="cuda:0")
        xk = torch.zeros_like(bt)
        for _ in range(max(1, min(args.steps, 3))):
            xk.zero_()
            solk.pcg(bt, xk, rtol=1e-8)
        msk, cntk = solk.kernel_time()
        solk.close()
        avgk = msk / max(cntk, 1)
        bytes_k = csr_smooth_step_bytes(stk, gt.fine.A.nnz)
        ach_k = bytes_k / (avgk * 1e-3) / 1e9
        log(f"THB fine smoothing step (CSR): {cntk} launches, avg {avgk * 1e3:.2f} us, {bytes_k / 1e6:.2f} MB, "
            f"{ach_k:.0f} GB/s")
        thb = {"workload": (f"2D Poisson, quadratic truncated hierarchical B-splines, {wt.n}^2 level-0 cells, "
                            f"cells cut by 40 seeded discs refined {wt.local_levels} times, f = 1, u = 0 on the "
                            f"box, {wt.levels}-level V(1,1) on meshes coarsened by Algorithm alg:coarsen, "
                            f"additive or multiplicative Schwarz (support-inclusion blocks), general sparse "
                            f"(CSR) levels"),
               "fine_dofs": gt.fine.n, "level_dofs": [lv.n for lv in gt.levels], "fine_nnz": int(gt.fine.A.nnz),
               "generate_s": round(gen_s, 1), "forms": res_t,
               "fine_smoothing_kernel": {"kernel": "k_csr_residual_smooth (finest level, FP64)",
                                         "avg_launch_us": round(avgk * 1e3, 2), "bytes_per_launch": int(bytes_k),
                                         "achieved_gbs": round(ach_k, 1),
                                         "frac_of_hbm_peak": round(ach_k / HBM_PEAK_GBS, 4),
                                         "launches": int(cntk),
                                         "traffic": PR.read_traffic(os.path.join(
                                             ROOT, "profiles", "traffic_k_csr_residual_smooth_thb_256_discs_fp64.txt"))}}
        del gt, gj
        # 2D linear elasticity on THB levels (the physics of the paper's THB example)
        we = W.thb_star_elasticity()
        t0 = time.time()
        ge = TB.generate(we)
        gen_e = time.time() - t0
        log(f"generated {we.name}: fine DOFs {ge.fine.n}, levels {[lv.n for lv in ge.levels]}, {gen_e:.1f} s")
        res_e = run_forms(we, ge, {"fp64": (S.FP64, "as", None, None), "ms-fp64": (S.FP64, "ms", None, None)},
                          args.steps, args.warmup)
        thb["elasticity"] = {
            "workload": (f"2D linear elasticity (lambda = mu = 1e3, load (0, -1)), quadratic THB-splines on the "
                         f"star domain, {we.n}^2 level-0 cells, cut cells refined {we.local_levels} times, "
                         f"penalty Dirichlet conditions (beta = 2/h of the boundary cells), {we.levels}-level "
                         f"V(1,1), per-component Schwarz blocks, general sparse (CSR) levels"),
            "fine_dofs": ge.fine.n, "level_dofs": [lv.n for lv in ge.levels], "generate_s": round(gen_e, 1),
            "forms": res_e}
        del ge

    # several right-hand sides with the C2 matrix: the 16-column form
    multi = None
    if args.nrhs > 1 and mg is not None:
        rng = np.random.Generator(np.random.PCG64(1000))
        nn = mg.fine.n
        U = rng.standard_normal((args.nrhs, nn))
        Bm = torch.tensor(np.stack([mg.M @ u for u in U]), device="cuda:0")  # load vectors of random L2 data
        Bm[0] = torch.tensor(mg.b, device="cuda:0")
        fm = {}
        for mode, label in ((0, "csr_fp64"), (2, "mfma_bf16")):
            sol = make(mg, mw, S.MIXED, block_gemm=mode)
            Xm = torch.zeros_like(Bm)
            sol.pcg_multi(Bm, Xm, rtol=1e-8)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tot_it = 0
            for _ in range(args.steps):
                Xm.zero_()
                infos = sol.pcg_multi(Bm, Xm, rtol=1e-8)
                tot_it += sum(i.iterations for i in infos)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            fm[label] = {"ms_per_solve": round(1e3 * dt / args.steps, 3),
                         "mdofs_x_iterations_per_s": round(nn * tot_it / dt / 1e6, 1),
                         "worst_true_rel_res": max(i.true_rel_res for i in infos)}
            log(f"{args.nrhs} right-hand sides ({label}): {fm[label]}")
            sol.close()
        multi = {"nrhs": args.nrhs, "general_blocks": fm,
                 "rhs": "column 0: the workload's load vector; others: load vectors M u of random normal u"}

    # batched: 64 independent problems (n in {64..512}^2, p in {1,2,3}), 16
    # right-hand sides each, one context and stream per problem, 16 host threads
    batched = None
    if not args.no_batched:
        from paper_1903_10977_amd import batch as BT
        batched = BT.run_batch(64, 16, workers=16, steps=2, precision=S.MIXED, block_gemm=0)
        batched["bf16_patch_gemms"] = BT.run_batch(64, 16, workers=16, steps=2, precision=S.MIXED, block_gemm=2)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded samples)")
        cpu = cpu_baseline()

    out = {
        "metric": METRIC, "value": hf["vcycle_mdofs"], "unit": "MDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hf["pcg_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"3D Poisson, quadratic B-splines, {w.n}^3 gyroid {{g < 0.3}} (two periods, seeded "
                                f"phase), f = 1, u = 0 on the box, {w.levels}-level V(1,1), PCG to 1e-8 from x0 = 0"
                                if w.dim == 3 else
                                f"2D Poisson, cubic B-splines, {w.n}^2 minus 200 seeded discs, manufactured "
                                f"solution, {w.levels}-level V(2,2), PCG to 1e-8 from x0 = 0"),
                   "fine_dofs": n, "headline_form": "fp64 (additive Schwarz V-cycle, FP64 everywhere)",
                   "value_is": "fine DOFs / median time of one V-cycle (50 timed cycles, HIP events)",
                   "ms_per_step_is": "one FP64 PCG solve from x0 = 0 to a true relative residual <= 1e-8",
                   "pcg_time_s": round(hf["pcg_ms"] / 1e3, 5), "forms": head,
                   "multigrid_solver": mg_forms,
                   "speedup_mixed_vs_fp64_pcg": (round(hf["pcg_ms"] / head["mixed"]["pcg_ms"], 3)
                                                 if "mixed" in head else None),
                   "second_workload": second, "elasticity": elastic, "thb": thb, "multi_rhs": multi,
                   "batched": batched},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_residual_smooth (finest level, FP64)", "bytes_per_launch": int(bytes_launch),
                     "avg_launch_us": round(avg_ms * 1e3, 2), "launches_per_event_pair": TIMED_REPS,
                     "device_copy_gbs": round(copy_gbs, 1) if copy_gbs else None,
                     "frac_of_device_copy": round(achieved / copy_gbs, 4) if copy_gbs else None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
