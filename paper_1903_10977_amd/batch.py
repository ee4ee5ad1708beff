"""Many independent problems, each with several right-hand sides, solved
concurrently on one GPU.

One library batch context (imsmg_setup_batched) holds the problems; each
problem gets its own child context and therefore its own HIP stream and its
own captured CG graph, and imsmg_pcg_solve_batched drives them from a pool
of native host threads, so the small, latency-bound V-cycles of different
problems overlap on the device instead of running one after the other.
Each problem uses the multi-column solve (all of its right-hand sides share
every kernel launch).

    python3 -m paper_1903_10977_amd.batch --problems 64 --nrhs 16
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import generator as GN
from . import solver as S


def _log(msg):
    print(f"[batch] {msg}", file=sys.stderr, flush=True)


class BatchSolver:
    def __init__(self, problems, nrhs=16, precision=S.MIXED, max_iter=2000, workers=16, block_gemm=0):
        import torch
        self.torch = torch
        self.problems = problems
        self.nrhs = nrhs
        self.workers = workers
        nus = {g.workload.nu for g in problems}
        if len(nus) != 1:
            raise ValueError("one batch shares its smoothing steps")
        nu = nus.pop()
        o = S.default_options(nu_pre=nu, nu_post=nu, precision=precision, max_iter=max_iter, block_gemm=block_gemm)
        self.ctx = S.BatchContext(0).setup(problems, o).factor()

    def rhs(self, seed0=1000):
        """nrhs right-hand sides per problem: load vectors b = M u of random
        data u ~ N(0, 1) per coefficient (PCG64 seed0 + index; M = the
        problem's mass matrix).  A standard-normal coefficient vector b itself
        is not a finite-element load vector: its components along the
        near-null modes of cut elements give solutions of size ~kappa |b|, for
        which an FP64 residual of 1e-8 is out of reach (eps kappa >= 1)."""
        out = []
        for i, g in enumerate(self.problems):
            if g.M is None:
                raise ValueError("batched right-hand sides need the mass matrices (generate with_mass=True)")
            rng = np.random.Generator(np.random.PCG64(seed0 + i))
            U = rng.standard_normal((self.nrhs, g.fine.n))
            out.append(self.torch.tensor(np.stack([g.M @ u for u in U]), device="cuda:0"))
        return out

    def solve(self, B, rtol=1e-8):
        """X (list of (nrhs, n) tensors), infos per problem, wall seconds; the
        library's batched solve drives the problems from `workers` host threads."""
        X = [self.torch.zeros_like(b) for b in B]
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = self.ctx.pcg(B, X, rtol=rtol, nthreads=self.workers, raise_on_error=False)
        self.torch.cuda.synchronize()
        return X, infos, time.perf_counter() - t0

    def close(self):
        self.ctx.close()


def run_batch(count=64, nrhs=16, workers=16, steps=2, precision=S.MIXED, block_gemm=0):
    import workloads as W
    t0 = time.time()
    probs = [GN.generate(W.batched_c4(i), with_mass=True) for i in range(count)]
    _log(f"generated {count} problems ({sum(g.fine.n for g in probs)} DOFs) in {time.time() - t0:.1f} s")
    bs = BatchSolver(probs, nrhs=nrhs, precision=precision, workers=workers, block_gemm=block_gemm)
    B = bs.rhs()
    bs.solve(B)  # warm-up: graph capture per context
    dof_it, wall, worst, status = 0, 0.0, 0.0, 0
    for _ in range(steps):
        X, infos, dt = bs.solve(B)
        wall += dt
        for g, inf in zip(probs, infos):
            dof_it += g.fine.n * sum(i.iterations for i in inf)
            worst = max(worst, max(i.true_rel_res for i in inf))
            status = status or next((i.status for i in inf if i.status != 0), 0)
    bs.close()
    res = {"problems": count, "nrhs": nrhs, "workers": workers, "block_gemm": block_gemm,
           "fine_dofs": int(sum(g.fine.n for g in probs)),
           "ms_per_batch": round(1e3 * wall / steps, 2), "mdofs": round(dof_it / wall / 1e6, 1),
           "worst_true_rel_res": worst, "status": status}
    _log(json.dumps(res))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", type=int, default=64)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--block-gemm", type=int, default=0, choices=[0, 1, 2],
                    help="general blocks: 0 CSR FP64, 1 FP64 patch GEMMs, 2 BF16 patch GEMMs (matrix cores)")
    a = ap.parse_args(argv)
    print(json.dumps(run_batch(a.problems, a.nrhs, a.workers, a.steps, block_gemm=a.block_gemm)))


if __name__ == "__main__":
    main()
