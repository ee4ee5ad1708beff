"""V-cycle and multigrid-preconditioned CG (oracle; test infrastructure only).

Algorithm alg:MGV, V-cycle(l, r_l):
  l > 1: x = 0; pre-smooth x = x + gamma M^{-1} r; update the residual;
         restrict r_{l-1} = R_l r; x_{l-1} = V-cycle(l-1, r_{l-1});
         prolongate x = x + R_l^T x_{l-1}; update the residual;
         post-smooth with the adjoint smoother (additive Schwarz is symmetric,
         so the adjoint is the same operator).
  l = 1: direct solve x = A_1^{-1} r.

Readings:
* the residual update after the prolongation is the residual of the current
  approximation, r_in - A x (the algorithm's second update read literally
  would subtract the pre-smoothed part twice);
* nu smoothing steps before and after (the paper uses one; the 1024^2
  cubic benchmark asks for two): each step is x += S (r_in - A x), with the
  smoother's pre-smoothing operator before and its adjoint after the coarse
  correction (additive Schwarz: the same symmetric operator; multiplicative
  Schwarz: the forward colour sweep before, the reversed one after);
* the coarsest "direct solve" is a dense Cholesky solve;
* the V-cycle is used as the preconditioner of CG (the paragraph after the
  algorithm), with x_0 = 0 and the stopping test ||r_k|| <= tol min(||r_0||,
  ||b||) in the 2-norm (the two agree for x_0 = 0); on stopping, the true
  residual ||b - A x|| / ||b|| is recomputed and, while it is above tol, CG is
  restarted from the current x (r = b - A x, fresh direction; the threshold
  and the iteration count carry over), at most three times; a solve that
  ends above tol reports that it did not converge;
* multigrid as a standalone solver (the same paragraph): x <- x + B(b - A x)
  from x0 until the relative residual meets tol; full multigrid (FMG, named
  there too) as nested iteration with one cycle per level;
* the paper names CG without a variant; besides the Hestenes-Stiefel beta the
  Polak-Ribiere ("flexible") form beta = r_{k+1}.(z_{k+1} - z_k) / r_k.z_k is
  offered, which equals it in exact arithmetic for a fixed SPD preconditioner
  (r_{k+1}.z_k = 0 there).  It is pinned only through that equality; how it
  behaves under a preconditioner that changes between iterations is parity
  unpinned (nothing here varies the V-cycle).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class VCycle:
    """cycle = 1: the V-cycle of Algorithm alg:MGV; cycle = 2: the W-cycle
    (the paragraph after the algorithm names W- and FMG-cycles as other
    multigrid cycles): on every level above level 1 the coarse correction is
    computed by two consecutive coarse cycles, the second on the residual the
    first leaves (level 1's coarse problem is solved directly, once)."""

    def __init__(self, A_list, R_list, smoothers, nu_pre=1, nu_post=1, cycle=1):
        self.A = A_list
        self.R = R_list
        self.S = smoothers          # index 0 (coarsest) unused
        self.nu_pre = nu_pre
        self.nu_post = nu_post
        self.cycle = cycle
        A1 = A_list[0].toarray()
        self.coarse_chol = sla.cho_factor(A1, lower=True)

    def apply(self, r: np.ndarray, level: int = None) -> np.ndarray:
        if level is None:
            level = len(self.A) - 1
        if level == 0:
            return sla.cho_solve(self.coarse_chol, r)
        A = self.A[level]
        S = self.S[level]
        x = S.pre(r)
        for _ in range(self.nu_pre - 1):
            x = x + S.pre(r - A @ x)
        rh = r - A @ x
        rc = self.R[level - 1] @ rh
        xc = self.apply(rc, level - 1)
        if level - 1 > 0:
            for _ in range(self.cycle - 1):
                xc = xc + self.apply(rc - self.A[level - 1] @ xc, level - 1)
        x = x + self.R[level - 1].T @ xc
        for _ in range(self.nu_post):
            x = x + S.post(r - A @ x)
        return x

    def dense(self, level: int = None) -> np.ndarray:
        """Matrix of the V-cycle operator B (z = B r) by unit-vector probing."""
        if level is None:
            level = len(self.A) - 1
        n = self.A[level].shape[0]
        Bm = np.zeros((n, n))
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            Bm[:, i] = self.apply(e, level)
        return Bm


MAX_RESTARTS = 3


def pcg(A, b, precond, tol=1e-8, max_iter=1000, x0=None, flexible=False, info=None):
    """Preconditioned CG (Hestenes-Stiefel; flexible=True: Polak-Ribiere beta).
    Returns (x, iterations, history) where history holds ||r_k|| / ||r_0|| of
    the first start.  If a dict is passed as `info` it receives the restart
    count, the final true relative residual and `converged`."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    r = b - A @ x
    r0 = np.linalg.norm(r)
    thr = tol * min(r0, bnorm)
    hist = [1.0]
    it = 0
    restarts = 0
    true_rel = r0 / bnorm if bnorm > 0 else 0.0
    while r0 > 0.0:
        z = precond(r)
        p = z.copy()
        rz = r @ z
        stopped = False
        while it < max_iter:
            q = A @ p
            alpha = rz / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            rn = np.linalg.norm(r)
            if restarts == 0:
                hist.append(rn / r0)
            if rn <= thr:
                stopped = True
                break
            z_old = z
            z = precond(r)
            rz_new = r @ z
            num = rz_new - r @ z_old if flexible else rz_new
            p = z + (num / rz) * p
            rz = rz_new
        r = b - A @ x
        true_rel = np.linalg.norm(r) / bnorm if bnorm > 0 else np.linalg.norm(r)
        if true_rel <= tol or not stopped or restarts == MAX_RESTARTS:
            break
        restarts += 1
    if info is not None:
        info.update(restarts=restarts, true_rel=true_rel, converged=bool(true_rel <= tol))
    return x, it, hist


def mg_solve(A, b, precond, tol=1e-8, max_cycles=500, x0=None):
    """Multigrid as a standalone solver (the paragraph after Algorithm
    alg:MGV): x <- x + B (b - A x) until ||b - A x|| <= tol ||b||.
    Returns (x, cycles, relative residual)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    k = 0
    while True:
        r = b - A @ x
        rel = np.linalg.norm(r) / bn if bn > 0 else np.linalg.norm(r)
        if rel <= tol or k >= max_cycles:
            return x, k, rel
        x = x + precond(r)
        k += 1


def fmg(vc: VCycle, b):
    """Full multigrid (the FMG cycle named after Algorithm alg:MGV; nested
    iteration): the right-hand side restricted to every level, the coarsest
    problem solved directly, and on every finer level the coarser solution,
    prolongated, improved by one cycle of that level."""
    L = len(vc.A)
    bs = [None] * L
    bs[L - 1] = b
    for l in range(L - 1, 0, -1):
        bs[l - 1] = vc.R[l - 1] @ bs[l]
    x = vc.apply(bs[0], level=0)
    for l in range(1, L):
        x = vc.R[l - 1].T @ x
        x = x + vc.apply(bs[l] - vc.A[l] @ x, level=l)
    return x
