"""Per-block damping: features, two-grid objective and stability check
(test infrastructure only).

The paper damps all additive Schwarz blocks of a level with one factor
gamma = 1 / max_K N_K (the damping discussion after eq:applyCS).  Per-block
weights omega_j generalize it: S_omega = sum_j omega_j P_j A_j^{-1} P_j^T.

* Objective.  The two-grid error propagation operator of the multigrid
  analysis (eq:eigenMulti) with one pre- and one post-smoothing step,
      E(omega) = (I - S_omega A)(I - R^T A_c^{-1} R A)(I - S_omega A),
  is scored on a fixed block of vectors Z in the energy norm, in which E is
  self-adjoint and (for stable weights) contractive:
      J(omega) = sum_cols ||E^k z||_A^2 / sum_cols ||z||_A^2,
  whose gradient follows from the adjoint recursion written out in
  `two_grid_objective`.
* Stability.  The smoother must keep lambda_max(S_omega A) below 2 so that
  I - S_omega A stays a contraction in the energy norm (the stability
  condition eq:stabilityMulti); learned weights are accepted only when
  lambda_max(S_omega A) < 2 (1 - 0.05).
* Features.  Sixteen scale-free numbers per final block, listed in
  `FEATURES`, computed from the block lists, the element incidence, the
  element volume fractions eta_K = |K cap Omega| / |K| and the block
  eigenvalues.

All FP64 dense NumPy (small problems only).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import assemble as AS

FEATURES = (
    "final block size / (2p+1)^d",
    "input block size / (2p+1)^d (1 for blocks added for uncovered DOFs)",
    "active elements in the block's support (union of its input members' supports) / (p+1)^d",
    "sum of eta_K over that support / (p+1)^d",
    "log10(max(min eta_K, 1e-16)) / 16 over that support",
    "mean over the support's cut elements (eta_K < 1 - 1e-12) of log10(max(eta_K, 1e-16)) / 16 (0 if none)",
    "max N_K over the support / (p+1)^d",
    "mean N_K over the support / (p+1)^d",
    "log10(lambda_max / lambda_min) / 16 of the final block",
    "log10(max(lambda_min / max diag, 1e-30)) / 16 of the input block (before removals)",
    "functions removed from the block / (2p+1)^d",
    "fraction of the final block's functions whose support holds a cut element",
    "x offset of the eta-weighted element centroid of the support from its unweighted centroid / (p+1)",
    "y offset (same)",
    "z offset (same; 0 in 2D)",
    "fraction of the level's active elements that are cut (eta_K < 1 - 1e-12)",
)
NFEAT = len(FEATURES)
SAFETY = 2.0 * (1.0 - 0.05)
CUT_ETA = 1.0 - 1e-12   # an element counts as cut when eta_K < CUT_ETA


def volume_fractions(hier, fine_vol_frac):
    """eta per level (dict: element linear index -> eta, active elements only).

    The finest level takes the assembled |K cap Omega_h| / |K|; a coarse
    element's fraction is the mean of its 2^d children's fractions (its
    volume is the sum of theirs)."""
    L = len(hier.levels)
    out = [None] * L
    out[L - 1] = dict(fine_vol_frac)
    for l in range(L - 2, -1, -1):
        fine, coarse = hier.levels[l + 1], hier.levels[l]
        d, nc = coarse.dim, coarse.n
        eta = {}
        for el in coarse.elem_funcs:
            e = _multi(el, nc, d)
            acc = 0.0
            for off in np.ndindex(*(2,) * d):
                child = tuple(2 * e[a] + off[a] for a in range(d))
                acc += out[l + 1].get(AS.element_lin(child, fine.n), 0.0)
            eta[el] = acc / 2 ** d
        out[l] = eta
    return out


def _multi(el, n, d):
    m = []
    for _ in range(d):
        m.append(el % n)
        el //= n
    return tuple(m)


def _func_elements(lev):
    """compact function index -> sorted list of active element linear indices"""
    pos = {int(L): i for i, L in enumerate(lev.active)}
    fe = [[] for _ in range(len(lev.active))]
    for el in sorted(lev.elem_funcs):
        for L in lev.elem_funcs[el]:
            i = pos.get(int(L))
            if i is not None:
                fe[i].append(el)
    return fe


def block_features(lev, A, sm, eta):
    """(nblocks x 16) features of the final blocks of smoother `sm` on a level
    (A: the level's operator, eta: its volume fractions)."""
    d, p = lev.dim, lev.p
    K = (2 * p + 1) ** d
    E = (p + 1) ** d
    A = sp.csr_matrix(A)
    fe = _func_elements(lev)
    # N_K over the final blocks
    nk = {}
    for blk in sm.blocks:
        els = set()
        for i in blk:
            els.update(fe[int(i)])
        for el in els:
            nk[el] = nk.get(el, 0) + 1
    cut_fn = np.array([any(eta[el] < CUT_ETA for el in fe[i]) for i in range(len(fe))], dtype=bool)
    nraw = len(sm.raw_blocks)
    cut_level = np.mean([v < CUT_ETA for v in eta.values()])
    F = np.zeros((len(sm.blocks), NFEAT))
    for j, blk in enumerate(sm.blocks):
        raw = np.asarray(sm.raw_blocks[j]) if j < nraw else np.asarray(blk)
        # support of the block: the union of its input members' supports (the
        # associated function's support, which contains all others)
        S = sorted(set().union(*(fe[int(i)] for i in raw)))
        et = np.array([eta[el] for el in S])
        F[j, 0] = len(blk) / K
        F[j, 1] = len(raw) / K
        F[j, 2] = len(S) / E
        F[j, 3] = et.sum() / E
        F[j, 4] = np.log10(max(et.min(), 1e-16)) / 16.0
        cut = et[et < CUT_ETA]
        F[j, 5] = np.mean(np.log10(np.maximum(cut, 1e-16))) / 16.0 if len(cut) else 0.0
        n_s = np.array([nk.get(el, 0) for el in S], dtype=np.float64)
        F[j, 6] = n_s.max() / E
        F[j, 7] = n_s.mean() / E
        if len(blk) >= 2:
            lam = np.linalg.eigvalsh(A[blk][:, blk].toarray())
            F[j, 8] = np.log10(lam[-1] / lam[0]) / 16.0
        Ar = A[raw][:, raw].toarray()
        lmin = np.linalg.eigvalsh(Ar)[0]
        F[j, 9] = np.log10(max(lmin / np.max(np.diag(Ar)), 1e-30)) / 16.0
        F[j, 10] = (len(raw) - len(blk)) / K if j < nraw else 0.0
        F[j, 11] = cut_fn[np.asarray(blk, dtype=np.int64)].mean() if len(blk) else 0.0
        cen = np.array([_multi(el, lev.n, d) for el in S], dtype=np.float64)
        off = (et @ cen) / et.sum() - cen.mean(axis=0)
        F[j, 12:12 + d] = off / (p + 1)
        F[j, 15] = cut_level
    return F


def smoother_dense(sm, omega):
    """S_omega = sum_j omega_j P_j A_j^{-1} P_j^T (dense)."""
    S = np.zeros((sm.n, sm.n))
    for wj, k, inv in zip(omega, sm.blocks, sm.inv):
        if len(k):
            S[np.ix_(k, k)] += wj * inv
    return S


def two_grid_objective(A, R, Ac, sm, omega, Z, k):
    """J(omega) = tr(X_k^T A X_k) / tr(Z^T A Z) with X_k = E^k Z, and dJ/domega_j.

    Forward: X_0 = Z, X_t = E X_{t-1} with E = M C M, M = I - S A,
    C = I - R^T A_c^{-1} R A.  Adjoint: Lambda_k = 2 A X_k / tr(Z^T A Z); for t = k..1
    with a = X_{t-1}, c = C M a:
        nu = (I - A S) Lambda_t,  mu = C^T nu,
        dJ/domega_j -= <P_j^T Lambda_t, A_j^{-1} P_j^T A c> + <P_j^T mu, A_j^{-1} P_j^T A a>,
        Lambda_{t-1} = (I - A S) mu      (= E^T Lambda_t),
    using dE/domega_j = -T_j A C M - M C T_j A with T_j = P_j A_j^{-1} P_j^T and
    M^T = I - A S, C^T = I - A R^T A_c^{-1} R (A, S, A_c symmetric)."""
    A = sp.csr_matrix(A).toarray()
    R = sp.csr_matrix(R).toarray()
    Ac = sp.csr_matrix(Ac).toarray()
    n = A.shape[0]
    S = smoother_dense(sm, omega)
    I = np.eye(n)
    Cc = I - R.T @ np.linalg.solve(Ac, R @ A)
    M = I - S @ A
    E = M @ Cc @ M
    Z = np.asarray(Z, dtype=np.float64).reshape(n, -1)
    X = [Z]
    for _ in range(k):
        X.append(E @ X[-1])
    nz = float(np.sum(Z * (A @ Z)))
    J = float(np.sum(X[-1] * (A @ X[-1]))) / nz
    lam = 2.0 * (A @ X[-1]) / nz
    g = np.zeros(len(sm.blocks))
    for t in range(k, 0, -1):
        a = X[t - 1]
        c = Cc @ (M @ a)
        Aa, Acv = A @ a, A @ c
        nu = lam - A @ (S @ lam)
        mu = Cc.T @ nu
        for j, (blk, inv) in enumerate(zip(sm.blocks, sm.inv)):
            if len(blk):
                g[j] -= np.sum(lam[blk] * (inv @ Acv[blk])) + np.sum(mu[blk] * (inv @ Aa[blk]))
        lam = mu - A @ (S @ mu)
    return J, g


def lambda_max_SA(A, sm, omega):
    """Largest eigenvalue of S_omega A (real: S_omega A is similar to the
    symmetric S^{1/2} A S^{1/2})."""
    S = smoother_dense(sm, omega)
    A = sp.csr_matrix(A).toarray()
    return float(np.max(np.linalg.eigvals(S @ A).real))
