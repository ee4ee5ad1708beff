"""Multigrid hierarchy (oracle; test infrastructure only).

Restriction, prolongation and coarse grid correction subsection:
* the level l-1 space is nested in the level l space, so there is a matrix
  R_l with Phi_{l-1} = R_l Phi_l (eq:coarsening); prolongation is R_l^T;
* Remark rem:gridParamCorr: the coarse problem is purely algebraic,
  A_{l-1} = R_l A_l R_l^T and r_{l-1} = R_l r_l (the penalty parameter is
  inherited unchanged).

R_l is obtained here from its definition: the 1D coarse functions are
sampled at n_f + p distinct points together with the 1D fine functions and
the interpolation system C = R1 F is solved (for B-splines the sample points
are the fine Greville abscissae, where the collocation matrix is
non-singular; for Lagrange functions they are the fine nodes, where F = I).
The multivariate R is the Kronecker product of the 1D matrices (x fastest),
restricted to active coarse rows and active fine columns.  Restricting the
columns is exact on Omega_h because inactive fine functions vanish there.

Readings: a coarse element is active when any child is active (equivalently
any leaf vertex inside it is positive); coarse active functions are those
non-zero on an active coarse element, minus the box-Dirichlet ones.  The
coarse pattern is the structural pattern of shared active coarse elements.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis as B
from .assemble import make_level, structural_pattern


def greville(n: int, p: int, lo: float, hi: float) -> np.ndarray:
    t = B.open_knots(n, p, lo, hi)
    if p == 0:
        return 0.5 * (t[:-1] + t[1:])
    return np.array([t[i + 1:i + p + 1].mean() for i in range(n + p)])


def two_scale_1d(basis: str, n_c: int, p: int, lo: float, hi: float) -> np.ndarray:
    """Dense 1D R with Phi_c(x) = R Phi_f(x), fine grid of 2 n_c elements."""
    n_f = 2 * n_c
    if basis == "bspline":
        x = greville(n_f, p, lo, hi)
    else:
        x = B.lagrange_nodes_1d(n_f, p, lo, hi)
    F = B.all_1d(basis, n_f, p, x, lo, hi)       # (nf_funcs, npts)
    C = B.all_1d(basis, n_c, p, x, lo, hi)       # (nc_funcs, npts)
    R = np.linalg.solve(F.T, C.T).T               # R F = C
    R[np.abs(R) < 1e-13] = 0.0
    return R


def restriction(basis: str, coarse, fine) -> sp.csr_matrix:
    """Masked tensor-product R (coarse active x fine active)."""
    R1 = two_scale_1d(basis, coarse.n, coarse.p, coarse.lo, coarse.hi)
    Rk = sp.csr_matrix(R1)
    for _ in range(coarse.dim - 1):
        Rk = sp.kron(sp.csr_matrix(R1), Rk, format="csr")  # x fastest: kron(R_y, R_x)
    Rm = Rk[coarse.active][:, fine.active]
    Rm = sp.csr_matrix(Rm)
    Rm.eliminate_zeros()
    Rm.sort_indices()
    return Rm


def galerkin(R: sp.csr_matrix, A: sp.csr_matrix, coarse) -> sp.csr_matrix:
    """A_c = R A R^T stored on the structural pattern of the coarse level."""
    Ac = (R @ A @ R.T).tocsr()
    P = structural_pattern(coarse)
    Ad = Ac.toarray() if Ac.shape[0] <= 6000 else None
    out = P.copy().astype(np.float64)
    if Ad is not None:
        r, c = P.nonzero()
        out = sp.csr_matrix((Ad[r, c], (r, c)), shape=P.shape)
        # nothing of R A R^T may fall outside the structural pattern
        mask = np.ones_like(Ad, dtype=bool)
        mask[r, c] = False
        assert np.all(Ad[mask] == 0.0)
    else:
        Ac = Ac.tocoo()
        lookup = {(i, j): v for i, j, v in zip(Ac.row, Ac.col, Ac.data)}
        r, c = P.nonzero()
        vals = np.array([lookup.get((i, j), 0.0) for i, j in zip(r, c)])
        pat = set(zip(r.tolist(), c.tolist()))
        assert all(((i, j) in pat) or v == 0.0 for (i, j), v in lookup.items())
        out = sp.csr_matrix((vals, (r, c)), shape=P.shape)
    out.sort_indices()
    return out


class Hierarchy:
    """Levels 1 (coarsest) .. L (finest), stored in lists indexed 0..L-1."""

    def __init__(self, w, fine_system, leaf):
        L = w.levels
        self.w = w
        self.levels = [None] * L
        self.A = [None] * L
        self.R = [None] * (L - 1)   # R[l] maps level l+1 (0-based index) -> level l
        self.levels[L - 1] = fine_system.level
        self.A[L - 1] = fine_system.A
        strong = w.bc == "box_dirichlet"
        for k in range(L - 2, -1, -1):
            fine = self.levels[k + 1]
            coarse = make_level(w, leaf, fine.n // 2, fine.depth + 1, strong)
            self.levels[k] = coarse
            self.R[k] = restriction(w.basis, coarse, fine)
            self.A[k] = galerkin(self.R[k], self.A[k + 1], coarse)
