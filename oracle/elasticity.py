"""Linear elasticity with penalty Dirichlet conditions (oracle; test
infrastructure only).

Immersed finite element formulation, eq:strongMulti / eq:weakMulti /
eq:operatorsMulti: find u_h in V_h^d with a_h(v, u_h) = b_h(v) for all v,

    a_h(v, u) = int_Omega grad^s v : sigma(u)
                + int_Gamma_D ( lambda beta (v.n)(u.n) + 2 mu beta v.u )
    b_h(v)    = int_Omega v.f + int_Gamma_D ( lambda beta (v.n)(g_D.n)
                + 2 mu beta v.g_D ) + int_Gamma_N v.g_N

with sigma(u) = lambda div(u) I + 2 mu grad^s u and beta = beta^lambda =
beta^mu = penalty_factor / h of the finest grid (the examples use 2/h).
The coarse levels inherit the fine weak form algebraically (Remark
rem:gridParamCorr), so the penalty parameter is not rescaled.

Basis and numbering.  V_h^d is spanned by phi_i e_c (c = 0 .. d-1) for the
active scalar functions phi_i of the scalar formulation (no function is
removed: the Dirichlet condition is weak).  Vector DOFs are numbered
component-major: DOF c N + i is component c of scalar function i (N active
scalar functions, ascending lattice index).

Entry of the stiffness between phi_a e_c and phi_b e_c' (from
grad^s(phi e_c) = (e_c (x) grad phi + grad phi (x) e_c) / 2):

    lambda d_c phi_a d_c' phi_b + mu ( delta_cc' grad phi_a . grad phi_b
                                       + d_c' phi_a d_c phi_b ).

Blocks of the Schwarz smoother (smoothers subsection): separate blocks for
the functions of each component, i.e. the scalar blocks by encapsulating
supports repeated for every component.  The relaxation gamma = 1 / max_K N_K
counts the blocks of every component that touch element K (the components
are coupled by A, so each of them enters the bound of eq:applyCS).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import assemble as AS
from . import geometry as G
from . import hierarchy as H
from . import multigrid as MG
from . import quadrature as Q
from . import schwarz as SW


def element_stiffness(vw, Gr, lam, mu):
    """(d, d) nested list of (nloc, nloc) blocks K[c][c'] of the element
    stiffness at quadrature weights vw and local gradients Gr (nloc, nq, d)."""
    d = Gr.shape[2]
    # D[c][e][a, b] = sum_q w_q d_c phi_a(x_q) d_e phi_b(x_q)
    D = [[(Gr[:, :, c] * vw) @ Gr[:, :, e].T for e in range(d)] for c in range(d)]
    lap = sum(D[e][e] for e in range(d))
    K = [[None] * d for _ in range(d)]
    for c in range(d):
        for e in range(d):
            blk = lam * D[c][e] + mu * D[e][c]
            if c == e:
                blk = blk + mu * lap
            K[c][e] = blk
    return K


def penalty_blocks(bw, Vb, bn, mask, lam, mu, beta):
    """(d, d) blocks of the Dirichlet penalty term on the boundary points with
    mask set: lambda beta (v.n)(u.n) + 2 mu beta v.u."""
    d = bn.shape[1]
    wq = bw * mask
    Mb = (Vb * wq) @ Vb.T
    K = [[None] * d for _ in range(d)]
    for c in range(d):
        for e in range(d):
            blk = lam * beta * ((Vb * (wq * bn[:, c] * bn[:, e])) @ Vb.T)
            if c == e:
                blk = blk + 2.0 * mu * beta * Mb
            K[c][e] = blk
    return K


@dataclass
class VectorSystem:
    level: AS.Level
    ncomp: int
    A: sp.csr_matrix
    b: np.ndarray
    M: sp.csr_matrix          # vector mass kron(I_d, M_scalar): the L2(Omega)^d metric
    omega_measure: float
    gamma_d_measure: float    # |Gamma_D| of the approximate boundary
    vol_frac: dict = None     # element linear index -> |K cap Omega_h| / |K|


def assemble_elasticity(w, leaf, n, depth, orders=None, force=None, g_dirichlet=None, traction=None,
                        traction_on="neumann", lam=None, mu=None, beta=None) -> VectorSystem:
    """Assemble A, b and the vector mass matrix on the level with n elements
    per axis.  force(pts) -> (nq, d) body load (default: w.force, constant);
    g_dirichlet(pts) -> (nq, d) Dirichlet data (default 0); traction(pts,
    normals) -> (nq, d) boundary traction applied on Gamma_N ("neumann") or on
    the whole approximate boundary ("all"; used by the consistency pin).
    lam, mu, beta override the workload's values (beta = 0: no penalty)."""
    lev = AS.make_level(w, leaf, n, depth, strong_box=False)
    d, p = w.dim, w.degree
    qc, qs, qb = orders if orders is not None else Q.default_orders(d, p)
    lam = w.lame_lambda if lam is None else lam
    mu = w.lame_mu if mu is None else mu
    beta = (w.penalty_factor / lev.h if w.bc == "penalty" else 0.0) if beta is None else beta
    fconst = np.zeros(d) if w.force is None else np.asarray(w.force, dtype=np.float64)
    N = len(lev.active)
    pos = {int(L): i for i, L in enumerate(lev.active)}
    rows, cols, vals = [], [], []
    mrows, mcols, mvals = [], [], []
    b = np.zeros(d * N)
    omega = 0.0
    gd_meas = 0.0
    vol_frac = {}
    for e in zip(*np.nonzero(lev.active_el)):
        el = AS.element_lin(e, n)
        fl = lev.elem_funcs[el]
        vp, vw, bp, bw, bn = Q.element_quadrature(leaf, e, depth, lev.lo, lev.h, qc, qs, qb)
        omega += float(vw.sum())
        vol_frac[el] = float(vw.sum()) / lev.h ** d
        V, Gr = AS.tensor_eval(lev, e, vp)
        K = element_stiffness(vw, Gr, lam, mu)
        Ml = (V * vw) @ V.T
        fv = force(vp) if force is not None else np.tile(fconst, (len(vw), 1))
        fb = [V @ (vw * fv[:, c]) for c in range(d)]
        if len(bw):
            Vb, _ = AS.tensor_eval(lev, e, bp)
            dmask = G.dirichlet_mask(w, bp).astype(np.float64)
            gd_meas += float(np.sum(bw * dmask))
            if beta > 0.0:
                P = penalty_blocks(bw, Vb, bn, dmask, lam, mu, beta)
                K = [[K[c][k] + P[c][k] for k in range(d)] for c in range(d)]
                if g_dirichlet is not None:
                    gd = g_dirichlet(bp)
                    gn = np.sum(gd * bn, axis=1)
                    for c in range(d):
                        rhs = lam * beta * gn * bn[:, c] + 2.0 * mu * beta * gd[:, c]
                        fb[c] = fb[c] + Vb @ (bw * dmask * rhs)
            if traction is not None:
                t = traction(bp, bn)
                where = (1.0 - dmask) if traction_on == "neumann" else np.ones_like(dmask)
                for c in range(d):
                    fb[c] = fb[c] + Vb @ (bw * where * t[:, c])
        loc = np.array([pos.get(L, -1) for L in fl])
        ok = loc >= 0
        li = loc[ok]
        ia, ib = np.meshgrid(np.nonzero(ok)[0], np.nonzero(ok)[0], indexing="ij")
        ra, rb = np.meshgrid(li, li, indexing="ij")
        for c in range(d):
            b[c * N + li] += fb[c][ok]
            for k in range(d):
                rows.append((c * N + ra).ravel())
                cols.append((k * N + rb).ravel())
                vals.append(K[c][k][ia, ib].ravel())
        mrows.append(ra.ravel())
        mcols.append(rb.ravel())
        mvals.append(Ml[ia, ib].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(d * N, d * N)).tocsr()
    A = 0.5 * (A + A.T)   # the blocks are symmetric up to rounding: exact symmetry
    A = A.tocsr()
    A.sort_indices()
    Ms = sp.coo_matrix((np.concatenate(mvals), (np.concatenate(mrows), np.concatenate(mcols))),
                       shape=(N, N)).tocsr()
    Ms = (0.5 * (Ms + Ms.T)).tocsr()
    M = sp.kron(sp.identity(d, format="csr"), Ms, format="csr")
    return VectorSystem(level=lev, ncomp=d, A=A, b=b, M=M, omega_measure=omega, gamma_d_measure=gd_meas,
                        vol_frac=vol_frac)


def vector_pattern(lev, d):
    """Structural pattern of the vector operator: every component pair on the
    scalar structural pattern."""
    P = AS.structural_pattern(lev)
    return sp.kron(sp.csr_matrix(np.ones((d, d))), P, format="csr")


def galerkin_vector(Rv, A, coarse, d):
    """A_c = R A R^T (R = I_d (x) R_scalar) on the coarse vector pattern."""
    Ac = (Rv @ A @ Rv.T).tocsr()
    P = vector_pattern(coarse, d).tocoo()
    Acc = Ac.tocoo()
    lookup = {(i, j): v for i, j, v in zip(Acc.row.tolist(), Acc.col.tolist(), Acc.data.tolist())}
    pat = set(zip(P.row.tolist(), P.col.tolist()))
    assert all(((i, j) in pat) or v == 0.0 for (i, j), v in lookup.items())
    vals = np.array([lookup.get((i, j), 0.0) for i, j in zip(P.row.tolist(), P.col.tolist())])
    out = sp.csr_matrix((vals, (P.row, P.col)), shape=P.shape)
    out.sort_indices()
    return out


class VectorHierarchy:
    """Levels 1 (coarsest) .. L (finest) of a vector problem, lists indexed
    0..L-1: scalar levels, vector operators, R[l] = I_d (x) R_scalar[l]."""

    def __init__(self, w, fine: VectorSystem, leaf):
        L = w.levels
        d = fine.ncomp
        self.ncomp = d
        self.levels = [None] * L
        self.A = [None] * L
        self.R = [None] * (L - 1)
        self.R_scalar = [None] * (L - 1)
        self.levels[L - 1] = fine.level
        self.A[L - 1] = fine.A
        for k in range(L - 2, -1, -1):
            f = self.levels[k + 1]
            coarse = AS.make_level(w, leaf, f.n // 2, f.depth + 1, False)
            self.levels[k] = coarse
            Rs = H.restriction(w.basis, coarse, f)
            self.R_scalar[k] = Rs
            self.R[k] = sp.kron(sp.identity(d, format="csr"), Rs, format="csr")
            self.A[k] = galerkin_vector(self.R[k], self.A[k + 1], coarse, d)


def vector_blocks(lev, d):
    """The scalar blocks by encapsulating supports, repeated per component
    (component c's copy shifted by c N), components in order."""
    sb, assoc = SW.select_blocks(lev)
    N = len(lev.active)
    blocks, vassoc = [], []
    for c in range(d):
        for blk, a in zip(sb, assoc):
            blocks.append(blk + c * N)
            vassoc.append(a + c * N)
    return blocks, vassoc


def max_NK_vector(lev, blocks, d) -> int:
    """max over active elements K of the number of blocks (of any component)
    holding a function non-zero on K."""
    N = len(lev.active)
    scalar = [np.unique(np.asarray(blk) % N) for blk in blocks]
    return SW.max_NK(lev, scalar)


class VectorSmoother(SW.Smoother):
    """Additive Schwarz with per-component blocks on one level of a vector
    problem."""

    def __init__(self, A, lev, d, blocks=None):
        if blocks is None:
            blocks, _ = vector_blocks(lev, d)
        self._vec = (lev, d)
        super().__init__(A, lev, blocks=blocks)

    def _gamma(self, lev, blocks):
        return 1.0 / max_NK_vector(lev, blocks, self._vec[1])


class VectorMultiplicativeSmoother(SW.MultiplicativeSmoother):
    """Multiplicative Schwarz (eq:multiplicativeSchwarz1) with per-component
    blocks.  Blocks of different components that share an element are coupled
    by A, so they need different colours: the block of component c associated
    with scalar function a takes c (p+1)^d + the scalar lattice colour of a
    (d (p+1)^d colours for uncut B-splines, three times the scalar count);
    added singletons are coloured greedily from d (p+1)^d."""

    def __init__(self, A, lev, d):
        blocks, vassoc = vector_blocks(lev, d)
        self._vec = (lev, d)
        SW.Smoother.__init__(self, A, lev, blocks=blocks)
        N = len(lev.active)
        q = (lev.p + 1) ** lev.dim
        given = [(a // N) * q + SW.lattice_colour(lev, lev.active[a % N]) for a in vassoc]
        self._order_blocks(A, lev, vassoc, given, lambda b: b % N, d * q)

    def _gamma(self, lev, blocks):
        return 1.0 / max_NK_vector(lev, blocks, self._vec[1])


@dataclass
class ElasticityProblem:
    w: object
    leaf: np.ndarray
    system: VectorSystem
    hier: VectorHierarchy
    smoothers: list
    vcycle: MG.VCycle

    @property
    def A(self):
        return self.system.A

    @property
    def b(self):
        return self.system.b

    def solve(self, b=None, tol=1e-8, max_iter=2000, flexible=False):
        b = self.b if b is None else b
        return MG.pcg(self.A, b, self.vcycle.apply, tol=tol, max_iter=max_iter, flexible=flexible)


def build(w, orders=None, smoothers=True) -> ElasticityProblem:
    leaf = G.leaf_values(w, w.n, w.depth)
    sysf = assemble_elasticity(w, leaf, w.n, w.depth, orders=orders)
    hier = VectorHierarchy(w, sysf, leaf)
    sm = [None] * w.levels
    vc = None
    if smoothers:
        for l in range(1, w.levels):
            A, lev = hier.A[l], hier.levels[l]
            kind = w.smoother if (l == w.levels - 1 or w.coarse_smoother == "same") else w.coarse_smoother
            if kind == "ms":
                sm[l] = VectorMultiplicativeSmoother(A, lev, sysf.ncomp)
            elif kind == "jacobi":
                # diagonal smoothing on the coarser levels (Remark rem:coarseGS),
                # damped by the additive rule with one block per DOF
                sm[l] = VectorSmoother(A, lev, sysf.ncomp, blocks=[np.array([i]) for i in range(A.shape[0])])
            elif kind == "as":
                sm[l] = VectorSmoother(A, lev, sysf.ncomp)
            else:
                raise ValueError(f"vector problems: smoother {kind}")
        vc = MG.VCycle(hier.A, hier.R, sm, nu_pre=w.nu, nu_post=w.nu, cycle=w.cycle)
    return ElasticityProblem(w=w, leaf=leaf, system=sysf, hier=hier, smoothers=sm, vcycle=vc)
