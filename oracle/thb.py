"""Truncated hierarchical B-splines and hierarchical coarsening (oracle; test
infrastructure only).

Immersed formulation section (Figure fig:THB): a hierarchical mesh has local
refinement levels m = 0..M, level-m cells being 2^m times narrower than the
level-0 cells.  Omega^m, the region covered by elements of level >= m, is a
union of level-m cells (children of refined level-(m-1) cells); the active
elements of level m are the level-m cells of Omega^m that are not refined.
A level-m B-spline belongs to the hierarchical basis when (i) it is non-zero
on at least one active element of level m and (ii) its whole support lies in
Omega^m.  The truncated basis replaces every such function by its truncation
with respect to the finer levels: written in the level-(m+1) B-splines by
the two-scale relation, the components on level-(m+1) B-splines whose support
lies in Omega^{m+1} are dropped; the rest is treated the same way at level
m+2, and so on up to level M.

Restriction subsection, Algorithm alg:coarsen: the coarse mesh starts as the
uniform mesh of twice the level-0 width; for m = 0..M-1 in turn, every coarse
element of local level m that intersects a fine element of local level > m is
refined (its four children become coarse elements of level m+1).

Readings (the paper fixes none of these):
* 2D, degree p, open uniform knot vectors on [lo, hi]^2 at every level;
* the input mesh: for m = 0..M-1 the level-m cells of Omega^m that hold a
  cut cell of the finest grid (volume fraction strictly between 0 and 1, to
  1e-12) are refined, so the boundary is resolved at level M;
* a coarse element "intersects" a fine element when they overlap with
  positive area (a fine element of level > m inside it);
* every function is stored by its coefficients C_ik in the B-splines B_k of
  one common uniform grid, the finest cells of the finest mesh; integrals
  are taken on that grid (A = C A_grid C^T, b = C b_grid: exactly
  a(phi_i, phi_j) because phi_i = sum_k C_ik B_k), with the cut-cell
  quadrature of the uniform case;
* a THB function is active when it has a non-zero coefficient on an active
  grid function and none on a function with a trace on the box faces
  (strong u = 0 there, as in the uniform case);
* an element of a hierarchical mesh is active when one of its grid cells is;
  E(k) = the active elements on which phi_k is non-zero (THB coefficients
  are non-negative, so phi_k is non-zero exactly on the cells its grid
  coefficients touch); blocks by support inclusion and N_K over these;
* R_l is the unique matrix with C_{l-1} = R_l C_l (the coarse THB space lies
  in the fine one), computed by the normal equations of that identity and
  restricted to active rows and columns; coarse operators are Galerkin
  products (Remark rem:gridParamCorr);
* numbering: by level m, then the level's lattice index (x fastest).

Linear elasticity on THB levels (the physics of the paper's THB example:
eq:weakMulti / eq:operatorsMulti, penalty Dirichlet conditions) takes the
same functions for every displacement component: DOF c N + i is component c
of THB function i (component-major), A = (I_d kron C) A_grid (I_d kron C)^T
with the vector grid operator of the uniform case, R_l = I_d kron R_l,scalar,
and the Schwarz blocks of the scalar level repeated per component (the
smoothers subsection's separate blocks per component); N_K counts the blocks
of every component, and the multiplicative smoother colours the vector
blocks greedily in block order, as on scalar THB levels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assemble as AS
from . import basis as B
from . import geometry as G
from . import hierarchy as H
from . import multigrid as MG
from . import schwarz as SW

CUT_TOL = 1e-12


@dataclass
class HMesh:
    """Hierarchical mesh of a square: n0 level-0 cells per axis, M local
    levels; dom[m] (bool, shape (n0 2^m,)*2, indexed [ix, iy]) marks the
    level-m cells of Omega^m (dom[0] is every cell)."""
    n0: int
    M: int
    dom: list

    def cells(self, m: int) -> int:
        return self.n0 * 2 ** m

    def refined(self, m: int) -> np.ndarray:
        if m >= self.M:
            return np.zeros((self.cells(m),) * 2, dtype=bool)
        return self.dom[m + 1][::2, ::2].copy()

    def active_cells(self, m: int) -> np.ndarray:
        return self.dom[m] & ~self.refined(m)

    def elements(self):
        """Active elements as (m, ex, ey), by level, then ey, then ex."""
        out = []
        for m in range(self.M + 1):
            act = self.active_cells(m)
            for ey in range(self.cells(m)):
                for ex in range(self.cells(m)):
                    if act[ex, ey]:
                        out.append((m, ex, ey))
        return out


def children(mask: np.ndarray) -> np.ndarray:
    return np.kron(mask, np.ones((2, 2), dtype=bool)).astype(bool)


def refine_at_boundary(n0: int, M: int, vol_frac: np.ndarray) -> HMesh:
    """The input mesh: level-m cells holding a cut grid cell are refined.
    vol_frac[ix, iy]: volume fractions of the cells of the n0 2^M grid."""
    n_grid = n0 * 2 ** M
    cut = (vol_frac > CUT_TOL) & (vol_frac < 1.0 - CUT_TOL)
    dom = [np.ones((n0, n0), dtype=bool)]
    for m in range(M):
        nm = n0 * 2 ** m
        s = n_grid // nm
        ref = np.zeros((nm, nm), dtype=bool)
        for ey in range(nm):
            for ex in range(nm):
                if dom[m][ex, ey] and cut[ex * s:(ex + 1) * s, ey * s:(ey + 1) * s].any():
                    ref[ex, ey] = True
        dom.append(children(ref))
    return HMesh(n0, M, dom)


def grid_volume_fractions(system, n_grid: int) -> np.ndarray:
    """[ix, iy] volume fractions of a uniform system (0 off the active cells)."""
    out = np.zeros((n_grid, n_grid))
    for el, v in system.vol_frac.items():
        out[el % n_grid, el // n_grid] = v
    return out


def coarsen(fine: HMesh) -> HMesh:
    """Algorithm alg:coarsen."""
    if fine.n0 % 2:
        raise ValueError("the level-0 cell count must be even to coarsen")
    n0c = fine.n0 // 2
    dom = [np.ones((n0c, n0c), dtype=bool)]          # uniform, unrefined coarse mesh
    for m in range(fine.M):
        ncm = n0c * 2 ** m                           # coarse level-m cells per axis
        # fine elements of local level > m cover Omega_h^{m+1}: level-(m+1)
        # fine cells, 4 x 4 of them inside one coarse level-m cell
        hi = fine.dom[m + 1]
        nxt = np.zeros((2 * ncm, 2 * ncm), dtype=bool)
        for ey in range(ncm):
            for ex in range(ncm):
                if not dom[m][ex, ey]:
                    continue                         # not an element of level m
                if hi[4 * ex:4 * ex + 4, 4 * ey:4 * ey + 4].any():
                    nxt[2 * ex:2 * ex + 2, 2 * ey:2 * ey + 2] = True   # refine k_i^m
        dom.append(nxt)
    return HMesh(n0c, fine.M, dom)


def _support(n: int, p: int, i: int):
    s = B.bspline_support(n, p, i)
    return slice(s.start, s.stop)


def thb_functions(mesh: HMesh, p: int):
    """(m, ix, iy) of the hierarchical basis (conditions (i) and (ii) of
    Figure fig:THB), by level, then lattice index (x fastest)."""
    out = []
    for m in range(mesh.M + 1):
        nm = mesh.cells(m)
        act = mesh.active_cells(m)
        for iy in range(nm + p):
            for ix in range(nm + p):
                sx, sy = _support(nm, p, ix), _support(nm, p, iy)
                if mesh.dom[m][sx, sy].all() and act[sx, sy].any():
                    out.append((m, ix, iy))
    return out


def _inside(mesh: HMesh, p: int, k: int) -> np.ndarray:
    """Level-k B-splines whose support lies in Omega^k."""
    nk = mesh.cells(k)
    out = np.zeros((nk + p, nk + p), dtype=bool)
    for iy in range(nk + p):
        for ix in range(nk + p):
            out[ix, iy] = mesh.dom[k][_support(nk, p, ix), _support(nk, p, iy)].all()
    return out


def coefficients(mesh: HMesh, p: int, funcs, n_grid: int, lo=0.0, hi=1.0, truncate=True) -> sp.csr_matrix:
    """C (len(funcs) x (n_grid + p)^2): coefficients of the (truncated)
    functions in the B-splines of the uniform grid with n_grid cells per
    axis, columns in lattice order (x fastest)."""
    top = mesh.cells(mesh.M)
    if n_grid % top:
        raise ValueError("the grid must refine the finest cells")
    extra = int(round(np.log2(n_grid // top)))
    nlev = mesh.M + 1 + extra
    R1 = [H.two_scale_1d("bspline", mesh.n0 * 2 ** k, p, lo, hi) for k in range(nlev - 1)]
    inside = [_inside(mesh, p, k) for k in range(mesh.M + 1)]
    rows = []
    for (m, ix, iy) in funcs:
        nm = mesh.cells(m)
        c = np.zeros((nm + p, nm + p))
        c[ix, iy] = 1.0
        for k in range(m + 1, nlev):
            c = R1[k - 1].T @ c @ R1[k - 1]          # the same function in level-k B-splines
            if truncate and k <= mesh.M:
                c[inside[k]] = 0.0                   # truncation with respect to level k
        rows.append(sp.csr_matrix(c.ravel(order="F")))
    C = sp.vstack(rows, format="csr")
    C.data[np.abs(C.data) < 1e-15] = 0.0
    C.eliminate_zeros()
    return C


@dataclass
class THBLevel:
    """One THB level in the form the Schwarz oracle reads (functions in
    compact order, elem_funcs over the active elements)."""
    mesh: HMesh
    p: int
    funcs: list                 # every hierarchical function (m, ix, iy)
    C_all: sp.csr_matrix        # their grid coefficients
    act: np.ndarray             # bool over funcs: active THB functions
    C: sp.csr_matrix            # rows of the active functions
    elems: list                 # active elements (m, ex, ey) of the mesh
    elem_on: np.ndarray         # bool over elems: element intersects Omega
    elem_funcs: dict = field(default_factory=dict)   # element -> compact function indices
    basis: str = "bspline"
    dim: int = 2

    @property
    def active(self):
        return np.arange(self.C.shape[0])


def build_level(mesh: HMesh, p: int, n_grid: int, grid_level, lo=0.0, hi=1.0) -> THBLevel:
    """THB level of `mesh` on the grid of the uniform system `grid_level`
    (an oracle.assemble.Level with n_grid cells per axis)."""
    funcs = thb_functions(mesh, p)
    C_all = coefficients(mesh, p, funcs, n_grid, lo, hi)
    nf1 = n_grid + p
    grid_act = np.zeros(nf1 * nf1, dtype=bool)
    grid_act[grid_level.active] = True
    ii = np.arange(nf1 * nf1)
    gx, gy = ii % nf1, ii // nf1
    boxf = (gx == 0) | (gx == nf1 - 1) | (gy == 0) | (gy == nf1 - 1)
    on_act = np.asarray((C_all[:, grid_act] != 0).sum(axis=1)).ravel() > 0
    on_box = np.asarray((C_all[:, boxf] != 0).sum(axis=1)).ravel() > 0
    act = on_act & ~on_box
    C = C_all[np.nonzero(act)[0]]
    # elements and the grid cells they cover
    elems = mesh.elements()
    owner = np.full((n_grid, n_grid), -1, dtype=np.int64)
    for e, (m, ex, ey) in enumerate(elems):
        s = n_grid // mesh.cells(m)
        owner[ex * s:(ex + 1) * s, ey * s:(ey + 1) * s] = e
    assert (owner >= 0).all()
    el_on = np.zeros(len(elems), dtype=bool)
    el_on[np.unique(owner[grid_level.active_el])] = True
    lev = THBLevel(mesh=mesh, p=p, funcs=funcs, C_all=C_all, act=act, C=C, elems=elems, elem_on=el_on)
    for i in range(C.shape[0]):
        ks = C.indices[C.indptr[i]:C.indptr[i + 1]]
        cells = np.zeros((n_grid, n_grid), dtype=bool)
        for k in ks:
            kx, ky = int(k % nf1), int(k // nf1)
            cells[_support(n_grid, p, kx), _support(n_grid, p, ky)] = True
        for e in np.unique(owner[cells]):
            if el_on[e]:
                lev.elem_funcs.setdefault(int(e), []).append(i)
    return lev


def embed(grid_level, A: sp.csr_matrix, nf1: int, d: int = 1) -> sp.csr_matrix:
    """A over the active grid functions (d components, component-major) ->
    over the whole (nf1^2) lattice, per component."""
    P = sp.csr_matrix((np.ones(len(grid_level.active)), (grid_level.active, np.arange(len(grid_level.active)))),
                      shape=(nf1 * nf1, len(grid_level.active)))
    P = sp.kron(sp.identity(d, format="csr"), P, format="csr")
    return (P @ A @ P.T).tocsr()


def per_component(X: sp.csr_matrix, d: int) -> sp.csr_matrix:
    """I_d kron X (one copy of X per displacement component)."""
    return X.tocsr() if d == 1 else sp.kron(sp.identity(d, format="csr"), X, format="csr")


def restriction(coarse: THBLevel, fine: THBLevel) -> sp.csr_matrix:
    """R with C_coarse = R C_fine over all functions (normal equations of the
    identity), restricted to active rows and columns."""
    Cf, Cc = fine.C_all, coarse.C_all
    G_ = (Cf @ Cf.T).tocsc()
    rhs = (Cf @ Cc.T).toarray()
    X = spla.splu(G_).solve(rhs)
    R = X.T
    R[np.abs(R) < 1e-12] = 0.0
    R = sp.csr_matrix(R)
    R = R[np.nonzero(coarse.act)[0]][:, np.nonzero(fine.act)[0]].tocsr()
    R.eliminate_zeros()
    R.sort_indices()
    return R


class THBHierarchy:
    """Levels 0 (coarsest) .. L-1 (finest); meshes by Algorithm alg:coarsen."""

    def __init__(self, w, orders=None):
        if w.dim != 2 or w.basis != "bspline":
            raise ValueError("THB levels are built for 2D B-splines")
        M, L, p = w.local_levels, w.levels, w.degree
        self.w = w
        self.n_grid = w.n * 2 ** M
        self.leaf = G.leaf_values(w, self.n_grid, w.depth)
        if getattr(w, "physics", "poisson") == "elasticity":
            from . import elasticity as EL
            self.grid = EL.assemble_elasticity(w, self.leaf, self.n_grid, w.depth, orders=orders)
            d = self.grid.ncomp
        else:
            self.grid = AS.assemble(w, self.leaf, self.n_grid, w.depth, orders=orders)
            d = 1
        self.ncomp = d
        nf1 = self.n_grid + p
        A_grid = embed(self.grid.level, self.grid.A, nf1, d)
        ng_act = len(self.grid.level.active)
        b_grid = np.zeros(d * nf1 * nf1)
        for c in range(d):
            b_grid[c * nf1 * nf1 + self.grid.level.active] = self.grid.b[c * ng_act:(c + 1) * ng_act]
        self.meshes = [None] * L
        self.meshes[L - 1] = refine_at_boundary(w.n, M, grid_volume_fractions(self.grid, self.n_grid))
        for k in range(L - 2, -1, -1):
            self.meshes[k] = coarsen(self.meshes[k + 1])
        self.levels = [build_level(m, p, self.n_grid, self.grid.level, w.box_lo, w.box_hi) for m in self.meshes]
        F = self.levels[L - 1]
        Cf = per_component(F.C, d)
        A = (Cf @ A_grid @ Cf.T).tocsr()
        self.A_direct = [(per_component(lv.C, d) @ A_grid @ per_component(lv.C, d).T).tocsr() for lv in self.levels]
        self.b = Cf @ b_grid
        # L2(Omega)^d Gram matrix of the THB functions (the grid's mass is
        # already one copy per component for elasticity)
        M_grid = embed(self.grid.level, self.grid.M, nf1, d)
        self.M = (Cf @ M_grid @ Cf.T).tocsr()
        self.A = [None] * L
        self.R = [None] * (L - 1)
        self.R_scalar = [None] * (L - 1)
        self.A[L - 1] = A
        for k in range(L - 2, -1, -1):
            self.R_scalar[k] = restriction(self.levels[k], self.levels[k + 1])
            self.R[k] = per_component(self.R_scalar[k], d)
            self.A[k] = (self.R[k] @ self.A[k + 1] @ self.R[k].T).tocsr()


class THBMultiplicativeSmoother(SW.MultiplicativeSmoother):
    """Multiplicative Schwarz (eq:multiplicativeSchwarz1) on a THB level.
    Reading: THB functions have no lattice position, so every block takes,
    in block order, the smallest colour that no block already coloured uses
    on a shared element (greedy from 0; same-colour blocks never share an
    element, as the subsection requires); kind "diagonal": one block per
    function (Gauss-Seidel, Remark rem:coarseGS)."""

    def __init__(self, A, lev, kind="schwarz"):
        if kind == "diagonal":
            blocks = [np.array([i], dtype=np.int64) for i in range(A.shape[0])]
            assoc = list(range(A.shape[0]))
        else:
            blocks, assoc = SW.select_blocks(lev)
        SW.Smoother.__init__(self, A, lev, blocks=blocks)
        self._order_blocks(A, lev, assoc, [None] * len(blocks), lambda b: b, 0)


class THBVectorMultiplicativeSmoother(SW.MultiplicativeSmoother):
    """Multiplicative Schwarz on a THB level of a vector problem: the scalar
    level's blocks repeated per component, coloured greedily in block order
    (blocks of different components that share an element are coupled by A,
    so they never share a colour); gamma is not used by this smoother."""

    def __init__(self, A, lev, d):
        from . import elasticity as EL
        blocks, vassoc = EL.vector_blocks(lev, d)
        N = lev.C.shape[0]
        self._d = d
        SW.Smoother.__init__(self, A, lev, blocks=blocks)
        self._order_blocks(A, lev, vassoc, [None] * len(blocks), lambda b: b % N, 0)

    def _gamma(self, lev, blocks):
        from . import elasticity as EL
        return 1.0 / EL.max_NK_vector(lev, blocks, self._d)


@dataclass
class THBProblem:
    w: object
    hier: THBHierarchy
    smoothers: list
    vcycle: MG.VCycle

    @property
    def A(self):
        return self.hier.A[-1]

    @property
    def b(self):
        return self.hier.b

    def solve(self, b=None, tol=1e-8, max_iter=1000):
        b = self.b if b is None else b
        return MG.pcg(self.A, b, self.vcycle.apply, tol=tol, max_iter=max_iter)


def build(w, orders=None) -> THBProblem:
    """The THB hierarchy with its smoothers (w.smoother on the finest level:
    "as" additive or "ms" multiplicative Schwarz over support-inclusion
    blocks; w.coarse_smoother on the others: "same", "jacobi" or "gs") and
    its V-cycle."""
    hier = THBHierarchy(w, orders)
    L = w.levels
    d = hier.ncomp
    sm = [None] * L
    for l in range(1, L):
        lev = hier.levels[l]
        fine = l == L - 1
        kind = w.smoother if (fine or w.coarse_smoother == "same") else w.coarse_smoother
        if d > 1:
            from . import elasticity as EL
            if kind == "as":
                sm[l] = EL.VectorSmoother(hier.A[l], lev, d)
            elif kind == "ms":
                sm[l] = THBVectorMultiplicativeSmoother(hier.A[l], lev, d)
            else:
                raise ValueError(f"vector THB levels: smoother {kind!r} not set up")
            continue
        if kind == "as":
            sm[l] = SW.Smoother(hier.A[l], lev)
        elif kind == "jacobi":
            sm[l] = SW.DiagonalSmoother(hier.A[l], lev)
        elif kind == "ms":
            sm[l] = THBMultiplicativeSmoother(hier.A[l], lev)
        elif kind == "gs":
            sm[l] = THBMultiplicativeSmoother(hier.A[l], lev, kind="diagonal")
        else:
            raise ValueError(f"THB levels: smoother {kind!r} not set up")
    vc = MG.VCycle(hier.A, hier.R, sm, nu_pre=w.nu, nu_post=w.nu, cycle=w.cycle)
    return THBProblem(w=w, hier=hier, smoothers=sm, vcycle=vc)
