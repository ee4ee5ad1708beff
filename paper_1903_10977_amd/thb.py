"""Locally refined problems for the solver library: truncated hierarchical
B-splines (THB) on hierarchically refined meshes (immersed formulation
section, Figure fig:THB) with the hierarchical coarsening of Algorithm
alg:coarsen (restriction subsection).

Host-side problem construction (not on the solve path): it produces, per
multigrid level, the operator, the restriction to the next coarser level,
the Schwarz blocks (support inclusion, smoothers subsection) and the element
incidence that the library's setup call takes.  THB levels carry no function
lattice: the library runs them as general sparse levels.

Construction (2D, degree p):
* meshes: dom[m] marks the level-m cells of Omega^m; the input mesh refines,
  for m = 0..M-1, the level-m cells of Omega^m holding a grid cell cut by the
  immersed boundary (volume fraction strictly between 0 and 1);
  coarser meshes follow Algorithm alg:coarsen (a coarse level-m element is
  refined when a fine element of local level > m lies inside it);
* basis: per level the B-splines whose support lies in Omega^m and meets an
  unrefined level-m cell; every function is carried as a row of grid
  coefficients (the B-splines of the uniform grid of the finest cells),
  computed for all functions of a level at once with sparse refinement
  matrices (Boehm knot insertion of the span midpoints) and the truncation
  masks of the finer levels;
* integrals: the uniform grid system of the native generator (cut-cell
  quadrature), A = C A_grid C^T and b = C b_grid; active functions touch an
  active grid function and have no trace on the box faces (strong u = 0);
* restriction: rows of R with C_coarse = R C_fine; a coarse function that is
  an untruncated B-spline whose two-scale children are all untruncated fine
  functions takes the two-scale coefficients, any other one a least-squares
  solve (normal equations, else an orthogonal solve) over the fine functions
  that share grid coefficients with it, accepted only when it reproduces the
  coarse row to 1e-12;
* blocks: E(k) = elements meeting Omega on which phi_k is non-zero; block of
  phi_j = {phi_k : E(k) within E(j)}; coarse operators R A R^T.
Numbering on every level: by level m, then lattice index of the level (x
fastest); elements likewise.

Linear elasticity (eq:weakMulti / eq:operatorsMulti with penalty Dirichlet
conditions, the physics of the paper's THB example): every displacement
component takes the same THB functions, DOF c N + i = component c of
function i; the grid operator is the generator's vector one, the THB
operator (I_d kron C) A_grid (I_d kron C)^T, R_l = I_d kron R_l,scalar, the
blocks those of the scalar level repeated per component, and every element
lists the DOFs of all components (the library runs such a level as a plain
general sparse level).
"""
from __future__ import annotations

import dataclasses
import time
from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp
from threadpoolctl import threadpool_limits

from . import generator as GEN

CUT_TOL = 1e-12


@dataclass
class Mesh:
    n0: int
    M: int
    dom: list   # dom[m]: bool (n0 2^m,)*2 indexed [ix, iy]

    def cells(self, m):
        return self.n0 << m

    def unrefined(self, m):
        if m == self.M:
            return self.dom[m]
        return self.dom[m] & ~self.dom[m + 1][::2, ::2]


def _up(mask):
    return mask.repeat(2, axis=0).repeat(2, axis=1)


def boundary_mesh(n0, M, eta_grid):
    """Input mesh: level-m cells of Omega^m holding a cut grid cell (volume
    fraction strictly between 0 and 1, to 1e-12) are refined.  eta_grid:
    grid-cell volume fractions [ix, iy] on the n0 2^M grid."""
    n_grid = n0 << M
    cut = (eta_grid > CUT_TOL) & (eta_grid < 1.0 - CUT_TOL)
    dom = [np.ones((n0, n0), dtype=bool)]
    for m in range(M):
        nm = n0 << m
        s = n_grid // nm
        holds = cut.reshape(nm, s, nm, s).any(axis=(1, 3))
        dom.append(_up(dom[m] & holds))
    return Mesh(n0, M, dom)


def coarsen(fine: Mesh) -> Mesh:
    """Algorithm alg:coarsen: coarse level-m elements (m < M) holding a fine
    level-(m+1) cell of Omega_h^{m+1} are refined."""
    n0c = fine.n0 // 2
    dom = [np.ones((n0c, n0c), dtype=bool)]
    for m in range(fine.M):
        ncm = n0c << m
        holds = fine.dom[m + 1].reshape(ncm, 4, ncm, 4).any(axis=(1, 3))
        dom.append(_up(dom[m] & holds))
    return Mesh(n0c, fine.M, dom)


_T_CACHE = {}


def insertion_matrix(n_c: int, p: int) -> np.ndarray:
    """T (n_f x n_c functions, n_f = 2 n_c + p) with fine coefficients = T
    coarse coefficients, by Boehm insertion of the midpoint of every span of
    the open uniform knot vector on [0, 1] (one knot at a time: the new
    coefficient i is (1 - a_i) P_{i-1} + a_i P_i inside the p affected
    positions, a copy elsewhere)."""
    key = (n_c, p)
    if key in _T_CACHE:
        return _T_CACHE[key]
    t = np.concatenate([np.zeros(p), np.arange(n_c + 1) / n_c, np.ones(p)])
    T = np.eye(n_c + p)
    for e in range(n_c):
        x = (e + 0.5) / n_c
        k = int(np.searchsorted(t, x, side="right")) - 1      # t[k] <= x < t[k+1]
        n = T.shape[0]
        Tn = np.empty((n + 1, T.shape[1]))
        lo = max(k - p + 1, 0)
        Tn[:lo] = T[:lo]
        Tn[k + 1:] = T[k:]
        for i in range(lo, k + 1):
            a = (x - t[i]) / (t[i + p] - t[i])
            Tn[i] = a * T[i] + ((1.0 - a) * T[i - 1] if i >= 1 else 0.0)
        T = Tn
        t = np.insert(t, k + 1, x)
    T[np.abs(T) < 1e-15] = 0.0
    _T_CACHE[key] = T
    return T


def _supports_in(mask, p):
    """Per level function (x fastest): is its support inside `mask` (cells)?
    Any: does it touch a True cell?"""
    n = mask.shape[0]
    f = n + p
    cnt = np.zeros((f, f), dtype=np.int64)
    tot = np.zeros((f, f), dtype=np.int64)
    m = mask.astype(np.int64)
    for dx in range(p + 1):
        for dy in range(p + 1):
            # function (ix, iy) touches cells (ix - dx, iy - dy)
            cnt[dx:dx + n, dy:dy + n] += m
            tot[dx:dx + n, dy:dy + n] += 1
    return cnt == tot, cnt > 0


@dataclass
class Space:
    mesh: Mesh
    funcs: np.ndarray          # (n, 3): m, ix, iy
    C: sp.csr_matrix           # grid coefficients of every function
    untrunc: np.ndarray        # bool: no coefficient removed by truncation


def build_space(mesh: Mesh, p: int, n_grid: int) -> Space:
    """THB functions of `mesh` with their grid coefficients."""
    top = mesh.cells(mesh.M)
    extra = int(round(np.log2(n_grid // top)))
    nlev = mesh.M + 1 + extra
    Tlev = []
    for k in range(nlev - 1):
        T1 = sp.csr_matrix(insertion_matrix(mesh.n0 << k, p))
        Tlev.append(sp.kron(T1, T1, format="csr"))        # x fastest on both sides
    keep = []
    for k in range(mesh.M + 1):
        inside, _ = _supports_in(mesh.dom[k], p)
        keep.append(sp.diags((~inside).ravel(order="F").astype(np.float64)))
    rows, funcs, untr = [], [], []
    for m in range(mesh.M + 1):
        inside, _ = _supports_in(mesh.dom[m], p)
        _, touches = _supports_in(mesh.unrefined(m), p)
        sel = (inside & touches).ravel(order="F")
        idx = np.nonzero(sel)[0]
        if len(idx) == 0:
            continue
        nf = (mesh.n0 << m) + p
        X = sp.csr_matrix((np.ones(len(idx)), (np.arange(len(idx)), idx)), shape=(len(idx), nf * nf))
        Xu = X
        for k in range(m + 1, nlev):
            X = (X @ Tlev[k - 1].T).tocsr()
            Xu = (Xu @ Tlev[k - 1].T).tocsr()
            if k <= mesh.M:
                X = (X @ keep[k]).tocsr()
        X.eliminate_zeros()
        d = abs(X - Xu)
        untr.append(np.asarray(d.max(axis=1).todense()).ravel() == 0.0)
        rows.append(X)
        funcs.append(np.stack([np.full(len(idx), m), idx % nf, idx // nf], axis=1))
    C = sp.vstack(rows, format="csr")
    C.sort_indices()
    return Space(mesh, np.concatenate(funcs), C, np.concatenate(untr))


def _dense_rows(M: sp.csr_matrix, rows, cols) -> np.ndarray:
    """M[rows][:, cols] as a dense array (cols sorted, holding every column
    the rows use)."""
    out = np.zeros((len(rows), len(cols)))
    for r, i in enumerate(rows):
        a, b = M.indptr[i], M.indptr[i + 1]
        out[r, np.searchsorted(cols, M.indices[a:b])] = M.data[a:b]
    return out


def _restriction_rows(cs: Space, fs: Space, p: int) -> sp.csr_matrix:
    """R (all coarse x all fine functions) with cs.C = R fs.C."""
    nc, nfine = cs.C.shape[0], fs.C.shape[0]
    rr, rc, rv = [], [], []
    fast = np.zeros(nc, dtype=bool)
    # two-scale rows: untruncated coarse B-splines of level m whose children
    # (level-m fine B-splines) are all untruncated fine functions
    for m in range(cs.mesh.M + 1):
        sel = np.nonzero((cs.funcs[:, 0] == m) & cs.untrunc)[0]
        if len(sel) == 0:
            continue
        n_c = cs.mesh.cells(m)
        T = insertion_matrix(n_c, p)                      # (2 n_c + p) x (n_c + p)
        nf1 = 2 * n_c + p
        fid = np.full((nf1, nf1), -1, dtype=np.int64)     # fine level-m function id by (ix, iy)
        fm = np.nonzero(fs.funcs[:, 0] == m)[0]
        fid[fs.funcs[fm, 1], fs.funcs[fm, 2]] = fm
        # children of every 1D coarse index (p + 2 at most), -1 padded
        ch = np.full((n_c + p, p + 2), -1, dtype=np.int64)
        co = np.zeros((n_c + p, p + 2))
        for i in range(n_c + p):
            nz = np.nonzero(T[:, i])[0]
            ch[i, :len(nz)] = nz
            co[i, :len(nz)] = T[nz, i]
        ix, iy = cs.funcs[sel, 1], cs.funcs[sel, 2]
        ax, ay = ch[ix][:, :, None], ch[iy][:, None, :]                 # (N, p+2, 1), (N, 1, p+2)
        cv = (co[ix][:, :, None] * co[iy][:, None, :]).reshape(len(sel), -1)
        valid = ((ax >= 0) & (ay >= 0)).reshape(len(sel), -1)
        kid = np.where(valid, fid[np.maximum(ax, 0), np.maximum(ay, 0)].reshape(len(sel), -1), -1)
        ok_kid = ~valid | ((kid >= 0) & fs.untrunc[np.maximum(kid, 0)])
        good = ok_kid.all(axis=1)
        for q in np.nonzero(good)[0]:
            v = valid[q]
            rr.append(np.full(int(v.sum()), sel[q]))
            rc.append(kid[q][v])
            rv.append(cv[q][v])
        fast[sel[good]] = True
    share = (cs.C @ fs.C.T).tocsr()          # coarse x fine: share a grid coefficient
    FT = fs.C.T.tocsr()                      # grid -> fine functions
    with threadpool_limits(1):               # many tiny dense solves: no BLAS threads
        _solve_rows(cs, fs, np.nonzero(~fast)[0], share, FT, rr, rc, rv)
    if not rr:
        return sp.csr_matrix((nc, nfine))
    return sp.csr_matrix((np.concatenate(rv), (np.concatenate(rr), np.concatenate(rc))), shape=(nc, nfine))


def _solve_rows(cs, fs, rows, share, FT, rr, rc, rv):
    for j in rows:
        cand = share.indices[share.indptr[j]:share.indptr[j + 1]]
        tcols = cs.C.indices[cs.C.indptr[j]:cs.C.indptr[j + 1]]
        tvals = cs.C.data[cs.C.indptr[j]:cs.C.indptr[j + 1]]
        done = False
        for _ in range(3):
            cols = np.unique(np.concatenate([fs.C.indices[fs.C.indptr[k]:fs.C.indptr[k + 1]] for k in cand]
                                            + [tcols]))
            Ms = _dense_rows(fs.C, cand, cols)
            tv = np.zeros(len(cols))
            tv[np.searchsorted(cols, tcols)] = tvals
            # normal equations of the (consistent) system Ms^T x = tv: the
            # grid-coefficient rows of neighbouring functions are far from
            # dependent, and the exactness check below guards the result
            try:
                x = np.linalg.solve(Ms @ Ms.T, Ms @ tv)
            except np.linalg.LinAlgError:
                x, *_ = np.linalg.lstsq(Ms.T, tv, rcond=None)
            if np.abs(Ms.T @ x - tv).max() > 1e-12:
                x, *_ = np.linalg.lstsq(Ms.T, tv, rcond=None)
            if np.abs(Ms.T @ x - tv).max() <= 1e-12:
                x[np.abs(x) < 1e-13] = 0.0
                nz = x != 0.0
                rr.append(np.full(int(nz.sum()), j))
                rc.append(np.asarray(cand)[nz])
                rv.append(x[nz])
                done = True
                break
            # widen: fine functions sharing a grid coefficient with the candidates
            cand = np.unique(FT[cols].indices)
        if not done:
            raise RuntimeError(f"coarse THB function {j} is not in the fine THB space")


@dataclass
class THBLevelData:
    space: Space
    act: np.ndarray            # bool over functions
    elems: np.ndarray          # (ne, 3): m, ex, ey of the active elements
    elem_on: np.ndarray        # bool: element meets Omega
    F: sp.csr_matrix           # active functions x elements meeting Omega (incidence)


def level_data(space: Space, p: int, n_grid: int, grid_active_funcs, grid_active_cells) -> THBLevelData:
    nf1 = n_grid + p
    mesh = space.mesh
    gact = np.zeros(nf1 * nf1, dtype=bool)
    gact[grid_active_funcs] = True
    g = np.arange(nf1 * nf1)
    gx, gy = g % nf1, g // nf1
    box = (gx == 0) | (gx == nf1 - 1) | (gy == 0) | (gy == nf1 - 1)
    C = space.C
    touch_act = np.asarray(C[:, gact].getnnz(axis=1)).ravel() > 0
    touch_box = np.asarray(C[:, box].getnnz(axis=1)).ravel() > 0
    act = touch_act & ~touch_box
    # active elements and the element owning every grid cell
    el, owner = [], np.full((n_grid, n_grid), -1, dtype=np.int64)
    for m in range(mesh.M + 1):
        u = mesh.unrefined(m)
        ey, ex = np.nonzero(u.T)          # by ey, then ex
        base = len(el)
        el.extend(zip([m] * len(ex), ex.tolist(), ey.tolist()))
        s = n_grid // mesh.cells(m)
        ids = np.full(u.shape, -1, dtype=np.int64)
        ids[ex, ey] = base + np.arange(len(ex))
        big = ids.repeat(s, axis=0).repeat(s, axis=1)
        owner = np.where(big >= 0, big, owner)
    elems = np.array(el, dtype=np.int64)
    on = np.zeros(len(elems), dtype=bool)
    on[np.unique(owner[grid_active_cells])] = True
    # grid cells touched by each active function: grid function k covers
    # cells (kx - p .. kx, ky - p .. ky); F = pattern(C) x (grid function ->
    # elements meeting Omega under its support)
    g2e_r, g2e_c = [], []
    for dx in range(p + 1):
        for dy in range(p + 1):
            cx, cy = gx - dx, gy - dy
            ok = (cx >= 0) & (cx < n_grid) & (cy >= 0) & (cy < n_grid)
            e = owner[cx[ok], cy[ok]]
            keep = on[e]
            g2e_r.append(g[ok][keep])
            g2e_c.append(e[keep])
    G2E = sp.csr_matrix((np.ones(sum(len(r) for r in g2e_r)), (np.concatenate(g2e_r), np.concatenate(g2e_c))),
                        shape=(nf1 * nf1, len(elems)))
    Ca = C[np.nonzero(act)[0]].copy()
    Ca.data[:] = 1.0
    F = (Ca @ G2E).tocsr()
    F.data[:] = 1.0
    F.sort_indices()
    return THBLevelData(space, act, elems, on, F)


def inclusion_blocks(F: sp.csr_matrix):
    """Block of every function j: {k : E(k) within E(j)} (ascending k)."""
    F = F.tocsr()
    sizes = np.asarray(F.sum(axis=1)).ravel()
    O = (F @ F.T).tocsr()                    # |E(j) cap E(k)|
    ptr, idx = [0], []
    for j in range(F.shape[0]):
        ks = O.indices[O.indptr[j]:O.indptr[j + 1]]
        ov = O.data[O.indptr[j]:O.indptr[j + 1]]
        sel = np.sort(ks[ov == sizes[ks]])
        idx.extend(sel.tolist())
        ptr.append(len(idx))
    return np.array(ptr, dtype=np.int32), np.array(idx, dtype=np.int32)


def _per_component(X: sp.csr_matrix, d: int) -> sp.csr_matrix:
    """I_d kron X."""
    return X.tocsr() if d == 1 else sp.kron(sp.identity(d, format="csr"), X, format="csr")


def generate(w, nthreads: int = 0):
    """GeneratedProblem of a THB workload (w.local_levels >= 0, 2D
    B-splines, Poisson or linear elasticity); levels 0 = coarsest, as the
    uniform generator."""
    physics = getattr(w, "physics", "poisson")
    if w.dim != 2 or w.basis != "bspline" or physics not in ("poisson", "elasticity"):
        raise ValueError("THB problems: 2D B-spline workloads (Poisson or linear elasticity)")
    if physics == "elasticity" and getattr(w, "coarse_smoother", "same") != "same":
        raise ValueError("vector THB problems: additive or multiplicative Schwarz on every level")
    t0 = time.perf_counter()
    M, L, p = w.local_levels, w.levels, w.degree
    n_grid = w.n << M
    wg = dataclasses.replace(w, n=n_grid, levels=1, local_levels=0)
    gp = GEN.generate(wg, nthreads=nthreads)
    grid = gp.levels[0]
    d = int(getattr(grid, "ncomp", 1))
    nf1 = n_grid + p
    gl = np.asarray(grid.dof_to_lattice, dtype=np.int64)
    eta = np.asarray(grid.eta).reshape(n_grid, n_grid, order="F")
    gcell = np.zeros((n_grid, n_grid), dtype=bool)
    eid = np.asarray(grid.elem_id, dtype=np.int64)
    gcell[eid % n_grid, eid // n_grid] = True
    P = sp.csr_matrix((np.ones(len(gl)), (gl, np.arange(len(gl)))), shape=(nf1 * nf1, len(gl)))
    P = _per_component(P, d)
    A_grid = (P @ grid.A @ P.T).tocsr()
    meshes: List[Mesh] = [None] * L
    meshes[L - 1] = boundary_mesh(w.n, M, eta)
    for k in range(L - 2, -1, -1):
        meshes[k] = coarsen(meshes[k + 1])
    spaces = [build_space(ms, p, n_grid) for ms in meshes]
    data = [level_data(s, p, n_grid, gl, gcell) for s in spaces]
    fine = data[L - 1]
    Cf = _per_component(fine.space.C[np.nonzero(fine.act)[0]], d)
    A = (Cf @ A_grid @ Cf.T).tocsr()
    A.sort_indices()
    levels = [None] * L
    Rs = [None] * L
    for k in range(L - 1, 0, -1):
        Rk = _restriction_rows(spaces[k - 1], spaces[k], p)
        Rk = Rk[np.nonzero(data[k - 1].act)[0]][:, np.nonzero(data[k].act)[0]].tocsr()
        Rk.eliminate_zeros()
        Rk = _per_component(Rk, d)
        Rk.sort_indices()
        Rs[k] = Rk
    As = [None] * L
    As[L - 1] = A
    for k in range(L - 1, 0, -1):
        Ac = (Rs[k] @ As[k] @ Rs[k].T).tocsr()
        Ac.sort_indices()
        As[k - 1] = Ac
    for l in range(L):
        dl = data[l]
        n = int(dl.act.sum())
        bp = bi = ba = None
        if l > 0:
            bp, bi = inclusion_blocks(dl.F)
            if 0 < l < L - 1 and getattr(w, "coarse_smoother", "same") in ("jacobi", "gs"):
                bp = np.arange(n + 1, dtype=np.int32)
                bi = np.arange(n, dtype=np.int32)
            # the scalar blocks once per component (component c shifted by c n)
            bp = np.concatenate([bp[:-1] + c * bp[-1] for c in range(d)] + [[d * bp[-1]]]).astype(np.int32)
            bi = np.concatenate([bi + c * n for c in range(d)]).astype(np.int32)
            ba = np.arange(d * n, dtype=np.int32)
        Ft = dl.F.T.tocsr()
        keep_el = np.nonzero(dl.elem_on)[0]
        Ft = Ft[keep_el]
        Ft = sp.hstack([Ft] * d, format="csr")   # every element lists the DOFs of all components
        Ft.sort_indices()
        levels[l] = GEN.GenLevel(n_elements=len(keep_el), lattice=(d * n,), dof_to_lattice=None, A=As[l], R=Rs[l],
                                 block_ptr=bp, block_idx=bi, block_assoc=ba, n_cut=0, eta_min=0.0, eta=None,
                                 elem_ptr=Ft.indptr.astype(np.int32), elem_idx=Ft.indices.astype(np.int32),
                                 elem_id=None, two_scale=None, block_colour=None)
    b = Cf @ (P @ np.asarray(gp.b))
    return GEN.GeneratedProblem(workload=w, levels=levels, b=b, M=None, seconds=time.perf_counter() - t0)


def with_coarse_diagonal(problem, kind: str = "jacobi"):
    """The same problem with one block per function on the levels between
    the coarsest and the finest (Remark rem:coarseGS: Jacobi, or
    Gauss-Seidel with kind "gs")."""
    levels = list(problem.levels)
    L = len(levels)
    for l in range(1, L - 1):
        n = levels[l].A.shape[0]
        levels[l] = dataclasses.replace(levels[l], block_ptr=np.arange(n + 1, dtype=np.int32),
                                        block_idx=np.arange(n, dtype=np.int32),
                                        block_assoc=np.arange(n, dtype=np.int32))
    w = dataclasses.replace(problem.workload, coarse_smoother=kind)
    return dataclasses.replace(problem, workload=w, levels=levels)
