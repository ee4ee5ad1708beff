"""Assembly of the immersed system (oracle; test infrastructure only).

eq:systemMulti: A x = b with A_ij = a_h(phi_i, phi_j) and b_i = b_h(phi_i).
The scalar analogue of eq:weakMulti / eq:operatorsMulti is used (the
benchmark problems are Poisson problems):

    a_h(v, u) = int_Omega grad v . grad u  [+ int_Gamma beta v u  (penalty)]
    b_h(v)    = int_Omega f v  + int_Gamma_N g v

with the penalty parameter beta = factor / h of the finest grid (the paper's
penalty method, parameter 2/h in its spectral study).  With the box Dirichlet
condition, functions with a non-zero trace on the box faces are removed
(strong u = 0) and the immersed boundary carries natural (Neumann) data.

V_h is spanned by the functions supported on Omega (immersed formulation
section): a lattice function is active when it is non-zero on at least one
active element, an element being active when any of its leaf vertices lies
in Omega.  The structural sparsity pattern couples two active functions that
share an active element; the pattern keeps entries whose value happens to be
zero.  Compact DOF numbering = ascending lattice index, x fastest.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import basis as B
from . import geometry as G
from . import quadrature as Q


@dataclass
class Level:
    """One discretization level (n elements per axis)."""
    dim: int
    p: int
    basis: str
    n: int
    depth: int            # bisection depth of this level's elements on the shared leaf lattice
    lo: float
    hi: float
    active_el: np.ndarray  # bool, shape (n,)*dim, indexed [e_x, e_y(, e_z)]
    active: np.ndarray     # sorted lattice indices of active functions
    nf1: int               # functions per axis
    elem_funcs: dict = field(default_factory=dict)  # element linear index -> lattice indices

    @property
    def h(self):
        return (self.hi - self.lo) / self.n

    @property
    def lattice_shape(self):
        return (self.nf1,) * self.dim

    def lat_to_multi(self, L):
        out = []
        for _ in range(self.dim):
            out.append(L % self.nf1)
            L = L // self.nf1
        return tuple(out)

    def multi_to_lat(self, m):
        L = 0
        for a in reversed(range(self.dim)):
            L = L * self.nf1 + m[a]
        return L


def element_lin(e, n):
    L = 0
    for a in reversed(range(len(e))):
        L = L * n + e[a]
    return L


def local_funcs(lev: Level, e):
    """Lattice indices of the (p+1)^d functions non-zero on element e,
    ordered with the x offset fastest."""
    first = [B.first_func_1d(lev.basis, lev.p, e[a]) for a in range(lev.dim)]
    out = []
    for off in itertools.product(range(lev.p + 1), repeat=lev.dim):
        m = [first[a] + off[lev.dim - 1 - a] for a in range(lev.dim)]
        out.append(lev.multi_to_lat(m))
    return out


def is_dirichlet(lev: Level, L: int) -> bool:
    m = lev.lat_to_multi(L)
    return any(mi == 0 or mi == lev.nf1 - 1 for mi in m)


def make_level(w, leaf, n, depth, strong_box: bool) -> Level:
    act_el = G.active_elements(leaf, n, depth)
    nf1 = B.nfuncs_1d(w.basis, n, w.degree)
    lev = Level(dim=w.dim, p=w.degree, basis=w.basis, n=n, depth=depth, lo=w.box_lo, hi=w.box_hi,
                active_el=act_el, active=np.zeros(0, dtype=np.int64), nf1=nf1)
    supported = set()
    for e in zip(*np.nonzero(act_el)):
        fl = local_funcs(lev, e)
        lev.elem_funcs[element_lin(e, n)] = fl
        supported.update(fl)
    act = sorted(L for L in supported if not (strong_box and is_dirichlet(lev, L)))
    lev.active = np.array(act, dtype=np.int64)
    return lev


def tensor_eval(lev: Level, e, pts):
    """Values (nloc, nq) and gradients (nloc, nq, d) of the local functions of
    element e at points pts (nq, d); local order as in local_funcs."""
    d = lev.dim
    vals1, ders1 = [], []
    for a in range(d):
        v, dv = B.eval_1d(lev.basis, lev.n, lev.p, int(e[a]), pts[:, a], lev.lo, lev.hi)
        vals1.append(v)
        ders1.append(dv)
    nq = pts.shape[0]
    nloc = (lev.p + 1) ** d
    V = np.zeros((nloc, nq))
    Gr = np.zeros((nloc, nq, d))
    for k, off in enumerate(itertools.product(range(lev.p + 1), repeat=d)):
        o = [off[d - 1 - a] for a in range(d)]
        v = np.ones(nq)
        for a in range(d):
            v = v * vals1[a][o[a]]
        V[k] = v
        for c in range(d):
            g = np.ones(nq)
            for a in range(d):
                g = g * (ders1[a][o[a]] if a == c else vals1[a][o[a]])
            Gr[k, :, c] = g
    return V, Gr


def _stiffness(vw, Gr):
    """K_ab = sum_q vw_q grad phi_a(x_q) . grad phi_b(x_q), as one matrix
    product over the (point, direction) pairs."""
    a, nq, d = Gr.shape
    G = Gr.reshape(a, nq * d)
    return (G * np.repeat(vw, d)) @ G.T


def manufactured(pts):
    """u* = prod_a sin(2 pi x_a); returns (u*, f = -lap u*, grad u*)."""
    d = pts.shape[1]
    s = np.sin(2 * np.pi * pts)
    c = np.cos(2 * np.pi * pts)
    u = np.prod(s, axis=1)
    f = d * (2 * np.pi) ** 2 * u
    g = np.zeros_like(pts)
    for a in range(d):
        t = 2 * np.pi * c[:, a]
        for b in range(d):
            if b != a:
                t = t * s[:, b]
        g[:, a] = t
    return u, f, g


@dataclass
class System:
    level: Level
    A: sp.csr_matrix
    b: np.ndarray
    M: sp.csr_matrix
    vol_frac: dict           # element linear index -> |K cap Omega_h| / |K|
    bnd_measure: dict        # element linear index -> |Gamma_h cap K|
    omega_measure: float


def assemble(w, leaf, n, depth, orders=None, with_rhs=True) -> System:
    """Assemble A, b and the mass matrix M on the level with n elements per
    axis, whose elements are bisected `depth` times on the shared leaf lattice."""
    strong = w.bc == "box_dirichlet"
    lev = make_level(w, leaf, n, depth, strong)
    d, p = w.dim, w.degree
    qc, qs, qb = orders if orders is not None else Q.default_orders(d, p)
    beta = w.penalty_factor / lev.h if w.bc == "penalty" else 0.0
    pos = {int(L): i for i, L in enumerate(lev.active)}
    rows, cols, vA, vM = [], [], [], []
    b = np.zeros(len(lev.active))
    vol_frac, bnd_meas = {}, {}
    omega = 0.0
    for e in zip(*np.nonzero(lev.active_el)):
        el = element_lin(e, n)
        fl = lev.elem_funcs[el]
        vp, vw, bp, bw, bn = Q.element_quadrature(leaf, e, depth, lev.lo, lev.h, qc, qs, qb)
        vol_frac[el] = float(vw.sum()) / lev.h ** d
        bnd_meas[el] = float(bw.sum())
        omega += float(vw.sum())
        V, Gr = tensor_eval(lev, e, vp)
        K = _stiffness(vw, Gr)
        Ml = (V * vw) @ V.T
        fb = np.zeros(len(fl))
        if with_rhs:
            if w.rhs == "one":
                fb += V @ vw
            elif w.rhs == "manufactured":
                _, f, _ = manufactured(vp)
                fb += V @ (vw * f)
        if len(bw):
            Vb, _ = tensor_eval(lev, e, bp)
            if beta > 0.0:
                K = K + beta * np.einsum("q,aq,bq->ab", bw, Vb, Vb)
            if with_rhs and w.rhs == "manufactured" and w.bc == "box_dirichlet":
                _, _, gu = manufactured(bp)
                gn = np.sum(gu * bn, axis=1)
                fb += Vb @ (bw * gn)
        # exact symmetry: keep the upper triangle and mirror it
        K = np.triu(K) + np.triu(K, 1).T
        Ml = np.triu(Ml) + np.triu(Ml, 1).T
        loc = [pos.get(L, -1) for L in fl]
        for a, ia in enumerate(loc):
            if ia < 0:
                continue
            b[ia] += fb[a]
            for c, ic in enumerate(loc):
                if ic < 0:
                    continue
                rows.append(ia)
                cols.append(ic)
                vA.append(K[a, c])
                vM.append(Ml[a, c])
    N = len(lev.active)
    A = _mirror(sp.coo_matrix((vA, (rows, cols)), shape=(N, N)).tocsr())
    M = _mirror(sp.coo_matrix((vM, (rows, cols)), shape=(N, N)).tocsr())
    return System(level=lev, A=A, b=b, M=M, vol_frac=vol_frac, bnd_measure=bnd_meas, omega_measure=omega)


def assemble_rows(w, leaf, n, depth, rows_lattice, orders=None):
    """Rows of A (and entries of b) for the active functions with the given
    lattice indices, from exactly the element contributions `assemble` adds
    for them, in the same element order: the same numbers as the full
    assembly, for problems too large to assemble whole.

    Returns (level, {row L: {column L': A value}}, {row L: b value})."""
    strong = w.bc == "box_dirichlet"
    lev = make_level(w, leaf, n, depth, strong)
    d, p = w.dim, w.degree
    qc, qs, qb = orders if orders is not None else Q.default_orders(d, p)
    beta = w.penalty_factor / lev.h if w.bc == "penalty" else 0.0
    active = set(int(L) for L in lev.active)
    want = set(int(L) for L in rows_lattice)
    if not want <= active:
        raise ValueError("requested rows must be active functions")
    # elements whose local functions include a requested row, ascending
    els = sorted(el for el, fl in lev.elem_funcs.items() if want.intersection(int(L) for L in fl))
    A = {L: {} for L in want}
    b = {L: 0.0 for L in want}
    for el in els:
        e = tuple(int(v) for v in np.unravel_index(el, (n,) * d, order="F"))
        fl = lev.elem_funcs[el]
        vp, vw, bp, bw, bn = Q.element_quadrature(leaf, e, depth, lev.lo, lev.h, qc, qs, qb)
        V, Gr = tensor_eval(lev, e, vp)
        K = _stiffness(vw, Gr)
        fb = np.zeros(len(fl))
        if w.rhs == "one":
            fb += V @ vw
        elif w.rhs == "manufactured":
            _, f, _ = manufactured(vp)
            fb += V @ (vw * f)
        if len(bw):
            Vb, _ = tensor_eval(lev, e, bp)
            if beta > 0.0:
                K = K + beta * np.einsum("q,aq,bq->ab", bw, Vb, Vb)
            if w.rhs == "manufactured" and w.bc == "box_dirichlet":
                _, _, gu = manufactured(bp)
                fb += Vb @ (bw * np.sum(gu * bn, axis=1))
        K = np.triu(K) + np.triu(K, 1).T
        for a, La in enumerate(fl):
            La = int(La)
            if La not in want:
                continue
            b[La] += fb[a]
            for c, Lc in enumerate(fl):
                Lc = int(Lc)
                if Lc in active:
                    A[La][Lc] = A[La].get(Lc, 0.0) + K[a, c]
    return lev, A, b


def _mirror(A: sp.csr_matrix) -> sp.csr_matrix:
    """Exactly symmetric copy: upper triangle (with diagonal) mirrored.  The
    structural pattern is kept (explicit zeros included)."""
    A = A.tocoo()
    up = A.row <= A.col
    r, c, v = A.row[up], A.col[up], A.data[up]
    off = r < c
    rr = np.concatenate([r, c[off]])
    cc = np.concatenate([c, r[off]])
    vv = np.concatenate([v, v[off]])
    out = sp.csr_matrix((vv, (rr, cc)), shape=A.shape)
    out.sort_indices()
    return out


def structural_pattern(lev: Level) -> sp.csr_matrix:
    """0/1 matrix of the structural pattern: active i, j sharing an active element."""
    pos = {int(L): i for i, L in enumerate(lev.active)}
    rows, cols = [], []
    for el, fl in lev.elem_funcs.items():
        loc = [pos[L] for L in fl if L in pos]
        for a in loc:
            for c in loc:
                rows.append(a)
                cols.append(c)
    N = len(lev.active)
    P = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N)).tocsr()
    P.data[:] = 1.0
    P.sort_indices()
    return P


def load_vector(w, leaf, n, depth, f=None, g=None, orders=None, strong_box=None):
    """v_i = int_Omega f phi_i + int_Gamma g(x, n) phi_i on the given level.

    f(points) and g(points, normals) are callables (either may be None)."""
    strong = (w.bc == "box_dirichlet") if strong_box is None else strong_box
    lev = make_level(w, leaf, n, depth, strong)
    qc, qs, qb = orders if orders is not None else Q.default_orders(w.dim, w.degree)
    pos = {int(L): i for i, L in enumerate(lev.active)}
    v = np.zeros(len(lev.active))
    for e in zip(*np.nonzero(lev.active_el)):
        fl = lev.elem_funcs[element_lin(e, n)]
        vp, vw, bp, bw, bn = Q.element_quadrature(leaf, e, depth, lev.lo, lev.h, qc, qs, qb)
        loc = np.zeros(len(fl))
        if f is not None and len(vw):
            V, _ = tensor_eval(lev, e, vp)
            loc += V @ (vw * f(vp))
        if g is not None and len(bw):
            Vb, _ = tensor_eval(lev, e, bp)
            loc += Vb @ (bw * g(bp, bn))
        for a, L in enumerate(fl):
            i = pos.get(L)
            if i is not None:
                v[i] += loc[a]
    return lev, v


def active_function_mask(active_el: np.ndarray, basis: str, p: int) -> np.ndarray:
    """Vectorised activation rule: lattice functions non-zero on at least one
    active element (no boundary removal).  Same rule as make_level, written
    with array shifts so that paper-size grids can be counted."""
    d = active_el.ndim
    n = active_el.shape[0]
    if basis == "bspline":
        out = np.zeros((n + p,) * d, dtype=bool)
        for off in itertools.product(range(p + 1), repeat=d):
            sl = tuple(slice(o, o + n) for o in off)
            out[sl] |= active_el
        return out
    out = np.zeros((p * n + 1,) * d, dtype=bool)
    for off in itertools.product(range(p + 1), repeat=d):
        sl = tuple(slice(o, o + p * n, p) for o in off)
        out[sl] |= active_el
    return out
