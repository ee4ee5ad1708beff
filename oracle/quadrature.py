"""Cut-cell quadrature (oracle; test infrastructure only).

Figure 1's caption (immersed formulation section): cut elements are bisected
recursively until a maximum integration depth is reached, the resulting cut
sub-cells are triangulated into integration subcells, standard Gauss points
are placed on the subcells for volume integrals, and boundary integrals use
Gauss quadrature on the approximate boundary formed by the subcell edges.

Readings taken here (the paper leaves them open; the native generator follows
the same readings in its own code):
* a sub-cell is inside / outside / cut according to the signs of the leaf
  vertices it contains; inside sub-cells get a tensor Gauss-Legendre rule,
  cut sub-cells are bisected until they are leaves;
* a cut leaf square is split along its (0,0)-(1,1) diagonal into the
  triangles (v00, v10, v11) and (v00, v11, v01); a cut leaf cube into the six
  Kuhn tetrahedra of the main diagonal, permutations in lexicographic order;
* each simplex is clipped by the linear interpolant of the snapped vertex
  values; in 2D the positive polygon is produced by walking the edges
  (a, b), (b, c), (c, a) and emitting a positive start vertex and every sign
  change, then fanned from its first vertex; in 3D the positive part is a
  tetrahedron or a wedge, the wedge cut into three tetrahedra;
* Gauss rules on simplices are collapsed (Duffy) tensor Gauss-Legendre
  rules; the boundary pieces are the clipped facets with the outward normal
  -grad(psi_lin)/|grad(psi_lin)|.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np


@functools.lru_cache(maxsize=None)
def _gauss01(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    x.flags.writeable = False
    w.flags.writeable = False
    return x, w


def gauss01(q: int):
    """Gauss-Legendre nodes and weights on [0, 1] (read-only arrays)."""
    return _gauss01(q)


def tensor_rule(lo: np.ndarray, hi: np.ndarray, q: int):
    """Tensor Gauss rule on the box [lo, hi] (d = len(lo))."""
    x, w = gauss01(q)
    d = len(lo)
    # all index tuples at once, the first axis slowest (itertools.product order)
    idx = np.array(list(itertools.product(range(q), repeat=d)))
    pts = lo[None, :] + (hi - lo)[None, :] * x[idx]
    wts = np.prod(w[idx], axis=1) * np.prod(hi - lo)
    return pts, wts


def triangle_rule(P: np.ndarray, q: int):
    """Collapsed Gauss rule on triangle P[0], P[1], P[2]:
    x = P0 + xi (P1 - P0) + eta (P2 - P1), xi = u, eta = u v, dxi deta = u du dv."""
    x, w = gauss01(q)
    J = abs(np.linalg.det(np.stack([P[1] - P[0], P[2] - P[1]], axis=1)))
    pts, wts = [], []
    for i in range(q):
        for j in range(q):
            u, v = x[i], x[j]
            xi, eta = u, u * v
            pts.append(P[0] + xi * (P[1] - P[0]) + eta * (P[2] - P[1]))
            wts.append(w[i] * w[j] * u * J)
    return np.array(pts), np.array(wts)


def tet_rule(P: np.ndarray, q: int):
    """Collapsed Gauss rule on tetrahedron P[0..3]:
    x = P0 + xi (P1-P0) + eta (P2-P1) + zeta (P3-P2), xi = u, eta = u v,
    zeta = u v w, Jacobian u^2 v."""
    x, w = gauss01(q)
    J = abs(np.linalg.det(np.stack([P[1] - P[0], P[2] - P[1], P[3] - P[2]], axis=1)))
    # all (i, j, k) at once, i slowest: the same products in the same order
    u, v, s = (a.reshape(-1) for a in np.meshgrid(x, x, x, indexing="ij"))
    wi, wj, wk = (a.reshape(-1) for a in np.meshgrid(w, w, w, indexing="ij"))
    xi, eta, zeta = u, u * v, u * v * s
    pts = (P[0] + xi[:, None] * (P[1] - P[0]) + eta[:, None] * (P[2] - P[1])
           + zeta[:, None] * (P[3] - P[2]))
    wts = wi * wj * wk * u * u * v * J
    return pts, wts


def segment_rule(A: np.ndarray, B: np.ndarray, q: int):
    x, w = gauss01(q)
    L = np.linalg.norm(B - A)
    pts = np.array([A + t * (B - A) for t in x])
    return pts, w * L


def surface_triangle_rule(P: np.ndarray, q: int):
    """Collapsed Gauss rule on a triangle embedded in 3D (area measure)."""
    x, w = gauss01(q)
    area2 = np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[1]))
    u, v = (a.reshape(-1) for a in np.meshgrid(x, x, indexing="ij"))
    wi, wj = (a.reshape(-1) for a in np.meshgrid(w, w, indexing="ij"))
    pts = P[0] + u[:, None] * (P[1] - P[0]) + (u * v)[:, None] * (P[2] - P[1])
    wts = wi * wj * u * area2
    return pts, wts


def _cross(a, b, fa, fb):
    """Point on segment a-b where the linear interpolant of (fa, fb) vanishes."""
    t = fa / (fa - fb)
    return a + t * (b - a)


def clip_triangle(P, f):
    """Positive part of triangle P (3x2) under the linear interpolant of f.

    Returns (list of triangles, boundary segment or None, gradient of the
    interpolant)."""
    poly = []
    for a in range(3):
        b = (a + 1) % 3
        if f[a] > 0.0:
            poly.append(P[a])
        if (f[a] > 0.0) != (f[b] > 0.0):
            poly.append(_cross(P[a], P[b], f[a], f[b]))
    tris = [np.array([poly[0], poly[k], poly[k + 1]]) for k in range(1, len(poly) - 1)]
    seg = None
    npos = int(sum(f > 0.0))
    if 0 < npos < 3:
        cuts = []
        for a in range(3):
            b = (a + 1) % 3
            if (f[a] > 0.0) != (f[b] > 0.0):
                cuts.append(_cross(P[a], P[b], f[a], f[b]))
        seg = (cuts[0], cuts[1])
    M = np.stack([P[1] - P[0], P[2] - P[0]])
    grad = np.linalg.solve(M, np.array([f[1] - f[0], f[2] - f[0]]))
    return tris, seg, grad


def _wedge(A, B, C, A2, B2, C2):
    """Triangular prism with bottom (A,B,C) and top (A2,B2,C2) joined A-A2,
    B-B2, C-C2, as three tetrahedra."""
    return [np.array([A, B, C, A2]), np.array([B, C, A2, B2]), np.array([C, A2, B2, C2])]


def clip_tet(P, f):
    """Positive part of tetrahedron P (4x3) under the linear interpolant of f.

    Returns (list of tetrahedra, list of boundary triangles, gradient)."""
    pos = [a for a in range(4) if f[a] > 0.0]
    neg = [a for a in range(4) if not f[a] > 0.0]
    I = lambda a, b: _cross(P[a], P[b], f[a], f[b])
    tets, faces = [], []
    if len(pos) == 4:
        tets = [P.copy()]
    elif len(pos) == 1:
        a = pos[0]
        b, c, d = neg
        tets = [np.array([P[a], I(a, b), I(a, c), I(a, d)])]
        faces = [np.array([I(a, b), I(a, c), I(a, d)])]
    elif len(pos) == 3:
        a, b, c = pos
        d = neg[0]
        tets = _wedge(P[a], P[b], P[c], I(a, d), I(b, d), I(c, d))
        faces = [np.array([I(a, d), I(b, d), I(c, d)])]
    elif len(pos) == 2:
        a, b = pos
        c, d = neg
        tets = _wedge(P[a], I(a, c), I(a, d), P[b], I(b, c), I(b, d))
        faces = [np.array([I(a, c), I(a, d), I(b, d)]), np.array([I(a, c), I(b, d), I(b, c)])]
    M = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]])
    grad = np.linalg.solve(M, np.array([f[1] - f[0], f[2] - f[0], f[3] - f[0]]))
    return tets, faces, grad


KUHN_PERMS = list(itertools.permutations(range(3)))


def element_quadrature(leaf, e, depth, lo, h, q_cell, q_simplex, q_bnd):
    """Quadrature for one element.

    leaf: snapped psi on the whole leaf lattice (indexed by leaf multi-index).
    e: element multi-index; h: element size; lo: box lower corner.
    Returns (vol_pts, vol_wts, bnd_pts, bnd_wts, bnd_normals)."""
    d = len(e)
    s = 2 ** depth
    hl = h / s
    vol_p, vol_w, bnd_p, bnd_w, bnd_n = [], [], [], [], []

    def corner(L):  # physical coordinates of leaf vertex multi-index L
        return np.array([lo + hl * L[a] for a in range(d)])

    def recurse(origin, size):
        idx = tuple(slice(origin[a], origin[a] + size + 1) for a in range(d))
        block = leaf[idx]
        npos = int(np.count_nonzero(block > 0.0))
        if npos == 0:
            return
        if npos == block.size:
            lo_c = np.array([lo + hl * origin[a] for a in range(d)])
            hi_c = np.array([lo + hl * (origin[a] + size) for a in range(d)])
            p, w = tensor_rule(lo_c, hi_c, q_cell)
            vol_p.append(p)
            vol_w.append(w)
            return
        if size > 1:
            half = size // 2
            for c in itertools.product(range(2), repeat=d):
                recurse(tuple(origin[a] + half * c[a] for a in range(d)), half)
            return
        # cut leaf
        if d == 2:
            ox, oy = origin
            V = {(i, j): (corner((ox + i, oy + j)), leaf[ox + i, oy + j]) for i in (0, 1) for j in (0, 1)}
            for tri in (((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))):
                P = np.array([V[t][0] for t in tri])
                f = np.array([V[t][1] for t in tri])
                tris, seg, grad = clip_triangle(P, f)
                for T in tris:
                    p, w = triangle_rule(T, q_simplex)
                    vol_p.append(p)
                    vol_w.append(w)
                if seg is not None:
                    p, w = segment_rule(seg[0], seg[1], q_bnd)
                    nrm = -grad / np.linalg.norm(grad)
                    bnd_p.append(p)
                    bnd_w.append(w)
                    bnd_n.append(np.tile(nrm, (len(w), 1)))
        else:
            for perm in KUHN_PERMS:
                L = [np.array(origin)]
                cur = np.array(origin)
                for ax in perm:
                    cur = cur.copy()
                    cur[ax] += 1
                    L.append(cur)
                P = np.array([corner(tuple(v)) for v in L])
                f = np.array([leaf[tuple(v)] for v in L])
                tets, faces, grad = clip_tet(P, f)
                for T in tets:
                    p, w = tet_rule(T, q_simplex)
                    vol_p.append(p)
                    vol_w.append(w)
                for F in faces:
                    p, w = surface_triangle_rule(F, q_bnd)
                    nrm = -grad / np.linalg.norm(grad)
                    bnd_p.append(p)
                    bnd_w.append(w)
                    bnd_n.append(np.tile(nrm, (len(w), 1)))

    recurse(tuple(ei * s for ei in e), s)
    cat = lambda L, k: np.concatenate(L) if L else np.zeros((0,) if k == 1 else (0, d))
    return (cat(vol_p, 2), cat(vol_w, 1), cat(bnd_p, 2), cat(bnd_w, 1), cat(bnd_n, 2))


def default_orders(dim: int, p: int):
    """(q_cell, q_simplex, q_bnd): tensor rule exact for the stiffness and mass
    integrands on whole cells (per-axis degree 2p), collapsed rules exact for
    the stiffness integrand on simplices (total degree 2 d p - 2 plus the Duffy
    Jacobian), boundary rules exact for the product of two functions on a
    facet."""
    q_cell = p + 1
    if dim == 2:
        return q_cell, max(2 * p, 1), 2 * p + 1
    return q_cell, 3 * p + 1, 3 * p + 1
