"""Level sets and the leaf-vertex sign lattice (oracle; test infrastructure only).

Immersed formulation section: the physical domain Omega sits inside a simple
embedding box carrying a tensor grid; elements that intersect Omega form the
background grid and the functions supported on Omega span V_h.  Figure 1's
caption describes the cut-cell integration: cut elements are bisected
recursively up to a maximum depth and then triangulated.

Readings taken here (the paper does not fix them):
* Omega = {psi > 0}; |psi| < 1e-13 is snapped to 0 and counts as outside.
* The geometry is sampled only at the vertices of the leaf lattice (spacing
  h / 2^depth).  An element is active when any of its leaf vertices is
  positive, inside when all are positive, cut otherwise.
"""
from __future__ import annotations

import numpy as np

SNAP = 1e-13


def psi_discs(points: np.ndarray, discs) -> np.ndarray:
    """Unit square minus discs: psi = min_k (|x - c_k| - r_k)."""
    x = points[..., 0]
    y = points[..., 1]
    out = np.full(x.shape, np.inf)
    for (cx, cy, r) in discs:
        dx = x - cx
        dy = y - cy
        d = np.sqrt(dx * dx + dy * dy) - r
        out = np.minimum(out, d)
    return out


def psi_gyroid(points: np.ndarray, phase, level: float) -> np.ndarray:
    """Gyroid with two periods on the unit cube: psi = level - g,
    g = sin X cos Y + sin Y cos Z + sin Z cos X, X = 4 pi x + phase_x."""
    X = 4.0 * np.pi * points[..., 0] + phase[0]
    Y = 4.0 * np.pi * points[..., 1] + phase[1]
    Z = 4.0 * np.pi * points[..., 2] + phase[2]
    g = np.sin(X) * np.cos(Y) + np.sin(Y) * np.cos(Z) + np.sin(Z) * np.cos(X)
    return level - g


def psi_star(points: np.ndarray) -> np.ndarray:
    """Figure 1: psi = 0.5 + 0.1 sin(5 theta) - r, theta = atan2(y, x)."""
    x = points[..., 0]
    y = points[..., 1]
    th = np.arctan2(y, x)
    r = np.sqrt(x * x + y * y)
    return 0.5 + 0.1 * np.sin(5.0 * th) - r


def apple_parts(points: np.ndarray):
    """The two level sets of the apple with a bite (numerical examples
    section, box (-2,2)^3): psi_1 = 1 - (z/1.7)^2 - (r/(1+z/17) - 0.7)^2 (the
    apple, r^2 = x^2 + y^2) and psi_2 = (x-2)^2 + y^2 + z^2 - 1 (the bite)."""
    x, y, z = points[..., 0], points[..., 1], points[..., 2]
    r = np.sqrt(x * x + y * y)
    p1 = 1.0 - (z / 1.7) ** 2 - (r / (1.0 + z / 17.0) - 0.7) ** 2
    p2 = (x - 2.0) ** 2 + y ** 2 + z ** 2 - 1.0
    return p1, p2


def psi_apple(points: np.ndarray) -> np.ndarray:
    """Apple with a bite: the intersection min(psi_1, psi_2)."""
    p1, p2 = apple_parts(points)
    return np.minimum(p1, p2)


def dirichlet_mask(w, points: np.ndarray) -> np.ndarray:
    """Which points of the approximate boundary carry the (penalty) Dirichlet
    condition.  "all": the whole immersed boundary.  "bite" (the apple
    example: homogeneous Dirichlet data on the surface of the bite only);
    reading: a boundary point belongs to the bite when the bite's level set
    is the smaller of the two there (it is the constraint that cuts)."""
    part = getattr(w, "dirichlet_part", "all")
    if part == "all":
        return np.ones(points.shape[0], dtype=bool)
    if part == "bite":
        p1, p2 = apple_parts(points)
        return p2 <= p1
    raise ValueError(part)


def psi_helix(points: np.ndarray) -> np.ndarray:
    """Triple helix joined by half rings (numerical examples section, box
    (-2,2)^3).  Reading: the three helices are the level set rotated by
    0, 2 pi/3, 4 pi/3 about the z axis, the domain is the union (max) of the
    helices and the two rings at z = -2 and z = +2."""
    x, y, z = points[..., 0], points[..., 1], points[..., 2]
    ri, Ro = 0.25, 1.5
    r = np.sqrt(x * x + y * y)
    out = np.full(x.shape, -np.inf)
    for k in range(3):
        a = 2.0 * np.pi * k / 3.0
        xr = np.cos(a) * x + np.sin(a) * y
        yr = -np.sin(a) * x + np.cos(a) * y
        p = ri ** 2 - (r - Ro) ** 2 - (z - 2.0 * np.arctan2(yr, xr) / np.pi) ** 2
        out = np.maximum(out, p)
    for s in (+1.0, -1.0):
        p = ri ** 2 - (r - Ro) ** 2 - (z + s * 2.0) ** 2
        out = np.maximum(out, p)
    return out


def psi_slab(points: np.ndarray, plane_x: float) -> np.ndarray:
    """Half of the box cut by the plane x = plane_x: psi = plane_x - x."""
    return plane_x - points[..., 0]


def level_set(w):
    """Return psi(points) for a workload description."""
    if w.geometry == "discs":
        return lambda P: psi_discs(P, w.discs)
    if w.geometry == "gyroid":
        return lambda P: psi_gyroid(P, w.phase, w.gyroid_level)
    if w.geometry == "star":
        return psi_star
    if w.geometry == "apple":
        return psi_apple
    if w.geometry == "helix":
        return psi_helix
    if w.geometry == "slab":
        return lambda P: psi_slab(P, w.plane_x)
    if w.geometry == "none":
        return lambda P: np.ones(P.shape[:-1])
    raise ValueError(w.geometry)


def snap(v: np.ndarray) -> np.ndarray:
    v = np.array(v, dtype=np.float64, copy=True)
    v[np.abs(v) < SNAP] = 0.0
    return v


def leaf_coords(lo: float, hi: float, nleaf: int) -> np.ndarray:
    """Leaf lattice coordinates lo + (hi - lo) * i / nleaf, i = 0..nleaf."""
    i = np.arange(nleaf + 1, dtype=np.float64)
    return (hi - lo) * i / nleaf + lo


def leaf_values(w, n: int, depth: int) -> np.ndarray:
    """Snapped psi on the leaf lattice of an n^d grid bisected `depth` times.

    Returns an array indexed [i_x, i_y(, i_z)] of shape (n 2^depth + 1)^d.
    """
    nleaf = n * (2 ** depth)
    c = leaf_coords(w.box_lo, w.box_hi, nleaf)
    grids = np.meshgrid(*([c] * w.dim), indexing="ij")
    P = np.stack(grids, axis=-1)
    return snap(level_set(w)(P))


def element_states(leaf: np.ndarray, n: int, depth: int):
    """Per element (indexed [e_x, e_y(, e_z)]): number of positive leaf vertices
    and total leaf vertices.  Active = any positive; inside = all positive."""
    d = leaf.ndim
    s = 2 ** depth
    pos = leaf > 0.0
    shape = (n,) * d
    npos = np.zeros(shape, dtype=np.int64)
    for off in np.ndindex(*([s + 1] * d)):
        sl = tuple(slice(o, o + n * s, s) for o in off)
        npos += pos[sl]
    total = (s + 1) ** d
    return npos, total


def active_elements(leaf: np.ndarray, n: int, depth: int) -> np.ndarray:
    npos, _ = element_states(leaf, n, depth)
    return npos > 0
