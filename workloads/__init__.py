"""Seeded synthetic inputs shared by the oracle, the generator binding and the tests.

This module draws random numbers and names workloads.  It holds none of the
solver's arithmetic: no level-set evaluation, quadrature, basis, assembly,
coarsening, smoothing or Krylov step lives here.  Both the CPU oracle
(``oracle/``) and the native generator receive the same plain numbers from it
(disc centres and radii, gyroid phase shifts, right-hand sides).

Geometry conventions (shared *data*, not code): the physical domain is
Omega = {x in box : psi(x) > 0}.  Disc sets remove discs from the unit square,
the gyroid keeps {sin X cos Y + sin Y cos Z + sin Z cos X < level} with
X = 4 pi x + phase_x (two periods over [0,1]), the star is the domain of the
paper's Figure 1 (immersed formulation section).
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional

import numpy as np


def disc_set(seed: int, n_discs: int, rmin: float, rmax: float, max_draws: int = 200000):
    """Random sequential addition of non-overlapping discs inside [0,1]^2.

    Each draw takes a radius r ~ U[rmin, rmax] and then a centre ~ U[r, 1-r]^2
    from one PCG64 stream; the disc is kept when it overlaps no kept disc
    (centre distance strictly larger than the radius sum).  Returns an
    (n_discs, 3) array of rows (cx, cy, r) in acceptance order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kept: List[tuple] = []
    draws = 0
    while len(kept) < n_discs:
        if draws >= max_draws:
            raise RuntimeError(f"disc_set: only {len(kept)} of {n_discs} discs placed in {max_draws} draws")
        draws += 1
        r = float(rng.uniform(rmin, rmax))
        cx = float(rng.uniform(r, 1.0 - r))
        cy = float(rng.uniform(r, 1.0 - r))
        ok = True
        for (ox, oy, orad) in kept:
            if math.hypot(cx - ox, cy - oy) <= r + orad:
                ok = False
                break
        if ok:
            kept.append((cx, cy, r))
    return np.array(kept, dtype=np.float64).reshape(-1, 3)


def single_disc(seed: int, radius: float = 0.25, lo: float = 0.4, hi: float = 0.6):
    """One disc of fixed radius with centre ~ U[lo, hi]^2 (PCG64 stream `seed`)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = float(rng.uniform(lo, hi))
    cy = float(rng.uniform(lo, hi))
    return np.array([[cx, cy, radius]], dtype=np.float64)


def gyroid_phase(seed: int):
    """Phase shift ~ U[0, 2 pi)^3 for the gyroid level set."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 2.0 * math.pi, size=3).astype(np.float64)


def random_rhs(seed: int, n: int, nrhs: int = 1):
    """Standard-normal right-hand sides, shape (n,) or (n, nrhs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(size=(n, nrhs))
    return v[:, 0].copy() if nrhs == 1 else v


@dataclass
class Workload:
    """A fully specified synthetic problem.

    geometry: "discs" (unit square minus discs), "gyroid" (unit cube),
              "star" ((-1,1)^2), "none" (whole box).
    basis: "bspline" (open uniform, maximal smoothness) or "lagrange".
    bc: "box_dirichlet" (u = 0 strongly on the box faces, natural on the
        immersed boundary) or "penalty" (u = 0 weakly on the immersed
        boundary with parameter beta = penalty_factor / h, no strong BCs).
    rhs: "one" (f = 1), "manufactured" (u* = prod sin(2 pi x_i), f = -lap u*,
         Neumann data grad u* . n on the immersed boundary), "zero".
    physics: "poisson" (scalar) or "elasticity" (displacement with dim
         components, Lame parameters lame_lambda / lame_mu, constant body
         load `force`; bc "penalty" applies the penalty Dirichlet condition
         on the part of the immersed boundary named by dirichlet_part: "all"
         or "bite" (the apple's bite), the rest is traction free).
    smoother: "as" (additive Schwarz) or "ms" (multiplicative Schwarz with
         colouring) on the finest level; coarse_smoother: "same" (the finest
         level's smoother on every level), "jacobi" or "gs" (one block per
         function on the coarser levels); cycle: 1 (V) or 2 (W).
    local_levels: 0 for uniform grids; M > 0 for hierarchically refined
         meshes (truncated hierarchical B-splines): n is then the number of
         level-0 cells per axis and the cells cut by the immersed boundary are
         refined, recursively, M times (finest cells n 2^M per axis).
    """
    name: str
    dim: int
    degree: int
    n: int
    depth: int
    levels: int
    geometry: str
    basis: str = "bspline"
    bc: str = "box_dirichlet"
    rhs: str = "one"
    nu: int = 1
    discs: Optional[list] = None
    phase: Optional[list] = None
    gyroid_level: float = 0.3
    box_lo: float = 0.0
    box_hi: float = 1.0
    penalty_factor: float = 2.0
    smoother: str = "as"
    coarse_smoother: str = "same"
    cycle: int = 1
    physics: str = "poisson"
    lame_lambda: float = 1.0e3
    lame_mu: float = 1.0e3
    force: Optional[list] = None
    dirichlet_part: str = "all"
    plane_x: float = 0.0
    local_levels: int = 0

    def to_json(self) -> str:
        return json.dumps(asdict(self), sort_keys=True)

    @staticmethod
    def from_json(s: str) -> "Workload":
        return Workload(**json.loads(s))


def c1(seed: int = 0) -> Workload:
    """2D Poisson, quadratic B-splines, 32^2, unit square minus one disc (r = 0.25,
    centre ~ U[0.4,0.6]^2), depth 3, f = 1, u = 0 on the box, 3 levels."""
    return Workload(name="C1", dim=2, degree=2, n=32, depth=3, levels=3, geometry="discs",
                    discs=single_disc(seed).tolist(), rhs="one", nu=1)


def c2(seed: int = 1, n: int = 1024, levels: int = 6, depth: int = 1) -> Workload:
    """2D Poisson, cubic B-splines, n^2 (1024^2 at full size), unit square minus
    200 non-overlapping discs with radii U[0.01,0.04], manufactured solution
    sin(2 pi x) sin(2 pi y), V(2,2)."""
    return Workload(name="C2" if n == 1024 else f"C2-{n}", dim=2, degree=3, n=n, depth=depth,
                    levels=levels, geometry="discs", discs=disc_set(seed, 200, 0.01, 0.04).tolist(),
                    rhs="manufactured", nu=2)


def c3(seed: int = 2, n: int = 128, levels: int = 4) -> Workload:
    """3D Poisson, quadratic B-splines, n^3 (128^3 at full size), gyroid
    {g < 0.3} with two periods and a seeded phase, f = 1, u = 0 on the box."""
    return Workload(name="C3" if n == 128 else f"C3-{n}", dim=3, degree=2, n=n, depth=0,
                    levels=levels, geometry="gyroid", phase=gyroid_phase(seed).tolist(),
                    rhs="one", nu=1)


def star(n: int = 16, degree: int = 2, depth: int = 3, levels: int = 2) -> Workload:
    """The paper's star-shaped domain psi = 0.5 + 0.1 sin(5 theta) - r on
    (-1,1)^2 with quadratic Lagrange functions and penalty 2/h (Figure 1 and
    the smoother study of the multigrid section)."""
    return Workload(name=f"star-{n}", dim=2, degree=degree, n=n, depth=depth, levels=levels,
                    geometry="star", basis="lagrange", bc="penalty", rhs="zero", nu=1,
                    box_lo=-1.0, box_hi=1.0)


def small_discs(seed: int, n: int, degree: int, levels: int, n_discs: int = 6,
                depth: int = 1, rmin: float = 0.05, rmax: float = 0.12,
                rhs: str = "one", nu: int = 1) -> Workload:
    """Small multi-disc 2D problem used for parity tests at oracle-friendly size."""
    return Workload(name=f"discs-s{seed}-n{n}-p{degree}", dim=2, degree=degree, n=n, depth=depth,
                    levels=levels, geometry="discs",
                    discs=disc_set(seed, n_discs, rmin, rmax).tolist(), rhs=rhs, nu=nu)


def small_gyroid(seed: int, n: int, degree: int = 2, levels: int = 2) -> Workload:
    return Workload(name=f"gyroid-s{seed}-n{n}", dim=3, degree=degree, n=n, depth=0, levels=levels,
                    geometry="gyroid", phase=gyroid_phase(seed).tolist(), rhs="one", nu=1)


def c5(seed: int = 5, n: int = 96, levels: int = 4) -> Workload:
    """3D Poisson, quadratic B-splines, n^3 gyroid {g < 0.3} (two periods,
    seeded phase), f = 1, u = 0 on the box, V(1,1): the learned-damping test."""
    return Workload(name="C5" if n == 96 else f"C5-{n}", dim=3, degree=2, n=n, depth=0, levels=levels,
                    geometry="gyroid", phase=gyroid_phase(seed).tolist(), rhs="one", nu=1)


def gyroid_window(seed: int, n: int = 16, resolution: int = 96, levels: int = 2) -> Workload:
    """An n^3 sub-window of the gyroid at the element size of a resolution^3
    grid of the unit cube: random offset along the diagonal, random phase."""
    rng = np.random.Generator(np.random.PCG64(seed))
    width = n / resolution
    lo = float(rng.uniform(0.0, 1.0 - width))
    return Workload(name=f"gyroid-window-s{seed}", dim=3, degree=2, n=n, depth=0, levels=levels,
                    geometry="gyroid", phase=gyroid_phase(seed + 7919).tolist(), rhs="one", nu=1,
                    box_lo=lo, box_hi=lo + width)


def batched_c4(index: int) -> Workload:
    """Problem `index` (0..63) of the batched workload: n ~ U{64,128,256,512},
    p ~ U{1,2,3}, 10..100 discs with radii U[0.01,0.04], depth log2(1024/n)."""
    rng = np.random.Generator(np.random.PCG64(100 + index))
    n = int(rng.choice([64, 128, 256, 512]))
    p = int(rng.choice([1, 2, 3]))
    nd = int(rng.integers(10, 101))
    depth = int(round(math.log2(1024 // n)))
    levels = int(round(math.log2(n // 16))) + 1
    return Workload(name=f"C4-{index}", dim=2, degree=p, n=n, depth=depth, levels=levels,
                    geometry="discs", discs=disc_set(100 + index, nd, 0.01, 0.04).tolist(),
                    rhs="zero", nu=1)


def apple(n: int = 80, levels: int = 4, nu: int = 1) -> Workload:
    """3D linear elasticity on the apple with a bite (numerical examples
    section): box (-2,2)^3, quadratic B-splines, n^3 elements (80^3 in the
    paper), integration depth 0, lambda = mu = 1e3, gravity load (0, 0, -1),
    homogeneous Dirichlet data on the bite by the penalty method with
    beta = 2/h, traction free elsewhere."""
    return Workload(name="apple" if n == 80 else f"apple-{n}", dim=3, degree=2, n=n, depth=0,
                    levels=levels, geometry="apple", basis="bspline", bc="penalty", rhs="force",
                    nu=nu, box_lo=-2.0, box_hi=2.0, penalty_factor=2.0, physics="elasticity",
                    lame_lambda=1.0e3, lame_mu=1.0e3, force=[0.0, 0.0, -1.0], dirichlet_part="bite")


def slab(n: int = 8, levels: int = 2, fraction: float = 0.37) -> Workload:
    """3D linear elasticity on the part x < x_c of the unit cube, clamped on
    the immersed plane x = x_c by the penalty method (beta = 2/h) and loaded
    by gravity (0, 0, -1), lambda = mu = 1e3, quadratic B-splines.  x_c lies
    `fraction` of a fine element past a grid plane, so every cut element keeps
    that volume fraction on every level (no near-singular cut blocks: a
    parity case whose Schwarz blocks are all well determined)."""
    h = 1.0 / n
    xc = (n // 2 + fraction) * h
    return Workload(name=f"slab-{n}", dim=3, degree=2, n=n, depth=0, levels=levels, geometry="slab",
                    basis="bspline", bc="penalty", rhs="force", nu=1, penalty_factor=2.0,
                    physics="elasticity", lame_lambda=1.0e3, lame_mu=1.0e3, force=[0.0, 0.0, -1.0],
                    dirichlet_part="all", plane_x=xc)


def thb_discs(seed: int = 7, n: int = 64, local_levels: int = 2, levels: int = 3, n_discs: int = 12,
              rmin: float = 0.04, rmax: float = 0.12, depth: int = 1) -> Workload:
    """2D Poisson with quadratic truncated hierarchical B-splines: unit square
    minus non-overlapping discs, n^2 level-0 cells, the cells cut by the disc
    boundaries refined local_levels times, f = 1, u = 0 on the box."""
    return Workload(name=f"thb-s{seed}-n{n}-m{local_levels}", dim=2, degree=2, n=n, depth=depth,
                    levels=levels, geometry="discs", discs=disc_set(seed, n_discs, rmin, rmax).tolist(),
                    rhs="one", nu=1, local_levels=local_levels)


def thb_256(seed: int = 7) -> Workload:
    """The larger THB problem: 256^2 level-0 cells, cut cells refined twice
    (finest cells 1024^2 near the boundaries), 40 seeded discs with radii
    U[0.02, 0.06], six multigrid levels."""
    return thb_discs(seed=seed, n=256, local_levels=2, levels=6, n_discs=40, rmin=0.02, rmax=0.06)


def thb_star_elasticity(n: int = 96, local_levels: int = 2, levels: int = 5, depth: int = 2) -> Workload:
    """2D linear elasticity with quadratic truncated hierarchical B-splines
    (the physics of the paper's THB example: lambda = mu = 1e3, penalty
    Dirichlet conditions, a constant load (0, -1)) on the star domain
    psi = 0.5 + 0.1 sin(5 theta) - r in (-1,1)^2, n^2 level-0 cells, the cut
    cells refined local_levels times and clamped by the penalty method with
    beta = 2/h of the (finest) boundary cells, which with two local levels
    is the example's 4 x 2/h of the unrefined cells.  The level counts are
    chosen so that the coarsest operator stays numerically positive definite
    (hierarchies whose coarsest mesh leaves tiny pieces of the star's arms
    get a coarsest operator with eigenvalues at rounding level, which no
    direct solver without regularization factorizes)."""
    return Workload(name=f"thb-star-el-n{n}-m{local_levels}", dim=2, degree=2, n=n, depth=depth, levels=levels,
                    geometry="star", basis="bspline", bc="penalty", rhs="force", nu=1, box_lo=-1.0, box_hi=1.0,
                    penalty_factor=2.0, physics="elasticity", lame_lambda=1.0e3, lame_mu=1.0e3,
                    force=[0.0, -1.0], dirichlet_part="all", local_levels=local_levels)
