"""Plain, slow FP64 CPU oracle for the immersed multigrid-preconditioned CG method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, the
native generator, the Python binding) may import, call, link or execute any
file in this directory.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.

Every function restates the paper (de Prenter et al., "Scalable multigrid
methods for immersed finite element methods and immersed isogeometric
analysis") and cites the section / equation / algorithm it follows.  The
oracle favours the plain definition of each object over speed:

* geometry.py   - level sets, leaf-vertex sign lattice, element states
                  (immersed formulation section, Figure 1).
* quadrature.py - cut-cell quadrature: bisection to a maximum depth,
                  triangulation, Gauss rules on the clipped simplices and on
                  the approximate boundary (Figure 1 caption).
* basis.py      - open uniform B-splines (Cox-de Boor recursion) and
                  Lagrange polynomials (immersed formulation section).
* assemble.py   - A_ij = a_h(phi_i, phi_j), b_i = b_h(phi_i)
                  (eq:weakMulti, eq:operatorsMulti, eq:systemMulti).
* hierarchy.py  - two-scale relation Phi_{l-1} = R_l Phi_l (eq:coarsening)
                  and Galerkin operators R A R^T (Remark rem:gridParamCorr).
* schwarz.py    - encapsulating-support blocks, the tiny-eigenvalue removal
                  remark, the additive Schwarz operator and its damping.
* multigrid.py  - the V-cycle (Algorithm alg:MGV) and CG preconditioned by it.
* mlp.py        - the per-block damping network (forward/backward/Adam).
* elasticity.py - linear elasticity with penalty Dirichlet conditions and
                  per-component Schwarz blocks (eq:weakMulti,
                  eq:operatorsMulti).
* thb.py        - truncated hierarchical B-splines (Figure fig:THB), the
                  hierarchical coarsening of Algorithm alg:coarsen and the THB
                  multigrid hierarchy, for Poisson and for 2D linear
                  elasticity (per-component blocks).
* learned.py    - per-block damping: block features, the two-grid objective
                  built on eq:eigenMulti with its adjoint gradient, and the
                  lambda_max(S A) < 2(1 - 0.05) stability check.

Parity unpinned (no independent pin exists): exact iteration counts against
the paper (its convergence figures are not in the text), removal decisions
whose eigenvalue ratio sits within a factor 10 of the 1e-16 threshold, and
learned damping weights (judged only against the uniform-damping fallback).
"""
