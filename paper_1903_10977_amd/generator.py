"""ctypes binding of the native problem generator (libimsmg_gen.so).

`generate(workload)` returns a GeneratedProblem holding, per level (0 =
coarsest), the active lattice indices, the CSR operator, the restriction to
the next coarser level and the Schwarz blocks, plus the fine right-hand side
(and optionally the fine mass matrix).  All arithmetic runs in the native
library; this module only marshals arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from . import LIB_DIR

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(LIB_DIR, "libimsmg_gen.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or python -m paper_1903_10977_amd.build")
    lib = C.CDLL(path)
    lib.imsmg_gen_build.argtypes = [C.POINTER(GenSpec), C.POINTER(C.c_void_p)]
    lib.imsmg_gen_build.restype = C.c_int
    lib.imsmg_gen_level_info_get.argtypes = [C.c_void_p, C.c_int, C.POINTER(LevelInfo)]
    lib.imsmg_gen_get_operator.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.imsmg_gen_get_operator_block.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]
    lib.imsmg_gen_get_restriction.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.imsmg_gen_get_blocks.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.imsmg_gen_get_block_colours.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    lib.imsmg_gen_lattice_colours.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p]
    lib.imsmg_gen_get_two_scale.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    lib.imsmg_gen_get_rhs.argtypes = [C.c_void_p, C.c_void_p]
    lib.imsmg_gen_get_elements.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.imsmg_gen_get_mass.argtypes = [C.c_void_p, C.c_void_p]
    lib.imsmg_gen_get_volume_fractions.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    lib.imsmg_gen_setup_seconds.argtypes = [C.c_void_p]
    lib.imsmg_gen_setup_seconds.restype = C.c_double
    lib.imsmg_gen_last_error.restype = C.c_char_p
    lib.imsmg_gen_free.argtypes = [C.c_void_p]
    _lib = lib
    return lib


class GenSpec(C.Structure):
    _fields_ = [("dim", C.c_int32), ("degree", C.c_int32), ("n", C.c_int32), ("depth", C.c_int32),
                ("levels", C.c_int32), ("basis", C.c_int32), ("bc", C.c_int32), ("rhs", C.c_int32),
                ("geometry", C.c_int32), ("ndiscs", C.c_int32), ("discs", C.POINTER(C.c_double)),
                ("phase", C.c_double * 3), ("gyroid_level", C.c_double), ("box_lo", C.c_double),
                ("box_hi", C.c_double), ("penalty_factor", C.c_double), ("q_cell", C.c_int32),
                ("q_simplex", C.c_int32), ("q_bnd", C.c_int32), ("nthreads", C.c_int32),
                ("with_mass", C.c_int32), ("physics", C.c_int32), ("dirichlet_part", C.c_int32),
                ("lame_lambda", C.c_double), ("lame_mu", C.c_double), ("force", C.c_double * 3),
                ("plane_x", C.c_double)]


class LevelInfo(C.Structure):
    _fields_ = [("n_active", C.c_int32), ("nnz", C.c_int64), ("lattice", C.c_int32 * 3),
                ("n_elements", C.c_int32), ("nblocks", C.c_int32), ("block_nnz", C.c_int64),
                ("r_nnz", C.c_int64), ("n_cut", C.c_int32), ("n_active_elements", C.c_int32),
                ("elem_nnz", C.c_int64), ("eta_min", C.c_double), ("ncomp", C.c_int32)]


_BASIS = {"bspline": 0, "lagrange": 1}
_BC = {"box_dirichlet": 0, "penalty": 1, "neumann": 2}
_RHS = {"one": 0, "manufactured": 1, "zero": 2, "force": 2}
_GEOM = {"none": 0, "discs": 1, "gyroid": 2, "star": 3, "apple": 4, "slab": 5}
_PHYSICS = {"poisson": 0, "elasticity": 1}
_DPART = {"all": 0, "bite": 1}


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


@dataclass
class GenLevel:
    """One level.  Vector problems (ncomp > 1): DOF c N + i is component c of
    scalar function i (N = len(dof_to_lattice)); A, R, the blocks, the
    element incidence and the colours are over these vector DOFs, the lattice
    fields describe the scalar functions."""
    n_elements: int
    lattice: tuple
    dof_to_lattice: np.ndarray
    A: sp.csr_matrix
    R: Optional[sp.csr_matrix]            # maps this level to the next coarser one
    block_ptr: Optional[np.ndarray]
    block_idx: Optional[np.ndarray]
    block_assoc: Optional[np.ndarray]
    n_cut: int
    eta_min: float
    eta: Optional[np.ndarray] = None      # per-element volume fractions (x fastest)
    elem_ptr: Optional[np.ndarray] = None  # active element -> active functions (CSR)
    elem_idx: Optional[np.ndarray] = None
    elem_id: Optional[np.ndarray] = None   # element index of each active element
    two_scale: Optional[np.ndarray] = None  # 1D factor of R (coarser 1D functions x these)
    block_colour: Optional[np.ndarray] = None  # colour of every block (multiplicative smoother)
    ncomp: int = 1
    scalar_indptr: Optional[np.ndarray] = None   # vector problems: the scalar pattern
    scalar_indices: Optional[np.ndarray] = None

    @property
    def n(self):
        return self.A.shape[0]

    def blocks(self) -> List[np.ndarray]:
        return [self.block_idx[self.block_ptr[j]:self.block_ptr[j + 1]] for j in range(len(self.block_ptr) - 1)]


@dataclass
class GeneratedProblem:
    workload: object
    levels: List[GenLevel]
    b: np.ndarray
    M: Optional[sp.csr_matrix]
    seconds: float

    @property
    def fine(self) -> GenLevel:
        return self.levels[-1]


def generate(w, with_mass: bool = False, nthreads: int = 0, orders=None) -> GeneratedProblem:
    lib = _load()
    spec = GenSpec()
    spec.dim, spec.degree, spec.n, spec.depth, spec.levels = w.dim, w.degree, w.n, w.depth, w.levels
    spec.basis, spec.bc, spec.rhs, spec.geometry = _BASIS[w.basis], _BC[w.bc], _RHS[w.rhs], _GEOM[w.geometry]
    discs = np.ascontiguousarray(np.array(w.discs if w.discs else [[0, 0, 0]], dtype=np.float64))
    spec.ndiscs = len(w.discs) if w.discs else 0
    spec.discs = discs.ctypes.data_as(C.POINTER(C.c_double))
    ph = w.phase if w.phase else [0.0, 0.0, 0.0]
    for a in range(3):
        spec.phase[a] = ph[a]
    spec.gyroid_level = w.gyroid_level
    spec.box_lo, spec.box_hi = w.box_lo, w.box_hi
    spec.penalty_factor = w.penalty_factor
    q = orders if orders is not None else (0, 0, 0)
    spec.q_cell, spec.q_simplex, spec.q_bnd = q
    spec.nthreads = nthreads
    spec.with_mass = 1 if with_mass else 0
    spec.physics = _PHYSICS[getattr(w, "physics", "poisson")]
    spec.dirichlet_part = _DPART[getattr(w, "dirichlet_part", "all")]
    spec.lame_lambda = getattr(w, "lame_lambda", 0.0)
    spec.lame_mu = getattr(w, "lame_mu", 0.0)
    f = getattr(w, "force", None) or [0.0, 0.0, 0.0]
    for a in range(3):
        spec.force[a] = f[a] if a < len(f) else 0.0
    spec.plane_x = getattr(w, "plane_x", 0.0)
    h = C.c_void_p()
    rc = lib.imsmg_gen_build(C.byref(spec), C.byref(h))
    if rc != 0:
        raise RuntimeError(f"imsmg_gen_build failed ({rc}): {lib.imsmg_gen_last_error().decode()}")
    try:
        levels = []
        for l in range(w.levels):
            info = LevelInfo()
            assert lib.imsmg_gen_level_info_get(h, l, C.byref(info)) == 0
            n, nnz = info.n_active, info.nnz
            d2l = np.zeros(n, dtype=np.int32)
            rp = np.zeros(n + 1, dtype=np.int32)
            col = np.zeros(nnz, dtype=np.int32)
            val = np.zeros(nnz, dtype=np.float64)
            assert lib.imsmg_gen_get_operator(h, l, _ptr(d2l), _ptr(rp), _ptr(col), _ptr(val)) == 0
            nc = info.ncomp
            if nc == 1:
                A = sp.csr_matrix((val, col, rp), shape=(n, n))
            else:
                blocks = [[None] * nc for _ in range(nc)]
                for ci in range(nc):
                    for cj in range(nc):
                        bv = np.zeros(nnz, dtype=np.float64)
                        assert lib.imsmg_gen_get_operator_block(h, l, ci, cj, _ptr(bv)) == 0
                        blocks[ci][cj] = sp.csr_matrix((bv, col.copy(), rp.copy()), shape=(n, n))
                A = sp.bmat(blocks, format="csr")
                A.sort_indices()
            R = None
            R1 = None
            if l > 0:
                ncs = len(levels[l - 1].dof_to_lattice)
                rrp = np.zeros(ncs + 1, dtype=np.int32)
                rcol = np.zeros(info.r_nnz, dtype=np.int32)
                rval = np.zeros(info.r_nnz, dtype=np.float64)
                assert lib.imsmg_gen_get_restriction(h, l, _ptr(rrp), _ptr(rcol), _ptr(rval)) == 0
                R = sp.csr_matrix((rval, rcol, rrp), shape=(ncs, n))
                if nc > 1:
                    R = sp.kron(sp.identity(nc, format="csr"), R, format="csr")
                R1 = np.zeros((levels[l - 1].lattice[0], info.lattice[0]), dtype=np.float64)
                assert lib.imsmg_gen_get_two_scale(h, l, _ptr(R1)) == 0
            bp = bi = ba = bc = None
            diagonal = 0 < l < w.levels - 1 and getattr(w, "coarse_smoother", "same") in ("jacobi", "gs")
            if diagonal:
                # one block per function on the coarser levels (Remark rem:coarseGS)
                bp = np.arange(n + 1, dtype=np.int32)
                bi = np.arange(n, dtype=np.int32)
                ba = np.arange(n, dtype=np.int32)
                bc = np.zeros(n, dtype=np.int32)
                assert lib.imsmg_gen_get_block_colours(h, l, 1, _ptr(bc)) == 0
            elif info.nblocks > 0:
                bp = np.zeros(info.nblocks + 1, dtype=np.int32)
                bi = np.zeros(info.block_nnz, dtype=np.int32)
                ba = np.zeros(info.nblocks, dtype=np.int32)
                assert lib.imsmg_gen_get_blocks(h, l, _ptr(bp), _ptr(bi), _ptr(ba)) == 0
                bc = np.zeros(info.nblocks, dtype=np.int32)
                assert lib.imsmg_gen_get_block_colours(h, l, 0, _ptr(bc)) == 0
            eta = np.zeros(info.n_elements ** w.dim, dtype=np.float64)
            assert lib.imsmg_gen_get_volume_fractions(h, l, _ptr(eta)) == 0
            ep = np.zeros(info.n_active_elements + 1, dtype=np.int32)
            ei = np.zeros(info.elem_nnz, dtype=np.int32)
            eid = np.zeros(info.n_active_elements, dtype=np.int32)
            assert lib.imsmg_gen_get_elements(h, l, _ptr(ep), _ptr(ei), _ptr(eid)) == 0
            if nc > 1:
                bp, bi, ba, bc, ep, ei = _vector_level_arrays(n, nc, bp, bi, ba, bc, ep, ei,
                                                              (w.degree + 1) ** w.dim)
            levels.append(GenLevel(n_elements=info.n_elements, lattice=tuple(info.lattice[:w.dim]),
                                   dof_to_lattice=d2l, A=A, R=R, block_ptr=bp, block_idx=bi,
                                   block_assoc=ba, n_cut=info.n_cut, eta_min=info.eta_min, eta=eta,
                                   elem_ptr=ep, elem_idx=ei, elem_id=eid,
                                   two_scale=R1 if l > 0 else None, block_colour=bc, ncomp=nc,
                                   scalar_indptr=rp if nc > 1 else None, scalar_indices=col if nc > 1 else None))
        nf = levels[-1].n
        b = np.zeros(nf, dtype=np.float64)
        lib.imsmg_gen_get_rhs(h, _ptr(b))
        M = None
        if with_mass:
            F = levels[-1]
            if F.ncomp == 1:
                mv = np.zeros(F.A.nnz, dtype=np.float64)
                assert lib.imsmg_gen_get_mass(h, _ptr(mv)) == 0
                M = sp.csr_matrix((mv, F.A.indices.copy(), F.A.indptr.copy()), shape=F.A.shape)
            else:
                ns = len(F.dof_to_lattice)
                mv = np.zeros(len(F.scalar_indices), dtype=np.float64)
                assert lib.imsmg_gen_get_mass(h, _ptr(mv)) == 0
                Ms = sp.csr_matrix((mv, F.scalar_indices.copy(), F.scalar_indptr.copy()), shape=(ns, ns))
                M = sp.kron(sp.identity(F.ncomp, format="csr"), Ms, format="csr")
        secs = lib.imsmg_gen_setup_seconds(h)
    finally:
        lib.imsmg_gen_free(h)
    return GeneratedProblem(workload=w, levels=levels, b=b, M=M, seconds=secs)


def _vector_level_arrays(n, nc, bp, bi, ba, bc, ep, ei, ncol):
    """Per-component copies of a level's scalar arrays (vector DOF c n + i):
    blocks repeated per component (smoothers subsection: separate blocks for
    the functions of each component), colours offset by ncol = (p+1)^d, the
    scalar lattice colour count, per component (blocks of different
    components that share an element are coupled by A), element incidence
    listing every component."""
    if bp is not None:
        nb, nnzb = len(bp) - 1, int(bp[-1])
        bp = np.concatenate([bp[:-1] + c * nnzb for c in range(nc)] + [np.array([nc * nnzb])]).astype(np.int32)
        bi = np.concatenate([bi + c * n for c in range(nc)]).astype(np.int32)
        ba = np.concatenate([ba + c * n for c in range(nc)]).astype(np.int32)
        if bc is not None:
            bc = np.concatenate([bc + c * ncol for c in range(nc)]).astype(np.int32)
    cnt = np.diff(ep)
    ei2 = np.concatenate([np.concatenate([ei[ep[k]:ep[k + 1]] + c * n for c in range(nc)])
                          for k in range(len(cnt))]) if len(cnt) else ei
    ep2 = np.concatenate([[0], np.cumsum(nc * cnt)]).astype(np.int32)
    return bp, bi, ba, bc, ep2, ei2.astype(np.int32)


def with_coarse_diagonal(problem, kind: str = "jacobi"):
    """A copy of a generated problem whose levels between the finest and the
    coarsest carry one block per function (Remark rem:coarseGS: diagonal
    smoothing on the coarser levels), coloured by the lattice rule for
    one-function blocks; the other arrays are shared."""
    import dataclasses
    lib = _load()
    w = dataclasses.replace(problem.workload, coarse_smoother=kind)
    levels = list(problem.levels)
    for l in range(1, len(levels) - 1):
        lev = levels[l]
        n = lev.n
        ns = len(lev.dof_to_lattice)
        scol = np.zeros(ns, dtype=np.int32)
        d2l = np.ascontiguousarray(lev.dof_to_lattice, dtype=np.int32)
        assert lib.imsmg_gen_lattice_colours(ns, _ptr(d2l), lev.lattice[0], w.dim, w.degree + 1, 1, _ptr(scol)) == 0
        # vector levels: component c's functions after the scalar colours of components < c
        q = (w.degree + 1) ** w.dim
        col = np.concatenate([scol + c * q for c in range(lev.ncomp)]).astype(np.int32)
        levels[l] = dataclasses.replace(lev, block_ptr=np.arange(n + 1, dtype=np.int32),
                                        block_idx=np.arange(n, dtype=np.int32),
                                        block_assoc=np.arange(n, dtype=np.int32), block_colour=col)
    return dataclasses.replace(problem, workload=w, levels=levels)
