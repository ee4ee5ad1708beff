"""ctypes binding of the HIP solver library libimsmg.so (same call names as the C ABI).

Argument marshalling only: every step of factorization, V-cycle and CG runs in
the library's HIP kernels.  Device vectors are torch tensors (float64, on the
library context's device); torch provides memory, nothing else.  The library
orders its work on its own stream and returns after completion; before each
call the binding synchronizes torch's device so that tensors written by torch
are complete.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import LIB_DIR

OK = 0
ERR = {-1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "NOT_SPD", -5: "NOT_CONVERGED", -6: "NAN", -7: "STATE"}
FP64, MIXED = 0, 1
ADDITIVE, MULTIPLICATIVE = 0, 1

_lib = None


class Csr(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class Patches(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("ptr", C.c_void_p), ("idx", C.c_void_p), ("colour", C.c_void_p)]


class Elements(C.Structure):
    _fields_ = [("nelements", C.c_int32), ("eptr", C.c_void_p), ("eidx", C.c_void_p), ("shape", C.c_int32 * 3),
                ("elem", C.c_void_p), ("eta", C.c_void_p)]


class Lattice(C.Structure):
    _fields_ = [("dim", C.c_int32), ("shape", C.c_int32 * 3), ("reach", C.c_int32), ("dof_to_lattice", C.c_void_p),
                ("two_scale", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("use_graph", C.c_int32), ("timing", C.c_int32), ("gamma", C.c_double),
                ("compress", C.c_int32), ("use_learned", C.c_int32), ("autotune", C.c_int32),
                ("block_gemm", C.c_int32), ("flexible_cg", C.c_int32), ("smoother", C.c_int32),
                ("coarse_smoother", C.c_int32), ("cycle", C.c_int32), ("flag_min_rows", C.c_int32),
                ("ncomp", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("solve_ms", C.c_double), ("restarts", C.c_int32),
                ("fallback_flags", C.c_int32), ("setup_ms", C.c_double), ("factor_ms", C.c_double)]


class LevelStats(C.Structure):
    _fields_ = [("n", C.c_int32), ("stencil", C.c_int32), ("stored_rows", C.c_int32), ("general_rows", C.c_int32),
                ("sg_nnz", C.c_int64), ("lattice", C.c_int64), ("value_bytes", C.c_int32), ("general_lanes", C.c_int32),
                ("patch_gemm", C.c_int32), ("bf16_blocks", C.c_int32)]


SYMBOLS = ["imsmg_default_options", "imsmg_create", "imsmg_setup", "imsmg_set_patch_weights",
           "imsmg_factor_patches", "imsmg_get_patches", "imsmg_get_patch_colours", "imsmg_get_gamma", "imsmg_vcycle", "imsmg_vcycle_time", "imsmg_pcg_solve", "imsmg_mg_solve",
           "imsmg_apply_operator", "imsmg_apply_smoother", "imsmg_apply_restriction", "imsmg_apply_prolongation",
           "imsmg_coarse_solve", "imsmg_get_level_stats", "imsmg_kernel_time", "imsmg_last_error", "imsmg_destroy",
           "imsmg_load_mlp", "imsmg_get_patch_features", "imsmg_get_patch_weights", "imsmg_set_block_weights",
           "imsmg_lambda_max", "imsmg_two_grid_objective", "imsmg_mlp_workspace_bytes", "imsmg_mlp_forward",
           "imsmg_mlp_loss_grad", "imsmg_mlp_loss_grad_noalloc", "imsmg_mlp_adam", "imsmg_vcycle_multi", "imsmg_pcg_solve_multi",
           "imsmg_setup_batched", "imsmg_batch_problem", "imsmg_pcg_solve_batched"]
MLP_PARAMS = 5313
NOALLOC_MAX_SAMPLES = 8192  # IMSMG_NOALLOC_MAX_SAMPLES
NFEAT = 16


def library_path() -> str:
    """The in-tree build, or the HIP library named by IMSMG_LIBRARY (another
    build of the same sources, e.g. for side-by-side timing)."""
    return os.environ.get("IMSMG_LIBRARY") or os.path.join(LIB_DIR, "libimsmg.so")


def load():
    """Load libimsmg.so; raises if it is not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    lib.imsmg_default_options.argtypes = [C.POINTER(Options)]
    lib.imsmg_default_options.restype = None
    lib.imsmg_create.argtypes = [C.POINTER(vp), i32, vp]
    lib.imsmg_setup.argtypes = [vp, i32, C.POINTER(Csr), C.POINTER(Csr), C.POINTER(Patches), C.POINTER(Lattice),
                                C.POINTER(Elements), C.POINTER(Options)]
    lib.imsmg_set_patch_weights.argtypes = [vp, i32, vp]
    lib.imsmg_factor_patches.argtypes = [vp]
    lib.imsmg_get_patches.argtypes = [vp, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int64), vp, vp]
    lib.imsmg_get_gamma.argtypes = [vp, i32, C.POINTER(C.c_double)]
    lib.imsmg_get_patch_colours.argtypes = [vp, i32, C.POINTER(C.c_int32), vp]
    lib.imsmg_vcycle.argtypes = [vp, vp, vp]
    lib.imsmg_vcycle_time.argtypes = [vp, vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.imsmg_pcg_solve.argtypes = [vp, vp, vp, dbl, C.POINTER(Info)]
    lib.imsmg_mg_solve.argtypes = [vp, vp, vp, dbl, i32, i32, C.POINTER(Info)]
    for f in ("imsmg_apply_operator", "imsmg_apply_smoother", "imsmg_apply_restriction", "imsmg_apply_prolongation"):
        getattr(lib, f).argtypes = [vp, i32, vp, vp]
    lib.imsmg_coarse_solve.argtypes = [vp, vp, vp]
    lib.imsmg_kernel_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), i32]
    lib.imsmg_get_level_stats.argtypes = [vp, i32, C.POINTER(LevelStats)]
    lib.imsmg_last_error.argtypes = [vp]
    lib.imsmg_last_error.restype = C.c_char_p
    lib.imsmg_destroy.argtypes = [vp]
    lib.imsmg_load_mlp.argtypes = [vp, vp, i64]
    lib.imsmg_get_patch_features.argtypes = [vp, i32, C.POINTER(C.c_int32), vp]
    lib.imsmg_get_patch_weights.argtypes = [vp, i32, C.POINTER(C.c_int32), vp, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_double)]
    lib.imsmg_set_block_weights.argtypes = [vp, i32, vp]
    lib.imsmg_lambda_max.argtypes = [vp, i32, i32, C.POINTER(C.c_double)]
    lib.imsmg_two_grid_objective.argtypes = [vp, i32, vp, i32, C.POINTER(C.c_double), vp]
    lib.imsmg_mlp_workspace_bytes.argtypes = [i32]
    lib.imsmg_mlp_forward.argtypes = [vp, vp, vp, i32, vp]
    lib.imsmg_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
    lib.imsmg_mlp_loss_grad_noalloc.argtypes = [vp, vp, vp, vp, i32, vp, vp]
    lib.imsmg_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float]
    lib.imsmg_vcycle_multi.argtypes = [vp, i32, vp, vp]
    lib.imsmg_pcg_solve_multi.argtypes = [vp, i32, vp, vp, dbl, C.POINTER(Info)]
    lib.imsmg_setup_batched.argtypes = [vp, i32, C.POINTER(C.c_int), C.POINTER(C.POINTER(Csr)),
                                        C.POINTER(C.POINTER(Csr)), C.POINTER(C.POINTER(Patches)),
                                        C.POINTER(C.POINTER(Lattice)), C.POINTER(C.POINTER(Elements)),
                                        C.POINTER(Options)]
    lib.imsmg_batch_problem.argtypes = [vp, i32, C.POINTER(vp)]
    lib.imsmg_pcg_solve_batched.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(vp), dbl, C.POINTER(Info), i32]
    for s in SYMBOLS:
        if s not in ("imsmg_default_options", "imsmg_last_error"):
            getattr(lib, s).restype = C.c_int
    lib.imsmg_mlp_workspace_bytes.restype = C.c_int64
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class SolverError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR.get(code, code)}: {msg}")
        self.code = code


def smoother_options(w) -> dict:
    """Options naming a workload's smoothers and cycle (the blocks of coarse
    diagonal smoothing come from the generator)."""
    fine = MULTIPLICATIVE if getattr(w, "smoother", "as") == "ms" else ADDITIVE
    cs = getattr(w, "coarse_smoother", "same")
    coarse = -1 if cs == "same" else (MULTIPLICATIVE if cs == "gs" else ADDITIVE)
    return dict(smoother=fine, coarse_smoother=coarse, cycle=getattr(w, "cycle", 1))


def default_options(**kw) -> Options:
    lib = load()
    o = Options()
    lib.imsmg_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclass
class SolveInfo:
    status: int
    iterations: int
    rel_res: float
    true_rel_res: float
    solve_ms: float
    restarts: int = 0
    fallback_flags: int = 0
    setup_ms: float = 0.0
    factor_ms: float = 0.0

    @staticmethod
    def of(i):
        return SolveInfo(i.status, i.iterations, i.rel_res, i.true_rel_res, i.solve_ms, i.restarts,
                         i.fallback_flags, i.setup_ms, i.factor_ms)


def problem_structs(problem, dim: int = None, reach: int = None, implicit_transfer=True):
    """The C-ABI arrays of one generated problem (levels 0 = coarsest):
    (nlevels, A, R, P, L, E, keep); keep holds the numpy arrays the structs
    point into and must outlive the setup call."""
    w = problem.workload
    dim = dim or w.dim
    reach = reach or w.degree
    L = len(problem.levels)
    keep = []
    A = (Csr * L)()
    R = (Csr * L)()
    P = (Patches * L)()
    Lt = (Lattice * L)()
    E = (Elements * L)()
    for l, lev in enumerate(problem.levels):
        rp, ci, va = _i32(lev.A.indptr), _i32(lev.A.indices), np.ascontiguousarray(lev.A.data, np.float64)
        keep += [rp, ci, va]
        A[l] = Csr(lev.A.shape[0], lev.A.shape[1], lev.A.nnz, _p(rp).value, _p(ci).value, _p(va).value)
        if lev.dof_to_lattice is None:
            # general sparse level (locally refined basis): no function lattice
            Lt[l] = Lattice(0, (C.c_int32 * 3)(lev.A.shape[0], 1, 1), 0, None, None)
        else:
            d2l = _i32(lev.dof_to_lattice)
            keep.append(d2l)
            shp = (C.c_int32 * 3)(*(list(lev.lattice) + [1] * (3 - len(lev.lattice))))
            ts = None
            if implicit_transfer and l > 0 and getattr(lev, "two_scale", None) is not None:
                ts = np.ascontiguousarray(lev.two_scale, dtype=np.float64)
                keep.append(ts)
            Lt[l] = Lattice(dim, shp, reach, _p(d2l).value, _p(ts).value if ts is not None else None)
        if l > 0:
            Rm = lev.R
            rrp, rci, rva = _i32(Rm.indptr), _i32(Rm.indices), np.ascontiguousarray(Rm.data, np.float64)
            keep += [rrp, rci, rva]
            R[l] = Csr(Rm.shape[0], Rm.shape[1], Rm.nnz, _p(rrp).value, _p(rci).value, _p(rva).value)
            bp, bi = _i32(lev.block_ptr), _i32(lev.block_idx)
            keep += [bp, bi]
            bc = None
            if getattr(lev, "block_colour", None) is not None:
                bc = _i32(lev.block_colour)
                keep.append(bc)
            P[l] = Patches(len(bp) - 1, _p(bp).value, _p(bi).value, _p(bc).value if bc is not None else None)
        if lev.elem_ptr is not None:
            ep, ei = _i32(lev.elem_ptr), _i32(lev.elem_idx)
            keep += [ep, ei]
            eshape = (C.c_int32 * 3)(*([lev.n_elements] * dim + [1] * (3 - dim)))
            el = et = None
            if getattr(lev, "elem_id", None) is not None:
                el = _i32(lev.elem_id)
                keep.append(el)
                if getattr(lev, "eta", None) is not None:
                    et = np.ascontiguousarray(np.asarray(lev.eta, np.float64)[lev.elem_id])
                    keep.append(et)
            E[l] = Elements(len(ep) - 1, _p(ep).value, _p(ei).value, eshape,
                            _p(el).value if el is not None else None, _p(et).value if et is not None else None)
    return L, A, R, P, Lt, E, keep


class Solver:
    """One library context bound to a HIP device."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        self._check(self.lib.imsmg_create(C.byref(h), device, None), h)
        self.h = h
        self.problem = None
        self._keep = []

    def _check(self, rc, h=None):
        if rc != OK:
            msg = self.lib.imsmg_last_error(h if h is not None else self.h)
            raise SolverError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.imsmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- setup
    def setup(self, problem, options: Options = None, dim: int = None, reach: int = None, implicit_transfer=True):
        """problem: a generator.GeneratedProblem (levels 0 = coarsest)."""
        w = problem.workload
        L, A, R, P, Lt, E, keep = problem_structs(problem, dim, reach, implicit_transfer)
        opt = options if options is not None else default_options(nu_pre=w.nu, nu_post=w.nu)
        if opt.ncomp == 1:
            opt.ncomp = getattr(problem.levels[-1], "ncomp", 1)   # vector problems: components per function
        self._check(self.lib.imsmg_setup(self.h, L, A, R, P, Lt, E, C.byref(opt)))
        self.problem = problem
        self.options = opt
        return self

    def set_patch_weights(self, level: int, omega):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        self._check(self.lib.imsmg_set_patch_weights(self.h, level, _p(om)))

    def factor(self):
        self._check(self.lib.imsmg_factor_patches(self.h))
        return self

    def get_patches(self, level: int):
        nb = C.c_int32()
        nnz = C.c_int64()
        self._check(self.lib.imsmg_get_patches(self.h, level, C.byref(nb), C.byref(nnz), None, None))
        ptr = np.zeros(nb.value + 1, np.int32)
        idx = np.zeros(nnz.value, np.int32)
        self._check(self.lib.imsmg_get_patches(self.h, level, C.byref(nb), C.byref(nnz), _p(ptr), _p(idx)))
        return ptr, idx

    def get_patch_colours(self, level: int):
        """(number of colours, colour of every post-removal block)."""
        nb = C.c_int32()
        self._check(self.lib.imsmg_get_patches(self.h, level, C.byref(nb), None, None, None))
        nc = C.c_int32()
        col = np.zeros(nb.value, np.int32)
        self._check(self.lib.imsmg_get_patch_colours(self.h, level, C.byref(nc), _p(col)))
        return nc.value, col

    # ------------------------------------------------- per-block damping
    def load_mlp(self, params):
        th = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.imsmg_load_mlp(self.h, _p(th), th.size))
        return self

    def features(self, level: int) -> np.ndarray:
        nb = C.c_int32()
        self._check(self.lib.imsmg_get_patch_features(self.h, level, C.byref(nb), None))
        F = np.zeros((nb.value, NFEAT), np.float32)
        self._check(self.lib.imsmg_get_patch_features(self.h, level, C.byref(nb), _p(F)))
        return F

    def weights(self, level: int):
        """(omega per final block, learned_status, lambda_max estimate)"""
        nb, st, lm = C.c_int32(), C.c_int32(), C.c_double()
        self._check(self.lib.imsmg_get_patch_weights(self.h, level, C.byref(nb), None, None, None))
        om = np.zeros(nb.value, np.float64)
        self._check(self.lib.imsmg_get_patch_weights(self.h, level, C.byref(nb), _p(om), C.byref(st), C.byref(lm)))
        return om, st.value, lm.value

    def set_block_weights(self, level: int, omega):
        om = np.ascontiguousarray(omega, dtype=np.float64)
        self._check(self.lib.imsmg_set_block_weights(self.h, level, _p(om)))

    def lambda_max(self, level: int, iters: int = 60) -> float:
        lm = C.c_double()
        self._check(self.lib.imsmg_lambda_max(self.h, level, iters, C.byref(lm)))
        return lm.value

    def two_grid_objective(self, Z, k: int = 1, grad: bool = True):
        """J and dJ/domega (final blocks of level 1) of a two-level hierarchy;
        Z: (n_1, m) host array."""
        Zc = np.asfortranarray(np.asarray(Z, np.float64).reshape(self._n(1), -1))
        J = C.c_double()
        g = np.zeros(len(self.weights(1)[0]), np.float64) if grad else None
        self._check(self.lib.imsmg_two_grid_objective(self.h, Zc.shape[1], Zc.ctypes.data_as(C.c_void_p), k,
                                                      C.byref(J), _p(g) if grad else None))
        return (J.value, g) if grad else J.value

    def gamma(self, level: int) -> float:
        g = C.c_double()
        self._check(self.lib.imsmg_get_gamma(self.h, level, C.byref(g)))
        return g.value

    # ---------------------------------------------------------- device ops
    def _dev(self, t):
        torch = self.torch
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
        return C.c_void_p(t.data_ptr())

    def _sync(self):
        self.torch.cuda.synchronize(self.device)

    def _n(self, level):
        return self.problem.levels[level].n

    def empty(self, level: int):
        return self.torch.zeros(self._n(level), dtype=self.torch.float64, device=f"cuda:{self.device}")

    def vcycle(self, r, z=None):
        z = self.empty(len(self.problem.levels) - 1) if z is None else z
        self._sync()
        self._check(self.lib.imsmg_vcycle(self.h, self._dev(r), self._dev(z)))
        return z

    def vcycle_time(self, r, reps: int = 50):
        """(median, mean) ms of one V-cycle over reps timed cycles."""
        med, mean = C.c_double(), C.c_double()
        self._sync()
        self._check(self.lib.imsmg_vcycle_time(self.h, self._dev(r), reps, C.byref(med), C.byref(mean)))
        return med.value, mean.value

    def pcg(self, b, x, rtol: float = 1e-8, raise_on_error: bool = True) -> SolveInfo:
        info = Info()
        self._sync()
        rc = self.lib.imsmg_pcg_solve(self.h, self._dev(b), self._dev(x), rtol, C.byref(info))
        if rc != OK and raise_on_error:
            self._check(rc)
        return SolveInfo.of(info)

    def mg_solve(self, b, x, rtol: float = 1e-8, max_cycles: int = 500, fmg: bool = False,
                 raise_on_error: bool = True) -> SolveInfo:
        """Multigrid as a standalone solver (imsmg_mg_solve): x <- x + B (b - A x),
        optionally started by a full multigrid pass (fmg=True, x's start ignored)."""
        info = Info()
        self._sync()
        rc = self.lib.imsmg_mg_solve(self.h, self._dev(b), self._dev(x), rtol, max_cycles, int(fmg), C.byref(info))
        if rc != OK and raise_on_error:
            self._check(rc)
        return SolveInfo.of(info)

    def _devm(self, t):
        torch = self.torch
        assert t.dtype == torch.float64 and t.is_cuda and t.dim() == 2 and t.is_contiguous()
        return C.c_void_p(t.data_ptr())

    def vcycle_multi(self, Rm, Zm=None):
        """Rm: (nrhs, n) device tensor (row k = right-hand side k)."""
        Zm = self.torch.zeros_like(Rm) if Zm is None else Zm
        self._sync()
        self._check(self.lib.imsmg_vcycle_multi(self.h, Rm.shape[0], self._devm(Rm), self._devm(Zm)))
        return Zm

    def pcg_multi(self, Bm, Xm, rtol: float = 1e-8, raise_on_error: bool = True, sync: bool = True):
        """Bm, Xm: (nrhs, n) device tensors; returns one SolveInfo per column.
        sync=False skips the device-wide synchronization before the call (the
        caller guarantees that Bm and Xm are complete, e.g. several contexts
        driven from host threads)."""
        k = Bm.shape[0]
        infos = (Info * k)()
        if sync:
            self._sync()
        rc = self.lib.imsmg_pcg_solve_multi(self.h, k, self._devm(Bm), self._devm(Xm), rtol, infos)
        if rc != OK and raise_on_error:
            self._check(rc)
        return [SolveInfo.of(i) for i in infos]

    def apply_operator(self, level, x, y=None):
        y = self.empty(level) if y is None else y
        self._sync()
        self._check(self.lib.imsmg_apply_operator(self.h, level, self._dev(x), self._dev(y)))
        return y

    def apply_smoother(self, level, r, y=None):
        y = self.empty(level) if y is None else y
        self._sync()
        self._check(self.lib.imsmg_apply_smoother(self.h, level, self._dev(r), self._dev(y)))
        return y

    def apply_restriction(self, level, rf, rc=None):
        rc = self.empty(level - 1) if rc is None else rc
        self._sync()
        self._check(self.lib.imsmg_apply_restriction(self.h, level, self._dev(rf), self._dev(rc)))
        return rc

    def apply_prolongation(self, level, xc, xf):
        self._sync()
        self._check(self.lib.imsmg_apply_prolongation(self.h, level, self._dev(xc), self._dev(xf)))
        return xf

    def coarse_solve(self, r, x=None):
        x = self.empty(0) if x is None else x
        self._sync()
        self._check(self.lib.imsmg_coarse_solve(self.h, self._dev(r), self._dev(x)))
        return x

    def level_stats(self, level: int) -> dict:
        st = LevelStats()
        self._check(self.lib.imsmg_get_level_stats(self.h, level, C.byref(st)))
        return {k: getattr(st, k) for k, _ in LevelStats._fields_}

    def kernel_time(self, reset: bool = False):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.imsmg_kernel_time(self.h, C.byref(ms), C.byref(n), 1 if reset else 0))
        return ms.value, n.value


# ------------------------------------------------------ damping network kernels
class BatchContext:
    """Many independent problems in one library batch context
    (imsmg_setup_batched): one child context and HIP stream per problem, the
    solves driven by the library's own pool of host threads."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.imsmg_create(C.byref(h), device, None)
        if rc != OK:
            raise SolverError(rc, "imsmg_create failed")
        self.h = h
        self.problems = []

    def _check(self, rc):
        if rc != OK:
            msg = self.lib.imsmg_last_error(self.h)
            raise SolverError(rc, msg.decode() if msg else "")

    def setup(self, problems, options: Options, implicit_transfer=True):
        """problems: generator.GeneratedProblem list; one options struct for all."""
        k = len(problems)
        structs = [problem_structs(g, implicit_transfer=implicit_transfer) for g in problems]
        nl = (C.c_int * k)(*[st[0] for st in structs])
        arr = lambda T, i: (C.POINTER(T) * k)(*[C.cast(st[i], C.POINTER(T)) for st in structs])
        self._check(self.lib.imsmg_setup_batched(self.h, k, nl, arr(Csr, 1), arr(Csr, 2), arr(Patches, 3),
                                                 arr(Lattice, 4), arr(Elements, 5), C.byref(options)))
        self.problems = list(problems)
        return self

    def factor(self):
        self._check(self.lib.imsmg_factor_patches(self.h))
        return self

    def problem_handle(self, p: int):
        ch = C.c_void_p()
        self._check(self.lib.imsmg_batch_problem(self.h, p, C.byref(ch)))
        return ch

    def level_stats(self, p: int, level: int) -> dict:
        st = LevelStats()
        ch = self.problem_handle(p)
        rc = self.lib.imsmg_get_level_stats(ch, level, C.byref(st))
        if rc != OK:
            raise SolverError(rc, (self.lib.imsmg_last_error(ch) or b"").decode())
        return {f: getattr(st, f) for f, _ in LevelStats._fields_}

    def pcg(self, B, X, rtol: float = 1e-8, nthreads: int = 4, raise_on_error: bool = True):
        """B, X: per problem a (nrhs, n_p) FP64 device tensor (row k = right-hand
        side k); returns per problem one SolveInfo per column."""
        torch = self.torch
        k = len(B)
        nrhs = B[0].shape[0]
        for b, x, g in zip(B, X, self.problems):
            assert b.shape == x.shape == (nrhs, g.fine.n) and b.dtype == x.dtype == torch.float64
            assert b.is_cuda and x.is_cuda and b.is_contiguous() and x.is_contiguous()
        torch.cuda.synchronize(self.device)
        bp = (C.c_void_p * k)(*[b.data_ptr() for b in B])
        xp = (C.c_void_p * k)(*[x.data_ptr() for x in X])
        infos = (Info * (k * nrhs))()
        rc = self.lib.imsmg_pcg_solve_batched(self.h, nrhs, bp, xp, rtol, infos, nthreads)
        if rc != OK and raise_on_error:
            self._check(rc)
        return [[SolveInfo.of(i)
                 for i in infos[p * nrhs:(p + 1) * nrhs]] for p in range(k)]

    def close(self):
        if getattr(self, "h", None):
            self.lib.imsmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def mlp_forward(params, X):
    """o for every row of X (torch float32 device tensors; params: 5313)."""
    import torch
    lib = load()
    assert params.dtype == torch.float32 and X.dtype == torch.float32 and params.numel() == MLP_PARAMS
    X = X.contiguous()
    out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    rc = lib.imsmg_mlp_forward(_stream(torch), C.c_void_p(params.data_ptr()), C.c_void_p(X.data_ptr()),
                               X.shape[0], C.c_void_p(out.data_ptr()))
    if rc != OK:
        raise SolverError(rc, "imsmg_mlp_forward")
    return out


def mlp_loss_grad_noalloc(params, X, t, loss=None, grad=None):
    """Loss and gradient of the damping network through the allocation-free
    entry point (the library's static workspace; at most
    NOALLOC_MAX_SAMPLES rows).  loss (1) and grad (5313) may be given as
    preallocated float32 device tensors; returns (loss, grad)."""
    import torch
    lib = load()
    X = X.contiguous()
    loss = torch.zeros(1, dtype=torch.float32, device=X.device) if loss is None else loss
    grad = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=X.device) if grad is None else grad
    rc = lib.imsmg_mlp_loss_grad_noalloc(_stream(torch), C.c_void_p(params.data_ptr()), C.c_void_p(X.data_ptr()),
                                         C.c_void_p(t.data_ptr()), X.shape[0], C.c_void_p(loss.data_ptr()),
                                         C.c_void_p(grad.data_ptr()))
    if rc != OK:
        raise SolverError(rc, "imsmg_mlp_loss_grad_noalloc")
    return loss, grad


class MlpTrainer:
    """Device-side training state of the damping network: parameters, Adam
    moments and the loss-gradient workspace (all torch float32 tensors)."""

    def __init__(self, params, n):
        import torch
        self.torch = torch
        self.lib = load()
        dev = params.device
        self.params = params.clone().contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.n = n
        self.work = torch.empty(int(self.lib.imsmg_mlp_workspace_bytes(n)), dtype=torch.uint8, device=dev)
        self.step_count = 0

    def loss_grad(self, X, t):
        assert X.shape == (self.n, NFEAT) and t.shape == (self.n,)
        rc = self.lib.imsmg_mlp_loss_grad(_stream(self.torch), C.c_void_p(self.params.data_ptr()),
                                          C.c_void_p(X.data_ptr()), C.c_void_p(t.data_ptr()), self.n,
                                          C.c_void_p(self.work.data_ptr()), C.c_void_p(self.loss.data_ptr()),
                                          C.c_void_p(self.grad.data_ptr()))
        if rc != OK:
            raise SolverError(rc, "imsmg_mlp_loss_grad")
        return self.loss, self.grad

    def step(self, X, t, lr):
        self.loss_grad(X, t)
        self.step_count += 1
        rc = self.lib.imsmg_mlp_adam(_stream(self.torch), C.c_void_p(self.params.data_ptr()),
                                     C.c_void_p(self.grad.data_ptr()), C.c_void_p(self.m.data_ptr()),
                                     C.c_void_p(self.v.data_ptr()), self.step_count, C.c_float(lr))
        if rc != OK:
            raise SolverError(rc, "imsmg_mlp_adam")
        return self.loss
