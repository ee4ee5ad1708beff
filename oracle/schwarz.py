"""Schwarz smoothers (oracle; test infrastructure only).

Smoothers subsection, "Additive Schwarz":
* M^{-1} = sum_j P_j (P_j^T A P_j)^{-1} P_j^T over N index blocks;
* block selection by encapsulating supports: for every basis function phi_j
  a block {phi_k : supp_Omega(phi_k) subset of supp_Omega(phi_j)};
  for Lagrange bases blocks are devised only for the nodal (vertex)
  functions;
* relaxation gamma = 1 / max_K N_K, N_K being the number of blocks that
  contain a function supported on element K (eq:applyASLemma,
  eq:applySummation, eq:applyCS): this keeps gamma lambda_max(M^{-1} A) <= 1;
* the remark on tiny eigenvalues: when a block matrix has an eigenvalue more
  than a factor 1e16 below its largest diagonal entry, the function that
  dominates that eigenvector is removed from the block.

Readings (not fixed by the paper):
* supp_Omega containment is decided on active elements: E(k) subset of E(j),
  E(k) = active elements on which phi_k is non-zero;
* the removal is repeated until no such eigenvalue remains; "dominant" =
  largest |v_i| (ties: lowest local index); a DOF left in no block gets the
  singleton block {i};
* blocks are kept in the order of their associated function; duplicates are
  kept (one block for every function).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis as B

REMOVAL_RATIO = 1e-16


def func_elements(lev):
    """Active-function compact index -> frozenset of active element linear indices."""
    pos = {int(L): i for i, L in enumerate(lev.active)}
    E = [set() for _ in range(len(lev.active))]
    for el, fl in lev.elem_funcs.items():
        for L in fl:
            i = pos.get(L)
            if i is not None:
                E[i].add(el)
    return [frozenset(s) for s in E]


def is_nodal(lev, L):
    if lev.basis == "bspline":
        return True
    m = lev.lat_to_multi(int(L))
    return all(mi % lev.p == 0 for mi in m)


def select_blocks(lev):
    """Blocks by encapsulating supports; returns list of sorted index arrays
    (compact indices) and the associated function of each block."""
    E = func_elements(lev)
    n = len(E)
    # candidates: functions sharing an element with j (others cannot be contained)
    el_to_f = {}
    for i, s in enumerate(E):
        for el in s:
            el_to_f.setdefault(el, []).append(i)
    blocks, assoc = [], []
    for j in range(n):
        if not is_nodal(lev, lev.active[j]):
            continue
        cand = set()
        for el in E[j]:
            cand.update(el_to_f[el])
        blk = sorted(k for k in cand if E[k] <= E[j])
        blocks.append(np.array(blk, dtype=np.int64))
        assoc.append(j)
    return blocks, assoc


def factor_block(A: sp.csr_matrix, idx: np.ndarray):
    """Eigen-factorize P^T A P with the tiny-eigenvalue removal.

    Returns (kept indices, inverse matrix, eigenvalues, removed indices)."""
    keep = list(idx)
    removed = []
    while True:
        Aj = A[keep][:, keep].toarray()
        lam, V = np.linalg.eigh(Aj)
        dmax = np.max(np.diag(Aj))
        k = int(np.argmin(lam))
        if lam[k] < REMOVAL_RATIO * dmax and len(keep) > 0:
            v = np.abs(V[:, k])
            i = int(np.argmax(v))  # first maximum = lowest local index on ties
            removed.append(keep[i])
            del keep[i]
            if not keep:
                return np.array([], dtype=np.int64), np.zeros((0, 0)), np.zeros(0), removed
            continue
        inv = (V / lam) @ V.T
        return np.array(keep, dtype=np.int64), inv, lam, removed


class Smoother:
    """Factored additive Schwarz smoother on one level."""

    def __init__(self, A: sp.csr_matrix, lev, blocks=None, omega=None):
        if blocks is None:
            blocks, assoc = select_blocks(lev)
        else:
            assoc = None
        self.n = A.shape[0]
        self.raw_blocks = blocks
        self.assoc = assoc
        self.blocks, self.inv, self.lam, self.removed = [], [], [], []
        for blk in blocks:
            k, inv, lam, rem = factor_block(A, blk)
            self.blocks.append(k)
            self.inv.append(inv)
            self.lam.append(lam)
            self.removed.append(rem)
        covered = np.zeros(self.n, dtype=bool)
        for k in self.blocks:
            covered[k] = True
        self.added = []
        for i in np.nonzero(~covered)[0]:
            k, inv, lam, rem = factor_block(A, np.array([i]))
            self.blocks.append(k)
            self.inv.append(inv)
            self.lam.append(lam)
            self.removed.append(rem)
            self.added.append(int(i))
        self.gamma = self._gamma(lev, self.blocks)
        self.omega = omega  # optional per-block weights; None -> uniform gamma

    def _gamma(self, lev, blocks):
        return 1.0 / max_NK(lev, blocks)

    def weights(self):
        if self.omega is None:
            return np.full(len(self.blocks), self.gamma)
        return np.asarray(self.omega, dtype=np.float64)

    def pre(self, r: np.ndarray) -> np.ndarray:
        """Pre-smoothing operator; additive Schwarz is symmetric, so the
        post-smoothing operator (its adjoint) is the same."""
        return self.apply(r)

    def post(self, r: np.ndarray) -> np.ndarray:
        return self.apply(r)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """y = sum_j w_j P_j A_j^{-1} P_j^T r (w_j = gamma unless weights given)."""
        y = np.zeros_like(r)
        for wj, k, inv in zip(self.weights(), self.blocks, self.inv):
            if len(k):
                y[k] += wj * (inv @ r[k])
        return y

    def dense(self) -> np.ndarray:
        """Dense sum_j w_j P_j A_j^{-1} P_j^T."""
        S = np.zeros((self.n, self.n))
        for wj, k, inv in zip(self.weights(), self.blocks, self.inv):
            if len(k):
                S[np.ix_(k, k)] += wj * inv
        return S


def block_elements(lev, blocks):
    """Active elements touched by each block: the union of E(k) over its
    members (two blocks interact through A only if these sets meet)."""
    E = func_elements(lev)
    return [frozenset().union(*[E[int(k)] for k in blk]) if len(blk) else frozenset() for blk in blocks]


def lattice_colour(lev, L, kind="schwarz"):
    """Colour of a block associated with the lattice function L, from its
    position (multiplicative Schwarz subsection: same-colour blocks must not
    share an element; (p+1)^d colours for B-splines, 2^d for Lagrange vertex
    blocks; the Gauss-Seidel footnote: (p+1)^d for single functions).
    Reading: B-splines and single-function blocks take sum_a (m_a mod (p+1))
    (p+1)^a; Lagrange vertex blocks (m_a = p v_a) take sum_a (v_a mod 2) 2^a."""
    m = lev.lat_to_multi(int(L))
    if kind == "schwarz" and lev.basis == "lagrange":
        q, pos = 2, [mi // lev.p for mi in m]
    else:
        q, pos = lev.p + 1, list(m)
    c = 0
    for a in reversed(range(lev.dim)):
        c = c * q + pos[a] % q
    return c


def colour_blocks(lev, blocks, given, base=None):
    """Colours of the final blocks: given[j] (an int) where known, else the
    smallest colour >= base (default: the number of lattice colours) that no
    block already coloured (in block order) uses on a shared element.  Raises
    if two same-colour given blocks share an element."""
    els = block_elements(lev, blocks)
    if base is None:
        base = (lev.p + 1) ** lev.dim   # above every lattice colour (2^d <= (p+1)^d)
    used = {}
    colours = []
    for j, es in enumerate(els):
        if given[j] is not None:
            c = int(given[j])
            for e in es:
                if c in used.get(e, ()):
                    raise ValueError(f"blocks of colour {c} share element {e}")
        else:
            taken = set()
            for e in es:
                taken |= used.get(e, set())
            c = base
            while c in taken:
                c += 1
        for e in es:
            used.setdefault(e, set()).add(c)
        colours.append(c)
    return colours


class MultiplicativeSmoother(Smoother):
    """Multiplicative Schwarz (eq:multiplicativeSchwarz1) with the graph
    colouring of the same subsection: the blocks are visited colour by colour
    and the residual is updated after every block,
        dy = P_j A_j^{-1} P_j^T r~,  y~ += dy,  r~ -= A dy,
    which equals the colour-wise form because blocks of one colour share no
    element (their updates do not change each other's residual).  No damping
    (unconditionally stable, as Gauss-Seidel).  The forward sweep visits the
    colours in ascending order (pre-smoothing); its adjoint visits them in
    descending order (post-smoothing), which keeps the V-cycle symmetric.
    kind = "schwarz": the encapsulating-support blocks; kind = "diagonal": one
    block per function (Gauss-Seidel, Remark rem:coarseGS)."""

    def __init__(self, A, lev, kind="schwarz"):
        if kind == "diagonal":
            blocks = [np.array([i], dtype=np.int64) for i in range(A.shape[0])]
            assoc = list(range(A.shape[0]))
        else:
            blocks, assoc = select_blocks(lev)
        super().__init__(A, lev, blocks=blocks)
        given = [lattice_colour(lev, lev.active[a], kind) for a in assoc]
        self._order_blocks(A, lev, assoc, given, lambda b: b, None)

    def _order_blocks(self, A, lev, assoc, given, to_scalar, base):
        """Colours (given ones for the input blocks, greedy from base for the
        singletons the factorization added; the element sets come from the
        blocks mapped by to_scalar), the sweep order and each block's reach."""
        self.assoc = assoc
        self.A = A
        given = list(given) + [None] * (len(self.blocks) - len(given))   # singletons added for uncovered DOFs
        self.colours = colour_blocks(lev, [to_scalar(np.asarray(b)) for b in self.blocks], given, base)
        self.order = sorted(range(len(self.blocks)), key=lambda j: (self.colours[j], j))
        # per block: the rows its update reaches (A[:, k] non-zero) and A[rows, k]
        Ac = A.tocsc()
        self._reach = []
        for k in self.blocks:
            sub = Ac[:, k]
            rows = np.unique(sub.indices)
            self._reach.append((rows, sub[rows].toarray()))

    def _sweep(self, r, order):
        y = np.zeros_like(r)
        rt = r.copy()
        for j in order:
            k, inv = self.blocks[j], self.inv[j]
            if not len(k):
                continue
            dy = inv @ rt[k]
            y[k] += dy
            rows, Ark = self._reach[j]
            rt[rows] -= Ark @ dy
        return y

    def forward(self, r):
        return self._sweep(r, self.order)

    def backward(self, r):
        return self._sweep(r, self.order[::-1])

    pre = forward
    post = backward

    def apply(self, r):
        return self.forward(r)


class DiagonalSmoother(Smoother):
    """Damped Jacobi as additive Schwarz with one block per function (Remark
    rem:coarseGS: diagonal smoothing suffices on the coarser levels); the
    damping follows the additive rule gamma = 1 / max_K N_K."""

    def __init__(self, A, lev):
        blocks = [np.array([i], dtype=np.int64) for i in range(A.shape[0])]
        super().__init__(A, lev, blocks=blocks)


def max_NK(lev, blocks) -> int:
    """max over active elements K of N_K = #blocks containing a function
    non-zero on K (eq:applyCS)."""
    pos = {int(L): i for i, L in enumerate(lev.active)}
    f_el = {}
    for el, fl in lev.elem_funcs.items():
        for L in fl:
            i = pos.get(L)
            if i is not None:
                f_el.setdefault(i, set()).add(el)
    count = {}
    for blk in blocks:
        els = set()
        for i in blk:
            els |= f_el.get(int(i), set())
        for el in els:
            count[el] = count.get(el, 0) + 1
    return max(count.values()) if count else 1
