"""Pins of the oracle's per-block damping pieces (network, features, two-grid
objective, stability check) against closed forms, finite differences and
independent routes (no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import assemble as AS
from oracle import learned as LR
from oracle import mlp as NN
from oracle import problem as P

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- network
def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_mlp_parameter_count():
    assert NN.NPARAM == 5313
    theta = np.arange(NN.NPARAM, dtype=np.float64)
    assert np.array_equal(NN.pack(*NN.unpack(theta)), theta)


def test_mlp_gradient_matches_central_differences():
    rng = _rng(3)
    theta = NN.init(rng)
    theta[NN.NPARAM - 1] = 0.3
    X = rng.standard_normal((9, NN.NFEAT))
    t = rng.standard_normal(9)
    L, g = NN.loss_and_grad(theta, X, t)
    idx = rng.choice(NN.NPARAM, size=40, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (NN.loss_and_grad(tp, X, t)[0] - NN.loss_and_grad(tm, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
    assert np.isclose(L, np.mean((NN.forward(theta, X) - t) ** 2))


def test_mlp_constant_network_closed_form():
    # all weights zero: o = b3 for every input; dL/db3 = 2 mean(b3 - t), the rest 0
    theta = np.zeros(NN.NPARAM)
    theta[-1] = 0.7
    X = _rng(4).standard_normal((5, NN.NFEAT))
    t = np.array([0.1, -0.2, 0.5, 1.0, 0.0])
    L, g = NN.loss_and_grad(theta, X, t)
    assert np.allclose(NN.forward(theta, X), 0.7)
    assert np.isclose(L, np.mean((0.7 - t) ** 2))
    assert np.isclose(g[-1], 2 * np.mean(0.7 - t))
    assert np.all(g[:-1] == 0.0)
    # omega = gamma exp(clip(o)): clipped at +-3
    theta[-1] = 10.0
    assert np.allclose(NN.weights(theta, X, 0.25), 0.25 * np.exp(3.0))


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([2.0, -0.5, 1e-3])
    th, m, v = NN.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# ---------------------------------------------------------------- problem
@pytest.fixture(scope="module")
def two_level():
    w = W.small_discs(seed=11, n=16, degree=2, levels=2, n_discs=3, rmin=0.08, rmax=0.15)
    op = P.build(w)
    return w, op


def test_two_grid_operator_is_identity_minus_BA(two_level):
    """eq:eigenMulti: with one smoothing step on each side, I - B A equals
    (I - S A)(I - R^T A_c^{-1} R A)(I - S A) for the V-cycle of Alg. MGV."""
    w, op = two_level
    sm = op.smoothers[1]
    A = op.hier.A[1].toarray()
    B = op.vcycle.dense(1)
    n = A.shape[0]
    Z = _rng(5).standard_normal((n, 4))
    omega = np.full(len(sm.blocks), sm.gamma)
    J, _ = LR.two_grid_objective(op.hier.A[1], op.hier.R[0], op.hier.A[0], sm, omega, Z, 1)
    E = np.eye(n) - B @ A
    EZ = E @ Z
    assert np.isclose(J, np.sum(EZ * (A @ EZ)) / np.sum(Z * (A @ Z)), rtol=1e-9)
    # gamma = 1 / max N_K keeps the smoother stable: E contracts in the energy norm
    assert J <= 1.0 + 1e-9


def test_two_grid_zero_weights_is_coarse_projection(two_level):
    """S = 0 leaves the coarse correction C = I - R^T A_c^{-1} R A, a projection:
    C^2 = C, so J(0) is the same for one and two applications."""
    _, op = two_level
    sm = op.smoothers[1]
    n = op.hier.A[1].shape[0]
    Z = _rng(6).standard_normal((n, 3))
    om0 = np.zeros(len(sm.blocks))
    J1, _ = LR.two_grid_objective(op.hier.A[1], op.hier.R[0], op.hier.A[0], sm, om0, Z, 1)
    J2, _ = LR.two_grid_objective(op.hier.A[1], op.hier.R[0], op.hier.A[0], sm, om0, Z, 2)
    assert np.isclose(J1, J2, rtol=1e-9)
    assert 0.0 < J1 <= 1.0 + 1e-12  # an A-orthogonal projection does not increase the energy norm


def test_two_grid_gradient_matches_central_differences(two_level):
    _, op = two_level
    sm = op.smoothers[1]
    rng = _rng(7)
    n = op.hier.A[1].shape[0]
    Z = rng.standard_normal((n, 3))
    omega = sm.gamma * np.exp(0.3 * rng.standard_normal(len(sm.blocks)))
    args = (op.hier.A[1], op.hier.R[0], op.hier.A[0], sm)
    J, g = LR.two_grid_objective(*args, omega, Z, 2)
    sizes = np.array([len(b) for b in sm.blocks])
    pick = list(rng.choice(np.nonzero(sizes == 1)[0], 4, replace=False)) + \
        list(rng.choice(np.nonzero(sizes > 1)[0], 4, replace=False))
    for j in pick:
        h = 1e-6 * omega[j]
        op_, om_ = omega.copy(), omega.copy()
        op_[j] += h
        om_[j] -= h
        fd = (LR.two_grid_objective(*args, op_, Z, 2)[0] - LR.two_grid_objective(*args, om_, Z, 2)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * max(abs(g[j]), 1e-3 * np.abs(g).max())


def test_lambda_max_scales_and_respects_the_schwarz_bound(two_level):
    """gamma = 1 / max_K N_K keeps lambda_max(gamma S A) <= 1 (the damping
    discussion after eq:applyCS); lambda_max is homogeneous in omega."""
    _, op = two_level
    sm = op.smoothers[1]
    om = np.full(len(sm.blocks), sm.gamma)
    lm = LR.lambda_max_SA(op.hier.A[1], sm, om)
    assert 0.1 < lm <= 1.0 + 1e-9
    assert np.isclose(LR.lambda_max_SA(op.hier.A[1], sm, 1.5 * om), 1.5 * lm, rtol=1e-9)


# ---------------------------------------------------------------- features
def test_coarse_volume_fractions_equal_direct_integration(two_level):
    """A coarse element's eta (mean of its children) equals the fraction
    integrated directly on the coarse level at one more bisection level."""
    w, op = two_level
    eta = LR.volume_fractions(op.hier, op.system.vol_frac)
    leaf = op.leaf
    coarse = AS.assemble(w, leaf, w.n // 2, w.depth + 1, with_rhs=False)
    assert set(coarse.vol_frac) == set(eta[0])
    for el, v in coarse.vol_frac.items():
        assert abs(v - eta[0][el]) <= 1e-12


def test_features_of_uncut_interior_blocks(two_level):
    """A singleton block whose support is inside Omega, away from the box and
    the cuts: sizes 1/K, full support, eta = 1, N_K = (p+1)^d (every function
    on the element owns one block), kappa = 1, no removal, no offset."""
    w, op = two_level
    sm = op.smoothers[1]
    eta = LR.volume_fractions(op.hier, op.system.vol_frac)
    F = LR.block_features(op.hier.levels[1], op.hier.A[1], sm, eta[1])
    K = (2 * w.degree + 1) ** 2
    full = (F[:, 2] == 1.0) & np.isclose(F[:, 3], 1.0, atol=1e-12) & (F[:, 0] == 1.0 / K) & (F[:, 11] == 0.0)
    assert full.sum() > 10
    row = F[full]
    assert np.allclose(row[:, [1, 4, 5, 8, 9, 10, 12, 13, 14]], [1.0 / K, 0, 0, 0, 0, 0, 0, 0, 0], atol=1e-12)
    assert np.allclose(row[:, 6], 1.0)
    assert np.allclose(F[:, 15], np.mean([v < LR.CUT_ETA for v in eta[1].values()])) and 0 < F[0, 15] < 1
    # invariants over all blocks
    assert np.all(F[:, 3] <= F[:, 2] + 1e-12) and np.all(F[:, 4] <= 1e-12)
    assert np.all(F[:, 0] <= F[:, 1] + 1e-15) and np.all(F[:, 9] <= 1e-12)
    assert np.all(np.abs(F[:, 12:15]) < 0.5)
    # a cut block has an eta below one and a shifted centroid
    cut = F[:, 11] > 0
    assert cut.any() and np.any(F[cut, 4] < 0.0) and np.any(np.abs(F[cut, 12:14]) > 0.0)
