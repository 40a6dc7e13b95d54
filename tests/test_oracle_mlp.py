"""CPU pins of the learned-weight oracle: finite differences for the gradient,
the convergence bound, the bfloat16 rounding, and the feature definition."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg_oracle as O
from oracle import mlp_oracle as M
from synthetic import problems as P


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.140625, 1e-3], np.float32)
    got = M.bf16(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1.0) wins;
    # 1 + 3*2^-8 ties between 1+2^-7 and 1+2^-6: even (1 + 2^-6) wins
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -7 and got[3] == 1.0 + 2 ** -6
    assert got[4] == -2.5 and got[5] == 3.140625
    assert abs(got[6] - 1e-3) <= 2 ** -9 * 1e-3


def test_features_hand_row():
    M_ = np.array([[4.0, -1.0, 0.0, -2.0], [-1.0, 2.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [-2.0, 0.0, 0.0, 8.0]])
    A = sp.csr_matrix(M_)
    F = M.features(A, 3)
    logd = np.log([4.0, 2.0, 1.0, 8.0])
    assert np.allclose(F[:, 0], logd - logd.mean())
    assert np.allclose(F[0, 1:7], [0.5, 0.25, 0, 0, 0, 0])
    assert np.allclose(F[:, 7], [0.25, 0.5, 1.0, 0.75])
    assert np.all(F[:, 8] == 3)


def test_omega_bound_makes_smoother_convergent():
    A = P.hetero3d(8, seed=2).to_scipy()
    w = M.init_weights(1)
    om = M.omega(w, A, M.features(A, 0))
    d = A.diagonal()
    Wi = om / d
    T = 2 * sp.diags(1.0 / Wi) - A
    # strictly diagonally dominant with a positive diagonal
    off = np.asarray(abs(T).sum(axis=1)).ravel() - np.abs(T.diagonal())
    assert np.all(T.diagonal() > off)
    # hence ||I - W A||_A < 1
    Ad = A.toarray()
    L = np.linalg.cholesky(Ad)
    S = np.eye(A.shape[0]) - np.diag(Wi) @ Ad
    Sa = L.T @ S @ np.linalg.inv(L.T)
    assert np.linalg.norm(Sa, 2) < 1.0


def test_projected_errors_have_no_coarse_component():
    A = P.hetero3d(10, seed=4).to_scipy()
    lv = O.coarsen_level(A, np.ones(A.shape[0]), O.Options.for_dim(3))
    E = M.projected_errors(A, lv.agg, lv.pval, lv.nc, 3, 7)
    assert np.abs(lv.P.T @ E).max() < 1e-13


def test_coarse_corrected_errors_are_the_a_orthogonal_complement():
    """e~ = (I - P A_c^-1 P^T A) e: P^T A e~ = 0 (A-orthogonal to the coarse
    space), a projection (applying it twice changes nothing), zero on range(P),
    and the A-norm minimiser of e - P y over every y (against random y)."""
    A = P.hetero3d(10, seed=4).to_scipy()
    lv = O.coarsen_level(A, np.ones(A.shape[0]), O.Options.for_dim(3))
    rng = np.random.default_rng(5)
    E = rng.standard_normal((A.shape[0], 3))
    T = M.coarse_corrected(A, lv.agg, lv.pval, lv.nc, E)
    scale = np.abs(lv.P.T @ (A @ E)).max()
    assert np.abs(lv.P.T @ (A @ T)).max() <= 1e-12 * scale
    T2 = M.coarse_corrected(A, lv.agg, lv.pval, lv.nc, T)
    assert np.abs(T2 - T).max() <= 1e-12 * np.abs(T).max()
    Z = M.coarse_corrected(A, lv.agg, lv.pval, lv.nc, lv.P @ rng.standard_normal((lv.nc, 2)))
    assert np.abs(Z).max() <= 1e-12
    anorm = lambda v: float(np.sqrt(v @ (A @ v)))   # noqa: E731
    for s in range(3):
        best = anorm(T[:, s])
        for _ in range(20):
            y = rng.standard_normal(lv.nc) * 0.1
            y += np.linalg.lstsq(lv.P.toarray(), E[:, s] - T[:, s], rcond=None)[0]
            assert anorm(E[:, s] - lv.P @ y) >= best * (1 - 1e-12)


def test_gradient_matches_central_differences():
    A = P.hetero3d(6, seed=3).to_scipy()
    lv = O.coarsen_level(A, np.ones(A.shape[0]), O.Options.for_dim(3))
    F = M.features(A, 1)
    E = M.projected_errors(A, lv.agg, lv.pval, lv.nc, 4, 11)
    w = M.init_weights(5)
    w[M.N_PARAMS - 1] = 0.3
    loss, g = M.loss_and_grad(w, A, F, E, round_bf16=False)
    rng = np.random.default_rng(0)
    idx = rng.choice(M.N_PARAMS, 40, replace=False)
    for k in list(idx) + [M.N_PARAMS - 1]:
        h = 1e-6 * max(1.0, abs(w[k]))
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (M.loss_and_grad(wp, A, F, E, False)[0] - M.loss_and_grad(wm, A, F, E, False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g).max()), (k, fd, g[k])
    assert 0.0 < loss < 1.0


def test_forward_hand_network():
    """A network small enough to evaluate by hand: only hidden unit 0 of each
    layer is wired, all values exact in bfloat16.
    x = (1, 2, 0, ..., 0): z1_0 = 0.5*1 + 0.25*2 + 1 = 2, h1_0 = 2;
    z1_1 = -3 (bias only) -> h1_1 = 0; z2_0 = 1.5*2 - 1 = 2, h2_0 = 2;
    y = 0.75*2 + 0.5 = 2."""
    d = {k: np.zeros(s) for k, s in M.SIZES}
    d["W1"][0, 0], d["W1"][0, 1], d["b1"][0], d["b1"][1] = 0.5, 0.25, 1.0, -3.0
    d["W2"][0, 0], d["W2"][0, 1], d["b2"][0] = 1.5, 7.0, -1.0
    d["W3"][0], d["b3"][0] = 0.75, 0.5
    F = np.zeros((2, M.N_IN))
    F[0, :2] = (1.0, 2.0)
    F[1, :2] = (-8.0, 0.0)   # z1_0 = -3 -> every hidden unit off: y = b3
    y, c = M.forward(M.pack(d), F)
    assert np.array_equal(y, [2.0, 0.5])
    assert c["h1"][0, 0] == 2.0 and c["h1"][0, 1] == 0.0 and c["h2"][0, 0] == 2.0


def test_forward_rounds_hidden_units_to_bfloat16():
    """1 + 2^-8 is a tie between 1 and 1 + 2^-7 (even mantissa wins): a hidden
    unit with that pre-activation enters the next layer as exactly 1."""
    d = {k: np.zeros(s) for k, s in M.SIZES}
    d["b1"][0] = 1.0 + 2.0 ** -8    # exact in FP32, a bfloat16 tie
    d["W2"][0, 0] = 1.0
    d["W3"][0] = 1.0
    y, c = M.forward(M.pack(d), np.zeros((1, M.N_IN)))
    assert c["z1"][0, 0] == 1.0 + 2.0 ** -8 and c["h1"][0, 0] == 1.0 and y[0] == 1.0
    y64, _ = M.forward(M.pack(d), np.zeros((1, M.N_IN)), round_bf16=False)
    assert y64[0] == 1.0 + 2.0 ** -8


def test_loss_omega_derivative_and_closed_form():
    """dL/domega against central differences; omega = 0 leaves every error
    unchanged (loss 1)."""
    A = P.hetero3d(5, seed=6).to_scipy()
    lv = O.coarsen_level(A, np.ones(A.shape[0]), O.Options.for_dim(3))
    E = M.projected_errors(A, lv.agg, lv.pval, lv.nc, 3, 5)
    assert M.loss_omega(A, E, np.zeros(A.shape[0]))[0] == pytest.approx(1.0, rel=1e-14)
    om = 0.3 + 0.4 * np.random.default_rng(2).random(A.shape[0])
    L, g = M.loss_omega(A, E, om)
    for i in (0, 17, A.shape[0] - 1):
        h = 1e-6
        e = np.zeros_like(om)
        e[i] = h
        fd = (M.loss_omega(A, E, om + e)[0] - M.loss_omega(A, E, om - e)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1e-3, np.abs(g).max())


def test_deviation_bounds_cover_fp32_evaluations():
    """The bounds the GPU tests use (tests/mlp_bounds.py) contain FP32
    evaluations of the same network in two different summation orders."""
    from tests import mlp_bounds as MB
    A = P.hetero3d(8, seed=4).to_scipy()
    w = M.init_weights(7)
    F = M.features(A, 1)
    om, dom, flips, fb = MB.omega_bounds(w, A, F)
    p = M.unpack(w)

    def fp32_forward(order):
        X = M.bf16(F).astype(np.float32)
        W1, W2, W3 = (M.bf16(p[k]).astype(np.float32) for k in ("W1", "W2", "W3"))

        def acc(bias, Xl, W):
            s = np.broadcast_to(np.asarray(bias, np.float32), (Xl.shape[0], W.shape[0])).copy()
            for q in order(Xl.shape[1]):
                s = s + Xl[:, q:q + 1] * W[:, q][None, :]
            return s

        h1 = M.bf16(np.maximum(acc(p["b1"], X, W1), 0)).astype(np.float32)
        h2 = M.bf16(np.maximum(acc(p["b2"], h1, W2), 0)).astype(np.float32)
        return acc(p["b3"], h2, W3[None, :])[:, 0].astype(np.float64)

    for order in (lambda m: range(m), lambda m: range(m - 1, -1, -1)):
        y32 = fp32_forward(order)
        assert np.all(np.abs(y32 - fb["y"]) <= fb["ey"])
        om32 = 1.0 / (1.0 + np.exp(-y32)) * M.omega_bound(A)
        assert np.all(np.abs(om32 - om) <= dom)
    assert 0.0 <= flips.mean() < 0.5
