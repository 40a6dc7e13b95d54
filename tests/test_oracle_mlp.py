"""CPU pins of the learned-weight oracle: finite differences for the gradient,
the convergence bound, the bfloat16 rounding, and the feature definition."""
import numpy as np
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


def test_fp32_accumulation_of_the_forward_pass():
    """The pre-activations accumulate in FP32 (bias first, ascending index):
    exact when every partial sum is representable, otherwise within one FP32
    rounding per step of the FP64 sum."""
    rng = np.random.default_rng(5)
    # small integers: products and partial sums exact in FP32 and FP64 alike
    X = rng.integers(-8, 9, size=(50, M.N_IN)).astype(np.float64)
    W = rng.integers(-8, 9, size=(M.N_H, M.N_IN)).astype(np.float64)
    b = rng.integers(-8, 9, size=M.N_H).astype(np.float64)
    assert np.array_equal(M._acc32(b, X, W), X @ W.T + b)
    # general bfloat16 operands: bounded by the FP32 rounding of each step
    X = M.bf16(rng.standard_normal((200, M.N_IN)))
    W = M.bf16(rng.standard_normal((M.N_H, M.N_IN)))
    b = rng.standard_normal(M.N_H).astype(np.float32).astype(np.float64)
    got, want = M._acc32(b, X, W), X @ W.T + b
    bound = (M.N_IN + 1) * 2.0 ** -24 * (np.abs(X) @ np.abs(W).T + np.abs(b))
    assert np.all(np.abs(got - want) <= bound)
