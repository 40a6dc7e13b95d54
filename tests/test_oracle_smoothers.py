"""CPU pins of the oracle's other smoothers: the Chebyshev polynomial smoother
(the paper's future work, Section 5) and multi-colour symmetric Gauss-Seidel
(Section 2.2.1), each against an independent formulation."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from numpy.polynomial import chebyshev as npcheb

from oracle import amg_oracle as O
from synthetic import problems as P


def _spd(rng, n):
    M = rng.standard_normal((n, n))
    A = M @ M.T + 0.5 * n * np.eye(n)
    return sp.csr_matrix(A)


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
def test_chebyshev_error_factor_is_scaled_chebyshev_polynomial(degree):
    """On every eigenvector v of D^-1 A (A v = lambda D v) one smoothing step
    multiplies the error by T_m((theta - lambda)/delta) / T_m(theta/delta),
    evaluated here with NumPy's Chebyshev series."""
    rng = np.random.default_rng(degree)
    n = 14
    A = _spd(rng, n)
    lam, V = sla.eigh(A.toarray(), np.diag(A.diagonal()))
    opts = O.Options(cheb_degree=degree, cheb_ratio=4.0, cheb_upper=1.1)
    lv = O.Level(A=A, B=np.ones(n))
    lv.smoother = "chebyshev"
    lv.cheb = O.chebyshev_interval(lam.max(), opts)
    theta, delta, _ = lv.cheb
    xs = rng.standard_normal(n)
    b = A @ xs
    Tm = np.zeros(degree + 1)
    Tm[degree] = 1.0
    for q in range(n):
        e0 = V[:, q]
        x1 = O.smooth(lv, b, xs - e0)
        want = npcheb.chebval((theta - lam[q]) / delta, Tm) / npcheb.chebval(theta / delta, Tm)
        assert np.allclose(xs - x1, want * e0, rtol=1e-9, atol=1e-12)
    # the interval: b = 1.1 rho, a = b / 4
    assert np.isclose(theta + delta, 1.1 * lam.max()) and np.isclose(theta - delta, 1.1 * lam.max() / 4)


def test_chebyshev_degree_one_is_damped_jacobi_with_weight_one_over_theta():
    rng = np.random.default_rng(3)
    A = _spd(rng, 9)
    lv = O.Level(A=A, B=np.ones(9))
    lv.smoother = "chebyshev"
    lv.cheb = (0.8, 0.5, 1)
    b, x = rng.standard_normal(9), rng.standard_normal(9)
    assert np.allclose(O.smooth(lv, b, x), x + (b - A @ x) / A.diagonal() / 0.8, rtol=1e-14)


def _random_pattern_matrix(rng, n, p):
    M = np.triu(rng.random((n, n)) < p, 1)
    M = M | M.T
    vals = np.where(M, -rng.random((n, n)), 0.0)
    vals = (vals + vals.T) / 2
    np.fill_diagonal(vals, np.abs(vals).sum(axis=1) + 1.0)
    A = sp.csr_matrix(vals)
    A.sort_indices()
    return A


def test_colouring_is_proper_and_rounds_equal_first_fit():
    rng = np.random.default_rng(8)
    for trial in range(40):
        n = int(rng.integers(1, 50))
        A = _random_pattern_matrix(rng, n, float(rng.uniform(0.02, 0.3)))
        col = O.color_greedy(A, trial)
        par, _ = O.color_parallel(A, trial)
        assert np.array_equal(col, par)
        rows = np.repeat(np.arange(n), np.diff(A.indptr))
        off = rows != A.indices
        assert np.all(col[rows[off]] != col[A.indices[off]])
        # first fit: a row of colour c has neighbours of every smaller colour
        for i in range(n):
            nb = A.indices[A.indptr[i]:A.indptr[i + 1]]
            assert set(range(col[i])) <= set(col[nb[nb != i]].tolist())


def test_colours_on_grids():
    """A row of a 5-point grid has 4 neighbours, of a 7-point grid 6: first fit
    needs at most 5 and 7 colours."""
    assert O.color_greedy(P.poisson2d(30).to_scipy(), 2).max() + 1 <= 5
    assert O.color_greedy(P.poisson3d(12).to_scipy(), 2).max() + 1 <= 7


def test_sgs_sweep_is_gauss_seidel_in_colour_order():
    """The colour-wise sweeps equal forward then backward Gauss-Seidel on the
    rows sorted by colour: x += (D + L)^-1 (b - A x), then
    x += (D + U)^-1 (b - A x), written as dense triangular solves."""
    rng = np.random.default_rng(12)
    for trial in range(10):
        n = int(rng.integers(5, 60))
        A = _random_pattern_matrix(rng, n, 0.15)
        lv = O.Level(A=A, B=np.ones(n))
        lv.smoother = "mcsgs"
        lv.colors = O.color_greedy(A, trial)
        b, x = rng.standard_normal(n), rng.standard_normal(n)
        perm = np.argsort(lv.colors, kind="stable")
        Ap = A.toarray()[np.ix_(perm, perm)]
        bp, xp = b[perm], x[perm]
        xp = xp + sla.solve_triangular(np.tril(Ap), bp - Ap @ xp, lower=True)
        xp = xp + sla.solve_triangular(np.triu(Ap), bp - Ap @ xp, lower=False)
        want = np.empty(n)
        want[perm] = xp
        assert np.allclose(O.smooth(lv, b, x), want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("smoother,kw", [("chebyshev", {}), ("chebyshev", {"cheb_degree": 3}), ("mcsgs", {})])
def test_smoothers_converge_and_beat_jacobi(smoother, kw):
    A = P.hetero3d(16, seed=5)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    ref = O.solve(O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(3)), b, 1e-8)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(3, smoother=smoother, **kw))
    res = O.solve(H, b, 1e-8)
    assert res.converged and res.relres <= 1e-8
    assert res.iters < ref.iters
