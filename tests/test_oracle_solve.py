"""CPU pins of the oracle's solve phase (Algorithms 4 and 5, outer Krylov).

Pins: the K-cycle's two-step update against the exact 2-D minimiser over
span{c, d}; flexible CG against a textbook PCG when the preconditioner is a
fixed symmetric V-cycle; the coarse solve against a dense solver; end-to-end
convergence to the true relative residual.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg_oracle as O
from synthetic import problems as P


def test_kcycle_cg_update_is_A_norm_minimiser():
    rng = np.random.default_rng(1)
    for _ in range(20):
        n = 30
        M = rng.standard_normal((n, n))
        A = M @ M.T + n * np.eye(n)
        r = rng.standard_normal(n)
        c, d = rng.standard_normal(n), rng.standard_normal(n)
        v = A @ c
        rho1, alpha1 = c @ v, c @ r
        rt = r - alpha1 / rho1 * v
        w = A @ d
        cc, cd = O.kcycle_coefficients(c, d, v, w, r, rt, "cg")
        G = np.array([[c @ A @ c, c @ A @ d], [d @ A @ c, d @ A @ d]])
        want = np.linalg.solve(G, np.array([c @ r, d @ r]))
        assert np.allclose([cc, cd], want, rtol=1e-10)


def test_kcycle_gmres_update_is_least_squares_minimiser():
    rng = np.random.default_rng(2)
    for _ in range(20):
        n = 30
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        r = rng.standard_normal(n)
        c, d = rng.standard_normal(n), rng.standard_normal(n)
        v, w = A @ c, A @ d
        rho1, alpha1 = v @ v, v @ r
        rt = r - alpha1 / rho1 * v
        cc, cd = O.kcycle_coefficients(c, d, v, w, r, rt, "gmres")
        want, *_ = np.linalg.lstsq(np.stack([v, w], 1), r, rcond=None)
        assert np.allclose([cc, cd], want, rtol=1e-10)


def test_coarse_solve_matches_dense_solver():
    A = P.poisson2d(20)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2, coarse_max=600))
    assert H.L == 0 and H.coarse_kind == "cholesky"
    b = np.random.default_rng(0).standard_normal(A.n)
    x = H.coarse_solve(b)
    Ad = A.to_scipy().toarray()
    assert np.linalg.norm(Ad @ x - b) <= 1e-13 * np.linalg.norm(Ad, 2) * np.linalg.norm(x)
    assert np.allclose(x, np.linalg.solve(Ad, b), rtol=1e-12, atol=1e-13)


def _textbook_pcg(A, b, M, iters):
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    hist = []
    for _ in range(iters):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        hist.append(np.linalg.norm(r) / np.linalg.norm(b))
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return hist


def test_fcg_with_vcycle_equals_textbook_pcg():
    """With V-cycles only (a fixed symmetric preconditioner) flexible CG is PCG."""
    A = P.poisson2d(64)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2, kcycle_levels=0))
    b = P.rhs(A, P.exact_solution(A.n, 1))
    res = O.solve(H, b, rtol=1e-10)
    pcg = _textbook_pcg(H.levels[0].A, b, lambda r: O.cycle(H, 0, r), len(res.history))
    k = min(len(pcg), 12)
    assert np.allclose(res.history[:k], pcg[:k], rtol=1e-6)


def test_vcycle_is_symmetric_operator():
    A = P.poisson2d(40)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2, kcycle_levels=0, coarse_max=100))
    rng = np.random.default_rng(3)
    u, w = rng.standard_normal(A.n), rng.standard_normal(A.n)
    lhs = u @ O.cycle(H, 0, w)
    rhs = w @ O.cycle(H, 0, u)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("krylov", ["fcg", "fgmres"])
def test_end_to_end_2d_poisson_128(krylov):
    A = P.poisson2d(128)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2, krylov=krylov))
    xs = P.exact_solution(A.n, 1)
    b = P.rhs(A, xs)
    res = O.solve(H, b, rtol=1e-8)
    assert res.converged and res.relres <= 1e-8
    assert res.iters <= 30
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-5


def test_end_to_end_heterogeneous_3d():
    A = P.hetero3d(20, seed=5)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(3))
    b = P.rhs(A, P.exact_solution(A.n, 1))
    res = O.solve(H, b, rtol=1e-8)
    assert res.converged and res.relres <= 1e-8 and res.iters <= 40


def test_fgmres_nonsymmetric_convection_diffusion():
    """GMRES path (K-cycle GMRES variant, LU coarse factor) on an upwinded
    convection-diffusion operator."""
    n = 48
    A = P.poisson2d(n).to_scipy().tolil()
    for i in range(n * n):
        if i % n:
            A[i, i - 1] -= 0.8
            A[i, i] += 0.8
    A = A.tocsr()
    A.sort_indices()
    H = O.setup(A.indptr, A.indices, A.data, O.Options.for_dim(2, krylov="fgmres", coarse_max=100))
    assert H.coarse_kind == "lu"
    b = A @ P.exact_solution(A.shape[0], 1)
    res = O.solve(H, b, rtol=1e-8)
    assert res.converged and res.relres <= 1e-8


def test_zero_rhs_and_nonfinite_rhs():
    A = P.poisson2d(16)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2, coarse_max=50))
    res = O.solve(H, np.zeros(A.n))
    assert res.iters == 0 and np.all(res.x == 0)
    b = np.ones(A.n)
    b[5] = np.inf
    with pytest.raises(O.OracleError):
        O.solve(H, b)


def test_max_iter_reports_not_converged():
    A = P.poisson2d(64)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2))
    res = O.solve(H, P.rhs(A, P.exact_solution(A.n, 1)), rtol=1e-8, max_iter=1)
    assert not res.converged and res.iters == 1


def test_batch_equals_individual_solves():
    mats = [P.poisson2d(s) for s in (20, 33, 27)]
    Abd, off = P.block_diag(mats)
    b = P.rhs(Abd, P.exact_solution(Abd.n, 1))
    opts = O.Options.for_dim(2, coarse_max=60)
    out = O.solve_batch(Abd.row_ptr, Abd.col, Abd.val, off, b, opts)
    for s, m in enumerate(mats):
        H = O.setup(m.row_ptr, m.col, m.val, opts)
        ref = O.solve(H, b[off[s]:off[s + 1]])
        assert out[s].iters == ref.iters and np.array_equal(out[s].x, ref.x)
