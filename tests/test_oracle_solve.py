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


def _three_level(krylov="fcg", kcycle_levels=1, t=0.25):
    A = P.poisson2d(48)
    H = O.setup(A.row_ptr, A.col, A.val,
                O.Options.for_dim(2, coarse_max=40, krylov=krylov, kcycle_levels=kcycle_levels, kcycle_t=t))
    assert H.L >= 2, "the K-cycle pin needs inner cycles on a level that is not the coarsest"
    return H


def _first_step(H, rc, cg):
    """c = one inner cycle on level 1 and what the best multiple of c leaves,
    written from the definition of the minimiser along c."""
    A1 = H.levels[1].A.toarray()
    c = O.cycle(H, 1, rc)
    if cg:   # argmin_a ||A1^-1 rc - a c||_A1: a = c'rc / c'A1 c
        a = (c @ rc) / (c @ A1 @ c)
    else:    # argmin_a ||rc - a A1 c||_2
        a = ((A1 @ c) @ rc) / ((A1 @ c) @ (A1 @ c))
    return A1, c, a, rc - a * (A1 @ c)


@pytest.mark.parametrize("krylov", ["fcg", "fgmres"])
def test_kcycle_correction_is_minimiser_over_two_inner_cycles(krylov):
    """With t = 0 the K-cycle always takes the second inner step; its coarse
    correction is then the minimiser over span{c, d} (A_1-norm error for CG,
    residual 2-norm for GMRES), solved here as a dense 2x2 Gram / least-squares
    system from the two inner cycles computed independently."""
    cg = krylov == "fcg"
    H = _three_level(krylov, t=0.0)
    rc = np.random.default_rng(11).standard_normal(H.levels[1].n)
    A1, c, _a, rt = _first_step(H, rc, cg)
    d = O.cycle(H, 1, rt)
    if cg:
        G = np.array([[c @ A1 @ c, c @ A1 @ d], [d @ A1 @ c, d @ A1 @ d]])
        y = np.linalg.solve(G, np.array([c @ rc, d @ rc]))
    else:
        y, *_ = np.linalg.lstsq(np.stack([A1 @ c, A1 @ d], 1), rc, rcond=None)
    e, steps = O.kcycle_correction(H, 1, rc)
    assert steps == 2
    want = y[0] * c + y[1] * d
    assert np.linalg.norm(e - want) <= 1e-10 * np.linalg.norm(want)
    # and it is a minimiser: the error (CG) or residual (GMRES) is orthogonal to the space
    res = rc - A1 @ e
    basis = (c, d) if cg else (A1 @ c, A1 @ d)
    for u in basis:
        assert abs(u @ res) <= 1e-10 * np.linalg.norm(u) * np.linalg.norm(rc)


@pytest.mark.parametrize("krylov", ["fcg", "fgmres"])
def test_kcycle_second_step_threshold(krylov):
    """The second inner step runs exactly when ||r~|| > t ||rc||: just above
    the measured ratio the correction is the best multiple of c, just below it
    the two-step minimiser."""
    cg = krylov == "fcg"
    H0 = _three_level(krylov)
    rc = np.random.default_rng(12).standard_normal(H0.levels[1].n)
    _A1, c, a, rt = _first_step(H0, rc, cg)
    q = np.linalg.norm(rt) / np.linalg.norm(rc)
    assert 0.0 < q < 1.0
    H0.opts.kcycle_t = q * 1.001
    e, steps = O.kcycle_correction(H0, 1, rc)
    assert steps == 1 and np.allclose(e, a * c, rtol=1e-12, atol=0)
    H0.opts.kcycle_t = q * 0.999
    e2, steps2 = O.kcycle_correction(H0, 1, rc)
    assert steps2 == 2 and not np.allclose(e2, a * c, rtol=1e-6)


def test_kcycle_nested_levels_and_v_only():
    """kcycle_levels = 0 makes cycle() the V-cycle everywhere; with two
    K-levels the level-0 cycle uses the level-1 K-cycle inside, and the
    resulting preconditioned solve still converges."""
    H = _three_level(kcycle_levels=0)
    b = np.random.default_rng(13).standard_normal(H.levels[0].n)
    assert np.array_equal(O.cycle(H, 0, b), O.vcycle(H, 0, b))
    H2 = _three_level(kcycle_levels=2)
    A = H2.levels[0].A
    res = O.solve(H2, b, rtol=1e-10)
    assert res.converged and np.linalg.norm(b - A @ res.x) <= 1e-10 * np.linalg.norm(b)


def test_kcycle_coefficients_guard_keeps_first_step():
    """rho2 <= 0 (d adds nothing: d parallel to c) keeps alpha1/rho1 c."""
    rng = np.random.default_rng(4)
    n = 12
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    r, c = rng.standard_normal(n), rng.standard_normal(n)
    d = 2.0 * c
    v, w = A @ c, A @ d
    rt = r - (c @ r) / (c @ v) * v
    cc, cd = O.kcycle_coefficients(c, d, v, w, r, rt, "cg")
    assert cd == 0.0 and cc == (c @ r) / (c @ v)
