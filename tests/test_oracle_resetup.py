"""Pins of the oracle's numeric re-setup on a fixed pattern (Section 3.1:
the Galerkin product's indices reused when only the values of A_0 change)."""
import numpy as np
import scipy.sparse as sp

from oracle import amg_oracle as O
from synthetic import problems as P


def _perturbed(A, seed, amp=0.3):
    """The same pattern with new symmetric values: a_ij *= 1 + amp u_ij
    (u symmetric in [0, 1)), the diagonal reset to keep every row dominant."""
    S = A.to_scipy().tocoo()
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, S.nnz)
    key_lo = np.minimum(S.row, S.col).astype(np.int64) * A.n + np.maximum(S.row, S.col)
    _, inv = np.unique(key_lo, return_inverse=True)
    w = rng.uniform(0.0, 1.0, inv.max() + 1)[inv]      # one factor per unordered pair
    data = S.data * (1.0 + amp * w)
    off = S.row != S.col
    T = sp.csr_matrix((np.where(off, data, 0.0), (S.row, S.col)), shape=S.shape)
    rowsum = -np.asarray(T.sum(axis=1)).ravel()
    data = np.where(off, data, rowsum[S.row] * (1.0 + 0.05 * u))
    M = sp.csr_matrix((data, (S.row, S.col)), shape=S.shape)
    M.sort_indices()
    assert np.array_equal(M.indptr, A.row_ptr) and np.array_equal(M.indices, A.col)
    return M.data


def test_resetup_with_the_same_values_reproduces_setup():
    A = P.poisson2d(30, 23)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2))
    R = O.resetup(H, A.val)
    assert R.L == H.L
    for a, b in zip(H.levels, R.levels):
        assert np.array_equal(a.A.data, b.A.data) and np.array_equal(a.A.indices, b.A.indices)
    for a, b in zip(H.levels[:-1], R.levels[:-1]):
        assert a.omega == b.omega and np.array_equal(a.agg, b.agg)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    r1, r2 = O.solve(H, b, 1e-8), O.solve(R, b, 1e-8)
    assert r1.iters == r2.iters and np.array_equal(r1.x, r2.x)


def test_resetup_scaling_by_two_is_exact():
    """2 A: every Galerkin term (P_i 2a_ij) P_j is exactly twice the old one,
    D^-1 A and so omega are unchanged, bit for bit."""
    A = P.hetero3d(9, seed=4)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(3))
    R = O.resetup(H, 2.0 * A.val)
    for a, b in zip(H.levels, R.levels):
        assert np.array_equal(2.0 * a.A.data, b.A.data)
    for a, b in zip(H.levels[:-1], R.levels[:-1]):
        assert a.omega == b.omega


def test_resetup_is_the_galerkin_product_of_the_fixed_p():
    """New values on the same pattern: the aggregates and P stay those of the
    first setup, every coarse matrix equals the dense P^T A_k P, the Jacobi
    estimate brackets rho(D^-1 A_k) as on any level, and the solve converges."""
    A = P.poisson2d(24, 17)
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(2))
    val = _perturbed(A, 5)
    R = O.resetup(H, val)
    assert np.array_equal(R.levels[0].A.data, val)
    for k, (old, lv) in enumerate(zip(H.levels[:-1], R.levels[:-1])):
        assert np.array_equal(lv.agg, old.agg) and np.array_equal(lv.pval, old.pval)
        Pd = np.zeros((lv.n, lv.nc))
        Pd[np.arange(lv.n), lv.agg] = lv.pval
        dense = Pd.T @ lv.A.toarray() @ Pd
        Ac = R.levels[k + 1].A.toarray()
        assert np.allclose(Ac, dense, rtol=0, atol=1e-13 * np.abs(dense).max())
        # the stored pattern keeps every structural (I, J), as the first setup
        assert np.array_equal(R.levels[k + 1].A.indices, H.levels[k + 1].A.indices)
        DA = lv.A.toarray() / lv.A.diagonal()[:, None]
        rho = np.max(np.abs(np.linalg.eigvals(DA)))
        assert 0.9 * rho <= lv.rho <= rho * (1 + 1e-12)
        assert not np.array_equal(lv.A.data, old.A.data)
    b = P.exact_solution(A.n, 1)
    res = O.solve(R, b, 1e-8)
    Anew = sp.csr_matrix((val, A.col, A.row_ptr), shape=(A.n, A.n))
    assert res.converged and np.linalg.norm(b - Anew @ res.x) <= 1e-8 * np.linalg.norm(b) * 1.0001
