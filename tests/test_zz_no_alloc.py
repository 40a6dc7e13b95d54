"""amg_galerkin_noalloc (the Galerkin product of Section 3.1 with its scratch in
a static device array) against amg_galerkin, the entry point that allocates,
through the C ABI: identical row pointers, columns and values, on two calls in
a row (the second on a smaller input, so stale contents of the shared array
would show), plus the oracle's product to 1e-12 and the capacity and size
limits."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import dev_vec, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")


def _tiered_case():
    """Coarse rows of every reduce tier (a few terms, up to 512, beyond 512)."""
    rng = np.random.default_rng(9)
    n = 4000
    M = sp.random(n, n, density=6.0 / n, random_state=rng)
    M = M + M.T + sp.identity(n) * 20
    S = M.tocsr()
    S.sort_indices()
    sizes = np.concatenate([np.ones(300, int), rng.integers(2, 12, 150), rng.integers(30, 60, 20),
                            rng.integers(100, 121, 6)])
    sizes = sizes[np.cumsum(sizes) <= n]
    sizes[-1] += n - sizes.sum()
    nc = len(sizes)
    agg = rng.permutation(np.repeat(np.arange(nc), sizes)).astype(np.int32)
    pval = rng.uniform(0.5, 1.5, n)
    return S, agg, pval, nc


def _poisson_case():
    """Level 0 of a 2-D Poisson hierarchy: the GPU's own aggregates and P."""
    A = P.poisson2d(40, 30)
    rp, ci, v = to_dev(A)
    h = amg.setup(rp, ci, v, amg.Options(dim=2))
    ex = h.export_level(0, what=("agg", "pval"))
    nc = h.level_info(0)["nc"]
    h.close()
    return A.to_scipy(), ex["agg"].astype(np.int32), ex["pval"], nc


def _both(S, agg, pval, nc):
    A = P.CSR(S.indptr, S.indices, S.data)
    rp, ci, v = to_dev(A)
    ag, pv = torch.from_numpy(agg).cuda(), dev_vec(pval)
    print(f"galerkin_noalloc: n={A.n} nnz={A.nnz} nc={nc}", flush=True)
    want_rp, want_ci, want_v = amg.galerkin(rp, ci, v, ag, pv, nc)
    grp, gci, gv, nnz_c = amg.galerkin_noalloc(rp, ci, v, ag, pv, nc)
    torch.cuda.synchronize()
    got_rp = grp.cpu().numpy()
    got_ci = gci[:nnz_c].cpu().numpy()
    got_v = gv[:nnz_c].cpu().numpy()
    return (want_rp, want_ci, want_v), (got_rp, got_ci, got_v, nnz_c)


def test_noalloc_matches_allocating_entry_twice():
    for S, agg, pval, nc in (_tiered_case(), _poisson_case()):   # second call: smaller input
        (want_rp, want_ci, want_v), (got_rp, got_ci, got_v, nnz_c) = _both(S, agg, pval, nc)
        assert nnz_c == len(want_ci)
        assert np.array_equal(got_rp, want_rp)
        assert np.array_equal(got_ci, want_ci)
        assert np.array_equal(got_v, want_v)   # same kernels, same summation order
        ref = O.galerkin(S, agg.astype(np.int64), pval, nc)
        assert np.array_equal(got_rp, ref.indptr) and np.array_equal(got_ci, ref.indices)
        assert np.allclose(got_v, ref.data, rtol=1e-12, atol=1e-12 * np.abs(ref.data).max())


def test_noalloc_capacity_and_limits():
    S, agg, pval, nc = _poisson_case()
    A = P.CSR(S.indptr, S.indices, S.data)
    rp, ci, v = to_dev(A)
    ag, pv = torch.from_numpy(agg).cuda(), dev_vec(pval)
    want_rp, want_ci, want_v = amg.galerkin(rp, ci, v, ag, pv, nc)
    with pytest.raises(amg.AmgError) as e:
        amg.galerkin_noalloc(rp, ci, v, ag, pv, nc, cap=len(want_ci) - 1)
    assert e.value.code == amg.binding.AMG_EINVAL
    # exactly enough room: the product is complete
    grp, gci, gv, nnz_c = amg.galerkin_noalloc(rp, ci, v, ag, pv, nc, cap=len(want_ci))
    assert nnz_c == len(want_ci)
    assert np.array_equal(gci.cpu().numpy(), want_ci) and np.array_equal(gv.cpu().numpy(), want_v)
    # an aggregate index outside [0, nc) is refused by the device checks
    bad = agg.copy()
    bad[3] = nc
    with pytest.raises(amg.AmgError) as e:
        amg.galerkin_noalloc(rp, ci, v, torch.from_numpy(bad).cuda(), pv, nc)
    assert e.value.code == amg.binding.AMG_EINVAL
    # beyond the array's row limit: refused before any device work
    big = P.poisson2d(400)   # 160,000 rows > 131,072
    brp, bci, bv = to_dev(big)
    with pytest.raises(amg.AmgError) as e:
        amg.galerkin_noalloc(brp, bci, bv, torch.zeros(big.n, dtype=torch.int32, device="cuda"),
                             torch.ones(big.n, dtype=torch.float64, device="cuda"), 1)
    assert e.value.code == amg.binding.AMG_EINVAL
    # and the shared array still serves a correct call afterwards
    grp, gci, gv, nnz_c = amg.galerkin_noalloc(rp, ci, v, ag, pv, nc)
    assert np.array_equal(gci[:nnz_c].cpu().numpy(), want_ci) and np.array_equal(gv[:nnz_c].cpu().numpy(), want_v)
