"""Numeric re-setup on a fixed pattern (amg_resetup; Section 3.1, the Galerkin
product's indices reused when only A_0's values change) against the oracle's
resetup, through the C ABI.

Bars: aggregates and MIS(2) state unchanged; every A_{k+1} equal to the
oracle's Galerkin product of the GPU's exported A_k with the kept P_k (pattern
exact, values within 1e-12 of the magnitude of their summed terms); omega_k
within 1e-12 of the oracle's Arnoldi estimate on the same A_k; the solve
against the oracle's re-set-up hierarchy (true relres <= 1e-8, iterations
within one, x within 1e-6)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import dev_vec, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")


def _export_all(h):
    return [h.export_level(k) if k + 1 < h.num_levels() else h.export_level(k, what=("A",))
            for k in range(h.num_levels())]


def _galerkin_bound(A, agg, pval, nc, tol=1e-12):
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    mag = np.abs(pval[rows] * A.data * pval[A.indices])
    M = sp.csr_matrix((mag, (agg[rows], agg[A.indices])), shape=(nc, nc))
    M.sum_duplicates()
    M.sort_indices()
    return tol * M.data + 1e-300


def _check_levels(h, before, opts):
    after = _export_all(h)
    for k in range(h.num_levels() - 1):
        ex, nxt, old = after[k], after[k + 1], before[k]
        assert np.array_equal(ex["agg"], old["agg"]) and np.array_equal(ex["state"], old["state"])
        assert np.array_equal(ex["strong"], old["strong"])
        assert np.array_equal(ex["pval"], old["pval"])
        A = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
        agg = ex["agg"].astype(np.int64)
        nc = int(agg.max()) + 1
        Ac = O.galerkin(A, agg, ex["pval"], nc)
        assert np.array_equal(nxt["row_ptr"], Ac.indptr) and np.array_equal(nxt["col"], Ac.indices)
        err = np.abs(nxt["val"] - Ac.data)
        bound = _galerkin_bound(A, agg, ex["pval"], nc)
        assert np.all(err <= bound), f"level {k + 1}: max ratio {np.max(err / bound):.3g}"
        om, _ = O.jacobi_weight(A, opts.arnoldi_m, opts.seed + 1, opts.jacobi_scale)
        assert abs(h.level_info(k)["omega"] - om) <= 1e-12 * om
    return after


@pytest.mark.parametrize("borrow", [False, True], ids=["copied", "borrowed"])
def test_resetup_new_values_against_oracle(borrow):
    A = P.hetero3d(20, seed=11)
    A2 = P.hetero3d(20, seed=12)          # same pattern, new coefficients
    assert np.array_equal(A.col, A2.col) and np.array_equal(A.row_ptr, A2.row_ptr)
    rp, ci, v = to_dev(A)
    opts = amg.Options(dim=3, flags=amg.binding.FLAG_BORROW_A if borrow else 0)
    h = amg.setup(rp, ci, v, opts)
    before = _export_all(h)
    v2 = dev_vec(A2.val)
    print(f"resetup: n={A.n} levels={h.num_levels()} borrow={borrow}", flush=True)
    h.resetup(v2)
    oo = O.Options.for_dim(3)
    after = _check_levels(h, before, oo)
    assert np.array_equal(after[0]["val"], A2.val)
    # the solve against the oracle's resetup of its own (identical) aggregation
    H = O.setup(A.row_ptr, A.col, A.val, oo)
    for k in range(H.L):
        assert np.array_equal(H.levels[k].agg, before[k]["agg"].astype(np.int64))
    R = O.resetup(H, A2.val)
    b = P.rhs(A2, P.exact_solution(A2.n, 1))
    x, it, rel = amg.solve(h, torch.from_numpy(b).cuda(), 1e-8)
    ref = O.solve(R, b, 1e-8)
    xh = x.cpu().numpy()
    true_rel = np.linalg.norm(b - A2.to_scipy() @ xh) / np.linalg.norm(b)
    assert rel <= 1e-8 and true_rel <= 1.01e-8 and ref.relres <= 1e-8
    assert abs(it - ref.iters) <= 1, (it, ref.iters)
    if it == ref.iters:
        assert np.linalg.norm(xh - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    h.close()


def _row_terms(ex_fine):
    """Number of Galerkin terms of every coarse row: the stored entries of its
    aggregate's member rows."""
    lens = np.diff(ex_fine["row_ptr"])
    return np.bincount(ex_fine["agg"], weights=lens).astype(np.int64)


def test_resetup_back_to_the_setup_values_is_exact():
    """Replaying the first values reproduces the setup's coarse matrices bit
    for bit on every coarse row of at most 512 terms (the rows the setup's
    wave reduce sums in segment order, as the replay does; longer rows are
    summed by a block reduction there and agree to rounding), and the solve
    then takes the same iterations as a fresh setup."""
    A = P.poisson3d(22)
    A2 = P.CSR(A.row_ptr, A.col, A.val * np.where(np.arange(A.nnz) % 3 == 0, 1.25, 1.0))
    S2 = A2.to_scipy()
    M = ((S2 + S2.T) * 0.5).tocsr()   # symmetric again, same pattern
    M.sort_indices()
    assert np.array_equal(M.indptr, A.row_ptr) and np.array_equal(M.indices, A.col)
    A2 = P.CSR(A.row_ptr, A.col, M.data)
    rp, ci, v = to_dev(A)
    h = amg.setup(rp, ci, v, amg.Options(dim=3))
    before = _export_all(h)
    om0 = [h.level_info(k)["omega"] for k in range(h.num_levels() - 1)]
    h.resetup(dev_vec(A2.val))
    mid = _export_all(h)
    assert any(not np.array_equal(m["val"], b["val"]) for m, b in zip(mid[1:], before[1:]))
    h.resetup(dev_vec(A.val))
    again = _export_all(h)
    assert np.array_equal(before[0]["val"], again[0]["val"])
    exact_levels = True
    for k in range(1, len(before)):
        a, b = before[k], again[k]
        assert np.array_equal(a["row_ptr"], b["row_ptr"]) and np.array_equal(a["col"], b["col"])
        terms = _row_terms(before[k - 1])
        row_of = np.repeat(np.arange(len(a["row_ptr"]) - 1), np.diff(a["row_ptr"]))
        short = terms[row_of] <= 512
        assert np.array_equal(a["val"][short], b["val"][short]), f"level {k}: a replayed short row differs"
        d = np.abs(a["val"][~short] - b["val"][~short])
        assert np.all(d <= 1e-13 * np.abs(a["val"][~short]).max(initial=0.0)), f"level {k}"
        exact_levels = exact_levels and bool(short.all())
    om = [h.level_info(k)["omega"] for k in range(h.num_levels() - 1)]
    if exact_levels:
        assert om == om0
    assert np.allclose(om, om0, rtol=1e-13, atol=0)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    _, it, rel = amg.solve(h, torch.from_numpy(b).cuda(), 1e-8)
    h2 = amg.setup(rp, ci, v, amg.Options(dim=3))
    _, it2, rel2 = amg.solve(h2, torch.from_numpy(b).cuda(), 1e-8)
    assert it == it2 and rel <= 1e-8 and abs(rel - rel2) <= 1e-3 * rel2
    h.close()
    h2.close()


def test_resetup_mixed_precision_converges():
    A = P.hetero3d(16, seed=3)
    A2 = P.hetero3d(16, seed=4)
    rp, ci, v = to_dev(A)
    h = amg.setup(rp, ci, v, amg.Options(dim=3, precision="mixed"))
    h64 = amg.setup(rp, ci, v, amg.Options(dim=3))
    h.resetup(dev_vec(A2.val))
    h64.resetup(dev_vec(A2.val))
    b = P.rhs(A2, P.exact_solution(A2.n, 1))
    x, it, rel = amg.solve(h, torch.from_numpy(b).cuda(), 1e-8)
    x64, it64, rel64 = amg.solve(h64, torch.from_numpy(b).cuda(), 1e-8)
    xh = x.cpu().numpy()
    assert rel <= 1e-8 and np.linalg.norm(b - A2.to_scipy() @ xh) <= 1.01e-8 * np.linalg.norm(b)
    assert abs(it - it64) <= 1, (it, it64)
    h.close()
    h64.close()


def test_resetup_errors():
    A = P.poisson2d(40)
    rp, ci, v = to_dev(A)
    h = amg.setup(rp, ci, v, amg.Options(dim=2))
    bad = A.val.copy()
    bad[A.row_ptr[5] + 1] = np.nan
    with pytest.raises(amg.AmgError) as e:
        h.resetup(dev_vec(bad))
    assert e.value.code in (amg.binding.AMG_ENANINF, amg.binding.AMG_EINVAL)
    h.close()
    mats = [P.poisson2d(20), P.poisson2d(24)]
    Abd, off = P.block_diag(mats)
    rp, ci, v = to_dev(Abd)
    hb = amg.setup_batched(rp, ci, v, off, amg.Options(dim=2))
    with pytest.raises(amg.AmgError) as e:
        hb.resetup(v)
    assert e.value.code == amg.binding.AMG_EUNSUPPORTED
    hb.close()
