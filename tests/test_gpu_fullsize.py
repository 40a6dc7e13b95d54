"""GPU parity at the full size of the headline workload (3-D 7-point Poisson
128^3, n = 2,097,152, nnz = 14,581,760), in the configuration the benchmark
times: FP64, K-cycle FCG, autotuned level kernels.

Every level the GPU builds is re-coarsened by the oracle from the GPU's own
exported A_k and B_k (strength mask, MIS(2) state and aggregates bit-exact;
A_{k+1} to 1e-12; omega to 1e-12), the level-0 sliced-ELL products (32-bit
columns and 16-bit offsets) are compared entry by entry with a CSR product,
and the solve is compared with the oracle's own full setup and solve.
"""
import numpy as np
import pytest

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import compare_level, dev_vec, oracle_level, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")


@pytest.fixture(scope="module")
def c2():
    A, dim, _ = P.config("C2")
    assert (A.n, int(A.row_ptr[-1])) == (2097152, 14581760)
    rp, ci, v = to_dev(A)
    h = amg.setup(rp, ci, v, amg.Options(dim=dim))
    return A, dim, (rp, ci, v), h


def test_c2_levels_match_oracle(c2):
    A, dim, _, h = c2
    oo = O.Options.for_dim(dim)
    L = h.num_levels()
    assert L >= 3
    for k in range(L - 1):
        ex = h.export_level(k)
        nxt = h.export_level(k + 1, what=("A", "B"))
        if k == 0:
            assert np.array_equal(ex["col"], A.col) and np.array_equal(ex["val"], A.val)
        lv = oracle_level(ex, oo)
        compare_level(ex, lv, nxt)
        assert np.allclose(nxt["B"], lv.Bc, rtol=1e-14, atol=0)
        omega, _ = O.jacobi_weight(lv.A, oo.arnoldi_m, oo.seed + 1, oo.jacobi_scale)
        assert abs(ex["omega"] - omega) <= 1e-12 * omega
        assert ex["mis_rounds"] == lv.mis_rounds
    assert h.export_level(L - 1, what=("A",))["n"] <= 600


@pytest.mark.parametrize("lanes", [-1, -2, 0])
def test_c2_level0_products_entrywise(c2, lanes):
    A, _, dev, _ = c2
    x = P.exact_solution(A.n, 7)
    y = amg.spmv(*dev, dev_vec(x), lanes_per_row=lanes).cpu().numpy()
    S = A.to_scipy()
    bound = 1e-15 * 8 * (abs(S) @ np.abs(x))
    assert np.all(np.abs(y - S @ x) <= bound)


def test_c2_tuned_level0_product_entrywise(c2):
    A, _, _, h = c2
    x = P.exact_solution(A.n, 9)
    y = h.level_spmv(0, dev_vec(x)).cpu().numpy()
    S = A.to_scipy()
    assert np.all(np.abs(y - S @ x) <= 1e-15 * 8 * (abs(S) @ np.abs(x)))


def test_c2_solve_matches_oracle(c2):
    A, dim, _, h = c2
    b = P.rhs(A, P.exact_solution(A.n, 1))
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8
    assert np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b) <= 1.01e-8
    ref = O.solve(O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(dim)), b, 1e-8)
    assert ref.relres <= 1e-8 and abs(it - ref.iters) <= 1
    if it == ref.iters:   # the same iteration on both sides, up to rounding
        assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e-6


# ---------------------------------------------------------------- C3
# 3-D heterogeneous finite-volume diffusion on 160^3 cells (k = exp(2g), seed 2),
# n = 4,096,000, nnz = 28,518,400: the largest single system, in the
# configuration the benchmark times.

@pytest.fixture(scope="module")
def c3():
    A, dim, _ = P.config("C3")
    assert (A.n, int(A.row_ptr[-1])) == (4096000, 28518400)
    rp, ci, v = to_dev(A)
    print(f"C3 full size: n={A.n} nnz={A.nnz}", flush=True)
    h = amg.setup(rp, ci, v, amg.Options(dim=dim))
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(dim))
    return A, dim, (rp, ci, v), h, H


def test_c3_levels_match_oracle(c3):
    A, dim, _, h, _ = c3
    oo = O.Options.for_dim(dim)
    L = h.num_levels()
    assert L >= 3
    for k in range(L - 1):
        ex = h.export_level(k)
        nxt = h.export_level(k + 1, what=("A", "B"))
        if k == 0:
            assert np.array_equal(ex["col"], A.col) and np.array_equal(ex["val"], A.val)
        lv = oracle_level(ex, oo)
        compare_level(ex, lv, nxt)
        assert np.allclose(nxt["B"], lv.Bc, rtol=1e-14, atol=0)
        omega, _ = O.jacobi_weight(lv.A, oo.arnoldi_m, oo.seed + 1, oo.jacobi_scale)
        assert abs(ex["omega"] - omega) <= 1e-12 * omega
        assert ex["mis_rounds"] == lv.mis_rounds


def test_c3_hierarchy_equals_oracle_setup(c3):
    """The oracle's own full setup builds the same hierarchy (level sizes and
    aggregates of every level) as the GPU."""
    _, _, _, h, H = c3
    assert h.num_levels() == len(H.levels)
    for k in range(h.num_levels() - 1):
        ex = h.export_level(k, what=("agg",))
        assert np.array_equal(ex["agg"].astype(np.int64), H.levels[k].agg), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c3_solve_matches_oracle(c3, precision):
    """FP64 and mixed (FP32 cycle, FP64 outer) solves against the oracle's FP64
    setup and solve: true relres <= 1e-8 on the host, iterations within one."""
    A, dim, dev, h64, H = c3
    h = h64 if precision == "fp64" else amg.setup(*dev, amg.Options(dim=dim, precision="mixed"))
    b = P.rhs(A, P.exact_solution(A.n, 1))
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8
    assert np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b) <= 1.01e-8
    ref = O.solve(H, b, 1e-8)
    assert ref.relres <= 1e-8 and abs(it - ref.iters) <= 1, (it, ref.iters)
    if it == ref.iters:
        assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e-6
    if h is not h64:
        h.close()


# ---------------------------------------------------------------- C4a
def test_c4a_full_size_multi_rhs_mixed():
    """3-D anisotropic 96^3 (eps_z = 1e-3) with 32 right-hand sides in one
    mixed-precision block solve: every column's true residual on the host, two
    columns against the oracle's solve."""
    A = P.aniso3d(96, 1e-3)
    assert (A.n, A.nnz) == (884736, 6137856)
    rp, ci, v = to_dev(A)
    print(f"C4a full size: n={A.n} R=32", flush=True)
    h = amg.setup(rp, ci, v, amg.Options(dim=3, precision="mixed"))
    X0 = P.multi_exact_solution(A.n, 32, 1)
    B = np.ascontiguousarray(P.rhs(A, X0))
    X, its, rels = amg.solve_multi(h, torch.from_numpy(B).cuda(), 1e-8)
    X = X.cpu().numpy()
    S = A.to_scipy()
    R = B - S @ X
    for c in range(32):
        assert rels[c] <= 1e-8
        assert np.linalg.norm(R[:, c]) <= 1.01e-8 * np.linalg.norm(B[:, c]), c
    H = O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(3))
    for c in (0, 31):
        ref = O.solve(H, B[:, c], 1e-8)
        assert ref.relres <= 1e-8 and abs(int(its[c]) - ref.iters) <= 1, (c, its[c], ref.iters)
        if int(its[c]) == ref.iters:
            assert np.linalg.norm(X[:, c] - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    h.close()
