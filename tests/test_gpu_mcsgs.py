"""Multi-colour symmetric Gauss-Seidel smoothing (Section 2.2.1) in the GPU
cycle against the oracle's, through the C ABI: the colouring of every level
bit-exact against the oracle's sequential first-fit colouring of the GPU's
exported A_k (same node-hash priorities), a proper colouring (no two coupled
rows share a colour), and the solve (iterations within one, true relres <=
1e-8, x within 1e-6 when the counts agree), FP64 and mixed."""
import numpy as np
import pytest

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import dev_vec, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")

CASES = [
    ("poisson2d_64x47", lambda: P.poisson2d(64, 47), 2),
    ("hetero3d_18", lambda: P.hetero3d(18, seed=11), 3),
    ("aniso2d_60", lambda: P.aniso2d(60, 1e-3), 2),
]


@pytest.mark.parametrize("name,make,dim", CASES, ids=[c[0] for c in CASES])
def test_mcsgs_colors_and_solve_match_oracle(name, make, dim):
    A = make()
    rp, ci, v = to_dev(A)
    print(f"mcsgs: {name}", flush=True)
    h = amg.setup(rp, ci, v, amg.Options(dim=dim, smoother="mcsgs"))
    oo = O.Options.for_dim(dim, smoother="mcsgs")
    H = O.setup(A.row_ptr, A.col, A.val, oo)
    assert h.num_levels() == len(H.levels)
    for k in range(h.num_levels() - 1):
        ex = h.export_level(k, what=("A",))
        Ak = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
        col, ncol = h.level_colors(k)
        want = O.color_greedy(Ak, oo.seed + 2)
        assert np.array_equal(col, want), k
        assert ncol == int(want.max()) + 1
        rows = np.repeat(np.arange(Ak.shape[0]), np.diff(Ak.indptr))
        off = rows != Ak.indices
        assert not np.any(col[rows[off]] == col[Ak.indices[off]])
        assert np.allclose(h.jacobi_weights(k), 1.0 / Ak.diagonal(), rtol=1e-15, atol=0)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    xh = x.cpu().numpy()
    ref = O.solve(H, b, 1e-8)
    assert rel <= 1e-8 and np.linalg.norm(b - A.to_scipy() @ xh) <= 1.01e-8 * np.linalg.norm(b)
    assert abs(it - ref.iters) <= 1, (it, ref.iters)
    if it == ref.iters:
        assert np.linalg.norm(xh - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    # mixed precision: within one iteration of the FP64 solve
    hm = amg.setup(rp, ci, v, amg.Options(dim=dim, smoother="mcsgs", precision="mixed"))
    xm, itm, relm = amg.solve(hm, dev_vec(b), 1e-8)
    assert relm <= 1e-8 and np.linalg.norm(b - A.to_scipy() @ xm.cpu().numpy()) <= 1.01e-8 * np.linalg.norm(b)
    assert abs(itm - it) <= 1, (itm, it)
    hm.close()
    h.close()
