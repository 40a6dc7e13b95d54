"""MIS(k), k > 2 (Section 2.1.2, aggressive coarsening) on the GPU against the
oracle, through the C ABI: every level re-coarsened by the oracle with the
same k from the GPU's exported A_k (strength mask, MIS(k) state and aggregates
bit-exact, round counts equal, A_{k+1} within 1e-12, omega within 1e-12), the
roots pairwise more than k apart and every node within k of one, and the
solve against the oracle's (iterations within one, true relres <= 1e-8)."""
import numpy as np
import pytest
import scipy.sparse.csgraph as csg

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import compare_level, dev_vec, oracle_level, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")

CASES = [
    ("poisson2d_64x47", lambda: P.poisson2d(64, 47), 2),
    ("aniso2d_80", lambda: P.aniso2d(80, 1e-3), 2),
    ("poisson3d_20", lambda: P.poisson3d(20), 3),
    ("hetero3d_18", lambda: P.hetero3d(18, seed=11), 3),
]


def _check_misk_property(ex, lv, k):
    """Roots pairwise farther than k in G; every node within k of a root."""
    roots = np.flatnonzero(ex["state"] == 1)
    d = csg.shortest_path(lv.G, unweighted=True, indices=roots)
    assert np.all(np.min(d, axis=0) <= k)
    dr = d[:, roots]
    np.fill_diagonal(dr, np.inf)
    assert np.all(dr > k)


@pytest.mark.parametrize("k", [3, 4])
@pytest.mark.parametrize("name,make,dim", CASES, ids=[c[0] for c in CASES])
def test_misk_levelwise_parity(name, make, dim, k):
    A = make()
    rp, ci, v = to_dev(A)
    print(f"misk: {name} k={k}", flush=True)
    h = amg.setup(rp, ci, v, amg.Options(dim=dim, mis_k=k))
    oo = O.Options.for_dim(dim, mis_k=k)
    L = h.num_levels()
    for lvl in range(L - 1):
        ex = h.export_level(lvl)
        nxt = h.export_level(lvl + 1, what=("A",))
        lv = oracle_level(ex, oo)
        compare_level(ex, lv, nxt)
        assert h.level_info(lvl)["mis_rounds"] == lv.mis_rounds
        om, _ = O.jacobi_weight(lv.A, oo.arnoldi_m, oo.seed + 1, oo.jacobi_scale)
        assert abs(h.level_info(lvl)["omega"] - om) <= 1e-12 * om
        if lvl == 0 and A.n <= 10000:
            _check_misk_property(ex, lv, k)
    # more aggressive than MIS(2): fewer coarse unknowns on level 1
    h2 = amg.setup(rp, ci, v, amg.Options(dim=dim))
    assert h.level_info(0)["nc"] < h2.level_info(0)["nc"]
    h2.close()
    b = P.rhs(A, P.exact_solution(A.n, 1))
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    xh = x.cpu().numpy()
    H = O.setup(A.row_ptr, A.col, A.val, oo)
    ref = O.solve(H, b, 1e-8)
    assert rel <= 1e-8 and np.linalg.norm(b - A.to_scipy() @ xh) <= 1.01e-8 * np.linalg.norm(b)
    assert abs(it - ref.iters) <= 1, (it, ref.iters)
    if it == ref.iters:
        assert np.linalg.norm(xh - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    h.close()
