"""Paper Table 1 on the GPU: the hierarchy of the 2-D anisotropic Poisson
problem on a 1000 x 1000 grid (eps = 1e-3, alpha = 0.25), level by level
against the oracle run on the GPU's own A_k (strength mask, MIS(2) state and
aggregates bit-exact, A_{k+1} within 1e-12, omega within 1e-12), and the level
sizes against the printed unsmoothed-aggregation column (levels 1-4 within
4 %, operator complexity within 1 %, as the oracle's own Table 1 pin)."""
import numpy as np
import pytest

from synthetic import problems as P
from tests.gpu_helpers import compare_level, oracle_level, to_dev
from oracle import amg_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")

TABLE1 = [(1000000, 4996000), (274979, 1770339), (77433, 525877), (21823, 147803), (6150, 39298), (938, 5128),
          (169, 641)]


def test_table1_hierarchy_levelwise():
    A = P.aniso2d(1000, 1e-3)
    rp, ci, v = to_dev(A)
    print(f"table1: n={A.n} nnz={A.nnz}", flush=True)
    h = amg.setup(rp, ci, v, amg.Options(dim=2))
    opts = O.Options.for_dim(2)
    L = h.num_levels()
    sizes = [(h.level_info(k)["n"], h.level_info(k)["nnz"]) for k in range(L)]
    assert sizes[0] == TABLE1[0]
    for k in range(1, 5):
        assert abs(sizes[k][0] - TABLE1[k][0]) <= 0.04 * TABLE1[k][0], (k, sizes[k])
    oc = sum(z for _, z in sizes) / sizes[0][1]
    paper_oc = sum(z for _, z in TABLE1) / TABLE1[0][1]
    assert abs(oc - paper_oc) <= 0.01 * paper_oc, (oc, paper_oc)
    for k in range(L - 1):
        ex = h.export_level(k)
        nxt = h.export_level(k + 1, what=("A",))
        lv = oracle_level(ex, opts)
        compare_level(ex, lv, nxt)
        assert lv.mis_rounds == h.level_info(k)["mis_rounds"]
        om, _ = O.jacobi_weight(lv.A, opts.arnoldi_m, opts.seed + 1, opts.jacobi_scale)
        assert abs(h.level_info(k)["omega"] - om) <= 1e-12 * om
    b = P.rhs(A, P.exact_solution(A.n, 1))
    x, it, rel = amg.solve(h, torch.from_numpy(b).cuda(), 1e-8)
    xh = x.cpu().numpy()
    assert rel <= 1e-8 and np.linalg.norm(b - A.to_scipy() @ xh) <= 1.01e-8 * np.linalg.norm(b)
    h.close()
