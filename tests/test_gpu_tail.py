"""The V-cycle levels below the K-cycle (and the coarse solve) as one
persistent launch per V-cycle (AMG_FLAG_PERSISTENT_TAIL): the same arithmetic
as the per-step kernels, so the solve gives the same iterate bit for bit, in
FP64 and mixed precision, with flexible CG and FGMRES, on hierarchies with one
to several tail levels; and the oracle's iteration count."""
import numpy as np
import pytest

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import dev_vec, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")

CASES = [
    ("hetero3d_30", lambda: P.hetero3d(30, seed=8), 3),
    ("poisson3d_48", lambda: P.poisson3d(48), 3),
    ("aniso2d_300", lambda: P.aniso2d(300, 1e-3), 2),
    ("poisson2d_700", lambda: P.poisson2d(700), 2),
]


@pytest.mark.parametrize("krylov", ["fcg", "fgmres"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,make,dim", CASES, ids=[c[0] for c in CASES])
def test_tail_launch_matches_per_step_kernels(name, make, dim, precision, krylov):
    A = make()
    rp, ci, v = to_dev(A)
    b = P.rhs(A, P.exact_solution(A.n, 3))
    print(f"tail: {name} {precision} {krylov}", flush=True)
    xs, its = [], []
    for flags in (amg.binding.FLAG_PERSISTENT_TAIL, 0):
        h = amg.setup(rp, ci, v, amg.Options(dim=dim, precision=precision, krylov=krylov, flags=flags))
        x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
        assert rel <= 1e-8
        x2, it2, _ = amg.solve(h, dev_vec(b), 1e-8)   # a replay of the captured launches
        assert it2 == it and torch.equal(x, x2)
        xs.append(x.cpu().numpy())
        its.append(it)
        h.close()
    assert its[0] == its[1]
    assert np.array_equal(xs[0], xs[1])
    if precision == "fp64" and krylov == "fcg" and A.n <= 30000:
        ref = O.solve(O.setup(A.row_ptr, A.col, A.val, O.Options.for_dim(dim)), b, 1e-8)
        assert abs(its[0] - ref.iters) <= 1


def test_tail_with_more_k_levels_and_no_graph():
    """kcycle_levels = 1 (the tail starts at level 1) and eager launches."""
    A = P.hetero3d(30, seed=9)
    rp, ci, v = to_dev(A)
    b = P.rhs(A, P.exact_solution(A.n, 4))
    out = []
    for flags in (amg.binding.FLAG_NO_GRAPH | amg.binding.FLAG_PERSISTENT_TAIL, amg.binding.FLAG_NO_GRAPH,
                  amg.binding.FLAG_PERSISTENT_TAIL):
        h = amg.setup(rp, ci, v, amg.Options(dim=3, kcycle_levels=1, flags=flags))
        x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
        assert rel <= 1e-8
        out.append((it, x.cpu().numpy()))
        h.close()
    assert out[0][0] == out[1][0] == out[2][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][1], out[2][1])
