"""GPU: independent systems in one batched hierarchy (block-diagonal input).

Each system must be set up and solved as if alone: on every level its block
of the batched hierarchy equals the hierarchy the library builds for that
system by itself (strength mask, MIS(2) state and aggregates bit-exact, A_{k+1}
to 1e-14 relative, the same coarsest level), its Jacobi weight agrees to
1e-12, and its solve converges like the single solve (iterations within one,
true relative residual <= 1e-8).  The oracle's batch semantics (solve_batch:
each system set up and solved alone) pins the reference.
"""
import numpy as np
import pytest

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import dev_vec, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")


def _systems():
    # sides chosen so that systems stop on levels 0 (9 x 9 = 81 <= 600), 1 and 2,
    # with one anisotropic system whose strength graph is one-dimensional
    return [P.poisson2d(40), P.poisson2d(9), P.poisson2d(71, 53), P.aniso2d(48, 1e-3), P.poisson2d(23),
            P.poisson2d(130)]


def _block(mats):
    Abd, off = P.block_diag(mats)
    return Abd, off


def _batched(mats, **kw):
    Abd, off = _block(mats)
    rp, ci, v = to_dev(Abd)
    h = amg.setup_batched(rp, ci, v, off, amg.Options(dim=2, **kw))
    return Abd, off, h


def _sub(ex, lo, hi):
    rp = ex["row_ptr"]
    a, b = rp[lo], rp[hi]
    return rp[lo:hi + 1] - a, ex["col"][a:b] - lo, ex["val"][a:b], (a, b)


def test_levels_match_single_setups():
    mats = _systems()
    Abd, off, h = _batched(mats)
    L = h.num_levels()
    for q, m in enumerate(mats):
        rp, ci, v = to_dev(m)
        hs = amg.setup(rp, ci, v, amg.Options(dim=2))
        Ls = hs.num_levels()
        for k in range(L):
            offk, om = h.batch_level(k)
            lo, hi = int(offk[q]), int(offk[q + 1])
            if k >= Ls:
                assert hi == lo, (q, k)
                continue
            exs = hs.export_level(k, what=("A",) if k == Ls - 1 else ("A", "strong", "state", "agg", "pval"))
            assert hi - lo == exs["n"], (q, k)
            coarsest = k == Ls - 1
            exb = h.export_level(k, what=("A",) if (coarsest or k == L - 1) else
                                 ("A", "strong", "state", "agg", "pval"))
            brp, bci, bval, (a, b) = _sub(exb, lo, hi)
            assert np.array_equal(brp, exs["row_ptr"]) and np.array_equal(bci, exs["col"]), (q, k)
            scale = np.abs(exs["val"]).max()
            assert np.all(np.abs(bval - exs["val"]) <= 1e-14 * scale), (q, k)
            if coarsest:
                continue
            assert np.array_equal(exb["strong"][a:b], exs["strong"]), (q, k)
            assert np.array_equal(exb["state"][lo:hi], exs["state"]), (q, k)
            offn, _ = h.batch_level(k + 1)
            assert np.array_equal(exb["agg"][lo:hi] - offn[q], exs["agg"]), (q, k)
            assert np.allclose(exb["pval"][lo:hi], exs["pval"], rtol=1e-15, atol=0)
            w_single = hs.level_info(k)["omega"]
            assert abs(om[q] - w_single) <= 1e-12 * w_single, (q, k, om[q], w_single)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solves_match_single_solves(precision):
    mats = _systems()
    Abd, off, h = _batched(mats, precision=precision)
    xs = P.exact_solution(Abd.n, 1)
    b = P.rhs(Abd, xs)
    x, it_max, rel_max = amg.solve(h, dev_vec(b), 1e-8)
    its, rels = h.batch_results()
    x = x.cpu().numpy()
    assert it_max == its.max() and rel_max == rels.max()
    for q, m in enumerate(mats):
        lo, hi = off[q], off[q + 1]
        rp, ci, v = to_dev(m)
        hs = amg.setup(rp, ci, v, amg.Options(dim=2, precision=precision))
        x1, it1, rel1 = amg.solve(hs, dev_vec(b[lo:hi]), 1e-8)
        x1 = x1.cpu().numpy()
        assert rels[q] <= 1e-8 and abs(int(its[q]) - it1) <= 1, (q, its[q], it1)
        true_rel = np.linalg.norm(b[lo:hi] - m.to_scipy() @ x[lo:hi]) / np.linalg.norm(b[lo:hi])
        assert true_rel <= 1.01e-8
        assert np.linalg.norm(x[lo:hi] - x1) <= 1e-6 * np.linalg.norm(x1)
    # the system that stops on level 0 is solved by its dense inverse: one
    # iteration in FP64, two when the inverse is applied in FP32
    assert its[1] == (1 if precision == "fp64" else 2)


def test_batch_against_oracle():
    mats = [P.poisson2d(37), P.aniso2d(30, 1e-3), P.poisson2d(19)]
    Abd, off, h = _batched(mats)
    b = P.rhs(Abd, P.exact_solution(Abd.n, 3))
    x, _, _ = amg.solve(h, dev_vec(b), 1e-8)
    its, rels = h.batch_results()
    x = x.cpu().numpy()
    ref = O.solve_batch(Abd.row_ptr, Abd.col, Abd.val, off, b, O.Options.for_dim(2))
    for q in range(len(mats)):
        lo, hi = off[q], off[q + 1]
        assert abs(int(its[q]) - ref[q].iters) <= 1 and rels[q] <= 1e-8, (q, its[q], ref[q].iters)
        assert np.linalg.norm(x[lo:hi] - ref[q].x) <= 1e-6 * np.linalg.norm(ref[q].x)


def test_zero_system_and_repeat_determinism():
    mats = [P.poisson2d(30), P.poisson2d(44), P.poisson2d(26)]
    Abd, off, h = _batched(mats, precision="mixed")
    b = P.rhs(Abd, P.exact_solution(Abd.n, 4))
    b[off[1]:off[2]] = 0.0
    x1, _, _ = amg.solve(h, dev_vec(b), 1e-8)
    its1, rels1 = h.batch_results()
    x2, _, _ = amg.solve(h, dev_vec(b), 1e-8)
    its2, _ = h.batch_results()
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    assert its1[1] == 0 and rels1[1] == 0.0 and np.all(x1[off[1]:off[2]] == 0.0)
    assert rels1[0] <= 1e-8 and rels1[2] <= 1e-8
    assert np.array_equal(x1, x2) and np.array_equal(its1, its2)


def test_max_levels_two_and_errors():
    mats = [P.poisson2d(50), P.poisson2d(64)]
    Abd, off, h = _batched(mats, max_levels=2)
    assert h.num_levels() == 2
    offk, _ = h.batch_level(1)
    for q, m in enumerate(mats):
        rp, ci, v = to_dev(m)
        hs = amg.setup(rp, ci, v, amg.Options(dim=2, max_levels=2))
        assert offk[q + 1] - offk[q] == hs.level_info(1)["n"]
    b = P.rhs(Abd, P.exact_solution(Abd.n, 5))
    _, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    assert rel <= 1e-8
    # an entry coupling two systems is rejected
    A = P.poisson2d(12)
    rp, ci, v = to_dev(A)
    with pytest.raises(amg.AmgError) as e:
        amg.setup_batched(rp, ci, v, [0, 70, A.n], amg.Options(dim=2))
    assert e.value.code == 1 and "couples" in str(e.value)
    with pytest.raises(amg.AmgError) as e:
        amg.solve_multi(h, torch.zeros((Abd.n, 2), dtype=torch.float64, device="cuda"))
    assert e.value.code == 8


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_c4b_full_size_sampled(precision):
    """The 64-system batch at full size in the benchmark's configuration (mixed)
    and in FP64: every system's true residual checked on the host, the three
    smallest systems against the oracle."""
    sides = P.batch_sides()
    mats = [P.poisson2d(int(s)) for s in sides]
    Abd, off, h = _batched(mats, precision=precision)
    b = P.rhs(Abd, P.exact_solution(Abd.n, 1))
    x, _, _ = amg.solve(h, dev_vec(b), 1e-8)
    its, rels = h.batch_results()
    x = x.cpu().numpy()
    S = Abd.to_scipy()
    r = b - S @ x
    for q in range(len(mats)):
        lo, hi = off[q], off[q + 1]
        assert np.linalg.norm(r[lo:hi]) <= 1.01e-8 * np.linalg.norm(b[lo:hi]), q
    for q in np.argsort(sides)[:3]:
        lo, hi = off[q], off[q + 1]
        m = mats[q]
        H = O.setup(m.row_ptr, m.col, m.val, O.Options.for_dim(2))
        ref = O.solve(H, b[lo:hi])
        assert abs(int(its[q]) - ref.iters) <= 1, (q, its[q], ref.iters)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_eager_launches(precision):
    mats = [P.poisson2d(41), P.poisson2d(29), P.aniso2d(33, 1e-3)]
    Abd, off, hg = _batched(mats, precision=precision)
    _, _, he = _batched(mats, precision=precision, flags=1)
    b = dev_vec(P.rhs(Abd, P.exact_solution(Abd.n, 6)))
    xg, _, _ = amg.solve(hg, b, 1e-8)
    itg, relg = hg.batch_results()
    xe, _, _ = amg.solve(he, b, 1e-8)
    ite, rele = he.batch_results()
    assert np.array_equal(itg, ite) and np.array_equal(relg, rele)
    assert torch.equal(xg, xe)
