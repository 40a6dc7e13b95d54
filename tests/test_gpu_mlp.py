"""GPU parity of the learned Jacobi weights against the FP64 oracle (same
bfloat16 rounding of inputs, weights and hidden units; sums in FP64 there,
FP32 in the kernels): features, omega, loss and gradient, each within the
bound that FP32 accumulation and the bfloat16 roundings it can flip allow
(tests/mlp_bounds.py); then training and the learned setup."""
import numpy as np
import pytest

from oracle import amg_oracle as O
from oracle import mlp_oracle as M
from synthetic import problems as P
from tests import mlp_bounds as MB
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")


def _setup(A, **kw):
    rp, ci, v = to_dev(A)
    return amg.setup(rp, ci, v, amg.Options(dim=3, **kw))


def _check_omega(om_gpu, w, S, F):
    om, dom, flips, _ = MB.omega_bounds(w.astype(np.float64), S, F)
    err = np.abs(om_gpu - om)
    assert np.all(err <= 1.5 * dom), f"omega off by {np.max(err / dom):.3g} of its bound"
    # rows whose bound allows no bfloat16 flip agree to the FP32 accumulation of y
    assert np.all(err[~flips] <= 1e-6 * om[~flips])
    return flips.mean()


def _check_loss_grad(loss, g, w, S, F, E):
    lo, dlo, go, dgo = MB.loss_grad_bounds(w.astype(np.float64), S, F, E)
    assert abs(loss - lo) <= 1.5 * dlo, (loss, lo, dlo)
    err = np.abs(np.asarray(g, np.float64) - go)
    assert np.all(err <= 1.5 * dgo), f"gradient off by {np.max(err / dgo):.3g} of its bound"
    # the bound itself stays small against the gradient (the check has teeth)
    assert np.linalg.norm(dgo) <= 1e-2 * np.linalg.norm(go)


def _weights(seed=3):
    w = M.init_weights(seed).astype(np.float32)
    w[-1] = 0.4
    return w


def test_features_match_oracle():
    A = P.hetero3d(14, seed=5)
    h = _setup(A)
    for k in range(h.num_levels() - 1):
        ex = h.export_level(k, what=("A",))
        S = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
        want = M.bf16(M.features(S, k))
        got = amg.mlp_features(h, k).cpu().numpy().astype(np.float64)
        # identical but for rare last-place differences of log() before rounding
        ulp = np.maximum(np.abs(want), 1e-30) * 2.0 ** -7
        assert np.all(np.abs(got - want) <= ulp)
        assert np.mean(got == want) > 0.999


def test_omega_loss_and_gradient_match_oracle():
    A = P.hetero3d(12, seed=8)
    h = _setup(A)
    w = _weights()
    wd = torch.from_numpy(w).cuda()
    for k in range(h.num_levels() - 1):
        ex = h.export_level(k)
        S = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
        F = amg.mlp_features(h, k).cpu().numpy().astype(np.float64)
        om = amg.mlp_omega(h, k, wd).cpu().numpy()
        assert _check_omega(om, w, S, F) < 0.5
        E = M.projected_errors(S, ex["agg"], ex["pval"], ex["nc"], 6, 77)
        g = torch.zeros_like(wd)
        loss = amg.mlp_loss_grad(h, k, wd, 6, 77, None, g)
        _check_loss_grad(loss, g.cpu().numpy(), w, S, F, E)


def test_extra_samples_and_accumulation():
    A = P.hetero3d(12, seed=9)
    h = _setup(A)
    wd = torch.from_numpy(_weights(4)).cuda()
    n = A.n
    extra = torch.from_numpy(np.random.default_rng(0).standard_normal((n, 2))).cuda()
    g1 = torch.zeros_like(wd)
    g2 = torch.zeros_like(wd)
    amg.mlp_loss_grad(h, 0, wd, 3, 5, extra, g1)
    amg.mlp_loss_grad(h, 0, wd, 3, 5, extra, g2)
    amg.mlp_loss_grad(h, 0, wd, 3, 5, extra, g2, accumulate=True)
    assert torch.allclose(2 * g1, g2, rtol=1e-6, atol=0)


def test_adam_step_matches_formula():
    rng = np.random.default_rng(1)
    w, m, v, g = (rng.standard_normal(1409).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    tw, tm, tv, tg = (torch.from_numpy(a.copy()).cuda() for a in (w, m, v, g))
    amg.mlp_adam(tw, tm, tv, tg, 3, 1e-2)
    m2 = 0.9 * m + 0.1 * g
    v2 = 0.999 * v + 0.001 * g * g
    w2 = w - 1e-2 * (m2 / (1 - 0.9 ** 3)) / (np.sqrt(v2 / (1 - 0.999 ** 3)) + 1e-8)
    assert np.allclose(tw.cpu().numpy(), w2, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss_and_learned_setup_is_safe():
    from paper_1403_1649_amd import learned as Ld
    train = [P.hetero3d(16, seed=100 + i) for i in range(3)]
    systems = []
    for A in train:
        h = _setup(A)
        systems.append((h, Ld.solver_errors(h, A, P.exact_solution(A.n, 1))))
    wd = torch.from_numpy(Ld.init_weights(0)).cuda()
    before = sum(amg.mlp_loss_grad(h, 0, wd, 8, 999) for h, _ in systems)
    w = Ld.train(systems, steps=60, lr=3e-3, samples=8)
    after = sum(amg.mlp_loss_grad(h, 0, torch.from_numpy(w).cuda(), 8, 999) for h, _ in systems)
    assert after < before
    A = P.hetero3d(20, seed=2)
    hl = _setup(A, mlp_weights=w)
    b = torch.from_numpy(P.rhs(A, P.exact_solution(A.n, 1))).cuda()
    x, it, rel = amg.solve(hl, b, 1e-8)
    assert rel <= 1e-8
    judge = hl.learned_judge()
    for k in range(hl.num_levels() - 1):
        learned, lp, ll = hl.smoother_info(k)
        assert lp > 0 and ll > 0
        assert learned == (judge["kept"] == 1)
        if learned:
            ex = hl.export_level(k, what=("A",))
            S = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
            F = amg.mlp_features(hl, k).cpu().numpy().astype(np.float64)
            _check_omega(hl.jacobi_weights(k) * S.diagonal(), w, S, F)


def test_learned_setup_rejects_bad_weights():
    A = P.hetero3d(10, seed=1)
    w = _weights()
    w[5] = np.nan
    with pytest.raises(amg.AmgError):
        _setup(A, mlp_weights=w)


def test_raw_extra_samples_and_learned_always():
    """AMG_MLP_RAW_EXTRA: the caller's samples enter the loss unprojected (the
    oracle's loss on [projected random | raw extra]); AMG_FLAG_LEARNED_ALWAYS
    keeps the learned weights on every level without validation."""
    A = P.hetero3d(12, seed=13)
    h = _setup(A)
    w = _weights(5)
    wd = torch.from_numpy(w).cuda()
    ex = h.export_level(0)
    S = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
    F = amg.mlp_features(h, 0).cpu().numpy().astype(np.float64)
    extra = np.random.default_rng(3).standard_normal((A.n, 2))
    E = np.concatenate([M.projected_errors(S, ex["agg"], ex["pval"], ex["nc"], 4, 21), extra], axis=1)
    g = torch.zeros_like(wd)
    loss = amg.mlp_loss_grad(h, 0, wd, 4, 21, torch.from_numpy(extra).cuda(), g, raw_extra=True)
    _check_loss_grad(loss, g.cpu().numpy(), w, S, F, E)
    hl = _setup(A, mlp_weights=w, flags=8)
    assert all(hl.smoother_info(k)[0] for k in range(hl.num_levels() - 1))
    b = torch.from_numpy(P.rhs(A, P.exact_solution(A.n, 1))).cuda()
    _, it, rel = amg.solve(hl, b, 1e-8)
    assert rel <= 1e-8


def test_learned_weights_judged_by_solve():
    """The method's judge of the learned weights (iteration count, then the
    final residual) on a 64^3 heterogeneous field (the training fields' size):
    the setup keeps them only when its probe solve needs fewer iterations than
    plain damped Jacobi; the full solve then needs no more iterations than the
    plain method, and a rejection leaves exactly the plain method."""
    from paper_1403_1649_amd import learned as Ld
    train = [P.hetero3d(16, seed=100 + i) for i in range(3)]
    systems = []
    for A in train:
        h = _setup(A)
        systems.append((h, Ld.solver_errors(h, A, P.exact_solution(A.n, 1))))
    w = Ld.train(systems, steps=60, lr=3e-3, samples=8)
    A = P.hetero3d(64, seed=7)
    print(f"learned judge: n={A.n}", flush=True)
    b = torch.from_numpy(P.rhs(A, P.exact_solution(A.n, 1))).cuda()
    hp = _setup(A)
    xp, itp, relp = amg.solve(hp, b, 1e-8)
    hl = _setup(A, mlp_weights=w)
    xl, itl, rell = amg.solve(hl, b, 1e-8)
    j = hl.learned_judge()
    assert rell <= 1e-8 and relp <= 1e-8
    assert j["kept"] in (-1, 0, 1)
    if j["kept"] == 1:
        assert j["iters_learned"] < j["iters_plain"] or (
            j["iters_learned"] == j["iters_plain"] and j["relres_learned"] < j["relres_plain"])
        assert itl <= itp, (itl, itp, j)
    else:
        assert all(not hl.smoother_info(k)[0] for k in range(hl.num_levels() - 1))
        assert itl == itp and np.array_equal(xl.cpu().numpy(), xp.cpu().numpy())
    hp.close()
    hl.close()


@pytest.mark.parametrize("name,make", [("hetero3d_16", lambda: P.hetero3d(16, seed=21)),
                                       ("aniso2d_64", lambda: P.aniso2d(64, 1e-2))])
def test_coarse_corrected_errors_match_oracle(name, make):
    """amg_mlp_coarse_corrected against the oracle's exact two-grid projection
    e - P A_c^-1 P^T A e on every level (A_c formed by the oracle from the
    GPU's exported A_k): exact coarse solve on the last level, 200 cycle steps
    from level k+1 above it (a stationary iteration whose factor per cycle is
    about 0.7 on the anisotropic case, so the result is exact to rounding)."""
    A = make()
    d = 3 if "3d" in name else 2
    h = amg.setup(*to_dev(A), amg.Options(dim=d))
    rng = np.random.default_rng(9)
    for k in range(h.num_levels() - 1):
        ex = h.export_level(k)
        S = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
        E = rng.standard_normal((ex["n"], 3))
        T = amg.mlp_coarse_corrected(h, k, torch.from_numpy(E).cuda(), cycles=200).cpu().numpy()
        R = M.coarse_corrected(S, ex["agg"], ex["pval"], ex["nc"], E)
        last = k == h.num_levels() - 2
        tol = 1e-10 if last else 1e-9
        assert np.linalg.norm(T - R) <= tol * np.linalg.norm(R), (k, np.linalg.norm(T - R) / np.linalg.norm(R))
    with pytest.raises(amg.AmgError):
        amg.mlp_coarse_corrected(h, h.num_levels() - 1, torch.zeros((1, 1), dtype=torch.float64, device="cuda"))
    hm = amg.setup(*to_dev(A), amg.Options(dim=d, precision="mixed"))
    with pytest.raises(amg.AmgError) as e:
        amg.mlp_coarse_corrected(hm, 0, torch.from_numpy(rng.standard_normal((A.n, 1))).cuda())
    assert e.value.code == 8
    h.close()
    hm.close()


def test_trained_network_gains_over_plain_jacobi():
    """The learned part end to end: the network trained on the GPU by the
    library's kernels (two-grid loss on four 64^3 heterogeneous fields), its
    output bias set by the solver's own judge on those fields (full solves),
    which also finds it better than plain damped Jacobi there; then, on
    held-out fields of the same distribution (64^3 and 96^3, other seeds), it
    needs fewer outer iterations than plain damped Jacobi at rtol 1e-8."""
    from paper_1403_1649_amd import learned as Ld
    systems, fields = [], []
    for q in range(4):
        At = P.hetero3d(64, seed=100 + q)
        dt = to_dev(At)
        h = amg.setup(*dt, amg.Options(dim=3))
        systems.append((h, Ld.solver_errors(h, At, P.exact_solution(At.n, 1))))
        fields.append(dt + (torch.from_numpy(P.rhs(At, P.exact_solution(At.n, 1))).cuda(),))
    w = Ld.train_two_grid(systems, steps=100, lr=3e-3, samples=8, pool=32)
    for h, _ in systems:
        h.close()
    cal = Ld.calibrate_bias(w, fields)
    assert cal["wins"], cal
    for A in (P.hetero3d(64, seed=7), P.hetero3d(96, seed=3)):
        print(f"learned vs plain: n={A.n}", flush=True)
        b = torch.from_numpy(P.rhs(A, P.exact_solution(A.n, 1))).cuda()
        hp = _setup(A)
        _, itp, relp = amg.solve(hp, b, 1e-8)
        hl = _setup(A, mlp_weights=cal["weights"], flags=amg.binding.FLAG_LEARNED_ALWAYS)
        xl, itl, rel = amg.solve(hl, b, 1e-8)
        S = A.to_scipy()
        assert rel <= 1e-8 and relp <= 1e-8
        assert np.linalg.norm(P.rhs(A, P.exact_solution(A.n, 1)) - S @ xl.cpu().numpy()) <= 1.01e-8 * np.linalg.norm(b.cpu().numpy())
        assert itl < itp, (A.n, itl, itp)
        hp.close()
        hl.close()
