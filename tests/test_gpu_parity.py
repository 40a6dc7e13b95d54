"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: integer decisions (strength mask, MIS(2) state, aggregates) bit-exact;
A_{k+1} to 1e-12 (normwise and per entry against the magnitude of its terms);
omega to 1e-12 relative; the solution to a true relative residual <= 1e-8 on
both sides with iteration counts within one.
"""
import numpy as np
import pytest

from oracle import amg_oracle as O
from synthetic import problems as P
from tests.gpu_helpers import compare_level, dev_vec, oracle_level, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")


def _setup(A, dim, **kw):
    rp, ci, v = to_dev(A)
    opts = amg.Options(dim=dim, **kw)
    return amg.setup(rp, ci, v, opts), opts


def _oracle_opts(dim, **kw):
    return O.Options.for_dim(dim, **kw)


def test_node_hash_bit_exact():
    for stream in (0, 1, 12345, 0xFFFFFFFF):
        n = (1 << 20) + 17
        got = amg.node_hash(n, stream).cpu().numpy().view(np.uint32)
        want = O.node_hash(np.arange(n), stream).astype(np.uint32)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("lpr", [-1, 0, 1, 2, 4, 8, 16, 32, 64])
def test_spmv_matches_oracle(lpr):
    A = P.hetero3d(24, seed=7)
    rp, ci, v = to_dev(A)
    x = P.exact_solution(A.n, 3)
    y = amg.spmv(rp, ci, v, dev_vec(x), lanes_per_row=lpr).cpu().numpy()
    S = A.to_scipy()
    want = S @ x
    bound = 1e-15 * 8 * (abs(S) @ np.abs(x))
    assert np.all(np.abs(y - want) <= bound + 1e-300)


def test_galerkin_worked_example_on_gpu():
    from tests.test_oracle_setup import _read_worked_example
    import scipy.sparse as sp
    pattern, aggmap, coarse = _read_worked_example()
    n = 8
    a = {(i, j): 10 * i + j + 1.0 / (i + j) for (i, j) in pattern}
    S = sp.csr_matrix(([a[p] for p in pattern], ([i - 1 for i, _ in pattern], [j - 1 for _, j in pattern])),
                      shape=(n, n))
    S.sort_indices()
    A = P.CSR(S.indptr, S.indices, S.data)
    agg = np.array([aggmap[i + 1] - 1 for i in range(n)], np.int32)
    rp, ci, v = to_dev(A)
    for pval in (np.ones(n), O.interpolation(agg, 3, np.ones(n))[0]):
        got_rp, got_ci, got_v = amg.galerkin(rp, ci, v, torch.from_numpy(agg).cuda(), dev_vec(pval), 3)
        want = O.galerkin(S, agg.astype(np.int64), pval, 3)
        assert np.array_equal(got_rp, want.indptr) and np.array_equal(got_ci, want.indices)
        assert np.allclose(got_v, want.data, rtol=1e-14, atol=0)


def test_galerkin_large_rows_path():
    """Aggregates whose segments exceed the LDS staging capacity (dense rows)."""
    rng = np.random.default_rng(4)
    n = 600
    import scipy.sparse as sp
    M = sp.random(n, n, density=0.08, random_state=rng)
    M = M + M.T + sp.identity(n) * 50
    S = M.tocsr()
    S.sort_indices()
    A = P.CSR(S.indptr, S.indices, S.data)
    nc = 7
    agg = np.concatenate([np.arange(nc), rng.integers(0, nc, n - nc)]).astype(np.int32)
    pval = rng.uniform(0.5, 1.5, n)
    rp, ci, v = to_dev(A)
    got_rp, got_ci, got_v = amg.galerkin(rp, ci, v, torch.from_numpy(agg).cuda(), dev_vec(pval), nc)
    want = O.galerkin(S, agg.astype(np.int64), pval, nc)
    assert np.array_equal(got_rp, want.indptr) and np.array_equal(got_ci, want.indices)
    assert np.allclose(got_v, want.data, rtol=1e-12, atol=1e-12 * np.abs(want.data).max())


def test_galerkin_every_row_tier():
    """Coarse rows of every size class in one product: a few terms (wave,
    two per lane), up to 512 terms (wave, eight per lane) and beyond (block
    extraction), with aggregates of 1 to 120 members in a random order."""
    rng = np.random.default_rng(9)
    import scipy.sparse as sp
    n = 4000
    M = sp.random(n, n, density=6.0 / n, random_state=rng)
    M = M + M.T + sp.identity(n) * 20
    S = M.tocsr()
    S.sort_indices()
    A = P.CSR(S.indptr, S.indices, S.data)
    sizes = np.concatenate([np.ones(300, int), rng.integers(2, 12, 150), rng.integers(30, 60, 20),
                            rng.integers(100, 121, 6)])
    sizes = sizes[np.cumsum(sizes) <= n]
    sizes[-1] += n - sizes.sum()
    nc = len(sizes)
    agg = rng.permutation(np.repeat(np.arange(nc), sizes)).astype(np.int32)
    pval = rng.uniform(0.5, 1.5, n)
    terms = np.bincount(agg, weights=np.diff(S.indptr), minlength=nc)
    assert terms.min() <= 128 and ((terms > 128) & (terms <= 512)).any() and terms.max() > 512
    rp, ci, v = to_dev(A)
    got_rp, got_ci, got_v = amg.galerkin(rp, ci, v, torch.from_numpy(agg).cuda(), dev_vec(pval), nc)
    want = O.galerkin(S, agg.astype(np.int64), pval, nc)
    assert np.array_equal(got_rp, want.indptr) and np.array_equal(got_ci, want.indices)
    assert np.allclose(got_v, want.data, rtol=1e-12, atol=1e-12 * np.abs(want.data).max())


CASES = [
    ("poisson2d_128", lambda: P.poisson2d(128), 2),
    ("poisson2d_37x53", lambda: P.poisson2d(37, 53), 2),
    ("aniso2d_90", lambda: P.aniso2d(90, 1e-3), 2),
    ("poisson3d_24", lambda: P.poisson3d(24), 3),
    ("hetero3d_20", lambda: P.hetero3d(20, seed=11), 3),
    ("aniso3d_18", lambda: P.aniso3d(18, 1e-3), 3),
]


@pytest.mark.parametrize("name,make,dim", CASES, ids=[c[0] for c in CASES])
def test_levelwise_setup_parity(name, make, dim):
    A = make()
    h, _ = _setup(A, dim)
    oo = _oracle_opts(dim)
    L = h.num_levels()
    assert L >= 2
    for k in range(L - 1):
        ex = h.export_level(k)
        nxt = h.export_level(k + 1, what=("A", "B"))
        if k == 0:
            assert np.array_equal(ex["row_ptr"], A.row_ptr) and np.array_equal(ex["val"], A.val)
        lv = oracle_level(ex, oo)
        compare_level(ex, lv, nxt)
        assert np.allclose(nxt["B"], lv.Bc, rtol=1e-14, atol=0)
        omega, _ = O.jacobi_weight(lv.A, oo.arnoldi_m, oo.seed + 1, oo.jacobi_scale)
        assert abs(ex["omega"] - omega) <= 1e-12 * omega
        assert ex["mis_rounds"] == lv.mis_rounds
    last = h.export_level(L - 1, what=("A",))
    assert last["n"] <= 600


@pytest.mark.parametrize("name,make,dim", CASES[:4] + CASES[4:5], ids=[c[0] for c in CASES[:5]])
def test_solve_matches_oracle(name, make, dim):
    A = make()
    xs = P.exact_solution(A.n, 1)
    b = P.rhs(A, xs)
    h, _ = _setup(A, dim)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    H = O.setup(A.row_ptr, A.col, A.val, _oracle_opts(dim))
    ref = O.solve(H, b, 1e-8)
    true_rel = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
    assert rel <= 1e-8 and true_rel <= 1.01e-8
    assert abs(it - ref.iters) <= 1, (it, ref.iters)
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("name,make,dim", [CASES[0], CASES[4]], ids=[CASES[0][0], CASES[4][0]])
def test_mixed_precision_solve(name, make, dim):
    A = make()
    xs = P.exact_solution(A.n, 1)
    b = P.rhs(A, xs)
    h64, _ = _setup(A, dim)
    _, it64, _ = amg.solve(h64, dev_vec(b), 1e-8)
    h, _ = _setup(A, dim, precision="mixed")
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8
    assert np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b) <= 1.01e-8
    assert abs(it - it64) <= 1, (it, it64)   # FP32 cycle: same iteration count up to one near-tie flip


def test_single_level_and_zero_rhs():
    A = P.poisson2d(20)              # 400 <= coarse_max: the preconditioner is the exact solve
    h, _ = _setup(A, 2)
    assert h.num_levels() == 1
    b = P.rhs(A, P.exact_solution(A.n, 1))
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    assert it == 1 and rel <= 1e-12
    x, it, rel = amg.solve(h, dev_vec(np.zeros(A.n)), 1e-8)
    assert it == 0 and rel == 0.0 and float(x.abs().max()) == 0.0


def test_error_paths():
    A = P.poisson2d(64)
    h, _ = _setup(A, 2, max_iter=1)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    with pytest.raises(amg.AmgError) as e:
        amg.solve(h, dev_vec(b), 1e-8)
    assert e.value.code == 4
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8, allow_notconv=True)
    assert it == 1 and rel > 1e-8
    bad = b.copy()
    bad[3] = np.nan
    h2, _ = _setup(A, 2)
    with pytest.raises(amg.AmgError) as e:
        amg.solve(h2, dev_vec(bad), 1e-8)
    assert e.value.code == 7
    # zero diagonal
    v = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    v[np.flatnonzero(A.col == rows)[5]] = 0.0
    with pytest.raises(amg.AmgError) as e:
        _setup(P.CSR(A.row_ptr, A.col, v), 2)
    assert e.value.code == 1
    # structurally nonsymmetric pattern
    import scipy.sparse as sp
    S = A.to_scipy().tolil()
    S[0, A.n - 1] = -0.5
    S = S.tocsr()
    S.sort_indices()
    with pytest.raises(amg.AmgError) as e:
        _setup(P.CSR(S.indptr, S.indices, S.data), 2)
    assert e.value.code == 1


def test_repeated_setup_is_deterministic():
    A = P.hetero3d(16, seed=3)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    outs = []
    for _ in range(2):
        h, _ = _setup(A, 3)
        x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
        outs.append((x.cpu().numpy(), it, rel, h.export_level(1, what=("A",))["val"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][3], outs[1][3])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_eager_launches(precision):
    """The captured outer iteration replayed many times (several solves with
    different right-hand sides, eager work and syncs in between) gives the
    same bits as launching every kernel from the host."""
    A = P.hetero3d(18, seed=9)
    hg, _ = _setup(A, 3, precision=precision)
    he, _ = _setup(A, 3, precision=precision, flags=1)
    for seed in (1, 2, 3):
        b = dev_vec(P.rhs(A, P.exact_solution(A.n, seed)))
        xg, itg, relg = amg.solve(hg, b, 1e-8)
        torch.cuda.synchronize()
        xe, ite, rele = amg.solve(he, b, 1e-8)
        assert itg == ite and relg == rele
        assert torch.equal(xg, xe)


@pytest.mark.parametrize("n,nonsym", [(1, False), (37, False), (143, False), (250, True), (600, False)])
def test_coarse_inverse_is_exact_solve(n, nonsym):
    """Single-level hierarchies: the preconditioner is the dense inverse, so one
    FCG step solves the system (covers one- and many-block eliminations)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(n)
    if n == 1:
        S = sp.csr_matrix(np.array([[3.0]]))
    else:
        A0 = P.hetero3d(int(round(n ** (1 / 3))) + 1, seed=n).to_scipy()[:n, :n].tocsr()
        S = A0 + sp.identity(n) * 1e-3
        if nonsym:
            S = S + sp.triu(S, 1) * 0.3
    S = S.tocsr()
    S.sort_indices()
    A = P.CSR(S.indptr, S.indices, S.data)
    h, _ = _setup(A, 3, coarse_max=600)
    assert h.num_levels() == 1
    b = rng.standard_normal(A.n)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    xs = np.linalg.solve(S.toarray(), b)
    assert it <= 2 and rel <= 1e-10
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("probe", ["l0_presmooth", "l0_postsmooth", "outer_spmv"])
def test_probe_timing_samples_in_solve(probe):
    A = P.poisson3d(40)
    h, _ = _setup(A, 3, probe=probe)
    b = dev_vec(P.rhs(A, P.exact_solution(A.n, 1)))
    _, it, rel = amg.solve(h, b, 1e-8)
    ms, n = h.probe_timing()
    assert rel <= 1e-8 and n >= 1 and 0.0 < ms < 50.0


@pytest.mark.parametrize("lanes", [-1, -2])
@pytest.mark.parametrize("make", [lambda: P.poisson2d(37, 53), lambda: P.hetero3d(17, seed=2)])
def test_sell_spmv_ragged_rows(make, lanes):
    """Sliced ELL (32-bit columns, or 16-bit offsets col - row) on ragged
    inputs: n not a multiple of 64, short boundary rows."""
    A = make()
    rp, ci, v = to_dev(A)
    x = P.exact_solution(A.n, 5)
    y = amg.spmv(rp, ci, v, dev_vec(x), lanes_per_row=lanes).cpu().numpy()
    S = A.to_scipy()
    assert np.all(np.abs(y - S @ x) <= 1e-15 * 8 * (abs(S) @ np.abs(x)) + 1e-300)


@pytest.mark.parametrize("make", [lambda: P.hetero3d(30, seed=8), lambda: P.poisson3d(42)])
def test_level_spmv_every_level(make):
    """amg_level_spmv on every level (fixed lanes on small levels, the tuned
    format on the 74,088-row level 0) against the exported A_k."""
    import scipy.sparse as sp
    A = make()
    h, _ = _setup(A, 3)
    for k in range(h.num_levels()):
        ex = h.export_level(k, what=("A",))
        S = sp.csr_matrix((ex["val"], ex["col"], ex["row_ptr"]), shape=(ex["n"], ex["n"]))
        x = P.exact_solution(ex["n"], 11 + k)
        y = h.level_spmv(k, dev_vec(x)).cpu().numpy()
        assert np.all(np.abs(y - S @ x) <= 1e-15 * 8 * (abs(S) @ np.abs(x)) + 1e-300), f"level {k}"
    with pytest.raises(amg.AmgError):
        h.level_spmv(h.num_levels(), dev_vec(np.zeros(1)))


def test_sell16_offsets_at_the_limits():
    """Couplings at offsets +-32767 fit the 16-bit columns, +-32768 (one
    past on the positive side) do not: the 16-bit form is refused, the 32-bit
    sliced ELL still serves."""
    import scipy.sparse as sp
    n = 40000
    for far, ok in ((32767, True), (32768, False)):
        S = sp.diags([-np.ones(n - 1), 4.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="lil")
        for i in (0, 5, n - far - 1):
            S[i, i + far] = -0.25
            S[i + far, i] = -0.25
        S = S.tocsr()
        S.sort_indices()
        A = P.CSR(S.indptr, S.indices, S.data)
        rp, ci, v = to_dev(A)
        x = P.exact_solution(n, 3)
        ref = S @ x
        y = amg.spmv(rp, ci, v, dev_vec(x), lanes_per_row=-1).cpu().numpy()
        assert np.all(np.abs(y - ref) <= 1e-15 * 8 * (abs(S) @ np.abs(x)))
        if ok:
            y = amg.spmv(rp, ci, v, dev_vec(x), lanes_per_row=-2).cpu().numpy()
            assert np.all(np.abs(y - ref) <= 1e-15 * 8 * (abs(S) @ np.abs(x)))
        else:
            with pytest.raises(amg.AmgError) as e:
                amg.spmv(rp, ci, v, dev_vec(x), lanes_per_row=-2)
            assert e.value.code == 1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_forced_formats_agree_on_a_tuned_level(precision, monkeypatch):
    """Above 65,536 rows the level kernels are chosen by timing; pin each
    format in turn (CSR, sliced ELL, sliced ELL with 16-bit offsets) and
    check the solves against the oracle's iteration count and each other."""
    A = P.poisson3d(42)   # 74,088 rows: level 0 is tuned
    b = P.rhs(A, P.exact_solution(A.n, 1))
    ref = O.solve(O.setup(A.row_ptr, A.col, A.val, _oracle_opts(3)), b, 1e-8)
    xs = []
    for fmt in ("csr", "sell", "sell16"):
        monkeypatch.setenv("AMG_TUNE_FORCE", fmt)
        h, _ = _setup(A, 3, precision=precision)
        x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
        assert rel <= 1e-8 and abs(it - ref.iters) <= 1
        xs.append(x.cpu().numpy())
    for x in xs[1:]:
        assert np.linalg.norm(x - xs[0]) / np.linalg.norm(xs[0]) < 1e-7


def test_tuned_and_untuned_kernels_agree():
    A = P.hetero3d(30, seed=8)
    b = dev_vec(P.rhs(A, P.exact_solution(A.n, 1)))
    ht, _ = _setup(A, 3)
    hu, _ = _setup(A, 3, flags=2)
    xt, it_t, rel_t = amg.solve(ht, b, 1e-8)
    xu, it_u, rel_u = amg.solve(hu, b, 1e-8)
    assert rel_t <= 1e-8 and rel_u <= 1e-8 and abs(it_t - it_u) <= 1
    assert float(torch.linalg.norm(xt - xu) / torch.linalg.norm(xu)) < 1e-7


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fgmres_matches_oracle(precision):
    A = P.hetero3d(16, seed=12)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    h, _ = _setup(A, 3, krylov="fgmres", precision=precision)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    H = O.setup(A.row_ptr, A.col, A.val, _oracle_opts(3, krylov="fgmres"))
    ref = O.solve(H, b, 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8 and np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b) <= 1.01e-8
    assert abs(it - ref.iters) <= 1, (it, ref.iters)


def test_fgmres_nonsymmetric_and_restart():
    n = 48
    S = P.poisson2d(n).to_scipy().tolil()
    for i in range(n * n):
        if i % n:
            S[i, i - 1] -= 0.8
            S[i, i] += 0.8
    S = S.tocsr()
    S.sort_indices()
    A = P.CSR(S.indptr, S.indices, S.data)
    b = S @ P.exact_solution(A.n, 1)
    for restart in (30, 4):
        h, _ = _setup(A, 2, krylov="fgmres", coarse_max=100, gmres_restart=restart)
        x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
        H = O.setup(A.row_ptr, A.col, A.val, _oracle_opts(2, krylov="fgmres", coarse_max=100, gmres_restart=restart))
        ref = O.solve(H, b, 1e-8)
        assert rel <= 1e-8 and abs(it - ref.iters) <= 1, (restart, it, ref.iters)


def test_omega_independent_of_recycled_device_memory():
    """Device memory of destroyed hierarchies is recycled without clearing;
    the Arnoldi estimate must only read what it wrote (regression: the
    Hessenberg entries below the subdiagonal were read from that memory)."""
    A0 = P.hetero3d(18, seed=6)
    rp, ci, v = to_dev(A0)
    h0 = amg.setup(rp, ci, v, amg.Options(dim=3, precision="mixed"))
    B = np.ascontiguousarray(P.rhs(A0, P.multi_exact_solution(A0.n, 8, 3)))
    amg.solve_multi(h0, torch.from_numpy(B).cuda(), 1e-8)
    del h0
    A = P.poisson2d(37, 53)
    h, _ = _setup(A, 2)
    oo = _oracle_opts(2)
    for k in range(h.num_levels() - 1):
        ex = h.export_level(k, what=("A",))
        S = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
        omega, _ = O.jacobi_weight(S, oo.arnoldi_m, oo.seed + 1, oo.jacobi_scale)
        assert abs(ex["omega"] - omega) <= 1e-12 * omega, (k, ex["omega"], omega)


def test_borrowed_matrix_and_cache_release():
    """AMG_FLAG_BORROW_A: the hierarchy reads the caller's arrays (identical
    hierarchy and solve); amg_release_cached_memory returns cached chunks once
    no hierarchy holds them."""
    A = P.poisson3d(24)
    rp, ci, v = to_dev(A)
    b = dev_vec(P.rhs(A, P.exact_solution(A.n, 1)))
    h1 = amg.setup(rp, ci, v, amg.Options(dim=3))
    x1, it1, rel1 = amg.solve(h1, b, 1e-8)
    h2 = amg.setup(rp, ci, v, amg.Options(dim=3, flags=amg.binding.FLAG_BORROW_A))
    x2, it2, rel2 = amg.solve(h2, b, 1e-8)
    assert it1 == it2 and rel2 <= 1e-8 and torch.equal(x1, x2)
    for k in range(h1.num_levels() - 1):
        e1, e2 = h1.export_level(k), h2.export_level(k)
        for key in ("row_ptr", "col", "val", "agg", "state"):
            assert np.array_equal(e1[key], e2[key]), (k, key)
    h1.close()
    h2.close()
    torch.cuda.synchronize()
    assert amg.release_cached_memory() > 0
    assert amg.release_cached_memory() == 0
