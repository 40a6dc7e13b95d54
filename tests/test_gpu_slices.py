"""The autotuner's other sparse layouts (Section 3's sparse products, in the
layouts that pad or move less): sliced ELL in 32- and 16-row slices (2 or 4
lanes per row, rows ordered by length within 64-row windows), for levels
whose rows vary in length, and sliced diagonals (per 64-row slice its
diagonal offsets and their values, no column indices), for levels from
structured grids.  Forced on the tuned levels of a 96^3 Poisson hierarchy
(level 0: 884,736 uniform rows; level 1: about 80,000 rows of uneven length)
and of a heterogeneous field, every product is checked entry by entry against
the exported A_k, the solve against the default hierarchy's, and a re-setup
on new values."""
import numpy as np
import pytest
import scipy.sparse as sp

from synthetic import problems as P
from tests.gpu_helpers import dev_vec, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amg = pytest.importorskip("paper_1403_1649_amd")

FMT = {"sell": 1, "sell16": 2}


@pytest.fixture(scope="module")
def base():
    A = P.poisson3d(96)
    dev = to_dev(A)
    b = P.rhs(A, P.exact_solution(A.n, 1))
    h = amg.setup(*dev, amg.Options(dim=3))
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    yield A, dev, b, x.cpu().numpy(), it
    h.close()


def _entrywise(h, k, seed):
    ex = h.export_level(k, what=("A",))
    S = sp.csr_matrix((ex["val"], ex["col"], ex["row_ptr"]), shape=(ex["n"], ex["n"]))
    x = P.exact_solution(ex["n"], seed)
    y = h.level_spmv(k, dev_vec(x)).cpu().numpy()
    rowlen = np.diff(ex["row_ptr"]).max()
    # both sides sum at most rowlen products: each within (rowlen - 1) u of the exact row sum
    assert np.all(np.abs(y - S @ x) <= 2.5e-16 * rowlen * (abs(S) @ np.abs(x)))


@pytest.mark.parametrize("slice_h,fmt", [(32, "sell"), (16, "sell"), (32, "sell16"), (16, "sell16")])
def test_short_slices_products_and_solve(base, slice_h, fmt, monkeypatch):
    A, dev, b, x0, it0 = base
    monkeypatch.setenv("AMG_TUNE_SLICE", str(slice_h))
    monkeypatch.setenv("AMG_TUNE_FORCE", f"{fmt}:{slice_h}")
    print(f"slices: {fmt} h={slice_h}", flush=True)
    h = amg.setup(*dev, amg.Options(dim=3))
    tuned = [k for k in range(h.num_levels() - 1) if h.level_info(k)["n"] > 65536]
    assert tuned[:2] == [0, 1]
    for k in tuned:
        f, lanes, _ = h.level_format(k)
        assert (f, lanes) == (FMT[fmt], 64 // slice_h), (k, f, lanes)
        _entrywise(h, k, 10 + k)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8 and abs(it - it0) <= 1
    assert np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - x0) <= 1e-7 * np.linalg.norm(x0)
    # new values on the same pattern: the short-slice copies take them too
    v2 = dev[2] * 2.0
    h.resetup(v2)
    for k in tuned:
        _entrywise(h, k, 20 + k)
    x2, it2, rel2 = amg.solve(h, dev_vec(b), 1e-8)
    assert rel2 <= 1e-8 and abs(it2 - it0) <= 1
    assert np.linalg.norm(x2.cpu().numpy() - 0.5 * x0) <= 1e-7 * np.linalg.norm(0.5 * x0)
    h.close()


@pytest.mark.parametrize("slice_h", [32, 16])
def test_short_slices_mixed_precision(base, slice_h, monkeypatch):
    A, dev, b, x0, it0 = base
    monkeypatch.setenv("AMG_TUNE_SLICE", str(slice_h))
    monkeypatch.setenv("AMG_TUNE_FORCE", f"sell16:{slice_h}")
    h = amg.setup(*dev, amg.Options(dim=3, precision="mixed"))
    assert h.level_format(1, "mixed")[:2] == (2, 64 // slice_h)
    assert h.level_format(0, "fp64")[:2] == (2, 64 // slice_h)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8 and abs(it - it0) <= 1
    assert np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-8 * np.linalg.norm(b)
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sliced_diagonals_products_and_solve(base, precision, monkeypatch):
    """Sliced diagonals (per 64-row slice its diagonal offsets and values, no
    column indices) on the 96^3 Poisson hierarchy's level 0 (seven diagonals):
    the product entry by entry against the exported A_0, the solve against the
    default hierarchy, and a re-setup on new values."""
    A, dev, b, x0, it0 = base
    monkeypatch.setenv("AMG_TUNE_FORCE", "sdia")
    print(f"sliced diagonals: {precision}", flush=True)
    h = amg.setup(*dev, amg.Options(dim=3, precision=precision))
    assert h.level_format(0, "fp64" if precision == "fp64" else "mixed")[:2] == (3, 1)
    if precision == "mixed":
        assert h.level_format(0, "fp64")[:2] == (3, 1)
    _entrywise(h, 0, 31)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8 and abs(it - it0) <= 1
    assert np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-8 * np.linalg.norm(b)
    if precision == "fp64":
        assert np.linalg.norm(x - x0) <= 1e-7 * np.linalg.norm(x0)
        h.resetup(dev[2] * 2.0)
        _entrywise(h, 0, 32)
        x2, it2, rel2 = amg.solve(h, dev_vec(b), 1e-8)
        assert rel2 <= 1e-8 and abs(it2 - it0) <= 1
        assert np.linalg.norm(x2.cpu().numpy() - 0.5 * x0) <= 1e-7 * np.linalg.norm(0.5 * x0)
    h.close()


def test_sliced_diagonals_on_the_heterogeneous_field(monkeypatch):
    """The 3-D heterogeneous finite-volume field (seven-point rows, fewer at
    the Dirichlet faces): forced sliced diagonals on level 0, its product
    entry by entry and the solve."""
    A = P.hetero3d(48, seed=5)
    dev = to_dev(A)
    b = P.rhs(A, P.exact_solution(A.n, 2))
    monkeypatch.setenv("AMG_TUNE_FORCE", "sdia")
    h = amg.setup(*dev, amg.Options(dim=3))
    assert h.level_format(0)[:2] == (3, 1)
    _entrywise(h, 0, 41)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    assert rel <= 1e-8
    assert np.linalg.norm(b - A.to_scipy() @ x.cpu().numpy()) <= 1.01e-8 * np.linalg.norm(b)
    h.close()


@pytest.mark.parametrize("fmt", ["sdia", "sell:32", "sell16:16", "csr16"])
def test_ragged_last_slice(fmt, monkeypatch):
    """A level whose row count is not a multiple of the slice height (43^3 =
    79,507 rows: the last 64-row slice holds 19 rows): the padded slots of the
    last slice (rows past n) contribute nothing and write nothing."""
    A = P.poisson3d(43)
    assert A.n % 64 != 0 and A.n > 65536
    dev = to_dev(A)
    b = P.rhs(A, P.exact_solution(A.n, 6))
    if ":" in fmt:
        monkeypatch.setenv("AMG_TUNE_SLICE", fmt.split(":")[1])
    monkeypatch.setenv("AMG_TUNE_FORCE", fmt)
    h = amg.setup(*dev, amg.Options(dim=3))
    f, lanes, _ = h.level_format(0)
    assert f == {"sdia": 3, "sell:32": 1, "sell16:16": 2, "csr16": 4}[fmt]
    _entrywise(h, 0, 51)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    assert rel <= 1e-8
    assert np.linalg.norm(b - A.to_scipy() @ x.cpu().numpy()) <= 1.01e-8 * np.linalg.norm(b)
    h.close()


@pytest.mark.parametrize("sched", ["contiguous", "sweep", "plane"])
@pytest.mark.parametrize("fmt", ["sdia", "sell", "sell16"])
def test_slice_schedules(base, fmt, sched, monkeypatch):
    """Every schedule of the slice kernels over the 96^3 Poisson level 0
    (3,456 steps of four slices; a grid plane is 36 steps): contiguous runs
    of steps per block, the XCD sweep (each XCD's blocks walk its eighth of
    the steps together) and plane-ordered.  The product entry by entry against
    the exported A_0 and the solve against the default hierarchy."""
    A, dev, b, x0, it0 = base
    monkeypatch.setenv("AMG_TUNE_FORCE", fmt)
    monkeypatch.setenv("AMG_TUNE_SCHEDULE", sched)
    print(f"schedule: {fmt} {sched}", flush=True)
    h = amg.setup(*dev, amg.Options(dim=3))
    assert h.level_format(0)[0] == {"sdia": 3, "sell": 1, "sell16": 2}[fmt]
    _entrywise(h, 0, 61)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8 and abs(it - it0) <= 1
    assert np.linalg.norm(x - x0) <= 1e-7 * np.linalg.norm(x0)
    h.close()


@pytest.mark.parametrize("fmt", ["sdia", "sell"])
def test_sweep_on_a_ragged_level(fmt, monkeypatch):
    """The XCD sweep where the steps do not divide evenly among the XCDs
    (43^3 = 79,507 rows: 311 steps over 304 blocks, 39 steps per XCD, the
    last XCD 38) and the last slice is partial."""
    A = P.poisson3d(43)
    dev = to_dev(A)
    b = P.rhs(A, P.exact_solution(A.n, 7))
    monkeypatch.setenv("AMG_TUNE_FORCE", fmt)
    monkeypatch.setenv("AMG_TUNE_SCHEDULE", "sweep")
    h = amg.setup(*dev, amg.Options(dim=3))
    _entrywise(h, 0, 71)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    assert rel <= 1e-8
    assert np.linalg.norm(b - A.to_scipy() @ x.cpu().numpy()) <= 1.01e-8 * np.linalg.norm(b)
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_csr_with_16bit_offsets(base, precision, monkeypatch):
    """The CSR row kernels reading the columns as 16-bit offsets col - row
    (forced on the tuned levels of the 96^3 Poisson hierarchy, whose offsets
    all fit): each product entry by entry against the exported A_k, the solve
    against the default hierarchy, and a re-setup on new values."""
    A, dev, b, x0, it0 = base
    monkeypatch.setenv("AMG_TUNE_FORCE", "csr16")
    print(f"csr16: {precision}", flush=True)
    h = amg.setup(*dev, amg.Options(dim=3, precision=precision))
    tuned = [k for k in range(h.num_levels() - 1) if h.level_info(k)["n"] > 65536]
    assert tuned[:2] == [0, 1]
    for k in tuned:
        f, lanes, _ = h.level_format(k, "fp64" if precision == "fp64" else "mixed")
        assert f == 4 and lanes in (2, 4, 8, 16, 32), (k, f, lanes)
    assert h.level_format(0, "fp64")[0] == 4
    for k in tuned:
        _entrywise(h, k, 81 + k)
    x, it, rel = amg.solve(h, dev_vec(b), 1e-8)
    x = x.cpu().numpy()
    assert rel <= 1e-8 and abs(it - it0) <= 1
    assert np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-8 * np.linalg.norm(b)
    if precision == "fp64":
        assert np.linalg.norm(x - x0) <= 1e-7 * np.linalg.norm(x0)
        h.resetup(dev[2] * 2.0)
        for k in tuned:
            _entrywise(h, k, 91 + k)
        x2, it2, rel2 = amg.solve(h, dev_vec(b), 1e-8)
        assert rel2 <= 1e-8 and abs(it2 - it0) <= 1
    h.close()
