"""CPU checks of the C ABI library: it loads, exports every symbol the header
declares, and its host-only entry points behave (no GPU work is issued)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg.h")

amg = pytest.importorskip("paper_1403_1649_amd")


def _lib_or_skip():
    if not os.path.exists(amg.library_path()):
        pytest.skip("libamg_hip.so not built")
    return amg.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("amg_setup", "amg_solve", "amg_destroy", "amg_export_level", "amg_spmv", "amg_galerkin"):
        assert name in syms
    assert set(syms) == set(amg.binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_default_options_follow_the_paper():
    _lib_or_skip()
    o2, o3 = amg.Options(dim=2), amg.Options(dim=3)
    assert o2.strength_alpha == 0.25 and o3.strength_alpha == 0.5
    assert o3.coarse_max == 600 and o3.kcycle_levels == 2 and o3.arnoldi_m == 5
    assert abs(o3.jacobi_scale - 4.0 / 3.0) < 1e-15 and o3.kcycle_t == 0.25


def test_status_strings():
    _lib_or_skip()
    for code in range(9):
        assert amg.status_string(code).startswith("AMG")


def test_hessenberg_radius_matches_numpy():
    _lib_or_skip()
    rng = np.random.default_rng(0)
    for m in range(1, 9):
        for _ in range(25):
            H = np.triu(rng.standard_normal((m, m)), -1)
            rho = amg.hessenberg_radius(H)
            want = np.abs(np.linalg.eigvals(H)).max()
            assert abs(rho - want) <= 1e-10 * max(1.0, want)
    # complex pair of modulus 2: rotation-scaled 2x2 block
    H = np.array([[0.0, -2.0], [2.0, 0.0]])
    assert abs(amg.hessenberg_radius(H) - 2.0) < 1e-14


def test_argument_validation_without_gpu():
    L = _lib_or_skip()
    h = C.c_void_p()
    assert L.amg_setup(None, None, None, C.byref(h)) == 1
    assert L.amg_solve(None, None, 1e-8, None, None, None, None) == 1
    A = amg.binding.AmgCsrC(0, 0, None, None, None)
    assert L.amg_spmv(C.byref(A), None, None, 0, None) == 1
    assert L.amg_node_hash(-1, 0, None, None) == 1
    assert L.amg_level_info(None, 0, None, None, None, None, None) == 1
    assert b"amg_level_info" in L.amg_last_error()


def test_batched_setup_validation_without_gpu():
    L = _lib_or_skip()
    h = C.c_void_p()
    dummy = np.zeros(8, np.int64)
    p = dummy.ctypes.data
    A = amg.binding.AmgCsrC(10, 28, p, p, p)   # never dereferenced: the checks fail first
    opts = amg.Options(dim=2)
    bad_offsets = ([1, 10], [0, 9], [0, 5, 5, 10], [0, 6, 4, 10])
    for off in bad_offsets:
        o = np.array(off, np.int32)
        assert L.amg_setup_batched(C.byref(A), len(off) - 1, o.ctypes.data, C.byref(opts.c), None,
                                   C.byref(h)) == 1, off
    o = np.array([0, 4, 10], np.int32)
    assert L.amg_setup_batched(C.byref(A), 0, o.ctypes.data, C.byref(opts.c), None, C.byref(h)) == 1
    assert L.amg_setup_batched(C.byref(A), 2, None, C.byref(opts.c), None, C.byref(h)) == 1
    fg = amg.Options(dim=2, krylov="fgmres")
    assert L.amg_setup_batched(C.byref(A), 2, o.ctypes.data, C.byref(fg.c), None, C.byref(h)) == 8
    assert b"flexible CG" in L.amg_last_error()
    assert L.amg_batch_results(None, None, None) == 1
    assert L.amg_batch_level(None, 0, None, None) == 1


def test_setup_rejects_too_many_kcycle_levels_without_gpu():
    """The K-cycle keeps per-level device slots for 24 levels: more is EINVAL
    before any device work (the matrix pointers are never dereferenced)."""
    L = _lib_or_skip()
    h = C.c_void_p()
    dummy = np.zeros(8, np.int64)
    p = dummy.ctypes.data
    A = amg.binding.AmgCsrC(10, 28, p, p, p)
    opts = amg.Options(dim=3, kcycle_levels=25, max_levels=40)
    assert L.amg_setup(C.byref(A), C.byref(opts.c), None, C.byref(h)) == 1
    assert b"option out of range" in L.amg_last_error()
    assert not h.value


def test_release_cached_memory_without_gpu():
    """Nothing is cached before any setup: the call frees nothing."""
    _lib_or_skip()
    assert amg.release_cached_memory() == 0


def test_setup_rejects_mis_k_out_of_range_without_gpu():
    """MIS(k) needs k >= 2 (the first sweep keeps settled maxima, which holds
    only when two roots never share a closed neighbourhood) and at most 8;
    batches coarsen by MIS(2) only.  Both are refused before any device work."""
    L = _lib_or_skip()
    h = C.c_void_p()
    dummy = np.zeros(8, np.int64)
    p = dummy.ctypes.data
    A = amg.binding.AmgCsrC(10, 28, p, p, p)
    for k in (1, 9):
        opts = amg.Options(dim=3, mis_k=k)
        assert L.amg_setup(C.byref(A), C.byref(opts.c), None, C.byref(h)) == 1
        assert b"mis_k" in L.amg_last_error()
        assert not h.value
    o = np.array([0, 5, 10], np.int32)
    opts = amg.Options(dim=2, mis_k=3)
    assert L.amg_setup_batched(C.byref(A), 2, o.ctypes.data, C.byref(opts.c), None, C.byref(h)) == 8


def test_default_options_extensions():
    o = amg.Options(dim=3)
    assert o.mis_k == 2 and o.cheb_degree == 2 and o.cheb_ratio == 4.0 and o.cheb_upper == 1.1
