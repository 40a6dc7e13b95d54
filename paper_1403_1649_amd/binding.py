"""ctypes marshalling for the C ABI in include/amg.h (argument passing only)."""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

AMG_OK, AMG_EINVAL, AMG_ENOMEM, AMG_EHIP, AMG_ENOTCONV = 0, 1, 2, 3, 4
AMG_EBREAKDOWN, AMG_ECOARSEN, AMG_ENANINF, AMG_EUNSUPPORTED = 5, 6, 7, 8
_PREC = {"fp64": 0, "mixed": 1}
_PROBE = {"none": 0, "l0_presmooth": 1, "l0_postsmooth": 2, "outer_spmv": 3}
_KRYLOV = {"fcg": 0, "fgmres": 1}
_SMOOTHER = {"jacobi": 0, "learned": 1, "chebyshev": 2, "mcsgs": 3}
FLAG_NO_GRAPH, FLAG_NO_TUNE, FLAG_LEARNED_ALWAYS, FLAG_BORROW_A, FLAG_PERSISTENT_TAIL = 1, 2, 8, 16, 32

EXPORTED = [
    "amg_default_options", "amg_status_string", "amg_last_error", "amg_setup", "amg_solve",
    "amg_destroy", "amg_num_levels", "amg_level_info", "amg_export_level", "amg_spmv",
    "amg_node_hash", "amg_galerkin", "amg_hessenberg_radius", "amg_timings", "amg_probe_timing",
    "amg_solve_multi", "amg_mlp_num_params", "amg_mlp_features", "amg_mlp_omega", "amg_mlp_loss_grad",
    "amg_mlp_adam", "amg_level_smoother", "amg_export_jacobi", "amg_setup_batched", "amg_batch_results",
    "amg_batch_level", "amg_level_format", "amg_level_spmv", "amg_release_cached_memory",
    "amg_setup_phases", "amg_galerkin_noalloc", "amg_resetup", "amg_resetup_time", "amg_level_colors", "amg_learned_judge",
    "amg_multi_tiles", "amg_mlp_coarse_corrected",
]


class AmgOptionsC(C.Structure):
    _fields_ = [
        ("strength_alpha", C.c_double), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
        ("kcycle_levels", C.c_int32), ("kcycle_t", C.c_double), ("jacobi_scale", C.c_double),
        ("arnoldi_m", C.c_int32), ("seed", C.c_uint32), ("krylov", C.c_int32),
        ("gmres_restart", C.c_int32), ("precision", C.c_int32), ("smoother", C.c_int32),
        ("max_iter", C.c_int32), ("dense_max", C.c_int32), ("probe", C.c_int32), ("check_every", C.c_int32),
        ("flags", C.c_uint32), ("mlp_weights", C.c_void_p), ("mis_k", C.c_int32), ("cheb_degree", C.c_int32),
        ("cheb_ratio", C.c_double), ("cheb_upper", C.c_double),
    ]


class AmgCsrC(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class AmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{status_string(code)} ({msg})")
        self.code = code


def library_path() -> str:
    return os.path.join(_HERE, "libamg_hip.so")


def lib():
    """Load libamg_hip.so (after torch, so both share one HIP runtime)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    try:
        import torch  # noqa: F401  (loads the HIP runtime the tensors use)
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, i32, u32, dbl = C.c_void_p, C.c_int32, C.c_uint32, C.c_double
    P = C.POINTER
    L.amg_default_options.argtypes = [P(AmgOptionsC), i32]
    L.amg_default_options.restype = None
    L.amg_status_string.argtypes = [i32]
    L.amg_status_string.restype = C.c_char_p
    L.amg_last_error.argtypes = []
    L.amg_last_error.restype = C.c_char_p
    L.amg_setup.argtypes = [P(AmgCsrC), P(AmgOptionsC), vp, P(vp)]
    L.amg_setup.restype = i32
    L.amg_solve.argtypes = [vp, vp, dbl, vp, P(i32), P(dbl), vp]
    L.amg_solve.restype = i32
    L.amg_destroy.argtypes = [vp]
    L.amg_destroy.restype = None
    L.amg_num_levels.argtypes = [vp]
    L.amg_num_levels.restype = i32
    L.amg_level_info.argtypes = [vp, i32, P(i32), P(i32), P(dbl), P(i32), P(i32)]
    L.amg_level_info.restype = i32
    L.amg_export_level.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.amg_export_level.restype = i32
    L.amg_spmv.argtypes = [P(AmgCsrC), vp, vp, i32, vp]
    L.amg_spmv.restype = i32
    L.amg_level_spmv.argtypes = [vp, i32, vp, vp, vp]
    L.amg_level_spmv.restype = i32
    L.amg_node_hash.argtypes = [i32, u32, vp, vp]
    L.amg_node_hash.restype = i32
    L.amg_galerkin.argtypes = [P(AmgCsrC), vp, vp, i32, P(i32), vp, vp, vp, i32, vp]
    L.amg_galerkin.restype = i32
    L.amg_galerkin_noalloc.argtypes = [P(AmgCsrC), vp, vp, i32, vp, vp, vp, i32, P(i32), vp]
    L.amg_galerkin_noalloc.restype = i32
    L.amg_resetup.argtypes = [vp, vp, vp]
    L.amg_resetup.restype = i32
    L.amg_resetup_time.argtypes = [vp, P(dbl)]
    L.amg_resetup_time.restype = i32
    L.amg_level_colors.argtypes = [vp, i32, vp, P(i32)]
    L.amg_level_colors.restype = i32
    L.amg_learned_judge.argtypes = [vp, P(i32), P(i32), P(dbl), P(i32), P(dbl)]
    L.amg_learned_judge.restype = i32
    L.amg_hessenberg_radius.argtypes = [vp, i32, P(dbl)]
    L.amg_hessenberg_radius.restype = i32
    L.amg_timings.argtypes = [vp, P(dbl), P(dbl)]
    L.amg_timings.restype = i32
    L.amg_solve_multi.argtypes = [vp, i32, vp, dbl, vp, vp, vp, vp]
    L.amg_solve_multi.restype = i32
    L.amg_mlp_num_params.argtypes = []
    L.amg_mlp_num_params.restype = i32
    L.amg_mlp_features.argtypes = [vp, i32, vp, vp]
    L.amg_mlp_features.restype = i32
    L.amg_mlp_omega.argtypes = [vp, i32, vp, vp, vp]
    L.amg_mlp_omega.restype = i32
    L.amg_mlp_loss_grad.argtypes = [vp, i32, vp, i32, u32, vp, i32, P(dbl), vp, i32, vp]
    L.amg_mlp_loss_grad.restype = i32
    L.amg_mlp_adam.argtypes = [vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.amg_mlp_adam.restype = i32
    L.amg_level_smoother.argtypes = [vp, i32, P(i32), P(dbl), P(dbl)]
    L.amg_level_smoother.restype = i32
    L.amg_export_jacobi.argtypes = [vp, i32, vp]
    L.amg_export_jacobi.restype = i32
    L.amg_probe_timing.argtypes = [vp, P(dbl), P(i32)]
    L.amg_probe_timing.restype = i32
    L.amg_setup_batched.argtypes = [P(AmgCsrC), i32, vp, P(AmgOptionsC), vp, P(vp)]
    L.amg_setup_batched.restype = i32
    L.amg_batch_results.argtypes = [vp, vp, vp]
    L.amg_batch_results.restype = i32
    L.amg_batch_level.argtypes = [vp, i32, vp, vp]
    L.amg_batch_level.restype = i32
    L.amg_level_format.argtypes = [vp, i32, i32, P(i32), P(i32), P(C.c_float)]
    L.amg_level_format.restype = i32
    L.amg_setup_phases.argtypes = [vp, P(dbl), P(dbl)]
    L.amg_setup_phases.restype = i32
    L.amg_multi_tiles.argtypes = [vp, i32, P(i32), i32, P(dbl)]
    L.amg_multi_tiles.restype = i32
    L.amg_mlp_coarse_corrected.argtypes = [vp, i32, vp, i32, i32, vp, vp]
    L.amg_mlp_coarse_corrected.restype = i32
    L.amg_release_cached_memory.argtypes = []
    L.amg_release_cached_memory.restype = C.c_size_t
    _LIB = L
    atexit.register(_teardown)
    return L


_LIVE = weakref.WeakSet()


def _teardown():
    """At interpreter exit, before the HIP runtime shuts down: destroy the
    hierarchies still alive and give the library's cached device memory back."""
    for h in list(_LIVE):
        h.close()
    if _LIB is not None:
        _LIB.amg_release_cached_memory()


def release_cached_memory() -> int:
    """amg_release_cached_memory: bytes of cached device chunks freed."""
    return int(lib().amg_release_cached_memory())


def status_string(code: int) -> str:
    return lib().amg_status_string(int(code)).decode()


def _check(code: int, allow=(AMG_OK,)):
    if code not in allow:
        raise AmgError(code, lib().amg_last_error().decode())
    return code


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _nptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


class Options:
    """Setup/solve options (amg_options); keyword names follow the C struct.

    ``mlp_weights`` takes a NumPy float32 array of amg_mlp_num_params()
    values and selects the learned smoother."""

    def __init__(self, dim: int = 3, **kw):
        self.c = AmgOptionsC()
        self._keep = None
        lib().amg_default_options(C.byref(self.c), int(dim))
        if kw.get("mlp_weights") is not None:
            w = np.ascontiguousarray(kw.pop("mlp_weights"), dtype=np.float32)
            if w.size != lib().amg_mlp_num_params():
                raise ValueError("mlp_weights has the wrong length")
            self._keep = w
            self.c.mlp_weights = w.ctypes.data
            self.c.smoother = 1
        kw.pop("mlp_weights", None)
        for k, v in kw.items():
            if k == "precision" and isinstance(v, str):
                v = _PREC[v]
            if k == "krylov" and isinstance(v, str):
                v = _KRYLOV[v]
            if k == "probe" and isinstance(v, str):
                v = _PROBE[v]
            if k == "smoother" and isinstance(v, str):
                v = _SMOOTHER[v]
            if not hasattr(self.c, k):
                raise KeyError(k)
            setattr(self.c, k, v)

    def __getattr__(self, k):
        return getattr(self.c, k)


def default_options(dim: int = 3) -> Options:
    return Options(dim)


def _csr(row_ptr, col, val) -> AmgCsrC:
    import torch
    for t, dt in ((row_ptr, torch.int32), (col, torch.int32), (val, torch.float64)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise TypeError("CSR arrays must be contiguous CUDA tensors (int32, int32, float64)")
    return AmgCsrC(int(row_ptr.numel() - 1), int(col.numel()), row_ptr.data_ptr(), col.data_ptr(),
                   val.data_ptr())


class Hierarchy:
    """An amg_hierarchy handle (destroyed with the object)."""

    def __init__(self, handle: C.c_void_p, n: int, opts: Options, nsys: int = 0, keep=None):
        self._h = handle
        self.n = n
        self.opts = opts
        self.nsys = nsys
        self._keep = keep   # borrowed device arrays (AMG_FLAG_BORROW_A) stay alive with the handle
        _LIVE.add(self)

    def close(self):
        """amg_destroy (also run when the object is collected)."""
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.amg_destroy(self._h)
        self._h = None
        self._keep = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    def num_levels(self) -> int:
        return lib().amg_num_levels(self._h)

    def level_info(self, k: int) -> dict:
        n, nnz, nc, rounds = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        om = C.c_double()
        _check(lib().amg_level_info(self._h, k, C.byref(n), C.byref(nnz), C.byref(om), C.byref(nc),
                                    C.byref(rounds)))
        return {"n": n.value, "nnz": nnz.value, "omega": om.value, "nc": nc.value,
                "mis_rounds": rounds.value}

    def export_level(self, k: int, what=("A", "strong", "state", "agg", "pval", "B")) -> dict:
        info = self.level_info(k)
        n, nnz = info["n"], info["nnz"]
        out = {}
        bufs = {
            "row_ptr": np.empty(n + 1, np.int32) if "A" in what else None,
            "col": np.empty(nnz, np.int32) if "A" in what else None,
            "val": np.empty(nnz, np.float64) if "A" in what else None,
            "strong": np.empty(nnz, np.uint8) if "strong" in what else None,
            "state": np.empty(n, np.int8) if "state" in what else None,
            "agg": np.empty(n, np.int32) if "agg" in what else None,
            "pval": np.empty(n, np.float64) if "pval" in what else None,
            "B": np.empty(n, np.float64) if "B" in what else None,
        }
        args = [(_nptr(b) if b is not None else None) for b in bufs.values()]
        _check(lib().amg_export_level(self._h, k, *args))
        for key, b in bufs.items():
            if b is not None:
                out[key] = b
        out.update(info)
        return out

    def timings(self):
        s, v = C.c_double(), C.c_double()
        _check(lib().amg_timings(self._h, C.byref(s), C.byref(v)))
        return s.value, v.value

    def resetup(self, val):
        """amg_resetup: new values of A_0 (device float64[nnz]) on the same pattern."""
        _check(lib().amg_resetup(self._h, _ptr(val), _stream()))
        if self._keep is not None and self.opts.c.flags & FLAG_BORROW_A:
            self._keep = (self._keep[0], self._keep[1], val)   # level 0 now reads these values

    def resetup_ms(self) -> float:
        ms = C.c_double()
        _check(lib().amg_resetup_time(self._h, C.byref(ms)))
        return ms.value

    def setup_phases(self):
        """(autotuner ms, graph capture ms) of the last setup (host wall clock)."""
        t, g = C.c_double(), C.c_double()
        _check(lib().amg_setup_phases(self._h, C.byref(t), C.byref(g)))
        return t.value, g.value

    def multi_tiles(self, nrhs: int):
        """(column tile per level, then of the FP64 level-0 products; tuner ms) of the
        block solve with nrhs columns."""
        cap = self.num_levels()
        t = (C.c_int32 * cap)()
        ms = C.c_double()
        _check(lib().amg_multi_tiles(self._h, nrhs, t, cap, C.byref(ms)))
        return list(t), ms.value

    def smoother_info(self, k: int):
        """(learned?, validation loss with plain omega, with learned weights)."""
        l, a, b = C.c_int32(), C.c_double(), C.c_double()
        _check(lib().amg_level_smoother(self._h, k, C.byref(l), C.byref(a), C.byref(b)))
        return bool(l.value), a.value, b.value

    def learned_judge(self) -> dict:
        """The setup's probe-solve judgement of the learned weights."""
        kept, ip, il = C.c_int32(), C.c_int32(), C.c_int32()
        rp, rl = C.c_double(), C.c_double()
        _check(lib().amg_learned_judge(self._h, C.byref(kept), C.byref(ip), C.byref(rp), C.byref(il), C.byref(rl)))
        return {"kept": kept.value, "iters_plain": ip.value, "relres_plain": rp.value, "iters_learned": il.value,
                "relres_learned": rl.value}

    def level_colors(self, k: int):
        """(colour of every row, number of colours) of level k (MC-SGS smoother)."""
        out = np.empty(self.level_info(k)["n"], np.int32)
        nc = C.c_int32()
        _check(lib().amg_level_colors(self._h, k, _nptr(out), C.byref(nc)))
        return out, nc.value

    def jacobi_weights(self, k: int) -> np.ndarray:
        """omega_i / a_ii of level k (host copy)."""
        out = np.empty(self.level_info(k)["n"], np.float64)
        _check(lib().amg_export_jacobi(self._h, k, _nptr(out)))
        return out

    def level_format(self, k: int, precision: str = "fp64"):
        """(format, lanes_per_row, timed us) the autotuner chose for level k;
        format 0 = CSR, 1 = sliced ELL, 2 = sliced ELL with 16-bit column
        offsets, 3 = sliced diagonals, 4 = CSR with 16-bit column offsets."""
        f, l, us = C.c_int32(), C.c_int32(), C.c_float()
        _check(lib().amg_level_format(self._h, int(k), _PREC[precision], C.byref(f), C.byref(l), C.byref(us)))
        return f.value, l.value, us.value

    def level_spmv(self, k: int, x, y=None):
        """y = A_k x with level k's tuned FP64 kernel (amg_level_spmv)."""
        import torch
        n = self.level_info(k)["n"]
        if x.numel() != n or x.dtype != torch.float64 or not x.is_cuda:
            raise ValueError(f"level_spmv: x must be a float64 device vector of {n} entries")
        if y is None:
            y = torch.empty(n, dtype=torch.float64, device=x.device)
        _check(lib().amg_level_spmv(self._h, int(k), _ptr(x), _ptr(y), _stream()))
        return y

    def batch_results(self):
        """Per-system (iters[], relres[]) of the last solve of a batched hierarchy."""
        it = np.zeros(self.nsys, np.int32)
        rel = np.zeros(self.nsys, np.float64)
        _check(lib().amg_batch_results(self._h, _nptr(it), _nptr(rel)))
        return it, rel

    def batch_level(self, k: int):
        """(sys_off[nsys+1], omega[nsys]) of level k of a batched hierarchy."""
        off = np.zeros(self.nsys + 1, np.int32)
        om = np.zeros(self.nsys, np.float64)
        _check(lib().amg_batch_level(self._h, int(k), _nptr(off), _nptr(om)))
        return off, om

    def probe_timing(self):
        """(average ms, samples) of the kernel selected by the probe option."""
        ms, n = C.c_double(), C.c_int32()
        _check(lib().amg_probe_timing(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


def setup(row_ptr, col, val, opts: Options | None = None, dim: int = 3) -> Hierarchy:
    """amg_setup on CUDA tensors; the current torch stream orders the work."""
    opts = opts or Options(dim)
    A = _csr(row_ptr, col, val)
    h = C.c_void_p()
    _check(lib().amg_setup(C.byref(A), C.byref(opts.c), _stream(), C.byref(h)))
    keep = (row_ptr, col, val) if opts.c.flags & FLAG_BORROW_A else None
    return Hierarchy(h, A.n, opts, keep=keep)


def setup_batched(row_ptr, col, val, sys_off, opts: Options | None = None, dim: int = 2) -> Hierarchy:
    """amg_setup_batched: independent systems on the block diagonal, system q
    owning rows [sys_off[q], sys_off[q+1]) (a host int sequence)."""
    opts = opts or Options(dim)
    A = _csr(row_ptr, col, val)
    off = np.ascontiguousarray(sys_off, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().amg_setup_batched(C.byref(A), int(off.size - 1), _nptr(off), C.byref(opts.c), _stream(),
                                   C.byref(h)))
    return Hierarchy(h, A.n, opts, nsys=int(off.size - 1))


def solve(h: Hierarchy, b, rtol: float = 1e-8, x=None, allow_notconv: bool = False):
    """amg_solve: returns (x, iters, relres)."""
    import torch
    if not (b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == h.n):
        raise TypeError("b must be a contiguous CUDA float64 tensor of length n")
    if x is None:
        x = torch.empty_like(b)
    it = C.c_int32()
    rel = C.c_double()
    code = lib().amg_solve(h.handle, _ptr(b), float(rtol), _ptr(x), C.byref(it), C.byref(rel), _stream())
    _check(code, (AMG_OK, AMG_ENOTCONV) if allow_notconv else (AMG_OK,))
    return x, it.value, rel.value


def solve_multi(h: Hierarchy, B, rtol: float = 1e-8, X=None, allow_notconv: bool = False):
    """amg_solve_multi on a row-major [n][nrhs] CUDA float64 block: (X, iters[], relres[])."""
    import torch
    if not (B.is_cuda and B.dtype == torch.float64 and B.is_contiguous() and B.dim() == 2
            and B.shape[0] == h.n):
        raise TypeError("B must be a contiguous CUDA float64 tensor of shape [n, nrhs]")
    R = int(B.shape[1])
    if X is None:
        X = torch.empty_like(B)
    it = np.zeros(R, np.int32)
    rel = np.zeros(R, np.float64)
    code = lib().amg_solve_multi(h.handle, R, _ptr(B), float(rtol), _ptr(X), _nptr(it), _nptr(rel), _stream())
    _check(code, (AMG_OK, AMG_ENOTCONV) if allow_notconv else (AMG_OK,))
    return X, it, rel


def spmv(row_ptr, col, val, x, y=None, lanes_per_row: int = 0):
    import torch
    A = _csr(row_ptr, col, val)
    if y is None:
        y = torch.empty(A.n, dtype=torch.float64, device=x.device)
    _check(lib().amg_spmv(C.byref(A), _ptr(x), _ptr(y), int(lanes_per_row), _stream()))
    return y


def node_hash(n: int, stream: int, device="cuda"):
    import torch
    out = torch.empty(n, dtype=torch.int32, device=device)
    _check(lib().amg_node_hash(int(n), int(stream) & 0xFFFFFFFF, _ptr(out), _stream()))
    return out


def galerkin(row_ptr, col, val, agg, pval, nc: int):
    """amg_galerkin: returns (row_ptr_c, col_c, val_c) as NumPy arrays."""
    A = _csr(row_ptr, col, val)
    nnz = C.c_int32()
    code = lib().amg_galerkin(C.byref(A), _ptr(agg), _ptr(pval), int(nc), C.byref(nnz), None, None, None,
                              0, _stream())
    if code != AMG_EINVAL or nnz.value <= 0:
        _check(code)
    rp = np.empty(nc + 1, np.int32)
    ci = np.empty(nnz.value, np.int32)
    v = np.empty(nnz.value, np.float64)
    _check(lib().amg_galerkin(C.byref(A), _ptr(agg), _ptr(pval), int(nc), C.byref(nnz), _nptr(rp),
                              _nptr(ci), _nptr(v), int(nnz.value), _stream()))
    return rp, ci, v


def galerkin_noalloc(row_ptr, col, val, agg, pval, nc: int, cap: int | None = None):
    """amg_galerkin_noalloc: returns (row_ptr_c, col_c, val_c) as device tensors
    (col_c / val_c of length cap, default nnz(A); the first nnz(A_c) entries hold
    the product) and nnz(A_c)."""
    import torch
    A = _csr(row_ptr, col, val)
    cap = int(A.nnz) if cap is None else int(cap)
    dev = row_ptr.device
    rp = torch.empty(nc + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    v = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    nnz = C.c_int32()
    _check(lib().amg_galerkin_noalloc(C.byref(A), _ptr(agg), _ptr(pval), int(nc), _ptr(rp), _ptr(ci), _ptr(v), cap,
                                      C.byref(nnz), _stream()))
    return rp, ci, v, nnz.value


def hessenberg_radius(H: np.ndarray) -> float:
    """Host-only: largest |eigenvalue| of a small upper Hessenberg matrix."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    rho = C.c_double()
    _check(lib().amg_hessenberg_radius(_nptr(H), int(H.shape[0]), C.byref(rho)))
    return rho.value


# ---------------------------------------------------------------- learned weights
def mlp_num_params() -> int:
    return lib().amg_mlp_num_params()


def mlp_features(h: Hierarchy, k: int):
    import torch
    n = h.level_info(k)["n"]
    F = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    _check(lib().amg_mlp_features(h.handle, k, _ptr(F), _stream()))
    return F


def mlp_omega(h: Hierarchy, k: int, w):
    import torch
    n = h.level_info(k)["n"]
    om = torch.empty(n, dtype=torch.float64, device="cuda")
    _check(lib().amg_mlp_omega(h.handle, k, _ptr(w), _ptr(om), _stream()))
    return om


def mlp_loss_grad(h: Hierarchy, k: int, w, nsamples: int, seed: int, extra=None, grad=None,
                  accumulate: bool = False, raw_extra: bool = False) -> float:
    """Smoothing loss (and gradient into grad); raw_extra: use the extra
    samples without removing their coarse-space component."""
    loss = C.c_double()
    n_extra = 0 if extra is None else int(extra.shape[1])
    flags = (1 if accumulate else 0) | (2 if raw_extra else 0)
    _check(lib().amg_mlp_loss_grad(h.handle, k, _ptr(w), int(nsamples), int(seed) & 0xFFFFFFFF,
                                   None if extra is None else _ptr(extra), n_extra, C.byref(loss),
                                   None if grad is None else _ptr(grad), flags, _stream()))
    return loss.value


def mlp_coarse_corrected(h: Hierarchy, k: int, E, cycles: int = 20, out=None):
    """amg_mlp_coarse_corrected: (I - P_k B P_k^T A_k) E for a device float64
    block E [n_k][S] (B the coarse inverse, or `cycles` cycle steps)."""
    import torch
    if E.dim() != 2 or E.dtype != torch.float64 or not E.is_cuda or not E.is_contiguous():
        raise ValueError("mlp_coarse_corrected: E must be a contiguous float64 device block [n_k][S]")
    if out is None:
        out = torch.empty_like(E)
    _check(lib().amg_mlp_coarse_corrected(h.handle, int(k), _ptr(E), int(E.shape[1]), int(cycles), _ptr(out),
                                          _stream()))
    return out


def mlp_adam(w, m, v, g, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    _check(lib().amg_mlp_adam(_ptr(w), _ptr(m), _ptr(v), _ptr(g), int(w.numel()), int(step), float(lr),
                              float(b1), float(b2), float(eps), _stream()))
