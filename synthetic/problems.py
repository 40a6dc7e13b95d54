"""Seeded synthetic linear systems A x = b (the problem statement of Section 2, eq. axb).

This module only builds inputs: finite-difference / finite-volume matrices in
0-based CSR (int32 row pointers, int32 sorted column indices, float64 values),
exact solutions drawn from NumPy's ``default_rng`` and right-hand sides
b = A x*.  It holds none of the multigrid method's arithmetic, so it is shared
by the CPU oracle tests and the GPU path alike.

Grid numbering is lexicographic with x fastest: i = x + nx*(y + ny*z).
Dirichlet boundaries are eliminated (their couplings simply drop out of the
stencil), unit mesh width.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CSR", "poisson1d", "poisson2d", "aniso2d", "poisson3d", "aniso3d",
    "hetero3d", "batch_sides", "block_diag", "exact_solution", "rhs",
    "multi_exact_solution", "config",
]


class CSR:
    """A square sparse matrix in 0-based CSR form with per-row sorted columns."""

    __slots__ = ("n", "row_ptr", "col", "val")

    def __init__(self, row_ptr, col, val):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def matvec(self, x):
        """y = A x in float64 (used only to form b = A x*)."""
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        return np.bincount(rows, weights=self.val * np.asarray(x, np.float64)[self.col],
                           minlength=self.n)


def _assemble(shape, faces, diag) -> CSR:
    """Assemble a 7-point (or 5/3-point) stencil on a [nz, ny, nx] grid.

    ``faces[axis]`` holds the coupling weight T between a cell and its +1
    neighbour along ``axis`` (array shape = grid shape with that axis one
    shorter), or None when the axis carries no couplings.  Off-diagonal
    entries are -T; ``diag`` is the full diagonal (cell order).
    """
    nz, ny, nx = shape
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    strides = {0: nx * ny, 1: nx, 2: 1}
    # slot order gives ascending column order: z-, y-, x-, diag, x+, y+, z+
    minus_slot = {0: 0, 1: 1, 2: 2}
    plus_slot = {2: 4, 1: 5, 0: 6}
    cols = np.zeros((n, 7), dtype=np.int64)
    vals = np.zeros((n, 7), dtype=np.float64)
    mask = np.zeros((n, 7), dtype=bool)
    cols[:, 3] = np.arange(n)
    vals[:, 3] = np.asarray(diag, dtype=np.float64).reshape(n)
    mask[:, 3] = True
    for axis, T in faces.items():
        if T is None or shape[axis] < 2:
            continue
        T = np.asarray(T, dtype=np.float64)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, shape[axis] - 1)
        hi[axis] = slice(1, shape[axis])
        lo_cells = idx[tuple(lo)].reshape(-1)
        hi_cells = idx[tuple(hi)].reshape(-1)
        t = T.reshape(-1)
        ps, ms = plus_slot[axis], minus_slot[axis]
        cols[lo_cells, ps] = lo_cells + strides[axis]
        vals[lo_cells, ps] = -t
        mask[lo_cells, ps] = True
        cols[hi_cells, ms] = hi_cells - strides[axis]
        vals[hi_cells, ms] = -t
        mask[hi_cells, ms] = True
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("matrix too large for int32 CSR")
    return CSR(row_ptr, cols[mask], vals[mask])


def _const_faces(shape, coef):
    faces = {}
    for axis, c in coef.items():
        s = list(shape)
        s[axis] -= 1
        faces[axis] = None if c is None or s[axis] <= 0 else np.full(s, float(c))
    return faces


def poisson1d(n: int) -> CSR:
    """tridiag(-1, 2, -1) of order n (1-D Dirichlet Poisson)."""
    shape = (1, 1, n)
    return _assemble(shape, _const_faces(shape, {2: 1.0}), np.full(n, 2.0))


def poisson2d(nx: int, ny: int | None = None) -> CSR:
    """5-point Dirichlet Poisson on an nx-by-ny interior grid: diag 4, off -1."""
    ny = nx if ny is None else ny
    shape = (1, ny, nx)
    return _assemble(shape, _const_faces(shape, {2: 1.0, 1: 1.0}), np.full(nx * ny, 4.0))


def aniso2d(nx: int, eps: float, ny: int | None = None) -> CSR:
    """5-point anisotropic Poisson: x couplings -1, y couplings -eps, diag 2+2eps."""
    ny = nx if ny is None else ny
    shape = (1, ny, nx)
    return _assemble(shape, _const_faces(shape, {2: 1.0, 1: eps}),
                     np.full(nx * ny, 2.0 + 2.0 * eps))


def poisson3d(n: int) -> CSR:
    """7-point Dirichlet Poisson on an n^3 interior grid: diag 6, off -1."""
    shape = (n, n, n)
    return _assemble(shape, _const_faces(shape, {2: 1.0, 1: 1.0, 0: 1.0}), np.full(n ** 3, 6.0))


def aniso3d(n: int, eps_z: float = 1e-3) -> CSR:
    """7-point anisotropic Poisson: x/y couplings -1, z couplings -eps_z, diag 4+2eps_z."""
    shape = (n, n, n)
    return _assemble(shape, _const_faces(shape, {2: 1.0, 1: 1.0, 0: eps_z}),
                     np.full(n ** 3, 4.0 + 2.0 * eps_z))


def hetero3d(n: int, seed: int = 2) -> CSR:
    """7-point two-point-flux finite-volume diffusion on an n^3 grid of unit cells.

    Cell permeability k = exp(2 g), g ~ N(0,1) i.i.d. (cell order, x fastest).
    Interior face transmissibility is the harmonic average 2 k_a k_b / (k_a + k_b);
    the two x-faces of the box are Dirichlet with half-cell transmissibility 2 k
    on the diagonal; y- and z-faces are no-flux.  a_ii = sum of the row's face
    transmissibilities, a_ij = -T.
    """
    shape = (n, n, n)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n ** 3).reshape(shape)
    k = np.exp(2.0 * g)
    faces = {}
    diag = np.zeros(shape)
    for axis in (0, 1, 2):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        ka, kb = k[tuple(lo)], k[tuple(hi)]
        T = 2.0 * ka * kb / (ka + kb)
        faces[axis] = T
        diag[tuple(lo)] += T
        diag[tuple(hi)] += T
    diag[:, :, 0] += 2.0 * k[:, :, 0]
    diag[:, :, n - 1] += 2.0 * k[:, :, n - 1]
    return _assemble(shape, faces, diag.reshape(-1))


def batch_sides(nsys: int = 64, seed: int = 3, lo: int = 64, hi: int = 512) -> np.ndarray:
    """Side lengths of the uneven 2-D Poisson batch: integers uniform in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=nsys)


def block_diag(mats) -> tuple[CSR, np.ndarray]:
    """Stack independent systems into one block-diagonal CSR; returns (A, sys_off)."""
    sizes = np.array([m.n for m in mats], dtype=np.int64)
    sys_off = np.zeros(len(mats) + 1, dtype=np.int64)
    np.cumsum(sizes, out=sys_off[1:])
    nnz_off = np.zeros(len(mats) + 1, dtype=np.int64)
    np.cumsum([m.nnz for m in mats], out=nnz_off[1:])
    if nnz_off[-1] >= 2 ** 31:
        raise ValueError("batch too large for int32 CSR")
    rp = np.concatenate([[0]] + [m.row_ptr[1:].astype(np.int64) + nnz_off[s]
                                 for s, m in enumerate(mats)])
    col = np.concatenate([m.col.astype(np.int64) + sys_off[s] for s, m in enumerate(mats)])
    val = np.concatenate([m.val for m in mats])
    return CSR(rp, col, val), sys_off.astype(np.int32)


def exact_solution(n: int, seed: int = 1) -> np.ndarray:
    """x* ~ U[-1, 1] i.i.d. from ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def multi_exact_solution(n: int, nrhs: int, seed: int = 1) -> np.ndarray:
    """X* ~ U[-1, 1], row-major [n][nrhs]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (n, nrhs))


def rhs(A: CSR, xstar: np.ndarray) -> np.ndarray:
    """b = A x* in float64 (column-wise for a 2-D x*)."""
    xstar = np.asarray(xstar, dtype=np.float64)
    if xstar.ndim == 1:
        return A.matvec(xstar)
    return np.stack([A.matvec(xstar[:, c]) for c in range(xstar.shape[1])], axis=1)


def config(name: str):
    """Named workloads: returns (A, dim, description).

    C1  2-D Poisson 128^2            C2  3-D Poisson 128^3
    C3  heterogeneous FV 160^3        C4a anisotropic 3-D 96^3 (eps_z = 1e-3)
    C5  heterogeneous FV 64^3 (training size; seeds 100-115 are separate fields)
    """
    if name == "C1":
        return poisson2d(128), 2, "2-D 5-point Poisson 128x128"
    if name == "C2":
        return poisson3d(128), 3, "3-D 7-point Poisson 128^3"
    if name == "C3":
        return hetero3d(160, seed=2), 3, "3-D heterogeneous FV diffusion 160^3, k=exp(2g)"
    if name == "C4a":
        return aniso3d(96, 1e-3), 3, "3-D anisotropic 7-point 96^3, eps_z=1e-3"
    if name == "C5":
        return hetero3d(64, seed=100), 3, "3-D heterogeneous FV diffusion 64^3"
    raise KeyError(name)
