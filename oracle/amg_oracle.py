"""Plain FP64 CPU oracle for aggregation AMG — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the HIP library: it takes plain CSR arrays
and returns plain arrays.  It is deliberately slow and literal: each function
follows one passage of Gandham, Esler & Zhang, "A GPU Accelerated Aggregation
Algebraic Multigrid Method" (arXiv 1403.1649), cited by section / algorithm /
equation, in the paper's order and notation.  Library primitives (a sparse
mat-vec, a sort, a segmented sum, a dense factorisation, a small eigenvalue
routine) stand in for single steps; nothing is blocked, fused or reordered.

Where the paper is silent, ambiguous or garbled, the reading taken here is
stated at the function that needs it:

* strength: strict ``>`` as printed; alpha*m_i is one FP64 multiply.
* the MIS graph is undirected, N_i = neighbours of i in G = C union C^T.
* the random r_i of Algorithm 2 is a seeded counter hash: r_i = H32(i)/2^32,
  H32 = the MurmurHash3 32-bit finaliser (a bijection of uint32), so tuples
  never tie.
* a non-root joins its nearest root in G (distance 1 before 2); among equally
  near roots, the one with the largest v; coarse ids number the roots in
  ascending node order.
* B_0 is the constant vector.
* the K-cycle's undefined initial guesses are 0; t = 0.25; the garbled
  residual update after prolongation reads r_k = b_k - A_k x_k, and the
  post-smoothing step is S_k(b_k, A_k, x_k).
* the coarsest system is solved by a dense factorisation (mathematically the
  exact solve the paper obtains with a sparse direct solver).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

MASK32 = 0xFFFFFFFF
GOLDEN32 = 0x9E3779B9  # Weyl increment that separates seeds


class OracleError(Exception):
    """Raised for inputs the method does not accept (mirrors the C status codes)."""

    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# Input validation (problem statement, Section 2, eq. axb)
# ---------------------------------------------------------------------------

def validate_csr(row_ptr, col, val) -> sp.csr_matrix:
    """Check a square 0-based CSR matrix: monotone row pointers, columns in
    range, strictly increasing within each row, a nonzero finite diagonal."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    n = row_ptr.shape[0] - 1
    if n < 1 or row_ptr[0] != 0 or row_ptr[-1] != col.shape[0] or col.shape != val.shape:
        raise OracleError("EINVAL", "malformed CSR arrays")
    if np.any(np.diff(row_ptr) < 0):
        raise OracleError("EINVAL", "row pointers decrease")
    if col.size and (col.min() < 0 or col.max() >= n):
        raise OracleError("EINVAL", "column index out of range")
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    same_row = rows[1:] == rows[:-1]
    if np.any(same_row & (col[1:] <= col[:-1])):
        raise OracleError("EINVAL", "columns not strictly increasing within a row")
    if not np.all(np.isfinite(val)):
        raise OracleError("ENANINF", "non-finite matrix entry")
    A = sp.csr_matrix((val, col, row_ptr), shape=(n, n))
    d = A.diagonal()
    if np.any(d == 0):
        raise OracleError("EINVAL", "zero or missing diagonal entry")
    return A


# ---------------------------------------------------------------------------
# Seeded counter hash (replaces the random r_i of Algorithm 2)
# ---------------------------------------------------------------------------

def fmix32(x):
    """MurmurHash3 32-bit finaliser: xor-shift 16, multiply 0x85ebca6b,
    xor-shift 13, multiply 0xc2b2ae35, xor-shift 16 (all mod 2^32).
    Every step is invertible, so the map is a bijection of uint32."""
    h = np.asarray(x, dtype=np.uint64) & MASK32
    h = h ^ (h >> np.uint64(16))
    h = (h * np.uint64(0x85EBCA6B)) & np.uint64(MASK32)
    h = h ^ (h >> np.uint64(13))
    h = (h * np.uint64(0xC2B2AE35)) & np.uint64(MASK32)
    h = h ^ (h >> np.uint64(16))
    return h


def node_hash(index, seed: int):
    """h_i = fmix32((i + seed * 0x9E3779B9) mod 2^32) for node index i."""
    i = np.asarray(index, dtype=np.uint64)
    return fmix32((i + np.uint64((seed * GOLDEN32) & MASK32)) & np.uint64(MASK32))


def unit_uniform(index, stream: int):
    """u_i = node_hash(i, stream) * 2^-31 - 1, an exact float64 in [-1, 1)."""
    return node_hash(index, stream).astype(np.float64) * 2.0 ** -31 - 1.0


# ---------------------------------------------------------------------------
# Section 2.1.1: classic strength of connection
# ---------------------------------------------------------------------------

def strength(A: sp.csr_matrix, alpha: float) -> np.ndarray:
    """C over A's pattern (bool per stored entry): C_ij = 1 iff
    -s_i A_ij > alpha * max_{j: -s_i A_ij > 0} (-s_i A_ij), s_i = sign(A_ii).

    The diagonal entry has -s_i A_ii < 0 and is never strong.  A row without
    any positive -s_i A_ij has an empty strong set (the max is then taken as 0,
    and no entry can exceed it while also being positive)."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    s = np.sign(A.diagonal())
    neg = -s[rows] * A.data                        # -s_i A_ij
    cand = np.where(neg > 0.0, neg, 0.0)
    m = _segmax(cand, A.indptr, 0.0)               # max over -s_i A_ij > 0
    threshold = alpha * m                          # one FP64 multiply per row
    return neg > threshold[rows]


def strong_graph(A: sp.csr_matrix, C: np.ndarray) -> sp.csr_matrix:
    """Undirected graph G = C union C^T (no self loops); N_i = row i of G."""
    n = A.shape[0]
    Cm = sp.csr_matrix((C.astype(np.int8), A.indices.copy(), A.indptr.copy()), shape=(n, n))
    Cm.eliminate_zeros()                               # copies above: A stays untouched
    G = ((Cm + Cm.T) != 0).astype(np.int8).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    return G


def influence_count(A: sp.csr_matrix, C: np.ndarray) -> np.ndarray:
    """#{j : C_ji = 1}: how many rows hold a strong entry in column i."""
    return np.bincount(A.indices[C], minlength=A.shape[0]).astype(np.int64)


# ---------------------------------------------------------------------------
# Algorithm 2: fine-grain parallel MIS(2)
# ---------------------------------------------------------------------------

def priorities(cnt: np.ndarray, seed: int) -> np.ndarray:
    """v_i = #{j : C_ji = 1} + r_i with r_i = h_i / 2^32 in [0, 1).

    Exact in float64 while the count stays below 2^21 (checked)."""
    if cnt.size and cnt.max() >= 2 ** 21:
        raise OracleError("EINVAL", "influence count too large for exact v")
    h = node_hash(np.arange(cnt.shape[0]), seed)
    return cnt.astype(np.float64) + h.astype(np.float64) * 2.0 ** -32


def mis_parallel(G: sp.csr_matrix, v: np.ndarray, k: int = 2):
    """Algorithm 2 in synchronous rounds, for MIS(k) (Section 2.1.2: roots
    more than k apart; Algorithm 2 is k = 2, with two sweeps).

    Tuples T_i = (s_i, v_i, i) are compared lexicographically.  Each round
    builds the tuples, takes k max sweeps over N_i (each sweep reads the
    previous sweep's tuples: double buffered), so every node sees the largest
    tuple within distance k; then every undecided node i becomes an MIS node
    if that tuple is its own, or a non-MIS node if it belongs to an MIS node.
    Returns (s, rounds) with s in {1 (MIS), -1 (non-MIS)}."""
    n = G.shape[0]
    ball = (G + sp.identity(n, dtype=np.int8, format="csr")).tocsr()  # N_i with i itself
    s = np.zeros(n, dtype=np.int64)
    nodes = np.arange(n)
    rounds = 0
    while np.any(s == 0):
        rounds += 1
        # T_i = (s_i, v_i, i): represent each tuple by its rank in lexicographic order
        order = np.lexsort((nodes, v, s))          # primary s, then v, then i
        T = np.empty(n, dtype=np.int64)
        T[order] = nodes
        for _d in range(k):
            T = np.maximum.reduceat(T[ball.indices], ball.indptr[:-1])   # T <- T-hat
        i_max = order[T]
        s_max = s[i_max]
        undecided = s == 0
        new_s = s.copy()
        new_s[undecided & (i_max == nodes)] = 1
        new_s[undecided & (i_max != nodes) & (s_max == 1)] = -1
        s = new_s
    return s, rounds


def mis2_parallel(G: sp.csr_matrix, v: np.ndarray):
    """Algorithm 2 as printed: MIS(2)."""
    return mis_parallel(G, v, 2)


def mis_greedy(G: sp.csr_matrix, v: np.ndarray, k: int = 2) -> np.ndarray:
    """Sequential greedy MIS(k): visit nodes by decreasing v; a node becomes an
    MIS node when no MIS node lies within graph distance k.  (Small graphs.)"""
    n = G.shape[0]
    nbr = [G.indices[G.indptr[i]:G.indptr[i + 1]] for i in range(n)]
    s = -np.ones(n, dtype=np.int64)
    blocked = np.zeros(n, dtype=bool)
    for i in np.argsort(-v, kind="stable"):
        if blocked[i]:
            continue
        s[i] = 1
        frontier, seen = [i], {i}
        for _d in range(k):                        # everything within distance k
            nxt = []
            for u in frontier:
                for j in nbr[u]:
                    if j not in seen:
                        seen.add(j)
                        nxt.append(j)
            frontier = nxt
        blocked[list(seen)] = True
    return s


def mis2_greedy(G: sp.csr_matrix, v: np.ndarray) -> np.ndarray:
    """Sequential greedy MIS(2)."""
    return mis_greedy(G, v, 2)


# ---------------------------------------------------------------------------
# Section 2.1.2 (end): aggregates around the MIS(2) roots
# ---------------------------------------------------------------------------

def aggregate(G: sp.csr_matrix, s: np.ndarray, v: np.ndarray, k: int = 2):
    """Every non-MIS node joins its nearest MIS node (graph distance in G, at
    most k for MIS(k) roots).

    Ties between equally near roots go to the root with the larger v; coarse
    ids number the roots in ascending node order.  Returns (agg, n_c)."""
    n = G.shape[0]
    is_root = s == 1
    roots = np.flatnonzero(is_root)
    coarse_id = np.full(n, -1, dtype=np.int64)
    coarse_id[roots] = np.arange(roots.shape[0])
    # rank of each node's v (ties impossible: v is injective through the hash)
    vrank = np.empty(n, dtype=np.int64)
    vrank[np.argsort(v, kind="stable")] = np.arange(n)
    order_to_node = np.argsort(v, kind="stable")

    def best_root(M):
        cand = np.where(is_root[M.indices], vrank[M.indices], -1)
        best = _segmax(cand, M.indptr, -1)
        return np.where(best >= 0, order_to_node[np.maximum(best, 0)], -1)

    # walks of length d reach exactly the roots at distance d from a node that
    # has none nearer, so the first d with a reachable root gives the nearest
    chosen = np.where(is_root, np.arange(n), -1)
    W = G.copy()
    for d in range(1, k + 1):
        if d > 1:
            W = (W @ G).tocsr()
            W.data[:] = 1
        W.sort_indices()
        bd = best_root(W)
        chosen = np.where(chosen >= 0, chosen, bd)
    if np.any(chosen < 0):
        raise OracleError("EINVAL", f"node farther than {k} from every MIS({k}) node")
    return coarse_id[chosen], int(roots.shape[0])


# ---------------------------------------------------------------------------
# Algorithm 3: interpolation with one nonzero per row
# ---------------------------------------------------------------------------

def interpolation(agg: np.ndarray, nc: int, B: np.ndarray):
    """P_k(i, Agg(i)) = B_k(i); B_{k+1}(I) = ||R_k(I, :)||_2; R and P are
    normalised by B_{k+1}, so P^T P = I and B_k = P_k B_{k+1} (eq. null_space).
    Returns (pval, B_next, P) with pval[i] = P_k(i, Agg(i))."""
    n = agg.shape[0]
    P = sp.csr_matrix((B.astype(np.float64), agg, np.arange(n + 1)), shape=(n, nc))
    R = P.T.tocsr()
    B_next = np.sqrt(np.asarray(R.multiply(R).sum(axis=1)).ravel())   # row 2-norms of R
    pval = B / B_next[agg]
    P = sp.csr_matrix((pval, agg, np.arange(n + 1)), shape=(n, nc))
    return pval, B_next, P


# ---------------------------------------------------------------------------
# Section 3.1: Galerkin product by aggregate index (eq. galerkin)
# ---------------------------------------------------------------------------

def galerkin(A: sp.csr_matrix, agg: np.ndarray, pval: np.ndarray, nc: int) -> sp.csr_matrix:
    """(A_{k+1})_IJ = sum_{i in G_I} sum_{j in G_J} P_iI A_ij P_jJ.

    Each stored (i, j) maps to (I, J) = (Agg(i), Agg(j)) and its coefficient
    is multiplied by P and R before the sort; the tuples are sorted
    lexicographically by (I, J), unique pairs are counted and duplicates
    summed by a segmented reduction.  Every structural (I, J) is kept."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    I = agg[rows]
    J = agg[A.indices]
    coef = (pval[rows] * A.data) * pval[A.indices]
    order = np.lexsort((J, I))                         # stable: I, then J
    I, J, coef = I[order], J[order], coef[order]
    head = np.ones(I.shape[0], dtype=bool)
    head[1:] = (I[1:] != I[:-1]) | (J[1:] != J[:-1])
    starts = np.flatnonzero(head)
    vals = np.add.reduceat(coef, starts)
    Ic, Jc = I[starts], J[starts]
    row_ptr = np.zeros(nc + 1, dtype=np.int64)
    np.cumsum(np.bincount(Ic, minlength=nc), out=row_ptr[1:])
    return sp.csr_matrix((vals, Jc, row_ptr), shape=(nc, nc))


# ---------------------------------------------------------------------------
# Section 2.2.1: damped Jacobi weight from Arnoldi (eq. damped_jacobi)
# ---------------------------------------------------------------------------

def arnoldi_hessenberg(A: sp.csr_matrix, m: int, stream: int):
    """m <= 5 Arnoldi steps (modified Gram-Schmidt) on M = D^{-1} A from the
    seeded start q_0 = u / ||u||, u_i = unit_uniform(i, stream).  Stops early
    when h_{j+1,j} <= 1e-14 ||M q_j||.  Returns the square Hessenberg block."""
    n = A.shape[0]
    m = min(m, n)
    dinv = 1.0 / A.diagonal()
    q = unit_uniform(np.arange(n), stream)
    Q = [q / np.linalg.norm(q)]
    H = np.zeros((m + 1, m))
    size = m
    for j in range(m):
        w = dinv * (A @ Q[j])
        wnorm = np.linalg.norm(w)
        for i in range(j + 1):
            H[i, j] = Q[i] @ w
            w = w - H[i, j] * Q[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= 1e-14 * wnorm:
            size = j + 1
            break
        Q.append(w / H[j + 1, j])
    return H[:size, :size]


def jacobi_weight(A: sp.csr_matrix, m: int, stream: int, scale: float = 4.0 / 3.0):
    """omega = (4/3) / rho(D^{-1} A), rho estimated as the largest modulus of
    the eigenvalues of the Arnoldi Hessenberg matrix.  Returns (omega, rho)."""
    H = arnoldi_hessenberg(A, m, stream)
    rho = float(np.max(np.abs(np.linalg.eigvals(H))))
    if not rho > 0.0 or not math.isfinite(rho):
        raise OracleError("EBREAKDOWN", "spectral radius estimate not positive")
    return scale / rho, rho


# ---------------------------------------------------------------------------
# Algorithm 1: setup
# ---------------------------------------------------------------------------

@dataclass
class Options:
    strength_alpha: float = 0.25     # 0.25 for 2-D problems, 0.5 for 3-D (Section 2.1.1)
    coarse_max: int = 600            # "about 600" unknowns on the coarsest level (Section 3)
    max_levels: int = 20
    kcycle_levels: int = 2           # K-cycles on the top two levels (Section 2.2)
    mis_k: int = 2                   # roots form an MIS(k) (Section 2.1.2; Algorithm 2 is k = 2)
    kcycle_t: float = 0.25
    jacobi_scale: float = 4.0 / 3.0
    arnoldi_m: int = 5
    seed: int = 0
    krylov: str = "fcg"              # "fcg" or "fgmres"
    gmres_restart: int = 30
    max_iter: int = 200
    dense_max: int = 4096            # largest coarsest level accepted after a stall
    # smoother S_k (Section 2.2.1): "jacobi" (damped Jacobi, eq. damped_jacobi),
    # "chebyshev" (polynomial smoother, Section 5) or "mcsgs" (multi-colour
    # symmetric Gauss-Seidel, Section 2.2.1)
    smoother: str = "jacobi"
    cheb_degree: int = 2             # SpMVs per Chebyshev smoothing step
    cheb_ratio: float = 4.0          # Chebyshev interval [b / ratio, b], b = cheb_upper * rho
    cheb_upper: float = 1.1          # margin over the Arnoldi estimate of rho(D^-1 A)

    @staticmethod
    def for_dim(dim: int, **kw) -> "Options":
        return Options(strength_alpha=0.25 if dim == 2 else 0.5, **kw)


@dataclass
class Level:
    A: sp.csr_matrix
    B: np.ndarray
    C: np.ndarray | None = None          # strong mask over A's pattern
    G: sp.csr_matrix | None = None
    cnt: np.ndarray | None = None
    v: np.ndarray | None = None
    s: np.ndarray | None = None          # MIS(2) state (1 / -1)
    mis_rounds: int = 0
    agg: np.ndarray | None = None
    nc: int = 0
    pval: np.ndarray | None = None
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    omega: float = 0.0
    rho: float = 0.0
    wdinv: np.ndarray | None = None      # omega / a_ii
    smoother: str = "jacobi"
    cheb: tuple | None = None            # (theta, delta, degree) of the Chebyshev smoother
    colors: np.ndarray | None = None     # colour of every row (multi-colour Gauss-Seidel)

    @property
    def n(self) -> int:
        return self.A.shape[0]


@dataclass
class Hierarchy:
    levels: list
    opts: Options
    coarse_factor: object = None
    coarse_kind: str = "cholesky"
    status: str = "OK"
    extra: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        """Index of the coarsest level."""
        return len(self.levels) - 1

    def coarse_solve(self, r):
        if self.coarse_kind == "cholesky":
            return sla.cho_solve(self.coarse_factor, r)
        return sla.lu_solve(self.coarse_factor, r)


def coarsen_level(A: sp.csr_matrix, B: np.ndarray, opts: Options) -> Level:
    """One pass of the loop body of Algorithm 1 (strength, aggregate, prolongate,
    Galerkin) plus the level's Jacobi weight; the coarse matrix is returned in
    ``lv.extra_Ac`` via the attribute ``Ac``."""
    lv = Level(A=A, B=B)
    lv.C = strength(A, opts.strength_alpha)
    lv.G = strong_graph(A, lv.C)
    lv.cnt = influence_count(A, lv.C)
    lv.v = priorities(lv.cnt, opts.seed)
    lv.s, lv.mis_rounds = mis_parallel(lv.G, lv.v, opts.mis_k)
    lv.agg, lv.nc = aggregate(lv.G, lv.s, lv.v, opts.mis_k)
    lv.pval, Bc, lv.P = interpolation(lv.agg, lv.nc, B)
    lv.R = lv.P.T.tocsr()
    lv.Ac = galerkin(A, lv.agg, lv.pval, lv.nc)
    lv.Bc = Bc
    return lv


def setup(row_ptr, col, val, opts: Options | None = None) -> Hierarchy:
    """Algorithm 1: coarsen while the level has more than ``coarse_max``
    unknowns; stop at ``max_levels`` or when coarsening stalls
    (n_{k+1} > 0.9 n_k).  Every non-coarsest level gets its damped Jacobi
    weight; the coarsest is factorised densely."""
    opts = opts or Options()
    A = validate_csr(row_ptr, col, val)
    B = np.ones(A.shape[0])
    levels = []
    while True:
        n = A.shape[0]
        if n <= opts.coarse_max or len(levels) + 1 >= opts.max_levels:
            levels.append(Level(A=A, B=B))
            break
        lv = coarsen_level(A, B, opts)
        if lv.nc > 0.9 * n or lv.nc == 0:
            levels.append(Level(A=A, B=B))             # stall: this level is the coarsest
            break
        lv.omega, lv.rho = jacobi_weight(A, opts.arnoldi_m, opts.seed + 1, opts.jacobi_scale)
        lv.wdinv = lv.omega / A.diagonal()
        lv.smoother = opts.smoother
        if opts.smoother == "chebyshev":
            lv.cheb = chebyshev_interval(lv.rho, opts)
        elif opts.smoother == "mcsgs":
            lv.colors = color_greedy(A, opts.seed + 2)
        elif opts.smoother != "jacobi":
            raise OracleError("EINVAL", f"unknown smoother {opts.smoother}")
        levels.append(lv)
        A, B = lv.Ac, lv.Bc
    H = Hierarchy(levels=levels, opts=opts)
    Ac = levels[-1].A
    if Ac.shape[0] > opts.dense_max:
        raise OracleError("ECOARSEN", f"coarsest level has {Ac.shape[0]} unknowns")
    coarse_factor(H)
    return H


def coarse_factor(H: Hierarchy) -> None:
    """Dense factorisation of the coarsest matrix: Cholesky for the CG path
    (LU when Cholesky fails), LU for the GMRES path."""
    dense = H.levels[-1].A.toarray()
    if H.opts.krylov == "fcg":
        try:
            H.coarse_factor = sla.cho_factor(dense, lower=True)
            H.coarse_kind = "cholesky"
            return
        except np.linalg.LinAlgError:
            pass
    H.coarse_factor = sla.lu_factor(dense)
    H.coarse_kind = "lu"


def resetup(H: Hierarchy, val) -> Hierarchy:
    """Numeric re-setup on a fixed pattern (Section 3.1: when only the values of
    A_0 change, as across Newton steps, the sort and segmented-reduction indices
    of the Galerkin product are stored and reused).  The aggregation of every
    level (strength, MIS(2), aggregates) and P_k are kept; A_0 takes the new
    values and, level by level, A_{k+1} = P_k^T A_k P_k is formed again with
    the same P_k, followed by the level's Jacobi weight and finally the coarse
    factorisation.  Returns a new hierarchy; H is left unchanged."""
    opts = H.opts
    A0 = H.levels[0].A
    val = np.asarray(val, dtype=np.float64)
    if val.shape != A0.data.shape:
        raise OracleError("EINVAL", "new values do not match the pattern")
    A = sp.csr_matrix((val.copy(), A0.indices.copy(), A0.indptr.copy()), shape=A0.shape)
    validate_csr(A.indptr, A.indices, A.data)
    levels = []
    for old in H.levels[:-1]:
        lv = Level(A=A, B=old.B, C=old.C, G=old.G, cnt=old.cnt, v=old.v, s=old.s, mis_rounds=old.mis_rounds,
                   agg=old.agg, nc=old.nc, pval=old.pval, P=old.P, R=old.R)
        lv.Ac = galerkin(A, lv.agg, lv.pval, lv.nc)
        lv.Bc = old.Bc
        lv.omega, lv.rho = jacobi_weight(A, opts.arnoldi_m, opts.seed + 1, opts.jacobi_scale)
        lv.wdinv = lv.omega / A.diagonal()
        lv.smoother = old.smoother
        if lv.smoother == "chebyshev":
            lv.cheb = chebyshev_interval(lv.rho, opts)
        elif lv.smoother == "mcsgs":
            lv.colors = old.colors                       # the graph of A_k is unchanged
        levels.append(lv)
        A = lv.Ac
    levels.append(Level(A=A, B=H.levels[-1].B))
    out = Hierarchy(levels=levels, opts=opts)
    if A.shape[0] > opts.dense_max:
        raise OracleError("ECOARSEN", f"coarsest level has {A.shape[0]} unknowns")
    coarse_factor(out)
    return out


# ---------------------------------------------------------------------------
# Algorithms 4 and 5: V-cycle and K-cycle (zero initial guess)
# ---------------------------------------------------------------------------

def smooth(lv: Level, b, x):
    """One smoothing step S_k(b, A_k, x) (Section 2.2.1): damped Jacobi
    (eq. damped_jacobi) x <- x + omega D^{-1} (b - A x) by default."""
    if lv.smoother == "chebyshev":
        return chebyshev_smooth(lv, b, x)
    if lv.smoother == "mcsgs":
        return sgs_smooth(lv, b, x)
    return x + lv.wdinv * (b - lv.A @ x)


# ---------------------------------------------------------------------------
# Other smoothers: polynomial (Section 5, future work) and multi-colour
# symmetric Gauss-Seidel (Section 2.2.1)
# ---------------------------------------------------------------------------

def chebyshev_interval(rho: float, opts: Options):
    """The interval [a, b] of the spectrum of D^-1 A that the polynomial damps:
    b = cheb_upper * rho (the Arnoldi estimate errs low), a = b / cheb_ratio.
    Returns (theta, delta, degree): centre, half-width, polynomial degree."""
    b = opts.cheb_upper * rho
    a = b / opts.cheb_ratio
    return 0.5 * (b + a), 0.5 * (b - a), opts.cheb_degree


def chebyshev_smooth(lv: Level, b, x):
    """Chebyshev acceleration of the Jacobi iteration (the three-term
    recurrence of the Chebyshev polynomials, scaled to [a, b]): after m steps
    the error is T_m((theta - M)/delta) / T_m(theta/delta) times the initial
    error, M = D^-1 A, which is at most 1/T_m(theta/delta) on [a, b]."""
    theta, delta, m = lv.cheb
    dinv = 1.0 / lv.A.diagonal()
    sigma = theta / delta
    r = dinv * (b - lv.A @ x)                          # preconditioned residual
    d = r / theta
    x = x + d
    rho_prev = 1.0 / sigma
    for _ in range(1, m):
        rho_k = 1.0 / (2.0 * sigma - rho_prev)
        r = r - dinv * (lv.A @ d)
        d = (rho_k * rho_prev) * d + (2.0 * rho_k / delta) * r
        x = x + d
        rho_prev = rho_k
    return x


def color_greedy(A: sp.csr_matrix, stream: int) -> np.ndarray:
    """First-fit colouring of the graph of A (off-diagonal pattern): rows in
    decreasing priority h_i = node_hash(i, stream) take the smallest colour no
    neighbour already holds."""
    n = A.shape[0]
    prio = node_hash(np.arange(n), stream)
    color = np.full(n, -1, dtype=np.int64)
    for i in np.argsort(-prio.astype(np.int64), kind="stable"):
        nb = A.indices[A.indptr[i]:A.indptr[i + 1]]
        used = set(int(c) for c in color[nb[nb != i]] if c >= 0)
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


def color_parallel(A: sp.csr_matrix, stream: int) -> tuple:
    """The same colouring in synchronous rounds (Jones-Plassmann): in each
    round every uncoloured row whose priority beats all its uncoloured
    neighbours takes the smallest colour its coloured neighbours leave free.
    Returns (colors, rounds)."""
    n = A.shape[0]
    prio = node_hash(np.arange(n), stream).astype(np.int64)
    color = np.full(n, -1, dtype=np.int64)
    rounds = 0
    while np.any(color < 0):
        rounds += 1
        new = color.copy()
        for i in np.flatnonzero(color < 0):
            nb = A.indices[A.indptr[i]:A.indptr[i + 1]]
            nb = nb[nb != i]
            if np.any((color[nb] < 0) & (prio[nb] > prio[i])):
                continue
            used = set(int(c) for c in color[nb] if c >= 0)
            c = 0
            while c in used:
                c += 1
            new[i] = c
        color = new
    return color, rounds


def sgs_smooth(lv: Level, b, x):
    """Symmetric Gauss-Seidel in colour order: a forward sweep over the
    colours (rows of one colour are not coupled, so each colour updates at
    once: x_i += (b - A x)_i / a_ii), then a backward sweep."""
    d = lv.A.diagonal()
    ncol = int(lv.colors.max()) + 1
    for c in list(range(ncol)) + list(range(ncol - 1, -1, -1)):
        rows = np.flatnonzero(lv.colors == c)
        x = x.copy()
        x[rows] += (b[rows] - lv.A[rows] @ x) / d[rows]
    return x


def kcycle_coefficients(c, d, v, w, r, rt, variant: str):
    """Coefficients of the two-step inner Krylov update of Algorithm 5.

    c, d: the two inner-cycle corrections; v = A c, w = A d; r: the coarse
    right-hand side; rt = r - (alpha1/rho1) v, what the first step leaves.
    The CG variant pairs each vector with c or d (A-norm error), the GMRES
    variant with v or w (residual 2-norm).  Returns (coef_c, coef_d) with
    x = coef_c c + coef_d d.  When the second direction adds nothing
    (rho2 = beta - gamma^2/rho1 <= 0, a guard the paper leaves open) the first
    step alone is kept: (alpha1/rho1, 0)."""
    if variant == "cg":
        rho1, alpha1 = c @ v, c @ r
        gamma, beta, alpha2 = d @ v, d @ w, d @ rt
    else:
        rho1, alpha1 = v @ v, v @ r
        gamma, beta, alpha2 = w @ v, w @ w, w @ rt
    rho2 = beta - gamma * gamma / rho1
    if not rho2 > 0.0:
        return alpha1 / rho1, 0.0
    return alpha1 / rho1 - gamma * alpha2 / (rho1 * rho2), alpha2 / rho2


def vcycle(H: Hierarchy, k: int, b):
    """Algorithm 4 with x_k = 0 on entry: smoothing around one coarse-grid
    correction by a recursive cycle (or the exact solve on the coarsest level)."""
    lv = H.levels[k]
    x = smooth(lv, b, np.zeros_like(b))
    rc = lv.R @ (b - lv.A @ x)
    if k + 1 == H.L:
        xc = H.coarse_solve(rc)
    else:
        xc = cycle(H, k + 1, rc)
    return smooth(lv, b, x + lv.P @ xc)


def kcycle_correction(H: Hierarchy, kc: int, rc):
    """The coarse-grid correction of Algorithm 5 on level kc for the restricted
    residual rc: the level's cycle is used as the preconditioner of at most two
    steps of a Krylov method on A_kc e = rc, started from e = 0.

    One inner cycle c gives the best multiple of c (A-norm error for the CG
    variant, residual 2-norm for the GMRES variant); if what it leaves,
    r~ = rc - A_kc (alpha1/rho1) c, is not below t ||rc||, a second inner cycle
    d on r~ and the best element of span{c, d} (kcycle_coefficients).
    Returns (e, steps) with steps the number of inner cycles that entered e.
    Guard the paper leaves open: rho1 <= 0 gives e = 0."""
    if kc == H.L:
        return H.coarse_solve(rc), 0
    cg = H.opts.krylov == "fcg"
    Ac = H.levels[kc].A
    c = cycle(H, kc, rc)
    v = Ac @ c
    rho1, alpha1 = ((c @ v), (c @ rc)) if cg else ((v @ v), (v @ rc))
    if not rho1 > 0.0:
        return np.zeros_like(rc), 0
    rt = rc - (alpha1 / rho1) * v
    if np.linalg.norm(rt) <= H.opts.kcycle_t * np.linalg.norm(rc):
        return (alpha1 / rho1) * c, 1
    d = cycle(H, kc, rt)
    coef_c, coef_d = kcycle_coefficients(c, d, v, Ac @ d, rc, rt, "cg" if cg else "gmres")
    return coef_c * c + coef_d * d, 2


def kcycle(H: Hierarchy, k: int, b):
    """Algorithm 5 with x_k = 0 on entry (readings in the module docstring):
    the V-cycle's smoothing and transfers around the Krylov-accelerated coarse
    correction of kcycle_correction."""
    lv = H.levels[k]
    x = smooth(lv, b, np.zeros_like(b))
    rc = lv.R @ (b - lv.A @ x)
    xc, _ = kcycle_correction(H, k + 1, rc)
    return smooth(lv, b, x + lv.P @ xc)


def cycle(H: Hierarchy, k: int, b):
    """K-cycle on the top ``kcycle_levels`` levels, V-cycle below (Section 2.2)."""
    if H.L == 0:
        return H.coarse_solve(b)
    if k < H.opts.kcycle_levels:
        return kcycle(H, k, b)
    return vcycle(H, k, b)


# ---------------------------------------------------------------------------
# Outer Krylov: flexible CG and flexible GMRES (Sections 2.2 and 4)
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    relres: float                     # true ||b - A x|| / ||b||
    converged: bool
    history: list


def fcg(A: sp.csr_matrix, b, precond, rtol: float, max_iter: int) -> SolveResult:
    """Flexible CG with one stored direction, x_0 = 0.  Stops when the
    recurrence residual satisfies ||r|| <= rtol ||b|| and the recomputed true
    residual agrees; otherwise it restarts from the true residual."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return SolveResult(x, 0, 0.0, True, [])
    r = b.copy()
    z = precond(r)
    p = z.copy()
    hist = []
    it = 0
    while it < max_iter:
        it += 1
        q = A @ p
        pq = p @ q
        if not pq > 0.0:
            raise OracleError("EBREAKDOWN", "p^T A p <= 0")
        alpha = (p @ r) / pq
        x = x + alpha * p
        r = r - alpha * q
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if rel <= rtol:
            r = b - A @ x
            if np.linalg.norm(r) / bnorm <= rtol:
                return SolveResult(x, it, np.linalg.norm(r) / bnorm, True, hist)
            z = precond(r)
            p = z.copy()
            continue
        z = precond(r)
        beta = -(z @ q) / pq
        p = z + beta * p
    rel = np.linalg.norm(b - A @ x) / bnorm
    return SolveResult(x, it, rel, rel <= rtol, hist)


def fgmres(A: sp.csr_matrix, b, precond, rtol: float, max_iter: int, restart: int) -> SolveResult:
    """Right-preconditioned flexible GMRES(restart), x_0 = 0 (Saad's FGMRES):
    the preconditioned vectors z_j are stored and x = x_0 + Z y."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return SolveResult(x, 0, 0.0, True, [])
    hist = []
    it = 0
    while it < max_iter:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta / bnorm <= rtol:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        Hm = np.zeros((m + 1, m))
        V[0] = r / beta
        g = np.zeros(m + 1)
        g[0] = beta
        cs = np.zeros(m)
        sn = np.zeros(m)
        j_done = 0
        for j in range(m):
            it += 1
            Z[j] = precond(V[j])
            w = A @ Z[j]
            for i in range(j + 1):
                Hm[i, j] = V[i] @ w
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0.0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):                         # apply previous rotations
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = math.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j], sn[j] = Hm[j, j] / den, Hm[j + 1, j] / den
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= rtol or it >= max_iter:
                break
        y = sla.solve_triangular(Hm[:j_done, :j_done], g[:j_done])
        x = x + Z[:j_done].T @ y
    rel = np.linalg.norm(b - A @ x) / bnorm
    return SolveResult(x, it, rel, rel <= rtol, hist)


def solve(H: Hierarchy, b, rtol: float = 1e-8, max_iter: int | None = None) -> SolveResult:
    """Outer Krylov solve of A_0 x = b preconditioned by one cycle(0)."""
    max_iter = H.opts.max_iter if max_iter is None else max_iter
    A = H.levels[0].A
    b = np.asarray(b, dtype=np.float64)
    if not np.all(np.isfinite(b)):
        raise OracleError("ENANINF", "non-finite right-hand side")

    def precond(r):
        return cycle(H, 0, r)

    if H.opts.krylov == "fcg":
        return fcg(A, b, precond, rtol, max_iter)
    return fgmres(A, b, precond, rtol, max_iter, H.opts.gmres_restart)


def solve_multi(H: Hierarchy, Bm, rtol: float = 1e-8):
    """Several right-hand sides: each column solved alone with the same hierarchy."""
    return [solve(H, Bm[:, c], rtol) for c in range(Bm.shape[1])]


def solve_batch(row_ptr, col, val, sys_off, b, opts: Options, rtol: float = 1e-8):
    """Independent systems on the block diagonal: each is set up and solved as
    if alone (its node hash uses the local row index)."""
    A = validate_csr(row_ptr, col, val)
    out = []
    for s in range(len(sys_off) - 1):
        lo, hi = int(sys_off[s]), int(sys_off[s + 1])
        As = A[lo:hi, lo:hi].tocsr()
        As.sort_indices()
        H = setup(As.indptr, As.indices, As.data, opts)
        out.append(solve(H, b[lo:hi], rtol))
    return out


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _segmax(vals, indptr, empty):
    """Max of vals over each CSR segment; ``empty`` for empty segments."""
    n = indptr.shape[0] - 1
    out = np.full(n, empty, dtype=np.asarray(vals).dtype)
    nonempty = indptr[1:] > indptr[:-1]
    if np.any(nonempty):
        out[nonempty] = np.maximum.reduceat(vals, indptr[:-1][nonempty])
    return out


def operator_complexity(H: Hierarchy) -> float:
    nnz0 = H.levels[0].A.nnz
    return sum(lv.A.nnz for lv in H.levels) / nnz0


def grid_complexity(H: Hierarchy) -> float:
    return sum(lv.n for lv in H.levels) / H.levels[0].n
