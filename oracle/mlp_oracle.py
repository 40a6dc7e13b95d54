"""FP64 oracle of the learned Jacobi weights — TEST INFRASTRUCTURE ONLY.

Not part of the paper (which fixes omega per level by eq. damped_jacobi and
Section 2.2.1); this is the extension that replaces the single omega_k by a
per-row omega_i predicted by a small MLP from local stencil features.  The
definitions below are the contract the HIP kernels follow:

features of row i on level k (9 values, then rounded to bfloat16):
  f0 = log|a_ii| - mean over the level of log|a_jj|
  f1..f6 = the six largest |a_ij| / |a_ii| over j != i, descending, zero-padded
  f7 = (sum_j a_ij) / a_ii
  f8 = k
MLP 9 -> 32 -> 32 -> 1 with ReLU: bfloat16 weights and inputs (round to
nearest even), FP32 biases; hidden activations are rounded to bfloat16 before
the next layer (straight-through in the backward pass).  Each pre-activation
is the FP64 sum of the bias and the products of bfloat16-rounded operands
(every such product is exact); the kernels accumulate in FP32, and the GPU
tests bound that difference, including the bfloat16 roundings of hidden units
that it can flip, instead of reproducing the kernel's summation order.
omega_i = sigmoid(y_i) * 2|a_ii| / (|a_ii| + sum_{j != i} |a_ij|): then
2 D Omega^-1 - A is strictly diagonally dominant with a positive diagonal, so
the smoother x += Omega D^-1 (b - A x) converges for SPD A.

Training loss on level k over S error samples e_s (the part of a vector that
the coarse space range(P_k) cannot represent, e = v - P P^T v, P^T P = I):
  L = (1/S) sum_s ||(I - W A) e_s||_A^2 / ||e_s||_A^2,   W = diag(omega_i / a_ii).
Two-grid training samples (the errors the smoother of level k meets in a
cycle, after the coarse correction of Algorithm 4 with an exact coarse solve):
  e~ = (I - P A_c^-1 P^T A) e,   A_c = P^T A P,
the A-orthogonal projection of e onto the complement of range(P); the loss
above on such samples is the two-grid post-smoothing factor.
Weight layout (1409 FP32 masters): W1[32][9], b1[32], W2[32][32], b2[32],
W3[32], b3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle.amg_oracle import unit_uniform

N_IN, N_H = 9, 32
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)   # 1409


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = w[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SIZES])


def bf16(x):
    """Round float32 values to bfloat16 (round to nearest, ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(A: sp.csr_matrix, level: int) -> np.ndarray:
    n = A.shape[0]
    d = A.diagonal()
    logd = np.log(np.abs(d))
    mean = logd.mean()
    F = np.zeros((n, N_IN))
    F[:, 0] = logd - mean
    for i in range(n):
        s, e = A.indptr[i], A.indptr[i + 1]
        cols, vals = A.indices[s:e], A.data[s:e]
        off = np.sort(np.abs(vals[cols != i]) / abs(d[i]))[::-1][:6]
        F[i, 1:1 + off.size] = off
        F[i, 7] = vals.sum() / d[i]
    F[:, 8] = level
    return F


def omega_bound(A: sp.csr_matrix) -> np.ndarray:
    d = np.abs(A.diagonal())
    rowabs = np.asarray(abs(A).sum(axis=1)).ravel()
    return 2.0 * d / (d + (rowabs - d))


def forward(w, F, round_bf16=True):
    """y = W3 h2 + b3, h2 = q(relu(W2 h1 + b2)), h1 = q(relu(W1 q(x) + b1)) with
    q = bfloat16 rounding (identity when round_bf16 is False) and the weights
    W1, W2, W3 rounded the same way; sums in FP64.  Returns y and the
    intermediates needed by backward."""
    p = unpack(w)
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    X = r(F)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    z1 = X @ W1.T + p["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + p["b2"]
    h2 = r(np.maximum(z2, 0.0))
    y = h2 @ W3 + p["b3"][0]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, W1=W1, W2=W2, W3=W3)


def omega(w, A, F, round_bf16=True):
    y, _ = forward(w, F, round_bf16)
    return 1.0 / (1.0 + np.exp(-y)) * omega_bound(A)


def projected_errors(A: sp.csr_matrix, agg, pval, nc: int, nsamples: int, seed: int) -> np.ndarray:
    """e_s = v_s - P P^T v_s with v_s[i] = unit_uniform(i, seed + s); [n][S]."""
    n = A.shape[0]
    P = sp.csr_matrix((pval, agg, np.arange(n + 1)), shape=(n, nc))
    E = np.zeros((n, nsamples))
    for s in range(nsamples):
        v = unit_uniform(np.arange(n), seed + s)
        E[:, s] = v - P @ (P.T @ v)
    return E


def coarse_corrected(A: sp.csr_matrix, agg, pval, nc: int, E) -> np.ndarray:
    """e~_s = e_s - P A_c^-1 P^T A e_s with A_c = P^T A P (sparse LU); [n][S]."""
    from scipy.sparse.linalg import splu
    n = A.shape[0]
    P = sp.csr_matrix((pval, agg, np.arange(n + 1)), shape=(n, nc))
    Ac = (P.T @ A @ P).tocsc()
    Y = splu(Ac).solve(np.asarray(P.T @ (A @ E)))
    return E - P @ Y


def loss_omega(A: sp.csr_matrix, E, om):
    """Smoothing loss as a function of the per-row weights omega and its
    derivative dL/domega_i (W = diag(omega_i / a_ii))."""
    a = A.diagonal()
    AE = A @ E
    ee = np.einsum("is,is->s", E, AE)
    E2 = E - (om / a)[:, None] * AE
    AE2 = A @ E2
    num = np.einsum("is,is->s", E2, AE2)
    S = E.shape[1]
    loss = float(np.mean(num / ee))
    domega = (-2.0 / S) * np.sum(AE2 * AE / ee[None, :], axis=1) / a
    return loss, domega


def loss_and_grad(w, A: sp.csr_matrix, F, E, round_bf16=True):
    """Smoothing loss and its gradient with respect to the 1409 weights
    (chain rule through omega_i = sigmoid(y_i) beta_i and the network)."""
    y, c = forward(w, F, round_bf16)
    beta = omega_bound(A)
    sig = 1.0 / (1.0 + np.exp(-y))
    loss, domega = loss_omega(A, E, sig * beta)
    dy = domega * beta * sig * (1.0 - sig)
    g = {}
    g["W3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, c["W3"])
    dz2 = dh2 * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ c["W2"]
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def init_weights(seed: int = 0) -> np.ndarray:
    """He-scaled normal weights; b3 = 1.5 so that sigmoid(y) starts near 0.8."""
    rng = np.random.default_rng(seed)
    d = {"W1": rng.standard_normal((N_H, N_IN)) * np.sqrt(2.0 / N_IN), "b1": np.zeros(N_H),
         "W2": rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H), "b2": np.zeros(N_H),
         "W3": rng.standard_normal(N_H) * np.sqrt(1.0 / N_H) * 0.1, "b3": np.array([1.5])}
    return pack(d)
