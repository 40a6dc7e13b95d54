"""How far the learned-weight kernels may lie from the FP64 oracle.

The kernels form every pre-activation of the network in FP32 (the bias, then
one fused multiply-add per input), the oracle in FP64.  A product of two
bfloat16 values is exact in either precision, so before a hidden unit is
quantised the only difference is the FP32 rounding of the running sum:
|z32 - z| <= gamma_m (|b| + sum |w x|), gamma_m = m u / (1 - m u), u = 2^-24,
m additions.  A unit whose interval [z - e, z + e] holds a bfloat16 rounding
boundary, or 0 where ReLU switches, may be quantised differently by the
kernel: it may move by one bfloat16 step and its ReLU mask may differ.  The
functions below carry these intervals through the network to y and omega,
and to first order through the loss and its weight gradient (the backward
kernel works in FP32 from dL/dy rounded to FP32).  They bound the kernel's
deviation; they do not reproduce its summation order.
"""
import numpy as np

from oracle import mlp_oracle as M

U32 = 2.0 ** -24


def gamma(m: int) -> float:
    return m * U32 / (1.0 - m * U32)


def forward_bounds(w, F):
    """Oracle forward pass plus, per row and hidden unit, how far the kernel's
    quantised activation may lie from the oracle's (d1, d2), which units may be
    quantised or masked differently (u1, u2), and the bound ey on |y_k - y|."""
    p = M.unpack(w)
    X = M.bf16(F)
    W1, W2, W3 = M.bf16(p["W1"]), M.bf16(p["W2"]), M.bf16(p["W3"])
    b1, b2, b3 = p["b1"], p["b2"], p["b3"][0]

    def q(a):
        return M.bf16(np.maximum(a, 0.0))

    z1 = X @ W1.T + b1
    e1 = gamma(M.N_IN) * (np.abs(X) @ np.abs(W1).T + np.abs(b1))
    h1, lo1, hi1 = q(z1), q(z1 - e1), q(z1 + e1)
    d1 = np.maximum(hi1 - h1, h1 - lo1)
    u1 = lo1 != hi1
    z2 = h1 @ W2.T + b2
    e2 = d1 @ np.abs(W2).T + gamma(M.N_H) * ((h1 + d1) @ np.abs(W2).T + np.abs(b2))
    h2, lo2, hi2 = q(z2), q(z2 - e2), q(z2 + e2)
    d2 = np.maximum(hi2 - h2, h2 - lo2)
    u2 = lo2 != hi2
    y = h2 @ W3 + b3
    ey = d2 @ np.abs(W3) + gamma(M.N_H) * ((h2 + d2) @ np.abs(W3) + abs(b3))
    return dict(X=X, W1=W1, W2=W2, W3=W3, z1=z1, z2=z2, h1=h1, h2=h2, d1=d1, d2=d2, u1=u1, u2=u2, y=y,
                ey=ey)


def omega_bounds(w, A, F):
    """(omega, bound on |omega_kernel - omega|, rows with a unit that may flip,
    forward intermediates).  The sigmoid moves by at most
    s(1-s)(e^ey - 1) <= s(1-s) ey e^ey; the kernel's FP64 sigmoid and row sums
    add rounding at the 1e-13 level."""
    fb = forward_bounds(w, F)
    sig = 1.0 / (1.0 + np.exp(-fb["y"]))
    beta = M.omega_bound(A)
    om = sig * beta
    s1 = sig * (1.0 - sig)
    dom = beta * s1 * fb["ey"] * np.exp(fb["ey"]) + 1e-13 * om
    flips = fb["u1"].any(axis=1) | fb["u2"].any(axis=1)
    fb.update(sig=sig, beta=beta, s1=s1)
    return om, dom, flips, fb


def loss_grad_bounds(w, A, F, E):
    """Oracle loss and gradient with bounds on the kernel's deviation:
    (loss, dloss, grad, dgrad) with dgrad elementwise over the 1409 weights."""
    om, dom, _flips, fb = omega_bounds(w, A, F)
    loss, g_om = M.loss_omega(A, E, om)
    a = A.diagonal()
    Aabs = abs(A)
    AE = A @ E
    ee = np.einsum("is,is->s", E, AE)
    S = E.shape[1]
    # loss: first order in delta omega, the quadratic term, FP64 rounding
    de = (dom / np.abs(a))[:, None] * np.abs(AE)
    quad = np.sum(np.einsum("is,is->s", de, Aabs @ de) / ee) / S
    dloss = float(np.abs(g_om) @ dom + quad + 1e-12 * loss)
    # dL/dy and how far the kernel's may lie from it
    dAE2 = Aabs @ de
    dg_om = (2.0 / S) * np.sum(dAE2 * np.abs(AE) / ee[None, :], axis=1) / np.abs(a)
    s1, beta, ey = fb["s1"], fb["beta"], fb["ey"]
    ds1 = s1 * ey * np.exp(ey)
    dy = g_om * beta * s1
    ddy = dg_om * beta * (s1 + ds1) + np.abs(g_om) * beta * ds1 + (U32 + 1e-12) * np.abs(dy)
    dyU = np.abs(dy) + ddy
    # backward, layer by layer (kernel: FP32, rows summed per block accumulator)
    n = A.shape[0]
    tiles = (n + 63) // 64
    gacc = gamma(64 * -(-tiles // min(tiles, 1024)))
    h1, h2, d1, d2, X = fb["h1"], fb["h2"], fb["d1"], fb["d2"], np.abs(fb["X"])
    W2a, W3a = np.abs(fb["W2"]), np.abs(fb["W3"])
    on2, on1 = fb["z2"] > 0, fb["z1"] > 0
    u2, u1 = fb["u2"], fb["u1"]
    gW3 = ddy @ (h2 + d2) + np.abs(dy) @ d2 + gacc * (dyU @ (h2 + d2))
    gb3 = ddy.sum() + gacc * dyU.sum()
    m2U = (on2 | u2) * dyU[:, None] * W3a[None, :]
    dz2 = on2 * dy[:, None] * fb["W3"][None, :]
    ddz2 = np.where(u2, m2U, on2 * ddy[:, None] * W3a[None, :]) + U32 * m2U
    gW2 = ddz2.T @ (h1 + d1) + np.abs(dz2).T @ d1 + gacc * (m2U.T @ (h1 + d1))
    gb2 = ddz2.sum(axis=0) + gacc * m2U.sum(axis=0)
    dh1 = dz2 @ fb["W2"]
    ddh1 = ddz2 @ W2a + gamma(M.N_H) * (m2U @ W2a)
    m1U = (on1 | u1) * (np.abs(dh1) + ddh1)
    ddz1 = np.where(u1, m1U, on1 * ddh1)
    gW1 = ddz1.T @ X + gacc * (m1U.T @ X)
    gb1 = ddz1.sum(axis=0) + gacc * m1U.sum(axis=0)
    # totals: the final FP64 sum of the block partials is stored in FP32
    bound = M.pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": np.array([gb3])})
    mag = M.pack({"W1": m1U.T @ X, "b1": m1U.sum(axis=0), "W2": m2U.T @ (h1 + d1), "b2": m2U.sum(axis=0),
                  "W3": dyU @ (h2 + d2), "b3": np.array([dyU.sum()])})
    _, grad = M.loss_and_grad(w, A, F, E)
    return loss, dloss, grad, bound + (U32 + 1e-10) * mag
