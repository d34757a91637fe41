"""FP64 numpy reference of the learned Newton guess (test infrastructure only).

The network: 5 invariant features -> 64 -> 64 -> 2, ReLU, outputs the
standardised (log(p/D), log Gamma) of the converged inversion.  Parameters in
one flat vector (the C ABI's layout):
  W1 [64][5] | b1 [64] | W2 [64][64] | b2 [64] | W3 [2][64] | b3 [2]
(row = output unit).  Loss: mean over the 2B outputs of (y - t)^2.
Optimiser: Adam (Kingma & Ba 2015) with bias correction.

Features of a conserved state (D, S, U, B), the five rotation invariants on
which the one-unknown inversion depends (it uses only D, U, S^2, B^2 and
tau = S.B):
  f0 = log(U/D), f1 = |S|/U, f2 = B^2/U, f3 = tau^2/(S^2 B^2 + 1e-300),
  f4 = log D.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 5, 64, 2
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def features(D, S, U, B):
    """D, U: (n,); S, B: (n, 3).  Returns (n, 5)."""
    S2 = np.sum(S * S, axis=1)
    B2 = np.sum(B * B, axis=1)
    tau = np.sum(S * B, axis=1)
    return np.stack([np.log(U / D), np.sqrt(S2) / U, B2 / U, tau * tau / (S2 * B2 + 1e-300),
                     np.log(D)], axis=1)


def targets(rho, v, p):
    """(log(p/D), log Gamma) of primitives rho (n,), v (n, 3), p (n,)."""
    v2 = np.sum(v * v, axis=1)
    lor = 1.0 / np.sqrt(1.0 - v2)
    return np.stack([np.log(p / (rho * lor)), np.log(lor)], axis=1)


def forward(theta, X):
    """X: (B, 5) standardised features.  Returns (Y (B, 2), cache)."""
    p = unpack(theta)
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ p["W3"].T + p["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss(Y, T):
    return float(np.mean((Y - T) ** 2))


def loss_grad(Y, T):
    return 2.0 * (Y - T) / Y.size


def backward(theta, cache, dY):
    """Gradient of the loss with respect to theta (flat), given dL/dY."""
    p = unpack(theta)
    X, Z1, H1, Z2, H2 = cache
    g = {}
    g["W3"] = dY.T @ H2
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ p["W3"]) * (Z2 > 0)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * (Z1 > 0)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)


def adam(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
