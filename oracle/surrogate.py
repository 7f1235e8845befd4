"""FP64 oracle of the learned surrogate (test infrastructure only).

The surrogate is an addition to the paper's method: a small MLP maps a
normalised window of the analytic fringe signal (Eq. 1) to (cos w, sin w),
and its prediction is accepted only after a MUSIC null-spectrum check and a
root-MUSIC refinement, with the plain method of Sec. 3 as the fallback.  This
module holds the plain definitions the GPU kernels are checked against:

  features    16 central samples of the window, de-rotated by the phase of the
              central sample and divided by the window's RMS magnitude,
              flattened as [Re(16), Im(16)]
  forward     32 -> GELU(64) -> GELU(64) -> 2, weights and activations rounded
              to bfloat16 (round to nearest even), accumulation in FP64 (or
              FP32 before each bfloat16 rounding, matching the kernel's
              precision where the rounding decides a value)
  loss        mean over the batch of the squared error to (cos w, sin w)
  backward    exact gradients of that loss; the bfloat16 roundings are
              treated as identity (straight-through)
  adam        Kingma and Ba's Adam with bias correction
  null_spectrum  1 - |u1^H a(w)|^2 / L: the MUSIC null spectrum a^H C a / L
              with C = I - u1 u1^H (Stoica and Moses), 0 at a true tone
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_FEAT_SAMPLES = 16
HIDDEN = 64
SHAPES = {"W1": (32, HIDDEN), "b1": (HIDDEN,), "W2": (HIDDEN, HIDDEN), "b2": (HIDDEN,),
          "W3": (HIDDEN, 2), "b3": (2,)}


def bf16_round(x) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest, ties to even); returned as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def features(win: np.ndarray) -> np.ndarray:
    """(M, N) complex windows, N >= 16 -> (M, 32) features."""
    win = np.asarray(win, dtype=np.complex128)
    N = win.shape[1]
    c = N // 2
    h = N_FEAT_SAMPLES // 2
    cen = win[:, c - h:c + h]
    g = win[:, c]
    mag = np.abs(g)
    rot = np.where(mag > 0, np.conj(g) / np.where(mag > 0, mag, 1.0), 1.0)
    rms = np.sqrt(np.mean(np.abs(win) ** 2, axis=1))
    rms = np.where(rms > 0, rms, 1.0)
    z = cen * (rot / rms)[:, None]
    return np.concatenate([z.real, z.imag], axis=1)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def init_params(seed: int) -> dict:
    """Seeded FP32 master weights (scaled normal initialisation)."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, s in SHAPES.items():
        if k.startswith("W"):
            p[k] = (rng.standard_normal(s) / math.sqrt(s[0])).astype(np.float32)
        else:
            p[k] = (0.1 * rng.standard_normal(s)).astype(np.float32)
    return p


def forward(p: dict, X: np.ndarray, quantize: bool = True, fp32_acc: bool = False) -> dict:
    """Forward pass; returns the cache (Z1, H1, Z2, H2, Y and the operands used)."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    acc = (lambda a: a.astype(np.float32).astype(np.float64)) if fp32_acc else (lambda a: a)
    Xq = q(X)
    W1, W2, W3 = q(p["W1"]), q(p["W2"]), q(p["W3"])
    b1, b2, b3 = (np.asarray(p[k], dtype=np.float64) for k in ("b1", "b2", "b3"))
    Z1 = acc(Xq @ W1 + b1)
    H1 = q(gelu(Z1))
    Z2 = acc(H1 @ W2 + b2)
    H2 = q(gelu(Z2))
    Y = acc(H2 @ W3 + b3)
    return {"X": Xq, "W1": W1, "W2": W2, "W3": W3, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2, "Y": Y}


def targets(w: np.ndarray) -> np.ndarray:
    return np.stack([np.cos(w), np.sin(w)], axis=1)


def loss(Y: np.ndarray, T: np.ndarray) -> float:
    return float(np.mean(np.sum((Y - T) ** 2, axis=1)))


def backward(cache: dict, T: np.ndarray) -> dict:
    """Gradients of loss(Y, T) with respect to every parameter."""
    Y = cache["Y"]
    B = Y.shape[0]
    dY = 2.0 * (Y - T) / B
    g = {"W3": cache["H2"].T @ dY, "b3": dY.sum(0)}
    dZ2 = (dY @ cache["W3"].T) * gelu_grad(cache["Z2"])
    g["W2"] = cache["H1"].T @ dZ2
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2 @ cache["W2"].T) * gelu_grad(cache["Z1"])
    g["W1"] = cache["X"].T @ dZ1
    g["b1"] = dZ1.sum(0)
    return g


def adam(p: dict, g: dict, m: dict, v: dict, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (t counts from 1); returns new (p, m, v) in float64."""
    P, M, V = {}, {}, {}
    for k in p:
        M[k] = b1 * m[k] + (1 - b1) * g[k]
        V[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = M[k] / (1 - b1 ** t)
        vh = V[k] / (1 - b2 ** t)
        P[k] = np.asarray(p[k], dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return P, M, V


def predict_omega(Y: np.ndarray) -> np.ndarray:
    return np.arctan2(Y[:, 1], Y[:, 0])


def null_spectrum(u1: np.ndarray, w: np.ndarray) -> np.ndarray:
    """1 - |u1^H a(w)|^2 / L for unit u1 (M, L) and frequencies w (M,)."""
    L = u1.shape[1]
    a = np.exp(1j * np.outer(w, np.arange(L)))
    return 1.0 - np.abs(np.sum(np.conj(u1) * a, axis=1)) ** 2 / L
