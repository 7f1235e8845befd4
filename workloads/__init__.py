"""Seeded synthetic fringe workloads.

This module only draws inputs; it holds none of the demodulation arithmetic.
Both sides of every parity check (the GPU library and the FP64 CPU oracle)
receive the exact bytes produced here.

Fringe model (paper, Sec. 2 and Eq. 1): a time-lapsed stack of carrier
fringes  I = a + b*cos(carrier + phi) + noise,  where phi is the
diffusion-induced phase.  The diffusion profile is the classical
error-function solution of Fick's second law (paper, Appendix, Eq. 16):
phi(y, t) = A * erf((y - y0) / w_t) with w_t = sqrt(4 D t).

Noise convention: real frames get i.i.d. N(0, s2) with
s2 = (b^2 / 2) * 10^(-SNR/10), i.e. SNR is measured against the AC fringe
power.  Complex frames (Eq. 1 directly) get circular noise with
E|eta|^2 = A^2 * 10^(-SNR/10).

Workload recipes (all seeded):
  cfg1  one 256x256 FP64 frame, carrier 1/8 cyc/px along x, phi = 2*erf((y-128)/16),
        SNR 20 dB, seed 0; x windows N=16, L=4.
  cfg2  100 frames of 1024x1024 FP32, carrier 0.1 cyc/px at 30 degrees,
        phi = 6*erf((y-512)/w_t), w_t = 8*32^(t/99), SNR 10 dB, seed t;
        x and y windows N=32, L=6.
  cfg3  64 frames of mixed sizes 512x512 ... 2048x1536, L in {4,6,8},
        N = 2L+8, SNR ~ U(5,20) dB, carrier ~ U(1/12,1/6) cyc/px at
        U(30,60) degrees, w ~ U(16,128) px, seed 3000+k; FP32.
  cfg4  16 frames of 4096x4096 stored FP16, carrier 1/8 cyc/px at 45 degrees,
        phi = 6*erf((y-2048)/w_t), w_t = 16*16^(t/15), SNR 10 dB, seed 4000+t;
        N=32, L=8.
  cfg5  training lines of 128 samples, random carrier 1/16..1/4 cyc/px,
        SNR 0..30 dB (surrogate training set).
  exp   stand-in for the paper's experimental series (Sec. 4): 19 frames of
        1850x700 8-bit samples taken at 120, 240, ..., 600 s and then every
        300 s to 4800 s; carrier 0.11 cyc/px at 35 degrees, phi = 5*erf((y-350)/w_t)
        with w_t = 6*sqrt(t/120 s) (Fick diffusion), SNR 12 dB before
        quantisation, seed 5000+i; line windows N = 15 (the paper's 2L+1 with
        L = 7) and covariance size 7.

  sweep window-size sweep field: phi = w0 (x + y) + A sin(k x) + A sin(k y),
        w0 = 1 rad/px, A k = 0.6 rad/px, k = 2 pi / 48, so the local frequency
        swings over 0.4 .. 1.6 rad/px and the third derivative of the phase
        (the bias of a window, which is exact for linear chirps) is 0.6 k^2.

8-bit frames are round(255 * I) clipped to 0..255.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import erf

A_DC = 0.5
B_AC = 0.4

CFG3_SIZES = [(512, 512), (768, 512), (768, 768), (1024, 768),
              (1024, 1024), (1536, 1024), (1536, 1536), (2048, 1536)]


@dataclass
class Frame:
    """One synthetic frame plus the closed-form truth of its local frequency."""
    data: np.ndarray            # (H, W) row-major; float16/32/64 or complex
    L: int
    N: int
    dirs: str                   # "x", "y" or "xy"
    truth_wx: object = None     # callable (ys, xs) -> rad/px, or None
    truth_wy: object = None
    meta: dict = field(default_factory=dict)

    @property
    def width(self) -> int:
        return self.data.shape[1]

    @property
    def height(self) -> int:
        return self.data.shape[0]


def _noise_sigma(snr_db: float) -> float:
    return math.sqrt(B_AC * B_AC / 2.0 * 10.0 ** (-snr_db / 10.0))


def erf_fringe(W, H, f0, angle_deg, amp, y0, w, snr_db, seed, dtype):
    """I = a + b cos(2 pi f0 (x cos t + y sin t) + amp*erf((y-y0)/w)) + noise."""
    th = math.radians(angle_deg)
    fx, fy = f0 * math.cos(th), f0 * math.sin(th)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    phase = 2.0 * math.pi * (fx * x + fy * y) + amp * erf((y - y0) / w)
    img = A_DC + B_AC * np.cos(phase)
    rng = np.random.default_rng(seed)      # an int seed or an existing Generator
    img = img + rng.standard_normal((H, W)) * _noise_sigma(snr_db)
    wx = 2.0 * math.pi * fx
    wy0 = 2.0 * math.pi * fy

    def truth_wx(ys, xs):
        return np.full(np.broadcast(ys, xs).shape, wx)

    def truth_wy(ys, xs):
        ys = np.asarray(ys, dtype=np.float64)
        val = wy0 + amp * 2.0 / math.sqrt(math.pi) * np.exp(-((ys - y0) / w) ** 2) / w
        return np.broadcast_to(val, np.broadcast(ys, xs).shape)

    if np.dtype(dtype) == np.uint8:
        return np.clip(np.rint(img * 255.0), 0, 255).astype(np.uint8), truth_wx, truth_wy
    return img.astype(dtype), truth_wx, truth_wy


def cfg1() -> Frame:
    """256x256 FP64, carrier 1/8 cyc/px along x, phi = 2 erf((y-128)/16), 20 dB, seed 0."""
    W = H = 256
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    img = A_DC + B_AC * np.cos(2.0 * math.pi * x / 8.0 + 2.0 * erf((y - 128.0) / 16.0))
    img = img + np.random.default_rng(0).standard_normal((H, W)) * _noise_sigma(20.0)
    return Frame(img.astype(np.float64), L=4, N=16, dirs="x",
                 truth_wx=lambda ys, xs: np.full(np.broadcast(ys, xs).shape, math.pi / 4),
                 meta={"cfg": 1})


def cfg2_frame(t: int) -> Frame:
    W = H = 1024
    w_t = 8.0 * 32.0 ** (t / 99.0)
    img, twx, twy = erf_fringe(W, H, 0.1, 30.0, 6.0, 512.0, w_t, 10.0, t, np.float32)
    return Frame(img, L=6, N=32, dirs="xy", truth_wx=twx, truth_wy=twy,
                 meta={"cfg": 2, "t": t, "w": w_t})


def cfg2(frames=range(100)) -> list:
    return [cfg2_frame(t) for t in frames]


def cfg3_frame(k: int) -> Frame:
    W, H = CFG3_SIZES[k % 8]
    L = [4, 6, 8][k % 3]
    rng = np.random.default_rng(3000 + k)
    snr = rng.uniform(5.0, 20.0)
    f0 = rng.uniform(1.0 / 12.0, 1.0 / 6.0)
    ang = rng.uniform(30.0, 60.0)
    w = rng.uniform(16.0, 128.0)
    # the noise continues the same generator stream after the four parameter draws
    img, twx, twy = erf_fringe(W, H, f0, ang, 6.0, H / 2.0, w, snr, rng, np.float32)
    return Frame(img, L=L, N=2 * L + 8, dirs="xy", truth_wx=twx, truth_wy=twy,
                 meta={"cfg": 3, "k": k, "snr": snr, "f0": f0, "angle": ang, "w": w})


def cfg3(frames=range(64)) -> list:
    return [cfg3_frame(k) for k in frames]


def cfg4_frame(t: int, size: int = 4096, dtype=np.float16) -> Frame:
    """Frame t of the FP16 series; dtype=np.float64 gives the same frame before its
    FP16 storage rounding (same seed, same noise draws)."""
    W = H = size
    w_t = 16.0 * 16.0 ** (t / 15.0)
    img, twx, twy = erf_fringe(W, H, 1.0 / 8.0, 45.0, 6.0, H / 2.0, w_t, 10.0, 4000 + t, dtype)
    return Frame(img, L=8, N=32, dirs="xy", truth_wx=twx, truth_wy=twy,
                 meta={"cfg": 4, "t": t, "w": w_t})


def cfg4(frames=range(16)) -> list:
    return [cfg4_frame(t) for t in frames]


EXP_TIMES_S = [120.0 * k for k in range(1, 6)] + [600.0 + 300.0 * k for k in range(1, 15)]


def exp_frame(i: int) -> Frame:
    """Frame i of the 19-frame 1850x700 8-bit stand-in series."""
    W, H = 1850, 700
    t = EXP_TIMES_S[i]
    w_t = 6.0 * math.sqrt(t / 120.0)
    img, twx, twy = erf_fringe(W, H, 0.11, 35.0, 5.0, H / 2.0, w_t, 12.0, 5000 + i, np.uint8)
    return Frame(img, L=7, N=15, dirs="xy", truth_wx=twx, truth_wy=twy,
                 meta={"cfg": "exp", "i": i, "t_s": t, "w": w_t})


def exp_series(frames=range(19)) -> list:
    return [exp_frame(i) for i in frames]


def sweep_frame(W, H, snr_db, seed, w0=1.0, dev=0.6, period=48.0, dtype=np.float64) -> Frame:
    """Fringe whose local frequency varies sinusoidally in x and y (window-size sweeps).

    truth_wx(ys, xs) = w0 + dev cos(k xs), truth_wy(ys, xs) = w0 + dev cos(k ys), and
    meta["phase"](ys, xs) is the fringe phase itself.
    """
    k = 2.0 * math.pi / period
    A = dev / k
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    phase = w0 * (x + y) + A * np.sin(k * x) + A * np.sin(k * y)
    img = A_DC + B_AC * np.cos(phase)
    img = img + np.random.default_rng(seed).standard_normal((H, W)) * _noise_sigma(snr_db)

    def truth_wx(ys, xs):
        return w0 + dev * np.cos(k * np.asarray(xs, dtype=np.float64)) + 0.0 * np.asarray(ys, dtype=np.float64)

    def truth_wy(ys, xs):
        return w0 + dev * np.cos(k * np.asarray(ys, dtype=np.float64)) + 0.0 * np.asarray(xs, dtype=np.float64)

    def phase_at(ys, xs):
        ys = np.asarray(ys, dtype=np.float64)
        xs = np.asarray(xs, dtype=np.float64)
        return w0 * (xs + ys) + A * np.sin(k * xs) + A * np.sin(k * ys)

    return Frame(img.astype(dtype), L=0, N=0, dirs="xy", truth_wx=truth_wx, truth_wy=truth_wy,
                 meta={"cfg": "sweep", "snr": snr_db, "phase": phase_at})


def complex_tone(W, H, wx, wy, alpha=0.3, amp=1.0, snr_db=None, seed=0):
    """Complex fringe of Eq. 1 with linear phase: A e^{j(alpha + wx x + wy y)} + eta."""
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    g = amp * np.exp(1j * (alpha + wx * x + wy * y))
    if snr_db is not None:
        rng = np.random.default_rng(seed)
        s = amp * math.sqrt(10.0 ** (-snr_db / 10.0) / 2.0)
        g = g + s * (rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W)))
    return g


def training_lines(n: int, seed: int, length: int = 128):
    """Surrogate training lines: 0.5 + 0.4 cos(w n + theta) + noise.

    w ~ U(2 pi/16, 2 pi/4), theta ~ U(0, 2 pi), SNR ~ U(0, 30) dB.
    Returns (lines[n, length] float64, w[n]).
    """
    rng = np.random.default_rng(seed)
    w = rng.uniform(2 * math.pi / 16, 2 * math.pi / 4, n)
    th = rng.uniform(0, 2 * math.pi, n)
    snr = rng.uniform(0.0, 30.0, n)
    m = np.arange(length, dtype=np.float64)[None, :]
    sig = np.sqrt(B_AC * B_AC / 2.0 * 10.0 ** (-snr / 10.0))[:, None]
    lines = A_DC + B_AC * np.cos(w[:, None] * m + th[:, None]) + rng.standard_normal((n, length)) * sig
    return lines, w


def random_frame(W, H, seed, dtype=np.float32, snr_db=10.0, f0=0.12, angle=40.0):
    """Small erf fringe with arbitrary (possibly ragged) size for parity tests."""
    img, twx, twy = erf_fringe(W, H, f0, angle, 4.0, H / 2.0, max(8.0, H / 6.0), snr_db, seed, dtype)
    return img


# ---------------------------------------------------------------------------
# Counter-based generator for the surrogate training lines
# ---------------------------------------------------------------------------
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32(ctr, key, rounds: int = 10):
    """Philox4x32 (Salmon, Moraes, Dror and Shaw, SC'11) on arrays of counters.

    ctr: (..., 4) uint32, key: (..., 2) uint32.  Each round multiplies words 0
    and 2 by the round constants, crosses the high halves with words 1 and 3
    and the key, and the key is bumped by the Weyl constants between rounds.
    """
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64)
    k1 = np.asarray(key[..., 1], dtype=np.uint64)
    mask = np.uint64(0xFFFFFFFF)
    for r in range(rounds):
        if r:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mask
            k1 = (k1 + np.uint64(PHILOX_W1)) & mask
        p0 = np.uint64(PHILOX_M0) * c[0]
        p1 = np.uint64(PHILOX_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def _uniform(u32):
    """(u + 0.5) / 2^32: uniform in (0, 1), never 0 or 1."""
    return (u32.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


TRAIN_LINE_LEN = 128


def philox_training_lines(line_ids, seed: int):
    """Training lines drawn by counter: the GPU generator draws the same numbers.

    Line i uses counter (i, 0, 0, 0) for its parameters
        w = 2 pi/16 + u0 (2 pi/4 - 2 pi/16),  theta = 2 pi u1,  SNR = 30 u2 dB,
    and counters (i, b+1, 0, 0), b < 32, for the noise of samples 4b..4b+3
    (two Box-Muller pairs per call).  Sample n is
        0.5 + 0.4 cos(w n + theta) + sqrt(0.08 10^(-SNR/10)) z_n.
    Returns (lines[M, 128] float64, w[M]).
    """
    ids = np.asarray(line_ids, dtype=np.uint64)
    M = ids.size
    key = np.broadcast_to(np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint32), (M, 2))
    ctr = np.zeros((M, 4), np.uint32)
    ctr[:, 0] = ids.astype(np.uint32)
    p = philox4x32(ctr, key)
    u = _uniform(p)
    w = 2 * math.pi / 16 + u[:, 0] * (2 * math.pi / 4 - 2 * math.pi / 16)
    th = 2 * math.pi * u[:, 1]
    snr = 30.0 * u[:, 2]
    nb = TRAIN_LINE_LEN // 4
    ctr2 = np.zeros((M, nb, 4), np.uint32)
    ctr2[:, :, 0] = ids.astype(np.uint32)[:, None]
    ctr2[:, :, 1] = np.arange(1, nb + 1, dtype=np.uint32)[None, :]
    q = _uniform(philox4x32(ctr2, np.broadcast_to(key[:, None, :], (M, nb, 2))))
    r0 = np.sqrt(-2.0 * np.log(q[..., 0]))
    r1 = np.sqrt(-2.0 * np.log(q[..., 2]))
    z = np.stack([r0 * np.cos(2 * math.pi * q[..., 1]), r0 * np.sin(2 * math.pi * q[..., 1]),
                  r1 * np.cos(2 * math.pi * q[..., 3]), r1 * np.sin(2 * math.pi * q[..., 3])], axis=-1)
    z = z.reshape(M, TRAIN_LINE_LEN)
    n = np.arange(TRAIN_LINE_LEN, dtype=np.float64)[None, :]
    sig = np.sqrt(B_AC * B_AC / 2.0 * 10.0 ** (-snr / 10.0))[:, None]
    lines = A_DC + B_AC * np.cos(w[:, None] * n + th[:, None]) + sig * z
    return lines, w
