#!/usr/bin/env python3
"""Throughput of sliding-window root-MUSIC demodulation on one MI355X.

Workload (default, cfg4): 16 time-lapsed 4096x4096 fringe frames stored FP16,
carrier 1/8 cyc/px at 45 degrees, erf diffusion phase, SNR 10 dB; local
frequency along x and y with windows of N=32 samples and L=8 covariances
(FP32 covariance, eigen-split and rooting, FP64 root polish), then FP64
integration of both maps to phase.  One step = one bosmusic_demodulate call
over all frames plus the integration of every frame, inputs resident in HBM.
The same frames are timed twice: with the plain root-MUSIC path (the line's
`value`) and with the learned surrogate (an MLP trained on the GPU on 10M
method-generated windows first), whose prediction seeds a power iteration for
the signal eigenvector that is accepted once proven converged and within the
MUSIC main lobe of the prediction, the plain eigen-split otherwise (the
`surrogate` object).

Prints one JSON line: Mpixel/s (frames*W*H / step time) of each mode, the
roofline of each mode's dominant kernel (algorithmic flops per launch / its
mean launch duration from HIP events on its stream), the error of each mode
against the FP64 oracle on the decoded FP16 frames (sampled rows and columns),
the error of omega_x, omega_y and phi against the FP64 oracle on the frames
before their FP16 storage rounding, and the oracle's own throughput on the
host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

PEAK_FP32_VECTOR = 157.3e12      # MI355X published FP32 vector peak (packed), FLOP/s
# mean eigenvalue Newton steps of the tridiagonal solver per window (L = 6, 8 at 10 dB, counted
# before the power route took most windows): the flop model's figure for the windows that fall
# back to it when the two routes are mixed in one counter
NEWTON_STEPS_TRIDIAG = 2.11
PEAK_HBM = 8.0e12
# HBM bytes per pixel and direction of the line-window root-MUSIC launch (L=8, N=32, FP16 4096x4096
# frames): FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 from rocprofv3 --pmc on two cfg4 frames
# (profiles/rootmusic_surrogate_cfg4_counters.md).  Valid only for that kernel and configuration;
# the other configurations report null.
TRAFFIC_BYTES_PER_PIXEL_DIR_CFG4 = (287208.0 * 2.0 + 262144.0) * 1024 / (2 * 2 * 4096 * 4096)
# The same for the surrogate kernel on those frames (same profile).
TRAFFIC_BYTES_PER_PIXEL_DIR_CFG4_SURROGATE = (287417.0 * 2.0 + 262144.0) * 1024 / (2 * 2 * 4096 * 4096)


def bairstow_flops(n: int) -> int:
    """One complex Newton step on a quadratic factor of a degree-n polynomial:
    two synthetic divisions (16 flops per coefficient each) and the 2x2 solve."""
    return 32 * (n + 1) + 60


def cpow_flops(k: int) -> int:
    """z^k by squaring (complex square 5 flops, complex product 6)."""
    if k <= 1:
        return 0
    return cpow_flops(k // 2) + 5 + (6 if k % 2 else 0)


def pair_newton_flops(L: int) -> int:
    """One Newton step for the signal root with its mate divided out, P = L z^(L-1) - B(z)^2
    evaluated from the signal vector: Horner for B and B' over its L coefficients (16 flops per
    step), z^(L-2) and z^(L-1), P and P' (16), and the corrected step (two reciprocals, ~62)."""
    return 16 * (L - 1) + cpow_flops(L - 2) + 6 + 16 + 62


def certificate_flops(L: int) -> tuple:
    """(FP64, FP32) flops of the certificate: the inner member and mate of the root (FP64) and
    the division by the pair's factor with the remainder test (FP32 for L <= 8, FP64 above), then
    the root count of the
    degree m = 2L-4 quotient at the fixed radius 0.8 (FP32): the closed-form first Schur-Cohn
    step (constant factors, two products per coefficient), the next step with a complex
    constant term (28 flops per coefficient pair), and the steps after it with the real one
    (20 per pair, 10 for a middle coefficient), 14 flops of pivots each.  The FP64 recount of
    the undecided windows is not counted."""
    n = 2 * L - 2
    m = n - 2
    division = 36 + 18 * (n + 1)
    if m <= 0:
        return division, 0
    if L <= 8:          # the division in FP32 too; the inner member and its mate stay FP64
        division32 = 18 * (n + 1)
        division, count0 = 36, division32
    else:
        count0 = 0
    d0 = m - 1
    schur = 28 * ((d0 + 1) // 2) + 16 if d0 >= 1 else 0
    schur += sum(20 * ((d - 1) // 2) + (10 if d % 2 == 0 else 0) + 14 for d in range(1, d0))
    return division, count0 + 2 * m + schur


def power_route_flops(L: int, steps: float) -> float:
    """The verified power iteration for the signal eigenvector: the start's half-angle
    (from the lag-1 sums, or the prediction's sincos), the real steering vector, tr T^2,
    `steps` products T v, the Rayleigh quotient / residual / bound test from the second
    step on, and the final normalisation."""
    half = 2 * (L - 1) + 12
    steer = 6 * (L - 1) + 6 * (L // 2) + 6
    trace2 = L + 3 * (L * (L - 1) // 2)
    return half + steer + trace2 + steps * 2 * L * L + max(0.0, steps - 1) * (8 * L + 20) + 3 * L + 2


def flops_per_window(L: int, N: int, newton: float, iters: float, pair_iters: float = 0.0,
                     cert_frac: float = 0.0, block: bool = False, pair_iters32: float = 0.0,
                     power_frac: float = 0.0, power_steps: float = 0.0, quad_lags: bool = True) -> dict:
    """Algorithmic flop count of one window of the root-MUSIC kernel.

    FMA = 2 flops; add, sub, mul, rcp, sqrt, rsq = 1 each.  `newton` is the
    measured mean number of Newton steps for the largest eigenvalue per
    window, `pair_iters32` and `pair_iters` the mean FP32 and FP64 Newton
    steps for the signal root before the certificate, `cert_frac` the fraction of windows
    finished by the certificate, and `iters` the mean simultaneous root
    iterations of the windows whose roots were all found.  Certificate work
    of a window that fails it is not counted.  `block`: the L x L block
    window, whose covariance is summed directly from its L snapshots.  `quad_lags`: the line
    kernel's lane-pair lag sums of four starts for L >= 7 (the surrogate kernel keeps two starts
    per lane).
    The eigenvalue Newton steps cost 8L flops each (the characteristic
    polynomial and its derivative), after a 7L + 2 flop start bound.  `power_frac` of
    the windows take the verified power iteration (`power_steps` steps each) instead of
    that solver.
    """
    K = N - L + 1
    n = 2 * L - 2
    if block:
        # block window: T summed straight from the L snapshots, a_k + j b_k = sqrt2 Q^H s_k
        # (2 L adds) and the upper triangle of a a^T + b b^T (two FMAs per entry)
        lag = L * (2 * L + 4 * (L * (L + 1) // 2))
    elif L >= 7 and quad_lags:
        # lag sums (complex MAC = 4 FMA; the zero lag is real, 2 FMA): a lane pair sums the
        # first of four starts directly (K L MACs) and slides to the next three (2 L MACs each)
        lag = (K * (8 * L - 4) + 3 * (16 * L - 8)) / 4
    else:
        # a lane sums its first start directly (K L MACs) and slides to its second (2 L MACs)
        lag = (K * (8 * L - 4) + 16 * L - 8) / 2
    # T from R (line windows) and the trace normalisation
    build_t = (0 if block else 3 * L * L) + L + L * (L + 1) // 2
    house = sum(2 * l * l + 2 * l * (l + 1) + 9 * l for l in range(2, L))
    newton_f = newton * 8 * L + 7 * L + 2
    inverse = 6 * L + 2 * 8 * L + sum(4 * l for l in range(2, L))
    eigen = (1.0 - power_frac) * (house + newton_f + inverse) + power_frac * power_route_flops(L, power_steps)
    coef = 2 * L + 8 * L * (L + 1) // 2
    # start of the signal-root Newton: two evaluations of the real spectral function g, g', g''
    # (half-angle powers and the L/2 terms), the peak step, the half-angle and the radius
    spectral_start = 2 * (6 * (L - 1) + 9 * L + 5) + 25
    common32 = lag + build_t + eigen + coef + 20 + spectral_start
    full = 1.0 - cert_frac
    start = 4 * n + 40
    aberth = iters * (n * (30 + 16 * n) + 12 * n * (n - 1) // 2 + 27 * n)
    select = 11 * n
    cert64, cert32 = certificate_flops(L)
    # the FP64 Newton stage: P and P' in FP64, the corrected step from them in FP32 (~62 flops)
    fp32 = (common32 + full * (start + aberth + select) + pair_iters32 * pair_newton_flops(L) + cert_frac * cert32
            + pair_iters * 62)
    fp64 = pair_iters * (pair_newton_flops(L) - 62) + cert_frac * cert64 + full * 3 * bairstow_flops(n)
    return {"fp32": fp32, "fp64": fp64, "total": fp32 + fp64}


def surrogate_flops_per_window(L: int, N: int) -> dict:
    """The surrogate kernel's own work per window beyond the plain path's: the features
    and the MLP of one window in 32 (matrix-core flops kept apart, GELU as its A&S
    erf: 16 flops) and the null spectrum at the prediction (its power route is counted
    with the plain path's).  Transcendentals count as one flop."""
    stride = 32                                       # one network prediction per 32 windows
    feat = (4 * N + 16 * 6 + 10) / stride
    mlp_mfma = 2 * (32 * 64 + 64 * 64 + 64 * 2) / stride
    mlp_valu = (2 * 64 * (16 + 1) + 2) / stride
    null = 2 * L + 2
    return {"predict": feat + mlp_valu + null, "mfma": mlp_mfma}


TRAIN_MFMA_FLOPS = 2 * (32 * 64 + 64 * 64 + 64 * 2) * 2 + 2 * 64 * 64   # forward, weight gradients, dH1


def train_surrogate(bm, torch, args):
    """Training set on the GPU, then minibatch Adam; returns (params, report)."""
    tr = bm.Demodulator(0, max_width=64, max_height=64)
    bm.bosmusic_surrogate_load(tr.h, bm.init_params(0))
    M = args.train_windows
    X = torch.empty((M, 32), device="cuda")
    T = torch.empty((M, 2), device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bm.bosmusic_surrogate_dataset(tr.h, 0, X, T, None, seed=2024)
    t_ds = time.perf_counter() - t0
    Mh = 65536
    Xh = torch.empty((Mh, 32), device="cuda")
    Th = torch.empty((Mh, 2), device="cuda")
    wh = torch.empty(Mh, device="cuda")
    bm.bosmusic_surrogate_dataset(tr.h, 1 << 31, Xh, Th, wh, seed=2024)
    print(f"# training set: {M} windows in {t_ds:.2f}s", file=sys.stderr, flush=True)
    s1 = (2 * args.train_steps) // 3
    t0 = time.perf_counter()
    l1 = bm.bosmusic_surrogate_train(tr.h, X, T, args.train_batch, s1, 2e-3)
    l2 = bm.bosmusic_surrogate_train(tr.h, X, T, args.train_batch, args.train_steps - s1, 2e-4)
    t_tr = time.perf_counter() - t0
    Y = torch.empty((Mh, 2), device="cuda")
    bm.bosmusic_surrogate_forward(tr.h, Xh, Y)
    torch.cuda.synchronize()
    y = Y.cpu().numpy().astype(np.float64)
    e = (np.arctan2(y[:, 1], y[:, 0]) - wh.cpu().numpy() + np.pi) % (2 * np.pi) - np.pi
    params = bm.bosmusic_surrogate_save(tr.h)
    tr.close()
    losses = np.concatenate([l1, l2])
    ws = args.train_steps * args.train_batch
    rep = {"windows": M, "steps": args.train_steps, "batch": args.train_batch, "lr": "2e-3 then 2e-4 (last third)",
           "dataset_s": round(t_ds, 3), "train_s": round(t_tr, 3), "window_steps_per_s": ws / t_tr,
           "mfma_tflops": ws * TRAIN_MFMA_FLOPS / t_tr / 1e12, "loss_first": float(losses[0]),
           "loss_last": float(losses[-20:].mean()), "held_out_rms_rad": float(np.sqrt(np.mean(e * e))),
           "held_out_windows": Mh}
    print(f"# trained {args.train_steps} steps x {args.train_batch} in {t_tr:.2f}s, loss {losses[0]:.4f} -> "
          f"{losses[-20:].mean():.5f}, held-out rms {rep['held_out_rms_rad']:.4f} rad", file=sys.stderr, flush=True)
    return params, rep


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample, on the host cores
# ---------------------------------------------------------------------------
_SAMPLE_FRAMES = {}


def _oracle_job(job):
    import oracle
    key, kind, idx, L, N = job
    f = _SAMPLE_FRAMES[key]
    if kind == "x":
        g = oracle.to_complex_field(f[idx:idx + 1], 1)
    else:
        g = oracle.to_complex_field(f[:, idx:idx + 1].T, 1)
    om = oracle.demod_lines(g, L, N)[0]
    return job, om


def sample_lines(H, W, N, lines_per_dir):
    """Rows and columns of the oracle sample: lines_per_dir evenly spaced ones (offset 37)
    plus the integration's anchor column N // 2."""
    rows = sorted({(37 + i * H // lines_per_dir) % H for i in range(lines_per_dir)})
    cols = sorted({(37 + i * W // lines_per_dir) % W for i in range(lines_per_dir)} | {N // 2})
    return rows, cols


def run_oracle(frames, meta, keys, lines, workers, timed=True):
    """The oracle on the given rows and columns of frames[key] with a process pool.

    Runs before the GPU is touched; the pool forks with the frames already in memory,
    so the timed region holds oracle work only.  Returns ({(key, kind, idx): omega},
    windows, seconds)."""
    import multiprocessing as mp
    _SAMPLE_FRAMES.clear()
    _SAMPLE_FRAMES.update({k: frames[k] for k in keys})
    jobs = []
    for k in keys:
        rows, cols = lines[k]
        jobs += [(k, "x", r, meta[k].L, meta[k].N) for r in rows]
        jobs += [(k, "y", c, meta[k].L, meta[k].N) for c in cols]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        if timed:
            pool.map(_oracle_job, jobs[:workers], chunksize=1)        # import warm-up, untimed
        t0 = time.perf_counter()
        res = pool.map(_oracle_job, jobs, chunksize=1)
        dt = time.perf_counter() - t0
    windows = sum(int(np.isfinite(om).sum()) for _, om in res)
    return {(j[0], j[1], j[2]): om for j, om in res}, windows, dt


def oracle_phi_rows(om, key, H, W, N, rows):
    """The oracle's phase on the sampled rows: its own trapezoid rule on its own omega
    (those rows and the anchor column)."""
    import oracle
    owx = np.full((H, W), np.nan)
    owy = np.full((H, W), np.nan)
    for (k, kind, idx), o in om.items():
        if k != key:
            continue
        if kind == "x":
            owx[idx] = o
        else:
            owy[:, idx] = o
    ref = oracle.integrate(owx, owy, N, N)
    return {r: ref[r] for r in rows}


def wrap(d):
    return (np.asarray(d) + np.pi) % (2 * np.pi) - np.pi


def omega_diffs(om, wx, wy, keys=None):
    """|d omega| of the GPU maps against oracle lines, per direction; NaN patterns must agree."""
    out = {"x": [], "y": []}
    for (k, kind, idx), o in om.items():
        if keys is not None and k not in keys:
            continue
        got = (wx[k][idx] if kind == "x" else wy[k][:, idx]).cpu().numpy().astype(np.float64)
        m = np.isfinite(o)
        assert np.array_equal(m, np.isfinite(got)), (k, kind, idx)
        out[kind].append(np.abs(wrap(got[m] - o[m])))
    return {d: np.concatenate(v) if v else np.zeros(0) for d, v in out.items()}


def stats_of(d, tol):
    return {"p50": float(np.quantile(d, 0.5)), "p99": float(np.quantile(d, 0.99)),
            "p999": float(np.quantile(d, 0.999)), "max": float(d.max()), "rms": float(np.sqrt(np.mean(d * d))),
            "windows": int(d.size), "tolerance": tol}


def workload(name, nframes):
    """Frames (numpy), per-frame (L, N, dirs) and a description of the workload."""
    if name == "cfg2":
        fr = [wl.cfg2_frame(t) for t in range(nframes or 100)]
        desc = (f"{len(fr)} time-lapsed 1024x1024 FP32 fringe frames, carrier 0.1 cyc/px at 30 deg, 6*erf "
                f"diffusion phase, SNR 10 dB; x and y windows N=32, L=6; plain root-MUSIC + FP64 phase integration")
    elif name == "cfg3":
        fr = [wl.cfg3_frame(k) for k in range(nframes or 64)]
        desc = (f"{len(fr)} uneven FP32 frames 512x512..2048x1536 ({sum(f.width * f.height for f in fr)} px), "
                f"L in {{4,6,8}}, N=2L+8, SNR 5-20 dB; one cached hipGraph replay per step, autotuned tiles; "
                f"plain root-MUSIC + FP64 phase integration")
    elif name in ("cfg4", "cfg5"):
        fr = [wl.cfg4_frame(t) for t in range(nframes or 16)]
        desc = (f"{len(fr)} time-lapsed 4096x4096 fringe frames stored FP16, carrier 1/8 cyc/px at 45 deg, 6*erf "
                f"diffusion phase, SNR 10 dB; x and y windows N=32, L=8; FP32 covariance/eigen/rooting, FP64 "
                f"root polish and phase prefix sums. Plain root-MUSIC (value) vs surrogate MLP 32-64-64-2 "
                f"(GELU, BF16 MFMA, FP32 accumulate) trained on the GPU on 10M method-generated windows "
                f"(carrier 1/16-1/4 cyc/px, SNR 0-30 dB, root-MUSIC L=8 N=32 labels) seeding a verified power "
                f"iteration for the signal eigenvector, plain eigen-split where it does not serve (surrogate)")
    elif name == "exp":
        fr = [wl.exp_frame(i) for i in range(nframes or 19)]
        desc = (f"{len(fr)} time-lapsed 1850x700 8-bit frames (stand-in for the paper's experimental diffusion "
                f"series), carrier 0.11 cyc/px at 35 deg, 5*erf phase, SNR 12 dB; x and y windows N=15, L=7; "
                f"analytic step through Bluestein's identity (neither length is 5-smooth); "
                f"plain root-MUSIC + FP64 phase integration")
    else:
        raise SystemExit(f"unknown workload {name}")
    return fr, desc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg4", choices=["cfg2", "cfg3", "cfg4", "cfg5", "exp"],
                    help="cfg4 (= cfg5): 16 FP16 4096x4096 frames, plain and surrogate")
    ap.add_argument("--modes", default="",
                    help="comma list of plain,surrogate (default: both on cfg4/cfg5, plain elsewhere)")
    ap.add_argument("--train-windows", type=int, default=10_000_000, help="surrogate: training set size")
    ap.add_argument("--train-steps", type=int, default=3000, help="surrogate: Adam steps")
    ap.add_argument("--train-batch", type=int, default=16384, help="surrogate: minibatch")
    ap.add_argument("--predictor", default="mlp", choices=["mlp", "lag1"],
                    help="surrogate: the trained MLP, or the non-learned lag-1 phase predictor")
    ap.add_argument("--frames", type=int, default=0, help="number of frames (0: the workload's own)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs")
    ap.add_argument("--cpu-lines", type=int, default=0,
                    help="oracle sample: lines per direction per sampled frame (0: the workload's default)")
    ap.add_argument("--block", type=int, default=0,
                    help="use the paper's M x M block window with this M (L = N = M) instead of line windows")
    ap.add_argument("--full-roots", action="store_true",
                    help="find every root of every window (no certified-pair shortcut)")
    ap.add_argument("--warm", action="store_true",
                    help="temporal warm start: frame t starts its Newton iterations at frame t-1's maps "
                         "(computed before the timed steps, as a streaming pipeline would have them)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (frames are independent; "
              "see the sharding notes in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    big = args.workload in ("cfg4", "cfg5")
    modes = [m for m in (args.modes or ("plain,surrogate" if big else "plain")).split(",") if m]
    if any(m not in ("plain", "surrogate") for m in modes) or not modes:
        raise SystemExit(f"--modes: {args.modes}")
    if args.block:
        args.no_cpu = True          # the oracle sample below is of line windows
        modes = ["plain"]

    t_gen = time.perf_counter()
    fr, desc = workload(args.workload, args.frames)
    frames = [f.data for f in fr]
    nf = len(fr)
    total_px = sum(f.width * f.height for f in fr)
    t_gen = time.perf_counter() - t_gen
    print(f"# generated {nf} frames ({total_px} px) in {t_gen:.1f}s", file=sys.stderr, flush=True)

    # ---- oracle legs (before the GPU is touched) ----------------------------
    cpu = None
    om = {}
    phi_ref = {}
    src = None
    workers = max(1, min(16, os.cpu_count() or 1))
    if not args.no_cpu:
        sf = sorted({0, nf - 1}) if big else sorted({0, nf // 3, (2 * nf) // 3, nf - 1})
        if args.cpu_lines <= 0:
            if big:
                args.cpu_lines = fr[0].height // 16           # every 16th row and column
            else:
                mean_len = np.mean([fr[t].width + fr[t].height for t in sf]) / 2
                args.cpu_lines = max(8, int(4e6 / (2 * len(sf) * mean_len)))
        lines = {t: sample_lines(fr[t].height, fr[t].width, fr[t].N, args.cpu_lines) for t in sf}
        om, windows, osec = run_oracle(frames, fr, sf, lines, workers)
        px_s = windows / osec / 2.0            # two directions per pixel
        cpu = {"value": px_s / 1e6, "unit": "Mpixel/s", "cores": workers, "kind": "oracle",
               "sample": f"{args.workload} frames {sf}, {args.cpu_lines} rows + {args.cpu_lines} columns each "
                         f"({windows} windows, {osec:.1f}s wall on {workers} processes); "
                         f"Mpixel/s = windows/s / 2 directions"}
        print(f"# oracle: {windows} windows in {osec:.2f}s on {workers} procs", file=sys.stderr, flush=True)
        for t in sf:
            phi_ref.update({(t, r): v for r, v in oracle_phi_rows(om, t, fr[t].height, fr[t].width, fr[t].N,
                                                                  lines[t][0]).items()})
        if big:
            # the same frames before their FP16 storage rounding, on every other sampled line
            srcf = {("src", t): wl.cfg4_frame(t, fr[t].width, np.float64).data for t in sf}
            smeta = {("src", t): fr[t] for t in sf}
            slines = {("src", t): (lines[t][0][::2], sorted(set(lines[t][1][::2]) | {fr[t].N // 2})) for t in sf}
            som, swin, ssec = run_oracle(srcf, smeta, list(srcf), slines, workers, timed=False)
            print(f"# FP64-source oracle: {swin} windows in {ssec:.2f}s", file=sys.stderr, flush=True)
            sphi = {}
            for t in sf:
                k = ("src", t)
                sphi.update({(t, r): v for r, v in oracle_phi_rows(som, k, fr[t].height, fr[t].width, fr[t].N,
                                                                   slines[k][0]).items()})
            src = {"om": {(k[1], kind, idx): v for (k, kind, idx), v in som.items()}, "phi": sphi,
                   "lines": {t: slines[("src", t)] for t in sf}}
            del srcf

    import torch
    import paper_1910_11872_amd as bm

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    maxw = max(f.width for f in fr)
    maxh = max(f.height for f in fr)
    d_frames = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in frames]
    wx = [torch.empty(f.shape, dtype=torch.float32, device=dev) for f in frames]
    wy = [torch.empty(f.shape, dtype=torch.float32, device=dev) for f in frames]
    phi = [torch.empty(f.shape, dtype=torch.float64, device=dev) for f in frames]
    if args.block:
        for f in fr:
            f.L = f.N = args.block
        desc += f"; the paper's {args.block}x{args.block} block window instead of line windows"
    bdir = bm.BM_BLOCK if args.block else 0
    specs = [bm.FrameSpec(d_frames[i], fr[i].L, fr[i].N, bm.BM_DIR_X | bm.BM_DIR_Y | bdir, wx[i], wy[i])
             for i in range(nf)]
    if args.warm:
        # the previous frame's maps, as a pipeline that demodulates frames in order holds them
        pdem = bm.Demodulator(0, max_width=maxw, max_height=maxh, max_batch_pixels=total_px)
        bm.bosmusic_demodulate(pdem.h, specs, bm.BM_PLAIN, torch.cuda.current_stream())
        torch.cuda.synchronize()
        pdem.close()
        for i in range(1, nf):
            if wx[i - 1].shape != wx[i].shape:
                continue
            specs[i].prev_omega_x = wx[i - 1].clone()
            specs[i].prev_omega_y = wy[i - 1].clone()
        desc += "; temporal warm start from the previous frame's maps"
    use_graph = args.workload == "cfg3"
    if use_graph:
        tdem = bm.Demodulator(0, max_width=maxw, max_height=maxh)
        for (L, N) in sorted({(f.L, f.N) for f in fr}):
            tdem.autotune(L, N, width=1024, lines=512)
        tdem.close()
    stream = torch.cuda.current_stream()
    params = train_rep = None
    if "surrogate" in modes and args.predictor == "mlp":
        params, train_rep = train_surrogate(bm, torch, args)

    if args.copy_mib > 0:
        nel = args.copy_mib * (1 << 20) // 4
        src_t = torch.ones(nel, dtype=torch.float32, device=dev)
        dst_t = torch.empty_like(src_t)
        torch.cuda.synchronize()
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t

    def make(mode, **kw):
        dm = bm.Demodulator(0, max_width=maxw, max_height=maxh, max_batch_pixels=total_px,
                            full_roots=args.full_roots, **kw)
        if mode == bm.BM_SURROGATE:
            if params is not None:
                bm.bosmusic_surrogate_load(dm.h, params)
            bm.bosmusic_surrogate_config(dm.h, 0.25, 1 if args.predictor == "lag1" else 0)
        return dm

    maps = [(wx[i], wy[i], fr[i].N, fr[i].N, 0.0, 0.0, phi[i]) for i in range(nf)]

    def step(dm, mode):
        bm.bosmusic_demodulate(dm.h, specs, mode, stream)
        bm.bosmusic_integrate_many(dm.h, maps, stream)

    def timed(dm, mode):
        for _ in range(args.warmup):
            step(dm, mode)
        torch.cuda.synchronize()
        dm.stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(dm, mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) * 1e3 / args.steps, dm.stats(reset=True)

    def roofline(mode, st):
        """Iteration counts per L from the counting variant of the kernels (outside the
        timed region), the flop model, and the timed launches' mean duration."""
        surrogate = mode == bm.BM_SURROGATE
        flops_step = 0.0
        mfma_step = 0.0
        per_L = {}
        for L in sorted({f.L for f in fr}):
            idx = [i for i in range(nf) if fr[i].L == L]
            sdem = make(mode, stats=True)
            sub = [specs[i] for i in idx[:3]]
            bm.bosmusic_demodulate(sdem.h, sub, mode, stream)
            ss = sdem.stats(reset=True)
            sdem.close()
            nwin = max(1, ss["windows"])
            # eig_iters holds the power steps of the power-route windows and the eigenvalue
            # Newton steps of the rest; the latter are taken at the tridiagonal solver's
            # measured mean when both routes are mixed
            pw = ss.get("power_windows", 0)
            if pw:
                newton = NEWTON_STEPS_TRIDIAG
                psteps = max(0.0, ss["eig_iters"] - (nwin - pw) * newton) / pw
            else:
                newton, psteps = ss["eig_iters"] / nwin, 0.0
            power_frac = pw / nwin
            pair_its32 = ss.get("pair_iters32", 0) / nwin
            if surrogate:
                # the certified fraction and the Aberth iterations come from a plain counting
                # pass (the surrogate's accepted/rejected counters are its own)
                pdem = make(bm.BM_PLAIN, stats=True)
                bm.bosmusic_demodulate(pdem.h, sub, bm.BM_PLAIN, stream)
                ps = pdem.stats(reset=True)
                pdem.close()
                pn = max(1, ps["windows"])
                iters = ps["root_iters"] / max(1, ps["sur_rejected"])
                pair_its, cert = ss["pair_iters"] / nwin, ps["sur_accepted"] / pn
            elif args.full_roots:
                iters = ss["root_iters"] / nwin
                pair_its, cert = 0.0, 0.0
            else:
                iters = ss["root_iters"] / max(1, ss["sur_rejected"])
                pair_its = ss["pair_iters"] / nwin
                cert = ss["sur_accepted"] / nwin
            wins = 0
            for i in idx:
                W, H, N = fr[i].width, fr[i].height, fr[i].N
                if args.block:
                    wins += 2 * max(0, W - N + 1) * max(0, H - N + 1)
                else:
                    wins += H * max(0, W - N + 1) + W * max(0, H - N + 1)
            fl = flops_per_window(L, fr[idx[0]].N, newton, iters, pair_its, cert, block=bool(args.block),
                                  pair_iters32=pair_its32, power_frac=power_frac, power_steps=psteps,
                                  quad_lags=not surrogate)
            per_win = fl["total"]
            entry = {"newton": round(newton, 2), "power_fraction": round(power_frac, 5),
                     "power_steps": round(psteps, 2), "root_iters": round(iters, 2), "windows_per_step": wins,
                     "pair_iters32": round(pair_its32, 2), "pair_iters": round(pair_its, 2),
                     "certified_fraction": round(cert, 5)}
            if surrogate:
                acc, rej = ss["sur_accepted"], ss["sur_rejected"]
                sfl = surrogate_flops_per_window(L, fr[idx[0]].N)
                per_win += sfl["predict"]
                mfma_step += wins * sfl["mfma"]
                entry.update({"surrogate_mfma_flop_per_window": sfl["mfma"],
                              "accepted_fraction": round(acc / max(1, acc + rej), 5)})
            entry["flop_per_window"] = round(per_win)
            flops_step += per_win * wins
            per_L[L] = entry
        rm_s = st["rm_time_ns"] / 1e9 / args.steps      # root-MUSIC (or surrogate) launch time per step
        achieved = flops_step / rm_s
        kname = "surrogate_kernel" if surrogate else "rootmusic_kernel"
        traffic = None
        if big and not (args.block or args.full_roots or args.warm or args.predictor != "mlp"):
            per_px = TRAFFIC_BYTES_PER_PIXEL_DIR_CFG4_SURROGATE if surrogate else TRAFFIC_BYTES_PER_PIXEL_DIR_CFG4
            traffic = per_px * 2 * total_px / max(1, st["rm_launches"] // args.steps)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE, scaled per pixel)",
                "kernel": f"{kname}, {st['rm_launches'] // args.steps} timed region(s)/step, mean "
                          f"{st['rm_time_ns'] / max(1, st['rm_launches']) / 1e6:.3f} ms (HIP events on its "
                          f"stream), per L: {json.dumps(per_L)}"}
        if surrogate:
            roof["mfma_tflops_in_mlp"] = mfma_step / rm_s / 1e12
        return roof, per_L

    results = {}
    for mname in modes:
        mode = bm.BM_SURROGATE if mname == "surrogate" else bm.BM_PLAIN
        # the production path (graph replay for the uneven batch; otherwise a batch's
        # two halves pipelined on two streams), then the same steps with HIP events
        # around every root-MUSIC launch, each launch alone on the chip, for the roofline
        pdem = make(mode, graph=True) if use_graph else make(mode)
        ms, _ = timed(pdem, mode)
        pdem.close()
        dem = make(mode, timing=True)
        ms_ev, st = timed(dem, mode)
        dem.close()
        mpx = total_px / (ms / 1e3) / 1e6
        print(f"# {mname}: {args.steps} steps, {ms:.2f} ms/step, {mpx:.1f} Mpixel/s (event-timed pass "
              f"{ms_ev:.2f} ms/step)", file=sys.stderr, flush=True)
        roof, per_L = roofline(mode, st)
        err = None
        if om:
            # the maps of the last timed step of this mode
            dd = omega_diffs(om, wx, wy)
            d = np.concatenate([dd["x"], dd["y"]])
            err = stats_of(d, "RMS <= 2e-3" if mname == "surrogate" else "p99.9 <= 1e-4")
            err = {("vs_oracle_" + k if k not in ("windows", "tolerance") else k): v for k, v in err.items()}
            err["unit"] = "rad/px"
            dphi = []
            for (t, r), refr in phi_ref.items():
                got = phi[t][r].cpu().numpy()
                m = np.isfinite(refr)
                assert np.array_equal(m, np.isfinite(got))
                dphi.append(np.abs(got[m] - refr[m]))
            dp = np.concatenate(dphi)
            err["phi_vs_oracle_max"] = float(dp.max())
            err["phi_vs_oracle_rms"] = float(np.sqrt(np.mean(dp * dp)))
            err["phi_unit"] = "rad (FP64 trapezoid of each side's own omega, sampled rows)"
        srcerr = None
        if src is not None and mname == "plain":
            # per output against the FP64 oracle on the frames before FP16 rounding; and the
            # oracle on the decoded FP16 frames against the same, on the same lines (the share
            # of the storage rounding)
            dd = omega_diffs(src["om"], wx, wy)
            dq = {"x": [], "y": []}
            for (t, kind, idx), o in src["om"].items():
                q = om[(t, kind, idx)]
                m = np.isfinite(o)
                dq[kind].append(np.abs(wrap(q[m] - o[m])))
            srcerr = {}
            for kname, d in (("omega_x", dd["x"]), ("omega_y", dd["y"])):
                q = np.concatenate(dq[kname[-1]])
                srcerr[kname] = {"gpu_vs_fp64_source": stats_of(d, None),
                                 "fp16_oracle_vs_fp64_source": stats_of(q, None)}
                for v in srcerr[kname].values():
                    v.pop("tolerance")
            dphi, qphi = [], []
            for (t, r), refr in src["phi"].items():
                got = phi[t][r].cpu().numpy()
                m = np.isfinite(refr)
                dphi.append(np.abs(got[m] - refr[m]))
                qphi.append(np.abs(phi_ref[(t, r)][m] - refr[m]))
            dp, qp = np.concatenate(dphi), np.concatenate(qphi)
            srcerr["phi"] = {"gpu_vs_fp64_source": {"max": float(dp.max()), "rms": float(np.sqrt(np.mean(dp * dp)))},
                             "fp16_oracle_vs_fp64_source": {"max": float(qp.max()),
                                                            "rms": float(np.sqrt(np.mean(qp * qp)))}}
            srcerr["unit"] = "rad/px (omega), rad (phi)"
            srcerr["sample"] = (f"frames {sorted(src['lines'])}, every {2 * (fr[0].height // args.cpu_lines)}th row "
                                f"and column (+ the anchor column), FP64 frames regenerated from the same seeds")
        acc = None
        if mode == bm.BM_SURROGATE:
            acc = {L: e.get("accepted_fraction") for L, e in per_L.items()}
        results[mname] = {"ms": ms, "mpx": mpx, "roofline": roof, "error": err, "source_error": srcerr,
                          "accepted": acc}

    first = results[modes[0]]
    out = {
        "metric": "Mpixel/s local-frequency demod (plain vs surrogate) at stated rad/px error",
        "value": first["mpx"],
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": first["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "frames": nf, "pixels": total_px,
                   "dirs": "xy", "mode": modes[0], "modes": modes, "graph": use_graph, "warm_start": args.warm,
                   "roots": "all" if args.full_roots else "certified pair, all roots where uncertified",
                   **({"predictor": args.predictor} if "surrogate" in modes else {})},
        "roofline": first["roofline"],
        "cpu_baseline": cpu,
        "error": first["error"],
    }
    if first["source_error"] is not None:
        out["source_error"] = first["source_error"]
    if "surrogate" in modes and modes[0] != "surrogate":
        s = results["surrogate"]
        out["surrogate"] = {"value": s["mpx"], "unit": "Mpixel/s", "ms_per_step": s["ms"],
                            "vs_plain": s["mpx"] / first["mpx"], "roofline": s["roofline"], "error": s["error"],
                            "accepted_fraction": s["accepted"], "training": train_rep,
                            "note": "same frames, same steps/warmup; value/ms_per_step of the line are the plain path"}
    elif "surrogate" in modes:
        out["training"] = train_rep
    print(json.dumps(out))


if __name__ == "__main__":
    main()
