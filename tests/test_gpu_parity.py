"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Sizes are chosen so the oracle finishes in seconds while the GPU launches span
several 256-wide window tiles and a ragged tail; full-size workloads are
compared on sampled lines.  Bar: |d omega| <= 1e-4 rad/px at the 99.9th
percentile, identical NaN patterns; phi to 1e-9 rad when integrating the same
omega maps.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare_omega, oracle_cols, oracle_rows, wrap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def dem(bm, torch):
    d = bm.Demodulator(0, max_width=4096, max_height=4096, stats=True)
    yield d
    d.close()


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run(dem, torch, img, L, N, dirs):
    wx, wy = dem.demodulate(to_dev(torch, img), L, N, dirs)
    torch.cuda.synchronize()
    return (wx.cpu().numpy() if wx is not None else None, wy.cpu().numpy() if wy is not None else None)


# ---------------------------------------------------------------------------
# cfg1 in full (256x256 FP64, x, L=4, N=16)
# ---------------------------------------------------------------------------
def test_cfg1_full(dem, torch):
    f = wl.cfg1()
    gx, _ = run(dem, torch, f.data, f.L, f.N, "x")
    ox, _ = oracle.demodulate(f.data, f.L, f.N, "x")
    s = compare_omega(gx, ox, "cfg1")
    print("cfg1", s)
    # accuracy against the truth is the oracle's, not worse
    v = np.isfinite(gx)
    assert math.sqrt(np.mean((gx[v] - math.pi / 4) ** 2)) < 1.1 * math.sqrt(np.mean((ox[v] - math.pi / 4) ** 2))


# ---------------------------------------------------------------------------
# Ragged sizes, every L, every real dtype, both directions
# ---------------------------------------------------------------------------
CASES = [
    # (W, H, L, N, dtype)
    (600, 40, 2, 6, np.float32),
    (300, 36, 3, 11, np.float64),
    (640, 30, 4, 16, np.float16),
    (270, 48, 5, 14, np.float32),
    (576, 40, 6, 32, np.float32),
    (250, 45, 7, 20, np.float64),
    (512, 32, 8, 32, np.float16),
    (360, 60, 8, 64, np.float32),
    (384, 50, 7, 15, np.uint8),
    (1100, 20, 7, 24, np.float32),   # lane-pair lag sums over three blocks and a ragged tail
    (700, 22, 7, 9, np.float32),     # K = 3 snapshots: fewer than one unrolled step of the sums
    (1030, 18, 8, 10, np.float16),
]


@pytest.mark.parametrize("W,H,L,N,dt", CASES)
def test_ragged_frames_both_directions(dem, torch, W, H, L, N, dt):
    img = wl.random_frame(W, H, seed=W + 7 * H + L, dtype=dt, snr_db=8.0)
    gx, gy = run(dem, torch, img, L, N, "xy")
    ox, oy = oracle.demodulate(img, L, N, "xy")
    print("x", compare_omega(gx, ox, f"x {W}x{H} L{L} N{N} {dt.__name__}"))
    print("y", compare_omega(gy, oy, f"y {W}x{H} L{L} N{N} {dt.__name__}"))


def test_complex_input_tones_exact(dem, torch):
    """C32 input (Gamma of Eq. 1 given directly): a linear-phase tone is exact to FP32."""
    W, H = 300, 70
    for (wx0, wy0) in [(0.7, -0.4), (-2.5, 1.9), (0.05, 3.0)]:
        g = wl.complex_tone(W, H, wx0, wy0).astype(np.complex64)
        gx, gy = run(dem, torch, g, 6, 20, "xy")
        assert np.nanmax(np.abs(wrap(gx - wx0))) < 2e-5
        assert np.nanmax(np.abs(wrap(gy - wy0))) < 2e-5
        ox, oy = oracle.demodulate(g, 6, 20, "xy")
        compare_omega(gx, ox, "tone x")
        compare_omega(gy, oy, "tone y")


def test_chirp_matches_derivative_at_window_centre(dem, torch):
    W, H = 512, 8
    m = np.arange(W)
    c = 1.5e-3
    g = np.exp(1j * (0.4 * m + c * m * m))[None, :].repeat(H, 0).astype(np.complex64)
    for L, N in [(4, 16), (8, 32), (5, 13)]:
        gx, _ = run(dem, torch, g, L, N, "x")
        lo, hi = oracle.valid_range(W, N)
        centre = np.arange(lo, hi + 1) - N // 2 + (N - 1) / 2
        err = np.abs(wrap(gx[:, lo:hi + 1] - (0.4 + 2 * c * centre)))
        assert err.max() < 5e-5, (L, N, err.max())


def test_noisy_complex_low_snr(dem, torch):
    """0 dB complex tones, small K: the regime where the selection is least stable."""
    g = wl.complex_tone(400, 60, 0.9, 0.3, snr_db=0.0, seed=11).astype(np.complex64)
    for L, N in [(4, 8), (4, 16), (8, 32)]:
        gx, gy = run(dem, torch, g, L, N, "xy")
        ox, oy = oracle.demodulate(g, L, N, "xy")
        print(L, N, compare_omega(gx, ox, f"0dB x L{L} N{N}"), compare_omega(gy, oy, f"0dB y L{L} N{N}"))


# ---------------------------------------------------------------------------
# Full-size workloads, sampled lines
# ---------------------------------------------------------------------------
def test_cfg2_frame_full_size_sampled(dem, torch):
    f = wl.cfg2_frame(50)
    gx, gy = run(dem, torch, f.data, f.L, f.N, "xy")
    rows = list(range(3, 1024, 97))
    cols = list(range(5, 1024, 101))
    print("x", compare_omega(gx[rows], oracle_rows(f.data, rows, f.L, f.N), "cfg2 x"))
    print("y", compare_omega(gy[:, cols].T, oracle_cols(f.data, cols, f.L, f.N), "cfg2 y"))


def test_cfg3_uneven_sampled(dem, torch):
    for k in (0, 4, 7, 11):
        f = wl.cfg3_frame(k)
        gx, gy = run(dem, torch, f.data, f.L, f.N, "xy")
        rows = list(range(1, f.height, f.height // 6))
        cols = list(range(2, f.width, f.width // 6))
        compare_omega(gx[rows], oracle_rows(f.data, rows, f.L, f.N), f"cfg3 k{k} x")
        compare_omega(gy[:, cols].T, oracle_cols(f.data, cols, f.L, f.N), f"cfg3 k{k} y")


def test_cfg4_frame_fp16_full_size_sampled(dem, torch):
    f = wl.cfg4_frame(15)
    gx, gy = run(dem, torch, f.data, f.L, f.N, "xy")
    rows = [7, 1500, 2047, 2048, 3999]
    cols = [9, 2048, 4000]
    print("x", compare_omega(gx[rows], oracle_rows(f.data, rows, f.L, f.N), "cfg4 x"))
    print("y", compare_omega(gy[:, cols].T, oracle_cols(f.data, cols, f.L, f.N), "cfg4 y"))


def test_experimental_series_u8_sampled(dem, torch):
    """Stand-in for the paper's experimental series: 1850 x 700 8-bit frames (neither
    length is 5-smooth), line windows N = 15, L = 7, first and last frame."""
    for i in (0, 18):
        f = wl.exp_frame(i)
        gx, gy = run(dem, torch, f.data, f.L, f.N, "xy")
        rows = [0, 7, 349, 350, 699]
        cols = [3, 925, 1849]
        print("x", compare_omega(gx[rows], oracle_rows(f.data, rows, f.L, f.N), f"exp {i} x"))
        print("y", compare_omega(gy[:, cols].T, oracle_cols(f.data, cols, f.L, f.N), f"exp {i} y"))


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def test_zero_frame_and_oversized_window_are_nan(dem, torch):
    z = np.zeros((40, 300), np.float32)
    gx, gy = run(dem, torch, z, 4, 12, "xy")
    assert np.all(np.isnan(gx)) and np.all(np.isnan(gy))
    img = wl.random_frame(30, 20, seed=3)
    gx, gy = run(dem, torch, img, 4, 32, "xy")        # N > W and N > H
    assert np.all(np.isnan(gx)) and np.all(np.isnan(gy))


def test_window_equal_to_L_and_nan_pixel(dem, torch):
    img = wl.random_frame(96, 24, seed=5, dtype=np.float64)
    gx, _ = run(dem, torch, img, 4, 4, "x")            # K = 1
    ox, _ = oracle.demodulate(img, 4, 4, "x")
    compare_omega(gx, ox, "K=1")
    g = wl.complex_tone(120, 4, 0.6, 0.0).astype(np.complex64)
    g[1, 50] = np.nan
    gx, _ = run(dem, torch, g, 3, 10, "x")
    ox, _ = oracle.demodulate(g, 3, 10, "x")
    compare_omega(gx, ox, "nan pixel")
    assert np.isnan(gx[1, 50]) and np.isfinite(gx[0, 50])


def test_max_fft_length_line(dem, torch, bm):
    d = bm.Demodulator(0, max_width=8192, max_height=16)
    img = wl.random_frame(8192, 3, seed=9)
    wx, _ = d.demodulate(to_dev(torch, img), 6, 24, "x")
    torch.cuda.synchronize()
    ox, _ = oracle.demodulate(img, 6, 24, "x")
    compare_omega(wx.cpu().numpy(), ox, "8192 line")
    d.close()


ANY_LENGTH = [
    # (W, H, L, N, dtype, dirs): line lengths with factors 7, 11, 13 take radix-7/11/13
    # passes; a prime factor above 13 takes Bluestein's identity.  Odd line counts leave
    # the last block of the two-line analytic kernel with a single line.
    (1850, 24, 7, 15, np.float32, "x"),      # the paper's experimental width (Sec. 4): 2 * 5^2 * 37, Bluestein
    (48, 700, 5, 15, np.float32, "y"),       # and its height: 2^2 * 5^2 * 7, radix 7
    (1001, 30, 6, 20, np.float64, "xy"),     # 7 * 11 * 13; 1001 columns of 30
    (520, 36, 6, 20, np.float64, "xy"),      # 2^3 * 5 * 13
    (263, 70, 4, 16, np.float16, "xy"),      # prime width (Bluestein); height 2 * 5 * 7
    (4093, 3, 6, 24, np.float32, "x"),       # the largest prime length taken
    (7, 11, 2, 5, np.float32, "xy"),         # shortest radix-7 and radix-11 lines
    (17, 19, 2, 6, np.float32, "xy"),        # shortest Bluestein lines
]


@pytest.mark.parametrize("W,H,L,N,dt,dirs", ANY_LENGTH)
def test_any_line_length(dem, torch, W, H, L, N, dt, dirs):
    img = wl.random_frame(W, H, seed=W + H, dtype=dt, snr_db=8.0)
    gx, gy = run(dem, torch, img, L, N, dirs)
    ox, oy = oracle.demodulate(img, L, N, dirs)
    if "x" in dirs:
        print("x", compare_omega(gx, ox, f"x {W}x{H} L{L} N{N}"))
    if "y" in dirs:
        print("y", compare_omega(gy, oy, f"y {W}x{H} L{L} N{N}"))


def test_flags_mark_borders(dem, torch):
    img = wl.random_frame(300, 40, seed=2)
    wx, wy, fl = dem.demodulate(to_dev(torch, img), 4, 16, "xy", flags=True)
    torch.cuda.synchronize()
    fl = fl.cpu().numpy()
    wx, wy = wx.cpu().numpy(), wy.cpu().numpy()
    assert np.array_equal((fl & 1) != 0, np.isnan(wx))
    assert np.array_equal((fl & 16) != 0, np.isnan(wy))


@pytest.mark.parametrize("L", [4, 6, 8])
def test_degenerate_signal_subspace_flagged(bm, torch, L):
    """Two complex tones of equal power whose steering vectors are orthogonal over L
    samples and whose cross terms cancel over the K = 4L sub-snapshots: lambda_1 =
    lambda_2, no one-dimensional signal subspace (Eq. 6-11): every valid window is NaN
    with BM_FLAG_DEGENERATE, as in the oracle, through the plain, all-roots, Jacobi and
    surrogate (lag-1 predictor) paths.  A power ratio of 1.01 is demodulated normally."""
    W, H, N = 256, 6, 5 * L - 1
    n = np.arange(W)
    w1, w2 = 0.4, 0.4 + 2 * np.pi / L
    for ratio in (1.0, 1.01):
        line = np.sqrt(ratio) * np.exp(1j * (w1 * n + 0.3)) + np.exp(1j * (w2 * n - 1.1))
        g = np.repeat(line[None], H, 0).astype(np.complex64)
        ref, _ = oracle.demodulate(g, L, N, "x")
        lo, hi = oracle.valid_range(W, N)
        assert np.all(np.isnan(ref[:, lo:hi + 1])) == (ratio == 1.0)
        for kw, mode in ((dict(), bm.BM_PLAIN), (dict(full_roots=True), bm.BM_PLAIN), (dict(jacobi=True), bm.BM_PLAIN),
                         (dict(), bm.BM_SURROGATE)):
            d = bm.Demodulator(0, max_width=W, max_height=H, **kw)
            if mode == bm.BM_SURROGATE:
                bm.bosmusic_surrogate_config(d.h, 0.25, 1)
            wx, _, fl = d.demodulate(to_dev(torch, g), L, N, "x", flags=True, mode=mode)
            torch.cuda.synchronize()
            wx, fl = wx.cpu().numpy(), fl.cpu().numpy()
            d.close()
            compare_omega(wx, ref, f"two tones L{L} ratio {ratio} {kw} mode {mode}")
            inner = fl[:, lo:hi + 1]
            if ratio == 1.0:
                assert np.all(inner == bm.BM_FLAG_DEGENERATE), (kw, mode, np.unique(inner))
            else:
                assert not np.any(fl & bm.BM_FLAG_DEGENERATE), (kw, mode)
                assert np.nanmax(np.abs(wrap(wx - w1))) < 1e-4
            assert np.all(fl[:, :lo] == bm.BM_FLAG_UNDEFINED) and np.all(fl[:, hi + 1:] == bm.BM_FLAG_UNDEFINED)


def test_deterministic_reruns(dem, torch):
    img = to_dev(torch, wl.random_frame(576, 64, seed=4))
    a = dem.demodulate(img, 6, 32, "xy")
    b = dem.demodulate(img, 6, 32, "xy")
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(torch.nan_to_num(u, 7.0), torch.nan_to_num(v, 7.0))


def test_invalid_arguments_enqueue_nothing(dem, torch, bm):
    img = to_dev(torch, wl.random_frame(64, 64, seed=1))
    wx = torch.full((64, 64), 5.0, device="cuda")
    bad = [
        bm.FrameSpec(img, 1, 16, bm.BM_DIR_X, wx),       # L < 2
        bm.FrameSpec(img, 9, 16, bm.BM_DIR_X, wx),       # L > 8
        bm.FrameSpec(img, 6, 5, bm.BM_DIR_X, wx),        # N < L
        bm.FrameSpec(img, 6, 65, bm.BM_DIR_X, wx),       # N > 64
        bm.FrameSpec(img, 6, 16, 0, wx),                 # no direction
        bm.FrameSpec(img, 6, 16, bm.BM_DIR_Y, wx, None),  # omega_y missing
    ]
    good = bm.FrameSpec(img, 6, 16, bm.BM_DIR_X, wx)
    for b in bad:
        with pytest.raises(bm.BosmusicError) as ei:
            bm.bosmusic_demodulate(dem.h, [good, b])
        assert ei.value.status == bm.BM_E_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(wx == 5.0)          # the valid first frame was not run either
    wide = bm.Demodulator(0, max_width=8192, max_height=8)
    odd = torch.zeros((4, 4099), device="cuda")          # 4099 is prime and above the Bluestein limit
    with pytest.raises(bm.BosmusicError) as ei:
        bm.bosmusic_demodulate(wide.h, [bm.FrameSpec(odd, 6, 16, bm.BM_DIR_X, torch.empty((4, 4099), device="cuda"))])
    assert ei.value.status == bm.BM_E_UNSUPPORTED
    wide.close()
    big = torch.zeros((10, 5000), device="cuda")
    with pytest.raises(bm.BosmusicError) as ei:
        bm.bosmusic_demodulate(dem.h, [bm.FrameSpec(big, 6, 16, bm.BM_DIR_X, torch.empty((10, 5000), device="cuda"))])
    assert ei.value.status == bm.BM_E_INVALID_ARG
    with pytest.raises(bm.BosmusicError) as ei:
        bm.bosmusic_demodulate(dem.h, [good], mode=bm.BM_SURROGATE)
    assert ei.value.status == bm.BM_E_UNSUPPORTED


def test_stats_count_windows(dem, torch):
    dem.stats(reset=True)
    img = wl.random_frame(300, 20, seed=8)
    dem.demodulate(to_dev(torch, img), 5, 20, "xy")
    s = dem.stats(reset=True)
    nx = 20 * (300 - 20 + 1)
    ny = 300 * (20 - 20 + 1)
    assert s["windows"] == nx + ny
    assert s["eig_iters"] >= s["windows"]
    assert s["sur_accepted"] + s["sur_rejected"] == s["windows"]        # certified pair or all roots
    assert s["pair_iters"] >= s["windows"] and s["root_iters"] >= s["sur_rejected"]
    # FP32 steps towards the signal root come first, at least one per window that took them
    assert s["pair_iters32"] >= s["sur_accepted"]
    print(s)


# ---------------------------------------------------------------------------
# Integration
# ---------------------------------------------------------------------------
def test_integrate_matches_oracle_on_same_omega(dem, torch):
    """The integration step alone: both sides integrate the same omega maps, which
    come from the oracle (FP32-rounded), never from the GPU."""
    f = wl.cfg2_frame(10)
    img = f.data[:512, :600]
    ox, oy = oracle.demodulate(img, 6, 32, "xy")
    ox32, oy32 = ox.astype(np.float32), oy.astype(np.float32)
    wx, wy = to_dev(torch, ox32), to_dev(torch, oy32)
    phi = dem.integrate(wx, wy, 32, 32, 0.3, 0.1)
    torch.cuda.synchronize()
    ref = oracle.integrate(ox32, oy32, 32, 32, 0.3, 0.1)
    got = phi.cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    m = np.isfinite(ref)
    assert np.max(np.abs(got[m] - ref[m])) < 1e-9
    # without omega_y
    phi2 = dem.integrate(wx, None, 32, 0)
    torch.cuda.synchronize()
    ref2 = oracle.integrate(ox32, None, 32, 0)
    got2 = phi2.cpu().numpy()
    assert np.array_equal(np.isnan(got2), np.isnan(ref2))
    m = np.isfinite(ref2)
    assert np.max(np.abs(got2[m] - ref2[m])) < 1e-9


def test_integrate_many_equals_single_calls(dem, torch, bm):
    """The batched integration gives bit for bit what one call per map gives."""
    rng = np.random.default_rng(4)
    maps = []
    for (W, H, nx, ny, with_y) in [(300, 40, 20, 12, True), (64, 100, 8, 8, False), (1024, 7, 32, 5, True),
                                   (50, 30, 60, 8, True)]:
        wx = to_dev(torch, (0.5 + 0.1 * rng.standard_normal((H, W))).astype(np.float32))
        wy = to_dev(torch, (0.2 + 0.1 * rng.standard_normal((H, W))).astype(np.float32)) if with_y else None
        maps.append((wx, wy, nx, ny, 0.1, -0.2))
    singles = [dem.integrate(wx, wy, nx, ny, cx, cy) for (wx, wy, nx, ny, cx, cy) in maps]
    outs = [torch.empty(m[0].shape, dtype=torch.float64, device="cuda") for m in maps]
    bm.bosmusic_integrate_many(dem.h, [m + (o,) for m, o in zip(maps, outs)])
    bm.bosmusic_integrate_many(dem.h, [m + (o,) for m, o in zip(maps, outs)])       # reuse of the tables
    torch.cuda.synchronize()
    for a, b in zip(singles, outs):
        assert torch.equal(torch.nan_to_num(a, 7.0), torch.nan_to_num(b, 7.0))
    assert torch.isnan(outs[3]).all()                                # Nx > W: nothing valid


def test_integrate_many_equals_single_calls_wide_rows(dem, torch, bm):
    """Rows go through registers (width a multiple of 4 up to 4096, 16-byte
    aligned maps) or through LDS (other widths, an 8-byte aligned phi); single and
    batched calls launch different block sizes and still agree bit for bit, and
    both match the FP64 oracle's trapezoid sums."""
    rng = np.random.default_rng(9)
    maps, outs = [], []
    for (W, H, nx, ny, with_y, shift) in [(4096, 12, 32, 8, True, 0), (1024, 9, 16, 4, True, 0),
                                          (2048, 5, 20, 6, False, 0), (1000, 12, 8, 8, True, 0),
                                          (1002, 10, 10, 6, True, 0), (512, 6, 12, 4, True, 1)]:
        wx = to_dev(torch, (0.5 + 0.1 * rng.standard_normal((H, W))).astype(np.float32))
        wy = to_dev(torch, (0.2 + 0.1 * rng.standard_normal((H, W))).astype(np.float32)) if with_y else None
        maps.append((wx, wy, nx, ny, 0.1, -0.2))
        buf = torch.empty(H * W + shift, dtype=torch.float64, device="cuda")
        outs.append(buf[shift:].view(H, W))                  # shift 1: phi only 8-byte aligned
    singles = [dem.integrate(wx, wy, nx, ny, cx, cy) for (wx, wy, nx, ny, cx, cy) in maps]
    bm.bosmusic_integrate_many(dem.h, [m + (o,) for m, o in zip(maps, outs)])
    torch.cuda.synchronize()
    for (wx, wy, nx, ny, cx, cy), a, b in zip(maps, singles, outs):
        assert torch.equal(torch.nan_to_num(a, 7.0), torch.nan_to_num(b, 7.0))
        ref = oracle.integrate(wx.cpu().numpy(), None if wy is None else wy.cpu().numpy(), nx, ny, cx, cy)
        got = b.cpu().numpy()
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        assert np.max(np.abs(got[ok] - ref[ok])) < 1e-9


def test_integrate_end_to_end_linear_phase(dem, torch):
    W, H = 240, 96
    wx0, wy0 = 2 * np.pi * 23 / W, 2 * np.pi * 9 / H
    x = np.arange(W)[None, :]
    y = np.arange(H)[:, None]
    img = (0.5 + 0.4 * np.cos(wx0 * x + wy0 * y + 0.2)).astype(np.float64)
    wx, wy = dem.demodulate(to_dev(torch, img), 5, 16, "xy")
    phi = dem.integrate(wx, wy, 16, 16).cpu().numpy()
    x0, _ = oracle.valid_range(W, 16)
    y0, _ = oracle.valid_range(H, 16)
    ref = np.broadcast_to(wx0 * (x - x0) + wy0 * (y - y0), (H, W))
    m = np.isfinite(phi)
    assert m.sum() == (W - 15) * (H - 15)
    assert np.max(np.abs(phi[m] - ref[m])) < 2e-3


def test_jacobi_option_agrees_with_default_solver(bm, torch):
    """Two independent eigensolvers for the signal subspace: each meets the parity bar
    against the FP64 oracle, and they agree with each other."""
    dj = bm.Demodulator(0, max_width=1024, max_height=1024, jacobi=True)
    dt = bm.Demodulator(0, max_width=1024, max_height=1024)
    for (W, H, L, N, snr) in [(600, 40, 4, 12, 3.0), (576, 40, 6, 32, 10.0), (512, 32, 8, 32, 6.0)]:
        img_np = wl.random_frame(W, H, seed=L, snr_db=snr)
        img = to_dev(torch, img_np)
        a = dj.demodulate(img, L, N, "xy")
        b = dt.demodulate(img, L, N, "xy")
        torch.cuda.synchronize()
        ref = oracle.demodulate(img_np, L, N, "xy")
        for u, v, o, name in zip(a, b, ref, "xy"):
            u, v = u.cpu().numpy(), v.cpu().numpy()
            compare_omega(u, o, f"jacobi vs oracle L{L} {name}")
            compare_omega(v, o, f"tridiagonal vs oracle L{L} {name}")
            compare_omega(u, v, f"jacobi vs tridiagonal L{L} {name}")
    dj.close()
    dt.close()


@pytest.mark.parametrize("L,N,snr", [(2, 8, 10.0), (4, 12, 0.0), (6, 32, 10.0), (8, 32, 3.0), (8, 64, 20.0)])
def test_certified_pair_agrees_with_all_roots(bm, torch, L, N, snr):
    """The certified-pair shortcut returns the pair that finding every root selects;
    both agree with the oracle, and most windows take the shortcut."""
    img_np = wl.random_frame(540, 36, seed=10 * L + N, snr_db=snr)
    img = to_dev(torch, img_np)
    dc = bm.Demodulator(0, max_width=1024, max_height=1024, stats=True)
    df = bm.Demodulator(0, max_width=1024, max_height=1024, stats=True, full_roots=True)
    a = dc.demodulate(img, L, N, "xy")
    b = df.demodulate(img, L, N, "xy")
    torch.cuda.synchronize()
    sc, sf = dc.stats(), df.stats()
    assert sf["sur_accepted"] == 0 and sf["sur_rejected"] == 0
    assert sc["sur_accepted"] + sc["sur_rejected"] == sc["windows"]
    ref = oracle.demodulate(img_np, L, N, "xy")
    for u, v, o, name in zip(a, b, ref, "xy"):
        u, v = u.cpu().numpy(), v.cpu().numpy()
        compare_omega(u, v, f"certified vs all roots L{L} {name}")
        compare_omega(u, o, f"certified vs oracle L{L} {name}")
    frac = sc["sur_accepted"] / max(1, sc["windows"])
    print(f"L{L} N{N} {snr} dB: certified {frac:.4f} of {sc['windows']} windows")
    # L = 2: the two roots of a quadratic conjugate-reciprocal polynomial often both lie on
    # the unit circle, which is not a mate pair, so those windows find all roots
    assert frac > (0.5 if snr < 5 or L == 2 else 0.9)
    dc.close()
    df.close()


def test_alloc_fault_in_create_reports_nomem_and_cleans_up(bm, torch, monkeypatch):
    """BOSMUSIC_FAULT=alloc fails the workspace allocation of create after its first buffer:
    BM_E_NOMEM with the reason, no handle, and a later create on the same device works."""
    monkeypatch.setenv("BOSMUSIC_FAULT", "alloc")
    with pytest.raises(bm.BosmusicError) as ei:
        bm.Demodulator(0, max_width=256, max_height=256)
    assert ei.value.status == bm.BM_E_NOMEM
    assert "workspace" in bm.bosmusic_last_error(None)
    monkeypatch.delenv("BOSMUSIC_FAULT")
    d = bm.Demodulator(0, max_width=256, max_height=256)
    img = torch.from_numpy(wl.random_frame(128, 16, seed=2)).cuda()
    wx, _ = d.demodulate(img, 4, 16, "x")
    torch.cuda.synchronize()
    assert np.isfinite(wx.cpu().numpy()).any()
    d.close()


def test_log_lines_on_request(bm, torch, monkeypatch, capfd):
    """BOSMUSIC_LOG=1 at create: one line for the handle and one per planned group."""
    monkeypatch.setenv("BOSMUSIC_LOG", "1")
    d = bm.Demodulator(0, max_width=256, max_height=256)
    monkeypatch.delenv("BOSMUSIC_LOG")
    img = torch.from_numpy(wl.random_frame(128, 16, seed=3)).cuda()
    d.demodulate(img, 4, 16, "xy")
    torch.cuda.synchronize()
    d.close()
    err = capfd.readouterr().err
    assert "[bosmusic] create: device 0" in err
    assert "[bosmusic] group frames 0..0" in err and "L4:" in err

