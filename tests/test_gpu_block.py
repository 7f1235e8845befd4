"""Block windows (the paper's L x L moving window, Sec. 3) on the GPU against the
block-mode oracle, through the C ABI.  Bar as for line windows: identical NaN
patterns and |d omega| <= 1e-4 rad/px at the 99.9th percentile."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare_omega, wrap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    # (W, H, M, dtype, snr)
    (300, 40, 2, np.float32, 8.0),
    (270, 45, 3, np.float64, 5.0),
    (640, 30, 4, np.float16, 10.0),
    (256, 50, 5, np.float32, 0.0),
    (576, 36, 6, np.float32, 8.0),
    (250, 48, 7, np.float64, 3.0),
    (512, 33, 8, np.float16, 10.0),
    (263, 30, 5, np.float32, 6.0),       # prime width: the row DFT goes through Bluestein's identity
]


@pytest.mark.parametrize("W,H,M,dt,snr", CASES)
def test_block_windows_match_oracle(bm, torch, W, H, M, dt, snr):
    d = bm.Demodulator(0, max_width=1024, max_height=1024)
    img = wl.random_frame(W, H, seed=W + M, dtype=dt, snr_db=snr)
    gx, gy = d.demodulate(dev(torch, img), M, M, "xy", block=True)
    torch.cuda.synchronize()
    ox, oy = oracle.demodulate_block(img, M)
    print("x", compare_omega(gx.cpu().numpy(), ox, f"block x {W}x{H} M{M}"))
    print("y", compare_omega(gy.cpu().numpy(), oy, f"block y {W}x{H} M{M}"))
    d.close()


def test_block_plane_waves_exact(bm, torch):
    d = bm.Demodulator(0, max_width=512, max_height=512)
    for M in (3, 5, 8):
        for (wx, wy) in [(0.7, -0.4), (-2.5, 1.9), (0.05, 3.0)]:
            g = wl.complex_tone(300, 70, wx, wy).astype(np.complex64)
            gx, gy = d.demodulate(dev(torch, g), M, M, "xy", block=True)
            torch.cuda.synchronize()
            gx, gy = gx.cpu().numpy(), gy.cpu().numpy()
            assert np.isfinite(gx).sum() == (70 - M + 1) * (300 - M + 1)
            assert np.nanmax(np.abs(wrap(gx - wx))) < 2e-5 and np.nanmax(np.abs(wrap(gy - wy))) < 2e-5
    d.close()


def test_block_paper_shape_low_snr_sampled(bm, torch):
    """The paper's simulation shape: a 512 x 512 fringe at 0 dB (Sec. 4), block 7 x 7."""
    d = bm.Demodulator(0, max_width=512, max_height=512)
    img = wl.random_frame(512, 512, seed=77, snr_db=0.0)
    gx, gy = d.demodulate(dev(torch, img), 7, 7, "xy", block=True)
    torch.cuda.synchronize()
    rows = [3, 100, 255, 400, 508]
    gxn, gyn = gx.cpu().numpy(), gy.cpu().numpy()
    for r in rows:
        sub = img[max(0, r - 3):r + 4]
        ox, oy = oracle.demodulate_block(sub, 7)
        k = r - max(0, r - 3)
        compare_omega(gxn[r], ox[k], f"paper shape x row {r}")
        compare_omega(gyn[r], oy[k], f"paper shape y row {r}")
    d.close()


def test_block_flags_and_mixed_batch(bm, torch):
    """Block and line frames of different L in one call give what separate calls give."""
    d = bm.Demodulator(0, max_width=1024, max_height=1024)
    a = wl.random_frame(300, 40, seed=1, snr_db=6.0)
    b = wl.random_frame(256, 64, seed=2, snr_db=6.0)
    da, db = dev(torch, a), dev(torch, b)
    ax = torch.empty_like(da)
    ay = torch.empty_like(da)
    af = torch.empty(da.shape, dtype=torch.uint8, device="cuda")
    bx = torch.empty_like(db)
    by = torch.empty_like(db)
    specs = [bm.FrameSpec(da, 5, 5, bm.BM_DIR_X | bm.BM_DIR_Y | bm.BM_BLOCK, ax, ay, af),
             bm.FrameSpec(db, 6, 24, bm.BM_DIR_X | bm.BM_DIR_Y, bx, by)]
    d.demodulate_many(specs)
    sx, sy, sf = d.demodulate(da, 5, 5, "xy", flags=True, block=True)
    lx, ly = d.demodulate(db, 6, 24, "xy")
    torch.cuda.synchronize()
    for u, v in ((ax, sx), (ay, sy), (bx, lx), (by, ly)):
        assert torch.equal(torch.nan_to_num(u, 9.0), torch.nan_to_num(v, 9.0))
    assert torch.equal(af, sf)
    f = af.cpu().numpy()
    assert np.array_equal((f & 1) != 0, np.isnan(ax.cpu().numpy()))
    assert np.array_equal((f & 16) != 0, np.isnan(ay.cpu().numpy()))
    d.close()


def test_block_graph_replays_match_eager(bm, torch):
    eager = bm.Demodulator(0, max_width=512, max_height=512)
    graph = bm.Demodulator(0, max_width=512, max_height=512, graph=True)
    img = dev(torch, wl.random_frame(384, 48, seed=5, snr_db=5.0))
    ex, ey = eager.demodulate(img, 7, 7, "xy", block=True)
    torch.cuda.synchronize()
    outs = [torch.empty_like(img) for _ in range(2)]
    spec = [bm.FrameSpec(img, 7, 7, bm.BM_DIR_X | bm.BM_DIR_Y | bm.BM_BLOCK, outs[0], outs[1])]
    for rep in range(3):
        for o in outs:
            o.fill_(-7.0)
        graph.demodulate_many(spec)
        torch.cuda.synchronize()
        junk = eager.demodulate(img, 4, 12, "x")[0]           # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk).any()
        assert torch.equal(torch.nan_to_num(outs[0], 9.0), torch.nan_to_num(ex, 9.0)), rep
        assert torch.equal(torch.nan_to_num(outs[1], 9.0), torch.nan_to_num(ey, 9.0)), rep
    eager.close()
    graph.close()


def test_block_certified_agrees_with_all_roots(bm, torch):
    img = dev(torch, wl.random_frame(300, 40, seed=8, snr_db=4.0))
    dc = bm.Demodulator(0, max_width=512, max_height=512, stats=True)
    df = bm.Demodulator(0, max_width=512, max_height=512, full_roots=True)
    a = dc.demodulate(img, 6, 6, "xy", block=True)
    b = df.demodulate(img, 6, 6, "xy", block=True)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        compare_omega(u.cpu().numpy(), v.cpu().numpy(), "block certified vs all roots")
    st = dc.stats()
    assert st["sur_accepted"] + st["sur_rejected"] == st["windows"] > 0
    dc.close()
    df.close()


def test_block_argument_checks(bm, torch):
    d = bm.Demodulator(0, max_width=256, max_height=256)
    img = dev(torch, wl.random_frame(128, 32, seed=1))
    with pytest.raises(bm.BosmusicError) as ei:
        d.demodulate(img, 5, 7, "xy", block=True)                # N != L
    assert ei.value.status == bm.BM_E_INVALID_ARG
    bm.bosmusic_surrogate_config(d.h, 0.25, 1)
    with pytest.raises(bm.BosmusicError) as ei:
        d.demodulate(img, 8, 8, "x", block=True, mode=bm.BM_SURROGATE)
    assert ei.value.status == bm.BM_E_UNSUPPORTED
    # a block larger than the frame: all NaN, not an error
    small = dev(torch, wl.random_frame(30, 6, seed=2))
    gx, gy = d.demodulate(small, 7, 7, "xy", block=True)
    torch.cuda.synchronize()
    assert torch.isnan(gx).all() and torch.isnan(gy).all()
    d.close()


@pytest.mark.parametrize("M,dt", [(5, np.float32), (7, np.float16), (4, np.float64)])
def test_block_phase_matches_oracle(bm, torch, M, dt):
    d = bm.Demodulator(0, max_width=512, max_height=512)
    img = wl.random_frame(320, 40, seed=3 * M, dtype=dt, snr_db=6.0)
    gx, gy, ph = d.demodulate(dev(torch, img), M, M, "xy", block=True, phase=True)
    torch.cuda.synchronize()
    ox, oy = oracle.demodulate_block(img, M)
    ref = oracle.block_phase(img, M, ox, oy)
    got = ph.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    v = np.isfinite(ref)
    e = np.abs(wrap(got[v] - ref[v]))
    print(f"block phase M{M}: p99.9 {np.quantile(e, 0.999):.2e} max {e.max():.2e}")
    assert np.quantile(e, 0.999) <= 1e-4
    d.close()


def test_block_phase_of_a_plane_wave(bm, torch):
    d = bm.Demodulator(0, max_width=512, max_height=512)
    W, H, wx, wy, a = 300, 50, 0.8, -0.45, 1.3
    g = wl.complex_tone(W, H, wx, wy, alpha=a).astype(np.complex64)
    _, _, ph = d.demodulate(dev(torch, g), 6, 6, "xy", block=True, phase=True)
    torch.cuda.synchronize()
    y, x = np.mgrid[0:H, 0:W]
    got = ph.cpu().numpy()
    v = np.isfinite(got)
    assert v.sum() == (H - 5) * (W - 5)
    assert np.max(np.abs(wrap(got[v] - (a + wx * x + wy * y)[v]))) < 5e-5
    with pytest.raises(bm.BosmusicError):
        d.demodulate(dev(torch, g), 6, 6, "x", block=True, phase=True)     # phase needs both directions
    d.close()


BIG_CASES = [
    # (W, H, M, dtype, snr): the paper's odd windows above 8 x 8, to the 17 x 17 of its table
    (220, 24, 9, np.float32, 5.0),
    (240, 28, 11, np.float16, 0.0),
    (200, 30, 13, np.float64, 8.0),
    (256, 32, 15, np.uint8, 10.0),
    (231, 34, 17, np.float32, 3.0),      # 231 = 3 * 7 * 11: the row DFT takes radix-7 and -11 passes
]


@pytest.mark.parametrize("W,H,M,dt,snr", BIG_CASES)
def test_big_block_windows_match_oracle(bm, torch, W, H, M, dt, snr):
    d = bm.Demodulator(0, max_width=1024, max_height=1024, stats=True)
    img = wl.random_frame(W, H, seed=W + M, dtype=dt, snr_db=snr)
    gx, gy = d.demodulate(dev(torch, img), M, M, "xy", block=True)
    torch.cuda.synchronize()
    st = d.stats()
    ox, oy = oracle.demodulate_block(img, M)
    print("x", compare_omega(gx.cpu().numpy(), ox, f"block x {W}x{H} M{M}"))
    print("y", compare_omega(gy.cpu().numpy(), oy, f"block y {W}x{H} M{M}"))
    print(f"M{M}: certified {st['sur_accepted']} of {st['windows']}")
    assert st["windows"] == 2 * (W - M + 1) * (H - M + 1)
    d.close()


def test_block_paper_simulation_shape_11x11(bm, torch):
    """The paper's simulation (Sec. 4): 512 x 512 at 0 dB with L = 5, i.e. an 11 x 11
    window; sampled rows against the oracle on the rows around them."""
    d = bm.Demodulator(0, max_width=512, max_height=512)
    img = wl.random_frame(512, 512, seed=78, snr_db=0.0)
    gx, gy = d.demodulate(dev(torch, img), 11, 11, "xy", block=True)
    torch.cuda.synchronize()
    gxn, gyn = gx.cpu().numpy(), gy.cpu().numpy()
    assert np.isfinite(gxn).sum() == 502 * 502
    for r in (5, 97, 256, 431, 506):
        sub = img[r - 5:r + 6]
        ox, oy = oracle.demodulate_block(sub, 11)
        compare_omega(gxn[r], ox[5], f"11x11 x row {r}")
        compare_omega(gyn[r], oy[5], f"11x11 y row {r}")
    d.close()


def test_big_block_plane_waves_exact_and_phase(bm, torch):
    d = bm.Demodulator(0, max_width=512, max_height=512)
    W, H = 200, 60
    for M in (9, 15):
        for (wx, wy, a) in [(0.7, -0.4, 0.3), (-2.5, 1.9, -1.2)]:
            g = wl.complex_tone(W, H, wx, wy, alpha=a).astype(np.complex64)
            gx, gy, ph = d.demodulate(dev(torch, g), M, M, "xy", block=True, phase=True)
            torch.cuda.synchronize()
            gx, gy, ph = gx.cpu().numpy(), gy.cpu().numpy(), ph.cpu().numpy()
            assert np.isfinite(gx).sum() == (H - M + 1) * (W - M + 1)
            assert np.nanmax(np.abs(wrap(gx - wx))) < 2e-5 and np.nanmax(np.abs(wrap(gy - wy))) < 2e-5
            y, x = np.mgrid[0:H, 0:W]
            v = np.isfinite(ph)
            assert np.max(np.abs(wrap(ph[v] - (a + wx * x + wy * y)[v]))) < 1e-4
    d.close()


def test_big_block_certified_agrees_with_all_roots_and_phase(bm, torch):
    img_np = wl.random_frame(220, 30, seed=9, snr_db=2.0)
    img = dev(torch, img_np)
    dc = bm.Demodulator(0, max_width=512, max_height=512, stats=True)
    df = bm.Demodulator(0, max_width=512, max_height=512, full_roots=True)
    a = dc.demodulate(img, 11, 11, "xy", block=True, phase=True)
    b = df.demodulate(img, 11, 11, "xy", block=True)
    torch.cuda.synchronize()
    for u, v in zip(a[:2], b):
        compare_omega(u.cpu().numpy(), v.cpu().numpy(), "11x11 certified vs all roots")
    st = dc.stats()
    assert st["sur_accepted"] + st["sur_rejected"] == st["windows"] > 0
    ox, oy = oracle.demodulate_block(img_np, 11)
    ref = oracle.block_phase(img_np, 11, ox, oy)
    got = a[2].cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    v = np.isfinite(ref)
    assert np.quantile(np.abs(wrap(got[v] - ref[v])), 0.999) <= 1e-4
    dc.close()
    df.close()


def test_big_block_argument_checks(bm, torch):
    d = bm.Demodulator(0, max_width=256, max_height=256)
    img = dev(torch, wl.random_frame(128, 40, seed=1))
    for M in (10, 16, 19):                 # above 8 x 8 only odd sizes up to 17
        with pytest.raises(bm.BosmusicError) as ei:
            d.demodulate(img, M, M, "xy", block=True)
        assert ei.value.status == bm.BM_E_INVALID_ARG
    with pytest.raises(bm.BosmusicError) as ei:
        d.demodulate(img, 9, 9, "xy")     # line windows stay at L <= 8
    assert ei.value.status == bm.BM_E_INVALID_ARG
    d.close()
