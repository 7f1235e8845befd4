"""Temporal warm start (the paper's time-lapsed series, Sec. 1 and 4: the phase
changes little between successive frames): the signal-root Newton of each window
starts at the previous frame's frequency at that pixel.  The certified pair is the
same, so the maps equal the cold-start ones and the oracle's; the test also prints
the Newton step counts of both starts (the evidence the option is judged on)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from parity_util import compare_omega

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def series_frame(t, W=512, H=384):
    """Successive frames of a diffusion series (erf phase widening with t)."""
    img, _, _ = wl.erf_fringe(W, H, 0.1, 30.0, 6.0, H / 2.0, 8.0 * 1.08 ** t, 10.0, 700 + t, np.float32)
    return img


@pytest.mark.parametrize("L,N", [(6, 32), (8, 32), (4, 16)])
def test_warm_start_matches_cold_start_and_oracle(bm, torch, L, N):
    d = bm.Demodulator(0, max_width=1024, max_height=1024, stats=True)
    f0, f1 = series_frame(0), series_frame(1)
    H, W = f1.shape
    p0 = d.demodulate(torch.from_numpy(f0).cuda(), L, N, "xy")
    torch.cuda.synchronize()
    d.stats(reset=True)
    g1 = torch.from_numpy(f1).cuda()
    cold = d.demodulate(g1, L, N, "xy")
    torch.cuda.synchronize()
    sc = d.stats(reset=True)
    wx = torch.empty((H, W), device="cuda")
    wy = torch.empty((H, W), device="cuda")
    bm.bosmusic_demodulate(d.h, [bm.FrameSpec(g1, L, N, 3, wx, wy, prev_omega_x=p0[0], prev_omega_y=p0[1])])
    torch.cuda.synchronize()
    sw = d.stats(reset=True)
    ref = oracle.demodulate(f1, L, N, "xy")
    for c, w, o, name in zip(cold, (wx, wy), ref, "xy"):
        c, w = c.cpu().numpy(), w.cpu().numpy()
        compare_omega(w, o, f"warm vs oracle L{L} {name}")
        compare_omega(w, c, f"warm vs cold L{L} {name}")
    per = lambda s, k: s[k] / max(1, s["windows"])
    print(f"L{L} N{N}: FP32/FP64 Newton steps per window cold {per(sc, 'pair_iters32'):.3f}/"
          f"{per(sc, 'pair_iters'):.3f}, warm {per(sw, 'pair_iters32'):.3f}/{per(sw, 'pair_iters'):.3f}; "
          f"certified cold {per(sc, 'sur_accepted'):.5f} warm {per(sw, 'sur_accepted'):.5f}")
    assert sw["windows"] == sc["windows"]
    d.close()


def test_warm_start_tolerates_nan_and_garbage_previous_maps(bm, torch):
    """NaN previous values fall back to the window's own start; a previous map of
    unrelated frequencies only costs iterations (or the all-roots path), never accuracy."""
    d = bm.Demodulator(0, max_width=1024, max_height=1024)
    f1 = series_frame(3)
    H, W = f1.shape
    g1 = torch.from_numpy(f1).cuda()
    rng = np.random.default_rng(0)
    junk = torch.from_numpy(rng.uniform(-3.1, 3.1, (H, W)).astype(np.float32)).cuda()
    junk[::3] = float("nan")
    wx = torch.empty((H, W), device="cuda")
    wy = torch.empty((H, W), device="cuda")
    bm.bosmusic_demodulate(d.h, [bm.FrameSpec(g1, 6, 32, 3, wx, wy, prev_omega_x=junk, prev_omega_y=junk)])
    torch.cuda.synchronize()
    ref = oracle.demodulate(f1, 6, 32, "xy")
    compare_omega(wx.cpu().numpy(), ref[0], "junk prev x")
    compare_omega(wy.cpu().numpy(), ref[1], "junk prev y")
    d.close()
