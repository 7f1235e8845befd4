"""Surrogate mode on the GPU: MLP forward parity with the oracle, and the
surrogate + plain-fallback maps against the FP64 oracle (RMS <= 2e-3 rad/px)."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import surrogate as S
from parity_util import compare_omega, wrap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rms_vs_oracle(got, ref):
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    m = np.isfinite(ref)
    d = wrap(got[m] - ref[m])
    return math.sqrt(np.mean(d * d)), np.abs(d)


def test_mlp_forward_matches_oracle(bm, torch):
    d = bm.Demodulator(0, max_width=256, max_height=256)
    p = S.init_params(21)
    bm.bosmusic_surrogate_load(d.h, p)
    back = bm.bosmusic_surrogate_save(d.h)
    assert np.array_equal(back, bm._flat_params(p))
    X = np.random.default_rng(5).standard_normal((1000, 32)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty((1000, 2), device="cuda")
    bm.bosmusic_surrogate_forward(d.h, Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    ref = S.forward(p, X, quantize=True, fp32_acc=True)["Y"]
    err = np.abs(Y - ref)
    scale = np.max(np.abs(ref))
    # equal up to bfloat16 rounding decisions taken on FP32 sums in another order
    assert np.quantile(err, 0.99) < 2e-3 * scale, np.quantile(err, 0.99)
    assert err.max() < 3e-2 * scale, err.max()
    d.close()


@pytest.mark.parametrize("predictor", [1, 0])
def test_surrogate_maps_match_oracle(bm, torch, predictor):
    """Lag-1 predictor, and an untrained MLP (most windows then take the fallback)."""
    d = bm.Demodulator(0, max_width=1024, max_height=1024, stats=True)
    if predictor == 0:
        bm.bosmusic_surrogate_load(d.h, S.init_params(3))
    bm.bosmusic_surrogate_config(d.h, 0.25, predictor)
    for (W, H, L, N, snr) in [(600, 48, 8, 32, 10.0), (512, 40, 6, 24, 5.0), (300, 64, 4, 16, 15.0)]:
        img = wl.random_frame(W, H, seed=L + W, snr_db=snr)
        wx, wy = d.demodulate(torch.from_numpy(img).cuda(), L, N, "xy", mode=bm.BM_SURROGATE)
        torch.cuda.synchronize()
        st = d.stats(reset=True)
        ox, oy = oracle.demodulate(img, L, N, "xy")
        for got, ref, name in ((wx, ox, "x"), (wy, oy, "y")):
            r, dd = rms_vs_oracle(got.cpu().numpy(), ref)
            print(f"pred={predictor} L{L} {name}: rms {r:.2e} p99.9 {np.quantile(dd, 0.999):.2e} "
                  f"accepted {st['sur_accepted']} rejected {st['sur_rejected']}")
            assert r <= 2e-3
        assert st["sur_accepted"] + st["sur_rejected"] > 0
        if predictor == 1:
            assert st["sur_accepted"] > 0.5 * (st["sur_accepted"] + st["sur_rejected"])
    d.close()


def test_surrogate_graph_replays_match_eager(bm, torch):
    eager = bm.Demodulator(0, max_width=1024, max_height=1024)
    graph = bm.Demodulator(0, max_width=1024, max_height=1024, graph=True)
    for h in (eager.h, graph.h):
        bm.bosmusic_surrogate_config(h, 0.25, 1)
    img = torch.from_numpy(wl.random_frame(600, 64, seed=2, snr_db=8.0)).cuda()
    wx = torch.empty((64, 600), device="cuda")
    wy = torch.empty((64, 600), device="cuda")
    spec = [bm.FrameSpec(img, 8, 32, 3, wx, wy)]
    bm.bosmusic_demodulate(eager.h, spec, bm.BM_SURROGATE)
    torch.cuda.synchronize()
    ref = (wx.clone(), wy.clone())
    for rep in range(3):
        wx.fill_(5.0)
        wy.fill_(5.0)
        bm.bosmusic_demodulate(graph.h, spec, bm.BM_SURROGATE)
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(wx, 9.0), torch.nan_to_num(ref[0], 9.0))
        assert torch.equal(torch.nan_to_num(wy, 9.0), torch.nan_to_num(ref[1], 9.0))
    eager.close()
    graph.close()


def test_surrogate_requires_parameters_and_long_windows(bm, torch):
    d = bm.Demodulator(0, max_width=256, max_height=256)
    img = torch.from_numpy(wl.random_frame(128, 32, seed=1)).cuda()
    with pytest.raises(bm.BosmusicError) as ei:
        d.demodulate(img, 6, 32, "x", mode=bm.BM_SURROGATE)
    assert ei.value.status == bm.BM_E_UNSUPPORTED
    bm.bosmusic_surrogate_config(d.h, 1e-3, 1)
    with pytest.raises(bm.BosmusicError) as ei:
        d.demodulate(img, 4, 12, "x", mode=bm.BM_SURROGATE)
    assert ei.value.status == bm.BM_E_UNSUPPORTED
    d.close()
