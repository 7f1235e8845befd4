"""The allocation-free integration entry point against bosmusic_integrate, through
the C ABI: the same kernels, so the phase maps must be identical bit for bit, on two
calls in a row (the second smaller, on the same fixed scratch) and with omega_y absent."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def maps(torch, W, H, N, seed):
    img = wl.random_frame(W, H, seed=seed, snr_db=10.0)
    ox, oy = oracle.demodulate(img, 6, N, "xy")
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    return to(ox), to(oy)


def test_noalloc_integrate_matches_handle_integrate(bm, torch):
    d = bm.Demodulator(0, max_width=1024, max_height=1024)
    for (W, H, N, seed, with_y) in [(700, 300, 24, 3, True), (260, 90, 16, 4, True), (300, 40, 20, 5, False)]:
        wx, wy = maps(torch, W, H, N, seed)
        if not with_y:
            wy = None
        ref = torch.full((H, W), 7.0, dtype=torch.float64, device="cuda")
        got = torch.full((H, W), -7.0, dtype=torch.float64, device="cuda")
        bm.bosmusic_integrate(d.h, wx, wy, N, N, 0.1, 0.05, ref)
        bm.bosmusic_integrate_noalloc(wx, wy, N, N, 0.1, 0.05, got)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(np.isnan(a), np.isnan(b))
        assert np.array_equal(a[np.isfinite(a)], b[np.isfinite(b)]), (W, H)
        assert np.isfinite(b).sum() == (W - N + 1) * ((H - N + 1) if with_y else H)
        # and against the oracle's own integration of the same maps
        ph = oracle.integrate(wx.cpu().numpy(), None if wy is None else wy.cpu().numpy(), N, N, 0.1, 0.05)
        m = np.isfinite(ph)
        assert np.array_equal(m, np.isfinite(b)) and np.max(np.abs(b[m] - ph[m])) < 1e-9
    d.close()


def test_noalloc_refuses_heights_beyond_its_scratch(bm, torch):
    L = bm.lib()
    buf = torch.zeros(16, device="cuda")
    st = L.bosmusic_integrate_noalloc(ctypes.c_void_p(buf.data_ptr()), None, 4, 65537, 2, 2, 0.0, 0.0,
                                      ctypes.c_void_p(buf.data_ptr()), None)
    assert st == bm.BM_E_INVALID_ARG
    assert "scratch" in bm.bosmusic_last_error(None)
    st = L.bosmusic_integrate_noalloc(None, None, 4, 4, 2, 2, 0.0, 0.0, None, None)
    assert st == bm.BM_E_INVALID_ARG
