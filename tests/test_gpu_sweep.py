"""Window-size sweep on the GPU (the paper's window-size study, Sec. 4, Table 1): the paper's
simulation shape (512 x 512 at 0 dB), a field whose frequency varies smoothly, line windows
N = 4 .. 64 and block windows 2 .. 8, then the paper's odd sizes to 17 x 17.  The frequency and the integrated phase are compared with
the field's own; the frequency error must be U-shaped in N (noise-limited small windows, model-
limited large ones).  The table is printed for the record."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _rms(d):
    d = d[np.isfinite(d)]
    d = (d + np.pi) % (2 * np.pi) - np.pi
    return float(np.sqrt(np.mean(d * d)))


def test_window_size_sweep_is_u_shaped(bm, torch):
    W = H = 512
    f = wl.sweep_frame(W, H, snr_db=0.0, seed=11, dtype=np.float32)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    d = bm.Demodulator(0, max_width=W, max_height=H)
    img = torch.from_numpy(f.data).to("cuda")
    rows = []
    for N in (4, 6, 8, 12, 16, 24, 32, 48, 64):
        L = max(2, min(8, N // 4))
        wx, wy = d.demodulate(img, L, N, "xy")
        phi = d.integrate(wx, wy, N, N)
        torch.cuda.synchronize()
        c = -(N // 2) + (N - 1) / 2
        ex = _rms(wx.cpu().numpy() - f.truth_wx(ys, xs + c))
        ey = _rms(wy.cpu().numpy() - f.truth_wy(ys + c, xs))
        p = phi.cpu().numpy()
        # phase relative to the anchor pixel (first valid row and column)
        a = (N // 2, N // 2)
        true = f.meta["phase"](ys + c, xs + c)
        ep = p - (true - true[a])
        ep = ep[np.isfinite(ep)]
        rows.append((N, L, ex, ey, float(np.sqrt(np.mean((ep - ep.mean()) ** 2)))))
    for M in list(range(2, 9)) + [9, 11, 13, 15, 17]:
        bx, by = d.demodulate(img, M, M, "xy", block=True)
        torch.cuda.synchronize()
        c = -(M // 2) + (M - 1) / 2
        rows.append((f"block {M}", M, _rms(bx.cpu().numpy() - f.truth_wx(ys, xs + c)),
                     _rms(by.cpu().numpy() - f.truth_wy(ys + c, xs)), float("nan")))
    d.close()
    print("\n  window      L   rms d omega_x   rms d omega_y   rms d phi (mean removed)")
    for r in rows:
        print(f"  {str(r[0]):9s} {r[1]:3d}   {r[2]:.4f}          {r[3]:.4f}          {r[4]:.4f}")
    line = [r for r in rows if isinstance(r[0], int)]
    block = [r for r in rows if not isinstance(r[0], int)]
    for group in (line, block):
        for k in (2, 3):
            e = [r[k] for r in group]
            i = int(np.argmin(e))
            assert 0 < i < len(e) - 1, e
            assert e[0] > 1.3 * e[i] and e[-1] > 1.3 * e[i], e
