"""Window size against accuracy (the paper's window-size study, Sec. 4, Table 1): a small
window is noise-limited and a large one breaks the local linear-phase model, so the error of
the estimated frequency is U-shaped in the window length.  The oracle must show that trade-off
on a field whose frequency varies smoothly (a linear chirp alone would not: the window centre
estimate is exact for it, pinned elsewhere)."""
import numpy as np

import oracle
import workloads as wl


def _rms(est, truth):
    v = np.isfinite(est)
    d = (est[v] - truth[v] + np.pi) % (2 * np.pi) - np.pi
    return float(np.sqrt(np.mean(d * d)))


def test_frequency_error_is_u_shaped_in_the_window_length():
    f = wl.sweep_frame(96, 96, snr_db=10.0, seed=3)
    ys, xs = np.mgrid[0:96, 0:96].astype(np.float64)
    err = {}
    for N in (4, 12, 48):
        L = max(2, min(8, N // 4))
        ox, oy = oracle.demodulate(f.data, L, N, "xy")
        c = -(N // 2) + (N - 1) / 2            # window centre relative to the pixel
        err[N] = (_rms(ox, f.truth_wx(ys, xs + c)), _rms(oy, f.truth_wy(ys + c, xs)))
    for d in (0, 1):
        assert err[12][d] < 0.7 * err[4][d], err
        assert err[12][d] < 0.5 * err[48][d], err


def test_block_window_error_is_u_shaped_in_the_block_size():
    """The same trade-off for the paper's own (2L+1) x (2L+1) block window (Sec. 3), over the
    sizes of its window table (Sec. 4, Table 1: L = 1 .. 8): 5 x 5 is noise-limited, 17 x 17
    model-limited, 11 x 11 (the paper's simulation choice, L = 5) near the minimum.  At 0 dB
    on a 160 x 160 field the oracle gives 0.18 / 0.037 / 0.10 rad/px (x) for 5 / 11 / 17."""
    f = wl.sweep_frame(96, 96, snr_db=0.0, seed=11)
    ys, xs = np.mgrid[0:96, 0:96].astype(np.float64)
    err = {}
    for M in (5, 11, 17):
        ox, oy = oracle.demodulate_block(f.data, M)
        c = -(M // 2) + (M - 1) / 2
        err[M] = (_rms(ox, f.truth_wx(ys, xs + c)), _rms(oy, f.truth_wy(ys + c, xs)))
    for d in (0, 1):
        assert err[11][d] < 0.5 * err[5][d], err
        assert err[11][d] < 0.6 * err[17][d], err
