"""Pins of the block-mode oracle (the paper's M x M moving window, Sec. 3)."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


@pytest.mark.parametrize("M", [2, 3, 5, 7, 8])
def test_plane_waves_are_exact_in_both_directions(M):
    """A complex plane wave A e^{j(alpha + wx x + wy y)} (Eq. 2-3 with a linear phase)
    gives omega_y = arg(z_y) and omega_x = -arg(z_x) exactly (Eq. 15)."""
    for (wx, wy) in [(0.7, -0.4), (-2.5, 1.9), (3.0, 0.05), (0.0, -3.1)]:
        g = wl.complex_tone(37, 29, wx, wy, alpha=1.1, amp=2.0)
        ox, oy = oracle.demodulate_block(g, M)
        v = np.isfinite(ox)
        assert v.sum() == (29 - M + 1) * (37 - M + 1)
        assert np.max(np.abs(ox[v] - wx)) < 1e-12
        assert np.max(np.abs(oy[v] - wy)) < 1e-12


def test_eigenvalues_of_a_noiseless_block():
    """Eq. 7-8: the signal autocorrelation is A^2 u1 u1^H, one eigenvalue M A^2, the others zero."""
    M, A = 7, 1.7
    g = wl.complex_tone(20, 20, 0.9, -0.6, amp=A)
    Ry, Rx = oracle.block_covariances(g, M)
    for R in (Ry[3, 4], Rx[3, 4]):
        lam = np.linalg.eigvalsh(R)
        assert abs(lam[-1] - M * A * A) < 1e-10
        assert np.max(np.abs(lam[:-1])) < 1e-10
    # Eq. 5: R_s[0, 1] = A^2 e^{-j omega_y}
    assert abs(Ry[3, 4][0, 1] - A * A * np.exp(-1j * -0.6)) < 1e-12


def test_real_fringe_on_the_dft_grid():
    """A real fringe a + b cos(2 pi k x / W + wy y + t): each row is on the DFT grid, so the
    row analytic signal is b e^{j(...)} exactly and both frequencies are exact."""
    W, H, k, wy = 64, 24, 9, 0.37
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    img = 0.5 + 0.4 * np.cos(2 * math.pi * k * x / W + wy * y + 0.2)
    ox, oy = oracle.demodulate_block(img, 5)
    v = np.isfinite(ox)
    assert np.max(np.abs(ox[v] - 2 * math.pi * k / W)) < 1e-11
    assert np.max(np.abs(oy[v] - wy)) < 1e-11


def test_block_placement_at_a_frequency_step():
    """Two plane-wave regions: a block wholly inside one region returns that region's
    frequencies, which pins the block's offset h = floor(M/2) and its extent."""
    W, H, M = 60, 20, 5
    h = M // 2
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    g = np.where(x < 30, np.exp(1j * (0.8 * x + 0.3 * y)), np.exp(1j * (-1.2 * x + 0.6 * y + 0.5)))
    ox, oy = oracle.demodulate_block(g, M)
    left = slice(h, 30 - M + h + 1)          # blocks [x-h, x-h+M) inside x < 30
    right = slice(30 + h, W - M + h + 1)
    rows = slice(h, H - M + h + 1)
    assert np.allclose(ox[rows, left], 0.8, atol=1e-11) and np.allclose(oy[rows, left], 0.3, atol=1e-11)
    assert np.allclose(ox[rows, right], -1.2, atol=1e-11) and np.allclose(oy[rows, right], 0.6, atol=1e-11)
    # the first straddling block is not exact
    assert abs(ox[5, 30 - M + h + 1] - 0.8) > 1e-6
    assert np.all(np.isnan(ox[:h])) and np.all(np.isnan(ox[:, W - M + h + 1:]))


def test_x_form_equals_y_form_of_the_transposed_field():
    """omega_x from E{Gamma^H Gamma} with -arg (Eq. 13, 15) is omega_y of the transposed
    block: B^T conj(B) = conj(B^H B) conjugates the roots."""
    g = wl.complex_tone(33, 27, 1.3, -0.2, snr_db=5.0, seed=4)
    ox, _ = oracle.demodulate_block(g, 6)
    _, oyt = oracle.demodulate_block(np.ascontiguousarray(g.T), 6)
    v = np.isfinite(ox)
    assert np.array_equal(v, np.isfinite(oyt.T))
    assert np.max(np.abs(ox[v] - oyt.T[v])) < 1e-9


def test_block_covariances_are_hermitian_and_psd():
    g = wl.complex_tone(20, 18, 0.5, 0.8, snr_db=0.0, seed=2)
    Ry, Rx = oracle.block_covariances(g, 4)
    for R in (Ry, Rx):
        assert np.allclose(R, np.conj(np.swapaxes(R, -1, -2)), atol=1e-14)
        assert np.min(np.linalg.eigvalsh(R)) > -1e-12
        # trace = mean energy per sample times M: sum |B|^2 / M
    B = g[2:6, 3:7]
    assert abs(np.trace(Ry[2, 3]) - np.sum(np.abs(B) ** 2) / 4) < 1e-12
    assert abs(np.trace(Rx[2, 3]) - np.sum(np.abs(B) ** 2) / 4) < 1e-12


def test_block_larger_than_frame_is_all_nan():
    g = wl.complex_tone(6, 5, 0.3, 0.3)
    ox, oy = oracle.demodulate_block(g, 7)
    assert np.all(np.isnan(ox)) and np.all(np.isnan(oy))


@pytest.mark.parametrize("M", [3, 5, 8])
def test_block_with_identical_snapshots_equals_line_mode(M):
    """When the field does not vary across the snapshots, every snapshot of the block is
    the same vector s, R = s s^H, and the block estimate must equal the line mode with a
    single sub-snapshot (L = N = M, K = 1) on that vector -- including its forward-backward
    averaging, which turns the rank-one s s^H into a rank-two matrix and moves omega."""
    rng = np.random.default_rng(M)
    f = rng.standard_normal(40) + 1j * rng.standard_normal(40)      # noise: no tone
    g_y = np.repeat(f[:, None], 19, axis=1)                          # constant along x
    _, oy = oracle.demodulate_block(g_y, M)
    line = oracle.demod_lines(f[None, :], M, M)[0]
    h = M // 2
    v = np.isfinite(oy[:, h])
    assert np.array_equal(v, np.isfinite(line))
    assert np.max(np.abs(oy[v, h] - line[v])) < 1e-9
    g_x = np.repeat(f[None, :], 17, axis=0)                          # constant along y
    ox, _ = oracle.demodulate_block(g_x, M)
    assert np.max(np.abs(ox[h, v] - line[v])) < 1e-9
    no_fb = oracle.demod_lines(f[None, :], M, M, fb=False)[0]
    assert np.max(np.abs(no_fb[v] - line[v])) > 1e-3                # the averaging matters here


def _wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


@pytest.mark.parametrize("M", [3, 6, 7])
def test_block_phase_of_a_plane_wave(M):
    """Eq. 15: for a linear phase alpha + wx x + wy y the block phase is that phase at the pixel."""
    W, H, wx, wy, a = 41, 30, 0.9, -0.35, 2.2
    g = wl.complex_tone(W, H, wx, wy, alpha=a, amp=1.5)
    ox, oy = oracle.demodulate_block(g, M)
    ph = oracle.block_phase(g, M, ox, oy)
    y, x = np.mgrid[0:H, 0:W]
    v = np.isfinite(ph)
    assert v.sum() == (H - M + 1) * (W - M + 1)
    assert np.max(np.abs(_wrap(ph - (a + wx * x + wy * y))[v])) < 1e-11


def test_block_phase_matches_integrated_phase_on_a_chirp():
    """A slowly varying frequency: the wrapped block phase and the trapezoid-integrated
    phase differ by a constant (the anchor's phase) up to the windowing error."""
    W, H, M = 80, 40, 5
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    phi = 0.6 * x + 1e-3 * x * x + 0.3 * y
    g = np.exp(1j * phi)
    ox, oy = oracle.demodulate_block(g, M)
    ph = oracle.block_phase(g, M, ox, oy)
    integ = oracle.integrate(ox, oy, M, M)
    v = np.isfinite(ph) & np.isfinite(integ)
    d = _wrap(ph[v] - integ[v])
    d0 = d[0]
    assert np.max(np.abs(_wrap(d - d0))) < 2e-3


def test_block_phase_with_given_frequencies_and_an_envelope():
    """With the true frequencies given, an amplitude envelope along x does not move the
    phase: mean(A e^{j phi} e^{-j(omega . d)}) = mean(A) e^{j phi(pixel)} with mean(A) > 0."""
    W, H, M, wx, wy, a = 50, 26, 5, 1.1, -0.5, -0.7
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    g = (1.0 + 0.5 * np.sin(0.3 * x)) * np.exp(1j * (a + wx * x + wy * y))
    ph = oracle.block_phase(g, M, np.full((H, W), wx), np.full((H, W), wy))
    v = np.isfinite(ph)
    assert v.sum() == (H - M + 1) * (W - M + 1)
    assert np.max(np.abs(_wrap(ph - (a + wx * x + wy * y))[v])) < 1e-11
