"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
closed form, an invariant, an independent library route or a brute-force
computation, chosen so that a plausible slip (a dropped term, a wrong sign or
index, a transposed operand, a reversed coefficient order, an off-by-one in
the window placement) fails at least one of them.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.signal

import oracle
import workloads as wl

RNG = np.random.default_rng(1234)


def wrap(d):
    return (np.asarray(d) + np.pi) % (2 * np.pi) - np.pi


# ---------------------------------------------------------------------------
# Single complex tone (Eq. 1 with constant phase slope; Eq. 5-8, 12, 15)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,N", [(2, 4), (3, 9), (4, 16), (5, 11), (6, 32), (7, 20), (8, 32), (8, 64)])
def test_single_tone_exact(L, N):
    """A noiseless tone A e^{j(w0 n + a)} is recovered exactly, for w0 of either sign.

    Eq. 8: the signal eigenvalue is M A^2 (here L A^2 with the 1/K scaling) and
    all others vanish; Eq. 15: omega = arg of the root on the unit circle.
    """
    for w0 in (-2.9, -1.1, -0.3, 0.05, 0.7, 1.9, 3.0):
        A = 1.7
        n = np.arange(N)
        win = A * np.exp(1j * (w0 * n + 0.4))
        om, info = oracle.demod_windows(win[None], L, details=True)
        assert abs(wrap(om[0] - w0)) < 1e-12
        lam = info["lam"][0]
        assert abs(lam[-1] - L * A * A) < 1e-12 * L * A * A
        assert np.max(np.abs(lam[:-1])) < 1e-12 * L * A * A


def test_tone_eigvector_is_steering_vector():
    """Eq. 6-8: the signal eigenvector is a(w0) = [1, e^{jw0}, ...]^T up to scale."""
    L, N, w0 = 6, 20, 0.83
    win = np.exp(1j * w0 * np.arange(N))
    R = oracle.fb_average(oracle.covariance(win, L))
    lam, V = np.linalg.eigh(R)
    u1 = V[:, -1]
    a = np.exp(1j * w0 * np.arange(L)) / math.sqrt(L)
    assert abs(abs(np.vdot(a, u1)) - 1.0) < 1e-12
    C, _ = oracle.noise_projector(R)
    # Eq. 9: the noise subspace is orthogonal to the steering vector
    assert np.linalg.norm(C @ a) < 1e-12


# ---------------------------------------------------------------------------
# Analytic step (Sec. 2 "bandpass filtering", reading R1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("W", [64, 96, 256, 243, 100])
def test_analytic_of_on_grid_cosine_is_exponential(W):
    """a + b cos(2 pi k x / W + t) maps to b e^{j(2 pi k x/W + t)} exactly."""
    x = np.arange(W)
    for k in (1, 5, W // 4, W // 2 - 1 if W % 2 == 0 else (W - 1) // 2):
        th = 0.37
        line = 0.5 + 0.4 * np.cos(2 * np.pi * k * x / W + th)
        g = oracle.analytic_signal(line)
        exp = 0.4 * np.exp(1j * (2 * np.pi * k * x / W + th))
        assert np.max(np.abs(g - exp)) < 1e-12


@pytest.mark.parametrize("W", [64, 128, 250])
def test_analytic_matches_scipy_hilbert_route(W):
    """scipy's analytic signal keeps DC and Nyquist (weights 1); ours drops both.

    So hilbert(x) - gamma = mean(x) + (X[W/2]/W) (-1)^n for even W, mean(x) for odd W.
    """
    x = RNG.standard_normal(W)
    g = oracle.analytic_signal(x)
    h = scipy.signal.hilbert(x)
    diff = h - g
    X = np.fft.fft(x)
    exp = np.full(W, x.mean(), dtype=complex)
    if W % 2 == 0:
        exp = exp + X[W // 2] / W * (-1.0) ** np.arange(W)
    assert np.max(np.abs(diff - exp)) < 1e-12


def test_real_tone_frame_gives_constant_omega():
    """Noiseless cfg1-shaped frame with the erf term removed: omega_x = pi/4 exactly."""
    W = H = 64
    x = np.arange(W)[None, :]
    y = np.arange(H)[:, None]
    img = 0.5 + 0.4 * np.cos(2 * np.pi * x / 8 + 0.3 * y)
    wx, wy = oracle.demodulate(img, 4, 16, "x")
    v = np.isfinite(wx)
    assert v.sum() == H * (W - 16 + 1)
    assert np.max(np.abs(wx[v] - np.pi / 4)) < 1e-12


# ---------------------------------------------------------------------------
# 2-D linear phase fringe and integration (P-c)
# ---------------------------------------------------------------------------
def test_linear_phase_fringe_and_integration():
    W, H = 96, 72
    kx, ky = 11, 7
    wx0, wy0 = 2 * np.pi * kx / W, 2 * np.pi * ky / H
    x = np.arange(W)[None, :]
    y = np.arange(H)[:, None]
    img = 0.5 + 0.4 * np.cos(wx0 * x + wy0 * y + 0.9)
    L, N = 5, 14
    wx, wy = oracle.demodulate(img, L, N, "xy")
    assert np.nanmax(np.abs(wx - wx0)) < 1e-12
    assert np.nanmax(np.abs(wy - wy0)) < 1e-12
    phi = oracle.integrate(wx, wy, N, N)
    x0, x1 = oracle.valid_range(W, N)
    y0, y1 = oracle.valid_range(H, N)
    ref = wx0 * (x - x0) + wy0 * (y - y0)
    inside = np.zeros((H, W), bool)
    inside[y0:y1 + 1, x0:x1 + 1] = True
    assert np.all(np.isnan(phi[~inside]))
    assert np.max(np.abs(phi[inside] - np.broadcast_to(ref, (H, W))[inside])) < 1e-9
    # carriers equal to the true slopes leave a flat phase
    phi0 = oracle.integrate(wx, wy, N, N, carrier_x=wx0, carrier_y=wy0)
    assert np.nanmax(np.abs(phi0)) < 1e-9


def test_integration_quadratic_phase_exact():
    """Trapezoid integration of a linear frequency ramp is exact (quadratic phase)."""
    H, W, N = 20, 50, 8
    x = np.arange(W, dtype=float)[None, :]
    y = np.arange(H, dtype=float)[:, None]
    c, d = 0.003, -0.002
    wx = np.broadcast_to(0.5 + 2 * c * x, (H, W)).copy()
    wy = np.broadcast_to(0.2 + 2 * d * y, (H, W)).copy()
    phi = oracle.integrate(wx, wy, N, N)
    x0, _ = oracle.valid_range(W, N)
    y0, _ = oracle.valid_range(H, N)
    fx = lambda t: 0.5 * t + c * t * t
    fy = lambda t: 0.2 * t + d * t * t
    ref = (fx(x) - fx(x0)) + (fy(y) - fy(y0))
    m = np.isfinite(phi)
    assert np.max(np.abs(phi[m] - np.broadcast_to(ref, (H, W))[m])) < 1e-12


def test_integration_mixed_quadratic_phase_exact():
    """phi = a x^2 + b x y + g y^2 has frequencies linear along every path the
    integration takes, so the trapezoid rule recovers phi - phi(anchor) exactly;
    the b x y term makes the result depend on which column anchors the rows."""
    H, W, Nx, Ny = 24, 40, 6, 10
    a, b, g = 0.002, 0.003, -0.001
    x = np.arange(W, dtype=float)[None, :]
    y = np.arange(H, dtype=float)[:, None]
    wx = np.broadcast_to(2 * a * x + b * y, (H, W)).copy()
    wy = np.broadcast_to(b * x + 2 * g * y, (H, W)).copy()
    phi = oracle.integrate(wx, wy, Nx, Ny)
    x0, _ = oracle.valid_range(W, Nx)
    y0, _ = oracle.valid_range(H, Ny)
    f = lambda xx, yy: a * xx * xx + b * xx * yy + g * yy * yy
    ref = np.broadcast_to(f(x, y) - f(x0, y0), (H, W))
    m = np.isfinite(phi)
    assert m.sum() == (H - Ny + 1) * (W - Nx + 1)
    assert np.max(np.abs(phi[m] - ref[m])) < 1e-12


def test_integration_without_omega_y_rows_start_at_zero():
    H, W, N = 6, 30, 10
    wx = np.full((H, W), 0.25)
    phi = oracle.integrate(wx, None, N, 0)
    x0, x1 = oracle.valid_range(W, N)
    assert np.all(phi[:, x0] == 0)
    assert np.allclose(phi[:, x1], 0.25 * (x1 - x0))
    assert np.all(np.isnan(phi[:, :x0])) and np.all(np.isnan(phi[:, x1 + 1:]))


# ---------------------------------------------------------------------------
# Quadratic phase (chirp): omega equals the phase derivative at the window
# centre x - 1/2 (pins the window placement of reading R2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,N", [(3, 9), (4, 16), (5, 11), (6, 32), (8, 32)])
@pytest.mark.parametrize("fb", [True, False])
def test_chirp_omega_is_derivative_at_window_centre(L, N, fb):
    W = 128
    m = np.arange(W)
    for c in (5e-4, 5e-3, 2e-2):
        g = np.exp(1j * (0.6 * m + c * m * m + 0.2))
        om = oracle.demod_lines(g[None], L, N, fb=fb)[0]
        lo, hi = oracle.valid_range(W, N)
        xs = np.arange(lo, hi + 1)
        centre = xs - N // 2 + (N - 1) / 2
        assert np.max(np.abs(wrap(om[lo:hi + 1] - (0.6 + 2 * c * centre)))) < 1e-11
        assert np.all(np.isnan(om[:lo])) and np.all(np.isnan(om[hi + 1:]))


# ---------------------------------------------------------------------------
# Coefficients against the quadratic form, roots against brute force (P-f)
# ---------------------------------------------------------------------------
def _noisy_windows(M, N, snr_db, seed, w0=0.9):
    rng = np.random.default_rng(seed)
    n = np.arange(N)
    s = math.sqrt(10 ** (-snr_db / 10) / 2)
    ph = rng.uniform(0, 2 * np.pi, M)[:, None]
    return np.exp(1j * (w0 * n[None, :] + ph)) + s * (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N)))


@pytest.mark.parametrize("L", [2, 3, 4, 6, 8])
def test_coefficients_equal_quadratic_form_on_unit_circle(L):
    """sum_k c_k z^k equals a(z)^H C a(z) for |z| = 1 (Eq. 12 expanded)."""
    win = _noisy_windows(20, 3 * L, 5.0, L)
    R = oracle.fb_average(oracle.covariance(win, L))
    C, _ = oracle.noise_projector(R)
    coef = oracle.poly_coeffs(C)            # highest power first
    for th in RNG.uniform(-np.pi, np.pi, 7):
        z = np.exp(1j * th)
        a = z ** np.arange(L)
        quad = np.einsum("i,mij,j->m", a.conj(), C, a)
        poly = np.polyval(coef.T, z) / z ** (L - 1)
        assert np.max(np.abs(poly - quad)) < 1e-12
        assert np.max(np.abs(quad.imag)) < 1e-12 and np.min(quad.real) > -1e-12


@pytest.mark.parametrize("L,N,snr", [(2, 4, 10.0), (3, 6, 5.0), (4, 8, 0.0), (4, 8, 20.0)])
def test_roots_and_selection_match_mpmath_brute_force(L, N, snr):
    """50-digit roots of the same coefficients give the same selected pair and omega."""
    win = _noisy_windows(12, N, snr, 7 + L)
    om, info = oracle.demod_windows(win, L, details=True)
    mpmath.mp.dps = 50
    for m in range(win.shape[0]):
        coef = [mpmath.mpc(complex(c)) for c in info["coef"][m]]
        rts = np.array([complex(r) for r in mpmath.polyroots(coef, maxsteps=400, extraprec=200)])
        dist = np.abs(np.abs(rts) - 1)
        i = int(np.argmin(dist))
        mir = 1 / np.conj(rts[i])
        d = np.abs(rts - mir)
        d[i] = np.inf
        j = int(np.argmin(d))
        om_bf = np.angle(rts[i] + rts[j])
        assert abs(wrap(om[m] - om_bf)) < 1e-10
        # the brute-force roots are the oracle's roots (as multisets)
        got = info["roots"][m]
        for r in rts:
            assert np.min(np.abs(got - r)) < 1e-6 * max(1.0, abs(r))


def test_roots_come_in_conjugate_reciprocal_pairs():
    win = _noisy_windows(50, 24, 3.0, 99)
    om, info = oracle.demod_windows(win, 6, details=True)
    for rts in info["roots"]:
        for r in rts:
            assert np.min(np.abs(rts - 1 / np.conj(r))) < 1e-6 * max(1, abs(r))


def test_selection_rule_on_known_root_sets():
    """Polynomials built from prescribed roots: the pair nearest the circle wins."""
    pairs = [(0.5, 0.3), (0.93, 1.1), (0.7, -2.0), (0.2, 2.5)]
    rts = []
    for r, th in pairs:
        rts += [r * np.exp(1j * th), np.exp(1j * th) / r]
    sel = oracle.select_root_pair(np.array(rts)[None])
    assert abs(sel["omega"][0] - 1.1) < 1e-12
    assert abs(abs(sel["zsel"][0]) - 0.93) < 1e-12
    # both members of a near-double pair pushed outside the circle by rounding:
    # the pair is still the selected one
    rts2 = [0.35 * np.exp(0.3j), np.exp(0.3j) / 0.35,
            1.0000001 * np.exp(0.8j), 1.0000003 * np.exp(0.8j)]
    sel2 = oracle.select_root_pair(np.array(rts2)[None])
    assert abs(sel2["omega"][0] - 0.8) < 1e-12


def test_null_spectrum_minimum_matches_selected_root():
    """Grid search of a(t)^H C a(t) finds its minimum where the selected root predicts.

    Near the pair r e^{jt_s}, e^{jt_s}/r the null spectrum is
    (1 + r^2 - 2 r cos(t - t_s)) G(t) / r, G the distance product over the other
    roots, so its minimum sits at t_s - (1-r)^2 G'(t_s) / (2 r G(t_s)) to
    second order.
    """
    win = _noisy_windows(40, 32, 25.0, 5)
    L = 6
    om, info = oracle.demod_windows(win, L, details=True)
    C = info["C"]
    grid = np.linspace(0.6, 1.2, 2 ** 16 + 1)
    step = grid[1] - grid[0]
    A = np.exp(1j * np.outer(grid, np.arange(L)))             # (G, L)
    for m in range(win.shape[0]):
        f = np.real(np.einsum("gi,ij,gj->g", A.conj(), C[m], A))
        tmin = grid[np.argmin(f)]
        zs = info["zsel"][m]
        r = abs(zs)
        if r > 1:
            r = 1 / r
        ts = np.angle(zs)
        others = [z for z in info["roots"][m] if abs(z - info["zsel"][m]) > 1e-12 and abs(z - info["zmate"][m]) > 1e-12]
        e = np.exp(1j * ts)
        # d/dt log G at t_s
        dlogG = sum(np.real(1j * e * np.conj(e - z)) / abs(e - z) ** 2 for z in others)
        pred = ts - (1 - r) ** 2 * dlogG / (2 * r)
        assert abs(tmin - pred) <= 1.5 * step + 10 * (1 - r) ** 3


# ---------------------------------------------------------------------------
# Invariants (P-g) and statistics (Eq. 10, P-h)
# ---------------------------------------------------------------------------
def test_invariants_on_noisy_windows():
    L = 6
    win = _noisy_windows(200, 32, 2.0, 3)
    om, info = oracle.demod_windows(win, L, details=True)
    R = info["R"]
    J = np.eye(L)[::-1]
    assert np.allclose(R, np.swapaxes(R.conj(), -1, -2), atol=1e-14)          # Hermitian
    assert np.allclose(R, J @ R.conj() @ J, atol=1e-14)                        # centro-Hermitian
    C = info["C"]
    assert np.allclose(C @ C, C, atol=1e-12)
    assert np.allclose(np.trace(C, axis1=1, axis2=2), L - 1, atol=1e-12)
    lam, V = np.linalg.eigh(R)
    u1 = V[..., -1]
    assert np.allclose(np.einsum("mij,mj->mi", C, u1), 0, atol=1e-12)
    # selected root is a root of the polynomial
    coef = info["coef"]
    for m in range(20):
        z = info["zsel"][m]
        val = np.polyval(coef[m], z)
        scale = np.polyval(np.abs(coef[m]), abs(z))
        assert abs(val) < 1e-10 * scale


def test_fb_average_keeps_single_tone():
    """J conj(a(w)) = e^{-jw(L-1)} a(w): FB averaging leaves a tone covariance unchanged."""
    L, N, w0 = 7, 21, 1.3
    win = 0.8 * np.exp(1j * w0 * np.arange(N))
    R = oracle.covariance(win, L)
    assert np.allclose(oracle.fb_average(R), R, atol=1e-14)
    a = np.exp(1j * w0 * np.arange(L))
    assert np.allclose(R, 0.64 * np.outer(a, a.conj()), atol=1e-14)


def test_noise_eigenvalues_statistics():
    """Eq. 10: with many snapshots the noise eigenvalues approach sigma^2 and
    the signal one L A^2 + sigma^2."""
    rng = np.random.default_rng(8)
    L, N = 4, 40000
    sig2 = 0.3
    noise = math.sqrt(sig2 / 2) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    tone = np.exp(1j * 0.7 * np.arange(N))
    R = oracle.covariance(tone + noise, L)
    lam = np.linalg.eigvalsh(R)
    assert np.all(np.abs(lam[:-1] - sig2) < 0.05 * sig2)
    assert abs(lam[-1] - (L + sig2)) < 0.02 * (L + sig2)
    lam0 = np.linalg.eigvalsh(oracle.covariance(noise, L))
    assert np.all(np.abs(lam0 - sig2) < 0.05 * sig2)


def test_zero_window_is_nan_and_border_is_nan():
    W, H = 40, 3
    img = np.zeros((H, W))
    wx, _ = oracle.demodulate(img, 4, 12, "x")
    assert np.all(np.isnan(wx))
    g = np.zeros((2, 10), complex)
    assert np.all(np.isnan(oracle.demod_lines(g, 3, 20)))     # window longer than the line


def test_cfg1_accuracy_against_truth():
    """cfg1 (20 dB): the local frequency sits near the true pi/4 (RMS ~ 6e-3)."""
    f = wl.cfg1()
    wx, _ = oracle.demodulate(f.data[::8], f.L, f.N, "x")
    v = np.isfinite(wx)
    rms = math.sqrt(np.mean((wx[v] - math.pi / 4) ** 2))
    assert 1e-3 < rms < 2e-2


def test_erf_phase_derivative_agreement():
    """Noiseless erf phase: omega tracks the analytic derivative away from the
    frame edges (approximate: window averaging of the curvature)."""
    W, H = 64, 256
    y = np.arange(H, dtype=float)[:, None]
    x = np.arange(W, dtype=float)[None, :]
    w = 40.0
    img = 0.5 + 0.4 * np.cos(2 * np.pi * (x / 8 + y / 10) + 3 * __import__("scipy").special.erf((y - 128) / w))
    _, wy = oracle.demodulate(img, 6, 24, "y")
    yy = np.arange(H, dtype=float)
    c = yy - 0.5
    truth = 2 * np.pi / 10 + 3 * 2 / math.sqrt(math.pi) * np.exp(-((c - 128) / w) ** 2) / w
    # third derivative bound of the erf phase times (N/2)^2/6, plus leakage allowance
    rows = slice(48, H - 48)
    err = np.abs(wy[rows, 20] - truth[rows])
    assert np.nanmax(err) < 3e-3


def two_tone_windows(L, ratio, w1=0.4):
    """Windows of two complex tones whose steering vectors are orthogonal over L samples
    (frequency spacing 2 pi / L) and whose cross terms cancel over the K = 4L sub-snapshots
    (K a multiple of L), so that R = P1 a1 a1^H + P2 a2 a2^H exactly, with eigenvalues
    L P1, L P2 and 0 (Eq. 8 for two sources), and FB averaging leaves it unchanged."""
    N = 5 * L - 1
    n = np.arange(N)
    w2 = w1 + 2 * np.pi / L
    win = np.sqrt(ratio) * np.exp(1j * (w1 * n + 0.3)) + np.exp(1j * (w2 * n - 1.1))
    return win[None], w1


@pytest.mark.parametrize("L", [2, 4, 6, 8])
def test_degenerate_signal_subspace_of_two_equal_tones(L):
    """Two tones of equal power: lambda_1 = lambda_2 = L, the one-dimensional signal
    subspace of Eq. 6-11 is not determined, omega is NaN (reading R10).  A power ratio of
    1.001 separates them and the stronger tone's frequency comes out exactly (its steering
    vector is then the top eigenvector); a ratio inside the bound is still degenerate."""
    win, w1 = two_tone_windows(L, 1.0)
    om, info = oracle.demod_windows(win, L, details=True)
    lam = info["lam"][0]
    assert np.allclose(lam[-2:], [L, L], rtol=0, atol=1e-10) and np.all(np.abs(lam[:-2]) < 1e-10)
    assert info["degenerate"][0] and np.isnan(om[0])
    win, w1 = two_tone_windows(L, 1.001)
    om, info = oracle.demod_windows(win, L, details=True)
    assert not info["degenerate"][0]
    assert abs(om[0] - w1) < 1e-9
    win, _ = two_tone_windows(L, 1.0 + 0.5 * oracle.DEGENERATE_REL)
    assert np.isnan(oracle.demod_windows(win, L)[0])
    win, _ = two_tone_windows(L, 1.0 + 3.0 * oracle.DEGENERATE_REL)
    assert np.isfinite(oracle.demod_windows(win, L)[0])
