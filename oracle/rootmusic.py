"""Plain FP64 root-MUSIC local-frequency demodulation (test oracle).

TEST INFRASTRUCTURE ONLY -- never imported by the library.

What is computed, in the paper's order:

  * analytic fringe signal Gamma (Eq. 1) from a real frame, by the
    band-pass step of Sec. 2 (reading R1 below);
  * per pixel, a window of N samples along one direction (Sec. 3, moving
    window; reading R2);
  * the autocorrelation matrix R of the window's length-L sub-snapshots
    (Eq. 4, sample form; reading R3) and its forward-backward average (R4);
  * its eigen-decomposition: largest eigenvalue -> signal subspace u1, the
    other L-1 eigenvectors -> noise subspace Un (Eq. 6-11);
  * the root-MUSIC polynomial a(z)^H Un Un^H a(z) (Eq. 12), whose
    coefficients are the diagonal sums of C = Un Un^H;
  * its roots as companion-matrix eigenvalues (Sec. 3, rooting);
  * the root inside the unit circle closest to it, and its angle as the
    local frequency (Eq. 15; reading R5 for the pair form);
  * trapezoid integration of the frequency maps to phase (reading R6).

Readings of points the paper leaves open (each also listed in the design notes):

  R1  Gamma = IFFT(FFT(row) * H) along the window direction, H[0] = 0,
      H[k] = 2 for 0 < k < W/2, H[W/2] = 0 (even W), H[k] = 0 above; odd W
      keeps 0 < k <= (W-1)/2.  The carrier is kept, so omega is the total
      local fringe frequency.  Complex input is taken as Gamma directly.
  R2  The window for pixel x starts at s = x - floor(N/2) and holds
      Gamma[s .. s+N-1]; the pixel is valid iff 0 <= s and s+N <= W.
      Invalid (border) pixels are NaN, as the paper neglects borders.
  R3  R = (1/K) sum_k s_k s_k^H with s_k = Gamma[s+k .. s+k+L-1], k = 0..K-1,
      K = N-L+1.  "L" here is the covariance size (the paper's M).
  R4  R_fb = (R + J conj(R) J) / 2, J the exchange matrix.
  R5  Roots come in pairs (z, 1/conj(z)) sharing one angle, because the
      coefficients satisfy c_{-k} = conj(c_k).  The paper keeps the root
      inside the unit circle that is closest to it, i.e. the inner member of
      the pair nearest the circle.  In exact arithmetic that pair also holds
      the root with the smallest ||z|-1| over all roots (an inner root at
      radius r is nearer the circle than its partner at 1/r), and this second
      form is the one evaluated, because rounding can push both members of a
      near-double pair to the same side of the circle.  z_sel is that root,
      z_mate the other root nearest 1/conj(z_sel), and
      omega = arg(z_sel + z_mate), which equals arg(z_sel) (Eq. 15) in exact
      arithmetic and does not depend on how rounding splits the near-double
      signal root.  With column snapshots in both directions omega = +arg for
      x and for y.
  R6  phi is integrated with the trapezoid rule in FP64 on the window-centre
      grid, anchored (phi = 0) at the first valid column and, when an
      omega_y map is given, the first valid row: first down the anchor column
      with omega_y, then along every row with omega_x.  Optional carriers are
      subtracted from each sample.  NaN outside the valid region.
  R7  A window whose covariance is identically zero (or non-finite) has no
      signal subspace; its omega is NaN.
  R8  Block mode (the paper's own window, Sec. 3): the block of pixel (y, x)
      is the M x M patch Gamma[y-h .. y-h+M-1, x-h .. x-h+M-1], h = floor(M/2)
      (centred for odd M = 2L+1 in the paper's notation), valid iff it fits.
      Gamma is the row-wise analytic signal of R1 (the paper forms one complex
      fringe field for the block; the row-wise one-sided mask is the 2-D
      half-plane mask k_x > 0).  R_y = B B^H / M (the block's columns are the
      snapshots, Eq. 4) gives z_y and omega_y = arg(z_y); R_x = B^H B / M (the
      autocorrelation E{Gamma^H Gamma}) gives z_x and omega_x = -arg(z_x)
      (Eq. 15).  FB averaging (R4) and the pair form of R5 are applied as in
      the line mode.
  R9  Block phase: Eq. 15's alpha = angle(mean(Gamma_w e^{-j(omega_x x +
      omega_y y)})) with (x, y) measured from the pixel, i.e. the wrapped
      phase of the block's linear model at the pixel.
  R10 The split of Eq. 6-11 into a one-dimensional signal subspace and the
      noise subspace needs a largest eigenvalue that stands apart: when
      lambda_1 <= lambda_2 (1 + DEGENERATE_REL) the signal eigenvector is not
      determined (any unit vector of a two-dimensional eigenspace qualifies,
      e.g. for two tones of equal power), and omega is NaN.  The bound,
      1e-5, sits above the resolution of eigenvalues computed in FP32 (a few
      1e-7 of the trace) so that the GPU's decision agrees with this one.
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

# R10: relative gap below which the signal subspace counts as undetermined
DEGENERATE_REL = 1e-5


# ---------------------------------------------------------------------------
# a1: analytic fringe signal (Sec. 2, Eq. 1; reading R1)
# ---------------------------------------------------------------------------
def analytic_mask(W: int) -> np.ndarray:
    """One-sided spectral mask H of reading R1 (length W, float64)."""
    H = np.zeros(W)
    if W % 2 == 0:
        H[1:W // 2] = 2.0
    else:
        H[1:(W - 1) // 2 + 1] = 2.0
    return H


def analytic_signal(lines: np.ndarray) -> np.ndarray:
    """Complex analytic signal of each real line (last axis), FP64.

    Paper Sec. 2: the complex fringe signal of Eq. 1 is obtained by bandpass
    filtering; here the filter is the exact one-sided DFT mask of reading R1.
    """
    x = np.asarray(lines, dtype=np.float64)
    W = x.shape[-1]
    X = np.fft.fft(x, axis=-1)
    return np.fft.ifft(X * analytic_mask(W), axis=-1)


# ---------------------------------------------------------------------------
# a2..a5: window, covariance, FB average, eigen-split (Eq. 2-11)
# ---------------------------------------------------------------------------
def valid_range(W: int, N: int):
    """First and last valid pixel index along a line of length W (reading R2)."""
    lo = N // 2
    hi = W - N + N // 2
    return lo, hi


def covariance(win: np.ndarray, L: int) -> np.ndarray:
    """Sample autocorrelation of the sub-snapshots of each window (Eq. 4; R3).

    win: (..., N) complex.  Returns (..., L, L) Hermitian.
    """
    N = win.shape[-1]
    K = N - L + 1
    S = sliding_window_view(win, L, axis=-1)          # (..., K, L): S[..., k, i] = win[k+i]
    assert S.shape[-2] == K
    return np.einsum("...ki,...kj->...ij", S, S.conj()) / K


def fb_average(R: np.ndarray) -> np.ndarray:
    """Forward-backward average (R + J conj(R) J)/2 (reading R4)."""
    RJ = R[..., ::-1, ::-1].conj()
    return 0.5 * (R + RJ)


def noise_projector(R: np.ndarray):
    """Signal/noise split of Eq. 6-11 for a one-dimensional signal subspace.

    Returns (C, lam) with C = Un Un^H (the projector that appears in Eq. 12)
    built from the L-1 eigenvectors of the smallest eigenvalues, and lam the
    eigenvalues in ascending order.  The paper computes the eigenvectors
    through an SVD; any Hermitian eigensolver gives the same subspaces.
    """
    lam, V = np.linalg.eigh(R)
    Un = V[..., :, :-1]
    C = Un @ np.swapaxes(Un.conj(), -1, -2)
    return C, lam


def degenerate(lam: np.ndarray) -> np.ndarray:
    """True where the two largest eigenvalues (ascending lam) are too close for
    a one-dimensional signal subspace (Eq. 6-11; reading R10)."""
    return lam[..., -1] <= lam[..., -2] * (1.0 + DEGENERATE_REL)


def poly_coeffs(C: np.ndarray) -> np.ndarray:
    """Coefficients of the root-MUSIC polynomial of Eq. 12.

    With a(z) = [1, z, ..., z^{L-1}]^T, a(z)^H C a(z) on the unit circle equals
    sum_{i,j} C[i,j] z^{j-i}, so the coefficient of z^k is the k-th diagonal
    sum c_k = sum_i C[i, i+k], k = -(L-1) .. L-1.  Returned highest power
    first, i.e. [c_{L-1}, ..., c_0, ..., c_{-(L-1)}], the polynomial being
    z^{L-1} * sum_k c_k z^k of degree 2L-2.
    """
    L = C.shape[-1]
    cols = [np.trace(C, offset=k, axis1=-2, axis2=-1) for k in range(L - 1, -L, -1)]
    return np.stack(cols, axis=-1)


def poly_roots(coef: np.ndarray) -> np.ndarray:
    """All roots as eigenvalues of the companion matrix (Sec. 3, rooting).

    coef: (..., n+1) highest power first.  Batched form of numpy.roots:
    companion matrix with first row -coef[1:]/coef[0] and ones on the
    sub-diagonal.  A window whose leading coefficient is exactly zero is
    handed to numpy.roots, which strips it, and padded with +inf roots.
    """
    coef = np.asarray(coef, dtype=np.complex128)
    shp = coef.shape[:-1]
    n = coef.shape[-1] - 1
    c = coef.reshape(-1, n + 1)
    out = np.full((c.shape[0], n), np.inf + 0j)
    good = (c[:, 0] != 0) & np.all(np.isfinite(c), axis=1)
    if np.any(good):
        cg = c[good]
        comp = np.zeros((cg.shape[0], n, n), dtype=np.complex128)
        comp[:, 0, :] = -cg[:, 1:] / cg[:, :1]
        idx = np.arange(n - 1)
        comp[:, idx + 1, idx] = 1.0
        out[good] = np.linalg.eigvals(comp)
    for i in np.nonzero(~good)[0]:
        if np.all(np.isfinite(c[i])) and np.any(c[i] != 0):
            r = np.roots(c[i])
            out[i, :r.size] = r
    return out.reshape(shp + (n,))


def select_root_pair(roots: np.ndarray):
    """Root selection of Sec. 3 and angle of Eq. 15 (reading R5).

    roots: (M, n) complex.  Returns dict with
      omega    angle of z_sel + z_mate (the parity output),
      omega1   angle of z_sel alone (the paper-literal output),
      zsel, zmate,
      margin   distance to the circle of the nearest root outside the
               selected pair minus that of z_sel (small values mark windows
               whose selection is ill-posed).
    """
    r = np.asarray(roots)
    M, n = r.shape
    a = np.abs(r)
    dist = np.abs(a - 1.0)
    sel = np.argmin(dist, axis=1)
    rows = np.arange(M)
    zsel = r[rows, sel]
    with np.errstate(divide="ignore", invalid="ignore"):
        mirror = 1.0 / np.conj(zsel)
    d = np.abs(r - mirror[:, None])
    d[rows, sel] = np.inf
    mate = np.argmin(d, axis=1)
    zmate = r[rows, mate]
    rest = dist.copy()
    rest[rows, sel] = np.inf
    rest[rows, mate] = np.inf
    nxt = np.min(rest, axis=1)
    return {
        "omega": np.angle(zsel + zmate),
        "omega1": np.angle(zsel),
        "zsel": zsel,
        "zmate": zmate,
        "margin": nxt - dist[rows, sel],
    }


def demod_windows(win: np.ndarray, L: int, fb: bool = True, details: bool = False):
    """Steps a3..a8 for a batch of windows (M, N) complex -> omega (M,).

    Windows whose covariance is identically zero or non-finite give NaN (R7),
    and so do windows whose signal subspace is not determined (R10).
    """
    win = np.asarray(win, dtype=np.complex128)
    M = win.shape[0]
    R = covariance(win, L)
    if fb:
        R = fb_average(R)
    tr = np.real(np.trace(R, axis1=-2, axis2=-1))
    ok = np.isfinite(tr) & (tr > 0)
    omega = np.full(M, np.nan)
    info = {"ok": ok}
    if np.any(ok):
        C, lam = noise_projector(R[ok])
        coef = poly_coeffs(C)
        rts = poly_roots(coef)
        sel = select_root_pair(rts)
        deg = degenerate(lam)
        omega[ok] = np.where(deg, np.nan, sel["omega"])
        if details:
            info.update(R=R, C=C, lam=lam, coef=coef, roots=rts, degenerate=deg, **sel)
    if details:
        return omega, info
    return omega


def demod_lines(gamma: np.ndarray, L: int, N: int, fb: bool = True, chunk: int = 32768):
    """omega along the last axis of a (H, W) complex array; NaN at borders."""
    gamma = np.asarray(gamma, dtype=np.complex128)
    H, W = gamma.shape
    out = np.full((H, W), np.nan)
    lo, hi = valid_range(W, N)
    if hi < lo:
        return out
    nv = hi - lo + 1
    wins = sliding_window_view(gamma, N, axis=1)[:, :nv, :]   # window for pixel lo+i starts at i
    flat = wins.reshape(H * nv, N)
    res = np.empty(H * nv)
    for s in range(0, H * nv, chunk):
        res[s:s + chunk] = demod_windows(flat[s:s + chunk], L, fb=fb)
    out[:, lo:hi + 1] = res.reshape(H, nv)
    return out


def to_complex_field(frame: np.ndarray, axis: int) -> np.ndarray:
    """Decode the stored frame to FP64 and form Gamma along ``axis`` (a0, a1)."""
    f = np.asarray(frame)
    if np.iscomplexobj(f):
        return f.astype(np.complex128)
    f = f.astype(np.float64)
    if axis == 1:
        return analytic_signal(f)
    return analytic_signal(f.T).T


def demodulate(frame: np.ndarray, L: int, N: int, dirs: str = "xy", fb: bool = True):
    """Whole-frame demodulation: returns (omega_x or None, omega_y or None)."""
    wx = wy = None
    if "x" in dirs:
        wx = demod_lines(to_complex_field(frame, 1), L, N, fb=fb)
    if "y" in dirs:
        g = to_complex_field(frame, 0)
        wy = demod_lines(g.T, L, N, fb=fb).T
    return wx, wy


# ---------------------------------------------------------------------------
# Block mode: the paper's M x M moving window (Sec. 3, Eq. 4-15; reading R8)
# ---------------------------------------------------------------------------
def block_covariances(gamma: np.ndarray, M: int):
    """R_y = B B^H / M and R_x = B^H B / M for every block that fits.

    gamma: (H, W) complex.  Returns (R_y, R_x), each (H-M+1, W-M+1, M, M);
    entry [a, b] belongs to the block whose top-left sample is gamma[a, b],
    i.e. to pixel (a + M//2, b + M//2).
    """
    B = sliding_window_view(gamma, (M, M))            # B[a, b, i, j] = gamma[a+i, b+j]
    Ry = np.einsum("...ij,...kj->...ik", B, B.conj()) / M
    Rx = np.einsum("...ri,...rk->...ik", B.conj(), B) / M
    return Ry, Rx


def _omega_from_cov(R: np.ndarray, fb: bool) -> np.ndarray:
    """Steps a4..a8 for covariances (n, M, M): pair-form angle, NaN where R is zero or
    not finite (R7) or the signal subspace is not determined (R10)."""
    if fb:
        R = fb_average(R)
    tr = np.real(np.trace(R, axis1=-2, axis2=-1))
    ok = np.isfinite(tr) & (tr > 0)
    out = np.full(R.shape[0], np.nan)
    if np.any(ok):
        C, lam = noise_projector(R[ok])
        w = select_root_pair(poly_roots(poly_coeffs(C)))["omega"]
        out[ok] = np.where(degenerate(lam), np.nan, w)
    return out


def demodulate_block(frame: np.ndarray, M: int, dirs: str = "xy", fb: bool = True, chunk: int = 16384):
    """Block-mode demodulation: (omega_x or None, omega_y or None), NaN where the block does not fit."""
    g = to_complex_field(frame, 1)
    H, W = g.shape
    wx = np.full((H, W), np.nan) if "x" in dirs else None
    wy = np.full((H, W), np.nan) if "y" in dirs else None
    if M > H or M > W:
        return wx, wy
    h = M // 2
    nr, nc = H - M + 1, W - M + 1
    for r0 in range(0, nr, max(1, chunk // nc)):
        r1 = min(nr, r0 + max(1, chunk // nc))
        Ry, Rx = block_covariances(g[r0:r1 + M - 1], M)
        if wy is not None:
            wy[r0 + h:r1 + h, h:h + nc] = _omega_from_cov(Ry.reshape(-1, M, M), fb).reshape(r1 - r0, nc)
        if wx is not None:
            # z_x = e^{-j omega_x}: omega_x = -arg(z_x)  (Eq. 15)
            wx[r0 + h:r1 + h, h:h + nc] = -_omega_from_cov(Rx.reshape(-1, M, M), fb).reshape(r1 - r0, nc)
    return wx, wy


def block_phase(frame: np.ndarray, M: int, omega_x: np.ndarray, omega_y: np.ndarray) -> np.ndarray:
    """Wrapped phase of the linear model of every block (Eq. 15, reading R9).

    The paper's alpha = angle(mean(Gamma_w e^{-j(omega_x x + omega_y y)})) with
    the block coordinates taken relative to the pixel, which makes alpha the
    model phase alpha_abs + omega_x x + omega_y y at the pixel itself, in
    (-pi, pi].  NaN where either frequency is NaN.
    """
    g = to_complex_field(frame, 1)
    H, W = g.shape
    out = np.full((H, W), np.nan)
    if M > H or M > W:
        return out
    h = M // 2
    B = sliding_window_view(g, (M, M))                # B[a, b, i, j] = g[a+i, b+j], pixel (a+h, b+h)
    wx = np.asarray(omega_x, dtype=np.float64)[h:h + H - M + 1, h:h + W - M + 1]
    wy = np.asarray(omega_y, dtype=np.float64)[h:h + H - M + 1, h:h + W - M + 1]
    d = np.arange(M) - h
    ex = np.exp(-1j * wx[..., None] * d)               # over the block's columns
    ey = np.exp(-1j * wy[..., None] * d)               # over its rows
    s = np.einsum("abij,abi,abj->ab", B, ey, ex) / (M * M)
    alpha = np.angle(s)
    alpha[~(np.isfinite(wx) & np.isfinite(wy))] = np.nan
    out[h:h + H - M + 1, h:h + W - M + 1] = alpha
    return out


# ---------------------------------------------------------------------------
# a10: integration of the frequency maps to phase (reading R6)
# ---------------------------------------------------------------------------
def integrate(omega_x, omega_y, Nx: int, Ny: int, carrier_x: float = 0.0, carrier_y: float = 0.0):
    wx = np.asarray(omega_x, dtype=np.float64) - carrier_x
    H, W = wx.shape
    phi = np.full((H, W), np.nan)
    x0, x1 = valid_range(W, Nx)
    if x1 < x0:
        return phi
    if omega_y is None:
        y0, y1 = 0, H - 1
        anchor = np.zeros(H)
    else:
        wy = np.asarray(omega_y, dtype=np.float64) - carrier_y
        y0, y1 = valid_range(H, Ny)
        if y1 < y0:
            return phi
        col = wy[y0:y1 + 1, x0]
        steps = 0.5 * (col[:-1] + col[1:])
        anchor = np.zeros(H)
        anchor[y0 + 1:y1 + 1] = np.cumsum(steps)
    rows = wx[y0:y1 + 1, x0:x1 + 1]
    steps = 0.5 * (rows[:, :-1] + rows[:, 1:])
    acc = np.zeros_like(rows)
    acc[:, 1:] = np.cumsum(steps, axis=1)
    phi[y0:y1 + 1, x0:x1 + 1] = acc + anchor[y0:y1 + 1, None]
    return phi
