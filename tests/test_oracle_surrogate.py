"""Pins of the surrogate oracle and of the counter-based training-line generator."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import surrogate as S


def test_philox_known_answer_vectors():
    """Published Philox4x32-10 known-answer vectors (Random123 test set)."""
    kat = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for c, k, e in kat:
        out = wl.philox4x32(np.array([c], np.uint32), np.array([k], np.uint32))[0]
        assert tuple(int(x) for x in out) == e


def test_training_lines_statistics_and_determinism():
    lines, w = wl.philox_training_lines(np.arange(4000), seed=7)
    assert lines.shape == (4000, 128)
    assert np.all(w >= 2 * np.pi / 16) and np.all(w <= 2 * np.pi / 4)
    again, w2 = wl.philox_training_lines(np.arange(2000, 2100), seed=7)
    assert np.array_equal(again, lines[2000:2100]) and np.array_equal(w2, w[2000:2100])
    other, _ = wl.philox_training_lines(np.arange(100), seed=8)
    assert not np.allclose(other, lines[:100])
    assert abs(lines.mean() - 0.5) < 0.01


def test_bf16_rounding_ties_to_even_and_matches_torch():
    one = np.float32(1.0)
    assert S.bf16_round(np.float32(1 + 2 ** -8)) == 1.0                 # halfway, even below
    assert S.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6     # halfway, even above
    assert S.bf16_round(one) == 1.0
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(S.bf16_round(x), ref)


def test_features_of_a_tone_and_invariances():
    N, w = 32, 0.9
    n = np.arange(N)
    win = 2.5 * np.exp(1j * (w * n + 0.3))
    f = S.features(win[None])[0]
    k = np.arange(16) - 8
    assert np.allclose(f[:16], np.cos(w * k), atol=1e-12)
    assert np.allclose(f[16:], np.sin(w * k), atol=1e-12)
    rng = np.random.default_rng(1)
    noisy = rng.standard_normal((5, N)) + 1j * rng.standard_normal((5, N))
    a = S.features(noisy)
    b = S.features(noisy * (0.3 - 1.7j))
    assert np.allclose(a, b, atol=1e-12)
    assert np.allclose(a[:, 16 + 8], 0.0, atol=1e-12) and np.all(a[:, 8] > 0)   # centre is real positive


def test_gelu_and_its_derivative():
    assert S.gelu(np.array(0.0)) == 0.0
    assert abs(S.gelu(np.array(6.0)) - 6.0) < 1e-8
    assert abs(S.gelu(np.array(-6.0))) < 1e-7
    x = np.linspace(-4, 4, 101)
    h = 1e-6
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - S.gelu_grad(x))) < 1e-8


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = {k: v.astype(np.float64) for k, v in S.init_params(11).items()}
    X = rng.standard_normal((7, 32))
    T = S.targets(rng.uniform(0, 2, 7))
    g = S.backward(S.forward(p, X, quantize=False), T)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = S.loss(S.forward(p, X, quantize=False)["Y"], T)
            flat[idx] = old - h
            lm = S.loss(S.forward(p, X, quantize=False)["Y"], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (k, idx, fd, an)


def test_adam_first_step_closed_form():
    p = {"W": np.array([1.0, -2.0, 3.0])}
    g = {"W": np.array([0.5, -4.0, 0.0])}
    zero = {"W": np.zeros(3)}
    P, M, V = S.adam(p, g, zero, zero, t=1, lr=0.01)
    # bias-corrected moments equal g and g^2 on the first step
    exp = p["W"] - 0.01 * g["W"] / (np.abs(g["W"]) + 1e-8)
    assert np.allclose(P["W"], exp, atol=1e-15)
    assert np.allclose(M["W"], 0.1 * g["W"]) and np.allclose(V["W"], 0.001 * g["W"] ** 2)


def test_null_spectrum_zero_at_tone_and_matches_projector():
    L, w = 8, 0.77
    a = np.exp(1j * w * np.arange(L))
    u = a / math.sqrt(L)
    assert abs(S.null_spectrum(u[None], np.array([w]))[0]) < 1e-14
    rng = np.random.default_rng(2)
    uu = rng.standard_normal((4, L)) + 1j * rng.standard_normal((4, L))
    uu /= np.linalg.norm(uu, axis=1, keepdims=True)
    ww = rng.uniform(-3, 3, 4)
    for i in range(4):
        aa = np.exp(1j * ww[i] * np.arange(L))
        C = np.eye(L) - np.outer(uu[i], uu[i].conj())
        assert abs(S.null_spectrum(uu[i:i + 1], ww[i:i + 1])[0] - np.real(aa.conj() @ C @ aa) / L) < 1e-12


def test_quantized_forward_close_to_exact():
    p = S.init_params(5)
    X = np.random.default_rng(4).standard_normal((64, 32))
    yq = S.forward(p, X)["Y"]
    ye = S.forward(p, X, quantize=False)["Y"]
    assert np.max(np.abs(yq - ye)) < 0.05 * max(1.0, np.max(np.abs(ye)))


def test_gelu_values_fixed_by_the_normal_cdf():
    """GELU(x) = x * Phi(x) with Phi the standard normal CDF.  Phi is taken here from
    tabulated values and, independently, by quadrature of the normal density; this
    fixes the 1/sqrt(2) inside erf and rules out the tanh approximation (which is off
    by ~1e-4 at x = 1 and by ~1.6e-4 at x = -1.5)."""
    from scipy.integrate import quad
    table = {1.0: 0.8413447460685429, -1.0: 0.15865525393145707, 2.0: 0.9772498680518208,
             -1.5: 0.06680720126885807, 0.5: 0.6914624612740131}
    dens = lambda t: math.exp(-0.5 * t * t) / math.sqrt(2.0 * math.pi)
    for x, phi in table.items():
        cdf = 0.5 + quad(dens, 0.0, x, epsabs=1e-15, epsrel=1e-15)[0]
        assert abs(cdf - phi) < 1e-13
        assert abs(float(S.gelu(np.float64(x))) - x * phi) < 1e-13, x
        # d/dx [x Phi(x)] = Phi(x) + x phi(x)
        assert abs(float(S.gelu_grad(np.float64(x))) - (phi + x * dens(x))) < 1e-13, x
    tanh_form = lambda x: 0.5 * x * (1 + math.tanh(math.sqrt(2 / math.pi) * (x + 0.044715 * x ** 3)))
    assert abs(tanh_form(-1.5) - float(S.gelu(np.float64(-1.5)))) > 1e-4


def test_features_fix_the_span_and_the_derotation_sample():
    """A tone plus an impulse on the window's centre sample N/2: the impulse must land on
    feature 8 (the 16-sample span is samples N/2-8 .. N/2+7), and the de-rotation must use
    the phase of that centre sample (every feature of the tone part then has the phase
    w (n - N/2)).  Values written out by hand for N = 32, w = 0.3, impulse 3 e^{j w 16}."""
    N, w = 32, 0.3
    n = np.arange(N)
    win = np.exp(1j * w * n)
    win[16] += 3.0 * np.exp(1j * w * 16)              # centre sample: 4 e^{j w 16}
    rms = math.sqrt((31.0 + 16.0) / 32.0)
    f = S.features(win[None])[0]
    expect = np.empty(16, complex)
    for k in range(16):
        expect[k] = np.exp(1j * w * (k - 8)) / rms
    expect[8] = 4.0 / rms
    assert np.allclose(f[:16], expect.real, atol=1e-12)
    assert np.allclose(f[16:], expect.imag, atol=1e-12)
    # shifting the impulse by one sample moves it to feature 9 and changes the rotation
    win2 = np.exp(1j * w * n)
    win2[17] += 3.0 * np.exp(1j * w * 17)
    f2 = S.features(win2[None])[0]
    assert abs(f2[9] - 4.0 / rms * math.cos(w)) < 1e-12 and abs(f2[8] - 1.0 / rms) < 1e-12
