"""Helpers shared by the parity tests: oracle references on sampled lines and
the omega comparison used as the parity bar."""
import math

import numpy as np

import oracle

# Parity bar of the plain path: |d omega| <= 1e-4 rad/px at the 99.9th percentile.
OMEGA_TOL = 1e-4
OMEGA_Q = 0.999


def wrap(d):
    return (np.asarray(d) + np.pi) % (2 * np.pi) - np.pi


def oracle_rows(frame: np.ndarray, rows, L: int, N: int) -> np.ndarray:
    """Oracle omega_x on the given rows of a real or complex frame (full-width lines)."""
    f = np.asarray(frame)[list(rows)]
    g = oracle.to_complex_field(f, 1)
    return oracle.demod_lines(g, L, N)


def oracle_cols(frame: np.ndarray, cols, L: int, N: int) -> np.ndarray:
    """Oracle omega_y on the given columns; returned as (len(cols), H)."""
    f = np.asarray(frame)[:, list(cols)].T
    g = oracle.to_complex_field(f, 1)      # analytic along the column, now the last axis
    return oracle.demod_lines(g, L, N)


def compare_omega(got: np.ndarray, ref: np.ndarray, what: str = "", tol: float = OMEGA_TOL, q: float = OMEGA_Q):
    """NaN patterns must agree exactly; finite values meet the percentile bar."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    gn, rn = np.isnan(got), np.isnan(ref)
    assert np.array_equal(gn, rn), f"{what}: NaN pattern differs in {np.sum(gn != rn)} of {gn.size} pixels"
    d = np.abs(wrap(got[~gn] - ref[~rn]))
    if d.size == 0:
        return {"n": 0}
    stats = {"n": int(d.size), "p50": float(np.quantile(d, 0.5)), "p999": float(np.quantile(d, q)),
             "max": float(d.max()), "frac_over": float(np.mean(d > tol))}
    assert stats["frac_over"] <= 1.0 - q, f"{what}: {stats}"
    return stats
