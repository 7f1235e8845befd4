"""FP64 CPU oracle for sliding-window root-MUSIC fringe demodulation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never
does, and the two share no code.

Every function follows the paper (Ramaiah, Ajithaprasad, Rajshekhar,
Ambrosini, "Fast and robust method for flow analysis using GPU assisted
diffractive optical element based background oriented schlieren") and cites
the section or equation it implements.  Readings of points the paper leaves
open are listed in the module docstring of ``oracle.rootmusic``.
"""
from .rootmusic import (  # noqa: F401
    analytic_signal,
    covariance,
    fb_average,
    noise_projector,
    degenerate,
    DEGENERATE_REL,
    poly_coeffs,
    poly_roots,
    select_root_pair,
    demod_windows,
    demod_lines,
    demodulate,
    integrate,
    valid_range,
    to_complex_field,
    analytic_mask,
    block_covariances,
    demodulate_block,
    block_phase,
)
