"""Pins for the oracle's direct transforms (eq. (fj)) and moments."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import wke_inputs as wi

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _signs(d, N):
    j = np.fft.fftfreq(N, 1.0 / N).astype(int)
    j[N // 2] = -N // 2
    s = 1.0
    for a in range(d):
        sh = [1] * d
        sh[a] = N
        s = s * ((-1.0) ** j).reshape(sh)
    return s


@pytest.mark.parametrize("d,N", [(1, 8), (2, 8), (2, 12), (3, 6)])
def test_spectrum_matches_numpy_fft(d, N):
    L = 3.7
    f = wi.random_smooth(d, N, L, 3) if d > 1 else np.exp(np.linspace(0, 1, N)) + 0j
    fh = oracle.spectrum(f, L)
    # with k_x = -L + h x, exp(-i pi j k_x / L) = (-1)^j exp(-2 pi i j x / N)
    ref = np.fft.fftn(f) / f.size * _signs(d, N)
    assert np.max(np.abs(fh - ref)) < 1e-14 * np.max(np.abs(ref)) * N


@pytest.mark.parametrize("d,N", [(2, 8), (2, 16), (3, 8)])
def test_synthesis_round_trip(d, N):
    L = 5.0
    f = wi.random_smooth(d, N, L, 7)
    g = oracle.synthesis(oracle.spectrum(f, L), L)
    assert np.max(np.abs(g - f)) < 1e-13


def test_single_mode_spectrum_is_a_delta():
    d, N, L = 2, 8, 4.0
    j0 = (2, -3)
    f = wi.single_mode(d, N, L, j0)
    fh = oracle.spectrum(f, L)
    expect = np.zeros_like(fh)
    expect[j0[0] % N, j0[1] % N] = 1.0
    assert np.max(np.abs(fh - expect)) < 1e-14


def test_eval_points_reproduces_grid_and_series():
    d, N, L = 2, 8, 4.0
    f = wi.random_smooth(d, N, L, 11)
    fh = oracle.spectrum(f, L)
    pts = np.stack([p.ravel() for p in wi.grid_points(d, N, L)], 1)
    assert np.max(np.abs(oracle.eval_points(fh, L, pts) - f.ravel())) < 1e-13
    # off-grid: the series of a single mode (including the kept -N/2 mode)
    for j0 in [(1, 2), (-4, 3), (-4, -4)]:
        g = oracle.spectrum(wi.single_mode(d, N, L, j0), L)
        k = np.array([[0.123, -1.7], [2.2, 0.31]])
        val = oracle.eval_points(g, L, k)
        ref = np.exp(1j * math.pi * (k @ np.array(j0, float)) / L)
        assert np.max(np.abs(val - ref)) < 1e-13


def test_moment_identity_rho_is_zero_mode():
    # rho = (2L)^d f_hat_0 for the rectangle rule (Appendix B)
    for d, N in [(2, 16), (3, 8)]:
        L = 6.0
        f = wi.random_smooth(d, N, L, 5, complex_valued=False)
        mom = oracle.moments(f, L)
        fh = oracle.spectrum(f, L)
        assert abs(mom[0] - (2 * L) ** d * fh[(0,) * d].real) < 1e-12 * abs(mom[0])


def test_moments_closed_form_gaussian():
    # rho, E, P of a shifted Gaussian (closed forms), rectangle rule is
    # spectrally accurate for smooth data that vanish at the box edge
    d, N, L = 2, 64, 10.0
    kx, ky = wi.grid_points(d, N, L)
    c = (0.7, -0.4)
    f = np.exp(-((kx - c[0]) ** 2 + (ky - c[1]) ** 2) / 2.0) + 0j
    mom = oracle.moments(f, L)
    rho = 2 * math.pi
    assert abs(mom[0] - rho) < 1e-12
    assert abs(mom[1] - rho * (2.0 + c[0] ** 2 + c[1] ** 2)) < 1e-11
    assert abs(mom[2] - rho * c[0]) < 1e-12 and abs(mom[3] - rho * c[1]) < 1e-12
    assert mom[4] == 0.0


def test_example3_initial_moments():
    """Example 3: rho(0) = 1, E(0) = 2 for the discontinuous data (paper,
    Section 4.1.2).  Rectangle rule with the average on k_1 = 0: O(h^2)."""
    g = GOLD["ex3_initial_moments"]
    errs = []
    for N in (32, 64, 128):
        f = wi.discontinuous_ex3(2, N, 10.0, g["rho1"], g["rho2"], g["T1"], g["T2"])
        mom = oracle.moments(f, 10.0)
        errs.append((abs(mom[0] - g["rho0"]), abs(mom[1] - g["E0"])))
    assert errs[-1][0] < 1e-10 and errs[-1][1] < 1e-9
