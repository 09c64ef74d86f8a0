"""Pins for the oracle's exact-weight reference system (Appendix B): the
Galerkin sums with the exact constraint and the weight functions integrated
in closed form over q-hat and sigma.  Checked against things other than
itself: the sphere means by direct quadrature, the zero mass mode the
appendix proves, and the convergence of the fast method (exact constraint)
to it as the fast method's quadrature is refined.
"""
import math

import numpy as np
import pytest

import oracle
import wke_inputs as wi


def _product_sphere(nt, nphi):
    t, w = np.polynomial.legendre.leggauss(nt)
    pts, wts = [], []
    for ct, wt in zip(t, w):
        st = math.sqrt(1.0 - ct * ct)
        for k in range(nphi):
            ph = 2.0 * math.pi * (k + 0.5) / nphi
            pts.append([st * math.cos(ph), st * math.sin(ph), ct])
            wts.append(wt * 2.0 * math.pi / nphi)
    return np.array(pts), np.array(wts)


def test_sphere_means_in_closed_form():
    """int e^{i x.s} ds over the circle is 2 pi J_0(|x|), over the sphere
    4 pi sin|x|/|x|: the identities the exact weights rest on."""
    from scipy.special import j0
    th = 2.0 * math.pi * (np.arange(64) + 0.5) / 64
    P, W = _product_sphere(24, 48)
    for x in (0.0, 0.3, 2.0, 7.5):
        circ = np.sum(np.exp(1j * x * np.cos(th))) * 2.0 * math.pi / 64
        assert abs(circ - 2.0 * math.pi * j0(x)) < 1e-12
        sph = np.sum(W * np.exp(1j * x * P[:, 2]))
        ref = 4.0 * math.pi * (np.sin(x) / x if x else 1.0)
        assert abs(sph - ref) < 1e-10


@pytest.mark.parametrize("d,N,L", [(2, 8, 8.0), (2, 12, 6.0), (3, 4, 6.0)])
def test_exact_system_conserves_mass(d, N, L):
    """Appendix B: the zeroth mode of the exact system vanishes."""
    f = wi.random_smooth(d, N, L, 4)
    _, Qh = oracle.Q_exact(f, d, N, L, return_hat=True)
    assert abs(Qh.flat[0]) <= 1e-14 * np.abs(Qh).sum()
    # a constant: only the zero mode, where the four weights coincide; the
    # bound is rounding on the size of one weight, S(0)^2 R^(2d-2) / (2d-2)
    R = oracle.default_R(L)
    s0 = 2.0 * math.pi if d == 2 else 4.0 * math.pi
    w0 = s0 * s0 * R ** (2 * d - 2) / (2 * d - 2)
    assert np.abs(oracle.Q_exact(np.full((N,) * d, 1.3 + 0j), d, N, L)).max() < 1e-14 * w0 * 1.3 ** 3


def test_fast_method_converges_to_exact_system_2d():
    """The double convolution with the exact constraint and Gauss-Legendre /
    midpoint quadrature approaches the exact weights spectrally."""
    d, N, L = 2, 8, 8.0
    f = wi.random_smooth(d, N, L, 3)
    Q = oracle.Q_exact(f, d, N, L)
    errs = [oracle.rel_l2(oracle.Q_fourier(f, oracle.nodes(d, N, L, nr, ns, ns, "midpoint"), linear=True), Q)
            for nr, ns in [(4, 8), (8, 16), (16, 32)]]
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 1e-8


def test_fast_method_converges_to_exact_system_3d():
    """3D, with Gauss-Legendre x midpoint product rules on the sphere (the
    closed-form designs are not refinable)."""
    d, N, L = 3, 4, 6.0
    f = wi.random_smooth(d, N, L, 3)
    Q = oracle.Q_exact(f, d, N, L)
    R = oracle.default_R(L)
    errs = []
    for nr, nt, nphi in [(3, 3, 6), (5, 4, 8)]:
        x, w = np.polynomial.legendre.leggauss(nr)
        P, W = _product_sphere(nt, nphi)
        nd = oracle.custom_nodes(d, N, L, 0.5 * R * (1 + x), 0.5 * R * w, P, W, P, W)
        errs.append(oracle.rel_l2(oracle.Q_fourier(f, nd, linear=True), Q))
    assert errs[0] > 4 * errs[1]
