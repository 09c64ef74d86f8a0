"""Pins for the oracle's quadrature (eq. (G1): Gauss-Legendre in |q|, the
midpoint rule on the circle, closed-form spherical designs on S^2)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("n", list(range(1, 25)) + [32, 64])
def test_gauss_legendre_matches_library(n):
    t, w = oracle.gauss_legendre(n)
    t_ref, w_ref = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(t - t_ref)) < 2e-15
    assert np.max(np.abs(w - w_ref)) < 2e-15 * max(1.0, n / 8)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13])
def test_gauss_legendre_exact_for_polynomials(n):
    t, w = oracle.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, t ** k) - exact) < 1e-14
    # and not exact one degree higher (a wrong node set can pass low degrees)
    k = 2 * n
    assert abs(np.dot(w, t ** k) - 2.0 / (k + 1)) > 1e-8


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 12])
def test_midpoint_rule_trig_exactness(n):
    pts, w = oracle.sphere_rule(2, "midpoint", n)
    th = np.arctan2(pts[:, 1], pts[:, 0])
    assert np.allclose(np.sum(pts ** 2, 1), 1.0, atol=1e-15)
    assert abs(w.sum() - 2 * math.pi) < 1e-14
    for k in range(-n + 1, n):
        exact = 2 * math.pi if k == 0 else 0.0
        assert abs(np.dot(w, np.exp(1j * k * th)) - exact) < 1e-13
    # the angles are (2i+1) pi / n
    ref = (2 * np.arange(n) + 1) * math.pi / n
    assert np.allclose(np.mod(th, 2 * math.pi), ref, atol=1e-14)


def _monomial_integral(e):
    """Exact integral of x^a y^b z^c over S^2 (textbook closed form)."""
    if any(v % 2 for v in e):
        return 0.0
    b = [(v + 1) / 2.0 for v in e]
    return 2.0 * math.prod(math.gamma(x) for x in b) / math.gamma(sum(b))


@pytest.mark.parametrize("rule,n,t", [("octahedron", 6, 3), ("cube", 8, 3), ("icosahedron", 12, 5)])
def test_spherical_designs(rule, n, t):
    pts, w = oracle.sphere_rule(3, rule, n)
    assert np.allclose(np.sum(pts ** 2, 1), 1.0, atol=1e-15)
    assert abs(w.sum() - GOLD["sphere_moments"]["area"]) < 1e-13
    for e in itertools.product(range(t + 1), repeat=3):
        if sum(e) > t:
            continue
        val = np.dot(w, pts[:, 0] ** e[0] * pts[:, 1] ** e[1] * pts[:, 2] ** e[2])
        assert abs(val - _monomial_integral(e)) < 1e-13, (rule, e)
    assert abs(np.dot(w, pts[:, 0] ** 2) - GOLD["sphere_moments"]["x2"]) < 1e-13
    if t >= 5:
        assert abs(np.dot(w, pts[:, 0] ** 4) - GOLD["sphere_moments"]["x4"]) < 1e-13
        assert abs(np.dot(w, pts[:, 0] ** 2 * pts[:, 1] ** 2) - GOLD["sphere_moments"]["x2y2"]) < 1e-13


@pytest.mark.parametrize("d,rule,n", [(2, "midpoint", 2), (2, "midpoint", 4), (2, "midpoint", 12),
                                      (3, "octahedron", 6), (3, "cube", 8), (3, "icosahedron", 12)])
def test_rules_are_antipodal(d, rule, n):
    pts, _ = oracle.sphere_rule(d, rule, n)
    for p in pts:
        assert np.min(np.max(np.abs(pts + p), axis=1)) < 1e-15


def test_midpoint_odd_is_not_antipodal():
    pts, _ = oracle.sphere_rule(2, "midpoint", 3)
    assert np.min(np.max(np.abs(pts + pts[0]), axis=1)) > 0.1


def test_default_R():
    # R = 2S with S = 2L/(3+sqrt 2): L = (3+sqrt 2) S / 2 (Section 3.2, Step 1)
    for L, R in [(8.0, 7.2493), (10.0, 9.0616), (12.0, 10.8740)]:
        assert abs(oracle.default_R(L) - R) < 1e-4
        S = oracle.default_R(L) / 2
        assert abs((3 + math.sqrt(2)) / 2 * S - L) < 1e-12
