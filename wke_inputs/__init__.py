"""Seeded synthetic inputs for the four-wave kinetic collision operator.

This module is shared by the test oracle and by the GPU path's tests and
benchmark.  It holds only workload descriptions (grid sizes, quadrature
counts, rule names) and the analytic initial data sampled on the uniform
grid; it contains none of the collision-operator arithmetic.

Grid convention (the paper only says "a uniform grid in D_L", Alg. 1): the
node x in {0..N-1} along each axis sits at k = -L + h*x with h = 2L/N, so -L
is a node and +L is not.  Arrays are row-major with the last axis fastest.
All grid data are complex128 (the Fourier truncation keeps the mode -N/2,
which makes the interpolant complex off the grid).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

__all__ = [
    "Workload", "grid_axis", "grid_points",
    "two_gaussians_c1", "three_bumps_2d", "aniso_gaussian_3d", "rj_profile",
    "rayleigh_jeans", "discontinuous_ex3", "two_bumps_3d", "constant",
    "single_mode", "random_smooth", "WORKLOADS", "workload",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One Q(f) problem shape.  rule is 'midpoint' (2D) or one of
    'octahedron', 'cube', 'icosahedron' (3D), used for both q-hat and sigma."""
    d: int
    N: int
    L: float
    Nr: int
    Ns: int
    Nsig: int
    rule: str

    @property
    def M(self) -> int:
        return self.Nr * self.Ns * self.Nsig

    @property
    def shape(self):
        return (self.N,) * self.d


def grid_axis(N: int, L: float) -> np.ndarray:
    """Node coordinates along one axis: -L + (2L/N) x, x = 0..N-1."""
    h = 2.0 * L / N
    return -L + h * np.arange(N, dtype=np.float64)


def grid_points(d: int, N: int, L: float) -> List[np.ndarray]:
    """Meshgrid (ij indexing) of the node coordinates, one array per axis."""
    ax = grid_axis(N, L)
    return list(np.meshgrid(*([ax] * d), indexing="ij"))


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a.astype(np.complex128))


def two_gaussians_c1(N: int = 16, L: float = 8.0) -> np.ndarray:
    """exp(-|k-(1,0)|^2/2) + exp(-|k+(1,0)|^2/2) on the 2D grid."""
    kx, ky = grid_points(2, N, L)
    f = np.exp(-((kx - 1.0) ** 2 + ky ** 2) / 2.0) + np.exp(-((kx + 1.0) ** 2 + ky ** 2) / 2.0)
    return _c(f)


def three_bumps_2d(N: int, L: float, seed: int) -> np.ndarray:
    """Sum of three isotropic Gaussians exp(-|k-c_i|^2/(2 w_i^2)).

    Per bump, three uniforms U1, U2, U3 are drawn in that order from
    numpy.random.default_rng(seed): the centre is 3*sqrt(U1)*(cos 2piU2,
    sin 2piU2) (uniform over the disc |k| <= 3) and the width w = 0.5 + U3.
    """
    rng = np.random.default_rng(seed)
    kx, ky = grid_points(2, N, L)
    f = np.zeros_like(kx)
    for _ in range(3):
        u1, u2, u3 = rng.random(3)
        rad = 3.0 * math.sqrt(u1)
        cx, cy = rad * math.cos(2 * math.pi * u2), rad * math.sin(2 * math.pi * u2)
        w = 0.5 + u3
        f += np.exp(-((kx - cx) ** 2 + (ky - cy) ** 2) / (2.0 * w * w))
    return _c(f)


def aniso_gaussian_3d(N: int, L: float) -> np.ndarray:
    """exp(-(kx^2/2 + ky^2/0.5 + kz^2))."""
    kx, ky, kz = grid_points(3, N, L)
    return _c(np.exp(-(kx ** 2 / 2.0 + ky ** 2 / 0.5 + kz ** 2)))


def rj_profile(d: int, N: int, L: float) -> np.ndarray:
    """The algebraic-tail check profile 1/(1+|k|^2)."""
    pts = grid_points(d, N, L)
    k2 = sum(p * p for p in pts)
    return _c(1.0 / (1.0 + k2))


def rayleigh_jeans(d: int, N: int, L: float, mu: float, nu, xi: float) -> np.ndarray:
    """1/(mu + nu.k + xi |k|^2) sampled on the grid."""
    pts = grid_points(d, N, L)
    den = mu + xi * sum(p * p for p in pts)
    for a in range(d):
        den = den + nu[a] * pts[a]
    if np.any(den <= 0):
        raise ValueError("mu + nu.k + xi|k|^2 must stay positive on the grid")
    return _c(1.0 / den)


def discontinuous_ex3(d: int, N: int, L: float,
                      rho1=6.0 / 5.0, rho2=4.0 / 5.0, T1=2.0 / 3.0, T2=3.0 / 2.0) -> np.ndarray:
    """Two half-space Maxwellians rho/(2 pi T) exp(-|k|^2/(2T)), the first for
    k_1 > 0 and the second for k_1 < 0; nodes on k_1 = 0 get the average."""
    pts = grid_points(d, N, L)
    k2 = sum(p * p for p in pts)
    g1 = rho1 / (2 * math.pi * T1) * np.exp(-k2 / (2 * T1))
    g2 = rho2 / (2 * math.pi * T2) * np.exp(-k2 / (2 * T2))
    f = np.where(pts[0] > 0, g1, np.where(pts[0] < 0, g2, 0.5 * (g1 + g2)))
    return _c(f)


def two_bumps_3d(N: int, L: float, seed: int) -> np.ndarray:
    """Two anisotropic Gaussians exp(-sum_a (k_a-c_a)^2/(2 w_a^2)).

    Per bump, six uniforms are drawn in order from default_rng(seed):
    U1 -> radius 3 U1^(1/3); U2 -> cos(theta) = 2U2-1; U3 -> phi = 2 pi U3
    (so the centre is uniform in the ball |k| <= 3); U4..U6 -> per-axis widths
    0.5 + U (uniform on [0.5, 1.5]).
    """
    rng = np.random.default_rng(seed)
    pts = grid_points(3, N, L)
    f = np.zeros_like(pts[0])
    for _ in range(2):
        u = rng.random(6)
        rad = 3.0 * u[0] ** (1.0 / 3.0)
        ct = 2.0 * u[1] - 1.0
        st = math.sqrt(max(0.0, 1.0 - ct * ct))
        ph = 2.0 * math.pi * u[2]
        c = (rad * st * math.cos(ph), rad * st * math.sin(ph), rad * ct)
        w = 0.5 + u[3:6]
        f += np.exp(-sum((pts[a] - c[a]) ** 2 / (2.0 * w[a] ** 2) for a in range(3)))
    return _c(f)


def constant(d: int, N: int, value: complex = 1.0) -> np.ndarray:
    return np.full((N,) * d, value, dtype=np.complex128)


def single_mode(d: int, N: int, L: float, j0) -> np.ndarray:
    """exp(i pi j0.k / L) on the grid, for an integer mode vector j0."""
    pts = grid_points(d, N, L)
    ph = sum(j0[a] * pts[a] for a in range(d))
    return np.ascontiguousarray(np.exp(1j * math.pi * ph / L))


def random_smooth(d: int, N: int, L: float, seed: int, complex_valued: bool = True) -> np.ndarray:
    """A seeded sum of four random anisotropic Gaussians with random complex
    amplitudes (for structural tests that should not rely on symmetry)."""
    rng = np.random.default_rng(seed)
    pts = grid_points(d, N, L)
    f = np.zeros(pts[0].shape, dtype=np.complex128)
    for _ in range(4):
        c = rng.uniform(-0.3 * L, 0.3 * L, size=d)
        w = rng.uniform(0.08 * L, 0.2 * L, size=d)
        amp = rng.uniform(0.5, 1.5) + (1j * rng.uniform(-0.5, 0.5) if complex_valued else 0.0)
        f += amp * np.exp(-sum((pts[a] - c[a]) ** 2 / (2 * w[a] ** 2) for a in range(d)))
    return np.ascontiguousarray(f)


# The five workload shapes used by the tests and the benchmark.
WORKLOADS = {
    "c1_2d_n16": Workload(2, 16, 8.0, 2, 4, 2, "midpoint"),
    "c2_2d_n64": Workload(2, 64, 10.0, 4, 4, 4, "midpoint"),
    "c3_3d_n32": Workload(3, 32, 10.0, 2, 8, 8, "cube"),
    "c4_2d_n32": Workload(2, 32, 10.0, 4, 4, 4, "midpoint"),
    "c4_2d_n48": Workload(2, 48, 10.0, 4, 4, 4, "midpoint"),
    "c4_2d_n64": Workload(2, 64, 10.0, 4, 4, 4, "midpoint"),
    "c4_2d_n96": Workload(2, 96, 10.0, 4, 4, 4, "midpoint"),
    "c5_3d_n64": Workload(3, 64, 12.0, 4, 8, 8, "cube"),
    # Example 3 (discontinuous data, 2D): N = N_r = 64, N_s = N_sigma = 12, S = 3
    "ex3_2d_n64": Workload(2, 64, (3.0 + math.sqrt(2.0)) * 3.0 / 2.0, 64, 12, 12, "midpoint"),
    # Example 6 (the same data in 3D): N = N_r, S = 0.33; N = 32 and the
    # 12-point design stand in for the unstated N and design size
    "ex6_3d_n32": Workload(3, 32, (3.0 + math.sqrt(2.0)) * 0.33 / 2.0, 32, 12, 12, "icosahedron"),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def c4_batch():
    """The uneven batch: 16 instances each of N = 32, 48, 64, 96 (in that
    order), instance s seeded with s and built with the three-bump recipe."""
    out = []
    s = 0
    for N in (32, 48, 64, 96):
        for _ in range(16):
            out.append((WORKLOADS["c4_2d_n%d" % N], three_bumps_2d(N, 10.0, s)))
            s += 1
    return out


def c5_batch():
    """Eight 3D N=64, L=12 instances, seeds 0..7, two anisotropic bumps each."""
    wl = WORKLOADS["c5_3d_n64"]
    return [(wl, two_bumps_3d(64, 12.0, s)) for s in range(8)]
