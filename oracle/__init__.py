"""CPU oracle for the spectrally truncated four-wave collision operator.

TEST INFRASTRUCTURE ONLY: this package may be imported by the tests, by the
smoke check and by the benchmark's CPU-baseline leg, never by the GPU path.
It shares no code with the GPU library.  Everything is IEEE double, with
direct sums and no FFT; the heavy loops live in ``wke_oracle.c`` (plain C,
OpenMP over output points, fixed summation order).

Paper: Qi, Shen, Wang, "A fast Fourier spectral method for wave kinetic
equation", arXiv 2503.12805.  Section 3.2 defines the truncation (Step 1),
the series f_N (eq. (fj)) and the Galerkin terms (eqs. (KK1)-(KK4)); Section
3.3 the quadrature decomposition (eq. (G1)) and the double convolution
(eq. (K1_con)); Alg. 1 the evaluation order.

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_*.py`` (closed forms, library routines, brute force over
the paper's weight functions G_1..G_4, Rayleigh-Jeans vanishing, moment
identities); nothing is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import sys
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wke_oracle.c")
_LIB = os.path.join(_HERE, "_wke_oracle.so")

RULES = {"midpoint": 0, "octahedron": 1, "cube": 2, "icosahedron": 3}
RULE_POINTS = {"octahedron": 6, "cube": 8, "icosahedron": 12}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fcx-limited-range", "-ffp-contract=off", "-D_DEFAULT_SOURCE",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.c_int
        node_args = [I, D, D, I, D, D, I, D, D]
        lib.oracle_gauss_legendre.argtypes = [I, D, D]
        lib.oracle_sphere_rule.argtypes = [I, I, I, D, D]
        lib.oracle_spectrum.argtypes = [I, I, ctypes.c_double, D, D]
        lib.oracle_synthesis.argtypes = [I, I, ctypes.c_double, D, D]
        lib.oracle_eval_points.argtypes = [I, I, ctypes.c_double, D, I, D, D]
        lib.oracle_Q_physical.argtypes = [I, I, ctypes.c_double] + node_args + [D, D, D]
        lib.oracle_Q_points.argtypes = [I, I, ctypes.c_double] + node_args + [
            D, I, ctypes.POINTER(ctypes.c_long), D]
        lib.oracle_Q_fourier.argtypes = [I, I, ctypes.c_double] + node_args + [I, D, D, D, D]
        lib.oracle_rk4.argtypes = [I, I, ctypes.c_double] + node_args + [D, ctypes.c_double, I]
        lib.oracle_moments.argtypes = [I, I, ctypes.c_double, D, D]
        lib.oracle_exact_system.argtypes = [I, I, ctypes.c_double, ctypes.c_double, I, D, D, D]
        for fn in ("oracle_gauss_legendre", "oracle_sphere_rule", "oracle_spectrum",
                   "oracle_synthesis", "oracle_eval_points", "oracle_Q_physical",
                   "oracle_Q_points", "oracle_Q_fourier", "oracle_rk4", "oracle_moments",
                   "oracle_exact_system"):
            getattr(lib, fn).restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc < 0:
        raise RuntimeError("%s failed with status %d" % (what, rc))
    return rc


# --------------------------------------------------------------------------
# Quadrature (eq. (G1))
# --------------------------------------------------------------------------

def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes/weights on [-1, 1] (Newton on the
    Legendre three-term recurrence)."""
    t = np.zeros(n)
    w = np.zeros(n)
    _check(_load().oracle_gauss_legendre(n, _dp(t), _dp(w)), "gauss_legendre")
    return t, w


def sphere_rule(d: int, rule: str, n: int):
    """Directions (n x d) and weights on S^{d-1}, total weight |S^{d-1}|."""
    pts = np.zeros((n, d))
    w = np.zeros(n)
    _check(_load().oracle_sphere_rule(d, RULES[rule], n, _dp(pts), _dp(w)), "sphere_rule")
    return pts, w


def default_R(L: float) -> float:
    """R = 2S with S = 2L/(3+sqrt 2): the equality case of the paper's
    anti-aliasing condition L >= (3+sqrt 2) S / 2 (Section 3.2, Step 1)."""
    return 4.0 * L / (3.0 + math.sqrt(2.0))


@dataclass
class Nodes:
    d: int
    N: int
    L: float
    r: np.ndarray      # radial nodes on [0, R]
    wr: np.ndarray     # radial weights
    qh: np.ndarray     # (Ns, d) directions q-hat
    ws: np.ndarray
    sg: np.ndarray     # (Nsig, d) collision angles sigma
    wsig: np.ndarray

    def args(self):
        return [len(self.r), _dp(self.r), _dp(self.wr), len(self.ws), _dp(self.qh), _dp(self.ws),
                len(self.wsig), _dp(self.sg), _dp(self.wsig)]

    @property
    def M(self):
        return len(self.r) * len(self.ws) * len(self.wsig)


def nodes(d, N, L, Nr, Ns, Nsig, rule="midpoint", R=None) -> Nodes:
    """Quadrature of eq. (G1): Gauss-Legendre in |q| on [0, R] (r = R/2 (1+t),
    w_r = R/2 w), and the sphere rule `rule` for both q-hat and sigma."""
    if R is None or R <= 0:
        R = default_R(L)
    t, w = gauss_legendre(Nr)
    r = 0.5 * R * (1.0 + t)
    wr = 0.5 * R * w
    qh, ws = sphere_rule(d, rule, Ns)
    sg, wsig = sphere_rule(d, rule, Nsig)
    return Nodes(d, N, L, np.ascontiguousarray(r), np.ascontiguousarray(wr),
                 np.ascontiguousarray(qh), np.ascontiguousarray(ws),
                 np.ascontiguousarray(sg), np.ascontiguousarray(wsig))


def nodes_for(wl, R=None) -> Nodes:
    return nodes(wl.d, wl.N, wl.L, wl.Nr, wl.Ns, wl.Nsig, wl.rule, R)


def custom_nodes(d, N, L, r, wr, qh, ws, sg, wsig) -> Nodes:
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return Nodes(d, N, L, f(r), f(wr), f(np.reshape(qh, (-1, d))), f(ws),
                 f(np.reshape(sg, (-1, d))), f(wsig))


# --------------------------------------------------------------------------
# Transforms (eq. (fj))
# --------------------------------------------------------------------------

def _cgrid(f, d, N):
    a = np.ascontiguousarray(np.asarray(f, dtype=np.complex128))
    if a.shape != (N,) * d:
        raise ValueError("expected shape %s, got %s" % ((N,) * d, a.shape))
    return a


def spectrum(f, L):
    """f_hat_j = N^-d sum_x f(k_x) exp(-i pi j.k_x/L), FFT index order."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.complex128))
    d, N = f.ndim, f.shape[0]
    out = np.zeros_like(f)
    _check(_load().oracle_spectrum(d, N, L, _dp(f), _dp(out)), "spectrum")
    return out


def synthesis(fhat, L):
    """g(k_x) = sum_j fhat_j exp(i pi j.k_x / L) on the grid."""
    fhat = np.ascontiguousarray(np.asarray(fhat, dtype=np.complex128))
    d, N = fhat.ndim, fhat.shape[0]
    out = np.zeros_like(fhat)
    _check(_load().oracle_synthesis(d, N, L, _dp(fhat), _dp(out)), "synthesis")
    return out


def eval_points(fhat, L, k):
    """f_N at arbitrary points k (npts x d) by the full direct sum."""
    fhat = np.ascontiguousarray(np.asarray(fhat, dtype=np.complex128))
    d, N = fhat.ndim, fhat.shape[0]
    if N > 512:
        raise ValueError("N <= 512")
    k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1, d))
    out = np.zeros(len(k), dtype=np.complex128)
    _check(_load().oracle_eval_points(d, N, L, _dp(fhat), len(k), _dp(k), _dp(out)), "eval_points")
    return out


# --------------------------------------------------------------------------
# The collision operator
# --------------------------------------------------------------------------

def Q_physical(f, nd: Nodes, return_terms=False):
    """Q on the grid from products of the interpolant at shifted points."""
    f = _cgrid(f, nd.d, nd.N)
    Q = np.zeros_like(f)
    K = np.zeros((4,) + f.shape, dtype=np.complex128) if return_terms else None
    _check(_load().oracle_Q_physical(nd.d, nd.N, nd.L, *nd.args(), _dp(f), _dp(Q),
                                     _dp(K) if return_terms else None), "Q_physical")
    return (Q, K) if return_terms else Q


def Q_fourier(f, nd: Nodes, linear=False, return_hat=False):
    """Q from the double convolution in Fourier space (cyclic by default)."""
    f = _cgrid(f, nd.d, nd.N)
    Q = np.zeros_like(f)
    Qh = np.zeros_like(f)
    Kh = np.zeros((4,) + f.shape, dtype=np.complex128)
    _check(_load().oracle_Q_fourier(nd.d, nd.N, nd.L, *nd.args(), int(bool(linear)),
                                    _dp(f), _dp(Q), _dp(Qh), _dp(Kh)), "Q_fourier")
    return (Q, Qh, Kh) if return_hat else Q


def Q_points(f, nd: Nodes, flat_idx):
    """Q at selected grid points (flat row-major indices), point by point."""
    f = _cgrid(f, nd.d, nd.N)
    idx = np.ascontiguousarray(np.asarray(flat_idx, dtype=np.int64))
    out = np.zeros(len(idx), dtype=np.complex128)
    _check(_load().oracle_Q_points(nd.d, nd.N, nd.L, *nd.args(), _dp(f), len(idx),
                                   idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out)),
           "Q_points")
    return out


def rk4(f, nd: Nodes, dt, nsteps):
    """Classical RK4 on the grid state; returns the new state."""
    y = _cgrid(f, nd.d, nd.N).copy()
    _check(_load().oracle_rk4(nd.d, nd.N, nd.L, *nd.args(), _dp(y), float(dt), int(nsteps)), "rk4")
    return y


def moments(f, L):
    """[rho, E, P_1..P_d, max|Im f|] by the rectangle rule on the grid."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.complex128))
    d, N = f.ndim, f.shape[0]
    out = np.zeros(d + 3)
    _check(_load().oracle_moments(d, N, L, _dp(f), _dp(out)), "moments")
    return out


def rel_l2(a, ref):
    a = np.asarray(a)
    ref = np.asarray(ref)
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


# --------------------------------------------------------------------------
# Exact-Galerkin (de-aliased) operator through twice the grid
# --------------------------------------------------------------------------
# The triple convolution with the exact constraint l + m + n = j (eq. (KK1);
# Q_fourier(linear=True)), restricted to j in [-N/2, N/2-1], equals the cyclic
# operator on the grid of P = 2N points applied to f_N sampled there,
# projected back onto the modes [-N/2, N/2-1]: a product of three series with
# modes in [-N/2, N/2-1] has modes in [-3N/2, 3N/2-3], none of which wraps
# into [-N/2, N/2-1] modulo 2N.  This route costs a physical-form evaluation
# on 2N points instead of the O(N^(2d)) direct sums, for sizes where those
# are too slow.  Parity pinned: equal to Q_fourier(linear=True) at 1e-13 on
# small grids (tests), and different from it with 3N/2 points.

def _mode_index(N, P):
    """P-grid FFT index of each N-grid FFT index (the same signed mode)."""
    i = np.arange(N)
    return np.where(i < N // 2, i, i - N) % P


def sample_fine(f, L, P):
    """f_N (modes [-N/2, N/2-1] of the grid function f) on the grid of P points."""
    f = np.asarray(f, dtype=np.complex128)
    d, N = f.ndim, f.shape[0]
    big = np.zeros((P,) * d, dtype=np.complex128)
    m = _mode_index(N, P)
    big[np.ix_(*([m] * d))] = spectrum(f, L)
    return synthesis(big, L)


def project_coarse(g, L, N):
    """Projection of a P-grid function onto the modes [-N/2, N/2-1], sampled
    on the grid of N points."""
    g = np.asarray(g, dtype=np.complex128)
    d, P = g.ndim, g.shape[0]
    m = _mode_index(N, P)
    return synthesis(spectrum(g, L)[np.ix_(*([m] * d))], L)


def Q_galerkin(f, wl, P=None):
    """Exact-Galerkin Q of the grid function f for the workload wl (d, L,
    Nr, Ns, Nsig, rule), through the cyclic operator on P (default 2N) points."""
    f = np.asarray(f, dtype=np.complex128)
    N = f.shape[0]
    P = 2 * N if P is None else P
    nd = nodes(wl.d, P, wl.L, wl.Nr, wl.Ns, wl.Nsig, wl.rule)
    return project_coarse(Q_physical(sample_fine(f, wl.L, P), nd), wl.L, N)


# --------------------------------------------------------------------------
# Nyquist-zero real form
# --------------------------------------------------------------------------
# The truncated series of eq. (fj) keeps the modes j_a = -N/2, which have no
# partner +N/2 in the box; they are what makes f_N complex off the grid for
# real data.  The real form drops every mode with a component -N/2 from the
# operator's input and takes Re f: Q_Z(f) = Q(P Re f).  Parity pinned by
# the tests: real output, equality with Q where f has no such modes, zero
# output for data made only of them, and the brute-force weight-function
# sums on the masked spectrum.

def nyquist_zero(f, L):
    """The grid function with every mode that has a component -N/2 removed."""
    f = np.asarray(f, dtype=np.complex128)
    d, N = f.ndim, f.shape[0]
    fh = spectrum(f, L)
    keep = np.ones(N, dtype=bool)
    keep[N // 2] = False
    mask = keep
    for _ in range(d - 1):
        mask = np.multiply.outer(mask, keep)
    return synthesis(np.where(mask, fh, 0.0), L)


def Q_zero(f, nd: Nodes):
    """The real form's operator Q(P Re f) on the grid (grid form)."""
    g = nyquist_zero(np.real(np.asarray(f)), nd.L)
    return Q_physical(g, nd)


# --------------------------------------------------------------------------
# Exact-weight reference system (Appendix B)
# --------------------------------------------------------------------------

def Q_exact(f, d, N, L, R=None, n_radial=256, return_hat=False):
    """The Galerkin system with the exact constraint and the weight functions
    integrated exactly over q-hat and sigma (|q| by n_radial-point
    Gauss-Legendre).  O(N^(3d)): tiny N."""
    f = _cgrid(f, d, N)
    R = default_R(L) if R is None else R
    Q = np.zeros_like(f)
    Qh = np.zeros_like(f)
    _check(_load().oracle_exact_system(d, N, L, R, int(n_radial), _dp(f), _dp(Q), _dp(Qh)), "exact_system")
    return (Q, Qh) if return_hat else Q
