"""Brute-force evaluation of the discrete operator from the paper's weight
functions G_1..G_4 (TEST INFRASTRUCTURE ONLY; tiny N).

Section 3.2 writes each Galerkin term as a weighted triple sum over modes,
  K_hat_{l,j} = sum_{l + m + n = j} G_l(...) f_hat_l f_hat_m f_hat_n,
(eqs. (KK1)-(KK4)), with G_1(l,m,n), G_2(m,n), G_3(l,n), G_4(l,m) given as
integrals over the ball B_R and the sphere.  Here each G is evaluated from
its own printed integrand with the integrals over |q|, q-hat and sigma
replaced by the same quadrature nodes that the fast method uses (eq. (G1)),
and the triple sum is taken literally, O(M N^(3d)).  Nothing here goes
through the shift factorisation alpha/beta/gamma, so it independently checks
the double-convolution form of the oracle.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _modes(N):
    return [i if i < N // 2 else i - N for i in range(N)]


def Q_hat_bruteforce(fhat, nd, linear=False):
    """Returns (Q_hat, [K_hat_1..K_hat_4]) in FFT index order.  cyclic: the
    constraint l + m + n = j is taken mod N (what size-N transforms compute);
    linear: exactly, as in eq. (KK1)."""
    d, N, L = nd.d, nd.N, nd.L
    fhat = np.asarray(fhat, dtype=np.complex128)
    modes = _modes(N)
    allj = list(itertools.product(range(N), repeat=d))           # slots
    sj = np.array([[modes[i] for i in s] for s in allj], dtype=np.float64)  # signed modes
    n = len(allj)
    fvec = np.array([fhat[s] for s in allj])
    # quadrature triples
    trip = []
    for p1 in range(len(nd.r)):
        for p2 in range(len(nd.ws)):
            for p3 in range(len(nd.wsig)):
                W = nd.wr[p1] * nd.r[p1] ** (2 * d - 3) * nd.ws[p2] * nd.wsig[p3]
                trip.append((W, nd.r[p1] * nd.qh[p2], nd.r[p1] * nd.sg[p3]))
    c = math.pi / L
    # G evaluated on all (l, m, n) of the mode box: arrays of shape (n, n, n)
    L_ = sj[:, None, None, :]
    M_ = sj[None, :, None, :]
    N_ = sj[None, None, :, :]
    G1 = np.zeros((n, n, n), dtype=np.complex128)
    G2 = np.zeros((n, n), dtype=np.complex128)   # (m, n)
    G3 = np.zeros((n, n), dtype=np.complex128)   # (l, n)
    G4 = np.zeros((n, n), dtype=np.complex128)   # (l, m)
    for W, q, rs in trip:
        # G_1: exp(-i pi/L (2m + l + n).q / 2) exp(+i pi/L |q| (l - n).sigma / 2)
        G1 += W * np.exp(-1j * c * 0.5 * ((2 * M_ + L_ + N_) @ q)) * np.exp(1j * c * 0.5 * ((L_ - N_) @ rs))
        # G_2: exp(-i pi/L (2m + n).q / 2) exp(-i pi/L |q| n.sigma / 2)
        mm, nn = sj[:, None, :], sj[None, :, :]
        G2 += W * np.exp(-1j * c * 0.5 * ((2 * mm + nn) @ q)) * np.exp(-1j * c * 0.5 * (nn @ rs))
        # G_3: exp(-i pi/L (l + n).q / 2) exp(+i pi/L |q| (l - n).sigma / 2)
        ll = sj[:, None, :]
        G3 += W * np.exp(-1j * c * 0.5 * ((ll + nn) @ q)) * np.exp(1j * c * 0.5 * ((ll - nn) @ rs))
        # G_4: exp(-i pi/L (2m + l).q / 2) exp(+i pi/L |q| l.sigma / 2)
        G4 += W * np.exp(-1j * c * 0.5 * ((2 * nn + ll) @ q)) * np.exp(1j * c * 0.5 * (ll @ rs))
    # note: G4 is indexed (l, m): row = l (ll), column = m (nn above)
    index = {tuple(int(v) for v in s): k for k, s in enumerate(sj)}
    K = [np.zeros(n, dtype=np.complex128) for _ in range(4)]
    half = N // 2
    for jk, jv in enumerate(sj):
        for lk in range(n):
            for mk in range(n):
                nv = jv - sj[lk] - sj[mk]
                if linear:
                    if np.any(nv < -half) or np.any(nv > half - 1):
                        continue
                else:
                    nv = (nv + half) % N - half
                nk = index[tuple(int(v) for v in nv)]
                prod = fvec[lk] * fvec[mk] * fvec[nk]
                K[0][jk] += G1[lk, mk, nk] * prod
                K[1][jk] += G2[mk, nk] * prod
                K[2][jk] += G3[lk, nk] * prod
                K[3][jk] += G4[lk, mk] * prod
    Kh = []
    for kv in K:
        a = np.zeros((N,) * d, dtype=np.complex128)
        for k, s in enumerate(allj):
            a[s] = kv[k]
        Kh.append(a)
    Qh = 2.0 ** (1 - d) * (Kh[0] - Kh[1] + Kh[2] - Kh[3])
    return Qh, Kh
