"""Pins for the oracle's collision operator.

Each test checks the oracle against something other than itself: the
paper's weight functions G_1..G_4 summed by brute force, closed forms,
the Rayleigh-Jeans vanishing identity, symmetries, the continuous operator
and the original delta-function form of the equation.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.brute import Q_hat_bruteforce
import wke_inputs as wi

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

SMALL = [
    (2, 8, 8.0, 2, 4, 2, "midpoint"),
    (2, 6, 5.0, 2, 3, 3, "midpoint"),       # odd angle count: not antipodal
    (3, 4, 6.0, 2, 6, 6, "octahedron"),
    (3, 4, 6.0, 1, 8, 8, "cube"),
]


def _terms_scale(K):
    return sum(np.linalg.norm(k) for k in K)


@pytest.mark.parametrize("case", SMALL)
def test_physical_form_equals_double_convolution(case):
    """Fourier-space double convolution (eq. (K1_con) and K_2..K_4, cyclic)
    and the product of shifted interpolants on the grid agree term by term."""
    d, N, L, Nr, Ns, Nsig, rule = case
    nd = oracle.nodes(d, N, L, Nr, Ns, Nsig, rule)
    f = wi.random_smooth(d, N, L, 1)
    Qp, K = oracle.Q_physical(f, nd, return_terms=True)
    Qf, Qh, Kh = oracle.Q_fourier(f, nd, return_hat=True)
    assert oracle.rel_l2(Qp, Qf) < 1e-13
    for l in range(4):
        assert oracle.rel_l2(K[l], oracle.synthesis(Kh[l], L)) < 1e-13
    # the returned Q_hat is the transform of Q
    assert oracle.rel_l2(oracle.spectrum(Qf, L), Qh) < 1e-13


@pytest.mark.parametrize("case", SMALL[:3])
@pytest.mark.parametrize("linear", [False, True])
def test_double_convolution_equals_weight_function_sum(case, linear):
    """Brute-force triple sum over modes with G_1..G_4 taken from their
    printed integrands (eqs. (KK1)-(KK4)) under the quadrature of eq. (G1)."""
    d, N, L, Nr, Ns, Nsig, rule = case
    nd = oracle.nodes(d, N, L, Nr, Ns, Nsig, rule)
    f = wi.random_smooth(d, N, L, 2)
    _, Qh, Kh = oracle.Q_fourier(f, nd, linear=linear, return_hat=True)
    Qb, Kb = Q_hat_bruteforce(oracle.spectrum(f, L), nd, linear=linear)
    assert oracle.rel_l2(Qb, Qh) < 1e-13
    for l in range(4):
        assert oracle.rel_l2(Kb[l], Kh[l]) < 1e-13


@pytest.mark.parametrize("case", SMALL)
def test_constant_state_gives_zero(case):
    d, N, L, Nr, Ns, Nsig, rule = case
    nd = oracle.nodes(d, N, L, Nr, Ns, Nsig, rule)
    f = wi.constant(d, N, 1.7 - 0.3j)
    Q, K = oracle.Q_physical(f, nd, return_terms=True)
    assert np.max(np.abs(Q)) < 1e-14 * _terms_scale(K)


@pytest.mark.parametrize("d,N,j0", [(2, 8, (1, -2)), (2, 8, (-4, 3)), (3, 4, (1, 0, -2))])
def test_single_mode_closed_form(d, N, j0):
    """f = exp(i pi j0.k/L): every shifted interpolant is f exp(-i theta.s),
    theta = pi j0 / L, so Q(k_x) = 2^(1-d) f(k_x)^3 sum_p W_p [e^{-2i theta.s_a}
    - e^{-i theta.(s_a+s_c)} + e^{-i theta.s_a} - e^{-i theta.(s_a+s_b)}]."""
    L = 5.0
    rule = "midpoint" if d == 2 else "icosahedron"
    nd = oracle.nodes(d, N, L, 2, 4 if d == 2 else 12, 4 if d == 2 else 12, rule)
    f = wi.single_mode(d, N, L, j0)
    Q = oracle.Q_physical(f, nd)
    th = math.pi * np.array(j0, float) / L
    tot = 0.0 + 0j
    for p1 in range(len(nd.r)):
        for p2 in range(len(nd.ws)):
            for p3 in range(len(nd.wsig)):
                r = nd.r[p1]
                sa = r * nd.qh[p2]
                sb = 0.5 * r * (nd.qh[p2] - nd.sg[p3])
                sc = 0.5 * r * (nd.qh[p2] + nd.sg[p3])
                W = nd.wr[p1] * r ** (2 * d - 3) * nd.ws[p2] * nd.wsig[p3]
                tot += W * (np.exp(-2j * th @ sa) - np.exp(-1j * th @ (sa + sc))
                            + np.exp(-1j * th @ sa) - np.exp(-1j * th @ (sa + sb)))
    expect = 2.0 ** (1 - d) * f ** 3 * tot
    assert np.max(np.abs(Q - expect)) < 1e-12 * max(1.0, abs(tot))


def _lattice_nodes(d, N, L):
    """Nodes whose shifts s_a = r qh, s_b, s_c = r (qh -+ sigma)/2 are all
    grid vectors: qh along the axes and sigma on integer directions of the
    same length (Pythagorean triples (3,4)/5 in 2D, quadruples (1,2,2)/3 in
    3D), with r chosen so that r qh and r sigma lie in 2h Z^d.  The resulting
    rectangles k, k', k_2, k'_2 are tilted, so a periodic wrap breaks the
    Rayleigh-Jeans identity (unlike axis-aligned ones)."""
    import itertools
    h = 2 * L / N
    qh = np.concatenate([np.eye(d), -np.eye(d)])
    if d == 2:
        base, scale, r = (3, 4), 5.0, 10 * h
    else:
        base, scale, r = (1, 2, 2), 3.0, 6 * h
    sg = set()
    for perm in itertools.permutations(base):
        for signs in itertools.product((1, -1), repeat=d):
            sg.add(tuple(s * v for s, v in zip(signs, perm)))
    sg = np.array(sorted(sg), float) / scale
    ws = np.full(len(qh), 1.0)
    wsig = np.linspace(0.5, 1.5, len(sg))
    wsig = 0.5 * (wsig + wsig[::-1])           # antipodal pairs share a weight
    reach = int(round(r / h))                  # largest shift component, in cells
    return oracle.custom_nodes(d, N, L, [r], [1.0], qh, ws, sg, wsig), reach


@pytest.mark.parametrize("d,N", [(2, 32), (3, 16)])
def test_rayleigh_jeans_vanishes_on_lattice_nodes(d, N):
    """With every shift a grid vector, the interpolant at the shifted points
    is f_eq itself there, and the bracket of eq. (WKE-Boltz) vanishes for
    f_eq = 1/(mu + nu.k + xi|k|^2) (momentum and energy conservation), so Q
    is zero at every node whose shifted points do not wrap around the box.
    Fixes the maps k', k'_2, k_2 and the signs of the four terms."""
    L = 8.0
    nd, reach = _lattice_nodes(d, N, L)
    nu = (0.3, -0.2, 0.25)[:d]
    f = wi.rayleigh_jeans(d, N, L, 2.0, nu, 0.5)
    Q, K = oracle.Q_physical(f, nd, return_terms=True)
    inner = tuple(slice(reach, N - reach) for _ in range(d))
    scale = np.max(np.abs(K[0][inner]))
    assert np.max(np.abs(Q[inner])) < 1e-14 * scale
    # near the edge the periodic wrap breaks the identity (the check has teeth)
    assert np.max(np.abs(Q)) > 1e-3 * np.max(np.abs(K[0]))


@pytest.mark.parametrize("d,rule,n", [(2, "midpoint", 4), (3, "cube", 8), (3, "icosahedron", 12)])
def test_antipodal_rules_give_equal_K2_K4(d, rule, n):
    N, L = (8, 6.0) if d == 2 else (4, 6.0)
    nd = oracle.nodes(d, N, L, 2, n, n, rule)
    f = wi.random_smooth(d, N, L, 4)
    _, K = oracle.Q_physical(f, nd, return_terms=True)
    assert oracle.rel_l2(K[1], K[3]) < 1e-14


def test_homogeneity_and_translation():
    d, N, L = 2, 16, 8.0
    nd = oracle.nodes(d, N, L, 2, 4, 2, "midpoint")
    f = wi.random_smooth(d, N, L, 9)
    Q = oracle.Q_physical(f, nd)
    lam = 1.7 - 0.4j
    assert oracle.rel_l2(oracle.Q_physical(lam * f, nd), lam ** 3 * Q) < 1e-14
    # translating the samples by a grid vector translates Q (periodic box)
    sh = (3, -5)
    Qs = oracle.Q_physical(np.roll(f, sh, axis=(0, 1)), nd)
    assert oracle.rel_l2(Qs, np.roll(Q, sh, axis=(0, 1))) < 1e-13


def _continuous_Q(fun, k, R, nr, nang):
    """K^R(f)(k) of eq. (WKE-Boltz) for an analytic f in 2D, |q| <= R, by a
    fine product rule: Gauss-Legendre (numpy) in |q|, uniform angles."""
    t, w = np.polynomial.legendre.leggauss(nr)
    r = 0.5 * R * (1 + t)
    wr = 0.5 * R * w
    th = 2 * np.pi * np.arange(nang) / nang
    u = np.stack([np.cos(th), np.sin(th)], 1)
    tot = 0.0
    for i in range(nr):
        q = r[i] * u                                     # (nang, 2) values of q
        k2 = k[None, :] - q                              # k_2 = k - q
        O = 0.5 * (k[None, :] + k2)
        for jq in range(nang):
            kp = O[jq][None, :] + 0.5 * r[i] * u         # k'  for every sigma
            kp2 = O[jq][None, :] - 0.5 * r[i] * u        # k'_2
            fk, f2 = fun(k[None, :])[0], fun(k2[jq][None, :])[0]
            fp, fp2 = fun(kp), fun(kp2)
            br = fp * f2 * fp2 - fk * f2 * fp2 + fp * fk * fp2 - fp * f2 * fk
            tot += wr[i] * r[i] * (2 * np.pi / nang) * np.sum(br) * (2 * np.pi / nang)
    return 0.5 * tot


def test_converges_to_continuous_operator():
    """The discrete operator converges to K^R of eq. (WKE-Boltz) for an
    analytic Gaussian as N and the quadrature are refined (pins the weights
    w_r |q|^(2d-3) w_s w_sig, the prefactor 2^(1-d) and the interpolant)."""
    L = 10.0
    c = np.array([0.4, -0.3])
    fun = lambda k: np.exp(-np.sum((k - c) ** 2, axis=-1) / 2.0)
    R = oracle.default_R(L)
    pts = [np.array([0.0, 0.0]), np.array([1.25, -1.25])]   # nodes for N = 32, 48, 64
    ref = [_continuous_Q(fun, k, R, 40, 96) for k in pts]
    errs = []
    for N, nr, na in [(32, 6, 6), (48, 16, 16), (64, 24, 24)]:
        nd = oracle.nodes(2, N, L, nr, na, na, "midpoint")
        kx, ky = wi.grid_points(2, N, L)
        f = fun(np.stack([kx, ky], -1)) + 0j
        h = 2 * L / N
        idx = [int(round((p[0] + L) / h)) * N + int(round((p[1] + L) / h)) for p in pts]
        # the two probe points are grid nodes for these N
        for p, i in zip(pts, idx):
            assert abs(-L + h * (i // N) - p[0]) < 1e-12 and abs(-L + h * (i % N) - p[1]) < 1e-12
        val = oracle.Q_points(f, nd, idx)
        errs.append(max(abs(v - r) / abs(r) for v, r in zip(val, ref)))
    assert errs[-1] < 1e-7
    assert errs[0] > errs[-1]


@pytest.mark.parametrize("d", [2, 3])
def test_sphere_form_matches_delta_form(d):
    """Appendix A: for fixed k, k_2 the energy delta over k_3 (with k_1 from
    the momentum delta) equals 2^(1-d) |k - k_2|^(d-2) times the sphere
    integral over sigma with k_1 = k', k_3 = k'_2.  Checked by a mollified
    delta on a Cartesian k_3 grid (independent of the derivation)."""
    rng = np.random.default_rng(0)
    k = rng.uniform(-0.5, 0.5, d)
    k2 = rng.uniform(-1.5, 1.5, d)
    a = rng.uniform(-0.5, 0.5, d)
    b = rng.uniform(-0.5, 0.5, d)
    Phi = lambda k1, k3: np.exp(-np.sum((k1 - a) ** 2, -1)) * np.exp(-0.5 * np.sum((k3 - b) ** 2, -1))
    eps = 0.03 if d == 2 else 0.05
    hgrid = 0.006 if d == 2 else 0.02
    lim = 4.0
    ax = np.arange(-lim, lim, hgrid) + hgrid / 2
    if d == 2:
        K3 = np.stack(np.meshgrid(ax, ax, indexing="ij"), -1)
    else:
        K3 = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1)
    K1 = k + k2 - K3
    g = 0.5 * (np.sum(K1 ** 2, -1) - k2 @ k2 + np.sum(K3 ** 2, -1) - k @ k)
    delta = np.exp(-0.5 * (g / eps) ** 2) / (math.sqrt(2 * math.pi) * eps)
    lhs = np.sum(Phi(K1, K3) * delta) * hgrid ** d
    # sphere side, fine rule on S^{d-1}
    if d == 2:
        th = 2 * np.pi * (np.arange(2000) + 0.5) / 2000
        sig = np.stack([np.cos(th), np.sin(th)], 1)
        wsig = 2 * np.pi / 2000
    else:
        t, w = np.polynomial.legendre.leggauss(60)
        ph = 2 * np.pi * np.arange(120) / 120
        ct, P = np.meshgrid(t, ph, indexing="ij")
        st = np.sqrt(1 - ct ** 2)
        sig = np.stack([st * np.cos(P), st * np.sin(P), ct], -1).reshape(-1, 3)
        wsig = (np.repeat(w, 120) * (2 * np.pi / 120))
    O = 0.5 * (k + k2)
    rad = 0.5 * np.linalg.norm(k - k2)
    rhs = 2.0 ** (1 - d) * np.linalg.norm(k - k2) ** (d - 2) * np.sum(Phi(O + rad * sig, O - rad * sig) * wsig)
    assert abs(lhs - rhs) < 5e-3 * abs(rhs)


def _rj_ratio(d, N, L, Nr, ns, rule, mu, nu, xi):
    nd = oracle.nodes(d, N, L, Nr, ns, ns, rule)
    f = wi.rayleigh_jeans(d, N, L, mu, nu, xi)
    Q, K = oracle.Q_physical(f, nd, return_terms=True)
    return np.linalg.norm(Q) / _terms_scale(K)


def test_rayleigh_jeans_residual_trend_2d():
    """Example 1 (Tables 1 and 3): the RJ residual falls as N and as
    N_s = N_sig grow.  The paper's digits are not parity targets (its norms,
    grid offset and L are not stated); the trend is."""
    g = GOLD["ex1_rj_2d"]
    L = (3 + math.sqrt(2)) / 2 * g["S"]
    by_n = [_rj_ratio(2, N, L, N, 12, "midpoint", g["mu"], g["nu"], g["xi"]) for N in (16, 32)]
    assert by_n[1] < 0.5 * by_n[0]
    by_s = [_rj_ratio(2, 32, L, 32, s, "midpoint", g["mu"], g["nu"], g["xi"]) for s in (3, 6, 12)]
    assert by_s[0] > by_s[1] > by_s[2]
    t1 = g["table1_Linf"]
    assert t1["16"] > t1["32"] > t1["64"] > t1["128"]


def test_rayleigh_jeans_residual_trend_3d():
    g = GOLD["ex5_rj_3d"]
    L = (3 + math.sqrt(2)) / 2 * g["S"]
    a = _rj_ratio(3, 8, L, 8, 6, "octahedron", g["mu"], g["nu"], g["xi"])
    b = _rj_ratio(3, 16, L, 16, 6, "octahedron", g["mu"], g["nu"], g["xi"])
    assert b < a


def test_mass_and_energy_conserved_to_spectral_accuracy():
    """The exact-weight system conserves mass (Appendix B); the fast method
    conserves mass and energy only up to the truncation error of f_N, which
    falls spectrally as N grows at a fixed quadrature."""
    L = 10.0
    rel = []
    for N in (32, 64):
        f = wi.three_bumps_2d(N, L, 0)
        kx, ky = wi.grid_points(2, N, L)
        nd = oracle.nodes(2, N, L, 8, 8, 8, "midpoint")
        Q, K = oracle.Q_physical(f, nd, return_terms=True)
        scale = sum(np.sum(np.abs(k)) for k in K)
        rel.append((abs(np.sum(Q)) / scale, abs(np.sum(Q * (kx ** 2 + ky ** 2))) / scale))
    assert rel[1][0] < 1e-3 * rel[0][0] and rel[1][1] < 1e-3 * rel[0][1]
    assert rel[1][0] < 1e-12 and rel[1][1] < 1e-10


def test_rk4_is_fourth_order():
    """Classical RK4: halving dt cuts the global error by about 2^4."""
    d, N, L = 2, 8, 6.0
    nd = oracle.nodes(d, N, L, 2, 4, 4, "midpoint")
    f0 = wi.random_smooth(d, N, L, 3) * 0.3
    T = 0.2
    ref = oracle.rk4(f0, nd, T / 256, 256)
    e = [np.linalg.norm(oracle.rk4(f0, nd, T / n, n) - ref) for n in (8, 16)]
    assert np.linalg.norm(ref - f0) > 1e-2          # the state really moves
    assert 14.0 < e[0] / e[1] < 18.5


GALERKIN = [
    wi.Workload(2, 8, 8.0, 2, 4, 2, "midpoint"),
    wi.Workload(2, 12, 6.0, 2, 3, 3, "midpoint"),     # odd angle count: not antipodal
    wi.Workload(3, 4, 6.0, 1, 6, 6, "octahedron"),
]


@pytest.mark.parametrize("wl", GALERKIN, ids=lambda w: "d%d_N%d_%d_%d_%d" % (w.d, w.N, w.Nr, w.Ns, w.Nsig))
def test_exact_galerkin_is_cyclic_on_twice_the_grid(wl):
    """The exact constraint l + m + n = j (the oracle's linear mode, itself
    pinned to the weight-function brute force above) equals the cyclic
    operator on 2N points of the sampled series, projected back onto
    [-N/2, N/2-1]; with 3N/2 points the wrapped modes alias into the box."""
    f = wi.random_smooth(wl.d, wl.N, wl.L, 5)
    nd = oracle.nodes(wl.d, wl.N, wl.L, wl.Nr, wl.Ns, wl.Nsig, wl.rule)
    lin = oracle.Q_fourier(f, nd, linear=True)
    assert oracle.rel_l2(oracle.Q_galerkin(f, wl), lin) < 1e-13
    assert oracle.rel_l2(oracle.Q_galerkin(f, wl, P=3 * wl.N // 2), lin) > 1e-6
    # and the cyclic operator on N points differs from both
    assert oracle.rel_l2(oracle.Q_fourier(f, nd), lin) > 1e-6


@pytest.mark.parametrize("wl", [wi.Workload(2, 12, 6.0, 2, 3, 3, "midpoint"),
                                wi.Workload(2, 12, 6.0, 2, 6, 6, "midpoint"),
                                wi.Workload(3, 6, 6.0, 1, 6, 6, "octahedron")],
                         ids=lambda w: "d%d_N%d_%d_%d_%d" % (w.d, w.N, w.Nr, w.Ns, w.Nsig))
def test_exact_galerkin_conserves_mass_when_rules_coincide(wl):
    """Appendix B: with the exact constraint the zeroth mode of the operator
    vanishes (the weak form with test function 1 cancels under the exchange
    of (k, k_2) with (k', k'_2)).  Under the quadrature of eq. (G1) that
    exchange swaps q-hat and sigma, so the cancellation survives when both
    use the same rule.  The cyclic constraint breaks it (wrapped modes)."""
    f = wi.random_smooth(wl.d, wl.N, wl.L, 8)
    nd = oracle.nodes_for(wl)
    _, Qh, _ = oracle.Q_fourier(f, nd, linear=True, return_hat=True)
    assert abs(Qh.flat[0]) <= 1e-13 * np.abs(Qh).sum()
    _, Qc, _ = oracle.Q_fourier(f, nd, return_hat=True)
    assert abs(Qc.flat[0]) > 1e-6 * np.abs(Qc).sum()


REAL_CASES = [
    wi.Workload(2, 8, 8.0, 2, 4, 2, "midpoint"),
    wi.Workload(2, 6, 5.0, 2, 3, 3, "midpoint"),     # not antipodal
    wi.Workload(3, 4, 6.0, 1, 8, 8, "cube"),
]


@pytest.mark.parametrize("wl", REAL_CASES, ids=lambda w: "d%d_N%d_%d_%d_%d" % (w.d, w.N, w.Nr, w.Ns, w.Nsig))
def test_nyquist_zero_form(wl):
    """Real form Q(P Re f): real for real data (every kept mode has its
    partner -j, so each shifted field is real), equal to Q on data without
    the dropped modes, zero on data made only of them, and equal to the
    brute-force weight-function sums on the masked spectrum.  Keeping the
    -N/2 modes (the plain operator) gives complex output for real data."""
    nd = oracle.nodes(wl.d, wl.N, wl.L, wl.Nr, wl.Ns, wl.Nsig, wl.rule)
    f = wi.random_smooth(wl.d, wl.N, wl.L, 9, complex_valued=False)
    Qz = oracle.Q_zero(f, nd)
    assert np.abs(Qz.imag).max() <= 1e-14 * np.abs(Qz).max()
    Qk = oracle.Q_physical(f, nd)
    assert np.abs(Qk.imag).max() > 1e-8 * np.abs(Qk).max()
    g = oracle.nyquist_zero(f, wl.L)
    assert oracle.rel_l2(oracle.Q_physical(g, nd), Qz) < 1e-14
    assert oracle.rel_l2(oracle.nyquist_zero(g, wl.L), g) < 1e-14
    # data made only of the dropped modes: (-1)^(x_0) times anything along the other axes
    alt = (f - g).real
    assert np.abs(oracle.Q_zero(alt, nd)).max() <= 1e-13 * np.abs(alt).max() ** 3
    if wl.d == 2:
        fh = oracle.spectrum(g, wl.L)
        Qb, _ = Q_hat_bruteforce(fh, nd)
        assert oracle.rel_l2(oracle.synthesis(Qb, wl.L), Qz) < 1e-13


def test_trivial_collisions_cancel():
    """With sigma = +-q-hat the collision partners coincide with the incoming
    pair (s_b = 0, s_c = s_a, or the reverse), so b c (a + F0) - F0 a (b + c)
    vanishes term by term: Q = 0 to rounding for (N_r, N_s, N_sigma) = (1,1,1)
    and (1,2,2) (the midpoint rules put sigma on +-q-hat), while the terms
    themselves do not."""
    for q in [(1, 1, 1), (1, 2, 2), (2, 1, 1)]:
        nd = oracle.nodes(2, 8, 8.0, *q, "midpoint")
        f = wi.random_smooth(2, 8, 8.0, 31)
        Q, K = oracle.Q_physical(f, nd, return_terms=True)
        assert np.abs(Q).max() <= 1e-14 * np.abs(K[0]).max()
        assert np.abs(K[0]).max() > 1e-3
