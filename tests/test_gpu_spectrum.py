"""GPU parity of the Fourier-coefficient output (wke_eval_Q_hat): Q_hat from
the GPU against the oracle's coefficients of the oracle's Q (the series of
eq. (fj), FFT index order), elementwise; for the exact-Galerkin plan also
against the oracle's linear double-convolution sums of Section 3 (eq. (KK1)
with l + m + n = j kept exactly); and the round trip back to the grid.
"""
import sys

import numpy as np
import pytest

import oracle
import wke_inputs as wi

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _wke():
    import paper_2503_12805_amd as wke
    wke.load_library()
    return wke


def _announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _grid(wl, seed):
    if wl.d == 2:
        return wi.three_bumps_2d(wl.N, wl.L, seed)
    return wi.random_smooth(3, wl.N, wl.L, seed)


def _max_rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _hat_and_grid(torch, wls, grids, precision, **kw):
    wke = _wke()
    plan = wke.Plan([wke.desc_from_workload(w) for w in wls], precision, **kw)
    f = plan.pack(grids)
    Qh = torch.zeros_like(f)
    Q = torch.zeros_like(f)
    plan.eval_Q_hat(f, Qh)
    plan.eval_Q(f, Q)
    torch.cuda.synchronize()
    out = plan.unpack(Qh), plan.unpack(Q)
    plan.close()
    return out


SHAPES = [
    ("c1_2d_n16", "f64", wi.workload("c1_2d_n16")),
    ("c1_2d_n16", "f32", wi.workload("c1_2d_n16")),
    ("c2_2d_n64", "f64", wi.workload("c2_2d_n64")),
    ("2d_n96", "f64", wi.workload("c4_2d_n96")),
    ("3d_n16", "f64", wi.Workload(3, 16, 6.0, 2, 6, 6, "octahedron")),
    ("3d_n32", "f32", wi.workload("c3_3d_n32")),
]


@pytest.mark.parametrize("name,prec,wl", SHAPES, ids=[s[0] + "_" + s[1] for s in SHAPES])
def test_q_hat_matches_oracle(torch_cuda, name, prec, wl):
    g = _grid(wl, 4)
    _announce("q_hat", name, prec)
    (qh,), (q,) = _hat_and_grid(torch_cuda, [wl], [g], prec)
    ref = oracle.spectrum(oracle.Q_physical(g, oracle.nodes_for(wl)), wl.L)
    err = _max_rel(qh, ref)
    print("max rel", err)
    assert err <= (F64_TOL if prec == "f64" else F32_TOL)
    # the coefficients resum to the grid values the plan gives directly
    assert _max_rel(oracle.synthesis(qh, wl.L), q) <= (1e-13 if prec == "f64" else 1e-6)


def test_q_hat_batch_of_sizes(torch_cuda):
    """Packed instances of different N: each instance's coefficients."""
    wls = [wi.workload("c4_2d_n32"), wi.workload("c4_2d_n48"), wi.workload("c1_2d_n16")]
    grids = [_grid(w, 9 + k) for k, w in enumerate(wls)]
    _announce("q_hat batch")
    qhs, _ = _hat_and_grid(torch_cuda, wls, grids, "f64")
    for w, g, qh in zip(wls, grids, qhs):
        ref = oracle.spectrum(oracle.Q_physical(g, oracle.nodes_for(w)), w.L)
        assert _max_rel(qh, ref) <= F64_TOL


def test_q_hat_exact_constraint(torch_cuda):
    """The exact-Galerkin plan's coefficients are the linear sums of
    eq. (KK1) (no wrap-around), modes [-N/2, N/2-1]."""
    wl = wi.Workload(2, 16, 8.0, 2, 4, 4, "midpoint")
    g = _grid(wl, 6)
    _announce("q_hat galerkin")
    (qh,), _ = _hat_and_grid(torch_cuda, [wl], [g], "f64", galerkin=True)
    _, ref, _ = oracle.Q_fourier(g, oracle.nodes_for(wl), linear=True, return_hat=True)
    assert _max_rel(qh, ref) <= F64_TOL
    _, cyc, _ = oracle.Q_fourier(g, oracle.nodes_for(wl), return_hat=True)
    assert _max_rel(qh, cyc) > 1e-6          # the cyclic sums differ


def test_q_hat_real_form(torch_cuda):
    """Nyquist-zero real form: the coefficients of the oracle's Q_zero."""
    wl = wi.workload("c1_2d_n16")
    g = _grid(wl, 2).real.astype(np.complex128)
    _announce("q_hat real form")
    (qh,), _ = _hat_and_grid(torch_cuda, [wl], [g], "f64", real=True)
    ref = oracle.spectrum(oracle.Q_zero(g, oracle.nodes_for(wl)), wl.L)
    assert _max_rel(qh, ref) <= F64_TOL
