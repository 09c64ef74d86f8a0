"""GPU parity of the Nyquist-zero real form (wke_plan_create_real) against
the oracle's Q_zero = Q(P Re f), P dropping every mode with a component
-N/2: element by element on real seeded data, in 2D and 3D, antipodal and
not, double (1e-12 relative L2) and float (1e-5); the imaginary part of the
output is exactly zero; RK4 against the oracle; the column-pass forms
against each other; and the item-slot form refused.
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


def _tol(precision):
    return F64_TOL if precision == "f64" else F32_TOL


def _eval(torch, wls, grids, precision, kind=None):
    wke = _wke()
    plan = wke.Plan([wke.desc_from_workload(w) for w in wls], precision, real=True)
    if kind is not None:
        plan.set_column_kernel(kind)
    f = plan.pack(grids)
    Q = torch.zeros_like(f)
    plan.eval_Q(f, Q)
    torch.cuda.synchronize()
    return plan, plan.unpack(Q)


SHAPES = [
    ("c1_2d_n16", wi.workload("c1_2d_n16"), lambda wl: wi.two_gaussians_c1()),
    ("c2_2d_n64", wi.workload("c2_2d_n64"), lambda wl: wi.three_bumps_2d(64, 10.0, 0)),
    ("2d_n32_odd", wi.Workload(2, 32, 7.0, 2, 3, 3, "midpoint"),
     lambda wl: wi.random_smooth(2, 32, 7.0, 11, complex_valued=False)),
    ("c4_2d_n96", wi.workload("c4_2d_n96"), lambda wl: wi.three_bumps_2d(96, 10.0, 40)),
    ("3d_n16_octa", wi.Workload(3, 16, 6.0, 2, 6, 6, "octahedron"),
     lambda wl: wi.random_smooth(3, 16, 6.0, 12, complex_valued=False)),
    ("c3_3d_n32", wi.workload("c3_3d_n32"), lambda wl: wi.aniso_gaussian_3d(32, 10.0)),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,wl,gen", SHAPES, ids=[c[0] for c in SHAPES])
def test_eval_matches_oracle(torch_cuda, name, wl, gen, precision):
    f = np.real(gen(wl))
    _announce("real eval", name, precision)
    _, (Q,) = _eval(torch_cuda, [wl], [f], precision)
    ref = oracle.Q_zero(f, oracle.nodes_for(wl))
    err = oracle.rel_l2(Q, ref)
    print("rel_l2", err)
    assert err <= _tol(precision)
    assert np.all(Q.imag == 0.0)


def test_imaginary_part_of_the_input_is_ignored(torch_cuda):
    wl = wi.workload("c2_2d_n64")
    g = wi.three_bumps_2d(64, 10.0, 1)
    _announce("real eval complex input")
    _, (Q1,) = _eval(torch_cuda, [wl], [g], "f64")
    _, (Q2,) = _eval(torch_cuda, [wl], [g + 0.3j * np.roll(g, 5)], "f64")
    assert np.array_equal(Q1, Q2)


@pytest.mark.parametrize("name,prec", [("c2_2d_n64", "f64"), ("c3_3d_n32", "f32"), ("c1_2d_n16", "f32")])
def test_column_forms_agree(torch_cuda, name, prec):
    wke = _wke()
    wl = wi.workload(name)
    f = wi.three_bumps_2d(wl.N, wl.L, 2) if wl.d == 2 else wi.aniso_gaussian_3d(wl.N, wl.L)
    _announce("real forms", name, prec)
    _, (Qa,) = _eval(torch_cuda, [wl], [f], prec, "fields")
    kinds = ["fields"]
    _, (Qh,) = _eval(torch_cuda, [wl], [f], prec, "fields_half")
    assert oracle.rel_l2(Qh, Qa) <= _tol(prec)
    kinds.append("fields_half")
    if wl.d == 2:
        try:
            _, (Qb,) = _eval(torch_cuda, [wl], [f], prec, "fused")
            assert oracle.rel_l2(Qb, Qa) <= _tol(prec)
            kinds.append("fused")
        except wke.WkeError as e:
            assert e.status == wke.WKE_ERR_UNSUPPORTED
    with pytest.raises(wke.WkeError) as e:
        _eval(torch_cuda, [wl], [f], prec, "slots")
    assert e.value.status == wke.WKE_ERR_UNSUPPORTED
    print("forms", kinds)


def _rk4_reference(f0, Qfun, dt, n):
    y = f0.copy()
    for _ in range(n):
        k1 = Qfun(y)
        k2 = Qfun(y + 0.5 * dt * k1)
        k3 = Qfun(y + 0.5 * dt * k2)
        k4 = Qfun(y + dt * k3)
        y = y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return y


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_rk4_matches_oracle(torch_cuda, precision):
    wke = _wke()
    wl = wi.workload("c1_2d_n16")
    f0 = wi.two_gaussians_c1()
    nd = oracle.nodes_for(wl)
    dt, n = 0.05, 3
    _announce("real rk4", precision)
    plan = wke.Plan([wke.desc_from_workload(wl)], precision, real=True)
    f = plan.pack([f0])
    plan.step(f, dt, n)
    torch_cuda.cuda.synchronize()
    (g,) = plan.unpack(f)
    ref = _rk4_reference(f0.real.astype(np.complex128), lambda y: oracle.Q_zero(y, nd), dt, n)
    err = oracle.rel_l2(g - f0, ref - f0)
    print("rel_l2 increment", err)
    assert err <= (1e-11 if precision == "f64" else 1e-5)
    assert np.all(g.imag == f0.imag)


def test_rk4_3d_and_split(torch_cuda):
    """3D, with the quadrature sum split over workgroups."""
    wke = _wke()
    wl = wi.Workload(3, 16, 6.0, 2, 8, 8, "cube")
    f0 = wi.random_smooth(3, 16, 6.0, 13, complex_valued=False)
    nd = oracle.nodes_for(wl)
    _announce("real rk4 3d")
    plan = wke.Plan([wke.desc_from_workload(wl)], "f64", real=True)
    plan.set_split(4)
    f = plan.pack([f0])
    plan.step(f, 1e-4, 2)       # |Q| is about 200 here, |f| about 2
    torch_cuda.cuda.synchronize()
    (g,) = plan.unpack(f)
    ref = _rk4_reference(f0, lambda y: oracle.Q_zero(y, nd), 1e-4, 2)
    assert oracle.rel_l2(g - f0, ref - f0) <= 1e-11


def test_batch_and_tuning(torch_cuda):
    wke = _wke()
    wls = [wi.workload("c4_2d_n32"), wi.workload("c4_2d_n48"), wi.workload("c4_2d_n32")]
    grids = [wi.three_bumps_2d(w.N, w.L, 20 + i) for i, w in enumerate(wls)]
    _announce("real batch")
    plan = wke.Plan([wke.desc_from_workload(w) for w in wls], "f32", real=True)
    f = plan.pack(grids)
    Q = torch_cuda.zeros_like(f)
    tuned = plan.tune(f, Q, reps=3)
    assert np.all(tuned[:, 0] >= 1)           # no item-slot form
    Q.zero_()
    plan.eval_Q(f, Q)
    torch_cuda.cuda.synchronize()
    for w, g, q in zip(wls, grids, plan.unpack(Q)):
        assert oracle.rel_l2(q, oracle.Q_zero(g, oracle.nodes_for(w))) <= F32_TOL
