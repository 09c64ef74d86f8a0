"""GPU parity on the discontinuous data of Examples 3 (2D) and 6 (3D): two
half-space Maxwellians joined across k_1 = 0, at the examples' own
quadrature sizes (N_r = N, N_s = N_sigma = 12, M = 9216 and 4608), and RK4
with their time step dt = 0.1.  The full-size checks use the oracle at
sampled grid points (direct sums per point); the float form is also checked
against the double form on the whole grid.  Tolerances: 1e-12 (double) and
1e-5 (float), relative to the largest |Q| at the sampled points.
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


def _eval(torch, wl, g, precision):
    wke = _wke()
    plan = wke.Plan([wke.desc_from_workload(wl)], precision)
    f = plan.pack([g])
    Q = torch.zeros_like(f)
    plan.eval_Q(f, Q)
    torch.cuda.synchronize()
    (q,) = plan.unpack(Q)
    plan.close()
    return q


def _sample(q, wl, rng):
    """Grid points where |Q| is largest, plus points on and beside the
    discontinuity k_1 = 0 (axis 0 index N/2 and its neighbours)."""
    top = np.argsort(np.abs(q).ravel())[::-1][:100]
    pick = list(rng.choice(top, 3, replace=False))
    N = wl.N
    rest = (N // 2 + 3,) * (wl.d - 1)
    for x0 in (N // 2 - 1, N // 2, N // 2 + 1):
        pick.append(int(np.ravel_multi_index((x0,) + rest, q.shape)))
    return np.array(pick)


@pytest.mark.parametrize("name", ["ex3_2d_n64", "ex6_3d_n32"])
def test_full_config_sampled_points(torch_cuda, name):
    wl = wi.workload(name)
    g = wi.discontinuous_ex3(wl.d, wl.N, wl.L)
    _announce(name, "f64")
    q64 = _eval(torch_cuda, wl, g, "f64")
    _announce(name, "f32")
    q32 = _eval(torch_cuda, wl, g, "f32")
    pick = _sample(q64, wl, np.random.default_rng(3))
    ref = oracle.Q_points(g, oracle.nodes_for(wl), pick)
    scale = np.max(np.abs(ref))
    e64 = np.max(np.abs(q64.ravel()[pick] - ref)) / scale
    e32 = np.max(np.abs(q32.ravel()[pick] - ref)) / scale
    print("sampled err f64 %.2e f32 %.2e; f32 vs f64 rel-L2 %.2e" % (e64, e32, oracle.rel_l2(q32, q64)))
    assert e64 <= F64_TOL
    assert e32 <= F32_TOL
    assert oracle.rel_l2(q32, q64) <= F32_TOL


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_rk4_dt_0_1_matches_oracle(torch_cuda, precision):
    """Example 3's data and time step on a reduced quadrature the oracle
    integrates in seconds: N = 32, N_r = 8, N_s = N_sigma = 6."""
    wke = _wke()
    full = wi.workload("ex3_2d_n64")
    wl = wi.Workload(2, 32, full.L, 8, 6, 6, "midpoint")
    f0 = wi.discontinuous_ex3(2, 32, wl.L)
    _announce("ex3 rk4", precision)
    plan = wke.Plan([wke.desc_from_workload(wl)], precision)
    f = plan.pack([f0])
    plan.step(f, 0.1, 3)
    torch_cuda.cuda.synchronize()
    (g,) = plan.unpack(f)
    ref = oracle.rk4(f0, oracle.nodes_for(wl), 0.1, 3)
    err = oracle.rel_l2(g - f0, ref - f0)
    print("rel_l2 increment", err)
    assert err <= (1e-11 if precision == "f64" else 1e-5)
