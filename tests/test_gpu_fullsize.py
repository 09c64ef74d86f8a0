"""GPU parity at full size, element by element on the whole grid.

Every full-size workload is compared with the oracle's grid form at every
grid point, in the launch configuration the benchmark times (the autotuner's
choice of column-pass form and work split) and in every other column-pass
form the plan can take:

* the 8-instance 3D N=64, L=12, (4,8,8) cube batch, every instance;
* the 64-instance uneven 2D batch (16 each of N = 32, 48, 64, 96), every
  instance;
* the discontinuous data of Examples 3 (2D, M = 9216) and 6 (3D, M = 4608)
  at their own quadrature sizes (Section 4, Examples 3 and 6): one
  evaluation, and two RK4 steps at the examples' dt = 0.1.

Bars: 1e-12 relative L2 for the double path and 1e-5 for the float path,
per instance over all grid points; RK4 compares the increment y - f0 at
1e-11 (double) and 1e-5 (float).  The oracle evaluations are computed once
per module (OpenMP over the host's cores: a few seconds each).
"""
import sys

import numpy as np
import pytest

import oracle
import wke_inputs as wi

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5
TOL = {"f64": F64_TOL, "f32": F32_TOL}
RK_TOL = {"f64": 1e-11, "f32": 1e-5}

_REF = {}


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


def _oracle_Q(key, i, wl, g):
    """The oracle's Q for instance i of workload key (cached per module)."""
    if (key, i) not in _REF:
        _REF[key, i] = oracle.Q_physical(g, oracle.nodes_for(wl))
    return _REF[key, i]


def _configurations(wke, plan, f, torch):
    """The tuned configuration first, then each other column-pass form the
    plan accepts, unsplit and split in two.  Yields a label per
    configuration, with the plan set to it."""
    tuned = plan.tune(f, torch.zeros_like(f), reps=3)
    _announce("tuned", tuned.tolist())
    yield "tuned"
    for kind in ("fields", "fields_half", "slots", "fused", "fused_mfma"):
        try:
            plan.set_column_kernel(kind)
        except wke.WkeError as e:
            assert e.status == wke.WKE_ERR_UNSUPPORTED
            continue
        for n in (1, 2):
            plan.set_split(n)
            yield "%s/split%d" % (kind, n)


def _check_batch(torch, key, batch, precision):
    wke = _wke()
    wls = [b[0] for b in batch]
    grids = [b[1] for b in batch]
    plan = wke.Plan([wke.desc_from_workload(w) for w in wls], precision)
    f = plan.pack(grids)
    worst = {}
    for label in _configurations(wke, plan, f, torch):
        _announce(key, precision, label)
        Q = torch.zeros_like(f)
        plan.eval_Q(f, Q)
        torch.cuda.synchronize()
        errs = [oracle.rel_l2(q, _oracle_Q(key, i, w, g))
                for i, (w, g, q) in enumerate(zip(wls, grids, plan.unpack(Q)))]
        worst[label] = max(errs)
        print(key, precision, label, "worst instance rel-L2 %.3e (instance %d)" % (max(errs), int(np.argmax(errs))),
              flush=True)
        assert max(errs) <= TOL[precision], (label, errs)
    plan.close()
    return worst


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_c5_batch_every_instance_full_grid(torch_cuda, precision):
    """3D N=64, L=12, (4,8,8) cube, 8 instances: every instance on all
    262144 grid points against the oracle."""
    _check_batch(torch_cuda, "c5", wi.c5_batch(), precision)


def test_c5_batch_float_against_double_everywhere(torch_cuda):
    """The float form against the double form of the same batch, after one
    evaluation and after five RK4 steps of dt = 1e-3."""
    wke = _wke()
    torch = torch_cuda
    batch = wi.c5_batch()
    out = {}
    for prec in ("f64", "f32"):
        _announce("c5 float vs double", prec)
        plan = wke.Plan([wke.desc_from_workload(w) for w, _ in batch], prec)
        f = plan.pack([g for _, g in batch])
        Q = torch.zeros_like(f)
        plan.eval_Q(f, Q)
        plan.step(f, 1e-3, 5)
        torch.cuda.synchronize()
        out[prec] = (plan.unpack(Q), plan.unpack(f))
        plan.close()
    for i, (_, g) in enumerate(batch):
        assert oracle.rel_l2(out["f32"][0][i], out["f64"][0][i]) <= F32_TOL
        assert oracle.rel_l2(out["f32"][1][i] - g, out["f64"][1][i] - g) <= F32_TOL


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_c4_batch_every_instance_full_grid(torch_cuda, precision):
    """64 uneven 2D instances (16 each of N = 32, 48, 64, 96) in one plan:
    every instance on its whole grid against the oracle."""
    _check_batch(torch_cuda, "c4", wi.c4_batch(), precision)


EXAMPLES = ["ex3_2d_n64", "ex6_3d_n32"]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", EXAMPLES)
def test_example_full_grid(torch_cuda, name, precision):
    wl = wi.workload(name)
    _check_batch(torch_cuda, name, [(wl, wi.discontinuous_ex3(wl.d, wl.N, wl.L))], precision)


def _oracle_rk(name, wl, g, dt, n):
    if (name, "rk", n) not in _REF:
        _REF[name, "rk", n] = oracle.rk4(g, oracle.nodes_for(wl), dt, n)
    return _REF[name, "rk", n]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", EXAMPLES)
def test_example_rk4_full_quadrature(torch_cuda, name, precision):
    """Two RK4 steps of dt = 0.1 at the example's own quadrature, against the
    oracle's RK4 (eight evaluations of its grid form), in the tuned
    configuration."""
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload(name)
    g0 = wi.discontinuous_ex3(wl.d, wl.N, wl.L)
    plan = wke.Plan([wke.desc_from_workload(wl)], precision)
    f = plan.pack([g0])
    _announce(name, "rk4", precision, plan.tune(f, torch.zeros_like(f), reps=3).tolist())
    plan.step(f, 0.1, 2)
    torch.cuda.synchronize()
    (g,) = plan.unpack(f)
    plan.close()
    ref = _oracle_rk(name, wl, g0, 0.1, 2)
    err = oracle.rel_l2(g - g0, ref - g0)
    print(name, precision, "rk4 increment rel-L2 %.3e, state rel-L2 %.3e" % (err, oracle.rel_l2(g, ref)))
    assert err <= RK_TOL[precision]
