"""GPU parity: the HIP path (through the C interface) against the CPU oracle,
element by element on the same seeded inputs.

Tolerances: the plain double path must match the oracle to 1e-12 relative
L2; the float path to 1e-5 relative L2 (the targets stated for the two
forms).  For near-equilibrium inputs, where Q nearly vanishes, the error is
normalised by the sum of the four term norms instead.
"""
import math
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


def _eval(torch, wls, grids, precision):
    wke = _wke()
    plan = wke.Plan([wke.desc_from_workload(w) for w in wls], precision)
    f = plan.pack(grids)
    Q = torch.zeros_like(f)
    plan.eval_Q(f, Q)
    torch.cuda.synchronize()
    return plan, plan.unpack(Q)


def _oracle_Q(wl, f):
    return oracle.Q_physical(f, oracle.nodes_for(wl))


CASES_2D = [
    ("c1_2d_n16", lambda wl: wi.two_gaussians_c1(wl.N, wl.L)),
    ("c2_2d_n64", lambda wl: wi.three_bumps_2d(wl.N, wl.L, 0)),
    ("c4_2d_n32", lambda wl: wi.three_bumps_2d(wl.N, wl.L, 3)),
    ("c4_2d_n48", lambda wl: wi.three_bumps_2d(wl.N, wl.L, 17)),
    ("c4_2d_n96", lambda wl: wi.three_bumps_2d(wl.N, wl.L, 40)),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,gen", CASES_2D, ids=[c[0] for c in CASES_2D])
def test_eval_2d_matches_oracle(torch_cuda, name, gen, precision):
    wl = wi.workload(name)
    f = gen(wl)
    _announce("eval", name, precision)
    _, (Q,) = _eval(torch_cuda, [wl], [f], precision)
    ref = _oracle_Q(wl, f)
    err = oracle.rel_l2(Q, ref)
    print("rel_l2", err)
    assert err <= (F64_TOL if precision == "f64" else F32_TOL)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_eval_c1_matches_double_convolution(torch_cuda, precision):
    """C1 against the Fourier-space double convolution itself (not only the
    equivalent grid form)."""
    wl = wi.workload("c1_2d_n16")
    f = wi.two_gaussians_c1()
    _announce("c1 vs fourier", precision)
    _, (Q,) = _eval(torch_cuda, [wl], [f], precision)
    ref = oracle.Q_fourier(f, oracle.nodes_for(wl))
    assert oracle.rel_l2(Q, ref) <= (F64_TOL if precision == "f64" else F32_TOL)


SMALL_SHAPES = [
    wi.Workload(2, 16, 6.0, 3, 3, 3, "midpoint"),      # odd angle count: separate b and c fields
    wi.Workload(2, 32, 7.0, 1, 2, 6, "midpoint"),
    wi.Workload(2, 128, 10.0, 1, 4, 4, "midpoint"),
    wi.Workload(3, 16, 6.0, 2, 6, 6, "octahedron"),
    wi.Workload(3, 16, 6.0, 1, 8, 8, "cube"),
    wi.Workload(3, 16, 6.0, 1, 12, 12, "icosahedron"),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("wl", SMALL_SHAPES, ids=lambda w: "d%d_N%d_%s_%d_%d_%d" % (w.d, w.N, w.rule, w.Nr, w.Ns, w.Nsig))
def test_eval_shapes_match_oracle(torch_cuda, wl, precision):
    f = wi.random_smooth(wl.d, wl.N, wl.L, 21)
    _announce("eval shape", wl, precision)
    _, (Q,) = _eval(torch_cuda, [wl], [f], precision)
    err = oracle.rel_l2(Q, _oracle_Q(wl, f))
    print("rel_l2", err)
    assert err <= (F64_TOL if precision == "f64" else F32_TOL)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_eval_c3_3d_n32(torch_cuda, precision):
    wl = wi.workload("c3_3d_n32")
    f = wi.aniso_gaussian_3d(wl.N, wl.L)
    _announce("eval c3", precision)
    _, (Q,) = _eval(torch_cuda, [wl], [f], precision)
    err = oracle.rel_l2(Q, _oracle_Q(wl, f))
    print("rel_l2", err)
    assert err <= (F64_TOL if precision == "f64" else F32_TOL)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_eval_c3_rayleigh_jeans_profile(torch_cuda, precision):
    """The 1/(1+|k|^2) check profile: Q is small, so the error is measured
    against the sum of the four term norms."""
    wl = wi.workload("c3_3d_n32")
    f = wi.rj_profile(3, wl.N, wl.L)
    _announce("eval c3 rj", precision)
    _, (Q,) = _eval(torch_cuda, [wl], [f], precision)
    ref, K = oracle.Q_physical(f, oracle.nodes_for(wl), return_terms=True)
    scale = sum(np.linalg.norm(k) for k in K) * 2.0 ** (1 - wl.d)
    err = np.linalg.norm(Q - ref) / scale
    print("err/sumK", err, "relQ", oracle.rel_l2(Q, ref))
    assert err <= (F64_TOL if precision == "f64" else F32_TOL)


def test_gpu_quadrature_matches_oracle(torch_cuda):
    wke = _wke()
    for wl in [wi.workload("c2_2d_n64"), wi.workload("c3_3d_n32"), SMALL_SHAPES[0], SMALL_SHAPES[3],
               SMALL_SHAPES[5], wi.Workload(2, 64, 10.0, 64, 12, 12, "midpoint")]:
        _announce("nodes", wl)
        plan = wke.Plan([wke.desc_from_workload(wl)], "f64")
        r, wr, qh, ws, sg, wsig = plan.nodes(0)
        nd = oracle.nodes_for(wl)
        assert np.max(np.abs(r - nd.r)) < 1e-14 * max(1, nd.r.max())
        assert np.max(np.abs(wr - nd.wr)) < 1e-13 * max(1, nd.wr.max())
        # the oracle rounds the angle (2i+1) pi / n before cos/sin, the GPU
        # evaluates sincospi((2i+1)/n): a few ulps of the angle apart
        assert np.max(np.abs(qh - nd.qh)) < 4e-15 and np.max(np.abs(sg - nd.sg)) < 4e-15
        assert np.max(np.abs(ws - nd.ws)) < 1e-15 and np.max(np.abs(wsig - nd.wsig)) < 1e-15
        plan.close()


def test_batch_of_uneven_sizes_matches_single_evals(torch_cuda):
    """A packed batch with different N gives, per instance, exactly what the
    single-instance plan gives, and matches the oracle."""
    wls = [wi.workload("c4_2d_n32"), wi.workload("c4_2d_n64"), wi.workload("c4_2d_n48"),
           wi.workload("c4_2d_n32"), wi.workload("c4_2d_n96")]
    grids = [wi.three_bumps_2d(w.N, w.L, s) for s, w in enumerate(wls)]
    for precision in ("f64", "f32"):
        _announce("batch", precision)
        _, Qs = _eval(torch_cuda, wls, grids, precision)
        for w, g, Q in zip(wls, grids, Qs):
            _, (Q1,) = _eval(torch_cuda, [w], [g], precision)
            # the split of the quadrature sum over workgroups depends on the
            # batch, so equality is to rounding, not bitwise
            assert oracle.rel_l2(Q, Q1) < (1e-14 if precision == "f64" else 1e-6)
            assert oracle.rel_l2(Q, _oracle_Q(w, g)) <= (F64_TOL if precision == "f64" else F32_TOL)


@pytest.mark.parametrize("kind", ["fused", "slots", "fields_half", "fused_mfma"])
def test_batch_in_each_column_form(torch_cuda, kind):
    """A packed batch of different N in the fused, the item-slot and the
    half-round field-parallel column forms (per-instance tables and offsets)
    matches the oracle per instance, for one evaluation and for two RK4
    steps."""
    wke = _wke()
    torch = torch_cuda
    wls = [wi.workload("c4_2d_n32"), wi.workload("c4_2d_n64"), wi.workload("c4_2d_n48"), wi.workload("c4_2d_n32")]
    grids = [wi.three_bumps_2d(w.N, w.L, 7 + s) for s, w in enumerate(wls)]
    for precision in ("f64", "f32"):
        _announce("batch form", kind, precision)
        plan = wke.Plan([wke.desc_from_workload(w) for w in wls], precision)
        plan.set_column_kernel(kind)
        f = plan.pack(grids)
        Q = torch.zeros_like(f)
        plan.eval_Q(f, Q)
        y = f.clone()
        plan.step(y, 1e-3, 2)
        torch.cuda.synchronize()
        tol = F64_TOL if precision == "f64" else F32_TOL
        for w, g, q, yy in zip(wls, grids, plan.unpack(Q), plan.unpack(y)):
            assert oracle.rel_l2(q, _oracle_Q(w, g)) <= tol
            ref = oracle.rk4(g, oracle.nodes_for(w), 1e-3, 2)
            assert oracle.rel_l2(yy - g, ref - g) <= (1e-11 if precision == "f64" else 1e-5)
        plan.close()


def test_repeat_runs_are_bitwise_identical(torch_cuda):
    wke = _wke()
    torch = torch_cuda
    for name, prec in [("c2_2d_n64", "f32"), ("c3_3d_n32", "f32"), ("c2_2d_n64", "f64")]:
        wl = wi.workload(name)
        f0 = wi.three_bumps_2d(wl.N, wl.L, 0) if wl.d == 2 else wi.aniso_gaussian_3d(wl.N, wl.L)
        _announce("determinism", name, prec)
        plan = wke.Plan([wke.desc_from_workload(wl)], prec)
        f = plan.pack([f0])
        Q1 = torch.zeros_like(f)
        Q2 = torch.zeros_like(f)
        plan.eval_Q(f, Q1)
        plan.eval_Q(f, Q2)
        torch.cuda.synchronize()
        assert torch.equal(Q1, Q2)


def test_constant_state_gives_zero(torch_cuda):
    wl = wi.workload("c2_2d_n64")
    f = wi.constant(2, wl.N, 0.8 + 0.1j)
    _announce("constant")
    _, (Q,) = _eval(torch_cuda, [wl], [f], "f64")
    _, K = oracle.Q_physical(f, oracle.nodes_for(wl), return_terms=True)
    assert np.max(np.abs(Q)) < 1e-13 * np.max(np.abs(K[0]))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_rk4_steps_match_oracle(torch_cuda, precision):
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload("c1_2d_n16")
    f0 = wi.two_gaussians_c1()
    nd = oracle.nodes_for(wl)
    dt, n = 0.05, 4
    _announce("rk4", precision)
    plan = wke.Plan([wke.desc_from_workload(wl)], precision)
    f = plan.pack([f0])
    plan.step(f, dt, n)
    torch.cuda.synchronize()
    (g,) = plan.unpack(f)
    ref = oracle.rk4(f0, nd, dt, n)
    err = oracle.rel_l2(g - f0, ref - f0)        # error of the increment
    print("rel_l2 increment", err)
    assert err <= (1e-11 if precision == "f64" else 1e-5)


def test_rk4_c2_shape_matches_oracle(torch_cuda):
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload("c2_2d_n64")
    f0 = wi.three_bumps_2d(wl.N, wl.L, 0)
    nd = oracle.nodes_for(wl)
    _announce("rk4 c2")
    plan = wke.Plan([wke.desc_from_workload(wl)], "f64")
    f = plan.pack([f0])
    plan.step(f, 1e-3, 3)
    torch.cuda.synchronize()
    (g,) = plan.unpack(f)
    ref = oracle.rk4(f0, nd, 1e-3, 3)
    assert oracle.rel_l2(g - f0, ref - f0) <= 1e-11
    assert oracle.rel_l2(g, ref) <= 1e-13


def test_step_in_chunks_equals_one_call(torch_cuda):
    """Resuming from a saved state: 2 x 3 steps equal 6 steps bitwise."""
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload("c2_2d_n64")
    f0 = wi.three_bumps_2d(wl.N, wl.L, 1)
    plan = wke.Plan([wke.desc_from_workload(wl)], "f32")
    a = plan.pack([f0])
    b = plan.pack([f0])
    _announce("chunks")
    plan.step(a, 1e-3, 6)
    plan.step(b, 1e-3, 3)
    saved = b.clone()
    plan.step(saved, 1e-3, 3)
    torch.cuda.synchronize()
    assert torch.equal(a, saved)


def test_moments_match_oracle(torch_cuda):
    wke = _wke()
    for wl, g in [(wi.workload("c2_2d_n64"), wi.three_bumps_2d(64, 10.0, 0)),
                  (wi.workload("c3_3d_n32"), wi.aniso_gaussian_3d(32, 10.0)),
                  (wi.Workload(2, 64, 10.0, 1, 2, 2, "midpoint"), wi.discontinuous_ex3(2, 64, 10.0))]:
        _announce("moments", wl)
        plan = wke.Plan([wke.desc_from_workload(wl)], "f64")
        f = plan.pack([g + 0.01j * np.roll(g.real, 3)])
        m = plan.moments(f)[0]
        ref = oracle.moments(g + 0.01j * np.roll(g.real, 3), wl.L)
        d = wl.d
        assert abs(m[0] - ref[0]) < 1e-13 * abs(ref[0])
        assert abs(m[1] - ref[1]) < 1e-13 * abs(ref[1])
        for a in range(d):
            assert abs(m[2 + a] - ref[2 + a]) < 1e-12 * abs(ref[0])
        assert m[5] == ref[2 + d]


def test_moments_flag_nonfinite(torch_cuda):
    wke = _wke()
    wl = wi.workload("c1_2d_n16")
    g = wi.two_gaussians_c1()
    g[3, 4] = np.nan
    plan = wke.Plan([wke.desc_from_workload(wl)], "f64")
    f = plan.pack([g])
    with pytest.raises(wke.WkeError) as e:
        plan.moments(f)
    assert e.value.status == wke.WKE_ERR_NONFINITE


def test_c5_full_size_sampled_points(torch_cuda):
    """3D N=64, L=12, (4,8,8), batch of 8: float path against the oracle at
    sampled grid points (the oracle evaluates each point by direct sums), and
    against the double GPU path everywhere."""
    import torch
    wke = _wke()
    batch = wi.c5_batch()
    wls = [b[0] for b in batch]
    grids = [b[1] for b in batch]
    _announce("c5 f64")
    _, Q64 = _eval(torch, wls, grids, "f64")
    _announce("c5 f32")
    _, Q32 = _eval(torch, wls, grids, "f32")
    rng = np.random.default_rng(5)
    for i in (0, 5):
        wl, g = wls[i], grids[i]
        nd = oracle.nodes_for(wl)
        # points near the bumps, where Q is not negligible
        flat = np.argsort(np.abs(Q64[i]).ravel())[::-1][:200]
        pick = rng.choice(flat, 3, replace=False)
        ref = oracle.Q_points(g, nd, pick)
        got64 = Q64[i].ravel()[pick]
        got32 = Q32[i].ravel()[pick]
        assert np.max(np.abs(got64 - ref)) <= F64_TOL * np.max(np.abs(ref))
        assert np.max(np.abs(got32 - ref)) <= F32_TOL * np.max(np.abs(ref))
    for i in range(8):
        assert oracle.rel_l2(Q32[i], Q64[i]) <= F32_TOL


def test_tuning_changes_only_rounding(torch_cuda):
    """The autotuner picks a work split; results stay within rounding of the
    untuned plan and within tolerance of the oracle."""
    wke = _wke()
    torch = torch_cuda
    for name, prec in [("c2_2d_n64", "f64"), ("c3_3d_n32", "f32"), ("c4_2d_n96", "f64")]:
        wl = wi.workload(name)
        g = wi.three_bumps_2d(wl.N, wl.L, 2) if wl.d == 2 else wi.aniso_gaussian_3d(wl.N, wl.L)
        _announce("tune", name, prec)
        plan = wke.Plan([wke.desc_from_workload(wl)], prec)
        f = plan.pack([g])
        Q0 = torch.zeros_like(f)
        plan.eval_Q(f, Q0)
        choice = plan.tune(f, torch.zeros_like(f), reps=3)
        print("tuned", choice)
        Q1 = torch.zeros_like(f)
        plan.eval_Q(f, Q1)
        torch.cuda.synchronize()
        (q0,), (q1,) = plan.unpack(Q0), plan.unpack(Q1)
        assert oracle.rel_l2(q1, q0) < (1e-14 if prec == "f64" else 1e-6)
        assert oracle.rel_l2(q1, _oracle_Q(wl, g)) <= (F64_TOL if prec == "f64" else F32_TOL)


def test_tuned_c5_batch_matches_untuned(torch_cuda):
    """3D N=64 float, batch of 8: the tuned evaluation (column-pass form and
    split) agrees with the untuned one to rounding, instance by instance."""
    wke = _wke()
    torch = torch_cuda
    batch = wi.c5_batch()
    _announce("tune c5 f32")
    plan = wke.Plan([wke.desc_from_workload(b[0]) for b in batch], "f32")
    f = plan.pack([b[1] for b in batch])
    Q0 = torch.zeros_like(f)
    plan.eval_Q(f, Q0)
    choice = plan.tune(f, torch.zeros_like(f), reps=3)
    print("tuned", choice)
    Q1 = torch.zeros_like(f)
    plan.eval_Q(f, Q1)
    torch.cuda.synchronize()
    for q0, q1 in zip(plan.unpack(Q0), plan.unpack(Q1)):
        assert oracle.rel_l2(q1, q0) < 1e-6
    plan.close()


@pytest.mark.parametrize("name,prec", [("c2_2d_n64", "f64"), ("c3_3d_n32", "f32")])
def test_graph_replay_matches_direct_launches(torch_cuda, name, prec):
    """wke_step replays a captured RK4 step; every replay, interleaved with
    other eager work and synchronisations, must equal direct launches."""
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload(name)
    g = wi.three_bumps_2d(wl.N, wl.L, 3) if wl.d == 2 else wi.aniso_gaussian_3d(wl.N, wl.L)
    pg = wke.Plan([wke.desc_from_workload(wl)], prec)
    pg.set_graphs(True)
    pe = wke.Plan([wke.desc_from_workload(wl)], prec)
    pe.set_graphs(False)
    a = pg.pack([g])
    b = pe.pack([g])
    _announce("graph", name, prec)
    for call in range(3):
        pg.step(a, 1e-3, 2)
        pe.step(b, 1e-3, 2)
        Q = torch.zeros_like(a)
        pg.eval_Q(a, Q)                 # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(a, b), "replay %d differs" % call
    # a new dt re-captures
    pg.step(a, 2e-3, 1)
    pe.step(b, 2e-3, 1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("form", ["fused", "fused_mfma"])
def test_single_instance_fused_matches_batched(torch_cuda, prec, form):
    """A single-instance plan with one item group runs the fused column pass
    in its single-instance variant (the task built from the kernel arguments,
    the descriptor requested at once); the same instance as the first of a
    batch of two runs the general variant.  Evaluations and RK4 steps are
    bitwise the same, and the evaluation matches the oracle."""
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload("c2_2d_n64")
    g0, g1 = wi.three_bumps_2d(wl.N, wl.L, 0), wi.three_bumps_2d(wl.N, wl.L, 5)
    d = wke.desc_from_workload(wl)
    p1 = wke.Plan([d], prec, stream=torch.cuda.current_stream())
    p2 = wke.Plan([d, d], prec, stream=torch.cuda.current_stream())
    for p in (p1, p2):
        p.set_column_kernel(form)
        p.set_split(1)
    _announce("single instance against batched", prec, form)
    a, b = p1.pack([g0]), p2.pack([g0, g1])
    Qa, Qb = torch.zeros_like(a), torch.zeros_like(b)
    p1.eval_Q(a, Qa)
    p2.eval_Q(b, Qb)
    torch.cuda.synchronize()
    qa, qb = p1.unpack(Qa)[0], p2.unpack(Qb)[0]
    assert np.array_equal(qa, qb)
    assert oracle.rel_l2(qa, _oracle_Q(wl, g0)) <= (F64_TOL if prec == "f64" else F32_TOL)
    p1.step(a, 1e-3, 2)
    p2.step(b, 1e-3, 2)
    torch.cuda.synchronize()
    assert np.array_equal(p1.unpack(a)[0], p2.unpack(b)[0])
    p1.close()
    p2.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_concurrent_groups_match_in_order_launches(torch_cuda, prec):
    """A batch of four grid sizes runs each N group on a stream of its own
    (the default) or every launch on the plan's stream: evaluations, direct
    RK4 steps and graph replays (every replay interleaved with eager work on
    the plan's stream and a synchronisation) are bitwise the same, and match
    the oracle per instance."""
    wke = _wke()
    torch = torch_cuda
    wls = [wi.workload("c4_2d_n96"), wi.workload("c4_2d_n32"), wi.workload("c4_2d_n64"), wi.workload("c4_2d_n48"),
           wi.workload("c4_2d_n32")]
    grids = [wi.three_bumps_2d(w.N, w.L, 11 + s) for s, w in enumerate(wls)]
    descs = [wke.desc_from_workload(w) for w in wls]
    pc = wke.Plan(descs, prec, stream=torch.cuda.current_stream())
    ps = wke.Plan(descs, prec, stream=torch.cuda.current_stream())
    assert pc.groups() == 4
    ps.set_concurrency(False)
    _announce("concurrent groups", prec)
    a, b = pc.pack(grids), ps.pack(grids)
    Qa, Qb = torch.zeros_like(a), torch.zeros_like(b)
    pc.eval_Q(a, Qa)
    ps.eval_Q(b, Qb)
    torch.cuda.synchronize()
    assert torch.equal(Qa, Qb)
    tol = F64_TOL if prec == "f64" else F32_TOL
    for w, g, q in zip(wls, grids, pc.unpack(Qa)):
        assert oracle.rel_l2(q, _oracle_Q(w, g)) <= tol
    pc.step(a, 1e-3, 2)
    ps.step(b, 1e-3, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    pc.set_graphs(True)
    for call in range(3):
        pc.step(a, 1e-3, 2)
        ps.step(b, 1e-3, 2)
        a.mul_(1.0)                     # eager work on the plan's stream between replays
        pc.eval_Q(a, Qa)
        torch.cuda.synchronize()
        assert torch.equal(a, b), "replay %d differs" % call
    pc.close()
    ps.close()


@pytest.mark.parametrize("name,prec,shape", [
    ("c2_2d_n64", "f64", None), ("c3_3d_n32", "f32", None),
    ("big2d", "f64", wi.Workload(2, 32, 8.0, 8, 8, 4, "midpoint")),      # 64 items: several rounds per slot
    ("c5one", "f32", wi.Workload(3, 64, 12.0, 4, 8, 8, "cube")),
])
def test_split_quadrature_sum_across_workgroups(torch_cuda, name, prec, shape):
    """Forcing the quadrature sum of each column block over several
    workgroups (partial sums published with a device-scope fence, combined
    by the last arriving workgroup) agrees with the one-workgroup sum to
    rounding and with the oracle; RK4 steps too."""
    wke = _wke()
    torch = torch_cuda
    wl = shape or wi.workload(name)
    g = wi.three_bumps_2d(wl.N, wl.L, 4) if wl.d == 2 else wi.two_bumps_3d(wl.N, wl.L, 1)
    plan = wke.Plan([wke.desc_from_workload(wl)], prec)
    f = plan.pack([g])
    results = []
    for n in (1, 2, 3, 64):
        _announce("split", name, prec, n)
        plan.set_split(n)
        Q = torch.zeros_like(f)
        plan.eval_Q(f, Q)
        plan.eval_Q(f, Q)             # the arrival counters must reset between launches
        y = f.clone()
        plan.step(y, 1e-3, 2)
        torch.cuda.synchronize()
        results.append((plan.unpack(Q)[0], plan.unpack(y)[0]))
    tol = 1e-14 if prec == "f64" else 1e-6
    for q, y in results[1:]:
        assert oracle.rel_l2(q, results[0][0]) < tol
        assert oracle.rel_l2(y - g, results[0][1] - g) < (1e-13 if prec == "f64" else 1e-5)
    if wl.N <= 32 or wl.d == 2:
        ref = _oracle_Q(wl, g)
        for q, _ in results:
            assert oracle.rel_l2(q, ref) <= (F64_TOL if prec == "f64" else F32_TOL)


def test_invalid_calls_report_errors(torch_cuda):
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload("c1_2d_n16")
    plan = wke.Plan([wke.desc_from_workload(wl)], "f64")
    f = plan.pack([wi.two_gaussians_c1()])
    with pytest.raises(ValueError):
        plan.eval_Q(f, torch.zeros(7, dtype=torch.complex128, device="cuda"))
    with pytest.raises(TypeError):
        plan.eval_Q(f, torch.zeros_like(f, dtype=torch.complex64))
    with pytest.raises(wke.WkeError):
        plan.eval_Q(f, f)                    # Q may not alias f
    with pytest.raises(wke.WkeError):
        plan.step(f, float("nan"), 1)
    with pytest.raises(wke.WkeError):
        plan.set_split(0)
    before = f.clone()
    plan.step(f, 1e-3, 0)                    # zero steps: no change
    torch.cuda.synchronize()
    assert torch.equal(before, f)


FORM_SHAPES = [
    ("c1", "f64", wi.workload("c1_2d_n16")),
    ("c2", "f64", wi.workload("c2_2d_n64")),
    ("c2", "f32", wi.workload("c2_2d_n64")),
    # 12 values per lane; the fused float form runs 768 lanes as 2 shares of
    # 6 x 48 (shares split wavefronts) over 9 slab fields (uneven shares):
    # tests/host/layout_check.cpp checks that this layout is that case
    ("n48", "f32", wi.workload("c4_2d_n48")),
    ("n96", "f64", wi.workload("c4_2d_n96")),                       # 12-lane transforms straddle wavefronts
    ("n128", "f64", wi.Workload(2, 128, 10.0, 1, 4, 4, "midpoint")),
    ("rounds", "f64", wi.Workload(2, 32, 8.0, 8, 8, 6, "midpoint")),  # 64 items: two rounds of fields
    ("odd", "f32", wi.Workload(2, 32, 7.0, 2, 3, 3, "midpoint")),     # no antipodes: b and c fields
    ("c3", "f64", wi.workload("c3_3d_n32")),
    ("c3", "f32", wi.workload("c3_3d_n32")),
    ("octa16", "f64", wi.Workload(3, 16, 6.0, 2, 6, 6, "octahedron")),
    ("ico16", "f32", wi.Workload(3, 16, 6.0, 1, 12, 12, "icosahedron")),
    ("cube16", "f64", wi.Workload(3, 16, 6.0, 3, 8, 8, "cube")),        # 24 items: rounds of fields
]


@pytest.mark.parametrize("name,prec,wl", FORM_SHAPES, ids=[s[0] + "_" + s[1] for s in FORM_SHAPES])
def test_column_pass_forms_agree(torch_cuda, name, prec, wl):
    """The item-slot and the field-parallel forms of the column pass give Q
    and RK4 steps within rounding of each other and within tolerance of the
    oracle, unsplit and with the quadrature sum split over workgroups."""
    wke = _wke()
    torch = torch_cuda
    g = wi.three_bumps_2d(wl.N, wl.L, 5) if wl.d == 2 else wi.two_bumps_3d(wl.N, wl.L, 5)
    ref = _oracle_Q(wl, g)
    plan = wke.Plan([wke.desc_from_workload(wl)], prec)
    f = plan.pack([g])
    got = {}
    for kind in ("slots", "fields", "fused", "fields_half", "fused_mfma"):
        if kind in ("fused", "fused_mfma"):
            try:
                plan.set_column_kernel(kind)
            except wke.WkeError as e:
                # 3D, more than 16 slab fields, or an interpolation sum too
                # long for the workgroup (double N > 64)
                assert e.status == wke.WKE_ERR_UNSUPPORTED
                assert wl.d == 3 or plan.field_counts(0)[1] > 16 or (prec == "f64" and wl.N > 64)
                continue
        for n in (1, 2):
            _announce("form", name, prec, kind, n)
            plan.set_column_kernel(kind)
            plan.set_split(n)
            Q = torch.zeros_like(f)
            plan.eval_Q(f, Q)
            y = f.clone()
            plan.step(y, 1e-3, 2)
            torch.cuda.synchronize()
            (q,), (yy,) = plan.unpack(Q), plan.unpack(y)
            err = oracle.rel_l2(q, ref)
            print(kind, n, "rel_l2", err)
            assert err <= (F64_TOL if prec == "f64" else F32_TOL)
            got[kind, n] = (q, yy)
    # in float each form sits about 1e-6 from the oracle by its own rounding
    # path.  The forms that transform the same slab fields differ only in the
    # order of the quadrature sum: 1e-6 between them.  The fused forms
    # interpolate where the others transform, so they may differ from those
    # by the sum of the two paths' errors: the parity bar itself.
    q0, y0 = got["slots", 1]
    for key, (q, yy) in got.items():
        fused = key[0].startswith("fused")
        bar = 1e-14 if prec == "f64" else (F32_TOL if fused else 1e-6)
        assert oracle.rel_l2(q, q0) < bar, key
        assert oracle.rel_l2(yy - g, y0 - g) < (1e-13 if prec == "f64" else (1e-5 if fused else 1e-6)), key


def test_column_form_choice(torch_cuda):
    """The 3D N=64 shape at full size: both column-pass forms agree to
    rounding (the oracle is checked on sampled points elsewhere); forms the
    plan cannot take are refused."""
    wke = _wke()
    torch = torch_cuda
    wl = wi.Workload(3, 64, 12.0, 1, 6, 6, "octahedron")
    g = wi.two_bumps_3d(wl.N, wl.L, 2)
    plan = wke.Plan([wke.desc_from_workload(wl)], "f32")
    f = plan.pack([g])
    out = []
    for kind in ("slots", "fields"):
        _announce("form 3d n64", kind)
        plan.set_column_kernel(kind)
        Q = torch.zeros_like(f)
        plan.eval_Q(f, Q)
        torch.cuda.synchronize()
        out.append(plan.unpack(Q)[0])
    assert oracle.rel_l2(out[1], out[0]) < 1e-6
    with pytest.raises(wke.WkeError):
        plan.set_column_kernel(7)
    wide = wke.Plan([wke.desc_from_workload(wi.Workload(2, 16, 6.0, 1, 1, 65, "midpoint"))], "f64")
    with pytest.raises(wke.WkeError):
        wide.set_column_kernel("fields")      # 65 product units per item
    wide.set_column_kernel("slots")


def _distinct_shift_counts(wl):
    """Shift vectors of Alg. 1 from the oracle's quadrature (r q-hat and
    r (q-hat - sigma) / 2 over every sigma node, which for an antipodal rule
    also covers r (q-hat + sigma) / 2), and how many distinct vectors they
    form on axes 1..d-1 and on all axes."""
    nd = oracle.nodes_for(wl)
    vecs = []
    for r in nd.r:
        for q in nd.qh:
            vecs.append(r * q)
            vecs.extend(0.5 * r * (q - s) for s in nd.sg)
    A = np.array(vecs)

    def distinct(B):
        return len({tuple(np.round(b / 1e-9).astype(np.int64)) for b in B})
    return len(A), distinct(A[:, 1:]), distinct(A)


@pytest.mark.parametrize("name", ["c2_2d_n64", "c3_3d_n32", "c5_3d_n64", "c1_2d_n16"])
def test_shared_field_counts(torch_cuda, name):
    """The library finds exactly the coincidences among the shift vectors
    that a direct count from the quadrature nodes finds (C2: 80 shifts, 9
    slab fields, 33 distinct vectors; the cube design in 3D: 144, 17, 53)."""
    wke = _wke()
    wl = wi.workload(name)
    plan = wke.Plan([wke.desc_from_workload(wl)], "f64")
    got = plan.field_counts(0)
    want = _distinct_shift_counts(wl)
    print(name, got, want)
    assert tuple(got) == want
    plan.close()


DEGENERATE = [
    # one quadrature point with sigma = q-hat: s_b = 0 and s_c = s_a, so every
    # product cancels (b = F0, c = a) and Q vanishes identically; likewise for
    # (1,2,2), where sigma = +-q-hat
    (wi.Workload(2, 16, 8.0, 1, 1, 1, "midpoint"), 0.0),
    (wi.Workload(2, 16, 8.0, 1, 2, 2, "midpoint"), 0.0),
    (wi.Workload(2, 16, 8.0, 1, 1, 2, "midpoint"), 0.0),     # one direction, one antipodal sigma pair
    (wi.Workload(2, 32, 6.0, 3, 1, 5, "midpoint"), 0.0),     # odd sigma count, single q-hat
    (wi.Workload(2, 16, 8.0, 2, 4, 4, "midpoint"), 16.0),    # R = 2L, the largest radius allowed
    (wi.Workload(3, 16, 6.0, 1, 6, 6, "octahedron"), 0.05),  # a tiny radius: shifts well below one cell
]


@pytest.mark.parametrize("wl,R", DEGENERATE, ids=["%d_%d_%d_R%g" % (w.Nr, w.Ns, w.Nsig, r) for w, r in DEGENERATE])
def test_degenerate_quadratures_and_radii(torch_cuda, wl, R):
    wke = _wke()
    torch = torch_cuda
    f = wi.random_smooth(wl.d, wl.N, wl.L, 30)
    _announce("degenerate", wl, R)
    d = wke.Desc(wl.d, wl.N, wl.L, wl.Nr, wl.Ns, wl.Nsig, wl.rule, R)
    for prec in ("f64", "f32"):
        plan = wke.Plan([d], prec)
        ft = plan.pack([f])
        Q = torch.zeros_like(ft)
        plan.eval_Q(ft, Q)
        torch.cuda.synchronize()
        nd = oracle.nodes(wl.d, wl.N, wl.L, wl.Nr, wl.Ns, wl.Nsig, wl.rule, R=R if R > 0 else None)
        ref, K = oracle.Q_physical(f, nd, return_terms=True)
        # measured against the size of the four terms, since Q itself can
        # vanish identically here
        scale = sum(np.linalg.norm(k) for k in K) * 2.0 ** (1 - wl.d)
        err = np.linalg.norm(plan.unpack(Q)[0] - ref) / scale
        print(prec, "err/sumK", err, "|Q|/sumK", np.linalg.norm(ref) / scale)
        assert err <= (F64_TOL if prec == "f64" else F32_TOL)
        plan.close()


def test_zero_state_gives_exact_zero(torch_cuda):
    wl = wi.workload("c3_3d_n32")
    _announce("zero state")
    for prec in ("f64", "f32"):
        _, (Q,) = _eval(torch_cuda, [wl], [np.zeros((32,) * 3, dtype=np.complex128)], prec)
        assert np.all(Q == 0)


def test_forced_allocation_failure_during_plan_creation(torch_cuda):
    """The allocation test hook makes each device allocation of plan
    creation fail in turn (plain, real and exact-Galerkin plans): every
    attempt reports WKE_ERR_NOMEM and releases what it had allocated, and a
    plan built afterwards evaluates correctly."""
    wke = _wke()
    torch = torch_cuda
    wl = wi.workload("c1_2d_n16")
    g = wi.two_gaussians_c1()
    ref = _oracle_Q(wl, g)
    desc = wke.desc_from_workload(wl)
    free0 = torch.cuda.mem_get_info()[0]
    for kw in ({}, {"real": True}, {"galerkin": True}):
        failures = 0
        for k in range(200):
            wke.wke_test_fail_allocations(k)
            try:
                plan = wke.Plan([desc], "f64", **kw)
            except wke.WkeError as e:
                assert e.status == wke.WKE_ERR_NOMEM, (kw, k, e)
                failures += 1
                continue
            finally:
                wke.wke_test_fail_allocations(-1)
            plan.close()
            break
        else:
            raise AssertionError("plan creation never completed")
        print(kw, "allocations before success:", failures)
        assert failures >= 10
    torch.cuda.synchronize()
    plan = wke.Plan([desc], "f64")
    f = plan.pack([g])
    Q = torch.zeros_like(f)
    plan.eval_Q(f, Q)
    torch.cuda.synchronize()
    assert oracle.rel_l2(plan.unpack(Q)[0], ref) <= F64_TOL
    plan.close()
    # the failed attempts freed their memory (allow for the caching of the
    # runtime and torch: a few MiB)
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)
