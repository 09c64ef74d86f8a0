"""GPU parity of the exact-weight reference system (wke_exact_system)
against the oracle's Q_exact (1e-12 relative L2, both double), its zero
mass mode, and its use: the fast method with the exact constraint
(wke_plan_create_galerkin) approaches it as the quadrature is refined.
"""
import sys

import numpy as np
import pytest

import oracle
import wke_inputs as wi

pytestmark = pytest.mark.gpu


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


def _exact_gpu(torch, d, N, L, f, n_radial=256):
    wke = _wke()
    ft = torch.from_numpy(np.ascontiguousarray(f, dtype=np.complex128).ravel()).cuda()
    Q = torch.zeros_like(ft)
    wke.wke_exact_system(wke.Desc(d, N, L, 1, 1, 1, "midpoint" if d == 2 else "cube"), ft, Q, n_radial)
    return Q.cpu().numpy().reshape((N,) * d)


CASES = [(2, 8, 8.0, 1), (2, 16, 8.0, 2), (2, 12, 6.0, 3), (3, 4, 6.0, 4), (3, 8, 6.0, 5)]


@pytest.mark.parametrize("d,N,L,seed", CASES, ids=["d%d_N%d" % (c[0], c[1]) for c in CASES])
def test_matches_oracle(torch_cuda, d, N, L, seed):
    f = wi.random_smooth(d, N, L, seed)
    print("[case] exact system", d, N, flush=True)
    sys.stdout.flush()
    Q = _exact_gpu(torch_cuda, d, N, L, f)
    ref = oracle.Q_exact(f, d, N, L)
    err = oracle.rel_l2(Q, ref)
    print("rel_l2", err)
    assert err <= 1e-12
    Qh = oracle.spectrum(Q, L)
    assert abs(Qh.flat[0]) <= 1e-13 * np.abs(Qh).sum()


def test_fast_method_approaches_it(torch_cuda):
    """2D N=16, C1 data: the exact-constraint fast method's distance to the
    reference system falls spectrally with N_r, N_s = N_sigma."""
    wke = _wke()
    torch = torch_cuda
    d, N, L = 2, 16, 8.0
    f = wi.two_gaussians_c1()
    ref = _exact_gpu(torch, d, N, L, f)
    errs = []
    for nr, ns in [(2, 4), (4, 8), (8, 16), (16, 32)]:
        plan = wke.Plan([wke.Desc(d, N, L, nr, ns, ns)], "f64", galerkin=True)
        ft = plan.pack([f])
        Q = torch.zeros_like(ft)
        plan.eval_Q(ft, Q)
        torch.cuda.synchronize()
        errs.append(oracle.rel_l2(plan.unpack(Q)[0], ref))
        plan.close()
    print("quadrature error", errs)
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-4        # 6.5e-6 on the oracle (exact constraint through 2N points)
