"""The allocation-free entry point wke_exact_system_noalloc (workspace in a
static device array) against wke_exact_system (workspace allocated per
call), through the C interface: two calls in a row, the second on a smaller
input, each equal to the allocating call's result to the double-precision
bar (1e-12 relative L2; the two run the same kernels, so the results are
expected to be bitwise equal).  Run alone and after the other tests."""
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


def _run(torch, fn, desc, g, nr):
    f = torch.from_numpy(np.ascontiguousarray(g).ravel()).cuda()
    Q = torch.full_like(f, complex(np.nan, np.nan))     # every element must be written
    fn(desc, f, Q, n_radial=nr, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    return Q.cpu().numpy().reshape(g.shape)


CASES = [
    # (d, N, L, n_radial, data): the first is the largest 2D size the static workspace holds
    (2, 16, 8.0, 256, lambda: wi.two_gaussians_c1(16, 8.0)),
    (2, 8, 6.0, 64, lambda: wi.random_smooth(2, 8, 6.0, 4)),
    (3, 4, 5.0, 32, lambda: wi.random_smooth(3, 4, 5.0, 9)),
]


def test_noalloc_matches_allocating_entry_point(torch_cuda):
    wke = _wke()
    for d, N, L, nr, gen in CASES:
        g = gen()
        desc = wke.Desc(d, N, L, 1, 1, 1, "midpoint" if d == 2 else "cube")
        print("[case] noalloc d=%d N=%d nr=%d" % (d, N, nr), flush=True)
        ref = _run(torch_cuda, wke.wke_exact_system, desc, g, nr)
        got = _run(torch_cuda, wke.wke_exact_system_noalloc, desc, g, nr)
        err = oracle.rel_l2(got, ref)
        print("rel-L2 %.3e, bitwise %s" % (err, np.array_equal(got, ref)), flush=True)
        assert np.all(np.isfinite(got))
        assert err <= 1e-12


def test_noalloc_in_order_on_one_stream(torch_cuda):
    """Two calls enqueued back to back on one stream without a wait between
    them (the second reuses the array the first used), then a third on the
    first input again."""
    wke = _wke()
    torch = torch_cuda
    g1, g2 = wi.two_gaussians_c1(16, 8.0), wi.random_smooth(2, 8, 6.0, 4)
    d1, d2 = wke.Desc(2, 16, 8.0, 1, 1, 1), wke.Desc(2, 8, 6.0, 1, 1, 1)
    r1 = _run(torch, wke.wke_exact_system, d1, g1, 128)
    r2 = _run(torch, wke.wke_exact_system, d2, g2, 128)
    s = torch.cuda.current_stream()
    f1 = torch.from_numpy(g1.ravel().copy()).cuda()
    f2 = torch.from_numpy(g2.ravel().copy()).cuda()
    Q1, Q2, Q3 = torch.zeros_like(f1), torch.zeros_like(f2), torch.zeros_like(f1)
    wke.wke_exact_system_noalloc(d1, f1, Q1, n_radial=128, stream=s)
    wke.wke_exact_system_noalloc(d2, f2, Q2, n_radial=128, stream=s)
    wke.wke_exact_system_noalloc(d1, f1, Q3, n_radial=128, stream=s)
    torch.cuda.synchronize()
    assert oracle.rel_l2(Q1.cpu().numpy().reshape(16, 16), r1) <= 1e-12
    assert oracle.rel_l2(Q2.cpu().numpy().reshape(8, 8), r2) <= 1e-12
    assert oracle.rel_l2(Q3.cpu().numpy().reshape(16, 16), r1) <= 1e-12


def test_noalloc_refuses_sizes_beyond_its_workspace(torch_cuda):
    wke = _wke()
    torch = torch_cuda
    f = torch.zeros(32 * 32, dtype=torch.complex128, device="cuda")
    Q = torch.zeros_like(f)
    with pytest.raises(wke.WkeError) as e:
        wke.wke_exact_system_noalloc(wke.Desc(2, 32, 8.0, 1, 1, 1), f, Q, n_radial=64)
    assert e.value.status == wke.WKE_ERR_UNSUPPORTED
