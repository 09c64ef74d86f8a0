"""CPU checks of the C interface: the library loads, exports every function
that include/wke.h declares, and rejects bad descriptors in its host-side
validation (which runs before any GPU call)."""
import ctypes
import os
import re

import pytest

import paper_2503_12805_amd as wke

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "wke.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wke_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_the_interface():
    names = _declared()
    for n in ["wke_plan_create", "wke_eval_Q", "wke_step", "wke_moments", "wke_plan_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = wke.load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(wke.EXPORTS) == _declared()


def _create(descs, precision=wke.WKE_F64):
    lib = wke.load_library()
    arr = (wke.wke_desc * len(descs))(*descs)
    h = ctypes.c_void_p()
    st = lib.wke_plan_create(ctypes.byref(h), arr, len(descs), precision, None)
    return st, h, lib.wke_last_error().decode()


def D(d=2, N=16, L=8.0, R=0.0, Nr=2, Ns=4, Nsig=2, rule=wke.WKE_MIDPOINT):
    return wke.wke_desc(d, N, L, R, Nr, Ns, Nsig, rule)


@pytest.mark.parametrize("desc,status,needle", [
    (D(d=4), wke.WKE_ERR_INVALID, "d must be"),
    (D(N=15), wke.WKE_ERR_INVALID, "even"),
    (D(N=40), wke.WKE_ERR_UNSUPPORTED, "not built"),
    (D(d=3, N=96, Ns=8, Nsig=8, rule=wke.WKE_CUBE), wke.WKE_ERR_UNSUPPORTED, "not built"),
    (D(L=-1.0), wke.WKE_ERR_INVALID, "L must be"),
    (D(Nr=0), wke.WKE_ERR_INVALID, "quadrature counts"),
    (D(rule=wke.WKE_CUBE), wke.WKE_ERR_INVALID, "2D uses"),
    (D(d=3, N=16, Ns=6, Nsig=8, rule=wke.WKE_CUBE), wke.WKE_ERR_INVALID, "design"),
    (D(d=3, N=16, Ns=8, Nsig=8, rule=wke.WKE_MIDPOINT), wke.WKE_ERR_INVALID, "design"),
    (D(R=17.0), wke.WKE_ERR_INVALID, "2L"),
    (D(R=float("nan")), wke.WKE_ERR_INVALID, "finite"),
])
def test_validation_rejects_bad_descriptors(desc, status, needle):
    st, h, msg = _create([desc])
    assert st == status
    assert needle in msg
    assert not h.value


def test_validation_rejects_mixed_dimensions_and_bad_precision():
    st, _, msg = _create([D(), D(d=3, N=16, Ns=8, Nsig=8, rule=wke.WKE_CUBE)])
    assert st == wke.WKE_ERR_INVALID and "share d" in msg
    st, _, msg = _create([D()], precision=7)
    assert st == wke.WKE_ERR_INVALID and "precision" in msg
    lib = wke.load_library()
    h = ctypes.c_void_p()
    assert lib.wke_plan_create(ctypes.byref(h), None, 1, 0, None) == wke.WKE_ERR_INVALID
    assert lib.wke_plan_create(None, None, 1, 0, None) == wke.WKE_ERR_INVALID


def test_null_plan_calls_fail_cleanly():
    lib = wke.load_library()
    assert lib.wke_eval_Q(None, None, None) == wke.WKE_ERR_INVALID
    assert lib.wke_eval_Q_hat(None, None, None) == wke.WKE_ERR_INVALID
    assert lib.wke_step(None, None, 0.1, 1) == wke.WKE_ERR_INVALID
    assert lib.wke_moments(None, None, None) == wke.WKE_ERR_INVALID
    assert lib.wke_field_counts(None, 0, None) == wke.WKE_ERR_INVALID
    assert lib.wke_offset(None, 0) == 0 and lib.wke_total_elems(None) == 0
    lib.wke_plan_destroy(None)
    assert lib.wke_status_string(wke.WKE_ERR_NONFINITE) == b"non-finite value"


def test_binding_refuses_missing_library(tmp_path):
    saved = wke._lib
    wke._lib = None
    try:
        with pytest.raises(ImportError):
            wke.load_library(str(tmp_path / "nope.so"))
    finally:
        wke._lib = saved


def test_galerkin_plan_validation_needs_no_gpu():
    """Argument and size checks of wke_plan_create_galerkin happen before
    any device call."""
    lib = wke.load_library()
    h = ctypes.c_void_p()

    def make(d, N, rule=wke.WKE_MIDPOINT, ns=4):
        arr = (wke.wke_desc * 1)(wke.wke_desc(d, N, 10.0, 0.0, 2, ns, ns, rule))
        return lib.wke_plan_create_galerkin(ctypes.byref(h), arr, 1, wke.WKE_F64, None)

    assert make(2, 96) == wke.WKE_ERR_UNSUPPORTED        # 2N = 192 is not built
    assert make(3, 64, wke.WKE_CUBE, 8) == wke.WKE_ERR_UNSUPPORTED
    assert make(2, 15) == wke.WKE_ERR_INVALID
    arr = (wke.wke_desc * 1)(wke.wke_desc(2, 16, 10.0, 0.0, 2, 4, 4, wke.WKE_MIDPOINT))
    assert lib.wke_plan_create_galerkin(ctypes.byref(h), arr, 0, wke.WKE_F64, None) == wke.WKE_ERR_INVALID
    assert lib.wke_plan_create_galerkin(None, arr, 1, wke.WKE_F64, None) == wke.WKE_ERR_INVALID
    assert lib.wke_plan_create_galerkin(ctypes.byref(h), arr, 1, 7, None) == wke.WKE_ERR_INVALID


def test_exact_system_validation_needs_no_gpu():
    lib = wke.load_library()
    big = wke.wke_desc(2, 64, 10.0, 0.0, 1, 1, 1, wke.WKE_MIDPOINT)
    dummy = ctypes.c_void_p(16)
    assert lib.wke_exact_system(ctypes.byref(big), 64, dummy, ctypes.c_void_p(32), None) == wke.WKE_ERR_UNSUPPORTED
    odd = wke.wke_desc(2, 15, 10.0, 0.0, 1, 1, 1, wke.WKE_MIDPOINT)
    assert lib.wke_exact_system(ctypes.byref(odd), 64, dummy, ctypes.c_void_p(32), None) == wke.WKE_ERR_INVALID
    ok = wke.wke_desc(2, 16, 10.0, 0.0, 1, 1, 1, wke.WKE_MIDPOINT)
    assert lib.wke_exact_system(ctypes.byref(ok), 0, dummy, ctypes.c_void_p(32), None) == wke.WKE_ERR_INVALID
    assert lib.wke_exact_system(None, 64, dummy, ctypes.c_void_p(32), None) == wke.WKE_ERR_INVALID


def test_noalloc_size_limit_needs_no_gpu():
    """The allocation-free reference system refuses, before any device call,
    sizes whose workspace exceeds its static array."""
    lib = wke.load_library()
    dummy = ctypes.c_void_p(16)
    too_big = wke.wke_desc(2, 32, 10.0, 0.0, 1, 1, 1, wke.WKE_MIDPOINT)
    st = lib.wke_exact_system_noalloc(ctypes.byref(too_big), 64, dummy, ctypes.c_void_p(32), None)
    assert st == wke.WKE_ERR_UNSUPPORTED
    assert b"static workspace" in lib.wke_last_error()
    wide = wke.wke_desc(2, 16, 10.0, 0.0, 1, 1, 1, wke.WKE_MIDPOINT)
    st = lib.wke_exact_system_noalloc(ctypes.byref(wide), 4096, dummy, ctypes.c_void_p(32), None)
    assert st == wke.WKE_ERR_UNSUPPORTED
    assert lib.wke_exact_system_noalloc(None, 64, dummy, dummy, None) == wke.WKE_ERR_INVALID


def test_forced_allocation_failure_reports_nomem():
    """The allocation test hook: the first device allocation of the
    allocating reference system fails, which it reports as WKE_ERR_NOMEM
    before any device call; with the hook off again the arguments are
    judged as before."""
    lib = wke.load_library()
    ok = wke.wke_desc(2, 16, 10.0, 0.0, 1, 1, 1, wke.WKE_MIDPOINT)
    dummy = ctypes.c_void_p(16)
    try:
        lib.wke_test_fail_allocations(0)
        st = lib.wke_exact_system(ctypes.byref(ok), 64, dummy, ctypes.c_void_p(32), None)
        assert st == wke.WKE_ERR_NOMEM
        assert b"allocation" in lib.wke_last_error()
    finally:
        lib.wke_test_fail_allocations(-1)
    assert lib.wke_exact_system(ctypes.byref(ok), 0, dummy, ctypes.c_void_p(32), None) == wke.WKE_ERR_INVALID
