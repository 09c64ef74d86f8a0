"""Python binding of libwke, the MI355X (gfx950) library for the spectrally
truncated four-wave collision operator (Qi, Shen, Wang, arXiv 2503.12805).

This module only marshals arguments: every step of the computation runs in
the HIP kernels of ``_wke.so`` behind the C interface of ``include/wke.h``.
The functions keep the C names.  Device buffers are torch tensors
(complex128, on the GPU, contiguous, packed as described by wke_offset);
torch provides memory and streams only.  There is no CPU fallback: if the
library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_wke.so")

WKE_OK = 0
WKE_ERR_INVALID = -1
WKE_ERR_UNSUPPORTED = -2
WKE_ERR_HIP = -3
WKE_ERR_NOMEM = -4
WKE_ERR_NONFINITE = -5

WKE_MIDPOINT, WKE_OCTAHEDRON, WKE_CUBE, WKE_ICOSAHEDRON = 0, 1, 2, 3
WKE_F64, WKE_F32 = 0, 1
RULE_IDS = {"midpoint": WKE_MIDPOINT, "octahedron": WKE_OCTAHEDRON, "cube": WKE_CUBE,
            "icosahedron": WKE_ICOSAHEDRON}
PRECISIONS = {"f64": WKE_F64, "f32": WKE_F32}
WKE_COLUMN_SLOTS, WKE_COLUMN_FIELDS, WKE_COLUMN_FUSED, WKE_COLUMN_FIELDS_HALF, WKE_COLUMN_FUSED_MFMA = 0, 1, 2, 3, 4
COLUMN_KINDS = {"slots": WKE_COLUMN_SLOTS, "fields": WKE_COLUMN_FIELDS, "fused": WKE_COLUMN_FUSED,
                "fields_half": WKE_COLUMN_FIELDS_HALF, "fused_mfma": WKE_COLUMN_FUSED_MFMA}

EXPORTS = ["wke_plan_create", "wke_plan_create_galerkin", "wke_plan_create_real", "wke_exact_system",
           "wke_exact_system_noalloc", "wke_plan_destroy", "wke_offset", "wke_total_elems", "wke_eval_Q",
           "wke_eval_Q_hat", "wke_step", "wke_set_graphs", "wke_moments", "wke_get_nodes", "wke_plan_tune",
           "wke_plan_set_split", "wke_plan_set_column_kernel", "wke_field_counts",
           "wke_time_kernels", "wke_work_model", "wke_plan_set_concurrency", "wke_plan_groups",
           "wke_status_string", "wke_last_error", "wke_test_fail_allocations"]


class WkeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("wke status %d: %s" % (status, msg))
        self.status = status


class wke_desc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int), ("L", ctypes.c_double),
                ("R", ctypes.c_double), ("N_r", ctypes.c_int), ("N_s", ctypes.c_int),
                ("N_sig", ctypes.c_int), ("sphere_rule", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load _wke.so (raises if it is absent: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libwke is not built (%s missing); run "
                          "`python -m paper_2503_12805_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    lib.wke_plan_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(wke_desc), ctypes.c_int,
                                    ctypes.c_int, P]
    lib.wke_plan_create.restype = ctypes.c_int
    lib.wke_plan_create_galerkin.argtypes = lib.wke_plan_create.argtypes
    lib.wke_plan_create_galerkin.restype = ctypes.c_int
    lib.wke_plan_create_real.argtypes = lib.wke_plan_create.argtypes
    lib.wke_plan_create_real.restype = ctypes.c_int
    lib.wke_exact_system.argtypes = [ctypes.POINTER(wke_desc), ctypes.c_int, P, P, P]
    lib.wke_exact_system.restype = ctypes.c_int
    lib.wke_exact_system_noalloc.argtypes = lib.wke_exact_system.argtypes
    lib.wke_exact_system_noalloc.restype = ctypes.c_int
    lib.wke_test_fail_allocations.argtypes = [ctypes.c_int]
    lib.wke_test_fail_allocations.restype = None
    lib.wke_plan_destroy.argtypes = [P]
    lib.wke_plan_destroy.restype = None
    lib.wke_offset.argtypes = [P, ctypes.c_int]
    lib.wke_offset.restype = ctypes.c_size_t
    lib.wke_total_elems.argtypes = [P]
    lib.wke_total_elems.restype = ctypes.c_size_t
    lib.wke_eval_Q.argtypes = [P, P, P]
    lib.wke_eval_Q.restype = ctypes.c_int
    lib.wke_eval_Q_hat.argtypes = [P, P, P]
    lib.wke_eval_Q_hat.restype = ctypes.c_int
    lib.wke_step.argtypes = [P, P, ctypes.c_double, ctypes.c_int]
    lib.wke_step.restype = ctypes.c_int
    lib.wke_set_graphs.argtypes = [P, ctypes.c_int]
    lib.wke_set_graphs.restype = ctypes.c_int
    lib.wke_plan_set_concurrency.argtypes = [P, ctypes.c_int]
    lib.wke_plan_set_concurrency.restype = ctypes.c_int
    lib.wke_plan_groups.argtypes = [P]
    lib.wke_plan_groups.restype = ctypes.c_int
    lib.wke_moments.argtypes = [P, P, D]
    lib.wke_moments.restype = ctypes.c_int
    lib.wke_get_nodes.argtypes = [P, ctypes.c_int, D, D, D, D, D, D]
    lib.wke_get_nodes.restype = ctypes.c_int
    lib.wke_plan_set_split.argtypes = [P, ctypes.c_int]
    lib.wke_plan_set_split.restype = ctypes.c_int
    lib.wke_plan_set_column_kernel.argtypes = [P, ctypes.c_int]
    lib.wke_plan_set_column_kernel.restype = ctypes.c_int
    lib.wke_field_counts.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.wke_field_counts.restype = ctypes.c_int
    lib.wke_plan_tune.argtypes = [P, P, P, ctypes.c_int, D]
    lib.wke_plan_tune.restype = ctypes.c_int
    lib.wke_time_kernels.argtypes = [P, P, P, ctypes.c_int, D]
    lib.wke_time_kernels.restype = ctypes.c_int
    lib.wke_work_model.argtypes = [P, D, D]
    lib.wke_work_model.restype = ctypes.c_int
    lib.wke_status_string.argtypes = [ctypes.c_int]
    lib.wke_status_string.restype = ctypes.c_char_p
    lib.wke_last_error.argtypes = []
    lib.wke_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != WKE_OK:
        lib = load_library()
        raise WkeError(status, (lib.wke_last_error() or b"").decode() or
                       lib.wke_status_string(status).decode())
    return status


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass(frozen=True)
class Desc:
    """One instance: d, N, L, (N_r, N_s, N_sig), rule; R <= 0 picks
    R = 4L/(3+sqrt 2)."""
    d: int
    N: int
    L: float
    N_r: int
    N_s: int
    N_sig: int
    rule: str = "midpoint"
    R: float = 0.0

    def to_c(self) -> wke_desc:
        return wke_desc(self.d, self.N, float(self.L), float(self.R), self.N_r, self.N_s,
                        self.N_sig, RULE_IDS[self.rule])


def desc_from_workload(wl) -> Desc:
    return Desc(wl.d, wl.N, wl.L, wl.Nr, wl.Ns, wl.Nsig, wl.rule)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _tensor_ptr(t, n_complex: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("%s must be a contiguous complex128 GPU tensor" % name)
    if t.numel() != n_complex:
        raise ValueError("%s has %d elements, the plan needs %d" % (name, t.numel(), n_complex))
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Owns one wke plan (quadrature tables and workspace on the GPU).
    galerkin=True builds the exact-Galerkin (de-aliased) form
    (wke_plan_create_galerkin), real=True the Nyquist-zero real form
    (wke_plan_create_real)."""

    def __init__(self, descs: Sequence[Desc], precision: str = "f64", stream=None, galerkin: bool = False,
                 real: bool = False):
        lib = load_library()
        if galerkin and real:
            raise ValueError("a plan is either exact-Galerkin or real, not both")
        arr = (wke_desc * len(descs))(*[d.to_c() for d in descs])
        h = ctypes.c_void_p()
        self._stream = stream
        create = (lib.wke_plan_create_galerkin if galerkin else
                  lib.wke_plan_create_real if real else lib.wke_plan_create)
        _check(create(ctypes.byref(h), arr, len(descs), PRECISIONS[precision], _stream_handle(stream)))
        self.handle = h
        self.descs = list(descs)
        self.precision = precision
        self.galerkin = bool(galerkin)
        self.real = bool(real)
        self.batch = len(descs)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().wke_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # layout -----------------------------------------------------------
    def offset(self, i: int) -> int:
        return int(load_library().wke_offset(self.handle, i))

    def total_elems(self) -> int:
        return int(load_library().wke_total_elems(self.handle))

    def pack(self, grids, device="cuda"):
        """Pack per-instance numpy grids into one complex128 device tensor."""
        import torch
        host = np.zeros(self.total_elems(), dtype=np.complex128)
        for i, g in enumerate(grids):
            n = g.size
            host[self.offset(i):self.offset(i) + n] = np.asarray(g, dtype=np.complex128).ravel()
        return torch.from_numpy(host).to(device)

    def unpack(self, t):
        h = t.detach().cpu().numpy()
        out = []
        for i, dsc in enumerate(self.descs):
            n = dsc.N ** dsc.d
            out.append(h[self.offset(i):self.offset(i) + n].reshape((dsc.N,) * dsc.d))
        return out

    # computation ------------------------------------------------------
    def eval_Q(self, f, Q):
        n = self.total_elems()
        _check(load_library().wke_eval_Q(self.handle, _tensor_ptr(f, n, "f"), _tensor_ptr(Q, n, "Q")))
        return Q

    def eval_Q_hat(self, f, Qhat):
        """Fourier coefficients of Q (FFT index order), per instance."""
        n = self.total_elems()
        _check(load_library().wke_eval_Q_hat(self.handle, _tensor_ptr(f, n, "f"), _tensor_ptr(Qhat, n, "Qhat")))
        return Qhat

    def step(self, f, dt: float, nsteps: int = 1):
        n = self.total_elems()
        _check(load_library().wke_step(self.handle, _tensor_ptr(f, n, "f"), float(dt), int(nsteps)))
        return f

    def set_graphs(self, enable: bool):
        _check(load_library().wke_set_graphs(self.handle, int(bool(enable))))

    def set_concurrency(self, enable: bool):
        _check(load_library().wke_plan_set_concurrency(self.handle, int(bool(enable))))

    def groups(self) -> int:
        return int(load_library().wke_plan_groups(self.handle))

    def moments(self, f) -> np.ndarray:
        out = np.zeros(6 * self.batch)
        st = load_library().wke_moments(self.handle, _tensor_ptr(f, self.total_elems(), "f"), _dptr(out))
        if st == WKE_ERR_NONFINITE:
            raise WkeError(st, "non-finite state")
        _check(st)
        return out.reshape(self.batch, 6)

    def nodes(self, i: int):
        dsc = self.descs[i]
        r = np.zeros(dsc.N_r); wr = np.zeros(dsc.N_r)
        qh = np.zeros(dsc.N_s * dsc.d); ws = np.zeros(dsc.N_s)
        sg = np.zeros(dsc.N_sig * dsc.d); wsig = np.zeros(dsc.N_sig)
        _check(load_library().wke_get_nodes(self.handle, i, _dptr(r), _dptr(wr), _dptr(qh), _dptr(ws),
                                            _dptr(sg), _dptr(wsig)))
        return r, wr, qh.reshape(-1, dsc.d), ws, sg.reshape(-1, dsc.d), wsig

    def tune(self, f, Q, reps: int = 10) -> np.ndarray:
        """Autotune the column pass (form and work split); returns
        (form, split, us) per N group."""
        n = self.total_elems()
        out = np.zeros(3 * 16)
        _check(load_library().wke_plan_tune(self.handle, _tensor_ptr(f, n, "f"), _tensor_ptr(Q, n, "Q"),
                                            int(reps), _dptr(out)))
        ngroups = len(dict.fromkeys(d.N for d in self.descs))
        return out[:3 * ngroups].reshape(ngroups, 3)

    def set_split(self, n: int):
        _check(load_library().wke_plan_set_split(self.handle, int(n)))

    def field_counts(self, i: int = 0):
        """(shifts, distinct slab fields, distinct shift vectors) of instance i."""
        out = (ctypes.c_int * 3)()
        _check(load_library().wke_field_counts(self.handle, int(i), out))
        return tuple(out)

    def set_column_kernel(self, kind):
        """kind: "slots", "fields", "fused", "fields_half" or "fused_mfma" (or the WKE_COLUMN_* values)."""
        _check(load_library().wke_plan_set_column_kernel(self.handle, COLUMN_KINDS.get(kind, kind)))

    def time_kernels(self, f, Q, reps: int = 20) -> np.ndarray:
        n = self.total_elems()
        out = np.zeros(4)
        _check(load_library().wke_time_kernels(self.handle, _tensor_ptr(f, n, "f"), _tensor_ptr(Q, n, "Q"),
                                               int(reps), _dptr(out)))
        return out

    def work_model(self):
        fl = np.zeros(3)
        by = np.zeros(3)
        _check(load_library().wke_work_model(self.handle, _dptr(fl), _dptr(by)))
        return fl, by


# The binding's public functions under the names of the C interface
# (include/wke.h), one per entry point; the Plan methods above are the same
# calls on a plan object.
def wke_plan_create(descs, precision="f64", stream=None) -> Plan:
    return Plan(descs, precision, stream)


def wke_plan_create_galerkin(descs, precision="f64", stream=None) -> Plan:
    return Plan(descs, precision, stream, galerkin=True)


def wke_plan_create_real(descs, precision="f64", stream=None) -> Plan:
    return Plan(descs, precision, stream, real=True)


def wke_exact_system(desc: Desc, f, Q, n_radial: int = 256, stream=None):
    """Exact-weight reference system on the GPU: Q (N^d complex128 tensor)
    from f; waits for completion."""
    c = desc.to_c()
    n = desc.N ** desc.d
    _check(load_library().wke_exact_system(ctypes.byref(c), int(n_radial), _tensor_ptr(f, n, "f"),
                                           _tensor_ptr(Q, n, "Q"), _stream_handle(stream)))
    return Q


def wke_exact_system_noalloc(desc: Desc, f, Q, n_radial: int = 256, stream=None):
    """The same system with its workspace in the library's static device
    array (no allocation, no wait): enqueued on `stream`."""
    c = desc.to_c()
    n = desc.N ** desc.d
    _check(load_library().wke_exact_system_noalloc(ctypes.byref(c), int(n_radial), _tensor_ptr(f, n, "f"),
                                                   _tensor_ptr(Q, n, "Q"), _stream_handle(stream)))
    return Q


def wke_test_fail_allocations(after: int):
    """Test hook: the device allocation after `after` more successful ones
    fails (after < 0: off)."""
    load_library().wke_test_fail_allocations(int(after))


def wke_plan_destroy(plan: Plan):
    plan.close()


def wke_eval_Q(plan: Plan, f, Q):
    return plan.eval_Q(f, Q)


def wke_step(plan: Plan, f, dt, nsteps=1):
    return plan.step(f, dt, nsteps)


def wke_set_graphs(plan: Plan, enable: bool):
    return plan.set_graphs(enable)


def wke_plan_set_concurrency(plan: Plan, enable: bool):
    return plan.set_concurrency(enable)


def wke_plan_groups(plan: Plan) -> int:
    return plan.groups()


def wke_moments(plan: Plan, f):
    return plan.moments(f)


def wke_offset(plan: Plan, i: int) -> int:
    return plan.offset(i)


def wke_total_elems(plan: Plan) -> int:
    return plan.total_elems()


def wke_get_nodes(plan: Plan, i: int):
    return plan.nodes(i)


def wke_plan_set_column_kernel(plan: Plan, kind):
    return plan.set_column_kernel(kind)


def wke_field_counts(plan: Plan, i: int = 0):
    return plan.field_counts(i)


def wke_plan_tune(plan: Plan, f, Q, reps=10):
    return plan.tune(f, Q, reps)


def wke_plan_set_split(plan: Plan, n: int):
    return plan.set_split(n)


def wke_time_kernels(plan: Plan, f, Q, reps=20):
    return plan.time_kernels(f, Q, reps)


def wke_work_model(plan: Plan):
    return plan.work_model()
