"""ctypes binding of ``libmss.so`` (the C ABI declared in ``include/mss.h``).

Argument marshalling only: every step of the solver runs in the HIP
kernels behind the C ABI.  Torch is used for device memory and streams.
If the library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmss.so")

MSS_MAX_TERMS = 32
MSS_MAX_SQUARES = 60

MSS_OK, MSS_E_INVALID, MSS_E_NOMEM, MSS_E_DEVICE, MSS_E_UNSUPPORTED, MSS_E_BUSY, \
    MSS_E_NOTREADY = range(7)

# every function include/mss.h declares
EXPORTS = [
    "mss_status_str", "mss_last_error", "mss_version", "mss_validate", "mss_plan_launch",
    "mss_workspace_size", "mss_propagate_workspace_size", "mss_integrate", "mss_propagate",
    "mss_solve",
]


class MssError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_STATUS_NAMES = {0: "MSS_OK", 1: "MSS_E_INVALID", 2: "MSS_E_NOMEM", 3: "MSS_E_DEVICE",
                 4: "MSS_E_UNSUPPORTED", 5: "MSS_E_BUSY", 6: "MSS_E_NOTREADY"}


class Term(C.Structure):
    _fields_ = [("kind", C.c_int32), ("comp", C.c_int32),
                ("a_slot", C.c_int32), ("f_slot", C.c_int32), ("phi_slot", C.c_int32),
                ("n_seg", C.c_int32), ("seg_a_slot", C.c_int32), ("seg_phi_slot", C.c_int32),
                ("a", C.c_double), ("f", C.c_double), ("phi", C.c_double),
                ("t_on", C.c_double), ("t_off", C.c_double),
                ("seg_t0", C.c_double), ("seg_len", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("spin_twice", C.c_int32), ("n_terms", C.c_int32),
                ("terms", C.POINTER(Term)), ("n_params", C.c_int32), ("n_fine", C.c_int32),
                ("n_samples", C.c_int64), ("t_start", C.c_double), ("dt_out", C.c_double),
                ("n_squares", C.c_int32), ("rotating_frame", C.c_int32)]


class Launch(C.Structure):
    _fields_ = [("slices", C.c_int32), ("block", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libmss.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        PP = C.POINTER(Problem)
        L.mss_status_str.restype = C.c_char_p
        L.mss_status_str.argtypes = [C.c_int]
        L.mss_last_error.restype = C.c_char_p
        L.mss_version.restype = C.c_char_p
        L.mss_validate.argtypes = [PP]
        L.mss_plan_launch.argtypes = [PP, C.POINTER(Launch)]
        L.mss_workspace_size.argtypes = [PP, C.c_int32, C.POINTER(sz)]
        L.mss_propagate_workspace_size.argtypes = [C.c_int32, C.c_int64, C.POINTER(sz)]
        L.mss_integrate.argtypes = [PP, vp, vp, vp, C.POINTER(Launch), vp]
        L.mss_propagate.argtypes = [C.c_int32, C.c_int64, vp, vp, vp, vp, vp, sz, vp]
        L.mss_solve.argtypes = [PP, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        for name in ("mss_validate", "mss_plan_launch", "mss_workspace_size",
                     "mss_propagate_workspace_size", "mss_integrate", "mss_propagate",
                     "mss_solve"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != MSS_OK:
        raise MssError(status, lib().mss_last_error().decode())


def last_error() -> str:
    return lib().mss_last_error().decode()


def version() -> str:
    return lib().mss_version().decode()


class PackedProblem:
    """A ctypes mss_problem with its term array kept alive."""

    def __init__(self, prob):
        terms = list(prob.terms)
        arr = (Term * max(1, len(terms)))()
        for i, t in enumerate(terms):
            arr[i] = Term(int(t.kind), int(t.comp), int(t.a_slot), int(t.f_slot),
                          int(t.phi_slot), int(t.n_seg), int(t.seg_a_slot), int(t.seg_phi_slot),
                          float(t.a), float(t.f), float(t.phi), float(t.t_on), float(t.t_off),
                          float(t.seg_t0), float(t.seg_len))
        self.terms = arr
        n_params = int(np.asarray(prob.params).size)
        self.c = Problem(int(prob.spin_twice), len(terms), arr, n_params, int(prob.n_fine),
                         int(prob.n_samples), float(prob.t_start), float(prob.dt_out),
                         int(prob.n_squares), int(bool(prob.rotating_frame)))
        self.dim = int(prob.spin_twice) + 1
        self.n_params = n_params

    @property
    def ref(self):
        return C.byref(self.c)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


def validate(prob) -> None:
    check(lib().mss_validate(PackedProblem(prob).ref))


def plan_launch(prob) -> tuple[int, int]:
    out = Launch()
    check(lib().mss_plan_launch(PackedProblem(prob).ref, C.byref(out)))
    return out.slices, out.block


def workspace_size(prob, store_u: bool) -> int:
    n = C.c_size_t()
    check(lib().mss_workspace_size(PackedProblem(prob).ref, int(bool(store_u)), C.byref(n)))
    return n.value


def propagate_workspace_size(spin_twice: int, n_samples: int) -> int:
    n = C.c_size_t()
    check(lib().mss_propagate_workspace_size(int(spin_twice), int(n_samples), C.byref(n)))
    return n.value


# ---- torch-facing wrappers (device tensors in, device tensors out) ---------

def device_params(prob, device="cuda"):
    import torch
    p = np.asarray(prob.params, dtype=np.float64).ravel()
    if p.size == 0:
        return None
    return torch.from_numpy(p.copy()).to(device)


def device_state(vec, device="cuda"):
    import torch
    v = np.ascontiguousarray(np.asarray(vec, dtype=np.complex128))
    return torch.from_numpy(v.copy()).to(device)


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def integrate(prob, params, U, time=None, launch: Optional[tuple[int, int]] = None,
              stream=None) -> None:
    """mss_integrate on device tensors (U: complex128 [K, N, N])."""
    pk = PackedProblem(prob)
    ln = C.byref(Launch(*launch)) if launch else None
    check(lib().mss_integrate(pk.ref, _ptr(params), _ptr(U), _ptr(time), ln, _stream(stream)))


def propagate(spin_twice: int, U, psi0, psi, psi_final=None, ws=None, stream=None) -> None:
    K = int(U.shape[0])
    nbytes = 0 if ws is None else int(ws.numel() * ws.element_size())
    check(lib().mss_propagate(int(spin_twice), K, _ptr(U), _ptr(psi0), _ptr(psi),
                              _ptr(psi_final), _ptr(ws), nbytes, _stream(stream)))


def solve_into(prob, params, psi0, psi, psi_final=None, U=None, time=None, ws=None,
               stream=None) -> None:
    pk = PackedProblem(prob)
    nbytes = 0 if ws is None else int(ws.numel() * ws.element_size())
    check(lib().mss_solve(pk.ref, _ptr(params), _ptr(psi0), _ptr(U), _ptr(psi),
                          _ptr(psi_final), _ptr(time), _ptr(ws), nbytes, _stream(stream)))


def solve(prob, store_u: bool = False, want_time: bool = False, device="cuda",
          stream=None) -> dict:
    """Allocate outputs on the device and run the whole path (mss_solve).
    Returns torch tensors: psi [K, N], psi_final [N], U [K, N, N] or None,
    time [K] or None."""
    import torch
    K, N = int(prob.n_samples), int(prob.spin_twice) + 1
    params = device_params(prob, device)
    psi0 = device_state(prob.psi0, device)
    psi = torch.empty((K, N), dtype=torch.complex128, device=device)
    fin = torch.empty((N,), dtype=torch.complex128, device=device)
    U = torch.empty((K, N, N), dtype=torch.complex128, device=device) if store_u else None
    time = torch.empty((K,), dtype=torch.float64, device=device) if want_time else None
    ws = alloc_workspace(workspace_size(prob, store_u), device)
    solve_into(prob, params, psi0, psi, fin, U, time, ws, stream)
    return {"psi": psi, "psi_final": fin, "U": U, "time": time}
