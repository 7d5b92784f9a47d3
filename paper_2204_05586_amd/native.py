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
    "mss_solve", "mss_spin_projection", "mss_batch_plan_create", "mss_batch_layout", "mss_batch_workspace_size",
    "mss_batch_info", "mss_batch_run", "mss_batch_integrate", "mss_batch_propagate",
    "mss_batch_check", "mss_batch_plan_destroy", "mss_server_create", "mss_server_submit", "mss_server_poll",
    "mss_server_wait", "mss_server_copy_out", "mss_server_release", "mss_server_stats_get",
    "mss_server_clock", "mss_server_destroy", "mss_server_request_slices",
    "mss_adjoint_plan_create",
    "mss_adjoint_workspace_size", "mss_adjoint_param_count", "mss_adjoint_run",
    "mss_adjoint_plan_destroy", "mss_sampler_create", "mss_sampler_log", "mss_sampler_integrate",
    "mss_sampler_solve", "mss_sampler_destroy", "mss_batch_plan_create_sampled",
    "mss_sampler_create_for_terms", "mss_sampler_min_params", "mss_propagate_spin",
    "mss_adjoint_plan_create_compiled", "mss_propagate_noalloc", "mss_solve_batch",
    "mss_adjoint_population",
]

MSS_REQ_QUEUED, MSS_REQ_RUNNING, MSS_REQ_DONE, MSS_REQ_FAILED = range(4)


class MssError(RuntimeError):
    """A non-OK status from the library; ``status`` holds the code.  Invalid
    arguments also raise as ValueError and out-of-memory as MemoryError
    (the subclasses below)."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class MssInvalidError(MssError, ValueError):
    pass


class MssNoMemoryError(MssError, MemoryError):
    pass


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
                ("n_squares", C.c_int32), ("rotating_frame", C.c_int32),
                ("method", C.c_int32)]


class Launch(C.Structure):
    _fields_ = [("slices", C.c_int32), ("block", C.c_int32)]


class BatchOptions(C.Structure):
    _fields_ = [("slices_spin_half", C.c_int32), ("slices_spin_one", C.c_int32),
                ("waves_per_simd", C.c_int32), ("use_graph", C.c_int32),
                ("scan_per_lane", C.c_int32), ("chained", C.c_int32),
                ("chain_wait_us", C.c_int32)]


class ServerOptions(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int32), ("slices", C.c_int32),
                ("iteration_steps", C.c_double)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("spin_twice", C.c_int32), ("n_samples", C.c_int64),
                ("psi", C.c_void_p), ("psi_final", C.c_void_p), ("U", C.c_void_p),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rounds", C.c_int64),
                ("queued", C.c_int32), ("active", C.c_int32), ("fine_steps", C.c_double),
                ("bytes_in_use", C.c_size_t), ("bytes_peak", C.c_size_t),
                ("budget", C.c_size_t)]


class BatchInfo(C.Structure):
    _fields_ = [("n_sims", C.c_int32), ("scan_levels", C.c_int32), ("grid_blocks", C.c_int32),
                ("pad", C.c_int32), ("n_items", C.c_int64), ("total_samples", C.c_int64)]


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
        L.mss_propagate_spin.argtypes = [C.c_int32, C.c_int64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.mss_propagate_noalloc.argtypes = [C.c_int32, C.c_int64, vp, vp, vp, vp, vp]
        L.mss_solve.argtypes = [PP, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.mss_spin_projection.argtypes = [C.c_int32, C.c_int64, vp, vp, vp]
        L.mss_spin_projection.restype = C.c_int
        i64p = C.POINTER(C.c_int64)
        L.mss_solve_batch.argtypes = [C.c_int32, PP, i64p, vp, vp, vp, vp, vp, vp]
        L.mss_adjoint_population.argtypes = [C.c_int32, PP, i64p, C.c_int32, vp, vp, vp, vp,
                                             vp, vp]
        L.mss_batch_plan_create.argtypes = [C.c_int32, PP, i64p, C.POINTER(BatchOptions),
                                            C.POINTER(vp)]
        L.mss_batch_plan_create_sampled.argtypes = [C.c_int32, PP, i64p,
                                                    C.POINTER(BatchOptions), vp, C.POINTER(vp)]
        L.mss_batch_layout.argtypes = [vp, i64p, i64p, i64p]
        L.mss_batch_workspace_size.argtypes = [vp, C.c_int32, C.POINTER(sz)]
        L.mss_batch_info.argtypes = [vp, C.POINTER(BatchInfo)]
        L.mss_batch_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.mss_batch_integrate.argtypes = [vp, vp, vp, vp, sz, vp]
        L.mss_batch_propagate.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
        L.mss_batch_check.argtypes = [vp, vp, vp]
        L.mss_server_create.argtypes = [C.POINTER(ServerOptions), C.POINTER(vp)]
        L.mss_server_submit.argtypes = [vp, PP, vp, vp, C.POINTER(C.c_uint64)]
        L.mss_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(RequestInfo)]
        L.mss_server_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(RequestInfo)]
        L.mss_server_copy_out.argtypes = [vp, C.c_uint64, vp, vp, vp, vp]
        L.mss_server_release.argtypes = [vp, C.c_uint64]
        L.mss_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
        L.mss_server_request_slices.argtypes = [vp, PP, C.POINTER(C.c_int32)]
        L.mss_server_clock.argtypes = [vp]
        L.mss_server_clock.restype = C.c_double
        L.mss_server_destroy.argtypes = [vp]
        L.mss_server_destroy.restype = None
        L.mss_adjoint_plan_create.argtypes = [C.c_int32, PP, i64p, C.c_int32, C.POINTER(vp)]
        L.mss_adjoint_plan_create_compiled.argtypes = [C.c_int32, PP, i64p, C.c_int32, vp,
                                                       C.POINTER(vp)]
        L.mss_adjoint_workspace_size.argtypes = [vp, C.POINTER(sz)]
        L.mss_adjoint_param_count.argtypes = [vp, i64p]
        L.mss_adjoint_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.mss_adjoint_plan_destroy.argtypes = [vp]
        L.mss_adjoint_plan_destroy.restype = None
        L.mss_batch_plan_destroy.argtypes = [vp]
        L.mss_batch_plan_destroy.restype = None
        L.mss_sampler_create.argtypes = [C.c_char_p, C.POINTER(C.c_char_p), C.c_int32,
                                         C.POINTER(vp)]
        L.mss_sampler_log.argtypes = [vp]
        L.mss_sampler_log.restype = C.c_char_p
        L.mss_sampler_integrate.argtypes = [vp, PP, vp, vp, vp, C.POINTER(Launch), vp]
        L.mss_sampler_solve.argtypes = [vp, PP, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.mss_sampler_create_for_terms.argtypes = [C.POINTER(Term), C.c_int32, C.POINTER(vp)]
        L.mss_sampler_min_params.argtypes = [vp]
        L.mss_sampler_min_params.restype = C.c_int32
        L.mss_sampler_destroy.argtypes = [vp]
        L.mss_sampler_destroy.restype = None
        for name in ("mss_validate", "mss_plan_launch", "mss_workspace_size",
                     "mss_propagate_workspace_size", "mss_integrate", "mss_propagate",
                     "mss_solve", "mss_spin_projection", "mss_batch_plan_create", "mss_batch_layout",
                     "mss_batch_workspace_size", "mss_batch_info", "mss_batch_run",
                     "mss_batch_integrate", "mss_batch_propagate", "mss_batch_check",
                     "mss_server_create",
                     "mss_server_submit", "mss_server_poll", "mss_server_wait",
                     "mss_server_copy_out", "mss_server_release", "mss_server_stats_get",
                     "mss_adjoint_plan_create", "mss_adjoint_workspace_size",
                     "mss_adjoint_param_count", "mss_adjoint_run", "mss_sampler_create",
                     "mss_sampler_integrate", "mss_sampler_solve",
                     "mss_batch_plan_create_sampled", "mss_sampler_create_for_terms",
                     "mss_propagate_spin", "mss_server_request_slices",
                     "mss_adjoint_plan_create_compiled", "mss_propagate_noalloc",
                     "mss_solve_batch", "mss_adjoint_population"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != MSS_OK:
        cls = {MSS_E_INVALID: MssInvalidError, MSS_E_NOMEM: MssNoMemoryError}.get(status, MssError)
        raise cls(status, lib().mss_last_error().decode())


def last_error() -> str:
    return lib().mss_last_error().decode()


def version() -> str:
    return lib().mss_version().decode()


def _term_array(terms):
    """A ctypes mss_term array of a term list (at least one element)."""
    terms = list(terms)
    arr = (Term * max(1, len(terms)))()
    for i, t in enumerate(terms):
        arr[i] = Term(int(t.kind), int(t.comp), int(t.a_slot), int(t.f_slot),
                      int(t.phi_slot), int(t.n_seg), int(t.seg_a_slot), int(t.seg_phi_slot),
                      float(t.a), float(t.f), float(t.phi), float(t.t_on), float(t.t_off),
                      float(t.seg_t0), float(t.seg_len))
    return arr


def _terms_key(terms) -> tuple:
    """Exact identity of a term list (every field, floats bit for bit)."""
    return tuple((int(t.kind), int(t.comp), int(t.a_slot), int(t.f_slot), int(t.phi_slot),
                  int(t.n_seg), int(t.seg_a_slot), int(t.seg_phi_slot),
                  float(t.a).hex(), float(t.f).hex(), float(t.phi).hex(), float(t.t_on).hex(),
                  float(t.t_off).hex(), float(t.seg_t0).hex(), float(t.seg_len).hex())
                 for t in terms)


class PackedProblem:
    """A ctypes mss_problem with its term array kept alive."""

    def __init__(self, prob):
        terms = list(prob.terms)
        arr = _term_array(terms)
        self.terms = arr
        n_params = int(np.asarray(prob.params).size)
        self.c = Problem(int(prob.spin_twice), len(terms), arr, n_params, int(prob.n_fine),
                         int(prob.n_samples), float(prob.t_start), float(prob.dt_out),
                         int(prob.n_squares), int(bool(prob.rotating_frame)),
                         int(getattr(prob, "method", 0)))
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


def propagate(spin_twice: int, U, psi0, psi, psi_final=None, ws=None, stream=None,
              spin=None) -> None:
    """mss_propagate; with a device tensor spin [K, 3] (float64),
    mss_propagate_spin: <J_x>, <J_y>, <J_z> of every state in the same pass."""
    K = int(U.shape[0])
    nbytes = 0 if ws is None else int(ws.numel() * ws.element_size())
    if spin is None:
        check(lib().mss_propagate(int(spin_twice), K, _ptr(U), _ptr(psi0), _ptr(psi),
                                  _ptr(psi_final), _ptr(ws), nbytes, _stream(stream)))
    else:
        check(lib().mss_propagate_spin(int(spin_twice), K, _ptr(U), _ptr(psi0), _ptr(psi),
                                       _ptr(psi_final), _ptr(spin), _ptr(ws), nbytes,
                                       _stream(stream)))


def propagate_noalloc(spin_twice: int, U, psi0, psi, psi_final=None, stream=None,
                      n_samples=None) -> None:
    """mss_propagate_noalloc: mss_propagate with the library's static scan
    scratch instead of a workspace (no allocation; calls overlapping on one
    GPU race).  n_samples defaults to U's length."""
    K = int(U.shape[0]) if n_samples is None else int(n_samples)
    check(lib().mss_propagate_noalloc(int(spin_twice), K, _ptr(U), _ptr(psi0), _ptr(psi),
                                      _ptr(psi_final), _stream(stream)))


def solve_into(prob, params, psi0, psi, psi_final=None, U=None, time=None, ws=None,
               stream=None) -> None:
    pk = PackedProblem(prob)
    nbytes = 0 if ws is None else int(ws.numel() * ws.element_size())
    check(lib().mss_solve(pk.ref, _ptr(params), _ptr(psi0), _ptr(U), _ptr(psi),
                          _ptr(psi_final), _ptr(time), _ptr(ws), nbytes, _stream(stream)))


def spin_projection(psi, stream=None):
    """<J_x>, <J_y>, <J_z> of each row of a device state tensor [K, N] -> [K, 3]."""
    import torch
    K, N = int(psi.shape[0]), int(psi.shape[1])
    out = torch.empty((K, 3), dtype=torch.float64, device=psi.device)
    check(lib().mss_spin_projection(N - 1, K, _ptr(psi.contiguous()), _ptr(out),
                                    _stream(stream)))
    return out


def solve(prob, store_u: bool = False, want_time: bool = False, device="cuda",
          stream=None, sampler: "Optional[Sampler]" = None, want_spin: bool = False) -> dict:
    """Allocate outputs on the device and run the whole path (mss_solve, or
    mss_sampler_solve when a sampler supplies the field; with want_spin the
    integrator then mss_propagate_spin).  Returns torch tensors: psi [K, N],
    psi_final [N], U [K, N, N] or None, time [K] or None, spin [K, 3] or None."""
    import torch
    K, N = int(prob.n_samples), int(prob.spin_twice) + 1
    params = device_params(prob, device)
    psi0 = device_state(prob.psi0, device)
    psi = torch.empty((K, N), dtype=torch.complex128, device=device)
    fin = torch.empty((N,), dtype=torch.complex128, device=device)
    U = torch.empty((K, N, N), dtype=torch.complex128, device=device) if store_u else None
    time = torch.empty((K,), dtype=torch.float64, device=device) if want_time else None
    if want_spin:
        Uw = U if U is not None else torch.empty((K, N, N), dtype=torch.complex128, device=device)
        if sampler is None:
            integrate(prob, params, Uw, time, stream=stream)
        else:
            sampler.integrate(prob, params, Uw, time, stream=stream)
        spin = torch.empty((K, 3), dtype=torch.float64, device=device)
        ws = alloc_workspace(propagate_workspace_size(prob.spin_twice, K), device)
        propagate(prob.spin_twice, Uw, psi0, psi, fin, ws, stream, spin=spin)
        return {"psi": psi, "psi_final": fin, "U": U, "time": time, "spin": spin}
    ws = alloc_workspace(workspace_size(prob, store_u), device)
    if sampler is None:
        solve_into(prob, params, psi0, psi, fin, U, time, ws, stream)
    else:
        sampler.solve_into(prob, params, psi0, psi, fin, U, time, ws, stream)
    return {"psi": psi, "psi_final": fin, "U": U, "time": time, "spin": None}


# ---- user field samplers ---------------------------------------------------

class Sampler:
    """A user field function in HIP C++, compiled at run time (hiprtc) into
    its own integrator (mss_sampler_create).  ``source`` defines
    ``__device__ void mss_user_field(double t, const double* params,
    double* field)`` setting f_x, f_y, f_z, f_q in Hz; problems solved with
    it carry no terms.  Compilation needs no GPU."""

    def __init__(self, source: str, options=()):
        opts = [str(o).encode() for o in options]
        arr = (C.c_char_p * max(1, len(opts)))(*opts) if opts else None
        h = C.c_void_p()
        check(lib().mss_sampler_create(source.encode(), arr, len(opts), C.byref(h)))
        self._h = h
        self.source = source
        self.terms = None

    @classmethod
    def for_terms(cls, terms) -> "Sampler":
        """The field program ``terms`` compiled into its own integrator
        (mss_sampler_create_for_terms): the interpreter's arithmetic for
        these terms, so the operators are bit for bit the interpreter's.
        Problems run with it carry no terms and at least ``min_params``
        parameters."""
        terms = list(terms)
        h = C.c_void_p()
        check(lib().mss_sampler_create_for_terms(_term_array(terms), len(terms), C.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.source = None
        self.terms = terms
        return self

    @property
    def min_params(self) -> int:
        return int(lib().mss_sampler_min_params(self._h))

    @property
    def log(self) -> str:
        return lib().mss_sampler_log(self._h).decode()

    def integrate(self, prob, params, U, time=None, launch: Optional[tuple[int, int]] = None,
                  stream=None) -> None:
        pk = PackedProblem(prob)
        ln = C.byref(Launch(*launch)) if launch else None
        check(lib().mss_sampler_integrate(self._h, pk.ref, _ptr(params), _ptr(U), _ptr(time), ln,
                                          _stream(stream)))

    def solve_into(self, prob, params, psi0, psi, psi_final=None, U=None, time=None, ws=None,
                   stream=None) -> None:
        pk = PackedProblem(prob)
        nbytes = 0 if ws is None else int(ws.numel() * ws.element_size())
        check(lib().mss_sampler_solve(self._h, pk.ref, _ptr(params), _ptr(psi0), _ptr(U),
                                      _ptr(psi), _ptr(psi_final), _ptr(time), _ptr(ws), nbytes,
                                      _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mss_sampler_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batches ---------------------------------------------------------------

def specialise(problems) -> "Optional[tuple[Sampler, list]]":
    """When every problem has the same term list, that field program
    compiled into its own integrator and the problems without their terms
    (what a sampler runs); None otherwise, and for full su(3) programs.  The
    caller owns the sampler."""
    problems = list(problems)
    if not problems or any(int(t.comp) >= 4 for t in problems[0].terms):
        return None  # full su(3) programs are interpreted
    key = _terms_key(problems[0].terms)
    if any(_terms_key(p.terms) != key for p in problems[1:]):
        return None
    return Sampler.for_terms(problems[0].terms), [p.replace(terms=[]) for p in problems]


class BatchPlan:
    """A planned batch of simulations (mss_batch_plan_create).

    The packed layout puts simulation i's initial/final state at
    psi0_off[i], its states at state_off[i] and its operators at op_off[i]
    (complex units).  Parameters are concatenated in simulation order.
    sampler: a ``Sampler`` giving every simulation's field (problems then
    carry no terms); kept alive by the plan.
    specialize: when every problem has the same term list (parameters may
    differ), compile that field program into its own integrator
    (``Sampler.for_terms``, bit-for-bit the interpreter's operators) and run
    the batch with it; otherwise the terms are interpreted.  The plan owns
    that sampler; ``specialized`` tells which happened.
    chained: ``run`` forms the states inside the integrator's launch (no
    operator buffer, no scan; see mss_batch_options.chained);
    chain_wait_us bounds one unit's wait for its entering state (0: 10 s),
    and ``check`` reports a run whose wait ran out."""

    def __init__(self, problems, slices_spin_half=0, slices_spin_one=0, waves_per_simd=0,
                 use_graph=False, scan_per_lane=0, sampler: "Optional[Sampler]" = None,
                 specialize: bool = False, chained: bool = False, chain_wait_us: int = 0):
        self.problems = list(problems)
        self._own_sampler = None
        self.specialized = False
        if specialize and sampler is None:
            sp = specialise(self.problems)
            if sp is not None:
                sampler, self.problems = sp
                self._own_sampler = sampler
                self.specialized = True
        n = len(self.problems)
        self.packed = [PackedProblem(p) for p in self.problems]
        arr = (Problem * max(1, n))()
        for i, pk in enumerate(self.packed):
            arr[i] = pk.c
        self._arr = arr
        counts = np.array([pk.n_params for pk in self.packed], dtype=np.int64)
        self.param_off = np.zeros(max(1, n), dtype=np.int64)
        if n:
            self.param_off[:n] = np.concatenate([[0], np.cumsum(counts)[:-1]])
        self.n_params_total = int(counts.sum())
        opt = BatchOptions(int(slices_spin_half), int(slices_spin_one), int(waves_per_simd),
                           int(bool(use_graph)), int(scan_per_lane), int(bool(chained)),
                           int(chain_wait_us))
        self.options = {"slices_spin_half": int(slices_spin_half),
                        "slices_spin_one": int(slices_spin_one),
                        "waves_per_simd": int(waves_per_simd), "use_graph": bool(use_graph),
                        "scan_per_lane": int(scan_per_lane), "chained": bool(chained),
                        "chain_wait_us": int(chain_wait_us)}
        self.chained = bool(chained)
        h = C.c_void_p()
        offp = self.param_off.ctypes.data_as(C.POINTER(C.c_int64))
        self.sampler = sampler
        if sampler is None:
            check(lib().mss_batch_plan_create(n, arr, offp, C.byref(opt), C.byref(h)))
        else:
            check(lib().mss_batch_plan_create_sampled(n, arr, offp, C.byref(opt), sampler._h,
                                                      C.byref(h)))
        self.handle = h
        self.n = n
        offs = [np.zeros(n + 1, dtype=np.int64) for _ in range(3)]
        check(lib().mss_batch_layout(self.handle,
                                     *[o.ctypes.data_as(C.POINTER(C.c_int64)) for o in offs]))
        self.psi0_off, self.state_off, self.op_off = offs

    def info(self) -> dict:
        bi = BatchInfo()
        check(lib().mss_batch_info(self.handle, C.byref(bi)))
        return {"n_sims": bi.n_sims, "scan_levels": bi.scan_levels,
                "grid_blocks": bi.grid_blocks, "n_items": bi.n_items,
                "total_samples": bi.total_samples}

    def workspace_size(self, store_u: bool) -> int:
        n = C.c_size_t()
        check(lib().mss_batch_workspace_size(self.handle, int(bool(store_u)), C.byref(n)))
        return n.value

    def params_host(self) -> np.ndarray:
        parts = [np.asarray(p.params, dtype=np.float64).ravel() for p in self.problems]
        return np.concatenate(parts) if self.n_params_total else np.zeros(0)

    def psi0_host(self) -> np.ndarray:
        return np.concatenate([np.asarray(p.psi0, dtype=np.complex128) for p in self.problems])

    def allocate(self, store_u=False, device="cuda") -> dict:
        import torch
        params = self.params_host()
        out = {
            "params": torch.from_numpy(params).to(device) if params.size else None,
            "psi0": torch.from_numpy(self.psi0_host()).to(device),
            "psi": torch.empty(int(self.state_off[-1]), dtype=torch.complex128, device=device),
            "psi_final": torch.empty(int(self.psi0_off[-1]), dtype=torch.complex128,
                                     device=device),
            "U": (torch.empty(int(self.op_off[-1]), dtype=torch.complex128, device=device)
                  if store_u else None),
        }
        out["ws"] = alloc_workspace(self.workspace_size(store_u), device)
        return out

    def run(self, bufs: dict, stream=None) -> None:
        ws = bufs["ws"]
        check(lib().mss_batch_run(self.handle, _ptr(bufs["params"]), _ptr(bufs["psi0"]),
                                  _ptr(bufs["psi"]), _ptr(bufs["psi_final"]), _ptr(bufs["U"]),
                                  _ptr(ws), int(ws.numel()), _stream(stream)))

    def integrate(self, bufs: dict, stream=None) -> None:
        ws = bufs["ws"]
        check(lib().mss_batch_integrate(self.handle, _ptr(bufs["params"]), _ptr(bufs["U"]),
                                        _ptr(ws), int(ws.numel()), _stream(stream)))

    def propagate(self, bufs: dict, stream=None) -> None:
        ws = bufs["ws"]
        check(lib().mss_batch_propagate(self.handle, _ptr(bufs["psi0"]), _ptr(bufs["psi"]),
                                        _ptr(bufs["psi_final"]), _ptr(bufs["U"]), _ptr(ws),
                                        int(ws.numel()), _stream(stream)))

    def check(self, bufs: dict, stream=None) -> None:
        """mss_batch_check: waits for the stream and raises MssError when a
        chained run failed (its states are then undefined)."""
        check(lib().mss_batch_check(self.handle, _ptr(bufs["ws"]), _stream(stream)))

    def split(self, bufs: dict, i: int) -> dict:
        """Views of simulation i's outputs: psi [K, N], psi_final [N], U [K, N, N]."""
        p = self.problems[i]
        K, N = int(p.n_samples), int(p.spin_twice) + 1
        a, b = int(self.state_off[i]), int(self.state_off[i + 1])
        out = {"psi": bufs["psi"][a:b].view(K, N),
               "psi_final": bufs["psi_final"][int(self.psi0_off[i]):int(self.psi0_off[i + 1])]}
        if bufs.get("U") is not None:
            a, b = int(self.op_off[i]), int(self.op_off[i + 1])
            out["U"] = bufs["U"][a:b].view(K, N, N)
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().mss_batch_plan_destroy(self.handle)
            self.handle = None
        if getattr(self, "_own_sampler", None) is not None:
            self._own_sampler.close()
            self._own_sampler = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _packed_problems(problems):
    packed = [PackedProblem(p) for p in problems]
    arr = (Problem * max(1, len(packed)))()
    for i, pk in enumerate(packed):
        arr[i] = pk.c
    counts = np.array([pk.n_params for pk in packed], dtype=np.int64)
    off = np.zeros(max(1, len(packed)), dtype=np.int64)
    if len(packed):
        off[:len(packed)] = np.concatenate([[0], np.cumsum(counts)[:-1]])
    return packed, arr, off, int(counts.sum())


def _host_params_psi0(problems, n_params):
    params = (np.concatenate([np.asarray(p.params, dtype=np.float64).ravel() for p in problems])
              if n_params else np.zeros(0))
    psi0 = np.concatenate([np.asarray(p.psi0, dtype=np.complex128) for p in problems])
    return params, psi0


def solve_batch(problems, store_u: bool = False, device="cuda", stream=None) -> dict:
    """mss_solve_batch: the whole batch in one synchronous call (a chained
    plan made, run and freed inside).  Returns the packed device arrays
    (psi0, psi, psi_final, U or None) and the offsets psi0_off, state_off,
    op_off (complex units, n + 1 entries)."""
    import torch
    problems = list(problems)
    packed, arr, off, n_params = _packed_problems(problems)
    params, psi0 = _host_params_psi0(problems, n_params)
    dims = np.array([p.spin_twice + 1 for p in problems], dtype=np.int64)
    ks = np.array([p.n_samples for p in problems], dtype=np.int64)
    psi0_off = np.concatenate([[0], np.cumsum(dims)])
    state_off = np.concatenate([[0], np.cumsum(ks * dims)])
    op_off = np.concatenate([[0], np.cumsum(ks * dims * dims)])
    out = {"params": torch.from_numpy(params).to(device) if params.size else None,
           "psi0": torch.from_numpy(psi0).to(device),
           "psi": torch.empty(int(state_off[-1]), dtype=torch.complex128, device=device),
           "psi_final": torch.empty(int(psi0_off[-1]), dtype=torch.complex128, device=device),
           "U": (torch.empty(int(op_off[-1]), dtype=torch.complex128, device=device)
                 if store_u else None),
           "psi0_off": psi0_off, "state_off": state_off, "op_off": op_off}
    check(lib().mss_solve_batch(len(problems), arr, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                _ptr(out["params"]), _ptr(out["psi0"]), _ptr(out["psi"]),
                                _ptr(out["psi_final"]), _ptr(out["U"]), _stream(stream)))
    return out


def adjoint_population(problems, level_m: int, device="cuda", stream=None) -> dict:
    """mss_adjoint_population: losses |psi_final_i[m]|^2 and their gradients
    with respect to every parameter in one synchronous call.  Returns loss
    [n], grad [total parameters] (simulation i's at param_off[i]),
    psi_final and param_off."""
    import torch
    problems = list(problems)
    packed, arr, off, n_params = _packed_problems(problems)
    params, psi0 = _host_params_psi0(problems, n_params)
    out = {"params": torch.from_numpy(params).to(device) if params.size else None,
           "psi0": torch.from_numpy(psi0).to(device),
           "loss": torch.empty(len(problems), dtype=torch.float64, device=device),
           "grad": torch.empty(max(1, n_params), dtype=torch.float64, device=device),
           "psi_final": torch.empty(psi0.size, dtype=torch.complex128, device=device),
           "param_off": off[:len(problems)]}
    check(lib().mss_adjoint_population(len(problems), arr,
                                       off.ctypes.data_as(C.POINTER(C.c_int64)), int(level_m),
                                       _ptr(out["params"]), _ptr(out["psi0"]),
                                       _ptr(out["loss"]), _ptr(out["grad"]),
                                       _ptr(out["psi_final"]), _stream(stream)))
    return out


# ---- serving ---------------------------------------------------------------

class Server:
    """Continuous-batching simulation server (mss_server_*).  slices: lanes
    per interval; 0 lets the server choose per request from its length
    (``request_slices``)."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 0, slices: int = 0,
                 iteration_steps: float = 0.0):
        opt = ServerOptions(int(hbm_budget), int(max_active), int(slices),
                            float(iteration_steps))
        h = C.c_void_p()
        check(lib().mss_server_create(C.byref(opt), C.byref(h)))
        self.handle = h

    def clock(self) -> float:
        return lib().mss_server_clock(self.handle)

    def request_slices(self, prob) -> int:
        """Lanes per interval the server gives this problem: its results are
        those of ``integrate(..., launch=(slices, 256))`` and ``propagate``."""
        pk = PackedProblem(prob)
        out = C.c_int32()
        check(lib().mss_server_request_slices(self.handle, pk.ref, C.byref(out)))
        return out.value

    def submit(self, prob) -> int:
        pk = PackedProblem(prob)
        params = np.ascontiguousarray(np.asarray(prob.params, dtype=np.float64).ravel())
        psi0 = np.ascontiguousarray(np.asarray(prob.psi0, dtype=np.complex128))
        t = C.c_uint64()
        check(lib().mss_server_submit(self.handle, pk.ref,
                                      params.ctypes.data if params.size else None,
                                      psi0.ctypes.data, C.byref(t)))
        return t.value

    @staticmethod
    def _info(ri: RequestInfo) -> dict:
        return {"state": ri.state, "spin_twice": ri.spin_twice, "n_samples": ri.n_samples,
                "t_submit": ri.t_submit, "t_admit": ri.t_admit, "t_done": ri.t_done}

    def poll(self, ticket: int) -> dict:
        ri = RequestInfo()
        check(lib().mss_server_poll(self.handle, ticket, C.byref(ri)))
        return self._info(ri)

    def wait(self, ticket: int, timeout: float = 60.0) -> dict:
        ri = RequestInfo()
        check(lib().mss_server_wait(self.handle, ticket, float(timeout), C.byref(ri)))
        return self._info(ri)

    def fetch(self, ticket: int, prob, want_u: bool = False, stream=None) -> dict:
        """Copy a finished request's results into new device tensors."""
        import torch
        K, N = int(prob.n_samples), int(prob.spin_twice) + 1
        psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
        U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda") if want_u else None
        check(lib().mss_server_copy_out(self.handle, ticket, _ptr(psi), _ptr(fin), _ptr(U),
                                        _stream(stream)))
        return {"psi": psi, "psi_final": fin, "U": U}

    def release(self, ticket: int) -> None:
        check(lib().mss_server_release(self.handle, ticket))

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().mss_server_stats_get(self.handle, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().mss_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- adjoint ---------------------------------------------------------------

class AdjointPlan:
    """Gradients of |psi_final[m]|^2 w.r.t. field parameters (mss_adjoint_*).
    specialize: when every problem has the same term list, its field program
    is compiled into the forward pass (mss_adjoint_plan_create_compiled; the
    losses and gradients are bit for bit those without); ``specialized``
    tells whether that happened.  The plan owns that sampler."""

    def __init__(self, problems, level_m: int, specialize: bool = False):
        self.problems = list(problems)
        n = len(self.problems)
        self.packed = [PackedProblem(p) for p in self.problems]
        arr = (Problem * max(1, n))()
        for i, pk in enumerate(self.packed):
            arr[i] = pk.c
        self._arr = arr
        counts = np.array([pk.n_params for pk in self.packed], dtype=np.int64)
        self.param_off = np.zeros(max(1, n), dtype=np.int64)
        if n:
            self.param_off[:n] = np.concatenate([[0], np.cumsum(counts)[:-1]])
        self._sampler = None
        sp = specialise(self.problems) if specialize else None
        if sp is not None:
            self._sampler = sp[0]
        self.specialized = self._sampler is not None
        h = C.c_void_p()
        offs = self.param_off.ctypes.data_as(C.POINTER(C.c_int64))
        if self._sampler is None:
            check(lib().mss_adjoint_plan_create(n, arr, offs, int(level_m), C.byref(h)))
        else:
            check(lib().mss_adjoint_plan_create_compiled(n, arr, offs, int(level_m),
                                                         self._sampler._h, C.byref(h)))
        self.handle = h
        self.n = n
        cnt = C.c_int64()
        check(lib().mss_adjoint_param_count(self.handle, C.byref(cnt)))
        self.n_grad = cnt.value
        nb = C.c_size_t()
        check(lib().mss_adjoint_workspace_size(self.handle, C.byref(nb)))
        self.ws_bytes = nb.value

    def allocate(self, device="cuda") -> dict:
        import torch
        params = np.concatenate([np.asarray(p.params, dtype=np.float64).ravel()
                                 for p in self.problems]) if self.n_grad else np.zeros(0)
        psi0 = np.concatenate([np.asarray(p.psi0, dtype=np.complex128) for p in self.problems])
        return {"params": torch.from_numpy(params).to(device) if params.size else None,
                "psi0": torch.from_numpy(psi0).to(device),
                "loss": torch.empty(self.n, dtype=torch.float64, device=device),
                "grad": torch.empty(max(1, self.n_grad), dtype=torch.float64, device=device),
                "psi_final": torch.empty(psi0.size, dtype=torch.complex128, device=device),
                "ws": alloc_workspace(self.ws_bytes, device)}

    def run(self, bufs: dict, stream=None) -> None:
        ws = bufs["ws"]
        check(lib().mss_adjoint_run(self.handle, _ptr(bufs["params"]), _ptr(bufs["psi0"]),
                                    _ptr(bufs["loss"]), _ptr(bufs["grad"]),
                                    _ptr(bufs.get("psi_final")), _ptr(ws), int(ws.numel()),
                                    _stream(stream)))

    def grad_of(self, bufs: dict, i: int):
        a = int(self.param_off[i])
        return bufs["grad"][a:a + self.packed[i].n_params]

    def close(self):
        if getattr(self, "handle", None):
            lib().mss_adjoint_plan_destroy(self.handle)
            self.handle = None
        if getattr(self, "_sampler", None) is not None:
            self._sampler.close()
            self._sampler = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
