"""ctypes front-end of the CPU oracle (``oracle/oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only callers.  Nothing in the GPU
library imports this module, and this module imports nothing from the GPU
library: problems are passed duck-typed (any object with the attributes
``spin_twice, terms, t_start, dt_out, n_samples, n_fine, n_squares,
rotating_frame, params, psi0`` and optionally ``method``; terms with ``kind, comp, a, f, phi, a_slot,
f_slot, phi_slot, t_on, t_off, n_seg, seg_t0, seg_len, seg_a_slot,
seg_phi_slot``).

What each function computes, and the passage of arXiv:2204.05586 it follows,
is documented in ``oracle.cpp``.  Pins: ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off"]


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (baseline x86-64, no FMA contraction)."""
    cmd = ["g++", *CXX_FLAGS, "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Term(C.Structure):
    _fields_ = [("kind", C.c_int32), ("comp", C.c_int32),
                ("a_slot", C.c_int32), ("f_slot", C.c_int32), ("phi_slot", C.c_int32),
                ("n_seg", C.c_int32), ("seg_a_slot", C.c_int32), ("seg_phi_slot", C.c_int32),
                ("a", C.c_double), ("f", C.c_double), ("phi", C.c_double),
                ("t_on", C.c_double), ("t_off", C.c_double),
                ("seg_t0", C.c_double), ("seg_len", C.c_double)]


class _Problem(C.Structure):
    _fields_ = [("spin_twice", C.c_int32), ("n_terms", C.c_int32), ("n_fine", C.c_int32),
                ("n_squares", C.c_int32), ("rotating_frame", C.c_int32), ("n_params", C.c_int32),
                ("method", C.c_int32), ("n_samples", C.c_int64), ("t_start", C.c_double), ("dt_out", C.c_double),
                ("terms", C.POINTER(_Term)), ("field_fn", C.c_void_p)]


# field function callback: (t, params, field[4]) with the paper's calling
# convention for a user field function
_FIELD_FN = C.CFUNCTYPE(None, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double))


class _FieldFn:
    """A Python field function fn(t, params, field) (field: float64 [4] to
    fill with f_x, f_y, f_z, f_q in Hz) as a C callback.  Exceptions raised
    inside are kept and re-raised after the oracle call returns."""

    def __init__(self, fn, n_params: int):
        self.error = None

        def cb(t, p, out):
            try:
                params = np.ctypeslib.as_array(p, shape=(max(n_params, 1),))[:n_params]
                fn(float(t), params, np.ctypeslib.as_array(out, shape=(4,)))
            except BaseException as e:  # noqa: BLE001 - re-raised by check()
                if self.error is None:
                    self.error = e

        self.c = _FIELD_FN(cb)

    def check(self):
        if self.error is not None:
            raise self.error


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_get_threads.restype = C.c_int
        L.oracle_field.argtypes = [C.POINTER(_Problem), dp, C.c_double, dp]
        L.oracle_exp_half.argtypes = [dp, dp]
        L.oracle_exp_one.argtypes = [dp, C.c_int, dp]
        L.oracle_lie_trotter_residual.argtypes = [dp, C.c_int, dp]
        L.oracle_exp_full.argtypes = [dp, C.c_int, dp]
        L.oracle_basis_operator.argtypes = [C.c_int, dp]
        L.oracle_operators.argtypes = [C.POINTER(_Problem), dp, C.c_int64, C.c_int64, dp]
        L.oracle_operators.restype = C.c_int
        L.oracle_states.argtypes = [C.c_int, C.c_int64, dp, dp, dp, dp]
        L.oracle_states.restype = C.c_int
        L.oracle_solve.argtypes = [C.POINTER(_Problem), dp, dp, dp, dp, dp]
        L.oracle_solve.restype = C.c_int
        L.oracle_spin_projection.argtypes = [C.c_int, C.c_int64, dp, dp]
        L.oracle_spin_projection.restype = C.c_int
        L.oracle_adjoint_population.argtypes = [C.POINTER(_Problem), dp, dp, C.c_int, dp, dp]
        L.oracle_adjoint_population.restype = C.c_int
        ldp = C.c_void_p
        L.oracle_solve_ld.argtypes = [C.POINTER(_Problem), ldp, ldp, ldp]
        L.oracle_solve_ld.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Packed:
    """Keeps the ctypes problem and its term array alive together."""

    def __init__(self, prob, field_fn=None):
        terms = list(prob.terms)
        if field_fn is not None and terms:
            raise ValueError("a problem with a field function carries no terms")
        arr = (_Term * max(1, len(terms)))()
        for i, t in enumerate(terms):
            arr[i] = _Term(int(t.kind), int(t.comp), int(t.a_slot), int(t.f_slot),
                           int(t.phi_slot), int(t.n_seg), int(t.seg_a_slot),
                           int(t.seg_phi_slot), float(t.a), float(t.f), float(t.phi),
                           float(t.t_on), float(t.t_off), float(t.seg_t0), float(t.seg_len))
        self.terms = arr
        params = np.ascontiguousarray(np.asarray(prob.params, dtype=np.float64).ravel())
        self.params = params if params.size else np.zeros(1)
        self.p = _Problem(int(prob.spin_twice), len(terms), int(prob.n_fine), int(prob.n_squares),
                          int(bool(prob.rotating_frame)), int(params.size),
                          int(getattr(prob, "method", 0)), int(prob.n_samples),
                          float(prob.t_start), float(prob.dt_out), arr)
        self.fn = None
        if field_fn is not None:
            self.fn = _FieldFn(field_fn, int(params.size))
            self.p.field_fn = C.cast(self.fn.c, C.c_void_p)
        self.dim = int(prob.spin_twice) + 1

    def call(self, f, *args):
        """Run oracle entry point f; a field function runs single-threaded
        (it holds the interpreter lock anyway) and its errors propagate."""
        if self.fn is None:
            return f(*args)
        n = get_threads()
        set_threads(1)
        try:
            rc = f(*args)
        finally:
            set_threads(n)
        self.fn.check()
        return rc


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return lib().oracle_get_threads()


def field(prob, t: float, field_fn=None) -> np.ndarray:
    """Field functions (f_x, f_y, f_z, f_q, f_u1, f_u2, f_v1, f_v2) in Hz at time t."""
    pk = _Packed(prob, field_fn)
    out = np.zeros(8)
    pk.call(lib().oracle_field, C.byref(pk.p), _dp(pk.params), float(t), _dp(out))
    return out


def _cmat(buf: np.ndarray, n: int) -> np.ndarray:
    return buf.view(np.complex128).reshape(n, n)


def exp_half(theta) -> np.ndarray:
    """exp(-i theta . J) for spin-1/2 (analytic SU(2) form)."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64)[:3])
    out = np.zeros(8)
    lib().oracle_exp_half(_dp(th), _dp(out))
    return _cmat(out, 2).copy()


def exp_one(theta, tau: int) -> np.ndarray:
    """Lie-Trotter exp(-i (theta_x J_x + theta_y J_y + theta_z J_z + theta_q Q)), n = 2^tau."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64)[:4])
    out = np.zeros(18)
    lib().oracle_exp_one(_dp(th), int(tau), _dp(out))
    return _cmat(out, 3).copy()


def exp_full(theta, tau: int) -> np.ndarray:
    """Full su(3) basis: exp(-i sum_j theta_j A_j) over (J_x, J_y, J_z, Q, U_1,
    U_2, V_1, V_2) by scaling and squaring (degree-4 Taylor residual of the
    2^-tau step, then tau residual squarings)."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64)[:8])
    out = np.zeros(18)
    lib().oracle_exp_full(_dp(th), int(tau), _dp(out))
    return _cmat(out, 3).copy()


def basis_operator(j: int) -> np.ndarray:
    """The spin-1 basis operator A_j, j = 0..7: J_x, J_y, J_z, Q, U_1, U_2, V_1, V_2."""
    out = np.zeros(18)
    lib().oracle_basis_operator(int(j), _dp(out))
    return _cmat(out, 3).copy()


def lie_trotter_residual(theta, tau: int) -> np.ndarray:
    """a = T - I of the symmetric Lie-Trotter factor (before any squaring)."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64)[:4])
    out = np.zeros(18)
    lib().oracle_lie_trotter_residual(_dp(th), int(tau), _dp(out))
    return _cmat(out, 3).copy()


def operators(prob, k0: int = 0, count: int | None = None, field_fn=None) -> np.ndarray:
    """U_k for k in [k0, k0 + count), shape [count, N, N] complex128."""
    pk = _Packed(prob, field_fn)
    if count is None:
        count = int(prob.n_samples) - k0
    U = np.zeros((count, pk.dim, pk.dim), dtype=np.complex128)
    rc = pk.call(lib().oracle_operators, C.byref(pk.p), _dp(pk.params), int(k0), int(count),
                 _dp(U.view(np.float64)))
    if rc:
        raise ValueError("oracle_operators: bad arguments")
    return U


def states(U: np.ndarray, psi0) -> tuple[np.ndarray, np.ndarray]:
    """Sequential state compilation: psi_0 = psi0, psi_{k+1} = U_k psi_k.
    Returns (psi [K, N], psi_final [N])."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    K, N, _ = U.shape
    v0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
    psi = np.zeros((K, N), dtype=np.complex128)
    fin = np.zeros(N, dtype=np.complex128)
    lib().oracle_states(N - 1, K, _dp(U.view(np.float64)), _dp(v0.view(np.float64)),
                        _dp(psi.view(np.float64)), _dp(fin.view(np.float64)))
    return psi, fin


def solve(prob, want_U: bool = False, field_fn=None) -> dict:
    """Full solve: operators U_k, states psi_k (k < K) and psi_final.
    field_fn(t, params, field) replaces the problem's terms when given."""
    pk = _Packed(prob, field_fn)
    K, N = int(prob.n_samples), pk.dim
    v0 = np.ascontiguousarray(np.asarray(prob.psi0, dtype=np.complex128))
    psi = np.zeros((K, N), dtype=np.complex128)
    fin = np.zeros(N, dtype=np.complex128)
    U = np.zeros((K, N, N), dtype=np.complex128) if want_U else None
    rc = pk.call(lib().oracle_solve, C.byref(pk.p), _dp(pk.params), _dp(v0.view(np.float64)),
                 _dp(U.view(np.float64)) if U is not None else None,
                 _dp(psi.view(np.float64)), _dp(fin.view(np.float64)))
    if rc:
        raise ValueError("oracle_solve: bad arguments")
    return {"U": U, "psi": psi, "psi_final": fin}


def final_state_ld(prob, params_ld: np.ndarray | None = None) -> np.ndarray:
    """psi_final in x86 extended precision (long double), as complex pairs
    [N, 2] of numpy.longdouble.  ``params_ld`` overrides the parameters."""
    pk = _Packed(prob)
    N = pk.dim
    if params_ld is None:
        params_ld = np.asarray(prob.params, dtype=np.longdouble)
    pl = np.ascontiguousarray(np.asarray(params_ld, dtype=np.longdouble).ravel())
    if pl.size == 0:
        pl = np.zeros(1, dtype=np.longdouble)
    v0 = np.asarray(prob.psi0, dtype=np.complex128)
    psi0 = np.ascontiguousarray(np.stack([v0.real, v0.imag], axis=1).astype(np.longdouble))
    out = np.zeros((N, 2), dtype=np.longdouble)
    rc = lib().oracle_solve_ld(C.byref(pk.p), pl.ctypes.data, psi0.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError("oracle_solve_ld: bad arguments")
    return out


def adjoint_population(prob, m: int) -> tuple[float, np.ndarray]:
    """loss = |psi_final[m]|^2 and its gradient w.r.t. every parameter slot
    (reverse mode through the same discrete map)."""
    pk = _Packed(prob)
    v0 = np.ascontiguousarray(np.asarray(prob.psi0, dtype=np.complex128))
    loss = np.zeros(1)
    grad = np.zeros(max(1, pk.p.n_params))
    rc = lib().oracle_adjoint_population(C.byref(pk.p), _dp(pk.params), _dp(v0.view(np.float64)),
                                         int(m), _dp(loss), _dp(grad))
    if rc == 2:
        raise ValueError("gradients need parameter slots on x and y terms only")
    if rc == 3:
        raise ValueError("gradients need the CF4 method")
    if rc == 5:
        raise ValueError("gradients are not defined for the full su(3) basis")
    if rc:
        raise ValueError("oracle_adjoint_population: bad arguments")
    return float(loss[0]), grad[:pk.p.n_params].copy()


def population_ld(prob, m: int, params_ld: np.ndarray) -> np.longdouble:
    """|psi_final[m]|^2 in extended precision at the given parameters."""
    out = final_state_ld(prob, params_ld)
    return out[m, 0] * out[m, 0] + out[m, 1] * out[m, 1]


def spin_projection(psi: np.ndarray) -> np.ndarray:
    """<J_x>, <J_y>, <J_z> of each state row of psi [K, N] -> [K, 3]."""
    psi = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    K, N = psi.shape
    out = np.zeros((K, 3))
    rc = lib().oracle_spin_projection(N - 1, K, _dp(psi.view(np.float64)), _dp(out))
    if rc:
        raise ValueError("oracle_spin_projection: bad arguments")
    return out
