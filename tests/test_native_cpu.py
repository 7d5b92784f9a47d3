"""Host-only checks of the C-ABI library: it loads, exports every function
include/mss.h declares, validates problems before any launch, and sizes
workspaces.  No GPU compute is called."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2204_05586_amd import native, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mss_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function():
    L = native.lib()
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert set(native.EXPORTS) <= set(declared) | {"mss_last_error"}


def test_version_and_status_strings():
    assert "gfx950" in native.version()
    assert native.lib().mss_status_str(1).decode() == "MSS_E_INVALID"


def _bad(prob, match):
    with pytest.raises(native.MssError, match=match) as e:
        native.validate(prob)
    assert e.value.status == native.MSS_E_INVALID


def test_validation_rejects_bad_problems():
    good = W.spin_one_sensing(n_samples=10)
    native.validate(good)
    _bad(good.replace(spin_twice=3), "spin_twice")
    _bad(good.replace(n_samples=0), "n_samples")
    _bad(good.replace(n_fine=0), "n_fine")
    _bad(good.replace(dt_out=0.0), "dt_out")
    _bad(good.replace(dt_out=float("nan")), "dt_out")
    _bad(good.replace(t_start=float("inf")), "t_start")
    _bad(good.replace(n_squares=61), "n_squares")
    half = W.spin_half_rabi(n_samples=10)
    _bad(half.replace(terms=half.terms + [W.Term(W.CONST, W.Q, a=1.0)]), "quadrupole")
    _bad(good.replace(terms=[W.Term(W.COS, W.X, a_slot=3)]), "slot")
    _bad(good.replace(terms=[W.Term(9, W.X)]), "kind")
    _bad(good.replace(terms=[W.Term(W.PWC, W.X, n_seg=4, seg_len=1.0, seg_a_slot=0)],
                      params=np.zeros(3)), "segment slots")
    _bad(good.replace(terms=[W.Term(W.PWC, W.X, n_seg=4, seg_len=0.0)]), "seg_len")
    _bad(good.replace(terms=[W.Term(W.CONST, W.X, a=float("nan"))]), "finite")
    _bad(good.replace(terms=[W.Term(W.CONST, W.X)] * 33), "terms")
    # full su(3) components: spin-1 only, and no component past V_2
    for c in (W.U1, W.U2, W.V1, W.V2):
        _bad(half.replace(terms=half.terms + [W.Term(W.CONST, c, a=1.0)]), "quadrupole")
        native.validate(good.replace(terms=good.terms + [W.Term(W.COS, c, a=1.0, f=2.0)]))
    _bad(good.replace(terms=[W.Term(W.CONST, 8, a=1.0)]), "comp")


def test_workspace_sizes():
    """Per level above the operators: aggregates and entering states."""
    tile = 256
    for spin_twice, K in [(1, 1), (1, 256), (2, 257), (2, 200_000), (2, 65_537), (1, 1 << 20),
                          (1, (1 << 20) + 1)]:
        N = spin_twice + 1
        expect = 0
        n = K
        sizes = []
        while n > tile:
            n = -(-n // tile)
            sizes.append(n)
            expect += -(-(n * 2 * N * N * 8) // 256) * 256 + -(-(n * 2 * N * 8) // 256) * 256
        assert native.propagate_workspace_size(spin_twice, K) == expect
        prob = W.random_problem(np.random.default_rng(0), spin_twice, K, 3)
        assert native.workspace_size(prob, True) == expect
        assert native.workspace_size(prob, False) == expect + -(-(K * N * N * 16) // 256) * 256


def test_launch_plan_is_valid():
    for prob in [W.spin_half_rabi(), W.spin_one_sensing(), W.spin_one_sensing(n_samples=7),
                 W.spin_half_rabi(n_samples=1, n_fine=1)]:
        S, B = native.plan_launch(prob)
        assert S >= 1 and S & (S - 1) == 0 and S <= min(64, prob.n_fine)
        assert B in (64, 128, 256)


def test_launch_plan_block_follows_the_wave_count():
    """Launches of at most 3 waves per SIMD (a 256-CU device when none is
    visible: 3072 waves) take one-wave workgroups, longer ones 256 lanes;
    a given block is kept."""
    half = W.spin_half_rabi()                       # 1e4 intervals x 16 slices: 2,500 waves
    assert native.plan_launch(half) == (16, 64)
    assert native.plan_launch(W.spin_one_sensing()) == (2, 256)   # 6,250 waves
    big = W.spin_half_rabi(n_samples=200_000)
    S, B = native.plan_launch(big)
    assert B == (64 if (big.n_samples * S + 63) // 64 <= 3072 else 256)


def test_solve_requires_buffers():
    prob = W.spin_half_rabi(n_samples=4)
    pk = native.PackedProblem(prob)
    st = native.lib().mss_solve(pk.ref, None, None, None, None, None, None, None, 0, None)
    assert st == native.MSS_E_INVALID
    assert "psi0" in native.last_error()


def test_errors_raise_as_python_kinds():
    """Invalid arguments raise ValueError, an impossible workspace
    MemoryError, both still MssError with the status code."""
    bad = W.spin_half_rabi(n_samples=4).replace(n_fine=0)
    with pytest.raises(ValueError) as e:
        native.check(native.lib().mss_validate(native.PackedProblem(bad).ref))
    assert isinstance(e.value, native.MssError) and e.value.status == native.MSS_E_INVALID
    with pytest.raises(MemoryError) as e:
        native.check(native.MSS_E_NOMEM)
    assert isinstance(e.value, native.MssError)


def test_compiled_adjoint_checks_its_sampler_before_any_allocation():
    """mss_adjoint_plan_create_compiled refuses a NULL sampler and one not
    generated from the problems' terms, before touching the device."""
    probs = W.control_batch(seed=6, n_inst=2, n_samples=20, n_fine=4)
    arr = (native.Problem * 2)()
    packed = [native.PackedProblem(p) for p in probs]
    for i, pk in enumerate(packed):
        arr[i] = pk.c
    offs = np.array([0, len(probs[0].params)], dtype=np.int64)
    offp = offs.ctypes.data_as(C.POINTER(C.c_int64))
    L = native.lib()
    st = L.mss_adjoint_plan_create_compiled(2, arr, offp, 1, None, C.byref(C.c_void_p()))
    assert st == native.MSS_E_INVALID and "NULL" in native.last_error()
    other = native.Sampler.for_terms(probs[0].terms[:1])
    st = L.mss_adjoint_plan_create_compiled(2, arr, offp, 1, other._h, C.byref(C.c_void_p()))
    assert st == native.MSS_E_INVALID and "not generated from its terms" in native.last_error()
    other.close()
    # a problem that claims terms but passes none is refused, not read
    own = native.Sampler.for_terms(probs[0].terms)
    arr[1].terms = None
    st = L.mss_adjoint_plan_create_compiled(2, arr, offp, 1, own._h, C.byref(C.c_void_p()))
    assert st == native.MSS_E_INVALID and "terms is NULL" in native.last_error()
    own.close()


def test_propagate_spin_requires_output():
    L = native.lib()
    buf = (C.c_double * 64)()
    st = L.mss_propagate_spin(1, 4, buf, buf, buf, None, None, None, 0, None)
    assert st == native.MSS_E_INVALID and "spin" in native.last_error()
    st = L.mss_propagate_spin(3, 4, buf, buf, buf, None, buf, None, 0, None)
    assert st == native.MSS_E_INVALID and "spin_twice" in native.last_error()


def test_batch_check_rejects_a_null_plan():
    """mss_batch_check validates its plan before any device call."""
    st = native.lib().mss_batch_check(None, None, None)
    assert st == native.MSS_E_INVALID and "plan" in native.last_error()


def test_propagate_noalloc_checks_before_any_device_call():
    """Bad arguments and sizes beyond the static scratch are refused on the
    host (this container has no GPU, so any device call would fail)."""
    L = native.lib()
    buf = (C.c_double * 64)()
    for spin_twice, kmax in ((2, 11_141_120), (1, 22_280_192)):
        st = L.mss_propagate_noalloc(spin_twice, kmax + 1, buf, buf, buf, None, None)
        assert st == native.MSS_E_INVALID and "scan scratch" in native.last_error()
        assert native.propagate_workspace_size(spin_twice, kmax) <= 8 << 20
    st = L.mss_propagate_noalloc(3, 4, buf, buf, buf, None, None)
    assert st == native.MSS_E_INVALID and "spin_twice" in native.last_error()
    st = L.mss_propagate_noalloc(2, 0, buf, buf, buf, None, None)
    assert st == native.MSS_E_INVALID and "n_samples" in native.last_error()


def test_one_shot_calls_check_before_any_device_call():
    L = native.lib()
    buf = (C.c_double * 64)()
    probs = [W.spin_half_rabi(n_samples=10, n_fine=2)]
    packed = [native.PackedProblem(p) for p in probs]
    arr = (native.Problem * 1)(packed[0].c)
    st = L.mss_solve_batch(1, arr, None, None, buf, None, None, None, None)
    assert st == native.MSS_E_INVALID and "psi" in native.last_error()
    st = L.mss_solve_batch(0, arr, None, None, buf, buf, None, None, None)
    assert st == native.MSS_E_INVALID and "at least one" in native.last_error()
    st = L.mss_adjoint_population(0, arr, None, 0, None, buf, buf, buf, None, None)
    assert st == native.MSS_E_INVALID


# ---- user field samplers (compiled at run time; needs no GPU) ---------------

def test_sampler_compiles_without_gpu():
    from tests import user_fields as F
    s = native.Sampler(F.CHIRP_SOURCE)
    assert isinstance(s.log, str)
    s.close()
    s.close()  # idempotent


def test_sampler_options_are_passed():
    src = "#ifndef AMP\n#error AMP undefined\n#endif\n" \
          "__device__ void mss_user_field(double t, const double* p, double* f) { f[0] = AMP; }\n"
    with pytest.raises(native.MssError, match="AMP undefined"):
        native.Sampler(src)
    native.Sampler(src, options=["-DAMP=2.0"]).close()


def test_sampler_compile_errors_name_the_user_line():
    src = "__device__ void mss_user_field(double t, const double* p, double* f) {\n" \
          "  f[0] = undefined_thing;\n}\n"
    with pytest.raises(native.MssError, match=r"user_field\.hip:2:.*undefined_thing") as e:
        native.Sampler(src)
    assert e.value.status == native.MSS_E_INVALID
    with pytest.raises(native.MssError, match="mss_user_field"):
        native.Sampler("int unrelated;")


def _kinds_terms(quad):
    T = W.Term
    terms = [T(W.CONST, W.Z, a=1.0e3), T(W.COS, W.X, a=2.0e2, f=1.0e3, phi=0.3),
             T(W.SIN, W.Y, a_slot=0, f_slot=1, phi_slot=2, t_on=1e-3, t_off=2e-3),
             T(W.PWC, W.X, n_seg=4, seg_a_slot=3, seg_t0=0.0, seg_len=1e-3),
             T(W.PWC_COS, W.X, f=5.0, n_seg=3, seg_a_slot=7, seg_phi_slot=10, seg_t0=0.0,
               seg_len=1e-3, t_off=0.5),
             T(W.PWC_SIN, W.Y, a=2.0, f=7.0, n_seg=2, seg_phi_slot=13, seg_t0=-1.0, seg_len=0.5,
               t_on=-0.1),
             T(W.COS, W.X, a=1.0, f=1.0, t_on=1.0, t_off=1.0)]
    if quad:
        terms.append(T(W.CONST, W.Q, a=-0.0))
    return terms


def test_sampler_for_terms_compiles_without_gpu():
    """Every term kind compiles into a specialised sampler; it needs the
    parameters up to the highest slot read (segment slots count n_seg)."""
    for quad in (False, True):
        s = native.Sampler.for_terms(_kinds_terms(quad))
        assert s.min_params == 15 and s.terms is not None
        s.close()
    s = native.Sampler.for_terms([])
    assert s.min_params == 0
    s.close()
    assert native.lib().mss_sampler_min_params(None) == 0


def test_sampler_for_terms_rejects_invalid_terms():
    T = W.Term
    for bad, msg in [([T(W.PWC, W.X, n_seg=0, seg_t0=0.0, seg_len=1.0)], "n_seg"),
                     ([T(7, W.X)], "unknown kind"),
                     ([T(W.COS, W.X, a=float("nan"))], "finite"),
                     ([T(W.CONST, W.X, t_on=float("nan"))], "NaN window"),
                     ([T(W.PWC, W.X, n_seg=2, seg_t0=0.0, seg_len=0.0)], "seg_len")]:
        with pytest.raises(native.MssError, match=msg):
            native.Sampler.for_terms(bad)
    h = C.c_void_p()
    assert native.lib().mss_sampler_create_for_terms(None, 1, C.byref(h)) == native.MSS_E_INVALID
    assert native.lib().mss_sampler_create_for_terms(None, 0, None) == native.MSS_E_INVALID


def test_full_basis_is_interpreted_and_has_no_adjoint():
    """Field programs on U_1, U_2, V_1, V_2 are not compiled into samplers (the
    batch plan keeps interpreting them) and have no adjoint."""
    T = W.Term
    terms = [T(W.CONST, W.Z, a=1e3), T(W.COS, W.V1, a=10.0, f=1e3)]
    with pytest.raises(native.MssError, match="su\\(3\\)") as e:
        native.Sampler.for_terms(terms)
    assert e.value.status == native.MSS_E_UNSUPPORTED
    assert native.specialise([W.Problem(2, terms, 0.0, 1e-6, 10, 2, 28, True)]) is None


def test_sampler_for_terms_checks_problems_before_launch():
    """A problem run with a specialised sampler carries the parameters its
    terms read, and spin-1 when they include a quadrupole term; the batch
    plan checks every simulation the same way.  All rejected before any
    device work."""
    s = native.Sampler.for_terms(_kinds_terms(True))
    L = native.lib()
    dummy = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    short = W.Problem(2, [], 0.0, 1e-6, 10, 2, 28, True, params=np.zeros(14))
    pk = native.PackedProblem(short)
    assert L.mss_sampler_integrate(s._h, pk.ref, dummy, dummy, None, None, None) == native.MSS_E_INVALID
    assert "15 parameters" in native.last_error()
    half = W.Problem(1, [], 0.0, 1e-6, 10, 2, 28, True, params=np.zeros(15))
    pk = native.PackedProblem(half)
    assert L.mss_sampler_integrate(s._h, pk.ref, dummy, dummy, None, None, None) == native.MSS_E_INVALID
    assert "spin-1 only" in native.last_error()
    with pytest.raises(native.MssError, match="15 parameters"):
        native.BatchPlan([short.replace(params=np.zeros(15)), short], sampler=s)
    s.close()


def test_sampler_integrate_validates_before_launch():
    from tests import user_fields as F
    s = native.Sampler(F.LZ_SOURCE)
    L = native.lib()
    prob = W.Problem(1, [W.Term(W.CONST, W.Z, a=1.0)], 0.0, 1e-6, 10, 2, 28, True)
    pk = native.PackedProblem(prob)
    dummy = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert L.mss_sampler_integrate(s._h, pk.ref, None, dummy, None, None, None) == native.MSS_E_INVALID
    assert "no terms" in native.last_error()
    pk = native.PackedProblem(prob.replace(terms=[], params=np.zeros(3)))
    assert L.mss_sampler_integrate(s._h, pk.ref, None, dummy, None, None, None) == native.MSS_E_INVALID
    assert "params" in native.last_error()
    assert L.mss_sampler_integrate(None, pk.ref, None, dummy, None, None, None) == native.MSS_E_INVALID
    s.close()
