"""The C ABI library loads and exports every entry point include/lbm.h
declares; host-only calls validate their arguments.  CPU only: nothing here
launches a kernel."""
import ctypes
import os
import re

import pytest

from paper_2607_05668_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = lbm.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    # and nothing else public
    out = os.popen(f"nm -D --defined-only {lbm.LIB_PATH}").read()
    exported = sorted(set(m for m in re.findall(r" T (lbm_\w+)", out)))
    assert exported == _declared()


def test_create_validates_arguments():
    lib = lbm.load_library()
    assert not lib.lbm_create(b"nope", b"D2Q9", 64, 64, 1, 0.6, 1e-3, 1e-2)
    assert b"unknown system" in lib.lbm_last_error(None)
    assert not lib.lbm_create(b"swe2d", b"D3Q7", 64, 64, 1, 0.6, 1e-3, 1e-2)
    assert not lib.lbm_create(b"swe2d", b"D2Q9", 64, 64, 2, 0.6, 1e-3, 1e-2)
    assert not lib.lbm_create(b"swe2d", b"D2Q9", 0, 64, 1, 0.6, 1e-3, 1e-2)
    assert b"invalid grid" in lib.lbm_last_error(None)
    assert not lib.lbm_create(b"swe2d", b"D2Q9", 64, 64, 1, 0.5, 1e-3, 1e-2)
    h = lib.lbm_create(b"swe2d", b"D2Q9", 64, 32, 1, 0.6, 1e-3, 1e-2)
    assert h
    h = ctypes.c_void_p(h)
    assert lib.lbm_num_fields(h) == 3 and lib.lbm_num_velocities(h) == 9
    assert lib.lbm_required_bytes(h, 0) == 3 * 9 * 64 * 32 * 4
    assert lib.lbm_set_storage(h, lbm.F16) == 0
    assert lib.lbm_required_bytes(h, 0) == 3 * 9 * 64 * 32 * 2
    assert lib.lbm_set_storage(h, 7) == lbm.LBM_EINVAL
    # tile-blocked layout: each z-slab padded to whole tiles of 64 cells
    r = ctypes.c_void_p(lib.lbm_create(b"nsf3d_trk17", b"D3Q7", 50, 37, 3, 0.6, 1e-3, 1e-2))
    assert lib.lbm_required_bytes(r, 0) == 17 * 7 * 3 * (50 * 37 + 6) * 4
    lib.lbm_destroy(r)
    assert lib.lbm_set_param(h, b"g", 9.81) == 0
    assert lib.lbm_set_param(h, b"mu", 1.0) == lbm.LBM_EINVAL
    assert b"unknown parameter" in lib.lbm_last_error(h)
    assert lib.lbm_step(h, 1) == lbm.LBM_ENOTBOUND
    assert lib.lbm_bind(h, None, None, None, None) == lbm.LBM_EINVAL
    lib.lbm_destroy(h)


def test_tracker_systems_need_g_tau():
    lib = lbm.load_library()
    h = ctypes.c_void_p(lib.lbm_create(b"advdiff_trk2d", b"D2Q5", 64, 64, 1, 0.6, 1e-3, 1e-2))
    # fake, aligned, distinct addresses: bind fails on the missing g_tau before
    # anything is dereferenced
    assert lib.lbm_bind(h, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(768), None) == lbm.LBM_EINVAL
    assert b"g_tau" in lib.lbm_last_error(h)
    lib.lbm_destroy(h)


def test_reference_rounds_to_float_for_single_precision_storage():
    lib = lbm.load_library()
    h = ctypes.c_void_p(lib.lbm_create(b"swe2d", b"D2Q9", 64, 64, 1, 0.6, 1e-3, 1e-2))
    import numpy as np
    q0 = np.array([1.1, 0.1, 0.0])
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.lbm_set_reference(h, q0.ctypes.data_as(dp)) == 0
    out = np.zeros(3)
    lib.lbm_get_reference(h, out.ctypes.data_as(dp))
    assert np.all(out == np.float32(q0).astype(np.float64))
    lib.lbm_destroy(h)


def test_hcnsf_reference_and_coefficient_field_validation():
    """hcnsf3d_trk14: default reference is the Mach-0.5 background (trackers
    zero); a reference with non-zero trackers is rejected (the flux's
    reference value must not depend on the porosity); the coefficient field
    is named "coef" and other systems do not take it."""
    import math

    import numpy as np
    lib = lbm.load_library()
    dp = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p(lib.lbm_create(b"hcnsf3d_trk14", b"D3Q7", 8, 8, 8, 0.6, 1e-3, 1e-2))
    assert h.value and lib.lbm_num_fields(h) == 14
    assert lib.lbm_set_storage(h, lbm.STORAGE["f64"]) == 0
    q0 = np.zeros(14)
    assert lib.lbm_get_reference(h, q0.ctypes.data_as(dp)) == 0
    u0 = 0.5 * math.sqrt(1.4)
    assert np.allclose(q0[:5], [1, u0, u0, u0, 2.5 + 1.5 * u0 * u0], rtol=1e-15) and not q0[5:].any()
    bad = q0.copy()
    bad[7] = 1e-3
    assert lib.lbm_set_reference(h, bad.ctypes.data_as(dp)) == lbm.LBM_EINVAL
    assert b"trackers" in lib.lbm_last_error(h)
    assert lib.lbm_set_field(h, b"coef", None) == 0
    assert lib.lbm_set_field(h, b"grad_zb", None) == lbm.LBM_EINVAL
    assert lib.lbm_set_param(h, b"eta", 0.0) == lbm.LBM_EINVAL
    lib.lbm_destroy(h)
    h = ctypes.c_void_p(lib.lbm_create(b"swe2d", b"D2Q9", 8, 8, 1, 0.6, 1e-3, 1e-2))
    assert lib.lbm_set_field(h, b"coef", None) == lbm.LBM_EINVAL
    lib.lbm_destroy(h)
    assert not lib.lbm_create(b"hcnsf3d_trk14", b"D2Q5", 8, 8, 1, 0.6, 1e-3, 1e-2)


def test_trt_parameters_and_bgk_only_paths():
    """trt_lambda: the rates in use after binding (omega- = the BGK rate,
    omega+ from the magic parameter, single-precision rounding of
    a = (omega+ + omega-)/2 and b = (omega+ - omega-)/2), rejection of the
    moment history / adjoint and of F16NE storage.  Binding with stand-in
    addresses touches no memory."""
    import numpy as np
    lib = lbm.load_library()
    v = ctypes.c_double()
    for storage, rtol in (("f64", 1e-15), ("f32", 1e-6)):
        h = ctypes.c_void_p(lib.lbm_create(b"swe2d", b"D2Q9", 64, 64, 1, 0.6, 1e-3, 1e-2))
        assert lib.lbm_set_param(h, b"trt_lambda", -1.0) == lbm.LBM_EINVAL
        assert lib.lbm_set_param(h, b"trt_lambda", 0.1875) == 0
        assert lib.lbm_set_storage(h, lbm.STORAGE[storage]) == 0
        assert lib.lbm_get_param(h, b"omega_plus", ctypes.byref(v)) == lbm.LBM_EINVAL    # not bound yet
        assert lib.lbm_bind(h, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(768), None) == 0
        lib.lbm_get_param(h, b"omega", ctypes.byref(v))
        wm = v.value
        lib.lbm_get_param(h, b"omega_plus", ctypes.byref(v))
        wp = v.value
        assert wm == pytest.approx(1 / 0.6, rel=rtol)
        assert (1 / wp - 0.5) * (1 / wm - 0.5) == pytest.approx(0.1875, rel=10 * rtol)
        if storage == "f32":
            a, b = 0.5 * (wp + wm), 0.5 * (wp - wm)
            assert np.float32(a) == a and np.float32(a - 1) == a - 1 and np.float32(b) == b
        assert lib.lbm_step_record(h, 1, ctypes.c_void_p(1024)) == lbm.LBM_EINVAL
        assert b"BGK" in lib.lbm_last_error(h)
        assert lib.lbm_adjoint_seed(h, ctypes.c_void_p(1024), ctypes.c_void_p(2048)) == lbm.LBM_EINVAL
        lib.lbm_destroy(h)
    h = ctypes.c_void_p(lib.lbm_create(b"neohooke2d", b"D2Q9", 64, 64, 1, 0.6, 1e-3, 1e-2))
    lib.lbm_set_param(h, b"trt_lambda", 0.25)
    lib.lbm_set_storage(h, lbm.STORAGE["f16ne"])
    assert lib.lbm_bind(h, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(768), None) == lbm.LBM_EINVAL
    lib.lbm_destroy(h)


def test_default_references():
    """Each system's default reference state (the shifted form's Q0)."""
    import numpy as np
    lib = lbm.load_library()
    dp = ctypes.POINTER(ctypes.c_double)
    cases = {b"burgers2d": [0.0], b"maxwell2d": [0.0, 0.0, 0.0], b"allencahn_trk2d": [0.0, 0.0, 0.0],
             b"swe2d": [1.0, 0.0, 0.0], b"euler2d": [1.0, 3.0, 3.0, 1 / 1.4 / 0.4 + 9.0],
             b"gen_euler2d": [1.0, 3.0, 3.0, 1 / 1.4 / 0.4 + 9.0], b"gen_advdiff_trk2d": [1.0, 0.0, 0.0]}
    for name, want in cases.items():
        h = ctypes.c_void_p(lib.lbm_create(name, b"D2Q5", 16, 16, 1, 0.6, 1e-3, 1e-2))
        assert h.value, name
        lib.lbm_set_storage(h, lbm.STORAGE["f64"])
        out = np.zeros(len(want))
        assert lib.lbm_get_reference(h, out.ctypes.data_as(dp)) == 0
        assert np.allclose(out, want, rtol=1e-15, atol=0), name
        lib.lbm_destroy(h)


def test_regularized_parameter_rules():
    lib = lbm.load_library()
    v = ctypes.c_double()
    h = ctypes.c_void_p(lib.lbm_create(b"swe2d", b"D2Q9", 64, 64, 1, 0.6, 1e-3, 1e-2))
    assert lib.lbm_set_param(h, b"regularized", 0.5) == lbm.LBM_EINVAL
    assert lib.lbm_set_param(h, b"regularized", 1.0) == 0
    assert lib.lbm_get_param(h, b"regularized", ctypes.byref(v)) == 0 and v.value == 1.0
    assert lib.lbm_set_param(h, b"trt_lambda", 0.25) == 0
    assert lib.lbm_bind(h, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(768), None) == lbm.LBM_EINVAL
    assert lib.lbm_set_param(h, b"trt_lambda", 0.0) == 0
    assert lib.lbm_bind(h, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(768), None) == 0
    assert lib.lbm_set_param(h, b"regularized", 0.0) == lbm.LBM_EINVAL    # fixed once bound
    assert lib.lbm_step_record(h, 1, ctypes.c_void_p(1024)) == lbm.LBM_EINVAL
    lib.lbm_destroy(h)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No CPU fallback: without the built HIP library the binding raises
    instead of computing anything."""
    monkeypatch.setattr(lbm, "LIB_PATH", str(tmp_path / "liblbm.so"))
    monkeypatch.setattr(lbm, "_lib", None)
    with pytest.raises(ImportError, match="not built"):
        lbm.load_library()


def test_check_every_and_static_reduce_host_checks():
    """Failure-detection interval: a non-negative whole step count, readable
    back; the static-workspace reduction refuses an unbound handle."""
    lib = lbm.load_library()
    h = ctypes.c_void_p(lib.lbm_create(b"swe2d", b"D2Q9", 64, 64, 1, 0.6, 1e-3, 1e-2))
    assert lib.lbm_set_param(h, b"check_every", -1.0) == lbm.LBM_EINVAL
    assert lib.lbm_set_param(h, b"check_every", 2.5) == lbm.LBM_EINVAL
    assert lib.lbm_set_param(h, b"check_every", 5.0) == 0
    v = ctypes.c_double()
    assert lib.lbm_get_param(h, b"check_every", ctypes.byref(v)) == 0 and v.value == 5.0
    out = (ctypes.c_double * 36)()
    assert lib.lbm_reduce_static(h, lbm.RED_SUMS, None, out) == lbm.LBM_ENOTBOUND
    lib.lbm_destroy(h)
