"""Shared pieces of the GPU parity tests.

* ``scheme(g, dx, dt, tau, ...)``: the scheme parameters an oracle twin takes
  from a stepper, each asserted against the value the test derives itself
  from the recipe it asked for (supplement, numerical configuration:
  ``lam = dt/dx``, ``omega = 1/tau_LB`` for conserved fields, ``1/(g_tau + 1)``
  for trackers, ``tau_grad = g_tau dt``) before the oracle is built from it.
  With single-precision arithmetic the library rounds ``dt/dx`` once to
  float, puts ``2 - omega`` on the 2^-24 grid and rounds the reference state
  to float; each reported value may differ from the test's by that one
  rounding and by nothing else.  With FP64 storage they must agree to the
  last bit of a double division.
* ``check_fields``: relative L2 (the validation section's norm) and
  relative L-infinity (max |a - b| / max |b|) per field group, both printed
  and asserted.  The L-infinity bar is ``LINF_FACTOR`` times the L2 bar: the
  rounding errors of single-precision storage behave like a smooth random
  field, whose maximum over 10^4 - 10^7 cells sits about 4-5 standard
  deviations out, while the maximum of the reference field is one to three
  times its RMS.  Where the flow itself amplifies rounding (a steepening
  front), the binary32 storage floor -- the FP64 oracle against itself with
  its populations rounded to binary32 every step, written by
  ``tests/golden/make_storage_floor.py`` -- can exceed that bar in a few
  cells; a test then passes ``floor`` and the group's L-infinity bar becomes
  ``FLOOR_FACTOR`` times the floor's, if that is larger.
"""
from __future__ import annotations

import math

import numpy as np

F32_STEP = 2.0 ** -24          # unit roundoff of binary32 (round to nearest)
F64_STEP = 2.0 ** -52
LINF_FACTOR = 5.0
FLOOR_FACTOR = 2.0


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def rel_linf(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b))) / float(np.max(np.abs(b)))


def linf_bar(tol, floor_linf=None):
    """L-infinity bar of a group with L2 bar tol and, if given, the
    storage floor's L-infinity distance."""
    bar = LINF_FACTOR * tol
    return bar if floor_linf is None else max(bar, FLOOR_FACTOR * floor_linf)


def check_fields(groups, Qg, Qo, tol, label="", floor=None):
    """Per field group (name -> index or slice into axis 0): relative L2 <=
    tol and relative L-infinity <= linf_bar(tol, floor[name]["linf"]) (floor:
    a storage-floor record of the group, or None).  Returns {name: (l2, linf)}."""
    out = {}
    for name, s in groups.items():
        e2, ei = rel_l2(Qg[s], Qo[s]), rel_linf(Qg[s], Qo[s])
        out[name] = (e2, ei)
        fl = "" if not floor else f"  (storage floor: L2 {floor[name]['l2']:.3e}, Linf {floor[name]['linf']:.3e})"
        print(f"{label}{name}: rel L2 {e2:.3e}  rel Linf {ei:.3e}{fl}", flush=True)
    for name, (e2, ei) in out.items():
        bar = linf_bar(tol, floor[name]["linf"] if floor else None)
        assert e2 <= tol, f"{label}{name}: rel L2 {e2:.3e} > {tol:.1e}"
        assert ei <= bar, f"{label}{name}: rel Linf {ei:.3e} > {bar:.1e}"
    return out


def _near(got, want, rel, what):
    assert abs(got - want) <= rel * abs(want) + 1e-300, f"{what}: library {got!r}, recipe {want!r}"


def scheme(g, dx, dt, tau, g_tau=None, Q0=None, trt_lambda=None):
    """Parameters in use by stepper ``g``, checked against the recipe values
    (dx, dt, tau_LB, g_tau, reference Q0) the test asked for.  Returns the
    keyword arguments of the oracle twin: dt, dx, tau, g_tau, Q0 and, where
    they apply, omega_tracker, omega_plus, omega_plus_tracker."""
    single = g.storage != "f64"
    r = F32_STEP if single else F64_STEP
    assert g.param("dx") == dx, "dx"
    lam = dt / dx
    _near(g.param("lambda"), lam, r, "lambda = dt/dx")
    _near(g.param("dt"), dt, r + 2 * F64_STEP, "dt")
    # conserved fields relax at 1/tau_LB; single precision moves 2 - omega
    # to the nearest point of the 2^-24 grid (at most half a step)
    om = 1.0 / tau
    om_tol = (F32_STEP / 2 if single else 2 * F64_STEP) * (4.0 if trt_lambda else 1.0)
    assert abs(g.param("omega") - om) <= om_tol, f"omega: library {g.param('omega')!r}, recipe {om!r}"
    out = {"dt": g.param("dt"), "dx": g.param("dx"), "tau": 1.0 / g.param("omega"), "g_tau": None,
           "Q0": g.reference}
    if g_tau is not None:
        assert g.param("g_tau") == g_tau, "g_tau"
        # trackers: tau_grad = g_tau dt inside flux and source, collision rate 1/(g_tau + 1)
        _near(g.param("tau_grad"), g_tau * dt, r + 4 * F64_STEP, "tau_grad = g_tau dt")
        omt = 1.0 / (g_tau + 1.0)
        assert abs(g.param("omega_tracker") - omt) <= om_tol, "omega_tracker = 1/(g_tau + 1)"
        out["g_tau"] = g_tau
        out["omega_tracker"] = g.param("omega_tracker")
    if trt_lambda:
        # symmetric rate from the magic parameter (1/w+ - 1/2)(1/w- - 1/2) = Lambda
        for key, wm in (("omega_plus", om), ("omega_plus_tracker", 1.0 / (g_tau + 1.0) if g_tau else om)):
            wp = 1.0 / (0.5 + trt_lambda / (1.0 / wm - 0.5))
            got = g.param(key)
            assert abs(got - wp) <= 4 * om_tol, f"{key}: library {got!r}, magic parameter gives {wp!r}"
            out[key] = got
    if Q0 is not None:
        ref = g.reference
        Q0 = np.asarray(Q0, dtype=np.float64)
        assert ref.shape == Q0.shape
        for k in range(len(Q0)):
            assert abs(ref[k] - Q0[k]) <= (F32_STEP if single else 0.0) * abs(Q0[k]), f"reference Q0[{k}]"
    return out


def recipe(n, scaling, f, tau_r):
    """(dx, dt, tau_LB) of the supplement's refinement recipe, derived here:
    dx = 1/N, dt = f dx (acoustic) or f dx^2 (diffusive), tau_LB = 1/2 + tau_R dt."""
    dx = 1.0 / n
    dt = f * dx if scaling == "acoustic" else f * dx * dx
    return dx, dt, 0.5 + tau_r * dt
