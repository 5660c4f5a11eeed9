"""Writes storage_floor.json: the binary32 storage floor of a workload -- the
relative L2 and L-infinity distance, per field group, between the FP64
oracle and the same oracle whose populations are rounded to binary32 after
the initialisation and after every step.  No single-precision stepper that
stores its populations in binary32 can be expected to sit closer to the FP64
oracle than this, element by element: where the flow amplifies rounding
(a steepening front), the floor's L-infinity distance shows by how much.

Cases (argument, default all):
  c2       shallow water, D2Q9, 1024^2 periodic, acoustic recipe f = 0.2,
           tau_R = 2, g = 1, 1000 steps, reference (1, 0, 0), initial
           fields inputs.swe_initial(1024)
  c3_64,   3D compressible NSF with 9 + 3 trackers, D3Q7, 64^3 / 128^3,
  c3_128   the configuration's recipe (acoustic f = 0.05, tau_R = 20,
           g_tau = 3), 500 steps of the manufactured solution with its
           forcing (SymPy residual, generated C), reference = background
  hcnsf_f16  homogenized NSF (14 fields), D3Q7, 24^3, acoustic f = 0.05,
           tau_R = 20, g_tau = 3, 60 steps from the manufactured state at
           t = 0.4 with its porosity / solid-velocity field held fixed
           (float32 values), reference = background, binary16 as for c5
  c5_f16_tau20,  neo-Hookean elastodynamics, D2Q9, 256^2, acoustic
  c5_f16_tau2    f = 0.1, tau_R = 20 (the binary16 recipe) or 2 (the
           single-precision rate), 2000 steps from inputs.neohooke_initial,
           reference F = I, v = 0; the populations rounded to binary16 after
           a per-field power-of-two scale 2^floor(log2(2048 / max |f_k|))
           chosen on the initial populations (the FP16 storage's rule)

Calls only the oracle, its forcing and the seeded input generators; c2
takes about five minutes on eight cores, c3_128 about half an hour.  Run
from the repository root:

    python tests/golden/make_storage_floor.py [c2 c3_64 c3_128 c5_f16_tau20 c5_f16_tau2]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import mms  # noqa: E402
from paper_2607_05668_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "storage_floor.json")


def _rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def _rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _binary32(f):
    return f.astype(np.float32).astype(np.float64)


def _binary16_rounder(f0):
    """Rounding to scaled binary16 with per-field scales 2^e, e =
    floor(log2(2048 / max |f_k|)) over the initial populations f0 [K, ...]."""
    K = f0.shape[0]
    m = np.abs(f0.reshape(K, -1)).max(axis=1)
    e = np.where(m > 0, np.floor(np.log2(2048.0 / np.where(m > 0, m, 1.0))), 0.0).clip(-24, 24)
    s = (2.0 ** e).reshape((K,) + (1,) * (f0.ndim - 1))
    return lambda f: (f * s).astype(np.float16).astype(np.float64) / s


def floor_run(make, Q, steps, groups, report_every=100, source=None, storage="binary32", coef=None):
    """(exact, rounded) oracle pair over `steps` (source(t): explicit source
    at t, or None; storage: binary32, or binary16 with per-field scales;
    coef: a fixed per-cell coefficient field, or None); returns
    {group: {l2, linf}}."""
    a, b = make(), make()
    a.init(Q, b=coef)
    b.init(Q, b=coef)
    rnd = _binary32 if storage == "binary32" else _binary16_rounder(b.f)
    b.f = rnd(b.f)
    t0 = time.time()
    while a.nsteps < steps:
        S = None if source is None else source(a.t + 0.5 * a.dt)
        a.step(1, source=None if S is None else (lambda t: S), b=coef)
        b.step(1, source=None if S is None else (lambda t: S), b=coef)
        b.f = rnd(b.f)
        if a.nsteps % report_every == 0:
            print(f"  step {a.nsteps}/{steps} ({time.time() - t0:.0f} s)", flush=True)
    Qa, Qb = a.moments(), b.moments()
    return {name: {"l2": _rel_l2(Qb[s], Qa[s]), "linf": _rel_linf(Qb[s], Qa[s])} for name, s in groups.items()}


def case_c2():
    n, steps, f, tau_r = 1024, 1000, 0.2, 2.0
    dx, dt, tau = oracle.recipe(n, "acoustic", f, tau_r)

    def make():
        return oracle.Oracle("swe2d", "D2Q9", (n, n), dt, dx, tau, None, {"g": 1.0}, Q0=[1.0, 0.0, 0.0])
    res = floor_run(make, inputs.swe_initial(n), steps, {"h": slice(0, 1), "hu": slice(1, 3)})
    return {"system": "swe2d", "lattice": "D2Q9", "n": n, "steps": steps, "f": f, "tau_r": tau_r, "groups": res}


def case_c3(n):
    steps, f, tau_r, g_tau = 500, 0.05, 20.0, 3.0
    dx, dt, tau = oracle.recipe(n, "acoustic", f, tau_r)
    m = inputs.NsfMms()
    par = {k: v for k, v in inputs.nsf_params(m).items() if k in ("gamma", "mu", "kappa")}

    def make():
        return oracle.Oracle("nsf3d_trk17", "D3Q7", (n, n, n), dt, dx, tau, g_tau, par, Q0=m.reference(),
                             omega_tracker=1.0 / (g_tau + 1.0))
    _, fS = mms.nsf17(m.gamma, m.rho0, m.p0, m.u0, m.amp, m.mu, m.kappa, g_tau * dt)
    fS = mms.compiled(fS)
    X, Y, Z = inputs.grid3(n)
    groups = {"rho": slice(0, 1), "m": slice(1, 4), "E": slice(4, 5), "G_u": slice(5, 14), "G_T": slice(14, 17)}
    res = floor_run(make, inputs.nsf_exact(n, 0.0, m), steps, groups, 50, source=lambda t: fS(X, Y, Z, t))
    return {"system": "nsf3d_trk17", "lattice": "D3Q7", "n": n, "steps": steps, "f": f, "tau_r": tau_r,
            "g_tau": g_tau, "groups": res}


def case_c5(tau_r):
    n, steps, f = 256, 2000, 0.1
    dx, dt, tau = oracle.recipe(n, "acoustic", f, tau_r)
    par = {"rho0": 1.0, "mu_s": 1.0, "lambda_s": 2.0}

    def make():
        return oracle.Oracle("neohooke2d", "D2Q9", (n, n), dt, dx, tau, None, par,
                             Q0=[1.0, 0.0, 0.0, 1.0, 0.0, 0.0])
    res = floor_run(make, inputs.neohooke_initial(n), steps, {"F": slice(0, 4), "v": slice(4, 6)}, 250,
                    storage="binary16")
    return {"system": "neohooke2d", "lattice": "D2Q9", "n": n, "steps": steps, "f": f, "tau_r": tau_r,
            "storage": "binary16, per-field power-of-two scale", "groups": res}


def case_hcnsf_f16():
    n, steps, f, tau_r, g_tau = 24, 60, 0.05, 20.0, 3.0
    dx, dt, tau = oracle.recipe(n, "acoustic", f, tau_r)
    par = {k: inputs.PRESETS["hcnsf256"].params[k] for k in ("gamma", "mu", "kappa", "eta")}
    coef = inputs.hcnsf_coefficients(n, 0.4).astype(np.float32).astype(np.float64)

    def make():
        return oracle.Oracle("hcnsf3d_trk14", "D3Q7", (n, n, n), dt, dx, tau, g_tau, par,
                             Q0=np.concatenate([inputs.HCNSF_MMS.reference()[:5], np.zeros(9)]),
                             omega_tracker=1.0 / (g_tau + 1.0))
    groups = {"rho": slice(0, 1), "m": slice(1, 4), "E": slice(4, 5), "G_u": slice(5, 11), "G_T": slice(11, 14)}
    res = floor_run(make, inputs.hcnsf_exact(n, 0.4), steps, groups, 20, storage="binary16", coef=coef)
    return {"system": "hcnsf3d_trk14", "lattice": "D3Q7", "n": n, "steps": steps, "f": f, "tau_r": tau_r,
            "g_tau": g_tau, "storage": "binary16, per-field power-of-two scale", "groups": res}


CASES = {"c2": case_c2, "c3_64": lambda: case_c3(64), "c3_128": lambda: case_c3(128),
         "c5_f16_tau20": lambda: case_c5(20.0), "c5_f16_tau2": lambda: case_c5(2.0), "hcnsf_f16": case_hcnsf_f16}


def main(names):
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    out["_source"] = "written by tests/golden/make_storage_floor.py from the FP64 oracle (no library values)"
    for name in names:
        print(f"{name}:", flush=True)
        out[name] = CASES[name]()
        print(json.dumps(out[name]["groups"]), flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or sorted(CASES))
