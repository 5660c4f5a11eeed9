"""GPU parity for the 3D homogenized compressible NSF system (14 fields:
strain-reduced velocity-gradient trackers and temperature-gradient trackers,
prescribed porosity and solid velocity per cell) against the FP64 oracle on
the same inputs, through the C ABI."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2607_05668_amd import inputs

import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2607_05668_amd import lbm  # noqa: E402

GROUPS = {"rho": slice(0, 1), "m": slice(1, 4), "E": slice(4, 5), "G_u": slice(5, 11), "G_T": slice(11, 14)}
FLOOR = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "storage_floor.json")))
PHYS = ("gamma", "mu", "kappa", "eta")


def rel(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def make_pair(shape, storage, Q, B, tau_r):
    pre = inputs.PRESETS["hcnsf256"]
    n = max(shape)
    dx = 1.0 / n
    dt = pre.f * dx
    g = lbm.Stepper("hcnsf3d_trk14", "D3Q7", shape, 0.5 + tau_r * dt, dt, dx, storage,
                    dict(pre.params, g_tau=pre.g_tau))
    if B is not None:
        g.set_field("coef", B)
    g.init(Q)
    c = parity.scheme(g, dx, dt, 0.5 + tau_r * dt, g_tau=pre.g_tau)
    o = oracle.Oracle("hcnsf3d_trk14", "D3Q7", shape, c["dt"], c["dx"], c["tau"], c["g_tau"],
                      {k: pre.params[k] for k in PHYS}, Q0=c["Q0"], omega_tracker=c["omega_tracker"])
    # the oracle gets the coefficient values the kernels read (the field is
    # held in the stepping arithmetic type)
    Bo = None if B is None else np.asarray(g._fields["coef"].cpu().numpy(), dtype=np.float64).reshape(B.shape)
    o.init(Q, b=Bo)
    return g, o, Bo


def advance(g, o, Bo, steps, tol=None, tol_trackers=None):
    """Step both; print rel L2 and rel Linf per field group; with tol, assert
    both (trackers against tol_trackers if given).  Returns the rel L2 errors."""
    g.step(steps)
    o.step(steps, b=Bo)
    Qg, Qo = g.moments().cpu().numpy(), o.moments()
    errs = {k: parity.rel_l2(Qg[s], Qo[s]) for k, s in GROUPS.items()}
    if tol is None:
        for k, s in GROUPS.items():
            print(f"step {g.steps} {k}: rel L2 {errs[k]:.3e} rel Linf {parity.rel_linf(Qg[s], Qo[s]):.3e}",
                  flush=True)
        return errs
    cons = {k: s for k, s in GROUPS.items() if not k.startswith("G_")}
    trk = {k: s for k, s in GROUPS.items() if k.startswith("G_")}
    parity.check_fields(cons, Qg, Qo, tol, label=f"step {g.steps} ")
    parity.check_fields(trk, Qg, Qo, tol_trackers or tol, label=f"step {g.steps} ")
    return errs


@pytest.mark.parametrize("storage,n,tol,coef", [("f32", 24, 1e-6, True), ("f32", 24, 1e-6, False),
                                                ("f64", 16, 1e-12, True)])
def test_hcnsf_with_porosity_matches_oracle(storage, n, tol, coef):
    """The paper's MMS state and coefficient fields at t = 0.4 (alpha over
    [0.1, 0.9], moving solid), held fixed, without forcing; and the same
    state as pure fluid (no coefficient field).  60 steps, then on to 150
    steps, where the drag has pulled the momentum of the solid region
    towards the solid velocity, 45% (RMS) away from the reference state,
    and single-precision storage of the shifted populations loses accuracy
    in proportion (measured with the porosity field: rho u 7.4e-8, G_u
    9.1e-7, G_T 6.3e-7 at 150 steps): every field within its tolerance at
    both."""
    print(f"hcnsf3d_trk14 D3Q7 {storage} {n}^3, coefficient field {coef}", flush=True)
    Q = inputs.hcnsf_exact(n, 0.4)
    B = inputs.hcnsf_coefficients(n, 0.4) if coef else None
    g, o, Bo = make_pair((n, n, n), storage, Q, B, 20.0 if storage == "f32" else 10.0)
    advance(g, o, Bo, 60, tol)
    advance(g, o, Bo, 90, tol)


def test_hcnsf_fp16_storage():
    """Binary16 shifted populations (per-field power-of-two scales, FP32
    arithmetic) on the porous MMS state: the conserved fields hold 1e-3
    (measured rho 2.3e-5, rho u 1.6e-4, E 3.8e-5 at 60 steps); the
    trackers follow the gradient of the velocity the binary16 momentum
    carries, which amplifies its rounding by |u| / |du| and 1 / (k dx):
    G_u 3.1e-3 and G_T 1.1e-3, above the FP16 tolerance (expected failure;
    a slower tracker relaxation, larger g_tau, measured worse).  The oracle
    with its own populations rounded to binary16 every step is above it too
    (G_u 2.2e-3, G_T 1.0e-3: the storage floor, printed beside)."""
    print("hcnsf3d_trk14 D3Q7 f16 24^3 60 steps, coefficient field", flush=True)
    n = 24
    g, o, Bo = make_pair((n, n, n), "f16", inputs.hcnsf_exact(n, 0.4), inputs.hcnsf_coefficients(n, 0.4), 20.0)
    errs = advance(g, o, Bo, 60)
    floor = FLOOR["hcnsf_f16"]["groups"]
    print("binary16 storage floor: " + "  ".join(f"{k} {v['l2']:.2e}" for k, v in floor.items()), flush=True)
    for k in ("rho", "m", "E"):
        assert errs[k] <= 1e-3, k
    if max(errs["G_u"], errs["G_T"]) > 1e-3:
        pytest.xfail(f"binary16 tracker populations: G_u {errs['G_u']:.1e}, G_T {errs['G_T']:.1e}")


def test_hcnsf_ragged_grid_pure_fluid():
    """7 x 13 x 40 cells (ragged tiles), no coefficient field (alpha = 1)."""
    print("hcnsf3d_trk14 D3Q7 f32 40x13x7 100 steps, no coefficient field", flush=True)
    shape = (7, 13, 40)
    z, y, x = np.meshgrid(np.arange(7) / 7, np.arange(13) / 13, np.arange(40) / 40, indexing="ij")
    u0 = 0.5 * math.sqrt(1.4)
    Q = np.zeros((14,) + shape)
    Q[0] = 1.0 + 0.05 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) * np.sin(2 * np.pi * z)
    for a in range(3):
        Q[1 + a] = u0 + 0.03 * np.cos(2 * np.pi * (x + a * y - z))
    Q[4] = 2.5 + 1.5 * u0 * u0 + 0.04 * np.cos(2 * np.pi * (x - z))
    Q[5:] = 0.1 * np.sin(2 * np.pi * (x + 2 * y + 3 * z))[None]
    g, o, Bo = make_pair(shape, "f32", Q, None, 20.0)
    advance(g, o, Bo, 100, 1e-6)
