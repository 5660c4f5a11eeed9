"""GPU parity of the two-relaxation-time collision (symmetric parts at
omega+, antisymmetric parts at the field's BGK rate omega-, omega+ from the
magic parameter) against the oracle's TRT, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from oracle import mms
from paper_2607_05668_amd import inputs

import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2607_05668_amd import lbm  # noqa: E402

MAGIC = 3.0 / 16.0


def rel(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def twin(g, system, lattice, params, trackers, rec):
    """Oracle with the stepper's rates, each checked first against the recipe
    rec = (dx, dt, tau) and the magic parameter."""
    phys = {k: v for k, v in params.items() if k not in ("g_tau", "trt_lambda")}
    g_tau = params.get("g_tau") if trackers else None
    c = parity.scheme(g, *rec, g_tau=g_tau, trt_lambda=params["trt_lambda"])
    kw = {"omega_plus": c["omega_plus"]}
    if trackers:
        kw.update(omega_tracker=c["omega_tracker"], omega_plus_tracker=c["omega_plus_tracker"])
    return oracle.Oracle(system, lattice, g.shape, c["dt"], c["dx"], c["tau"], c["g_tau"], phys, Q0=c["Q0"], **kw)


@pytest.mark.parametrize("storage,lattice,shape,tol", [("f32", "D2Q9", (48, 64), 1e-6),
                                                      ("f64", "D2Q9", (48, 64), 1e-12),
                                                      ("f32", "D2Q5", (37, 50), 1e-6),
                                                      ("f16", "D2Q9", (64, 64), 1e-3)])
def test_swe_trt_matches_oracle(storage, lattice, shape, tol):
    """Shallow water from the seeded 8-mode depth field, 300 steps; the
    FP32 path is the float-float one (only the TRT term b d_ib added)."""
    print(f"swe2d {lattice} {storage} {shape} TRT 300 steps", flush=True)
    ny, nx = shape
    dx = 1.0 / max(shape)
    dt = 0.2 * dx
    params = {"g": 1.0, "trt_lambda": MAGIC}
    g = lbm.Stepper("swe2d", lattice, shape, 0.5 + 2.0 * dt, dt, dx, storage, params)
    Q = inputs.swe_initial(max(shape))[:, :ny, :nx]
    g.init(Q)
    g.step(300)
    assert g.param("omega_plus") != pytest.approx(g.param("omega"), rel=1e-3)
    o = twin(g, "swe2d", lattice, params, False, (dx, dt, 0.5 + 2.0 * dt))
    o.init(Q)
    o.step(300)
    Qg, Qo = g.moments().cpu().numpy(), o.moments()
    parity.check_fields({"h": slice(0, 1), "hu": slice(1, None)}, Qg, Qo, tol)


@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("f64", 1e-12)])
def test_cnsf_trt_with_trackers_matches_oracle(storage, tol):
    """2D compressible NSF (12 fields, trackers with their own omega- and
    omega+), the paper's Mach-3/2 state, 300 steps."""
    print(f"cnsf_trk2d D2Q5 {storage} 48x48 TRT 300 steps", flush=True)
    n = 48
    mu, K = 3.52 / (1.225 * 340.2), 4980.0 / (287.0 * 1.225 * 340.2)
    params = {"gamma": 1.4, "mu": mu, "kappa": K, "R_gas": 1.0, "g_tau": 6.0, "trt_lambda": MAGIC}
    dx = 1.0 / n
    dt = 2.0 * dx * dx
    g = lbm.Stepper("cnsf_trk2d", "D2Q5", (n, n), 0.5 + 60.0 * dt, dt, dx, storage, params)
    fQ, _ = mms.cnsf2d_paper(mu, K)
    X, Y = inputs.grid2(n)
    Q = fQ(X, Y, 0.0)
    g.init(Q)
    g.step(300)
    o = twin(g, "cnsf_trk2d", "D2Q5", params, True, (dx, dt, 0.5 + 60.0 * dt))
    o.init(Q)
    o.step(300)
    Qg, Qo = g.moments().cpu().numpy(), o.moments()
    parity.check_fields({"rho": slice(0, 1), "m": slice(1, 3), "E": slice(3, 4), "G": slice(4, None)}, Qg, Qo, tol)


def test_hcnsf_trt_matches_oracle():
    """3D homogenized NSF with the porosity field, D3Q7, FP32, 60 steps."""
    print("hcnsf3d_trk14 D3Q7 f32 20^3 TRT 60 steps", flush=True)
    n = 20
    pre = inputs.PRESETS["hcnsf256"]
    params = dict(pre.params, g_tau=pre.g_tau, trt_lambda=MAGIC)
    dx = 1.0 / n
    dt = pre.f * dx
    g = lbm.Stepper("hcnsf3d_trk14", "D3Q7", (n, n, n), 0.5 + 20.0 * dt, dt, dx, "f32", params)
    B = inputs.hcnsf_coefficients(n, 0.4)
    g.set_field("coef", B)
    Q = inputs.hcnsf_exact(n, 0.4)
    g.init(Q)
    g.step(60)
    Bo = g._fields["coef"].cpu().numpy().astype(np.float64).reshape(B.shape)
    o = twin(g, "hcnsf3d_trk14", "D3Q7", params, True, (dx, dt, 0.5 + 20.0 * dt))
    o.init(Q, b=Bo)
    o.step(60, b=Bo)
    Qg, Qo = g.moments().cpu().numpy(), o.moments()
    parity.check_fields({"rho": slice(0, 1), "m": slice(1, 4), "E": slice(4, 5), "G_u": slice(5, 11), "G_T": slice(11, None)}, Qg, Qo, 1e-6)


@pytest.mark.parametrize("storage,lattice,tol", [("f32", "D2Q9", 1e-6), ("f64", "D2Q9", 1e-12),
                                                 ("f32", "D2Q5", 1e-6)])
def test_swe_regularized_matches_oracle(storage, lattice, tol):
    """Regularized collision (non-equilibrium projected on the first-order
    Hermite polynomial), shallow water from the seeded depth field, 300
    steps at tau_R = 20 (omega = 1.78).  With the C2 rate tau_R = 2 (omega
    = 1.975) this operator is unstable for this flow, in the oracle as on
    the GPU: it relaxes the symmetric non-equilibrium at rate one, the
    two-relaxation-time limit of a vanishing magic parameter."""
    print(f"swe2d {lattice} {storage} 48x64 regularized 300 steps", flush=True)
    shape = (48, 64)
    dx = 1.0 / 64
    dt = 0.2 * dx
    g = lbm.Stepper("swe2d", lattice, shape, 0.5 + 20.0 * dt, dt, dx, storage, {"g": 1.0, "regularized": 1})
    Q = inputs.swe_initial(64)[:, :48, :64]
    g.init(Q)
    g.step(300)
    c = parity.scheme(g, dx, dt, 0.5 + 20.0 * dt, Q0=[1.0, 0.0, 0.0])
    o = oracle.Oracle("swe2d", lattice, shape, c["dt"], c["dx"], c["tau"], None, {"g": 1.0}, Q0=c["Q0"],
                      regularized=True)
    o.init(Q)
    o.step(300)
    Qg, Qo = g.moments().cpu().numpy(), o.moments()
    parity.check_fields({"h": slice(0, 1), "hu": slice(1, None)}, Qg, Qo, tol)


def test_nsf17_regularized_matches_oracle():
    """Regularized collision on the 3D 17-field cascade (trackers at their
    own rate), D3Q7 FP32, 24^3 MMS state, 60 steps without forcing."""
    print("nsf3d_trk17 D3Q7 f32 24^3 regularized 60 steps", flush=True)
    n = 24
    pre = inputs.PRESETS["nsf256"]
    params = dict(pre.params, mms=0.0, g_tau=pre.g_tau, regularized=1)
    dx = 1.0 / n
    dt = pre.f * dx
    g = lbm.Stepper("nsf3d_trk17", "D3Q7", (n, n, n), 0.5 + pre.tau_r * dt, dt, dx, "f32", params)
    Q = inputs.nsf_exact(n, 0.3)
    g.init(Q)
    g.step(60)
    phys = {k: pre.params[k] for k in ("gamma", "mu", "kappa")}
    c = parity.scheme(g, dx, dt, 0.5 + pre.tau_r * dt, g_tau=pre.g_tau, Q0=inputs.NsfMms().reference())
    o = oracle.Oracle("nsf3d_trk17", "D3Q7", (n, n, n), c["dt"], c["dx"], c["tau"], c["g_tau"], phys, Q0=c["Q0"],
                      omega_tracker=c["omega_tracker"], regularized=True)
    o.init(Q)
    o.step(60)
    Qg, Qo = g.moments().cpu().numpy(), o.moments()
    parity.check_fields({"rho": slice(0, 1), "m": slice(1, 4), "E": slice(4, 5), "G": slice(5, None)}, Qg, Qo, 1e-6)
