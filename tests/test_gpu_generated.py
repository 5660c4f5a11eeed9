"""GPU parity of the systems the compiler slice emitted from declared
conservation laws (gen_*), against the oracle's hand-written systems of the
same physics, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from oracle import mms

import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2607_05668_amd import inputs, lbm  # noqa: E402


def rel(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def run_pair(gen, system, lattice, shape, f, tau_r, steps, storage, params, Q, diffusive=False):
    ny, nx = shape
    dx = 1.0 / max(nx, ny)
    dt = f * dx * dx if diffusive else f * dx
    g = lbm.Stepper(gen, lattice, shape, 0.5 + tau_r * dt, dt, dx, storage, params)
    g.init(Q)
    g.step(steps)
    Qg = g.moments().cpu().numpy()
    phys = {k: v for k, v in params.items() if k != "g_tau"}
    c = parity.scheme(g, dx, dt, 0.5 + tau_r * dt, g_tau=params.get("g_tau"))
    kw = {"omega_tracker": c["omega_tracker"]} if "g_tau" in params else {}
    o = oracle.Oracle(system, lattice, shape, c["dt"], c["dx"], c["tau"], c["g_tau"], phys, Q0=c["Q0"], **kw)
    o.init(Q)
    o.step(steps)
    return Qg, o.moments()


@pytest.mark.parametrize("lattice,shape,storage,f,tol", [
    ("D2Q5", (64, 64), "f64", 0.05, 1e-12), ("D2Q5", (128, 128), "f32", 0.05, 1e-6),
    ("D2Q9", (40, 56), "f32", 0.025, 1e-6)])
def test_generated_euler_matches_oracle(lattice, shape, storage, f, tol):
    """The paper's Mach-3 Euler state at t = 0, unforced, 400 steps (the
    configuration of the hand-written Euler's parity test)."""
    print(f"gen_euler2d {lattice} {storage} {shape} 400 steps", flush=True)
    fQ, _ = mms.euler_paper()
    X, Y = np.meshgrid(np.arange(shape[1]) / shape[1], np.arange(shape[0]) / shape[0], indexing="xy")
    Qg, Qo = run_pair("gen_euler2d", "euler2d", lattice, shape, f, 5.0 if storage == "f32" else 0.2, 400,
                      storage, {"gamma": 1.4}, fQ(X, Y, 0.0))
    parity.check_fields({"rho": slice(0, 1), "m": slice(1, 3), "E": slice(3, 4)}, Qg, Qo, tol)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_generated_advdiff_matches_oracle(storage, tol):
    """The C1 workload (64^2, a = (0.1, 0.05), nu = 0.01, reaction off)
    with the compiled advection-diffusion system, 200 steps."""
    print(f"gen_advdiff_trk2d D2Q5 {storage} 64x64 200 steps", flush=True)
    p = inputs.PRESETS["advdiff64"]
    Qg, Qo = run_pair("gen_advdiff_trk2d", "advdiff_trk2d", "D2Q5", (64, 64), p.f, p.tau_r, 200, storage,
                      dict(p.params, g_tau=p.g_tau), inputs.advdiff_initial(64), diffusive=True)
    parity.check_fields({"c": slice(0, 1), "G": slice(1, None)}, Qg, Qo, tol)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_generated_cnsf_matches_oracle(storage, tol):
    """The paper's 2D compressible NSF state at t = 0 (Mach 3 / 2), with
    the 8 conserved-field trackers the compiler derived by the chain rule,
    diffusive recipe f = 2, tau_R = 60, g_tau = 6, 300 steps."""
    print(f"gen_cnsf_trk2d D2Q5 {storage} 48x48 300 steps", flush=True)
    mu, K = 3.52 / (1.225 * 340.2), 4980.0 / (287.0 * 1.225 * 340.2)
    fQ, _ = mms.cnsf2d_paper(mu, K)
    X, Y = inputs.grid2(48)
    Qg, Qo = run_pair("gen_cnsf_trk2d", "cnsf_trk2d", "D2Q5", (48, 48), 2.0, 60.0, 300, storage,
                      {"gamma": 1.4, "mu": mu, "kappa": K, "R_gas": 1.0, "g_tau": 6.0}, fQ(X, Y, 0.0),
                      diffusive=True)
    parity.check_fields({"rho": slice(0, 1), "m": slice(1, 3), "E": slice(3, 4), "G": slice(4, None)}, Qg, Qo, tol)


def test_generated_cnsf_from_si_runs_in_lattice_units():
    """Alg. 1's Dedimensionalize step end to end: the 2D compressible NSF
    declared in SI units (the supplement's listing: density and gas
    constant as references, rho0 = 1.225 kg/m^3 and c_s = 340 m/s as working
    scales) gives nondimensional parameters equal to those derived by hand;
    scaled on to lattice units by dx^-p dt^-q (parameters, initial fields,
    reference state) it runs with dx = dt = 1, and scaled back its FP64 fields
    equal those of the nondimensional run with explicit dt and dx to 1e-12."""
    from paper_2607_05668_amd import compiler as C
    from paper_2607_05668_amd import declared
    print("gen_cnsf_trk2d D2Q5 f64 48x48 300 steps: SI -> lattice units vs nondimensional", flush=True)
    s = declared.cnsf2d()
    si = {"gamma": 1.4, "mu": 3.52, "kappa": 4980.0, "R_gas": 287.0}
    char = [(C.LENGTH, 1.0), (C.VELOCITY, 340.0), (C.DENSITY, 1.225), (C.GAS_CONSTANT, 287.0)]
    nd = C.nondimensional(s, si, char)
    hand = {"gamma": 1.4, "mu": 3.52 / (1.225 * 340.0), "kappa": 4980.0 / (287.0 * 1.225 * 340.0), "R_gas": 1.0}
    for k, v in hand.items():
        assert abs(nd[k] - v) <= 1e-12 * abs(v), k
    n, steps, g_tau = 48, 300, 6.0
    dx, dt = 1.0 / n, 2.0 / n ** 2
    tau = 0.5 + 60.0 * dt
    fQ, _ = mms.cnsf2d_paper(nd["mu"], nd["kappa"])
    X, Y = inputs.grid2(n)
    Q = fQ(X, Y, 0.0)
    a = lbm.Stepper("gen_cnsf_trk2d", "D2Q5", (n, n), tau, dt, dx, "f64", dict(nd, g_tau=g_tau))
    a.init(Q)
    a.step(steps)
    Qa = a.moments().cpu().numpy()
    lat = C.lattice_values(s, nd, dx, dt)
    fac = np.array(C.field_factors(s, dx, dt))
    ref = a.reference * fac
    b = lbm.Stepper("gen_cnsf_trk2d", "D2Q5", (n, n), tau, 1.0, 1.0, "f64", dict(lat, g_tau=g_tau), reference=ref)
    assert b.param("lambda") == 1.0
    b.init(Q * fac[:, None, None])
    b.step(steps)
    Qb = b.moments().cpu().numpy() / fac[:, None, None]
    parity.check_fields({"rho": slice(0, 1), "m": slice(1, 3), "E": slice(3, 4), "G": slice(4, None)}, Qb, Qa,
                        1e-12)
