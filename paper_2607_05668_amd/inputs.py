"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds input data only: a counter-free pseudo-random generator,
random Fourier-mode fields with their analytic gradients, the closed-form
initial fields of each workload, and the workload presets as plain numbers.
It contains none of the scheme's arithmetic (no equilibria, fluxes,
collision or streaming), so importing it on either side shares no method
code.  It imports numpy only.

Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written from its published
description: add the golden-gamma increment to the state, then apply the
two xor-shift-multiply finalisation rounds.  Doubles in [0,1) take the top
53 bits.

Random Fourier fields: ``sum_m A_m cos(2 pi (kx x + ky y) + phi_m)`` with
integer wavenumbers ``k = floor(u (2K+1)) - K`` drawn per component, the
pair (0,0) rejected, and ``phi = 2 pi u``.  Grid nodes sit at ``x_j = j/N``
on the periodic unit square (the paper's periodic domains, Sec. 3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


class SplitMix64:
    """SplitMix64 stream; ``next_u64`` and ``next_double`` in [0, 1)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def next_double(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


@dataclass(frozen=True)
class Modes:
    kx: tuple
    ky: tuple
    phi: tuple
    amp: tuple


def draw_modes(seed: int, nmodes: int, kmax: int, amp_per_mode: float) -> Modes:
    """Draw ``nmodes`` (kx, ky, phase) triples with |k|_inf <= kmax, k != 0."""
    rng = SplitMix64(seed)
    kx, ky, ph = [], [], []
    while len(kx) < nmodes:
        a = int(math.floor(rng.next_double() * (2 * kmax + 1))) - kmax
        b = int(math.floor(rng.next_double() * (2 * kmax + 1))) - kmax
        if a == 0 and b == 0:
            continue
        kx.append(a)
        ky.append(b)
        ph.append(2.0 * math.pi * rng.next_double())
    return Modes(tuple(kx), tuple(ky), tuple(ph), tuple([amp_per_mode] * nmodes))


def grid2(n: int):
    """Node coordinates (X, Y), each [n, n] with X varying along the last axis."""
    x = np.arange(n, dtype=np.float64) / n
    return np.meshgrid(x, x, indexing="xy")


def grid3(n: int):
    """Node coordinates (X, Y, Z), each [n, n, n] indexed [z, y, x]."""
    x = np.arange(n, dtype=np.float64) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def fourier_field(n: int, modes: Modes):
    """Return (value, d/dx, d/dy) of the mode sum on the n x n grid, [n, n] each."""
    X, Y = grid2(n)
    v = np.zeros((n, n))
    gx = np.zeros((n, n))
    gy = np.zeros((n, n))
    two_pi = 2.0 * math.pi
    for a, b, p, A in zip(modes.kx, modes.ky, modes.phi, modes.amp):
        arg = two_pi * (a * X + b * Y) + p
        v += A * np.cos(arg)
        s = -A * np.sin(arg) * two_pi
        gx += s * a
        gy += s * b
    return v, gx, gy


# --------------------------------------------------------------------------
# Workload presets (plain numbers).  f, tau_R, g_tau are the paper's
# convergence-study recipes (supplement, numerical configuration table):
# dt = f dx (acoustic) or f dx^2 (diffusive), tau_LB = 1/2 + tau_R dt,
# tau_grad = g_tau dt, tracker collision rate 1/(g_tau + 1).
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Preset:
    name: str
    system: str
    lattice: str
    n: int
    storage: str
    steps: int
    scaling: str            # "acoustic" | "diffusive"
    f: float
    tau_r: float
    g_tau: float | None
    params: dict = field(default_factory=dict)


PRESETS = {
    "advdiff64": Preset("advdiff64", "advdiff_trk2d", "D2Q5", 64, "f64", 200,
                        "diffusive", 1.9, 50.0, 6.0,
                        {"ax": 0.1, "ay": 0.05, "nu": 0.01, "R": 0.0}),
    "swe1024": Preset("swe1024", "swe2d", "D2Q9", 1024, "f32", 1000,
                      "acoustic", 0.2, 2.0, None, {"g": 1.0}),
    "sweadj512": Preset("sweadj512", "swe2d", "D2Q9", 512, "f32", 500,
                        "acoustic", 0.2, 2.0, None, {"g": 1.0}),
    # binary16 storage: tau_R = 20 (the paper raises tau_R as it lowers the
    # precision; at its single-precision tau_R = 2, omega = 1.997 and the
    # rounding of the stored non-equilibrium part decays over ~300 steps)
    "neohooke2048": Preset("neohooke2048", "neohooke2d", "D2Q9", 2048, "f16", 2000,
                           "acoustic", 0.1, 20.0, None,
                           {"rho0": 1.0, "mu_s": 1.0, "lambda_s": 2.0}),
    # the paper's suite on the same kernel (single-precision recipes of its
    # configuration table, D2Q5 as in the paper)
    "burgers2048": Preset("burgers2048", "burgers2d", "D2Q5", 2048, "f32", 100,
                          "acoustic", 0.2, 2.0, None, {}),
    "euler2048": Preset("euler2048", "euler2d", "D2Q5", 2048, "f32", 100,
                        "acoustic", 0.05, 5.0, None, {"gamma": 1.4}),
    "maxwell2048": Preset("maxwell2048", "maxwell2d", "D2Q5", 2048, "f32", 100,
                          "acoustic", 0.2, 0.2, None, {"c": 1.0}),
    "allencahn2048": Preset("allencahn2048", "allencahn_trk2d", "D2Q5", 2048, "f32", 100,
                            "diffusive", 1.9, 50.0, 6.0, {"nu": 0.01, "R": 1.0}),
    "relhydro2048": Preset("relhydro2048", "relhydro2d", "D2Q5", 2048, "f32", 100,
                           "acoustic", 0.2, 0.2, None, {}),
    "nse2048": Preset("nse2048", "nse_trk2d", "D2Q5", 2048, "f32", 100,
                      "diffusive", 2.0, 90.0, 6.0, {"cs_phys": 1.0, "mu": 0.01}),
    "cnsf2048": Preset("cnsf2048", "cnsf_trk2d", "D2Q5", 2048, "f32", 100,
                       "diffusive", 2.0, 60.0, 6.0,
                       {"gamma": 1.4, "mu": 3.52 / (1.225 * 340.2), "kappa": 4980.0 / (287.0 * 1.225 * 340.2),
                        "R_gas": 1.0}),
    "mhd2048": Preset("mhd2048", "mhd_trk2d", "D2Q5", 2048, "f32", 100,
                      "acoustic", 0.025, 160.0, 4.0,
                      {"gamma": 1.4, "mu": 4.165 / (1.225 * 340.0), "kappa": 4.165 / (1.225 * 340.0),
                       "eta": 3.4 / 340.0}),
}

# Seeds of the random fields.
SEED_SWE_H = 1
SEED_SWE_TARGET = 2
SEED_TOPOGRAPHY = 3
SEED_FD_DIRECTIONS = 4
SEED_DISPLACEMENT = (5, 6)


# --------------------------------------------------------------------------
# Initial fields, SoA [K, ...] float64.
# --------------------------------------------------------------------------

def advdiff_initial(n: int):
    """u0 = 1 + 0.1 sin(2 pi x) sin(2 pi y) and its analytic gradient, [3, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    u = 1.0 + 0.1 * np.sin(k * X) * np.sin(k * Y)
    gx = 0.1 * k * np.cos(k * X) * np.sin(k * Y)
    gy = 0.1 * k * np.sin(k * X) * np.cos(k * Y)
    return np.stack([u, gx, gy])


def advdiff_exact(n: int, t: float, ax: float, ay: float, nu: float):
    """Closed-form decaying solution of u_t + a.grad u = nu lap u and its gradient."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    d = math.exp(-2.0 * k * k * nu * t)
    sx, cx = np.sin(k * (X - ax * t)), np.cos(k * (X - ax * t))
    sy, cy = np.sin(k * (Y - ay * t)), np.cos(k * (Y - ay * t))
    u = 1.0 + 0.1 * d * sx * sy
    return np.stack([u, 0.1 * d * k * cx * sy, 0.1 * d * k * sx * cy])


def swe_height(n: int, seed: int = SEED_SWE_H, h0: float = 1.0):
    """h = h0 + sum of 8 random modes of amplitude 0.05 each, |k|_inf <= 8."""
    m = draw_modes(seed, 8, 8, 0.05)
    v, _, _ = fourier_field(n, m)
    return h0 + v


def swe_initial(n: int, seed: int = SEED_SWE_H):
    """(h, hu, hv) with fluid at rest, [3, n, n]."""
    h = swe_height(n, seed)
    z = np.zeros_like(h)
    return np.stack([h, z, z])


def topography_gradient(n: int, seed: int = SEED_TOPOGRAPHY):
    """b = grad z_b, z_b = sum of 8 modes of amplitude 0.01/8, |k|_inf <= 4; [2, n, n]."""
    m = draw_modes(seed, 8, 4, 0.01 / 8.0)
    _, gx, gy = fourier_field(n, m)
    return np.stack([gx, gy])


def burgers_initial(n: int, amp: float = 1.3):
    """The paper's Burgers profile at t = 0: u = A sin(2 pi x) sin(2 pi y), [1, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    return (amp * np.sin(k * X) * np.sin(k * Y))[None]


def euler_initial(n: int, gamma: float = 1.4):
    """The paper's Euler profile at t = 0 in units rho0 = cs = 1: rho = 1 +
    0.3 sin(2 pi x) cos(2 pi y), velocity (3, 3) (the velocity and pressure
    modes carry sin t), p = 1/gamma + (rho - 1); conserved [4, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    rho = 1.0 + 0.3 * np.sin(k * X) * np.cos(k * Y)
    p = 1.0 / gamma + (rho - 1.0)
    E = p / (gamma - 1.0) + 0.5 * rho * (3.0 ** 2 + 3.0 ** 2)
    return np.stack([rho, 3.0 * rho, 3.0 * rho, E])


def maxwell_initial(n: int, amp: float = 0.5):
    """The paper's TM pattern at t = 0: E_z = A sin(2 pi x) sin(4 pi y), H = 0."""
    X, Y = grid2(n)
    Ez = amp * np.sin(2.0 * math.pi * X) * np.sin(4.0 * math.pi * Y)
    return np.stack([Ez, np.zeros_like(Ez), np.zeros_like(Ez)])


def allencahn_initial(n: int, amp: float = 0.7):
    """The paper's Allen-Cahn profile at t = 0, phi = 0.7 sin(2 pi x) cos(2 pi y),
    with its analytic gradient as the tracker fields, [3, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    phi = amp * np.sin(k * X) * np.cos(k * Y)
    return np.stack([phi, amp * k * np.cos(k * X) * np.cos(k * Y), -amp * k * np.sin(k * X) * np.sin(k * Y)])


def relhydro_initial(n: int):
    """The paper's ultrarelativistic profile at t = 0: E = 3 + 0.4 sin sin,
    S = (1.2, 1.2), [3, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    E = 3.0 + 0.4 * np.sin(k * X) * np.sin(k * Y)
    return np.stack([E, np.full_like(E, 1.2), np.full_like(E, 1.2)])


def nse_initial(n: int, U: float = 0.1):
    """The paper's Taylor-Green state at t = 0 (rho0 = cs = 1): rho = 1 + p,
    p = -U^2 (cos 2kx + cos 2ky) / 4, m = rho u, and the exact momentum
    gradients d_b m_a as tracker fields, [7, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    u = -U * np.cos(k * X) * np.sin(k * Y)
    v = U * np.sin(k * X) * np.cos(k * Y)
    rho = 1.0 - 0.25 * U * U * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    drx = 0.5 * U * U * k * np.sin(2 * k * X)
    dry = 0.5 * U * U * k * np.sin(2 * k * Y)
    dux, duy = U * k * np.sin(k * X) * np.sin(k * Y), -U * k * np.cos(k * X) * np.cos(k * Y)
    dvx, dvy = U * k * np.cos(k * X) * np.cos(k * Y), -U * k * np.sin(k * X) * np.sin(k * Y)
    return np.stack([rho, rho * u, rho * v, drx * u + rho * dux, dry * u + rho * duy,
                     drx * v + rho * dvx, dry * v + rho * dvy])


def cnsf2d_initial(n: int, gamma: float = 1.4):
    """The paper's 2D compressible NSF state at t = 0 in units rho0 = cs = 1:
    rho = 1 + 0.2 sin(2 pi x) cos(2 pi y), u = 3, v = 2 + 0.15 sin sin,
    p = 1/gamma + (rho - 1), conserved fields and their analytic gradients
    (rho, m0, m1, E, G_rho, G_m0, G_m1, G_E), [12, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    sx, cx, sy, cy = np.sin(k * X), np.cos(k * X), np.sin(k * Y), np.cos(k * Y)
    rho = 1.0 + 0.2 * sx * cy
    rx, ry = 0.2 * k * cx * cy, -0.2 * k * sx * sy
    u = np.full_like(rho, 3.0)
    v = 2.0 + 0.15 * sx * sy
    vx, vy = 0.15 * k * cx * sy, 0.15 * k * sx * cy
    p = 1.0 / gamma + (rho - 1.0)
    kin = 0.5 * (u * u + v * v)
    E = p / (gamma - 1.0) + rho * kin
    Ex = rx / (gamma - 1.0) + rx * kin + rho * v * vx
    Ey = ry / (gamma - 1.0) + ry * kin + rho * v * vy
    return np.stack([rho, rho * u, rho * v, E, rx, ry, rx * u, ry * u, rx * v + rho * vx, ry * v + rho * vy,
                     Ex, Ey])


def mhd_initial(n: int, gamma: float = 1.4):
    """The paper's resistive MHD state at t = 0 in units rho0 = cs = 1:
    rho = 1 + 0.3 sin(2 pi x) cos(2 pi y), u = v = 3, B = (0.5, 0.5),
    p = 1/gamma + (rho - 1); conserved fields and their analytic gradients
    (rho, m0, m1, E, B0, B1, G_rho, G_m0, G_m1, G_E, G_B0, G_B1), [18, n, n]."""
    X, Y = grid2(n)
    k = 2.0 * math.pi
    sx, cx, sy, cy = np.sin(k * X), np.cos(k * X), np.sin(k * Y), np.cos(k * Y)
    rho = 1.0 + 0.3 * sx * cy
    rx, ry = 0.3 * k * cx * cy, -0.3 * k * sx * sy
    p = 1.0 / gamma + (rho - 1.0)
    E = p / (gamma - 1.0) + 9.0 * rho + 0.25
    c = 1.0 / (gamma - 1.0) + 9.0
    z = np.zeros_like(rho)
    return np.stack([rho, 3.0 * rho, 3.0 * rho, E, z + 0.5, z + 0.5, rx, ry, 3.0 * rx, 3.0 * ry, 3.0 * rx, 3.0 * ry,
                     c * rx, c * ry, z, z, z, z])


def neohooke_initial(n: int, seeds=SEED_DISPLACEMENT):
    """F = I + grad w, v = 0 for a random displacement w; [6, n, n] as (F00,F01,F10,F11,v0,v1)."""
    out = np.zeros((6, n, n))
    for a, s in enumerate(seeds):
        m = draw_modes(s, 8, 4, 0.01 / 8.0)
        _, dx, dy = fourier_field(n, m)
        out[2 * a + 0] = (1.0 if a == 0 else 0.0) + dx   # F_a0 = delta_a0 + d w_a / dx
        out[2 * a + 1] = (1.0 if a == 1 else 0.0) + dy   # F_a1 = delta_a1 + d w_a / dy
    return out


# ----- 3D compressible NSF manufactured solution (shape of the paper's
# homogenized-NSF MMS, supplement, with porosity 1) --------------------------

@dataclass(frozen=True)
class NsfMms:
    gamma: float = 1.4
    rho0: float = 1.0
    p0: float = 1.0
    mach: float = 0.1
    reynolds: float = 100.0
    prandtl: float = 0.71
    amp: float = 0.05

    @property
    def cbar2(self):            # mean adiabatic sound speed squared, gamma p0 / rho0
        return self.gamma * self.p0 / self.rho0

    @property
    def u0(self):               # per-axis drift
        return self.mach * math.sqrt(self.cbar2)

    @property
    def mu(self):               # dynamic viscosity from Re = rho0 U0 L / mu, L = 1
        return self.rho0 * self.u0 / self.reynolds

    @property
    def kappa(self):            # heat-flux coefficient mu c_p / Pr with c_p = gamma/(gamma-1), R = 1
        return self.mu * self.gamma / (self.gamma - 1.0) / self.prandtl

    @property
    def E0(self):
        return self.p0 / (self.gamma - 1.0) + 1.5 * self.rho0 * self.u0 ** 2

    def reference(self):
        """Background state (rho, rho u, E, trackers = 0), 17 values."""
        q = np.zeros(17)
        q[0] = self.rho0
        q[1:4] = self.rho0 * self.u0
        q[4] = self.E0
        return q


def nsf_params(mms: NsfMms = NsfMms()):
    """Parameters of the 3D NSF workload: gas, transport coefficients from
    Re and Pr, and the manufactured-solution shape (mms_* entries)."""
    return {"gamma": mms.gamma, "mu": mms.mu, "kappa": mms.kappa, "mms": 1.0, "mms_amp": mms.amp,
            "mms_rho0": mms.rho0, "mms_p0": mms.p0, "mms_u0": mms.u0}


PRESETS["nsf256"] = Preset("nsf256", "nsf3d_trk17", "D3Q7", 256, "f32", 500,
                           "acoustic", 0.05, 20.0, 3.0, nsf_params())


def nsf_exact(n: int, t: float, mms: NsfMms = NsfMms()):
    """Exact fields [17, n, n, n] (indexed [k, z, y, x]) at time t.

    Order: rho, rho u (3), E, G_ab = d_b u_a (9, index 5 + 3a + b), grad T (3).
    """
    X, Y, Z = grid3(n)
    k = 2.0 * math.pi
    A, p0, c2 = mms.amp, mms.p0, mms.cbar2
    sx, cx = np.sin(k * X), np.cos(k * X)
    sy, cy = np.sin(k * Y), np.cos(k * Y)
    sz, cz = np.sin(k * Z), np.cos(k * Z)
    st, ct = math.sin(t), math.cos(t)
    U0 = mms.u0
    rho = mms.rho0 + A * sx * cy * sz * ct
    u = [U0 + A * cx * sy * sz * st,
         U0 + A * sx * cy * sz * st,
         U0 + A * sx * sy * cz * st]
    p = p0 + c2 * (rho - mms.rho0) + A * p0 * cx * sy * cz * st
    E = p / (mms.gamma - 1.0) + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    # gradients of u (rows a, columns b = d/dx_b)
    Ak = A * k * st
    du = [[-Ak * sx * sy * sz, Ak * cx * cy * sz, Ak * cx * sy * cz],
          [Ak * cx * cy * sz, -Ak * sx * sy * sz, Ak * sx * cy * cz],
          [Ak * cx * sy * cz, Ak * sx * cy * cz, -Ak * sx * sy * sz]]
    drho = [A * k * ct * cx * cy * sz, -A * k * ct * sx * sy * sz, A * k * ct * sx * cy * cz]
    dpi = [-A * p0 * k * st * sx * sy * cz, A * p0 * k * st * cx * cy * cz,
           -A * p0 * k * st * cx * sy * sz]
    T = p / rho
    out = np.zeros((17, n, n, n))
    out[0] = rho
    for a in range(3):
        out[1 + a] = rho * u[a]
    out[4] = E
    for a in range(3):
        for b in range(3):
            out[5 + 3 * a + b] = du[a][b]
    for b in range(3):
        dp = c2 * drho[b] + dpi[b]
        out[14 + b] = (dp - T * drho[b]) / rho
    return out


# --------------------------------------------------------------------------
# 3D homogenized NSF (14 fields): the paper's MMS working point (Ma 0.5,
# amplitude 0.2, rho0 = cs = 1 with isothermal cs, p0 = 1), SI transport
# coefficients (mu = kappa = 3.52 Pa s, eta = 0.348 ms at rho0 = 1.225,
# cs = 287.4) read in those units; single-precision recipe.
# --------------------------------------------------------------------------
HCNSF_MMS = NsfMms(mach=0.5, amp=0.2)
PRESETS["hcnsf256"] = Preset("hcnsf256", "hcnsf3d_trk14", "D3Q7", 256, "f32", 100,
                             "acoustic", 0.05, 20.0, 3.0,
                             {"gamma": 1.4, "mu": 3.52 / (1.225 * 287.4), "kappa": 3.52 / (1.225 * 287.4),
                              "eta": 0.000348 * 287.4})


def hcnsf_exact(n: int, t: float):
    """Exact fields [14, n, n, n] of the homogenized-NSF MMS at time t:
    rho, rho u (3), E, sym grad u as (00, 11, 22, 01, 02, 12), grad T."""
    q = nsf_exact(n, t, HCNSF_MMS)
    out = np.zeros((14, n, n, n))
    out[:5] = q[:5]
    for s, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        out[5 + s] = 0.5 * (q[5 + 3 * a + b] + q[5 + 3 * b + a])
    out[11:14] = q[14:17]
    return out


def hcnsf_coefficients(n: int, t: float):
    """Prescribed (alpha, u_s) [4, n, n, n] of the homogenized-NSF MMS at time
    t: solid velocity = rotation (0.2) + translation (0.1, -0.1, 0.05) +
    oscillation (0.1); porosity 1/2 + [sin k xi_0 + sin k xi_1 + sin k xi_2 +
    2 sin k xi_0 sin k xi_1 sin k xi_2] / 10 along xi = x - d,
    d = r(x) sin t + c t (r: the rotation's spatial profile)."""
    X, Y, Z = grid3(n)
    k = 2.0 * math.pi
    c = (0.1, -0.1, 0.05)
    r = [0.2 * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z),
         -0.2 * np.cos(k * X) * np.sin(k * Y) * np.cos(k * Z),
         0.2 * np.cos(k * X) * np.cos(k * Y) * np.sin(k * Z)]
    st, ct = math.sin(t), math.cos(t)
    out = np.zeros((4, n, n, n))
    out[1] = r[0] * ct + c[0] + 0.1 * st * np.cos(k * Z)
    out[2] = r[1] * ct + c[1] + 0.1 * ct * np.cos(k * X)
    out[3] = r[2] * st + c[2] + 0.1 * st * np.cos(k * Y)
    s = [np.sin(k * (v - (r[i] * st + c[i] * t))) for i, v in enumerate((X, Y, Z))]
    out[0] = 0.5 + (s[0] + s[1] + s[2] + 2.0 * s[0] * s[1] * s[2]) / 10.0
    return out
