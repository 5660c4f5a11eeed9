"""Manufactured-solution forcing for the oracle -- TEST INFRASTRUCTURE ONLY.

The validation section of the paper forces each system with the continuous
residual of an analytic profile,
    S_MMS(x, t) = d_t Q_exact + div Phi(Q_exact) - S(Q_exact),
injected through the source term of eq. (lbe_update) at t + dt/2.  Here the
residual is formed symbolically with SymPy from the exact fields and the
fluxes written in the paper's tensor notation, then turned into a numpy
function of (x, y[, z], t) with ``lambdify``.  Nothing here is shared with
the HIP library.

Cases:
* ``swe_paper``  -- the paper's shallow-water MMS (supplement, SWE MMS):
  h = 0.04 sin sin cos t + 0.1, hu = 0.02 cos cos sin t + 0.03,
  hv = 0.02 sin sin sin t + 0.03 over z_b = 0.01 sin(2 pi x) cos(2 pi y).
* ``adr_paper``  -- the paper's advection-diffusion-reaction MMS
  (supplement, ADR MMS), with the tracker initialised at grad c.
* ``neohooke_paper`` -- the paper's finite-strain elasticity MMS
  (supplement, elasticity MMS) with mu_s/rho0 = 1, lambda_s/rho0 = 2.
* ``burgers_paper`` -- the paper's inviscid-Burgers MMS (amplitude 1.3).
* ``euler_paper`` -- the paper's compressible-Euler MMS, nondimensional
  (rho0 = 1, cs = 1: background Mach 3 per axis).
* ``maxwell_paper`` -- the paper's Maxwell TM MMS (c = 1).
* ``allencahn_paper`` -- the paper's Allen-Cahn MMS, trackers exact.
* ``relhydro_paper`` -- the paper's ultrarelativistic-fluid MMS.
* ``nse_paper``  -- the paper's weakly compressible NSE (Taylor-Green) MMS,
  nondimensional, trackers exact.
* ``cnsf2d_paper`` -- the paper's 2D compressible NSF MMS (Mach 3 / 2),
  trackers exact.
* ``mhd_paper``  -- the paper's resistive-MHD MMS, trackers exact.
* ``hcnsf_paper`` -- the paper's 3D homogenized-NSF MMS (14 fields, Ma 0.5,
  amplitude 0.2) with its prescribed porosity and solid velocity.
* ``nsf17``      -- the 3D compressible NSF manufactured solution with the
  shapes of the paper's homogenized-NSF MMS (porosity 1), conserved rows
  forced; tracker rows are forced only when ``force_trackers`` is set.
"""
from __future__ import annotations

import ctypes
import functools
import hashlib
import math
import os
import subprocess

import numpy as np
import sympy as sp

X, Y, Z, T = sp.symbols("x y z t", real=True)
PI2 = 2 * sp.pi


def _div(Phi_row, coords):
    return sum(sp.diff(Phi_row[a], coords[a]) for a in range(len(coords)))


# ---------------------------------------------------------------- SWE ----
def swe_exact_exprs():
    h = sp.Rational(1, 25) * sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.cos(T) + sp.Rational(1, 10)
    hu = sp.Rational(1, 50) * sp.cos(PI2 * X) * sp.cos(PI2 * Y) * sp.sin(T) + sp.Rational(3, 100)
    hv = sp.Rational(1, 50) * sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.sin(T) + sp.Rational(3, 100)
    return [h, hu, hv]


def swe_topography_expr():
    return sp.Rational(1, 100) * sp.sin(PI2 * X) * sp.cos(PI2 * Y)


@functools.lru_cache(maxsize=None)
def swe_exprs(g: float):
    """Symbolic (exact fields, forcing, topography gradient) of the SWE MMS."""
    gs = sp.Float(g)
    Q = swe_exact_exprs()
    h, mx, my = Q
    Phi = [[mx, my],
           [gs * h ** 2 / 2 + mx ** 2 / h, mx * my / h],
           [mx * my / h, gs * h ** 2 / 2 + my ** 2 / h]]
    zb = swe_topography_expr()
    S = [sp.Integer(0), -gs * h * sp.diff(zb, X), -gs * h * sp.diff(zb, Y)]
    res = [sp.diff(Q[k], T) + _div(Phi[k], (X, Y)) - S[k] for k in range(3)]
    return Q, res, [sp.diff(zb, X), sp.diff(zb, Y)]


@functools.lru_cache(maxsize=None)
def swe_paper(g: float):
    """Return (exact(x, y, t) -> [3, ...], forcing(x, y, t) -> [3, ...], b(x, y) -> [2, ...])."""
    Q, res, b = swe_exprs(g)
    fQ = sp.lambdify((X, Y, T), Q, "numpy")
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    fb = sp.lambdify((X, Y), b, "numpy")
    return _wrap2(fQ), _wrap2(fS), _wrap2b(fb)


# ---------------------------------------------------------------- ADR ----
@functools.lru_cache(maxsize=None)
def adr_paper(u0=0.1, u1=-0.1, D=0.01, R=1.0, tau_grad=None):
    """Paper's ADR MMS; trackers (d c/dx, d c/dy) exact, not forced."""
    c = sp.Rational(1, 2) + sp.Rational(1, 2) * sp.exp(-T) * sp.sin(PI2 * (X - u0 * T)) \
        * sp.cos(PI2 * (Y - u1 * T))
    gx, gy = sp.diff(c, X), sp.diff(c, Y)
    Phi_c = [c * u0 - D * gx, c * u1 - D * gy]
    S_c = R * c * (1 - c)
    res_c = sp.diff(c, T) + _div(Phi_c, (X, Y)) - S_c
    fQ = sp.lambdify((X, Y, T), [c, gx, gy], "numpy")
    fS = sp.lambdify((X, Y, T), [res_c, sp.Integer(0), sp.Integer(0)], "numpy", cse=True)
    return _wrap2(fQ), _wrap2(fS)


# ------------------------------------------------------------ BURGERS ----
@functools.lru_cache(maxsize=None)
def burgers_paper(amp=1.3):
    """The paper's inviscid-Burgers MMS (supplement, Burgers MMS):
    u = A sin(2 pi x) sin(2 pi y) cos t with A = 1.3, flux (u^2/2, u^2/2)."""
    A = sp.Float(amp)
    u = A * sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.cos(T)
    res = sp.diff(u, T) + sp.diff(u ** 2 / 2, X) + sp.diff(u ** 2 / 2, Y)
    fQ = sp.lambdify((X, Y, T), [u], "numpy")
    fS = sp.lambdify((X, Y, T), [res], "numpy", cse=True)
    return _wrap2(fQ, [u]), _wrap2(fS, [res])


# -------------------------------------------------------------- EULER ----
def euler_exact_exprs(rho0=1.0, cs=1.0, gamma=1.4):
    """The paper's compressible-Euler MMS (supplement, Euler MMS): per-axis
    Mach-3 background u0 = v0 = 3 cs, p0 = rho0 cs^2 / gamma, fluctuations
    0.3 rho0, 0.3 cs and c_s^2 d rho + 0.2 p0 in the printed modes."""
    r0, c, gm = sp.Float(rho0), sp.Float(cs), sp.Float(gamma)
    p0 = r0 * c ** 2 / gm
    drho = sp.Rational(3, 10) * r0 * sp.sin(PI2 * X) * sp.cos(PI2 * Y) * sp.cos(T)
    du = sp.Rational(3, 10) * c * sp.cos(PI2 * X) * sp.sin(PI2 * Y) * sp.sin(T)
    dv = sp.Rational(3, 10) * c * sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.sin(T)
    dp = c ** 2 * drho + sp.Rational(1, 5) * p0 * sp.cos(PI2 * X) * sp.sin(PI2 * Y) * sp.sin(T)
    rho = r0 + drho
    u, v = 3 * c + du, 3 * c + dv
    p = p0 + dp
    E = p / (gm - 1) + rho * (u ** 2 + v ** 2) / 2
    return [rho, rho * u, rho * v, E], gm


@functools.lru_cache(maxsize=None)
def euler_exprs(rho0=1.0, cs=1.0, gamma=1.4):
    """Symbolic (exact fields, forcing) of the Euler MMS."""
    Q, gm = euler_exact_exprs(rho0, cs, gamma)
    rho, mx, my, E = Q
    p = (gm - 1) * (E - (mx ** 2 + my ** 2) / (2 * rho))
    Phi = [[mx, my],
           [mx ** 2 / rho + p, mx * my / rho],
           [mx * my / rho, my ** 2 / rho + p],
           [(E + p) * mx / rho, (E + p) * my / rho]]
    res = [sp.diff(Q[k], T) + _div(Phi[k], (X, Y)) for k in range(4)]
    return Q, res


def torch_fields(exprs):
    """f(Xg, Yg, t) -> [K, ...] torch tensor on the device and dtype of Xg,
    evaluating SymPy expressions of (x, y, t) with torch (test inputs such
    as a manufactured forcing evaluated next to the GPU stepper)."""
    import torch
    # numeric constants folded first (torch's pow takes no plain-number pair)
    fn = sp.lambdify((X, Y, T), [sp.N(e) for e in exprs], "torch", cse=True)

    def f(Xg, Yg, t):
        """t: a number (-> [K, *Xg.shape]) or a 1-D tensor of times
        (-> [len(t), K, *Xg.shape], all steps of a batch at once)."""
        tt = torch.as_tensor(t, dtype=Xg.dtype, device=Xg.device)
        if tt.dim() == 1:
            tt = tt.reshape((-1,) + (1,) * Xg.dim())
        shape = torch.broadcast_shapes(Xg.shape, tt.shape)
        vals = [v if torch.is_tensor(v) else torch.tensor(float(v), dtype=Xg.dtype, device=Xg.device)
                for v in fn(Xg, Yg, tt)]
        return torch.stack([v.expand(shape) for v in vals], dim=-Xg.dim() - 1).contiguous()
    return f


@functools.lru_cache(maxsize=None)
def euler_paper(rho0=1.0, cs=1.0, gamma=1.4):
    """(exact(x, y, t) -> [4, ...], forcing(x, y, t) -> [4, ...])."""
    Q, res = euler_exprs(rho0, cs, gamma)
    fQ = sp.lambdify((X, Y, T), Q, "numpy")
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    return _wrap2(fQ, Q), _wrap2(fS, res)


# ------------------------------------------------------------ MAXWELL ----
@functools.lru_cache(maxsize=None)
def maxwell_paper(amp=0.5, omega=4.0, c=1.0):
    """The paper's Maxwell TM MMS (supplement, Maxwell MMS): kx = 2 pi,
    ky = 4 pi, E_z ~ cos(omega t), H ~ sin(omega t), div H = 0."""
    A, w, cc = sp.Float(amp), sp.Float(omega), sp.Float(c)
    kx, ky = PI2, 2 * PI2
    Ez = A * sp.sin(kx * X) * sp.sin(ky * Y) * sp.cos(w * T)
    Hx = A * sp.sin(kx * X) * sp.cos(ky * Y) * sp.sin(w * T)
    Hy = -A * (kx / ky) * sp.cos(kx * X) * sp.sin(ky * Y) * sp.sin(w * T)
    Q = [Ez, Hx, Hy]
    Phi = [[-cc * Hy, cc * Hx], [sp.Integer(0), cc * Ez], [-cc * Ez, sp.Integer(0)]]
    res = [sp.diff(Q[k], T) + _div(Phi[k], (X, Y)) for k in range(3)]
    fQ = sp.lambdify((X, Y, T), Q, "numpy")
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    return _wrap2(fQ, Q), _wrap2(fS, res)


# --------------------------------------------------------- ALLEN-CAHN ----
@functools.lru_cache(maxsize=None)
def allencahn_paper(gamma=0.01, r=1.0):
    """The paper's Allen-Cahn MMS (supplement, Allen-Cahn MMS):
    phi = 0.7 sin(2 pi x) cos(2 pi y) cos t, trackers exact (grad phi), not
    forced; the phi row is forced with the flux at the exact trackers."""
    phi = sp.Rational(7, 10) * sp.sin(PI2 * X) * sp.cos(PI2 * Y) * sp.cos(T)
    gx, gy = sp.diff(phi, X), sp.diff(phi, Y)
    res = sp.diff(phi, T) + _div([-gamma * gx, -gamma * gy], (X, Y)) - r * (phi - phi ** 3)
    fQ = sp.lambdify((X, Y, T), [phi, gx, gy], "numpy")
    fS = sp.lambdify((X, Y, T), [res, sp.Integer(0), sp.Integer(0)], "numpy", cse=True)
    return _wrap2(fQ), _wrap2(fS)


# -------------------------------------------------- ULTRARELATIVISTIC ----
def relhydro_exact_exprs():
    """The paper's ultrarelativistic MMS (supplement): fluctuations of 0.4 about
    (E, S0, S1) = (3, 1.2, 1.2)."""
    a = sp.Rational(2, 5)
    E = a * sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.cos(T) + 3
    S0 = a * sp.cos(PI2 * X) * sp.cos(PI2 * Y) * sp.sin(T) + sp.Rational(6, 5)
    S1 = a * sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.sin(T) + sp.Rational(6, 5)
    return [E, S0, S1]


@functools.lru_cache(maxsize=None)
def relhydro_paper():
    Q = relhydro_exact_exprs()
    E, S0, S1 = Q
    p = (sp.sqrt(4 * E ** 2 - 3 * (S0 ** 2 + S1 ** 2)) - E) / 3
    v = [S0 / (E + p), S1 / (E + p)]
    Phi = [[S0, S1], [S0 * v[0] + p, S0 * v[1]], [S1 * v[0], S1 * v[1] + p]]
    res = [sp.diff(Q[k], T) + _div(Phi[k], (X, Y)) for k in range(3)]
    fQ = sp.lambdify((X, Y, T), Q, "numpy")
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    return _wrap2(fQ, Q), _wrap2(fS, res)


# ----------------------------------------------------------------- NSE ----
def nse_exact_exprs(rho0=1.0, cs=1.0, U=0.1, mu=0.01):
    """The paper's weakly compressible NSE MMS (supplement): Taylor-Green
    vortex with decay D = exp(-2 (nu / cs) k^2 t), rho = rho0 + p / cs^2,
    m = rho u; read nondimensionally (rho0 = cs = 1, U = 0.1, mu = 0.01:
    Ma 0.1, Re 10).  Returns (rho, m0, m1) and the exact trackers d_b m_a."""
    r0, c, Uu = sp.Float(rho0), sp.Float(cs), sp.Float(U)
    nu = sp.Float(mu) / r0
    k = PI2
    Dc = sp.exp(-2 * (nu / c) * k ** 2 * T)
    u = -Uu * sp.cos(k * X) * sp.sin(k * Y) * Dc
    v = Uu * sp.sin(k * X) * sp.cos(k * Y) * Dc
    p = -sp.Rational(1, 4) * r0 * Uu ** 2 * (sp.cos(2 * k * X) + sp.cos(2 * k * Y)) * Dc ** 2
    rho = r0 + p / c ** 2
    m = [rho * u, rho * v]
    G = [[sp.diff(m[a], (X, Y)[b]) for b in range(2)] for a in range(2)]
    return [rho, m[0], m[1]], G


@functools.lru_cache(maxsize=None)
def nse_paper(rho0=1.0, cs=1.0, U=0.1, mu=0.01):
    """Conserved rows forced with the flux at the exact trackers; tracker rows
    not forced (as for the other tracker systems)."""
    (rho, m0, m1), G = nse_exact_exprs(rho0, cs, U, mu)
    m = [m0, m1]
    cs2, muf = sp.Float(cs) ** 2, sp.Float(mu)
    Phi = [[m0, m1]]
    for a in range(2):
        Phi.append([m[a] * m[c] / rho + (rho * cs2 if a == c else 0) - muf * (G[a][c] + G[c][a]) / rho
                    for c in range(2)])
    Q = [rho, m0, m1, G[0][0], G[0][1], G[1][0], G[1][1]]
    res = [sp.diff(Q[k], T) + _div(Phi[k], (X, Y)) for k in range(3)] + [sp.Integer(0)] * 4
    fQ = sp.lambdify((X, Y, T), Q, "numpy")
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    return _wrap2(fQ, Q), _wrap2(fS, res)


# ------------------------------------------------------------- CNSF 2D ----
def cnsf2d_exact_exprs(rho0=1.0, cs=1.0, gamma=1.4):
    """The paper's 2D compressible NSF MMS (supplement): per-axis Mach 3 and 2
    background, fluctuations 0.20 rho0, 0.20 cs, 0.15 cs and cs^2 d rho +
    0.20 p0 in the printed modes, p0 = rho0 cs^2 / gamma."""
    r0, c, gm = sp.Float(rho0), sp.Float(cs), sp.Float(gamma)
    p0 = r0 * c ** 2 / gm
    drho = sp.Rational(1, 5) * r0 * sp.sin(PI2 * X) * sp.cos(PI2 * Y) * sp.cos(T)
    du = sp.Rational(1, 5) * c * sp.cos(PI2 * X) * sp.sin(PI2 * Y) * sp.sin(T)
    dv = sp.Rational(3, 20) * c * sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.cos(T)
    dp = c ** 2 * drho + sp.Rational(1, 5) * p0 * sp.cos(PI2 * X) * sp.sin(PI2 * Y) * sp.sin(T)
    rho = r0 + drho
    u, v = 3 * c + du, 2 * c + dv
    p = p0 + dp
    E = p / (gm - 1) + rho * (u ** 2 + v ** 2) / 2
    return [rho, rho * u, rho * v, E]


@functools.lru_cache(maxsize=None)
def cnsf2d_paper(mu, kappa, R=1.0, gamma=1.4, rho0=1.0, cs=1.0):
    """(exact(x, y, t) -> [12, ...], forcing -> [12, ...]): conserved rows
    forced with the flux at the exact trackers, tracker rows not forced."""
    Qc = cnsf2d_exact_exprs(rho0, cs, gamma)
    G = [sp.diff(Qc[j], v) for j in (0, 1, 2, 3) for v in (X, Y)]
    Q = Qc + G
    gm, muf, Kf, Rf = sp.Float(gamma), sp.Float(mu), sp.Float(kappa), sp.Float(R)
    rho, m0, m1, E = Qc
    u = [m0 / rho, m1 / rho]
    p = (gm - 1) * (E - (m0 * u[0] + m1 * u[1]) / 2)
    Gr = [G[0], G[1]]
    Gm = [[G[2], G[3]], [G[4], G[5]]]
    GE = [G[6], G[7]]
    du = [[(Gm[a][b] - u[a] * Gr[b]) / rho for b in range(2)] for a in range(2)]
    div = du[0][0] + du[1][1]
    tau = [[muf * (du[a][b] + du[b][a] - (sp.Rational(2, 3) * div if a == b else 0)) for b in range(2)]
           for a in range(2)]
    gT = []
    for b in range(2):
        gp = (gm - 1) * (GE[b] - (u[0] * Gm[0][b] + u[1] * Gm[1][b]) + (u[0] ** 2 + u[1] ** 2) * Gr[b] / 2)
        gT.append((gp - p * Gr[b] / rho) / (Rf * rho))
    Phi = [[m0, m1]]
    for a in range(2):
        Phi.append([(m0, m1)[a] * u[c] + (p if a == c else 0) - tau[a][c] for c in range(2)])
    Phi.append([(E + p) * u[c] - (tau[c][0] * u[0] + tau[c][1] * u[1]) - Kf * gT[c] for c in range(2)])
    res = [sp.diff(Qc[k], T) + _div(Phi[k], (X, Y)) for k in range(4)] + [sp.Integer(0)] * 8
    fQ = sp.lambdify((X, Y, T), Q, "numpy", cse=True)
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    return _wrap2(fQ), _wrap2(fS)


# ----------------------------------------------------------------- MHD ----
def mhd_exact_exprs(rho0=1.0, cs=1.0, gamma=1.4):
    """The paper's resistive-MHD MMS (supplement): per-axis Mach-3 flow, field
    in Alfven units with background (0.5, 0.5) cs, fluctuations 0.3 rho0 and
    0.3 cs in the printed modes (div dB = 0), dp = cs^2 drho + 0.2 p0 mode."""
    r0, c, gm = sp.Float(rho0), sp.Float(cs), sp.Float(gamma)
    p0 = r0 * c ** 2 / gm
    k = PI2
    drho = sp.Rational(3, 10) * r0 * sp.sin(k * X) * sp.cos(k * Y) * sp.cos(T)
    dp = c ** 2 * drho + sp.Rational(1, 5) * p0 * sp.cos(k * X) * sp.sin(k * Y) * sp.sin(T)
    u = 3 * c + sp.Rational(3, 10) * c * sp.cos(k * X) * sp.sin(k * Y) * sp.sin(T)
    v = 3 * c + sp.Rational(3, 10) * c * sp.sin(k * X) * sp.sin(k * Y) * sp.sin(T)
    Bx = c / 2 - sp.Rational(3, 10) * c * sp.cos(k * X) * sp.sin(k * Y) * sp.sin(T)
    By = c / 2 + sp.Rational(3, 10) * c * sp.sin(k * X) * sp.cos(k * Y) * sp.sin(T)
    rho = r0 + drho
    p = p0 + dp
    E = p / (gm - 1) + rho * (u ** 2 + v ** 2) / 2 + (Bx ** 2 + By ** 2) / 2
    return [rho, rho * u, rho * v, E, Bx, By]


@functools.lru_cache(maxsize=None)
def mhd_paper(mu, kappa, eta, gamma=1.4, rho0=1.0, cs=1.0):
    """(exact -> [18, ...], forcing -> [18, ...]): conserved rows forced with
    the flux and the Powell source at the exact trackers, tracker rows not."""
    Qc = mhd_exact_exprs(rho0, cs, gamma)
    G = [sp.diff(Qc[f], v) for f in range(6) for v in (X, Y)]
    gm, muf, Kf, ef = sp.Float(gamma), sp.Float(mu), sp.Float(kappa), sp.Float(eta)
    rho, m0, m1, E, B0, B1 = Qc
    m, B = [m0, m1], [B0, B1]
    u = [m0 / rho, m1 / rho]
    pg = (gm - 1) * (E - (m0 * u[0] + m1 * u[1]) / 2 - (B0 ** 2 + B1 ** 2) / 2)
    ptot = pg + (B0 ** 2 + B1 ** 2) / 2
    Gr, Gm, GE, GB = G[0:2], [G[2:4], G[4:6]], G[6:8], [G[8:10], G[10:12]]
    du = [[(Gm[a][b] - u[a] * Gr[b]) / rho for b in range(2)] for a in range(2)]
    div = du[0][0] + du[1][1]
    tau = [[muf * (du[a][b] + du[b][a] - (sp.Rational(2, 3) * div if a == b else 0)) for b in range(2)]
           for a in range(2)]
    gT = []
    for b in range(2):
        gp = (gm - 1) * (GE[b] - (u[0] * Gm[0][b] + u[1] * Gm[1][b]) + (u[0] ** 2 + u[1] ** 2) * Gr[b] / 2
                         - (B0 * GB[0][b] + B1 * GB[1][b]))
        gT.append((gp - pg * Gr[b] / rho) / rho)
    j = GB[1][0] - GB[0][1]
    uB = u[0] * B0 + u[1] * B1
    jxB = [-j * B1, j * B0]
    divB = GB[0][0] + GB[1][1]
    Phi = [[m0, m1]]
    for a in range(2):
        Phi.append([m[a] * u[c] + (ptot if a == c else 0) - B[a] * B[c] - tau[a][c] for c in range(2)])
    Phi.append([(E + ptot) * u[c] - B[c] * uB - (tau[c][0] * u[0] + tau[c][1] * u[1]) - Kf * gT[c] + ef * jxB[c]
                for c in range(2)])
    for a in range(2):
        Phi.append([B[a] * u[c] - u[a] * B[c] - ef * GB[a][c] for c in range(2)])
    S = [0, -divB * B0, -divB * B1, -divB * uB, -divB * u[0], -divB * u[1]]
    res = [sp.diff(Qc[k], T) + _div(Phi[k], (X, Y)) - S[k] for k in range(6)] + [sp.Integer(0)] * 12
    fQ = sp.lambdify((X, Y, T), Qc + G, "numpy", cse=True)
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    return _wrap2(fQ, Qc + G), _wrap2(fS, res)


# ------------------------------------------------------------ ELASTIC ----
@functools.lru_cache(maxsize=None)
def neohooke_paper(rho0=1.0, mu_s=1.0, lam_s=2.0, amp=0.06):
    """The paper's neo-Hookean MMS (supplement, elasticity MMS): F = I + grad w,
    v = d_t w for the printed displacement potential w of amplitude 0.06."""
    A = sp.Float(amp)
    w0 = A * (sp.sin(PI2 * X) * sp.sin(PI2 * Y) * sp.cos(T) + sp.sin(PI2 * X) * sp.cos(PI2 * Y) * sp.sin(T) / 2
              + sp.cos(PI2 * (X + Y)) * sp.cos(T) / 4)
    w1 = A * (sp.cos(PI2 * X) * sp.cos(PI2 * Y) * sp.sin(T) + sp.cos(PI2 * X) * sp.sin(PI2 * Y) * sp.cos(T) / 2
              + sp.sin(PI2 * (X - Y)) * sp.sin(T) / 4)
    w = [w0, w1]
    F = [[sp.Integer(1 if a == b else 0) + sp.diff(w[a], (X, Y)[b]) for b in range(2)] for a in range(2)]
    v = [sp.diff(w[a], T) for a in range(2)]
    J = F[0][0] * F[1][1] - F[0][1] * F[1][0]
    FiT = [[F[1][1] / J, -F[1][0] / J], [-F[0][1] / J, F[0][0] / J]]
    P = [[mu_s * (F[a][c] - FiT[a][c]) + lam_s * sp.log(J) * FiT[a][c] for c in range(2)] for a in range(2)]
    Q = [F[0][0], F[0][1], F[1][0], F[1][1], v[0], v[1]]
    Phi = [[-v[a] if b == c else sp.Integer(0) for c in range(2)] for a in range(2) for b in range(2)]
    Phi += [[-P[a][c] / rho0 for c in range(2)] for a in range(2)]
    res = [sp.diff(Q[k], T) + _div(Phi[k], (X, Y)) for k in range(6)]
    fQ = sp.lambdify((X, Y, T), Q, "numpy")
    fS = sp.lambdify((X, Y, T), res, "numpy", cse=True)
    return _wrap2(fQ, Q), _wrap2(fS, res)


# ---------------------------------------------------------------- NSF ----
def nsf_exact_exprs(gamma, rho0, p0, u0, amp):
    k = PI2
    A = sp.Float(amp)
    c2 = sp.Float(gamma * p0 / rho0)
    rho = rho0 + A * sp.sin(k * X) * sp.cos(k * Y) * sp.sin(k * Z) * sp.cos(T)
    u = [u0 + A * sp.cos(k * X) * sp.sin(k * Y) * sp.sin(k * Z) * sp.sin(T),
         u0 + A * sp.sin(k * X) * sp.cos(k * Y) * sp.sin(k * Z) * sp.sin(T),
         u0 + A * sp.sin(k * X) * sp.sin(k * Y) * sp.cos(k * Z) * sp.sin(T)]
    p = p0 + c2 * (rho - rho0) + A * p0 * sp.cos(k * X) * sp.sin(k * Y) * sp.cos(k * Z) * sp.sin(T)
    E = p / (gamma - 1) + rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / 2
    Tm = p / rho
    coords = (X, Y, Z)
    G = [[sp.diff(u[a], coords[b]) for b in range(3)] for a in range(3)]
    GT = [sp.diff(Tm, coords[b]) for b in range(3)]
    return rho, u, p, E, Tm, G, GT


def nsf_flux_exprs(Q, gamma, mu, kappa, tau_grad):
    """Phi (17 x 3) of the tracker-cascaded compressible NSF system, tensor form."""
    rho, m, E = Q[0], Q[1:4], Q[4]
    G = [[Q[5 + 3 * a + b] for b in range(3)] for a in range(3)]
    GT = Q[14:17]
    u = [m[a] / rho for a in range(3)]
    p = (gamma - 1) * (E - (m[0] * u[0] + m[1] * u[1] + m[2] * u[2]) / 2)
    Tm = p / rho
    trG = G[0][0] + G[1][1] + G[2][2]
    tau = [[mu * (G[a][b] + G[b][a] - (sp.Rational(2, 3) * trG if a == b else 0)) for b in range(3)]
           for a in range(3)]
    Phi = [[None] * 3 for _ in range(17)]
    for c in range(3):
        Phi[0][c] = m[c]
        for a in range(3):
            Phi[1 + a][c] = m[a] * u[c] + (p if a == c else 0) - tau[a][c]
        Phi[4][c] = (E + p) * u[c] - sum(tau[c][b] * u[b] for b in range(3)) - kappa * GT[c]
        for a in range(3):
            for b in range(3):
                Phi[5 + 3 * a + b][c] = G[a][b] * u[c] - (u[a] / tau_grad if b == c else 0)
        for a in range(3):
            Phi[14 + a][c] = GT[a] * u[c] - (Tm / tau_grad if a == c else 0)
    return Phi


@functools.lru_cache(maxsize=None)
def nsf17(gamma, rho0, p0, u0, amp, mu, kappa, tau_grad, force_trackers=False):
    """(exact(x,y,z,t) -> [17,...], forcing(x,y,z,t) -> [17,...])."""
    rho, u, p, E, Tm, G, GT = nsf_exact_exprs(gamma, rho0, p0, u0, amp)
    Q = [rho] + [rho * u[a] for a in range(3)] + [E] + [G[a][b] for a in range(3) for b in range(3)] + GT
    Phi = nsf_flux_exprs(Q, gamma, mu, kappa, tau_grad)
    coords = (X, Y, Z)
    S = [0] * 5 + [-Q[k] / tau_grad for k in range(5, 17)]
    rows = range(17) if force_trackers else range(5)
    res = []
    for k in range(17):
        if k in rows:
            res.append(sp.diff(Q[k], T) + _div(Phi[k], coords) - S[k])
        else:
            res.append(sp.Integer(0))
    fQ = sp.lambdify((X, Y, Z, T), Q, "numpy", cse=True)
    fS = sp.lambdify((X, Y, Z, T), res, "numpy", cse=True)
    return _wrap3(fQ, Q), _wrap3(fS, res)


# -------------------------------------------------------------- HCNSF ----
def hcnsf_coef_exprs():
    """Prescribed coefficient fields of the paper's homogenized-NSF MMS
    (supplement): solid velocity u_s = rotation (amplitude 0.2) + uniform
    translation c = (0.1, -0.1, 0.05) + oscillation (amplitude 0.1), and the
    porosity alpha = 1/2 + [sin k xi_0 + sin k xi_1 + sin k xi_2
    + 2 sin k xi_0 sin k xi_1 sin k xi_2] / 10 advected along xi = x - d,
    d_i = r_i(x) sin t + c_i t, with r the rotation's spatial profile
    (the reading of the printed displacement).  Velocities in units of cs."""
    k = PI2
    c = (sp.Rational(1, 10), -sp.Rational(1, 10), sp.Rational(1, 20))
    a2 = sp.Rational(1, 5)
    r = [a2 * sp.sin(k * X) * sp.cos(k * Y) * sp.cos(k * Z),
         -a2 * sp.cos(k * X) * sp.sin(k * Y) * sp.cos(k * Z),
         a2 * sp.cos(k * X) * sp.cos(k * Y) * sp.sin(k * Z)]
    us = [r[0] * sp.cos(T) + c[0] + sp.sin(T) * sp.cos(k * Z) / 10,
          r[1] * sp.cos(T) + c[1] + sp.cos(T) * sp.cos(k * X) / 10,
          r[2] * sp.sin(T) + c[2] + sp.sin(T) * sp.cos(k * Y) / 10]
    xi = [v - (r[i] * sp.sin(T) + c[i] * T) for i, v in enumerate((X, Y, Z))]
    s = [sp.sin(k * v) for v in xi]
    alpha = sp.Rational(1, 2) + (s[0] + s[1] + s[2] + 2 * s[0] * s[1] * s[2]) / 10
    return alpha, us


def hcnsf_exact_exprs(gamma=1.4, amp=0.2, mach=0.5):
    """14 exact fields of the paper's homogenized-NSF MMS in units
    rho0 = cs = 1 (p0 = 1, mean sound speed sqrt(gamma), drift Ma sqrt(gamma)):
    rho, rho u, E, sym grad u as (00, 11, 22, 01, 02, 12), grad T."""
    gm = sp.Float(gamma)
    rho, u, p, E, Tm, G, GT = nsf_exact_exprs(gm, 1, 1, sp.Float(mach) * sp.sqrt(gm), amp)
    sym = [(G[a][b] + G[b][a]) / 2 for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))]
    return [rho] + [rho * u[a] for a in range(3)] + [E] + sym + list(GT)


def hcnsf_flux_source_exprs(Q, b, gamma, mu, kappa, eta):
    """Phi (conserved rows, 5 x 3) and S (5) of the homogenized NSF system in
    tensor form (paper Sec. 3), at the exact trackers."""
    alpha, us = b[0], b[1:4]
    rho, m, E = Q[0], Q[1:4], Q[4]
    idx = {(0, 0): 5, (1, 1): 6, (2, 2): 7, (0, 1): 8, (0, 2): 9, (1, 2): 10}
    G = [[Q[idx[(min(a, c), max(a, c))]] for c in range(3)] for a in range(3)]
    GT = Q[11:14]
    u = [m[a] / rho for a in range(3)]
    p = (gamma - 1) * (E - (m[0] * u[0] + m[1] * u[1] + m[2] * u[2]) / 2)
    trG = G[0][0] + G[1][1] + G[2][2]
    tau = [[mu * (2 * G[a][c] - (sp.Rational(2, 3) * trG if a == c else 0)) for c in range(3)] for a in range(3)]
    Phi = [[m[c] for c in range(3)]]
    for a in range(3):
        Phi.append([m[a] * u[c] + (p if a == c else 0) - alpha * tau[a][c] for c in range(3)])
    Phi.append([(E + p) * u[c] - alpha * sum(tau[c][d] * u[d] for d in range(3)) - alpha * kappa * GT[c]
                for c in range(3)])
    drag = (1 - alpha) / eta
    Sm = [drag * (rho * us[a] - m[a]) for a in range(3)]
    S = [0] + Sm + [sum(Sm[a] * u[a] for a in range(3))]
    return Phi, S


@functools.lru_cache(maxsize=None)
def hcnsf_paper(mu, kappa, eta, gamma=1.4, amp=0.2, mach=0.5):
    """(exact -> [14, ...], forcing -> [14, ...], coefficients -> [4, ...]),
    all functions of (x, y, z, t): conserved rows forced with the flux and the
    drag source at the exact trackers and the prescribed (alpha, u_s),
    tracker rows not."""
    Q = hcnsf_exact_exprs(gamma, amp, mach)
    alpha, us = hcnsf_coef_exprs()
    b = [alpha] + us
    Phi, S = hcnsf_flux_source_exprs(Q, b, sp.Float(gamma), sp.Float(mu), sp.Float(kappa), sp.Float(eta))
    coords = (X, Y, Z)
    res = [sp.diff(Q[k], T) + _div(Phi[k], coords) - S[k] for k in range(5)] + [sp.Integer(0)] * 9
    fQ = sp.lambdify((X, Y, Z, T), Q, "numpy", cse=True)
    fS = sp.lambdify((X, Y, Z, T), res, "numpy", cse=True)
    fB = sp.lambdify((X, Y, Z, T), b, "numpy", cse=True)
    return _wrap3(fQ, Q), _wrap3(fS, res), _wrap3(fB, b)


# ------------------------------------------------------------- helpers ----
def _broadcast(vals, shape):
    return np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), shape) for v in vals])


def _wrap2(fn, exprs=None):
    def f(Xg, Yg, t):
        return _broadcast(fn(Xg, Yg, t), Xg.shape)
    f.exprs = exprs           # the SymPy expressions, for other evaluators
    return f


def _wrap2b(fn):
    def f(Xg, Yg):
        return _broadcast(fn(Xg, Yg), Xg.shape)
    return f


def _wrap3(fn, exprs=None):
    def f(Xg, Yg, Zg, t):
        return _broadcast(fn(Xg, Yg, Zg, t), Xg.shape)
    f.exprs = exprs
    return f


def rel_l2(a, b):
    """Paper's relative L2 error (validation section): ||a-b|| / ||b|| with
    ||f|| = (N^-1 sum f^2)^(1/2); the N^-1 cancels."""
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def eoc(ns, errs):
    """Negative least-squares slope of log2 err against log2 N."""
    x = np.log2(np.asarray(ns, dtype=float))
    y = np.log2(np.asarray(errs, dtype=float))
    return -float(np.polyfit(x, y, 1)[0])


# ------------------------------------------------ compiled evaluation ----
_GEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_gen")


def compiled(f3):
    """The same SymPy expressions as the 3D field function ``f3`` (made by
    ``_wrap3``), evaluated by generated C: common subexpressions eliminated
    by SymPy, each printed with ``ccode`` (17 significant digits), one
    OpenMP loop over the grid points, gcc -O2 without FMA contraction.  The
    values agree with numpy's evaluation of the same expressions up to
    rounding order (a few 1e-16 relative); it is some 20 times faster on a
    64^3 grid, which is what lets the 3D parity tests run the oracle for
    hundreds of steps."""
    exprs = [sp.sympify(e) for e in f3.exprs]
    repl, red = sp.cse(exprs)
    body = [f"        const double {s} = {sp.ccode(e)};" for s, e in repl]
    body += [f"        out[(size_t){k} * n + j] = {sp.ccode(e)};" for k, e in enumerate(red)]
    src = ("#include <math.h>\n#include <stddef.h>\n"
           "void eval(size_t n, const double *X, const double *Y, const double *Z, double t, double *out)\n"
           "{\n#pragma omp parallel for schedule(static)\n    for (size_t j = 0; j < n; ++j) {\n"
           "        const double x = X[j], y = Y[j], z = Z[j];\n"
           "        (void)x; (void)y; (void)z; (void)t;\n" + "\n".join(body) + "\n    }\n}\n")
    key = hashlib.sha256(src.encode()).hexdigest()[:20]
    os.makedirs(_GEN_DIR, exist_ok=True)
    so = os.path.join(_GEN_DIR, f"f_{key}.so")
    if not os.path.exists(so):
        c = os.path.join(_GEN_DIR, f"f_{key}.c")
        with open(c, "w") as fh:
            fh.write(src)
        tmp = so + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", c, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, so)
    lib = ctypes.CDLL(so)
    P = ctypes.POINTER(ctypes.c_double)
    lib.eval.argtypes = [ctypes.c_size_t, P, P, P, ctypes.c_double, P]
    K = len(exprs)

    def f(Xg, Yg, Zg, t):
        Xc, Yc, Zc = (np.ascontiguousarray(np.broadcast_to(a, Xg.shape), dtype=np.float64) for a in (Xg, Yg, Zg))
        out = np.empty((K,) + Xg.shape)
        lib.eval(Xc.size, Xc.ctypes.data_as(P), Yc.ctypes.data_as(P), Zc.ctypes.data_as(P), float(t),
                 out.ctypes.data_as(P))
        return out
    f.exprs = f3.exprs
    return f
