"""Conservation laws declared for the compiler slice (``compiler.py``): the
paper's systems written once in SI form, compiled into the gradient-free
tracker systems the step kernel runs.  Each function returns the compiled
``Scheme``; ``GENERATED`` lists the ones emitted into the library as
``gen_<name>`` systems."""
from __future__ import annotations

import functools

from .compiler import (DENSITY, DYNAMIC_VISCOSITY, GAS_CONSTANT, LENGTH, ONE, PRESSURE, THERMAL_CONDUCTIVITY,
                       TIME, VELOCITY, Model, div, dot, dt, eye, grad, outer, trace)


@functools.lru_cache(maxsize=None)
def euler2d():
    """Compressible Euler (Sec. 3): rho, rho u, E of an ideal gas."""
    m = Model("euler2d", 2)
    rho = m.state("rho", DENSITY)
    mom = m.state("m", DENSITY * VELOCITY, rank=1)
    E = m.state("E", PRESSURE)
    gamma = m.param("gamma", ONE)
    u = mom / rho
    p = (gamma - 1) * (E - dot(mom, u) / 2)
    m.law(dt(rho) + div(mom))
    m.law(dt(mom) + div(outer(mom, u) + p * eye(2)))
    m.law(dt(E) + div((E + p) * u))
    return m.compile()


@functools.lru_cache(maxsize=None)
def advdiff2d():
    """Advection-diffusion-reaction (Sec. 3): dt c + div(a c - nu grad c) =
    R c (1 - c); the diffusive gradient becomes a tracker advected with a."""
    m = Model("advdiff_trk2d", 2)
    c = m.state("c", ONE)
    ax, ay = m.param("ax", VELOCITY), m.param("ay", VELOCITY)
    nu = m.param("nu", LENGTH ** 2 / TIME)
    R = m.param("R", ONE / TIME)
    from sympy import Matrix
    a = Matrix([ax, ay])
    m.tracker_velocity(a)
    m.law(dt(c) + div(a * c - nu * grad(c)) - R * c * (1 - c))
    return m.compile()


@functools.lru_cache(maxsize=None)
def cnsf2d():
    """Compressible Navier-Stokes-Fourier in 2D (Sec. 3): the viscous stress
    and the heat flux are written with grad u and grad T of the derived
    velocity and temperature T = p / (R rho); Cascade expands both over the
    conserved fields and tracks grad rho, grad(rho u), grad E."""
    m = Model("cnsf_trk2d", 2)
    rho = m.state("rho", DENSITY)
    mom = m.state("m", DENSITY * VELOCITY, rank=1)
    E = m.state("E", PRESSURE)
    gamma = m.param("gamma", ONE)
    mu = m.param("mu", DYNAMIC_VISCOSITY)
    kappa = m.param("kappa", THERMAL_CONDUCTIVITY)
    Rg = m.param("R_gas", GAS_CONSTANT)
    u = mom / rho
    p = (gamma - 1) * (E - dot(mom, u) / 2)
    T = p / (Rg * rho)
    gu = grad(u)
    tau = mu * (gu + gu.T - 2 * trace(gu) / 3 * eye(2))
    q = -kappa * grad(T)
    m.tracker_velocity(u)
    m.law(dt(rho) + div(mom))
    m.law(dt(mom) + div(outer(mom, u) + p * eye(2) - tau))
    m.law(dt(E) + div((E + p) * u - tau * u + q))
    return m.compile()


@functools.lru_cache(maxsize=None)
def nsf3d17():
    """Compressible NSF in 3D with the velocity and the temperature T = p /
    rho tracked directly (9 + 3 trackers; the homogenized NSF at porosity 1
    with the full gradient basis)."""
    m = Model("nsf3d_trk17", 3)
    rho = m.state("rho", DENSITY)
    mom = m.state("m", DENSITY * VELOCITY, rank=1)
    E = m.state("E", PRESSURE)
    gamma = m.param("gamma", ONE)
    mu = m.param("mu", DYNAMIC_VISCOSITY)
    kappa = m.param("kappa", DYNAMIC_VISCOSITY)
    uex = mom / rho
    pex = (gamma - 1) * (E - dot(mom, uex) / 2)
    u = m.tracked("u", uex)
    T = m.tracked("T", pex / rho)
    gu = grad(u)
    tau = mu * (gu + gu.T - 2 * trace(gu) / 3 * eye(3))
    m.tracker_velocity(u)
    m.law(dt(rho) + div(mom))
    m.law(dt(mom) + div(outer(mom, u) + pex * eye(3) - tau))
    m.law(dt(E) + div((E + pex) * u - tau * u - kappa * grad(T)))
    return m.compile()


@functools.lru_cache(maxsize=None)
def nsf3d_strain():
    """The same 3D NSF with the velocity and T = p / rho tracked, compiled with
    Alg. 1's strain reduction: the stress depends on the velocity gradient
    only through its symmetric part, so its 9 trackers become the 6 strain
    trackers (00, 11, 22, 01, 02, 12), and the state is the 14-field basis
    of the paper's homogenized NSF at porosity 1."""
    m = Model("nsf3d_strain", 3)
    rho = m.state("rho", DENSITY)
    mom = m.state("m", DENSITY * VELOCITY, rank=1)
    E = m.state("E", PRESSURE)
    gamma = m.param("gamma", ONE)
    mu = m.param("mu", DYNAMIC_VISCOSITY)
    kappa = m.param("kappa", DYNAMIC_VISCOSITY)
    uex = mom / rho
    pex = (gamma - 1) * (E - dot(mom, uex) / 2)
    u = m.tracked("u", uex, VELOCITY)
    T = m.tracked("T", pex / rho, PRESSURE / DENSITY)
    gu = grad(u)
    tau = mu * (gu + gu.T - 2 * trace(gu) / 3 * eye(3))
    m.tracker_velocity(u)
    m.law(dt(rho) + div(mom))
    m.law(dt(mom) + div(outer(mom, u) + pex * eye(3) - tau))
    m.law(dt(E) + div((E + pex) * u - tau * u - kappa * grad(T)))
    return m.compile(strain="u")


# Systems emitted into the library: (library name, declaration, parameter
# defaults, default reference state).  The references are the backgrounds of
# the paper's manufactured solutions in units rho0 = cs = 1, as for the
# hand-written systems of the same name without the prefix.
GENERATED = [
    ("gen_euler2d", euler2d, {"gamma": 1.4}, [1.0, 3.0, 3.0, 1.0 / 1.4 / 0.4 + 9.0]),
    ("gen_advdiff_trk2d", advdiff2d, {"ax": 0.1, "ay": 0.05, "nu": 0.01, "R": 0.0}, [1.0, 0.0, 0.0]),
    ("gen_cnsf_trk2d", cnsf2d, {"gamma": 1.4, "mu": 0.01, "kappa": 0.04, "R_gas": 1.0},
     [1.0, 3.0, 2.0, 1.0 / 1.4 / 0.4 + 6.5] + [0.0] * 8),
]
