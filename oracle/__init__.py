"""FP64 CPU oracle of the collide-and-stream scheme -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never uses it and
shares no code with it; the only thing both sides import is the seeded input
module ``paper_2607_05668_amd.inputs`` (random fields and presets, no method
arithmetic).

The stepping itself is plain C (``lbm_oracle.c``, IEEE double, no FMA
contraction, OpenMP over cells); this module only marshals numpy arrays and
derives the scheme's parameters from the paper's recipe:

* time step: ``dt = f dx`` (acoustic) or ``f dx^2`` (diffusive), ``dx = 1/N``
  (supplement, numerical configuration);
* ``tau_LB = 1/2 + tau_R dt`` (Sec. 2.4.1), conserved fields collide at
  ``omega = 1/tau_LB``;
* trackers: ``tau_grad = g_tau dt`` inside flux and source (Sec. 2.1.1), and
  they collide at the fixed rate ``1/(g_tau + 1)`` (supplement);
* ``lam = dt/dx`` multiplies the flux in the equilibrium (eq. feq).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

SYSTEMS = {"advdiff_trk2d": 0, "swe2d": 1, "neohooke2d": 2, "nsf3d_trk17": 3, "burgers2d": 4, "euler2d": 5,
           "maxwell2d": 6, "allencahn_trk2d": 7, "relhydro2d": 8, "nse_trk2d": 9,
           "cnsf_trk2d": 10, "mhd_trk2d": 11, "hcnsf3d_trk14": 12}
LATTICES = {"D2Q5": 0, "D2Q9": 1, "D3Q7": 2}
LATTICE_DIM = {"D2Q5": 2, "D2Q9": 2, "D3Q7": 3}
SYSTEM_DIM = {"advdiff_trk2d": 2, "swe2d": 2, "neohooke2d": 2, "nsf3d_trk17": 3, "burgers2d": 2, "euler2d": 2,
              "maxwell2d": 2, "allencahn_trk2d": 2, "relhydro2d": 2, "nse_trk2d": 2,
              "cnsf_trk2d": 2, "mhd_trk2d": 2, "hcnsf3d_trk14": 3}
PARAM_INDEX = {"g": 0, "ax": 1, "ay": 2, "az": 3, "nu": 4, "R": 5, "tau_grad": 6,
               "gamma": 7, "mu": 8, "kappa": 9, "rho0": 10, "mu_s": 11, "lambda_s": 12,
               "c": 13, "cs_phys": 14, "R_gas": 15,
               "eta": 4}
TRACKER_FIELDS = {"advdiff_trk2d": range(1, 3), "nsf3d_trk17": range(5, 17), "allencahn_trk2d": range(1, 3),
                  "nse_trk2d": range(3, 7), "cnsf_trk2d": range(4, 12),
                  "mhd_trk2d": range(6, 18), "hcnsf3d_trk14": range(5, 14)}
# components of the per-cell coefficient field b ([NB, ...]): the homogenized
# NSF system's (alpha, u_s); otherwise one per dimension (SWE: grad z_b)
COEF_COMPONENTS = {"hcnsf3d_trk14": 4}
MAXK = 18


class _Cfg(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int), ("lattice", ctypes.c_int),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("shifted", ctypes.c_int),
                ("lam", ctypes.c_double), ("dt", ctypes.c_double),
                ("omega", ctypes.c_double * MAXK), ("Q0", ctypes.c_double * MAXK),
                ("par", ctypes.c_double * 16),
                ("trt", ctypes.c_int), ("omega_plus", ctypes.c_double * MAXK)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        d = P(ctypes.c_double)
        c = P(_Cfg)
        lib.oracle_init.argtypes = [c, d, d, d]
        lib.oracle_moments.argtypes = [c, d, d]
        lib.oracle_step.argtypes = [c, d, d, d, d]
        lib.oracle_flux.argtypes = [c, d, d, d]
        lib.oracle_source.argtypes = [c, d, d, d]
        lib.oracle_adjoint_step.argtypes = [c, d, d, d, d, d]
        lib.oracle_init_adjoint.argtypes = [c, d, d, d]
        lib.oracle_num_fields.argtypes = [ctypes.c_int]
        lib.oracle_num_velocities.argtypes = [ctypes.c_int]
        lib.oracle_lattice.argtypes = [ctypes.c_int, P(ctypes.c_int), d, d]
        lib.oracle_num_threads.argtypes = []
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice(name: str):
    """(c [Q, 3] int, w [Q], cs2) of the oracle's velocity set."""
    lib = _load()
    c = np.zeros(27 * 3, dtype=np.int32)
    w = np.zeros(27)
    cs2 = ctypes.c_double()
    q = lib.oracle_lattice(LATTICES[name], c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(w),
                           ctypes.byref(cs2))
    return c[:3 * q].reshape(q, 3).copy(), w[:q].copy(), cs2.value


def num_threads() -> int:
    """Threads the oracle's OpenMP loops run on."""
    return int(_load().oracle_num_threads())


def recipe(n: int, scaling: str, f: float, tau_r: float):
    """(dx, dt, tau_LB) of the paper's refinement recipe."""
    dx = 1.0 / n
    dt = f * dx if scaling == "acoustic" else f * dx * dx
    return dx, dt, 0.5 + tau_r * dt


class Oracle:
    """FP64 stepper on an nx x ny (x nz) periodic grid.

    Arrays use the SoA layout ``[K, (nz,) ny, nx]`` for fields and
    ``[K, Q, (nz,) ny, nx]`` for populations, x fastest.  ``omega_tracker``
    overrides the trackers' collision rate 1/(g_tau + 1), e.g. to run exactly
    the rate a single-precision stepper rounded it to.
    """

    def __init__(self, system, lattice, shape, dt, dx, tau, g_tau=None, params=None,
                 Q0=None, shifted=True, omega_tracker=None, trt_lambda=None, omega_plus=None,
                 omega_plus_tracker=None, regularized=False):
        if LATTICE_DIM[lattice] != SYSTEM_DIM[system]:
            raise ValueError("lattice dimension does not match the system")
        self.lib = _load()
        self.system, self.lattice = system, lattice
        self.shape = tuple(shape)                     # (ny, nx) or (nz, ny, nx)
        nz, ny, nx = (1,) * (3 - len(shape)) + self.shape
        self.K = self.lib.oracle_num_fields(SYSTEMS[system])
        self.Q = self.lib.oracle_num_velocities(LATTICES[lattice])
        self.C = nx * ny * nz
        self.dt, self.dx, self.tau = dt, dx, tau
        cfg = _Cfg()
        cfg.system, cfg.lattice = SYSTEMS[system], LATTICES[lattice]
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.shifted = 1 if shifted else 0
        cfg.lam = dt / dx
        cfg.dt = dt
        params = dict(params or {})
        if g_tau is not None:
            params["tau_grad"] = g_tau * dt
        for k in range(MAXK):
            cfg.omega[k] = 1.0 / tau
        for k in TRACKER_FIELDS.get(system, ()):
            if g_tau is None:
                raise ValueError("system has tracker fields: g_tau required")
            cfg.omega[k] = 1.0 / (g_tau + 1.0) if omega_tracker is None else omega_tracker
        for name, v in params.items():
            cfg.par[PARAM_INDEX[name]] = float(v)
        # two-relaxation-time collision: the symmetric rate from the magic
        # parameter, or given explicitly (conserved fields, trackers)
        if regularized:
            cfg.trt = 2
        elif trt_lambda is not None or omega_plus is not None:
            cfg.trt = 1
            trk = set(TRACKER_FIELDS.get(system, ()))
            for k in range(MAXK):
                given = omega_plus_tracker if k in trk else omega_plus
                cfg.omega_plus[k] = given if given is not None else trt_omega_plus(cfg.omega[k], trt_lambda)
        if shifted:
            if Q0 is None:
                raise ValueError("shifted form needs a reference state Q0")
            for k in range(self.K):
                cfg.Q0[k] = float(Q0[k])
        self.cfg = cfg
        self.params = params
        self.f = np.zeros((self.K, self.Q) + self.shape)
        self.t = 0.0
        self.nsteps = 0

    # ---- single-state evaluations -------------------------------------
    def flux(self, q, b=None):
        q = np.ascontiguousarray(q, dtype=np.float64)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        out = np.zeros(self.K * 3)
        self.lib.oracle_flux(ctypes.byref(self.cfg), _ptr(q), _ptr(bb), _ptr(out))
        return out.reshape(self.K, 3)

    def source(self, q, b=None):
        q = np.ascontiguousarray(q, dtype=np.float64)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        out = np.zeros(self.K)
        self.lib.oracle_source(ctypes.byref(self.cfg), _ptr(q), _ptr(bb), _ptr(out))
        return out

    # ---- fields ---------------------------------------------------------
    def init(self, Qf, b=None):
        """Populations at the (shifted) equilibrium of the fields ``Qf``; ``b``
        is the per-cell coefficient field at t = 0 when the flux reads one."""
        Qf = np.ascontiguousarray(Qf, dtype=np.float64).reshape((self.K,) + self.shape)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        self.lib.oracle_init(ctypes.byref(self.cfg), _ptr(Qf), _ptr(bb), _ptr(self.f))
        self.t = 0.0
        self.nsteps = 0

    def moments(self, f=None):
        f = self.f if f is None else np.ascontiguousarray(f)
        out = np.zeros((self.K,) + self.shape)
        self.lib.oracle_moments(ctypes.byref(self.cfg), _ptr(f), _ptr(out))
        return out

    def step(self, n=1, source=None, b=None, history=None):
        """Advance n steps.  ``source(t)`` returns an explicit [K, ...] source
        evaluated at the given time (called with t_n + dt/2); ``b`` is the
        per-cell coefficient field [NB, ...], or a function of time giving it
        (called with t_n + dt/2, like the source); ``history`` (a list)
        receives a copy of the pre-collision populations of every step taken."""
        bb = None if (b is None or callable(b)) else np.ascontiguousarray(b, dtype=np.float64)
        out = np.empty_like(self.f)
        for _ in range(n):
            S = None
            if source is not None:
                S = np.ascontiguousarray(source(self.t + 0.5 * self.dt), dtype=np.float64)
            if callable(b):
                bb = np.ascontiguousarray(b(self.t + 0.5 * self.dt), dtype=np.float64)
            if history is not None:
                history.append(self.f.copy())
            self.lib.oracle_step(ctypes.byref(self.cfg), _ptr(self.f), _ptr(out), _ptr(S), _ptr(bb))
            self.f, out = out, self.f
            self.nsteps += 1
            self.t = self.nsteps * self.dt

    # ---- discrete adjoint ----------------------------------------------
    def adjoint_step(self, lam_next, f_n, b=None, grad_b=None):
        lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
        f_n = np.ascontiguousarray(f_n, dtype=np.float64)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        out = np.empty_like(lam_next)
        self.lib.oracle_adjoint_step(ctypes.byref(self.cfg), _ptr(lam_next), _ptr(out), _ptr(f_n),
                                     _ptr(bb), _ptr(grad_b))
        return out

    def init_adjoint(self, lam0, Qf):
        lam0 = np.ascontiguousarray(lam0, dtype=np.float64)
        Qf = np.ascontiguousarray(Qf, dtype=np.float64).reshape((self.K,) + self.shape)
        out = np.zeros((self.K,) + self.shape)
        self.lib.oracle_init_adjoint(ctypes.byref(self.cfg), _ptr(lam0), _ptr(Qf), _ptr(out))
        return out


def trt_omega_plus(omega_minus: float, magic: float) -> float:
    """Symmetric TRT rate from the antisymmetric one and the magic parameter
    Lambda = (1/omega+ - 1/2)(1/omega- - 1/2) (Ginzburg's TRT)."""
    return 1.0 / (0.5 + magic / (1.0 / omega_minus - 0.5))


def make(preset, n=None, shifted=True, Q0=None, params=None, tau_r=None, f=None):
    """Oracle for a workload preset (paper_2607_05668_amd.inputs.PRESETS)."""
    n = preset.n if n is None else n
    dx, dt, tau = recipe(n, preset.scaling, preset.f if f is None else f,
                         preset.tau_r if tau_r is None else tau_r)
    dim = SYSTEM_DIM[preset.system]
    shape = (n,) * dim
    p = dict(preset.params)
    p.update(params or {})
    p = {k: v for k, v in p.items() if k in PARAM_INDEX}
    return Oracle(preset.system, preset.lattice, shape, dt, dx, tau, preset.g_tau, p,
                  Q0=Q0, shifted=shifted)
