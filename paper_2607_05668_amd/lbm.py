"""Python binding of the HIP collide-and-stream library (include/lbm.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch provides device memory and the stream; the library is
bound to ``torch.cuda.current_stream()`` at construction, so torch events
recorded on that stream time its kernels.  There is no CPU fallback: if the
library is not built, or no GPU is present, this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOTBOUND, LBM_EHIP, LBM_ESUBCHAR, LBM_ENONFINITE = 0, -1, -2, -3, -4, -5
F64, F32, F16, F16NE = 0, 1, 2, 3
RED_SUMS, RED_RELL2, RED_RELLINF, RED_MAXSPEED, RED_NONFINITE = 0, 1, 2, 3, 4
STORAGE = {"f64": F64, "f32": F32, "f16": F16, "f16ne": F16NE}

EXPORTS = ["lbm_create", "lbm_last_error", "lbm_num_fields", "lbm_num_velocities", "lbm_set_param", "lbm_get_param",
           "lbm_set_storage", "lbm_set_reference", "lbm_get_reference", "lbm_required_bytes", "lbm_bind",
           "lbm_set_field", "lbm_init_moments", "lbm_step", "lbm_step_record", "lbm_moments", "lbm_reduce", "lbm_reduce_static",
           "lbm_step_count", "lbm_time", "lbm_adjoint_seed", "lbm_adjoint_step", "lbm_adjoint_to_initial",
           "lbm_save", "lbm_load", "lbm_snapshot", "lbm_restore", "lbm_bw_copy", "lbm_bw_streams", "lbm_bw_streams3",
           "lbm_destroy"]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load liblbm.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, c_int, c_double, c_size = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.POINTER(c_double)
    lib.lbm_create.restype = vp
    lib.lbm_create.argtypes = [ctypes.c_char_p, ctypes.c_char_p, c_int, c_int, c_int, c_double, c_double, c_double]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_last_error.argtypes = [vp]
    for name in ("lbm_num_fields", "lbm_num_velocities"):
        getattr(lib, name).argtypes = [vp]
    lib.lbm_set_param.argtypes = [vp, ctypes.c_char_p, c_double]
    lib.lbm_get_param.argtypes = [vp, ctypes.c_char_p, dp]
    lib.lbm_set_storage.argtypes = [vp, c_int]
    lib.lbm_set_reference.argtypes = [vp, dp]
    lib.lbm_get_reference.argtypes = [vp, dp]
    lib.lbm_required_bytes.restype = c_size
    lib.lbm_required_bytes.argtypes = [vp, c_int]
    lib.lbm_bind.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_set_field.argtypes = [vp, ctypes.c_char_p, vp]
    lib.lbm_init_moments.argtypes = [vp, vp]
    lib.lbm_step.argtypes = [vp, c_int]
    lib.lbm_step_record.argtypes = [vp, c_int, vp]
    lib.lbm_moments.argtypes = [vp, vp, c_int, c_int]
    lib.lbm_reduce.argtypes = [vp, c_int, vp, dp]
    lib.lbm_reduce_static.argtypes = [vp, c_int, vp, dp]
    lib.lbm_step_count.restype = ctypes.c_longlong
    lib.lbm_step_count.argtypes = [vp]
    lib.lbm_time.restype = c_double
    lib.lbm_time.argtypes = [vp]
    lib.lbm_adjoint_seed.argtypes = [vp, vp, vp]
    lib.lbm_adjoint_step.argtypes = [vp, c_int, vp, vp, vp, vp]
    lib.lbm_adjoint_to_initial.argtypes = [vp, vp, vp, vp]
    lib.lbm_save.argtypes = [vp, vp, ctypes.POINTER(c_size)]
    lib.lbm_load.argtypes = [vp, vp, c_size]
    lib.lbm_snapshot.argtypes = [vp, vp]
    lib.lbm_restore.argtypes = [vp, vp, ctypes.c_longlong]
    lib.lbm_bw_copy.argtypes = [vp, vp, c_size, vp]
    lib.lbm_bw_streams.argtypes = [vp, vp, c_int, c_int, c_int, vp]
    lib.lbm_bw_streams3.argtypes = [vp, vp, c_int, c_int, c_int, c_int, vp]
    lib.lbm_destroy.restype = None
    lib.lbm_destroy.argtypes = [vp]
    _lib = lib
    return lib


def recipe(n: int, scaling: str, f: float, tau_r: float):
    """(dx, dt, tau_LB): dx = 1/N, dt = f dx (acoustic) or f dx^2 (diffusive),
    tau_LB = 1/2 + tau_R dt (paper, supplement, numerical configuration)."""
    dx = 1.0 / n
    dt = f * dx if scaling == "acoustic" else f * dx * dx
    return dx, dt, 0.5 + tau_r * dt


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the collide-and-stream library runs only on the device")
    return torch


class Stepper:
    """One collide-and-stream problem bound to torch-owned device memory."""

    def __init__(self, system, lattice, shape, tau, dt, dx, storage="f32", params=None, reference=None,
                 device=None):
        torch = _torch()
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device or "cuda")
        shape = tuple(int(s) for s in shape)
        nz, ny, nx = (1,) * (3 - len(shape)) + shape
        self.shape = shape
        h = self.lib.lbm_create(system.encode(), lattice.encode(), nx, ny, nz, tau, dt, dx)
        if not h:
            raise LbmError(LBM_EINVAL, self.lib.lbm_last_error(None).decode())
        self.h = ctypes.c_void_p(h)
        self.K = self.lib.lbm_num_fields(self.h)
        self.Q = self.lib.lbm_num_velocities(self.h)
        self.C = nx * ny * nz
        self.system, self.lattice = system, lattice
        self.tau, self.dt, self.dx = tau, dt, dx
        self.storage = storage
        for name, v in (params or {}).items():
            self._check(self.lib.lbm_set_param(self.h, name.encode(), float(v)))
        self._check(self.lib.lbm_set_storage(self.h, STORAGE[storage]))
        if reference is not None:
            ref = np.ascontiguousarray(reference, dtype=np.float64)
            self._check(self.lib.lbm_set_reference(self.h, ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        nbytes = self.lib.lbm_required_bytes(self.h, 0)
        aux = self.lib.lbm_required_bytes(self.h, 1)
        with torch.cuda.device(self.device):
            self.pop_a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.pop_b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.aux = torch.empty(aux, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.lbm_bind(self.h, self.pop_a.data_ptr(), self.pop_b.data_ptr(), self.aux.data_ptr(),
                                      ctypes.c_void_p(self.stream.cuda_stream)))
        self.real = torch.float64 if storage == "f64" else torch.float32
        self._fields = {}
        # parameters in use (single-precision arithmetic rounds dt/dx and 2 - omega once)
        self.dt, self.tau = self.param("dt"), self.param("tau")

    # ---- plumbing -------------------------------------------------------
    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field_tensor(self, x, dtype, k):
        t = self.torch.as_tensor(x, device=self.device, dtype=dtype).reshape(k, *self.shape).contiguous()
        return t

    # ---- API ------------------------------------------------------------
    @property
    def reference(self):
        out = np.zeros(self.K)
        self._check(self.lib.lbm_get_reference(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    @property
    def steps(self):
        return int(self.lib.lbm_step_count(self.h))

    @property
    def time(self):
        return float(self.lib.lbm_time(self.h))

    def param(self, name):
        """A parameter in use (see lbm_get_param): dt, dx, lambda, tau, omega, omega_tracker, tau_grad, ..."""
        v = ctypes.c_double()
        self._check(self.lib.lbm_get_param(self.h, name.encode(), ctypes.byref(v)))
        return v.value

    def set_param(self, name, value):
        self._check(self.lib.lbm_set_param(self.h, name.encode(), float(value)))

    # values per cell of each named per-cell field
    FIELD_COMPONENTS = {"grad_zb": 2, "coef": 4}

    def set_field(self, name, value):
        """Attach a per-cell field: "grad_zb" (swe2d, [2, ...]), "coef"
        (hcnsf3d_trk14: alpha, u_s, [4, ...]) or "source" (any system: an
        explicit source [K, ...] added to S_k); keeps a reference.  The
        tensor may be rewritten in place between steps."""
        if value is None:
            self._fields.pop(name, None)
            self._check(self.lib.lbm_set_field(self.h, name.encode(), None))
            return
        t = self.torch.as_tensor(value, device=self.device, dtype=self.real).contiguous()
        nb = self.K if name == "source" else self.FIELD_COMPONENTS.get(name)
        if nb is not None and t.numel() != nb * self.C:
            raise ValueError(f"field {name!r} needs {nb} x {self.C} values, got {t.numel()}")
        self._fields[name] = t
        self._check(self.lib.lbm_set_field(self.h, name.encode(), t.data_ptr()))

    def init(self, Q):
        """Equilibrium initialisation from fields Q [K, ...] (cast to float64)."""
        q = self._field_tensor(Q, self.torch.float64, self.K)
        self._check(self.lib.lbm_init_moments(self.h, q.data_ptr()))

    def step(self, n=1):
        self._check(self.lib.lbm_step(self.h, int(n)))

    def step_record(self, n, hist):
        """n steps writing the pre-collision deviations dQ into hist [n, K, ...]."""
        assert hist.is_contiguous() and hist.dtype == self.real and hist.numel() >= n * self.K * self.C
        self._check(self.lib.lbm_step_record(self.h, int(n), hist.data_ptr()))

    def moments(self, absolute=True, dtype=None, out=None):
        dtype = dtype or self.torch.float64
        if out is None:
            out = self.torch.empty((self.K,) + self.shape, dtype=dtype, device=self.device)
        code = F64 if out.dtype == self.torch.float64 else F32
        self._check(self.lib.lbm_moments(self.h, out.data_ptr(), 1 if absolute else 0, code))
        return out

    def reduce(self, what, ref=None, static=False):
        """FP64 reduction (lbm_reduce; with static=True lbm_reduce_static,
        which uses the library's static workspace instead of the bound one)."""
        out = np.zeros(2 * 18)
        rp = None
        if ref is not None:
            ref = self._field_tensor(ref, self.torch.float64, self.K)
            rp = ref.data_ptr()
        fn = self.lib.lbm_reduce_static if static else self.lib.lbm_reduce
        self._check(fn(self.h, what, rp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        n = {RED_SUMS: self.K, RED_RELL2: self.K, RED_RELLINF: self.K, RED_MAXSPEED: 2, RED_NONFINITE: 1}[what]
        return out[:n].copy()

    def save(self):
        n = ctypes.c_size_t(0)
        self._check(self.lib.lbm_save(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.lib.lbm_save(self.h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.lbm_load(self.h, buf, len(blob)))

    def snapshot(self, buf=None):
        """Device copy of the current populations (a uint8 tensor)."""
        if buf is None:
            buf = self.torch.empty_like(self.pop_a)
        self._check(self.lib.lbm_snapshot(self.h, buf.data_ptr()))
        return buf

    def restore(self, buf, step):
        self._check(self.lib.lbm_restore(self.h, buf.data_ptr(), int(step)))

    # ---- adjoint --------------------------------------------------------
    def new_adjoint(self):
        return self.torch.empty((self.K, self.Q) + self.shape, dtype=self.real, device=self.device)

    def adjoint_seed(self, dLdQ, lam):
        g = self._field_tensor(dLdQ, self.real, self.K)
        self._check(self.lib.lbm_adjoint_seed(self.h, g.data_ptr(), lam.data_ptr()))

    def adjoint_step(self, n, lam, tmp, hist, grad_field=None):
        """n adjoint steps from lam using hist [n, K, ...]; returns the buffer holding the result."""
        gp = None if grad_field is None else grad_field.data_ptr()
        self._check(self.lib.lbm_adjoint_step(self.h, int(n), lam.data_ptr(), tmp.data_ptr(),
                                              hist.data_ptr(), gp))
        return lam if n % 2 == 0 else tmp

    def adjoint_to_initial(self, lam0, Q_init):
        q = self._field_tensor(Q_init, self.torch.float64, self.K)
        out = self.torch.empty((self.K,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.lbm_adjoint_to_initial(self.h, lam0.data_ptr(), q.data_ptr(), out.data_ptr()))
        return out


def from_preset(preset, n=None, storage=None, params=None, reference=None, tau_r=None, f=None, lattice=None):
    """Stepper for a workload preset (paper_2607_05668_amd.inputs.PRESETS)."""
    n = preset.n if n is None else n
    dx, dt, tau = recipe(n, preset.scaling, preset.f if f is None else f,
                         preset.tau_r if tau_r is None else tau_r)
    dim = 3 if preset.lattice == "D3Q7" else 2
    p = dict(preset.params)
    if preset.g_tau is not None:
        p["g_tau"] = preset.g_tau
    p.update(params or {})
    return Stepper(preset.system, lattice or preset.lattice, (n,) * dim, tau, dt, dx, storage or preset.storage, p,
                   reference=reference)


def bw_streams(dst, src, nx, ny, fields, stream=None):
    """D2Q9 step memory-pattern probe: 9 fields planes of nx*ny floats pulled
    at the lattice offsets and stored (no arithmetic); see include/lbm.h."""
    lib = load_library()
    torch = _torch()
    need = 36 * fields * ((nx * ny + 63) // 64 * 64)       # tile-blocked, padded to 64 cells
    if dst.numel() * dst.element_size() < need or src.numel() * src.element_size() < need:
        raise ValueError(f"bw_streams needs {need} bytes per buffer")
    s = stream or torch.cuda.current_stream()
    rc = lib.lbm_bw_streams(dst.data_ptr(), src.data_ptr(), int(nx), int(ny), int(fields),
                            ctypes.c_void_p(s.cuda_stream))
    if rc != LBM_OK:
        raise LbmError(rc, "bw_streams failed")


def bw_streams3(dst, src, nx, ny, nz, fields, stream=None):
    """D3Q7 step memory-pattern probe: 7 fields planes of nx*ny*nz floats
    pulled at the lattice offsets and stored (no arithmetic); see include/lbm.h."""
    lib = load_library()
    torch = _torch()
    need = 28 * fields * ((nx * ny + 63) // 64 * 64) * nz    # tile-blocked z-slabs, padded to 64 cells
    if dst.numel() * dst.element_size() < need or src.numel() * src.element_size() < need:
        raise ValueError(f"bw_streams3 needs {need} bytes per buffer")
    s = stream or torch.cuda.current_stream()
    rc = lib.lbm_bw_streams3(dst.data_ptr(), src.data_ptr(), int(nx), int(ny), int(nz), int(fields),
                             ctypes.c_void_p(s.cuda_stream))
    if rc != LBM_OK:
        raise LbmError(rc, "bw_streams3 failed")


def bw_copy(dst, src, nbytes, stream=None):
    """Copy probe: nbytes from src to dst (16-byte non-temporal lanes)."""
    lib = load_library()
    torch = _torch()
    if dst.numel() * dst.element_size() < nbytes or src.numel() * src.element_size() < nbytes:
        raise ValueError(f"bw_copy needs {nbytes} bytes per buffer")
    s = stream or torch.cuda.current_stream()
    rc = lib.lbm_bw_copy(dst.data_ptr(), src.data_ptr(), int(nbytes), ctypes.c_void_p(s.cuda_stream))
    if rc != LBM_OK:
        raise LbmError(rc, "bw_copy failed")
