"""Checkpointed differentiable rollout of the shallow-water stepper.

Forward: initialise the populations at the equilibrium of (h0, 0, 0), run
``steps`` collide-and-stream steps with the topography-gradient source
b = grad z_b, keeping a device snapshot of the populations every ``ckpt``
steps, and return the final depth h^N.

Backward (discrete adjoint of the scheme, eq. lbe_update): seed
lam_{h,i} = dL/dh^N, then for each segment from last to first restore its
snapshot, recompute it while recording the pre-collision moment deviations,
and run the adjoint steps backwards through it, accumulating dL/db.
Finally map lam^0 through the equilibrium initialisation to dL/dh0.  All of
it runs in the library's HIP kernels; this module only orders the calls.

``rollout(h0, b, runner)`` wraps this in a ``torch.autograd.Function``.
"""
from __future__ import annotations

import math

from . import lbm


class SweRollout:
    def __init__(self, n=512, steps=500, ckpt=50, g=1.0, f=0.2, tau_r=2.0, storage="f32"):
        torch = lbm._torch()
        self.torch = torch
        dx, dt, tau = lbm.recipe(n, "acoustic", f, tau_r)
        self.stepper = lbm.Stepper("swe2d", "D2Q9", (n, n), tau, dt, dx, storage, {"g": g})
        self.n, self.steps, self.ckpt = n, int(steps), int(ckpt)
        self.nseg = int(math.ceil(self.steps / self.ckpt))
        s = self.stepper
        self.snaps = [torch.empty_like(s.pop_a) for _ in range(self.nseg)]
        self.hist = torch.empty((self.ckpt, s.K) + s.shape, dtype=s.real, device=s.device)
        self.lam = s.new_adjoint()
        self.tmp = s.new_adjoint()
        # one gradient buffer for every backward, so that the adjoint launches
        # captured for small grids keep their arguments
        self.grad_b = torch.zeros((2,) + s.shape, dtype=s.real, device=s.device)
        self.Q_init = None
        self.b = None
        self.generation = 0          # forwards run so far; backward must follow its own forward

    def forward(self, h0, b):
        torch, s = self.torch, self.stepper
        self.generation += 1
        h0 = h0.to(device=s.device, dtype=torch.float64)
        self.b = b.to(device=s.device, dtype=s.real).contiguous()
        s.set_field("grad_zb", self.b)
        z = torch.zeros_like(h0)
        self.Q_init = torch.stack([h0, z, z]).contiguous()
        s.init(self.Q_init)
        for j in range(self.nseg):
            s.snapshot(self.snaps[j])
            s.step(min(self.ckpt, self.steps - j * self.ckpt))
        return s.moments(dtype=torch.float64)[0]

    def backward(self, dL_dhN):
        torch, s = self.torch, self.stepper
        g = dL_dhN.to(device=s.device, dtype=s.real)
        z = torch.zeros_like(g)
        lam, tmp = self.lam, self.tmp
        s.adjoint_seed(torch.stack([g, z, z]), lam)
        grad_b = self.grad_b
        grad_b.zero_()
        for j in reversed(range(self.nseg)):
            m = min(self.ckpt, self.steps - j * self.ckpt)
            s.restore(self.snaps[j], j * self.ckpt)
            s.step_record(m, self.hist)
            out = s.adjoint_step(m, lam, tmp, self.hist, grad_b)
            if out is tmp:
                lam, tmp = tmp, lam
        dQ0 = s.adjoint_to_initial(lam, self.Q_init)
        return dQ0[0], grad_b.clone()


def _function():
    torch = lbm._torch()

    class _Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, h0, b, runner):
            ctx.runner = runner
            ctx.b_dtype = b.dtype
            ctx.h_dtype = h0.dtype
            out = runner.forward(h0, b)
            # the runner keeps one set of snapshots: remember which forward
            # they belong to, and let torch's version counters catch in-place
            # edits of h0 or b between forward and backward
            ctx.generation = runner.generation
            ctx.save_for_backward(h0, b)
            return out

        @staticmethod
        def backward(ctx, grad_hN):
            ctx.saved_tensors                     # raises if h0 or b changed in place
            if ctx.runner.generation != ctx.generation:
                raise RuntimeError("SweRollout ran another forward since this graph was built: its snapshots "
                                   "belong to that later forward; use one runner per pending backward")
            dh0, db = ctx.runner.backward(grad_hN)
            return dh0.to(ctx.h_dtype), db.to(ctx.b_dtype), None

    return _Rollout


_FN = None


def rollout(h0, b, runner: SweRollout):
    """h^N of the checkpointed rollout, differentiable w.r.t. h0 and b."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(h0, b, runner)
