"""lbm_reduce_static (the reductions with the library's static per-GPU
workspace, for callers that cannot allocate) against lbm_reduce (the bound
workspace), through the C ABI: every reduction, two calls in a row on
different handles, the second on a smaller grid.  Same kernels in the same
order, so the results must agree bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2607_05668_amd import inputs, lbm  # noqa: E402

WHATS = [lbm.RED_SUMS, lbm.RED_RELL2, lbm.RED_RELLINF, lbm.RED_MAXSPEED, lbm.RED_NONFINITE]


def _stepper(system, shape, storage):
    if system == "swe2d":
        ny, nx = shape
        dx = 1.0 / max(shape)
        g = lbm.Stepper("swe2d", "D2Q9", shape, 0.5 + 2.0 * 0.2 * dx, 0.2 * dx, dx, storage, {"g": 1.0})
        Q = inputs.swe_initial(max(shape))[:, :ny, :nx]
    else:
        n = max(shape)
        pre = inputs.PRESETS["nsf256"]
        dx = 1.0 / n
        dt = pre.f * dx
        g = lbm.Stepper(pre.system, pre.lattice, shape, 0.5 + pre.tau_r * dt, dt, dx, storage,
                        dict(pre.params, g_tau=pre.g_tau))
        Q = inputs.nsf_exact(n, 0.0)[:, :shape[0], :shape[1], :shape[2]]
    g.init(np.ascontiguousarray(Q))
    g.step(7)
    return g


def _compare(g, seed):
    M = g.moments().cpu().numpy()
    ref = M + 1e-3 * np.random.default_rng(seed).normal(size=M.shape)
    for what in WHATS:
        r = ref if what in (lbm.RED_RELL2, lbm.RED_RELLINF) else None
        a = g.reduce(what, r)
        b = g.reduce(what, r, static=True)
        print(f"{g.system} {g.shape} what={what}: bound {a[:3]} static {b[:3]}", flush=True)
        assert np.array_equal(a, b), what


@pytest.mark.parametrize("system,big,small,storage", [
    ("swe2d", (96, 128), (40, 50), "f32"),
    ("swe2d", (64, 64), (17, 30), "f16"),
    ("nsf3d_trk17", (24, 24, 32), (8, 12, 16), "f32"),
])
def test_reduce_static_matches_bound_workspace(system, big, small, storage):
    print(f"reduce_static {system} {storage}: {big} then {small}", flush=True)
    g1 = _stepper(system, big, storage)
    _compare(g1, 1)
    g2 = _stepper(system, small, storage)
    _compare(g2, 2)
    # the first handle again, after the smaller one left its partials behind
    _compare(g1, 3)
