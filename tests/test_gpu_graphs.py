"""Small-grid launch batching: runs of step and adjoint launches replayed from
captured HIP graphs give bit-identical results to one launch per step, on
every replay, with other work on the stream between replays, after the
kernel arguments change (a new source field, a re-initialisation), and for
the moment history and the adjoint of the checkpointed rollout."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2607_05668_amd import inputs, lbm, rollout  # noqa: E402


def _pair(make):
    a, b = make(), make()
    b.set_param("graphs", 0)
    assert a.param("graphs") == 1 and b.param("graphs") == 0
    return a, b


def test_swe_steps_replayed_from_graphs_are_bit_identical():
    print("swe2d D2Q9 f32 96x128: graphs vs one launch per step", flush=True)

    def make():
        dx = 1.0 / 128
        return lbm.Stepper("swe2d", "D2Q9", (96, 128), 0.5 + 2 * 0.2 * dx, 0.2 * dx, dx, "f32", {"g": 1.0})
    a, b = _pair(make)
    Q = inputs.swe_initial(128)[:, :96, :]
    bf = 20 * inputs.topography_gradient(128)[:, :96, :]
    for s in (a, b):
        s.set_field("grad_zb", bf)
        s.init(np.ascontiguousarray(Q))
    for rep, n in enumerate((37, 100, 5, 3, 64, 37, 37)):
        a.step(n)
        b.step(n)
        ma, mb = a.moments(), b.moments()          # eager work between the replays
        sa, sb = a.reduce(lbm.RED_SUMS), b.reduce(lbm.RED_SUMS)
        assert a.steps == b.steps
        assert torch.equal(ma, mb), f"replay {rep} ({n} steps)"
        assert np.array_equal(sa, sb)
        if rep == 3:                               # new argument: a different topography field
            bf2 = -0.5 * bf
            a.set_field("grad_zb", bf2)
            b.set_field("grad_zb", bf2)
    # re-initialisation resets the A/B parity and the step count
    for s in (a, b):
        s.init(np.ascontiguousarray(Q))
        s.step(41)
    assert torch.equal(a.moments(), b.moments())


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_other_storage_replayed_from_graphs(storage):
    print(f"advdiff_trk2d D2Q5 {storage} 64x64: graphs vs one launch per step", flush=True)
    p = inputs.PRESETS["advdiff64"]
    a, b = _pair(lambda: lbm.from_preset(p, storage=storage))
    Q = inputs.advdiff_initial(64)
    for s in (a, b):
        s.init(Q)
    for n in (200, 13, 1):
        a.step(n)
        b.step(n)
        assert torch.equal(a.moments(), b.moments())


def test_history_and_adjoint_replayed_from_graphs():
    """The checkpointed rollout (64^2, 130 steps, snapshot every 50, last
    segment ragged) with graphs and without: identical final depth and
    identical gradients, twice in a row."""
    print("swe2d adjoint 64x64 130 steps: graphs vs one launch per step", flush=True)
    n = 64
    ra = rollout.SweRollout(n=n, steps=130, ckpt=50)
    rb = rollout.SweRollout(n=n, steps=130, ckpt=50)
    rb.stepper.set_param("graphs", 0)
    h0 = torch.tensor(inputs.swe_height(n), device="cuda")
    b = torch.tensor(20 * inputs.topography_gradient(n), device="cuda", dtype=torch.float32)
    tgt = torch.tensor(inputs.swe_height(n, seed=inputs.SEED_SWE_TARGET), device="cuda")
    for rep in range(2):
        ha, hb = ra.forward(h0, b), rb.forward(h0, b)
        assert torch.equal(ha, hb), rep
        ga, gb = ra.backward((ha - tgt) / ha.numel()), rb.backward((hb - tgt) / hb.numel())
        assert torch.equal(ga[0], gb[0]) and torch.equal(ga[1], gb[1]), rep
