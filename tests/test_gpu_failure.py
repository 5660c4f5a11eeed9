"""Runtime failure detection (Sec. 2.4.2): the sub-characteristic check of
the initialisation, and the non-finite scan of lbm_step every check_every
steps.  The non-finite value is planted as data (a NaN written by torch into
one population of the bound buffer); every kernel runs normally."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2607_05668_amd import inputs, lbm  # noqa: E402


def _swe(n, g=1.0, check_subchar=True):
    dx = 1.0 / n
    dt = 0.2 * dx
    params = {"g": g}
    if not check_subchar:
        params["check_subchar"] = 0.0
    return lbm.Stepper("swe2d", "D2Q9", (n, n), 0.5 + 2.0 * dt, dt, dx, "f32", params)


def test_nonfinite_population_stops_stepping():
    print("swe2d D2Q9 f32 64x64: NaN planted, check_every 5", flush=True)
    s = _swe(64)
    s.init(inputs.swe_initial(64))
    s.set_param("check_every", 5)
    assert s.param("check_every") == 5
    s.step(7)                                        # finite: no error
    assert s.reduce(lbm.RED_NONFINITE)[0] == 0
    torch.cuda.synchronize()
    cur = s.pop_b if s.steps % 2 else s.pop_a       # the buffer holding step 7's populations
    cur.view(torch.float32)[3 * 64 * 64 + 1234] = float("nan")
    with pytest.raises(lbm.LbmError) as e:
        s.step(10)
    assert e.value.code == lbm.LBM_ENONFINITE
    assert "non-finite populations after step 10" in str(e.value)
    assert s.steps == 10                             # stopped at the first scan after the NaN
    assert s.reduce(lbm.RED_NONFINITE)[0] > 0


def test_nonfinite_is_silent_without_check():
    s = _swe(64)
    s.init(inputs.swe_initial(64))
    torch.cuda.synchronize()
    s.pop_a.view(torch.float32)[777] = float("inf")
    s.step(6)
    assert s.steps == 6
    assert s.reduce(lbm.RED_NONFINITE)[0] > 0


def test_subcharacteristic_violation_is_rejected():
    """Shallow water at rest with g = 10, h = 1: lam sqrt(g h) = 0.2 sqrt(10)
    = 0.632 exceeds cs = 1/sqrt(3) = 0.577."""
    n = 32
    Q = np.stack([np.ones((n, n)), np.zeros((n, n)), np.zeros((n, n))])
    s = _swe(n, g=10.0)
    with pytest.raises(lbm.LbmError) as e:
        s.init(Q)
    assert e.value.code == lbm.LBM_ESUBCHAR
    assert "sub-characteristic" in str(e.value)
    sp = _swe(n, g=10.0, check_subchar=False)
    sp.init(Q)                                       # the check can be switched off
    assert sp.reduce(lbm.RED_MAXSPEED)[1] == pytest.approx(0.2 * np.sqrt(10.0) * np.sqrt(3.0), rel=1e-6)
    ok = _swe(n, g=1.0)
    ok.init(Q)                                       # 0.2 < 0.577: accepted
