"""Pins of the oracle's two-relaxation-time collision (the operator family
the paper names as consuming its equilibria unchanged; textbook TRT): with
equal rates it is BGK; on a single periodic cell (streaming is the identity)
one step relaxes the first moment's non-equilibrium part at omega- and the
second moment's at omega+, and conserves the zeroth moment.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2607_05668_amd import inputs


def _swe(shape, lattice="D2Q9", **kw):
    n = max(shape)
    dx, dt, tau = oracle.recipe(n, "acoustic", 0.2, 2.0)
    return oracle.Oracle("swe2d", lattice, shape, dt, dx, tau, None, {"g": 1.0}, Q0=[1.0, 0.0, 0.0], **kw)


def test_magic_parameter():
    for om in (0.3, 1.0, 1.7, 1.999):
        for lam in (1 / 4, 3 / 16, 1 / 12):
            op = oracle.trt_omega_plus(om, lam)
            assert (1 / op - 0.5) * (1 / om - 0.5) == pytest.approx(lam, rel=1e-14)


@pytest.mark.parametrize("lattice", ["D2Q5", "D2Q9"])
def test_equal_rates_reduce_to_bgk(lattice):
    a, b = _swe((24, 24), lattice), _swe((24, 24), lattice)
    b_trt = _swe((24, 24), lattice, omega_plus=1.0 / a.tau)
    Q = inputs.swe_initial(24)
    for o in (a, b_trt):
        o.init(Q)
        o.step(40)
    assert np.abs(a.moments() - b_trt.moments()).max() < 1e-13
    assert np.abs(a.f - b_trt.f).max() < 1e-13


@pytest.mark.parametrize("lattice", ["D2Q5", "D2Q9"])
def test_single_cell_moment_relaxation(lattice):
    """Unforced SWE on a 1 x 1 periodic grid: post - eq moments equal
    (1 - omega-) and (1 - omega+) times the pre-collision ones."""
    cl, _, cs2 = oracle.lattice(lattice)
    c = cl[:, :2].astype(float)
    nq = len(c)
    rng = np.random.default_rng(91)
    o = _swe((1, 1), lattice, trt_lambda=3 / 16)
    om_m, om_p = 1.0 / o.tau, o.cfg.omega_plus[0]
    assert om_p != pytest.approx(om_m)
    for _ in range(10):
        f = rng.uniform(-0.05, 0.05, (3, nq, 1, 1))
        o.f = f.copy()
        q = o.moments()[:, 0, 0]
        eq1 = (o.dt / o.dx) * (o.flux(q) - o.flux([1.0, 0.0, 0.0]))[:, :2]
        o.step(1)
        post = o.f[:, :, 0, 0]
        pre = f[:, :, 0, 0]
        dq = q - np.array([1.0, 0.0, 0.0])
        for k in range(3):
            assert post[k].sum() == pytest.approx(pre[k].sum(), abs=1e-15)
            m1_pre, m1_post = c.T @ pre[k], c.T @ post[k]
            assert np.allclose(m1_post - eq1[k], (1 - om_m) * (m1_pre - eq1[k]), rtol=1e-12, atol=1e-16)
            m2_pre = np.einsum("ia,ib,i->ab", c, c, pre[k])
            m2_post = np.einsum("ia,ib,i->ab", c, c, post[k])
            m2_eq = cs2 * dq[k] * np.eye(2)
            assert np.allclose(m2_post - m2_eq, (1 - om_p) * (m2_pre - m2_eq), rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("lattice", ["D2Q5", "D2Q9"])
def test_regularized_single_cell(lattice):
    """Regularized collision on one periodic cell: the zeroth moment is
    conserved, the first moment's non-equilibrium part relaxes by exactly
    (1 - omega), and every second-moment non-equilibrium part vanishes."""
    cl, _, cs2 = oracle.lattice(lattice)
    c = cl[:, :2].astype(float)
    nq = len(c)
    rng = np.random.default_rng(93)
    o = _swe((1, 1), lattice, regularized=True)
    om = 1.0 / o.tau
    for _ in range(10):
        f = rng.uniform(-0.05, 0.05, (3, nq, 1, 1))
        o.f = f.copy()
        q = o.moments()[:, 0, 0]
        eq1 = (o.dt / o.dx) * (o.flux(q) - o.flux([1.0, 0.0, 0.0]))[:, :2]
        o.step(1)
        post, pre = o.f[:, :, 0, 0], f[:, :, 0, 0]
        dq = q - np.array([1.0, 0.0, 0.0])
        for k in range(3):
            assert post[k].sum() == pytest.approx(pre[k].sum(), abs=1e-15)
            assert np.allclose(c.T @ post[k] - eq1[k], (1 - om) * (c.T @ pre[k] - eq1[k]), rtol=1e-12, atol=1e-16)
            m2 = np.einsum("ia,ib,i->ab", c, c, post[k])
            assert np.allclose(m2, cs2 * dq[k] * np.eye(2), rtol=1e-12, atol=1e-15)


def test_regularized_is_trt_with_unit_symmetric_rate_on_d2q5():
    """On D2Q5 the first-order projection keeps exactly the antisymmetric
    non-equilibrium parts: regularized = TRT with omega+ = 1."""
    a = _swe((16, 16), "D2Q5", regularized=True)
    b = _swe((16, 16), "D2Q5", omega_plus=1.0)
    Q = inputs.swe_initial(16)
    for o in (a, b):
        o.init(Q)
        o.step(30)
    assert np.abs(a.f - b.f).max() < 1e-14
