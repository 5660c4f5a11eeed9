"""The seeded input module's closed-form fields agree with the oracle's
independently written (SymPy) manufactured solutions where both exist.  CPU
only."""
import numpy as np
import pytest

from oracle import mms
from paper_2607_05668_amd import inputs


@pytest.mark.parametrize("t", [0.0, 0.37, 1.3])
def test_hcnsf_inputs_match_the_oracle_mms(t):
    fQ, _, fB = mms.hcnsf_paper(0.01, 0.01, 0.1)
    n = 7
    X, Y, Z = inputs.grid3(n)
    assert np.abs(inputs.hcnsf_exact(n, t) - fQ(X, Y, Z, t)).max() < 1e-14
    assert np.abs(inputs.hcnsf_coefficients(n, t) - fB(X, Y, Z, t)).max() < 1e-14


def test_mhd_and_cnsf_initial_states_match_the_oracle_mms():
    n = 16
    X, Y = inputs.grid2(n)
    fQ, _ = mms.mhd_paper(0.01, 0.01, 0.01)
    assert np.abs(inputs.mhd_initial(n) - fQ(X, Y, 0.0)).max() < 1e-13
    fQ, _ = mms.cnsf2d_paper(0.01, 0.04)
    assert np.abs(inputs.cnsf2d_initial(n) - fQ(X, Y, 0.0)).max() < 1e-13
