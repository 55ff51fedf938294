"""Physical-unit front end (Sec. 4): unit conversions and the Gaussian width fit."""
import math
import numpy as np
import pytest

from paper_2009_02044_amd import physunits as pu


def test_rhic_setup_against_the_printed_set_up():
    s = pu.rhic_setup()
    # a (6 fm)^3 box on 2048 x 192^2 cells
    assert s.nz * s.a_L_fm == pytest.approx(6.0) and s.nt * s.a_T * s.a_L_fm == pytest.approx(6.0)
    assert s.a_T == pytest.approx(2048 / 192)
    # the printed Landau width for RHIC 200 GeV: sqrt(ln gamma) ~ 2.15 with gamma = 100
    assert s.gamma == pytest.approx(100.0) and s.sigma_landau == pytest.approx(2.15, abs=0.005)
    # Q_s^2 = 200^0.25 GeV^2
    assert s.Qs_GeV ** 2 == pytest.approx(200 ** 0.25)
    # L = m_N R / sqrt(s), R = 1.2 * 197^(1/3) fm
    assert s.L_fm == pytest.approx(1.2 * 197 ** (1 / 3) / 200)
    # conversions through hbar c: 1 fm = 5.0677 / GeV
    assert s.tau0 * s.a_L_fm == pytest.approx(1.0)
    assert s.m_ir / s.a_L_fm == pytest.approx(0.2 / pu.HBARC_GEV_FM)
    assert s.uv_cut / s.m_ir == pytest.approx(50.0)
    assert s.mu / s.m_ir == pytest.approx(s.Qs_GeV / 0.75 / 0.2)
    # the nucleus spans about 12 cells at this resolution
    assert 11.0 < s.sigma < 13.0


def test_gaussian_width_fit_recovers_a_gaussian():
    eta = np.linspace(-2.5, 2.5, 41)
    for sig in (1.28, 1.66, 2.34):
        assert pu.gaussian_width(eta, 3.0 * np.exp(-eta ** 2 / (2 * sig ** 2))) == pytest.approx(sig, rel=1e-12)
    assert pu.gaussian_width(eta, np.exp(0.1 * eta ** 2)) == math.inf
