"""Pins of the material law (Section 2): closed forms and calculus
identities that a slip in the oracle's formulas would break."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import material as M
from workloads import Material


MAT = Material()
TS = np.concatenate([np.linspace(100.0, 3500.0, 341), [300.0, 1563.0, 1593.0, 1623.0]])


def test_endpoints_and_clamp():
    assert M.heat_capacity(300.0, MAT) == pytest.approx(450.0)
    assert M.heat_capacity(1563.0, MAT) == pytest.approx(700.0)
    assert M.heat_capacity(5000.0, MAT) == pytest.approx(700.0)
    assert M.heat_capacity(100.0, MAT) == pytest.approx(450.0)
    assert M.conductivity(300.0, MAT) == pytest.approx(10.0)
    assert M.conductivity(1563.0, MAT) == pytest.approx(30.0)
    assert M.conductivity(0.5 * (300 + 1563), MAT) == pytest.approx(20.0)


def test_sensible_integral_matches_quadrature():
    # int_{T_lo}^{T} c(s) ds by adaptive quadrature of the clamped-linear c
    for T in (150.0, 300.0, 800.0, 1563.0, 2500.0):
        ref, _ = quad(lambda s: float(M.heat_capacity(s, MAT)), MAT.T_lo, T,
                      points=[MAT.T_lo, MAT.T_hi] if T > MAT.T_hi else None, limit=200)
        assert float(M.sensible_integral(T, MAT)) == pytest.approx(ref, rel=1e-12, abs=1e-9)


def test_enthalpy_slope_is_derivative():
    h = 1e-3
    fd = (M.enthalpy(TS + h, MAT) - M.enthalpy(TS - h, MAT)) / (2 * h)
    an = M.enthalpy_slope(TS, MAT)
    # away from the kinks of the clamped c(T) the derivative is smooth
    ok = (np.abs(TS - MAT.T_lo) > 2 * h) & (np.abs(TS - MAT.T_hi) > 2 * h)
    assert np.allclose(fd[ok], an[ok], rtol=1e-8, atol=0)


def test_phase_fraction_properties():
    Tm = 0.5 * (MAT.T_sol + MAT.T_liq)
    assert float(M.phase_fraction(Tm, MAT)) == pytest.approx(0.5, abs=1e-15)
    # the slope integrates to one: all latent heat is released exactly once
    tot, _ = quad(lambda s: float(M.phase_fraction_slope(s, MAT)), Tm - 2000, Tm + 2000,
                  points=[Tm], limit=400)
    assert tot == pytest.approx(1.0, abs=1e-12)
    # share of the latent heat released between solidus and liquidus:
    # tanh(S (T_liq - T_sol) / 2) = tanh(1.5) ~ 0.905
    share = float(M.phase_fraction(MAT.T_liq, MAT) - M.phase_fraction(MAT.T_sol, MAT))
    assert share == pytest.approx(np.tanh(1.5), rel=1e-14)
    assert share == pytest.approx(0.905, abs=5e-4)


def test_enthalpy_jump_across_melting():
    # H(hot) - H(cold) = rho int c + rho chi (f(hot) - f(cold))
    lo, hi = 1400.0, 1800.0
    dH = float(M.enthalpy(hi, MAT) - M.enthalpy(lo, MAT))
    sens = MAT.rho * (MAT.c_hi * (hi - MAT.T_hi)
                      + quad(lambda s: float(M.heat_capacity(s, MAT)), lo, MAT.T_hi)[0])
    lat = MAT.rho * MAT.latent * float(M.phase_fraction(hi, MAT) - M.phase_fraction(lo, MAT))
    assert dH == pytest.approx(sens + lat, rel=1e-12)
    assert lat == pytest.approx(MAT.rho * MAT.latent, rel=1e-5)
