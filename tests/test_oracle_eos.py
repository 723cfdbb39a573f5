"""Pins of the oracle's equation of state (App. B, Supplemental item 1).

Independent references: numerical quadrature of psi (the definition of
c_s^2 through psi = d ln c_s^2 / d rho), Richardson-extrapolated finite
differences of p(rho) for dp/drho and rho d2p/drho2, the identity
p - rho dp/drho = -rho^2 d(p/rho)/drho of item 1, the statements of App. B
(c_s^2 equal below rho1 and above rho3, A = 0 is an ideal gas, the example
A = 1.2 is admissible in 2D), and the equal-area form of the Maxwell
construction.
"""
import math

import numpy as np
import pytest
from scipy import integrate


def _model(orc, **kw):
    prm = dict(Q=21, nx=4, ny=4, nz=1, rho1=0.5, rho2=1.0, A=1.2, cs2_1=0.6)
    prm.update(kw)
    return orc.Model(**prm)


def _psi(m, r):
    rho3 = 2 * m.rho2 - m.rho1
    if m.rho1 < r < rho3:
        return m.A * math.sin(math.pi * (r - m.rho1) / (m.rho2 - m.rho1))
    return 0.0


def _deriv(f, x, h=1e-3, order=1):
    """Richardson-extrapolated central difference (error O(h^6))."""
    def d(hh):
        if order == 1:
            return (f(x + hh) - f(x - hh)) / (2 * hh)
        return (f(x + hh) - 2 * f(x) + f(x - hh)) / hh**2
    d1, d2, d4 = d(h), d(h / 2), d(h / 4)
    r1 = (4 * d2 - d1) / 3
    r2 = (4 * d4 - d2) / 3
    return (16 * r2 - r1) / 15


@pytest.mark.parametrize("prm", [dict(), dict(rho1=0.3, A=0.9, cs2_1=0.45), dict(rho1=0.3, A=0.8, cs2_1=0.39)])
def test_cs2_is_exp_integral_of_psi(orc, prm):
    m = _model(orc, **prm)
    for r in np.linspace(0.05, 2.5, 57):
        pts = [x for x in (m.rho1, m.rho2, 2 * m.rho2 - m.rho1) if min(m.rho1, r) < x < max(m.rho1, r)]
        I, _ = integrate.quad(lambda x: _psi(m, x), m.rho1, r, points=pts or None,
                              epsabs=1e-14, epsrel=1e-14, limit=200)
        assert orc.eos(m, r)[0, 0] == pytest.approx(m.cs2_1 * math.exp(I), rel=1e-12)


@pytest.mark.parametrize("prm", [dict(), dict(rho1=0.3, A=0.9, cs2_1=0.45)])
def test_eos_derivatives(orc, prm):
    m = _model(orc, **prm)
    rho3 = 2 * m.rho2 - m.rho1
    p = lambda r: orc.eos(m, r)[0, 1]
    # smooth points only (psi' jumps at rho1 and rho3)
    for r in list(np.linspace(m.rho1 + 0.05, rho3 - 0.05, 13)) + [0.2, rho3 + 0.3]:
        cs2, pp, dp, P1, P2, psi = orc.eos(m, r)[0]
        assert pp == pytest.approx(r * cs2, rel=1e-15)
        assert dp == pytest.approx(_deriv(p, r), rel=1e-9, abs=1e-11)
        assert P2 == pytest.approx(r * _deriv(p, r, order=2), rel=1e-6, abs=1e-8)
        assert P1 == pytest.approx(-r**2 * _deriv(lambda x: p(x) / x, r), rel=1e-9, abs=1e-11)
        assert psi == pytest.approx(_psi(m, r), abs=1e-15)


def test_cs2_same_outside_interval_and_ideal_gas(orc):
    m = _model(orc)
    rho3 = 2 * m.rho2 - m.rho1
    for r in [0.1, 0.3, m.rho1, rho3, rho3 + 0.5, 3.0]:
        assert orc.eos(m, r)[0, 0] == pytest.approx(m.cs2_1, rel=1e-15)
    g = _model(orc, A=0.0)
    for r in [0.2, 0.7, 1.3, 2.9]:
        cs2, p, dp, P1, P2, psi = orc.eos(g, r)[0]
        assert (cs2, dp, P1, P2) == pytest.approx((g.cs2_1, g.cs2_1, 0.0, 0.0), abs=1e-15)


def test_paper_example_is_admissible_in_2d(orc):
    """App. B: rho1=0.5, rho2=1, A=1.2, c_s^2(rho1)=0.6, d=2 satisfies all
    three conditions; in 3D the bulk-viscosity condition fails."""
    from oracle import eos_tools as E
    ad = E.admissibility(_model(orc))
    assert ad["weights_positive"] and ad["two_phase"] and ad["bulk_viscosity_positive"]
    ad3 = E.admissibility(_model(orc, Q=59, nz=4))
    assert ad3["weights_positive"] and ad3["two_phase"] and not ad3["bulk_viscosity_positive"]
    # too small an amplitude: no coexistence; A = 0 is an ideal gas
    assert not E.admissibility(_model(orc, A=0.5))["two_phase"]


@pytest.mark.parametrize("prm", [dict(), dict(rho1=0.3, A=0.9, cs2_1=0.45), dict(rho1=0.3, A=0.8, cs2_1=0.39)])
def test_maxwell_equal_area(orc, prm):
    """Coexistence: equal pressure, and the equal-area rule in the p(1/rho)
    plane, int_{v_l}^{v_g} p dv = p_c (v_g - v_l), computed by quadrature."""
    from oracle import eos_tools as E
    m = _model(orc, **prm)
    rg, rl, pc = E.maxwell(m)
    assert rg < rl
    assert E.pressure(m, rg) == pytest.approx(pc, rel=1e-12)
    assert E.pressure(m, rl) == pytest.approx(pc, rel=1e-12)
    vg, vl = 1 / rg, 1 / rl
    area, _ = integrate.quad(lambda v: E.pressure(m, 1 / v), vl, vg, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert area == pytest.approx(pc * (vg - vl), rel=1e-9)
