"""Equation-of-state utilities of App. B, on top of the oracle's EOS.

TEST INFRASTRUCTURE ONLY (used to derive workload parameters and by tests).

* ``admissibility``: the three conditions of App. B -- positive weights
  (c_s^2 inside the window of Sec. III), two-phase coexistence
  (psi < -1/rho somewhere) and positive bulk viscosity
  (psi < (2/d)/rho everywhere, Sec. VII).
* ``maxwell``: coexistence densities by the Maxwell construction of App. B
  (equal pressure and equal chemical potential, with the free energy per unit
  mass f obtained by integrating df/drho = p/rho^2 and normalised by
  f(rho1) = 0).
* ``kappa_for_width``: interfacial stiffness giving a planar tanh profile of a
  requested width.  Not from the paper: for the square-gradient free energy
  whose force is kappa rho grad lap rho (Sec. II), a planar interface obeys
  (kappa/2) rho'^2 = W(rho), W the excess grand-potential density; matching the
  peak slope of rho_bar + (drho/2) tanh(z/w) gives kappa = 8 w^2 W_max / drho^2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

from . import oracle

# Weight-positivity windows for c_s^2 printed in Sec. III and App. B.
WINDOW_2D = (0.3510760, 1.3333333)
WINDOW_3D = (0.3850612, 1.1917145)


def _eos1(m, rho):
    return oracle.eos(m, rho)[0]


def pressure(m, rho):
    return _eos1(m, rho)[1]


def cs2_range(m):
    """c_s^2 takes its extremes at rho1 (and outside (rho1, rho3)) and at rho2."""
    lo = m.cs2_1
    hi = m.cs2_1 * math.exp(2.0 * m.A * (m.rho2 - m.rho1) / math.pi)
    return min(lo, hi), max(lo, hi)


def admissibility(m, npts: int = 20001):
    """Return dict with the three App. B conditions and diagnostics."""
    d = m.dim
    rho3 = 2 * m.rho2 - m.rho1
    rr = np.linspace(m.rho1, rho3, npts)[1:-1]
    e = oracle.eos(m, rr)
    psi = e[:, 5]
    lo, hi = cs2_range(m)
    win = WINDOW_3D if d == 3 else WINDOW_2D
    return dict(
        weights_positive=(lo > win[0] and hi < win[1]),
        two_phase=bool(np.min(psi + 1.0 / rr) < 0.0),
        bulk_viscosity_positive=bool(np.max(rr * psi) < 2.0 / d),
        cs2_min=lo, cs2_max=hi, max_rho_psi=float(np.max(rr * psi)),
        min_psi_plus_inv_rho=float(np.min(psi + 1.0 / rr)),
    )


def free_energy_per_mass(m, rho):
    """f(rho) = int_{rho1}^{rho} p(r)/r^2 dr (App. B normalisation f(rho1)=0)."""
    rho3 = 2 * m.rho2 - m.rho1
    pts = [x for x in (m.rho1, m.rho2, rho3) if min(m.rho1, rho) < x < max(m.rho1, rho)]
    val, _ = integrate.quad(lambda r: pressure(m, r) / r**2, m.rho1, rho, points=pts or None,
                            epsabs=1e-14, epsrel=1e-13, limit=400)
    return val


def chemical_potential(m, rho):
    return free_energy_per_mass(m, rho) + pressure(m, rho) / rho


def spinodals(m):
    """Densities where dp/drho = 0 inside (rho2, rho3) (1 + rho psi = 0)."""
    rho3 = 2 * m.rho2 - m.rho1
    g = lambda r: 1.0 + r * _eos1(m, r)[5]
    rr = np.linspace(m.rho2, rho3, 4001)
    v = np.array([g(r) for r in rr])
    roots = []
    for k in range(len(rr) - 1):
        if v[k] == 0 or v[k] * v[k + 1] < 0:
            roots.append(optimize.brentq(g, rr[k], rr[k + 1], xtol=1e-15))
    return roots


def maxwell(m):
    """Coexistence densities (rho_g, rho_l) and pressure p_c."""
    sp = spinodals(m)
    if len(sp) < 2:
        raise ValueError("no two-phase region for this EOS")
    s1, s2 = sp[0], sp[-1]
    p_lo, p_hi = pressure(m, s2), pressure(m, s1)   # p decreases between spinodals

    def branches(pc):
        rg = optimize.brentq(lambda r: pressure(m, r) - pc, 1e-6, s1, xtol=1e-15)
        rl = optimize.brentq(lambda r: pressure(m, r) - pc, s2, 20.0, xtol=1e-15)
        return rg, rl

    def dmu(pc):
        rg, rl = branches(pc)
        return chemical_potential(m, rg) - chemical_potential(m, rl)

    eps = 1e-12 * abs(p_hi)
    pc = optimize.brentq(dmu, p_lo + eps, p_hi - eps, xtol=1e-15, rtol=1e-15)
    rg, rl = branches(pc)
    return rg, rl, pc


def excess_grand_potential(m, rho, rho_g, p_c):
    mu_c = chemical_potential(m, rho_g)
    return rho * free_energy_per_mass(m, rho) - mu_c * rho + p_c


def kappa_for_width(m, width: float = 3.0):
    rg, rl, pc = maxwell(m)
    res = optimize.minimize_scalar(lambda r: -excess_grand_potential(m, r, rg, pc),
                                   bounds=(rg, rl), method="bounded",
                                   options=dict(xatol=1e-12))
    wmax = -res.fun
    return 8.0 * width**2 * wmax / (rl - rg) ** 2, dict(rho_g=rg, rho_l=rl, p_c=pc, W_max=wmax)


def critical_amplitude(m):
    """Smallest A with psi(rho) = -1/rho solvable (mean-field critical point)."""
    rho3 = 2 * m.rho2 - m.rho1
    D = m.rho2 - m.rho1
    rr = np.linspace(m.rho2, rho3, 200001)[1:-1]
    # psi = A sin(pi (rho - rho1)/D) < 0 on (rho2, rho3): need A >= min(1/(rho |sin|))
    s = np.sin(np.pi * (rr - m.rho1) / D)
    return float(np.min(1.0 / (rr * np.abs(s))))


def max_amplitude(m):
    """Largest A with rho psi < 2/d on (rho1, rho2) (positive bulk viscosity)."""
    D = m.rho2 - m.rho1
    rr = np.linspace(m.rho1, m.rho2, 200001)[1:-1]
    s = np.sin(np.pi * (rr - m.rho1) / D)
    return float(np.min((2.0 / m.dim) / (rr * s)))
