"""Pins of the oracle's finite differences and implicit solve (Secs. IV, VI,
IX; Supplemental items 2-8).

* The force stencil (Sec. IV E) and the first-derivative stencil (Sec. IV B)
  are exact on polynomials of degree <= 4 (their Taylor conditions in Sec. IV),
  so on a periodic lattice they reproduce the continuum derivatives (sympy) at
  every site farther than the stencil radius from the periodic seam.
* The Laplacian and traceless second-derivative stencils (Secs. IV C, IV D)
  are exact on polynomials of degree <= 3 and not on quartics (their Taylor
  conditions leave the fourth-order term): second-order accurate.
* Sec. VI: the total lattice force vanishes on a periodic lattice.
* Sec. IX: the iteration solves a linear system; the iterate matches a dense
  direct solve built column by column from the one-pass map.
"""
import numpy as np
import pytest
import sympy as sp


def _poly_field(shape, expr, syms, shift):
    coords = np.meshgrid(*[np.arange(n, dtype=float) - shift for n in shape[::-1]], indexing="ij")[::-1]
    f = sp.lambdify(syms, expr, "numpy")
    v = f(*coords)
    return np.broadcast_to(v, coords[0].shape).ravel().astype(float)


def _interior(shape, r):
    coords = np.meshgrid(*[np.arange(n) for n in shape[::-1]], indexing="ij")[::-1]
    ok = np.ones(coords[0].shape, dtype=bool)
    for c, n in zip(coords, shape):
        ok &= (c >= r) & (c < n - r)
    return ok.ravel()


@pytest.mark.parametrize("Q,shape", [(21, (24, 20)), (59, (14, 12, 13))])
def test_force_exact_on_quartics(orc, Q, shape):
    d = len(shape)
    syms = sp.symbols("x y z")[:d]
    rng = np.random.default_rng(3)
    # random polynomial of total degree <= 4 around 1.4
    expr = sp.Float(1.4)
    for exps in __import__("itertools").product(range(5), repeat=d):
        if 0 < sum(exps) <= 4:
            expr += sp.Float(rng.uniform(-1, 1) * 10.0 ** (-1 - sum(exps))) * sp.Mul(
                *[s**e for s, e in zip(syms, exps)])
    shift = [n / 2 for n in shape]
    rho = _poly_field(shape, expr, syms, shift[0])  # same shift on all axes (centred box)
    kappa = 0.37
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, kappa=kappa)
    n = orc.init(m, rho, np.zeros((rho.size, d)))
    F = orc.fields(m, n)
    lap = sum(sp.diff(expr, s, 2) for s in syms)
    ok = _interior(shape, 2)
    for a, s in enumerate(syms):
        exact = kappa * rho * _poly_field(shape, sp.diff(lap, s), syms, shift[0])
        tol = 1e-10 * np.abs(exact).max()   # FP64 rounding of the 1.4 offset
        np.testing.assert_allclose(F["f"][ok, a], exact[ok], rtol=0, atol=tol)


@pytest.mark.parametrize("Q,shape", [(21, (16, 12)), (59, (9, 10, 11))])
def test_total_force_vanishes(orc, Q, shape):
    d = len(shape)
    rng = np.random.default_rng(5)
    rho = 1.3 + 0.2 * rng.uniform(-1, 1, int(np.prod(shape)))
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, kappa=0.5)
    F = orc.fields(m, orc.init(m, rho, np.zeros((rho.size, d))))
    assert np.abs(F["f"].sum(axis=0)).max() <= 1e-13 * np.abs(F["f"]).max() * rho.size
    assert np.abs(F["f"]).max() > 1e-3


@pytest.mark.parametrize("Q,shape", [(21, (26, 22)), (59, (16, 15, 14))])
def test_jtilde_map_exact_on_polynomial_velocity(orc, Q, shape):
    """Uniform rho: j~new_a = -(1/12) d_b [P1 d_ab div u + p (d_b u_a + d_a u_b)]
    with exact derivatives wherever the two nested stencils stay off the seam."""
    d = len(shape)
    syms = sp.symbols("x y z")[:d]
    rng = np.random.default_rng(9)
    us = []
    for a in range(d):
        e = sp.Float(0)
        for exps in __import__("itertools").product(range(5), repeat=d):
            if 0 < sum(exps) <= 4:
                e += sp.Float(rng.uniform(-1, 1) * 10.0 ** (-2 - sum(exps))) * sp.Mul(
                    *[s**k for s, k in zip(syms, exps)])
        us.append(e)
    rho0 = 1.35
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, A=0.8,
                  rho1=0.3, rho2=1.0, cs2_1=0.45)
    cs2, p, dp, P1, P2, psi = orc.eos(m, rho0)[0]
    shift = shape[0] / 2
    N = int(np.prod(shape))
    rho = np.full(N, rho0)
    u = np.zeros((N, 3))
    for a in range(d):
        u[:, a] = _poly_field(shape, us[a], syms, shift)
    j0p = rho[:, None] * u
    jt_new = orc.jtilde_map(m, rho, j0p, np.zeros((N, 3)))
    div = sum(sp.diff(us[b], syms[b]) for b in range(d))
    ok = _interior(shape, 4)
    for a in range(d):
        expr = 0
        for b in range(d):
            q_ab = (P1 * div if a == b else 0) + p * (sp.diff(us[a], syms[b]) + sp.diff(us[b], syms[a]))
            expr += sp.diff(q_ab, syms[b])
        exact = -_poly_field(shape, expr, syms, shift) / 12.0
        np.testing.assert_allclose(jt_new[ok, a], exact[ok], rtol=0, atol=1e-10 * np.abs(exact).max())


@pytest.mark.parametrize("Q,shape", [(21, (12, 10)), (59, (9, 9, 9))])
def test_jtilde_invariants(orc, Q, shape):
    """Uniform u gives j~ = 0; the map output sums to zero (a divergence)."""
    d = len(shape)
    N = int(np.prod(shape))
    rng = np.random.default_rng(2)
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, A=0.8, cs2_1=0.45)
    rho = 1.4 + 0.1 * rng.uniform(-1, 1, N)
    U = np.array([0.01, -0.02, 0.015 if d == 3 else 0.0])
    jt = orc.jtilde_map(m, rho, rho[:, None] * U[None, :], np.zeros((N, 3)))
    assert np.abs(jt).max() < 1e-16
    j0p = rng.uniform(-0.01, 0.01, (N, 3))
    if d == 2:
        j0p[:, 2] = 0
    jt = orc.jtilde_map(m, rho, j0p, np.zeros((N, 3)))
    assert np.abs(jt).max() > 1e-6
    assert np.abs(jt.sum(axis=0)).max() < 1e-15 * N


@pytest.mark.parametrize("Q,shape", [(21, (9, 9)), (59, (9, 9, 9))])
def test_iteration_matches_direct_solve(orc, Q, shape):
    """Items 3-8 converge to the solution of the linear system
    j~ = T(j0' + j~) (Sec. IX), T the one-pass map of items 3-5."""
    d = len(shape)
    N = int(np.prod(shape))
    rng = np.random.default_rng(4)
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, A=0.8,
                  rho1=0.3, rho2=1.0, cs2_1=0.45 if d == 2 else 0.39, kappa=0.05, tol=1e-15,
                  max_iter=5000)
    rho = 1.35 + 0.15 * rng.uniform(-1, 1, N)
    u = 0.01 * rng.uniform(-1, 1, (N, d))
    n = orc.init(m, rho, u)
    F = orc.fields(m, n)
    assert F["converged"]
    j0p = F["j0"] + 0.5 * F["f"]
    # T is linear in (j0' + j~): build its matrix on the d*N unknowns
    nun = d * N
    Tm = np.zeros((nun, nun))
    for k in range(nun):
        e = np.zeros((N, 3))
        e[k // d, k % d] = 1.0
        Tm[:, k] = orc.jtilde_map(m, F["rho"], e, np.zeros((N, 3)))[:, :d].ravel()
    rhs = Tm @ j0p[:, :d].ravel()
    jt_direct = np.linalg.solve(np.eye(nun) - Tm, rhs).reshape(N, d)
    scale = np.abs(jt_direct).max()
    assert np.abs(F["jt"][:, :d] - jt_direct).max() <= 1e-11 * scale
    # the spectral radius of T is below one here (the iteration converges)
    assert np.max(np.abs(np.linalg.eigvals(Tm))) < 1.0


def _poly(d, deg, rng, scale):
    syms = sp.symbols("x y z")[:d]
    e = sp.Float(0.7)
    for exps in __import__("itertools").product(range(deg + 1), repeat=d):
        if 0 < sum(exps) <= deg:
            e += sp.Float(rng.uniform(-1, 1) * scale ** sum(exps)) * sp.Mul(*[s**k for s, k in zip(syms, exps)])
    return syms, e


@pytest.mark.parametrize("Q,shape", [(21, (14, 12)), (59, (9, 10, 8))])
def test_second_derivative_stencils_exact_on_cubics(orc, Q, shape):
    """d_a d_b g from the Table III Laplacian + traceless stencils equals the
    exact Hessian of any cubic at every site one step off the seam, and
    misses that of a quartic by the fourth-order term."""
    d = len(shape)
    rng = np.random.default_rng(21)
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1)
    shift = shape[0] / 2
    ok = _interior(shape, 1)
    for deg, exact_expected in ((3, True), (4, False)):
        syms, e = _poly(d, deg, rng, 0.1)
        g = _poly_field(shape, e, syms, shift)
        H = orc.hessian(m, g)
        err = 0.0
        scale = 0.0
        for a in range(d):
            for b in range(d):
                ref = _poly_field(shape, sp.diff(e, syms[a], syms[b]), syms, shift)
                err = max(err, np.abs(H[ok, a, b] - ref[ok]).max())
                scale = max(scale, np.abs(ref[ok]).max())
        if exact_expected:
            assert err <= 1e-12 * max(scale, 1.0), (deg, err)
        else:
            assert err > 1e-6 * scale, (deg, err)
