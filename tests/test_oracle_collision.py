"""Pins of the oracle's collision operators and of whole steps.

Per-site moment identities (exact): Sec. V (momentum transfer), Sec. VI
(Delta^int: mass-neutral, first moment (1+gamma)/2 h f, second moment zero,
third moment (1+gamma)/2 h c0^2 (f d + perm)), Sec. VIII (Delta^corr: mass 0,
first moment (gamma-1) j~, second moment Sigma, third moment
Xi = Xi' + (gamma-1) c0^2 (d j~ + perm)).

Lattice invariants: mass and total momentum are conserved (Sec. VI); a
uniform state (rest or moving) is a fixed point whose second moment is the
Euler stress p(rho) d + rho u u with the prescribed EOS (Sec. III).

Textbook limit: A = 0, kappa = 0, no correction is lattice BGK with
c_s^2 = c_s^2(rho1); a shear wave decays with nu = c_s^2 (1+gamma)/(2(1-gamma))
(Sec. VII: eta = (h/2)(1+gamma)/(1-gamma) p), up to O(k^2) lattice terms.
"""
import numpy as np
import pytest


def _sym_random(rng, d, scale):
    S = rng.uniform(-scale, scale, (3, 3))
    S = 0.5 * (S + S.T)
    S[d:, :] = 0
    S[:, d:] = 0
    return S


def _sym3_random(rng, d, scale):
    import itertools
    X = np.zeros((3, 3, 3))
    for a, b, c in itertools.combinations_with_replacement(range(d), 3):
        v = rng.uniform(-scale, scale)
        for p in set(itertools.permutations((a, b, c))):
            X[p] = v
    return X


@pytest.mark.parametrize("Q", [21, 59])
@pytest.mark.parametrize("gamma", [-0.5, 0.0, 0.6])
def test_collision_moments(orc, Q, gamma):
    d = 3 if Q == 59 else 2
    m = orc.Model(Q=Q, nx=8, ny=8, nz=8 if d == 3 else 1, gamma=gamma, A=0.8, rho1=0.3, rho2=1.0,
                  cs2_1=0.42, rho0=0.3)
    c0sq = orc.eos(m, m.rho0)[0, 0]
    c, _ = orc.velocities(Q)
    c = c.astype(float)
    I = np.eye(3)
    I[d:, d:] = 0
    rng = np.random.default_rng(21)
    for _ in range(5):
        rho = rng.uniform(1.1, 1.7)
        f = np.zeros(3); f[:d] = rng.uniform(-1e-2, 1e-2, d)
        jt = np.zeros(3); jt[:d] = rng.uniform(-1e-3, 1e-3, d)
        u = np.zeros(3); u[:d] = rng.uniform(-0.05, 0.05, d)
        Sig = _sym_random(rng, d, 1e-3)
        Xip = _sym3_random(rng, d, 1e-3)
        # pre-collision populations whose j0 makes u the hydrodynamic velocity:
        # j = j0 + f/2 + j~ (Sec. V)
        n = orc.equilibrium(m, rho, u[:d]) + rng.uniform(-1e-4, 1e-4, Q)
        n -= n.mean() - orc.equilibrium(m, rho, u[:d]).mean()       # keep sum n = rho
        j0 = n @ c
        u_h = (j0 + 0.5 * f + jt) / rho
        db, di, dc = orc.site_collision(m, n, rho, u_h, f, jt, Sig, Xip)
        # Delta^int (Sec. VI)
        assert abs(di.sum()) < 1e-16
        np.testing.assert_allclose(di @ c, 0.5 * (1 + gamma) * f, atol=1e-15)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", di, c, c), 0, atol=1e-15)
        third = 0.5 * (1 + gamma) * c0sq * (np.einsum("a,bg->abg", f, I) + np.einsum("b,ag->abg", f, I)
                                            + np.einsum("g,ab->abg", f, I))
        np.testing.assert_allclose(np.einsum("i,ia,ib,ig->abg", di, c, c, c), third, atol=1e-15)
        # Delta^corr (Sec. VIII)
        assert abs(dc.sum()) < 1e-16
        np.testing.assert_allclose(dc @ c, (gamma - 1) * jt, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", dc, c, c), Sig, atol=1e-16)
        Xi = Xip + (gamma - 1) * c0sq * (np.einsum("g,ab->abg", jt, I) + np.einsum("b,ag->abg", jt, I)
                                         + np.einsum("a,bg->abg", jt, I))
        np.testing.assert_allclose(np.einsum("i,ia,ib,ig->abg", dc, c, c, c), Xi, atol=1e-16)
        # Delta^bulk is mass-neutral; total momentum transfer is h f (Sec. V)
        assert abs(db.sum()) < 1e-15
        np.testing.assert_allclose((db + di + dc) @ c, f, atol=1e-15)


@pytest.mark.parametrize("Q,shape", [(21, (24, 20)), (59, (12, 10, 9))])
def test_mass_and_momentum_conserved(orc, Q, shape):
    d = len(shape)
    N = int(np.prod(shape))
    rng = np.random.default_rng(31)
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, gamma=0.0,
                  kappa=0.16 if d == 2 else 0.0124, A=0.8 if d == 2 else 0.745, rho1=0.3, rho2=1.0,
                  cs2_1=0.45 if d == 2 else 0.39, rho0=0.3, tol=1e-14, max_iter=3000)
    rho = 1.38 + 0.05 * rng.uniform(-1, 1, N)
    u = 0.003 * rng.uniform(-1, 1, (N, d))
    n = orc.init(m, rho, u)
    M0, P0 = orc.totals(m, n)
    orc.step(m, n, 5)
    M1, P1 = orc.totals(m, n)
    assert abs(M1 - M0) <= 1e-13 * M0
    assert np.abs(P1 - P0).max() <= 1e-13 * M0


@pytest.mark.parametrize("Q,shape", [(21, (10, 9)), (59, (9, 9, 9))])
@pytest.mark.parametrize("moving", [False, True])
def test_uniform_state_is_fixed_point(orc, Q, shape, moving):
    d = len(shape)
    N = int(np.prod(shape))
    m = orc.Model(Q=Q, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, gamma=0.3,
                  kappa=0.2, A=0.8, rho1=0.3, rho2=1.0, cs2_1=0.45 if d == 2 else 0.42, rho0=0.3)
    rho0 = 1.42
    U = np.array([0.03, -0.02, 0.01])[:d] if moving else np.zeros(d)
    n = orc.init(m, np.full(N, rho0), np.tile(U, (N, 1)))
    n_start = n.copy()
    orc.step(m, n, 3)
    np.testing.assert_allclose(n, n_start, rtol=0, atol=1e-15)
    # second moment = Euler stress with the prescribed EOS
    c, _ = orc.velocities(Q)
    c = c.astype(float)[:, :d]
    p = orc.eos(m, rho0)[0, 1]
    Pi = np.einsum("i,ia,ib->ab", n[:, 0], c, c)
    np.testing.assert_allclose(Pi, p * np.eye(d) + rho0 * np.outer(U, U), atol=1e-15)


def _shear_rate(orc, gamma, ny, cs2=0.45, nx=8, steps=20, blocks=4):
    m = orc.Model(Q=21, nx=nx, ny=ny, gamma=gamma, A=0.0, cs2_1=cs2, rho0=0.3, flags=orc.NO_CORR)
    N = nx * ny
    y = (np.arange(N) // nx).astype(float)
    k = 2 * np.pi / ny
    u = np.zeros((N, 2))
    u[:, 0] = 1e-6 * np.sin(k * y)
    n = orc.init(m, np.ones(N), u)
    amps = []
    for _ in range(blocks):
        orc.step(m, n, steps)
        F = orc.fields(m, n)
        amps.append(2 * np.mean(F["u"][:, 0] * np.sin(k * y)))
    return -np.mean(np.diff(np.log(amps))) / steps / k**2


@pytest.mark.parametrize("gamma", [-0.4, 0.0, 0.4])
def test_bgk_shear_wave_viscosity(orc, gamma):
    """Ideal gas, no force, no correction: u_x = U sin(k y) decays as
    exp(-nu k^2 t), nu = c_s^2 (1+gamma)/(2(1-gamma)) (Sec. VII), up to a
    relative O(k^2) lattice term removed by Richardson extrapolation."""
    cs2 = 0.45
    nu_k = _shear_rate(orc, gamma, 32, cs2)
    nu_k2 = _shear_rate(orc, gamma, 64, cs2)
    nu0 = (4 * nu_k2 - nu_k) / 3
    nu = cs2 * (1 + gamma) / (2 * (1 - gamma))
    assert nu0 == pytest.approx(nu, rel=2e-4)
