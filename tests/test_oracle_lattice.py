"""Pins of the oracle's velocity sets, weights and equilibrium (Sec. III).

Every expected value here comes from the paper's statements, not from the
oracle: the moment conditions of Sec. III (eqs. tensor0_revised ...
tensor6_revised), the weight-positivity windows printed in Sec. III / App. B,
the projection of D3Q59 onto D2Q21 (Sec. III), and the moments of n_eq
(eqs. mass00 ... psi00).
"""
import itertools

import numpy as np
import pytest

SHELLS_3D = [1, 6, 12, 8, 6, 12, 8, 6]       # Table I, column b
SHELLS_2D = [1, 4, 4, 4, 4, 4]               # Table II, column b


def _moment(w, c, axes):
    return float(np.sum(w * np.prod(c[:, axes], axis=1))) if axes else float(np.sum(w))


@pytest.mark.parametrize("Q,sizes", [(59, SHELLS_3D), (21, SHELLS_2D)])
def test_shell_sizes(orc, Q, sizes):
    c, sh = orc.velocities(Q)
    assert len(c) == Q
    assert [int(np.sum(sh == k)) for k in range(len(sizes))] == sizes
    # distinct vectors, closed under reflection
    assert len({tuple(v) for v in c}) == Q
    assert {tuple(-v) for v in c} == {tuple(v) for v in c}
    assert np.abs(c).max() == 4


@pytest.mark.parametrize("Q", [59, 21])
@pytest.mark.parametrize("s", [0.36, 0.40, 0.45, 0.6, 0.9, 1.1])
def test_isotropy_to_sixth_rank(orc, Q, s):
    """sum w = 1, sum w c c = s d, 4th rank s^2 (dd+perm), 6th rank s^3 (ddd+perm)."""
    c, _ = orc.velocities(Q)
    c = c.astype(float)
    w = orc.weights(Q, s)
    d = 3 if Q == 59 else 2
    assert _moment(w, c, []) == pytest.approx(1.0, abs=1e-14)
    # Gaussian (Wick) moments: E[prod c_a] for isotropic Gaussian of variance s
    for order in range(1, 7):
        for axes in itertools.combinations_with_replacement(range(d), order):
            counts = [axes.count(a) for a in range(d)]
            if any(k % 2 for k in counts):
                expect = 0.0
            else:
                expect = 1.0
                for k in counts:
                    # (k-1)!! s^(k/2)
                    expect *= float(np.prod(np.arange(k - 1, 0, -2))) * s ** (k // 2)
            assert _moment(w, c, list(axes)) == pytest.approx(expect, abs=2e-14), (order, axes)


def _window(orc, Q):
    """Interval of sigma2 where every weight is positive, by bisection."""
    def minw(s):
        return orc.weights(Q, s).min()

    def root(lo, hi):
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if (minw(mid) > 0) == (minw(lo) > 0):
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)
    inside = 0.6
    assert minw(inside) > 0
    return root(inside, 0.2), root(inside, 2.0)


@pytest.mark.parametrize("Q,lo,hi", [(21, 0.3510760, 1.3333333), (59, 0.3850612, 1.1917145)])
def test_positivity_window_matches_printed_values(orc, Q, lo, hi):
    """Sec. III prints c_s,min^2 and c_s,max^2 to seven digits.  For D3Q59 the
    upper end is only reproduced with w0 fixed by the normalisation (the
    printed Table I w0 is inconsistent with it)."""
    a, b = _window(orc, Q)
    assert a == pytest.approx(lo, abs=6e-8)
    assert b == pytest.approx(hi, abs=6e-8)


@pytest.mark.parametrize("s", [0.4, 0.45, 0.6, 1.0])
def test_projection_3d_onto_2d(orc, s):
    """Sec. III: D2Q21 is D3Q59 projected onto a plane; summing the 3D weights
    over c_z gives the 2D weight of (c_x, c_y)."""
    c3, _ = orc.velocities(59)
    c2, _ = orc.velocities(21)
    w3 = orc.weights(59, s)
    w2 = orc.weights(21, s)
    proj = {}
    for v, w in zip(c3, w3):
        proj[(v[0], v[1])] = proj.get((v[0], v[1]), 0.0) + w
    assert len(proj) == 21
    for v, w in zip(c2, w2):
        assert proj[(v[0], v[1])] == pytest.approx(w, abs=1e-15)


@pytest.mark.parametrize("Q", [59, 21])
def test_equilibrium_moments(orc, Q):
    """eqs. mass00-psi00: moments of n_eq up to fourth order, with the local
    c_s^2 = p/rho of the EOS (App. B)."""
    d = 3 if Q == 59 else 2
    m = orc.Model(Q=Q, nx=4, ny=4, nz=4 if d == 3 else 1, A=0.8, rho1=0.3, rho2=1.0, cs2_1=0.42)
    rng = np.random.default_rng(7)
    c, _ = orc.velocities(Q)
    c = c.astype(float)[:, :d]
    I = np.eye(d)
    for _ in range(6):
        rho = rng.uniform(0.5, 2.0)
        u = rng.uniform(-0.1, 0.1, d)
        cs2 = orc.eos(m, rho)[0, 0]
        p = rho * cs2
        n = orc.equilibrium(m, rho, u)
        assert n.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(n @ c, rho * u, atol=1e-15)
        pi = np.einsum("i,ia,ib->ab", n, c, c)
        np.testing.assert_allclose(pi, p * I + rho * np.outer(u, u), atol=2e-15)
        phi = np.einsum("i,ia,ib,ig->abg", n, c, c, c)
        phi_ex = rho * cs2 * (np.einsum("ab,g->abg", I, u) + np.einsum("ag,b->abg", I, u)
                              + np.einsum("bg,a->abg", I, u))
        np.testing.assert_allclose(phi, phi_ex, atol=2e-15)
        psi = np.einsum("i,ia,ib,ig,id->abgd", n, c, c, c, c)
        uu = np.outer(u, u)
        psi_ex = (rho * cs2**2 * (np.einsum("ab,gd->abgd", I, I) + np.einsum("ag,bd->abgd", I, I)
                                  + np.einsum("ad,bg->abgd", I, I))
                  + rho * cs2 * (np.einsum("ab,gd->abgd", I, uu) + np.einsum("ag,bd->abgd", I, uu)
                                 + np.einsum("ad,bg->abgd", I, uu))
                  + rho * cs2 * (np.einsum("gd,ab->abgd", I, uu) + np.einsum("bd,ag->abgd", I, uu)
                                 + np.einsum("bg,ad->abgd", I, uu)))
        np.testing.assert_allclose(psi, psi_ex, atol=4e-15)
