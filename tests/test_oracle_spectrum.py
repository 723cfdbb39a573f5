"""The spectrum of the j~ map's linear part (Sec. IX), which the Chebyshev
solver relies on.

With j0' = 0 the map G of items 3-5 is linear: G = (1/12) D^T C D R, where
D is the first-derivative stencil (Sec. IV B) as a gradient, C the per-site
map G -> P1 tr(G) I + p (G + G^T) and R = diag(1/rho).  D^T C D is symmetric
and, when the bulk viscosity is positive (App. B), positive semi-definite,
so G is similar to a symmetric PSD operator: its eigenvalues are real and
non-negative.  The plane-wave bound b = 1.05 |s|^2_max/12 * max c_s^2 (2 -
rho psi) (written out here independently of the library) must not be
exceeded.  The dense matrix is built column by column from the oracle's
own map on small grids.
"""
import numpy as np
import pytest

import lb2p_workloads as W


def _bound(model, dim):
    k = np.linspace(0.0, np.pi, 4001)
    smax = np.max(((4.0 / 3.0) * np.sin(k) - (1.0 / 6.0) * np.sin(2 * k)) ** 2)
    e = model["eos"]
    r1, r2, A, c1 = e["rho1"], e["rho2"], e["A"], e["cs2_1"]
    r3, dl = 2 * r2 - r1, r2 - r1
    r = np.linspace(r1, r3, 4001)
    inside = (r > r1) & (r < r3)
    th = np.pi * (r - r1) / dl
    psi = np.where(inside, A * np.sin(th), 0.0)
    cs2 = np.where(inside, c1 * np.exp(A * dl / np.pi * (1 - np.cos(th))), c1)
    return 1.05 * dim * smax * np.max(cs2 * np.maximum(2 - r * psi, 1.0)) / 12.0


@pytest.mark.parametrize("name,shape", [("d2q21_64_droplet", (12, 10)), ("d3q59_256_slab", (6, 6, 8))])
@pytest.mark.parametrize("field", ["droplet", "random"])
def test_map_spectrum_real_nonnegative_and_bounded(orc, name, shape, field):
    entry = W.load_params()[name]
    model = entry["model"]
    d = len(shape)
    m = orc.Model(nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, **W.oracle_kwargs(model))
    N = m.N
    if field == "droplet":
        rho, _ = W.droplet(shape, radius=0.3 * min(shape), rho_g=model["rho_g"], rho_l=model["rho_l"],
                           width=1.5, noise=0.0)
    else:
        rho = np.random.default_rng(3).uniform(model["rho_g"], model["rho_l"], N)
    M = np.zeros((N * d, N * d))
    zero = np.zeros((N, 3))
    for col in range(N * d):
        e = np.zeros((N, 3))
        e[col // d, col % d] = 1.0
        M[:, col] = orc.jtilde_map(m, rho, zero, e)[:, :d].ravel()
    ev = np.linalg.eigvals(M)
    lam = float(np.max(ev.real))
    b = _bound(model, d)
    print(name, field, f"lambda_max {lam:.4f} bound {b:.4f} min {ev.real.min():.2e}", flush=True)
    assert np.max(np.abs(ev.imag)) <= 1e-9 * lam
    assert ev.real.min() >= -1e-12 * lam
    assert lam <= b
    assert lam >= 0.5 * b     # the bound is not vacuous on these states


def _symbol(shape):
    """|s(k)|^2 of the first-derivative stencil (Sec. IV B) at every wave
    vector of a periodic grid."""
    tot = 0.0
    for a, n in enumerate(shape):
        k = 2.0 * np.pi * np.arange(n) / n
        s2 = ((4.0 / 3.0) * np.sin(k) - (1.0 / 6.0) * np.sin(2.0 * k)) ** 2
        tot = np.add.outer(tot, s2) if a else s2
    return np.asarray(tot).ravel()


def test_uniform_state_spectrum_is_the_plane_wave_symbol(orc):
    """On a uniform density the map's linear part is diagonal in plane waves:
    per wave vector the transverse velocities have c_s^2 |s|^2 / 12 and the
    longitudinal one c_s^2 (2 - rho psi) |s|^2 / 12.  These are the
    eigenvalues whose largest value sets the iteration's convergence, and
    whose continuity in k makes the implicit system singular on large grids
    once that largest value exceeds 1."""
    model = W.load_params()["d3q59_256_slab"]["model"]
    shape = (6, 6, 8)
    m = orc.Model(nx=shape[0], ny=shape[1], nz=shape[2], **W.oracle_kwargs(model))
    N, d = m.N, 3
    r0 = 1.279
    rho = np.full(N, r0)
    M = np.zeros((N * d, N * d))
    zero = np.zeros((N, 3))
    for col in range(N * d):
        e = np.zeros((N, 3))
        e[col // d, col % d] = 1.0
        M[:, col] = orc.jtilde_map(m, rho, zero, e)[:, :d].ravel()
    ev = np.sort(np.linalg.eigvals(M).real)
    cs2, psi = orc.eos(m, r0)[0][[0, 5]]
    s2 = _symbol(shape)
    pred = np.sort(np.concatenate([cs2 * s2 / 12.0, cs2 * s2 / 12.0, cs2 * (2.0 - r0 * psi) * s2 / 12.0]))
    assert np.abs(ev - pred).max() <= 1e-12 * pred.max()


def test_unit_crossing_makes_the_implicit_system_ill_conditioned():
    """Beyond a largest eigenvalue of 1 no solver helps: the plane-wave
    eigenvalues c_s^2 (2 - rho psi) |s(k)|^2 / 12 fill [0, lambda_max]
    continuously, so on a growing grid some 1 - lambda(k) approaches 0 and
    the correction current j~ = (I - M)^-1 c amplifies that mode without
    bound.  Below 1 the amplification stays bounded by 1/(1 - lambda_max)."""
    def worst(g, L):
        lam = _symbol((L, L, L)) * g / 12.0
        return 1.0 / np.abs(1.0 - lam).min()
    g_over = 12.0 * 1.14 / (3 * 1.8829929668)     # lambda_max = 1.14
    g_under = 12.0 * 0.66 / (3 * 1.8829929668)    # the 3D workloads' 0.66
    amp_over = [worst(g_over, L) for L in (16, 64, 256)]
    amp_under = [worst(g_under, L) for L in (16, 64, 256)]
    assert amp_over[-1] > 1e4 and amp_over[-1] > 100 * amp_over[0]
    assert max(amp_under) <= 1.0 / (1.0 - 0.66) * (1 + 1e-9)
