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
