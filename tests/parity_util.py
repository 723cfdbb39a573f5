"""Helpers shared by the GPU parity tests and the smoke check: run the same
seeded input through the HIP library and the FP64 oracle and compare.

Error measure (per field): max_r |G - O| / max_r |O| over every component.
"""
from __future__ import annotations

import numpy as np

import lb2p_workloads as W

# 3D component order of the library: Sigma xx yy zz xy xz yz,
# Xi' xxx yyy zzz xxy xxz xyy xzz yyz yzz xyz ; 2D: xx yy xy / xxx yyy xxy xyy.
SIG3 = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
SIG2 = [(0, 0), (1, 1), (0, 1)]
XI3 = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 2, 2), (1, 1, 2),
       (1, 2, 2), (0, 1, 2)]
XI2 = [(0, 0, 0), (1, 1, 1), (0, 0, 1), (0, 1, 1)]


def rel_err(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    scale = np.max(np.abs(o))
    if scale == 0.0:
        return float(np.max(np.abs(g)))
    return float(np.max(np.abs(g - o)) / scale)


def oracle_sigma_components(Sig, d):
    idx = SIG3 if d == 3 else SIG2
    return np.stack([Sig[:, a, b] for a, b in idx])


def oracle_xi_components(Xi, d):
    idx = XI3 if d == 3 else XI2
    return np.stack([Xi[:, a, b, c] for a, b, c in idx])


def match_populations(c_lib, c_orc):
    """Permutation p with c_orc[p[i]] == c_lib[i]."""
    lut = {tuple(v): k for k, v in enumerate(np.asarray(c_orc))}
    return np.array([lut[tuple(v)] for v in np.asarray(c_lib)])


# Linearly stable parameter sets (uniform-state spectral radius 1 at both
# coexistence densities): 2D A=0.8, c_s^2(rho1)=0.45, kappa for width 3;
# 3D near the critical point, A=0.745, c_s^2(rho1)=0.39, kappa for width 2.
STABLE = {21: dict(A=0.8, cs2_1=0.45, kappa=0.1594, rg=1.2285, rl=1.5454),
          59: dict(A=0.745, cs2_1=0.39, kappa=0.0124, rg=1.3127, rl=1.4589)}


def small_case(lattice, shape, seed=11, gamma=0.0, u_amp=1e-3):
    """A droplet with noise and a random velocity field (all terms non-zero)."""
    d = len(shape)
    st = STABLE[lattice]
    A, cs2_1, kappa, rg, rl = st["A"], st["cs2_1"], st["kappa"], st["rg"], st["rl"]
    rho, u = W.droplet(shape, radius=0.3 * min(shape), rho_g=rg, rho_l=rl, width=2.0,
                       noise=1e-3, seed=seed)
    rng = np.random.default_rng(seed + 1)
    u = rng.uniform(-u_amp, u_amp, size=(d, rho.size))
    model = dict(Q=lattice, nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, gamma=gamma,
                 kappa=kappa, rho1=0.3, rho2=1.0, A=A, cs2_1=cs2_1, rho0=0.3)
    return rho, u, model


def oracle_reference(orc, model, rho, u, nsteps_long=10, tol=1e-14):
    """Oracle fields at t=0, the closure of t=0, populations at t=1 and
    (rho, u) at t=nsteps_long."""
    m = orc.Model(**model, tol=tol, max_iter=2000)
    d = m.dim
    n0 = orc.init(m, rho, u.T.copy())
    F0 = orc.fields(m, n0)
    j = F0["rho"][:, None] * F0["u"]
    Sig, Xi = orc.closure(m, F0["rho"], j, F0["jt"])
    n1 = n0.copy()
    orc.step(m, n1, 1)
    nL = n1.copy()
    if nsteps_long > 1:
        orc.step(m, nL, nsteps_long - 1)
    FL = orc.fields(m, nL)
    return dict(m=m, d=d, F0=F0, Sig=oracle_sigma_components(Sig, d),
                Xi=oracle_xi_components(Xi, d), n1=n1, FL=FL)


def gpu_run(L, model, storage, rho, u, nsteps_long=10, tol=None, **extra):
    d = 3 if model["Q"] == 59 else 2
    P = L.Params(lattice=model["Q"], nx=model["nx"], ny=model["ny"], nz=model["nz"],
                 storage=storage, gamma=model["gamma"], kappa=model["kappa"], rho1=model["rho1"],
                 rho2=model["rho2"], A=model["A"], cs2_rho1=model["cs2_1"], rho0=model["rho0"],
                 tol=tol, max_iter=2000, **extra)
    out = {}
    with L.Context(P) as ctx:
        ctx.init(np.ascontiguousarray(rho, dtype=np.float64), np.ascontiguousarray(u, dtype=np.float64))
        out["n0"] = ctx.populations()
        r0, u0 = ctx.moments()
        out["rho0"], out["u0"] = r0, u0
        out["j00"] = ctx.field(L.FIELD_J0)
        out["f0"] = ctx.field(L.FIELD_FORCE)
        out["jt0"] = ctx.field(L.FIELD_JTILDE)
        out["stats0"] = ctx.stats()
        ctx.step(1)
        out["Sig0"] = ctx.field(L.FIELD_SIGMA)
        out["Xi0"] = ctx.field(L.FIELD_XI)
        out["n1"] = ctx.populations()
        out["stats1"] = ctx.stats()
        if nsteps_long > 1:
            ctx.step(nsteps_long - 1)
        rL, uL = ctx.moments()
        out["rhoL"], out["uL"] = rL, uL
        out["statsL"] = ctx.stats()
    out["c"] = L.velocities(model["Q"])
    return out


def compare(orc, ref, gpu):
    """Dict of relative errors for every compared quantity."""
    d = ref["d"]
    c_orc, _ = orc.velocities(ref["m"].Q)
    perm = match_populations(gpu["c"], c_orc)
    F0, FL = ref["F0"], ref["FL"]
    e = {}
    e["rho_t0"] = rel_err(gpu["rho0"], F0["rho"])
    e["u_t0"] = rel_err(gpu["u0"], F0["u"][:, :d].T)
    e["j0_t0"] = rel_err(gpu["j00"], F0["j0"][:, :d].T)
    e["force_t0"] = rel_err(gpu["f0"], F0["f"][:, :d].T)
    e["jtilde_t0"] = rel_err(gpu["jt0"], F0["jt"][:, :d].T)
    e["sigma_t0"] = rel_err(gpu["Sig0"], ref["Sig"])
    e["xi_t0"] = rel_err(gpu["Xi0"], ref["Xi"])
    e["pop_t1"] = rel_err(gpu["n1"], ref["n1"][perm])
    e["rho_tL"] = rel_err(gpu["rhoL"], FL["rho"])
    e["u_tL"] = rel_err(gpu["uL"], FL["u"][:, :d].T)
    return e
