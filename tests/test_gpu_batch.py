"""GPU checks of batched contexts (several independent lattices advanced by
one set of launches), HIP-graph replay and the block-shape autotuner.

A batched context must give every domain exactly what a context of that
domain alone gives (each domain has its own constants, periodic wrap and
stop rule of Sec. IX), and that in turn matches the FP64 oracle.
"""
import numpy as np
import pytest

import lb2p_workloads as W
from parity_util import match_populations, rel_err, small_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1402_2920_amd import lb2p
    lb2p.lib()
    return lb2p


def _params(L, model, storage, **extra):
    kw = dict(max_iter=2000)
    kw.update(extra)
    return L.Params(lattice=model["Q"], nx=model["nx"], ny=model["ny"], nz=model["nz"], storage=storage,
                    gamma=model["gamma"], kappa=model["kappa"], rho1=model["rho1"], rho2=model["rho2"],
                    A=model["A"], cs2_rho1=model["cs2_1"], rho0=model["rho0"], **kw)


def _domains_3d():
    """Three 3D domains of different sizes and constants (gamma, kappa)."""
    out = []
    for shape, seed, gamma, kappa in (((20, 12, 10), 21, 0.0, 0.0124), ((16, 16, 12), 22, 0.2, 0.008),
                                      ((40, 24, 36), 23, -0.1, 0.0124)):
        rho, u, m = small_case(59, shape, seed=seed, gamma=gamma)
        m["kappa"] = kappa
        out.append((m, rho, u))
    return out


def _domains_2d(n=4):
    out = []
    for ent, shape, rho, u in W.build_batch("d2q21_batch512", n):
        m = dict(Q=21, nx=shape[0], ny=shape[1], nz=1, gamma=ent["gamma"], kappa=ent["kappa"],
                 rho1=ent["eos"]["rho1"], rho2=ent["eos"]["rho2"], A=ent["eos"]["A"],
                 cs2_1=ent["eos"]["cs2_1"], rho0=ent["rho0"])
        rng = np.random.default_rng(ent["seed"] + 7)
        u = rng.uniform(-1e-3, 1e-3, size=u.shape)
        out.append((m, rho, u))
    return out


def _run_batch(L, doms, storage, nsteps, **extra):
    plist = [_params(L, m, storage, **extra) for m, _, _ in doms]
    rho = np.concatenate([r for _, r, _ in doms])
    u = np.concatenate([uu for _, _, uu in doms], axis=1)
    with L.Context(plist) as ctx:
        ctx.init(rho, np.ascontiguousarray(u))
        tot0 = ctx.domain_totals()
        ctx.step(nsteps)
        n = ctx.populations()
        r, uu = ctx.moments()
        tot = ctx.domain_totals()
        st = ctx.stats()
        off = ctx.offsets
    return [dict(n=n[:, off[k]:off[k + 1]], rho=r[off[k]:off[k + 1]], u=uu[:, off[k]:off[k + 1]],
                 tot0=tot0[k], tot=tot[k]) for k in range(len(doms))], st


def _run_single(L, m, rho, u, storage, nsteps, **extra):
    with L.Context(_params(L, m, storage, **extra)) as ctx:
        ctx.init(rho, np.ascontiguousarray(u))
        ctx.step(nsteps)
        n = ctx.populations()
        r, uu = ctx.moments()
        return dict(n=n, rho=r, u=uu, iters=ctx.stats()["iters"])


@pytest.mark.parametrize("flags", [0, 2])   # 2: the stencil formulation of items 10-11
@pytest.mark.parametrize("dim", [2, 3])
def test_batch_matches_oracle_per_domain(orc, L, dim, flags):
    doms = _domains_2d() if dim == 2 else _domains_3d()
    nsteps = 4
    res, _ = _run_batch(L, doms, L.STORE_F64, nsteps, tol=1e-14, flags=flags)
    c_lib = L.velocities(doms[0][0]["Q"])
    for k, (m, rho, u) in enumerate(doms):
        om = orc.Model(**m, tol=1e-14, max_iter=2000, flags=flags)
        n = orc.init(om, rho, u.T.copy())
        orc.step(om, n, nsteps)
        F = orc.fields(om, n)
        perm = match_populations(c_lib, orc.velocities(m["Q"])[0])
        e = dict(pop=rel_err(res[k]["n"], n[perm]), rho=rel_err(res[k]["rho"], F["rho"]),
                 u=rel_err(res[k]["u"], F["u"][:, :dim].T))
        print("domain", k, (m["nx"], m["ny"], m["nz"]), {a: f"{b:.2e}" for a, b in e.items()}, flush=True)
        for name, v in e.items():
            assert v <= 1e-10, (k, name, v)
        # per-domain conservation (FP64 sums)
        assert abs(res[k]["tot"][0] - res[k]["tot0"][0]) <= 1e-13 * res[k]["tot0"][0]
        assert np.max(np.abs(res[k]["tot"][1:] - res[k]["tot0"][1:])) <= 1e-13 * res[k]["tot0"][0]


@pytest.mark.parametrize("storage", ["STORE_F64", "STORE_F32", "STORE_BF16"])
def test_batch_equals_single_domain_contexts(L, storage):
    """Bit-identical to running each domain in a context of its own (same
    kernels, same per-site arithmetic, per-domain stop rule)."""
    st = getattr(L, storage)
    doms = _domains_3d()
    tol = 1e-14 if st == L.STORE_F64 else 1e-6
    res, stats = _run_batch(L, doms, st, 3, tol=tol)
    iters = []
    for k, (m, rho, u) in enumerate(doms):
        one = _run_single(L, m, rho, u, st, 3, tol=tol)
        iters.append(one["iters"])
        for name in ("n", "rho", "u"):
            d = np.max(np.abs(res[k][name] - one[name]))
            assert d == 0.0, (k, name, d)
    assert stats["iters"] == max(iters)


@pytest.mark.parametrize("lattice,shape", [(21, (40, 24)), (59, (40, 24, 36))])
def test_graph_replay_equals_eager(L, lattice, shape):
    """Steps replayed from a captured HIP graph (fixed iteration count) give
    exactly the eager result, for both buffer parities and a remainder."""
    rho, u, m = small_case(lattice, shape)
    outs = []
    for gs in (0, 4):
        with L.Context(_params(L, m, L.STORE_F32, fixed_iter=6, graph_steps=gs)) as ctx:
            ctx.init(rho, np.ascontiguousarray(u))
            ctx.step(6)   # eager (no previous j~) + one replay + eager: parity even
            ctx.step(9)   # two replays + one eager step
            ctx.step(4)   # one replay
            outs.append(ctx.populations())
    assert np.isfinite(outs[0]).all()
    assert np.array_equal(outs[0], outs[1])


def test_autotune_keeps_state_and_results(L):
    rho, u, m = small_case(59, (40, 24, 36))
    P = _params(L, m, L.STORE_F32, tol=1e-6)
    with L.Context(P) as a, L.Context(P) as b:
        a.init(rho, np.ascontiguousarray(u))
        b.init(rho, np.ascontiguousarray(u))
        n_before = a.populations()
        a.autotune(2)
        assert np.array_equal(a.populations(), n_before)
        a.step(3)
        b.step(3)
        na, nb = a.populations(), b.populations()
    assert np.array_equal(na, nb), np.max(np.abs(na - nb))



def test_site_tilings_give_identical_results(L):
    """The site kernels' block shape and the solve pass's chunk length
    change which thread handles a site, not what it computes: plane patches,
    linear tiles of 256 consecutive sites and 8- or 32-plane chunks
    (lb2p_set_tiling) give the same populations to the bit, for a 3D domain
    and for a batch of narrow 2D domains; other shapes are refused."""
    rho, u, m = small_case(59, (40, 24, 36))
    P = _params(L, m, L.STORE_F32, tol=1e-6)
    doms = _domains_2d(8)
    plist = [_params(L, mm, L.STORE_F32, tol=1e-6) for mm, _, _ in doms]
    rho2 = np.concatenate([r for _, r, _ in doms])
    u2 = np.ascontiguousarray(np.concatenate([uu for _, _, uu in doms], axis=1))
    for params, r_, u_ in ((P, rho, np.ascontiguousarray(u)), (plist, rho2, u2)):
        outs = []
        # (bx, by, solve-pass chunk planes)
        for shape in ((64, 4, 32), (256, 0, 32), (32, 8, 32), (64, 4, 8)):
            with L.Context(params) as ctx:
                ctx.set_tiling(*shape)
                ctx.init(r_, u_)
                ctx.step(3)
                outs.append(ctx.populations())
        assert all(np.array_equal(outs[0], o) for o in outs[1:])
    with L.Context(P) as ctx:
        for bad in ((128, 4, 32), (256, 1, 0), (255, 0, 32), (0, 256, 32)):
            assert L.lib().lb2p_set_tiling(ctx._ctx, *bad) == L.EINVAL, bad


@pytest.mark.parametrize("storage,bound", [("STORE_F32", 1e-9), ("STORE_BF16", 1e-6)])
def test_batch_reduced_storage_conserves_mass(L, storage, bound):
    """FP32/BF16 storage: the rest population carries the site's mass balance
    at higher precision, so each domain's mass stays put over a graph-replayed
    run (a systematic rounding of the populations would drift it by about
    1e-8 per step)."""
    doms = _domains_2d(8)
    plist = [_params(L, m, getattr(L, storage), fixed_iter=6, graph_steps=100) for m, _, _ in doms]
    rho = np.concatenate([r for _, r, _ in doms])
    u = np.ascontiguousarray(np.concatenate([uu for _, _, uu in doms], axis=1))
    with L.Context(plist) as ctx:
        ctx.init(rho, u)
        t0 = ctx.domain_totals()
        ctx.step(301)
        t1 = ctx.domain_totals()
        assert not ctx.stats()["nonfinite"]
    dm = np.abs(t1[:, 0] - t0[:, 0]) / t0[:, 0]
    print(storage, "per-domain relative mass drift over 301 steps: max", f"{dm.max():.2e}", flush=True)
    assert dm.max() <= bound


def test_domain_solve_reports_each_domains_stop_rule(L):
    """lb2p_domain_solve: the stop rule of Sec. IX holds per domain of a
    batch.  In tolerance mode each domain's last residual meets its own rule,
    resid <= tol * max|j0'| of that domain; with a fixed pass count every
    domain reports that count; with max_iter 1 and a tolerance no pass can
    meet, every domain reports that its rule did not hold."""
    doms = _domains_2d()
    rho = np.concatenate([r for _, r, _ in doms])
    u = np.concatenate([uu for _, _, uu in doms], axis=1)
    tol = 1e-10
    with L.Context([_params(L, m, L.STORE_F64, tol=tol) for m, _, _ in doms]) as ctx:
        with pytest.raises(L.Lb2pError):
            ctx.domain_solve()          # no solve since init
        ctx.init(rho, np.ascontiguousarray(u))
        ctx.step(3)
        ds = ctx.domain_solve()
        assert ds["converged"].all() and (ds["iters"] >= 1).all()
        assert np.all(ds["resid"] <= tol * ds["jscale"]), (ds["resid"], ds["jscale"])
        assert np.all(ds["jscale"] > 0)
    with L.Context([_params(L, m, L.STORE_F64, fixed_iter=5) for m, _, _ in doms]) as ctx:
        ctx.init(rho, np.ascontiguousarray(u))
        ctx.step(2)
        ds = ctx.domain_solve()
        assert (ds["iters"] == 5).all() and ds["converged"].all()
    with L.Context([_params(L, m, L.STORE_F64, tol=1e-30, max_iter=1) for m, _, _ in doms]) as ctx:
        ctx.init(rho, np.ascontiguousarray(u))
        ctx.step(1, allow=(L.ENOCONV,))
        ds = ctx.domain_solve()
        assert (ds["iters"] == 1).all() and not ds["converged"].any()
        assert np.all(ds["resid"] > 0)
