"""C-ABI entry points without a test elsewhere: lb2p_set_populations (a
state handed in from outside, then advanced) and the diagnostic profiler
(lb2p_profile_enable / lb2p_profile_read / lb2p_profile_classes)."""
import numpy as np
import pytest

from parity_util import match_populations, rel_err, small_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1402_2920_amd import lb2p
    lb2p.lib()
    return lb2p


def _params(L, model, storage, **kw):
    return L.Params(lattice=model["Q"], nx=model["nx"], ny=model["ny"], nz=model["nz"], storage=storage,
                    gamma=model["gamma"], kappa=model["kappa"], rho1=model["rho1"], rho2=model["rho2"],
                    A=model["A"], cs2_rho1=model["cs2_1"], rho0=model["rho0"], **kw)


@pytest.mark.parametrize("lattice,shape", [(21, (40, 24)), (59, (20, 12, 10))])
def test_set_populations_then_step_matches_oracle(orc, L, lattice, shape):
    """Populations the oracle reached after 3 steps, handed to a fresh
    context (no lb2p_init), read back unchanged (FP64 storage) and advanced
    2 steps: equal to the oracle's steps 4 and 5 (1e-10)."""
    rho, u, model = small_case(lattice, shape)
    m = orc.Model(**model, tol=1e-14, max_iter=2000)
    n = orc.init(m, rho, u.T.copy())
    orc.step(m, n, 3)
    n3 = n.copy()
    orc.step(m, n, 2)
    perm = match_populations(L.velocities(lattice), orc.velocities(m.Q)[0])
    with L.Context(_params(L, model, L.STORE_F64, tol=1e-14, max_iter=2000)) as ctx:
        ctx.set_populations(n3[perm])
        back = ctx.populations()
        ctx.step(2)
        n5 = ctx.populations()
    assert np.array_equal(back, n3[perm])
    e = rel_err(n5, n[perm])
    print(lattice, "set + 2 steps vs oracle", f"{e:.2e}", flush=True)
    assert e <= 1e-10


def test_set_populations_f32_round_trip(L):
    """FP32 storage keeps the rest population (FP64 plane) exactly and each
    moving one as its deviation from the rest-equilibrium offset o_k of the
    reference density's record (set_populations has no local density):
    one FP32 rounding of (n - o_k)/W_k and one of the product W_k b, i.e.
    |error| <= 2^-23 |n - o_k| with |o_k| <= w_1 rho_ref < 0.1 here."""
    rho, u, model = small_case(59, (20, 12, 10))
    rng = np.random.default_rng(5)
    with L.Context(_params(L, model, L.STORE_F32)) as ctx:
        n = 0.02 + 0.01 * rng.random((59, ctx.N))
        ctx.set_populations(n)
        back = ctx.populations()
    assert np.array_equal(back[0], n[0])
    assert np.abs(back[1:] - n[1:]).max() <= 2.0**-23 * 0.13


def test_profiler_counts_launches(L):
    """Every time step launches moments, force, both closure kernels and the
    collision once, and the solve pass at least once.  lb2p_profile_enable
    resets the totals whether it switches timing on or off; while off, steps
    add nothing."""
    rho, u, model = small_case(59, (20, 12, 10))
    with L.Context(_params(L, model, L.STORE_F32, tol=1e-6, max_iter=200)) as ctx:
        ctx.init(rho, u)
        ctx.profile_enable(True)
        ctx.step(3)
        p = ctx.profile_read()
        for k in ("moments", "force", "closure1", "closure2", "collide"):
            assert p[k][1] == 3, (k, p[k])
            assert p[k][0] > 0.0
        assert p["iter_fused"][1] >= 3 and p["iter_fused"][0] > 0.0
        assert p["iter_q"][1] == 0 and p["iter_jt"][1] == 0   # the fused solve only
        ctx.profile_enable(False)
        ctx.step(2)
        assert all(v == (0.0, 0) for v in ctx.profile_read().values())
        ctx.profile_enable(True)
        ctx.step(1)
        q = ctx.profile_read()
        assert q["moments"][1] == 1 and q["collide"][1] == 1
        # one class timed, every class still counted
        ctx.profile_classes(["collide"])
        ctx.profile_enable(True)
        ctx.step(2)
        r = ctx.profile_read()
        assert r["collide"][1] == 2 and r["collide"][0] > 0.0
        for k in ("moments", "force", "closure1", "closure2"):
            assert r[k] == (0.0, 2), (k, r[k])
        assert r["iter_fused"][1] >= 2 and r["iter_fused"][0] == 0.0
        assert L.lib().lb2p_profile_classes(ctx._ctx, 1 << len(L.KERNEL_NAMES)) == L.EINVAL
        ctx.profile_classes(None)
        ctx.profile_enable(True)
        ctx.step(1)
        assert all(v[1] >= 1 and v[0] > 0.0 for k, v in ctx.profile_read().items()
                   if k not in ("iter_q", "iter_jt"))


def test_profiler_counts_working_passes(L):
    """lb2p_profile_passes counts the solve passes that did work: per step
    the pass count of its solve (lb2p_stats_get), while the launch count
    also holds the launches after the stop rule held."""
    import ctypes
    rho, u, model = small_case(59, (20, 12, 10))
    with L.Context(_params(L, model, L.STORE_F32, tol=1e-6, max_iter=200)) as ctx:
        ctx.init(rho, u)
        ctx.step(2)
        ctx.profile_enable(True)
        iters = []
        for _ in range(4):
            ctx.step(1)
            iters.append(ctx.stats()["iters"])
        passes = ctx.profile_passes()
        launches = ctx.profile_read()["iter_fused"][1]
        assert passes == sum(iters) and 4 <= passes <= launches, (iters, passes, launches)
        assert L.lib().lb2p_profile_passes(ctx._ctx, None) == L.EINVAL
        ctx.profile_enable(True)
        assert ctx.profile_passes() == 0


def test_profiler_teardown_leaves_no_hip_error(L):
    """Launches of classes the profiler only counts leave records without
    events; a context destroyed with such records pending (here the moments
    launch of lb2p_stats_get) must not leave a HIP error behind for the
    caller's next runtime call."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipGetLastError.restype = ctypes.c_int
    rho, u, model = small_case(59, (20, 12, 10))
    hip.hipGetLastError()
    with L.Context(_params(L, model, L.STORE_F32, tol=1e-6, max_iter=200)) as ctx:
        ctx.init(rho, u)
        ctx.profile_classes(["iter_fused"])
        ctx.profile_enable(True)
        ctx.step(2)
        ctx.profile_read()
        ctx.stats()
    assert hip.hipGetLastError() == 0
