"""lb2p_moments_noalloc through the C ABI: the same outputs as lb2p_moments,
bit for bit, on two calls in a row (the second on a smaller context, so the
static staging array keeps the first call's larger contents beyond the
second's range), for host and device outputs of both precisions; sizes
beyond the staging array are refused with LB2P_ESIZE before any work."""
import ctypes

import numpy as np
import pytest

from parity_util import small_case

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


def _both(L, ctx, dtype, device):
    """(lb2p_moments, lb2p_moments_noalloc) outputs of one state."""
    out = []
    for noalloc in (False, True):
        if device:
            import torch
            td = torch.float64 if dtype == np.float64 else torch.float32
            r = torch.full((ctx.N,), -1.0, dtype=td, device="cuda")
            u = torch.full((ctx.dim, ctx.N), -1.0, dtype=td, device="cuda")
            ctx.moments_into(r, u, noalloc=noalloc)
            torch.cuda.synchronize()
            out.append((r.cpu().numpy(), u.cpu().numpy()))
        else:
            r = np.full(ctx.N, -1.0, dtype=dtype)
            u = np.full((ctx.dim, ctx.N), -1.0, dtype=dtype)
            ctx.moments_into(r, u, noalloc=noalloc)
            out.append((r, u))
    return out


@pytest.mark.parametrize("storage", [1, 0])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("device", [False, True])
def test_noalloc_matches_moments_on_two_calls(L, storage, dtype, device):
    big = small_case(59, (40, 24, 20))
    small = small_case(21, (24, 16))
    for rho, u, model in (big, small):
        print("noalloc case", model["Q"], model["nx"], model["ny"], model["nz"], "storage", storage,
              "dtype", np.dtype(dtype).name, "device", device, flush=True)
        with L.Context(_params(L, model, storage)) as ctx:
            ctx.init(rho, u)
            ctx.step(2)
            (r1, u1), (r2, u2) = _both(L, ctx, dtype, device)
            assert ctx.last_status == L.OK
            assert np.array_equal(r1, r2) and np.array_equal(u1, u2)
            assert np.isfinite(r2).all() and (r2 > 0).all()
            # a later step is unaffected by either query
            ctx.step(1)
            assert ctx.last_status == L.OK


def test_noalloc_refuses_outputs_beyond_the_staging_array(L):
    """160^3 D3Q59 with FP32 fields: FP64 host output of u needs 3 * 160^3 * 8
    bytes = 98 MB > 64 MiB.  Refused with ESIZE before the state is touched
    (the context is not even initialised); FP32 output (no conversion) and
    device outputs need no staging."""
    n = 160
    assert 3 * n**3 * 8 > L.NOALLOC_STAGE_BYTES
    P = L.Params(lattice=59, nx=n, ny=n, nz=n, storage=L.STORE_F32, A=0.745, cs2_rho1=0.39, kappa=0.0124)
    with L.Context(P) as ctx:
        r = np.zeros(ctx.N)
        u = np.zeros((3, ctx.N))
        st = L.lib().lb2p_moments_noalloc(ctx._ctx, ctypes.c_void_p(r.ctypes.data),
                                          ctypes.c_void_p(u.ctypes.data), L.DTYPE_F64, 0, None)
        assert st == L.ESIZE
        r32 = np.zeros(ctx.N, dtype=np.float32)
        u32 = np.zeros((3, ctx.N), dtype=np.float32)
        st = L.lib().lb2p_moments_noalloc(ctx._ctx, ctypes.c_void_p(r32.ctypes.data),
                                          ctypes.c_void_p(u32.ctypes.data), L.DTYPE_F32, 0, None)
        assert st == L.ESTATE      # passed the size check; not initialised
