"""CPU checks of the C-ABI library: it loads, exports every function that
include/lb2p.h declares, and its host-side validation and tables behave
(no GPU compute is called here).

Failure injection on the host: an inadmissible equation of state (App. B)
gives LB2P_EEOS, out-of-range gamma (Sec. II) or a grid side below 8 gives
LB2P_EINVAL, before any device call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1402_2920_amd import build, lb2p
    build.build(force=False)
    lb2p.lib()
    return lb2p


def test_every_declared_symbol_is_exported(L):
    hdr = open(os.path.join(ROOT, "include", "lb2p.h")).read()
    names = set(re.findall(r"\b(lb2p_[a-z_]+)\s*\(", hdr))
    assert len(names) >= 12
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(L.EXPORTED)


@pytest.mark.parametrize("Q", [21, 59])
def test_velocity_table(L, orc, Q):
    c = L.velocities(Q)
    assert c.shape == (Q, 3)
    co, _ = orc.velocities(Q)
    assert {tuple(v) for v in c} == {tuple(v) for v in co}
    assert tuple(c[0]) == (0, 0, 0)
    # antipodal pairs (2p+1, 2p+2)
    for p in range((Q - 1) // 2):
        assert tuple(c[2 * p + 2]) == tuple(-c[2 * p + 1])


def test_default_params(L):
    prm = L._Params()
    st = L.lib().lb2p_default_params(59, 32, 32, 32, L.STORE_F32, ctypes.byref(prm))
    assert st == L.OK
    assert (prm.nx, prm.ny, prm.nz, prm.storage) == (32, 32, 32, L.STORE_F32)
    assert prm.gamma == 0.0 and prm.tol == 4e-7 and prm.max_iter == 200 and prm.warm_start == 1
    assert prm.iter_prec == L.ITER_AUTO
    assert prm.eos.rho1 == 0.3 and prm.eos.rho2 == 1.0 and prm.rho0 == 0.3
    assert L.lib().lb2p_default_params(59, 8, 8, 8, L.STORE_F64, None) == L.EINVAL
    # the binding's default tolerance per storage is the library's
    for stg in (L.STORE_F64, L.STORE_F32, L.STORE_BF16, L.STORE_F16):
        assert L.lib().lb2p_default_params(59, 32, 32, 32, stg, ctypes.byref(prm)) == L.OK
        assert prm.tol == L.DEFAULT_TOL[stg] == L.Params(lattice=59, nx=8, ny=8, nz=8, storage=stg).to_c().tol
    assert L.DEFAULT_TOL[L.STORE_BF16] == 2.0**-9 and L.DEFAULT_TOL[L.STORE_F16] == 2.0**-12


def test_profile_classes_rejects_null_context(L):
    assert L.lib().lb2p_profile_classes(None, 1) == L.EINVAL
    assert L.lib().lb2p_profile_classes(None, 0) == L.EINVAL
    n = ctypes.c_longlong(0)
    assert L.lib().lb2p_profile_passes(None, ctypes.byref(n)) == L.EINVAL
    assert L.lib().lb2p_set_tiling(None, 256, 0, 128) == L.EINVAL


def _p(L, **kw):
    base = dict(lattice=59, nx=16, ny=16, nz=16, A=0.745, cs2_rho1=0.39, kappa=0.01)
    base.update(kw)
    return L.Params(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(gamma=1.0), "EINVAL"), (dict(gamma=-1.0), "EINVAL"), (dict(nx=7), "EINVAL"),
    (dict(lattice=21, nz=4), "EINVAL"), (dict(lattice=20), "EINVAL"), (dict(kappa=-1.0), "EINVAL"),
    (dict(tol=-1.0), "EINVAL"), (dict(max_iter=0), "EINVAL"), (dict(storage=7), "EINVAL"),
    # a domain of 2^29 sites or more: its FP64 plane would pass 4 GiB, beyond
    # the kernels' 32-bit byte offsets (refused before any allocation)
    (dict(nx=813, ny=813, nz=813), "EINVAL"),
    # App. B: the paper's example EOS violates positive bulk viscosity in 3D
    (dict(A=1.2, rho1=0.5, cs2_rho1=0.6), "EEOS"),
    # weights negative for c_s^2 below the Sec. III window
    (dict(cs2_rho1=0.38), "EEOS"),
    # A > 0 without a two-phase region
    (dict(A=0.5), "EEOS"),
    # non-finite or out-of-range settings are refused before any device call
    (dict(kappa=float("nan")), "EINVAL"), (dict(gamma=float("nan")), "EINVAL"),
    (dict(rho0=float("nan")), "EINVAL"), (dict(rho0=0.0), "EINVAL"),
    (dict(tol=float("nan")), "EINVAL"), (dict(A=float("nan")), "EINVAL"),
    (dict(cs2_rho1=float("nan")), "EINVAL"), (dict(rho1=1.2), "EINVAL"),
    (dict(warm_start=4), "EINVAL"), (dict(warm_start=-1), "EINVAL"),
    (dict(fixed_iter=-1), "EINVAL"), (dict(graph_steps=-1), "EINVAL"),
    (dict(iter_prec=3), "EINVAL"), (dict(iter_prec=-1), "EINVAL"),
    # FP64 storage computes in FP64: an FP32 iteration is not offered
    (dict(storage=0, iter_prec=1), "EINVAL"),
])
def test_create_rejects_bad_parameters(L, kw, status):
    assert L.create_status(_p(L, **kw)) == getattr(L, status)


def test_strerror(L):
    for s in range(9):
        assert isinstance(L.strerror(s), str) and L.strerror(s)
    assert L.strerror(99) == "unknown status"


def test_batch_rejects_mixed_shared_settings(L):
    """Domains of one batched context share lattice, storage and iteration
    settings; a mismatch is refused on the host before any allocation."""
    a = L.Params(lattice=59, nx=16, ny=16, nz=16, A=0.745, cs2_rho1=0.39, kappa=0.01)
    b = L.Params(lattice=59, nx=20, ny=12, nz=10, A=0.745, cs2_rho1=0.39, kappa=0.02,
                 storage=L.STORE_F64)
    with pytest.raises(L.Lb2pError) as ei:
        L.Context([a, b])
    assert ei.value.status == L.EINVAL
    c = L.Params(lattice=21, nx=16, ny=16, A=0.8, cs2_rho1=0.45, kappa=0.1)
    with pytest.raises(L.Lb2pError) as ei:
        L.Context([a, c])
    assert ei.value.status == L.EINVAL


def test_solver_settings_validated(L):
    base = dict(lattice=59, nx=16, ny=16, nz=16, A=0.745, cs2_rho1=0.39, kappa=0.01)
    assert L.create_status(L.Params(**base, solver=2)) == L.EINVAL
    assert L.create_status(L.Params(**base, solver=1, spectral_bound=1.0)) == L.EINVAL
    assert L.create_status(L.Params(**base, solver=1, spectral_bound=-0.1)) == L.EINVAL
    # an EOS whose plane-wave bound reaches 1: the semi-iteration does not apply
    hot = dict(base, A=0.9, cs2_rho1=0.8)
    assert L.create_status(L.Params(**hot, solver=1)) in (L.EINVAL, L.EEOS)
