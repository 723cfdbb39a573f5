"""ctypes binding of the FP64 CPU oracle (``lb2p_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this module.  The GPU package never does.

Arrays follow the oracle's conventions: populations ``n[Q, N]`` (pre-collision,
site index ``x + nx*(y + ny*z)``), vector fields ``[N, 3]``, rank-2 tensors
``[N, 3, 3]``, rank-3 tensors ``[N, 3, 3, 3]``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("Q", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("gamma", ctypes.c_double), ("kappa", ctypes.c_double),
        ("rho1", ctypes.c_double), ("rho2", ctypes.c_double), ("A", ctypes.c_double),
        ("cs2_1", ctypes.c_double), ("rho0", ctypes.c_double),
        ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("flags", ctypes.c_int),
    ]


class OrcInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("resid", ctypes.c_double),
                ("jscale", ctypes.c_double), ("converged", ctypes.c_int)]


NO_CORR = 1
STENCIL_CLOSURE = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP, -O2)."""
    from . import build_oracle
    return build_oracle.build(force=force)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(OrcParams)
        L.orc_velocities.argtypes = [ctypes.c_int, ip, ip]
        L.orc_weights.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc_eos.argtypes = [pp, ctypes.c_double, dp]
        L.orc_equilibrium.argtypes = [pp, ctypes.c_double, dp, dp]
        L.orc_init.argtypes = [pp, dp, dp, dp]
        L.orc_fields.argtypes = [pp, dp, dp, dp, dp, dp, dp, ctypes.POINTER(OrcInfo)]
        L.orc_closure.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_site_collision.argtypes = [pp, dp, ctypes.c_double, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_step.argtypes = [pp, dp, ctypes.c_int, ctypes.POINTER(OrcInfo)]
        L.orc_totals.argtypes = [pp, dp, dp, dp]
        L.orc_jtilde_map.argtypes = [pp, dp, dp, dp, dp]
        L.orc_hessian.argtypes = [pp, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Model:
    """Parameters of one run (lattice units h = a = 1)."""
    Q: int
    nx: int
    ny: int
    nz: int = 1
    gamma: float = 0.0
    kappa: float = 0.0
    rho1: float = 0.3
    rho2: float = 1.0
    A: float = 0.0
    cs2_1: float = 0.45
    rho0: float = 0.3
    tol: float = 1e-13
    max_iter: int = 1000
    flags: int = 0

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dim(self) -> int:
        return 3 if self.Q == 59 else 2

    def c_params(self) -> OrcParams:
        return OrcParams(self.Q, self.nx, self.ny, self.nz, self.gamma, self.kappa,
                         self.rho1, self.rho2, self.A, self.cs2_1, self.rho0,
                         self.tol, self.max_iter, self.flags)


def velocities(Q: int):
    c = np.zeros((Q, 3), dtype=np.int32)
    sh = np.zeros(Q, dtype=np.int32)
    r = lib().orc_velocities(Q, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                             sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    assert r == Q
    return c, sh


def weights(Q: int, sigma2: float) -> np.ndarray:
    w = np.zeros(Q)
    lib().orc_weights(Q, float(sigma2), _p(w))
    return w


def eos(m: Model, rho) -> np.ndarray:
    """EOS at each density: columns cs2, p, dp/drho, P1, P2, psi."""
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    out = np.zeros((rho.size, 6))
    prm = m.c_params()
    buf = np.zeros(6)
    for k, r in enumerate(rho.ravel()):
        lib().orc_eos(ctypes.byref(prm), float(r), _p(buf))
        out[k] = buf
    return out


def equilibrium(m: Model, rho: float, u) -> np.ndarray:
    u3 = np.zeros(3)
    u3[:len(u)] = u
    out = np.zeros(m.Q)
    prm = m.c_params()
    lib().orc_equilibrium(ctypes.byref(prm), float(rho), _p(u3), _p(out))
    return out


def _vec3(u, N):
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = u.reshape(N, -1)
    out = np.zeros((N, 3))
    out[:, :u.shape[1]] = u.reshape(N, -1)
    return np.ascontiguousarray(out)


def init(m: Model, rho, u) -> np.ndarray:
    """n_i = n_eq(rho, u); rho is [N] (any shape flattening to N), u [N, d]."""
    N = m.N
    rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(N))
    u3 = _vec3(np.asarray(u).reshape(N, -1), N)
    n = np.zeros((m.Q, N))
    prm = m.c_params()
    lib().orc_init(ctypes.byref(prm), _p(rho), _p(u3), _p(n))
    return n


def fields(m: Model, n: np.ndarray):
    """Items 1-8: returns dict(rho, j0, f, jt, u, info)."""
    N = m.N
    n = np.ascontiguousarray(n, dtype=np.float64)
    rho = np.zeros(N); j0 = np.zeros((N, 3)); f = np.zeros((N, 3))
    jt = np.zeros((N, 3)); u = np.zeros((N, 3))
    info = OrcInfo()
    prm = m.c_params()
    rc = lib().orc_fields(ctypes.byref(prm), _p(n), _p(rho), _p(j0), _p(f), _p(jt), _p(u),
                          ctypes.byref(info))
    return dict(rho=rho, j0=j0, f=f, jt=jt, u=u, converged=(rc == 0), iters=info.iters,
                resid=info.resid, jscale=info.jscale)


def closure(m: Model, rho, j, jt):
    N = m.N
    Sig = np.zeros((N, 3, 3)); Xi = np.zeros((N, 3, 3, 3))
    prm = m.c_params()
    lib().orc_closure(ctypes.byref(prm), _p(np.ascontiguousarray(rho, dtype=np.float64)),
                      _p(np.ascontiguousarray(j, dtype=np.float64)),
                      _p(np.ascontiguousarray(jt, dtype=np.float64)), _p(Sig), _p(Xi))
    return Sig, Xi


def site_collision(m: Model, n_site, rho, u, f, jt, Sigma, Xip):
    prm = m.c_params()
    db = np.zeros(m.Q); di = np.zeros(m.Q); dc = np.zeros(m.Q)
    lib().orc_site_collision(ctypes.byref(prm), _p(np.ascontiguousarray(n_site, dtype=np.float64)),
                             float(rho), _p(_vec3(u, 1)[0].copy()), _p(_vec3(f, 1)[0].copy()),
                             _p(_vec3(jt, 1)[0].copy()),
                             _p(np.ascontiguousarray(Sigma, dtype=np.float64).reshape(9).copy()),
                             _p(np.ascontiguousarray(Xip, dtype=np.float64).reshape(27).copy()),
                             _p(db), _p(di), _p(dc))
    return db, di, dc


def step(m: Model, n: np.ndarray, nsteps: int = 1):
    """Advance n (in place) by nsteps; returns (n, info dict)."""
    assert n.dtype == np.float64 and n.flags.c_contiguous and n.shape == (m.Q, m.N)
    info = OrcInfo()
    prm = m.c_params()
    rc = lib().orc_step(ctypes.byref(prm), _p(n), int(nsteps), ctypes.byref(info))
    return n, dict(converged=(rc == 0), iters=info.iters, resid=info.resid, jscale=info.jscale)


def totals(m: Model, n: np.ndarray):
    mass = np.zeros(1); mom = np.zeros(3)
    prm = m.c_params()
    lib().orc_totals(ctypes.byref(prm), _p(np.ascontiguousarray(n)), _p(mass), _p(mom))
    return float(mass[0]), mom


def jtilde_map(m: Model, rho, j0p, jt):
    N = m.N
    out = np.zeros((N, 3))
    prm = m.c_params()
    lib().orc_jtilde_map(ctypes.byref(prm), _p(np.ascontiguousarray(rho, dtype=np.float64)),
                         _p(_vec3(j0p, N)), _p(_vec3(jt, N)), _p(out))
    return out


def hessian(m: Model, g) -> np.ndarray:
    """d_a d_b g [N, 3, 3] from the Table III Laplacian and traceless stencils."""
    out = np.zeros((m.N, 3, 3))
    prm = m.c_params()
    lib().orc_hessian(ctypes.byref(prm), _p(np.ascontiguousarray(g, dtype=np.float64).reshape(m.N)), _p(out))
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())
