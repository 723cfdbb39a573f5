"""ctypes binding of ``liblb2p.so`` (C ABI in ``include/lb2p.h``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Host arrays are numpy; device arrays are torch tensors on the GPU
(PyTorch is used for device memory and streams only).  The library must have
been built (``paper_1402_2920_amd/build.py``); importing this module without
it raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblb2p.so")

OK, EINVAL, EEOS, ENOCONV, ENONFINITE, ENOMEM, EHIP, ESTATE, ESIZE = range(9)
NOALLOC_STAGE_BYTES = 64 << 20
D2Q21, D3Q59 = 21, 59
STORE_F64, STORE_F32, STORE_BF16, STORE_F16 = 0, 1, 2, 3
DTYPE_F64, DTYPE_F32 = 0, 1
FIELD_RHO, FIELD_J0, FIELD_FORCE, FIELD_JTILDE, FIELD_U, FIELD_SIGMA, FIELD_XI = range(7)
FLAG_UNFUSED_SOLVE = 1
FLAG_STENCIL_CLOSURE = 2
SOLVER_FIXED_POINT, SOLVER_CHEBYSHEV = 0, 1
ITER_AUTO, ITER_F32, ITER_F64 = 0, 1, 2
F32_TOL_FLOOR = 2e-7
F32_TOL_DEFAULT = 4e-7
# lb2p_default_params: FP64 1e-13, FP32 4e-7, BF16/F16 half the format's unit roundoff
DEFAULT_TOL = {0: 1e-13, 1: F32_TOL_DEFAULT, 2: 2.0**-9, 3: 2.0**-12}
STORAGE_NAMES = {"f64": STORE_F64, "f32": STORE_F32, "bf16": STORE_BF16, "f16": STORE_F16}


class Lb2pError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


class _Eos(ctypes.Structure):
    _fields_ = [("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
                ("A", ctypes.c_double), ("cs2_rho1", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("storage", ctypes.c_int), ("gamma", ctypes.c_double),
                ("kappa", ctypes.c_double), ("eos", _Eos), ("rho0", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("fixed_iter", ctypes.c_int),
                ("warm_start", ctypes.c_int), ("check_every", ctypes.c_int),
                ("store_rho_ref", ctypes.c_double), ("flags", ctypes.c_int),
                ("graph_steps", ctypes.c_int), ("solver", ctypes.c_int),
                ("spectral_bound", ctypes.c_double), ("iter_prec", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("mom", ctypes.c_double * 3), ("iters", ctypes.c_int),
                ("resid", ctypes.c_double), ("jscale", ctypes.c_double), ("nonfinite", ctypes.c_int)]


EXPORTED = [
    "lb2p_default_params", "lb2p_create", "lb2p_create_batch", "lb2p_domain_totals", "lb2p_domain_solve",
    "lb2p_autotune", "lb2p_init", "lb2p_step", "lb2p_moments", "lb2p_moments_noalloc",
    "lb2p_get_field", "lb2p_get_populations", "lb2p_set_populations", "lb2p_velocities",
    "lb2p_stats_get", "lb2p_profile_enable", "lb2p_profile_read", "lb2p_profile_classes", "lb2p_profile_passes",
    "lb2p_set_tiling", "lb2p_destroy", "lb2p_strerror",
]
KERNEL_NAMES = ["moments", "force", "iter_q", "iter_jt", "closure1", "closure2", "collide",
                "iter_fused"]

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1402_2920_amd/build.py")
        # One HIP runtime per process: PyTorch ships its own libamdhip64, and
        # device pointers and streams it hands over are only valid in that
        # runtime.  Loading torch first makes the library bind to the same
        # copy (by soname); loading it second leaves torch without a device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        pp = ctypes.POINTER(_Params)
        L.lb2p_default_params.argtypes = [ctypes.c_int] * 5 + [pp]
        L.lb2p_create.argtypes = [pp, vp, ctypes.POINTER(vp)]
        L.lb2p_create_batch.argtypes = [ctypes.c_int, pp, vp, ctypes.POINTER(vp)]
        L.lb2p_domain_totals.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.lb2p_domain_solve.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.lb2p_autotune.argtypes = [vp, ctypes.c_int]
        L.lb2p_init.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int]
        L.lb2p_step.argtypes = [vp, ctypes.c_int]
        L.lb2p_moments.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Stats)]
        L.lb2p_moments_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Stats)]
        L.lb2p_get_field.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int]
        L.lb2p_get_populations.argtypes = [vp, vp, ctypes.c_int]
        L.lb2p_set_populations.argtypes = [vp, vp, ctypes.c_int]
        L.lb2p_velocities.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.lb2p_stats_get.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.lb2p_profile_enable.argtypes = [vp, ctypes.c_int]
        L.lb2p_profile_classes.argtypes = [vp, ctypes.c_uint]
        L.lb2p_set_tiling.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.lb2p_profile_passes.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
        L.lb2p_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_longlong)]
        L.lb2p_destroy.argtypes = [vp]
        L.lb2p_destroy.restype = None
        L.lb2p_strerror.argtypes = [ctypes.c_int]
        L.lb2p_strerror.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("lb2p_destroy", "lb2p_strerror"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().lb2p_strerror(int(status)).decode()


def velocities(lattice: int) -> np.ndarray:
    c = (ctypes.c_int * (3 * 64))()
    q = ctypes.c_int(0)
    st = lib().lb2p_velocities(int(lattice), c, ctypes.byref(q))
    if st != OK:
        raise Lb2pError(st, "lb2p_velocities")
    return np.array(c[: 3 * q.value], dtype=np.int64).reshape(q.value, 3)


@dataclass
class Params:
    """Mirror of ``lb2p_params`` (lattice units h = a = 1)."""
    lattice: int
    nx: int
    ny: int
    nz: int = 1
    storage: int = STORE_F32
    gamma: float = 0.0
    kappa: float = 0.0
    rho1: float = 0.3
    rho2: float = 1.0
    A: float = 0.0
    cs2_rho1: float = 0.45
    rho0: float = 0.3
    tol: float | None = None
    max_iter: int = 200
    fixed_iter: int = 0
    warm_start: int = 1
    check_every: int = 0
    store_rho_ref: float = 0.0
    flags: int = 0
    graph_steps: int = 0
    solver: int = SOLVER_FIXED_POINT
    spectral_bound: float = 0.0
    iter_prec: int = ITER_AUTO

    def to_c(self) -> _Params:
        tol = self.tol if self.tol is not None else DEFAULT_TOL.get(self.storage, F32_TOL_DEFAULT)
        return _Params(self.lattice, self.nx, self.ny, self.nz, self.storage, self.gamma, self.kappa,
                       _Eos(self.rho1, self.rho2, self.A, self.cs2_rho1), self.rho0, tol,
                       self.max_iter, self.fixed_iter, self.warm_start, self.check_every,
                       self.store_rho_ref, self.flags, self.graph_steps, self.solver,
                       self.spectral_bound, self.iter_prec)

    @property
    def dim(self) -> int:
        return 3 if self.lattice == D3Q59 else 2

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz


def create_status(params: Params) -> int:
    """Status lb2p_create returns for these parameters (context freed)."""
    ctx = ctypes.c_void_p()
    prm = params.to_c()
    st = lib().lb2p_create(ctypes.byref(prm), None, ctypes.byref(ctx))
    if ctx.value:
        lib().lb2p_destroy(ctx)
    return st


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype_code: int):
    """(pointer, on_device) for a numpy array or torch tensor of the dtype."""
    if _is_torch(x):
        import torch
        want = torch.float64 if dtype_code == DTYPE_F64 else torch.float32
        if x.dtype != want or not x.is_contiguous():
            raise ValueError("torch buffer must be contiguous and of the requested dtype")
        return ctypes.c_void_p(x.data_ptr()), int(x.is_cuda)
    want = np.float64 if dtype_code == DTYPE_F64 else np.float32
    if x.dtype != want or not x.flags.c_contiguous:
        raise ValueError("numpy buffer must be C-contiguous and of the requested dtype")
    return ctypes.c_void_p(x.ctypes.data), 0


class Context:
    """One lattice (``lb2p_create``), or a batch of independent lattices
    (``lb2p_create_batch``) when ``params`` is a list; buffers then hold the
    domains packed in order (``offsets``)."""

    def __init__(self, params, stream=None):
        batch = isinstance(params, (list, tuple))
        plist = list(params) if batch else [params]
        self.params = params
        self.domains = plist
        self._ctx = ctypes.c_void_p()
        arr = (_Params * len(plist))(*[p.to_c() for p in plist])
        handle = None
        if stream is not None:
            handle = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        if batch:
            st = lib().lb2p_create_batch(len(plist), arr, handle, ctypes.byref(self._ctx))
        else:
            st = lib().lb2p_create(arr, handle, ctypes.byref(self._ctx))
        if st != OK:
            raise Lb2pError(st, "lb2p_create_batch" if batch else "lb2p_create")
        self.Q = plist[0].lattice
        self.dim = plist[0].dim
        self.N = sum(p.N for p in plist)
        self.offsets = np.cumsum([0] + [p.N for p in plist])
        self.last_status = OK

    def _check(self, st, where, allow=()):
        self.last_status = st
        if st != OK and st not in allow:
            raise Lb2pError(st, where)
        return st

    def close(self):
        if self._ctx is not None and self._ctx.value:
            lib().lb2p_destroy(self._ctx)
        self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def init(self, rho, u):
        """rho [N] and u [d][N] (numpy host or torch device, FP64 or FP32)."""
        code = DTYPE_F64 if str(rho.dtype).endswith("float64") else DTYPE_F32
        pr, dev = _ptr(rho, code)
        pu, dev2 = _ptr(u, code)
        assert dev == dev2
        return self._check(lib().lb2p_init(self._ctx, pr, pu, code, dev), "lb2p_init")

    def step(self, nsteps: int = 1, allow=(ENOCONV,)):
        return self._check(lib().lb2p_step(self._ctx, int(nsteps)), "lb2p_step", allow)

    def moments(self, dtype=np.float64, allow=(ENOCONV,)):
        """(rho [N], u [d][N]) of the current state as numpy arrays."""
        code = DTYPE_F64 if dtype == np.float64 else DTYPE_F32
        rho = np.zeros(self.N, dtype=dtype)
        u = np.zeros((self.dim, self.N), dtype=dtype)
        st = _Stats()
        self._check(lib().lb2p_moments(self._ctx, _ptr(rho, code)[0], _ptr(u, code)[0], code, 0,
                                       ctypes.byref(st)), "lb2p_moments", allow)
        return rho, u

    def moments_into(self, rho, u, allow=(ENOCONV,), noalloc=False):
        """Write into caller buffers (torch device tensors or numpy);
        ``noalloc`` calls lb2p_moments_noalloc."""
        code = DTYPE_F64 if str(rho.dtype).endswith("float64") else DTYPE_F32
        pr, dev = _ptr(rho, code)
        pu, _ = _ptr(u, code)
        fn = lib().lb2p_moments_noalloc if noalloc else lib().lb2p_moments
        name = "lb2p_moments_noalloc" if noalloc else "lb2p_moments"
        return self._check(fn(self._ctx, pr, pu, code, dev, None), name, allow)

    def field(self, which: int, dtype=np.float64) -> np.ndarray:
        ncomp = {FIELD_RHO: 1, FIELD_SIGMA: 6 if self.dim == 3 else 3,
                 FIELD_XI: 10 if self.dim == 3 else 4}.get(which, self.dim)
        code = DTYPE_F64 if dtype == np.float64 else DTYPE_F32
        out = np.zeros((ncomp, self.N), dtype=dtype)
        self._check(lib().lb2p_get_field(self._ctx, int(which), _ptr(out, code)[0], code, 0),
                    "lb2p_get_field")
        return out[0] if which == FIELD_RHO else out

    def populations(self) -> np.ndarray:
        out = np.zeros((self.Q, self.N))
        self._check(lib().lb2p_get_populations(self._ctx, ctypes.c_void_p(out.ctypes.data), 0),
                    "lb2p_get_populations")
        return out

    def populations_into(self, out):
        """Decoded populations [Q][N] FP64 into a caller buffer (a contiguous
        torch FP64 device tensor, or a numpy array)."""
        p, dev = _ptr(out, DTYPE_F64)
        return self._check(lib().lb2p_get_populations(self._ctx, p, dev), "lb2p_get_populations")

    def set_populations(self, n: np.ndarray):
        n = np.ascontiguousarray(n, dtype=np.float64)
        assert n.shape == (self.Q, self.N)
        return self._check(lib().lb2p_set_populations(self._ctx, ctypes.c_void_p(n.ctypes.data), 0),
                           "lb2p_set_populations")

    def profile_enable(self, on: bool = True):
        return self._check(lib().lb2p_profile_enable(self._ctx, int(on)), "lb2p_profile_enable")

    def profile_classes(self, names=None):
        """Bracket only the named kernel classes with events (None: all);
        the others are counted."""
        mask = (1 << len(KERNEL_NAMES)) - 1 if names is None else sum(1 << KERNEL_NAMES.index(k) for k in names)
        return self._check(lib().lb2p_profile_classes(self._ctx, mask), "lb2p_profile_classes")

    def profile_passes(self) -> int:
        """Solve passes that did work since profile_enable (the solve-pass
        launch count also holds launches after the stop rule held)."""
        n = ctypes.c_longlong(0)
        self._check(lib().lb2p_profile_passes(self._ctx, ctypes.byref(n)), "lb2p_profile_passes")
        return n.value

    def profile_read(self) -> dict:
        """{kernel class: (total ms, launches)} since profile_enable."""
        n = len(KERNEL_NAMES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        self._check(lib().lb2p_profile_read(self._ctx, ms, cnt), "lb2p_profile_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_NAMES)}

    def domain_totals(self) -> np.ndarray:
        """[ndom, 4] FP64: mass and momentum (x, y, z) per domain."""
        out = np.zeros((len(self.domains), 4))
        self._check(lib().lb2p_domain_totals(self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "lb2p_domain_totals")
        return out

    def domain_solve(self) -> dict:
        """Per domain, the last j~ solve: passes, last residual, max|j0'| and
        whether the stop rule held (numpy arrays of ndom entries)."""
        n = len(self.domains)
        it = np.zeros(n, dtype=np.int32)
        res = np.zeros(n)
        js = np.zeros(n)
        cv = np.zeros(n, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(lib().lb2p_domain_solve(self._ctx, it.ctypes.data_as(ip), res.ctypes.data_as(dp),
                                            js.ctypes.data_as(dp), cv.ctypes.data_as(ip)), "lb2p_domain_solve")
        return dict(iters=it, resid=res, jscale=js, converged=cv.astype(bool))

    def autotune(self, steps: int = 2):
        return self._check(lib().lb2p_autotune(self._ctx, int(steps)), "lb2p_autotune")

    def set_tiling(self, bx: int, by: int, tz: int = 128):
        """The site kernels' block shape (bx * by = 256, or bx = 256, by = 0
        for blocks of 256 consecutive sites) and the 3D solve chunk length."""
        return self._check(lib().lb2p_set_tiling(self._ctx, int(bx), int(by), int(tz)), "lb2p_set_tiling")

    def stats(self) -> dict:
        st = _Stats()
        self._check(lib().lb2p_stats_get(self._ctx, ctypes.byref(st)), "lb2p_stats_get")
        return dict(mass=st.mass, mom=np.array(st.mom[:]), iters=st.iters, resid=st.resid,
                    jscale=st.jscale, nonfinite=bool(st.nonfinite))
