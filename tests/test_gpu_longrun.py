"""Long runs at the configurations' stated lengths, every storage form
against an FP64 reference.

References: the FP64 oracle (tests/golden/longrun/, written by
tests/golden/make_longrun_refs.py, which calls the oracle only; C1 is run
here) -- rho and u at a seeded sample of sites, with max|u| and max rho of
the whole lattice as the error scales -- and, for the 512^3 two-droplet case
that no host can hold in FP64, the library's FP64 path (itself within 1e-10
of the oracle wherever the oracle can run).

e_rho = max |rho_G - rho_O| / max rho_O, e_u = max |u_G - u_O| / max |u_O|
(max over the sampled sites, scale over all sites).  Stated bounds (FP32
fields at the default tolerance 4e-7; FP32 storage with FP64 fields at tol
1e-13; BF16 and FP16 deviation storage, FP32 fields):
  FP32            e_rho 1e-7, e_u 1e-5, except the slab column, whose flow
                  decays to 2e-5 after a few hundred steps: there the FP32
                  fields' rounding (|u_G - u_O| about 4e-10) allows e_u 5e-5;
  FP32 + FP64 fields  e_rho 1e-8, e_u 1e-5;
  FP16            e_rho 3e-4, e_u 0.15;
  BF16            e_rho 2e-2, e_u 0.5 (and |u_G - u_O| <= 5e-4).
"""
import json
import os
import time

import numpy as np
import pytest

import lb2p_workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "longrun")

BOUNDS = {  # form: (e_rho, e_u)
    "f32": (1e-7, 1e-5),
    "f32_f64fields": (1e-8, 1e-5),
    "f16": (3e-4, 0.15),
    "bf16": (2e-2, 0.5),
}
SLAB_F32_EU = 5e-5
BF16_ABS_U = 5e-4


@pytest.fixture(scope="module")
def L():
    from paper_1402_2920_amd import lb2p
    lb2p.lib()
    return lb2p


def _form(L, name):
    """(storage, iter_prec, tol) of a storage form."""
    return {"f32": (L.STORE_F32, L.ITER_F32, None), "f32_f64fields": (L.STORE_F32, L.ITER_F64, 1e-13),
            "f16": (L.STORE_F16, L.ITER_F32, None), "bf16": (L.STORE_BF16, L.ITER_F32, None),
            "f64": (L.STORE_F64, L.ITER_AUTO, 1e-13)}[name]


def _run(L, params_of, rho, u, checkpoints, idx=None):
    """(rho, u) at each checkpoint, restricted to the sample idx."""
    out = []
    with L.Context(params_of()) as ctx:
        ctx.init(rho, np.ascontiguousarray(u))
        done = 0
        for c in checkpoints:
            ctx.step(c - done)
            done = c
            r, v = ctx.moments()
            out.append((r if idx is None else r[idx], v if idx is None else v[:, idx]))
    return out


def _errors(got, ref_rho, ref_u, rhomax, umax):
    r, v = got
    e_rho = float(np.abs(r - ref_rho).max() / rhomax)
    du = np.sqrt(((v - ref_u) ** 2).sum(0))
    return e_rho, float(du.max() / umax), float(du.max())


def _check(name, form, cp, e_rho, e_u, abs_u):
    b_rho, b_u = BOUNDS[form]
    if form == "f32" and name in ("slab_column", "c3"):
        b_u = SLAB_F32_EU
    print(f"{name} {form} step {cp}: e_rho {e_rho:.2e} (<= {b_rho:g}) e_u {e_u:.2e} (<= {b_u:g}) "
          f"|du| {abs_u:.2e}", flush=True)
    assert e_rho <= b_rho and e_u <= b_u, (name, form, cp, e_rho, e_u)
    if form == "bf16":
        assert abs_u <= BF16_ABS_U


def _golden(name):
    meta = json.load(open(os.path.join(GOLD, "longrun.json")))[name]
    idx = np.load(os.path.join(GOLD, f"{name}_idx.npy"))
    vals = np.load(os.path.join(GOLD, f"{name}_vals.npy"))
    return meta, idx, vals


@pytest.fixture(scope="module")
def c1_ref(orc):
    entry, shape, rho, u = W.build("d2q21_64_droplet")
    m = orc.Model(nx=shape[0], ny=shape[1], nz=1, tol=1e-13, max_iter=2000, **W.oracle_kwargs(entry["model"]))
    n = orc.init(m, rho, u.T.copy())
    out, done = [], 0
    for c in (100, 1000):
        orc.step(m, n, c - done)
        done = c
        F = orc.fields(m, n)
        out.append((c, F["rho"].copy(), F["u"][:, :2].T.copy()))
    return entry, shape, rho, u, out


@pytest.mark.parametrize("form", ["f32", "f32_f64fields", "f16", "bf16"])
def test_c1_1000_steps(L, c1_ref, form):
    entry, shape, rho, u, ref = c1_ref
    st, ip, tol = _form(L, form)
    got = _run(L, lambda: L.Params(nx=shape[0], ny=shape[1], nz=1, storage=st, iter_prec=ip, tol=tol,
                                   max_iter=500, **W.model_kwargs(entry["model"])), rho, u, [c for c, _, _ in ref])
    for (c, rr, ur), g in zip(ref, got):
        umax = float(np.sqrt((ur**2).sum(0)).max())
        _check("c1", form, c, *_errors(g, rr, ur, float(rr.max()), umax))


def _against_gpu_f64(L, workload, checkpoints, forms, nsample, seed):
    """Run the workload at full size in FP64 and in each storage form, one
    after the other, and return per form the (rho, u) sample at each
    checkpoint plus the FP64 run's whole-lattice max rho and max|u| there."""
    import torch
    entry, shape, rho, u = W.build(workload)
    N = rho.size
    idx = np.sort(np.random.default_rng(seed).choice(N, size=min(nsample, N), replace=False))
    torch.cuda.set_device(0)
    res = {}
    for form in ("f64",) + tuple(forms):
        st, ip, tol = _form(L, form)
        P = L.Params(nx=shape[0], ny=shape[1], nz=shape[2], storage=st, iter_prec=ip, tol=tol, max_iter=300,
                     **W.model_kwargs(entry["model"]))
        t0 = time.time()
        out = []
        with L.Context(P, stream=torch.cuda.current_stream()) as ctx:
            ctx.init(torch.tensor(rho, device="cuda:0"), torch.tensor(u, device="cuda:0").contiguous())
            done = 0
            rd = torch.empty(N, dtype=torch.float64, device="cuda:0")
            ud = torch.empty((3, N), dtype=torch.float64, device="cuda:0")
            ti = torch.as_tensor(idx, device="cuda:0")
            for c in checkpoints:
                while done < c:
                    k = min(100, c - done)
                    ctx.step(k)
                    done += k
                    print(f"{workload} {form}: step {done}, {time.time() - t0:.0f} s", flush=True)
                ctx.moments_into(rd, ud)
                out.append((rd[ti].cpu().numpy(), ud[:, ti].cpu().numpy(), float(rd.max()),
                            float(ud.square().sum(0).sqrt().max())))
            del rd, ud, ti
        res[form] = out
        torch.cuda.empty_cache()
    return res


@pytest.mark.timeout(900)
def test_c5_512_two_droplets_500_steps_against_gpu_f64(L):
    """512^3 two droplets colliding, 500 steps: FP32 and BF16 storage against
    the library's FP64 path (flagged: the host cannot hold the FP64 oracle's
    2 x 63 GB of populations).  rho and u come back to the host at a seeded
    sample of 2^20 sites."""
    entry = W.load_params()["d3q59_512_two_droplets"]
    steps = entry["steps"]
    res = _against_gpu_f64(L, "d3q59_512_two_droplets", [steps], ("f32", "bf16"), 1 << 20, 1406)
    rr, ur, rhomax, umax = res["f64"][0]
    assert umax > 1e-3   # the droplets still move
    for form in ("f32", "bf16"):
        _check("c5", form, steps, *_errors(res[form][0][:2], rr, ur, rhomax, umax))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,workload,checkpoints", [("c2", "d3q59_128_droplet", [100, 1000]),
                                                       ("c3", "d3q59_256_slab", [500, 1000, 2000])])
def test_full_size_run_against_gpu_f64(L, name, workload, checkpoints):
    """The 128^3 droplet for its 1000 steps and the 256^3 slab for its 2000,
    at full size, in FP32, FP16 and BF16 storage against the library's FP64
    path (itself within 1e-10 of the oracle on every window the oracle can
    run), at the stated bounds; the oracle references of the same workloads
    on reduced grids are in test_gpu_longrun_oracle.py."""
    forms = ("f32", "f16", "bf16")
    res = _against_gpu_f64(L, workload, checkpoints, forms, 1 << 20, 1407)
    for k, c in enumerate(checkpoints):
        rr, ur, rhomax, umax = res["f64"][k]
        for form in forms:
            _check(name, form, c, *_errors(res[form][k][:2], rr, ur, rhomax, umax))
