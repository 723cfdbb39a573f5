"""Long runs against the FP64 oracle's stored references
(tests/golden/longrun/, written by tests/golden/make_longrun_refs.py, which
calls the oracle only): the 256^3 slab workload on a 16 x 16 x 256 column
for its 2000 steps, the 128^3 droplet workload reduced to 48^3 for its 1000
steps, the first 16 domains of the batched workload for its 1000 steps, and
all 512 of its domains for 100 steps.
The error measures and stated bounds are those of test_gpu_longrun.py.
"""
import time

import numpy as np
import pytest

import lb2p_workloads as W
from test_gpu_longrun import _check, _errors, _form, _golden, _run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1402_2920_amd import lb2p
    lb2p.lib()
    return lb2p


@pytest.mark.parametrize("name,workload,shape", [("slab_column", "d3q59_256_slab", (16, 16, 256)),
                                                 ("droplet48", "d3q59_128_droplet", (48, 48, 48))])
@pytest.mark.parametrize("form", ["f32", "f32_f64fields", "f16", "bf16"])
def test_3d_long_run_against_oracle(L, name, workload, shape, form):
    meta, idx, vals = _golden(name)
    entry, shape, rho, u = W.build(workload, shape)
    assert list(shape) == meta["shape"]
    st, ip, tol = _form(L, form)
    t0 = time.time()
    got = _run(L, lambda: L.Params(nx=shape[0], ny=shape[1], nz=shape[2], storage=st, iter_prec=ip, tol=tol,
                                   max_iter=500, **W.model_kwargs(entry["model"])), rho, u,
               meta["checkpoints"], idx)
    print(f"{name} {form}: {meta['checkpoints'][-1]} steps in {time.time() - t0:.1f} s", flush=True)
    for k, c in enumerate(meta["checkpoints"]):
        _check(name, form, c, *_errors(got[k], vals[k, 0], vals[k, 1:], meta["rhomax"][k], meta["umax"][k]))


@pytest.mark.parametrize("form", ["f32", "f32_f64fields", "bf16"])
def test_batch16_1000_steps_against_oracle(L, form):
    """The first 16 domains of the batched workload in one batched context
    (per-domain stop rule), each domain against its own oracle run.  e_rho
    and |du| are the worst over the domains.  The FP32 forms hold e_u per
    domain (each domain's own max|u| as the scale).  BF16 resolves u to an
    absolute 2e-4 here, which is more than the whole flow of the quietest
    domains (max|u| about 2e-4): its e_u takes the batch's largest flow as
    the scale, beside the absolute bound |du| <= 5e-4."""
    meta, idx, vals = _golden("batch16")
    doms = W.build_batch("d2q21_batch512", limit=meta["ndom"])
    st, ip, tol = _form(L, form)
    rho = np.concatenate([d[2] for d in doms])
    u = np.concatenate([d[3] for d in doms], axis=1)
    got = _run(L, lambda: [L.Params(nx=s[0], ny=s[1], nz=1, storage=st, iter_prec=ip, tol=tol, max_iter=500,
                                    **W.model_kwargs(dd)) for dd, s, _, _ in doms], rho, u, meta["checkpoints"], idx)
    sizes = [s[0] * s[1] for _, s, _, _ in doms]
    dom_of = np.searchsorted(np.cumsum(sizes), idx, side="right")
    for k, c in enumerate(meta["checkpoints"]):
        vk = vals[k]   # [3, sites]: rho, u_x, u_y
        worst = (0.0, 0.0, 0.0)
        for d in range(meta["ndom"]):
            sel = dom_of == d
            e = _errors((got[k][0][sel], got[k][1][:, sel]), vk[0, sel], vk[1:, sel],
                        meta["rhomax_per_domain"][d][k], meta["umax_per_domain"][d][k])
            worst = tuple(max(a, b) for a, b in zip(worst, e))
        e_rho, e_u_dom, du = worst
        if form == "bf16":
            umax_batch = max(meta["umax_per_domain"][d][k] for d in range(meta["ndom"]))
            print(f"batch16 bf16 step {c}: worst per-domain e_u {e_u_dom:.2e}", flush=True)
            _check("batch16", form, c, e_rho, du / umax_batch, du)
        else:
            _check("batch16", form, c, e_rho, e_u_dom, du)


@pytest.mark.parametrize("form", ["f32", "bf16"])
def test_batch512_100_steps_against_oracle(L, form):
    """All 512 domains of the batched workload, 100 steps in one batched
    context (per-domain stop rule), 32 sampled sites per domain against each
    domain's own oracle run (the bounds and scales of the 16-domain case)."""
    meta, idx, vals = _golden("batch512_100")
    doms = W.build_batch("d2q21_batch512", limit=meta["ndom"])
    st, ip, tol = _form(L, form)
    rho = np.concatenate([d[2] for d in doms])
    u = np.concatenate([d[3] for d in doms], axis=1)
    got = _run(L, lambda: [L.Params(nx=s[0], ny=s[1], nz=1, storage=st, iter_prec=ip, tol=tol, max_iter=500,
                                    **W.model_kwargs(dd)) for dd, s, _, _ in doms], rho, u, meta["checkpoints"], idx)
    sizes = [s[0] * s[1] for _, s, _, _ in doms]
    dom_of = np.searchsorted(np.cumsum(sizes), idx, side="right")
    vk = vals[0]
    worst = (0.0, 0.0, 0.0)
    for d in range(meta["ndom"]):
        sel = dom_of == d
        e = _errors((got[0][0][sel], got[0][1][:, sel]), vk[0, sel], vk[1:, sel],
                    meta["rhomax_per_domain"][d][0], meta["umax_per_domain"][d][0])
        worst = tuple(max(a, b) for a, b in zip(worst, e))
    e_rho, e_u_dom, du = worst
    if form == "bf16":
        umax_batch = max(meta["umax_per_domain"][d][0] for d in range(meta["ndom"]))
        print(f"batch512 bf16: worst per-domain e_u {e_u_dom:.2e}", flush=True)
        _check("batch512_100", form, 100, e_rho, du / umax_batch, du)
    else:
        _check("batch512_100", form, 100, e_rho, e_u_dom, du)
