"""Throughput of the consistent two-phase LB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--storage f32]

Prints ONE JSON line.  A step is one full time step (Supplemental items 1-12:
moments, force, the implicit j~/u solve to the paper's stop rule, closure,
collision, streaming) over the whole lattice; value = lattice sites x steps /
wall time of the timed region / 1e6 (MLUPS), inputs already in HBM.  The
timed window follows --settle steps (default 200) of the run from the
synthetic start: the first steps relax the initial tanh walls and noise and
need up to twice the solve passes of the rest of a 2000-step run.

roofline: the kernel class with the largest share of the timed region,
its algorithmic bytes per launch (per-site bytes x sites) over its average
HIP-event duration on the library's stream, against 8 TB/s.  For the solve
pass the per-site bytes are the pass's minimum, (1 + 3D) r (rho, j0', the
iterate in and out); the bytes the fused pass moves by design (it also
reads p and P1) are reported beside them.
step_hbm: the whole step's bandwidth (population floor 2 Q s per site, the
kernels' algorithmic bytes, the counters' measured bytes) against 8 TB/s and
against a streaming copy measured in the same run.
cpu_baseline: the FP64 oracle, unchanged, on a bounded sample of the same
workload (a 16 x 16 x nz column for 3D grids), on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "d3q59_256_slab"


def site_bytes(kernel, Q, D, s, r, warm, cheb=False, pull=False):
    """Algorithmic bytes per site of one launch of a kernel class: every
    population or field word the kernel must read or write once (stencil
    neighbours are reuse, not extra traffic).  The rest population is one
    plane of t0 bytes (FP64 beside FP64/FP32 storage, FP32 beside BF16/FP16);
    the deviation forms (FP32, BF16, FP16 storage) add the writer's 2-byte
    density record per site.  The moments
    kernel writes the exact pulled mass (FP64), which the collision reads in
    place of the pulled populations when gamma = 0 (pull=False); with
    gamma != 0 the collision pulls the populations again."""
    nsig = 6 if D == 3 else 3
    nxi = 10 if D == 3 else 4
    t0 = 8 if s >= 4 else 4
    rec = 0 if s == 8 else 2     # the writer's density record of the deviation forms
    pops = (Q - 1) * s + t0 + rec
    return {
        # pulled populations; writes rho, j0, the FP64 mass and the four
        # per-step EOS planes (p - p_ref, P1, 1/rho, c_s^2 - c_s^2_ref)
        "moments": pops + (1 + D) * r + 8 + 4 * r,
        # reads the FP64 mass (stencil) and j0; warm: 0 zero start, 1 previous
        # j~, 2/3 extrapolated (history read and written); writes f, j0', u
        "force": 8 + D * r + (D * r if warm else 0) + (2 * D * r * (warm - 1) if warm >= 2 else 0)
                 + 3 * D * r,
        "iter_q": (2 + D) * r + nsig * r,
        "iter_jt": (nsig + 1 + 2 * D) * r + 2 * D * r + (D * r if cheb else 0),
        # reads u, p - p_ref, c_s^2 - c_s^2_ref, P1, 1/rho and (to form j~ =
        # rho u - j0' after the velocity-form solve) rho and j0'; writes X, T,
        # Y, Xi' and j~ (the copy of u when the solve ended in the second
        # buffer is not counted)
        "closure1": (5 + 2 * D) * r + (1 + nsig + D + nxi + D) * r,
        "closure2": (2 + nsig + 2 * D) * r + nsig * r,
        # fields u, f, j~, Sigma, Xi' and the FP64 mass
        "collide": (2 * pops if pull else pops + 8) + (3 * D + nsig + nxi) * r,
        # fused pass (velocity form): read u, p, P1 and (own site) j0', rho;
        # write the next u (Chebyshev: also read u_{k-1})
        "iter_fused": (3 + 2 * D) * r + D * r + (D * r if cheb else 0),
    }[kernel]


STORE_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}


SOLVERS = {"fixed_point": 0, "chebyshev": 1}


def dominant_class(prof):
    """The kernel class with the largest summed event time."""
    total = {k: v[0] for k, v in prof.items()}
    return max(total, key=total.get)


def run_gpu(workload, storage, steps, warmup, shape=None, profile=True, tol=None, solver="fixed_point",
            autotune=True, warm_start=1, settle=0, prof_steps=5):
    """Time `steps` steps after `settle` + `warmup` untimed ones.  With
    profile: `prof_steps` steps between them bracket every kernel class with
    HIP events (the per-kernel table and the dominant class); the timed
    steps then bracket only the dominant class (each bracketed launch adds
    two event records that the GPU processes between kernels) and count the
    launches of every class."""
    import torch
    import lb2p_workloads as W
    from paper_1402_2920_amd import lb2p
    entry, shape, rho, u = W.build(workload, shape)
    d = len(shape)
    st = lb2p.STORAGE_NAMES[storage]
    P = lb2p.Params(nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, storage=st,
                    tol=tol, max_iter=200, warm_start=warm_start, solver=SOLVERS[solver],
                    **W.model_kwargs(entry["model"]))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    dt = torch.float64
    rho_d = torch.tensor(rho, dtype=dt, device="cuda:0")
    u_d = torch.tensor(u, dtype=dt, device="cuda:0").contiguous()
    out = {}
    with lb2p.Context(P, stream=stream) as ctx:
        ctx.init(rho_d, u_d)
        del rho_d, u_d
        if autotune:
            ctx.autotune(2)
        # the synthetic start (tanh walls plus noise) relaxes over the first
        # steps, which need up to twice the solve passes of the rest of the
        # run; the timed window samples the run after that transient
        ctx.step(settle + warmup)
        prof_all = dom = None
        passes_all = passes = None
        if profile:
            ctx.profile_enable(True)
            ctx.step(prof_steps)
            prof_all = ctx.profile_read()
            passes_all = ctx.profile_passes()
            dom = dominant_class(prof_all)
            ctx.profile_classes([dom])
            ctx.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if profile:
            prof = ctx.profile_read()
            passes = ctx.profile_passes()
        else:
            prof = None
        stats = ctx.stats()
        out.update(seconds=t1 - t0, prof=prof, prof_all=prof_all, dominant=dom, passes=passes,
                   passes_all=passes_all,
                   prof_steps=prof_steps if profile else 0, stats=stats, N=P.N, Q=P.lattice, D=d,
                   shape=shape, params=P, pull=P.gamma != 0.0, workload=workload, storage=storage,
                   tol=P.to_c().tol)
    return out


def run_batch(workload, steps, warmup, fixed_iter, graph=True, limit=None, autotune=True):
    """Batched workload: every domain in one context, `fixed_iter` passes of
    the j~ iteration per step, the timed steps replayed from one captured HIP
    graph.  A short eager pass with per-kernel events follows for the
    roofline (events cannot sit inside a graph)."""
    import torch
    import lb2p_workloads as W
    from paper_1402_2920_amd import lb2p
    doms = W.build_batch(workload, limit)
    plist = [lb2p.Params(nx=sh[0], ny=sh[1], nz=1, storage=lb2p.STORE_F32, max_iter=200, warm_start=1,
                         fixed_iter=fixed_iter, graph_steps=steps if graph else 0,
                         **W.model_kwargs(ent))
             for ent, sh, _, _ in doms]
    rho = np.concatenate([r for _, _, r, _ in doms])
    u = np.ascontiguousarray(np.concatenate([uu for _, _, _, uu in doms], axis=1))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    out = {}
    with lb2p.Context(plist, stream=stream) as ctx:
        ctx.init(torch.tensor(rho, device="cuda:0"), torch.tensor(u, device="cuda:0"))
        if autotune:
            ctx.autotune(2)
        ctx.step(1)
        tot0 = ctx.domain_totals()
        # warm-up: the first steps-long call captures and instantiates the graph
        ctx.step(steps if graph else warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = ctx.stats()
        ds = ctx.domain_solve()
        tot = ctx.domain_totals()
        ctx.profile_enable(True)
        ctx.step(4)
        prof = ctx.profile_read()
        passes = ctx.profile_passes()
        ctx.profile_enable(False)
        out.update(seconds=t1 - t0, prof=prof, passes=passes, stats=st, N=ctx.N, Q=21, D=2, ndom=len(doms),
                   resid_ratio=ds["resid"] / np.maximum(ds["jscale"], 1e-300), resid_jscale=ds["jscale"],
                   pull=any(p.gamma != 0.0 for p in plist), workload=workload, storage="f32",
                   mass_drift=float(np.max(np.abs(tot[:, 0] - tot0[:, 0]) / tot0[:, 0])))
    return out


def minimal_pass_bytes(D, r, cheb=False):
    """Bytes per site that one pass of the j~ fixed point (items 3-8) cannot
    do without: rho and j0' at the site, the current iterate in, the next one
    out ((1 + 3D) r; Chebyshev also reads the iterate before).  The fused
    pass moves 2 r more: it reads the per-step planes p - p_ref and P1
    (formed in FP64 by the moments kernel) instead of evaluating the EOS's
    exp, sin and cos at every stencil point of every pass."""
    return (1 + 3 * D) * r + (D * r if cheb else 0)


def roofline(res, storage, warm=2, cheb=False):
    """The dominant kernel class's algorithmic bytes per launch over its
    average event time in the timed steps, and the per-kernel table (from
    the instrumented steps before them when the run has them)."""
    prof = res["prof"]
    Q, D, N = res["Q"], res["D"], res["N"]
    s = STORE_BYTES[storage]
    r = res.get("rsize", 8 if storage == "f64" else 4)
    pull = res.get("pull", False)
    dom = res.get("dominant") or dominant_class(prof)
    ms, n = prof[dom]
    # the solve pass: per pass that did work (launches after the stop rule
    # held return at once; their few microseconds stay in the total)
    work = work_launches(dom, n, res.get("passes"))
    avg_s = ms / 1e3 / max(work, 1)
    design = site_bytes(dom, Q, D, s, r, warm, cheb, pull)
    alg = minimal_pass_bytes(D, r, cheb) if dom == "iter_fused" else design
    achieved = alg * N / avg_s / 1e9
    pk = res.get("prof_all") or prof
    pk_passes = res.get("passes_all") if res.get("prof_all") else res.get("passes")
    per_kernel = {}
    for k, v in pk.items():
        w = work_launches(k, v[1], pk_passes)
        per_kernel[k] = dict(ms_total=round(v[0], 3), launches=v[1], working_launches=w,
                             avg_us=round(1e3 * v[0] / max(w, 1), 2),
                             gbs=round(site_bytes(k, Q, D, s, r, warm, cheb, pull) * N / (v[0] / 1e3 / max(w, 1)) / 1e9, 1)
                             if v[1] else None)
    traffic = measured_traffic(dom, res)
    out = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, bytes_per_site=alg, launches=n,
               working_launches=work, avg_launch_us=round(avg_s * 1e6, 2))
    if alg != design:
        out.update(design_bytes_per_site=design, design_frac=round(design * N / avg_s / 1e9 / HBM_PEAK_GBS, 4))
    return out, per_kernel


def work_launches(kernel, launches, passes):
    """Launches of a kernel class that did work: for the solve pass, the
    passes the library counted (`lb2p_profile_passes`), when known."""
    if kernel in ("iter_fused", "iter_q", "iter_jt") and passes is not None and launches:
        return min(launches, passes)
    return launches


def traffic_table(res):
    """Per-kernel-class HBM bytes per launch from committed rocprofv3
    FETCH_SIZE/WRITE_SIZE counters (scaled by a plain copy kernel's reading),
    if they were taken on the current kernel source and on this workload and
    storage (profiles/traffic.json: one entry per "workload storage"); else
    None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            t = json.load(fh)
        from paper_1402_2920_amd import build as B
        if t.get("src_sha") != B.source_sha():
            return None
        key = f"{res.get('workload')} {res.get('storage')}"
        ent = t.get("workloads", {}).get(key)
        if ent is None and t.get("workload") == key:
            ent = t
        if ent is None:
            return None
        return {k: v["bytes_per_launch"] for k, v in ent["kernels"].items()}
    except Exception:
        return None


def measured_traffic(kernel, res):
    t = traffic_table(res)
    return None if t is None else t.get(kernel)


def copy_rate_gbs(nbytes=2 << 30, reps=5):
    """Streaming-copy rate of this GPU: torch's device copy of nbytes, read
    plus write bytes over HIP-event time (the practical HBM ceiling that the
    memory-bound kernels are compared with)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    rate = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return rate


def step_hbm(res, storage, warm, cheb, steps, secs, copy_gbs):
    """Whole-step bandwidth three ways, each as GB/s and as a fraction of the
    8 TB/s peak and of the measured copy rate: the population floor 2 Q s per
    site (every word read and written once), the kernels' algorithmic bytes
    (the per-site table x launches) and the counters' measured bytes."""
    prof = res["prof"]
    Q, D, N = res["Q"], res["D"], res["N"]
    s = STORE_BYTES[storage]
    r = 8 if storage == "f64" else 4
    pull = res.get("pull", False)

    def rate(total_bytes):
        gbs = total_bytes / secs / 1e9
        return dict(gbs=round(gbs, 1), frac_peak=round(gbs / HBM_PEAK_GBS, 4),
                    frac_copy=round(gbs / copy_gbs, 4) if copy_gbs else None,
                    bytes_per_site_step=round(total_bytes / (N * steps), 1))

    floor = rate(2 * Q * s * N * steps)
    work = {k: work_launches(k, v[1], res.get("passes")) for k, v in prof.items()}
    model = rate(sum(site_bytes(k, Q, D, s, r, warm, cheb, pull) * N * work[k] for k, v in prof.items() if v[1]))
    tt = traffic_table(res)
    meas = None
    if tt is not None and all(k in tt for k, v in prof.items() if v[1]):
        meas = rate(sum(tt[k] * work[k] for k, v in prof.items() if v[1]))
    return dict(peak_gbs=HBM_PEAK_GBS, copy_gbs=round(copy_gbs, 1) if copy_gbs else None,
                population_floor=floor, algorithmic=model, measured=meas,
                note="time: the whole timed region; bytes: every kernel launch in it that did work (the "
                     "solve-pass launches after the stop rule held return at once), except the residual "
                     "reductions (a few KB each)")


def cpu_baseline(workload, nsteps_max=30, budget_s=15.0):
    """Oracle MLUPS on a bounded sample of the workload (16 x 16 x nz column
    in 3D, 64 x 64 in 2D); returns (dict, sample results for the error check)."""
    from oracle import build_oracle, oracle as orc
    import lb2p_workloads as W
    build_oracle.build(force=False)
    full = tuple(W.load_params()[workload]["shape"])
    shape = (16, 16, full[2]) if len(full) == 3 else (64, 64)
    entry, shape, rho, u = W.build(workload, shape)
    d = len(shape)
    m = orc.Model(nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, tol=1e-13, max_iter=2000,
                  **W.oracle_kwargs(entry["model"]))
    n = orc.init(m, rho, u.T.copy())
    t0 = time.perf_counter()
    steps = 0
    while steps < nsteps_max and time.perf_counter() - t0 < budget_s:
        orc.step(m, n, 1)
        steps += 1
    dt = time.perf_counter() - t0
    F = orc.fields(m, n)
    N = int(np.prod(shape))
    res = dict(value=round(N * steps / dt / 1e6, 4), unit="MLUPS", cores=orc.num_threads(), kind="oracle",
               sample=f"{'x'.join(map(str, shape))} sample of the {workload} workload (same EOS, kappa, "
                      f"profile), {steps} steps, FP64, j~ from zero, tol 1e-13, {dt:.1f} s")
    return res, dict(shape=shape, steps=steps, rho=F["rho"], u=F["u"][:, :d].T.copy())


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_CORE = '''
import sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as orc
import lb2p_workloads as W
workload, budget = sys.argv[2], float(sys.argv[3])
full = tuple(W.load_params()[workload]["shape"])
shape = (16, 16, full[2]) if len(full) == 3 else (64, 64)
entry, shape, rho, u = W.build(workload, shape)
d = len(shape)
m = orc.Model(nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, tol=1e-13, max_iter=2000,
              **W.oracle_kwargs(entry["model"]))
n = orc.init(m, rho, u.T.copy())
t0 = time.perf_counter(); steps = 0
while steps < 30 and time.perf_counter() - t0 < budget:
    orc.step(m, n, 1); steps += 1
dt = time.perf_counter() - t0
print(m.N * steps / dt / 1e6, steps, orc.num_threads())
'''


def cpu_one_core(workload, budget_s=10.0):
    """The same oracle sample on one host core (OMP_NUM_THREADS=1, its own
    process): (MLUPS, steps)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    p = subprocess.run([sys.executable, "-c", _ONE_CORE, ROOT, workload, str(budget_s)], env=env,
                       capture_output=True, text=True, timeout=300)
    if p.returncode != 0:
        return None, 0
    mlups, steps, threads = p.stdout.split()[-3:]
    return (round(float(mlups), 4), int(steps)) if int(threads) == 1 else (None, 0)


def sample_errors(workload, storage, ref, iter_prec=0):
    """max and RMS error of rho and u on the cpu-baseline sample after the
    same number of steps (GPU in `storage`, at the tolerance of the timed
    runs, vs the FP64 oracle); iter_prec 2: FP64 fields at tol 1e-13."""
    import lb2p_workloads as W
    from paper_1402_2920_amd import lb2p
    entry, shape, rho, u = W.build(workload, ref["shape"])
    d = len(shape)
    P = lb2p.Params(nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1,
                    storage=lb2p.STORAGE_NAMES[storage], max_iter=500, warm_start=1, iter_prec=iter_prec,
                    tol=1e-13 if storage == "f64" or iter_prec == 2 else None, **W.model_kwargs(entry["model"]))
    with lb2p.Context(P) as ctx:
        ctx.init(rho, u)
        ctx.step(ref["steps"])
        rg, ug = ctx.moments()
    er = rg - ref["rho"]
    eu = np.sqrt(((ug - ref["u"]) ** 2).sum(axis=0))
    umag = np.sqrt((ref["u"] ** 2).sum(axis=0))
    return dict(e_rho_max=float(np.abs(er).max() / np.abs(ref["rho"]).max()),
                e_rho_rms=float(np.sqrt((er**2).mean()) / np.abs(ref["rho"]).max()),
                e_u_max=float(eu.max() / max(umag.max(), 1e-300)),
                e_u_rms=float(np.sqrt((eu**2).mean()) / max(umag.max(), 1e-300)),
                u_max=float(umag.max()), steps=ref["steps"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--storage", default="f32", choices=list(STORE_BYTES))
    ap.add_argument("--solver", default="fixed_point", choices=list(SOLVERS),
                    help="j~ solver: the paper's fixed point, or Chebyshev semi-iteration on the same map")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default block shapes")
    ap.add_argument("--warm-start", type=int, default=1, choices=(0, 1, 2, 3),
                    help="start of the j~ iteration: zero, previous step, extrapolated linearly from two "
                         "steps or quadratically from three (after the initial transient the previous step's "
                         "j~ needs the fewest passes on these workloads: extrapolation amplifies the "
                         "step-to-step fluctuation of j~)")
    ap.add_argument("--settle", type=int, default=200,
                    help="steps run before warm-up and timing: the relaxation of the synthetic start, whose "
                         "solves need more passes than the rest of the run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-whole-run", action="store_true",
                    help="skip the configuration's whole run (all its steps from the synthetic start)")
    ap.add_argument("--no-variants", action="store_true", help="skip the BF16/F16 storage lines")
    ap.add_argument("--batch-steps", type=int, default=1000,
                    help="steps of the 512-domain batched workload in one graph (0: skip)")
    # 7: the fewest fixed passes with which every domain's last residual
    # stays within the FP32 default tolerance (4e-7 of its max|j0'|)
    ap.add_argument("--batch-iters", type=int, default=7, help="fixed j~ passes per batched step")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the step would shard by z-slabs with halo exchange; not built).", file=sys.stderr)
        sys.exit(2)

    import lb2p_workloads as W
    entry = W.load_params()[args.workload]
    warm_of = lambda stg: args.warm_start
    args_warm = warm_of(args.storage)
    res = run_gpu(args.workload, args.storage, args.steps, args.warmup, solver=args.solver,
                  autotune=not args.no_autotune, warm_start=args_warm, settle=args.settle)
    N, K = res["N"], args.steps
    secs = res["seconds"]
    roof, per_kernel = roofline(res, args.storage, warm=args_warm, cheb=args.solver == "chebyshev")
    shape = res["shape"]
    line = dict(
        metric="MLUPS and % HBM peak, D3Q59 FP32 vs BF16-storage at stated error",
        value=round(N * K / secs / 1e6, 2), unit="MLUPS", n_gpus=1, steps=K, warmup=args.warmup,
        ms_per_step=round(1e3 * secs / K, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=args.storage, data="synthetic",
        config=dict(workload=f"{args.workload}: D{len(shape)}Q{res['Q']} {'x'.join(map(str, shape))} "
                             f"periodic, {entry['kind']}, {args.storage} populations",
                    sites=N, parallelism="single GPU",
                    solve=("j~ fixed point" if args.solver == "fixed_point" else "Chebyshev semi-iteration")
                    + f" to the paper's stop rule, tol {res['tol']:.0e} x max|j0'|, "
                    + ["zero start", "warm start", "extrapolated warm start", "quadratic warm start"][args_warm],
                    iters_last_step=res["stats"]["iters"],
                    timed_after_step=args.settle + args.warmup + res["prof_steps"]),
        roofline=dict(roof, note="HIP events around the dominant class only, in the timed steps"),
        kernels=per_kernel,
        kernels_note=f"HIP events around every kernel class over the {res['prof_steps']} steps right before "
                     f"the timed steps",
    )
    line["step_hbm"] = step_hbm(res, args.storage, args_warm, args.solver == "chebyshev", K, secs,
                                copy_rate_gbs())
    # the configuration's whole run from the synthetic start (the first steps
    # relax the initial walls and noise and need more solve passes)
    wsteps = entry.get("steps", 0)
    if wsteps and not args.no_whole_run:
        wr = run_gpu(args.workload, args.storage, wsteps, 0, profile=False, solver=args.solver,
                     autotune=not args.no_autotune, warm_start=args_warm, settle=0)
        line["whole_run"] = dict(steps=wsteps, value=round(N * wsteps / wr["seconds"] / 1e6, 2), unit="MLUPS",
                                 ms_per_step=round(1e3 * wr["seconds"] / wsteps, 4),
                                 note="all steps of the configuration from its synthetic start, transient "
                                      "included, one timed region")
    ref = None
    if not args.no_cpu:
        cb, ref = cpu_baseline(args.workload)
        one, one_steps = cpu_one_core(args.workload)
        cb["one_core"] = dict(value=one, unit="MLUPS", steps=one_steps)
        cb["host_cpu"] = cpu_model()
        line["cpu_baseline"] = cb
    if not args.no_variants and args.storage == "f32":
        var = {}
        other = "chebyshev" if args.solver == "fixed_point" else "fixed_point"
        for stg, sol in (("bf16", args.solver), ("f16", args.solver), ("f32", other), ("bf16", other)):
            r2 = run_gpu(args.workload, stg, K, args.warmup, solver=sol, autotune=not args.no_autotune,
                         warm_start=warm_of(stg), settle=args.settle)
            rf, _ = roofline(r2, stg, warm=warm_of(stg), cheb=sol == "chebyshev")
            var[f"{stg}_{sol}"] = dict(value=round(N * K / r2["seconds"] / 1e6, 2), unit="MLUPS",
                                       ms_per_step=round(1e3 * r2["seconds"] / K, 4),
                                       roofline_frac=rf["frac"], dominant=rf["kernel"],
                                       iters_last_step=r2["stats"]["iters"], warm_start=warm_of(stg))
        line["variants"] = var
    if args.batch_steps > 0:
        bw = "d2q21_batch512"
        bres = run_batch(bw, args.batch_steps, args.warmup, args.batch_iters)
        broof, bkern = roofline(bres, "f32", warm=1)
        bN = bres["N"]
        line["batched"] = dict(
            workload=f"{bw}: {bres['ndom']} periodic D2Q21 domains, sides 32..256, one droplet each, "
                     f"per-domain EOS (T_r 0.89..0.97) and kappa, f32 populations",
            value=round(bN * args.batch_steps / bres["seconds"] / 1e6, 2), unit="MLUPS",
            sites=bN, steps=args.batch_steps, ms_per_step=round(1e3 * bres["seconds"] / args.batch_steps, 4),
            solve=f"{args.batch_iters} j~ passes per step (fixed), all timed steps in one HIP graph launch",
            resid_over_jscale=dict(
                worst=float(f"{bres['resid_ratio'].max():.3e}"),
                worst_domain_max_j0p=float(f"{bres['resid_jscale'][int(bres['resid_ratio'].argmax())]:.3e}"),
                median=float(f"{np.median(bres['resid_ratio']):.3e}"),
                note="per domain: the last pass's residual / the domain's max|j0'| (the stop rule's two sides); "
                     "a domain whose droplet has dissolved has max|j0'| near 0 and its residual at the FP32 "
                     "floor, so its ratio grows without the iteration being any less converged"),
            max_rel_mass_drift=float(f"{bres['mass_drift']:.3e}"),
            roofline=dict(broof, note="per-kernel HIP events from 4 eager steps after the graph run"),
            kernels={k: v for k, v in bkern.items() if v["launches"]})
    if ref is not None:
        errs = {}
        stgs = [args.storage] + ([] if args.no_variants or args.storage != "f32" else ["bf16", "f16"])
        for stg in stgs:
            errs[stg] = {k: (float(f"{v:.3e}") if isinstance(v, float) else v)
                         for k, v in sample_errors(args.workload, stg, ref).items()}
        if args.storage == "f32":
            errs["f32_storage_f64_fields"] = {k: (float(f"{v:.3e}") if isinstance(v, float) else v)
                                              for k, v in sample_errors(args.workload, "f32", ref, 2).items()}
        line["errors_vs_oracle"] = errs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
