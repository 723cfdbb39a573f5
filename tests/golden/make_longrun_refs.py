"""Write the FP64 oracle references of the long-run GPU tests
(tests/golden/longrun/): the workloads at their stated run lengths, on grids
the oracle finishes in minutes.

Cases (inputs from lb2p_workloads, the same builders the GPU side uses):
  slab_column  D3Q59 16 x 16 x 256 column of the 256^3 slab workload,
               2000 steps, references at steps 500, 1000 and 2000;
  droplet48    D3Q59 48^3 reduction of the 128^3 droplet workload (radius
               scaled to 12), 1000 steps, references at 100 and 1000;
  batch16      the first 16 domains of the 512-domain D2Q21 batch (their own
               EOS and kappa), 1000 steps, references at 100 and 1000;
  batch512_100 all 512 domains of the batch, 100 steps, reference at 100.
Each reference keeps rho and u at a seeded sample of sites (every site of
8 sampled (x, y) columns for the slab, 4096 sites for the droplet, 512 per
domain for batch16, 32 per domain for batch512_100) plus max|u| and max rho over all sites, the scales of
the relative errors.  The oracle runs its own stop rule from a zero start
(tol 1e-13).

Calls the oracle only.  Run:  python tests/golden/make_longrun_refs.py [case ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import build_oracle  # noqa: E402
from oracle import oracle as O  # noqa: E402
import lb2p_workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "longrun")
TOL = 1e-13


def sample_slab(shape, rng):
    nx, ny, nz = shape
    cols = rng.choice(nx * ny, size=8, replace=False)
    return np.sort(np.concatenate([c + nx * ny * np.arange(nz) for c in cols]))


def run_single(case, workload, shape, checkpoints, nsample):
    entry, shape, rho, u = W.build(workload, shape)
    d = len(shape)
    m = O.Model(nx=shape[0], ny=shape[1], nz=shape[2] if d == 3 else 1, tol=TOL, max_iter=4000,
                **W.oracle_kwargs(entry["model"]))
    rng = np.random.default_rng(1402 + len(case))
    idx = sample_slab(shape, rng) if case == "slab_column" else np.sort(
        rng.choice(m.N, size=nsample, replace=False))
    n = O.init(m, rho, u.T.copy())
    vals, umax, rmax = [], [], []
    done, t0 = 0, time.time()
    for c in checkpoints:
        O.step(m, n, c - done)
        done = c
        F = O.fields(m, n)
        assert F["converged"]
        uu = F["u"][:, :d]
        vals.append(np.concatenate([F["rho"][idx][None], uu[idx].T], axis=0))
        umax.append(float(np.sqrt((uu**2).sum(axis=1)).max()))
        rmax.append(float(F["rho"].max()))
        print(f"{case}: step {c} done, {time.time() - t0:.0f} s", flush=True)
    np.save(os.path.join(OUT, f"{case}_idx.npy"), idx.astype(np.int64))
    np.save(os.path.join(OUT, f"{case}_vals.npy"), np.stack(vals))
    return dict(workload=workload, shape=list(shape), checkpoints=checkpoints, umax=umax, rhomax=rmax,
                tol=TOL, oracle_seconds=round(time.time() - t0, 1), threads=O.num_threads())


def _batch_domain(args):
    """One domain of a batch case (runs in a worker process)."""
    k, ndom, checkpoints, idx = args
    entry = W.load_params()["d2q21_batch512"]
    dd = entry["domains"][k]
    shape = (dd["nx"], dd["ny"])
    rho, u = W.droplet(shape, dd["radius"], dd["rho_g"], dd["rho_l"], width=dd["width"], noise=entry["noise"],
                       seed=dd["seed"])
    m = O.Model(nx=shape[0], ny=shape[1], nz=1, tol=TOL, max_iter=4000, **W.oracle_kwargs(dd))
    n = O.init(m, rho, u.T.copy())
    done, vv, um, rm = 0, [], [], []
    for c in checkpoints:
        O.step(m, n, c - done)
        done = c
        F = O.fields(m, n)
        assert F["converged"]
        uu = F["u"][:, :2]
        vv.append(np.concatenate([F["rho"][idx][None], uu[idx].T], axis=0))
        um.append(float(np.sqrt((uu**2).sum(axis=1)).max()))
        rm.append(float(F["rho"].max()))
    return k, shape, np.stack(vv), um, rm


def run_batch(case, ndom, checkpoints, per_dom, workers=1):
    """Domains one by one (the oracle's threads within each) or, with
    workers > 1, one domain per single-threaded worker process."""
    doms = W.build_batch("d2q21_batch512", limit=ndom)
    rng = np.random.default_rng(1402016)
    idxs = []
    for dd, shape, rho, u in doms:
        N = shape[0] * shape[1]
        idxs.append(np.sort(rng.choice(N, size=min(per_dom, N), replace=False)))
    t0 = time.time()
    jobs = [(k, ndom, checkpoints, idxs[k]) for k in range(len(doms))]
    results = [None] * len(doms)
    if workers > 1:
        import multiprocessing as mp
        os.environ["OMP_NUM_THREADS"] = "1"
        with mp.get_context("spawn").Pool(workers) as pool:
            for r in pool.imap_unordered(_batch_domain, jobs):
                results[r[0]] = r
                print(f"{case}: domain {r[0]} {r[1]} done, {time.time() - t0:.0f} s", flush=True)
    else:
        for j in jobs:
            r = _batch_domain(j)
            results[r[0]] = r
            print(f"{case}: domain {r[0]} {r[1]} done, {time.time() - t0:.0f} s", flush=True)
    idx_all, vals_dom, umax, rmax = [], [], [], []
    off = 0
    for k, (dd, shape, rho, u) in enumerate(doms):
        _, _, vv, um, rm = results[k]
        idx_all.append(idxs[k] + off)
        vals_dom.append(vv)                    # [ncp, 3, nsample_dom]
        umax.append(um)
        rmax.append(rm)
        off += shape[0] * shape[1]
    np.save(os.path.join(OUT, f"{case}_idx.npy"), np.concatenate(idx_all).astype(np.int64))
    np.save(os.path.join(OUT, f"{case}_vals.npy"), np.concatenate(vals_dom, axis=2))
    return dict(workload="d2q21_batch512", ndom=ndom, checkpoints=checkpoints,
                umax_per_domain=umax, rhomax_per_domain=rmax, per_domain_sample=per_dom, tol=TOL,
                oracle_seconds=round(time.time() - t0, 1),
                threads=1 if workers > 1 else O.num_threads(), workers=workers)


CASES = {
    "slab_column": lambda: run_single("slab_column", "d3q59_256_slab", (16, 16, 256), [500, 1000, 2000], 0),
    "droplet48": lambda: run_single("droplet48", "d3q59_128_droplet", (48, 48, 48), [100, 1000], 4096),
    "batch16": lambda: run_batch("batch16", 16, [100, 1000], 512),
    "batch512_100": lambda: run_batch("batch512_100", 512, [100], 32, workers=8),
}


def main():
    build_oracle.build(force=False)
    os.makedirs(OUT, exist_ok=True)
    meta_path = os.path.join(OUT, "longrun.json")
    meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
    for name in (sys.argv[1:] or list(CASES)):
        meta[name] = CASES[name]()
        with open(meta_path, "w") as fh:
            json.dump(meta, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
