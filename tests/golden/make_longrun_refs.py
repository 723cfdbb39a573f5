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


def run_batch(case, ndom, checkpoints, per_dom):
    doms = W.build_batch("d2q21_batch512", limit=ndom)
    rng = np.random.default_rng(1402016)
    idx_all, vals_dom, umax, rmax = [], [], [], []
    t0 = time.time()
    off = 0
    for k, (dd, shape, rho, u) in enumerate(doms):
        m = O.Model(nx=shape[0], ny=shape[1], nz=1, tol=TOL, max_iter=4000, **W.oracle_kwargs(dd))
        idx = np.sort(rng.choice(m.N, size=min(per_dom, m.N), replace=False))
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
        idx_all.append(idx + off)
        vals_dom.append(np.stack(vv))          # [ncp, 3, nsample_dom]
        umax.append(um)
        rmax.append(rm)
        off += m.N
        print(f"{case}: domain {k} {shape} done, {time.time() - t0:.0f} s", flush=True)
    np.save(os.path.join(OUT, f"{case}_idx.npy"), np.concatenate(idx_all).astype(np.int64))
    np.save(os.path.join(OUT, f"{case}_vals.npy"), np.concatenate(vals_dom, axis=2))
    return dict(workload="d2q21_batch512", ndom=ndom, checkpoints=checkpoints,
                umax_per_domain=umax, rhomax_per_domain=rmax, per_domain_sample=per_dom, tol=TOL,
                oracle_seconds=round(time.time() - t0, 1), threads=O.num_threads())


CASES = {
    "slab_column": lambda: run_single("slab_column", "d3q59_256_slab", (16, 16, 256), [500, 1000, 2000], 0),
    "droplet48": lambda: run_single("droplet48", "d3q59_128_droplet", (48, 48, 48), [100, 1000], 4096),
    "batch16": lambda: run_batch("batch16", 16, [100, 1000], 512),
    "batch512_100": lambda: run_batch("batch512_100", 512, [100], 32),
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
