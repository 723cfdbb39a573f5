"""Stability of the 3D model on the FP64 oracle, the evidence for the
near-critical EOS of the 3D workloads: D3Q59 32^3 periodic boxes, a droplet
(radius 8, the 128^3 droplet workload scaled) and a liquid slab (z in
[8, 24)), interfaces of tanh width 3 between the Maxwell coexistence
densities, kappa for that width, gamma = 0, rho0 = rho1, noise 1e-3; each
run to 2000 steps or until it diverges (a non-finite density or max|u| > 0.1,
from a start at rest).  Parameter sets: the workloads' A = 0.74,
c_s^2(rho1) = 0.39; A = 0.76 at the same c_s^2; and A = 0.90,
c_s^2(rho1) = 0.45 (a deeper quench at a larger sound speed).

Calls the oracle only; writes tests/golden/stability_3d.json.
Run:  python tests/golden/oracle_stability_3d.py
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
from oracle import eos_tools as E  # noqa: E402
from oracle import oracle as O  # noqa: E402
import lb2p_workloads as W  # noqa: E402

SETS = [("A0.74_cs0.39", 0.74, 0.39), ("A0.76_cs0.39", 0.76, 0.39), ("A0.90_cs0.45", 0.90, 0.45)]
SHAPE = (32, 32, 32)
STEPS = 2000


def run(A, cs2, kind):
    m0 = O.Model(Q=59, nx=8, ny=8, nz=8, rho1=0.3, rho2=1.0, A=A, cs2_1=cs2)
    kappa, info = E.kappa_for_width(m0, 3.0)
    if kind == "droplet":
        rho, u = W.droplet(SHAPE, 8.0, info["rho_g"], info["rho_l"], width=3.0, noise=1e-3, seed=1404)
    else:
        rho, u = W.slab(SHAPE, 8, 24, info["rho_g"], info["rho_l"], width=3.0, noise=1e-3, seed=1405)
    m = O.Model(Q=59, nx=SHAPE[0], ny=SHAPE[1], nz=SHAPE[2], rho1=0.3, rho2=1.0, A=A, cs2_1=cs2,
                kappa=kappa, rho0=0.3, tol=1e-13, max_iter=3000)
    n = O.init(m, rho, u.T.copy())
    umax_hist = []
    for s in range(1, STEPS + 1):
        _, inf = O.step(m, n, 1)
        if s % 50 == 0 or s < 50:
            F = O.fields(m, n)
            umax = float(np.abs(F["u"]).max()) if np.isfinite(F["u"]).all() else float("inf")
            if s % 50 == 0:
                umax_hist.append((s, umax))
            if not np.isfinite(F["rho"]).all() or not umax < 0.1 or not inf["converged"]:
                return dict(diverged_at=s, umax=umax_hist, kappa=kappa, rho_g=info["rho_g"],
                            rho_l=info["rho_l"], converged=inf["converged"])
    return dict(diverged_at=None, umax=umax_hist, kappa=kappa, rho_g=info["rho_g"], rho_l=info["rho_l"])


def main():
    build_oracle.build(force=False)
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stability_3d.json")
    res = json.load(open(out_path)) if os.path.exists(out_path) else {}
    for name, A, cs2 in SETS:
        for kind in ("slab", "droplet"):
            key = f"{name} {kind}"
            if key in res:
                continue
            t0 = time.time()
            r = run(A, cs2, kind)
            r["seconds"] = round(time.time() - t0, 1)
            res[key] = r
            print(key, "diverged at", r["diverged_at"], f"({r['seconds']} s)", flush=True)
            with open(out_path, "w") as fh:
                json.dump(dict(res, shape=list(SHAPE), steps=STEPS, threads=O.num_threads()), fh, indent=1)


if __name__ == "__main__":
    main()
