"""Write lb2p_workloads/params.json: the model parameters of every synthetic
workload, derived with the oracle's equation-of-state tools only.

For each workload: the App. B EOS (rho1, rho2, A, c_s^2(rho1)), the Maxwell
coexistence densities rho_g, rho_l (App. B), the interfacial stiffness kappa
for a planar tanh profile of width 3, gamma = 0 and rho0 = rho1.

The EOS scale and amplitude are chosen inside App. B's admissible set AND
where the full step stays stable over thousands of steps with interfaces
present (the paper reports no runs; the model is unstable for deeper
quenches, larger c_s^2 or larger gamma, see the design notes):
  2D: rho1 0.3, rho2 1, c_s^2(rho1) 0.45, A 0.80 (5000 steps of the 64^2
      droplet stay bounded);
  3D: rho1 0.3, rho2 1, c_s^2(rho1) 0.39, A 0.74 (T_r 0.988; a droplet, a
      slab and two colliding droplets stay bounded for 3000 steps, while
      A >= 0.76 diverges within 250 steps);
  batched 2D: reduced temperature T_r = A_c / A uniform in [0.89, 0.97].

Run:  python tests/golden/make_workload_params.py
"""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import eos_tools as E  # noqa: E402
from oracle import oracle as O  # noqa: E402
import lb2p_workloads as W  # noqa: E402

WIDTH = 3.0
EOS2 = dict(rho1=0.3, rho2=1.0, cs2_1=0.45, A=0.80)
EOS3 = dict(rho1=0.3, rho2=1.0, cs2_1=0.39, A=0.74)
TR_RANGE = (0.89, 0.97)


def model_entry(Q, eos):
    m = O.Model(Q=Q, nx=8, ny=8, nz=8 if Q == 59 else 1, **eos)
    adm = E.admissibility(m)
    assert adm["weights_positive"] and adm["two_phase"] and adm["bulk_viscosity_positive"], adm
    kappa, info = E.kappa_for_width(m, WIDTH)
    return dict(lattice=Q, gamma=0.0, kappa=kappa, rho0=eos["rho1"], eos=dict(eos),
                rho_g=info["rho_g"], rho_l=info["rho_l"], p_c=info["p_c"], width=WIDTH,
                A_c=E.critical_amplitude(m))


def main():
    out = {}
    m2 = model_entry(21, EOS2)
    m3 = model_entry(59, EOS3)
    out["d2q21_64_droplet"] = dict(model=m2, shape=[64, 64], kind="droplet", radius=16.0,
                                   noise=1e-3, seed=1403, steps=1000, storage="f64")
    out["d3q59_128_droplet"] = dict(model=m3, shape=[128, 128, 128], kind="droplet", radius=32.0,
                                    noise=1e-3, seed=1404, steps=1000, storage="f32")
    out["d3q59_256_slab"] = dict(model=m3, shape=[256, 256, 256], kind="slab", z_lo=64, z_hi=192,
                                 noise=1e-3, seed=1405, steps=2000, storage="f32")
    out["d3q59_512_two_droplets"] = dict(model=m3, shape=[512, 512, 512], kind="two_droplets",
                                         radius=64.0, separation=150.0, speed=0.02, noise=1e-3,
                                         seed=1406, steps=500, storage="f32")
    # batched 2D: 512 domains
    doms = W.batch_domains(512, 32, 256, seed=1402000)
    base = O.Model(Q=21, nx=8, ny=8, **EOS2)
    A_c = E.critical_amplitude(base)
    batch = []
    for k, dd in enumerate(doms):
        tr = TR_RANGE[0] + (TR_RANGE[1] - TR_RANGE[0]) * dd["t_unit"]
        eos = dict(EOS2, A=A_c / tr)
        e = model_entry(21, eos)
        e.update(nx=dd["nx"], ny=dd["ny"], radius=dd["radius"], T_r=tr, seed=1402000 + k)
        batch.append(e)
    out["d2q21_batch512"] = dict(kind="batch", domains=batch, noise=1e-3, steps=1000, storage="f32",
                                 T_r_range=list(TR_RANGE))
    with open(W.PARAMS_PATH, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", W.PARAMS_PATH)


if __name__ == "__main__":
    main()
