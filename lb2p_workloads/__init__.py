"""Seeded synthetic initial conditions shared by the tests, the smoke check
and the benchmark.

This module holds no arithmetic of the lattice Boltzmann method: it builds
density and velocity fields (tanh interfaces between two given densities plus
uniform noise) and reads the per-workload model parameters from
``params.json``.  That file is written by ``tests/golden/make_workload_params.py``
from the oracle's equation-of-state tools (coexistence densities by the Maxwell
construction of App. B, interfacial stiffness for a given tanh width).

Layout: site index x + nx*(y + ny*z); rho is [N], u is [d][N].
Noise: numpy PCG64 with the given seed, uniform in [-amp, amp), added to rho
in site order.
"""
from __future__ import annotations

import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(_HERE, "params.json")


def load_params() -> dict:
    with open(PARAMS_PATH) as fh:
        return json.load(fh)


def _grid(shape):
    """Coordinates of every site, x fastest."""
    if len(shape) == 2:
        nx, ny = shape
        y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                           indexing="ij")
        return [x.ravel(), y.ravel()]
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return [x.ravel(), y.ravel(), z.ravel()]


def _min_image(d, n):
    return (d + 0.5 * n) % n - 0.5 * n


def _noise(rho, amp, seed):
    if amp > 0:
        rng = np.random.default_rng(seed)
        rho = rho + rng.uniform(-amp, amp, size=rho.size)
    return rho


def droplet(shape, radius, rho_g, rho_l, width=3.0, centre=None, noise=1e-3, seed=1403):
    """Circle (2D) or sphere (3D) of liquid in gas, periodic minimum-image
    distance, rho = mean + (drho/2) tanh((R - |r - r_c|)/width); u = 0."""
    coords = _grid(shape)
    if centre is None:
        centre = [0.5 * n for n in shape]
    r2 = sum(_min_image(c - c0, n) ** 2 for c, c0, n in zip(coords, centre, shape))
    dist = np.sqrt(r2)
    rho = 0.5 * (rho_g + rho_l) + 0.5 * (rho_l - rho_g) * np.tanh((radius - dist) / width)
    rho = _noise(rho, noise, seed)
    u = np.zeros((len(shape), rho.size))
    return rho, u


def slab(shape, z_lo, z_hi, rho_g, rho_l, width=3.0, noise=1e-3, seed=1404):
    """Liquid for z in [z_lo, z_hi) in gas (two tanh walls, periodic in z)."""
    coords = _grid(shape)
    z = coords[-1]
    n = shape[-1]
    mid = 0.5 * (z_lo + z_hi)
    half = 0.5 * (z_hi - z_lo)
    dist = np.abs(_min_image(z - mid + 0.5, n))   # distance from the slab centre plane
    rho = 0.5 * (rho_g + rho_l) + 0.5 * (rho_l - rho_g) * np.tanh((half - dist) / width)
    rho = _noise(rho, noise, seed)
    u = np.zeros((len(shape), rho.size))
    return rho, u


def two_droplets(shape, radius, separation, rho_g, rho_l, speed, width=3.0, noise=1e-3, seed=1405):
    """Two spheres on the x axis through the box centre, separation apart,
    moving towards each other with +-speed along x, each velocity weighted by
    that droplet's tanh liquid fraction."""
    coords = _grid(shape)
    cx = 0.5 * shape[0]
    centres = [[cx - 0.5 * separation] + [0.5 * n for n in shape[1:]],
               [cx + 0.5 * separation] + [0.5 * n for n in shape[1:]]]
    phi = []
    for c0 in centres:
        r2 = sum(_min_image(c - c_, n) ** 2 for c, c_, n in zip(coords, c0, shape))
        phi.append(0.5 * (1.0 + np.tanh((radius - np.sqrt(r2)) / width)))
    frac = np.clip(phi[0] + phi[1], 0.0, 1.0)
    rho = rho_g + (rho_l - rho_g) * frac
    rho = _noise(rho, noise, seed)
    u = np.zeros((len(shape), rho.size))
    u[0] = speed * phi[0] - speed * phi[1]
    return rho, u


def batch_domains(n_domains, side_lo, side_hi, seed=1402000):
    """Per-domain (nx, ny) drawn uniformly from [side_lo, side_hi] and a radius
    fraction uniform in [0.15, 0.35] (one droplet per domain)."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(side_lo, side_hi + 1, size=n_domains)
    ny = rng.integers(side_lo, side_hi + 1, size=n_domains)
    frac = rng.uniform(0.15, 0.35, size=n_domains)
    tr = rng.uniform(0.0, 1.0, size=n_domains)
    return [dict(nx=int(a), ny=int(b), radius=float(f * min(a, b)), t_unit=float(t))
            for a, b, f, t in zip(nx, ny, frac, tr)]


def model_kwargs(model: dict) -> dict:
    """lb2p.Params keyword arguments of a params.json model entry."""
    e = model["eos"]
    return dict(lattice=model["lattice"], gamma=model["gamma"], kappa=model["kappa"], rho1=e["rho1"],
                rho2=e["rho2"], A=e["A"], cs2_rho1=e["cs2_1"], rho0=model["rho0"])


def oracle_kwargs(model: dict) -> dict:
    """Oracle Model keyword arguments of a params.json model entry."""
    e = model["eos"]
    return dict(Q=model["lattice"], gamma=model["gamma"], kappa=model["kappa"], rho1=e["rho1"],
                rho2=e["rho2"], A=e["A"], cs2_1=e["cs2_1"], rho0=model["rho0"])


def build(name: str, shape=None):
    """(entry, shape, rho, u) of a named workload; `shape` overrides the grid
    (the initial condition keeps its geometry relative to the box: droplet
    radius and slab walls scale with the box)."""
    entry = load_params()[name]
    full = tuple(entry["shape"])
    shape = tuple(shape) if shape is not None else full
    scale = shape[-1] / full[-1]
    m = entry["model"]
    if entry["kind"] == "droplet":
        rho, u = droplet(shape, entry["radius"] * min(shape) / min(full), m["rho_g"], m["rho_l"],
                         width=m["width"], noise=entry["noise"], seed=entry["seed"])
    elif entry["kind"] == "slab":
        rho, u = slab(shape, entry["z_lo"] * scale, entry["z_hi"] * scale, m["rho_g"], m["rho_l"],
                      width=m["width"], noise=entry["noise"], seed=entry["seed"])
    elif entry["kind"] == "two_droplets":
        sx = shape[0] / full[0]
        rho, u = two_droplets(shape, entry["radius"] * sx, entry["separation"] * sx, m["rho_g"],
                              m["rho_l"], entry["speed"], width=m["width"], noise=entry["noise"],
                              seed=entry["seed"])
    else:
        raise ValueError(name)
    return entry, shape, rho, u


def build_batch(name: str, limit=None):
    """[(model, shape, rho, u)] of a batched workload: one droplet per domain
    (the domain's own EOS, kappa and radius), noise seeded per domain."""
    entry = load_params()[name]
    if entry["kind"] != "batch":
        raise ValueError(name)
    out = []
    for d in entry["domains"][:limit]:
        shape = (d["nx"], d["ny"])
        rho, u = droplet(shape, d["radius"], d["rho_g"], d["rho_l"], width=d["width"],
                         noise=entry["noise"], seed=d["seed"])
        out.append((d, shape, rho, u))
    return out
