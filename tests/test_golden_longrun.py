"""The stored long-run references (tests/golden/longrun/, written by
tests/golden/make_longrun_refs.py from the FP64 oracle) are whole and
consistent with their metadata: sample indices in range and unique, one
(rho, u) record per checkpoint and sampled site, finite values, densities
inside the workloads' range and flows no larger than their stated maxima."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "longrun")


def _meta():
    with open(os.path.join(GOLD, "longrun.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name", ["slab_column", "droplet48", "batch16", "batch512_100"])
def test_reference_is_consistent(name):
    meta = _meta()[name]
    idx = np.load(os.path.join(GOLD, f"{name}_idx.npy"))
    vals = np.load(os.path.join(GOLD, f"{name}_vals.npy"))
    ncp = len(meta["checkpoints"])
    assert meta["tol"] <= 1e-13
    assert vals.shape[0] == ncp and vals.shape[2] == idx.size
    assert np.all(np.isfinite(vals))
    assert np.unique(idx).size == idx.size and idx.min() >= 0
    if name.startswith("batch"):
        assert vals.shape[1] == 3   # rho, u_x, u_y
        umax = np.array(meta["umax_per_domain"]).T      # [checkpoint][domain]
        rmax = np.array(meta["rhomax_per_domain"]).T
        assert umax.shape == (ncp, meta["ndom"])
        for k in range(ncp):
            assert np.abs(vals[k, 1:]).max() <= umax[k].max() * (1 + 1e-12)
            assert vals[k, 0].max() <= rmax[k].max() * (1 + 1e-12)
    else:
        assert vals.shape[1] == 4   # rho, u_x, u_y, u_z
        assert idx.max() < int(np.prod(meta["shape"]))
        for k in range(ncp):
            speed = np.sqrt((vals[k, 1:] ** 2).sum(0))
            assert speed.max() <= meta["umax"][k] * (1 + 1e-12)
            assert vals[k, 0].max() <= meta["rhomax"][k] * (1 + 1e-12)
    # the 3D model's coexisting densities lie inside (1.2, 1.6); the batch's
    # lowest-temperature domains reach about 1.75
    assert 1.0 < vals[:, 0].min() and vals[:, 0].max() < 1.9
