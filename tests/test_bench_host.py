"""Host-side logic of bench.py: the per-site byte model, the whole-step
bandwidth report and the single-GPU guard (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_site_bytes_d3q59_f32():
    # the per-kernel byte table of the 3D FP32 step (gamma = 0, previous-step
    # warm start): populations 58 x 4 + FP64 rest plane + 2-byte density
    # record, fields 4 B, the FP64 mass 8 B
    sb = lambda k: bench.site_bytes(k, 59, 3, 4, 4, 1)
    pops = 58 * 4 + 8 + 2
    assert sb("moments") == pops + 4 * 4 + 8 + 4 * 4
    assert sb("force") == 8 + 3 * 4 + 3 * 4 + 9 * 4
    assert sb("iter_fused") == 48
    assert sb("closure1") == 11 * 4 + 23 * 4
    assert sb("closure2") == 80
    assert sb("collide") == pops + 8 + (9 + 6 + 10) * 4
    # gamma != 0: the collision pulls the populations again
    assert bench.site_bytes("collide", 59, 3, 4, 4, 1, pull=True) == 2 * pops + 25 * 4
    # FP64 storage has no density record
    assert bench.site_bytes("moments", 59, 3, 8, 8, 1) == 58 * 8 + 8 + 4 * 8 + 8 + 4 * 8
    # Chebyshev reads u_{k-1} too
    assert bench.site_bytes("iter_fused", 59, 3, 4, 4, 1, cheb=True) == 60


def test_step_hbm_sums_launches():
    N, steps, secs = 1000, 2, 1e-3
    prof = {k: (0.0, 0) for k in ("moments", "force", "iter_q", "iter_jt", "closure1", "closure2",
                                  "collide", "iter_fused")}
    prof.update(moments=(0.1, 2), force=(0.1, 2), closure1=(0.1, 2), closure2=(0.1, 2), collide=(0.1, 2),
                iter_fused=(0.5, 26))
    res = dict(prof=prof, Q=59, D=3, N=N, workload="none", storage="f32")
    out = bench.step_hbm(res, "f32", 1, False, steps, secs, copy_gbs=5000.0)
    assert out["population_floor"]["bytes_per_site_step"] == 2 * 59 * 4
    per_step = 282 + 68 + 136 + 80 + 350 + 13 * 48
    assert out["algorithmic"]["bytes_per_site_step"] == per_step
    gbs = per_step * N * steps / secs / 1e9
    assert out["algorithmic"]["gbs"] == pytest.approx(gbs, abs=0.1)
    assert out["algorithmic"]["frac_peak"] == pytest.approx(gbs / 8000.0, abs=1e-4)
    assert out["algorithmic"]["frac_copy"] == pytest.approx(gbs / 5000.0, abs=1e-4)
    # no committed counters for this workload: measured stays null
    assert out["measured"] is None


def test_roofline_solve_pass_on_its_minimal_bytes():
    # the solve pass is priced on the bytes a pass cannot do without, rho,
    # j0' and the iterate in and out: (1 + 3D) r, 40 B in 3D FP32, 28 B in 2D
    assert bench.minimal_pass_bytes(3, 4) == 40
    assert bench.minimal_pass_bytes(2, 4) == 28
    assert bench.minimal_pass_bytes(3, 4, cheb=True) == 52
    N = 1 << 20
    prof = {k: (0.0, 0) for k in ("moments", "force", "closure1", "closure2", "collide")}
    prof.update(collide=(1.0, 1), iter_fused=(2.0, 10))
    res = dict(prof=prof, Q=59, D=3, N=N, workload="none", storage="f32")
    roof, _ = bench.roofline(res, "f32", warm=1)
    assert roof["kernel"] == "iter_fused" and roof["bytes_per_site"] == 40
    assert roof["design_bytes_per_site"] == 48
    assert roof["achieved"] == pytest.approx(40 * N / 200e-6 / 1e9, abs=0.1)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0, abs=1e-4)
    # another dominant kernel keeps its own algorithmic bytes
    prof.update(collide=(5.0, 1))
    roof, _ = bench.roofline(dict(res, prof=prof), "f32", warm=1)
    assert roof["kernel"] == "collide" and roof["bytes_per_site"] == 350 and "design_bytes_per_site" not in roof


def test_solve_pass_priced_per_working_pass():
    # launches after the stop rule held return at once: the solve pass's
    # average is taken over the passes that did work, when they are known
    N = 1 << 20
    prof = {k: (0.0, 0) for k in ("moments", "force", "closure1", "closure2", "collide")}
    prof.update(collide=(1.0, 5), iter_fused=(4.0, 29))
    res = dict(prof=prof, Q=59, D=3, N=N, workload="none", storage="f32", passes=25)
    roof, kern = bench.roofline(res, "f32", warm=1)
    assert roof["kernel"] == "iter_fused" and roof["launches"] == 29 and roof["working_launches"] == 25
    assert roof["avg_launch_us"] == pytest.approx(4000.0 / 25, abs=0.01)
    assert kern["iter_fused"]["working_launches"] == 25 and kern["collide"]["working_launches"] == 5
    # without the count, every launch counts
    roof, _ = bench.roofline(dict(res, passes=None), "f32", warm=1)
    assert roof["working_launches"] == 29
    assert bench.work_launches("collide", 5, 3) == 5
    assert bench.work_launches("iter_fused", 29, 40) == 29


def test_traffic_table_matches_workload_only():
    res = dict(workload="no_such_workload", storage="f32")
    assert bench.traffic_table(res) is None
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(path):
        with open(path) as fh:
            t = json.load(fh)
        from paper_1402_2920_amd import build as B
        for key, ent in t["workloads"].items():
            wl, stg = key.split()
            tt = bench.traffic_table(dict(workload=wl, storage=stg))
            if t["src_sha"] == B.source_sha():
                assert tt is not None and tt["iter_fused"] == ent["kernels"]["iter_fused"]["bytes_per_launch"]
            else:
                assert tt is None
        # another storage of a profiled workload has no entry
        wl = next(iter(t["workloads"])).split()[0]
        assert bench.traffic_table(dict(workload=wl, storage="f64")) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
