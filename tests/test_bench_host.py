"""Host-side logic of bench.py (no GPU): the algorithmic byte counts per kernel, the lookup of the
counter-measured traffic in profiles/, and the single-GPU contract."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    import bench as b
    return b


def test_kernel_bytes(bench):
    # fields moved per point by each TTI launch (FP32): two-pass six-field, fused, two-pass
    # four-field, split
    assert bench.kernel_bytes(0, 0) == 10 * 4 and bench.kernel_bytes(1, 0) == 15 * 4
    assert bench.kernel_bytes(1, 0, adjoint=True) == 17 * 4
    assert bench.kernel_bytes(0, 4) == 4 * 4 and bench.kernel_bytes(1, 4) == 12 * 4
    assert bench.kernel_bytes(1, 4, adjoint=True) == 15 * 4
    assert bench.kernel_bytes(1, 2) == 11 * 4 == bench.METHOD_BYTES_PER_PT["tti"]
    assert bench.kernel_bytes(1, 2, adjoint=True) == 15 * 4
    # four-field: pass 1 reads u, v, n_x, n_y and writes t (3) and n . grad v; pass 2 reads n_x, n_y
    # in place of s_x, s_y, so it moves what the six-field pass 2 moves
    assert bench.kernel_bytes(0, 3) == 8 * 4 and bench.kernel_bytes(0, 3, adjoint=True) == 8 * 4
    assert bench.kernel_bytes(1, 3) == bench.kernel_bytes(1, 0)
    assert bench.kernel_bytes(1, 3, adjoint=True) == bench.kernel_bytes(1, 0, adjoint=True)
    assert bench.kernel_bytes(2) == 13 * 4 and bench.kernel_bytes(3) == 17 * 4
    assert bench.kernel_bytes(4) == 21 * 4 == bench.METHOD_BYTES_PER_PT["elastic"]


def test_traffic_lookup_follows_the_committed_counters(bench):
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as fh:
        rec = json.load(fh)
    npts = 512 ** 3
    for key, ent in rec.items():
        if key == "calibration":
            continue
        kclass, scheme, so = key.split("/")
        got = bench.traffic_from_profiles(int(kclass), npts, int(scheme), ent["tile"], int(so[2:]))
        # counters taken on another kernel source are not reported
        fresh = ent["source_hash"] == bench.kernel_source_hash(int(scheme))
        assert got == (ent["bytes_per_launch"] if fresh else None), key
        assert ent["bytes_per_launch"] > bench.kernel_bytes(int(kclass), int(scheme)) * npts   # halos
        assert bench.traffic_from_profiles(int(kclass), npts, int(scheme), [9, 9], int(so[2:])) is None
        assert bench.traffic_from_profiles(int(kclass), npts + 1, int(scheme), ent["tile"], int(so[2:])) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_fast_model_recipe_is_seeded_and_in_range():
    """The fast FP32 recipe used for the 64-shot model: the same arrays for any thread count, the
    parameter ranges of the default recipe, epsilon >= delta, and a layered velocity trend."""
    import numpy as np
    from paper_2004_10519_amd import inputs
    a = inputs.tti_model((48, 40, 96), 8, 4, parallel=3)
    b = inputs.tti_model((48, 40, 96), 8, 4, parallel=5)
    for k in a:
        assert a[k].dtype == np.float32 and a[k].shape == (96, 40, 48)
        assert np.array_equal(a[k], b[k]), k
    assert a["vp"].min() >= 1500.0 * 0.95 - 1e-3 and a["vp"].max() <= 4500.0 * 1.05 + 1e-3
    assert a["eps"].min() == 0.0 and abs(a["eps"].max() - 0.3) < 1e-6
    assert np.all(a["eps"] >= a["delta"])
    for k in ("theta", "phi"):
        assert abs(np.abs(a[k]).max() - np.pi / 4) < 1e-6
    vz = a["vp"].mean(axis=(1, 2))
    assert vz[-10:].mean() > vz[:10].mean() + 1000.0
    m = inputs.slowness_squared(a["vp"], threads=4)
    assert np.array_equal(m, inputs.slowness_squared(a["vp"]))
