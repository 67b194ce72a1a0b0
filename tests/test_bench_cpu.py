"""Host-side accounting of bench.py (CPU): size buckets, the voxels each solver
family's launch takes, the algorithmic work per voxel, the arithmetic label and
the guard on stored counter readings."""
import json

import numpy as np

import bench


def test_bucket_boundaries():
    n = np.array([1, 16, 17, 32, 33, 64, 65, 96, 97, 128, 129, 256, 257, 512])
    assert bench.bucket_of(n).tolist() == [0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6, 6]


def test_family_buckets_follow_the_launch_choices():
    tun = {"tiled_merge": 0, "tile_first_bucket": 3}
    assert bench.family_buckets("fit_f64_n512", tun, 512) == (6,)
    assert bench.family_buckets("fit_f64_n256", tun, 512) == (5,)
    merged = dict(tun, tiled_merge=1)
    # the merged launch takes the 256-point bucket's voxels too
    assert bench.family_buckets("fit_f64_n512", merged, 512) == (5, 6)
    assert bench.family_buckets("fit_mix_n512", merged, 512) == (5, 6)
    # ... but not when the 512-point bucket is not launched, nor for the FP64 re-solve family
    assert bench.family_buckets("fit_f64_n512", merged, 256) == (6,)
    assert bench.family_buckets("refine_f64_n512", merged, 512) == (6,)
    # nor when the 256-point bucket is not a tiled one
    assert bench.family_buckets("fit_f64_n512", dict(merged, tile_first_bucket=6), 512) == (6,)
    assert bench.family_buckets("fit_f32_n16", merged, 512) == (0,)


def test_voxel_flops_and_bytes():
    n, m = np.array([1, 10]), 4
    # n^3/3 + n^2 m + 2 n^2 + 4 n m + 6 (n^2/2 + n m)
    expect = [1 / 3 + 4 + 2 + 16 + 6 * (0.5 + 4), 1000 / 3 + 400 + 200 + 160 + 6 * (50 + 40)]
    assert np.allclose(bench.voxel_flops(n, m), expect, rtol=0, atol=1e-9)
    assert bench.voxel_bytes(np.array([10]), 4).tolist() == [12 * 10 + 16 + 16 * 4 + 2]


def test_precision_split_labels():
    n = np.array([10, 20, 300])
    solved = np.array([True, True, True])
    tun = {"tile_first_bucket": 3, "fp32_last_bucket": 0}
    fl = bench.voxel_flops(n, 16)
    sp = bench.precision_split(n, solved, 16, tun, "fp32")
    assert sp["dtype"] == "f64"
    assert np.isclose(sp["flop_share"]["f32"], fl[0] / fl.sum())
    assert bench.precision_split(n, solved, 16, tun, "fp64")["flop_share"] == {"f64": 1.0}
    # MIXED: the tiled bucket's tiles are FP32
    mx = bench.precision_split(n, solved, 16, tun, "mixed")
    assert np.isclose(mx["flop_share"]["f32"], (fl[0] + fl[2]) / fl.sum())


def test_stored_traffic_needs_matching_sources_and_choices(tmp_path, monkeypatch):
    tun = {"streams": 3}
    rec = {"source_hash": bench.source_hash(), "tuning": tun, "precision": "fp32",
           "families": {"fit_f64_n512": {"bytes_per_launch": 123.0}}}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setitem(bench.TRAFFIC_FILES, "aggregated", str(f))
    assert bench.measured_traffic("aggregated", "fit_f64_n512", tun, "fp32") == 123.0
    assert bench.measured_traffic("aggregated", "fit_f64_n512", {"streams": 1}, "fp32") is None
    assert bench.measured_traffic("aggregated", "fit_f64_n512", tun, "fp64") is None
    f.write_text(json.dumps(dict(rec, source_hash="0" * 16)))
    assert bench.measured_traffic("aggregated", "fit_f64_n512", tun, "fp32") is None
