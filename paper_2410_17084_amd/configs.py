"""Workload presets: hyper-parameters and input recipes of the synthetic workloads.

Plain data only. Each preset names the scan generator and the Voxel-GPR
hyper-parameters it runs with. Values the paper fixes come from its Table S6
(voxel 0.2 m, tau 10, n_s = n_r = 3, eta 0.3) and Sec. 3.1 (lambda = 1); the
rest are the synthetic workloads' own choices (length scale half a voxel,
noise variance 1e-3 m^2, tau 3 for the single-scan workloads).
"""
from __future__ import annotations

WORKLOADS = {
    # 20k points on 3 tilted planes in a 20 m cube; the small case the oracle
    # finishes in seconds.
    "planes": dict(
        desc="planes: 20k points on 3 random planes in a 20 m cube + N(0, 0.02 m) normal noise, "
             "voxel 1 m, cap 32, tau 3, 4x4 grid",
        voxel_size=1.0, max_pts=32, min_pts=3, grid_side=4, signal_var=1.0, length_scale=0.5, noise_var=1e-3,
        converge_var=0.3),
    # one 32-beam x 1800-azimuth spinning scan of the box scene.
    "spin32": dict(
        desc="spin32: 32-beam x 1800-azimuth spinning scan (57.6k rays, about 40k returns) of a 100 m box "
             "scene, range noise N(0, 0.02 m), voxel 0.5 m, cap 128, tau 3, 8x8 grid",
        voxel_size=0.5, max_pts=128, min_pts=3, grid_side=8, signal_var=1.0, length_scale=0.25, noise_var=1e-3,
        converge_var=0.3, n_beams=32, n_az=1800),
    # paper-shaped serving streams: voxel 0.2 m, tau 10, n_s = n_r = 3.
    "paper_stream": dict(
        desc="paper-shaped stream: voxel 0.2 m, tau 10, 9x9 grid (n_s = n_r = 3), eta 0.3",
        voxel_size=0.2, max_pts=64, min_pts=10, grid_side=9, signal_var=1.0, length_scale=0.1, noise_var=1e-3,
        converge_var=0.3),
    # batched uneven voxels: one 128-beam x 1024-azimuth scan (or a rosette
    # scan) at 1 m voxels, up to 256 points per voxel, 8x8 grid.
    "batched": dict(
        desc="batched: 128-beam x 1024-azimuth spinning scan (131k rays) or a 100k-point rosette scan of the box "
             "scene, voxel 1 m, cap 256, tau 3, 8x8 grid",
        voxel_size=1.0, max_pts=256, min_pts=3, grid_side=8, signal_var=1.0, length_scale=0.5, noise_var=1e-3,
        converge_var=0.3, n_beams=128, n_az=1024),
    # large aggregated map update: 10 scans of 128 x 1024 with pose noise,
    # voxel 0.1 m, up to 512 points per voxel, length scale from PCA, 16x16 grid.
    "aggregated": dict(
        desc="aggregated: 10 scans of 128 beams x 1024 azimuths 0.05 m apart along a path with N(0, 0.01 m) "
             "pose noise, scene cleared within 2 m (about 1M points, voxels up to the 512 cap), voxel 0.1 m, "
             "cap 512, tau 3, 16x16 grid, length scale from PCA",
        voxel_size=0.1, max_pts=512, min_pts=3, grid_side=16, signal_var=1.0, length_scale=0.05, noise_var=1e-3,
        converge_var=0.3, ls_mode=1, n_beams=128, n_az=1024),
}


def params_for(name: str, **overrides) -> dict:
    """Hyper-parameters of a workload (without its descriptive / generator keys)."""
    w = dict(WORKLOADS[name])
    for k in ("desc", "n_beams", "n_az"):
        w.pop(k, None)
    w.update(overrides)
    return w
