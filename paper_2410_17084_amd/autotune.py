"""Launch autotuner of vgpr_fit_predict.

Searches the launch choices of `vgpr_tuning` (which buckets try FP32 first,
which use the one-voxel-per-wavefront solver, which use the tiled
matrix-core solver, one or three streams and which stream each bucket takes,
the persistent grid size of each bucket) by coordinate descent, timing the real
workload on the device with HIP events. A candidate is accepted only if its
outputs stay within the accuracy tolerances of an FP64 reference run of the
same call (mean 1e-4 m, variance 1e-3 s_f^2, identical status and axis), so
tuning never trades accuracy for speed. Results are cached as JSON per
(grid side, cap, precision, device name).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")

MEAN_TOL = 1e-4
VAR_TOL_REL = 1e-3


def cache_key(params, device_name: str) -> str:
    return f"nq={params.grid_side},cap={params.max_pts},prec={params.precision},dev={device_name}"


def load_cached(params, device_name: str, path: str = DEFAULT_CACHE):
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh).get(cache_key(params, device_name))


def save_cached(params, device_name: str, entry: dict, path: str = DEFAULT_CACHE):
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[cache_key(params, device_name)] = entry
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def _time_fit(ctx, xyz, vox, params, out, reps: int) -> float:
    torch = ctx.torch
    ctx.fit_predict(xyz, vox, params, out=out)  # warm
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        start.record(ctx.stream)
        ctx.fit_predict(xyz, vox, params, out=out)
        end.record(ctx.stream)
        end.synchronize()
        best = min(best, start.elapsed_time(end))
    return best


def _within(out, ref, sf2: float) -> bool:
    o, a, s = (t.cpu().numpy() for t in out)
    ro, ra, rs = (t.cpu().numpy() for t in ref)
    solved = (rs & 1) != 0
    # solved / below tau / capped / near-tie must match; refined and converged may differ
    if not np.array_equal(a, ra) or not np.array_equal(s & 0x47, rs & 0x47):
        return False
    if not solved.any():
        return True
    ax = ra[solved]
    go, gr = o[solved], ro[solved]
    idx = np.arange(len(ax))
    em = np.abs(go[idx, :, ax] - gr[idx, :, ax]).max()
    ev = np.abs(go[:, :, 3] - gr[:, :, 3]).max()
    return bool(em <= MEAN_TOL and ev <= VAR_TOL_REL * sf2)


def tune(ctx, xyz, vox, params, reps: int = 5, log=print) -> dict:
    """Coordinate-descent search; returns {"tuning": ..., "ms": ..., "baseline_ms": ...}."""
    from . import vgpr
    torch = ctx.torch
    V = vox.n_vox
    m = params.grid_side ** 2
    mk = lambda: (torch.empty((V, m, 4), dtype=torch.float32, device=xyz.device),  # noqa: E731
                  torch.empty(V, dtype=torch.int8, device=xyz.device),
                  torch.empty(V, dtype=torch.uint8, device=xyz.device))
    ref = mk()
    ctx.fit_predict(xyz, vox, params.replace(precision=vgpr.PREC_FP64), out=ref)
    out = mk()
    cur = ctx.tuning().as_dict()
    ctx.set_tuning(vgpr.Tuning.from_dict(cur))
    base = _time_fit(ctx, xyz, vox, params, out, reps)
    best_ms = base
    log(f"[autotune] baseline {base:.3f} ms {cur}")
    fp32_opts = [-1, 0, 1, 2, 3, 4] if params.precision in (vgpr.PREC_FP32, vgpr.PREC_MIXED) else [cur["fp32_last_bucket"]]
    space = [("streams", [1, 3]), ("wave_last_bucket", [0, 1, 2]), ("fp32_last_bucket", fp32_opts)]
    space.append(("tiled_first", [0, 1]))
    if params.max_pts > 32:
        tiles = [b for b in (2, 3, 4, 5) if params.max_pts > (16, 32, 64, 96, 128)[b - 1]] or [5]
        space.append(("tile_first_bucket", tiles))
        # which buckets are tiled and whether they run before the fork interact: search them together
        space.append((("joint", "tile_first_bucket", "tiled_first"), [(b, f) for b in tiles for f in (0, 1)]))
    # bucket -> stream maps (0: the context's stream, 1..3: side streams): the default, the
    # 256-point bucket ahead of the 96/128-point ones, the 96-point bucket with the 32/64-point ones
    space.append(("bucket_stream", [list(vgpr.DEFAULT_BUCKET_STREAM), [0, 2, 2, 1, 1, 1, 3], [0, 2, 2, 2, 1, 1, 3]]))
    if params.max_pts > 256:
        space.append(("tiled_merge", [0, 1]))
    caps = (0, 16, 32, 64, 96, 128, 256)  # lower bound of each bucket
    space += [(("grid_scale", b), [2, 4, 8, 16]) for b in range(7) if params.max_pts > caps[b]]
    t0 = time.perf_counter()
    for _ in range(2):  # two sweeps of coordinate descent
        improved = False
        for key, options in space:
            for opt in options:
                cand = json.loads(json.dumps(cur))
                if isinstance(key, tuple) and key[0] == "joint":
                    if all(cand[k] == o for k, o in zip(key[1:], opt)):
                        continue
                    for k, o in zip(key[1:], opt):
                        cand[k] = o
                elif isinstance(key, tuple):
                    if cand["grid_scale"][key[1]] == opt:
                        continue
                    cand["grid_scale"][key[1]] = opt
                else:
                    if cand[key] == opt:
                        continue
                    cand[key] = opt
                ctx.set_tuning(vgpr.Tuning.from_dict(cand))
                ms = _time_fit(ctx, xyz, vox, params, out, reps)
                ok = _within(out, ref, params.signal_var)
                if ok and ms < best_ms * 0.98:
                    best_ms, cur, improved = ms, cand, True
                    log(f"[autotune] {ms:.3f} ms {cur}")
        if not improved:
            break
    ctx.set_tuning(vgpr.Tuning.from_dict(cur))
    return {"tuning": cur, "ms": best_ms, "baseline_ms": base, "search_s": time.perf_counter() - t0}
