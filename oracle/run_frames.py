"""Run the oracle over whole frames on a pool of worker processes (test
infrastructure, like the rest of oracle/).

The CPU baseline of the benchmark starts this as a child process of its own
(python -m oracle.run_frames ...): a fresh interpreter that never touches the
GPU forks its workers, each voxelizing one frame and fitting every voxel with
the FP64 oracle, BLAS limited to one thread per worker. With --split-voxels
(batches of a few large frames) the interpreter voxelizes every frame itself,
then forks the workers, which fit interleaved slices of each frame's voxels.
Prints one JSON line. Holds no method arithmetic of its own.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import time

import numpy as np

_XYZ = None
_FO = None
_PRM = None


def _init(xyz_path: str, fo_path: str, params: dict) -> None:
    global _XYZ, _FO, _PRM
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    _XYZ = np.load(xyz_path, mmap_mode="r")
    _FO = np.load(fo_path)
    _PRM = params


def fit_frame(f: int) -> tuple:
    """Oracle voxelize + fit of every voxel of frame f: (solved, voxels, seconds)."""
    from oracle import vgpr_oracle as O
    keys = {k for k in O.Params.__dataclass_fields__}
    prm = O.Params(**{k: v for k, v in _PRM.items() if k in keys})
    xf = np.ascontiguousarray(_XYZ[int(_FO[f]):int(_FO[f + 1])])
    t0 = time.perf_counter()
    ov = O.voxelize(xf, prm.voxel_size)
    solved = 0
    for v in range(len(ov["keys"])):
        r = O.fit_predict_voxel(O.voxel_points(xf, ov, v), ov["keys"][v], prm)
        solved += bool(r["status"] & O.ST_SOLVED)
    return solved, len(ov["keys"]), time.perf_counter() - t0


_OV = None


def fit_slice(task: tuple) -> tuple:
    """Oracle fit of voxels lo, lo + step, ... of frame f, voxelized before the fork."""
    from oracle import vgpr_oracle as O
    f, lo, step = task
    keys = {k for k in O.Params.__dataclass_fields__}
    prm = O.Params(**{k: v for k, v in _PRM.items() if k in keys})
    xf = np.ascontiguousarray(_XYZ[int(_FO[f]):int(_FO[f + 1])])
    ov = _OV[f]
    t0 = time.perf_counter()
    solved = 0
    for v in range(lo, len(ov["keys"]), step):
        r = O.fit_predict_voxel(O.voxel_points(xf, ov, v), ov["keys"][v], prm)
        solved += bool(r["status"] & O.ST_SOLVED)
    return solved, len(range(lo, len(ov["keys"]), step)), time.perf_counter() - t0


def split_voxels(a, params: dict) -> dict:
    global _OV
    from threadpoolctl import threadpool_limits

    from oracle import vgpr_oracle as O
    threadpool_limits(limits=1)
    _init(a.xyz, a.fo, params)
    n_frames = len(_FO) - 1
    slices = 8 * a.workers
    t0 = time.perf_counter()
    _OV = [O.voxelize(np.ascontiguousarray(_XYZ[int(_FO[f]):int(_FO[f + 1])]), params["voxel_size"])
           for f in range(n_frames)]
    t_vox = time.perf_counter() - t0
    with mp.get_context("fork").Pool(a.workers) as pool:
        res = pool.map(fit_slice, [(f, k, slices) for f in range(n_frames) for k in range(slices)], chunksize=1)
    wall = time.perf_counter() - t0
    return {"frames": n_frames, "solved": int(sum(r[0] for r in res)), "voxels": int(sum(r[1] for r in res)),
            "wall_s": wall, "worker_s": float(sum(r[2] for r in res)) + t_vox, "voxelize_s": t_vox,
            "workers": a.workers, "pid": os.getpid()}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--xyz", required=True)
    ap.add_argument("--fo", required=True)
    ap.add_argument("--params", required=True, help="JSON of the hyper-parameters")
    ap.add_argument("--workers", type=int, required=True)
    ap.add_argument("--split-voxels", action="store_true",
                    help="voxelize each frame here, then fit slices of its voxels on the workers")
    a = ap.parse_args()
    params = json.loads(a.params)
    if a.split_voxels:
        print(json.dumps(split_voxels(a, params)), flush=True)
        return
    fo = np.load(a.fo)
    n_frames = len(fo) - 1
    with mp.get_context("fork").Pool(a.workers, initializer=_init, initargs=(a.xyz, a.fo, params)) as pool:
        pool.map(fit_frame, range(min(a.workers, n_frames)))  # start-up outside the clock
        t0 = time.perf_counter()
        res = pool.map(fit_frame, range(n_frames), chunksize=1)
        wall = time.perf_counter() - t0
    print(json.dumps({"frames": n_frames, "solved": int(sum(r[0] for r in res)),
                      "voxels": int(sum(r[1] for r in res)), "wall_s": wall,
                      "worker_s": float(sum(r[2] for r in res)), "workers": a.workers, "pid": os.getpid()}),
          flush=True)


if __name__ == "__main__":
    main()
