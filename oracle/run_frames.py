"""Run the oracle over whole frames on a pool of worker processes (test
infrastructure, like the rest of oracle/).

The CPU baseline of the benchmark starts this as a child process of its own
(python -m oracle.run_frames ...): a fresh interpreter that never touches the
GPU forks its workers, each voxelizing one frame and fitting every voxel with
the FP64 oracle, BLAS limited to one thread per worker. Prints one JSON line.
Holds no method arithmetic of its own.
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


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--xyz", required=True)
    ap.add_argument("--fo", required=True)
    ap.add_argument("--params", required=True, help="JSON of the hyper-parameters")
    ap.add_argument("--workers", type=int, required=True)
    a = ap.parse_args()
    params = json.loads(a.params)
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
