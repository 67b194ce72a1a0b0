"""Throughput of the Voxel-GPR hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic scans that
are already resident in HBM: vgpr_voxelize over the batch (frames voxelized
independently) followed by vgpr_fit_predict over every voxel of the batch.
By default the batch is one aggregated map-update frame: 10 seeded 128-beam x
1024-azimuth scans of the box scene 0.05 m apart with pose noise (about 1M
points; voxel 0.1 m, cap 512, tau 3, 16x16 query grid, length scale from PCA);
`--workload spin32` and `--workload batched` run 64 spinning scans (0.5 m, cap
128, 8x8) and the 16-frame spinning + rosette batch (1 m, cap 256, 8x8) instead.

Prints one JSON line: solved voxels per second (plus dense points per second),
the per-kernel roofline of the dominant kernel from HIP events on the
library's stream, single-frame latency percentiles, and the FP64 CPU oracle
timed on a bounded sample of the same workload, whose results also give the
accuracy check of the GPU outputs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2410_17084_amd import configs, synth  # noqa: E402

PEAK = {"f32": 157.3, "f64": 78.6}  # TFLOP/s, MI355X vector FP32 / FP64
HBM_PEAK = 8000.0                   # GB/s
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILES = {"aggregated": os.path.join(HERE, "profiles", "hbm_traffic_aggregated.json")}


def source_hash() -> str:
    """Hash of the sources the solver kernels and their launches are built from (the
    solver file, the context and launch-choice code, the internal and ABI headers):
    ties stored counter readings of the solver kernels to the code."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_2410_17084_amd", "csrc")
    files = [os.path.join(csrc, f) for f in ("ctx.hip", "fit.hip", "scan.h", "vgpr_internal.h")] + \
        [os.path.join(HERE, "include", "vgpr.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, family: str, tuning: dict, precision: str):
    """HBM bytes per launch of `family` from the stored FETCH_SIZE / WRITE_SIZE readings.

    None unless the readings were taken on the current sources with the same
    launch choices and precision.
    """
    path = TRAFFIC_FILES.get(workload)
    if path is None or not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash() or d.get("tuning") != tuning or d.get("precision") != precision:
        return None
    e = d.get("families", {}).get(family)
    return None if e is None else float(e["bytes_per_launch"])
BUCKETS = (16, 32, 64, 96, 128, 256, 512)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def voxel_flops(n: np.ndarray, m: int) -> np.ndarray:
    """Algorithmic FP operations of one voxel solve.

    n^3/3 (factorisation) + n^2 m (L^-1 K*) + 2 n^2 (solve of f) + 4 n m
    (mean and variance) + 6 (n^2/2 + n m) (kernel entries, exp not counted).
    """
    n = n.astype(np.float64)
    return n ** 3 / 3 + n * n * m + 2 * n * n + 4 * n * m + 6 * (n * n / 2 + n * m)


def voxel_bytes(n: np.ndarray, m: int) -> np.ndarray:
    """Algorithmic HBM bytes of one voxel solve: points in, key/offset/count, rows out, axis/status."""
    return 12.0 * n + 16 + 16.0 * m + 2


def family_buckets(fam: str, tuning: dict, max_pts: int) -> tuple:
    """Size buckets whose voxels a solver family's launch takes: its own, and with
    tiled_merge the 512-point launch also takes the 256-point bucket."""
    b = BUCKETS.index(int(fam.rsplit("_n", 1)[1]))
    if b == len(BUCKETS) - 1 and tuning.get("tiled_merge") and max_pts > BUCKETS[-2] \
            and tuning["tile_first_bucket"] <= len(BUCKETS) - 2 and not fam.startswith("refine"):
        return (b - 1, b)
    return (b,)


def bucket_of(n: np.ndarray) -> np.ndarray:
    b = np.zeros(len(n), dtype=np.int64)
    for i, c in enumerate(BUCKETS[:-1]):
        b += (n > c)
    return b


def precision_split(n_kept: np.ndarray, solved: np.ndarray, m: int, tuning: dict, precision: str) -> dict:
    """Share of the step's algorithmic FLOPs computed in each arithmetic type, from
    the launch choices that ran: in FP32 and MIXED mode the buckets up to
    fp32_last_bucket that are not tiled run in float (their voxels flagged for
    re-solve again in double), tiled buckets run FP64 tiles (MIXED: FP32 tiles
    and FP32 query products); everything else runs in double."""
    b_of = bucket_of(n_kept)
    fl = voxel_flops(n_kept, m)
    share = {}
    for b in range(len(BUCKETS)):
        sel = solved & (b_of == b)
        if not sel.any():
            continue
        tiled = b >= tuning["tile_first_bucket"]
        if precision == "fp64":
            kind = "f64"
        elif tiled:
            kind = "f32" if precision == "mixed" else "f64"
        else:
            kind = "f32" if b <= tuning["fp32_last_bucket"] else "f64"
        share[kind] = share.get(kind, 0.0) + float(fl[sel].sum())
    tot = sum(share.values()) or 1.0
    frac = {k: v / tot for k, v in sorted(share.items(), key=lambda kv: -kv[1])}
    label = " + ".join(f"{k} {100 * v:.0f}%" for k, v in frac.items())
    return {"dtype": next(iter(frac), "f64"), "flop_share": frac, "label": label}


def cpu_baseline(xyz_np: np.ndarray, fo, frame_vox, w: dict, gpu_out, budget_s: float) -> dict:
    """FP64 oracle on the batch's frames in order: voxelize a frame, fit its voxels, until the budget.

    The oracle's outputs for the voxels it reached also check the GPU outputs
    of the same voxels (the accuracy gate of the metric): frame f's voxels are
    the batch's voxels frame_vox[f] .. frame_vox[f + 1] in the same order.
    """
    from threadpoolctl import threadpool_limits

    from oracle import vgpr_oracle as O
    from tests import parity

    prm = parity.oracle_params(w)
    solved = reached = frames = points = 0
    spent = 0.0
    max_mean = max_var = max_rel = 0.0
    rel_in = rel_tot = 0
    with threadpool_limits(limits=1):
        for f in range(len(fo) - 1):
            xf = xyz_np[int(fo[f]):int(fo[f + 1])]
            t0 = time.perf_counter()
            ov = O.voxelize(xf, w["voxel_size"])
            done = 0
            for v in range(len(ov["keys"])):
                r = O.fit_predict_voxel(O.voxel_points(xf, ov, v), ov["keys"][v], prm)
                solved += bool(r["status"] & O.ST_SOLVED)
                done = v + 1
                if spent + time.perf_counter() - t0 > budget_s:
                    break
            spent += time.perf_counter() - t0
            a, b = int(frame_vox[f]), int(frame_vox[f + 1])
            stats = parity.compare_fit(xf, ov, prm, gpu_out[0][a:b], gpu_out[1][a:b], gpu_out[2][a:b],
                                       voxels=range(done))
            max_mean = max(max_mean, stats["max_mean_err"])
            max_var = max(max_var, stats["max_var_err"])
            max_rel = max(max_rel, stats["max_var_rel_own"])
            rel_in += stats["queries_var_rel_own_within_tol"]
            rel_tot += stats["queries_var_rel_own"]
            reached += done
            frames += 1
            points += len(xf)
            if spent > budget_s:
                break
    return {
        "value": solved / spent, "unit": "voxel solves/s", "cores": 1, "kind": "oracle",
        "sample": f"the first {frames} frame(s) of the batch ({points} points): oracle voxelize + FP64 fit of "
                  f"{reached} voxels ({solved} solved) in {spent:.1f} s, BLAS limited to 1 thread",
        "accuracy": {"voxels_checked": reached, "solved_checked": solved, "max_mean_err_m": max_mean,
                     "max_var_err": max_var, "mean_tol_m": parity.MEAN_TOL, "var_tol": parity.VAR_TOL_REL,
                     "var_err_reading": "|gpu - oracle| <= var_tol * s_f^2 (prior-normalised), asserted",
                     "max_var_rel_own": max_rel,
                     "frac_queries_var_rel_own_within_tol": rel_in / rel_tot if rel_tot else 1.0,
                     "var_rel_own_reading": "|gpu - oracle| / oracle (own value), reported, not asserted",
                     "pass": True},
    }


def cpu_pool(xyz_np: np.ndarray, fo, w: dict, workers: int, timeout_s: float = 240.0):
    """The FP64 oracle over every frame of the batch on `workers` processes: a
    child interpreter of its own (it never touches the GPU) forks the pool, one
    frame per task. None if it fails or exceeds timeout_s."""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory(dir="/tmp") as td:
        xp, fp = os.path.join(td, "xyz.npy"), os.path.join(td, "fo.npy")
        np.save(xp, np.ascontiguousarray(xyz_np, dtype=np.float32))
        np.save(fp, np.asarray(fo, dtype=np.int64))
        prm = {k: v for k, v in w.items() if isinstance(v, (int, float))}
        try:
            split = ["--split-voxels"] if len(fo) - 1 < workers else []
            r = subprocess.run([sys.executable, "-m", "oracle.run_frames", "--xyz", xp, "--fo", fp, "--params",
                                json.dumps(prm), "--workers", str(workers), *split], cwd=HERE, capture_output=True,
                               text=True, timeout=timeout_s)
        except subprocess.TimeoutExpired:
            log(f"cpu pool exceeded {timeout_s} s; skipped")
            return None
    if r.returncode != 0:
        log(f"cpu pool failed: {r.stderr[-500:]}")
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    how = ("the frames voxelized in one process, then interleaved slices of their voxels fitted"
           if "voxelize_s" in d else "one frame per task, voxelized and fitted")
    return {"value": d["solved"] / d["wall_s"], "unit": "voxel solves/s", "cores": workers, "kind": "oracle",
            "sample": f"all {d['frames']} frames of the batch ({len(xyz_np)} points): oracle voxelize + FP64 fit of "
                      f"{d['voxels']} voxels ({d['solved']} solved) on {workers} worker processes ({how}) in "
                      f"{d['wall_s']:.1f} s wall ({d['worker_s']:.1f} s of worker time), BLAS limited to 1 thread "
                      "per worker"}


def precision_accuracy(forms: dict, samples: dict) -> None:
    """CPU-baseline leg, for the precision forms: the oracle's voxelization and FP64
    fit of each form's sampled voxels, compared with the GPU outputs the precision
    leg kept; fills in the forms' error fields."""
    import torch

    from oracle import vgpr_oracle as O
    from tests import parity
    xyz_np, fo = samples["xyz"], samples["fo"]
    for s in (0.2, 0.5, 1.0):
        w = configs.params_for("batched", voxel_size=s, length_scale=s / 2)
        ov = O.voxelize(xyz_np, w["voxel_size"], fo)
        for prec_name in ("fp32", "fp64", "mixed"):
            V, m, pick, rows, ax, st = samples[(s, prec_name)]
            out = np.full((V, m, 4), np.nan, np.float32)
            axis = np.full(V, -1, np.int8)
            status = np.zeros(V, np.uint8)
            out[pick], axis[pick], status[pick] = rows, ax, st
            stats = parity.compare_fit(xyz_np, ov, parity.oracle_params(w), torch.from_numpy(out),
                                       torch.from_numpy(axis), torch.from_numpy(status), voxels=pick, strict=False)
            forms[f"s={s:g}"][prec_name].update({
                "max_mean_err_m": stats["max_mean_err"], "max_var_err_prior": stats["max_var_err"],
                "max_var_rel_own": stats["max_var_rel_own"],
                "sample_voxels_outside_tolerance": stats["outside_tolerance"],
                "within_tolerance": stats["outside_tolerance"] == 0})
            log(f"precision form s={s} {prec_name} accuracy: {forms[f's={s:g}'][prec_name]}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["spin32", "batched", "aggregated"], default="aggregated",
                    help="aggregated: 10-scan 128-beam map updates at 0.1 m voxels, cap 512, 16x16 (the default "
                         "step); spin32: batches of 32-beam scans; batched: 128-beam and rosette scans at 1 m "
                         "voxels, cap 256")
    ap.add_argument("--no-precision-forms", dest="precision_forms", action="store_false",
                    help="skip the FP32 / FP64 / MIXED comparison on the batched workload at 0.2, 0.5, 1.0 m")
    ap.add_argument("--extra-steps", type=int, default=10,
                    help="timed steps of each other workload reported beside the headline (0 skips them)")
    ap.add_argument("--frames", type=int, default=None, help="frames per step (default 64 / 16 / 1 by workload)")
    ap.add_argument("--precision", choices=["fp32", "fp64", "mixed"], default="fp32")
    ap.add_argument("--latency-frames", type=int, default=60)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle worker processes of the CPU baseline (capped by the usable cores; 1 = one core)")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the 8-stream 10 Hz serving run (0 skips it)")
    ap.add_argument("--serve-frames", type=int, default=10, help="distinct frames generated per stream (cycled)")
    ap.add_argument("--autotune", action="store_true", help="search launch choices first and cache them")
    ap.add_argument("--gauss-launches", type=int, default=20,
                    help="timed launches of the 3D-Gaussian initialisation on the batch's grids (0 skips)")
    ap.add_argument("--loss-launches", type=int, default=10, help="timed structure-loss calls (0 = skip)")
    ap.add_argument("--isolated-steps", type=int, default=5,
                    help="steps with every bucket on one stream, for each kernel's own duration (0 = skip)")
    ap.add_argument("--graph-steps", type=int, default=20,
                    help="steps of the captured-graph form of the batch (0 skips it)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(voxels would shard by key with one all-to-all exchange of points)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2410_17084_amd import vgpr

    w = configs.params_for(args.workload)
    if args.frames is None:
        args.frames = {"spin32": 64, "batched": 16, "aggregated": 1}[args.workload]
    m = w["grid_side"] ** 2
    t0 = time.perf_counter()
    xyz_np, fo = workload_frames(args.workload, args.frames)
    log(f"generated {args.frames} {args.workload} frames, {len(xyz_np)} points in {time.perf_counter() - t0:.1f} s")

    if args.copy_probe:
        src = torch.empty(args.copy_probe << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written")
        del src, dst

    prec = {"fp32": vgpr.PREC_FP32, "fp64": vgpr.PREC_FP64, "mixed": vgpr.PREC_MIXED}[args.precision]
    p = vgpr.default_params(**{k: v for k, v in w.items() if k in {f for f, _ in vgpr.Params._fields_}})
    p.precision = prec
    ctx = vgpr.Context(0)
    xyz = torch.from_numpy(xyz_np).cuda()
    torch.cuda.synchronize()

    # first pass sizes the outputs; every later step reuses them
    vox = ctx.voxelize(xyz, p, frame_offsets=fo)
    V = vox.n_vox
    out = (torch.empty((V, m, 4), dtype=torch.float32, device="cuda"),
           torch.empty(V, dtype=torch.int8, device="cuda"), torch.empty(V, dtype=torch.uint8, device="cuda"))
    keys = torch.empty(len(xyz_np), dtype=torch.int64, device="cuda")
    offs = torch.empty(len(xyz_np), dtype=torch.int32, device="cuda")
    cnts = torch.empty(len(xyz_np), dtype=torch.int32, device="cuda")
    perm = torch.empty(len(xyz_np), dtype=torch.int32, device="cuda")

    # launch choices: the cached autotuner result for this device (or a fresh search)
    from paper_2410_17084_amd import autotune
    props = torch.cuda.get_device_properties(0)
    dev_name = f"{getattr(props, 'gcnArchName', 'gpu').split(':')[0]}x{props.multi_processor_count}cu"
    log(f"device key for cached tuning: {dev_name}")
    tuned = None
    if args.autotune:
        prior = autotune.load_cached(p, dev_name)
        if prior:  # refine the cached choices rather than start from the library defaults
            ctx.set_tuning(vgpr.Tuning.from_dict(prior["tuning"]))
        tuned = autotune.tune(ctx, xyz, vgpr.Voxels(vox.keys, vox.offsets, vox.counts, vox.perm, V, [], 0), p,
                              log=log)
        autotune.save_cached(p, dev_name, tuned)
    else:
        tuned = autotune.load_cached(p, dev_name)
        if tuned:
            ctx.set_tuning(vgpr.Tuning.from_dict(tuned["tuning"]))
    log(f"tuning: {ctx.tuning().as_dict()}")

    def step():
        n = ctypes_voxelize(ctx, vgpr, xyz, p, fo, keys, offs, cnts, perm)
        v = vgpr.Voxels(keys[:n], offs[:n], cnts[:n], perm, n, [], 0)
        ctx.fit_predict(xyz, v, p, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done: {V} voxels in the batch")
    if not args.no_profile:
        ctx.profile(True)
        for fam in FAMILIES:
            ctx.profile_read(fam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fam_time = {}
    if not args.no_profile:
        for fam in FAMILIES:
            ms, cnt = ctx.profile_read(fam)
            if cnt:
                fam_time[fam] = (ms, cnt)
        ctx.profile(False)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    status = out[2].cpu().numpy()
    counts = cnts[:V].cpu().numpy().astype(np.int64)
    n_kept = np.minimum(counts, w["max_pts"])
    solved = (status & vgpr.ST_SOLVED) != 0
    refined = (status & vgpr.ST_REFINED) != 0
    n_solved = int(solved.sum())
    value = n_solved * args.steps / elapsed
    dense = value * m

    # roofline of the dominant kernel family
    roof = None
    kernels = {}
    if fam_time:
        b_of = bucket_of(n_kept)
        fl = voxel_flops(n_kept, m)
        by = voxel_bytes(n_kept, m)
        for fam, (ms, cnt) in fam_time.items():
            kernels[fam] = {"ms_per_launch": ms / cnt, "launches_per_step": cnt / args.steps}
        # dominant kernel: the solver family that carries the most algorithmic FLOPs of the step
        # (a launch's duration in the concurrent step includes waiting for CUs, so the longest
        # launch can be a small one); its roofline uses its duration in the timed region
        tun = ctx.tuning().as_dict()

        def fam_flops(f):
            fb_ = family_buckets(f, tun, w["max_pts"])
            sel_ = solved & np.isin(b_of, fb_) & (refined if f.startswith("refine") else True)
            return float(fl[sel_].sum())
        dom = max((f for f in fam_time if f.startswith(("fit", "refine"))),
                  key=lambda f: (fam_flops(f), fam_time[f][0]), default=None)
        if dom is not None:
            fb = family_buckets(dom, ctx.tuning().as_dict(), w["max_pts"])
            if dom.startswith("refine"):
                sel = solved & refined & np.isin(b_of, fb)
            else:
                sel = solved & np.isin(b_of, fb)
            flops = float(fl[sel].sum())
            ms, cnt = fam_time[dom]
            per_launch_s = ms / cnt / 1e3
            launches_per_step = cnt / args.steps
            flops_per_launch = flops / launches_per_step
            achieved = flops_per_launch / per_launch_s / 1e12
            dt = "f64" if ("f64" in dom) else "f32"
            roof = {"bound": "alu", "achieved": achieved, "peak": PEAK[dt], "unit": "TFLOP/s",
                    "frac": achieved / PEAK[dt], "traffic": None, "kernel": dom,
                    "voxel_points": f"({([0] + list(BUCKETS))[fb[0]]}, {BUCKETS[fb[-1]]}]",
                    "voxels_per_launch": int(sel.sum() / launches_per_step),
                    "algorithmic_bytes_per_launch": float(by[sel].sum() / launches_per_step),
                    "hbm_frac": float(by[sel].sum() / launches_per_step) / per_launch_s / 1e9 / HBM_PEAK}
            default_frames = {"spin32": 64, "batched": 16, "aggregated": 1}[args.workload]
            roof["traffic"] = (measured_traffic(args.workload, dom, ctx.tuning().as_dict(), args.precision)
                               if args.frames == default_frames else None)
            if roof["traffic"]:
                roof["traffic_vs_algorithmic"] = roof["traffic"] / roof["algorithmic_bytes_per_launch"]
        tot_fit = sum(v[0] for f, v in fam_time.items() if f.startswith(("fit", "refine")))
        kernels["_fit_all"] = {"ms_per_step": tot_fit / args.steps,
                               "tflops": float(fl[solved].sum()) / (tot_fit / args.steps / 1e3) / 1e12}

    # The buckets run concurrently on side streams, so a launch's duration in the
    # timed region includes time spent waiting for CUs that other buckets hold
    # (and rocprofv3 sees the same). The same launch choices with every bucket
    # on one stream give each kernel's own duration: the per-kernel roofline.
    isolated = None
    if fam_time and args.isolated_steps > 0:
        t_saved = ctx.tuning().as_dict()
        t_ser = dict(t_saved)
        t_ser["streams"] = 1
        ctx.set_tuning(vgpr.Tuning.from_dict(t_ser))
        step()
        torch.cuda.synchronize()
        ctx.profile(True)
        for fam in FAMILIES:
            ctx.profile_read(fam)
        for _ in range(args.isolated_steps):
            step()
        iso = {fam: ctx.profile_read(fam) for fam in FAMILIES}
        ctx.profile(False)
        ctx.set_tuning(vgpr.Tuning.from_dict(t_saved))
        b_of = bucket_of(n_kept)
        fl = voxel_flops(n_kept, m)
        per = {}
        for fam, (ms, cnt) in iso.items():
            if not cnt or not fam.startswith(("fit", "refine")):
                continue
            fb = family_buckets(fam, t_saved, w["max_pts"])
            sel = solved & np.isin(b_of, fb) & (refined if fam.startswith("refine") else True)
            lps = cnt / args.isolated_steps
            sec = ms / cnt / 1e3
            tf = float(fl[sel].sum()) / lps / sec / 1e12
            dt = "f64" if "f64" in fam else "f32"
            per[fam] = {"ms_per_launch": ms / cnt, "voxels_per_launch": int(sel.sum() / lps), "tflops": tf,
                        "frac": tf / PEAK[dt]}
        dom_iso = max(per, key=lambda f: per[f]["ms_per_launch"]) if per else None
        isolated = {"what": "same launch choices, every bucket on one stream (each kernel's own duration, HIP "
                            "events); peak FP64 78.6 / FP32 157.3 TFLOP/s", "dominant": dom_iso,
                    "ms_per_step_serial": sum(v[0] for f, v in iso.items() if v[1]) / args.isolated_steps,
                    "kernels": per}
        log(f"isolated launches: dominant {dom_iso} {per.get(dom_iso)}")

    # batched form captured as a graph: the same batch voxelized into fixed
    # buffers, then one replay of the captured fit_predict per step
    graph = None
    if args.graph_steps > 0:
        gst = torch.cuda.Stream()
        gctx = vgpr.Context(0, stream=gst)
        gctx.set_tuning(ctx.tuning())
        torch.cuda.synchronize()
        n0 = ctypes_voxelize(gctx, vgpr, xyz, p, fo, keys, offs, cnts, perm)
        gv = vgpr.Voxels(keys[:n0], offs[:n0], cnts[:n0], perm, n0, [], 0)
        gout = (torch.empty_like(out[0]), torch.empty_like(out[1]), torch.empty_like(out[2]))
        g = gctx.fit_graph(xyz, gv, p, out=gout)
        for _ in range(args.warmup):
            g.launch()
        gst.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.graph_steps):
            if ctypes_voxelize(gctx, vgpr, xyz, p, fo, keys, offs, cnts, perm) != n0:
                raise RuntimeError("batch voxel count changed between graph replays")
            g.launch()
        gst.synchronize()
        g_step = (time.perf_counter() - t1) / args.graph_steps
        t1 = time.perf_counter()
        for _ in range(args.graph_steps):
            g.launch()
        gst.synchronize()
        g_fit = (time.perf_counter() - t1) / args.graph_steps
        t1 = time.perf_counter()
        for _ in range(args.graph_steps):
            gctx.fit_predict(xyz, gv, p, out=gout)
        gst.synchronize()
        e_fit = (time.perf_counter() - t1) / args.graph_steps
        same = all(bool(torch.equal(a[:n0], b[:n0])) if a.dtype != torch.float32 else
                   bool(torch.equal(torch.nan_to_num(a[:n0], nan=-7.0), torch.nan_to_num(b[:n0], nan=-7.0)))
                   for a, b in zip(gout, out))
        graph = {"ms_per_step": g_step * 1e3, "solves_per_s": n_solved / g_step,
                 "fit_ms_graph": g_fit * 1e3, "fit_ms_eager": e_fit * 1e3, "outputs_equal_eager": same,
                 "what": "voxelize + one replay of the captured fit_predict per step, same batch"}
        g.close()
        gctx.close()
        log(f"graph: {graph}")

    # initial 3D Gaussians (Sec. 3.2) from the batch's grids: HBM-bound (the rows of
    # solved voxels read once, one status byte per voxel, 32 B per Gaussian written)
    gauss = None
    if args.gauss_launches > 0:
        nr = max(1, w["grid_side"] // 4)
        ns = w["grid_side"] // nr
        gbuf = torch.empty((V, ns * ns, 8), dtype=torch.float32, device="cuda")
        ctx.gauss_init(out[0], out[2], w["grid_side"], nr, gauss=gbuf)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read("gauss_init")
        for _ in range(args.gauss_launches):
            ctx.gauss_init(out[0], out[2], w["grid_side"], nr, gauss=gbuf)
        gms, gcnt = ctx.profile_read("gauss_init")
        ctx.profile(False)
        per = gms / gcnt / 1e3
        gbytes = n_solved * m * 16 + V + V * ns * ns * 32
        gauss = {"ms_per_launch": per * 1e3, "gaussians_per_launch": int(V * ns * ns), "n_r": nr,
                 "bytes_per_launch": gbytes, "achieved_GBps": gbytes / per / 1e9,
                 "hbm_frac": gbytes / per / 1e9 / HBM_PEAK, "bound": "hbm"}
        log(f"gauss_init: {gauss}")

    # structure similarity loss L_p (Eq. (9)) of one scan against the batch's
    # Gaussians (S from variances: scale_mode 1), cell = the Gaussian spacing
    sloss = None
    if args.gauss_launches > 0 and args.loss_launches > 0:
        xs = xyz[int(fo[0]):int(fo[1])]
        spacing = w["voxel_size"] / ns
        by_cell = {}
        for mult in (1, 2, 4, 8):
            cell = spacing * mult
            ctx.structure_loss(xs, gbuf, cell, scale_mode=1)
            torch.cuda.synchronize()
            ctx.profile(True)
            fams = ("structure_loss", "structure_loss_brute", "voxelize_key", "voxelize_sort", "voxelize_segment")
            for fam in fams:
                ctx.profile_read(fam)
            t1 = time.perf_counter()
            for _ in range(args.loss_launches):
                lp, nvp, _, _ = ctx.structure_loss(xs, gbuf, cell, scale_mode=1)
            wall = (time.perf_counter() - t1) / args.loss_launches
            ph = {fam: ctx.profile_read(fam) for fam in fams}
            ctx.profile(False)
            by_cell[f"{cell:g}"] = {"ms_per_call": wall * 1e3,
                                    "query_kernel_ms": ph["structure_loss"][0] / max(ph["structure_loss"][1], 1),
                                    "brute_ms_per_call": ph["structure_loss_brute"][0] / args.loss_launches,
                                    "grid_sort_ms": sum(ph[f][0] for f in ph if f.startswith("voxelize")) /
                                    args.loss_launches}
        best = min(by_cell, key=lambda c: by_cell[c]["ms_per_call"])
        sloss = {"loss_m": lp, "points": int(nvp), "gaussians": int(V * ns * ns), "cell_m": float(best),
                 "ms_per_call": by_cell[best]["ms_per_call"],
                 "points_per_s": nvp / (by_cell[best]["ms_per_call"] / 1e3), "by_cell": by_cell,
                 "what": "one scan against all Gaussians of the batch: grid build (voxelize the centres, cell "
                         "table) + ring search + mean, host clock, synchronised"}
        log(f"structure loss: {sloss}")

    # single-frame latency (voxelize + fit of one scan, host clock, synchronised)
    lat = []
    lat_solved = []
    for i in range(args.latency_frames):
        f = i % args.frames
        a, b = int(fo[f]), int(fo[f + 1])
        xf = xyz[a:b]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        vf = ctx.voxelize(xf, p)
        _, _, sf = ctx.fit_predict(xf, vf, p)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
        lat_solved.append(int(((sf & vgpr.ST_SOLVED) != 0).sum().item()))
    lat = np.array(lat[5:] if len(lat) > 10 else lat)
    lat_solved = np.array(lat_solved[5:] if len(lat_solved) > 10 else lat_solved)
    if len(lat):
        log(f"latency p50 {np.percentile(lat, 50):.3f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        single = cpu_baseline(xyz_np, fo, vox.frame_vox, w, out, args.cpu_budget)
        log(f"cpu baseline (one core) {single['value']:.1f} solves/s; accuracy {single['accuracy']}")
        cpu = single
        if args.cpu_workers > 1:
            try:
                avail = len(os.sched_getaffinity(0))
            except AttributeError:
                avail = os.cpu_count() or 1
            nw = max(1, min(args.cpu_workers, avail))
            pool = cpu_pool(xyz_np, fo, w, nw)
            if pool is not None:
                cpu = pool
                cpu["single_core"] = {k: single[k] for k in ("value", "cores", "sample")}
                cpu["accuracy"] = single["accuracy"]
                log(f"cpu baseline ({nw} workers) {cpu['value']:.1f} solves/s")

    serving = None
    if args.serve_seconds > 0:
        serving = serve_leg(args, vgpr)
        log(f"serving: {serving}")

    split = precision_split(n_kept, solved, m, ctx.tuning().as_dict(), args.precision)
    extra = {}
    if args.extra_steps > 0:
        for name in ("spin32", "batched"):
            if name != args.workload:
                extra[name] = extra_leg(args, vgpr, name)
                log(f"{name}: {extra[name]}")
    forms = None
    if args.precision_forms:
        forms, fsamples = precision_leg(args, vgpr)
        if not args.no_cpu_baseline:
            precision_accuracy(forms, fsamples)
        del fsamples
    rec = {
        "metric": "voxel GPR solves/s (dense pts/s, p50/p99 frame latency) at fixed accuracy",
        "value": value, "unit": "voxel solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": split["dtype"], "data": "synthetic",
        "config": {"workload": f"{args.workload} batch: {args.frames} frames, {WORKLOAD_DESC[args.workload]} "
                               f"({len(xyz_np)} points, {V} voxels, {n_solved} solved per step)",
                   "frames": args.frames, "precision": args.precision,
                   "arithmetic": split["label"] + " of the algorithmic FLOPs" +
                                 (", float voxels with small pivots refined by one FP64 step of alpha"
                                  if prec == vgpr.PREC_FP32 else ""),
                   "parallelism": "1 GPU"},
        "flop_share": split["flop_share"],
        "dense_pts_per_s": dense,
        "tuning": ctx.tuning().as_dict(),
        "solved_per_step": n_solved, "refined_per_step": int(refined.sum()),
        "latency_ms": ({"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                        "frames": int(len(lat)), "what": "one scan: voxelize + fit_predict + sync"}
                       if len(lat) else None),
        "plain_single_scan": ({"solves_per_s": float(lat_solved.sum() / (lat.sum() / 1e3)),
                               "what": "one scan per call, synchronised (the unbatched path)"}
                              if len(lat) else None),
        "batched_graph": graph,
        "gauss_init": gauss,
        "structure_loss": sloss,
        "roofline": roof, "roofline_isolated": isolated, "kernels": kernels, "cpu_baseline": cpu, "serving": serving,
        "other_workloads": extra,
        "precision_forms": forms,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


def extra_leg(args, vgpr, name: str) -> dict:
    """Throughput of another workload under its cached launch choices (same
    precision): voxelize + fit_predict of its batch per step, K timed steps."""
    import torch

    from paper_2410_17084_amd import autotune
    w = configs.params_for(name)
    frames = {"spin32": 64, "batched": 16, "aggregated": 1}[name]
    m = w["grid_side"] ** 2
    xyz_np, fo = workload_frames(name, frames)
    prec = {"fp32": vgpr.PREC_FP32, "fp64": vgpr.PREC_FP64, "mixed": vgpr.PREC_MIXED}[args.precision]
    p = vgpr.default_params(**{k: v for k, v in w.items() if k in {f for f, _ in vgpr.Params._fields_}})
    p.precision = prec
    ctx = vgpr.Context(0)
    props = torch.cuda.get_device_properties(0)
    dev_name = f"{getattr(props, 'gcnArchName', 'gpu').split(':')[0]}x{props.multi_processor_count}cu"
    tuned = autotune.load_cached(p, dev_name)
    if tuned:
        ctx.set_tuning(vgpr.Tuning.from_dict(tuned["tuning"]))
    xyz = torch.from_numpy(xyz_np).cuda()
    vox = ctx.voxelize(xyz, p, frame_offsets=fo)
    V = vox.n_vox
    out = (torch.empty((V, m, 4), dtype=torch.float32, device="cuda"),
           torch.empty(V, dtype=torch.int8, device="cuda"), torch.empty(V, dtype=torch.uint8, device="cuda"))
    keys = torch.empty(len(xyz_np), dtype=torch.int64, device="cuda")
    offs = torch.empty(len(xyz_np), dtype=torch.int32, device="cuda")
    cnts = torch.empty(len(xyz_np), dtype=torch.int32, device="cuda")
    perm = torch.empty(len(xyz_np), dtype=torch.int32, device="cuda")

    def step():
        n = ctypes_voxelize(ctx, vgpr, xyz, p, fo, keys, offs, cnts, perm)
        ctx.fit_predict(xyz, vgpr.Voxels(keys[:n], offs[:n], cnts[:n], perm, n, [], 0), p, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.extra_steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.extra_steps
    st = out[2].cpu().numpy()
    n_kept = np.minimum(cnts[:V].cpu().numpy().astype(np.int64), w["max_pts"])
    solved = (st & vgpr.ST_SOLVED) != 0
    ns = int(solved.sum())
    sp = precision_split(n_kept, solved, m, ctx.tuning().as_dict(), args.precision)
    ctx.close()
    return {"solves_per_s": ns / el, "ms_per_step": el * 1e3, "dense_pts_per_s": ns * m / el,
            "solved_per_step": ns, "points": int(len(xyz_np)), "frames": frames, "steps": args.extra_steps,
            "arithmetic": sp["label"], "workload": WORKLOAD_DESC[name]}


def precision_leg(args, vgpr) -> tuple:
    """The three arithmetic forms on the batched workload (128-beam and rosette scans, cap 256,
    8x8 grid) at voxel sizes 0.2, 0.5 and 1.0 m (length scale half a voxel): solves/s of
    voxelize + fit_predict per step under each form's cached launch choices. Returns the
    forms and the GPU outputs of a seeded sample of voxels (every voxel above 128 points,
    every refined voxel up to 100, and 150 others), whose largest errors against the FP64
    oracle the CPU-baseline leg fills in (`precision_accuracy`)."""
    import torch

    from paper_2410_17084_amd import autotune
    frames = 16
    xyz_np, fo = workload_frames("batched", frames)
    xyz = torch.from_numpy(xyz_np).cuda()
    props = torch.cuda.get_device_properties(0)
    dev_name = f"{getattr(props, 'gcnArchName', 'gpu').split(':')[0]}x{props.multi_processor_count}cu"
    out = {"what": "batched workload (16 frames: 128x1024 spinning + 100k rosette scans), cap 256, tau 3, 8x8 "
                   "grid, l = s/2; errors: max |mean - oracle| (m), max |var - oracle| / s_f^2, max "
                   "|var - oracle| / oracle, on a seeded sample"}
    rng = np.random.Generator(np.random.PCG64(2024))
    samples = {"xyz": xyz_np, "fo": fo}
    for s in (0.2, 0.5, 1.0):
        w = configs.params_for("batched", voxel_size=s, length_scale=s / 2)
        m = w["grid_side"] ** 2
        row = {}
        for prec_name, prec in (("fp32", vgpr.PREC_FP32), ("fp64", vgpr.PREC_FP64), ("mixed", vgpr.PREC_MIXED)):
            p = vgpr.default_params(**{k: v for k, v in w.items() if k in {f for f, _ in vgpr.Params._fields_}})
            p.precision = prec
            ctx = vgpr.Context(0)
            tuned = autotune.load_cached(p, dev_name)
            if tuned:
                ctx.set_tuning(vgpr.Tuning.from_dict(tuned["tuning"]))
            vox = ctx.voxelize(xyz, p, frame_offsets=fo)
            V = vox.n_vox
            res = (torch.empty((V, m, 4), dtype=torch.float32, device="cuda"),
                   torch.empty(V, dtype=torch.int8, device="cuda"), torch.empty(V, dtype=torch.uint8, device="cuda"))
            for _ in range(args.warmup):
                ctx.voxelize(xyz, p, frame_offsets=fo)
                ctx.fit_predict(xyz, vox, p, out=res)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            steps = max(args.extra_steps, 1)
            for _ in range(steps):
                v2 = ctx.voxelize(xyz, p, frame_offsets=fo)
                ctx.fit_predict(xyz, v2, p, out=res)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            st = res[2].cpu().numpy()
            cnt = vox.counts.cpu().numpy().astype(np.int64)
            solved = (st & vgpr.ST_SOLVED) != 0
            big = np.flatnonzero(solved & (np.minimum(cnt, w["max_pts"]) > 128))
            refd = np.flatnonzero(solved & ((st & vgpr.ST_REFINED) != 0))[:100]
            rest = np.flatnonzero(solved)
            pick = np.union1d(np.union1d(big, refd), rng.choice(rest, size=min(150, len(rest)), replace=False))
            # the sampled voxels' outputs, checked against the oracle by the CPU-baseline leg
            samples[(s, prec_name)] = (V, m, pick, res[0][torch.from_numpy(pick).cuda()].cpu().numpy(),
                                       res[1].cpu().numpy()[pick], st[pick])
            ns = int(solved.sum())
            row[prec_name] = {"solves_per_s": ns / el, "ms_per_step": el * 1e3, "solved_per_step": ns,
                              "refined_per_step": int(((st & vgpr.ST_REFINED) != 0).sum()),
                              "arithmetic": precision_split(np.minimum(cnt, w["max_pts"]), solved, m,
                                                            ctx.tuning().as_dict(), prec_name)["label"],
                              "sample_voxels": int(len(pick)), "max_mean_err_m": None, "max_var_err_prior": None,
                              "max_var_rel_own": None, "sample_voxels_outside_tolerance": None,
                              "within_tolerance": None}
            ctx.close()
            log(f"precision form s={s} {prec_name}: {row[prec_name]}")
        out[f"s={s:g}"] = row
    return out, samples


def serve_leg(args, vgpr) -> dict:
    """Eight sensor streams at 10 Hz through device maps (paper-shaped parameters).

    Each stream's frames are generated once along its trajectory and cycled;
    frames arrive on a wall-clock schedule, are admitted as worker slots and the
    HBM budget allow, and their latency is arrival -> completion.
    """
    from paper_2410_17084_amd import serve
    t0 = time.perf_counter()
    scene = synth.box_scene(clear_radius=12.0)
    frames = [synth.stream_frames(j, args.serve_frames, scene=scene) for j in range(len(synth.STREAM_SENSORS))]
    log(f"serving frames generated in {time.perf_counter() - t0:.1f} s")
    w = configs.params_for("paper_stream")
    p = vgpr.default_params(**{k: v for k, v in w.items() if k in {f for f, _ in vgpr.Params._fields_}})
    be = serve.GpuBackend(p, frames, max_voxels=250000)
    be.warmup()
    sizes = [[len(f) for f in fr] for fr in frames]
    st = serve.serve(be, sizes, rate_hz=10.0, duration_s=args.serve_seconds, workers=8, budget_bytes=8 << 30,
                     m=p.grid_side ** 2)
    out = st.summary()
    out["arrivals"] = "sensors phase-shifted by 1/80 s"
    # held for good by the eight contexts (scratch, map staging, maps), beside the
    # per-frame admission estimate of the frames in flight (max_inflight_bytes)
    out["device_bytes_held"] = be.device_bytes()
    be.close()
    # the same streams with every sensor ticking at the same instant (synchronised sensors):
    # eight frames arrive together each 100 ms, so admission and device overlap are exercised
    be = serve.GpuBackend(p, frames, max_voxels=250000)
    be.warmup()
    sa = serve.serve(be, sizes, rate_hz=10.0, duration_s=max(args.serve_seconds / 2, 1.0), workers=8,
                     budget_bytes=8 << 30, m=p.grid_side ** 2, offsets_s=[0.0] * len(frames)).summary()
    sa["arrivals"] = "all sensors at the same instant"
    out["synchronised"] = sa
    out["streams"] = [f"{b}x{a}" for b, a in synth.STREAM_SENSORS]
    out["points_per_tick"] = int(sum(s[0] for s in sizes))
    out["config"] = "voxel 0.2 m, tau 10, cap 64, 9x9 grid, eta 0.3; 10 frames per stream cycled"
    be.close()
    # throughput of the served form: the same frames as a backlog (all queued at
    # t = 0), continuous batching over 8 worker slots vs one frame at a time,
    # each on fresh maps
    backlog = {}
    for workers in (8, 1):
        be = serve.GpuBackend(p, frames, max_voxels=250000)
        be.warmup()
        sb = serve.serve(be, sizes, rate_hz=10.0, duration_s=1.0, workers=workers, budget_bytes=8 << 30,
                         m=p.grid_side ** 2, realtime=False).summary()
        be.close()
        backlog[f"workers{workers}"] = {k: sb[k] for k in ("frames", "failed", "solves", "solves_per_s", "wall_s",
                                                           "max_inflight")}
    backlog["speedup"] = backlog["workers8"]["solves_per_s"] / backlog["workers1"]["solves_per_s"]
    # the same backlog through maps with the covariance-centred update of type (c)
    # voxels (every re-solve of a voxel in the map stacks its 81 carried rows)
    be = serve.GpuBackend(p, frames, max_voxels=250000, feedback=True)
    be.warmup()
    sb = serve.serve(be, sizes, rate_hz=10.0, duration_s=1.0, workers=8, budget_bytes=8 << 30,
                     m=p.grid_side ** 2, realtime=False).summary()
    conv = sum(mp.stats()["converged"] for mp in be.maps)
    be.close()
    backlog["feedback_workers8"] = {k: sb[k] for k in ("frames", "failed", "solves", "solves_per_s", "wall_s",
                                                       "max_inflight")}
    backlog["feedback_workers8"]["converged_voxels"] = int(conv)
    out["backlog"] = backlog
    return out


FAMILIES = ["voxelize_key", "voxelize_sort", "voxelize_segment", "classify", "nan_rows"] + \
    [f"fit_f32_n{c}" for c in BUCKETS] + [f"fit_f64_n{c}" for c in BUCKETS] + [f"refine_f64_n{c}" for c in BUCKETS] + \
    ["refine_f32_n16"] + \
    [f"fit_mix_n{c}" for c in BUCKETS] + ["gauss_init"]


WORKLOAD_DESC = {
    "spin32": "seeded 32-beam x 1800-azimuth spinning scans, voxel 0.5 m, cap 128, tau 3, 8x8 grid, l 0.25 m, "
              "noise 1e-3",
    "batched": "alternating seeded 128-beam x 1024-azimuth spinning scans and 100k-ray rosette scans (17/23 Hz "
               "petals), voxel 1 m, cap 256, tau 3, 8x8 grid, l 0.5 m, noise 1e-3",
    "aggregated": "each 10 seeded 128-beam x 1024-azimuth scans 0.05 m apart along a path with N(0, 0.01 m) pose "
                  "noise, box scene cleared within 2 m (about 1M points, voxels up to the 512 cap), voxel 0.1 m, "
                  "cap 512, tau 3, 16x16 grid, length scale from PCA, noise 1e-3",
}


def workload_frames(name: str, n_frames: int):
    """Seeded frames of a workload, concatenated, with their frame offsets."""
    if name == "spin32":
        wl = configs.WORKLOADS["spin32"]
        return synth.scan_batch(2, n_frames, n_beams=wl["n_beams"], n_az=wl["n_az"])
    scene = synth.box_scene()
    frames = []
    for k in range(n_frames):
        if name == "batched":
            frames.append(synth.spin_scan(synth.frame_seed(3, k), n_beams=128, n_az=1024, scene=scene) if k % 2 == 0
                          else synth.rosette_scan(synth.frame_seed(3, k), n_pts=100000, frame_index=k, scene=scene))
        else:
            frames.append(synth.aggregated_scans(synth.frame_seed(5, k)))
    offs = np.zeros(n_frames + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(f) for f in frames])
    return np.ascontiguousarray(np.concatenate(frames)), offs


def ctypes_voxelize(ctx, vgpr, xyz, p, fo, keys, offs, cnts, perm) -> int:
    """vgpr_voxelize into preallocated buffers; returns the voxel count."""
    import ctypes as C
    nf = len(fo) - 1
    fo_c = (C.c_int64 * (nf + 1))(*[int(x) for x in fo])
    nv = C.c_int64()
    n = xyz.numel() // 3
    st = ctx.lib.vgpr_voxelize(ctx.h, C.c_void_p(xyz.data_ptr()), n, fo_c, nf, C.byref(p),
                               C.c_void_p(keys.data_ptr()), C.c_void_p(offs.data_ptr()), C.c_void_p(cnts.data_ptr()),
                               C.c_void_p(perm.data_ptr()), n, C.byref(nv), None, None)
    ctx._check(st, "vgpr_voxelize")
    return nv.value


if __name__ == "__main__":
    main()
