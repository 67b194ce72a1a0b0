"""Continuous-batching frame server over device-resident voxel maps.

Each sensor stream owns a context, a HIP stream and a device voxel map
(`vgpr_map`, the global map C of Alg. S1 with the voxel states of Sec. 3.3).
Frames arrive on a wall-clock schedule (10 Hz per sensor by default). A
scheduler admits a frame as soon as
  - its stream has no frame in flight (a map is updated in frame order),
  - a worker slot is free, and
  - the HBM working set of the frames in flight plus this frame's estimate
    fits the admission budget;
admitted frames run `vgpr_map_update` on their own HIP stream from worker
threads (the C calls release the GIL), so frames of different streams
overlap on the device while later arrivals wait for slots. A frame's latency
is its completion time minus its arrival time.

Only scheduling lives here; every step of the hot path runs in the HIP library.
"""
from __future__ import annotations

import heapq
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    stream: int
    index: int           # frame number within its stream
    arrival: float       # scheduled arrival time (s, relative to the run start)
    n_pts: int
    est_bytes: int
    admitted: float = 0.0
    done: float = 0.0
    n_upd: int = 0
    error: str | None = None


@dataclass
class ServeStats:
    requests: list = field(default_factory=list)
    wall: float = 0.0
    max_inflight: int = 0
    max_inflight_bytes: int = 0

    def latencies_ms(self) -> np.ndarray:
        return np.array([(r.done - r.arrival) * 1e3 for r in self.requests if r.error is None])

    def summary(self) -> dict:
        lat = self.latencies_ms()
        solves = sum(r.n_upd for r in self.requests if r.error is None)
        return {
            "frames": len(self.requests),
            "failed": sum(1 for r in self.requests if r.error is not None),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "max_ms": float(lat.max()) if len(lat) else None,
            "solves": int(solves),
            "solves_per_s": solves / self.wall if self.wall else None,
            "wall_s": self.wall,
            "max_inflight": self.max_inflight,
            "max_inflight_bytes": self.max_inflight_bytes,
        }


def working_set_bytes(n_pts: int, m: int) -> int:
    """Upper estimate of the device bytes one frame update touches besides the map.

    Voxelize scratch (~21 B/point), solver scratch (~84 B/voxel) and the output
    rows (16 m B/voxel) with at most one voxel per point. What each stream's
    context holds for good (its scratch and map staging, grown to its largest
    update, and its map) is not part of this per-frame estimate;
    `GpuBackend.device_bytes` reports it.
    """
    return int(n_pts * (21 + 84 + 16 * m + 24))


class Backend:
    """What the scheduler drives: one map update per (stream, frame)."""

    def update(self, stream: int, frame_index: int):  # pragma: no cover - interface
        raise NotImplementedError


class GpuBackend(Backend):
    """Per-stream context, HIP stream and device map; frames resident in HBM.
    feedback=True gives every stream a map with the covariance-centred update of
    type (c) voxels (update mode 1)."""

    def __init__(self, params, frames_by_stream, max_voxels: int, device: int = 0, feedback: bool = False):
        import torch
        self.max_voxels = max_voxels
        self.feedback = feedback

        from . import vgpr
        self.torch = torch
        self.vgpr = vgpr
        self.params = params
        self.m = params.grid_side * params.grid_side
        self.streams = []
        self.ctxs = []
        self.maps = []
        self.frames = []
        self.outs = []
        for frames in frames_by_stream:
            st = torch.cuda.Stream(device=device)
            ctx = vgpr.Context(device, stream=st)
            self.streams.append(st)
            self.ctxs.append(ctx)
            self.maps.append(vgpr.Map(ctx, params, max_voxels, feedback=feedback))
            dev = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(f"cuda:{device}") for f in frames]
            self.frames.append(dev)
            cap = max(len(f) for f in frames)
            self.outs.append((torch.empty(cap, dtype=torch.int64, device=f"cuda:{device}"),
                              torch.empty((cap, self.m, 4), dtype=torch.float32, device=f"cuda:{device}"),
                              torch.empty(cap, dtype=torch.int8, device=f"cuda:{device}"),
                              torch.empty(cap, dtype=torch.uint8, device=f"cuda:{device}")))
        torch.cuda.synchronize(device)
        self.results = {}
        self.keep_results = False

    def warmup(self):
        """Grow each context's scratch and load its kernels before anything is timed.

        Runs voxelize + fit_predict on the stream's largest frame, then the
        stream's first frames through a map of its own (the same update mode),
        so that the map kernels and the fits of re-solved voxels (with the
        feedback update: their carried rows stacked with the new points) have
        run once and the workspace has grown to their size. The stream's own map
        is untouched.
        """
        for s, frames in enumerate(self.frames):
            x = max(frames, key=lambda t: t.shape[0])
            ctx = self.ctxs[s]
            vox = ctx.voxelize(x, self.params)
            ctx.fit_predict(x, vox, self.params)
            scratch_map = self.vgpr.Map(ctx, self.params, self.max_voxels, feedback=self.feedback)
            for f in frames[:3]:
                scratch_map.update(f, out=self.outs[s])
            self.streams[s].synchronize()
            scratch_map.close()

    def device_bytes(self) -> int:
        """Device bytes the streams' contexts hold: scratch, map staging and maps."""
        return sum(c.workspace_bytes() for c in self.ctxs)

    def update(self, stream: int, frame_index: int):
        frames = self.frames[stream]
        x = frames[frame_index % len(frames)]
        k, o, a, s = self.maps[stream].update(x, out=self.outs[stream])
        self.streams[stream].synchronize()
        if self.keep_results:
            self.results[(stream, frame_index)] = (k.cpu().numpy().copy(), o.cpu().numpy().copy(),
                                                   a.cpu().numpy().copy(), s.cpu().numpy().copy())
        return len(k)

    def close(self):
        for mp in self.maps:
            mp.close()
        for c in self.ctxs:
            c.close()


def serve(backend: Backend, frame_sizes: list, rate_hz: float, duration_s: float, workers: int,
          budget_bytes: int, m: int, offsets_s: list | None = None, streams: list | None = None,
          realtime: bool = True) -> ServeStats:
    """Run the arrival schedule through the backend; returns per-request timings.

    frame_sizes[s] lists the point counts of stream s's frames (cycled).
    `streams` restricts the run to a subset of streams (the others send nothing).
    With realtime=False every frame arrives at t = 0 (a backlog), which measures
    throughput rather than latency.
    """
    S = len(frame_sizes)
    active = list(range(S)) if streams is None else list(streams)
    offsets_s = offsets_s or [s / (S * rate_hz) for s in range(S)]
    arrivals = []
    for s in active:
        k = 0
        while True:
            t = offsets_s[s] + k / rate_hz if realtime else 0.0
            if (realtime and t >= duration_s) or (not realtime and k >= int(duration_s * rate_hz)):
                break
            n = frame_sizes[s][k % len(frame_sizes[s])]
            arrivals.append(Request(s, k, t, n, working_set_bytes(n, m)))
            k += 1
    arrivals.sort(key=lambda r: (r.arrival, r.stream))
    pending = {s: deque() for s in active}
    stats = ServeStats()
    lock = threading.Condition()
    busy = set()
    inflight_bytes = [0]
    inflight = [0]
    finished = []

    def run_one(req: Request, t0: float):
        try:
            req.n_upd = backend.update(req.stream, req.index)
        except Exception as e:  # a failed frame is reported, the server keeps going
            req.error = repr(e)
        req.done = time.perf_counter() - t0
        with lock:
            busy.discard(req.stream)
            inflight_bytes[0] -= req.est_bytes
            inflight[0] -= 1
            finished.append(req)
            lock.notify_all()

    t0 = time.perf_counter()
    nxt = 0
    with ThreadPoolExecutor(max_workers=workers) as pool:
        with lock:
            while len(finished) < len(arrivals):
                now = time.perf_counter() - t0
                while nxt < len(arrivals) and arrivals[nxt].arrival <= now:
                    pending[arrivals[nxt].stream].append(arrivals[nxt])
                    nxt += 1
                # admit in arrival order across streams
                cand = [(q[0].arrival, s) for s, q in pending.items() if q and s not in busy]
                heapq.heapify(cand)
                while cand and inflight[0] < workers:
                    _, s = heapq.heappop(cand)
                    req = pending[s][0]
                    if inflight[0] > 0 and inflight_bytes[0] + req.est_bytes > budget_bytes:
                        break  # wait for memory; a lone frame is always admitted
                    pending[s].popleft()
                    busy.add(s)
                    inflight[0] += 1
                    inflight_bytes[0] += req.est_bytes
                    stats.max_inflight = max(stats.max_inflight, inflight[0])
                    stats.max_inflight_bytes = max(stats.max_inflight_bytes, inflight_bytes[0])
                    req.admitted = now
                    pool.submit(run_one, req, t0)
                wait = None
                if nxt < len(arrivals):
                    wait = max(0.0, arrivals[nxt].arrival - (time.perf_counter() - t0))
                lock.wait(timeout=wait if wait is not None else 1.0)
    stats.wall = time.perf_counter() - t0
    stats.requests = sorted(finished, key=lambda r: (r.stream, r.index))
    return stats
