"""Seeded synthetic LiDAR inputs shared by the HIP path, its tests and the bench.

This module only *generates* point clouds. It holds none of the Voxel-GPR
arithmetic (no voxel keys, no frames, no kernels, no solves), so the oracle and
the HIP path can both consume its output without sharing method code.

Every generator takes an explicit seed and returns float32 points of shape
(N, 3) in the world frame (metres), the layout both sides read (12 B/point,
x, y, z interleaved).

Shapes follow the sensors the paper evaluates on (Sec. 4.1 and the
supplementary dataset description): multi-line spinning LiDARs at 10 Hz, a
non-repetitive rosette scanner, and a 0.2 m default voxel (Table S6). The
paper's recorded datasets are not available, so these scenes stand in for them.

Scene recipe (one shared box world): a 100 m square [-50, 50]^2, ground plane
z = 0, 200 axis-aligned boxes whose three sides are U(0.5, 5) m, standing on
the ground with centres uniform in the square; boxes whose footprint comes
within 4 m of the origin are removed so that sensors near the origin start
in free space.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "BoxScene", "box_scene", "planes_cloud", "spin_directions", "rosette_directions",
    "cast_rays", "spin_scan", "rosette_scan", "scan_batch", "yaw_matrix", "rotation_rpy",
    "spline_trajectory", "stream_frames", "STREAM_SENSORS", "frame_seed", "SCENE_SEED",
]

# (beams, azimuth steps) of the eight serving streams: 16- to 128-beam spinning
# LiDARs at 512..2048 azimuth steps, 630,784 rays per 10 Hz tick in total.
STREAM_SENSORS = [(16, 512), (16, 2048), (32, 1024), (32, 2048), (64, 512), (64, 1024), (128, 1024), (128, 2048)]

SCENE_SEED = 0


def frame_seed(config: int, k: int) -> int:
    """Seed of frame k of workload `config` (1-based config index)."""
    return 1000 * config + k


@dataclass(frozen=True)
class BoxScene:
    lo: np.ndarray  # (B, 3) box minimum corners, float64
    hi: np.ndarray  # (B, 3) box maximum corners, float64
    half_extent: float = 50.0


def box_scene(seed: int = SCENE_SEED, n_boxes: int = 200, half_extent: float = 50.0,
              clear_radius: float = 4.0) -> BoxScene:
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.uniform(0.5, 5.0, size=(n_boxes, 3))
    cxy = rng.uniform(-half_extent, half_extent, size=(n_boxes, 2))
    lo = np.empty((n_boxes, 3))
    hi = np.empty((n_boxes, 3))
    lo[:, :2] = cxy - sides[:, :2] / 2
    hi[:, :2] = cxy + sides[:, :2] / 2
    lo[:, 2] = 0.0
    hi[:, 2] = sides[:, 2]
    # distance from the origin to each footprint rectangle
    dx = np.maximum(np.maximum(lo[:, 0], -hi[:, 0]), 0.0)
    dy = np.maximum(np.maximum(lo[:, 1], -hi[:, 1]), 0.0)
    keep = np.hypot(dx, dy) >= clear_radius
    return BoxScene(lo=lo[keep], hi=hi[keep], half_extent=half_extent)


def planes_cloud(seed: int, n_pts: int = 20000, cube: float = 20.0, n_planes: int = 3,
                 noise: float = 0.02) -> np.ndarray:
    """Points uniform on `n_planes` random planes clipped to a cube, plus normal noise.

    Planes have random unit normals and pass through random centres inside the
    inner half of the cube [-cube/2, cube/2]^3. Each point gets N(0, noise^2)
    displacement along its plane's normal.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = cube / 2
    per = [n_pts // n_planes + (1 if i < n_pts % n_planes else 0) for i in range(n_planes)]
    out = []
    for npl in per:
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        c = rng.uniform(-h / 2, h / 2, size=3)
        a = np.cross(nrm, [1.0, 0.0, 0.0] if abs(nrm[0]) < 0.9 else [0.0, 1.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(nrm, a)
        r = cube * math.sqrt(3.0)
        got = []
        n_got = 0
        while n_got < npl:
            uv = rng.uniform(-r, r, size=(4 * npl, 2))
            p = c + uv[:, :1] * a + uv[:, 1:] * b
            inside = np.all(np.abs(p) <= h, axis=1)
            p = p[inside]
            got.append(p)
            n_got += len(p)
        p = np.concatenate(got)[:npl]
        p = p + rng.normal(0.0, noise, size=(npl, 1)) * nrm
        out.append(p)
    pts = np.concatenate(out)
    pts = pts[rng.permutation(len(pts))]
    return np.ascontiguousarray(pts, dtype=np.float32)


def yaw_matrix(yaw: float) -> np.ndarray:
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rotation_rpy(roll: float, pitch: float, yaw: float) -> np.ndarray:
    """Rotation R = Rz(yaw) Ry(pitch) Rx(roll) (sensor to world)."""
    cr, sr = math.cos(roll), math.sin(roll)
    cp, sp = math.cos(pitch), math.sin(pitch)
    rx = np.array([[1.0, 0.0, 0.0], [0.0, cr, -sr], [0.0, sr, cr]])
    ry = np.array([[cp, 0.0, sp], [0.0, 1.0, 0.0], [-sp, 0.0, cp]])
    return yaw_matrix(yaw) @ ry @ rx


def spline_trajectory(seed: int, n_frames: int, rate_hz: float = 10.0, speed=(1.0, 10.0), radius: float = 9.0,
                      tilt_deg: float = 2.0):
    """Poses along a uniform cubic B-spline through seeded waypoints in a disc of `radius`.

    The sensor moves at a seeded constant speed in [speed[0], speed[1]] m/s,
    yaws along the tangent, and rolls / pitches with N(0, tilt_deg) noise.
    Returns a list of (position (3,), rotation (3, 3)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.uniform(*speed)
    n_way = 12
    ang = np.sort(rng.uniform(0, 2 * np.pi, n_way))
    rad = radius * np.sqrt(rng.uniform(0.2, 1.0, n_way))
    way = np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)
    way = np.concatenate([way, way[:3]])  # closed loop
    # dense sampling of the B-spline, then constant-speed reparametrisation
    ts = np.linspace(0, 1, 64, endpoint=False)
    basis = np.stack([(1 - ts) ** 3, 3 * ts ** 3 - 6 * ts ** 2 + 4, -3 * ts ** 3 + 3 * ts ** 2 + 3 * ts + 1,
                      ts ** 3], 1) / 6.0
    curve = np.concatenate([basis @ way[i:i + 4] for i in range(n_way)])
    seg = np.linalg.norm(np.diff(curve, axis=0, append=curve[:1]), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    total = arc[-1]
    poses = []
    for k in range(n_frames):
        s_ = (v * k / rate_hz) % total
        i = int(np.searchsorted(arc, s_, side="right") - 1)
        i = min(i, len(curve) - 1)
        a, b = curve[i], curve[(i + 1) % len(curve)]
        t = (s_ - arc[i]) / max(seg[i], 1e-9)
        pos = a + t * (b - a)
        yaw = math.atan2(b[1] - a[1], b[0] - a[0])
        roll, pitch = np.deg2rad(rng.normal(0, tilt_deg, 2))
        poses.append((np.array([pos[0], pos[1], 1.8]), rotation_rpy(roll, pitch, yaw)))
    return poses


def spin_directions(n_beams: int, n_az: int, elev_deg=(-15.0, 15.0)) -> np.ndarray:
    """Unit ray directions of a spinning LiDAR in the sensor frame, beam-major."""
    el = np.deg2rad(np.linspace(elev_deg[0], elev_deg[1], n_beams))
    az = 2 * np.pi * np.arange(n_az) / n_az
    el, az = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], axis=-1)
    return d.reshape(-1, 3)


def rosette_directions(n_pts: int, t0: float, duration: float = 0.1, f1: float = 17.0,
                       f2: float = 23.0, half_fov_deg: float = 35.0) -> np.ndarray:
    """Non-repetitive rosette scan pattern (two counter-rotating prisms), forward = +x.

    The deflection is the half-sum of two unit phasors turning at f1 and -f2 Hz,
    scaled to the half field of view; time continues across frames through t0.
    """
    t = t0 + duration * np.arange(n_pts) / n_pts
    a = 2 * np.pi * f1 * t
    b = 2 * np.pi * f2 * t
    u = 0.5 * (np.cos(a) + np.cos(b))
    v = 0.5 * (np.sin(a) - np.sin(b))
    th = np.deg2rad(half_fov_deg)
    ang_y = th * u
    ang_z = th * v
    d = np.stack([np.ones_like(ang_y), np.tan(ang_y), np.tan(ang_z)], axis=-1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def cast_rays(scene: BoxScene, origin: np.ndarray, dirs: np.ndarray, max_range: float = 120.0,
              n_bins: int = 720) -> np.ndarray:
    """Nearest hit distance of each ray against the ground plane and the boxes (inf if none).

    Boxes are culled per ray by azimuth: each box covers an azimuth interval
    seen from the origin, rays are binned by azimuth, and only (ray, box) pairs
    sharing a bin go through the slab test.
    """
    origin = np.asarray(origin, dtype=np.float64)
    dirs = np.asarray(dirs, dtype=np.float64)
    t = np.full(len(dirs), np.inf)
    down = dirs[:, 2] < -1e-12
    t[down] = -origin[2] / dirs[down, 2]
    if len(scene.lo):
        binw = 2 * np.pi / n_bins
        az = np.mod(np.arctan2(dirs[:, 1], dirs[:, 0]), 2 * np.pi)
        rbin = np.minimum((az / binw).astype(np.int64), n_bins - 1)
        order = np.argsort(rbin, kind="stable")
        starts = np.searchsorted(rbin[order], np.arange(n_bins + 1))
        cx = np.stack([scene.lo[:, 0], scene.hi[:, 0], scene.hi[:, 0], scene.lo[:, 0]], 1) - origin[0]
        cy = np.stack([scene.lo[:, 1], scene.lo[:, 1], scene.hi[:, 1], scene.hi[:, 1]], 1) - origin[1]
        mid = np.arctan2(cy.mean(1), cx.mean(1))
        rel = np.mod(np.arctan2(cy, cx) - mid[:, None] + np.pi, 2 * np.pi) - np.pi
        a0 = mid + rel.min(1) - binw
        a1 = mid + rel.max(1) + binw
        b0 = np.floor(a0 / binw).astype(np.int64)
        b1 = np.floor(a1 / binw).astype(np.int64)
        ray_idx = []
        box_idx = []
        for k in range(len(scene.lo)):
            bins = np.mod(np.arange(b0[k], b1[k] + 1), n_bins)
            rs = np.concatenate([order[starts[b]:starts[b + 1]] for b in bins])
            ray_idx.append(rs)
            box_idx.append(np.full(len(rs), k))
        ri = np.concatenate(ray_idx)
        bi = np.concatenate(box_idx)
        d = dirs[ri]
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / d
            t1 = (scene.lo[bi] - origin) * inv
            t2 = (scene.hi[bi] - origin) * inv
        tn = np.nanmax(np.minimum(t1, t2), axis=1)
        tf = np.nanmin(np.maximum(t1, t2), axis=1)
        hit = (tf >= tn) & (tn > 1e-6)
        np.minimum.at(t, ri[hit], tn[hit])
    t[t > max_range] = np.inf
    return t


def spin_scan(seed: int, n_beams: int = 32, n_az: int = 1800, position=None, yaw=None,
              scene: BoxScene | None = None, sensor_height: float = 1.8, range_noise: float = 0.02,
              max_range: float = 120.0, elev_deg=(-15.0, 15.0), rotation=None) -> np.ndarray:
    """One spinning-LiDAR scan of the box scene, world frame, misses dropped.

    Without an explicit pose the sensor sits at a seeded position within 2 m of
    the origin (inside the box-free disc) with a seeded yaw.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = scene if scene is not None else box_scene()
    if position is None:
        r = 2.0 * math.sqrt(rng.uniform())
        phi = rng.uniform(0, 2 * np.pi)
        position = (r * math.cos(phi), r * math.sin(phi))
    if yaw is None:
        yaw = rng.uniform(0, 2 * np.pi)
    z = position[2] if len(position) > 2 else sensor_height
    o = np.array([position[0], position[1], z], dtype=np.float64)
    R = yaw_matrix(yaw) if rotation is None else np.asarray(rotation, dtype=np.float64)
    d = spin_directions(n_beams, n_az, elev_deg) @ R.T
    t = cast_rays(scene, o, d, max_range)
    ok = np.isfinite(t)
    t = t[ok] + rng.normal(0.0, range_noise, size=int(ok.sum()))
    pts = o + t[:, None] * d[ok]
    return np.ascontiguousarray(pts, dtype=np.float32)


def rosette_scan(seed: int, n_pts: int = 100000, frame_index: int = 0, position=None, yaw=None,
                 scene: BoxScene | None = None, sensor_height: float = 1.8, pitch_deg: float = -10.0,
                 range_noise: float = 0.02, max_range: float = 120.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = scene if scene is not None else box_scene()
    if position is None:
        r = 2.0 * math.sqrt(rng.uniform())
        phi = rng.uniform(0, 2 * np.pi)
        position = (r * math.cos(phi), r * math.sin(phi))
    if yaw is None:
        yaw = rng.uniform(0, 2 * np.pi)
    d = rosette_directions(n_pts, t0=0.1 * frame_index)
    p = math.radians(pitch_deg)
    pitch = np.array([[math.cos(p), 0, -math.sin(p)], [0, 1, 0], [math.sin(p), 0, math.cos(p)]])
    d = d @ pitch.T @ yaw_matrix(yaw).T
    o = np.array([position[0], position[1], sensor_height], dtype=np.float64)
    t = cast_rays(scene, o, d, max_range)
    ok = np.isfinite(t)
    t = t[ok] + rng.normal(0.0, range_noise, size=int(ok.sum()))
    pts = o + t[:, None] * d[ok]
    return np.ascontiguousarray(pts, dtype=np.float32)


def scan_batch(config: int, n_frames: int, first: int = 0, **kw):
    """`n_frames` seeded spinning scans (seeds frame_seed(config, first + k)).

    Returns (points (N, 3) float32, frame_offsets (n_frames + 1,) int64) with the
    frames concatenated in order.
    """
    scene = kw.pop("scene", None) or box_scene()
    frames = [spin_scan(frame_seed(config, first + k), scene=scene, **kw) for k in range(n_frames)]
    offs = np.zeros(n_frames + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(f) for f in frames])
    return np.ascontiguousarray(np.concatenate(frames)), offs


def aggregated_scans(seed: int, n_scans: int = 10, n_beams: int = 128, n_az: int = 1024, spacing: float = 0.05,
                     pose_noise: float = 0.01, scene: BoxScene | None = None, clear_radius: float = 2.0) -> np.ndarray:
    """A map-update frame: `n_scans` scans taken along a straight path, concatenated.

    Scan k is taken at start + k * spacing along a seeded heading (0.05 m: a
    platform at 0.5 m/s scanning at 10 Hz), with the position perturbed by
    N(0, pose_noise) m per axis (a registration error), and the same heading as
    yaw. Without an explicit scene the box world is cleared only within
    `clear_radius` of the origin, so that surfaces 2-3 m from the sensor are hit
    by every scan and their 0.1 m voxels fill to several hundred points (about
    1M points per frame, voxels up to and beyond a 512-point cap). Seeds: path
    `seed`, scan k seed + 1 + k.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    scene = scene if scene is not None else box_scene(clear_radius=clear_radius)
    heading = rng.uniform(0, 2 * np.pi)
    start = rng.uniform(-1.0, 1.0, size=2) - 0.5 * (n_scans - 1) * spacing * np.array([math.cos(heading),
                                                                                        math.sin(heading)])
    scans = []
    for k in range(n_scans):
        xy = start + k * spacing * np.array([math.cos(heading), math.sin(heading)])
        pos = np.array([xy[0], xy[1], 1.8]) + rng.normal(0.0, pose_noise, size=3)
        scans.append(spin_scan(seed + 1 + k, n_beams=n_beams, n_az=n_az, position=tuple(pos), yaw=heading,
                               scene=scene))
    return np.ascontiguousarray(np.concatenate(scans))


def stream_frames(stream: int, n_frames: int, rate_hz: float = 10.0, scene: BoxScene | None = None):
    """Seeded frames of serving stream `stream` (sensor STREAM_SENSORS[stream]) along its trajectory.

    The scene has a 12 m clearing around the origin so the trajectories stay in
    free space; seeds: trajectory 10^4 (stream + 1), frame k 10^4 (stream + 1) + k.
    """
    scene = scene if scene is not None else box_scene(clear_radius=12.0)
    beams, az = STREAM_SENSORS[stream % len(STREAM_SENSORS)]
    poses = spline_trajectory(10 ** 4 * (stream + 1), n_frames, rate_hz)
    return [spin_scan(10 ** 4 * (stream + 1) + k, n_beams=beams, n_az=az, position=pos, rotation=R, scene=scene)
            for k, (pos, R) in enumerate(poses)]
