"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every case prints what names it before touching the GPU.
"""
import numpy as np
import pytest

from oracle import vgpr_oracle as O
from paper_2410_17084_amd import configs, synth
from tests import parity

pytestmark = pytest.mark.gpu


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2410_17084_amd import vgpr
    ctx = vgpr.Context(0)
    yield torch, vgpr, ctx
    torch.cuda.synchronize()
    ctx.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def say(*a):
    print("[case]", *a, flush=True)


# ---------------------------------------------------------------------------
# voxelize: bit-exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["planes", "spin32"])
def test_voxelize_workloads(env, name):
    torch, vgpr, ctx = env
    w = configs.WORKLOADS[name]
    xyz = synth.planes_cloud(synth.frame_seed(1, 0)) if name == "planes" else synth.spin_scan(synth.frame_seed(2, 0))
    say("voxelize", name, xyz.shape)
    p = parity.gpu_params(vgpr, w)
    gv = ctx.voxelize(dev(torch, xyz), p)
    parity.compare_voxelize(O.voxelize(xyz, w["voxel_size"]), gv)


def test_voxelize_edge_values(env):
    torch, vgpr, ctx = env
    r = rng(7)
    s = 0.25
    xyz = r.uniform(-3, 3, size=(9001, 3)).astype(np.float32)          # ragged tail over 4096-tiles
    xyz[:300] = (r.integers(-12, 12, size=(300, 3)) * s).astype(np.float32)  # on voxel boundaries
    xyz[300] = [-0.0, 0.0, -0.0]
    xyz[301:320] = xyz[301]                                              # duplicates
    xyz[400] = [np.nan, 0, 0]
    xyz[401] = [0, np.inf, 0]
    xyz[402] = [0, 0, -np.inf]
    xyz[9000] = [1e-30, -1e-30, 0.0]
    say("voxelize edge values", xyz.shape)
    gv = ctx.voxelize(dev(torch, xyz), vgpr.default_params(voxel_size=s))
    parity.compare_voxelize(O.voxelize(xyz, s), gv)


@pytest.mark.parametrize("n", [0, 1, 2, 4095, 4096, 4097, 200003])
def test_voxelize_sizes(env, n):
    torch, vgpr, ctx = env
    xyz = rng(100 + n).normal(0, 20, size=(n, 3)).astype(np.float32)
    say("voxelize size", n)
    gv = ctx.voxelize(dev(torch, xyz.reshape(-1, 3)) if n else torch.zeros((0, 3), device="cuda"),
                      vgpr.default_params(voxel_size=0.2))
    parity.compare_voxelize(O.voxelize(xyz.reshape(-1, 3), 0.2), gv)


def test_voxelize_frame_batch(env):
    torch, vgpr, ctx = env
    r = rng(8)
    frames = [r.normal(0, 5, size=(k, 3)).astype(np.float32) for k in (5000, 0, 1, 12000, 3)]
    frames[3][7] = np.nan
    xyz = np.concatenate(frames)
    offs = np.cumsum([0] + [len(f) for f in frames])
    say("voxelize frame batch", [len(f) for f in frames])
    gv = ctx.voxelize(dev(torch, xyz), vgpr.default_params(voxel_size=0.5), frame_offsets=offs)
    parity.compare_voxelize(O.voxelize(xyz, 0.5, offs), gv)


def test_voxelize_many_frames(env):
    torch, vgpr, ctx = env
    xyz, offs = synth.scan_batch(2, 3, n_beams=16, n_az=900)
    # 300 frames of small slices exercise the second frame-digit pass
    cut = np.linspace(0, len(xyz), 301).astype(np.int64)
    say("voxelize 300 frames", len(xyz))
    gv = ctx.voxelize(dev(torch, xyz), vgpr.default_params(voxel_size=0.5), frame_offsets=cut)
    parity.compare_voxelize(O.voxelize(xyz, 0.5, cut), gv)


def test_voxelize_range_and_capacity_errors(env):
    torch, vgpr, ctx = env
    xyz = np.array([[0, 0, 0], [(2 ** 20) * 0.5, 0, 0]], np.float32)
    say("voxelize range error")
    with pytest.raises(vgpr.VgprError) as ei:
        ctx.voxelize(dev(torch, xyz), vgpr.default_params(voxel_size=0.5))
    assert ei.value.status == vgpr.E_RANGE
    xyz = rng(9).uniform(-5, 5, size=(1000, 3)).astype(np.float32)
    nv = len(O.voxelize(xyz, 0.5)["keys"])
    say("voxelize capacity error", nv)
    with pytest.raises(vgpr.VgprError) as ei:
        ctx.voxelize(dev(torch, xyz), vgpr.default_params(voxel_size=0.5), cap_vox=nv - 1)
    assert ei.value.status == vgpr.E_CAPACITY


# ---------------------------------------------------------------------------
# fit_predict: tolerances of tests/parity.py
# ---------------------------------------------------------------------------
def run_fit(env, xyz, w, **kw):
    torch, vgpr, ctx = env
    p = parity.gpu_params(vgpr, w, **kw)
    x = dev(torch, xyz)
    gv = ctx.voxelize(x, p)
    out = ctx.fit_predict(x, gv, p)
    torch.cuda.synchronize()
    return gv, out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["planes", "spin32"])
def test_fit_workloads(env, name, prec):
    torch, vgpr, ctx = env
    w = configs.WORKLOADS[name]
    xyz = synth.planes_cloud(synth.frame_seed(1, 0)) if name == "planes" else synth.spin_scan(synth.frame_seed(2, 0))
    say("fit", name, prec, xyz.shape)
    gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_FP32 if prec == "fp32" else vgpr.PREC_FP64)
    ov = O.voxelize(xyz, w["voxel_size"])
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
    print(name, prec, stats)
    assert stats["solved"] > 1000


def test_fit_bench_batch_sampled(env):
    """The timed step at full size: the 64-scan spinning batch (2.55M points) voxelized and fitted in
    one call each, in FP32 mode, under the launch choices taken from the tuning cache for this
    device (as the bench does). The voxel arrays are compared in full; outputs for a seeded sample
    (40 voxels of every scan, and every voxel with more than 64 kept points) against the oracle
    voxel by voxel."""
    torch, vgpr, ctx = env
    from paper_2410_17084_amd import autotune
    w = configs.WORKLOADS["spin32"]
    xyz, offs = synth.scan_batch(2, 64, n_beams=w["n_beams"], n_az=w["n_az"])
    p = parity.gpu_params(vgpr, w, precision=vgpr.PREC_FP32)
    props = torch.cuda.get_device_properties(0)
    dev_name = f"{getattr(props, 'gcnArchName', 'gpu').split(':')[0]}x{props.multi_processor_count}cu"
    default = ctx.tuning().as_dict()
    tuned = autotune.load_cached(p, dev_name)
    say("fit 64-scan batch", xyz.shape, tuned["tuning"] if tuned else "library defaults")
    try:
        if tuned:
            ctx.set_tuning(vgpr.Tuning.from_dict(tuned["tuning"]))
        x = dev(torch, xyz)
        gv = ctx.voxelize(x, p, frame_offsets=offs)
        out, axis, status = ctx.fit_predict(x, gv, p)
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning(vgpr.Tuning.from_dict(default))
    ov = O.voxelize(xyz, w["voxel_size"], offs)
    parity.compare_voxelize(ov, gv)
    r = rng(64)
    fv = ov["frame_vox"]
    sample = set()
    for f in range(len(offs) - 1):
        lo, hi = int(fv[f]), int(fv[f + 1])
        sample.update(r.choice(np.arange(lo, hi), size=min(40, hi - lo), replace=False).tolist())
    sample.update(np.nonzero(np.minimum(ov["counts"], w["max_pts"]) > 64)[0].tolist())
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status, voxels=sorted(sample))
    print("64-scan batch", len(sample), stats)
    assert stats["solved"] > 2000


def _ragged_voxels(seed, sizes, s=0.5, noise=0.01, tilt=True):
    """One voxel per requested point count, on a noisy (tilted) plane, scattered in space."""
    r = rng(seed)
    pts = []
    for i, n in enumerate(sizes):
        k = np.array([3 * i - 500, (7 * i) % 200 - 100, (i % 11) - 5])
        uv = r.uniform(0.02, 0.98, size=(n, 2)) * s
        h = 0.5 * s + (0.2 * uv[:, 0] - 0.1 * uv[:, 1] if tilt else 0) + r.normal(0, noise, n)
        p = np.stack([uv[:, 0], uv[:, 1], np.clip(h, 0.01 * s, 0.99 * s)], 1) + k * s
        pts.append(p)
    xyz = np.concatenate(pts).astype(np.float32)
    return xyz[r.permutation(len(xyz))]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fit_every_size_in_one_call(env, prec):
    """n = 1..160 in one launch: every bucket, its edges, the cap and tau."""
    torch, vgpr, ctx = env
    sizes = list(range(1, 161))
    xyz = _ragged_voxels(11, sizes)
    w = dict(configs.params_for("spin32"), max_pts=128, min_pts=3)
    say("fit every size", prec, len(xyz))
    gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_FP32 if prec == "fp32" else vgpr.PREC_FP64)
    ov = O.voxelize(xyz, w["voxel_size"])
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
    assert stats["solved"] == 160 - 2
    caps = status.cpu().numpy() & vgpr.ST_CAPPED
    assert caps.astype(bool).sum() == 32


LARGE_SIZES = [3, 40, 100, 129, 130, 160, 161, 200, 255, 256, 257, 300, 384, 511, 512, 513, 700]


@pytest.mark.parametrize("nq,ls_mode", [(4, 0), (9, 0), (16, 0), (16, 1)])
def test_fit_large_voxels(env, nq, ls_mode):
    """Voxels of 129..512 kept points (tiled solver) beside small ones, every grid size class."""
    torch, vgpr, ctx = env
    xyz = _ragged_voxels(21 + nq + ls_mode, LARGE_SIZES)
    w = dict(configs.params_for("spin32"), max_pts=512, min_pts=3, grid_side=nq, ls_mode=ls_mode)
    for prec in (vgpr.PREC_FP32, vgpr.PREC_FP64):
        say("fit large voxels", nq, ls_mode, prec, len(xyz))
        gv, (out, axis, status) = run_fit(env, xyz, w, precision=prec)
        ov = O.voxelize(xyz, w["voxel_size"])
        stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
        assert stats["solved"] == len(LARGE_SIZES)
        assert (status.cpu().numpy() & vgpr.ST_CAPPED).astype(bool).sum() == 2
        print(stats)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fit_tiled_merge(env, prec):
    """The 256- and 512-point buckets as one longest-first launch of the 512-point solver:
    every voxel is solved the same way as in its own bucket's launch (bit-identical), and
    matches the oracle."""
    torch, vgpr, ctx = env
    p_ = {"fp64": vgpr.PREC_FP64, "mixed": vgpr.PREC_MIXED}[prec]
    sizes = LARGE_SIZES + [140, 250, 260, 380, 500] * 3
    xyz = _ragged_voxels(77, sizes)
    w = dict(configs.params_for("spin32"), max_pts=512, min_pts=3, grid_side=16, ls_mode=1)
    default = ctx.tuning().as_dict()
    outs = []
    try:
        for merge in (0, 1):
            say("fit tiled merge", prec, merge, len(xyz))
            t = dict(default)
            t.update(tiled_merge=merge, tile_first_bucket=4)
            ctx.set_tuning(vgpr.Tuning.from_dict(t))
            gv, res = run_fit(env, xyz, w, precision=p_)
            outs.append([r.cpu().numpy() for r in res])
    finally:
        ctx.set_tuning(vgpr.Tuning.from_dict(default))
    for g, r in zip(outs[1], outs[0]):
        assert np.array_equal(g, r, equal_nan=True)
    ov = O.voxelize(xyz, w["voxel_size"])
    out, axis, status = (torch.from_numpy(x) for x in outs[1])
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
    assert stats["solved"] == len(sizes)
    print(stats)


@pytest.mark.parametrize("tile_first", [2, 5])
def test_fit_mixed_precision(env, tile_first):
    """MIXED mode (FP32 tiles, the query rows as one FP32 product with the formed inverse,
    FP64 mean and refinement) on every size class, two grid sizes, and a 128-beam scan at
    1 m and 0.5 m voxels (at 0.5 m split-BF16 tile products in the triangular recurrence
    left a 198-point voxel with 1.3e-3 s_f^2 of variance error): within the tolerances."""
    torch, vgpr, ctx = env
    default = ctx.tuning().as_dict()
    t = dict(default)
    t["tile_first_bucket"] = tile_first
    ctx.set_tuning(vgpr.Tuning.from_dict(t))
    try:
        for nq, ls_mode in ((8, 0), (16, 1)):
            xyz = _ragged_voxels(31 + nq, LARGE_SIZES)
            w = dict(configs.params_for("spin32"), max_pts=512, min_pts=3, grid_side=nq, ls_mode=ls_mode)
            say("fit mixed", tile_first, nq, ls_mode, len(xyz))
            gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_MIXED)
            ov = O.voxelize(xyz, w["voxel_size"])
            stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
            assert stats["solved"] == len(LARGE_SIZES)
            print("mixed", tile_first, nq, stats)
        xyz = synth.spin_scan(synth.frame_seed(3, 0), n_beams=128, n_az=1024)
        for vs in (1.0, 0.5):
            w = configs.params_for("batched", voxel_size=vs, length_scale=vs / 2)
            say("fit mixed batched", tile_first, "voxel", vs, len(xyz))
            gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_MIXED)
            ov = O.voxelize(xyz, w["voxel_size"])
            stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
            print("mixed batched", tile_first, vs, stats)
    finally:
        ctx.set_tuning(vgpr.Tuning.from_dict(default))


def test_fit_mixed_batched_batch_large_voxels(env):
    """MIXED mode on the 16-frame batched batch (128-beam and rosette scans) at 1 m voxels under
    the cached launch choices, every voxel above 128 points against the oracle. With one FP64
    refinement step of alpha, five of these voxels (condition n s_f^2 / sigma^2 up to 2.6e5) kept
    up to 1.5e-4 m of mean error; two steps bring them within the tolerance."""
    torch, vgpr, ctx = env
    from paper_2410_17084_amd import autotune
    frames = []
    scene = synth.box_scene()
    for k in range(16):
        frames.append(synth.spin_scan(synth.frame_seed(3, k), n_beams=128, n_az=1024, scene=scene) if k % 2 == 0
                      else synth.rosette_scan(synth.frame_seed(3, k), n_pts=100000, frame_index=k, scene=scene))
    xyz = np.concatenate(frames)
    offs = np.cumsum([0] + [len(f) for f in frames])
    w = configs.params_for("batched")
    p = parity.gpu_params(vgpr, w, precision=vgpr.PREC_MIXED)
    props = torch.cuda.get_device_properties(0)
    dev_name = f"{getattr(props, 'gcnArchName', 'gpu').split(':')[0]}x{props.multi_processor_count}cu"
    default = ctx.tuning().as_dict()
    tuned = autotune.load_cached(p, dev_name)
    say("fit mixed, batched batch", xyz.shape, tuned["tuning"] if tuned else "library defaults")
    try:
        if tuned:
            ctx.set_tuning(vgpr.Tuning.from_dict(tuned["tuning"]))
        x = dev(torch, xyz)
        gv = ctx.voxelize(x, p, frame_offsets=offs)
        out, axis, status = ctx.fit_predict(x, gv, p)
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning(vgpr.Tuning.from_dict(default))
    ov = O.voxelize(xyz, w["voxel_size"], offs)
    big = np.flatnonzero(np.minimum(ov["counts"], w["max_pts"]) > 128)
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status, voxels=big)
    print("mixed batched batch, voxels above 128 points", len(big), stats)
    assert stats["solved"] == len(big) > 500


@pytest.mark.parametrize("scan", ["spin128", "rosette"])
def test_fit_batched_workload(env, scan):
    """128-beam spinning scan and rosette scan at 1 m voxels, cap 256: every voxel against the oracle."""
    torch, vgpr, ctx = env
    if scan == "spin128":
        xyz = synth.spin_scan(synth.frame_seed(3, 0), n_beams=128, n_az=1024)
    else:
        xyz = synth.rosette_scan(synth.frame_seed(3, 1), n_pts=100000)
    w = configs.params_for("batched")
    say("fit batched workload", scan, len(xyz))
    gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_FP32)
    ov = O.voxelize(xyz, w["voxel_size"])
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
    print(scan, stats)


def test_fit_aggregated_workload_sampled(env):
    """About 0.9M aggregated points, voxel 0.1 m, cap 512, 16x16 grid, PCA length scale.

    Keys and order are compared in full; GP outputs on every voxel above 64
    points and a seeded 1% sample of the rest.
    """
    torch, vgpr, ctx = env
    xyz = synth.aggregated_scans(synth.frame_seed(5, 0))
    w = configs.params_for("aggregated")
    say("fit aggregated workload", len(xyz))
    gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_FP32)
    ov = O.voxelize(xyz, w["voxel_size"])
    parity.compare_voxelize(ov, gv)
    counts = ov["counts"]
    pick = np.flatnonzero(counts > 64)
    rest = np.flatnonzero(counts <= 64)
    pick = np.union1d(pick, rng(15).choice(rest, size=len(rest) // 100, replace=False))
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status, voxels=pick)
    print(stats)
    st = status.cpu().numpy()
    assert (st & vgpr.ST_SOLVED).astype(bool).sum() == int((np.minimum(counts, 512) >= 3).sum())


@pytest.mark.parametrize("nq", [8, 16])
def test_fit_fp32_refinement_pass(env, nq):
    """FP32 mode: the 16-point wave bucket hands voxels with small pivots to a second FP32 pass
    that takes one FP64 refinement step of alpha with the float factor. With a conditioning
    threshold of 1 every solved voxel of the bucket goes through it (REFINED set, outputs within
    the tolerances); with both thresholds out of reach none does (unrefined FP32 means may then
    exceed 1e-4 m, which is what the thresholds are for: only the bits are checked there)."""
    torch, vgpr, ctx = env
    w = dict(configs.params_for("spin32"), grid_side=nq)
    xyz = synth.spin_scan(synth.frame_seed(2, 7))
    ov = O.voxelize(xyz, w["voxel_size"])
    small = np.flatnonzero((np.minimum(ov["counts"], w["max_pts"]) >= w["min_pts"]) &
                           (np.minimum(ov["counts"], w["max_pts"]) <= 16))
    for cond, thr, expect in ((1.0, 40.0, True), (1e30, 1e30, False)):
        say("fp32 refinement pass, grid", nq, "cond threshold", cond, "refine threshold", thr)
        gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_FP32, cond_threshold=cond,
                                          refine_threshold=thr)
        st = status.cpu().numpy()
        ref_bits = (st[small] & vgpr.ST_REFINED) != 0
        assert ref_bits.all() if expect else not ref_bits.any(), (int(ref_bits.sum()), len(small))
        if expect:
            stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status, voxels=small)
            print("every small voxel refined, grid", nq, stats)
            assert stats["solved"] >= 0.9 * len(small)


@pytest.mark.parametrize("cap,tau,nq", [(20, 5, 3), (128, 10, 9), (64, 1, 16), (7, 7, 1)])
def test_fit_cap_tau_grid(env, cap, tau, nq):
    xyz = synth.spin_scan(synth.frame_seed(2, 1), n_beams=16, n_az=1024)
    w = dict(configs.params_for("spin32"), max_pts=cap, min_pts=tau, grid_side=nq)
    say("fit cap/tau/grid", cap, tau, nq)
    gv, (out, axis, status) = run_fit(env, xyz, w)
    ov = O.voxelize(xyz, w["voxel_size"])
    parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)


def test_fit_length_scale_from_pca(env):
    xyz = synth.spin_scan(synth.frame_seed(2, 2), n_beams=16, n_az=1024)
    w = dict(configs.params_for("spin32"), ls_mode=1)
    say("fit ls_mode 1")
    gv, (out, axis, status) = run_fit(env, xyz, w)
    ov = O.voxelize(xyz, w["voxel_size"])
    parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)


def test_fit_per_point_noise(env):
    torch, vgpr, ctx = env
    xyz = synth.spin_scan(synth.frame_seed(2, 3), n_beams=16, n_az=1024)
    noise = rng(12).uniform(2e-4, 5e-3, size=len(xyz)).astype(np.float32)
    w = configs.params_for("spin32")
    p = parity.gpu_params(vgpr, w)
    x = dev(torch, xyz)
    say("fit per-point noise")
    gv = ctx.voxelize(x, p)
    out = ctx.fit_predict(x, gv, p, noise_var=torch.from_numpy(noise).cuda())
    ov = O.voxelize(xyz, w["voxel_size"])
    parity.compare_fit(xyz, ov, parity.oracle_params(w), *out, noise=noise.astype(np.float64))


def test_fit_degenerate_voxels(env):
    """Duplicated points, collinear points and single points."""
    torch, vgpr, ctx = env
    s = 0.5
    dup = np.tile([[0.1, 0.2, 0.3]], (12, 1))                            # all identical
    line = np.stack([np.linspace(0.05, 0.45, 9) + 1.0, np.full(9, 0.2), np.full(9, 0.25)], 1)  # collinear
    one = np.array([[2.2, 0.1, 0.1]])
    xyz = np.concatenate([dup, line, one]).astype(np.float32)
    w = dict(configs.params_for("spin32"), min_pts=1)
    say("fit degenerate voxels")
    gv, (out, axis, status) = run_fit(env, xyz, w)
    ov = O.voxelize(xyz, s)
    stats = parity.compare_fit(xyz, ov, parity.oracle_params(w), out, axis, status)
    assert stats["solved"] == 3


@pytest.mark.parametrize("n", [6, 40, 80, 120, 200])
def test_fit_zero_noise_duplicates_flags_failure(env, n):
    """sigma^2 = 0 with n copies of one point makes K singular (every pivot after the first is
    zero): each solver shape of the default launch choices (wave: 6, 40; workgroup: 80, 120;
    tiled: 200) must flag it or stay finite, and not hang."""
    torch, vgpr, ctx = env
    xyz = np.tile([[0.1, 0.2, 0.3]], (n, 1)).astype(np.float32)
    w = dict(configs.params_for("spin32"), min_pts=1, max_pts=256, noise_var=0.0)
    say(f"fit zero-noise duplicates n={n}")
    gv, (out, axis, status) = run_fit(env, xyz, w, precision=vgpr.PREC_FP64)
    st = int(status.cpu()[0])
    o = out.cpu().numpy()
    if st & vgpr.ST_FACTOR_FAIL:
        # a failed FP64 factorisation is not SOLVED and leaves NaN rows
        assert not st & vgpr.ST_SOLVED and np.isnan(o[..., 3]).all()
    else:
        assert st & vgpr.ST_SOLVED and np.isfinite(o).all()


# ---------------------------------------------------------------------------
# map_update (Sec. 3.3 state machine)
# ---------------------------------------------------------------------------
def test_map_update_matches_oracle_state_machine(env):
    torch, vgpr, ctx = env
    w = dict(configs.params_for("paper_stream"), max_pts=48, converge_var=0.05)
    prm = parity.oracle_params(w)
    p = parity.gpu_params(vgpr, w)
    om = O.VoxelMap(prm)
    gm = vgpr.Map(ctx, p, max_voxels=200000)
    for k in range(4):
        xyz = synth.spin_scan(synth.frame_seed(4, k), n_beams=16, n_az=512, position=(0.3 * k, 0.1 * k), yaw=0.1 * k)
        say("map frame", k, len(xyz))
        keys, out, axis, status = gm.update(dev(torch, xyz))
        ref = om.update(xyz)
        # keys exact; SOLVED / CAPPED / BELOW_TAU / CONVERGED equal; an axis mismatch only on a
        # flagged near tie; rows within the fit tolerances
        _, stt, n_cmp = _compare_map_frame(ref, keys, out, axis, status, prm.signal_var, prm.converge_var)
        say("map frame", k, "compared", n_cmp, "of", len(ref["keys"]), "converged",
            int(((stt & O.ST_CONVERGED) != 0).sum()))
        assert n_cmp >= 0.9 * int(((ref["status"] & O.ST_SOLVED) != 0).sum())
        st = gm.stats()
        assert st["voxels"] == len(om.points)
        assert st["points"] == sum(len(v) for v in om.points.values())


def _compare_map_frame(o_ref, keys, out, axis, status, sf2, eta, rotated=False):
    """One frame of map updates: keys exact, SOLVED / CAPPED / BELOW_TAU equal,
    CONVERGED equal unless the oracle's max variance is within tolerance of eta,
    rows within the fit tolerances where both took the same value axis (frame
    mode 1: all three coordinates within MEAN_TOL, frames flagged as near ties
    skipped, as in the rotated fit tests)."""
    assert np.array_equal(parity.as_u64(keys), o_ref["keys"])
    o = out.cpu().numpy().astype(np.float64)
    ax = axis.cpu().numpy()
    stt = status.cpu().numpy()
    n_cmp = 0
    for i in range(len(o_ref["keys"])):
        for bit in (O.ST_SOLVED, O.ST_CAPPED, O.ST_BELOW_TAU):
            assert bool(stt[i] & bit) == bool(o_ref["status"][i] & bit), (i, stt[i], o_ref["status"][i])
        if not o_ref["status"][i] & O.ST_SOLVED:
            continue
        a = o_ref["axis"][i]
        tie = (stt[i] & O.ST_AXIS_TIE) or (o_ref["status"][i] & O.ST_AXIS_TIE)
        if ax[i] != a:
            assert tie, i
            continue
        if rotated:
            if tie:
                continue
            assert np.abs(o[i][:, :3] - o_ref["out"][i][:, :3]).max() <= parity.MEAN_TOL, i
            assert np.abs(o[i][:, 3] - o_ref["out"][i][:, 3]).max() <= parity.VAR_TOL_REL * sf2, i
            n_cmp += 1
            continue
        u, wv = O.PARAM_AXES[a]
        assert np.array_equal(o[i][:, u].astype(np.float32), o_ref["out"][i][:, u].astype(np.float32))
        assert np.array_equal(o[i][:, wv].astype(np.float32), o_ref["out"][i][:, wv].astype(np.float32))
        assert np.abs(o[i][:, a] - o_ref["out"][i][:, a]).max() <= parity.MEAN_TOL, i
        assert np.abs(o[i][:, 3] - o_ref["out"][i][:, 3]).max() <= parity.VAR_TOL_REL * sf2, i
        mv = o_ref["out"][i][:, 3].max()
        if abs(mv - eta) > parity.VAR_TOL_REL * sf2:
            assert bool(stt[i] & O.ST_CONVERGED) == bool(mv <= eta), (i, mv)
        n_cmp += 1
    return o, stt, n_cmp


def _grid_normal_angle(a, b):
    """Angle between the least-scatter directions of two sets of grid points."""
    def normal(p):
        c = p - p.mean(axis=0)
        return np.linalg.eigh(c.T @ c)[1][:, 0]
    return float(np.arccos(min(1.0, abs(float(normal(a) @ normal(b))))))


def _feedback_no_resync(env, prec, frame_mode):
    """Five frames through a feedback map (update mode 1) on the GPU and in the
    oracle, each side carrying its own float32 rows from frame to frame. Every
    voxel both sides update is compared within the fit tolerances (axis-aligned
    grids: parameter coordinates bit-exact as float32; rotated grids: all three
    coordinates within the mean tolerance, near-tie frames skipped). A voxel whose
    value axis was a flagged near tie, whose CONVERGED decision fell within the
    tolerance of eta, or (rotated grids) whose two grids' normals differ by more
    than 5e-5 rad, its frame having been taken from each side's own carried rows
    where the PCA normal is ill-conditioned, may take a different branch on the
    two sides; it is followed no further (at most 2% of the compared voxels). Returns (max mean error, max variance error, voxels
    compared, type (c) re-solves among them, diverged voxels)."""
    torch, vgpr, ctx = env
    w = dict(configs.params_for("paper_stream"), max_pts=48, converge_var=2e-4, frame_mode=frame_mode)
    prm = parity.oracle_params(w)
    p = parity.gpu_params(vgpr, w, precision=vgpr.PREC_FP32 if prec == "fp32" else vgpr.PREC_FP64)
    om = O.VoxelMap(prm, feedback=True)
    gm = vgpr.Map(ctx, p, max_voxels=200000, feedback=True)
    diverged = set()
    n_resolved = n_cmp = 0
    max_mean = max_var = 0.0
    for k in range(5):
        xyz = synth.spin_scan(synth.frame_seed(5, k), n_beams=32, n_az=1024, position=(0.05 * k, 0.02 * k),
                              yaw=0.05 * k)
        say("feedback map without re-sync", prec, "frame mode", frame_mode, "frame", k, len(xyz))
        before = set(om.pred)
        keys, out, axis, status = gm.update(dev(torch, xyz))
        ref = om.update(xyz)
        gkeys = parity.as_u64(keys).tolist()
        o = out.cpu().numpy().astype(np.float64)
        ax = axis.cpu().numpy()
        stt = status.cpu().numpy()
        gi = {key: i for i, key in enumerate(gkeys)}
        ri = {key: i for i, key in enumerate(ref["keys"].tolist())}
        # a key updated on one side only must belong to a voxel that already diverged
        for key in set(gi) ^ set(ri):
            assert key in diverged, key
        solved_rows = []
        for key, i in ri.items():
            if key in diverged or key not in gi:
                continue
            j = gi[key]
            rs = int(ref["status"][i])
            for bit in (O.ST_SOLVED, O.ST_CAPPED, O.ST_BELOW_TAU):
                assert bool(stt[j] & bit) == bool(rs & bit), (k, key, stt[j], rs)
            if not rs & O.ST_SOLVED:
                continue
            solved_rows.append(o[j])
            a = int(ref["axis"][i])
            tie = bool((stt[j] & O.ST_AXIS_TIE) or (rs & O.ST_AXIS_TIE))
            if ax[j] != a:
                assert tie, (k, key)
                diverged.add(key)
                continue
            e = ref["out"][i]
            if frame_mode == 1:
                if tie:
                    diverged.add(key)
                    continue
                em = np.abs(o[j][:, :3] - e[:, :3]).max()
                if em > parity.MEAN_TOL and _grid_normal_angle(o[j][:, :3], e[:, :3]) > 5e-5:
                    # each side took this voxel's frame from its own carried rows; where the PCA
                    # normal is ill-conditioned (curved patches) their normals differ measurably
                    # and the two grids sample the surface at different places: a valid
                    # difference, followed no further (5e-5 rad moves a grid corner 7e-6 m)
                    diverged.add(key)
                    continue
            else:
                u, wv = O.PARAM_AXES[a]
                assert np.array_equal(o[j][:, u].astype(np.float32), e[:, u].astype(np.float32)), (k, key)
                assert np.array_equal(o[j][:, wv].astype(np.float32), e[:, wv].astype(np.float32)), (k, key)
                em = np.abs(o[j][:, a] - e[:, a]).max()
            ev = np.abs(o[j][:, 3] - e[:, 3]).max()
            assert em <= parity.MEAN_TOL and ev <= parity.VAR_TOL_REL * prm.signal_var, (k, key, em, ev)
            max_mean, max_var = max(max_mean, em), max(max_var, ev)
            mv = e[:, 3].max()
            if bool(stt[j] & O.ST_CONVERGED) != bool(rs & O.ST_CONVERGED):
                assert abs(mv - prm.converge_var) <= parity.VAR_TOL_REL * prm.signal_var, (k, key, mv)
                diverged.add(key)
            n_cmp += 1
            n_resolved += key in before
        if solved_rows:
            # axis-aligned grids take grid_side distinct values per parameter coordinate, rotated ones more
            distinct = np.median([min(len(np.unique(r[:, c].astype(np.float32))) for c in range(3))
                                  for r in solved_rows[:200]])
            assert (distinct > prm.grid_side) == (frame_mode == 1), distinct
        st = gm.stats()
        assert st["voxels"] == len(om.points)
        if not diverged:
            assert st["points"] == sum(len(v) for v in om.points.values())
            assert st["converged"] == sum(om.converged.values())
    say("no re-sync", prec, frame_mode, ": compared", n_cmp, "type (c) re-solves", n_resolved, "diverged",
        len(diverged), "max mean err", max_mean, "max var err", max_var)
    assert n_resolved >= 200
    assert len(diverged) <= 0.02 * n_cmp
    return max_mean, max_var, n_cmp, n_resolved, diverged


@pytest.mark.parametrize("prec,frame_mode", [("fp32", 0), ("fp32", 1), ("fp64", 1)])
def test_map_feedback_matches_oracle(env, prec, frame_mode):
    """Update mode 1 (covariance-centred update of type (c) voxels) over five frames,
    each side carrying its own state; every frame within the fit tolerances (the
    FP64 axis-aligned case, with its drift bound, is the test below)."""
    _feedback_no_resync(env, prec, frame_mode)


def test_map_feedback_multiframe_no_resync_fp64(env):
    """The FP64 axis-aligned case against a drift bound derived for it.

    In FP64 each re-solve agrees to ~1e-7 m, but the carried rows are rounded to
    float32 on both sides, and world coordinates of tens of metres have an ulp of up
    to 3.8e-6 m, so a carried row may differ by one ulp; the carried rows enter with
    their posterior variance as noise (floored at 1e-6 s_f^2), so the re-solve nearly
    interpolates them and passes such a difference on with a gain of about one. Five
    frames therefore stay within 5 x 3.8e-6 m, far inside the 1e-4 m mean tolerance
    (and the variances, which depend on coordinates only through the kernel, within
    1e-3 s_f^2)."""
    max_mean, _, _, _, _ = _feedback_no_resync(env, "fp64", 0)
    # the drift bound above: five frames of one-ulp differences in the carried rows
    assert max_mean <= 5 * (3.9e-6 + 1e-6), max_mean


def test_map_feedback_closed_form_frames(env):
    """The l -> 0 frames of the oracle's closed-form pin through the GPU map, compared
    with the oracle without any re-synchronisation: four solves, variance 1, 1/2,
    1/3, 1/4 (converged), CAPPED on the fourth frame, then skipped."""
    torch, vgpr, ctx = env
    w = dict(voxel_size=1.0, grid_side=2, min_pts=3, max_pts=8, signal_var=1.0, length_scale=1e-3,
             noise_var=1e-3, converge_var=0.3)
    prm = parity.oracle_params(w)
    r = rng(90)
    sites = [0.05, 0.15, 0.35, 0.45, 0.55, 0.65, 0.85, 0.95]

    def frame(n, z):
        idx = r.choice(64, n, replace=False)
        return np.stack([[sites[i // 8] for i in idx], [sites[i % 8] for i in idx], z], 1).astype(np.float32)
    frames = [frame(5, 0.5 + r.uniform(-0.01, 0.01, 5)), frame(4, 0.5 + r.uniform(-0.01, 0.01, 4)),
              frame(3, 0.5 + r.uniform(-0.01, 0.01, 3)),
              frame(11, np.concatenate([0.5 + r.uniform(-0.01, 0.01, 8), [0.56] * 3])), frame(2, [0.5, 0.5])]
    for prec in (vgpr.PREC_FP32, vgpr.PREC_FP64):
        om = O.VoxelMap(prm, feedback=True)
        gm = vgpr.Map(ctx, parity.gpu_params(vgpr, w, precision=prec), max_voxels=16, feedback=True)
        for k, F in enumerate(frames):
            say("feedback closed form", prec, k)
            keys, out, axis, status = gm.update(dev(torch, F))
            ref = om.update(F)
            _, stt, _ = _compare_map_frame(ref, keys, out, axis, status, 1.0, 0.3)
            if k < 4:
                assert abs(out.cpu().numpy()[0, :, 3].max() - 1.0 / (k + 1)) <= 1e-6
        gm.close()


def test_map_feedback_argument_errors(env):
    torch, vgpr, ctx = env
    p = parity.gpu_params(vgpr, configs.params_for("paper_stream"))
    say("feedback map argument errors")
    with pytest.raises(vgpr.VgprError) as ei:
        h = vgpr.C.c_void_p()
        ctx._check(ctx.lib.vgpr_map_create_ex(ctx.h, vgpr.C.byref(p), 100, 2, vgpr.C.byref(h)), "create_ex")
    assert ei.value.status == vgpr.E_INVALID
    big = parity.gpu_params(vgpr, configs.params_for("paper_stream"), max_pts=512)  # 81 + 512 > 512
    with pytest.raises(vgpr.VgprError) as ei:
        vgpr.Map(ctx, big, max_voxels=100, feedback=True)
    assert ei.value.status == vgpr.E_INVALID
    vgpr.Map(ctx, big, max_voxels=100).close()  # mode 0 accepts it


def test_map_update_output_capacity_reports_required_size(env):
    """cap_upd below the number of re-solved voxels: E_CAPACITY with *h_n_upd = the
    required count (the oracle map's), the first cap_upd outputs equal to those of
    a call with room for all, and the frame applied to the map."""
    torch, vgpr, ctx = env
    C = vgpr.C
    w = dict(configs.params_for("paper_stream"), max_pts=48)
    p = parity.gpu_params(vgpr, w)
    xyz = synth.spin_scan(synth.frame_seed(7, 3), n_beams=32, n_az=1024)
    ref = O.VoxelMap(parity.oracle_params(w)).update(xyz)
    full = vgpr.Map(ctx, p, max_voxels=100000)
    k_full, o_full, a_full, s_full = [t.cpu().numpy() for t in full.update(dev(torch, xyz))]
    small = vgpr.Map(ctx, p, max_voxels=100000)
    cap = 5
    m = p.grid_side ** 2
    keys = torch.empty(cap, dtype=torch.int64, device="cuda")
    out = torch.empty((cap, m, 4), dtype=torch.float32, device="cuda")
    axis = torch.empty(cap, dtype=torch.int8, device="cuda")
    status = torch.empty(cap, dtype=torch.uint8, device="cuda")
    nu = C.c_int64()
    x = dev(torch, xyz)
    say("map update output capacity", cap)
    st = ctx.lib.vgpr_map_update(small.h, C.c_void_p(x.data_ptr()), len(xyz), C.c_void_p(keys.data_ptr()),
                                 C.c_void_p(out.data_ptr()), C.c_void_p(axis.data_ptr()),
                                 C.c_void_p(status.data_ptr()), cap, C.byref(nu))
    torch.cuda.synchronize()
    assert st == vgpr.E_CAPACITY and nu.value == len(ref["keys"]) == len(k_full) > cap
    assert np.array_equal(keys.cpu().numpy(), k_full[:cap])
    assert np.array_equal(out.cpu().numpy(), o_full[:cap], equal_nan=True)
    assert np.array_equal(status.cpu().numpy(), s_full[:cap])
    assert small.stats()["voxels"] == full.stats()["voxels"]
    small.close()
    full.close()


def test_map_capacity_rejects_frame(env):
    torch, vgpr, ctx = env
    p = parity.gpu_params(vgpr, configs.params_for("paper_stream"))
    gm = vgpr.Map(ctx, p, max_voxels=10)
    xyz = rng(13).uniform(-5, 5, size=(500, 3)).astype(np.float32)
    say("map capacity")
    with pytest.raises(vgpr.VgprError) as ei:
        gm.update(dev(torch, xyz))
    assert ei.value.status == vgpr.E_CAPACITY
    assert gm.stats()["voxels"] == 0


def test_map_update_scratch_scales_with_the_update(env):
    """A 2M-voxel map (48 points a voxel: about 1.25 GB of pool and table) updated
    with a small frame under a 2 GB context budget: the solve stages only the
    re-solved voxels' points, so the update fits (a point scratch sized by the
    map's capacity, 16 B x 96M slots, would exceed the budget), and its output
    agrees with the oracle's map on two frames."""
    torch, vgpr, _ = env
    w = dict(configs.params_for("paper_stream"), max_pts=48)
    prm = parity.oracle_params(w)
    p = parity.gpu_params(vgpr, w)
    big = vgpr.Context(0, hbm_budget=2 << 30)
    gm = vgpr.Map(big, p, max_voxels=2_000_000)
    held_map = big.workspace_bytes()  # device bytes the context holds: the map's own so far
    om = O.VoxelMap(prm)
    n_solved = 0
    for k in range(2):
        xyz = synth.spin_scan(synth.frame_seed(7, 3 + k), n_beams=32, n_az=1024, position=(0.2 * k, 0.0))
        say("map update scratch, frame", k, len(xyz))
        keys, out, axis, status = gm.update(dev(torch, xyz))
        ref = om.update(xyz)
        _, _, n_cmp = _compare_map_frame(ref, keys, out, axis, status, prm.signal_var, prm.converge_var)
        solved = int(((ref["status"] & O.ST_SOLVED) != 0).sum())
        assert n_cmp >= 0.9 * solved
        n_solved += solved
    assert n_solved > 0
    assert big.workspace_bytes() - held_map < (256 << 20)  # the updates' scratch and staging
    gm.close()
    big.close()


def test_budget_exhaustion(env):
    torch, vgpr, _ = env
    small = vgpr.Context(0, hbm_budget=1 << 16)
    xyz = rng(14).uniform(-5, 5, size=(100000, 3)).astype(np.float32)
    say("budget exhaustion")
    with pytest.raises(vgpr.VgprError) as ei:
        small.voxelize(dev(torch, xyz), vgpr.default_params(voxel_size=0.5))
    assert ei.value.status == vgpr.E_BUDGET
    small.close()


def test_tuning_choices(env):
    """streams / grid scale are bit-identical; solver and FP32 choices stay within the oracle tolerances."""
    torch, vgpr, ctx = env
    xyz = synth.spin_scan(synth.frame_seed(2, 4), n_beams=32, n_az=1024)
    w = configs.params_for("spin32")
    p = parity.gpu_params(vgpr, w, precision=vgpr.PREC_FP64)
    x = dev(torch, xyz)
    gv = ctx.voxelize(x, p)
    default = ctx.tuning().as_dict()
    ref = [t.cpu().numpy() for t in ctx.fit_predict(x, gv, p)]
    ov = O.voxelize(xyz, w["voxel_size"])
    prm = parity.oracle_params(w)
    try:
        for change in [dict(streams=1), dict(grid_scale=[1, 2, 16, 8, 3, 2, 1]), dict(streams=1, grid_scale=[64] * 7),
                       dict(tiled_first=1), dict(tiled_first=1, streams=1),
                       dict(bucket_stream=[0, 1, 2, 3, 1, 2, 3]), dict(bucket_stream=[0] * 7),
                       dict(bucket_stream=[3, 3, 2, 2, 1, 1, 0])]:
            say("tuning (bit-identical)", change)
            t = dict(default)
            t.update(change)
            ctx.set_tuning(vgpr.Tuning.from_dict(t))
            got = [t_.cpu().numpy() for t_ in ctx.fit_predict(x, gv, p)]
            for g, r in zip(got, ref):
                assert np.array_equal(g, r, equal_nan=True)
        for change, prec in [(dict(wave_last_bucket=-1), vgpr.PREC_FP64), (dict(wave_last_bucket=0), vgpr.PREC_FP64),
                             (dict(fp32_last_bucket=2), vgpr.PREC_FP32), (dict(fp32_last_bucket=-1), vgpr.PREC_FP32),
                             (dict(tile_first_bucket=3), vgpr.PREC_FP64), (dict(tile_first_bucket=4), vgpr.PREC_FP32),
                             (dict(tile_first_bucket=2), vgpr.PREC_FP64), (dict(tile_first_bucket=2), vgpr.PREC_MIXED)]:
            say("tuning (within tolerance)", change, prec)
            t = dict(default)
            t.update(change)
            ctx.set_tuning(vgpr.Tuning.from_dict(t))
            out = ctx.fit_predict(x, gv, p.replace(precision=prec))
            parity.compare_fit(xyz, ov, prm, *out)
        # tiled buckets before the fork or with the others: bit-identical (only the schedule differs)
        outs = []
        for tf in (0, 1):
            say("tuning tiled_first", tf)
            t = dict(default)
            t.update(tile_first_bucket=4, tiled_first=tf)
            ctx.set_tuning(vgpr.Tuning.from_dict(t))
            outs.append([t_.cpu().numpy() for t_ in ctx.fit_predict(x, gv, p)])
        for g, r in zip(outs[1], outs[0]):
            assert np.array_equal(g, r, equal_nan=True)
        for key, val in (("streams", 2), ("tile_first_bucket", 1), ("wave_last_bucket", 3), ("tiled_first", 2),
                         ("bucket_stream", [0, 1, 2, 4, 1, 2, 3]), ("bucket_stream", [-1] + [0] * 6),
                         ("tiled_merge", 2)):
            with pytest.raises(vgpr.VgprError):
                bad = dict(default)
                bad[key] = val
                ctx.set_tuning(vgpr.Tuning.from_dict(bad))
    finally:
        ctx.set_tuning(vgpr.Tuning.from_dict(default))



def test_fit_graph_replays(env):
    """Captured fit_predict: each replay (with eager work and syncs in between)
    equals the eager call bit for bit, and a replay after the inputs change
    computes the new inputs (checked against the oracle)."""
    torch, vgpr, _ = env
    st = torch.cuda.Stream()
    ctx = vgpr.Context(0, stream=st)
    try:
        xyz = synth.spin_scan(synth.frame_seed(2, 5), n_beams=32, n_az=1024)
        w = configs.params_for("spin32")
        p = parity.gpu_params(vgpr, w)
        x = dev(torch, xyz)
        noise = torch.full((len(xyz),), 1e-3, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        say("fit graph: capture", len(xyz))
        vox = ctx.voxelize(x, p)
        ref = [t.cpu().numpy() for t in ctx.fit_predict(x, vox, p, noise_var=noise)]
        g = ctx.fit_graph(x, vox, p, noise_var=noise)
        for rep in range(3):
            say("fit graph: replay", rep)
            eager = ctx.fit_predict(x, vox, p, noise_var=noise)
            st.synchronize()
            out = g.launch()
            st.synchronize()
            for what, got in (("graph", out), ("eager", eager)):
                for name, a, b in zip(("out", "axis", "status"), got, ref):
                    a = a.cpu().numpy()
                    if not np.array_equal(a, b, equal_nan=True):
                        bad = np.flatnonzero(~((a == b) | (np.isnan(a) & np.isnan(b))).reshape(len(a), -1).all(1))
                        cnts = vox.counts.cpu().numpy()[bad[:8]]
                        raise AssertionError(f"{what} replay {rep}: {name} differs in {len(bad)} voxels, "
                                             f"first {bad[:8].tolist()} counts {cnts.tolist()} "
                                             f"status {ref[2][bad[:8]].tolist()} vs {got[2].cpu().numpy()[bad[:8]].tolist()}")
        new_noise = rng(16).uniform(2e-4, 5e-3, size=len(xyz)).astype(np.float32)
        noise.copy_(torch.from_numpy(new_noise))
        torch.cuda.synchronize()
        say("fit graph: replay on new noise")
        out = g.launch()
        st.synchronize()
        ov = O.voxelize(xyz, w["voxel_size"])
        parity.compare_fit(xyz, ov, parity.oracle_params(w), *out, noise=new_noise.astype(np.float64))
        eager = ctx.fit_predict(x, vox, p, noise_var=noise)
        st.synchronize()
        for a, b in zip(out, eager):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy(), equal_nan=True)
        g.close()
        with pytest.raises(vgpr.VgprError):
            vgpr.Context(0, stream=torch.cuda.default_stream()).fit_graph(x, vox, p)
    finally:
        st.synchronize()
        ctx.close()


# ---------------------------------------------------------------------------
# PCA-rotated local frame (frame_mode 1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "fp64", "mixed"])
def test_fit_rotated_frame(env, prec):
    """frame_mode 1 on the planes and spinning-scan workloads and on ragged voxels of 3..700
    points (every solver shape, 8x8 and 16x16 grids) against the oracle."""
    torch, vgpr, ctx = env
    pm = {"fp32": vgpr.PREC_FP32, "fp64": vgpr.PREC_FP64, "mixed": vgpr.PREC_MIXED}[prec]
    default = ctx.tuning().as_dict()
    try:
        if prec == "mixed":
            t = dict(default)
            t["tile_first_bucket"] = 2
            ctx.set_tuning(vgpr.Tuning.from_dict(t))
        cases = [("planes", synth.planes_cloud(synth.frame_seed(1, 2)), dict(configs.params_for("planes"))),
                 ("spin32", synth.spin_scan(synth.frame_seed(2, 7)), dict(configs.params_for("spin32"))),
                 ("ragged8", _ragged_voxels(61, LARGE_SIZES), dict(configs.params_for("spin32"), max_pts=512, min_pts=3)),
                 ("ragged16", _ragged_voxels(62, LARGE_SIZES),
                  dict(configs.params_for("spin32"), max_pts=512, min_pts=3, grid_side=16))]
        for name, xyz, w in cases:
            w["frame_mode"] = 1
            say("fit rotated frame", prec, name, len(xyz))
            gv, (out, axis, status) = run_fit(env, xyz, w, precision=pm)
            ov = O.voxelize(xyz, w["voxel_size"])
            stats = parity.compare_fit_rotated(xyz, ov, parity.oracle_params(w), out, axis, status)
            print(prec, name, stats)
            assert stats["solved"] > 0 and stats["skipped_ties"] <= max(2, stats["solved"] // 50)
    finally:
        ctx.set_tuning(vgpr.Tuning.from_dict(default))


def test_fit_rotated_frame_reproduces_tilted_planes(env):
    """Noiseless points on planes of several tilts (dyadic coordinates, exact in float32):
    every predicted point lies on its plane to float32 rounding of the output (a fit in
    the world-axis frame misses tilted planes by ~1e-3 m)."""
    torch, vgpr, ctx = env
    r = rng(63)
    pts, planes = [], []
    for i, (a, b) in enumerate([(0.5, 0.25), (-0.75, 0.5), (1.5, -0.25), (0.25, 2.0), (-1.0, -1.0)]):
        xy = r.integers(0, 32, size=(60, 2)) / 64.0 + np.array([4.0 * i, 0.0])  # one 4 m voxel column each
        z = a * xy[:, 0] + b * xy[:, 1] + 0.125 - a * 4.0 * i
        pts.append(np.stack([xy[:, 0], xy[:, 1], z], 1))
        planes.append((a, b, 0.125 - a * 4.0 * i))
    xyz = np.concatenate(pts).astype(np.float32)
    w = dict(configs.params_for("spin32"), voxel_size=4.0, min_pts=3, grid_side=8, length_scale=0.5,
             frame_mode=1)
    say("fit rotated frame, tilted planes", len(xyz))
    for prec in (vgpr.PREC_FP32, vgpr.PREC_FP64):
        gv, (out, axis, status) = run_fit(env, xyz, w, precision=prec)
        o = out.cpu().numpy().astype(np.float64)
        assert ((status.cpu().numpy() & vgpr.ST_SOLVED) != 0).all()
        for v in range(gv.n_vox):
            xyzv = o[v, :, :3]
            res = [np.abs(a * xyzv[:, 0] + b * xyzv[:, 1] + c - xyzv[:, 2]).max() for a, b, c in planes]
            assert min(res) <= 1e-5, (v, res)  # float32 rounding of outputs up to ~17 m


@pytest.mark.parametrize("feedback", [False, True])
def test_map_export_import_resumes_identically(env, feedback):
    """Checkpoint / resume: a map exported after two frames and imported into a
    new map continues bit-identically to the original over two more frames."""
    torch, vgpr, ctx = env
    w = dict(configs.params_for("paper_stream"), max_pts=48, converge_var=2e-4)
    p = parity.gpu_params(vgpr, w)
    a = vgpr.Map(ctx, p, max_voxels=150000, feedback=feedback)
    frames = [synth.spin_scan(synth.frame_seed(6, k), n_beams=32, n_az=1024, position=(0.05 * k, 0.02 * k),
                              yaw=0.05 * k) for k in range(4)]
    for k in range(2):
        say("map export/import", feedback, "frame", k)
        a.update(dev(torch, frames[k]))
    data = a.export()
    st = a.stats()
    assert len(data) >= 80 and data[:8] == b"VGPRMAP1"
    b = vgpr.Map.load(ctx, data, max_voxels=160000)
    assert b.feedback == feedback and b.stats() == st
    assert b.export() == data
    for k in range(2, 4):
        say("map export/import", feedback, "resume frame", k)
        ra = [t.cpu().numpy() for t in a.update(dev(torch, frames[k]))]
        rb = [t.cpu().numpy() for t in b.update(dev(torch, frames[k]))]
        assert len(ra[0]) > 100
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y, equal_nan=True)
    assert a.stats() == b.stats()
    with pytest.raises(vgpr.VgprError) as ei:
        vgpr.Map.load(ctx, data, max_voxels=st["voxels"] - 1)
    assert ei.value.status == vgpr.E_INVALID
    dup = bytearray(data)
    dup[88:96] = dup[80:88]  # the second voxel key repeats the first
    for bad in (b"XGPRMAP1" + data[8:], data[:len(data) - 5], data[:40], bytes(dup)):
        with pytest.raises(vgpr.VgprError) as ei:
            vgpr.Map.load(ctx, bad, max_voxels=160000)
        assert ei.value.status == vgpr.E_INVALID
    a.close()
    b.close()


def test_binding_rejects_unsuitable_tensors(env):
    """The binding hands raw device pointers to the library: non-contiguous,
    non-float32 or host tensors are refused before any GPU work."""
    torch, vgpr, ctx = env
    p = vgpr.default_params(voxel_size=0.5)
    good = torch.zeros((100, 3), dtype=torch.float32, device="cuda")
    say("binding input checks")
    for bad in (good.double(), good.cpu(), good.t().contiguous().t(), good[:, :2]):
        with pytest.raises(ValueError):
            ctx.voxelize(bad, p)
    g = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        ctx.structure_loss(good, g.double(), cell_size=1.0)
