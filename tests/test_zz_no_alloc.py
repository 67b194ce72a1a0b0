"""vgpr_fit_predict_noalloc (fixed device scratch, no allocation) against
vgpr_fit_predict through the C ABI: two calls in a row, the second on a smaller
input, each compared with the allocating entry point's outputs on the same
inputs (the same kernels run, so the outputs must be bit-identical); a call
whose scratch exceeds the fixed array is rejected without running."""
import numpy as np
import pytest

from paper_2410_17084_amd import configs, synth
from tests import parity

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _same(a, b):
    import torch
    if a.dtype == torch.float32:
        return bool(torch.equal(torch.nan_to_num(a, nan=-7.0), torch.nan_to_num(b, nan=-7.0)))
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_fit_predict_twice(prec):
    import torch
    from paper_2410_17084_amd import vgpr
    ctx = vgpr.Context(0)
    try:
        w = configs.WORKLOADS["spin32"]
        p = parity.gpu_params(vgpr, w, precision=vgpr.PREC_FP32 if prec == "fp32" else vgpr.PREC_FP64)
        m = p.grid_side ** 2
        big = synth.spin_scan(synth.frame_seed(2, 3))
        small = synth.spin_scan(synth.frame_seed(2, 4), n_beams=16, n_az=900)
        held0 = None
        for name, xyz in (("first call", big), ("second call, smaller input", small)):
            x = torch.from_numpy(xyz).cuda()
            vox = ctx.voxelize(x, p)
            V = vox.n_vox
            say("noalloc", prec, name, len(xyz), "points", V, "voxels")
            ref = ctx.fit_predict(x, vox, p)
            torch.cuda.synchronize()
            if held0 is None:
                held0 = ctx.lib.vgpr_workspace_bytes(ctx.h)
            out = (torch.full((V, m, 4), 123.0, device="cuda"), torch.full((V,), 5, dtype=torch.int8, device="cuda"),
                   torch.full((V,), 255, dtype=torch.uint8, device="cuda"))
            got = ctx.fit_predict_noalloc(x, vox, p, out)
            torch.cuda.synchronize()
            for a, b in zip(got, ref):
                assert _same(a, b), name
            # the no-allocation call did not grow the context's device memory
            assert ctx.lib.vgpr_workspace_bytes(ctx.h) == held0
            solved = int(((got[2] & vgpr.ST_SOLVED) != 0).sum())
            say("noalloc", prec, name, "bit-identical,", solved, "solved")
            assert solved > 100
    finally:
        ctx.close()


def test_noalloc_rejects_oversized_calls():
    import torch
    from paper_2410_17084_amd import vgpr
    ctx = vgpr.Context(0)
    try:
        # a cap above 128 in MIXED mode needs the tiled solvers' scratch areas (hundreds of MB)
        p = vgpr.default_params(voxel_size=0.1, max_pts=512, min_pts=3, grid_side=16, precision=vgpr.PREC_MIXED)
        xyz = synth.spin_scan(synth.frame_seed(2, 5), n_beams=16, n_az=512)
        x = torch.from_numpy(xyz).cuda()
        vox = ctx.voxelize(x, p)
        V = vox.n_vox
        out = (torch.zeros((V, 256, 4), device="cuda"), torch.zeros(V, dtype=torch.int8, device="cuda"),
               torch.zeros(V, dtype=torch.uint8, device="cuda"))
        say("noalloc oversized: MIXED, cap 512", V, "voxels")
        with pytest.raises(vgpr.VgprError) as ei:
            ctx.fit_predict_noalloc(x, vox, p, out)
        assert ei.value.status == vgpr.E_CAPACITY
        torch.cuda.synchronize()
        assert bool((out[2] == 0).all())  # nothing ran
    finally:
        ctx.close()
