"""Register and private-memory use of the solver kernels, read from the compiler's
resource report (CPU only: hipcc cross-compiles for gfx950).

The wave and block solvers must not spill registers to private (scratch) memory:
they run concurrently on several streams and inside captured graphs, and a spill
there once coincided with outputs that differed between graph replays. The tiled
solvers spill a few loop-invariant words per lane (written when a wavefront starts,
read back once per voxel or row block, outside the pivot and tile-update loops); their
budget is stated here so that growth shows up.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_17084_amd", "csrc")

# private bytes per lane allowed per kernel family (anything not listed: 0)
BUDGET = {"fit_tile_kernel": 80}


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not available")


def _resources(src: str) -> dict:
    from paper_2410_17084_amd import build
    cmd = [_hipcc(), *build.HIPCC_FLAGS, "--offload-device-only", "-c", os.path.join(CSRC, src), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\])?: (\d+)", line)
        if m and name:
            out[name][m.group(1).strip()] = int(m.group(2))
    return out


def test_solver_kernels_do_not_spill():
    res = _resources("fit.hip")
    kernels = {k: v for k, v in res.items() if "_kernel" in k}
    assert any("fit_wave_kernel" in k for k in kernels) and any("fit_block_kernel" in k for k in kernels)
    for name, r in kernels.items():
        allowed = max([b for fam, b in BUDGET.items() if fam in name], default=0)
        assert r.get("ScratchSize", 0) <= allowed, (name, r)
        if allowed == 0:
            assert r.get("VGPRs Spill", 0) == 0, (name, r)
