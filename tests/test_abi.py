"""CPU checks of the C-ABI library: it loads, exports every declared entry point,
and its host-only calls behave (no GPU compute here)."""
import ctypes as C
import os
import re

import pytest

from paper_2410_17084_amd import vgpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "vgpr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vgpr_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(vgpr.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = vgpr.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_library_exports_only_the_abi():
    """Internal C++ symbols stay hidden (default visibility only on the ABI)."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", vgpr.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    ours = {s for s in exported if "vgpr" in s}
    assert ours == set(declared_symbols())


def test_params_default_are_the_papers():
    p = vgpr.default_params()
    assert p.voxel_size == pytest.approx(0.2)
    assert p.min_pts == 10 and p.grid_side == 9
    assert p.converge_var == pytest.approx(0.3)
    assert 1.0 / (2 * p.length_scale ** 2) == pytest.approx(1.0, rel=1e-6)
    assert p.signal_var == 1.0 and p.precision == vgpr.PREC_FP32 and p.frame_mode == 0


def test_params_struct_layout_matches_header():
    # 13 four-byte fields, no padding
    assert C.sizeof(vgpr.Params) == 52


def test_status_strings():
    lib = vgpr.load()
    names = [lib.vgpr_status_str(i).decode() for i in range(8)]
    assert names == ["VGPR_OK", "VGPR_E_INVALID", "VGPR_E_NOMEM", "VGPR_E_CAPACITY", "VGPR_E_RANGE",
                     "VGPR_E_BUDGET", "VGPR_E_DEVICE", "VGPR_E_UNSUPPORTED"]


def test_null_arguments_rejected_on_host():
    lib = vgpr.load()
    assert lib.vgpr_create(0, None, 0, None) == vgpr.E_INVALID
    assert lib.vgpr_destroy(None) == vgpr.E_INVALID
    assert lib.vgpr_map_destroy(None) == vgpr.E_INVALID
    n = C.c_int64()
    p = vgpr.default_params()
    assert lib.vgpr_voxelize(None, None, 0, None, 1, C.byref(p), None, None, None, None, 0, C.byref(n), None,
                             None) == vgpr.E_INVALID


def test_library_binds_to_torchs_hip_runtime():
    """Loaded first in a fresh process, libvgpr.so must still share PyTorch's HIP
    runtime (one libamdhip64 mapped), or torch's tensors and streams would belong
    to another runtime than the library's."""
    import subprocess
    import sys
    code = ("from paper_2410_17084_amd import vgpr\n"
            "vgpr.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"
