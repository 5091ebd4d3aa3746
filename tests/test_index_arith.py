"""CPU check of the HIP kernels' index arithmetic (tests/index/index_check.cpp): the
workgroup maps (XCD remap, stencil tiles, DST plane slabs), the stencil and one-sweep PCG
tilings from the library's own planner (exact partition of every grid, points per thread,
halo rows, LDS), the fast-Poisson plans (slabs, pencils, padding, LDS) and the row-blocked
BF16 operand layout, over the launch shapes the API admits.  Built with hipcc against
libqo_hip.so; runs on the host only."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_index_arithmetic(tmp_path):
    from paper_2605_25149_amd import build as hb

    if not os.path.exists(hb.LIB):
        pytest.skip("libqo_hip.so not built")
    try:
        hipcc = hb.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "index_check")
    libdir = os.path.dirname(hb.LIB)
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-I", hb.CSRC,
                        os.path.join(ROOT, "tests", "index", "index_check.cpp"), "-L", libdir,
                        "-lqo_hip", f"-Wl,-rpath,{libdir}", "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout
