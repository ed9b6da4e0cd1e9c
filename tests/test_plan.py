"""Host logic of the plan (CPU): the nested-dissection tree eliminates every interface unknown
once, the extend-add maps place each child's boundary unknowns at the parent's matching
positions (and the inverse maps point back), node storage ranges are disjoint with each level's
fronts contiguous, the fused bottom levels cover every node of their levels once with consistent
places, parents and x_B sources, and workspace offsets are aligned and in bounds; for constant
and linear interface spaces, ragged trees, one subdomain, many-line subdomains and the metric
workload."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2103_11050_amd", "csrc")
INC = os.path.join(HERE, "..", "include")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_plan_consistency(tmp_path):
    exe = tmp_path / "plan_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, "-I", INC, os.path.join(HERE, "plan_check.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.count(": ok") == 16
    # the metric workload fuses four levels in 256 subtrees; ragged trees and the linear spaces
    # fuse too
    assert "1024x1024 sub 16x16 ne 8,8 deg 0: ok" in out.stdout and "fused 4 subtrees 256 +flux" in out.stdout
    fused = [l for l in out.stdout.splitlines() if ": ok" in l and " fused 0 " not in l]
    assert len(fused) >= 10
    # the ctypes descriptor of the binding has the C layout
    import ctypes

    from paper_2103_11050_amd import binding
    line = [l for l in out.stdout.splitlines() if l.startswith("desc ")][0].split()
    D = binding.Desc
    assert [int(x) for x in line[1:]] == [ctypes.sizeof(D), D.bc_value.offset, D.iface_degree.offset,
                                          D.refine_rtol.offset]
