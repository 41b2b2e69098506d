"""Workspace layouts against their consumers, on the CPU: ws_layout_check.cpp
lays out every entry point's workspace over a fake address for a grid of
sizes (nothing is allocated or dereferenced) and checks that each slice holds
the largest index the kernels that use it can reach."""
import os
import shutil
import subprocess

import pytest

from paper_2204_04898_amd import pm4g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2204_04898_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc is not installed")
    pm4g.load()   # the library must be built
    exe = str(tmp_path_factory.mktemp("wslayout") / "ws_layout_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(PKG, "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "ws_layout_check.cpp"), "-L", PKG, "-lpm4g", "-Wl,-rpath," + PKG, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


def test_every_slice_holds_its_consumers(checker):
    r = subprocess.run([checker], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert "0 failures" in r.stdout
