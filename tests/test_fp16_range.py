"""The FP16 range test of the FP32 solvers' stored block multipliers (the
lfits/lnarrow helpers of csrc/segprec.h), checked on the host: hipcc builds a
host-only program from tests/fp16_range_check.hip and runs it (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_fp16_multiplier_range_edge(tmp_path):
    exe = str(tmp_path / "fp16_range_check")
    cmd = [HIPCC, "--offload-host-only", "-std=c++17", "-O1",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2307_13483_amd", "csrc"),
           os.path.join(ROOT, "tests", "fp16_range_check.hip"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=60)
    assert r.returncode == 0, r.stdout[-3000:]
    assert r.stdout.strip().endswith("(0 failures)")
