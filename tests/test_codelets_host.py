"""The radix-7 codelet (Rader's algorithm, the remark after Algorithm 1)
compiled for the host and checked against the DFT definition (no GPU)."""
import os
import shutil
import subprocess

import pytest

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_rader_seven_point_codelet(tmp_path):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "dft7_check")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-I", os.path.join(root, "paper_0808_0487_amd", "csrc"), "-I", os.path.join(root, "include"),
                    os.path.join(root, "tests", "dft7_check.hip"), "-o", exe], check=True, timeout=300,
                   capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout
