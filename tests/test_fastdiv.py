"""CPU check of the fixed-divisor division of the device code (txs::FastDiv):
a host program built from the library's own header against plain division."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_fastdiv_matches_division():
    d = tempfile.mkdtemp()
    try:
        exe = os.path.join(d, "fastdiv_check")
        subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                               "-I", os.path.join(ROOT, "include"),
                               "-I", os.path.join(ROOT, "paper_2305_04966_amd", "csrc"),
                               os.path.join(ROOT, "tests", "cpp", "fastdiv_check.cpp"),
                               "-o", exe], stderr=subprocess.DEVNULL)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
    finally:
        shutil.rmtree(d, ignore_errors=True)
