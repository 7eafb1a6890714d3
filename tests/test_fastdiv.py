"""CPU check of the multiply-shift division (fdiv / make_fastdiv) that the
lattice kernels use in place of run-time integer division: compiled for the
host with hipcc from the library's own header and compared with n / d over
every divisor up to 4096, powers of two and their neighbours up to 2^31, and
numerators across the 32-bit range."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_fastdiv_matches_integer_division():
    tmp = tempfile.mkdtemp()
    try:
        exe = os.path.join(tmp, "fastdiv_check")
        subprocess.run([HIPCC, "-std=c++17", "-O2", "--offload-arch=gfx950",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_1809_00828_amd", "csrc"),
                        os.path.join(ROOT, "tests", "fastdiv_check.cpp"), "-o", exe],
                       check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "mismatches 0" in r.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
