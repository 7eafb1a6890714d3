"""CPU checks of device helpers, compiled for the host with hipcc from the
library's own headers:
- the multiply-shift division (fdiv / make_fastdiv) that the lattice kernels
  use in place of run-time integer division, against n / d over every
  divisor up to 4096, powers of two and their neighbours up to 2^31, and
  numerators across the 32-bit range;
- the stored layout of the symmetric local inverses (sym_offset): one-to-one
  for every block size, paired rows adjacent for m <= 64."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run_check(name):
    tmp = tempfile.mkdtemp()
    try:
        exe = os.path.join(tmp, name)
        subprocess.run([HIPCC, "-std=c++17", "-O2", "--offload-arch=gfx950",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_1809_00828_amd", "csrc"),
                        os.path.join(ROOT, "tests", name + ".cpp"), "-o", exe],
                       check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr
        return r.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_fastdiv_matches_integer_division():
    assert "mismatches 0" in _run_check("fastdiv_check")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_symmetric_inverse_layout():
    assert "failures 0" in _run_check("layout_check")
