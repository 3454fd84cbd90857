"""Host check of the library's register FFTs (csrc/fft.hpp): every grid
length the kernels are instantiated for, and the radix-5 and radix-7
sub-lengths, against a direct DFT in long double (tests/fft_host_check.cpp,
compiled for the host with hipcc)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_register_fft_lengths_match_direct_dft(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fft_host_check")
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", os.path.join(HERE, "fft_host_check.cpp"), "-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, check=True).stdout
    seen = set()
    for line in out.split("\n"):
        if not line.strip():
            continue
        n, ef, ei = line.split()
        seen.add(int(n))
        # inputs in [-0.5, 0.5]^2, so |X_k| <= N/sqrt(2); a few ulps per stage
        assert float(ef) <= 4e-17 * int(n) ** 1.5 + 1e-16, line
        assert float(ei) <= 4e-17 * int(n) ** 1.5 + 1e-16, line
    assert {5, 7, 10, 14, 40, 56, 48, 32}.issubset(seen)
