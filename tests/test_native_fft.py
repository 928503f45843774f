"""Host emulation of the fixed-length lane FFT used by the transform kernels
(one host thread per lane, a std::barrier for the block barrier), against a
direct DFT for every compiled length and both directions."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_lane_fft_matches_direct_dft(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "fft_lane_check"
    src = os.path.join(HERE, "native", "fft_lane_check.cpp")
    subprocess.run([hipcc, "-std=c++20", "-O2", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", src, "-o", str(exe), "-lpthread"], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ALL OK" in out.stdout
