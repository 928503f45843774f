"""The host code of the C ABI (host_setup.cpp, tc_api.cpp) built with
AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer, driven by
tests/native/abi_sanitize.cpp through geometry validation and host-only
(TC_FLAG_DRYRUN) contexts of several shapes and instance counts.  No GPU is
needed: nothing in the driver reaches the device.  The HIP kernels' object is
linked unsanitised (the library's own build, or a fresh hipcc compile)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_0711_1429_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def test_abi_host_code_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not gxx or not os.path.exists(hipcc):
        pytest.skip("g++ or hipcc not available")
    objs = []
    for name in ("host_setup.cpp", "tc_api.cpp"):
        obj = str(tmp_path / (name + ".o"))
        subprocess.run([gxx, "-std=c++17", "-O1", "-g", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-c", os.path.join(CSRC, name), "-o", obj], check=True)
        objs.append(obj)
    drv = str(tmp_path / "drv.o")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", *SAN, "-c", os.path.join(HERE, "native", "abi_sanitize.cpp"),
                    "-o", drv], check=True)
    kobj = os.path.join(ROOT, "paper_0711_1429_amd", "_build", "kernels.hip.o")
    if not os.path.exists(kobj):
        kobj = str(tmp_path / "kernels.o")
        subprocess.run([hipcc, "-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-c",
                        os.path.join(CSRC, "kernels.hip"), "-o", kobj], check=True)
    exe = str(tmp_path / "abi_sanitize")
    subprocess.run([gxx, *SAN, drv, *objs, kobj, "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx",
                    "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(out.stdout[-3000:], out.stderr[-3000:])
    assert out.returncode == 0, out.stdout[-3000:] + out.stderr[-3000:]
    assert "ALL OK" in out.stdout
    assert "ERROR: AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr
