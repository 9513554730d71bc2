"""The library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged), driven on the CPU by
``tests/sanitize/host_abi_check.cpp``: the host-only entry points (grids,
Gauss-Legendre panel coefficients, admission footprint, default options) with
valid and invalid arguments and the refusals of the device entry points.
Any memory or undefined-behaviour error aborts the driver."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_02930_amd", "csrc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SAN = "address,undefined"


def _runtime_dir():
    hits = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return os.path.dirname(hits[0]) if hits else None


@pytest.mark.slow
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    if not shutil.which("hipcc") or not os.path.exists(CLANG) or _runtime_dir() is None:
        pytest.skip("hipcc, clang++ or the sanitizer runtime is missing")
    srcs = sorted(os.path.basename(p) for p in glob.glob(os.path.join(CSRC, "*.hip")) +
                  glob.glob(os.path.join(CSRC, "*.cpp")))
    # sanitizer options go to the host half of each compilation only
    host_san = ["-Xarch_host", "-fsanitize=" + SAN, "-Xarch_host", "-fno-omit-frame-pointer",
                "-Xarch_host", "-fno-sanitize-recover=undefined"]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        cmd = ["hipcc", "--offload-arch=gfx950", "-O2", "-g", "-std=c++17", "-fPIC", "-pthread",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
               "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-x", "hip", "-c", os.path.join(CSRC, src),
               "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libite_san.so")
    # host-only link and driver: plain clang++ with the shared sanitizer runtime
    r = subprocess.run([CLANG, "-shared", "-fPIC", "-pthread", "-fsanitize=" + SAN, "-shared-libsan", "-o", lib,
                        *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "host_abi_check")
    r = subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=" + SAN, "-shared-libsan",
                        "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
                        "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "host_abi_check.cpp"),
                        "-o", exe, "-L" + str(tmp_path), "-lite_san", "-Wl,-rpath," + str(tmp_path)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               LD_LIBRARY_PATH=_runtime_dir() + ":" + os.environ.get("LD_LIBRARY_PATH", ""))
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host ABI checks passed" in r.stdout
