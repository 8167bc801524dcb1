"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The host side of every csrc/*.hip source is compiled with -fsanitize=address,undefined (host
pass only: no device code is built or run), linked into a shared library, and driven by
tests/sanitize/abi_sanitize.cpp, a sanitized executable that repeats the argument-validation
cases of test_abi_cpu.py, the size queries at the edges of their ranges, the deterministic-mode
switch and a parser run over well-formed, truncated, corrupt and random tuning-cache files.
A sanitizer report fails the run.  (A Python process cannot host the ASan runtime unless it is
preloaded, hence the C++ driver.)"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_16121_amd", "csrc")
ROCM = "/opt/rocm"
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not found")
def test_host_code_under_asan_and_ubsan(tmp_path):
    out = str(tmp_path)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def compile_one(src):
        obj = os.path.join(out, os.path.basename(src)[:-4] + ".o")
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN, "-c", src, "-o", obj],
             timeout=600)
        return obj

    with cf.ThreadPoolExecutor(min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = os.path.join(out, "libsvdlut_san.so")
    _run([CLANG, "-shared", "-o", lib, *objs, f"-L{ROCM}/lib", "-lamdhip64"], timeout=300)
    exe = os.path.join(out, "abi_sanitize")
    _run([CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__",
          os.path.join(ROOT, "tests", "sanitize", "abi_sanitize.cpp"), "-o", exe, f"-L{out}", "-lsvdlut_san",
          f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{out}", f"-Wl,-rpath,{ROCM}/lib"], timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"{r.stdout[-4000:]}\n{r.stderr[-6000:]}"
    assert r.stdout.startswith("OK "), r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
