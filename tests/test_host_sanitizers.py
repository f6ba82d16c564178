"""The host side of the library (argument checks, basis tabulation, incidence and
workspace bookkeeping: basis.cpp, api.cpp, solver.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host compilation pass only, and the host-only ABI
checks of test_abi.py run against that build in a child process.  The kernel objects are
the regular ones; nothing here launches a kernel, so no GPU is needed."""
import glob
import os
import re
import subprocess
import sys

import pytest

from _support import ROOT, ensure_built

HIPCC = "/opt/rocm/bin/hipcc"
# every sanitizer flag is scoped to the host pass: device code is built as usual
SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()
SAN_EXTRA = "-Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined".split()

CHILD = """
import os, sys
sys.path[:0] = [{root!r}, {tests!r}]
import pytest
from paper_2204_01722_amd import binding
binding.LIB_PATH = {lib!r}
rc = pytest.main([{abi!r}, "-q", "-p", "no:cacheprovider", "-m", "not gpu"])
maps = open("/proc/self/maps").read()
print("sanitized library loaded:", {lib!r} in maps)
print("in-tree library loaded:", os.path.join({root!r}, "paper_2204_01722_amd", "libhpmg.so") in maps)
sys.exit(int(rc))
"""


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    runtime = _asan_runtime()
    if not os.path.exists(HIPCC) or runtime is None:
        pytest.skip("hipcc or the AddressSanitizer runtime is not installed")
    ensure_built()
    from paper_2204_01722_amd import build
    kernels = [os.path.join(build.BUILD, s + ".o") for s in ("op_kernels.hip", "vec_kernels.hip")]
    if not all(os.path.exists(k) for k in kernels):
        build.build()
    csrc = os.path.join(ROOT, "paper_2204_01722_amd", "csrc")
    flags = ["-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include"), *SAN, *SAN_EXTRA]
    procs, objs = [], []
    for src in ("basis.cpp", "api.cpp", "solver.cpp"):
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, "-x", "hip", *flags, "-c", os.path.join(csrc, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out = p.communicate()[0]
        assert p.returncode == 0, out[-3000:]
    lib = str(tmp_path / "libhpmg_san.so")
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan", *SAN, "-o", lib,
                          *objs, *kernels], capture_output=True, text=True)
    assert res.returncode == 0, (res.stdout + res.stderr)[-3000:]

    tests = os.path.join(ROOT, "tests")
    child = CHILD.format(root=ROOT, tests=tests, lib=lib, abi=os.path.join(tests, "test_abi.py"))
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-c", child], env=env, capture_output=True, text=True,
                         timeout=900, cwd=ROOT)
    log = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, log
    assert "sanitized library loaded: True" in res.stdout, log
    assert "in-tree library loaded: False" in res.stdout, log
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, log
    passed = re.search(r"(\d+) passed", res.stdout)
    assert passed and int(passed.group(1)) >= 15, log
