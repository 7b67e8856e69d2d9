"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the host sources are rebuilt with both sanitizers (device code
unchanged), linked with tests/host_sanitize_driver.cpp, and run.  The driver
exercises a device-less context: template preparation (k-means, NNF,
counts, weighted banks, RGB templates, batched), every getter, PCA, the
error-bound getter, and the argument checks of every GPU call.  Any
sanitizer report or failed check fails the test."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2306_15010_amd import build as LB  # noqa: E402

CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]


def test_host_code_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(LB.HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain not found")
    objs, jobs = [], []
    for src in LB.HOST_SOURCES:
        o = str(tmp_path / (src + ".o"))
        jobs.append([LB.HIPCC, *LB.COMMON, *LB.HOST_FLAGS, *SAN_HOST, "-c", os.path.join(LB.CSRC, src), "-o", o])
        objs.append(o)
    for src in LB.DEVICE_SOURCES:
        o = os.path.join(LB.BUILD, src + ".o")
        s = os.path.join(LB.CSRC, src)
        if not (os.path.exists(o) and os.path.getmtime(o) >= os.path.getmtime(s)):
            o = str(tmp_path / (src + ".o"))
            jobs.append([LB.HIPCC, *LB.COMMON, *LB.DEVICE_FLAGS, "-c", s, "-o", o])
        objs.append(o)
    drv = str(tmp_path / "driver.o")
    jobs.append([CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
                 "-o", drv])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    exe = str(tmp_path / "host_sanitize_driver")
    _run([CLANG, "-fsanitize=address,undefined", drv, *objs, "-o", exe, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-lpthread"])
    sup = tmp_path / "lsan.supp"
    # allocations the HIP runtime keeps for the life of the process
    sup.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               LSAN_OPTIONS=f"suppressions={sup}", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert "all checks passed" in r.stdout
