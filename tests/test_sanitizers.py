"""Sanitizer builds on the CPU (no GPU needed).

- The float64 oracle (plain C) is built with AddressSanitizer and
  UndefinedBehaviorSanitizer and every entry point is run on small synthetic
  inputs (tests/sanitize/oracle_driver.c); the run must end cleanly, with the
  recovered poses close to the truth.
- The C-ABI library's host code is built with the same sanitizers (hipcc,
  -Xarch_host, so the GPU code is built as usual) and every host-side entry
  point (argument checks, planning of batches of 1 to 40 queries, workspace
  and staging sizes, paper settings, context creation on a machine without a
  device) is called (tests/sanitize/runtime_driver.cpp); leaks are checked.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_asan"
    srcs = [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")] + \
        [os.path.join(ROOT, "oracle", f) for f in ("imloc_oracle.c", "triangulate.c", "rig.c")]
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                    *srcs, "-o", str(exe), "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=SAN_ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "0 failure(s)" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.skipif(_gpu_present(), reason="checks context creation failing without a device")
def test_runtime_host_code_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2601_04185_amd", "csrc")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-I", os.path.join(ROOT, "include"), "-I", csrc]
    units = [os.path.join(csrc, f) for f in ("rounds.hip", "sample_p3p.hip", "score.hip", "refine.hip", "lift.hip",
                                              "triangulate.hip", "runtime.cpp")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([HIPCC, *flags, "-x", "hip", "-c", src, "-o", obj], check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, units))
    drv = str(tmp_path / "driver.o")
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-Xarch_host",
                    "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-c",
                    os.path.join(ROOT, "tests", "sanitize", "runtime_driver.cpp"), "-o", drv],
                   check=True, capture_output=True)
    exe = str(tmp_path / "runtime_asan")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", drv, *objs, "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "0 failure(s)" in r.stdout
    shutil.rmtree(str(tmp_path), ignore_errors=True)
