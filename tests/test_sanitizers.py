"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's validation, workspace sizing and planning (bq_engine.cpp,
  built with host-side sanitizers and linked with the ordinary kernel
  objects) driven by tests/sanitize/validate_driver.cpp over 200 000
  argument combinations: null and misaligned pointers, negative, huge and
  empty shapes, bad leading dimensions, ops, precisions, slice counts and
  workspace sizes.  No HIP call is made.
* The oracle (bq_oracle.c, gcc) on small integer products against a product
  written out in tests/sanitize/oracle_driver.c.

Any sanitizer report aborts the driver (halt_on_error, no recovery), so a
zero exit status means none was found.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(HERE, "_build")
CSRC = os.path.join(ROOT, "paper_2609_02081_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_2609_02081_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, timeout=600):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=timeout, env=ENV)
    return r.returncode, r.stdout


def _host_san():
    # Sanitizers on the host pass only (the device code is not instrumented).
    return ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_engine_validation_under_sanitizers():
    from paper_2609_02081_amd import build as lib_build

    kernels = [os.path.join(OBJ, os.path.splitext(f)[0] + ".o") for f in lib_build.SOURCES if f.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        pytest.skip("library objects not built (run the build first)")
    os.makedirs(OUT, exist_ok=True)
    eng = os.path.join(OUT, "bq_engine_san.o")
    exe = os.path.join(OUT, "validate_driver")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    rc, out = _run([HIPCC, *common, *_host_san(), "-c", os.path.join(CSRC, "bq_engine.cpp"), "-o", eng])
    assert rc == 0, out
    drv = os.path.join(OUT, "validate_driver.o")
    rc, out = _run([HIPCC, *common, *_host_san(), "-c", os.path.join(HERE, "validate_driver.cpp"), "-o", drv])
    assert rc == 0, out
    rc, out = _run([HIPCC, "--offload-arch=gfx950", *_host_san(), drv, eng, *kernels,
                    "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe])
    assert rc == 0 and "0 failures" in out, out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_sanitizers():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    rc, out = _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "oracle", "bq_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
                    "-o", exe, "-lm"])
    assert rc == 0, out
    rc, out = _run([exe])
    assert rc == 0 and "0 failures" in out, out
