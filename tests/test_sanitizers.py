"""The oracle and the host-side parsing code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU (no GPU needed).

``tests/sanitize/oracle_check.c`` drives the FP64 oracle over every raster kind its tables
handle (walls, outflow segments, periodic sides including a one-column strip, a masked
domain with an OUTFLOW rim, a Dirichlet ring, a given-flux column), runs steps with rain,
plant drag, the viscous flux and infiltration, and checks the neighbour relation, the books
and the hex convolution's adjoint.  ``tests/sanitize/tune_check.cpp`` stores, reads back
and feeds malformed files to the autotuner's JSON cache.  A sanitizer report aborts the
driver, so the test fails on any out-of-bounds access, use after free, leak or undefined
operation.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-std=c99", "-Wall", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-ffp-contract=off",
          "-fopenmp", "-I", os.path.join(ROOT, "oracle"), os.path.join(SAN, "oracle_check.c"),
          os.path.join(ROOT, "oracle", "hexsv_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert r.stdout.strip().endswith("OK")


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not installed")
def test_tune_cache_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tune_check")
    csrc = os.path.join(ROOT, "paper_2406_14933_amd", "csrc")
    _run([HIPCC, "-x", "hip", "--cuda-host-only", "-std=c++17", "-g", "-O1",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", csrc,
          os.path.join(SAN, "tune_check.cpp"), os.path.join(csrc, "hexsv_tune.cpp"), "-o", exe])
    r = _run([exe, str(tmp_path)], env=ENV, timeout=120)
    assert r.stdout.strip().endswith("OK")
