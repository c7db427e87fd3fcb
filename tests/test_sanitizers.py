"""Host sanitizer builds, run on the CPU only: the oracle (gcc with
AddressSanitizer and UndefinedBehaviorSanitizer) through every entry point on
small and degenerate systems, and the host code of libpasta (hipcc with the
sanitizers on the host side only) through the argument checks of every
entry point, which refuse before any device is touched.  A sanitizer report
or an unexpected return code fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1412_8502_amd", "csrc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


def _clean(out):
    return "AddressSanitizer" not in out and "runtime error" not in out and \
        "LeakSanitizer" not in out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    rc, out = _run(["gcc", "-O1", "-g", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
                    "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-lm"])
    assert rc == 0, out
    rc, out = _run([exe], env=SAN_ENV, timeout=300)
    print(out)
    assert rc == 0 and _clean(out) and "oracle sanitizer run ok" in out, out


def _hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if p and os.path.exists(p):
            return p
    return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not found")
def test_abi_checks_under_sanitizers(tmp_path):
    cc = _hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    common = ["--offload-arch=gfx950", "-O1", "-fPIC", "-std=c++17", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument"]
    srcs = ["api.hip", "cells.hip", "forces.hip", "integrate.hip", "cluster.hip", "batch.hip"]
    procs, objs = [], []
    for s in srcs:
        o = str(tmp_path / s.replace(".hip", ".o"))
        extra = ["-ffp-contract=off"] if s == "cluster.hip" else (
            ["-mllvm", "-amdgpu-dpp-combine=false"] if s == "forces.hip" else [])
        procs.append(subprocess.Popen([cc, *common, *san, *extra, "-c", os.path.join(CSRC, s),
                                       "-o", o], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
        objs.append(o)
    drv = str(tmp_path / "abi_checks.o")
    procs.append(subprocess.Popen([cc, *common, *san, "-c",
                                   os.path.join(ROOT, "tests", "sanitize", "abi_checks.cpp"),
                                   "-o", drv], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                  text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    exe = str(tmp_path / "abi_checks")
    rc, out = _run([cc, "--offload-arch=gfx950", *san, drv, *objs, "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=SAN_ENV, timeout=300)
    print(out)
    assert rc == 0 and _clean(out) and "abi checks ok" in out, out
