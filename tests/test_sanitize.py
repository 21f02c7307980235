"""Host code under AddressSanitizer (with leak detection) and UndefinedBehaviorSanitizer, on
the CPU: the fit's host numerics (eigensolver, Haar rotation, logistic regression, the
significance quantiles, key selection, OPQ allocation) built with g++, and the library's
host sources (argument and file checks, fault-spec parsing, server creation checks) built by
hipcc with the sanitizers on the host side only, linked with the unchanged device objects and
driven by a C program that expects every call to be refused before any device call."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_16322_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_host_numerics_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_checks")
    _run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", f"-I{CSRC}", os.path.join(CSRC, "host_math.cpp"),
          os.path.join(HERE, "host_checks.cpp"), "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "ok (0 failures)" in r.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2404_16322_amd import build as B
    hipcc = B._hipcc()
    kernels = [os.path.join(B.BUILD, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        B.build(verbose=False)
    host = [s for s in B.SOURCES if not s.endswith(".hip")]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", f"-I{B.INCLUDE}", f"-I{CSRC}"]
    procs, objs = [], []
    for s in host:
        o = str(tmp_path / (s + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen([hipcc, *flags, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, err[-3000:]
    drv = str(tmp_path / "abi_checks.o")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", f"-I{B.INCLUDE}", "-c",
          os.path.join(HERE, "abi_checks.c"), "-o", drv])
    exe = str(tmp_path / "abi_checks")
    _run([hipcc, "--offload-arch=gfx950",
          "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", *objs, drv, *kernels, "-o", exe])
    r = _run([exe, str(tmp_path)], env=ENV, timeout=300)
    assert "ok (0 failures)" in r.stdout
