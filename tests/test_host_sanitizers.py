"""Host code under AddressSanitizer and UBSan (CPU only).

The C oracle, and the library's host code (level plans, constants,
tolerance schedules, batch sizing, argument validation), are built with
-fsanitize=address,undefined and run through small drivers in
tests/sanitize/.  The library's device objects are linked in unchanged (no
sanitizer in device code); the driver only takes paths that fail
validation before any HIP call, so no GPU is needed or touched.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_DIR = os.path.join(ROOT, "tests", "sanitize")
ORACLE = os.path.join(ROOT, "oracle")
PKG = os.path.join(ROOT, "paper_2010_05872_amd")
CSRC = os.path.join(PKG, "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))}\n{r.stdout}\n{r.stderr}"
    return r


def _env(leaks):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={1 if leaks else 0}:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.pop("LD_PRELOAD", None)
    return env


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c99", *SAN, "-ffp-contract=off", "-I", ORACLE, os.path.join(ORACLE, "mgard_oracle.c"),
          os.path.join(SAN_DIR, "oracle_driver.c"), "-o", exe, "-lm"])
    r = _run([exe], env=_env(leaks=True))
    assert "oracle sanitizer driver: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not found")
def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2010_05872_amd import build as B
    objs = []
    for src, extra in B.SOURCES:
        if not src.endswith(".hip"):
            continue
        obj = os.path.join(B.BUILD_DIR, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj):  # device objects as the library build makes them (no sanitizer)
            os.makedirs(B.BUILD_DIR, exist_ok=True)
            _run(["hipcc", *B.COMMON, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    host = []
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__=1"]
    for src in ("plan.cpp", "capi.cpp"):
        obj = str(tmp_path / (src + ".o"))
        _run([CLANG, "-std=c++17", *SAN, "-ffp-contract=off", *inc, "-c", os.path.join(CSRC, src), "-o", obj])
        host.append(obj)
    drv = str(tmp_path / "driver.o")
    _run([CLANG, "-std=c++17", *SAN, *inc, "-c", os.path.join(SAN_DIR, "host_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "host_san")
    _run([CLANG, *SAN, drv, *host, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    # the HIP runtime keeps allocations of its own until exit: leak checking off
    r = _run([exe], env=_env(leaks=False))
    assert "host sanitizer driver: ok" in r.stdout
