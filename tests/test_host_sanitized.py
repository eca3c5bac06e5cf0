"""The C++ host side of the library -- the FP64 set-up (HEALPix directions,
phase matrix scaling, ray lattice, coefficients, cone sets, pulse weights,
interface interceptions), the C-ABI's descriptor checks and host-table calls
-- built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only,
with g++; the HIP kernels are linked unchanged) and exercised by the host-table
tests in a child process.  Any out-of-bounds access, use after free or
undefined behaviour aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2105_01028_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitized")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def _device_objects():
    """The HIP kernel objects of the regular build (built here if missing)."""
    from paper_2105_01028_amd import build_lib
    objs = [os.path.join(build_lib.BUILD, s + ".o") for s in build_lib.SOURCES
            if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in objs):
        build_lib.build(verbose=False)
    return objs


def _gcc_lib(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()


def test_host_side_clean_under_asan_and_ubsan():
    asan, ubsan = _gcc_lib("libasan.so"), _gcc_lib("libubsan.so")
    if not (os.path.isabs(asan) and os.path.isabs(ubsan)):
        pytest.skip("gcc sanitizer runtimes not installed")
    os.makedirs(OUT, exist_ok=True)
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-std=c++17", "-fPIC",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", "/opt/rocm/include",
             "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src in ("host_setup.cpp", "capi.cpp", "serve.cpp"):
        o = os.path.join(OUT, src + ".o")
        _run(["g++"] + flags + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    lib = os.path.join(OUT, "libtrinity_sanitized.so")
    _run(["g++", "-shared", "-fsanitize=address,undefined", "-o", lib] + objs +
         _device_objects() + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms   # instrumented
    env = dict(os.environ, TRINITY_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_host_tables.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
