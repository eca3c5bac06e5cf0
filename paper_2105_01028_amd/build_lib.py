"""Build libtrinity.so (the HIP kernels, the C-ABI and the C++ host set-up) in
the package directory for gfx950.  Run `python -m paper_2105_01028_amd.build_lib`."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtrinity.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["kernels.hip", "capi.cpp", "serve.cpp", "host_setup.cpp", "twolevel.hip",
           "probe.hip"]
ARCH = "gfx950"


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags(src):
    f = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    if src.endswith(".hip"):
        # packed fp32 instructions stay off: the compiler may form them from
        # float code, and they are avoided on this hardware
        f += ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]
    else:
        f += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
    return f


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for s in SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        cmds.append([cc] + _flags(s) + ["-c", os.path.join(CSRC, s), "-o", o])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)

    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        list(ex.map(run, cmds))
    tmp = LIB + ".tmp"
    run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
