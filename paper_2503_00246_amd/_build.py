"""Build libghost.so in-tree with hipcc for gfx950.

    python -m paper_2503_00246_amd._build

Host C++ sources are compiled as plain C++ (no device pass); HIP sources for
gfx950 only.  Packed-FP32 instructions are disabled for all device code.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libghost.so")

HOST_SOURCES = ["ghost_plan.cpp", "ghost_abi.cpp"]
HIP_SOURCES = ["ghost_kernels.hip", "ghost_cg.hip"]
GEN_SOURCE = "gen_tables.cpp"  # host program run at build time; writes _build/ghost_tables_gen.h


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _common():
    return ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", BUILD]


def _compile(src):
    hipcc = _hipcc()
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".cpp"):
        cmd = [hipcc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-ffp-contract=off",
               "-c", path, "-o", obj] + _common()
    else:
        cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-munsafe-fp-atomics",
               "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-c", path, "-o", obj] + _common()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _generate_tables(host_objs):
    """Link and run gen_tables: the 1D tables as compile-time constants for the kernels."""
    gen_obj = _compile(GEN_SOURCE)
    exe = os.path.join(BUILD, "gen_tables")
    plan_obj = [o for o in host_objs if os.path.basename(o).startswith("ghost_plan")]
    cmd = [_hipcc(), "-o", exe, gen_obj] + plan_obj
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    r = subprocess.run([exe, os.path.join(BUILD, "ghost_tables_gen.h")], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gen_tables failed\n{r.stdout}\n{r.stderr}")


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(HOST_SOURCES))) as ex:
        host_objs = list(ex.map(_compile, HOST_SOURCES))
    _generate_tables(host_objs)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(HIP_SOURCES))) as ex:
        objs = host_objs + list(ex.map(_compile, HIP_SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    try:
        build()
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
