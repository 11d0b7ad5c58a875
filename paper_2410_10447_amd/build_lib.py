"""Build the HIP library libdockmi.so in-tree with hipcc for gfx950.

Usage: python -m paper_2410_10447_amd.build_lib [--jobs N] [--sanitized]

--sanitized builds libdockmi_san.so instead: the host code only (ligand
preparation and the C ABI, with host stand-ins for the kernel launchers,
csrc/dock_hoststub.cpp) compiled by g++ with AddressSanitizer and UBSan, for
running the CPU tests of the host code under the sanitizers.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdockmi.so")
LIB_SAN = os.path.join(PKG, "libdockmi_san.so")
SAN_SOURCES = ["dock_abi.cpp", "dock_prep.cpp", "dock_hoststub.cpp"]
ARCH = "gfx950"

SOURCES = ["dock_kernels.hip", "dock_ga.hip", "dock_static.hip", "dock_abi.cpp", "dock_prep.cpp"]

# Packed FP32 VALU instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str) -> None:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
           "-I" + INCLUDE, "-I" + CSRC, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if not src.endswith(".hip"):
        cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
               "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def build(jobs: int = 3) -> str:
    """Compile every source and link libdockmi.so (always rebuilds)."""
    with tempfile.TemporaryDirectory(prefix="dockmi_build_") as tmp:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
            list(ex.map(lambda a: _compile(*a), zip(SOURCES, objs)))
        out_tmp = LIB + ".tmp"
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(out_tmp, LIB)
    return LIB


def build_sanitized() -> str:
    """Host code with -fsanitize=address,undefined (g++, no device code)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    out_tmp = LIB_SAN + ".tmp"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"), "-I" + INCLUDE, "-I" + CSRC,
           *[os.path.join(CSRC, s) for s in SAN_SOURCES],
           "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib"),
           "-o", out_tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(out_tmp, LIB_SAN)
    return LIB_SAN


if __name__ == "__main__":
    if "--sanitized" in sys.argv:
        print(build_sanitized())
        sys.exit(0)
    j = 3
    if "--jobs" in sys.argv:
        j = int(sys.argv[sys.argv.index("--jobs") + 1])
    print(build(j))
