"""Build libhm.so: HIP kernels for gfx950 (hipcc) + host C++ (ROCm clang).

Every call compiles from source; objects go to _build/ next to this file and
the shared library to paper_2308_10960_amd/libhm.so.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libhm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
# packed FP32 instructions are disabled for all device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

HIP_SOURCES = ["hm_kernels.hip", "hm_kernels_batch.hip", "hm_kernels_util.hip", "hm_construct.hip", "hm_lu.hip"]
HOST_SOURCES = ["hm_host.cpp", "hm_server.cpp", "hm_construct_host.cpp", "hm_lu_host.cpp"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HOST_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([CLANG, *COMMON, "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-pthread",
                     "-c", path, "-o", obj])
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-pthread", *objs, "-o", tmp,
          f"-L{ROCM}/lib", "-lamdhip64"], verbose)
    os.replace(tmp, OUT)
    return OUT


SAN_OUT = os.path.join(BUILD, "libhm_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    """The clang AddressSanitizer runtime a process must preload to load
    the sanitized library."""
    res = subprocess.run([CLANG, "-print-resource-dir"], capture_output=True, text=True, check=True).stdout.strip()
    return os.path.join(res, "lib", "linux", "libclang_rt.asan-x86_64.so")


def build_sanitized(verbose: bool = False) -> str:
    """libhm_san.so: the host code (plan, packing, request loop, construction
    host side) built with AddressSanitizer and UndefinedBehaviorSanitizer,
    linked with the device objects of build().  For CPU tests only: load it
    with HM_LIBRARY set to its path and the runtime of sanitizer_runtime()
    preloaded."""
    os.makedirs(BUILD, exist_ok=True)
    dev = [os.path.join(BUILD, src + ".o") for src in HIP_SOURCES]
    if not all(os.path.exists(o) for o in dev):
        build(verbose)
    objs = list(dev)
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".san.o")
        objs.append(obj)
        jobs.append([CLANG, "-O1", "-g", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", *SAN_FLAGS,
                     "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-pthread", "-c", os.path.join(CSRC, src),
                     "-o", obj])
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = SAN_OUT + ".tmp"
    _run([CLANG, "-shared", "-fPIC", *SAN_FLAGS, "-shared-libsan", "-pthread", *objs, "-o", tmp,
          f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"], verbose)
    os.replace(tmp, SAN_OUT)
    return SAN_OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
