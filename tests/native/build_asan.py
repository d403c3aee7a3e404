"""Build the AddressSanitizer check of the serving queue: the library with
its host code instrumented (device code unchanged, gfx950) and the threaded
driver serve_threads.cpp, into tests/native/build/.  Run by
__graft_entry__.build(), so the GPU test that executes the driver finds it.
(ThreadSanitizer is not usable here: under its memory layout the ROCm
runtime finds no device.)"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from paper_2111_11788_amd import build as lib_build  # noqa: E402

OUT = os.path.join(HERE, "build")
LIB = os.path.join(OUT, "libmlmc_asan.so")
DRIVER = os.path.join(OUT, "serve_threads")
CLANG = "/opt/rocm/llvm/bin/clang++"
# instrument the host pass only: each sanitizer flag behind -Xarch_host
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT, "obj", src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [lib_build.HIPCC, *lib_build.COMMON, *lib_build.EXTRA.get(src, []), *HOST_SAN, *lang, "-c",
           os.path.join(lib_build.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(OUT, "obj"), exist_ok=True)
    with cf.ThreadPoolExecutor(min(len(lib_build.SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, lib_build.SOURCES))
    steps = [
        [lib_build.HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={lib_build.ARCH}", *objs, "-o", LIB],
        [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "serve_threads.cpp"), "-L", OUT, "-lmlmc_asan",
         "-L/opt/rocm/lib", "-lamdhip64", "-pthread", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath,/opt/rocm/lib", "-o", DRIVER],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", DRIVER)
    return DRIVER


if __name__ == "__main__":
    build(verbose=True)
