"""Build the HIP library in-tree: ``paper_1711_10579_amd/_lib/libexagridpf.so``.

Every call recompiles all sources for gfx950 with hipcc (objects in
``_build/``), then links the shared library.  ``python -m
paper_1711_10579_amd.build`` runs it from the command line.

``build(sanitize=True)`` makes the host-sanitizer variant instead
(``_lib_san/libexagridpf.so``, objects in ``_build_san/``): host code built
with AddressSanitizer and UndefinedBehaviorSanitizer (clang's runtime, which
the process must preload), device code as usual; see ``sanitize.py``.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libexagridpf.so")
BUILD_SAN = os.path.join(ROOT, "_build_san")
LIBDIR_SAN = os.path.join(HERE, "_lib_san")
LIB_SAN = os.path.join(LIBDIR_SAN, "libexagridpf.so")

SOURCES = [
    "ordering.cpp",
    "analysis.cpp",
    "api.cpp",
    "newton.cpp",
    "serve.cpp",
    "hostcheck.cpp",
    "krylov_analysis.cpp",
    "nk.cpp",
    "krylov_check.cpp",
    "tune.cpp",
    "dense_plan.cpp",
    "precond_check.cpp",
    "kernels.hip",
    "dense.hip",
    "krylov.hip",
    "noalloc.hip",
]

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions stay disabled (some of their forms are unsafe here)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]


CXX = os.environ.get("CXX_HOST", "g++")
HOST = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-D__HIP_PLATFORM_AMD__",
    "-I/opt/rocm/include",
    f"-I{os.path.join(ROOT, 'include')}",
]


# host sanitizers: one runtime (clang's) for the host parts of every object,
# so the host-only sources go through the same clang as hipcc's host side;
# on hipcc lines each -fsanitize= applies to the host compilation only
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN_HOST = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
SAN_HIP = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _compile(src, sanitize=False):
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, os.path.basename(src) + ".o")
    if src.endswith(".cpp"):
        # host-only sources: plain C++ against the HIP runtime headers
        if sanitize:
            cmd = [CLANGXX, *[f for f in HOST if f != "-O3"], "-O1", *SAN_HOST, "-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd = [CXX, *HOST, "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, *(SAN_HIP if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{out}")
    return obj, out


def _torch_libdir():
    """PyTorch's lib directory, found without importing torch."""
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return None
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None


def _runtime_link():
    """Link the HIP runtime that PyTorch ships when it is installed, so that a
    process using both holds one HIP runtime; else the system one."""
    tl = _torch_libdir()
    if tl is None:
        return []
    return [f"-L{tl}", f"-Wl,-rpath,{tl}", "-Wl,-rpath,/opt/rocm/lib"]


def build(verbose=False, jobs=None, sanitize=False):
    bdir, ldir, lib = (BUILD_SAN, LIBDIR_SAN, LIB_SAN) if sanitize else (BUILD, LIBDIR, LIB)
    os.makedirs(bdir, exist_ok=True)
    os.makedirs(ldir, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for (o, msg) in results:
            if msg:
                print(msg)
    tmp = lib + ".tmp"
    # the sanitizer variant leaves the runtime's symbols to the preloaded runtime
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *_runtime_link(), *objs,
           "-lpthread", *([] if sanitize else ["-Wl,--no-undefined"])]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stdout + r.stderr)
    shutil.move(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
