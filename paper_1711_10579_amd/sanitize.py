"""Host sanitizer run of the library: ``python -m paper_1711_10579_amd.sanitize [--gpu]``.

1. Builds the host-sanitizer variant of the library (AddressSanitizer and
   UndefinedBehaviorSanitizer on every host part, clang's runtime;
   ``build(sanitize=True)``) and the harness ``sanitize/leakcheck.cpp``.
2. Runs the harness: the host analysis, the Krylov analysis and the input
   validation in loops (and, with ``--gpu``, context and case creation,
   solves, a batch, a served request, the no-allocation solve and
   destruction in loops), with LeakSanitizer on at exit; the HIP runtime's
   own lifetime allocations are suppressed by library name.
3. Runs ``tests/test_host_library.py`` against the sanitizer variant (runtime
   preloaded into Python; leak detection off there, since the interpreter
   keeps its own allocations at exit).
Exit status 0 only if every step passes.
"""

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def asan_runtime():
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not c:
        raise RuntimeError("clang's AddressSanitizer runtime not found under /opt/rocm/llvm")
    return c[-1]


def main():
    from paper_1711_10579_amd import build

    gpu = "--gpu" in sys.argv
    lib = build.build(sanitize=True)
    rt = asan_runtime()
    exe = os.path.join(build.BUILD_SAN, "leakcheck")
    cmd = [build.CLANGXX, "-std=c++17", "-O1", "-g", *build.SAN_HOST, "-shared-libsan",
           os.path.join(HERE, "sanitize", "leakcheck.cpp"), "-o", exe, lib,
           f"-Wl,-rpath,{os.path.dirname(lib)}", f"-Wl,-rpath,{os.path.dirname(rt)}"]
    tl = build._torch_libdir()
    if tl:
        cmd.append(f"-Wl,-rpath,{tl}")
    subprocess.run(cmd, check=True)
    supp = os.path.join(build.BUILD_SAN, "lsan.supp")
    with open(supp, "w") as f:
        f.write("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\nleak:librocprofiler\n")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={supp}:print_suppressions=0"
    r = subprocess.run([exe, "gpu" if gpu else "host", "3"], env=env)
    print(f"sanitize: harness exit {r.returncode}", flush=True)
    ok = r.returncode == 0
    env2 = dict(os.environ)
    env2["LD_PRELOAD"] = rt
    env2["PF_LIB"] = lib
    env2["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:exitcode=23"
    env2["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r2 = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                         os.path.join(ROOT, "tests", "test_host_library.py")], env=env2, cwd=ROOT)
    print(f"sanitize: host-library tests under the sanitizers exit {r2.returncode}", flush=True)
    ok = ok and r2.returncode == 0
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
