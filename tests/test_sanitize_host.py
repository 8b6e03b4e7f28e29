"""Host code of the library under AddressSanitizer, UndefinedBehaviorSanitizer
and LeakSanitizer (the sanitizer variant of the build and the harness
paper_1711_10579_amd/sanitize/leakcheck.cpp): the symbolic analysis of every
schedule, the Krylov analysis and the input validation's error paths, in
loops; the process must end without a sanitizer report and with nothing of the
library's left allocated."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def test_host_code_clean_under_sanitizers():
    from paper_1711_10579_amd import build, sanitize

    lib = build.LIB_SAN if os.path.exists(build.LIB_SAN) else build.build(sanitize=True)
    exe = os.path.join(build.BUILD_SAN, "leakcheck")
    rt = sanitize.asan_runtime()
    cmd = [build.CLANGXX, "-std=c++17", "-O1", "-g", *build.SAN_HOST, "-shared-libsan",
           os.path.join(ROOT, "paper_1711_10579_amd", "sanitize", "leakcheck.cpp"), "-o", exe, lib,
           f"-Wl,-rpath,{os.path.dirname(lib)}", f"-Wl,-rpath,{os.path.dirname(rt)}"]
    tl = build._torch_libdir()
    if tl:
        cmd.append(f"-Wl,-rpath,{tl}")
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe, "host", "2"], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
