"""The host code of libhm (plan and store layout, packing and conversion,
request-loop bookkeeping, construction host side, H-LU validation) built with
AddressSanitizer and UndefinedBehaviorSanitizer, running the CPU tests of
the plan, the construction layout and the H-LU object's validation in a
child process: any
out-of-bounds access, use after free, signed overflow or misaligned access
in those paths aborts the child and fails this test.  No GPU."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_asan_ubsan():
    from paper_2308_10960_amd import build
    lib = build.build_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = build.sanitizer_runtime()
    env["HM_LIBRARY"] = lib
    # Python itself is not instrumented: leak reports would be its own
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_plan_cpu.py"),
                        os.path.join(ROOT, "tests", "test_construct_cpu.py"),
                        os.path.join(ROOT, "tests", "test_lu_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    # the child really loaded the sanitized build
    assert "passed" in r.stdout
