"""The library's plain C++ host code under the compiler's sanitizers (no GPU).

tests/sanitize/host_check.cpp drives the fusion planners (every score, the
cap search, repeated rounds, the layout-swap pass), the diagonal cover (also
that it allocates nothing after a thread's first call), the batched path's
host pass with its threaded packing, the host MLP forward on seeded
random inputs and bad arguments, and the layout permutations' host side
(exchange lists and their tile passes; the LDS swizzle of a pass:
bijective, linear, two lanes per bank slot).  It is built with g++ together with the
library's host-only sources, once with AddressSanitizer and
UndefinedBehaviorSanitizer and once with ThreadSanitizer; a sanitizer report
or a failed check fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_16940_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "sanitize", "host_check.cpp")] + [
    os.path.join(CSRC, f) for f in ("sv_plan.cpp", "sv_batch_host.cpp", "sv_mlp_host.cpp", "sv_host.cpp")]
OUT = os.path.join(ROOT, "_build")


def build_and_run(tag, sanitize_flags, env_extra):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "host_check_" + tag)
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *sanitize_flags,
           "-Wno-mismatched-new-delete", "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SOURCES,
           "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host checks passed" in r.stdout


def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    build_and_run("asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                  {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})


def test_host_code_under_thread_sanitizer():
    build_and_run("tsan", ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
