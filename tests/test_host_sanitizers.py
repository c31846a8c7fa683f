"""The library's host code (argument validation, plan and stream
bookkeeping) under the address and undefined-behaviour sanitizers, on the
CPU: a build whose host code carries them runs tests/host_validation.c, every
documented rejection with no device."""
import os
import subprocess

import pytest

from paper_1411_0436_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_host_validation_under_address_and_ub_sanitizers(tmp_path):
    lib = build.build_host_sanitized(str(tmp_path))
    exe = str(tmp_path / "host_validation")
    clang = "/opt/rocm/llvm/bin/clang"
    subprocess.check_call([clang, "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g",
                           "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "host_validation.c"),
                           "-L" + str(tmp_path), "-lpfbspec", "-Wl,-rpath," + str(tmp_path), "-o", exe])
    env = dict(os.environ)
    # the HIP runtime's own allocations outlive main(); only errors in this
    # library's code are of interest here
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""      # no device, wherever this runs
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host validation ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
