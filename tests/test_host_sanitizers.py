"""The host code of the library (checkpoint schedules, the recovery model of
the two-level checkpoints, argument validation, the error paths of plan
creation) under AddressSanitizer and UBSan: the CPU tests of the C ABI re-run
in a child process against the sanitizer build of the library
(paper_2509_10103_amd/build.py --asan; the device code is not instrumented)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_abi_checks_pass_under_address_and_undefined_behaviour_sanitizers():
    from paper_2509_10103_amd import build
    if not os.path.exists(build.ASAN_OUT):
        pytest.skip("sanitizer build not present (paper_2509_10103_amd/build.py --asan)")
    rt = build.asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    env = dict(os.environ, LD_PRELOAD=rt, NPO_LIBRARY=build.ASAN_OUT, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_capi.py")],
                       env=env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    # the child loaded the sanitizer build
    probe = ("from paper_2509_10103_amd import npo; npo.lib(); "
             "print(any('libnpo_asan.so' in l for l in open('/proc/self/maps')))")
    r = subprocess.run([sys.executable, "-c", probe], env=env, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip().endswith("True"), r.stdout + r.stderr
