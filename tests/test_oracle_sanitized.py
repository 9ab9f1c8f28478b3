"""The oracle's CPU pins again with the oracle built under AddressSanitizer
and UndefinedBehaviorSanitizer (every report fatal): oracle/build.py
build_sanitized() -> oracle/libqso_san.so, loaded through QSO_LIB by a pytest
subprocess that preloads the ASan runtime (leak checks off: the interpreter's
own allocations are not the oracle's)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_oracle_pins_pass_under_asan_and_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime")
    sys.path.insert(0, ROOT)
    from oracle import build
    lib = build.build_sanitized()
    tests = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py")
                   and f != os.path.basename(__file__))
    env = dict(os.environ, QSO_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow",
                        "-p", "no:cacheprovider"] + tests, cwd=ROOT, env=env,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
