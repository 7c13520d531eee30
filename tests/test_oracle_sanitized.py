"""The oracle's pins once more with the oracle built under AddressSanitizer
and UndefinedBehaviorSanitizer, aborting on the first report: out-of-bounds
accesses, use after free, signed overflow, shifts out of range and
misaligned or undersized loads in the C oracle fail the run."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = str(tmp_path / "liboracle_san.so")
    O.build(lib, sanitize=True)
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, SFHE_ORACLE_LIB=lib, LD_PRELOAD=libasan + (":" + pre if pre else ""),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(HERE, "test_oracle_pins.py")],
                       cwd=os.path.dirname(HERE), env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert " passed" in r.stdout and "failed" not in r.stdout
