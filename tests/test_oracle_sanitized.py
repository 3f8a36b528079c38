"""The oracle's pins again, against a build of the C oracle with
AddressSanitizer and UndefinedBehaviorSanitizer: no out-of-bounds access, use
after free or undefined behaviour on any path the pins reach."""
import os
import subprocess
import sys

import pytest

from oracle import henn_oracle as ho

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = ho.build_sanitized(str(tmp_path / "libhenn_oracle_san.so"))
    env = dict(os.environ, HENN_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the pins that go through the C oracle (the Gram brute force is NumPy/torch)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(HERE, "test_oracle_pins.py"), os.path.join(HERE, "test_oracle_near_ties.py"),
           "-k", "not gram"]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
