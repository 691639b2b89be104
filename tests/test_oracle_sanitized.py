"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, g++) and run over every entry point: no out-of-bounds access, no
undefined behaviour, and the same results as the regular build."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "tl_oracle.cpp")
DRIVER = os.path.join(HERE, "oracle_driver.cpp")


def _build(tmp, flags, name):
    exe = os.path.join(tmp, name)
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", *flags, SRC, DRIVER,
                    "-o", exe], check=True)
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_sanitized_oracle(tmp_path):
    san = _build(str(tmp_path), ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                 "-fno-omit-frame-pointer", "-static-libasan"], "driver_san")
    plain = _build(str(tmp_path), [], "driver_plain")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([san], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    ref = subprocess.run([plain], capture_output=True, text=True, check=True)
    assert r.stdout == ref.stdout
    assert r.stdout.count("expr ") == 17
