"""The oracle's C code under the sanitizers (CPU only).

`sanitize_oracle_driver.c` calls every oracle route on small random inputs
with several threads and checks that they agree (exactly for 0/1 matrices).
It is built together with oracle/perm_oracle.c twice: with AddressSanitizer
and UndefinedBehaviorSanitizer (any report aborts the run), and with
ThreadSanitizer for the thread split of the ranges.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "tests", "sanitize_oracle_driver.c"),
           os.path.join(ROOT, "oracle", "perm_oracle.c")]
PASS = "oracle sanitizer driver: all routes agree"


def build_and_run(tmp_path, name, flags):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / name)
    b = subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-o", exe,
                        *SOURCES, "-lpthread", "-lm"], capture_output=True, text=True)
    if b.returncode != 0:
        if "cannot find" in b.stderr and "san" in b.stderr:
            pytest.skip(f"sanitizer runtime not installed: {b.stderr.strip()[:200]}")
        raise AssertionError(b.stderr)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    return r


def test_address_and_undefined(tmp_path):
    r = build_and_run(tmp_path, "asan",
                      ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    assert r.returncode == 0 and PASS in r.stdout, r.stdout + r.stderr


def test_threads(tmp_path):
    r = build_and_run(tmp_path, "tsan", ["-fsanitize=thread"])
    if r.returncode != 0 and "unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot map its shadow memory on this kernel")
    assert r.returncode == 0 and PASS in r.stdout, r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
