"""Runs the C test drivers against the oracle: the brute-force topology check
on every 3x3 field over a 5-value alphabet (plus random 4x4, 3x3x3, 4x4x4
fields) and the sanitizer-built corrupted-stream fuzzer."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DRV = os.path.join(HERE, "drivers")
SRC = os.path.join(ROOT, "oracle", "toposzp_oracle.c")


def _build(tmp_path, name, extra):
    exe = str(tmp_path / name)
    subprocess.check_call(["gcc", "-std=c11", "-ffp-contract=off", *extra, "-o", exe,
                           os.path.join(DRV, name + ".c"), SRC, "-lm"])
    return exe


def test_bruteforce_tiny_fields(tmp_path):
    exe = _build(tmp_path, "bf_tiny", ["-O2"])
    out = subprocess.run([exe, "1"], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "failures 0" in out.stdout


def test_corrupt_stream_fuzz_sanitized(tmp_path):
    exe = _build(tmp_path, "fuzz_corrupt",
                 ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    out = subprocess.run([exe, "4000"], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad 0" in out.stdout
