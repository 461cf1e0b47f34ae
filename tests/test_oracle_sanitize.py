"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code only) and driven through every entry point on small inputs and edge cases
by tests/oracle_sanitize_main.c: out-of-bounds accesses, use after free, leaks,
signed overflow, invalid shifts and float-to-integer conversions out of range
abort the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "orc_san")
    cmd = ["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-O1", "-g",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-Wall", "-Wno-unknown-pragmas", "-I" + os.path.join(ROOT, "oracle"),
           os.path.join(HERE, "oracle_sanitize_main.c"), os.path.join(ROOT, "oracle", "sr_oracle.c"),
           "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtimes not installed")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip().endswith("ok")
    assert "runtime error" not in run.stderr
