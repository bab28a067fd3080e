"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): tests/oracle_sanitize.c calls every public oracle function on
small seeded inputs, including the smallest image the census window allows,
ragged sizes, a disparity range next to the width, both aggregation forms,
short and zero arm limits, the Eq. 4 vote, the contour filter and the soft
path.  Any out-of-bounds access, leak, overflow of a signed integer or
other undefined behaviour aborts the run.  CPU only."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.check_call(
        ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-ffp-contract=off", "-std=c99", "-o", exe,
         os.path.join(HERE, "oracle_sanitize.c"), os.path.join(ROOT, "oracle", "dco_oracle.c"),
         "-lm"])
    # verify_asan_link_order=0: a library preloaded by the environment is
    # tolerated instead of refused (the environment is left as it is)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "sanitized oracle run: ok" in r.stdout
