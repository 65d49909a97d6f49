"""The FP64 oracle under the host sanitizers (CPU).

tests/oracle_asan_driver.c runs tiny solves through every path of the
oracle's source iteration (walls, rows of unequal height, Maxwell walls,
sliding wall, periodic cell with a delta field, a one-column channel,
rejected inputs, the quadrature); here it is compiled together with
oracle/dvm_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer
and must finish with no report."""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no host C compiler")
    exe = tmp_path / "oracle_asan"
    subprocess.run([cc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", str(exe),
                    str(ROOT / "tests" / "oracle_asan_driver.c"), str(ROOT / "oracle" / "dvm_oracle.c"), "-lm"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok"), res.stdout
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr, res.stderr
