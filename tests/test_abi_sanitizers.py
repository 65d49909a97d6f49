"""The C ABI's host layer under the host sanitizers (CPU, no GPU needed).

tests/abi_asan_driver.c calls what runs on the host only: argument checks of
dvm_create, dvm_set_geometry (stencil codes, percolation of every fluid
component, wall faces), dvm_set_row_heights, dvm_set_driving, the host-side
checks of dvm_solve, dvm_flow_rate before a solve, dvm_permeability and
dvm_destroy.  The library's HIP sources are compiled with their host code
under AddressSanitizer and UndefinedBehaviorSanitizer (device code as
usual), linked with the driver, and run; it must finish with no report
(leak detection on)."""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1704_03126_amd" / "csrc"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def test_abi_host_layer_clean_under_asan_and_ubsan(tmp_path):
    if not (Path(HIPCC).exists() and Path(CLANG).exists()):
        pytest.skip("no ROCm compilers")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN]
    srcs = ["dvm_kernels", "dvm_vec", "dvm_api"]
    objs = [tmp_path / f"{s}.o" for s in srcs]

    def cc(args):
        res = subprocess.run(args, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-4000:]

    with ThreadPoolExecutor(len(srcs)) as ex:
        list(ex.map(cc, [[HIPCC, *flags, "-c", str(CSRC / f"{s}.hip"), "-o", str(o)]
                         for s, o in zip(srcs, objs)]))
    drv = tmp_path / "driver.o"
    cc([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-c",
        str(ROOT / "tests" / "abi_asan_driver.c"), "-o", str(drv)])
    exe = tmp_path / "abi_asan"
    cc([HIPCC, "--offload-arch=gfx950", *HOST_SAN, *map(str, objs), str(drv), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]
    assert res.stdout.strip().endswith("ok"), res.stdout
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr, res.stderr
