"""Host-side logic of bench.py (no GPU): the one-GPU guard, the validity
check of the profiled traffic figures and the comparison with the stored
FP64 oracle results."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_no_gpu_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _run("--steps", "1", "--warmup", "0", "--no-cpu")
    assert r.returncode == 1
    assert "no GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_traffic_figures_only_for_the_profiled_kernel():
    import bench
    path = os.path.join(ROOT, "profiles", "k_sweep_traffic.json")
    with open(path) as f:
        tr = json.load(f)
    with open(os.path.join(ROOT, "paper_1704_03126_amd", "csrc", "dvm_kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    got = bench.measured_traffic(tr["schedule"], *tr["shape"])
    if not sha.startswith(tr["kernel_source_sha256_prefix"]):
        # the kernel changed since the counters were taken: no figures
        assert got is None
        return
    assert got is not None and got["fetch_bytes"] > 0 and got["write_bytes"] > 0
    other = "skew" if tr["schedule"] != "skew" else "wrap"
    assert bench.measured_traffic(other, *tr["shape"]) is None
    assert bench.measured_traffic(tr["schedule"], tr["shape"][0] * 2, tr["shape"][1]) is None


def test_stored_oracle_error():
    import bench
    from paper_1704_03126_amd.geometry import cfg_rough_channel
    g = cfg_rough_channel()
    with open(os.path.join(ROOT, "tests", "golden", f"rough_channel_{g.nx}x{g.ny}_nv{bench.NV}.json")) as f:
        ref = {float(r["delta"]): r["Q"] for r in json.load(f)["results"]}
    qs = [ref[d] * (1.0 + 1e-7 * (i + 1)) for i, d in enumerate(bench.DELTAS)]
    err = bench.stored_oracle_error(g, qs)
    for i, d in enumerate(bench.DELTAS):
        assert abs(err[str(d)] - 1e-7 * (i + 1)) < 1e-12
