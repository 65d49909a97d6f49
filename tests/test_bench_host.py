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
    """Profiler byte counts are reported only for the kernel source, workload,
    precision, order and launch shape they were taken on."""
    import bench
    path = os.path.join(ROOT, "profiles", "k_sweep_traffic.json")
    with open(path) as f:
        entries = json.load(f)
    if isinstance(entries, dict):
        entries = [entries]
    h = hashlib.sha256()
    for name in ("dvm_kernels.hip", "dvm_sweep_body.inc", "dvm_internal.h"):
        with open(os.path.join(ROOT, "paper_1704_03126_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()
    assert sha == bench.kernel_source_sha256()
    for tr in entries:
        wl, prec = tr.get("workload_key", "rough_channel"), tr.get("precision", "fp64")
        got = bench.measured_traffic(wl, prec, *tr["shape"], schedule=tr.get("schedule"))
        if not sha.startswith(tr["kernel_source_sha256_prefix"]):
            # the kernel changed since the counters were taken: no figures
            assert got is None
            continue
        assert got is not None and got["fetch_bytes"] > 0 and got["write_bytes"] > 0
        other = "fp32" if prec == "fp64" else "fp64"
        assert bench.measured_traffic(wl, other, *tr["shape"]) is None
        assert bench.measured_traffic(wl, prec, tr["shape"][0] * 2, tr["shape"][1]) is None
        assert bench.measured_traffic("no_such_workload", prec, *tr["shape"]) is None


def test_batch_oracle_error():
    import bench
    path = os.path.join(ROOT, "tests", "golden", "batch64_subset_nv48.json")
    if not os.path.exists(path):
        pytest.skip("stored batch results not generated")
    with open(path) as f:
        ref = json.load(f)["instances"]
    qs = [1.0] * 64
    for k, r in enumerate(ref):
        qs[r["index"]] = r["Q"] * (1.0 + 1e-7 * (k + 1))
    err = bench.batch_oracle_error(qs)
    for k, r in enumerate(ref):
        assert abs(err[str(r["index"])] - 1e-7 * (k + 1)) < 1e-12


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
