"""Host-side logic of bench.py (no GPU): the one-GPU rule, the counter
bookkeeping behind the roofline's traffic field, and the work formulas."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_is_reported_only_for_the_source_it_was_measured_on():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for name, r in rec.items():
        src = open(os.path.join(ROOT, r["source"]), "rb").read()
        want = r["bytes_per_launch"] if hashlib.sha256(src).hexdigest() == r["source_sha256"] else None
        assert bench.measured_traffic(name) == want
        # bytes = FETCH_SIZE x its copy-kernel scale + WRITE_SIZE x its scale (KiB per dispatch)
        kib = r["fetch_KiB_per_dispatch"] * r["fetch_scale"] + r["write_KiB_per_dispatch"] * r["write_scale"]
        assert abs(kib * 1024 - r["bytes_per_launch"]) <= 1e-4 * r["bytes_per_launch"] + 1024
    assert bench.measured_traffic("no_such_kernel") is None


def test_heff_flops_closed_form():
    # two environment contractions (2 w d^2 D^3 each) and two one-site MPO
    # stages (2 w^2 d^3 D^2 each) at equal bonds
    D, d, w = 1024, 2, 5
    assert bench.heff_flops(D, d, w) == 4 * w * d * d * D ** 3 + 4 * w * w * d ** 3 * D ** 2
    assert abs(bench.heff_flops(D, d, w) / 1e9 - 86.74) < 0.01


@pytest.mark.parametrize("L", [6, 10])
def test_block_equivalents_of_a_uniform_chain(L):
    # all bonds at the cap: every one of the 2 (L - 1) blocks counts once
    chi = 8
    dims = [chi] * (L + 1)
    assert abs(bench.block_equivalents(dims, 2, 5) - 2 * (L - 1)) < 1e-12


def test_cpu_baseline_reports_all_threads_and_one_thread():
    # the oracle leg at a small bond (the bench runs it at the workload's):
    # the all-thread block and the same block on one thread, both extrapolated
    # by the same block equivalents
    from paper_2606_02930_amd import hamiltonians
    W = hamiltonians.heisenberg(8)
    dims = [1, 2, 4, 8, 16, 8, 4, 2, 1]
    cb = bench.cpu_baseline(dims, 2, W)
    assert cb["kind"] == "oracle" and cb["value"] > 0.0 and cb["cores"] >= 1
    single = cb["single_core"]
    assert "error" in single or (single["cores"] == 1 and single["value"] > 0.0 and single["block_s"] > 0.0)
