"""Host-side logic of bench.py (no GPU): the traffic record is used only for
the kernel source it was measured on, the workloads have the sizes the
metric is quoted on, and the CPU baseline reports the oracle's rate on a
bounded sample with the fields the benchmark line carries."""
import hashlib
import json
import os

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_record_used_only_for_its_sweep_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    src = open(os.path.join(ROOT, "paper_2511_11425_amd", "csrc", "sph_sweep.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()
    for kernel, r in rec.items():
        want = r["fetch_bytes"] + r["write_bytes"] if r["source_sha256"] == sha else None
        assert bench.traffic_of(kernel, r["workload"]) == want, kernel
        # the counters are scaled by what they read for a copy of known size
        assert r["fetch_bytes"] == pytest.approx(r["fetch_kib_counter"] * 1024 * r["fetch_factor"])
        assert r["write_bytes"] == pytest.approx(r["write_kib_counter"] * 1024 * r["write_factor"])


def test_traffic_is_withheld_for_another_workload_or_kernel():
    assert bench.traffic_of("k_forces<2, true>", "two_phase") is None
    assert bench.traffic_of("no_such_kernel", "large") is None


def test_headline_workload_sizes():
    c = bench.make_workload("large", small=True)
    assert c["n"] == 64 ** 3 and c["ngroups"] == 64 ** 3 // 64
    assert c["params"]["kernel"] == "wc4" and c["params"]["n_ngb"] == 200.0
    assert bench._ngroups([64, 65, 1]) == 1 + 2 + 1


def test_cpu_baseline_on_a_small_sample(orc):
    c = bench.make_workload("large", small=True)
    r = bench.cpu_baseline(c, seconds=1.5)
    assert r["kind"] == "oracle" and r["unit"] == "pair interactions/s"
    assert r["value"] > 0 and np.isfinite(r["value"])
    assert r["cores"] >= 1
    assert "particles" in r["sample"] and "median of 3 runs" in r["sample"]
