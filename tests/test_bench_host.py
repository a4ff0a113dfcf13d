"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the roofline
arithmetic over the library's per-pass timing records, the rule that attaches
measured HBM traffic only to the kernels it was taken on, and the recovery
check that decides whether a step counts."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports neither torch nor the library at module level)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


class _FakeTorch:
    class cuda:
        @staticmethod
        def synchronize():
            pass


class _FakeLib:
    """Stands in for the binding's profiling calls with fixed records."""

    def __init__(self, records):
        self.records = records
        self.enabled = []
        self.resets = 0

    def cs_prof_reset(self):
        self.resets += 1

    def cs_prof_enable(self, on):
        self.enabled.append(on)
        return True

    def cs_prof_read(self):
        return self.records


RECORDS = {
    # 10 launches of 8 MB in 0.1 ms total: 10 us each, 800 GB/s
    "row_happly": {"launches": 10, "total_ms": 0.1, "bytes": 10 * 8e6},
    # 10 launches of 4 MB in 0.05 ms total
    "col_fwd": {"launches": 10, "total_ms": 0.05, "bytes": 10 * 4e6},
    # a class that never ran is ignored
    "col_inv": {"launches": 0, "total_ms": 0.0, "bytes": 0.0},
}


def _roofline(traffic_file, shape, steps=5):
    calls = []
    lib = _FakeLib(RECORDS)
    roof, prof = bench.profiled_roofline(_FakeTorch, lib, lambda: calls.append(1), steps, traffic_file, shape)
    assert len(calls) == steps
    assert lib.resets == 1 and lib.enabled == [True, False]
    assert prof is RECORDS
    return roof


def test_roofline_arithmetic():
    roof = _roofline("no_such_traffic_file.json", [9, 10, 2, 2])
    assert roof["kernel"] == "row_happly"             # the largest share of pass time
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["avg_launch_us"] == pytest.approx(10.0)
    assert roof["algorithmic_bytes_per_launch"] == pytest.approx(8e6)
    assert roof["achieved"] == pytest.approx(800.0)
    assert roof["frac"] == pytest.approx(0.1)
    assert roof["launches_per_step"] == pytest.approx(2.0)
    assert roof["share_of_transform_time"] == pytest.approx(0.1 / 0.15, abs=1e-3)
    # every pass together: 120 MB in 0.15 ms
    assert roof["all_transform_passes"]["achieved"] == pytest.approx(800.0)
    assert roof["traffic"] is None                    # no counter file: nothing to attach


def test_roofline_without_records():
    lib = _FakeLib({"row_happly": {"launches": 0, "total_ms": 0.0, "bytes": 0.0}})
    roof, _ = bench.profiled_roofline(_FakeTorch, lib, lambda: None, 1, "x.json", [1])
    assert roof is None


def test_traffic_attached_only_to_the_profiled_kernels():
    name = "traffic_sp_ompr_n2p20_sp.json"
    t = json.load(open(os.path.join(ROOT, "profiles", name)))
    shape = list(t["shape"])
    want = t["classes"]["row_happly"]["hbm_bytes_per_launch"] if t["source_hash"] == bench.source_hash() else None
    assert _roofline(name, shape)["traffic"] == want
    # another transform shape: the counters describe other kernels
    other = shape[:-1] + [shape[-1] + 1]
    assert _roofline(name, other)["traffic"] is None


def test_source_hash_is_stable():
    h = bench.source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.source_hash() == h


def test_recovered_rule():
    supp = np.array([1, 4, 7])
    vals = np.array([1.0, -2.0, 0.5])
    s = np.zeros(10)
    s[supp] = vals
    assert bench.recovered(s, supp, None)[0] is False
    ok, err = bench.recovered(s, supp, (supp, vals))
    assert ok and err == 0.0
    # within the relative tolerance
    s2 = s.copy()
    s2[4] += 1e-6
    ok, err = bench.recovered(s2, supp, (supp, vals))
    assert ok and err == pytest.approx(1e-6 / np.linalg.norm(vals))
    # outside it
    s3 = s.copy()
    s3[4] += 1e-3
    assert bench.recovered(s3, supp, (supp, vals))[0] is False
    # a different support never counts, however close the values
    assert bench.recovered(s, np.array([1, 4, 8]), (supp, vals))[0] is False
