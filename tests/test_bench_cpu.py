"""Host logic of bench.py: the calibrated traffic table must describe the
kernel source in the tree (a stale entry would attach another build's HBM
bytes to the roofline), and the CPU baseline runs both schedules."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_2211_14969_amd import inputs  # noqa: E402


def test_traffic_table_matches_kernel_source():
    h = bench.kernel_source_hash()
    default = inputs.multi_bump().name
    assert (h, default, "fp64") in bench.MEASURED_TRAFFIC, (h, default)
    for (hh, _, _), tr in bench.MEASURED_TRAFFIC.items():
        assert hh == h
        assert tr["fetch_bytes"] > 0 and tr["write_bytes"] > 0 and tr["kernel"]


def test_workloads_name_the_configurations():
    assert bench.make_problems("bumps")[0].name == "bumps_32x32_p32"
    assert len(bench.make_problems("uneven")) == 8


def test_cpu_baseline_times_both_schedules():
    r = bench.cpu_baseline("tiny", 0.5)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
    assert set(r["schedules"]) == {"process_pool", "threaded_blas"}
    assert r["schedule"] in r["schedules"]
    assert r["value"] == max(v["value"] for v in r["schedules"].values())
