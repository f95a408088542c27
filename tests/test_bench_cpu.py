"""Host logic of bench.py: the calibrated traffic table must describe the
kernel source in the tree (a stale entry would attach another build's HBM
bytes to the roofline)."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_2211_14969_amd import inputs  # noqa: E402


def test_traffic_table_matches_kernel_source():
    h = bench.kernel_source_hash()
    default = inputs.single_bump().name
    for prec in ("fp64", "fp32"):
        assert (h, default, prec) in bench.MEASURED_TRAFFIC, (h, default, prec)
    for (hh, _, _), tr in bench.MEASURED_TRAFFIC.items():
        assert hh == h
        assert tr["fetch_bytes"] > 0 and tr["write_bytes"] > 0 and tr["kernel"]

