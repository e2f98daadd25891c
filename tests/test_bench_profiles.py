"""The committed rocprofv3 summaries that bench.py reads: the HBM traffic of
the headline kernel and the VALU instruction counts of every 256^3 form.
Both carry a digest of the step kernels' sources; while it matches, every
form the bench times must find its kernels' counts (so its VALU-roofline
fraction is reported), and the traffic must be the calibrated bytes of one
launch."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_valu_counts_cover_every_form():
    counts = bench.read_valu_counts()
    if not counts:
        pytest.skip("VALU counts taken on other kernel sources (profiles need a new run)")
    for name, storage, streaming, var in bench.FORMS_256:
        t = bench.valu_issue_ms(counts, storage, streaming, var, bench.N)
        assert t is not None and t > 0, name
    # the headline form as well
    assert bench.valu_issue_ms(counts, "F64", "PULL", None, bench.N) > 0


def test_headline_traffic_is_one_launch_of_calibrated_bytes():
    traffic = bench.read_counters()
    if traffic is None:
        pytest.skip("traffic counters taken on other kernel sources (profiles need a new run)")
    algorithmic = 432 * bench.N ** 3
    assert 0.98 * algorithmic < traffic < 1.1 * algorithmic
