"""The integer-VALU throughput probe behind the roofline's measured peak:
every probed instruction runs at a plausible rate for 256 compute units
(between a quarter of and twice the published 39.3 T lane-ops/s), and the
peaks the bench takes never exceed the published ones."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_probe_rates_and_peaks():
    import torch
    torch.cuda.init()
    vp = bench.valu_peak(iters=2000)
    rates = vp["rates_tinst_s"]
    assert set(rates) == set(bench.VALU_OPS)
    for name, r in rates.items():
        assert 0.25 * 39.3 < r < 2 * 39.3, (name, r)
    assert vp["peak16"] <= bench.PEAK_OPS16 and vp["peak32"] <= bench.PEAK_OPS32
    assert vp["peak16"] > 0.5 * bench.PEAK_OPS16 and vp["peak32"] > 0.5 * bench.PEAK_OPS32
