"""The bench reports HBM traffic only from counters taken on the kernel
source and the launch it timed: any other block size, job size, LDS window
or kind of map add gives no figure (no GPU needed)."""
import json

import pytest

from paper_1711_03244_amd import roofline


def committed_launch():
    with open(roofline.COUNTERS) as f:
        c = json.load(f)
    (window, e), = c["by_window"].items()
    took = e["launch"]
    return c, {"block_size": took["block_size"], "refill_chunk": took["refill_chunk"],
               "lds_window_cells": int(window),
               "map_adds": {"64-bit": 1, "32-bit with carry": 2}[took["map_adds"]]}


def test_traffic_only_for_the_profiled_launch():
    c, launch = committed_launch()
    if c["kernel_source_sha256"] != roofline.kernel_source_hash():
        pytest.skip("the committed counters predate the current kernel source")
    n = c["photons"]
    t = roofline.measured_traffic(n, launch)
    assert t is not None and t > 0
    assert roofline.measured_traffic(2 * n, launch) == pytest.approx(2 * t, rel=1e-12)
    for key, other in [("block_size", 768), ("refill_chunk", 256), ("lds_window_cells", 16384),
                       ("map_adds", 3 - launch["map_adds"])]:
        assert roofline.measured_traffic(n, dict(launch, **{key: other})) is None, key


def test_no_traffic_when_the_source_changed(monkeypatch):
    _, launch = committed_launch()
    monkeypatch.setattr(roofline, "kernel_source_hash", lambda: "0" * 64)
    assert roofline.measured_traffic(10**8, launch) is None
