"""Host arithmetic of the roofline figures the benchmark reports (no GPU):
the FP32 lane-rate peak from the chip's unit counts and clock, the work
model's linearity in the event counts, the VALU and atomic fractions, and
the gating of the HBM traffic figure on the kernel source hash and the LDS
window the committed counters were taken with."""
import json

import pytest

from paper_1711_03244_amd import roofline as R

EVENTS = ["events", "scatters", "face_events", "fresnel_draws", "launched"]
PER_EVENT = [R.SEGMENT, R.SCATTER, R.FACE, R.FRESNEL, R.LAUNCH]


def test_peak_is_the_fp32_lane_rate():
    assert R.VALU_PEAK == pytest.approx(256 * 64 * 2.4e9)
    assert R.VALU_PEAK / 1e12 == pytest.approx(39.3216)
    # a Philox4x32-10 block costs the 60 issue slots the microbenchmark measured
    assert R.PHILOX_BLOCK == 60


def test_work_model_is_linear_in_the_event_counts():
    zero = dict.fromkeys(EVENTS, 0)
    assert R.algorithmic_ops(zero) == 0
    for name, per in zip(EVENTS, PER_EVENT):
        assert R.algorithmic_ops(dict(zero, **{name: 7})) == 7 * per
    mixed = dict(zip(EVENTS, [378, 50, 300, 9, 1]))
    assert R.algorithmic_ops(mixed) == sum(R.algorithmic_ops(dict(zero, **{k: v}))
                                           for k, v in mixed.items())
    # every event kind costs more than its bare bookkeeping
    assert min(PER_EVENT) > 10 and R.SCATTER > R.PHILOX_BLOCK and R.FRESNEL > R.PHILOX_BLOCK


def test_fractions():
    stats = dict(zip(EVENTS, [4e9, 1e9, 3e9, 1e8, 1e7]), flushes=1.18e10)
    ops = R.algorithmic_ops(stats)
    v = R.valu_roofline(stats, 0.5)
    assert v["bound"] == "alu" and v["ops_per_launch"] == ops
    assert v["frac"] == pytest.approx(ops / 0.5 / R.VALU_PEAK)
    assert v["achieved"] / v["peak"] == pytest.approx(v["frac"])
    a = R.atomic_roofline(stats, 0.5)
    assert a["frac"] == pytest.approx(1.18e10 / 0.5 / 2.36e10)
    assert a["atomics_per_photon"] == pytest.approx(1180.0)


def counters(tmp_path, monkeypatch, sha, window=1000, key=None):
    c = {"kernel_source_sha256": sha, "photons": 1_000_000, "fetch_factor": 2.0,
         "write_factor": 1.0,
         "by_window": {str(key or window): {"launch": {"lds_window_cells": window},
                                           "fetch_kib": 1.5, "write_kib": 4.0}}}
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(c))
    monkeypatch.setattr(R, "COUNTERS", str(path))


def test_traffic_scales_the_counters_per_photon(tmp_path, monkeypatch):
    counters(tmp_path, monkeypatch, R.kernel_source_hash())
    per_photon = (1.5 * 2.0 + 4.0 * 1.0) * 1024 / 1e6
    assert R.measured_traffic(1_000_000, 1000) == pytest.approx(per_photon * 1e6)
    assert R.measured_traffic(5_000_000, 1000) == pytest.approx(per_photon * 5e6)
    assert R.measured_traffic(1_000_000, 2000) is None          # no entry for this window


def test_traffic_is_null_for_other_source_or_a_mislabelled_entry(tmp_path, monkeypatch):
    counters(tmp_path, monkeypatch, "0" * 64)
    assert R.measured_traffic(1_000_000, 1000) is None
    counters(tmp_path, monkeypatch, R.kernel_source_hash(), window=1000, key=2000)
    assert R.measured_traffic(1_000_000, 2000) is None
    monkeypatch.setattr(R, "COUNTERS", str(tmp_path / "missing.json"))
    assert R.measured_traffic(1_000_000, 1000) is None


def test_committed_counters_give_the_profiled_traffic():
    with open(R.COUNTERS) as f:
        c = json.load(f)
    if c["kernel_source_sha256"] != R.kernel_source_hash():
        pytest.skip("transport source changed since the counters were taken")
    # 1e8-photon sphere benchmark, 18432-cell window: 417.6 GB per launch
    assert R.measured_traffic(100_000_000, 18432) / 1e9 == pytest.approx(417.6, abs=0.1)
    assert R.measured_traffic(100_000_000, 8192) is None
