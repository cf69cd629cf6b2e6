"""Host-side logic of the denoiser evaluation and the bench's argument
checks (no GPU).

The time-to-equal-error arithmetic (denoise.summarise) is checked on
synthetic rows whose errors follow c / sqrt(n) and whose times follow
T = a n + T0 exactly, so every expected value is a closed form.
"""
import math
import os
import subprocess
import sys

import pytest

from paper_1711_03244_amd import denoise

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def plain_err(n, c=300.0):
    return c / math.sqrt(n)


def test_equivalent_photons_inverts_a_power_law():
    curve = [(n, plain_err(n)) for n in (1e5, 1e6, 1e7, 1e9)]
    for n_eq in (3e5, 2.5e6, 4e7, 5e8):          # inside the measured range
        assert denoise._equivalent_photons(curve, plain_err(n_eq)) == pytest.approx(n_eq, rel=1e-9)
    for n_eq in (2e4, 4e9):                        # extrapolated from the nearest pair
        assert denoise._equivalent_photons(curve, plain_err(n_eq)) == pytest.approx(n_eq, rel=1e-9)
    assert denoise._equivalent_photons(curve[:1], 1.0) is None
    assert denoise._equivalent_photons(curve, 0.0) is None


def synthetic_rows(inputs, n_eq, plain, a, t0, infer_ms, ref_err=0.0):
    """Rows as evaluate() builds them: every input's denoised error equals
    the plain error at n_eq[i] photons (with the reference share added in
    quadrature to every measured error)."""
    def measured(e):
        return math.sqrt(e * e + ref_err * ref_err)
    row = {"seed": 1, "mask_voxels": 100, "ref_err": ref_err, "plain_err": measured(plain_err(plain)),
           "plain_ms": a * plain + t0, "inputs": []}
    for n, ne in zip(inputs, n_eq):
        row["inputs"].append({"photons": int(n), "sim_ms": a * n + t0, "infer_ms": infer_ms,
                              "noisy_err": measured(plain_err(n)),
                              "denoised_err": measured(plain_err(ne))})
    return [row, dict(row, seed=2)]


@pytest.mark.parametrize("ref_err", [0.0, 0.004])
def test_summarise_time_ratios_are_the_closed_forms(ref_err):
    inputs, n_eq = [1e5, 1e6, 1e7], [4e6, 3e7, 1.5e8]
    a, t0, inf = 8e-6, 26.0, 0.4
    out = denoise.summarise(synthetic_rows(inputs, n_eq, 1e9, a, t0, inf, ref_err), 1e9, inputs)
    assert out["plain_time_model"]["ms_per_photon"] == pytest.approx(a, rel=1e-9)
    assert out["plain_time_model"]["overhead_ms"] == pytest.approx(t0, rel=1e-6)
    assert out["plain_err_debiased"] == pytest.approx(plain_err(1e9), rel=1e-9)
    for r, n, ne in zip(out["per_input"], inputs, n_eq):
        assert r["denoised_err_debiased"] == pytest.approx(plain_err(ne), rel=1e-9)
        assert r["equal_error_plain_photons"] == pytest.approx(ne, rel=1e-6)
        assert r["time_ratio"] == pytest.approx((a * ne + t0) / (a * n + t0 + inf), rel=1e-6)
    assert out["best_time_ratio"] == max(r["time_ratio"] for r in out["per_input"])
    # no input reaches the plain run's error: the strict ratio is absent
    assert out["time_ratio"] is None and out["equal_error_photons"] is None
    assert "batched" not in out


def test_summarise_batched_ratios_use_the_batched_model():
    inputs, n_eq = [1e5, 1e6, 1e7], [4e6, 3e7, 1.5e8]
    a, t0, inf = 8e-6, 26.0, 0.4
    ab, t0b = 6e-6, 2.5                      # per-volume batched model
    batched = [(n, ab * n + t0b) for n in inputs + [3e7]]
    out = denoise.summarise(synthetic_rows(inputs, n_eq, 1e9, a, t0, inf), 1e9, inputs, batched)
    b = out["batched"]
    assert b["time_model"]["ms_per_photon"] == pytest.approx(ab, rel=1e-9)
    assert b["time_model"]["overhead_ms"] == pytest.approx(t0b, rel=1e-6)
    for r, n, ne in zip(out["per_input"], inputs, n_eq):
        assert r["batched_sim_ms"] == pytest.approx(ab * n + t0b, rel=1e-12)
        assert r["batched_time_ratio"] == pytest.approx((ab * ne + t0b) / (ab * n + t0b + inf),
                                                        rel=1e-6)
    assert b["best_time_ratio"] == max(r["batched_time_ratio"] for r in out["per_input"])


def test_summarise_reports_the_strict_ratio_when_an_input_reaches_the_plain_error():
    inputs, n_eq = [1e5, 1e6], [2e7, 2e9]    # the second input beats the 1e9 run
    a, t0, inf = 8e-6, 26.0, 0.4
    out = denoise.summarise(synthetic_rows(inputs, n_eq, 1e9, a, t0, inf), 1e9, inputs)
    assert out["equal_error_photons"] == 1_000_000
    assert out["time_ratio"] == pytest.approx((a * 1e9 + t0) / (a * 1e6 + t0 + inf), rel=1e-9)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bf16_bits_round_to_nearest_even_like_torch():
    """The checkpoint's BF16 rounding equals torch's float32 -> bfloat16
    conversion (round to nearest even) on normal, subnormal, tie, huge and
    special values."""
    import numpy as np
    import torch
    from paper_1711_03244_amd import nn
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32),
                        (rng.normal(size=2000) * 1e-39).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, -2.5, np.inf, -np.inf, 3.4e38, -3.4e38,
                                  1.00390625, 1.01171875, 1e-45], np.float32)])
    # exact ties: low 16 bits 0x8000 with even and odd upper halves
    ties = (np.arange(1000, dtype=np.uint32) << 16 | 0x8000).astype(np.uint32) + (0x3f80 << 16)
    x = np.concatenate([x, ties.view(np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(nn.bf16_bits(x), want)
    nanbits = nn.bf16_bits(np.array([np.nan], np.float32))
    assert (nanbits[0] & 0x7f80) == 0x7f80 and (nanbits[0] & 0x7f) != 0


def test_strict_error_estimators_recover_known_noise():
    """Closed form: maps = truth * exp(noise) with independent Gaussian log
    noise.  K runs of sigma_run each estimate a plain run of K times their
    photons, whose log error is sigma_run / sqrt(K); a map with log noise
    sigma_m compared against their mean has error sigma_m once the
    reference's own share is removed."""
    import numpy as np
    rng = np.random.default_rng(7)
    shape = (40, 40, 40)
    truth = np.exp(rng.uniform(-10, -2, shape))
    mask = np.ones(shape, bool)
    K, s_run, s_m = 2, 0.02, 0.011
    runs = [truth * np.exp(rng.normal(0, s_run, shape)) for _ in range(K)]
    ref = np.mean(runs, axis=0)
    ep2 = denoise.plain_error_sq(runs, mask)
    assert math.sqrt(ep2) == pytest.approx(s_run / math.sqrt(K), rel=0.01)
    m = truth * np.exp(rng.normal(0, s_m, shape))
    e2 = denoise.error_sq_against(m, ref, mask, ep2)
    assert math.sqrt(e2) == pytest.approx(s_m, rel=0.03)


def test_committed_inference_checkpoint_is_plain_arrays_with_provenance():
    """The bench's denoiser checkpoint loads without unpickling and says how
    it was made: the command, the training-volume seeds (disjoint from the
    held-out seeds 900001.. the bench evaluates), the photon counts and the
    source commit."""
    import json
    import os
    import numpy as np
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1711_03244_amd", "checkpoints", "denoiser_64cube.npz")
    with np.load(path, allow_pickle=False) as z:
        assert z["weights_bf16"].dtype == np.uint16 and z["biases"].dtype == np.float32
        assert tuple(z["channels"]) == (32, 64, 128, 256) and tuple(z["shape"]) == (64, 64, 64)
        assert np.all(np.isfinite(z["biases"]))
        w = (z["weights_bf16"].astype(np.uint32) << 16).view(np.float32)
        assert np.all(np.isfinite(w)) and np.abs(w).max() < 100
        meta = json.loads(str(z["meta"]))
    h = meta["history"][-1]
    lo, hi = h["train_volume_seeds"]
    assert hi < 900001
    assert h["target"] == 1e9 and "denoise" in h["command"] and h["source_commit"]
