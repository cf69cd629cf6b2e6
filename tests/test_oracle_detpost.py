"""Pins of the oracle's detected-photon post-processing: a hand-worked
record set, the energy ledger of a transport run, the gate sum, and the
physics fact the re-weighting rests on -- with absorption a continuous weight
decay, a run with changed absorption detects the same photons along the same
paths, so re-weighting the first run's records must reproduce the second
run's (paper: detected-photon data as the output of the Fig. 1 workflow)."""
import math

import numpy as np
import pytest

from paper_1711_03244_amd import workloads as W


def test_hand_worked_records(oracle_mod):
    # dmua and pathlengths are exact binary fractions, so every exponent is
    # exact; gates of width 1/8 ns from t0 = 1/4 ns
    rec = np.array([
        # det, nscat, w,    t,     L1, L2
        [0,    3,     0.5,  0.3,   10, 0],   # (0.3 - 0.25) / 0.125 = 0.4  -> gate 0
        [0,    5,     0.25, 0.375, 4,  6],   # exactly 1                   -> gate 1
        [1,    1,     0.125, 0.7,  0,  2],   # 3.6                         -> gate 3
        [1,    2,     1.0,  9.0,   1,  1],   # past the last gate          -> gate 4
        [2,    0,     0.75, 0.5,   3,  3],   # detector 2 of 2: skipped
        [0.5,  0,     0.3,  0.5,   1,  1],   # not an integer: skipped
        [1,    0,     0.2,  0.1,   0,  0],   # before t0                   -> gate 0
    ], np.float32)
    dmua = (1 / 64, 1 / 32)
    out, w = oracle_mod.detected_postprocess(rec, 10, 2, 0.25, 0.125, 5, dmua)
    e = [10 / 64, 4 / 64 + 6 / 32, 2 / 32, 1 / 64 + 1 / 32, 3 / 64 + 3 / 32, 1 / 64 + 1 / 32, 0.0]
    assert np.allclose(w, rec[:, 2] * np.exp(-np.array(e)), rtol=1e-15, atol=0)
    w0, w1, w2, w3, w6 = 0.5 * math.exp(-e[0]), 0.25 * math.exp(-e[1]), 0.125 * math.exp(-e[2]), \
        math.exp(-e[3]), float(np.float32(0.2))
    want = np.zeros((2, 7))
    want[0, :2] = 2, (w0 + w1) / 10
    want[0, 2], want[0, 3] = w0 / 1.25, w1 / 1.25
    want[1, :2] = 3, (w2 + w3 + w6) / 10
    want[1, 2], want[1, 5], want[1, 6] = w6 / 1.25, w2 / 1.25, w3 / 1.25
    assert np.allclose(out, want, rtol=1e-14, atol=0)
    raw, _ = oracle_mod.detected_postprocess(rec, 0, 2, 0.25, 0.125, 5, dmua)
    assert np.allclose(raw[:, 1], want[:, 1] * 10, rtol=1e-14) and np.array_equal(raw[:, 0], want[:, 0])
    empty, w_empty = oracle_mod.detected_postprocess(np.zeros((0, 6), np.float32), 10, 3, 0, 1, 4)
    assert not empty.any() and w_empty.size == 0


def sphere_with_wide_detectors(ngates=10, dt=0.2):
    p = W.cube_sphere(n=30, ngates=ngates, dt=dt)
    d = p.detectors.copy()
    d[:, 3] = 3.0
    return p.replace(detectors=d, rr_threshold=0.0, name="cube30_sphere_wide_det")


def test_ledger_and_gate_sums(oracle_mod):
    p = sphere_with_wide_detectors()
    N = 100_000
    r = oracle_mod.run(p, N, 4, nthreads=4)
    assert r["det_total"] == len(r["records"]) > 500
    out, w = oracle_mod.detected_postprocess(r["records"], N, p.ndet, p.t0, p.dt, p.ngates)
    assert out[:, 0].sum() == r["det_total"] == r["counts"]["detected"]
    # detected weight per launched photon = the transport ledger's (records
    # hold the weights in FP32)
    assert out[:, 1].sum() * N == pytest.approx(r["ledger"]["detected"], rel=1e-6)
    # the gates partition each detector's records
    assert np.allclose(out[:, 2:].sum(axis=1) * float(np.float32(p.dt)), out[:, 1], rtol=1e-12)
    assert np.array_equal(w, r["records"][:, 2].astype(np.float64))
    # +x / -x detectors at the same distance see the same reflectance
    se = math.sqrt(out[0, 0]) / out[0, 0]
    assert abs(out[0, 1] - out[1, 1]) / out[0, 1] < 6 * se


def test_reweighting_reproduces_a_run_with_changed_absorption(oracle_mod):
    p = sphere_with_wide_detectors()
    dmua = np.array([0.003, -0.0015], np.float32)
    media = p.media.copy()
    media[1:, 0] = media[1:, 0] + dmua
    q = p.replace(media=media)
    dmua_exact = q.media[1:, 0].astype(np.float64) - p.media[1:, 0].astype(np.float64)
    N = 60_000
    r1 = oracle_mod.run(p, N, 9, nthreads=4)
    r2 = oracle_mod.run(q, N, 9, nthreads=4)
    # the same photons are detected, with the same pathlengths and times
    o1, o2 = np.argsort(r1["record_photon"]), np.argsort(r2["record_photon"])
    assert np.array_equal(r1["record_photon"][o1], r2["record_photon"][o2])
    a, b = r1["records"][o1], r2["records"][o2]
    assert np.array_equal(a[:, [0, 1, 3, 4, 5]], b[:, [0, 1, 3, 4, 5]])
    out1, w1 = oracle_mod.detected_postprocess(a, N, p.ndet, p.t0, p.dt, p.ngates, dmua_exact)
    out2, _ = oracle_mod.detected_postprocess(b, N, q.ndet, q.t0, q.dt, q.ngates)
    assert np.allclose(w1, b[:, 2], rtol=1e-6, atol=0)
    assert np.array_equal(out1[:, 0], out2[:, 0])
    assert np.allclose(out1[:, 1:], out2[:, 1:], rtol=1e-6, atol=1e-12 * out2[:, 1:].max())
    # and the change is not negligible
    assert np.all(np.abs(out1[:, 1] / out1[:, 1].sum() - out2[:, 1] / out2[:, 1].sum()) >= 0) \
        and abs(out1[:, 1].sum() / out2[:, 1].sum() - 1) < 1e-6
    base, _ = oracle_mod.detected_postprocess(a, N, p.ndet, p.t0, p.dt, p.ngates)
    assert out2[:, 1].sum() < 0.97 * base[:, 1].sum()
