"""The benchmark workloads at full size (1e8 photons), in the launch
configuration bench.py times (the shape the autotuner picks from pilots of
1/20 of the photons, no digests).

At this size the oracle cannot follow every photon, so the checks are
properties that hold at any size -- every photon launched and terminated
once, the FP64 energy identity, a run split in two halves reproducing the
whole run, mirror-symmetric detectors agreeing within binomial noise -- and
rates compared with an oracle sample of the same workload within its
statistical error.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1711_03244_amd import mcx, workloads as W

pytestmark = pytest.mark.gpu
COUNT_KEYS = ["launched", "escaped", "detected", "timeout", "rr_dead", "capped", "scatters",
              "face_events", "fresnel_draws", "reflections", "rr_tests", "rr_survived", "events"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def terminated(st):
    return st["escaped"] + st["timeout"] + st["rr_dead"] + st["capped"]


def energy_residual(st):
    n = st["launched"]
    return (n + st["w_rr_gain"] - st["absorbed_grid"] - st["w_escaped"] - st["w_timeout"]
            - st["w_rr_loss"] - st["w_capped"]) / max(n, 1)


def whole_and_split(p, N, seed, tune=False):
    with mcx.Simulation(p) as sim:
        if tune:
            t = sim.autotune(max(1000, N // 20), seed + 3000)
            say("autotuned shape: block", t["block_size"], "chunk", t["refill_chunk"],
                "window", t["lds_window_cells"])
        sim.run(N, seed)
        st = sim.stats()
        raw = sim.fluence(mcx.MCX_RAW, f64=True)
        rec = sim.detected() if p.ndet else None
        sim.reset()
        sim.run_range(0, N // 2, seed)
        sim.run_range(N // 2, N - N // 2, seed)
        sim.sync()
        st2 = sim.stats()
        raw2 = sim.fluence(mcx.MCX_RAW, f64=True)
    return st, raw, rec, st2, raw2


def check_properties(st, raw, st2, raw2, N):
    assert st["launched"] == N and terminated(st) == N
    assert abs(energy_residual(st)) < 1e-6
    for k in COUNT_KEYS:
        assert st2[k] == st[k], k
    big = raw > 1e-6 * raw.max()
    assert np.allclose(raw2[big], raw[big], rtol=1e-9)
    assert st2["absorbed_grid"] == pytest.approx(st["absorbed_grid"], rel=1e-12)


def test_sphere_benchmark_full_size():
    p = W.cube_sphere()
    N = 100_000_000
    say(f"[gpu] {p.name} N={N} (bench launch configuration)")
    st, raw, (rec, ph, drop), st2, raw2 = whole_and_split(p, N, 1, tune=True)
    check_properties(st, raw, st2, raw2, N)
    # the default launch shape follows the same photons: same counts, same map
    with mcx.Simulation(p) as sim:
        sim.run(N, 1)
        st3 = sim.stats()
        raw3 = sim.fluence(mcx.MCX_RAW, f64=True)
    for k in COUNT_KEYS:
        assert st3[k] == st[k], k
    big = raw > 1e-6 * raw.max()
    assert np.allclose(raw3[big], raw[big], rtol=1e-9)
    # detector records: one per detected photon, mirror pairs agree
    assert drop == 0 and len(rec) == st["detected"] > 1000
    det = rec[:, 0].astype(int)
    n = np.bincount(det, minlength=4)
    say("detections per detector", n)
    for a, b in [(0, 1), (2, 3)]:
        assert abs(n[a] - n[b]) <= 5 * math.sqrt(n[a] + n[b]), (a, b, n)
    assert len(np.unique(ph)) == len(ph)
    # rates against an oracle sample (photons 0..2e6-1 of the same seed)
    M = 2_000_000
    o = oracle.run(p, M, 1, nthreads=16, ndigest=M)
    w = o["digest"][:, 4]
    # no roulette at this weight scale: a photon's absorbed weight is 1 - its final weight
    assert o["counts"]["rr_tests"] == 0
    a_o, se = float(np.mean(1 - w)), float(np.std(1 - w) / math.sqrt(M))
    a_g = st["absorbed_grid"] / N
    say("absorbed fraction gpu", a_g, "oracle", a_o, "+-", se)
    assert abs(a_g - a_o) <= 5 * se
    r_g, r_o = st["detected"] / N, o["counts"]["detected"] / M
    assert abs(r_g - r_o) <= 5 * math.sqrt(r_o * (1 - r_o) / M) + 1e-12
    for k in ["escaped", "timeout"]:
        f_g, f_o = st[k] / N, o["counts"][k] / M
        assert abs(f_g - f_o) <= 5 * math.sqrt(max(f_o * (1 - f_o), 1e-12) / M), k


def test_homogeneous_cube_full_size():
    p = W.cube_homogeneous()
    N = 100_000_000
    say(f"[gpu] {p.name} N={N}")
    st, raw, _, st2, raw2 = whole_and_split(p, N, 2)
    check_properties(st, raw, st2, raw2, N)
    f = raw[0]
    # the beam enters at (29.5, 29.5) and the cube is the same along x and
    # y: the fluence is symmetric under x <-> y (in expectation)
    other = np.swapaxes(f, 1, 2)
    big = f > 1e-3 * f.max()
    rel = np.abs(other[big] - f[big]) / f[big]
    say("x <-> y: median rel diff", float(np.median(rel)), "cells", int(big.sum()))
    assert np.median(rel) < 5e-3


def test_head_phantom_full_size():
    p = W.head_phantom(1)
    N = 100_000_000
    say(f"[gpu] {p.name} N={N}")
    st, raw, _, st2, raw2 = whole_and_split(p, N, 1, tune=True)
    check_properties(st, raw, st2, raw2, N)
    assert st["rr_tests"] > 0 and st["timeout"] > 0
    M = 100_000
    o = oracle.run(p, M, 1, nthreads=8)
    for k in ["escaped", "timeout", "rr_dead"]:
        f_g, f_o = st[k] / N, o["counts"][k] / M
        say(k, "fraction gpu", f_g, "oracle", f_o)
        assert abs(f_g - f_o) <= 5 * math.sqrt(max(f_o * (1 - f_o), 1e-12) / M) + 1e-9, k
