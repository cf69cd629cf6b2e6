"""Detected-photon post-processing on the GPU against the oracle's
post-processing of the same records (paper: detected-photon data as the
output of the Fig. 1 workflow).

Both sides sum FP64 values, the oracle in record order and the GPU over
per-workgroup partial sums, so sums agree to rounding order (1e-12
relative); record counts and per-record re-weighted weights agree exactly up
to the last bit of exp (1e-14)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1711_03244_amd import mcx, workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def wide_detectors(p, r):
    d = p.detectors.copy()
    d[:, 3] = r
    return p.replace(detectors=d)


def check_against_oracle(out, w, rec, N, p, dmua):
    ref, wref = oracle.detected_postprocess(rec, N, p.ndet, p.t0, p.dt, p.ngates, dmua)
    assert np.array_equal(out[:, 0], ref[:, 0])
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-15 * np.abs(ref[:, 1:]).max())
    if w is not None:
        assert np.allclose(w, wref, rtol=1e-14, atol=0)
    return ref


@pytest.mark.parametrize("dmua", [None, (0.002, -0.001)])
def test_detected_process_matches_oracle(dmua):
    p = wide_detectors(W.cube_sphere(n=30, ngates=10, dt=0.2), 3.0).replace(name="cube30_sphere")
    N = 200_000
    say(f"[gpu] {p.name} N={N} dmua={dmua}")
    with mcx.Simulation(p) as sim:
        sim.run(N, 2)
        st = sim.stats()
        rec, _, dropped = sim.detected()
        out, w = sim.detected_process(dmua, weights=True)
    assert dropped == 0 and len(rec) == st["detected"] > 1000
    ref = check_against_oracle(out, w, rec, N, p, dmua)
    say("records", len(rec), "reflectance", ref[:, 1])
    if dmua is None:
        # the ledger's detected weight is the FP64 sum of the same weights
        assert out[:, 1].sum() * N == pytest.approx(st["w_detected"], rel=1e-6)
        assert out[:, 0].sum() == st["detected"]


def test_reweighting_matches_a_gpu_run_with_changed_absorption():
    """With roulette off, a run with absorption mua + dmua follows the same
    paths (stepping depends on the scattering properties only): its detector
    outputs equal the first run's records re-weighted by dmua.

    Both runs carry each photon's weight in FP32 through its segments (one
    multiply and one subtraction per segment) and sum its pathlengths in
    FP32, so a record's weight differs between the re-weighted and the
    direct run by a sum of roundings: with up to ~2000 segments per photon
    (2 ns at 1 mm steps) about sqrt(3 * 2000) * 2^-24 / sqrt(3) ~ 3e-6
    relative at one standard deviation.  Bars: 3e-5 per record (about 10
    sigma), 1e-5 for the per-detector and per-gate sums."""
    p = wide_detectors(W.cube_sphere(n=30, ngates=10, dt=0.2), 3.0).replace(rr_threshold=0.0)
    dmua = np.array([0.003, -0.0015], np.float32)
    media = p.media.copy()
    media[1:, 0] = media[1:, 0] + dmua
    q = p.replace(media=media)
    exact = q.media[1:, 0].astype(np.float64) - p.media[1:, 0].astype(np.float64)
    N = 200_000
    say(f"[gpu] reweighting, N={N}")
    with mcx.Simulation(p) as a, mcx.Simulation(q) as b:
        a.run(N, 6)
        b.run(N, 6)
        out_a, w_a = a.detected_process(exact, weights=True)
        out_b, _ = b.detected_process()
        plain_a, _ = a.detected_process()
        rec_a, ph_a, _ = a.detected()
        rec_b, ph_b, _ = b.detected()
    oa, ob = np.argsort(ph_a), np.argsort(ph_b)
    assert np.array_equal(ph_a[oa], ph_b[ob])
    assert np.array_equal(rec_a[oa][:, [0, 1]], rec_b[ob][:, [0, 1]])
    rel = np.abs(w_a[oa] - rec_b[ob][:, 2]) / rec_b[ob][:, 2]
    say(f"records {len(rel)}, per-record relative difference median {np.median(rel):.2e}, "
        f"max {rel.max():.2e}")
    assert rel.max() <= 3e-5
    assert np.array_equal(out_a[:, 0], out_b[:, 0])
    assert np.allclose(out_a[:, 1:], out_b[:, 1:], rtol=1e-5, atol=1e-12 * out_b[:, 1:].max())
    assert out_b[:, 1].sum() < 0.97 * plain_a[:, 1].sum()


def test_detpost_device_many_detectors_and_edge_cases():
    """Synthetic records in device memory: 300 detectors x 40 gates need two
    passes over detector ranges; records with detector indices outside the
    range, non-integer, or NaN, times before t0 and past the last gate; an
    empty record set; raw sums (nphoton = 0)."""
    import torch
    rng = np.random.default_rng(5)
    n, npath, ndet, ngates = 200_000, 3, 300, 40
    rec = np.empty((n, 4 + npath), np.float32)
    rec[:, 0] = rng.integers(-5, ndet + 10, n)
    rec[rng.random(n) < 0.01, 0] += 0.5
    rec[rng.random(n) < 0.001, 0] = np.nan
    rec[:, 1] = rng.integers(0, 500, n)
    rec[:, 2] = rng.random(n)
    rec[:, 3] = rng.uniform(-0.5, 6.0, n)
    rec[:, 4:] = rng.exponential(20.0, (n, npath))
    spec = dict(ndet=ndet, npath=npath, t0=0.25, dt=0.125, ngates=ngates, nphoton=1_000_000)
    dmua = np.array([0.01, -0.002, 0.0005], np.float32)
    say(f"[gpu] detpost device: {n} records, {ndet} detectors x {ngates} gates")
    drec = torch.as_tensor(rec).cuda()
    out, w = mcx.mcx_detpost_device(drec, spec, torch.as_tensor(dmua).cuda(), weight=True)
    torch.cuda.synchronize()
    ref, wref = oracle.detected_postprocess(rec, spec["nphoton"], ndet, spec["t0"], spec["dt"],
                                            ngates, dmua)
    got = out.cpu().numpy()
    assert np.array_equal(got[:, 0], ref[:, 0]) and ref[:, 0].sum() < n
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15 * ref[:, 1:].max())
    assert np.allclose(w.cpu().numpy(), wref, rtol=1e-14, atol=0)
    raw, _ = mcx.mcx_detpost_device(drec, dict(spec, nphoton=0))
    rref, _ = oracle.detected_postprocess(rec, 0, ndet, spec["t0"], spec["dt"], ngates)
    assert np.allclose(raw.cpu().numpy(), rref, rtol=1e-12, atol=0)
    empty, _ = mcx.mcx_detpost_device(torch.zeros((0, 4 + npath), device="cuda"), spec)
    assert not empty.cpu().numpy().any()
    with pytest.raises(mcx.McxError) as e:
        mcx.mcx_detpost_device(drec, dict(spec, ngates=0))
    assert e.value.status == mcx.MCX_EINVAL


def test_sphere_benchmark_reflectance_and_tpsf():
    """The sphere benchmark's four 1 mm detectors over 1e7 photons: the
    per-detector outputs against the oracle's post-processing of the same
    records, the ledger's detected weight, and the +x / -x and +y / -y
    detector pairs (mirror images under the sphere's symmetry) within their
    counting noise."""
    p = W.cube_sphere()
    N = 10_000_000
    say(f"[gpu] {p.name} N={N}")
    with mcx.Simulation(p) as sim:
        sim.run(N, 1)
        st = sim.stats()
        rec, _, dropped = sim.detected()
        out, _ = sim.detected_process()
    assert dropped == 0
    check_against_oracle(out, None, rec, N, p, None)
    assert out[:, 1].sum() * N == pytest.approx(st["w_detected"], rel=1e-6)
    for a, b in [(0, 1), (2, 3)]:
        se = math.sqrt(1 / out[a, 0] + 1 / out[b, 0])
        say("detectors", a, b, "records", out[a, 0], out[b, 0], "R", out[a, 1], out[b, 1])
        assert abs(math.log(out[a, 1] / out[b, 1])) < 6 * se
    # the 10 mm pair sees more light, and earlier, than the 20 mm pair
    assert out[0, 1] > 3 * out[2, 1]
    mean_t = lambda d: (out[d, 2:] * (np.arange(p.ngates) + 0.5)).sum() / out[d, 2:].sum()
    assert mean_t(0) < mean_t(2)
