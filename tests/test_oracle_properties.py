"""Property tests of the FP64 oracle on random small problems (hypothesis):
random grids of 1-5 voxels per side with holes (label 0), up to three media
(absorbing or not, scattering or not, any anisotropy and index), Fresnel on
or off, 1-4 gates, voxel sizes 0.5-2 mm, disk detectors and an event cap.
Whatever the inputs, every photon is launched and ends once, the FP64
ledger balances (launched + roulette gain = absorbed + escaped + timed out
+ roulette loss + capped), the tally is non-negative, and the absorbed
weight equals the sum of mua * tally over the absorbing voxels (the
track-length deposit w (1 - e^{-mua l}) / mua times mua is exactly the
weight lost on the segment).
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
from paper_1711_03244_amd import workloads as W


@st.composite
def problems(draw):
    nx, ny, nz = (draw(st.integers(1, 5)) for _ in range(3))
    nmed = draw(st.integers(1, 3))
    labels = np.array(draw(st.lists(st.integers(0, nmed), min_size=nx * ny * nz,
                                    max_size=nx * ny * nz)), np.uint8).reshape(nz, ny, nx)
    sx, sy = draw(st.integers(0, nx - 1)), draw(st.integers(0, ny - 1))
    labels[0, sy, sx] = draw(st.integers(1, nmed))          # the source voxel is medium
    rows = [(draw(st.sampled_from([0.0, 0.01, 0.3, 2.0])), draw(st.sampled_from([0.0, 0.5, 5.0, 20.0])),
             draw(st.floats(-0.9, 0.95)), draw(st.floats(1.0, 1.6))) for _ in range(nmed)]
    h = draw(st.sampled_from([0.5, 1.0, 2.0]))
    ndet = draw(st.integers(0, 2))
    det = [(draw(st.floats(0, nx * h)), draw(st.floats(0, ny * h)), 0.0, draw(st.floats(0.2, 2.0)))
           for _ in range(ndet)]
    return W.Problem(labels=labels, media=W._media(*rows),
                     src_pos=((sx + 0.5) * h, (sy + 0.5) * h, 0.0), src_dir=(0.0, 0.0, 1.0), h=h,
                     detectors=np.array(det, np.float32).reshape(-1, 4),
                     t0=0.0, dt=draw(st.sampled_from([0.01, 0.1, 1.0])),
                     ngates=draw(st.integers(1, 4)), reflect=draw(st.booleans()),
                     max_events=20_000)


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow],
          derandomize=True)
@given(p=problems(), seed=st.integers(0, 2**32 - 1))
def test_ledger_balances_and_tally_matches_absorption(p, seed):
    N = 300
    r = oracle.run(p, N, seed, nthreads=2)
    c, L = r["counts"], r["ledger"]
    assert c["launched"] == N
    assert c["escaped"] + c["timeout"] + c["rr_dead"] + c["capped"] == N
    assert c["detected"] <= c["escaped"] and L["detected"] <= L["escaped"] + 1e-12
    lhs = L["launched"] + L["rr_gain"]
    rhs = L["absorbed"] + L["escaped"] + L["timeout"] + L["rr_loss"] + L["capped"]
    assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-9)
    tally = r["tally"]
    assert np.all(tally >= 0)
    mua = np.asarray(p.media, np.float64)[:, 0][p.labels]
    absorbing = mua > 0
    from_tally = float((tally[:, absorbing] * mua[absorbing]).sum())
    assert from_tally == pytest.approx(L["absorbed"], rel=1e-9, abs=1e-12)
