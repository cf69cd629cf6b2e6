"""Pins of the oracle's transport loop: closed forms with scattering off
(Beer-Lambert, time gates, Fresnel round trips), hand-worked paths on tiny
grids, exact energy conservation, detector records, and the invariants the
method's construction fixes (prefix property, thread independence,
trajectories independent of absorption, unbiased roulette, x/y symmetry)."""
import math

import numpy as np
import pytest

from paper_1711_03244_amd import workloads as W

C = 299.792458


def energy_residual(p, r):
    """N + roulette gain - (absorbed from the grid + escaped + timeout +
    roulette loss + capped), relative to N."""
    L = r["ledger"]
    n = L["launched"]
    mua = np.asarray(p.media, np.float64)[:, 0][p.labels]
    absorbed = float((r["tally"].sum(axis=0) * mua).sum())
    return (n + L["rr_gain"] - absorbed - L["escaped"] - L["timeout"] - L["rr_loss"]
            - L["capped"]) / n


# ------------------------------------------------------------ Beer-Lambert

@pytest.mark.parametrize("mua", [0.005, 0.08, 0.0])
def test_beer_lambert_column(oracle_mod, mua):
    p = W.slab_column(nz=60, mua=mua, mus=0.0)
    mua = float(p.media[1, 0])  # the stored float32 value
    N = 1000
    r = oracle_mod.run(p, N, seed=5, nthreads=2)
    t = r["tally"][0] / N
    k = np.arange(60)
    expect = np.exp(-mua * k) * (-np.expm1(-mua)) / mua if mua > 0 else np.ones(60)
    assert np.allclose(t[:, 1, 1], expect, rtol=1e-12, atol=0)
    mask = np.ones_like(t, bool)
    mask[:, 1, 1] = False
    assert not t[mask].any()
    assert r["counts"]["escaped"] == N and r["counts"]["scatters"] == 0
    assert r["ledger"]["escaped"] / N == pytest.approx(math.exp(-60 * mua), rel=1e-12)
    assert abs(energy_residual(p, r)) < 1e-12


def test_beer_lambert_gates(oracle_mod):
    # Straight flight at c/n: the segment through voxel k starts at
    # t = k h n / c and is booked in gate floor(t / dt).
    dt = 0.02
    p = W.slab_column(nz=60, mua=0.01, mus=0.0, ngates=20, dt=dt)
    r = oracle_mod.run(p, 10, seed=1, nthreads=1)
    t = r["tally"][:, :, 1, 1] / 10
    mua, n = float(p.media[1, 0]), float(p.media[1, 3])
    for k in range(60):
        gate = min(int(math.floor(k * n / C / p.dt)), 19)
        expect = math.exp(-mua * k) * (-math.expm1(-mua)) / mua
        assert t[gate, k] == pytest.approx(expect, rel=1e-12), k
        assert t[:, k].sum() == pytest.approx(expect, rel=1e-12)


def test_beer_lambert_timeout(oracle_mod):
    # A 0.1 ns window ends the flight after c*0.1/n mm.
    p = W.slab_column(nz=60, mua=0.01, mus=0.0, ngates=1, dt=0.1)
    r = oracle_mod.run(p, 10, seed=1, nthreads=1)
    mua, n = float(p.media[1, 0]), float(p.media[1, 3])
    depth = C * p.dt / n
    assert r["counts"]["timeout"] == 10
    assert r["ledger"]["timeout"] / 10 == pytest.approx(math.exp(-mua * depth), rel=1e-12)
    t = r["tally"][0, :, 1, 1] / 10
    kl = int(depth)
    assert t[kl + 1:].sum() == 0 and t[kl] > 0
    assert t[kl] == pytest.approx(math.exp(-mua * kl) * -math.expm1(-mua * (depth - kl)) / mua,
                                  rel=1e-10)


@pytest.mark.parametrize("h,dt", [(0.5, 0.02), (2.0, 0.05)])
def test_normalised_kinds_at_other_voxel_sizes(oracle_mod, h, dt):
    """Fluence and fluence rate of a straight, non-scattering beam down a
    column of voxels of h mm, against the closed form.  Voxel k covers depths
    [k h, (k + 1) h) and the beam enters it with weight exp(-mua k h), so its
    track-length fluence per launched photon is the weight integrated over
    the voxel's depth divided by the voxel volume,
    exp(-mua k h) (1 - exp(-mua h)) / (mua h^3), booked in the gate of the
    entry time k h n / c; the rate divides that by the gate width.  And the
    absorbed fraction, sum of mua h^3 times the fluence, is the weight that
    did not leave the far end, 1 - exp(-mua nz h)."""
    nz = 40
    base = W.slab_column(nz=nz, mua=0.02, mus=0.0, ngates=30, dt=dt)
    p = base.replace(h=h, src_pos=(1.5 * h, 1.5 * h, 0.0), dt=dt)
    mua, n = float(p.media[1, 0]), float(p.media[1, 3])
    h, dt = p.h, p.dt   # the stored float32 values
    N = 50
    r = oracle_mod.run(p, N, seed=2, nthreads=1)
    k1 = oracle_mod.normalise(r["tally"], N, h, dt, 1)
    k2 = oracle_mod.normalise(r["tally"], N, h, dt, 2)
    assert np.array_equal(oracle_mod.normalise(r["tally"], N, h, dt, 0), r["tally"])
    expect = np.zeros_like(k1)
    for k in range(nz):
        gate = min(int(math.floor(k * h * n / C / dt)), p.ngates - 1)
        expect[gate, k, 1, 1] = math.exp(-mua * k * h) * -math.expm1(-mua * h) / (mua * h ** 3)
    assert np.allclose(k1, expect, rtol=1e-12, atol=0)
    assert np.allclose(k2, expect / dt, rtol=1e-12, atol=0)
    absorbed = float((k1.sum(axis=0) * mua * h ** 3).sum())
    assert absorbed == pytest.approx(-math.expm1(-mua * nz * h), rel=1e-12)
    assert r["ledger"]["escaped"] / N == pytest.approx(math.exp(-mua * nz * h), rel=1e-12)


def test_fresnel_round_trips(oracle_mod):
    # mus = 0, reflection on: the beam bounces between the end faces with
    # R0 = ((n-1)/(n+1))^2 per face.  Expected tally per voxel is the
    # geometric series of passes; the count of reflections at the far face is
    # Binomial(N, R0).
    p = W.slab_column(nz=60, mua=0.005, mus=0.0, n=1.37, reflect=True)
    mua, n = float(p.media[1, 0]), float(p.media[1, 3])
    N = 200000
    r = oracle_mod.run(p, N, seed=11, nthreads=8)
    R = ((n - 1) / (n + 1)) ** 2
    a = math.exp(-60 * mua)
    c = -math.expm1(-mua) / mua
    k = np.arange(60)
    series = 1 / (1 - (R * a) ** 2)
    expect = c * (np.exp(-mua * k) + R * a * np.exp(-mua * (59 - k))) * series
    got = r["tally"][0, :, 1, 1] / N
    sigma = math.sqrt(R * (1 - R) / N) * c
    assert np.all(np.abs(got - expect) < 5 * sigma + 1e-12)
    refl = r["counts"]["reflections"]
    assert abs(refl - N * R * (1 + R * a * a)) < 5 * math.sqrt(N * R)
    assert r["counts"]["tir"] == 0
    assert abs(energy_residual(p, r)) < 1e-12


# --------------------------------------------------------------- tiny grids

def tiny(labels, pos, d, mua=0.1, reflect=False, n=1.37, nout=1.0, dets=None, media=None):
    labels = np.asarray(labels, np.uint8)
    if media is None:
        media = np.array([(0, 0, 1, 1), (mua, 0.0, 0.0, n)], np.float32)
    d = np.asarray(d, float)
    d = d / np.linalg.norm(d)
    return W.Problem(labels=labels, media=media, src_pos=pos, src_dir=tuple(d), dt=50.0,
                     reflect=reflect, n_out=nout,
                     detectors=np.zeros((0, 4), np.float32) if dets is None else dets)


def c_of(mua, l):
    mua = float(np.float32(mua))
    return -math.expm1(-mua * l) / mua


def e_of(mua, l):
    return math.exp(-float(np.float32(mua)) * l)


def test_tiny_single_voxel_axis(oracle_mod):
    p = tiny([[[1]]], (0.5, 0.5, 0.5), (1, 0, 0))
    r = oracle_mod.run(p, 3, seed=1, nthreads=1)
    assert r["tally"][0, 0, 0, 0] / 3 == pytest.approx(c_of(0.1, 0.5), rel=1e-14)
    assert r["ledger"]["escaped"] / 3 == pytest.approx(e_of(0.1, 0.5), rel=1e-14)


def test_tiny_diagonal_two_voxels(oracle_mod):
    # 2x1x1 grid, start (0.5, 0.25, 0.5) mm, direction (1,1,0)/sqrt2: x face
    # after 0.5*sqrt2, then the y face after another 0.25*sqrt2 (escape).
    p = tiny([[[1, 1]]], (0.5, 0.25, 0.5), (1, 1, 0))
    r = oracle_mod.run(p, 2, seed=1, nthreads=1)
    vx, vy = p.src_dir[0], p.src_dir[1]   # float32 components, equal
    l0, l1 = 0.5 / vx, 0.25 / vy
    assert r["tally"][0, 0, 0, 0] / 2 == pytest.approx(c_of(0.1, l0), rel=1e-12)
    assert r["tally"][0, 0, 0, 1] / 2 == pytest.approx(e_of(0.1, l0) * c_of(0.1, l1),
                                                       rel=1e-12)
    assert r["counts"]["entries"] == 2 and r["counts"]["face_events"] == 4


def test_tiny_corner_tie_breaks_on_lowest_axis(oracle_mod):
    # From the centre of voxel (0,0) of a 2x2x1 grid along (1,1,0): x and y
    # faces tie; x is crossed first (into voxel (1,0)), then y with a zero
    # segment (into voxel (1,1)), which the photon then crosses fully.
    p = tiny([[[1, 1], [1, 1]]], (0.5, 0.5, 0.5), (1, 1, 0), mua=0.2)
    r = oracle_mod.run(p, 1, seed=1, nthreads=1, ndigest=1)
    l0 = 0.5 / p.src_dir[0]
    t = r["tally"][0, 0]
    assert t[0, 0] == pytest.approx(c_of(0.2, l0), rel=1e-12)
    assert t[0, 1] == 0.0     # zero-length segment in (1,0)
    assert t[1, 0] == 0.0
    assert t[1, 1] == pytest.approx(e_of(0.2, l0) * c_of(0.2, 2 * l0), rel=1e-12)
    assert r["digest"][0][3] == 3  # ends in voxel (1,1): 1 + 2*1


def test_label_zero_inside_grid_is_outside(oracle_mod):
    p = tiny([[[1, 0, 1]]], (0.5, 0.5, 0.5), (1, 0, 0))
    r = oracle_mod.run(p, 4, seed=1, nthreads=1)
    t = r["tally"][0, 0, 0]
    assert t[0] > 0 and t[1] == 0 and t[2] == 0
    assert r["counts"]["escaped"] == 4


def test_total_internal_reflection_on_grazing_exit(oracle_mod):
    # Leaving n = 1.37 for air at 60 degrees from the normal is beyond the
    # 46.9 degree critical angle: reflected without a draw, every time.
    ang = math.radians(60)
    p = tiny([[[1, 1, 1, 1]]], (0.5, 0.5, 0.5), (math.sin(ang), 0, math.cos(ang)),
             reflect=True)
    r = oracle_mod.run(p, 5, seed=1, nthreads=1, ndigest=5)
    assert r["counts"]["tir"] >= 5 and r["counts"]["fresnel_draws"] >= 5
    assert abs(energy_residual(p, r)) < 1e-13


def test_refraction_bends_by_snell(oracle_mod):
    # Two media with n 1.0 -> 1.5, mus = 0: the transmitted photons continue
    # at sin(t) = sin(i)/1.5; the exit point on the far face shows the angle.
    media = np.array([(0, 0, 1, 1), (0.0, 0.0, 0.0, 1.0), (0.0, 0.0, 0.0, 1.5)], np.float32)
    labels = np.ones((2, 1, 8), np.uint8)
    labels[1] = 2
    i = math.radians(30)
    p = tiny(labels, (0.5, 0.5, 0.5), (math.sin(i), 0, math.cos(i)), reflect=True, media=media,
             nout=1.0)
    p = p.replace(detectors=np.zeros((0, 4), np.float32))
    r = oracle_mod.run(p, 4000, seed=2, nthreads=2, ndigest=4000)
    vx, vz = p.src_dir[0], p.src_dir[2]          # float32 sin(i), cos(i)
    st = vx / 1.5                                # Snell: sin(t) = sin(i) n1/n2
    ct = math.sqrt(1 - st * st)
    # transmitted photons cross the z=1 interface at x = 0.5 + 0.5 tan(i), then
    # travel 1 mm in z inside medium 2, exiting the top at x1:
    x1 = 0.5 + 0.5 * vx / vz + st / ct
    ends = r["digest"]
    # exit time of the transmitted, unreflected photons: 0.5/cos(i) mm at
    # n = 1 plus 1/cos(t) mm at n = 1.5
    t_exit = (0.5 / vz * 1.0 + 1.0 / ct * 1.5) / C
    direct = np.isclose(ends[:, 5], t_exit, rtol=1e-12, atol=0)
    # about (1-R)^2 of them; R ~ 0.04 per interface at 30 degrees
    assert direct.sum() > 3400
    assert np.all(ends[direct, 3] == int(x1) + 8)  # voxel (int(x1), 0, 1)


# ---------------------------------------------------------- energy identity

@pytest.mark.parametrize("case", ["c1", "c2", "rand0", "rand1", "rand2", "roulette"])
def test_energy_identity(oracle_mod, case):
    if case == "c1":
        p, N = W.cube_homogeneous(), 3000
    elif case == "c2":
        p, N = W.cube_sphere(sphere_n=1.0), 2000
    elif case == "roulette":
        p = W.cube_homogeneous(n=20)
        p = W.with_medium(p, 1, (0.1, 2.0, 0.5, 1.37)).replace(rr_threshold=0.3, reflect=True)
        N = 3000
    else:
        p, N = W.random_small(int(case[-1])), 3000
    r = oracle_mod.run(p, N, seed=3, nthreads=4)
    assert r["counts"]["launched"] == N
    c = r["counts"]
    assert c["escaped"] + c["timeout"] + c["rr_dead"] + c["capped"] == N
    assert abs(energy_residual(p, r)) < 1e-12
    # the ledger's own absorbed sum agrees with the grid
    mua = np.asarray(p.media, np.float64)[:, 0][p.labels]
    assert r["ledger"]["absorbed"] == pytest.approx(float((r["tally"].sum(0) * mua).sum()),
                                                    rel=1e-11, abs=1e-12)
    if case == "roulette":
        assert c["rr_tests"] > 0 and c["rr_survived"] > 0 and c["rr_dead"] > 0


# -------------------------------------------------------------- invariants

def test_prefix_and_split_runs(oracle_mod):
    p = W.cube_sphere(sphere_n=1.0, ngates=5, dt=1.0)
    a = oracle_mod.run(p, 2000, seed=9, nthreads=4)
    b1 = oracle_mod.run(p, 1000, seed=9, first=0, nthreads=3)
    b2 = oracle_mod.run(p, 1000, seed=9, first=1000, nthreads=1)
    assert np.allclose(a["tally"], b1["tally"] + b2["tally"], rtol=1e-12, atol=1e-15)
    for k in ["scatters", "face_events", "fresnel_draws", "escaped", "detected"]:
        assert a["counts"][k] == b1["counts"][k] + b2["counts"][k]
    # photon-index-keyed random numbers: the first 1000 are the same photons
    assert np.array_equal(np.sort(a["record_photon"][a["record_photon"] < 1000]),
                          np.sort(b1["record_photon"]))


def test_thread_count_does_not_change_results(oracle_mod):
    p = W.cube_homogeneous()
    a = oracle_mod.run(p, 1500, seed=4, nthreads=1)
    b = oracle_mod.run(p, 1500, seed=4, nthreads=7)
    assert np.allclose(a["tally"], b["tally"], rtol=1e-12, atol=1e-15)
    assert a["counts"] == b["counts"]


def test_seed_changes_results(oracle_mod):
    p = W.cube_homogeneous()
    a = oracle_mod.run(p, 500, seed=1, nthreads=2)
    b = oracle_mod.run(p, 500, seed=2, nthreads=2)
    assert a["counts"]["scatters"] != b["counts"]["scatters"]


def test_trajectories_do_not_depend_on_absorption(oracle_mod):
    # Free paths are drawn in scattering depth only, so changing mua (with
    # roulette off) leaves every path unchanged; detected weights are then
    # exp(-sum_i mua_i L_i) and exit times sum_i L_i n_i / c.
    base = W.cube_sphere(sphere_n=1.0, ngates=1, dt=5.0).replace(rr_threshold=0.0)
    other = W.with_medium(W.with_medium(base, 1, (0.02, 1.0, 0.01, 1.37)), 2,
                          (0.0, 5.0, 0.9, 1.0))
    N = 20000
    a = oracle_mod.run(base, N, seed=21, nthreads=8)
    b = oracle_mod.run(other, N, seed=21, nthreads=8)
    for k in ["scatters", "face_events", "fresnel_draws", "detected", "escaped", "timeout"]:
        assert a["counts"][k] == b["counts"][k]
    assert a["det_total"] > 10
    assert np.array_equal(a["record_photon"], b["record_photon"])
    assert np.array_equal(a["records"][:, 4:], b["records"][:, 4:])
    for p, r in [(base, a), (other, b)]:
        rec = r["records"].astype(np.float64)
        mua = np.asarray(p.media, np.float64)[1:, 0]
        nn = np.asarray(p.media, np.float64)[1:, 3]
        L = rec[:, 4:]
        assert np.allclose(rec[:, 2], np.exp(-(L * mua).sum(1)), rtol=2e-6)
        assert np.allclose(rec[:, 3], (L * nn).sum(1) / C, rtol=2e-6)
    # detectors: +-x pair at 10 mm, +-y pair at 20 mm; exit points within r
    ids = a["records"][:, 0].astype(int)
    assert set(ids) <= {0, 1, 2, 3}
    assert (ids <= 1).sum() > (ids >= 2).sum()


def test_detector_capture_geometry(oracle_mod):
    # mus = 0 photon leaving the far face at (1.5, 1.5, 3): caught by a disk
    # centred there, missed by one 1.01 mm away with r = 1.
    labels = np.ones((3, 3, 3), np.uint8)
    dets = np.array([(1.5 + 1.01, 1.5, 3.0, 1.0), (1.5, 1.5 + 0.99, 3.0, 1.0),
                     (1.5, 1.5, 3.0, 0.5)], np.float32)
    p = tiny(labels, (1.5, 1.5, 0.0), (0, 0, 1), mua=0.05, dets=dets)
    r = oracle_mod.run(p, 6, seed=1, nthreads=1)
    assert r["det_total"] == 6
    rec = r["records"]
    assert np.all(rec[:, 0] == 1)     # first detector in index order that contains the point
    assert np.all(rec[:, 1] == 0)
    assert np.allclose(rec[:, 2], e_of(0.05, 3.0), rtol=1e-6)
    assert np.allclose(rec[:, 4], 3.0, rtol=1e-7)


def test_roulette_is_unbiased(oracle_mod):
    # Same medium with and without roulette: the absorbed fraction agrees
    # within its batch-estimated noise.
    base = W.with_medium(W.cube_homogeneous(n=16), 1, (0.15, 3.0, 0.6, 1.37))
    base = base.replace(dt=50.0)
    rr = base.replace(rr_threshold=0.2)
    off = base.replace(rr_threshold=0.0)
    fr, fo = [], []
    for s in range(10):
        a = oracle_mod.run(rr, 3000, seed=100 + s, nthreads=8)
        b = oracle_mod.run(off, 3000, seed=200 + s, nthreads=8)
        fr.append(a["ledger"]["absorbed"] / 3000)
        fo.append(b["ledger"]["absorbed"] / 3000)
        assert a["counts"]["rr_tests"] > 0 and b["counts"]["rr_tests"] == 0
    fr, fo = np.array(fr), np.array(fo)
    se = math.sqrt(fr.var(ddof=1) / 10 + fo.var(ddof=1) / 10)
    assert abs(fr.mean() - fo.mean()) < 4 * se


def test_xy_symmetry_of_cube(oracle_mod):
    # The homogeneous cube and the beam at (29.5, 29.5) are symmetric under
    # x <-> y, so the tally's x and y moments agree within noise.
    p = W.cube_homogeneous()
    mx, my = [], []
    for s in range(8):
        r = oracle_mod.run(p, 2500, seed=50 + s, nthreads=8)
        t = r["tally"][0]
        tot = t.sum()
        x = np.arange(60) + 0.5
        mx.append(((t.sum((0, 1)) * (x - 30) ** 2).sum() / tot))
        my.append(((t.sum((0, 2)) * (x - 30) ** 2).sum() / tot))
    mx, my = np.array(mx), np.array(my)
    d = mx - my
    assert abs(d.mean()) < 4 * d.std(ddof=1) / math.sqrt(len(d)) + 1e-12


def test_visit_counter_counts_runs_of_one_photons_deposits(oracle_mod):
    """Pins of the oracle's per-cell visit counter (a visit = a maximal run
    of one photon's consecutive deposits into one cell): a straight column
    visits every cell once per photon; a photon scattering inside a single
    voxel until it escapes leaves one visit however many segments it
    deposits; and visits never exceed deposits."""
    N = 500
    p = W.slab_column(nz=20, mua=0.01, mus=0.0)
    r = oracle_mod.run(p, N, 1, nthreads=2, deposits=True, visits=True)
    on_axis = r["visits"][0, :, 1, 1]
    assert np.all(on_axis == N) and np.array_equal(r["visits"], r["deposits"])
    q = W.cube_homogeneous(n=1).replace(src_pos=(0.5, 0.5, 0.0), reflect=True,
                                        media=np.array([[0, 0, 1, 1], [0.01, 3.0, 0.5, 1.37]],
                                                       np.float32))
    r = oracle_mod.run(q, N, 2, nthreads=2, deposits=True, visits=True)
    assert r["visits"].sum() == N and r["deposits"].sum() > 3 * N
    c = W.cube_homogeneous(n=12).replace(src_pos=(5.5, 5.5, 0.0))
    r = oracle_mod.run(c, 2000, 3, nthreads=2, deposits=True, visits=True)
    assert np.all(r["visits"] <= r["deposits"]) and r["visits"].sum() < r["deposits"].sum()
