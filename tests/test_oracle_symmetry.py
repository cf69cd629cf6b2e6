"""Symmetry of the transport under the x-y symmetries of a volume, the fact
behind the denoiser's training augmentation (a symmetry applied to an
(input, target) pair of fluence maps gives the pair of the transformed
volume with the source moved to match).

The oracle runs a random two-medium volume and its image under a mirror in
x and under the x <-> y transpose, each with the source at the image of the
original position.  Trajectories are not mapped one to one (the random
draws act in a basis the symmetry does not preserve), so the comparison is
statistical: each side is R independent seeded runs, whose spread gives
the standard error of the absorbed fraction, of the absorption per
z-layer and of the absorption map summed over z.  The maps must agree
pixel by pixel in aggregate (mean squared z-score near 1), and the same
statistic must reject the untransformed map, so the check has power.
"""
import numpy as np
import pytest

import oracle
from paper_1711_03244_amd import workloads as W

R, N = 8, 4000                     # runs per side, photons per run
NX = 12


def problem(labels, sx, sy):
    media = W._media((0.02, 1.0, 0.8, 1.37), (0.1, 5.0, 0.6, 1.45))
    return W.Problem(labels=labels, media=media, src_pos=(sx, sy, 0.0), src_dir=(0.0, 0.0, 1.0),
                     t0=0.0, dt=1.0, ngates=2, reflect=True)


def absorption(p, seed0):
    """Per run: absorbed fraction, absorption per z-layer, absorption map
    over (y, x) summed over z, all per launched photon."""
    mua = np.asarray(p.media, np.float64)[:, 0][p.labels]
    tot, layers, maps = [], [], []
    for k in range(R):
        r = oracle.run(p, N, seed0 + k, nthreads=8)
        a = r["tally"].sum(0) * mua / N          # [z][y][x]
        tot.append(r["ledger"]["absorbed"] / N)
        layers.append(a.sum(axis=(1, 2)))
        maps.append(a.sum(axis=0))
    return np.array(tot), np.array(layers), np.array(maps)


def mean_se(v):
    return v.mean(0), v.std(0, ddof=1) / np.sqrt(len(v))


def z2(a, b, keep):
    (ma, sa), (mb, sb) = mean_se(a), mean_se(b)
    return float(np.mean(((ma - mb)[keep] / np.hypot(sa, sb)[keep]) ** 2))


@pytest.mark.parametrize("sym", ["mirror_x", "transpose_xy"])
def test_symmetric_volume_gives_the_symmetric_absorption(sym):
    rng = np.random.default_rng(5)
    labels = np.where(rng.random((8, NX, NX)) < 0.3, 2, 1).astype(np.uint8)
    sx, sy = 3.5, 5.5                              # off the centre lines
    if sym == "mirror_x":
        img_labels, img_src = labels[:, :, ::-1], (NX - sx, sy)
        img_map = lambda m: m[..., ::-1]           # noqa: E731
    else:
        img_labels, img_src = labels.transpose(0, 2, 1), (sy, sx)
        img_map = lambda m: np.swapaxes(m, -1, -2)  # noqa: E731
    p = problem(labels, sx, sy)
    q = problem(np.ascontiguousarray(img_labels), *img_src)
    ta, la, ma = absorption(p, 100)
    tb, lb, mb = absorption(q, 200)
    (mta, sta), (mtb, stb) = mean_se(ta), mean_se(tb)
    assert abs(mta - mtb) <= 4 * np.hypot(sta, stb), (mta, mtb, sta, stb)
    assert 0.05 < mta < 0.95                       # a non-trivial split of the weight
    layer = la.mean(0) > 0.02 * la.mean(0).max()
    assert z2(la, lb, layer) < 3.0
    dense = ma.mean(0) > 0.05 * ma.mean(0).max()
    assert dense.sum() >= 20
    assert z2(img_map(ma), mb, dense) < 3.0
    # the statistic sees the difference when the map is not transformed
    assert z2(ma, mb, dense) > 20.0
