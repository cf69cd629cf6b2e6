"""The seeded input generators: determinism and the structure each workload
promises (label ranges, nesting, source placement, geometry)."""
import hashlib

import numpy as np
import pytest

from paper_1711_03244_amd import workloads as W


@pytest.fixture(scope="module")
def head():
    return W.head_phantom(1)


def test_head_is_deterministic(head):
    again = W.head_phantom.__wrapped__(1)
    assert np.array_equal(again.labels, head.labels)
    assert again.src_pos == head.src_pos and again.src_dir == head.src_dir
    other = W.head_phantom.__wrapped__(2)
    assert not np.array_equal(other.labels, head.labels)


def test_head_layout(head):
    assert head.labels.shape == (181, 217, 181)
    assert head.labels.max() == 5 and head.nmedia == 6
    counts = np.bincount(head.labels.ravel(), minlength=6)
    assert all(c > 50_000 for c in counts[1:])
    assert np.allclose(head.media[1:], np.array(W.HEAD_MEDIA, np.float32))
    assert head.ngates == 10 and head.dt == 0.5 and head.reflect


def test_head_shells_are_nested(head):
    # walking outward from the centre along any ray, labels never increase
    rng = np.random.default_rng(0)
    nz, ny, nx = head.labels.shape
    c = np.array([nx / 2, ny / 2, nz / 2])
    for _ in range(60):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        prev = 5
        for r in np.arange(0, 130, 0.25):
            x = c + r * u
            i, j, k = (int(np.floor(v)) for v in x)
            if not (0 <= i < nx and 0 <= j < ny and 0 <= k < nz):
                break
            lab = int(head.labels[k, j, i])
            assert lab <= prev
            prev = lab
        assert prev == 0


def test_head_source_enters_scalp_along_inward_normal(head):
    i, j, k = (int(np.floor(v)) for v in head.src_pos)
    assert head.labels[k, j, i] == 1
    d = np.array(head.src_dir)
    assert abs(np.linalg.norm(d) - 1) < 1e-6
    nz, ny, nx = head.labels.shape
    centre = np.array([nx / 2, ny / 2, nz / 2])
    assert d @ (centre - np.array(head.src_pos)) > 0
    # one voxel back along the beam is outside
    x = np.array(head.src_pos) - 1.0 * d
    i, j, k = (int(np.floor(v)) for v in x)
    assert head.labels[k, j, i] == 0
    # the scalp then skull are crossed within ~20 mm along the beam
    seen = []
    for r in np.arange(0, 25, 0.2):
        x = np.array(head.src_pos) + r * d
        i, j, k = (int(np.floor(v)) for v in x)
        seen.append(int(head.labels[k, j, i]))
    assert 2 in seen and 3 in seen


def test_cube_workloads():
    p = W.cube_homogeneous()
    assert p.labels.shape == (60, 60, 60) and (p.labels == 1).all()
    assert p.src_pos == (29.5, 29.5, 0.0) and not p.reflect
    q = W.cube_sphere()
    assert (q.labels == 2).sum() == int(W.sphere_mask((60, 60, 60), (30, 30, 30), 15).sum())
    assert q.ndet == 4 and q.ngates == 50 and q.reflect
    d = np.hypot(q.detectors[:, 0] - 29.5, q.detectors[:, 1] - 29.5)
    assert np.allclose(sorted(d), [10, 10, 20, 20])


def test_random_small_is_seeded():
    a, b = W.random_small(3), W.random_small(3)
    assert np.array_equal(a.labels, b.labels) and a.src_pos == b.src_pos
    i, j, k = (int(np.floor(v)) for v in a.src_pos)
    assert a.labels[k, j, i] != 0


def test_batch_workload_recipe():
    items = W.batch_workload()
    assert len(items) == 256
    sides = {it.problem.shape[0] for it in items}
    assert sides == set(W.BATCH_SIDES)
    n = np.array([it.nphoton for it in items])
    assert n.min() >= 1e5 and n.max() <= 1e7
    assert 4.5e8 < n.sum() < 6.5e8            # mean of log-uniform [1e5, 1e7] ~ 2.15e6 each
    for it in items[:40]:
        p = it.problem
        s = p.shape[0]
        assert p.shape == (s, s, s) and p.reflect and p.ngates == 1 and p.dt == 5.0
        assert p.src_pos == (s / 2 - 0.5, s / 2 - 0.5, 0.0)
        k = p.nmedia - 2                         # inclusions
        assert 1 <= k <= 3 and set(np.unique(p.labels)) <= set(range(1, 2 + k))
        mua, mus, g, nn = p.media[1:].T
        assert (mua >= 0.001 - 1e-9).all() and (mua <= 0.05 + 1e-9).all()
        assert (mus >= 0.5 - 1e-6).all() and (mus <= 20 + 1e-5).all()
        assert (g >= 0.5).all() and (g <= 0.95).all() and (nn == np.float32(1.37)).all()
    # seeded and independent of other draws
    again = W.batch_workload(nsims=3)
    for a, b in zip(items[:3], again):
        assert np.array_equal(a.problem.labels, b.problem.labels) and a.seed == b.seed


def test_denoiser_volume_recipe():
    a, b = W.denoiser_volume(5), W.denoiser_volume(5)
    assert np.array_equal(a.labels, b.labels) and np.array_equal(a.media, b.media)
    assert a.shape == (64, 64, 64) and a.src_pos == (31.5, 31.5, 0.0) and a.reflect
    counts = [W.denoiser_volume(s, 32).nmedia - 2 for s in range(1, 30)]
    assert min(counts) >= 1 and max(counts) <= 5 and len(set(counts)) >= 3
    assert not np.array_equal(W.denoiser_volume(6).labels, a.labels)
