"""Seeded synthetic inputs: voxel volumes, optical properties, sources, gates.

This module only builds inputs.  It holds none of the transport arithmetic;
the GPU library and the CPU checker each consume a :class:`Problem` through
their own code.

The cube workloads follow the paper's benchmark description (60 x 60 x 60 mm
domain, mua 0.005/mm, mus 1.0/mm, g 0.01, n 1.37, air outside, pencil beam
along +z; B2/B2a add a 15 mm sphere with Fresnel boundaries).  Coordinates
start at the grid corner, voxel (i, j, k) covers [i, i+1) * h along x, and
volumes are stored x-fastest as numpy arrays of shape (nz, ny, nx).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    """One simulation: domain, media table, source, detectors, time gates."""

    labels: np.ndarray                 # uint8 (nz, ny, nx), 0 = outside
    media: np.ndarray                  # float32 (nmedia, 4): mua, mus, g, n; row 0 = outside
    src_pos: tuple                     # mm from the grid corner
    src_dir: tuple                     # unit vector
    h: float = 1.0                     # voxel edge, mm
    detectors: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros((0, 4), np.float32))  # (ndet, 4): x, y, z, r (mm)
    t0: float = 0.0                    # ns
    dt: float = 5.0                    # ns
    ngates: int = 1
    reflect: bool = False
    n_out: float = 1.0
    rr_threshold: float = 1e-4
    rr_m: float = 10.0
    max_events: int = 10_000_000
    name: str = ""

    def __post_init__(self):
        self.labels = np.ascontiguousarray(self.labels, dtype=np.uint8)
        self.media = np.ascontiguousarray(self.media, dtype=np.float32)
        self.detectors = np.ascontiguousarray(
            np.asarray(self.detectors, dtype=np.float32).reshape(-1, 4))
        # Every scalar is stored as its float32 value so that both consumers
        # see bit-identical inputs.
        self.src_pos = tuple(float(np.float32(x)) for x in self.src_pos)
        self.src_dir = tuple(float(np.float32(x)) for x in self.src_dir)
        self.h = float(np.float32(self.h))
        self.t0 = float(np.float32(self.t0))
        self.dt = float(np.float32(self.dt))
        self.n_out = float(np.float32(self.n_out))
        self.rr_threshold = float(np.float32(self.rr_threshold))
        self.rr_m = float(np.float32(self.rr_m))

    @property
    def shape(self):
        return self.labels.shape  # (nz, ny, nx)

    @property
    def nvox(self) -> int:
        return int(self.labels.size)

    @property
    def nmedia(self) -> int:
        return int(self.media.shape[0])

    @property
    def ndet(self) -> int:
        return int(self.detectors.shape[0])

    @property
    def tally_shape(self):
        return (self.ngates,) + tuple(self.labels.shape)

    @property
    def record_len(self) -> int:
        return 4 + self.nmedia - 1

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ------------------------------------------------------------------ cubes

CUBE_MEDIUM = (0.005, 1.0, 0.01, 1.37)      # background of the paper's benchmarks
SPHERE_MEDIUM = (0.002, 5.0, 0.9, 1.37)     # inclusion; the paper's B2 uses n = 1.0


def _media(*rows) -> np.ndarray:
    return np.array([(0.0, 0.0, 1.0, 1.0)] + [tuple(r) for r in rows], np.float32)


def sphere_mask(shape, centre, radius, h=1.0) -> np.ndarray:
    """Voxels whose centre lies within `radius` (mm) of `centre` (mm)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                          (np.arange(nx) + 0.5) * h, indexing="ij")
    cx, cy, cz = centre
    return (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= radius ** 2


def cube_homogeneous(n: int = 60, nphoton: int = 100_000) -> Problem:
    """Homogeneous 60 mm cube, pencil beam at (29.5, 29.5, 0) along +z, one
    0-5 ns gate, photons end at the cube boundary (no reflection)."""
    labels = np.ones((n, n, n), np.uint8)
    return Problem(labels=labels, media=_media(CUBE_MEDIUM),
                   src_pos=(n / 2 - 0.5, n / 2 - 0.5, 0.0), src_dir=(0.0, 0.0, 1.0),
                   t0=0.0, dt=5.0, ngates=1, reflect=False, name="cube60_homogeneous")


def cube_sphere(n: int = 60, sphere_n: float = 1.37, ngates: int = 50, dt: float = 0.1,
                detectors: bool = True) -> Problem:
    """Heterogeneous 60 mm cube with a centred r = 15 mm sphere, Fresnel
    boundaries on, 50 gates of 0.1 ns, four r = 1 mm disk detectors on the
    z = 0 face at 10 mm (+x, -x) and 20 mm (+y, -y) from the source."""
    labels = np.ones((n, n, n), np.uint8)
    labels[sphere_mask(labels.shape, (n / 2, n / 2, n / 2), n / 4)] = 2
    sx, sy = n / 2 - 0.5, n / 2 - 0.5
    dets = np.array([(sx + 10, sy, 0, 1), (sx - 10, sy, 0, 1),
                     (sx, sy + 20, 0, 1), (sx, sy - 20, 0, 1)], np.float32)
    sphere = SPHERE_MEDIUM[:3] + (sphere_n,)
    return Problem(labels=labels, media=_media(CUBE_MEDIUM, sphere),
                   src_pos=(sx, sy, 0.0), src_dir=(0.0, 0.0, 1.0),
                   detectors=dets if detectors else np.zeros((0, 4), np.float32),
                   t0=0.0, dt=dt, ngates=ngates, reflect=True, name="cube60_sphere")


def slab_column(nz: int = 60, mua: float = 0.005, mus: float = 0.0, n: float = 1.37,
                reflect: bool = False, ngates: int = 1, dt: float = 5.0, nxy: int = 3) -> Problem:
    """Narrow column of one medium with a pencil beam down its axis; with
    mus = 0 every photon follows the same straight line."""
    labels = np.ones((nz, nxy, nxy), np.uint8)
    c = nxy / 2
    return Problem(labels=labels, media=_media((mua, mus, 0.0, n)),
                   src_pos=(c, c, 0.0), src_dir=(0.0, 0.0, 1.0),
                   t0=0.0, dt=dt, ngates=ngates, reflect=reflect, name="slab_column")


def random_small(seed: int, max_side: int = 12, nmedia: int = 4) -> Problem:
    """Small random heterogeneous volume with random media and a random
    interior pencil beam; for property tests and edge cases."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in rng.integers(2, max_side + 1, size=3))
    labels = rng.integers(1, nmedia, size=(nz, ny, nx)).astype(np.uint8)
    holes = rng.random((nz, ny, nx)) < 0.1
    labels[holes] = 0
    rows = []
    for _ in range(nmedia - 1):
        rows.append((10 ** rng.uniform(-3, -0.5), 10 ** rng.uniform(-1, 1.2),
                     rng.uniform(-0.5, 0.95), float(rng.choice([1.0, 1.33, 1.37, 1.5]))))
    i, j, k = (int(rng.integers(0, d)) for d in (nx, ny, nz))
    if labels[k, j, i] == 0:
        labels[k, j, i] = 1
    pos = (i + rng.uniform(0.05, 0.95), j + rng.uniform(0.05, 0.95), k + rng.uniform(0.05, 0.95))
    d = rng.normal(size=3)
    d = d / np.linalg.norm(d)
    d32 = d.astype(np.float32)
    d32 = d32 / np.float32(np.sqrt(np.sum(d32.astype(np.float64) ** 2)))
    return Problem(labels=labels, media=_media(*rows), src_pos=pos, src_dir=tuple(d32),
                   t0=0.0, dt=float(rng.uniform(0.2, 1.0)), ngates=int(rng.integers(1, 6)),
                   reflect=bool(rng.integers(0, 2)), name=f"random_small_{seed}")


def with_medium(p: Problem, row: int, values) -> Problem:
    media = p.media.copy()
    media[row] = values
    return p.replace(media=media)


def photons_and_seed(name: str) -> tuple:
    """Photon count and seed each named workload is quoted at."""
    return {"cube60_homogeneous": (100_000, 1), "cube60_sphere": (100_000_000, 1)}[name]


def describe(p: Problem, nphoton: Optional[int] = None) -> dict:
    nz, ny, nx = p.shape
    d = {"workload": p.name, "grid": [nx, ny, nz], "voxel_mm": p.h, "nmedia": p.nmedia - 1,
         "ngates": p.ngates, "gate_ns": p.dt, "ndet": p.ndet, "reflect": bool(p.reflect)}
    if nphoton is not None:
        d["photons"] = int(nphoton)
    return d
