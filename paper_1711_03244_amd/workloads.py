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
import functools
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
    cx, cy, cz = centre
    dx2 = (((np.arange(nx) + 0.5) * h - cx) ** 2)[None, None, :]
    dy2 = (((np.arange(ny) + 0.5) * h - cy) ** 2)[None, :, None]
    dz2 = (((np.arange(nz) + 0.5) * h - cz) ** 2)[:, None, None]
    return dx2 + dy2 + dz2 <= radius ** 2


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


# ------------------------------------------------------------------ head

HEAD_SHAPE = (181, 217, 181)                 # (nz, ny, nx) voxels of 1 mm
HEAD_TISSUES = ("scalp", "skull", "csf", "gray", "white")
HEAD_MEDIA = ((0.019, 7.8, 0.89, 1.37), (0.019, 7.8, 0.89, 1.37), (0.004, 0.009, 0.89, 1.37),
              (0.02, 9.0, 0.89, 1.37), (0.08, 40.9, 0.84, 1.37))
HEAD_SEMI_AXES = (75.0, 95.0, 80.0)          # outer scalp surface, mm (x, y, z)
HEAD_DEPTHS = (0.0, 5.0, 12.0, 14.0, 18.0)   # outer boundary of each shell below the scalp, mm


def _angle_field(rng, amp: float, lmax: int = 3):
    """Seeded smooth function of direction (polar t, azimuth f) with
    |value| <= amp: a sum of low-order cosine products."""
    terms = []
    for l in range(1, lmax + 1):
        for m in range(0, lmax + 1):
            terms.append((l, m, rng.normal(), rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)))
    norm = sum(abs(a) for _, _, a, _, _ in terms)
    cache = {}

    def f(t, ph):
        # the azimuth factors are reused across calls on the same grid
        key = id(ph)
        if key not in cache:
            cache.clear()
            cache[key] = (ph, [a * np.cos(m * ph + c) for _, m, a, _, c in terms])
        phis = cache[key][1]
        out = np.zeros(np.broadcast(t, ph).shape)
        for (l, _, _, b, _), cp in zip(terms, phis):
            out += np.cos(l * t + b) * cp
        return out * (amp / norm)
    return f


@functools.lru_cache(maxsize=4)
def head_phantom(seed: int = 1) -> Problem:
    """Synthetic layered head: five nested ellipsoidal shells (scalp, skull,
    CSF, gray, white matter) centred in a 181 x 217 x 181 grid of 1 mm
    voxels, each boundary scaled along every direction by 1 + a seeded
    low-order perturbation (a shared field up to 4% plus a per-shell field up
    to 1%, nesting kept with >= 1 mm between boundaries).  Pencil beam along
    the inward normal of the perturbed scalp surface at a seeded point on the
    upper half; it starts where that ray first enters a tissue voxel.  Ten
    0.5 ns gates, Fresnel boundaries on."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = HEAD_SHAPE
    centre = np.array([nx / 2, ny / 2, nz / 2])
    shared = _angle_field(rng, 0.04)
    own = [_angle_field(rng, 0.01) for _ in HEAD_DEPTHS]
    semi = np.array(HEAD_SEMI_AXES)

    def boundary_radius(k, t, ph):
        """Radius scale of boundary k along a direction (1 = unperturbed)."""
        return 1.0 + shared(t, ph) + own[k](t, ph)

    def level(k, pts):
        """< 1 inside boundary k, for points (..., 3) in mm."""
        d = pts - centre
        a = semi - HEAD_DEPTHS[k]
        rho = np.sqrt(((d / a) ** 2).sum(-1))
        r = np.sqrt((d ** 2).sum(-1))
        t = np.arccos(np.clip(d[..., 2] / np.maximum(r, 1e-9), -1, 1))
        ph = np.arctan2(d[..., 1], d[..., 0])
        return rho / boundary_radius(k, t, ph)

    labels = np.zeros(HEAD_SHAPE, np.uint8)
    Y, X = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    dx, dy = X - centre[0], Y - centre[1]
    ph = np.arctan2(dy, dx)
    for iz in range(nz):
        dz = iz + 0.5 - centre[2]
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        t = np.arccos(np.clip(dz / np.maximum(r, 1e-9), -1, 1))
        common = 1.0 + shared(t, ph)
        lab = np.zeros((ny, nx), np.uint8)
        for k in range(len(HEAD_DEPTHS)):
            a = semi - HEAD_DEPTHS[k]
            rho = np.sqrt((dx / a[0]) ** 2 + (dy / a[1]) ** 2 + (dz / a[2]) ** 2)
            lab[rho <= common + own[k](t, ph)] = k + 1
        labels[iz] = lab
    # nesting: along any ray from the centre the labels never increase outward
    # (each inner boundary lies >= 1 mm inside the one before it by
    # construction: depths differ by >= 2 mm and perturbations by <= 1% each)

    # source: seeded direction in the upper half, surface point, inward normal
    t0 = rng.uniform(np.radians(15), np.radians(60))
    f0 = rng.uniform(0, 2 * np.pi)
    u = np.array([np.sin(t0) * np.cos(f0), np.sin(t0) * np.sin(f0), np.cos(t0)])
    lo, hi = 0.0, 2.0 * semi.max()
    for _ in range(60):  # bisection on the outer level function along the ray
        mid = 0.5 * (lo + hi)
        if level(0, centre + mid * u) <= 1.0:
            lo = mid
        else:
            hi = mid
    surf = centre + lo * u
    eps = 1e-3
    grad = np.array([(level(0, surf + eps * e) - level(0, surf - eps * e)) / (2 * eps)
                     for e in np.eye(3)])
    normal = grad / np.linalg.norm(grad)
    d = (-normal).astype(np.float32)
    d = (d / np.float32(np.sqrt((d.astype(np.float64) ** 2).sum()))).astype(np.float32)
    # march in from outside until the first tissue voxel
    pos = surf + 4.0 * normal
    step = 1e-3
    for _ in range(20000):
        i, j, k = (int(np.floor(c)) for c in pos)
        if 0 <= i < nx and 0 <= j < ny and 0 <= k < nz and labels[k, j, i] != 0:
            break
        pos = pos + step * d.astype(np.float64)
    pos32 = tuple(float(np.float32(c)) for c in pos)
    i, j, k = (int(np.floor(c)) for c in pos32)
    if labels[k, j, i] == 0:
        raise RuntimeError("head source does not start in tissue")
    return Problem(labels=labels, media=_media(*HEAD_MEDIA), src_pos=pos32, src_dir=tuple(d),
                   t0=0.0, dt=0.5, ngates=10, reflect=True, name=f"head_{seed}")


# ------------------------------------------------------------------ batch

BATCH_SIDES = (32, 48, 64, 96, 128)
BATCH_MUA = (0.001, 0.05)       # 1/mm, log-uniform
BATCH_MUS = (0.5, 20.0)         # 1/mm, log-uniform
BATCH_G = (0.5, 0.95)           # uniform
BATCH_PHOTONS = (1e5, 1e7)      # log-uniform


@dataclasses.dataclass
class BatchItem:
    problem: Problem
    nphoton: int
    seed: int


def _log_uniform(rng, lo, hi):
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


def batch_cube(rng, side: int, name: str = "") -> Problem:
    """One cube of the batched workload: `side`^3 voxels of 1 mm, label 1
    background with 1-3 spherical inclusions (labels 2..4, radius uniform in
    [side/10, side/4], centre uniform where the sphere fits, later ones
    painted over earlier ones), every label's mua / mus log-uniform and g
    uniform in the batch ranges, n = 1.37, pencil beam along +z at the
    voxel-centred middle of the z = 0 face, one 0-5 ns gate, Fresnel
    boundaries on."""
    labels = np.ones((side, side, side), np.uint8)
    ninc = int(rng.integers(1, 4))
    for k in range(ninc):
        r = float(rng.uniform(side / 10, side / 4))
        c = tuple(float(rng.uniform(r, side - r)) for _ in range(3))
        labels[sphere_mask(labels.shape, c, r)] = 2 + k
    rows = [(_log_uniform(rng, *BATCH_MUA), _log_uniform(rng, *BATCH_MUS),
             float(rng.uniform(*BATCH_G)), 1.37) for _ in range(1 + ninc)]
    c = side / 2 - 0.5
    return Problem(labels=labels, media=_media(*rows), src_pos=(c, c, 0.0),
                   src_dir=(0.0, 0.0, 1.0), t0=0.0, dt=5.0, ngates=1, reflect=True,
                   name=name or f"batch_cube{side}")


def batch_workload(nsims: int = 256, seed: int = 1, sides=BATCH_SIDES,
                   photons=BATCH_PHOTONS, scale: float = 1.0) -> list:
    """The batched workload: `nsims` independent cubes (`batch_cube`) with
    sides drawn uniformly from `sides` and photon counts log-uniform in
    `photons` (times `scale`, at least 1), each with its own seed, all drawn
    from one numpy PCG64 stream seeded with `seed`."""
    rng = np.random.default_rng(seed)
    items = []
    for i in range(nsims):
        side = int(rng.choice(np.asarray(sides)))
        prob = batch_cube(rng, side, name=f"batch{seed}_{i}_cube{side}")
        n = max(1, int(round(_log_uniform(rng, *photons) * scale)))
        items.append(BatchItem(prob, n, int(rng.integers(1, 2 ** 32))))
    return items


# ------------------------------------------------------------------ denoiser

DENOISER_CHANNELS = (32, 64, 128, 256)


def denoiser_layer_shapes(channels=DENOISER_CHANNELS) -> list:
    """(kind, taps, cin, cout) of the denoiser's layers in forward order:
    input conv, level-0 conv, then per deeper level a stride-2 down conv and
    a conv, one more conv at the bottom, then per level back up a stride-2
    transposed conv and a conv, and the one-channel output conv."""
    c = list(channels)
    out = [("conv3", 27, 1, c[0]), ("conv3", 27, c[0], c[0])]
    for l in range(1, len(c)):
        out += [("down", 8, c[l - 1], c[l]), ("conv3", 27, c[l], c[l])]
    out.append(("conv3", 27, c[-1], c[-1]))
    for l in range(len(c) - 2, -1, -1):
        out += [("up", 8, c[l + 1], c[l]), ("conv3", 27, c[l], c[l])]
    out.append(("conv3", 27, c[0], 1))
    return out


def denoiser_weights(channels=DENOISER_CHANNELS, seed: int = 1, zero_output: bool = True,
                     bias_scale: float = 0.0) -> list:
    """Seeded initial weights: He-normal (std sqrt(2 / (taps * cin))) float32
    weights [taps][cin][cout] and biases (zero, or normal with std
    `bias_scale`), in forward layer order, from numpy PCG64 `seed`.  With
    `zero_output` the output layer starts at zero, so an untrained network
    returns its input."""
    rng = np.random.default_rng(seed)
    shapes = denoiser_layer_shapes(channels)
    out = []
    for i, (kind, taps, ci, co) in enumerate(shapes):
        w = rng.normal(0.0, np.sqrt(2.0 / (taps * ci)), size=(taps, ci, co)).astype(np.float32)
        b = (rng.normal(0.0, bias_scale, size=co) if bias_scale else np.zeros(co)).astype(np.float32)
        if zero_output and i == len(shapes) - 1:
            w[...] = 0.0
            b[...] = 0.0
        out.append((w, b))
    return out


def denoiser_volume(seed: int, side: int = 64) -> Problem:
    """One volume of the denoiser's data set: `side`^3 voxels of 1 mm, label 1
    background with 1-5 randomly oriented ellipsoidal inclusions (labels
    2..6, semi-axes uniform in [side/10, side/4], centres uniform where the
    largest semi-axis fits, later ones painted over earlier ones), every
    label's mua / mus log-uniform and g uniform in the batched workload's
    ranges, n = 1.37; pencil beam along +z at the voxel-centred middle of the
    z = 0 face, one 0-5 ns gate, Fresnel boundaries on.  numpy PCG64 `seed`."""
    rng = np.random.default_rng(seed)
    labels = np.ones((side, side, side), np.uint8)
    ninc = int(rng.integers(1, 6))
    c1 = np.arange(side) + 0.5
    z, y, x = np.meshgrid(c1, c1, c1, indexing="ij")
    pts = np.stack([x, y, z], axis=-1)
    for k in range(ninc):
        axes = rng.uniform(side / 10, side / 4, size=3)
        rmax = float(axes.max())
        centre = rng.uniform(rmax, side - rmax, size=3)
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        d = (pts - centre) @ q          # coordinates along the ellipsoid's axes
        labels[((d / axes) ** 2).sum(-1) <= 1.0] = 2 + k
    rows = [(_log_uniform(rng, *BATCH_MUA), _log_uniform(rng, *BATCH_MUS),
             float(rng.uniform(*BATCH_G)), 1.37) for _ in range(1 + ninc)]
    c = side / 2 - 0.5
    return Problem(labels=labels, media=_media(*rows), src_pos=(c, c, 0.0),
                   src_dir=(0.0, 0.0, 1.0), t0=0.0, dt=5.0, ngates=1, reflect=True,
                   name=f"denoise_{seed}")


def with_medium(p: Problem, row: int, values) -> Problem:
    media = p.media.copy()
    media[row] = values
    return p.replace(media=media)


def photons_and_seed(name: str) -> tuple:
    """Photon count and seed each named workload is quoted at."""
    return {"cube60_homogeneous": (100_000, 1), "cube60_sphere": (100_000_000, 1),
            "head_1": (100_000_000, 1)}[name]


def describe(p: Problem, nphoton: Optional[int] = None) -> dict:
    nz, ny, nx = p.shape
    d = {"workload": p.name, "grid": [nx, ny, nz], "voxel_mm": p.h, "nmedia": p.nmedia - 1,
         "ngates": p.ngates, "gate_ns": p.dt, "ndet": p.ndet, "reflect": bool(p.reflect)}
    if nphoton is not None:
        d["photons"] = int(nphoton)
    return d
