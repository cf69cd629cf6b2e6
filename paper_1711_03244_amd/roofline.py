"""Algorithmic work model of the transport loop, for roofline fractions.

Counts the VALU lane-operations the method itself needs per event -- the
arithmetic of the formulas, not the instructions a compiler happens to emit
-- with full-rate FP32/integer operations (add, mul, fma, compare, select,
min/max, conversion, bit operation) as 1 slot, transcendental unit
operations (exp, log, sqrt, rcp, rsq, sin, cos) as 4 slots, and the 32x32->64
multiply Philox needs as 2 slots (the issue cost measured on gfx950 by the
microbenchmark: a Philox4x32-10 block costs 60 slots).  Multiplying by the
event counts a run reports gives the run's algorithmic work; divided by the
kernel time and by the chip's FP32 VALU lane rate it is the fraction of the
VALU roofline achieved.

Peak: 256 compute units x 64 FP32 lanes per clock x 2.4 GHz = 39.32e12
lane-operations per second (non-packed; packed FP32 is disabled in the build).
"""
import hashlib
import json
import os

CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
VALU_PEAK = CUS * LANES * CLOCK_HZ            # lane-op slots per second
ATOMIC_PEAK_F64 = 2.36e10                     # measured FP64 no-return atomics/s, distinct addresses

PHILOX_BLOCK = 10 * (2 * 2 + 2)                # 10 rounds: two 32x32->64 products, two 3-input xors
UNIFORM = 3                                    # shift, or, convert-and-scale

# every segment: 3 face distances (gap, clamp, scale, zero-velocity select:
# 5 each), argmin (4), scattering distance (2), time distance (3), event
# choice (5), gate index (6), deposit: mua*l, 1-exp (exp + 1), scale by w and
# 1/mua with the mua = 0 select (4), weight update (1), visit accumulation
# (2), move: 3 fma + 3 clamps, time, depth and its clamp (10), segment count (2)
SEGMENT = 15 + 4 + 2 + 3 + 5 + 6 + (1 + 4 + 1 + 4 + 1) + 2 + 10 + 2
# scattering: one Philox block and 3 uniforms; HG inverse CDF (13 incl. one
# rcp); sin(theta) (7 incl. sqrt); sin/cos of the azimuth (9); Duff et al.
# basis (15 incl. one rcp); rotation (12); renormalisation (10 incl. rsq);
# three h/|v| (21 incl. three rcp); new free path -ln u (5); roulette test (1)
SCATTER = PHILOX_BLOCK + 3 * UNIFORM + 13 + 7 + 9 + 15 + 12 + 10 + 21 + 5 + 1
# voxel face event: axis components (6), neighbour index and bounds (6),
# index comparison (2), face snap (2), entering the neighbour (3)
FACE = 6 + 6 + 2 + 2 + 3
# Fresnel test with a draw: n1/n2 (rcp + 1), sin^2 t (3), TIR test (1),
# cos t (sqrt + 2), reflectance (two rcp + 10), one Philox block + uniform,
# refraction or reflection update with new h/|v| (24)
FRESNEL = 5 + 3 + 1 + 6 + 18 + PHILOX_BLOCK + UNIFORM + 24
# photon launch: one Philox block, uniform, -ln u, state set-up (20)
LAUNCH = PHILOX_BLOCK + UNIFORM + 5 + 20


def algorithmic_ops(stats: dict) -> float:
    """Lane-op slots of the method for a run's event counts."""
    return (SEGMENT * stats["events"] + SCATTER * stats["scatters"] + FACE * stats["face_events"]
            + FRESNEL * stats["fresnel_draws"] + LAUNCH * stats["launched"])


def valu_roofline(stats: dict, kernel_s: float) -> dict:
    ops = algorithmic_ops(stats)
    achieved = ops / kernel_s
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "T lane-op/s", "frac": achieved / VALU_PEAK,
            "ops_per_launch": ops}


def atomic_roofline(stats: dict, kernel_s: float) -> dict:
    rate = stats["flushes"] / kernel_s
    return {"bound": "memory-side atomics", "achieved": rate, "peak": ATOMIC_PEAK_F64,
            "unit": "atomics/s", "frac": rate / ATOMIC_PEAK_F64,
            "atomics_per_photon": stats["flushes"] / max(1, stats["launched"])}


HERE = os.path.dirname(os.path.abspath(__file__))
COUNTERS = os.path.join(os.path.dirname(HERE), "profiles", "transport_cube60_sphere_counters.json")


def kernel_source_hash() -> str:
    """SHA-256 of the transport kernel's sources (kernel, internal header and
    the host code that lays out its launch and LDS window)."""
    h = hashlib.sha256()
    for f in ["mcx_transport.hip", "mcx_internal.hpp", "mcx_runtime.hip"]:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(photons: int, lds_window_cells: int):
    """HBM-side bytes per transport launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counters (one entry per LDS window size they
    were taken with), scaled by the copy-kernel calibration and by photons;
    None when the counters were taken on other kernel source or no entry
    has this LDS window (the window decides how many deposits reach memory
    as atomics)."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    e = c.get("by_window", {}).get(str(lds_window_cells))
    if e is None or e["launch"]["lds_window_cells"] != lds_window_cells:
        return None
    per_photon = (e["fetch_kib"] * c["fetch_factor"] + e["write_kib"] * c["write_factor"]) * 1024.0 \
        / c["photons"]
    return per_photon * photons
