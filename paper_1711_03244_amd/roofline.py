"""Roofline figures of the transport loop: the two ceilings that bind it.

**FP32 VALU.**  Peak: 256 compute units x 64 FP32 lanes per clock x 2.4 GHz
= 39.32e12 lane-operations per second (non-packed; packed FP32 is disabled
in the build).  The algorithmic work of a run is the method's own
arithmetic per event, counted by a fixed convention written down before
anything was measured, times the event counts the run reports:

* a random uniform costs its share of a Philox4x32-10 block: ten rounds of
  two 32x32 multiplies, each giving a high and a low word, and four
  xor/add, plus two, 82 operations per block or about 20 per uniform;
  integer multiplies issue at a quarter of the FP32 rate, so with each of
  the 40 multiplies weighted 4 a block costs 202 and a uniform 50.5;
* a segment (free path, voxel hop and deposit): about 25 FP32 operations,
  one exp (4) and one 1 - exp(-x) (about 6) -> 35;
* a scattering: 3 uniforms, one log (4), one sqrt (4), a sine and a cosine
  (4 each) and about 30 FMA (HG inversion, basis, rotation, renormalising)
  -> 46 + 3 uniforms;
* a Fresnel test: about 20 operations, one sqrt (4) and one uniform;
* a roulette test: one compare and one uniform;
* a launch: one uniform and its log (4).

Transcendentals (v_exp, v_log, v_sqrt, v_sin, v_cos, v_rcp) are
quarter-rate and count 4.  Two figures come out: with the multiplies
weighted 4 (the convention's primary count) and unweighted.  A third,
finer model of the issue slots each event's instructions take on gfx950
(segment 60, scattering 162, face event 19, Fresnel test 120, launch 88,
with the Philox block at the 60 slots the microbenchmark measures) is kept
beside them as `issue_model`.

**Memory-side atomics.**  Every atomic add on device memory executes at the
memory side at a fixed aggregate rate, measured by the microbenchmark on
distinct addresses (the published specifications give no such figure):
2.36e10/s for 64-bit (and FP64) adds without a return, 2.59e10/s for
returning 32-bit adds followed by the carry test the map's 32-bit mode
uses.  The atomics a launch issues are counted by the kernel itself
(`flushes`: every cell-visit sum added to the map by a global atomic; a
carry's second add, once per ~4000 adds to a cell, is not counted) and
agree with the TCC_ATOMIC counter.  Algorithmic bytes of the map traffic
are 8 per deposit (one map update per segment) plus one label byte per face
event; HBM traffic measured by FETCH_SIZE / WRITE_SIZE is reported against
them.
"""
import hashlib
import json
import os

CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
VALU_PEAK = CUS * LANES * CLOCK_HZ            # lane-op slots per second
ATOMIC_PEAK_F64 = 2.36e10                     # measured FP64 no-return atomics/s, distinct addresses
ATOMIC_PEAK_U64 = 2.36e10                     # measured 64-bit integer no-return adds/s (the same)
ATOMIC_PEAK_U32_CARRY = 2.59e10               # measured returning 32-bit adds/s with the carry test
MAP_ADDS_32 = 2                               # mcx_run_stats.map_adds of a 32-bit-add launch

# --- the frozen per-event convention
PHILOX_BLOCK_OPS = 10 * (2 + 2 + 4) + 2       # 82: per round 2 mul_hi, 2 mul_lo, 4 xor/add
PHILOX_BLOCK_OPS_MUL4 = 10 * (4 * 4 + 4) + 2  # 202: the 40 multiplies weighted 4
TRANS = 4                                     # exp, log, sqrt, sin, cos, rcp


def per_event(uniform: float) -> dict:
    """Operations per event of the convention, for a uniform costing `uniform`."""
    return {
        "segment": 25 + TRANS + 6,
        "scatter": 3 * uniform + TRANS + TRANS + 2 * TRANS + 30,
        "fresnel": 20 + TRANS + uniform,
        "roulette": 1 + uniform,
        "launch": uniform + TRANS,
    }


CONVENTION = per_event(PHILOX_BLOCK_OPS_MUL4 / 4)
CONVENTION_UNWEIGHTED = per_event(PHILOX_BLOCK_OPS / 4)


def convention_ops(stats: dict, table: dict = CONVENTION) -> float:
    """Algorithmic lane-operations of a run: per-event work x event counts."""
    return (table["segment"] * stats["events"] + table["scatter"] * stats["scatters"]
            + table["fresnel"] * stats["fresnel_draws"] + table["roulette"] * stats["rr_tests"]
            + table["launch"] * stats["launched"])


# --- the finer issue-slot model (full-rate operation 1 slot, transcendental
# 4, 32x32->64 multiply 2; Philox block 60 slots as measured)
PHILOX_BLOCK_SLOTS = 10 * (2 * 2 + 2)
UNIFORM_SLOTS = 3                              # shift, or, convert-and-scale
ISSUE_MODEL = {
    # 3 face distances (5 each), argmin 4, scattering distance 2, time
    # distance 3, event choice 5, gate 6, deposit 11, visit accumulation 2,
    # move 10, segment count 2
    "segment": 15 + 4 + 2 + 3 + 5 + 6 + 11 + 2 + 10 + 2,
    # Philox block + 3 uniforms, HG 13, sin theta 7, azimuth 9, basis 15,
    # rotation 12, renormalising 10, three h/|v| 21, new free path 5, roulette 1
    "scatter": PHILOX_BLOCK_SLOTS + 3 * UNIFORM_SLOTS + 13 + 7 + 9 + 15 + 12 + 10 + 21 + 5 + 1,
    # axis components 6, neighbour index and bounds 6, comparison 2, face
    # snap 2, entering 3
    "face": 6 + 6 + 2 + 2 + 3,
    # n1/n2 5, sin^2 t 3, TIR test 1, cos t 6, reflectance 18, Philox block +
    # uniform, direction update with new h/|v| 24
    "fresnel": 5 + 3 + 1 + 6 + 18 + PHILOX_BLOCK_SLOTS + UNIFORM_SLOTS + 24,
    # Philox block, uniform, -ln u, state set-up 20
    "launch": PHILOX_BLOCK_SLOTS + UNIFORM_SLOTS + 5 + 20,
}


def issue_model_ops(stats: dict) -> float:
    m = ISSUE_MODEL
    return (m["segment"] * stats["events"] + m["scatter"] * stats["scatters"]
            + m["face"] * stats["face_events"] + m["fresnel"] * stats["fresnel_draws"]
            + m["launch"] * stats["launched"])


def valu_roofline(stats: dict, kernel_s: float) -> dict:
    ops = convention_ops(stats)
    ops_u = convention_ops(stats, CONVENTION_UNWEIGHTED)
    ops_i = issue_model_ops(stats)
    return {"bound": "alu", "achieved": ops / kernel_s / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "T lane-op/s", "frac": ops / kernel_s / VALU_PEAK, "ops_per_launch": ops,
            "frac_unweighted_multiplies": ops_u / kernel_s / VALU_PEAK,
            "issue_model": {"frac": ops_i / kernel_s / VALU_PEAK, "ops_per_launch": ops_i}}


def algorithmic_bytes(stats: dict) -> float:
    """Map traffic the method needs: one 8-byte map update per deposit
    (segment) and one label byte per face event."""
    return 8.0 * stats["events"] + 1.0 * stats["face_events"]


def atomic_roofline(stats: dict, kernel_s: float) -> dict:
    """Map atomics of a launch against the measured rate of the kind of add
    it used (stats["map_adds"]): 64-bit adds without a return, or 32-bit
    returning adds with the carry test."""
    rate = stats["flushes"] / kernel_s
    if stats.get("map_adds") == MAP_ADDS_32:
        peak, src = ATOMIC_PEAK_U32_CARRY, ("measured: returning 32-bit atomic adds with the "
                                            "carry test on distinct addresses (microbenchmark)")
    else:
        peak, src = ATOMIC_PEAK_U64, ("measured: 64-bit no-return atomic adds on distinct "
                                      "addresses (microbenchmark)")
    return {"bound": "atomics", "achieved": rate, "peak": peak, "peak_source": src,
            "unit": "atomics/s", "frac": rate / peak,
            "atomics_per_photon": stats["flushes"] / max(1, stats["launched"]),
            "deposits_per_photon": stats["events"] / max(1, stats["launched"])}


def binding(stats: dict, kernel_s: float) -> dict:
    """The roofline of the ceiling that binds: the larger of the memory-side
    atomic fraction and the VALU fraction (convention count), with the other
    one attached."""
    a = atomic_roofline(stats, kernel_s)
    v = valu_roofline(stats, kernel_s)
    if a["frac"] >= v["frac"]:
        out = dict(a)
        out["valu"] = v
    else:
        out = dict(v)
        out["atomics"] = a
    out["algorithmic_bytes"] = algorithmic_bytes(stats)
    return out


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


def measured_traffic(photons: int, launch: dict):
    """HBM-side bytes per transport launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counters, scaled by the copy-kernel calibration
    and by photons; None when the counters were taken on other kernel
    source or with another launch (block size, photons per job, LDS window
    and kind of map add decide how many deposits reach memory, and how).
    launch: {"block_size", "refill_chunk", "lds_window_cells", "map_adds"}
    with map_adds as mcx_run_stats reports it (1: 64-bit, 2: 32-bit)."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    e = c.get("by_window", {}).get(str(launch["lds_window_cells"]))
    if e is None:
        return None
    took = e["launch"]
    adds = {"64-bit": 1, "32-bit with carry": 2}.get(took.get("map_adds"))
    if (took["block_size"], took["refill_chunk"], took["lds_window_cells"], adds) != (
            launch["block_size"], launch["refill_chunk"], launch["lds_window_cells"],
            launch["map_adds"]):
        return None
    per_photon = (e["fetch_kib"] * c["fetch_factor"] + e["write_kib"] * c["write_factor"]) * 1024.0 \
        / c["photons"]
    return per_photon * photons
