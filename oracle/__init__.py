"""FP64 CPU oracle of voxel Monte Carlo photon transport -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps oracle/libmcx_oracle.so (plain C, double
precision) with ctypes and adds the post-processing step of the paper's
workflow (normalising the read-back tally into fluence) written out in
numpy.  Nothing here is shared with, or imported from, the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np

from . import build as _build

LEDGER = ["absorbed", "escaped", "detected", "timeout", "rr_gain", "rr_loss", "capped",
          "launched"]
COUNTS = ["launched", "escaped", "detected", "timeout", "rr_dead", "capped", "scatters",
          "face_events", "fresnel_draws", "tir", "reflections", "rr_tests", "rr_survived",
          "deposits", "events", "max_events", "entries"]
DIGEST = ["reason", "nscat", "events", "voxel", "w", "t", "blocks", "det"]
C_MM_PER_NS = 299.792458


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
                ("labels", C.c_void_p), ("nmedia", C.c_int32), ("media", C.c_void_p),
                ("src_pos", C.c_double * 3), ("src_dir", C.c_double * 3),
                ("ndet", C.c_int32), ("det", C.c_void_p),
                ("t0", C.c_double), ("dt", C.c_double), ("ngates", C.c_int32),
                ("reflect", C.c_int32), ("n_out", C.c_double), ("rr_threshold", C.c_double),
                ("rr_m", C.c_double), ("max_events", C.c_uint64)]


class _Output(C.Structure):
    _fields_ = [("tally", C.c_void_p), ("deposits", C.c_void_p),
                ("ledger", C.c_double * len(LEDGER)), ("counts", C.c_int64 * len(COUNTS)),
                ("det_rec", C.c_void_p), ("det_photon", C.c_void_p), ("det_cap", C.c_uint64),
                ("det_total", C.c_uint64), ("det_written", C.c_uint64),
                ("digest", C.c_void_p), ("ndigest", C.c_uint64), ("visits", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # MCX_ORACLE_LIB lets a checker point the wrapper at another build of
        # this same source (e.g. a deliberately broken copy, to verify that
        # the pins catch it).
        path = os.environ.get("MCX_ORACLE_LIB") or _build.build(force=False)
        L = C.CDLL(path)
        L.orc_run.argtypes = [C.POINTER(_Problem), C.c_uint64, C.c_uint64, C.c_uint64, C.c_int,
                              C.POINTER(_Output)]
        L.orc_run.restype = C.c_int
        L.orc_validate.argtypes = [C.POINTER(_Problem)]
        L.orc_validate.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_hg_cos.argtypes = [C.c_double, C.c_double]
        L.orc_hg_cos.restype = C.c_double
        L.orc_scatter_dir.argtypes = [C.POINTER(C.c_double), C.c_double, C.c_double,
                                      C.POINTER(C.c_double)]
        L.orc_fresnel.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_fresnel.restype = C.c_double
        _lib = L
    return _lib


def _pack(p):
    """Marshal a workloads.Problem into the C struct; the arrays are kept
    alive by the returned tuple."""
    labels = np.ascontiguousarray(p.labels, np.uint8)
    media = np.ascontiguousarray(p.media, np.float64)
    det = np.ascontiguousarray(p.detectors, np.float64).reshape(-1, 4)
    nz, ny, nx = labels.shape
    s = _Problem()
    s.nx, s.ny, s.nz, s.h = nx, ny, nz, p.h
    s.labels = labels.ctypes.data
    s.nmedia = media.shape[0]
    s.media = media.ctypes.data
    s.src_pos = (C.c_double * 3)(*p.src_pos)
    s.src_dir = (C.c_double * 3)(*p.src_dir)
    s.ndet = det.shape[0]
    s.det = det.ctypes.data if det.size else None
    s.t0, s.dt, s.ngates = p.t0, p.dt, p.ngates
    s.reflect = int(bool(p.reflect))
    s.n_out, s.rr_threshold, s.rr_m = p.n_out, p.rr_threshold, p.rr_m
    s.max_events = int(p.max_events)
    return s, (labels, media, det)


def validate(p) -> int:
    s, keep = _pack(p)
    return lib().orc_validate(C.byref(s))


def run(p, nphoton: int, seed: int, first: int = 0, nthreads: int | None = None,
        deposits: bool = False, det_cap: int = 1 << 20, ndigest: int = 0,
        visits: bool = False) -> dict:
    """Simulate photons [first, first+nphoton) and return the raw tally
    (ngates, nz, ny, nx) in weight*mm, the ledger, counters, detector
    records and optional per-photon digests; with `deposits` the segments
    that deposited into each cell, with `visits` the photon visits of each
    cell (maximal runs of one photon's consecutive deposits into it)."""
    if nthreads is None:
        nthreads = min(os.cpu_count() or 1, 16)
    s, keep = _pack(p)
    tally = np.zeros(p.tally_shape, np.float64)
    dep = np.zeros(p.tally_shape, np.int64) if deposits else None
    vis = np.zeros(p.tally_shape, np.int64) if visits else None
    rec = np.zeros((det_cap, p.record_len), np.float32)
    rec_ph = np.zeros(det_cap, np.uint64)
    dig = np.zeros((ndigest, len(DIGEST)), np.float64) if ndigest else None
    o = _Output()
    o.tally = tally.ctypes.data
    o.deposits = dep.ctypes.data if dep is not None else None
    o.visits = vis.ctypes.data if vis is not None else None
    o.det_rec = rec.ctypes.data if det_cap else None
    o.det_photon = rec_ph.ctypes.data if det_cap else None
    o.det_cap = det_cap
    o.digest = dig.ctypes.data if dig is not None else None
    o.ndigest = ndigest
    t = time.perf_counter()
    rc = lib().orc_run(C.byref(s), first, nphoton, seed, nthreads, C.byref(o))
    wall = time.perf_counter() - t
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    nw = int(o.det_written)
    return {"tally": tally, "deposits": dep, "visits": vis,
            "ledger": dict(zip(LEDGER, list(o.ledger))),
            "counts": dict(zip(COUNTS, list(o.counts))),
            "records": rec[:nw].copy(), "record_photon": rec_ph[:nw].copy(),
            "det_total": int(o.det_total), "digest": dig, "wall_s": wall,
            "nthreads": nthreads, "nphoton": nphoton, "seed": seed, "first": first}


# ---------------------------------------------------------------- pieces

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform(word: int) -> float:
    return lib().orc_uniform(int(word) & 0xFFFFFFFF)


def hg_cos(g: float, u: float) -> float:
    return lib().orc_hg_cos(g, u)


def scatter_dir(v, cos_theta: float, u_phi: float):
    vin = (C.c_double * 3)(*v)
    out = (C.c_double * 3)()
    lib().orc_scatter_dir(vin, cos_theta, u_phi, out)
    return np.array(list(out))


def fresnel(n1: float, n2: float, cos_i: float) -> float:
    return lib().orc_fresnel(n1, n2, cos_i)


# ------------------------------------------------------ post-processing

def normalise(tally: np.ndarray, nphoton: int, h: float, dt: float, kind: int) -> np.ndarray:
    """The paper's post-processing of the read-back map.  kind 0: raw tally
    (weight*mm per cell); 1: fluence per launched photon, 1/mm^2 (tally /
    (N h^3)); 2: fluence rate, 1/(mm^2 ns) (fluence / gate width)."""
    if kind == 0:
        return tally.copy()
    phi = tally / (float(nphoton) * h ** 3)
    return phi if kind == 1 else phi / dt


def detected_postprocess(records, nphoton: int, ndet: int, t0: float, dt: float, ngates: int,
                         dmua=None):
    """Post-processing of detected-photon records (the step after detection
    in the paper's workflow, Fig. 1).  Rows are {detector, scatterings, exit
    weight w, exit time t, pathlength L_1 .. L_npath per medium}.

    Re-weighting for an absorption change: absorption is a continuous weight
    decay along the path, so a photon's exit weight under absorption
    mua_i + dmua_i is w exp(-sum_i dmua_i L_i); the exponent is summed in
    medium order.  Per detector d (rows of the result): the number of
    records, the re-weighted weight summed and divided by the launched
    photons (reflectance), and the same sum split by the gate of the exit
    time, g = min(max(floor((t - t0) / dt), 0), ngates - 1), divided by
    photons x dt (the time-resolved reflectance).  nphoton = 0 keeps the raw
    sums.  Records whose detector column is not an integer in [0, ndet) are
    left out.  Returns (result (ndet, 2 + ngates), re-weighted weights)."""
    rec = np.asarray(records, np.float32).astype(np.float64).reshape(-1, np.shape(records)[-1])
    n, npath = rec.shape[0], rec.shape[1] - 4
    w = rec[:, 2].copy()
    if dmua is not None:
        e = np.zeros(n)
        for i in range(npath):
            e = e + float(np.float32(dmua[i])) * rec[:, 4 + i]
        w = w * np.exp(-e)
    t0 = float(np.float32(t0))
    dt = float(np.float32(dt))
    det = rec[:, 0]
    ok = (det >= 0) & (det < ndet) & (det == np.floor(det))
    gate = np.floor((rec[:, 3] - t0) / dt)
    gate = np.where(gate >= 0, gate, 0.0)          # NaN and negative -> gate 0
    gate = np.minimum(gate, ngates - 1).astype(np.int64)
    d = det[ok].astype(np.int64)
    out = np.zeros((ndet, 2 + ngates))
    np.add.at(out[:, 0], d, 1.0)
    np.add.at(out[:, 1], d, w[ok])
    np.add.at(out, (d, 2 + gate[ok]), w[ok])
    if nphoton:
        out[:, 1] /= float(nphoton)
        out[:, 2:] /= float(nphoton) * dt
    return out, w
