"""ctypes binding of libmcx.so, the C ABI declared in include/mcx.h.

Argument marshalling only: every step of the simulation runs in the HIP
library.  The functions keep the C names; :class:`Simulation` bundles them
for a :class:`paper_1711_03244_amd.workloads.Problem`.  PyTorch is used only
when the caller hands over device tensors or streams.

Importing this module does not load the library; the first call does, and it
raises if ``libmcx.so`` has not been built (``python -m
paper_1711_03244_amd.build``).  There is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcx.so")

MCX_OK, MCX_EINVAL, MCX_ENOMEM, MCX_ENODEV, MCX_EDEVICE, MCX_ESTATE, MCX_ERANGE = (
    0, -1, -2, -3, -4, -5, -6)
MCX_RAW, MCX_FLUENCE, MCX_FLUENCE_RATE = 0, 1, 2
STATUS_NAMES = {0: "MCX_OK", -1: "MCX_EINVAL", -2: "MCX_ENOMEM", -3: "MCX_ENODEV",
                -4: "MCX_EDEVICE", -5: "MCX_ESTATE", -6: "MCX_ERANGE"}
DIGEST = ["reason", "nscat", "events", "voxel", "w", "t", "blocks", "det"]

EXPORTS = ["mcx_default_options", "mcx_create", "mcx_run", "mcx_run_range", "mcx_reset",
           "mcx_sync", "mcx_ncells", "mcx_fluence", "mcx_fluence_f64", "mcx_fluence_device",
           "mcx_detected", "mcx_stats", "mcx_digest", "mcx_last_error", "mcx_destroy",
           "mcx_batch_create", "mcx_batch_size", "mcx_batch_ncells", "mcx_batch_run",
           "mcx_batch_run_range", "mcx_batch_fluence", "mcx_batch_fluence_f64",
           "mcx_batch_stats", "mcx_batch_detected", "mcx_batch_digest", "mcx_set_launch",
           "mcx_autotune", "mcx_detpost_device", "mcx_detpost_device_noalloc",
           "mcx_detected_process", "mcx_fit_linear",
           "mcx_fit_runtime", "mcx_set_balance", "mcx_shape_window", "mcx_set_map_adds"]


class McxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class mcx_medium(C.Structure):
    _fields_ = [("mua", C.c_float), ("mus", C.c_float), ("g", C.c_float), ("n", C.c_float)]


class mcx_volume(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("voxel_mm", C.c_float),
                ("labels", C.c_void_p), ("media", C.c_void_p), ("nmedia", C.c_int32)]


class mcx_source(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("dir", C.c_float * 3)]


class mcx_detector(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("radius", C.c_float)]


class mcx_gates(C.Structure):
    _fields_ = [("t0_ns", C.c_float), ("dt_ns", C.c_float), ("ngates", C.c_int32)]


class mcx_sim(C.Structure):
    _fields_ = [("vol", mcx_volume), ("src", mcx_source), ("det", C.c_void_p),
                ("ndet", C.c_int32), ("gates", mcx_gates), ("reflect", C.c_int32),
                ("n_outside", C.c_float)]


class mcx_tune_result(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("refill_chunk", C.c_int32),
                ("lds_window_cells", C.c_int32), ("candidates", C.c_int32),
                ("default_ms", C.c_double), ("best_ms", C.c_double),
                ("ms_per_photon", C.c_double), ("overhead_ms", C.c_double),
                ("map_adds", C.c_int32), ("reserved", C.c_int32)]

# how the transport kernel adds to map cells (mcx_set_map_adds)
MAP_ADDS_AUTO, MAP_ADDS_64, MAP_ADDS_32 = 0, 1, 2


class mcx_options(C.Structure):
    _fields_ = [("reflect", C.c_int32), ("n_outside", C.c_float), ("rr_threshold", C.c_float),
                ("rr_m", C.c_float), ("max_detected", C.c_uint64), ("max_events", C.c_uint64),
                ("device", C.c_int32), ("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("refill_chunk", C.c_int32), ("ndigest", C.c_uint64),
                ("lds_window_cells", C.c_int32), ("accurate_math", C.c_int32),
                ("kernel_variant", C.c_int32)]


class mcx_detpost(C.Structure):
    _fields_ = [("ndet", C.c_int32), ("npath", C.c_int32), ("t0_ns", C.c_float),
                ("dt_ns", C.c_float), ("ngates", C.c_int32), ("nphoton", C.c_uint64)]


class mcx_run_stats(C.Structure):
    _fields_ = ([(n, C.c_uint64) for n in
                 ["launched", "escaped", "detected", "timeout", "rr_dead", "capped", "scatters",
                  "face_events", "fresnel_draws", "reflections", "rr_tests", "rr_survived",
                  "events", "lane_slots", "flushes", "det_records", "det_dropped"]]
                + [(n, C.c_double) for n in
                   ["w_launched", "w_escaped", "w_detected", "w_timeout", "w_rr_gain",
                    "w_rr_loss", "w_capped", "tally_sum", "absorbed_grid", "kernel_ms",
                    "run_ms"]]
                + [("grid_blocks", C.c_int32), ("block_size", C.c_int32),
                   ("map_adds", C.c_int32), ("reserved", C.c_int32)])


_lib = None


def lib() -> C.CDLL:
    """Load libmcx.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "`python -m paper_1711_03244_amd.build`")
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7
        # and loads it by path, so load it first and let libmcx bind to the
        # same copy (same soname) instead of pulling in a second runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, u64, i32 = C.c_void_p, C.c_uint64, C.c_int32
        sig = {
            "mcx_default_options": (None, [C.POINTER(mcx_options)]),
            "mcx_create": (C.c_int, [C.POINTER(mcx_volume), C.POINTER(mcx_source),
                                     C.POINTER(mcx_detector), i32, C.POINTER(mcx_gates),
                                     C.POINTER(mcx_options), C.POINTER(vp)]),
            "mcx_run": (C.c_int, [vp, u64, u64]),
            "mcx_run_range": (C.c_int, [vp, u64, u64, u64, vp]),
            "mcx_reset": (C.c_int, [vp, vp]),
            "mcx_sync": (C.c_int, [vp]),
            "mcx_ncells": (u64, [vp]),
            "mcx_fluence": (C.c_int, [vp, i32, vp, u64]),
            "mcx_fluence_f64": (C.c_int, [vp, i32, vp, u64]),
            "mcx_fluence_device": (C.c_int, [vp, i32, vp, u64, vp]),
            "mcx_detected": (C.c_int, [vp, vp, vp, u64, C.POINTER(u64), C.POINTER(u64)]),
            "mcx_stats": (C.c_int, [vp, C.POINTER(mcx_run_stats)]),
            "mcx_digest": (C.c_int, [vp, vp, u64]),
            "mcx_last_error": (C.c_char_p, []),
            "mcx_destroy": (None, [vp]),
            "mcx_batch_create": (C.c_int, [C.POINTER(mcx_sim), i32, C.POINTER(mcx_options),
                                           C.POINTER(vp)]),
            "mcx_batch_size": (i32, [vp]),
            "mcx_batch_ncells": (u64, [vp, i32]),
            "mcx_batch_run": (C.c_int, [vp, vp, vp]),
            "mcx_batch_run_range": (C.c_int, [vp, vp, vp, vp, vp]),
            "mcx_batch_fluence": (C.c_int, [vp, i32, i32, vp, u64]),
            "mcx_batch_fluence_f64": (C.c_int, [vp, i32, i32, vp, u64]),
            "mcx_batch_stats": (C.c_int, [vp, i32, C.POINTER(mcx_run_stats)]),
            "mcx_batch_detected": (C.c_int, [vp, i32, vp, vp, u64, C.POINTER(u64),
                                             C.POINTER(u64)]),
            "mcx_batch_digest": (C.c_int, [vp, i32, vp, u64]),
            "mcx_set_launch": (C.c_int, [vp, i32, i32, i32]),
            "mcx_autotune": (C.c_int, [vp, vp, vp, C.POINTER(mcx_tune_result)]),
            "mcx_detpost_device": (C.c_int, [vp, u64, C.POINTER(mcx_detpost), vp, vp, vp, vp]),
            "mcx_detpost_device_noalloc": (C.c_int, [vp, u64, C.POINTER(mcx_detpost), vp, vp, vp,
                                                     vp]),
            "mcx_detected_process": (C.c_int, [vp, i32, vp, vp, u64, vp, u64]),
            "mcx_fit_linear": (C.c_int, [vp, vp, i32, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]),
            "mcx_fit_runtime": (C.c_int, [vp, vp, vp, vp, vp, vp]),
            "mcx_set_balance": (C.c_int, [vp, vp]),
            "mcx_shape_window": (C.c_int, [vp, vp, vp, i32]),
            "mcx_set_map_adds": (C.c_int, [vp, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != MCX_OK:
        raise McxError(status, mcx_last_error())


def mcx_last_error() -> str:
    return lib().mcx_last_error().decode()


def mcx_default_options(**overrides) -> mcx_options:
    o = mcx_options()
    lib().mcx_default_options(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class _Inputs:
    """C structs for a Problem; holds the arrays they point into."""

    def __init__(self, p):
        self.labels = np.ascontiguousarray(p.labels, np.uint8)
        self.media = np.ascontiguousarray(p.media, np.float32)
        nz, ny, nx = self.labels.shape
        self.vol = mcx_volume(nx, ny, nz, p.h, self.labels.ctypes.data, self.media.ctypes.data,
                              self.media.shape[0])
        self.src = mcx_source((C.c_float * 3)(*p.src_pos), (C.c_float * 3)(*p.src_dir))
        dets = np.ascontiguousarray(p.detectors, np.float32).reshape(-1, 4)
        self.ndet = dets.shape[0]
        self.det = (mcx_detector * max(1, self.ndet))()
        for i, d in enumerate(dets):
            self.det[i] = mcx_detector((C.c_float * 3)(*d[:3]), float(d[3]))
        self.gates = mcx_gates(p.t0, p.dt, p.ngates)


def _options(**options) -> mcx_options:
    o = mcx_default_options()
    for k, v in options.items():
        setattr(o, k, v)
    return o


def mcx_batch_create(problems, **options) -> C.c_void_p:
    """One context for a list of workloads.Problem (one launch serves all).
    Roulette settings and the event cap come from the first problem."""
    p0 = problems[0]
    o = mcx_default_options(rr_threshold=p0.rr_threshold, rr_m=p0.rr_m,
                            max_events=int(p0.max_events))
    for k, v in options.items():
        setattr(o, k, v)
    keep = [_Inputs(p) for p in problems]
    sims = (mcx_sim * len(problems))()
    for i, (p, inp) in enumerate(zip(problems, keep)):
        sims[i] = mcx_sim(inp.vol, inp.src, C.cast(inp.det, C.c_void_p) if inp.ndet else None,
                          inp.ndet, inp.gates, int(bool(p.reflect)), p.n_out)
    ctx = C.c_void_p()
    _check(lib().mcx_batch_create(sims, len(problems), C.byref(o), C.byref(ctx)))
    return ctx


def mcx_batch_size(ctx) -> int:
    return int(lib().mcx_batch_size(ctx))


def mcx_batch_ncells(ctx, sim: int) -> int:
    return int(lib().mcx_batch_ncells(ctx, sim))


def _u64(values):
    return np.ascontiguousarray(np.asarray(values, dtype=np.uint64))


def mcx_batch_run(ctx, nphoton, seed):
    n, s = _u64(nphoton), _u64(seed)
    _check(lib().mcx_batch_run(ctx, n.ctypes.data, s.ctypes.data))


def mcx_batch_run_range(ctx, first, n, seed, stream=None):
    f = _u64(first) if first is not None else None
    nn, s = _u64(n), _u64(seed)
    _check(lib().mcx_batch_run_range(ctx, f.ctypes.data if f is not None else None,
                                     nn.ctypes.data, s.ctypes.data, _stream(stream)))


def mcx_batch_fluence(ctx, sim: int, kind: int = MCX_FLUENCE) -> np.ndarray:
    out = np.empty(mcx_batch_ncells(ctx, sim), np.float32)
    _check(lib().mcx_batch_fluence(ctx, sim, int(kind), out.ctypes.data, out.size))
    return out


def mcx_batch_fluence_f64(ctx, sim: int, kind: int = MCX_FLUENCE) -> np.ndarray:
    out = np.empty(mcx_batch_ncells(ctx, sim), np.float64)
    _check(lib().mcx_batch_fluence_f64(ctx, sim, int(kind), out.ctypes.data, out.size))
    return out


def mcx_batch_detected(ctx, sim: int, cap: int, rec_len: int):
    rec = np.zeros((cap, rec_len), np.float32)
    ph = np.zeros(cap, np.uint64)
    nrec, ndrop = C.c_uint64(), C.c_uint64()
    _check(lib().mcx_batch_detected(ctx, sim, rec.ctypes.data if cap else None,
                                    ph.ctypes.data if cap else None, cap, C.byref(nrec),
                                    C.byref(ndrop)))
    n = int(nrec.value)
    return rec[:n].copy(), ph[:n].copy(), int(ndrop.value)


def mcx_batch_digest(ctx, sim: int, nrows: int) -> np.ndarray:
    out = np.zeros((nrows, len(DIGEST)), np.float64)
    _check(lib().mcx_batch_digest(ctx, sim, out.ctypes.data, nrows))
    return out


def mcx_batch_stats(ctx, sim: int) -> dict:
    s = mcx_run_stats()
    _check(lib().mcx_batch_stats(ctx, sim, C.byref(s)))
    return {name: getattr(s, name) for name, _ in mcx_run_stats._fields_}


def mcx_set_launch(ctx, block_size: int = 0, refill_chunk: int = 0, lds_window_cells: int = 0):
    _check(lib().mcx_set_launch(ctx, block_size, refill_chunk, lds_window_cells))


def mcx_set_map_adds(ctx, mode: int):
    _check(lib().mcx_set_map_adds(ctx, int(mode)))


def mcx_autotune(ctx, pilot_photons, seed) -> dict:
    n, s = _u64(pilot_photons), _u64(seed)
    r = mcx_tune_result()
    _check(lib().mcx_autotune(ctx, n.ctypes.data, s.ctypes.data, C.byref(r)))
    return {name: getattr(r, name) for name, _ in mcx_tune_result._fields_}


def mcx_shape_window(ctx, pilot_photons, seed, lds_window_cells: int):
    """Shape the LDS window from a flush census pilot (see include/mcx.h)."""
    n, s = _u64(pilot_photons), _u64(seed)
    _check(lib().mcx_shape_window(ctx, n.ctypes.data, s.ctypes.data, int(lds_window_cells)))


def mcx_fit_linear(x, y):
    """Least-squares line y = a x + b (host only); returns (a, b)."""
    xs = np.ascontiguousarray(np.asarray(x, np.float64))
    ys = np.ascontiguousarray(np.asarray(y, np.float64))
    if xs.shape != ys.shape:
        raise ValueError("x and y differ in length")
    a, b = C.c_double(), C.c_double()
    _check(lib().mcx_fit_linear(xs.ctypes.data, ys.ctypes.data, xs.size, C.byref(a), C.byref(b)))
    return a.value, b.value


def mcx_fit_runtime(ctx, n1=None, n2=None, seed=None):
    """T = a n + T0 per simulation from pilots of n1 and n2 photons (None:
    1e6 and 5e6); returns (a, t0) arrays (ms per photon, ms)."""
    ns = mcx_batch_size(ctx)
    a, t0 = np.zeros(ns), np.zeros(ns)
    u1 = _u64(n1) if n1 is not None else None
    u2 = _u64(n2) if n2 is not None else None
    sd = _u64(seed if seed is not None else [1] * ns)
    _check(lib().mcx_fit_runtime(ctx, u1.ctypes.data if u1 is not None else None,
                                 u2.ctypes.data if u2 is not None else None, sd.ctypes.data,
                                 a.ctypes.data, t0.ctypes.data))
    return a, t0


def mcx_set_balance(ctx, cost_per_photon=None):
    """Home waves by estimated work cost_i n_i (None: by job counts)."""
    if cost_per_photon is None:
        _check(lib().mcx_set_balance(ctx, None))
        return
    c = np.ascontiguousarray(np.asarray(cost_per_photon, np.float64))
    assert c.size == mcx_batch_size(ctx)
    _check(lib().mcx_set_balance(ctx, c.ctypes.data))


def mcx_create(p, **options) -> C.c_void_p:
    """Create a context for a workloads.Problem; keyword arguments override
    mcx_options fields (block_size, refill_chunk, ndigest, device, ...)."""
    o = mcx_default_options(reflect=int(bool(p.reflect)), n_outside=p.n_out,
                            rr_threshold=p.rr_threshold, rr_m=p.rr_m,
                            max_events=int(p.max_events))
    for k, v in options.items():
        setattr(o, k, v)
    inp = _Inputs(p)
    ctx = C.c_void_p()
    _check(lib().mcx_create(C.byref(inp.vol), C.byref(inp.src),
                            inp.det if inp.ndet else None, inp.ndet, C.byref(inp.gates),
                            C.byref(o), C.byref(ctx)))
    return ctx


def mcx_run(ctx, nphoton: int, seed: int):
    _check(lib().mcx_run(ctx, int(nphoton), int(seed)))


def mcx_run_range(ctx, first: int, n: int, seed: int, stream=None):
    _check(lib().mcx_run_range(ctx, int(first), int(n), int(seed), _stream(stream)))


def mcx_reset(ctx, stream=None):
    _check(lib().mcx_reset(ctx, _stream(stream)))


def mcx_sync(ctx):
    _check(lib().mcx_sync(ctx))


def mcx_ncells(ctx) -> int:
    return int(lib().mcx_ncells(ctx))


def mcx_fluence(ctx, kind: int = MCX_FLUENCE, out: Optional[np.ndarray] = None) -> np.ndarray:
    n = mcx_ncells(ctx)
    if out is None:
        out = np.empty(n, np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous
    _check(lib().mcx_fluence(ctx, int(kind), out.ctypes.data, out.size))
    return out


def mcx_fluence_f64(ctx, kind: int = MCX_FLUENCE, out: Optional[np.ndarray] = None) -> np.ndarray:
    n = mcx_ncells(ctx)
    if out is None:
        out = np.empty(n, np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous
    _check(lib().mcx_fluence_f64(ctx, int(kind), out.ctypes.data, out.size))
    return out


def mcx_fluence_device(ctx, kind: int, tensor, stream=None):
    """Write the normalised map into a contiguous float32 torch tensor on the
    context's device, enqueued on `stream` (None: torch's current stream, so
    that torch's later work on the tensor sees the result; torch's default
    stream is the null stream, which the C call takes for NULL).  The
    library orders it after the context's last clear or launch on any
    stream, so no synchronisation is needed in between."""
    import torch
    assert tensor.is_cuda and tensor.dtype == torch.float32 and tensor.is_contiguous()
    if stream is None:
        stream = torch.cuda.current_stream(tensor.device)
    _check(lib().mcx_fluence_device(ctx, int(kind), C.c_void_p(tensor.data_ptr()),
                                    tensor.numel(), _stream(stream)))
    return tensor


def mcx_detected(ctx, cap: int, rec_len: int):
    rec = np.zeros((cap, rec_len), np.float32)
    ph = np.zeros(cap, np.uint64)
    nrec, ndrop = C.c_uint64(), C.c_uint64()
    _check(lib().mcx_detected(ctx, rec.ctypes.data if cap else None, ph.ctypes.data if cap else None,
                              cap, C.byref(nrec), C.byref(ndrop)))
    n = int(nrec.value)
    return rec[:n].copy(), ph[:n].copy(), int(ndrop.value)


def mcx_stats(ctx) -> dict:
    s = mcx_run_stats()
    _check(lib().mcx_stats(ctx, C.byref(s)))
    return {name: getattr(s, name) for name, _ in mcx_run_stats._fields_}


def mcx_digest(ctx, nrows: int) -> np.ndarray:
    out = np.zeros((nrows, len(DIGEST)), np.float64)
    _check(lib().mcx_digest(ctx, out.ctypes.data, nrows))
    return out


def mcx_detpost_device(rec, spec: dict, dmua=None, out=None, weight=None, stream=None,
                       noalloc: bool = False):
    """Post-process detector records held in a float32 torch tensor (nrec,
    4 + npath) on the GPU: `spec` has ndet, npath, t0, dt, ngates, nphoton;
    `dmua` an optional float32 device tensor of npath absorption changes.
    Returns the (ndet, 2 + ngates) float64 device tensor `out` (count,
    reflectance, TPSF per gate) and, if `weight` is given or True, the
    re-weighted weight of every record.  noalloc=True calls
    mcx_detpost_device_noalloc (the library's own workspace, no stream wait);
    pass `out` (and a `weight` tensor) to keep the call free of allocations."""
    import torch
    assert rec.is_cuda and rec.dtype == torch.float32 and rec.is_contiguous()
    sp = mcx_detpost(int(spec["ndet"]), int(spec["npath"]), float(spec["t0"]),
                     float(spec["dt"]), int(spec["ngates"]), int(spec["nphoton"]))
    nrec = rec.shape[0] if rec.dim() == 2 else 0
    if nrec:
        assert rec.shape[1] == 4 + sp.npath, "records need 4 + npath columns"
    if out is None:
        out = torch.empty((sp.ndet, 2 + sp.ngates), dtype=torch.float64, device=rec.device)
    if weight is True:
        weight = torch.empty(nrec, dtype=torch.float64, device=rec.device)
    if dmua is not None:
        assert dmua.is_cuda and dmua.dtype == torch.float32 and dmua.numel() >= sp.npath
    fn = lib().mcx_detpost_device_noalloc if noalloc else lib().mcx_detpost_device
    _check(fn(C.c_void_p(rec.data_ptr()) if nrec else None, nrec, C.byref(sp),
              C.c_void_p(dmua.data_ptr()) if dmua is not None else None,
              C.c_void_p(out.data_ptr()),
              C.c_void_p(weight.data_ptr()) if weight is not None else None,
              _stream(stream)))
    return out, weight


def mcx_detected_process(ctx, sim: int, ndet: int, ngates: int, npath: int, dmua=None,
                         weights: bool = False, nrec: int = 0):
    """Post-process the stored records of simulation `sim` on the GPU:
    returns (out (ndet, 2 + ngates) float64, weights of the nrec records in
    record order or None)."""
    out = np.zeros((ndet, 2 + ngates), np.float64)
    w = np.zeros(max(nrec, 1), np.float64) if weights else None
    d = None if dmua is None else np.ascontiguousarray(np.asarray(dmua, np.float32).ravel()[:npath])
    if d is not None and d.size < npath:
        raise ValueError(f"need {npath} absorption changes")
    _check(lib().mcx_detected_process(ctx, int(sim), d.ctypes.data if d is not None else None,
                                      out.ctypes.data, out.size,
                                      w.ctypes.data if w is not None else None,
                                      w.size if w is not None else 0))
    return out, (w[:nrec] if w is not None else None)


def mcx_destroy(ctx):
    if ctx:
        lib().mcx_destroy(ctx)


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return C.c_void_p(s)
    handle = getattr(s, "cuda_stream", None)  # torch.cuda.Stream
    return C.c_void_p(handle if handle is not None else int(s))


class Batch:
    """One context for many Problems, run by one persistent launch."""

    def __init__(self, problems, **options):
        self.problems = list(problems)
        self.ctx = mcx_batch_create(self.problems, **options)
        self.ndigest = int(options.get("ndigest", 0))

    def __len__(self):
        return len(self.problems)

    def run(self, nphoton, seed) -> "Batch":
        mcx_batch_run(self.ctx, nphoton, seed)
        return self

    def run_range(self, first, n, seed, stream=None) -> "Batch":
        mcx_batch_run_range(self.ctx, first, n, seed, stream)
        return self

    def reset(self, stream=None):
        mcx_reset(self.ctx, stream)

    def sync(self):
        mcx_sync(self.ctx)

    def fluence(self, sim: int, kind: int = MCX_FLUENCE, f64: bool = False) -> np.ndarray:
        f = (mcx_batch_fluence_f64 if f64 else mcx_batch_fluence)(self.ctx, sim, kind)
        return f.reshape(self.problems[sim].tally_shape)

    def stats(self, sim: int) -> dict:
        return mcx_batch_stats(self.ctx, sim)

    def detected(self, sim: int, cap: Optional[int] = None):
        if cap is None:
            cap = int(self.stats(sim)["det_records"])
        return mcx_batch_detected(self.ctx, sim, cap, self.problems[sim].record_len)

    def digest(self, sim: int, nrows: Optional[int] = None) -> np.ndarray:
        return mcx_batch_digest(self.ctx, sim, self.ndigest if nrows is None else nrows)

    def detected_process(self, sim: int, dmua=None, weights: bool = False):
        p = self.problems[sim]
        nrec = int(self.stats(sim)["det_records"]) if weights else 0
        return mcx_detected_process(self.ctx, sim, p.ndet, p.ngates, p.nmedia - 1, dmua,
                                    weights, nrec)

    def autotune(self, pilot_photons, seed) -> dict:
        return mcx_autotune(self.ctx, pilot_photons, seed)

    def set_launch(self, block_size=0, refill_chunk=0, lds_window_cells=0):
        mcx_set_launch(self.ctx, block_size, refill_chunk, lds_window_cells)

    def set_map_adds(self, mode: int):
        mcx_set_map_adds(self.ctx, mode)

    def fit_runtime(self, n1=None, n2=None, seed=None):
        return mcx_fit_runtime(self.ctx, n1, n2, seed)

    def set_balance(self, cost_per_photon=None):
        mcx_set_balance(self.ctx, cost_per_photon)

    def close(self):
        if self.ctx:
            mcx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation:
    """One context for one Problem."""

    def __init__(self, problem, **options):
        self.problem = problem
        self.ctx = mcx_create(problem, **options)
        self.ndigest = int(options.get("ndigest", 0))

    def run(self, nphoton: int, seed: int) -> "Simulation":
        mcx_run(self.ctx, nphoton, seed)
        return self

    def run_range(self, first: int, n: int, seed: int, stream=None) -> "Simulation":
        mcx_run_range(self.ctx, first, n, seed, stream)
        return self

    def reset(self, stream=None):
        mcx_reset(self.ctx, stream)

    def sync(self):
        mcx_sync(self.ctx)

    def fluence(self, kind: int = MCX_FLUENCE, f64: bool = False) -> np.ndarray:
        f = mcx_fluence_f64(self.ctx, kind) if f64 else mcx_fluence(self.ctx, kind)
        return f.reshape(self.problem.tally_shape)

    def detected(self, cap: Optional[int] = None):
        if cap is None:
            cap = int(self.stats()["det_records"])
        return mcx_detected(self.ctx, cap, self.problem.record_len)

    def stats(self) -> dict:
        return mcx_stats(self.ctx)

    def digest(self, nrows: Optional[int] = None) -> np.ndarray:
        return mcx_digest(self.ctx, self.ndigest if nrows is None else nrows)

    def detected_process(self, dmua=None, weights: bool = False):
        """Per-detector record count, reflectance and TPSF (and optionally
        the re-weighted record weights) from the stored detector records,
        for absorption changes dmua (one per medium 1..nmedia-1)."""
        p = self.problem
        nrec = int(self.stats()["det_records"]) if weights else 0
        return mcx_detected_process(self.ctx, 0, p.ndet, p.ngates, p.nmedia - 1, dmua,
                                    weights, nrec)

    def autotune(self, pilot_photons: int, seed: int) -> dict:
        return mcx_autotune(self.ctx, [pilot_photons], [seed])

    def shape_window(self, pilot_photons: int, seed: int, lds_window_cells: int):
        mcx_shape_window(self.ctx, [pilot_photons], [seed], lds_window_cells)

    def fit_runtime(self, n1: int = 1_000_000, n2: int = 5_000_000, seed: int = 1):
        """The paper's T = a n + T0 from two pilots; returns (a, t0)."""
        a, t0 = mcx_fit_runtime(self.ctx, [n1], [n2], [seed])
        return float(a[0]), float(t0[0])

    def set_launch(self, block_size=0, refill_chunk=0, lds_window_cells=0):
        mcx_set_launch(self.ctx, block_size, refill_chunk, lds_window_cells)

    def set_map_adds(self, mode: int):
        mcx_set_map_adds(self.ctx, mode)

    def close(self):
        if self.ctx:
            mcx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
