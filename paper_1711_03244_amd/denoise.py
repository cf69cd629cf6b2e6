"""Training data, training loop and time-to-equal-error evaluation of the
fluence denoiser (include/mcx_nn.h), all on one GPU.

Data: seeded random heterogeneous volumes (workloads.denoiser_volume), each
simulated by the library's batched transport at a low photon count (the
network input; several counts per volume) and a high one (the target),
with independent seeds.  Maps are fluence per launched photon of the single
gate.  Training: Adam with a cosine learning-rate decay over the
(input, target) pairs in a seeded random order, on the mean gradient of a
few volumes per step, clipped to a global norm.

Evaluation on held-out volumes: the reference map is the mean of K
independent runs at the plain photon count; the error of a map is the RMS,
over the medium voxels where the reference is at least 1e-8 of its
maximum, of ln max(phi, 1e-12) - ln max(phi_ref, 1e-12).  The reference's
own noise inflates every measured error; its share, estimated from the
spread of the K runs (variance of the log map / K), is reported and
subtracted in quadrature.  Times: the plain run's and each low-photon run's
HIP-event time (clear + transport + reductions) plus the network's
inference time (HIP events on the inference stream).

Two timings are reported.  Single volume: each run in its own launch, so a
low-photon run pays the whole latency of its longest photons (tens of ms in
these media).  Batched: K volumes share one launch of the batched transport
at each photon count; the per-volume time is the launch time / K, and the
plain runs' per-volume time model T = a n + T0 is fitted over the same
batched launches.  Batching changes no result (a batched simulation
reproduces its single run photon for photon), only the time.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import mcx, nn, workloads as W

EPS = 1e-12
MASK_FLOOR = 1e-8


def _torch():
    import torch
    return torch


def simulate(problems, nphoton, seeds):
    """Fluence maps (per launched photon, gate 0) of every problem, one
    batched launch; returns (maps as float32 arrays, launch run_ms)."""
    n = [int(nphoton)] * len(problems) if np.isscalar(nphoton) else [int(v) for v in nphoton]
    with mcx.Batch(problems) as b:
        b.run(n, [int(s) for s in seeds])
        maps = [b.fluence(i, mcx.MCX_FLUENCE)[0].copy() for i in range(len(problems))]
        run_ms = b.stats(0)["run_ms"]
    return maps, run_ms


def simulate_one(problem, nphoton, seed):
    """One simulation in its own context; returns (map, run_ms)."""
    with mcx.Simulation(problem) as s:
        s.run(int(nphoton), int(seed))
        return s.fluence(mcx.MCX_FLUENCE)[0].copy(), s.stats()["run_ms"]


def error_mask(ref, labels):
    return (labels != 0) & (ref >= MASK_FLOOR * ref.max())


def log_rms(phi, ref, mask) -> float:
    d = np.log(np.maximum(phi, EPS)) - np.log(np.maximum(ref, EPS))
    return float(np.sqrt(np.mean(d[mask] ** 2)))


@dataclass
class DataSet:
    volumes: list
    inputs: list = field(default_factory=list)    # (volume index, photons, torch map)
    targets: list = field(default_factory=list)   # torch map per volume
    sim_ms: float = 0.0


def simulate_groups(vols, nphoton, seeds, max_photons=5e9):
    """`simulate` in batches of at most max_photons photons per launch."""
    per = max(1, int(max_photons // max(1.0, float(nphoton))))
    maps, ms = [], 0.0
    for g in range(0, len(vols), per):
        m, t = simulate(vols[g:g + per], nphoton, seeds[g:g + per])
        maps += m
        ms += t
    return maps, ms


def make_dataset(seeds, side, input_photons, target_photons, seed_base=1_000_000, say=print):
    """Simulate every volume at each input photon count and at the target
    count (independent seeds)."""
    t = _torch()
    seeds = [int(s) for s in seeds]
    vols = [W.denoiser_volume(s, side) for s in seeds]
    ds = DataSet(vols)
    for j, n_in in enumerate(input_photons):
        maps, ms = simulate_groups(vols, n_in, [seed_base * (j + 1) + s for s in seeds])
        ds.sim_ms += ms
        for i, m in enumerate(maps):
            ds.inputs.append((i, int(n_in), t.as_tensor(m).cuda()))
        say(f"[data] {len(vols)} volumes x {n_in:.0e} photons: {ms:.0f} ms")
    maps = []
    per = max(1, int(5e9 // float(target_photons)))
    for g in range(0, len(vols), per):
        m, ms = simulate(vols[g:g + per], target_photons,
                         [seed_base * 97 + s for s in seeds[g:g + per]])
        maps += m
        ds.sim_ms += ms
        say(f"[data] targets {g + len(m)}/{len(vols)} x {target_photons:.0e} photons: {ms:.0f} ms")
    ds.targets = [t.as_tensor(m).cuda() for m in maps]
    return ds


def train(den: nn.Denoiser, ds: DataSet, steps: int, lr: float = 1e-3, lr_min: float = 1e-5,
          seed: int = 1, log_every: int = 0, batch: int = 1, max_norm: float = 0.0,
          augment: bool = False, say=print) -> dict:
    """Adam steps over the pairs in a seeded random order, each on the mean
    gradient of `batch` pairs, clipped to global norm `max_norm` (> 0), with
    a cosine-decayed learning rate; with `augment`, every pair passes
    through one of the eight x-y symmetries (seeded draw) first.  Returns
    losses and wall time."""
    t = _torch()
    rng = np.random.default_rng(seed)
    order = []
    losses = []
    if augment:
        xa = t.empty_like(ds.targets[0])
        ta = t.empty_like(ds.targets[0])
    t.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        rate = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * k / max(1, steps)))
        want = bool(log_every) and (k % log_every == 0 or k == steps - 1)
        step_loss = []
        for b in range(batch):
            if not order:
                order = list(rng.permutation(len(ds.inputs)))
            vi, _, x = ds.inputs[order.pop()]
            y = ds.targets[vi]
            if augment:
                op = int(rng.integers(8))
                x, y = nn.mcx_nn_mirror_xy(x, op, xa), nn.mcx_nn_mirror_xy(y, op, ta)
            step_loss.append(den.loss_grad(x, y, want_loss=want, accumulate=b > 0))
        den.adam(rate, 1.0 / batch, max_norm)
        if want:
            loss = float(np.mean(step_loss))
            losses.append((k, loss))
            say(f"[train] step {k} lr {rate:.2e} loss {loss:.5f}")
    t.cuda.synchronize()
    return {"steps": steps, "batch": batch, "max_norm": max_norm, "augment": augment,
            "seconds": time.perf_counter() - t0, "losses": losses}


def infer_timed(den: nn.Denoiser, phi, symmetries: int = 1):
    """Denoise one map (averaged over `symmetries` x-y symmetries of the
    input, Denoiser.forward); returns (map as numpy, inference ms by HIP
    events)."""
    t = _torch()
    x = t.as_tensor(phi).cuda()
    out = t.empty_like(x)
    s = t.cuda.current_stream()
    e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
    e0.record(s)
    den.forward(x, phi_out=out, stream=s, symmetries=symmetries)
    e1.record(s)
    e1.synchronize()
    return out.cpu().numpy(), e0.elapsed_time(e1)


def evaluate(den: nn.Denoiser, seeds, side, plain_photons, ref_runs, input_photons,
             seed_base=5_000_000, say=print, batch_seeds=(), batch_extra=(3e7,)) -> dict:
    """Time-to-equal-error on held-out volumes (see the module docstring);
    with `batch_seeds`, also per-volume times of those volumes in batched
    launches at the input counts and at `batch_extra` counts."""
    batched = None
    if len(batch_seeds):
        counts = sorted(set(float(n) for n in list(input_photons) + list(batch_extra)))
        batched = batch_timing(side, batch_seeds, counts, say=say)
    rows = []
    for s in seeds:
        p = W.denoiser_volume(int(s), side)
        refs = []
        for k in range(ref_runs):
            m, _ = simulate_one(p, plain_photons, seed_base + 1000 * int(s) + 11 + k)
            refs.append(m.astype(np.float64))
        ref = np.mean(refs, axis=0)
        mask = error_mask(ref, p.labels)
        logs = np.log(np.maximum(np.stack(refs), EPS))
        ref_err = float(np.sqrt(np.mean(np.var(logs, axis=0, ddof=1)[mask]) / ref_runs))
        plain, plain_ms = simulate_one(p, plain_photons, seed_base + 1000 * int(s) + 1)
        row = {"seed": int(s), "mask_voxels": int(mask.sum()), "ref_err": ref_err,
               "plain_err": log_rms(plain, ref, mask), "plain_ms": plain_ms, "inputs": []}
        for j, n in enumerate(input_photons):
            lo, lo_ms = simulate_one(p, n, seed_base + 1000 * int(s) + 100 + j)
            dn, inf_ms = infer_timed(den, lo)
            infer_timed(den, lo)  # the first call includes weight packing; time a second
            dn, inf_ms = infer_timed(den, lo)
            row["inputs"].append({"photons": int(n), "sim_ms": lo_ms, "infer_ms": inf_ms,
                                  "noisy_err": log_rms(lo, ref, mask),
                                  "denoised_err": log_rms(dn, ref, mask)})
        rows.append(row)
        say(f"[eval] volume {s}: plain {plain_photons:.0e} err {row['plain_err']:.4f} "
            f"(ref share {ref_err:.4f}), " + ", ".join(
                f"{r['photons']:.0e}: noisy {r['noisy_err']:.4f} denoised {r['denoised_err']:.4f}"
                for r in row["inputs"]))
    return summarise(rows, plain_photons, input_photons, batched)


def plain_error_sq(runs, mask) -> float:
    """Squared log-RMS error of a plain run with as many photons as the K
    runs `runs` together (each with 1/K of them): the mean over the mask of
    the unbiased per-voxel variance of the K log maps, divided by K."""
    logs = np.log(np.maximum(np.stack([np.asarray(r, np.float64) for r in runs]), EPS))
    return float(np.mean(np.var(logs, axis=0, ddof=1)[mask]) / len(runs))


def error_sq_against(m, ref, mask, ref_sq) -> float:
    """Squared log-RMS error of map m against the truth, from its mean
    squared log difference to a reference whose own squared error is
    ref_sq (independent of m): the difference of the two."""
    d = np.log(np.maximum(np.asarray(m, np.float64), EPS)) - np.log(np.maximum(ref, EPS))
    return float(np.mean(d[mask] ** 2)) - ref_sq


def evaluate_strict(den: nn.Denoiser, seeds, side, input_photons, plain_photons=1e9,
                    ref_runs=2, timed_plain=2, seed_base=6_000_000, say=print,
                    symmetries: int = 1) -> dict:
    """Whether denoised low-photon maps reach the plain high-photon run's
    error, and in how much less time, on held-out volumes.

    Per volume: `ref_runs` independent plain runs of plain_photons /
    ref_runs photons each (all volumes in one batched launch per run; a
    batched simulation equals its single run photon for photon).  Their
    mean R is a plain run of plain_photons photons; the error a plain run
    of that size makes, E_p, is estimated from their spread: with K runs
    of n/K photons, var(ln of a run of n) = var(ln of a run of n/K) / K, and
    the mean over voxels of the unbiased per-voxel variance of the K log
    maps, divided by K, estimates E_p^2.  A map M is compared with R: the
    mean of (ln M - ln R)^2 over the mask is E(M)^2 + var(ln R), so E(M)^2 =
    that mean - E_p^2 (R's own noise, the same size as a plain run's).
    Mask: medium voxels with R >= 1e-8 max R.  Low-photon maps: one
    single-volume run per input count (its HIP-event time: clear,
    transport, reductions), denoised (inference time by HIP events).
    Plain-run time: single-volume runs of plain_photons photons timed on
    the first `timed_plain` volumes; for every volume, T = a n + T0 fitted
    to its own input runs, checked against those timed runs.  The target
    is met at an input count whose RMS (over volumes) denoised error is at
    most the RMS plain error; its time ratio is the mean plain time over
    the mean time of the input run plus inference.  symmetries: inference
    averaged over that many x-y symmetries of the input (its cost is in the
    inference time)."""
    seeds = [int(s) for s in seeds]
    vols = [W.denoiser_volume(s, side) for s in seeds]
    K = int(ref_runs)
    per_run = int(plain_photons) // K
    runs = []
    group = max(1, int(4e9 // per_run))  # photons per batched launch <= 4e9
    for k in range(K):
        maps = []
        for g in range(0, len(vols), group):
            m, ms = simulate(vols[g:g + group], per_run,
                             [seed_base + 1000 * int(s) + 11 + k for s in seeds[g:g + group]])
            maps += [x.astype(np.float64) for x in m]
            say(f"[strict] reference run {k + 1}/{K}, volumes {g + 1}-{g + len(m)} x "
                f"{per_run:.1e} photons: {ms / 1e3:.1f} s")
        runs.append(maps)
    rows = []
    for i, (s, p) in enumerate(zip(seeds, vols)):
        ref = np.mean([runs[k][i] for k in range(K)], axis=0)
        mask = error_mask(ref, p.labels)
        ep2 = plain_error_sq([runs[k][i] for k in range(K)], mask)
        row = {"seed": int(s), "mask_voxels": int(mask.sum()), "plain_err": math.sqrt(ep2),
               "inputs": []}
        ns, ts = [], []
        for j, n in enumerate(input_photons):
            lo, lo_ms = simulate_one(p, n, seed_base + 1000 * int(s) + 100 + j)
            infer_timed(den, lo, symmetries)  # the first call includes weight packing
            dn, inf_ms = infer_timed(den, lo, symmetries)
            e_n = error_sq_against(lo, ref, mask, ep2)
            e_d = error_sq_against(dn, ref, mask, ep2)
            row["inputs"].append({"photons": int(n), "sim_ms": lo_ms, "infer_ms": inf_ms,
                                  "noisy_err": math.sqrt(max(e_n, 0.0)),
                                  "denoised_err": math.sqrt(max(e_d, 0.0)),
                                  "denoised_sq": e_d})
            ns.append(float(n))
            ts.append(lo_ms)
        a, t0 = np.polyfit(np.array(ns), np.array(ts), 1)
        row["plain_ms_model"] = float(a * plain_photons + t0)
        if i < timed_plain:
            _, row["plain_ms"] = simulate_one(p, plain_photons, seed_base + 1000 * int(s) + 1)
        rows.append(row)
        say(f"[strict] volume {s}: plain {plain_photons:.0e} err {row['plain_err']:.4f}, " +
            ", ".join(f"{r['photons']:.0e}: noisy {r['noisy_err']:.4f} denoised "
                      f"{r['denoised_err']:.4f}" for r in row["inputs"]))
    plain = float(np.sqrt(np.mean([r["plain_err"] ** 2 for r in rows])))
    measured = [(r["plain_ms"], r["plain_ms_model"]) for r in rows if "plain_ms" in r]
    plain_ms = float(np.mean([r["plain_ms_model"] for r in rows]))
    out = {"volumes": len(rows), "plain_photons": int(plain_photons), "ref_runs": K,
           "symmetries": int(symmetries),
           "plain_err": plain, "plain_ms": plain_ms,
           "plain_ms_measured": [m for m, _ in measured],
           "plain_ms_model_error": (max(abs(mod / m - 1.0) for m, mod in measured)
                                    if measured else None),
           "per_input": [], "equal_error_photons": None, "time_ratio": None}
    for j, n in enumerate(input_photons):
        den2 = float(np.mean([r["inputs"][j]["denoised_sq"] for r in rows]))
        den_err = math.sqrt(max(den2, 0.0))
        noisy = float(np.sqrt(np.mean([r["inputs"][j]["noisy_err"] ** 2 for r in rows])))
        sim_ms = float(np.mean([r["inputs"][j]["sim_ms"] for r in rows]))
        inf_ms = float(np.mean([r["inputs"][j]["infer_ms"] for r in rows]))
        wins = sum(r["inputs"][j]["denoised_err"] <= r["plain_err"] for r in rows)
        out["per_input"].append({"photons": int(n), "noisy_err": noisy, "denoised_err": den_err,
                                 "sim_ms": sim_ms, "infer_ms": inf_ms,
                                 "time_ratio": plain_ms / (sim_ms + inf_ms),
                                 "volumes_at_or_below_plain": int(wins)})
    for r in sorted(out["per_input"], key=lambda r: r["photons"]):
        if r["denoised_err"] <= plain:
            out["equal_error_photons"] = r["photons"]
            out["time_ratio"] = r["time_ratio"]
            break
    return out


def batch_timing(side, seeds, photon_counts, seed_base=7_000_000, say=print) -> list:
    """Per-volume time of plain runs when the volumes `seeds` share one
    batched launch, at every photon count: [(photons, launch run_ms / K)]
    (HIP events: clear + launch + per-simulation reductions), after a
    warm-up launch."""
    vols = [W.denoiser_volume(int(s), side) for s in seeds]
    K = len(vols)
    out = []
    with mcx.Batch(vols) as b:
        b.run([1000] * K, [seed_base + int(s) for s in seeds])
        for j, n in enumerate(photon_counts):
            b.run([int(n)] * K, [seed_base + 1000 * (j + 1) + int(s) for s in seeds])
            ms = b.stats(0)["run_ms"]
            out.append((float(n), ms / K))
            say(f"[batch] {K} volumes x {n:.0e} photons: {ms:.1f} ms, {ms / K:.2f} ms per volume")
    return out


def _debias(e, r):
    return math.sqrt(max(e * e - r * r, 0.0))


def _equivalent_photons(n_err, err):
    """Photon count at which plain runs reach `err`: log-log interpolation
    between the two measured plain points that bracket it (extrapolation
    from the two nearest ones outside the measured range).  n_err:
    [(photons, error), ...]; None when the curve cannot be used."""
    pts = sorted((n, e) for n, e in n_err if e > 0)
    if len(pts) < 2 or err <= 0:
        return None
    if err >= pts[0][1]:
        pair = pts[0], pts[1]
    elif err <= pts[-1][1]:
        pair = pts[-2], pts[-1]
    else:
        pair = next((p, q) for p, q in zip(pts, pts[1:]) if p[1] >= err >= q[1])
    (n0, e0), (n1, e1) = pair
    if e0 == e1:
        return None
    slope = math.log(e1 / e0) / math.log(n1 / n0)
    return n0 * (err / e0) ** (1.0 / slope)


def summarise(rows, plain_photons, input_photons, batched=None) -> dict:
    """Errors (reference share removed in quadrature), the plain runs'
    error curve and time model T = a n + T0 over all plain photon counts
    (the low-photon runs are plain runs too), and for every input count the
    plain photon count of equal error and the time ratio of that plain run
    to the low-photon run plus inference.  `batched` (from batch_timing,
    covering every input count) adds the same ratios with per-volume times
    of batched launches."""
    ref = float(np.sqrt(np.mean([r["ref_err"] ** 2 for r in rows])))
    plain = float(np.sqrt(np.mean([r["plain_err"] ** 2 for r in rows])))
    plain_ms = float(np.mean([r["plain_ms"] for r in rows]))
    curve = [(float(plain_photons), _debias(plain, ref))]
    times = [(float(plain_photons), plain_ms)]
    per_n = []
    for j, n in enumerate(input_photons):
        den = float(np.sqrt(np.mean([r["inputs"][j]["denoised_err"] ** 2 for r in rows])))
        noisy = float(np.sqrt(np.mean([r["inputs"][j]["noisy_err"] ** 2 for r in rows])))
        sim_ms = float(np.mean([r["inputs"][j]["sim_ms"] for r in rows]))
        inf_ms = float(np.mean([r["inputs"][j]["infer_ms"] for r in rows]))
        curve.append((float(n), _debias(noisy, ref)))
        times.append((float(n), sim_ms))
        per_n.append({"photons": int(n), "noisy_err": noisy, "denoised_err": den,
                      "noisy_err_debiased": _debias(noisy, ref),
                      "denoised_err_debiased": _debias(den, ref), "sim_ms": sim_ms,
                      "infer_ms": inf_ms, "sim_plus_infer_ms": sim_ms + inf_ms})
    ns = np.array([t[0] for t in times])
    ts = np.array([t[1] for t in times])
    a, t0 = np.polyfit(ns, ts, 1)
    for r in per_n:
        neq = _equivalent_photons(curve, r["denoised_err_debiased"])
        r["equal_error_plain_photons"] = neq
        r["time_ratio"] = (a * neq + t0) / r["sim_plus_infer_ms"] if neq else None
    out = {"volumes": len(rows), "plain_photons": int(plain_photons), "plain_err": plain,
           "plain_err_debiased": _debias(plain, ref), "ref_err": ref, "plain_ms": plain_ms,
           "plain_time_model": {"ms_per_photon": float(a), "overhead_ms": float(t0)},
           "plain_error_curve": curve, "per_input": per_n, "equal_error_photons": None,
           "time_ratio": None, "best_time_ratio": None}
    ratios = [r["time_ratio"] for r in per_n if r["time_ratio"]]
    out["best_time_ratio"] = max(ratios) if ratios else None
    if batched:
        bn = np.array([b[0] for b in batched])
        bt = np.array([b[1] for b in batched])
        ab, t0b = np.polyfit(bn, bt, 1)
        per_vol = dict(batched)
        for r in per_n:
            lo = per_vol[float(r["photons"])]
            neq = r["equal_error_plain_photons"]
            r["batched_sim_ms"] = lo
            r["batched_time_ratio"] = (ab * neq + t0b) / (lo + r["infer_ms"]) if neq else None
        br = [r["batched_time_ratio"] for r in per_n if r["batched_time_ratio"]]
        out["batched"] = {"per_volume_ms": [list(b) for b in batched],
                          "time_model": {"ms_per_photon": float(ab), "overhead_ms": float(t0b)},
                          "best_time_ratio": max(br) if br else None}
    for r in per_n:
        if r["denoised_err_debiased"] <= out["plain_err_debiased"]:
            out["equal_error_photons"] = r["photons"]
            out["time_ratio"] = plain_ms / r["sim_plus_infer_ms"]
            break
    return out


def time_passes(den: nn.Denoiser, side: int, reps: int = 50, seed: int = 900001) -> dict:
    """Kernel time (HIP events on the current stream, mean over `reps`
    calls after three warm-up calls) of one forward pass, of the forward
    pass averaged over the 8 x-y symmetries, and of one loss-and-gradient
    pass (fused backward, and without the fusion), on the 1e6-photon map of
    a held-out volume (target: its 1e7-photon map)."""
    t = _torch()
    p = W.denoiser_volume(seed, side)
    x = t.as_tensor(simulate_one(p, 1e6, seed + 1)[0]).cuda()
    y = t.as_tensor(simulate_one(p, 1e7, seed + 2)[0]).cuda()
    out = t.empty_like(x)
    s = t.cuda.current_stream()

    def timed(fn, n):
        for _ in range(3):
            fn()
        t.cuda.synchronize()
        e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(n):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    r = {"forward_ms": timed(lambda: den.forward(x, phi_out=out, stream=s), reps),
         "forward_8_symmetries_ms": timed(
             lambda: den.forward(x, phi_out=out, stream=s, symmetries=8), max(1, reps // 4))}
    # the two backward modes alternately, twice each (clock drift over a
    # run otherwise favours whichever is timed second)
    times = {True: [], False: []}
    for fused in (False, True, True, False):
        den.set_fused_backward(fused)
        times[fused].append(timed(lambda: den.loss_grad(x, y, want_loss=False, stream=s), reps))
    den.set_fused_backward(True)
    r["loss_grad_ms"] = float(np.mean(times[True]))
    r["loss_grad_unfused_ms"] = float(np.mean(times[False]))
    return r


def main(argv=None) -> dict:
    """Command line: simulate a training set, train, evaluate; prints JSON.

        python -m paper_1711_03244_amd.denoise [--train 64] [--steps 20000]
            [--side 64] [--inputs 1e5,1e6,1e7] [--target 1e8] [--eval 2]
            [--plain 1e9] [--ref-runs 2] [--lr 1e-3] [--batch 4] [--max-norm 0.1]
            [--augment 1] [--batch-volumes 32] [--train-first 1] [--init CKPT]
            [--save CKPT]
        python -m paper_1711_03244_amd.denoise --time-passes CKPT
    """
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(prog="python -m paper_1711_03244_amd.denoise")
    ap.add_argument("--train", type=int, default=64)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--side", type=int, default=64)
    ap.add_argument("--inputs", default="1e5,1e6,1e7")
    ap.add_argument("--target", type=float, default=1e8)
    ap.add_argument("--eval", type=int, default=2)
    ap.add_argument("--plain", type=float, default=1e9)
    ap.add_argument("--ref-runs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--max-norm", type=float, default=0.1)
    ap.add_argument("--augment", type=int, default=1,
                    help="1: pass training pairs through random x-y symmetries")
    ap.add_argument("--batch-volumes", type=int, default=32,
                    help="volumes per batched launch in the batched timing (0 = none)")
    ap.add_argument("--train-first", type=int, default=1,
                    help="seed of the first training volume (volumes first .. first+train-1)")
    ap.add_argument("--init", default=None,
                    help="start from this inference checkpoint instead of the seeded weights")
    ap.add_argument("--save", default=None, help="write an inference checkpoint here")
    ap.add_argument("--time-passes", default=None, metavar="CHECKPOINT",
                    help="only time forward and loss-and-gradient passes of this inference "
                         "checkpoint (time_passes) and print them")
    a = ap.parse_args(argv)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)
    if a.time_passes:
        with nn.Denoiser(W.DENOISER_CHANNELS, (a.side,) * 3) as d:
            d.load_inference(a.time_passes)
            res = time_passes(d, a.side)
        print(json.dumps(res))
        return res
    inputs = [float(v) for v in a.inputs.split(",")]
    ch = W.DENOISER_CHANNELS
    t0 = time.perf_counter()
    seeds = range(a.train_first, a.train_first + a.train)
    ds = make_dataset(seeds, a.side, inputs, a.target, say=log)
    data_s = time.perf_counter() - t0
    with nn.Denoiser(ch, (a.side,) * 3) as d:
        history = []
        if a.init:
            history = d.load_inference(a.init).get("history", [])
        else:
            d.set_params(W.denoiser_weights(ch, seed=1))
        tr = train(d, ds, a.steps, lr=a.lr, log_every=max(1, a.steps // 5), batch=a.batch,
                   max_norm=a.max_norm, augment=bool(a.augment), say=log)
        if a.save:
            stage = {"command": "python -m paper_1711_03244_amd.denoise " + " ".join(
                         argv if argv is not None else sys.argv[1:]),
                     "train_volume_seeds": [seeds.start, seeds.stop - 1], "inputs": inputs,
                     "target": a.target, "steps": a.steps, "batch": a.batch, "lr": a.lr,
                     "max_norm": a.max_norm, "augment": bool(a.augment),
                     "data_s": data_s, "train_s": tr["seconds"],
                     "final_loss": tr["losses"][-1][1] if tr["losses"] else None}
            d.save_inference(a.save, {"channels": list(ch), "side": a.side,
                                      "history": history + [stage]})
            log(f"[save] {a.save}")
        ev = evaluate(d, range(900001, 900001 + a.eval), a.side, a.plain, a.ref_runs, inputs,
                      say=log, batch_seeds=range(800001, 800001 + a.batch_volumes)) \
            if a.eval > 0 else None
    out = {"channels": list(ch), "side": a.side, "train_volumes": a.train, "inputs": inputs,
           "target": a.target, "data_s": data_s, "train_steps": a.steps, "augment": bool(a.augment),
           "train_s": tr["seconds"], "losses": tr["losses"], "evaluation": ev}
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
