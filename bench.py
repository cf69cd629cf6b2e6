"""Throughput benchmark of the photon-transport hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--photons N]
                    [--launch BLOCK,CHUNK,WINDOW[,ADDS]] [--head-launch BLOCK,CHUNK,WINDOW[,ADDS]]
                    [--no-cpu-baseline] [--head-photons M] [--no-head] [--no-batch]
                    [--no-denoise] [--no-scaling]

Workload: the paper's heterogeneous cube benchmark as configured here -- a
60 x 60 x 60 grid of 1 mm voxels, background mua 0.005/mm, mus 1.0/mm,
g 0.01, n 1.37 and a centred 15 mm sphere with mua 0.002/mm, mus 5.0/mm,
g 0.9, n 1.37, Fresnel boundaries, pencil beam at (29.5, 29.5, 0) along +z,
50 gates of 0.1 ns and four 1 mm disk detectors, 1e8 photons per step.
Inputs are synthetic (the phantom is generated, not read).  A step is one
full pass of the path: clear, transport (launch, free paths, hops, deposits,
scattering, boundaries, roulette, detection, ledger), FP64 reductions and
normalisation of the map into a device tensor.  Problem creation and upload
(the paper's host overhead) happen once, before the timed region.

Prints one JSON line.  `roofline` is the ceiling that binds the transport
kernel -- the memory-side FP64 atomic rate (measured peak) on this workload --
with the other one (FP32 VALU, the method's per-event operation count over
the kernel's HIP-event time) attached, and the kernel's HBM traffic against
its algorithmic bytes; `cpu_baseline` the FP64 oracle on the host cores
available to this process over a prefix of the same photons, best of 3.  The launch shape of the timed steps is the one the library's
autotuner picks (before the timed region) from pilot launches of 1/20 of the
photons, with the kind of map add decided by one untimed full-size run of
each; the rate of the default shape is reported beside it.  Two further workloads are reported beside the main one, each
timed once after a warm-up launch: `head_volume` (the seeded 181 x 217 x
181 layered head phantom, 10 gates of 0.5 ns, 1e8 photons) and `batched`
(256 generated cubes of 32-128 mm with 1-3 inclusions and 1e5-1e7 photons
each, 5.4e8 photons in one launch, with the fixed launch shape -- 64-thread
workgroups, one photon per lane per job, direct atomics -- and with the
shape the autotuner picks from pilot launches of 1/50 of the photons).
The batch leg also fits the paper's device model per simulation from
pilots of 1e6 and 5e6 photons and reruns the batch with home waves spread
by the estimated work a_i n_i (the paper's throughput partition S2) instead
of job counts.  `photon_scaling` runs the sphere benchmark at 1e6 .. 1e9
photons and fits the device model T = a n + T0.  `ablations` times the
paper's benchmark variants of the event loop (non-atomic deposits, B2;
branch-reduced loop, Opt3) against the default loop at 3e7 photons.
`denoiser` evaluates the 3-D U-Net of the committed inference checkpoint
(trained on simulator pairs of 64^3 volumes with 1e9-photon targets; the
file records how) on 16 held-out volumes: the error of denoised 5e7, 7e7,
8e7 and 9e7-photon maps (each the mean, in log space, of the network's
outputs for the 8 x-y symmetries of the input) against the error of a
plain 1e9-photon run, and the wall-time ratio at equal error (see
denoise.evaluate_strict).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photons/ms at 60³ & head volume; time-to-equal-error denoised vs plain MC"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--photons", type=int, default=100_000_000)
    ap.add_argument("--cpu-photons", type=int, default=2_000_000,
                    help="photons per CPU-baseline run (3 runs, best kept)")
    ap.add_argument("--launch", default=None, metavar="BLOCK,CHUNK,WINDOW[,ADDS]",
                    help="fix the transport launch shape and optionally the map adds "
                         "(1: 64-bit, 2: 32-bit with carry; default automatic); skips the "
                         "autotuner and the default-shape context run, e.g. for profiling")
    ap.add_argument("--head-launch", default=None, metavar="BLOCK,CHUNK,WINDOW[,ADDS]",
                    help="the same for the head-volume leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--head-photons", type=int, default=100_000_000)
    ap.add_argument("--no-head", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-denoise", action="store_true")
    ap.add_argument("--no-scaling", action="store_true")
    ap.add_argument("--no-ablations", action="store_true")
    ap.add_argument("--dn-train", type=int, default=64, help="denoiser training volumes")
    ap.add_argument("--dn-steps", type=int, default=20000, help="denoiser training steps")
    ap.add_argument("--dn-batch", type=int, default=4, help="volumes per training step")
    ap.add_argument("--dn-clip", type=float, default=0.1, help="gradient-norm clip")
    ap.add_argument("--dn-target", type=float, default=1e8, help="target photons per volume")
    ap.add_argument("--dn-eval", type=int, default=2, help="held-out volumes")
    ap.add_argument("--dn-plain", type=float, default=1e9, help="plain-run photons")
    ap.add_argument("--dn-ref-runs", type=int, default=2, help="reference runs per volume")
    ap.add_argument("--dn-augment", type=int, default=1,
                    help="1: random x-y symmetries of the training pairs")
    ap.add_argument("--dn-batch-volumes", type=int, default=32,
                    help="volumes per batched launch in the denoiser's batched timing")
    ap.add_argument("--dn-checkpoint", default=CHECKPOINT,
                    help="inference checkpoint evaluated by the denoiser leg")
    ap.add_argument("--dn-train-in-bench", action="store_true",
                    help="train the denoiser in the bench instead of loading the checkpoint")
    ap.add_argument("--dn-eval-strict", type=int, default=16,
                    help="held-out volumes of the checkpoint's evaluation")
    ap.add_argument("--dn-inputs", default="5e7,7e7,8e7,9e7",
                    help="low-photon counts of the checkpoint's evaluation")
    ap.add_argument("--dn-symmetries", type=int, default=8,
                    help="x-y symmetries averaged at inference (1, 2, 4 or 8)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the transport runs on a single MI355X "
              "(photons would shard across GPUs by index range; no multi-GPU launch is "
              "provided); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_03244_amd import mcx, roofline, workloads as W
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)

    p = W.cube_sphere()
    N = args.photons
    t_create = time.perf_counter()
    sim = mcx.Simulation(p)
    create_ms = (time.perf_counter() - t_create) * 1e3
    out = torch.empty(p.tally_shape, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    if args.launch:
        blk, chunk, win, *adds = (int(v) for v in args.launch.split(","))
        if win > 0:  # the window boxes the autotuner would shape for this size
            sim.shape_window(max(1000, N // 20), args.seed + 3000, win)
        sim.set_launch(blk, chunk, win)
        sim.set_map_adds(adds[0] if adds else mcx.MAP_ADDS_AUTO)
        default_rate = None
        tune = {"refill_chunk": chunk, "lds_window_cells": win}
        chosen_by = "--launch"
    else:
        # the library's default launch shape, for context, then the shape the
        # autotuner picks from pilot launches of N/20 photons (kept for the
        # steps; shorter pilots overweight the end-of-launch window flush)
        sim.run(N // 100, args.seed + 2000)
        sim.run(N, args.seed + 2001)
        default_rate = N / sim.stats()["kernel_ms"]
        t_tune = time.perf_counter()
        tune = sim.autotune(max(1000, N // 20), args.seed + 3000)
        adds_note = map_adds_at_full_size(mcx, sim, N, args.seed + 4000)
        chosen_by = (f"autotuner, {tune['candidates']} shapes, pilots of {N // 20} photons, "
                     f"{time.perf_counter() - t_tune:.1f} s before the timed steps; {adds_note}")

    def step(i):
        mcx.mcx_reset(sim.ctx)
        mcx.mcx_run_range(sim.ctx, 0, N, args.seed + i)
        mcx.mcx_fluence_device(sim.ctx, mcx.MCX_FLUENCE_RATE, out)
        return sim.stats()  # waits for the context's stream

    log("launch shape:", chosen_by)
    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    kernel_ms, stats = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = step(i)
        kernel_ms.append(st["kernel_ms"])
        stats.append(st)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ms_per_step = wall_ms / args.steps
    value = N * args.steps / wall_ms

    last = stats[-1]
    ksec = sum(kernel_ms) / len(kernel_ms) / 1e3
    roof = roofline.binding(last, ksec)
    roof["traffic"] = roofline.measured_traffic(
        N, {"block_size": last["block_size"], "refill_chunk": tune["refill_chunk"],
            "lds_window_cells": tune["lds_window_cells"], "map_adds": last["map_adds"]})
    roof["traffic_over_algorithmic"] = (roof["traffic"] / roof["algorithmic_bytes"]
                                        if roof["traffic"] else None)
    log(f"timed steps: {value:.1f} photons/ms")
    scaling = None if args.no_scaling else scaling_leg(sim, args.seed)
    shape = (last["block_size"], tune["refill_chunk"], tune["lds_window_cells"])
    sim.close()
    log("ablations")
    ablations = None if args.no_ablations else ablation_leg(mcx, W, shape, args.seed)
    log("homogeneous cube and head volume")

    cube1 = None if args.no_head else cube1_leg(mcx, W)
    head = None if args.no_head else head_leg(mcx, roofline, W, args.head_photons, args.seed,
                                              args.head_launch)
    log("batched workload")
    batched = None if args.no_batch else batch_leg(mcx, W)
    log("denoiser")
    denoised = None if args.no_denoise else denoise_leg(args)

    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        log("CPU baseline")
        cpu, cpu1 = cpu_baseline(p, args.cpu_photons, args.seed)

    ks = sorted(kernel_ms)
    line = {
        "metric": METRIC, "value": value, "unit": "photons/ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cube60_sphere_b2a", "grid": [60, 60, 60], "voxel_mm": 1.0,
                   "photons_per_step": N, "gates": 50, "gate_ns": 0.1, "detectors": 4,
                   "reflect": True, "seed": args.seed, "tally": "u64 deposit units"},
        "kernel_ms_per_step": sum(kernel_ms) / len(kernel_ms),
        "kernel_photons_per_ms": N / (sum(kernel_ms) / len(kernel_ms)),
        "kernel_photons_per_ms_best": N / ks[0],
        "kernel_photons_per_ms_median": N / ks[len(ks) // 2],
        "kernel_photons_per_ms_default_launch": default_rate,
        "launch": {"block_size": last["block_size"], "grid_blocks": last["grid_blocks"],
                   "refill_chunk": tune["refill_chunk"],
                   "lds_window_cells": tune["lds_window_cells"],
                   "map_adds": {1: "64-bit", 2: "32-bit with carry"}[last["map_adds"]],
                   "chosen_by": chosen_by},
        "create_ms": create_ms,
        "events_per_photon": last["events"] / N,
        "lane_utilisation": last["events"] / max(1, last["lane_slots"]),
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_single_thread": cpu1,
        "photon_scaling": scaling,
        "homogeneous_cube": cube1,
        "head_volume": head,
        "batched": batched,
        "ablations": ablations,
        "denoiser": denoised,
    }
    print(json.dumps(line), flush=True)


def _sha16(path) -> str:
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def host_cpu() -> dict:
    """The host's CPU model, its logical CPU count, the CPUs this process may
    run on and the cgroup's CPU quota (in CPUs), as far as they are readable."""
    info = {"model": None, "nproc": os.cpu_count(), "affinity": None, "cgroup_quota": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
        if q != "max":
            info["cgroup_quota"] = float(q) / float(per)
    except (OSError, ValueError):
        pass
    return info


def cpu_baseline(p, n, seed):
    """The FP64 oracle, as it stands, on every CPU this process may use (the
    affinity set, capped by the cgroup quota), 3 runs of photons [0, n) of
    the same workload and seed, best kept; and on one thread over n/16
    photons, best of 3."""
    import math
    import oracle
    cpu = host_cpu()
    cores = cpu["affinity"] or cpu["nproc"] or 1
    if cpu["cgroup_quota"]:
        cores = max(1, min(cores, int(math.ceil(cpu["cgroup_quota"]))))
    walls = [oracle.run(p, n, seed, nthreads=cores)["wall_s"] for _ in range(3)]
    n1 = max(1, n // 16)
    walls1 = [oracle.run(p, n1, seed, nthreads=1)["wall_s"] for _ in range(3)]
    best = {"value": n / (min(walls) * 1e3), "unit": "photons/ms", "cores": cores,
            "kind": "oracle",
            "sample": f"photons 0..{n - 1} of the same workload and seed, FP64, {cores} threads, "
                      f"best of 3 runs ({', '.join(f'{w:.2f}' for w in walls)} s)",
            "median": n / (sorted(walls)[1] * 1e3), "host": cpu}
    one = {"value": n1 / (min(walls1) * 1e3), "unit": "photons/ms", "cores": 1, "kind": "oracle",
           "sample": f"photons 0..{n1 - 1}, one thread, best of 3 runs "
                     f"({', '.join(f'{w:.2f}' for w in walls1)} s)"}
    return best, one


def scaling_leg(sim, seed):
    """The sphere benchmark at 1e6 .. 1e9 photons with the timed steps'
    launch shape: run time (clear + transport + reductions, HIP events)
    against photons, and the paper's device model T = a n + T0 fitted to
    it (the study of its Fig. 3(b))."""
    import numpy as np
    counts = [1_000_000, 10_000_000, 100_000_000, 1_000_000_000]
    kernel, run = [], []
    for n in counts:
        sim.run(n, seed + 5000)
        st = sim.stats()
        kernel.append(st["kernel_ms"])
        run.append(st["run_ms"])
    a, t0 = np.polyfit(np.array(counts, float), np.array(run), 1)
    return {"photons": counts, "kernel_ms": kernel, "run_ms": run,
            "photons_per_ms": [n / t for n, t in zip(counts, run)],
            "model": {"ms_per_photon": float(a), "overhead_ms": float(t0)}}


def best_median(mcx, sim, N, seeds):
    """Kernel-time photons/ms of one run per seed: best and median (the
    paper reports the best of three runs)."""
    rates, stats = [], []
    for sd in seeds:
        sim.run(N, sd)
        st = sim.stats()
        stats.append(st)
        rates.append(N / st["kernel_ms"])
    r = sorted(rates)
    return r[-1], r[len(r) // 2], stats


def cube1_leg(mcx, W):
    """The homogeneous 60^3 cube at 1e8 photons, seeds 1-3; plus, for
    context, 1e7 photons with the paper's baseline launch of 2^14 threads
    in 64-thread workgroups."""
    p = W.cube_homogeneous()
    N = 100_000_000
    with mcx.Simulation(p) as sim:
        sim.run(N // 100, 99)
        best, med, st = best_median(mcx, sim, N, [1, 2, 3])
    with mcx.Simulation(p, block_size=64, blocks_per_cu=1, lds_window_cells=-1) as sim:
        sim.run(100_000, 99)
        sim.run(N // 10, 1)
        base = sim.stats()
    return {"workload": "cube60_homogeneous", "photons": N, "photons_per_ms_best": best,
            "photons_per_ms_median": med, "events_per_photon": st[-1]["events"] / N,
            "paper_baseline_launch": {"threads": base["grid_blocks"] * base["block_size"],
                                      "block_size": base["block_size"], "photons": N // 10,
                                      "photons_per_ms": (N // 10) / base["kernel_ms"]}}


def map_adds_at_full_size(mcx, sim, N, seed):
    """The kind of map add for the timed runs, from one untimed run of N
    photons with each kind at the tuned shape: on the autotuner's short
    pilots the two kinds come within timing noise of each other, at full
    size they do not (sphere: 32-bit adds ahead; head phantom: 64-bit)."""
    ms = {}
    for kind in (mcx.MAP_ADDS_32, mcx.MAP_ADDS_64):
        sim.set_map_adds(kind)
        sim.run(N, seed)
        ms[kind] = sim.stats()["kernel_ms"]
    kind = min(ms, key=ms.get)
    sim.set_map_adds(kind)
    return (f"map adds from one full-size run of each kind: 32-bit {ms[mcx.MAP_ADDS_32]:.1f} ms, "
            f"64-bit {ms[mcx.MAP_ADDS_64]:.1f} ms")


def head_leg(mcx, roofline, W, N, seed, launch=None):
    p = W.head_phantom(1)
    with mcx.Simulation(p) as sim:
        if launch:
            blk, chunk, win, *adds = (int(v) for v in launch.split(","))
            if win > 0:
                sim.shape_window(max(1000, N // 50), seed + 3000, win)
            sim.set_launch(blk, chunk, win)
            sim.set_map_adds(adds[0] if adds else mcx.MAP_ADDS_AUTO)
            default_med, tune = None, {"refill_chunk": chunk, "lds_window_cells": win}
            sim.run(N // 100, seed + 1000)  # warm-up
        else:
            sim.run(N // 100, seed + 1000)  # warm-up
            _, default_med, _ = best_median(mcx, sim, N, [seed, seed + 1, seed + 2])
            tune = sim.autotune(max(1000, N // 50), seed + 3000)
            map_adds_at_full_size(mcx, sim, N, seed + 4000)
        best, med, runs = best_median(mcx, sim, N, [seed, seed + 1, seed + 2])
        st = runs[0]
    ksec = st["kernel_ms"] / 1e3
    return {"workload": "head_1", "grid": [181, 217, 181], "gates": 10, "gate_ns": 0.5,
            "photons": N, "photons_per_ms": N / st["run_ms"], "photons_per_ms_best": best,
            "photons_per_ms_median": med, "photons_per_ms_median_default_launch": default_med,
            "launch": {"block_size": st["block_size"], "refill_chunk": tune["refill_chunk"],
                       "lds_window_cells": tune["lds_window_cells"],
                       "map_adds": {1: "64-bit", 2: "32-bit with carry"}[st["map_adds"]]},
            "kernel_ms": st["kernel_ms"],
            "run_ms": st["run_ms"], "events_per_photon": st["events"] / N,
            "roofline": roofline.binding(st, ksec)}


def ablation_leg(mcx, W, shape, seed, N=30_000_000):
    """The paper's benchmark study (Fig. 2) on this chip: the event-loop
    variants at the timed steps' launch shape on the sphere benchmark --
    default loop, non-atomic map deposits (B2; the weight the races lose is
    reported against the atomic run of the same photons), branch-reduced
    loop (Opt3) -- and default vs branch-reduced on the head phantom with
    the library's default shape.  Kernel-time photons/ms, best of 2 seeds."""
    out = {"photons": N}

    def rates(p, variant, launch=None):
        with mcx.Simulation(p, kernel_variant=variant) as sim:
            if launch:
                sim.set_launch(*launch)
            sim.run(N // 30, seed + 7000)  # warm-up
            best, _, st = best_median(mcx, sim, N, [seed + 7001, seed + 7002])
        return best, st[0]

    p = W.cube_sphere()
    d, st_d = rates(p, 0, shape)
    r, st_r = rates(p, 1, shape)
    f, _ = rates(p, 2, shape)
    out["sphere"] = {"launch": list(shape), "default": d, "non_atomic_b2": r,
                     "branch_reduced_opt3": f,
                     "atomic_overhead": d and (r / d - 1.0),
                     "non_atomic_weight_lost": 1.0 - st_r["absorbed_grid"] / st_d["absorbed_grid"]}
    h = W.head_phantom(1)
    hd, _ = rates(h, 0)
    hf, _ = rates(h, 2)
    out["head"] = {"launch": "library default", "default": hd, "branch_reduced_opt3": hf}
    return out


def batch_leg(mcx, W):
    items = W.batch_workload()
    n = [it.nphoton for it in items]
    seeds = [it.seed for it in items]
    total = sum(n)
    out = {"workload": "batch_256_cubes", "simulations": len(items), "photons": total,
           "sides": list(W.BATCH_SIDES), "seed": 1}
    with mcx.Batch([it.problem for it in items]) as b:
        def timed(label):
            b.run([max(1, x // 100) for x in n], [s + 1 for s in seeds])  # warm-up
            b.run(n, seeds)
            st = b.stats(0)
            out[label] = {"photons_per_ms": total / st["run_ms"], "run_ms": st["run_ms"],
                          "kernel_ms": st["kernel_ms"], "block_size": st["block_size"],
                          "grid_blocks": st["grid_blocks"],
                          "map_adds": {1: "64-bit", 2: "32-bit with carry"}[st["map_adds"]]}
        b.set_launch(64, 64, -1)
        b.set_map_adds(mcx.MAP_ADDS_64)  # the fixed baseline: plain 64-bit atomic adds
        timed("fixed")
        out["fixed"]["refill_chunk"] = 64
        t0 = time.perf_counter()
        tune = b.autotune([max(1000, x // 50) for x in n], seeds)
        out["autotune_s"] = time.perf_counter() - t0
        timed("autotuned")
        out["autotuned"]["refill_chunk"] = tune["refill_chunk"]
        out["autotune"] = tune
        # the paper's device model per simulation from pilots of 1e6 and 5e6
        # photons, then home waves in proportion to a_i n_i (its throughput
        # partition S2) instead of job counts, same launch shape
        t0 = time.perf_counter()
        a, t_over = b.fit_runtime(seed=[s + 11 for s in seeds])
        out["fit_s"] = time.perf_counter() - t0
        b.set_balance(a)
        timed("autotuned_s2")
        b.set_balance(None)
        out["runtime_model"] = {"pilots": [1_000_000, 5_000_000],
                                "ms_per_photon_min": float(min(a)),
                                "ms_per_photon_max": float(max(a)),
                                "overhead_ms_median": float(sorted(t_over)[len(t_over) // 2])}
    out["speedup"] = out["autotuned"]["photons_per_ms"] / out["fixed"]["photons_per_ms"]
    out["s2_over_job_counts"] = (out["autotuned_s2"]["photons_per_ms"]
                                 / out["autotuned"]["photons_per_ms"])
    return out


CHECKPOINT = os.path.join(ROOT, "paper_1711_03244_amd", "checkpoints", "denoiser_64cube.npz")


def denoise_leg(args):
    """Time-to-equal-error of the denoiser: the network of the committed
    inference checkpoint (trained by `python -m paper_1711_03244_amd.denoise`
    on simulator pairs with 1e9-photon targets; its provenance is in the
    file and in the line) on held-out volumes against the plain 1e9-photon
    run (denoise.evaluate_strict).  With --dn-train-in-bench, or without
    the checkpoint, the network is trained here instead on the smaller
    configuration below and evaluated by denoise.evaluate."""
    from paper_1711_03244_amd import denoise, nn, workloads as W
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    side = 64
    ch = W.DENOISER_CHANNELS
    if os.path.exists(args.dn_checkpoint) and not args.dn_train_in_bench:
        inputs = [float(v) for v in args.dn_inputs.split(",")]
        with nn.Denoiser(ch, (side, side, side)) as d:
            meta = d.load_inference(args.dn_checkpoint)
            ev = denoise.evaluate_strict(d, range(900001, 900001 + args.dn_eval_strict), side,
                                         inputs, plain_photons=args.dn_plain, ref_runs=2,
                                         say=log, symmetries=args.dn_symmetries)
        return {"workload": "denoise_64cubes", "channels": list(ch), "side": side,
                "checkpoint": os.path.relpath(args.dn_checkpoint, ROOT),
                "checkpoint_sha256_16": _sha16(args.dn_checkpoint),
                "training": meta.get("history"), "held_out_seeds": [900001,
                                                                     900000 + args.dn_eval_strict],
                **ev}
    t0 = time.perf_counter()
    inputs = [1e5, 1e6, 1e7]
    ds = denoise.make_dataset(range(1, args.dn_train + 1), side, inputs, args.dn_target, say=log)
    data_s = time.perf_counter() - t0
    with nn.Denoiser(ch, (side, side, side)) as d:
        d.set_params(W.denoiser_weights(ch, seed=1))
        tr = denoise.train(d, ds, args.dn_steps, lr=1e-3, log_every=max(1, args.dn_steps // 5),
                           batch=args.dn_batch, max_norm=args.dn_clip,
                           augment=bool(args.dn_augment), say=log)
        ev = denoise.evaluate(d, range(900001, 900001 + args.dn_eval), side, args.dn_plain,
                              args.dn_ref_runs, inputs, say=log,
                              batch_seeds=range(800001, 800001 + args.dn_batch_volumes))
    del ds
    return {"workload": "denoise_64cubes", "channels": list(ch), "side": side,
            "train_volumes": args.dn_train, "train_inputs": inputs, "train_target": args.dn_target,
            "data_s": data_s, "train_steps": tr["steps"], "train_batch": tr["batch"],
            "train_clip": tr["max_norm"], "train_augment": tr["augment"], "train_s": tr["seconds"],
            "final_loss": tr["losses"][-1][1] if tr["losses"] else None, **ev}


if __name__ == "__main__":
    main()
