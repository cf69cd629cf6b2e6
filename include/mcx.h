/*
 * mcx.h -- C ABI of the MI355X voxel Monte Carlo photon-transport library
 * (libmcx.so, HIP for gfx950).
 *
 * What the library computes is the paper's per-thread photon simulation
 * (Yu, Nina-Paravecino, Kaeli and Fang, "Scalable and massively parallel
 * Monte Carlo photon transport simulations for heterogeneous computing
 * platforms"): from domain settings, optical properties, a source,
 * detectors and random seeds (the problem statement before Fig. 1) it
 * produces 3-D time-resolved fluence maps and detected-photon data, then
 * post-processes them.  The benchmark domains of the paper's Fig. 2
 * experiments (60 mm cube, optional 15 mm sphere, pencil beam, Fresnel
 * boundaries, atomic deposits) are expressible directly.
 *
 * Conventions shared by every entry point:
 *  - Units: mm, 1/mm, ns.  Coordinates start at the grid corner; voxel
 *    (i, j, k) covers [i, i+1) x [j, j+1) x [k, k+1) voxel edges.
 *  - Volumes and fluence maps are x-fastest: cell = i + nx*(j + ny*k); a
 *    fluence map is [gate][k][j][i], ngates*nx*ny*nz cells.
 *  - Ownership: inputs are deep-copied by mcx_create; the caller may free
 *    them on return.  Outputs go to caller-owned buffers whose capacity is
 *    passed in; the library never frees caller memory.  Pointers named
 *    `host_*` are host memory, pointers named `dev_*` are device memory on
 *    the context's device.
 *  - Errors: every call returns an mcx_status and never throws.  On error
 *    mcx_last_error() (thread-local) describes it.  Argument validation
 *    happens before any HIP call, so invalid input is reported without a
 *    GPU.  A context is used by one host thread at a time.
 *  - Random numbers: photon k of a run with seed S draws from the
 *    counter-based Philox4x32-10 generator with key (S mod 2^32, S div 2^32)
 *    and counter (k mod 2^32, k div 2^32, b, 0); block b = 0 launches the
 *    photon and each scattering event or Fresnel test takes the next b.  A
 *    run over photons [first, first+n) therefore produces exactly the same
 *    photons however it is split or scheduled.
 */
#ifndef MCX_H
#define MCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcx_ctx mcx_ctx; /* opaque; owns all of its device memory */

typedef enum {
  MCX_OK = 0,
  MCX_EINVAL = -1,  /* invalid argument; nothing was changed */
  MCX_ENOMEM = -2,  /* host or device allocation failed */
  MCX_ENODEV = -3,  /* no usable HIP device */
  MCX_EDEVICE = -4, /* a HIP call failed; the context should be destroyed */
  MCX_ESTATE = -5,  /* call not valid in the context's current state */
  MCX_ERANGE = -6   /* caller buffer too small */
} mcx_status;

/* Optical properties of one medium: absorption and scattering coefficients
 * (1/mm), Henyey-Greenstein anisotropy g in [-1, 1], refractive index >= 1. */
typedef struct {
  float mua, mus, g, n;
} mcx_medium;

/* Voxelised domain.  labels[nx*ny*nz] holds medium indices into media[];
 * label 0 is the outside (its media row is ignored), so nmedia counts the
 * outside row too (2 <= nmedia <= 256). */
typedef struct {
  int32_t nx, ny, nz;
  float voxel_mm;
  const uint8_t *labels;
  const mcx_medium *media;
  int32_t nmedia;
} mcx_volume;

/* Pencil beam: start point (mm, inside a voxel with label != 0) and unit
 * direction (|dir| within 1e-5 of 1). */
typedef struct {
  float pos[3];
  float dir[3];
} mcx_source;

/* Disk detector: an escaping photon whose exit point lies within `radius`
 * (mm) of `pos` is recorded (first detector in index order wins). */
typedef struct {
  float pos[3];
  float radius;
} mcx_detector;

/* Time gates: ngates gates of width dt_ns starting at t0_ns; photons start at
 * t0_ns and end at t0_ns + ngates*dt_ns. */
typedef struct {
  float t0_ns;
  float dt_ns;
  int32_t ngates;
} mcx_gates;

/* Options; fill with mcx_default_options() then override. */
typedef struct {
  int32_t reflect;        /* 1: Fresnel reflect/refract where n changes, incl. at escape */
  float n_outside;        /* refractive index of label 0 and off-grid (default 1.0) */
  float rr_threshold;     /* Russian roulette when w < this after a scattering (1e-4) */
  float rr_m;             /* roulette: survive with probability 1/M, w *= M (10) */
  uint64_t max_detected;  /* detected-photon record capacity (default 1<<20) */
  uint64_t max_events;    /* per-photon segment cap, a safety stop (default 1e8) */
  int32_t device;         /* HIP device ordinal (default 0) */
  int32_t block_size;     /* threads per workgroup, multiple of 64; 0 = library default */
  int32_t blocks_per_cu;  /* resident workgroups per compute unit; 0 = occupancy maximum */
  int32_t refill_chunk;   /* photons a wave takes per refill grab; 0 = library default */
  uint64_t ndigest;       /* per-photon digest rows kept for photons [first, first+ndigest) */
  int32_t lds_window_cells; /* cells around the source summed per workgroup in LDS before they
                               reach the map (32-bit integer sums of deposit units, 4 bytes
                               each); 0 =
                               library default (16384), < 0 = none, at most 36864
                               (144 KB) */
  int32_t accurate_math;  /* 0: hardware transcendentals (~1 ulp); 1: device math library */
  int32_t kernel_variant; /* event loop (the paper's benchmark study, Fig. 2): 0 = default;
                             1 = map deposits by a plain, non-atomic read-add-write (the
                             paper's B2: concurrent updates of one cell can be lost, for
                             speed studies only; needs accurate_math = 0 and ndigest = 0);
                             2 = branch-reduced loop (the paper's Opt3: every lane computes
                             the scattering and the face-crossing updates and keeps its own
                             by selection; same results as 0; needs accurate_math = 0) */
} mcx_options;

/* Run statistics, accumulated since the last mcx_reset / mcx_run. */
typedef struct {
  uint64_t launched, escaped, detected, timeout, rr_dead, capped;
  uint64_t scatters, face_events, fresnel_draws, reflections, rr_tests, rr_survived;
  uint64_t events;          /* segments simulated (lane iterations with a live photon) */
  uint64_t lane_slots;      /* wave iterations x 64 (events / lane_slots = lane utilisation) */
  uint64_t flushes;         /* cell visits added to the map by a global atomic (not via LDS) */
  uint64_t det_records;     /* records written (<= max_detected) */
  uint64_t det_dropped;     /* detected photons without room for a record */
  double w_launched, w_escaped, w_detected, w_timeout, w_rr_gain, w_rr_loss, w_capped;
  double tally_sum;         /* FP64 sum of all raw tally cells (weight*mm) */
  double absorbed_grid;     /* FP64 sum of mua(voxel)*tally, i.e. absorbed weight */
  double kernel_ms;         /* transport kernel time of the last run (HIP events) */
  double run_ms;            /* whole last run: clear + transport + reductions */
  int32_t grid_blocks, block_size;
  int32_t map_adds;         /* MCX_MAP_ADDS_64 or MCX_MAP_ADDS_32: the last launch's map adds */
  int32_t reserved;
} mcx_run_stats;

/* One simulation of a batch (mcx_batch_create): everything mcx_create takes
 * for one problem, with the boundary settings per simulation. */
typedef struct {
  mcx_volume vol;
  mcx_source src;
  const mcx_detector *det; /* may be NULL when ndet == 0 */
  int32_t ndet;
  mcx_gates gates;
  int32_t reflect;         /* Fresnel reflect/refract where n changes */
  float n_outside;         /* refractive index of label 0 and off-grid */
} mcx_sim;

/* Result of mcx_autotune. */
typedef struct {
  int32_t block_size;       /* chosen threads per workgroup */
  int32_t refill_chunk;     /* chosen photons per job */
  int32_t lds_window_cells; /* chosen LDS window (-1 = none) */
  int32_t candidates;       /* launch shapes timed */
  double default_ms;        /* pilot kernel time with the default shape */
  double best_ms;           /* pilot kernel time with the chosen shape */
  double ms_per_photon;     /* slope a of T = a n + T0 fitted from two pilot sizes */
  double overhead_ms;       /* intercept T0 of that fit */
  int32_t map_adds;         /* chosen MCX_MAP_ADDS_64 or MCX_MAP_ADDS_32 */
  int32_t reserved;
} mcx_tune_result;

/* How the transport kernel adds to the map (mcx_set_map_adds): the atomic
 * accumulation of absorbed weight into the fluence map (the paper's
 * benchmark B2a, whose atomic operations its B2 variant removes, Fig. 2).
 * The map holds one 64-bit integer per cell: the count of deposit units u (a power
 * of two, 2^-20 of the voxel size or just below) the cell received; every
 * cell-visit sum is rounded to whole units, so sums are exact and results
 * do not depend on the order of the additions.  MCX_MAP_ADDS_64: one 64-bit
 * atomic add per visit.  MCX_MAP_ADDS_32: a 32-bit atomic add to the low
 * word whose returned value tells whether it carried into the high word
 * (then one more add); faster at the memory side, but the wave waits for
 * the returned value.  MCX_MAP_ADDS_AUTO: 32-bit adds when at least 16
 * waves per compute unit are resident.  The maps are bit-identical. */
enum { MCX_MAP_ADDS_AUTO = 0, MCX_MAP_ADDS_64 = 1, MCX_MAP_ADDS_32 = 2 };

/* Output kinds for mcx_fluence*. */
enum {
  MCX_RAW = 0,          /* weight*mm deposited per cell */
  MCX_FLUENCE = 1,      /* per launched photon, 1/mm^2: raw / (N h^3) */
  MCX_FLUENCE_RATE = 2  /* per launched photon, 1/(mm^2 ns): fluence / dt */
};

void mcx_default_options(mcx_options *opt);

/* Validate and deep-copy the problem, pick the device, allocate the tally
 * (one 64-bit count of deposit units per cell, 8 bytes) and upload.
 * `det` may be NULL when ndet == 0; `opt` may be NULL for defaults.
 * Errors: MCX_EINVAL (bad argument, message says which), MCX_ENODEV,
 * MCX_ENOMEM, MCX_EDEVICE.  *out is set only on MCX_OK. */
mcx_status mcx_create(const mcx_volume *vol, const mcx_source *src, const mcx_detector *det,
                      int32_t ndet, const mcx_gates *gates, const mcx_options *opt,
                      mcx_ctx **out);

/* Many independent simulations in one context, served by one persistent
 * launch per run (each wave works on one simulation at a time and moves on
 * when its lanes are done), as in the batched workload of the project (256
 * cubes of different sizes and photon counts).  Validation, ownership and
 * errors as for mcx_create; simulation i's messages are prefixed with its
 * index.  The single-simulation calls below act on simulation 0, and
 * mcx_run / mcx_run_range run every simulation of the context with the same
 * photon range and seed. */
mcx_status mcx_batch_create(const mcx_sim *sims, int32_t nsims, const mcx_options *opt,
                            mcx_ctx **out);
int32_t mcx_batch_size(const mcx_ctx *ctx);
uint64_t mcx_batch_ncells(const mcx_ctx *ctx, int32_t sim);

/* Clear, then run photons [0, nphoton[i]) of simulation i with seed[i], all
 * in one launch (split only past 2^31 photons per simulation); blocking. */
mcx_status mcx_batch_run(mcx_ctx *ctx, const uint64_t *nphoton, const uint64_t *seed);

/* Enqueue photons [first[i], first[i] + n[i]) (first may be NULL for 0) of
 * every simulation with seed[i] on hip_stream, accumulating; async. */
mcx_status mcx_batch_run_range(mcx_ctx *ctx, const uint64_t *first, const uint64_t *n,
                               const uint64_t *seed, void *hip_stream);

/* Normalised map, statistics, detector records and digests of simulation
 * `sim` (as mcx_fluence, mcx_fluence_f64, mcx_stats, mcx_detected and
 * mcx_digest for one simulation; kernel_ms and run_ms are those of the whole
 * launch).  MCX_EINVAL when sim is not in [0, mcx_batch_size). */
mcx_status mcx_batch_fluence(mcx_ctx *ctx, int32_t sim, int32_t kind, float *host_out,
                             uint64_t ncells);
mcx_status mcx_batch_fluence_f64(mcx_ctx *ctx, int32_t sim, int32_t kind, double *host_out,
                                 uint64_t ncells);
mcx_status mcx_batch_stats(mcx_ctx *ctx, int32_t sim, mcx_run_stats *out);
mcx_status mcx_batch_detected(mcx_ctx *ctx, int32_t sim, float *host_rec, uint64_t *host_photon,
                              uint64_t cap, uint64_t *nrec, uint64_t *ndropped);
mcx_status mcx_batch_digest(mcx_ctx *ctx, int32_t sim, double *host_out, uint64_t nrows);

/* Launch shape: threads per workgroup (0 = the size that keeps the most waves
 * resident), photons per job (0 = default 256), LDS window cells (0 = default
 * 16384, < 0 = none, at most 36864; in a batch each workgroup keeps the window
 * of the simulation its first wave starts on).  The window covers, per early
 * gate, a box of cells: by default one box round the source over the gates of
 * the first ~0.5 ns; after mcx_autotune on a single simulation, the boxes
 * its flush census shaped for that cell count.  Waits for the stream. */
mcx_status mcx_set_launch(mcx_ctx *ctx, int32_t block_size, int32_t refill_chunk,
                          int32_t lds_window_cells);

/* How later launches add to the map (the atomic deposit of the paper's
 * benchmark B2a, Fig. 2): MCX_MAP_ADDS_AUTO (the default), MCX_MAP_ADDS_64
 * or MCX_MAP_ADDS_32.  Only the speed changes, never a
 * result.  MCX_EINVAL for another value.  Waits for the stream. */
mcx_status mcx_set_map_adds(mcx_ctx *ctx, int32_t mode);

/* Shape the LDS window of a single-simulation context (hardware math, no
 * digests) for lds_window_cells cells from a flush census -- one pilot of
 * pilot_photons[0] photons (seed[0]) counting, per map cell, the cell visits
 * the kernel adds to the map -- as mcx_autotune does for its candidates, and
 * use it from the next launch (keeping the block size and job size; a later
 * mcx_set_launch with the same cell count keeps the shaped boxes).  Other
 * contexts keep the default boxes.  Tallies are cleared on return.
 * MCX_EINVAL for a cell count outside [1, 36864].  Blocking. */
mcx_status mcx_shape_window(mcx_ctx *ctx, const uint64_t *pilot_photons, const uint64_t *seed,
                            int32_t lds_window_cells);

/* Autotuner: times pilot launches of pilot_photons[i] photons (seed[i]) per
 * simulation over block sizes {64, 256, 448, 512, 768, 1024} x jobs of {64,
 * 256, 1024} photons (1 to 16 photons per lane) x deposit schemes {direct
 * global atomics, LDS window of 8192, 16384, 32768 or 36864 cells} (shapes that
 * do not fit on a compute unit are skipped; each timed with the map adds
 * MCX_MAP_ADDS_AUTO picks for it, and the four fastest again with the other
 * kind), keeps the fastest shape -- with the map adds MCX_MAP_ADDS_AUTO picks
 * for it unless the other kind is more than 10 % faster over three alternate
 * re-timings of both -- and fits
 * (single simulations without digests and with hardware math: the window boxes
 * are first shaped by a flush census -- one pilot counting, per map cell, the
 * cell visits the kernel adds to the map -- per gate the box grown from its
 * busiest cell by the densest slabs that fit the candidate's cell count),
 * the linear device runtime model T = a n + T0 of the paper's device-level
 * load balancing (the study of Fig. 3(b)) from pilots of n and n/2 photons.
 * Results do not depend on the shape (the random numbers are keyed by photon
 * index); tallies are cleared on return.  Blocking. */
mcx_status mcx_autotune(mcx_ctx *ctx, const uint64_t *pilot_photons, const uint64_t *seed,
                        mcx_tune_result *out);

/* Least-squares line y = a x + b through k >= 2 points (host only, no GPU):
 * the fit of the paper's device runtime model T = a n + T0 (device-level
 * load balancing, Fig. 3(b)).  MCX_EINVAL for NULL arrays, k < 2, a
 * non-finite point or fewer than two distinct x. */
mcx_status mcx_fit_linear(const double *x, const double *y, int32_t k, double *a, double *b);

/* The paper's device runtime model per simulation: T = a n + T0 (kernel
 * time in ms against photons) from two timed pilot launches of n1[i] and
 * n2[i] photons (NULL: the paper's 1e6 and 5e6) of simulation i alone, with
 * seed[i] and the current launch shape.  a[i] (ms per photon; 1/a is the
 * throughput) and t0[i] (ms) receive the fit.  Tallies are cleared on
 * return.  Blocking. */
mcx_status mcx_fit_runtime(mcx_ctx *ctx, const uint64_t *n1, const uint64_t *n2,
                           const uint64_t *seed, double *a, double *t0);

/* Device-level load balancing inside one launch, by throughput (the paper's
 * S2 partition, shares proportional to the work estimated from 1/a): with
 * cost_per_photon[i] = a_i (e.g. from mcx_fit_runtime), every later launch
 * spreads the waves' home simulations in proportion to a_i n_i instead of
 * the job counts; NULL restores job counts.  Only the schedule changes:
 * every photon's history and every result stay the same.  MCX_EINVAL for a
 * negative or non-finite cost. */
mcx_status mcx_set_balance(mcx_ctx *ctx, const double *cost_per_photon);

/* Clear tallies, detector records, ledger and counters, run photons
 * [0, nphoton) with `seed`, reduce, and wait.  Blocking. */
mcx_status mcx_run(mcx_ctx *ctx, uint64_t nphoton, uint64_t seed);

/* Enqueue photons [first, first+n) with `seed` on `hip_stream` (a
 * hipStream_t; NULL = the context's own stream), accumulating into the
 * current tallies; returns without waiting.  Runs with different seeds may
 * be accumulated; the normalisation divides by the total photon count.
 * The work of one context is ordered whatever streams it is enqueued on:
 * every clear, launch and device-side normalisation first waits (on the
 * device) for the context's previous one, and every call that reads results
 * back to the host waits for it too. */
mcx_status mcx_run_range(mcx_ctx *ctx, uint64_t first, uint64_t n, uint64_t seed,
                         void *hip_stream);

/* Clear tallies, records, ledger and counters (enqueued on hip_stream). */
mcx_status mcx_reset(mcx_ctx *ctx, void *hip_stream);

/* Wait for all work enqueued on the context's stream. */
mcx_status mcx_sync(mcx_ctx *ctx);

/* Number of fluence cells (ngates*nx*ny*nz). */
uint64_t mcx_ncells(const mcx_ctx *ctx);

/* Normalised map (kind = MCX_RAW / MCX_FLUENCE / MCX_FLUENCE_RATE), computed
 * on the GPU in FP64 from the map's integer counts and rounded once.  host_out
 * must hold ncells >= mcx_ncells() values (else MCX_ERANGE).  Blocking. */
mcx_status mcx_fluence(mcx_ctx *ctx, int32_t kind, float *host_out, uint64_t ncells);
mcx_status mcx_fluence_f64(mcx_ctx *ctx, int32_t kind, double *host_out, uint64_t ncells);

/* Same, written to device memory dev_out (ncells floats) on hip_stream
 * (NULL = the null stream, as for the other calls that write into the
 * caller's device memory; not the context's own stream), after the
 * context's last clear or launch on any stream; async. */
mcx_status mcx_fluence_device(mcx_ctx *ctx, int32_t kind, float *dev_out, uint64_t ncells,
                              void *hip_stream);

/* Detected-photon records, each 4 + (nmedia - 1) floats:
 * {detector index, scattering count, exit weight, exit time (ns),
 *  pathlength in medium 1, ..., pathlength in medium nmedia-1 (mm)},
 * plus the photon index of each record in host_photon (may be NULL).
 * Copies min(cap, records) rows; *nrec = rows copied, *ndropped = detected
 * photons that found the record buffer full.  Record order is unspecified.
 * Blocking. */
mcx_status mcx_detected(mcx_ctx *ctx, float *host_rec, uint64_t *host_photon, uint64_t cap,
                        uint64_t *nrec, uint64_t *ndropped);

/* ------------------------------------------------ detected-photon post-processing
 *
 * The step after detection in the paper's workflow (Fig. 1: detected-photon
 * data are read back and processed).  Records are rows of 4 + npath floats,
 * as mcx_detected returns them: {detector, scatterings, exit weight w, exit
 * time t (ns), pathlength L_1 .. L_npath in media 1 .. npath (mm)}.
 *
 * Per record: w' = w exp(-(dmua[0] L_1 + ... + dmua[npath-1] L_npath)), the
 * weight the photon would have left with had medium i's absorption been
 * mua_i + dmua[i-1]: absorption is a continuous weight decay, so paths depend
 * only on the scattering properties and the stored pathlengths fix the
 * detected weight for any absorption change (valid while roulette, whose
 * decisions depend on the weight, did not act on the photon).  dmua NULL:
 * w' = w.  The exponent is summed in medium order in FP64, each product
 * rounded on its own.
 *
 * Per detector d, row d of `out` (2 + ngates doubles):
 *   out[d][0]      number of records of detector d;
 *   out[d][1]      sum of w' / nphoton: detected weight per launched photon
 *                  (the detector's diffuse reflectance, not divided by its area);
 *   out[d][2 + g]  sum of w' over the records whose exit time is in gate g,
 *                  g = min(max(floor((t - t0) / dt), 0), ngates - 1) in FP64,
 *                  / (nphoton dt): the time-resolved reflectance (TPSF), 1/ns
 *                  per launched photon.
 * nphoton = 0 returns the raw sums (no division at all).  Records whose
 * detector column is not an integer in [0, ndet) are skipped.  Sums are FP64
 * over per-workgroup partial sums added in a fixed order. */
typedef struct {
  int32_t ndet;     /* detectors, 1..4096 */
  int32_t npath;    /* pathlength columns (nmedia - 1), 1..255; rows have 4 + npath floats */
  float t0_ns;      /* start of gate 0 (finite) */
  float dt_ns;      /* gate width (> 0, finite) */
  int32_t ngates;   /* 1..8190 */
  uint64_t nphoton; /* launched photons to divide by; 0 = raw sums */
} mcx_detpost;

/* Post-process nrec records in device memory (dev_rec, nrec rows; may be
 * NULL when nrec == 0) into dev_out (ndet * (2 + ngates) doubles, device)
 * and, when dev_weight is not NULL, the re-weighted weight of every record
 * (nrec doubles, device, record order).  dev_dmua: npath floats in device
 * memory, or NULL.  Enqueued on hip_stream (NULL = the null stream); the
 * per-workgroup partial sums go to a workspace the call allocates, and it
 * waits for the stream before returning to free it.  Errors: MCX_EINVAL for
 * a bad spec or NULL buffers (checked before any HIP call), MCX_ENOMEM,
 * MCX_EDEVICE. */
mcx_status mcx_detpost_device(const float *dev_rec, uint64_t nrec, const mcx_detpost *spec,
                              const float *dev_dmua, double *dev_out, double *dev_weight,
                              void *hip_stream);

/* mcx_detpost_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results and errors, but the partial sums go
 * to a workspace the library keeps in device memory for the life of the
 * process (128 x 8192 doubles, 8 MB per device, its address looked up on
 * the first call on each device), and the call returns once the work is
 * enqueued (no stream wait).  At most 128 workgroups per pass, so for more
 * than 32768 records the partial sums are added in another order than
 * mcx_detpost_device's (results agree to FP64 rounding).  A pass that would
 * need more workspace than the library holds is rejected with MCX_ERANGE;
 * none can with the current limits (ngates <= 8190, passes over detector
 * ranges).  Every call on one device shares the workspace: calls that
 * overlap on one device (different streams, or threads) race and must be
 * ordered by the caller.  No hipMalloc, hipFree or allocating library
 * routine is called. */
mcx_status mcx_detpost_device_noalloc(const float *dev_rec, uint64_t nrec,
                                      const mcx_detpost *spec, const float *dev_dmua,
                                      double *dev_out, double *dev_weight, void *hip_stream);

/* The same for the records simulation `sim` of a context holds (those
 * mcx_batch_detected would return, in the same order): ndet, npath and the
 * gates are the simulation's, nphoton the photons run since the last reset.
 * host_dmua: npath = nmedia - 1 floats, or NULL.  host_out must hold nout >=
 * ndet * (2 + ngates) doubles (else MCX_ERANGE); host_weight (may be NULL)
 * nweight >= stored records.  MCX_ESTATE when no photons were run since the
 * last reset.  Blocking. */
mcx_status mcx_detected_process(mcx_ctx *ctx, int32_t sim, const float *host_dmua,
                                double *host_out, uint64_t nout, double *host_weight,
                                uint64_t nweight);

/* Statistics of the runs since the last reset (waits for the stream). */
mcx_status mcx_stats(mcx_ctx *ctx, mcx_run_stats *out);

/* Per-photon digests (needs opt.ndigest > 0): rows of 8 doubles
 * {end reason (1 escape, 2 time, 3 roulette, 4 cap), scatterings,
 *  segments, last voxel, final weight, final time, random blocks used,
 *  detector or -1} for photons first..first+ndigest-1 of the last run.
 * Blocking. */
mcx_status mcx_digest(mcx_ctx *ctx, double *host_out, uint64_t nrows);

/* Message of the last failed call on this thread ("" if none). */
const char *mcx_last_error(void);

/* Release the context and all its device memory.  NULL is ignored. */
void mcx_destroy(mcx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MCX_H */
