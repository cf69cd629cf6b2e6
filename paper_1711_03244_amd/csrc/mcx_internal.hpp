// Internal interfaces between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcx.h"

namespace mcx {

// Set the calling thread's mcx_last_error message; returns st.
mcx_status report(mcx_status st, const char* message);

// Ledger slots (FP64 weight sums) and counter slots accumulated per simulation.
enum LedgerSlot {
  kLedEscaped = 0, kLedDetected, kLedTimeout, kLedRrGain, kLedRrLoss, kLedCapped,
  kLedgerN = 8
};
enum CountSlot {
  kCntLaunched = 0, kCntEscaped, kCntDetected, kCntTimeout, kCntRrDead, kCntCapped,
  kCntScatters, kCntFaceEvents, kCntFresnel, kCntReflections, kCntRrTests, kCntRrSurvived,
  kCntEvents, kCntLaneSlots, kCntFlushes,
  kCountN = 16
};
constexpr int kDigestN = 8;
constexpr int kMaxWavesPerBlock = 16;
constexpr int kMaxWinGates = 16;  // gates an LDS window can cover

// One simulation: domain, media, source, gates, photon range and outputs.
// Lives in device memory; a wave reads the fields of its current
// simulation with scalar loads.
struct SimDesc {
  // domain, x-fastest
  const uint8_t* labels;
  int32_t nx, ny, nz;
  uint32_t nvox, stride_y, stride_z;
  float h, inv_h;
  // tables: [0, nmedia) (mua, mus, g, n); [nmedia, 2 nmedia) (1/mus or inf,
  // n/c, c/n, 1/mua or 0); [2 nmedia, 3 nmedia) HG (1-g, 2g, 2(1+g^2), (1-g)^2);
  // then ndet detector rows (x, y, z, r^2)
  const float4* tables;
  int32_t nmedia, ndet;
  // source
  int32_t src_ix, src_iy, src_iz, src_label;
  uint32_t src_lin;
  float src_fx, src_fy, src_fz, src_vx, src_vy, src_vz;
  // gates
  float t0, inv_dt, t_end;
  int32_t ngates;
  // boundaries
  int32_t reflect;
  float n_out;
  // photons [first, first + nphoton) with key (key0, key1)
  uint64_t first, nphoton;
  uint32_t key0, key1;
  // outputs
  uint64_t* tally;               // ngates * nvox sums, integer counts of q_unit
  double* ledger;                // kLedgerN
  unsigned long long* counts;    // kCountN
  float* det_rec;
  unsigned long long* det_photon;
  unsigned long long* det_count;
  uint64_t det_cap;
  int32_t rec_len;
  double* digest;
  uint64_t ndigest;
  // Deposit unit: every cell-visit sum is rounded to a whole number of
  // q_unit (a power of two, 2^-20 of the voxel size or just below; q_inv =
  // 1 / q_unit) before it reaches the map or the window; the map holds
  // those numbers.
  float q_unit, q_inv;
  // LDS window of this simulation (wng = 0: none): for each gate g < wng
  // the cells of a box [x0, x0 + nx) x [y0, y0 + ny) x [z0, z0 + nz), at
  // window slots off + ((z - z0) ny + (y - y0)) nx + (x - x0); wbox holds
  // per gate the rows (x0, y0, z0, off) and (nx, ny, nz, 0); wcount slots in
  // all.  The window holds 32-bit integer sums of deposit units.
  const int4* wbox;
  int32_t wng, wcount;
};

// One launch over `nsims` simulations.  Photons are handed out in jobs of
// `chunk` photons of one simulation: simulation s has jobs
// job_start[s+1] - job_start[s], taken in order through its own counter.
// Each wave starts on a home simulation (waves are spread over simulations
// in proportion to their shares, see home_start) and moves on to the
// following simulations once its home has no jobs left.
struct LaunchParams {
  const SimDesc* sims;
  int32_t nsims;
  const uint64_t* job_start;     // nsims + 1 entries, prefix sums of job counts
  uint64_t njobs;
  uint32_t chunk;
  unsigned long long* job_counters;  // nsims entries, zero at launch
  // Shares of the home simulations: prefix sums (nsims + 1 entries) of each
  // simulation's job count, or of its estimated work a_i n_i scaled to
  // integers; nhome = home_start[nsims] (> 0).
  const uint64_t* home_start;
  uint64_t nhome;
  float rr_threshold, rr_p, rr_m;
  uint32_t max_events;
  int32_t table_rows;            // LDS rows per wave for the current simulation's tables
  int32_t nmedia_max;            // for the per-lane pathlength array (detectors)
  // LDS window capacity in cells (0: no window).  Each workgroup keeps the
  // window of one simulation -- the home simulation of its first wave -- and
  // its waves use it while they work on that simulation.
  int32_t window_cells;
  // How the kernel adds to map cells: 1 a returning 32-bit add with a carry
  // into the cell's high word, 0 one 64-bit add (see map_add).
  int32_t map32;
};

size_t transport_smem_bytes(int table_rows, int nmedia_max, int block, bool detect,
                            int window_cells);
// `variant`: 0 the default event loop, 1 non-atomic map deposits, 2 the
// branch-reduced loop (mcx_options.kernel_variant), 3 the flush census: the
// default loop adding 1 to a map cell for every cell visit it flushes, with
// no window (the window shaping reads it).
constexpr int kVariantCensus = 3;
bool transport_variant_available(bool detect, bool diag, bool accurate, int variant);
hipError_t transport_occupancy(int* blocks_per_cu, int block, size_t smem, bool detect,
                               bool diag, bool accurate, int variant);
// `host` is the host copy (for the shared-memory size); `dev` must hold the
// same bytes in device memory by the time the kernel runs.
hipError_t launch_transport(const LaunchParams& host, const LaunchParams* dev, int grid,
                            int block, hipStream_t s, bool detect, bool diag, bool accurate,
                            int variant);

// Zero `ncells` tally cells and `nsims` ledgers, counters and record counts.
hipError_t launch_clear(uint64_t* tally, uint64_t ncells, double* ledger,
                        unsigned long long* counts, unsigned long long* det_count,
                        int nsims, hipStream_t s);
hipError_t launch_reset_counters(unsigned long long* counters, int n, hipStream_t s);
// out2[0] += unit * sum of the cells, out2[1] += unit * sum of mua * cell.
hipError_t launch_reduce(const uint64_t* tally, double unit, const uint8_t* labels,
                         const float4* media, uint32_t nvox, int ngates, double* out2,
                         hipStream_t s);
// out[i] = tally[i] * scale (scale includes the deposit unit).
hipError_t launch_normalise_f32(const uint64_t* tally, uint64_t ncells, double scale, float* out,
                                hipStream_t s);
hipError_t launch_normalise_f64(const uint64_t* tally, uint64_t ncells, double scale,
                                double* out, hipStream_t s);

}  // namespace mcx
