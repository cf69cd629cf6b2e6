// Internal interfaces between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcx {

// Ledger slots (FP64 weight sums) and counter slots accumulated on the GPU.
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

// Everything one transport launch needs; passed by value as the kernel
// argument block.
struct TransportParams {
  // domain
  const uint8_t* labels;   // nx*ny*nz, x-fastest
  int32_t nx, ny, nz;
  uint32_t nvox;
  float h, inv_h;
  // media: nmedia rows each of the three float4 tables below
  const float4* media;     // [0, nmedia): (mua, mus, g, n)
                           // [nmedia, 2 nmedia): (1/mus or inf, n/c, c/n, 1/mua or 0)
                           // [2 nmedia, 3 nmedia): HG (1-g, 2g, 2(1+g^2), (1-g)^2)
                           // then ndet rows of detectors (x, y, z, r^2)
  int32_t nmedia;
  int32_t ndet;
  // source
  int32_t src_ix, src_iy, src_iz, src_label;
  float src_fx, src_fy, src_fz;
  float src_vx, src_vy, src_vz;
  // gates
  float t0, inv_dt, t_end;
  int32_t ngates;
  // options
  int32_t reflect;
  float n_out, rr_threshold, rr_p, rr_m;
  uint32_t max_events;
  // run
  uint64_t first, nphoton;
  uint32_t key0, key1;
  uint32_t chunk;
  // LDS window: cells [wx0, wx0+wnx) x [wy0, ...) x [wz0, ...) of gates
  // [0, wng) are summed per workgroup in LDS and flushed once at the end
  int32_t wx0, wy0, wz0, wnx, wny, wnz, wng;
  // outputs
  double* tally;                     // FP64 sum per cell
  unsigned long long* photon_counter;  // next unclaimed photon offset
  double* ledger;                    // kLedgerN
  unsigned long long* counts;        // kCountN
  float* det_rec;
  unsigned long long* det_photon;
  unsigned long long* det_count;
  uint64_t det_cap;
  int32_t rec_len;
  double* digest;
  uint64_t ndigest;
};

// `p` is the host copy (used for the launch shape); `dev_params` must hold the
// same bytes in device memory by the time the kernel runs (copied on `s`).
hipError_t launch_transport(const TransportParams& p, TransportParams* dev_params, int grid,
                            int block, hipStream_t s, bool detect, bool diag, bool accurate);
// Shared-memory bytes the transport kernel needs for a launch shape.
size_t transport_smem_bytes(int nmedia, int ndet, int block, bool detect, int window_cells);
// Occupancy query (resident workgroups per CU) for a launch shape.
hipError_t transport_occupancy(int* blocks_per_cu, int block, size_t smem, bool detect,
                               bool diag, bool accurate);

hipError_t launch_clear(double* tally, uint64_t ncells, double* ledger,
                        unsigned long long* counts, unsigned long long* det_count,
                        double* reduce, hipStream_t s);
hipError_t launch_reset_counter(unsigned long long* counter, hipStream_t s);
hipError_t launch_reduce(const double* tally, const uint8_t* labels, const float4* media,
                         uint32_t nvox, int ngates, double* out2, hipStream_t s);
hipError_t launch_normalise_f32(const double* tally, uint64_t ncells, double scale, float* out,
                                hipStream_t s);
hipError_t launch_normalise_f64(const double* tally, uint64_t ncells, double scale, double* out,
                                hipStream_t s);

}  // namespace mcx
