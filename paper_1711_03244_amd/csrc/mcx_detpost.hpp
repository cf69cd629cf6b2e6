// Internal interface of the detected-photon post-processing kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcx {

// LDS budget of one histogram pass: detectors x (2 + gates) FP64 sums.
constexpr int kDetpostHistMax = 8192;
// Workgroups of the partial-sum launch (each owns one histogram of partials).
constexpr int kDetpostMaxBlocks = 1024;

struct DetpostArgs {
  const float* rec;     // device, nrec rows of rec_len floats
  uint64_t nrec;
  int rec_len, npath;   // rec_len = 4 + npath
  const float* dmua;    // device, npath values, or nullptr
  int ndet;
  float t0, dt;
  int ngates;
  uint64_t nphoton;     // divisor; 0 = raw sums
  double* out;          // device, ndet * (2 + ngates)
  double* weight_out;   // device, nrec, or nullptr
};

// Workgroups of a pass of the entry point that allocates nothing, and the
// doubles of its device-resident workspace: every pass (at most
// kDetpostHistMax histogram entries per workgroup) fits it.
constexpr int kDetpostNoallocBlocks = 128;
constexpr uint64_t kDetpostScratch =
    static_cast<uint64_t>(kDetpostNoallocBlocks) * kDetpostHistMax;  // 8 MB

// Detectors one pass can hold, and the workgroups of a pass over nrec records.
int detpost_dets_per_pass(int ngates);
int detpost_blocks(uint64_t nrec);

// One pass over detectors [det_lo, det_hi): partial sums into `partial`
// (nblocks * (det_hi - det_lo) * (2 + ngates) doubles), then the scaled
// totals into a.out.  Pass det_lo = 0 also writes the re-weighted weights.
hipError_t launch_detpost(const DetpostArgs& a, double* partial, int nblocks, int det_lo,
                          int det_hi, hipStream_t s);

// Address, on the current device, of the library's own workspace of
// kDetpostScratch doubles (looked up once per device, then cached).  The
// workspace lives as long as the process; every call on a device shares it.
hipError_t detpost_scratch(double** ptr);

}  // namespace mcx
