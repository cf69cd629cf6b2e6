// Detected-photon post-processing on the GPU (the step after detection in
// the paper's workflow, Fig. 1: detected-photon data are read back and
// turned into measurements).
//
// Input: detector records as the transport kernel writes them, one row of
// 4 + npath floats per detected photon {detector, scatterings, exit weight,
// exit time (ns), pathlength in medium 1 .. npath (mm)}.  Per record the
// weight is optionally re-weighted for an absorption change dmua of every
// medium, w' = w exp(-sum_i dmua_i L_i): with absorption applied as a
// continuous weight decay, trajectories depend only on the scattering
// properties, so the stored partial pathlengths fix the detected weight for
// any absorption map.  Per detector the kernels sum the record count, the
// weights (reflectance, per launched photon) and the weights by exit-time
// gate (time-resolved reflectance, the TPSF, per launched photon and ns).
//
// Two launches, both HBM-light: each workgroup sums its records into an FP64
// histogram in LDS and writes it to its own slot of a workspace of partial
// sums; a second launch adds the partials of each histogram entry in
// workgroup order (so a given launch shape always sums in the same order)
// and scales them.  Detectors whose histogram does not fit the LDS budget
// are processed in several passes over detector ranges.
#include <math.h>

#include <mutex>

#include "mcx_detpost.hpp"

namespace mcx {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxDevices = 64;

// Workspace of partial sums for callers that cannot allocate device memory.
// In host code this name stands for the variable, not for its device
// address: kernels get the address detpost_scratch() looks up.
static __device__ __align__(256) double scratch[kDetpostScratch];

__global__ void __launch_bounds__(kBlock)
    detpost_partial_kernel(const float* __restrict__ rec, uint64_t nrec, int rec_len, int npath,
                           const float* __restrict__ dmua, int det_lo, int det_hi, double t0,
                           double dt, int ngates, double* __restrict__ weight_out,
                           double* __restrict__ partial) {
  extern __shared__ double hist[];
  const int cols = 2 + ngates;
  const int hist_len = (det_hi - det_lo) * cols;
  for (int i = threadIdx.x; i < hist_len; i += blockDim.x) hist[i] = 0.0;
  __syncthreads();
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t r = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < nrec;
       r += stride) {
    const float* row = rec + r * static_cast<uint64_t>(rec_len);
    // the exponent is summed medium by medium, each product rounded on its
    // own (no fused multiply-add), in FP64
    double w = static_cast<double>(row[2]);
    if (dmua) {
#pragma clang fp contract(off)
      double e = 0.0;
      for (int i = 0; i < npath; ++i)
        e = e + static_cast<double>(dmua[i]) * static_cast<double>(row[4 + i]);
      w = w * exp(-e);
    }
    if (weight_out && det_lo == 0) weight_out[r] = w;
    // a record counts for detector d only if its first column is exactly d
    // (range checked in float before any conversion; NaN fails it)
    const float df = row[0];
    if (!(df >= static_cast<float>(det_lo) && df < static_cast<float>(det_hi))) continue;
    const int d = static_cast<int>(df);
    if (static_cast<float>(d) != df) continue;
    // gate of the exit time, clamped to [0, ngates - 1] (NaN -> 0)
    double q = floor((static_cast<double>(row[3]) - t0) / dt);
    q = q >= 0.0 ? q : 0.0;
    const int gate = q >= static_cast<double>(ngates - 1) ? ngates - 1 : static_cast<int>(q);
    double* h = hist + (d - det_lo) * cols;
    atomicAdd(h, 1.0);
    atomicAdd(h + 1, w);
    atomicAdd(h + 2 + gate, w);
  }
  __syncthreads();
  double* mine = partial + static_cast<uint64_t>(blockIdx.x) * hist_len;
  for (int i = threadIdx.x; i < hist_len; i += blockDim.x) mine[i] = hist[i];
}

// out[det_lo * cols + i] = scale(i) * sum over workgroups b (in order) of
// partial[b][i]; column 0 (record count) is not scaled, column 1 by
// 1 / nphoton, columns 2.. by 1 / (nphoton dt).
__global__ void __launch_bounds__(kBlock)
    detpost_final_kernel(const double* __restrict__ partial, int nparts, int hist_len, int cols,
                         double s_sum, double s_gate, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= hist_len) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += partial[static_cast<int64_t>(b) * hist_len + i];
  const int c = i % cols;
  out[i] = c == 0 ? acc : acc * (c == 1 ? s_sum : s_gate);
}

}  // namespace

hipError_t detpost_scratch(double** ptr) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

int detpost_dets_per_pass(int ngates) {
  return kDetpostHistMax / (2 + ngates);
}

int detpost_blocks(uint64_t nrec) {
  const uint64_t want = (nrec + kBlock - 1) / kBlock;
  return static_cast<int>(want < 1 ? 1 : (want > kDetpostMaxBlocks ? kDetpostMaxBlocks : want));
}

hipError_t launch_detpost(const DetpostArgs& a, double* partial, int nblocks, int det_lo,
                          int det_hi, hipStream_t s) {
  const int cols = 2 + a.ngates;
  const int hist_len = (det_hi - det_lo) * cols;
  const size_t smem = static_cast<size_t>(hist_len) * sizeof(double);
  hipLaunchKernelGGL(detpost_partial_kernel, dim3(nblocks), dim3(kBlock), smem, s, a.rec, a.nrec,
                     a.rec_len, a.npath, a.dmua, det_lo, det_hi, static_cast<double>(a.t0),
                     static_cast<double>(a.dt), a.ngates, a.weight_out, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // nphoton = 0: raw sums, no scaling
  const double n = static_cast<double>(a.nphoton);
  const double s_sum = a.nphoton > 0 ? 1.0 / n : 1.0;
  const double s_gate = a.nphoton > 0 ? 1.0 / (n * static_cast<double>(a.dt)) : 1.0;
  hipLaunchKernelGGL(detpost_final_kernel, dim3((hist_len + kBlock - 1) / kBlock), dim3(kBlock),
                     0, s, partial, nblocks, hist_len, cols, s_sum, s_gate,
                     a.out + static_cast<uint64_t>(det_lo) * cols);
  return hipGetLastError();
}

}  // namespace mcx
