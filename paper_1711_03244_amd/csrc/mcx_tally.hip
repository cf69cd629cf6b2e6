// Tally maintenance kernels: clearing, the FP64 reductions of the finished
// map (total deposit and absorbed weight) and normalisation to fluence.
// The map holds 64-bit integer counts of the simulation's deposit unit; a
// count converts to FP64 exactly up to 2^53 units.  All are grid-stride
// loops over the cells with coalesced 8-byte accesses.
#include "mcx_internal.hpp"

namespace mcx {
namespace {

__global__ void clear_kernel(uint64_t* tally, uint64_t ncells, double* ledger,
                             unsigned long long* counts, unsigned long long* det_count,
                             int nsims) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  const uint64_t first = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (uint64_t i = first; i < ncells; i += stride) tally[i] = 0ull;
  for (uint64_t i = first; i < static_cast<uint64_t>(nsims) * kLedgerN; i += stride)
    ledger[i] = 0.0;
  for (uint64_t i = first; i < static_cast<uint64_t>(nsims) * kCountN; i += stride)
    counts[i] = 0ull;
  for (uint64_t i = first; i < static_cast<uint64_t>(nsims); i += stride) det_count[i] = 0ull;
}

__global__ void reset_counters_kernel(unsigned long long* counters, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    counters[i] = 0ull;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// out[0] += sum over cells, out[1] += sum of mua(label) * cell: total
// deposited weight*mm and the absorbed weight it implies.  Per-thread and
// per-block sums in FP64.
__global__ void __launch_bounds__(256) reduce_kernel(const uint64_t* tally, double unit,
                                                     const uint8_t* labels, const float4* media,
                                                     uint32_t nvox, uint64_t ncells, double* out) {
  __shared__ double part[2][4];
  double a = 0.0, b = 0.0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < ncells;
       i += stride) {
    const double v = static_cast<double>(tally[i]) * unit;
    a += v;
    b += static_cast<double>(media[labels[i % nvox]].x) * v;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][wv] = a;
    part[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < static_cast<int>(blockDim.x >> 6); ++k) {
      sa += part[0][k];
      sb += part[1][k];
    }
    unsafeAtomicAdd(out, sa);
    unsafeAtomicAdd(out + 1, sb);
  }
}

template <typename T>
__global__ void normalise_kernel(const uint64_t* tally, uint64_t ncells, double scale, T* out) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < ncells;
       i += stride)
    out[i] = static_cast<T>(static_cast<double>(tally[i]) * scale);
}

int grid_for(uint64_t n, int block, int cap) {
  const uint64_t g = (n + block - 1) / block;
  return static_cast<int>(g < static_cast<uint64_t>(cap) ? (g ? g : 1) : cap);
}

}  // namespace

hipError_t launch_clear(uint64_t* tally, uint64_t ncells, double* ledger,
                        unsigned long long* counts, unsigned long long* det_count,
                        int nsims, hipStream_t s) {
  const uint64_t n = ncells > static_cast<uint64_t>(nsims) * kCountN
                         ? ncells : static_cast<uint64_t>(nsims) * kCountN;
  clear_kernel<<<grid_for(n, 256, 8192), 256, 0, s>>>(tally, ncells, ledger, counts, det_count,
                                                      nsims);
  return hipGetLastError();
}

hipError_t launch_reset_counters(unsigned long long* counters, int n, hipStream_t s) {
  reset_counters_kernel<<<(n + 255) / 256, 256, 0, s>>>(counters, n);
  return hipGetLastError();
}

hipError_t launch_reduce(const uint64_t* tally, double unit, const uint8_t* labels,
                         const float4* media, uint32_t nvox, int ngates, double* out2,
                         hipStream_t s) {
  const uint64_t n = static_cast<uint64_t>(nvox) * ngates;
  reduce_kernel<<<grid_for(n, 256, 4096), 256, 0, s>>>(tally, unit, labels, media, nvox, n,
                                                        out2);
  return hipGetLastError();
}

hipError_t launch_normalise_f32(const uint64_t* tally, uint64_t ncells, double scale, float* out,
                                hipStream_t s) {
  normalise_kernel<float><<<grid_for(ncells, 256, 8192), 256, 0, s>>>(tally, ncells, scale, out);
  return hipGetLastError();
}

hipError_t launch_normalise_f64(const uint64_t* tally, uint64_t ncells, double scale,
                                double* out, hipStream_t s) {
  normalise_kernel<double><<<grid_for(ncells, 256, 8192), 256, 0, s>>>(tally, ncells, scale,
                                                                       out);
  return hipGetLastError();
}

}  // namespace mcx
