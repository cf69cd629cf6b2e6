// Microbenchmarks behind the transport kernel's design choices on gfx950:
//  - global atomic add throughput: FP32 with and without a returned value,
//    FP64 and 64- and 32-bit integers without a return, on distinct
//    addresses spread over working sets that fit L2 (4 MB per XCD), the
//    MALL, or only HBM, on a few hot addresses shared by every wave, and
//    with a wave's lanes on consecutive cells;
//  - FP32 VALU issue rate (dependent FMA chains) and the Philox block rate,
//    to anchor the ALU roofline of the transport kernel.
// Prints one JSON object per measurement.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define CHECK(x)                                                                    \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
      exit(1);                                                                      \
    }                                                                               \
  } while (0)

__device__ __forceinline__ uint32_t mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Each thread performs `iters` atomics; the index is a hash of (thread,
// iteration) masked to `mask` (a power of two minus one), or fixed among
// `hot` addresses when hot > 0.  Modes: 0 FP32 no return, 1 FP32 with the
// returned value used, 2 FP64 no return, 3 64-bit integer no return, 4 32-bit
// integer no return, 5 FP64 no return with the 64 lanes of a wave on 64
// consecutive cells (8 cache lines of 64 B per instruction), 6 32-bit integer
// add into the low word of a 64-bit cell with the returned value checked for
// a carry into the high word (an exact 64-bit integer sum from 32-bit
// atomics), 7 the same without a return (low words of 64-bit cells).
template <int kMode>
__global__ void __launch_bounds__(256) atomic_kernel(float* f32, double* f64, uint32_t mask,
                                                     uint32_t hot, int iters, float* sink) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  float acc = 0.f;
  for (int i = 0; i < iters; ++i) {
    uint32_t h = mix(tid * 0x9E3779B9u + i);
    if constexpr (kMode == 5) h = mix((tid >> 6) * 0x9E3779B9u + i);
    uint32_t idx = hot ? (h % hot) * 32u : (h & mask);
    if constexpr (kMode == 5) idx = hot ? idx : ((h & mask & ~63u) | (tid & 63u));
    const float v = 1.0f + (h & 0xff) * 1e-3f;
    if constexpr (kMode == 0) {
      unsafeAtomicAdd(f32 + idx, v);
    } else if constexpr (kMode == 1) {
      acc += unsafeAtomicAdd(f32 + idx, v);
    } else if constexpr (kMode == 2 || kMode == 5) {
      unsafeAtomicAdd(f64 + idx, static_cast<double>(v));
    } else if constexpr (kMode == 3) {
      atomicAdd(reinterpret_cast<unsigned long long*>(f64) + idx,
                static_cast<unsigned long long>(h & 0xffffu));
    } else if constexpr (kMode == 4) {
      atomicAdd(reinterpret_cast<unsigned int*>(f32) + idx, h & 0xffffu);
    } else if constexpr (kMode == 6) {
      unsigned int* w = reinterpret_cast<unsigned int*>(f64) + 2 * static_cast<uint64_t>(idx);
      const unsigned int add = (h & 0xffffu) << 12;
      const unsigned int old = atomicAdd(w, add);
      if (old + add < old) atomicAdd(w + 1, 1u);
    } else {
      atomicAdd(reinterpret_cast<unsigned int*>(f64) + 2 * static_cast<uint64_t>(idx),
                (h & 0xffffu) << 12);
    }
  }
  if (kMode == 1 && acc == -1.f) sink[0] = acc;
}

template <int kMode>
static void launch_atomic(int grid, int block, float* f32, double* f64, uint32_t mask,
                          uint32_t hot, int iters, float* sink) {
  atomic_kernel<kMode><<<grid, block>>>(f32, f64, mask, hot, iters, sink);
}

static void launch_atomic_mode(int mode, int grid, int block, float* f32, double* f64,
                               uint32_t mask, uint32_t hot, int iters, float* sink) {
  switch (mode) {
    case 0: launch_atomic<0>(grid, block, f32, f64, mask, hot, iters, sink); break;
    case 1: launch_atomic<1>(grid, block, f32, f64, mask, hot, iters, sink); break;
    case 2: launch_atomic<2>(grid, block, f32, f64, mask, hot, iters, sink); break;
    case 3: launch_atomic<3>(grid, block, f32, f64, mask, hot, iters, sink); break;
    case 4: launch_atomic<4>(grid, block, f32, f64, mask, hot, iters, sink); break;
    case 5: launch_atomic<5>(grid, block, f32, f64, mask, hot, iters, sink); break;
    case 6: launch_atomic<6>(grid, block, f32, f64, mask, hot, iters, sink); break;
    default: launch_atomic<7>(grid, block, f32, f64, mask, hot, iters, sink); break;
  }
}

// Independent FMA chains: 8 per thread, `iters` rounds.
__global__ void __launch_bounds__(256) fma_kernel(float* out, int iters, float a, float b) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = threadIdx.x * 1e-3f + k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  if (s == -1.f) out[0] = s;
}

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, uint32_t k0, uint32_t k1) {
  const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
  const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
  const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
  const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
  c1 = static_cast<uint32_t>(p1);
  c3 = static_cast<uint32_t>(p0);
  c0 = n0;
  c2 = n2;
}

__global__ void __launch_bounds__(256) philox_kernel(uint32_t* out, int iters, uint32_t key0,
                                                     uint32_t key1) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (int i = 0; i < iters; ++i) {
    uint32_t c0 = tid, c1 = 0, c2 = static_cast<uint32_t>(i), c3 = 0, k0 = key0, k1 = key1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      philox_round(c0, c1, c2, c3, k0, k1);
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    acc ^= c0 ^ c1 ^ c2 ^ c3;
  }
  if (acc == 0x12345678u) out[0] = acc;
}

// Plain streaming copy, the reference for HBM byte counters: reads and
// writes `n` float4 values once.
__global__ void __launch_bounds__(256) copy_kernel(const float4* __restrict__ in,
                                                   float4* __restrict__ out, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    out[i] = in[i];
}

static float time_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, a, b));
  return ms;
}

static int run_copy() {
  const uint64_t bytes = 1ull << 30;  // 1 GiB read + 1 GiB written
  const uint64_t n = bytes / sizeof(float4);
  float4 *a = nullptr, *b = nullptr;
  CHECK(hipMalloc(&a, bytes));
  CHECK(hipMalloc(&b, bytes));
  CHECK(hipMemset(a, 1, bytes));
  CHECK(hipMemset(b, 0, bytes));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  for (int rep = 0; rep < 3; ++rep) {
    CHECK(hipEventRecord(e0));
    copy_kernel<<<8192, 256>>>(a, b, n);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    const double ms = time_ms(e0, e1);
    printf("{\"bench\": \"copy\", \"bytes_read\": %llu, \"bytes_written\": %llu, "
           "\"GBps\": %.1f, \"ms\": %.3f}\n",
           static_cast<unsigned long long>(bytes), static_cast<unsigned long long>(bytes),
           2.0 * bytes / (ms * 1e-3) / 1e9, ms);
  }
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && strcmp(argv[1], "copy") == 0) return run_copy();
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  const int block = 256, per_cu = 8;
  const int grid = cus * per_cu;
  const uint64_t threads = static_cast<uint64_t>(grid) * block;
  const int iters = 64;
  const size_t max_bytes = 1ull << 30;  // 1 GiB of FP64 cells at most
  float* f32 = nullptr;
  double* f64 = nullptr;
  float* sink = nullptr;
  CHECK(hipMalloc(&f32, max_bytes));
  CHECK(hipMalloc(&f64, max_bytes));
  CHECK(hipMalloc(&sink, 64));
  CHECK(hipMemset(f32, 0, max_bytes));
  CHECK(hipMemset(f64, 0, max_bytes));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));

  const char* modes[8] = {"f32_noret", "f32_ret", "f64_noret", "u64_noret", "u32_noret",
                          "f64_noret_wave_lines", "u32_ret_carry_in_u64", "u32_noret_in_u64"};
  // working sets in bytes of FP64 cells (FP32 uses half the bytes, same count)
  const uint64_t sets[] = {1ull << 20, 2ull << 20, 64ull << 20, 512ull << 20};
  for (int mode = 0; mode < 8; ++mode) {
    for (uint64_t ws : sets) {
      const uint32_t cells = static_cast<uint32_t>(ws / 8);
      const uint32_t mask = cells - 1;
      for (int rep = 0; rep < 2; ++rep) {
        CHECK(hipEventRecord(e0));
        launch_atomic_mode(mode, grid, block, f32, f64, mask, 0, iters, sink);
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        if (rep == 1) {
          const double ms = time_ms(e0, e1);
          printf("{\"bench\": \"atomic\", \"mode\": \"%s\", \"cells\": %u, \"working_set_MB\": %.1f, "
                 "\"atomics_per_s\": %.4g, \"ms\": %.3f}\n",
                 modes[mode], cells, cells * (mode == 0 || mode == 1 || mode == 4 ? 4.0 : 8.0) / 1048576.0,
                 threads * iters / (ms * 1e-3), ms);
        }
      }
    }
    for (uint32_t hot : {1u, 8u, 64u, 512u}) {
      for (int rep = 0; rep < 2; ++rep) {
        const int it = hot < 64 ? 4 : iters;
        CHECK(hipEventRecord(e0));
        launch_atomic_mode(mode, grid, block, f32, f64, 0, hot, it, sink);
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        if (rep == 1) {
          const double ms = time_ms(e0, e1);
          printf("{\"bench\": \"atomic_hot\", \"mode\": \"%s\", \"hot_addresses\": %u, "
                 "\"atomics_per_s\": %.4g, \"ms\": %.3f}\n",
                 modes[mode], hot, threads * it / (ms * 1e-3), ms);
        }
      }
    }
  }

  {
    const int it = 4096;
    for (int rep = 0; rep < 2; ++rep) {
      CHECK(hipEventRecord(e0));
      fma_kernel<<<grid, block>>>(sink, it, 0.999f, 0.001f);
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      if (rep == 1) {
        const double ms = time_ms(e0, e1);
        const double lane_ops = static_cast<double>(threads) * it * 8;
        printf("{\"bench\": \"fma_f32\", \"lane_fma_per_s\": %.4g, \"tflops\": %.2f, \"ms\": %.3f}\n",
               lane_ops / (ms * 1e-3), 2 * lane_ops / (ms * 1e-3) / 1e12, ms);
      }
    }
  }
  {
    const int it = 256;
    for (int rep = 0; rep < 2; ++rep) {
      CHECK(hipEventRecord(e0));
      philox_kernel<<<grid, block>>>(reinterpret_cast<uint32_t*>(sink), it, 1u, 0u);
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      if (rep == 1) {
        const double ms = time_ms(e0, e1);
        printf("{\"bench\": \"philox4x32_10\", \"blocks_per_s\": %.4g, \"ms\": %.3f}\n",
               static_cast<double>(threads) * it / (ms * 1e-3), ms);
      }
    }
  }
  CHECK(hipFree(f32));
  CHECK(hipFree(f64));
  CHECK(hipFree(sink));
  return 0;
}
