// gfx950 kernels of the fluence denoiser: BF16 MFMA convolutions with FP32
// accumulation (forward, input gradient, weight gradient) and the
// element-wise steps around them.
//
// Activations are channels-last BF16 arrays [voxel][channel], voxels
// x-fastest.  A convolution is an implicit GEMM: rows m are the voxels of
// the grid the kernel iterates, columns n the output channels, and the
// reduction index k = tap * Cin + ci walks the input channels of every tap.
// The A operand is gathered from the activation array on the fly (zero
// outside the volume), the B operand is the weight matrix packed as BF16
// rows Bt[n][k] (k contiguous, padded with zeros to the tile sizes).
// Four gather geometries cover the forward pass and the input gradient of
// all three layer kinds:
//   kConv3   y[v] += x[v + d(t)] W[t]        (3x3x3, stride 1, zero pad)
//   kConv3T  y[v] += x[v - d(t)] W[t]        (its input gradient)
//   kDown    y[v] += x[2v + e(t)] W[t]       (2x2x2, stride 2)
//   kUp      y[2v + e(c)] = x[v] W[c]        (2x2x2 transposed, one parity
//                                             class c per grid z-slice)
// The down layer's input gradient is a kUp product and the up layer's a
// kDown product, each with transposed weights.
//
// Kernels: conv_kernel is the generic implicit GEMM (every geometry);
// 3x3x3 products get dedicated kernels that stage operands in LDS --
// conv3_resident_kernel (exactly 32 gathered channels on large grids: the
// weights stay in LDS, input planes stream in by direct global-to-LDS
// loads), conv3_brick_kernel (other multiples of 32 gathered channels),
// conv3_scalar_kernel (one gathered channel), wgrad_slab_kernel and
// wgrad_onechannel_kernel
// (weight gradients) -- and wgrad_kernel covers the remaining weight
// gradients.  Products that launch too few workgroups split their
// reduction and finish in split_reduce_kernel / wgrad_reduce_kernel, which
// add FP32 partial sums in a fixed order.
//
// MFMA v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8(l / 16) + j]
// and B[8(l / 16) + j][l % 16] (j = 0..7) and receives
// D[4(l / 16) + i][l % 16] (i = 0..3).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "nn_internal.hpp"

namespace mcx {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

constexpr int kBM = 64;   // rows per workgroup tile (4 waves x 16)
constexpr int kBK = 32;   // reduction step
constexpr int kPadK = 8;  // LDS row padding (bf16 elements)

// float -> bf16 bits, round to nearest even: the kernels run with FP32
// denormals kept and round-to-nearest-even, so gfx950's conversion
// instruction gives exactly that rounding, denormals included (NaN stays NaN)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// voxel index of the A operand for row m (grid coordinates z, y, x) and
// tap t, or -1 when it lies outside the input volume
__device__ __forceinline__ int64_t gather_at(const ConvArgs& a, int z, int y, int x, int t) {
  int iz, iy, ix;
  if (a.geo == kConv3 || a.geo == kConv3T) {
    const int s = a.geo == kConv3 ? 1 : -1;
    iz = z + s * (t / 9 - 1);
    iy = y + s * ((t / 3) % 3 - 1);
    ix = x + s * (t % 3 - 1);
    if (iz < 0 || iy < 0 || ix < 0 || iz >= a.in_d || iy >= a.in_h || ix >= a.in_w) return -1;
  } else if (a.geo == kDown) {
    iz = 2 * z + (t >> 2);
    iy = 2 * y + ((t >> 1) & 1);
    ix = 2 * x + (t & 1);
  } else {
    iz = z;
    iy = y;
    ix = x;
  }
  return (static_cast<int64_t>(iz) * a.in_h + iy) * a.in_w + ix;
}

// ------------------------------------------------------------ forward GEMM
// One workgroup: 64 rows x 16*NB columns; wave w owns rows 16w..16w+15.
// KS reduction steps of 32 are staged per pair of barriers.
template <int NB, bool kVec, int KS>
__global__ void __launch_bounds__(256) conv_kernel(ConvArgs a) {
  __shared__ uint16_t sA[kBM][KS * kBK + kPadK];
  __shared__ uint16_t sB[16 * NB][KS * kBK + kPadK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * kBM;
  const int n0 = blockIdx.y * 16 * NB;
  const int cls = blockIdx.z;  // parity class of kUp, else 0
  const int64_t M = static_cast<int64_t>(a.d) * a.h * a.w;
  const int koff = a.geo == kUp ? cls * a.cin : 0;

  // this thread's A row and 8-wide k chunk for the loads
  const int lr = tid >> 2, lc = (tid & 3) * 8;
  const int64_t lm = m0 + lr;
  int lz = 0, ly = 0, lx = 0;
  if (lm < M) {
    lx = static_cast<int>(lm % a.w);
    ly = static_cast<int>((lm / a.w) % a.h);
    lz = static_cast<int>(lm / (static_cast<int64_t>(a.w) * a.h));
  }

  floatx4 acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // this thread's 8 k of row lr of the A tile at reduction step k0
  auto load_a = [&](int k0) -> uint4 {
    const int k = k0 + lc;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (lm >= M) return v;
    if constexpr (kVec) {
      if (k < a.k) {
        const int t = k / a.cin, ci = k - t * a.cin;
        const int64_t src = gather_at(a, lz, ly, lx, t);
        if (src >= 0) v = *reinterpret_cast<const uint4*>(a.x + src * a.cin + ci);
      }
    } else {
      uint16_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        e[j] = 0;
        const int kk = k + j;
        if (kk < a.k) {
          const int t = kk / a.cin, ci = kk - t * a.cin;
          const int64_t src = gather_at(a, lz, ly, lx, t);
          if (src >= 0) e[j] = a.x[src * a.cin + ci];
        }
      }
      v = make_uint4(e[0] | (uint32_t(e[1]) << 16), e[2] | (uint32_t(e[3]) << 16),
                     e[4] | (uint32_t(e[5]) << 16), e[6] | (uint32_t(e[7]) << 16));
    }
    return v;
  };
  // this thread's 8 k of one B row (threads 0 .. 64*NB-1), Bt[n][koff + k]
  const bool has_b = tid < 16 * NB * 4;
  const int br = tid >> 2, bc = (tid & 3) * 8;
  const uint16_t* brow = a.bt + static_cast<int64_t>(n0 + br) * a.kpad + koff;
  auto load_b = [&](int k0) -> uint4 {
    const int k = k0 + bc;
    if (k + 8 <= a.k && (koff & 7) == 0) return *reinterpret_cast<const uint4*>(brow + k);
    uint16_t e[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) e[j] = (k + j < a.k) ? brow[k + j] : 0;
    return make_uint4(e[0] | (uint32_t(e[1]) << 16), e[2] | (uint32_t(e[3]) << 16),
                      e[4] | (uint32_t(e[5]) << 16), e[6] | (uint32_t(e[7]) << 16));
  };

  // software pipeline: the next stage's global loads are in flight while
  // the matrix cores work on the current stage's tiles
  constexpr int kStage = KS * kBK;
  // kDown with gridDim.z = S > 1: this workgroup's reduction range (a
  // multiple of kStage; the last range ends at a.k)
  int k_begin = 0, k_end = a.k;
  if (a.geo != kUp && gridDim.z > 1) {
    const int len = (a.k / static_cast<int>(gridDim.z) + kStage - 1) / kStage * kStage;
    k_begin = static_cast<int>(blockIdx.z) * len;
    k_end = min(a.k, k_begin + len);
  }
  uint4 va[KS], vb[KS];
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    va[q] = k_begin + q * kBK < k_end ? load_a(k_begin + q * kBK) : make_uint4(0u, 0u, 0u, 0u);
    vb[q] = has_b && k_begin + q * kBK < k_end ? load_b(k_begin + q * kBK)
                                               : make_uint4(0u, 0u, 0u, 0u);
  }
  for (int k0 = k_begin; k0 < k_end; k0 += kStage) {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      *reinterpret_cast<uint4*>(&sA[lr][q * kBK + lc]) = va[q];
      if (has_b) *reinterpret_cast<uint4*>(&sB[br][q * kBK + bc]) = vb[q];
    }
    __syncthreads();
    if (k0 + kStage < k_end) {
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        const int kn = k0 + kStage + q * kBK;
        va[q] = kn < k_end ? load_a(kn) : make_uint4(0u, 0u, 0u, 0u);
        if (has_b) vb[q] = kn < k_end ? load_b(kn) : make_uint4(0u, 0u, 0u, 0u);
      }
    }
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      if (k0 + q * kBK >= k_end) break;
      const bf16x8 af =
          *reinterpret_cast<const bf16x8*>(&sA[wave * 16 + (lane & 15)][q * kBK + (lane >> 4) * 8]);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const bf16x8 bf =
            *reinterpret_cast<const bf16x8*>(&sB[j * 16 + (lane & 15)][q * kBK + (lane >> 4) * 8]);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // epilogue: bias, skip, ReLU, store; with gridDim.z = S > 1 (kDown only)
  // the raw sums of this reduction range go to part[z][m][cout] instead
  const bool split = a.geo != kUp && gridDim.z > 1;
  float* part = split ? a.part + static_cast<int64_t>(blockIdx.z) * M * a.cout : nullptr;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + wave * 16 + (lane >> 4) * 4 + i;
    if (m >= M) continue;
    int64_t o = m;
    if (a.geo == kUp) {
      // grids hold at most 2^30 voxels: 32-bit arithmetic
      const uint32_t mm = static_cast<uint32_t>(m);
      const uint32_t x = mm % static_cast<uint32_t>(a.w);
      const uint32_t rest = mm / static_cast<uint32_t>(a.w);
      const uint32_t y = rest % static_cast<uint32_t>(a.h);
      const uint32_t z = rest / static_cast<uint32_t>(a.h);
      o = (static_cast<int64_t>(2 * z + (cls >> 2)) * (2 * a.h) + 2 * y + ((cls >> 1) & 1)) *
              (2 * a.w) + 2 * x + (cls & 1);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + j * 16 + (lane & 15);
      if (n >= a.cout) continue;
      if (split) {
        part[o * a.cout + n] = acc[j][i];
        continue;
      }
      float v = acc[j][i] + (a.bias ? a.bias[n] : 0.f);
      if (a.skip) v += from_bf16(a.skip[o * a.cout + n]);
      if (a.relu) v = fmaxf(v, 0.f);
      if (a.y_f32)
        static_cast<float*>(a.y)[o * a.cout + n] = v;
      else
        static_cast<uint16_t*>(a.y)[o * a.cout + n] = to_bf16(v);
    }
  }
}

// ------------------------------------------------- 3x3x3 conv from an LDS brick
// kConv3 / kConv3T with cin a multiple of 32: a workgroup owns a 4 x 4 x 4MZ
// tile of output voxels (wave w: the z-slices MZ w .. MZ w + MZ - 1, one
// 16-row MFMA block each) and 16 NB output channels.  Per chunk of 32 input
// channels it stages the 6 x 6 x (4MZ + 2) input brick (tile plus halo, zero
// outside the volume) in LDS once, and per plane of 9 taps the weights of
// those taps for its channels; every tap then reads its A fragments from
// the brick and its B fragments from the staged weights, so each weight
// fragment feeds MZ NB matrix instructions.
// With gridDim.z = S > 1 the chunks are split into S equal ranges, one per
// grid z index, and each workgroup stores its raw sums to the workspace
// part[z][out voxel][cout] for split_reduce_kernel to finish.
template <int NB, int MZ>
__global__ void __launch_bounds__(256) conv3_brick_kernel(ConvArgs a) {
  constexpr int BZ = 4 * MZ + 2;
  constexpr int BV = 36 * BZ;
  __shared__ uint16_t sBr[BV][kBK + kPadK];
  __shared__ uint16_t sW[9][16 * NB][kBK + kPadK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tx_n = (a.w + 3) >> 2, ty_n = (a.h + 3) >> 2;
  const int tile = blockIdx.x;
  const int bx = (tile % tx_n) * 4;
  const int by = ((tile / tx_n) % ty_n) * 4;
  const int bz = (tile / (tx_n * ty_n)) * (4 * MZ);
  const int n0 = blockIdx.y * 16 * NB;
  const int sgn = a.geo == kConv3 ? 1 : -1;
  const int r = lane & 15;            // A row of this lane: voxel (r & 3, r >> 2) of a slice
  const int ox = r & 3, oy = r >> 2;
  const int kq = (lane >> 4) * 8;     // this lane's 8 reduction (channel) positions

  floatx4 acc[MZ][NB];
#pragma unroll
  for (int q = 0; q < MZ; ++q)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[q][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int split_len = a.cin / static_cast<int>(gridDim.z);  // a multiple of kBK
  const int c_begin = static_cast<int>(blockIdx.z) * split_len;
  for (int c0 = c_begin; c0 < c_begin + split_len; c0 += kBK) {
    __syncthreads();  // the previous chunk's fragments have been read
    for (int i = tid; i < BV * 4; i += 256) {
      const int v = i >> 2, cc = (i & 3) * 8;
      const int vx = v % 6, vy = (v / 6) % 6, vz = v / 36;
      const int gx = bx + vx - 1, gy = by + vy - 1, gz = bz + vz - 1;
      uint4 val = make_uint4(0u, 0u, 0u, 0u);
      if (gx >= 0 && gy >= 0 && gz >= 0 && gx < a.in_w && gy < a.in_h && gz < a.in_d)
        val = *reinterpret_cast<const uint4*>(
            a.x + ((static_cast<int64_t>(gz) * a.in_h + gy) * a.in_w + gx) * a.cin + c0 + cc);
      *reinterpret_cast<uint4*>(&sBr[v][cc]) = val;
    }
    for (int pz = 0; pz < 3; ++pz) {
      if (pz > 0) __syncthreads();  // the previous plane's weights have been read
      // weights of taps 9 pz .. 9 pz + 8: rows n0 .. n0 + 16 NB - 1 of bt (the
      // packed rows extend to a multiple of 64 >= n0 + 16 NB), 32 columns each
      for (int i = tid; i < 9 * 16 * NB * 4; i += 256) {
        const int tt = i / (16 * NB * 4), rem = i % (16 * NB * 4);
        const int row = rem >> 2, cc = (rem & 3) * 8;
        *reinterpret_cast<uint4*>(&sW[tt][row][cc]) = *reinterpret_cast<const uint4*>(
            a.bt + static_cast<int64_t>(n0 + row) * a.kpad + (9 * pz + tt) * a.cin + c0 + cc);
      }
      __syncthreads();
      const int dz = sgn * (pz - 1);
#pragma unroll
      for (int tt = 0; tt < 9; ++tt) {
        const int dy = sgn * (tt / 3 - 1), dx = sgn * (tt % 3 - 1);
        bf16x8 bc[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j)
          bc[j] = *reinterpret_cast<const bf16x8*>(&sW[tt][16 * j + r][kq]);
#pragma unroll
        for (int q = 0; q < MZ; ++q) {
          const int oz = wave * MZ + q;
          const int v = ((oz + 1 + dz) * 6 + (oy + 1 + dy)) * 6 + (ox + 1 + dx);
          const bf16x8 af = *reinterpret_cast<const bf16x8*>(&sBr[v][kq]);
#pragma unroll
          for (int j = 0; j < NB; ++j)
            acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bc[j], acc[q][j], 0, 0, 0);
        }
      }
    }
  }

  // epilogue: rows 4 (lane >> 4) + e of each of the wave's slices
  const bool split = gridDim.z > 1;
  float* part = split ? a.part + static_cast<int64_t>(blockIdx.z) * a.d * a.h * a.w * a.cout
                      : nullptr;
#pragma unroll
  for (int q = 0; q < MZ; ++q)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + j * 16 + (lane & 15);
      if (n >= a.cout) continue;
      const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = (lane >> 4) * 4 + e;
        const int x = bx + (rr & 3), y = by + (rr >> 2), z = bz + wave * MZ + q;
        if (x >= a.w || y >= a.h || z >= a.d) continue;
        const int64_t o = (static_cast<int64_t>(z) * a.h + y) * a.w + x;
        if (split) {
          part[o * a.cout + n] = acc[q][j][e];
          continue;
        }
        float v = acc[q][j][e] + bias;
        if (a.skip) v += from_bf16(a.skip[o * a.cout + n]);
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.y_f32)
          static_cast<float*>(a.y)[o * a.cout + n] = v;
        else
          static_cast<uint16_t*>(a.y)[o * a.cout + n] = to_bf16(v);
      }
    }
}

// --------------------------------- 3x3x3 conv, 32 input channels, weights resident
// kConv3 / kConv3T with cin == 32 on large grids (the full-resolution layers):
// the reduction is one chunk of 32 channels, so a workgroup's weights (27
// taps x 16 NB output channels) fit in LDS and stay there while the
// workgroup walks its columns of tiles (columns blockIdx.x, blockIdx.x +
// gridDim.x, ... of 4 x 4 x 8-voxel tiles stacked along z).  Waves 0-3
// compute (wave w: z-slices 2w, 2w + 1 of the tile, NB 16-column MFMA blocks
// each) and leave each tile's outputs in LDS; wave 4 streams the input
// planes of the column (6 x 6 voxels of 32 channels, z = -1 .. 8 per tile
// count + 1) into a ring of plane slots with direct global-to-LDS loads,
// A tiles ahead (a tile reuses two planes of the previous one and loads
// eight; zeros outside the volume come from g_zero16); waves 5 and 6
// write the previous tile's outputs from LDS to global memory.  The compute
// waves issue no global memory operation; each data wave waits only for its
// own transfers (the plane wave for all but the newest A - 1 tiles' loads,
// which complete in issue order): one barrier per tile.  Plane layout: voxel
// (y, x) of the plane at (y * 6 + x) * 64 bytes, its 16-byte chunk j
// (channels 8j .. 8j + 7) in slot j ^ (y & 3), so that the 16 rows of an A
// fragment (a 4 x 4 patch of voxels) fall on 16 different bank groups; the
// weights of output channel n likewise at n * 64 bytes, chunk j in slot
// j ^ ((n >> 2) & 3).
constexpr int kResPlane = 36 * 64;  // bytes per plane slot
// The source of the zero padding: 64 KB of zeros, each lane reading its
// own 16 bytes (offset by workgroup and load), so that the zero chunks --
// whole planes at z = -1 and z = d, and the volume's sides -- spread over
// many cache lines instead of sending every compute unit to one address.
constexpr int kZeroChunks = 4096;
__device__ __align__(16) uint4 g_zero16[kZeroChunks];

// Byte offset of byte `byte` of local voxel vl's outputs in an output tile
// of the resident kernel (rows of NB 16 outputs of ES bytes).  For NB == 2
// the rows and 16-byte chunks are permuted within each group of 16 voxels
// by g = (vl >> 2) & 3, the group of lanes that writes them in the
// epilogue (lanes 16 g .. 16 g + 15), so that each epilogue write
// instruction hits 64 different banks: BF16 rows (64 bytes) go to row
// vl ^ g with the two 32-byte halves swapped for odd g; FP32 rows (128
// bytes) to row vl ^ (g >> 1) with the halves swapped for odd g.
template <int NB, int ES>
__device__ __forceinline__ int sout_off(int vl, int byte) {
  if constexpr (NB != 2) {
    return vl * (16 * NB * ES) + byte;
  } else {
    const int g = (vl >> 2) & 3;
    if constexpr (ES == 2)
      return (vl ^ g) * 64 + (byte ^ ((g & 1) << 5));
    else
      return (vl ^ (g >> 1)) * 128 + (byte ^ ((g & 1) << 6));
  }
}

// Makes the compiler produce v here (an empty instruction that takes it as
// input): loads of values used only under a condition are otherwise moved
// into the conditional code, one load and one wait at a time.
__device__ __forceinline__ void pin(const uint4& v) {
  asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

// tiles of planes in flight: all that fit in LDS beside the weights and
// two output tiles (three, or two for 32 FP32 output columns)
constexpr int res_ahead(int nb, bool f32) { return nb == 2 && f32 ? 2 : 3; }

// kGrad: an input gradient with the next backward step folded in
// (ConvArgs::gmask): the compute waves leave FP32 sums in LDS, the output
// waves apply the ReLU mask, round to BF16, store, and sum each channel's
// BF16 values; the workgroup's sums go to gpart.
template <int NB, bool kF32, bool kGrad>
__global__ void __launch_bounds__(448) conv3_resident_kernel(ConvArgs a) {
  constexpr int NC = 16 * NB;                 // output channels of the workgroup
  constexpr int ES = kF32 || kGrad ? 4 : 2;   // bytes per output in LDS
  constexpr int A = res_ahead(NB, kF32 || kGrad);
  constexpr int kRing = 8 * A + 10;           // plane slots: tiles k .. k + A
  __shared__ uint4 sW[27][NC][4];
  __shared__ uint4 sRing[kRing * kResPlane / 16];
  __shared__ uint4 sOut[2][128 * NC * ES / 16];  // 128 voxels x NC outputs
  __shared__ float sBias[NC];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tx_n = (a.w + 3) >> 2, ty_n = (a.h + 3) >> 2, tz_n = (a.d + 7) >> 3;
  const int ncol = tx_n * ty_n;
  const int n0 = blockIdx.y * NC;
  const int ncols = min(NC, a.cout - n0);

  // weights and bias, once.  The weights by direct global-to-LDS loads of
  // 64 slots (1 KB) each, all in flight together, from every wave but the
  // plane wave (which starts on the first column's planes meanwhile): lane
  // L of block bl fills slot 64 bl + L, i.e. row (16 bl + L / 4) of the
  // flattened [27][NC] rows, chunk slot L % 4, with the chunk
  // (L % 4) ^ ((row >> 2) & 3) of that row.
  if (wave != 4) {
    const int w6 = wave < 4 ? wave : wave - 1;
    for (int bl = w6; bl < 27 * NC / 16; bl += 6) {
      const int fr = 16 * bl + (lane >> 2), tt = fr / NC, row = fr % NC;
      const int j = (lane & 3) ^ ((row >> 2) & 3);
      __builtin_amdgcn_global_load_lds(
          (__attribute__((address_space(1))) void*)(a.bt + static_cast<int64_t>(n0 + row) * a.kpad +
                                                     tt * 32 + j * 8),
          (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(sW) + bl * 1024), 16, 0,
          0);
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's weight transfers have landed
  }
  for (int i = tid; i < NC; i += blockDim.x) sBias[i] = (a.bias && i < ncols) ? a.bias[n0 + i] : 0.f;

  // wave 4: plane z of the column at (bx, by) into its ring slot, in three
  // loads of 64 lanes (144 chunks: the last load has 16 lanes).  A chunk's
  // offset and position in the plane are the same for every plane.
  int64_t rel[3];
  int pos[3];  // x | y << 4 of the chunk's voxel in the plane, or -1 past it
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int c = k * 64 + lane;  // chunk slot within the plane
    const int vp = c >> 2, y = vp / 6, x = vp % 6, j = (c & 3) ^ (y & 3);
    rel[k] = (static_cast<int64_t>(y - 1) * a.in_w + (x - 1)) * 32 + j * 8;
    pos[k] = c < 144 ? (x | y << 4) : -1;
  }
  const uint16_t* zero = reinterpret_cast<const uint16_t*>(g_zero16);
  auto load_plane = [&](int bx, int by, int z) {
    const int64_t base = (static_cast<int64_t>(z) * a.in_h + by) * a.in_w * 32 +
                         static_cast<int64_t>(bx) * 32;
    const bool zin = z >= 0 && z < a.in_d;
    const bool xyin = bx >= 1 && by >= 1 && bx + 5 <= a.in_w && by + 5 <= a.in_h;
    char* slot = reinterpret_cast<char*>(sRing) + ((z + 1) % kRing) * kResPlane;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (pos[k] < 0) continue;
      bool in = zin && xyin;
      if (zin && !xyin) {
        const int gx = bx + (pos[k] & 15) - 1, gy = by + (pos[k] >> 4) - 1;
        in = gx >= 0 && gy >= 0 && gx < a.in_w && gy < a.in_h;
      }
      const uint16_t* src =
          in ? a.x + base + rel[k] : zero + ((blockIdx.x * 192 + k * 64 + lane) & (kZeroChunks - 1)) * 8;
      __builtin_amdgcn_global_load_lds(
          (__attribute__((address_space(1))) void*)(src),
          (__attribute__((address_space(3))) void*)(slot + k * 1024), 16, 0, 0);
    }
  };
  // waves 5 and 6: the outputs of the tile at (bx, by, bz) from sOut[b] to
  // y, every other 64 pieces each
  const int s0 = lane + 64 * (wave - 5);
  // kGrad: this lane's channel sums, and the ReLU mask of its pieces of
  // the next tile to store (loaded a tile ahead: the output path is the
  // kernel's bound)
  constexpr int kGP = NC * 2 / 16;  // 16-byte BF16 pieces per voxel
  float gsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  uint4 gm[kGP];
  auto piece = [&](int bx, int by, int bz, int mm, int64_t& e0) {
    const int i = s0 + 128 * mm;
    const int vl = i / kGP, k = i % kGP;
    const int x = bx + (vl & 3), y = by + ((vl >> 2) & 3), z = bz + (vl >> 4);
    e0 = ((static_cast<int64_t>(z) * a.h + y) * a.w + x) * a.cout + n0 + k * 8;
    return x < a.w && y < a.h && z < a.d;
  };
  auto load_mask = [&](int bx, int by, int bz) {
#pragma unroll
    for (int mm = 0; mm < kGP; ++mm) {
      int64_t e0;
      gm[mm] = piece(bx, by, bz, mm, e0) ? *reinterpret_cast<const uint4*>(a.gmask + e0)
                                          : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store_out = [&](int bx, int by, int bz, int b) {
    const char* src = reinterpret_cast<const char*>(sOut[b]);
    if constexpr (kGrad) {
      // 16-byte BF16 pieces of 8 channels (NC == cout): a lane always has
      // channels 8 (lane % 4) .. + 7; their FP32 sums (32 bytes at byte 32 i
      // of the tile for piece i) are read from LDS first
      float fv[kGP][8];
#pragma unroll
      for (int mm = 0; mm < kGP; ++mm) {
        const int i = s0 + 128 * mm;  // piece i: voxel i / kGP, channels 8 (i % kGP) ..
        const uint4* q = reinterpret_cast<const uint4*>(src + sout_off<NB, 4>(i / kGP, (i % kGP) * 32));
        *reinterpret_cast<uint4*>(&fv[mm][0]) = q[0];
        *reinterpret_cast<uint4*>(&fv[mm][4]) = q[1];
      }
#pragma unroll
      for (int mm = 0; mm < kGP; ++mm) {
        pin(*reinterpret_cast<uint4*>(&fv[mm][0]));
        pin(*reinterpret_cast<uint4*>(&fv[mm][4]));
      }
#pragma unroll
      for (int mm = 0; mm < kGP; ++mm) {
        int64_t e0;
        if (!piece(bx, by, bz, mm, e0)) continue;
        const float* f = fv[mm];
        const uint16_t* mh = reinterpret_cast<const uint16_t*>(&gm[mm]);
        uint4 o;
        uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float v = f[j];
          if (!(from_bf16(mh[j]) > 0.f)) v = 0.f;
          oh[j] = to_bf16(v);
          gsum[j] += from_bf16(oh[j]);
        }
        *reinterpret_cast<uint4*>(static_cast<uint16_t*>(a.y) + e0) = o;
      }
      return;
    }
    const int out_bytes = ncols * ES;
    if (ncols == NC && (a.cout * ES) % 16 == 0) {  // whole rows of 16-byte pieces
      constexpr int per = NC * ES / 16;
      // all of this lane's pieces from LDS first: one wait for the LDS
      // reads (which queue behind the compute waves' fragment reads), not
      // one per piece
      uint4 v[per];
#pragma unroll
      for (int mm = 0; mm < per; ++mm)  // piece i = s0 + 128 mm at byte 16 i of the tile
        v[mm] = *reinterpret_cast<const uint4*>(
            src + sout_off<NB, ES>((s0 + 128 * mm) / per, (s0 + 128 * mm) % per * 16));
#pragma unroll
      for (int mm = 0; mm < per; ++mm) pin(v[mm]);
#pragma unroll
      for (int mm = 0; mm < per; ++mm) {  // 128 * per pieces, 128 per step
        const int i = s0 + 128 * mm;
        const int vl = i / per, k = i % per;
        const int x = bx + (vl & 3), y = by + ((vl >> 2) & 3), z = bz + (vl >> 4);
        if (x >= a.w || y >= a.h || z >= a.d) continue;
        const int64_t o = (static_cast<int64_t>(z) * a.h + y) * a.w + x;
        *reinterpret_cast<uint4*>(static_cast<char*>(a.y) + (o * a.cout + n0) * ES + k * 16) =
            v[mm];
      }
    } else if (out_bytes % 16 == 0 && (a.cout * ES) % 16 == 0) {
      const int per = out_bytes / 16;
      for (int i = s0; i < 128 * per; i += 128) {
        const int vl = i / per, k = i % per;
        const int x = bx + (vl & 3), y = by + ((vl >> 2) & 3), z = bz + (vl >> 4);
        if (x >= a.w || y >= a.h || z >= a.d) continue;
        const int64_t o = (static_cast<int64_t>(z) * a.h + y) * a.w + x;
        *reinterpret_cast<uint4*>(static_cast<char*>(a.y) + (o * a.cout + n0) * ES + k * 16) =
            *reinterpret_cast<const uint4*>(src + sout_off<NB, ES>(vl, k * 16));
      }
    } else {
      for (int i = s0; i < 128 * ncols; i += 128) {
        const int vl = i / ncols, n = i % ncols;
        const int x = bx + (vl & 3), y = by + ((vl >> 2) & 3), z = bz + (vl >> 4);
        if (x >= a.w || y >= a.h || z >= a.d) continue;
        const int64_t o = (static_cast<int64_t>(z) * a.h + y) * a.w + x;
        if constexpr (kF32)
          static_cast<float*>(a.y)[o * a.cout + n0 + n] =
              *reinterpret_cast<const float*>(src + sout_off<NB, ES>(vl, n * 4));
        else
          static_cast<uint16_t*>(a.y)[o * a.cout + n0 + n] =
              *reinterpret_cast<const uint16_t*>(src + sout_off<NB, ES>(vl, n * 2));
      }
    }
  };

  const int sgn = a.geo == kConv3 ? 1 : -1;
  const int r = lane & 15;
  const int ox = r & 3, oy = r >> 2;
  const int kq = lane >> 4;  // this lane's 16-byte chunk of the 32 channels
  for (int col = blockIdx.x; col < ncol; col += gridDim.x) {
    const int bx = (col % tx_n) * 4, by = (col / tx_n) * 4;
    // planes -1 .. 8 min(tz_n, A): the first A tiles; wait for tile 0's
    // (all loads but those of the tiles after it, 24 per tile)
    if (wave == 4) {
      const int zend = 8 * min(tz_n, A);
      for (int z = -1; z <= zend; ++z) load_plane(bx, by, z);
      const int pending = min(tz_n, A) - 1;
      if (pending >= 2)
        __builtin_amdgcn_s_waitcnt(0xCF70);  // vmcnt(48), other counters not waited
      else if (pending == 1)
        __builtin_amdgcn_s_waitcnt(0x4F78);  // vmcnt(24)
      else
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    for (int k = 0; k < tz_n; ++k) {
      if (wave == 4) {
        // the eight new planes of tile k + A (their slots held planes no tile
        // from k on needs); then wait until tile k + 1's planes have arrived:
        // all loads but those of the tiles after it (24 per tile)
        const int last = min(k + A, tz_n - 1);  // the newest tile loaded
        if (k + A < tz_n)
          for (int z = 8 * (k + A) + 1; z <= 8 * (k + A) + 8; ++z) load_plane(bx, by, z);
        const int pending = last - (k + 1);  // tiles whose loads may stay in flight
        if (pending >= 2)
          __builtin_amdgcn_s_waitcnt(0xCF70);  // vmcnt(48), other counters not waited
        else if (pending == 1)
          __builtin_amdgcn_s_waitcnt(0x4F78);  // vmcnt(24)
        else
          __builtin_amdgcn_s_waitcnt(0);
      } else if (wave >= 5) {
        if (k > 0) store_out(bx, by, 8 * (k - 1), (k - 1) & 1);
        if constexpr (kGrad) load_mask(bx, by, 8 * k);  // for the store of tile k
      } else {
        floatx4 acc[2][NB];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[q][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        const char* ring = reinterpret_cast<const char*>(sRing);
        // fragments of tap tt: B from the weights, A from the planes (voxel
        // of row r shifted by the tap); the next tap's are read while this
        // tap's matrix instructions run
        auto frags = [&](int tt, bf16x8 (&bc)[NB], bf16x8 (&af)[2]) {
          const int dz = sgn * (tt / 9 - 1), dy = sgn * ((tt / 3) % 3 - 1), dx = sgn * (tt % 3 - 1);
#pragma unroll
          for (int j = 0; j < NB; ++j)
            bc[j] = *reinterpret_cast<const bf16x8*>(&sW[tt][16 * j + r][kq ^ ((r >> 2) & 3)]);
          const int yy = oy + 1 + dy;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int zs = (8 * k + wave * 2 + q + 1 + dz) % kRing;  // plane z = 8k + zi - 1
            af[q] = *reinterpret_cast<const bf16x8*>(
                ring + zs * kResPlane + (yy * 6 + ox + 1 + dx) * 64 + ((kq ^ (yy & 3)) << 4));
          }
        };
        bf16x8 bc[2][NB], af[2][2];
        frags(0, bc[0], af[0]);
#pragma unroll
        for (int tt = 0; tt < 27; ++tt) {
          const int cur = tt & 1;
          if (tt + 1 < 27) frags(tt + 1, bc[cur ^ 1], af[cur ^ 1]);
          __builtin_amdgcn_sched_barrier(0);  // keep those reads ahead of the MFMAs below
#pragma unroll
          for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int j = 0; j < NB; ++j)
              acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[cur][q], bc[cur][j],
                                                                  acc[q][j], 0, 0, 0);
        }
        // epilogue into sOut: row 4 (lane >> 4) + e of slice 2 wave + q is
        // local voxel (x, y, z) = (rr & 3, rr >> 2, 2 wave + q)
        char* dst = reinterpret_cast<char*>(sOut[k & 1]);
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const int nl = j * 16 + (lane & 15);
            const int vl0 = ((wave * 2 + q) * 4 + (lane >> 4)) * 4;  // the voxel of e = 0
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              v[e] = acc[q][j][e] + sBias[nl];
              if (a.relu) v[e] = fmaxf(v[e], 0.f);
            }
            if constexpr (kF32 || kGrad) {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                *reinterpret_cast<float*>(dst + sout_off<NB, 4>(vl0 + e, nl * 4)) = v[e];
            } else {
              // two adjacent channels of one voxel per 32-bit write: lanes
              // 2m and 2m + 1 (channels nl, nl + 1) swap one value, the even
              // lane then holds voxel e0's pair, the odd lane voxel e0 + 1's
              const bool odd = lane & 1;
#pragma unroll
              for (int e0 = 0; e0 < 4; e0 += 2) {
                const float send = odd ? v[e0] : v[e0 + 1];
                const float recv = __int_as_float(
                    __builtin_amdgcn_mov_dpp(__float_as_int(send), 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
                floatx2 pr;
                pr.x = odd ? recv : v[e0];
                pr.y = odd ? v[e0 + 1] : recv;
                *reinterpret_cast<uint32_t*>(dst + sout_off<NB, 2>(vl0 + e0 + (odd ? 1 : 0), (nl & ~1) * 2)) =
                    __builtin_bit_cast(uint32_t, __builtin_convertvector(pr, bf16x2v));
              }
            }
          }
      }
      __syncthreads();
    }
    // the column's last tile; the ring and the output tiles are reused next
    if (wave >= 5) store_out(bx, by, 8 * (tz_n - 1), (tz_n - 1) & 1);
    __syncthreads();
  }
  if constexpr (kGrad) {
    // the workgroup's channel sums, added in a fixed order
    __shared__ float sRed[2][64][8];
    if (wave >= 5)
#pragma unroll
      for (int j = 0; j < 8; ++j) sRed[wave - 5][lane][j] = gsum[j];
    __syncthreads();
    if (tid < NC) {
      const int k = tid >> 3, j = tid & 7;
      float sum = 0.f;
      for (int w = 0; w < 2; ++w)
        for (int l = k; l < 64; l += 4) sum += sRed[w][l][j];
      a.gpart[static_cast<int64_t>(blockIdx.x) * a.cout + n0 + tid] = sum;
    }
  }
}

// ------------------------------------------ 3x3x3 conv with one gathered channel
// kConv3 / kConv3T with cin == 1 (the input layer's forward pass, the output
// layer's input gradient): the 27 taps are the reduction axis (one MFMA
// step, taps 27..31 zero).  A workgroup owns a 4 x 4 x 4 tile (wave w: the
// z-slice w) and 16 NB output channels; the tile's 6 x 6 x 6 input brick is
// staged in LDS and the B fragments Bt[n][t] are read once from the packed
// weights (kpad >= 32, zero beyond tap 26).
template <int NB>
__global__ void __launch_bounds__(256) conv3_scalar_kernel(ConvArgs a) {
  __shared__ uint16_t sB[216];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tx_n = (a.w + 3) >> 2, ty_n = (a.h + 3) >> 2;
  const int tile = blockIdx.x;
  const int bx = (tile % tx_n) * 4;
  const int by = ((tile / tx_n) % ty_n) * 4;
  const int bz = (tile / (tx_n * ty_n)) * 4;
  const int n0 = blockIdx.y * 16 * NB;
  const int sgn = a.geo == kConv3 ? 1 : -1;
  const int r = lane & 15, g = lane >> 4;
  for (int v = tid; v < 216; v += 256) {
    const int gx = bx + v % 6 - 1, gy = by + (v / 6) % 6 - 1, gz = bz + v / 36 - 1;
    uint16_t val = 0;
    if (gx >= 0 && gy >= 0 && gz >= 0 && gx < a.in_w && gy < a.in_h && gz < a.in_d)
      val = a.x[(static_cast<int64_t>(gz) * a.in_h + gy) * a.in_w + gx];
    sB[v] = val;
  }
  bf16x8 bf[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j)
    bf[j] = *reinterpret_cast<const bf16x8*>(a.bt + static_cast<int64_t>(n0 + 16 * j + r) * a.kpad +
                                            8 * g);
  __syncthreads();
  // A row r = voxel (r & 3, r >> 2, wave) of the tile; k = tap 8 g + j
  bf16x8 af;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int t = 8 * g + j;
    uint16_t e = 0;
    if (t < 27) {
      const int dz = sgn * (t / 9 - 1), dy = sgn * ((t / 3) % 3 - 1), dx = sgn * (t % 3 - 1);
      e = sB[((wave + 1 + dz) * 6 + ((r >> 2) + 1 + dy)) * 6 + ((r & 3) + 1 + dx)];
    }
    af[j] = __builtin_bit_cast(__bf16, e);
  }
  floatx4 acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j)
    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[j], floatx4{0.f, 0.f, 0.f, 0.f}, 0,
                                                     0, 0);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int n = n0 + j * 16 + r;
    if (n >= a.cout) continue;
    const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int rr = 4 * g + e;
      const int x = bx + (rr & 3), y = by + (rr >> 2), z = bz + wave;
      if (x >= a.w || y >= a.h || z >= a.d) continue;
      const int64_t o = (static_cast<int64_t>(z) * a.h + y) * a.w + x;
      float v = acc[j][e] + bias;
      if (a.skip) v += from_bf16(a.skip[o * a.cout + n]);
      if (a.relu) v = fmaxf(v, 0.f);
      if (a.y_f32)
        static_cast<float*>(a.y)[o * a.cout + n] = v;
      else
        static_cast<uint16_t*>(a.y)[o * a.cout + n] = to_bf16(v);
    }
  }
}

// Finish a split product: y[o][n] = [relu](sum over splits of part[s][o][n]
// + bias[n] [+ skip[o][n]]), splits summed in order.
__global__ void __launch_bounds__(256) split_reduce_kernel(ConvArgs a, int nsplit) {
  const int64_t n_out = static_cast<int64_t>(a.d) * a.h * a.w * a.cout;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n_out;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int n = static_cast<int>(i % a.cout);
    float v = a.part[i];
    for (int sp = 1; sp < nsplit; ++sp) v += a.part[sp * n_out + i];
    v += a.bias ? a.bias[n] : 0.f;
    if (a.skip) v += from_bf16(a.skip[i]);
    if (a.relu) v = fmaxf(v, 0.f);
    if (a.y_f32)
      static_cast<float*>(a.y)[i] = v;
    else
      static_cast<uint16_t*>(a.y)[i] = to_bf16(v);
  }
}

// ------------------------------------------------------------ weight GEMM
// gw[p][n] += sum over the workgroup's voxels of A(m, p) gy(m, n), with
// p = t * cin + ci.  kConv3 / kDown: m runs over the output grid, A is x
// gathered at the tap; kUp: m runs over the input grid, A = x[m] and gy is
// read at the parity-class position of tap t (all rows of a tile share t).
template <int NB, bool kVec>
__global__ void __launch_bounds__(256) wgrad_kernel(WgradArgs a) {
  __shared__ uint16_t sA[kBM][kBK + kPadK];       // [p][m]
  __shared__ uint16_t sB[16 * NB][kBK + kPadK];   // [n][m]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t M = static_cast<int64_t>(a.d) * a.h * a.w;
  const int64_t mb = static_cast<int64_t>(blockIdx.x) * a.m_per_block;
  const int64_t me = mb + a.m_per_block < M ? mb + a.m_per_block : M;
  const int n0 = blockIdx.z * 16 * NB;
  const int P = a.taps * a.cin;
  // rows of this tile
  int p0, t_up = 0, prow_lim;
  if (a.geo == kUp) {
    const int tiles = (a.cin + kBM - 1) / kBM;
    t_up = blockIdx.y / tiles;
    p0 = t_up * a.cin + (blockIdx.y % tiles) * kBM;
    prow_lim = t_up * a.cin + a.cin;
  } else {
    p0 = blockIdx.y * kBM;
    prow_lim = P;
  }

  floatx4 acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int64_t m0 = mb; m0 < me; m0 += kBK) {
    // A: 64 rows (p) x 32 voxels, loaded 8 rows of one voxel per thread
    {
      const int mm = tid >> 3, rc = (tid & 7) * 8;
      const int64_t m = m0 + mm;
      uint16_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = 0;
      if (m < me) {
        const int x = static_cast<int>(m % a.w);
        const int y = static_cast<int>((m / a.w) % a.h);
        const int z = static_cast<int>(m / (static_cast<int64_t>(a.w) * a.h));
        const int p = p0 + rc;
        if constexpr (kVec) {
          if (p < prow_lim) {
            const int t = p / a.cin, ci = p - t * a.cin;
            const int64_t src = a.geo == kUp ? m : gather_at(a.g, z, y, x, t);
            if (src >= 0) {
              const uint4 v = *reinterpret_cast<const uint4*>(a.x + src * a.cin + ci);
              e[0] = v.x & 0xffff; e[1] = v.x >> 16; e[2] = v.y & 0xffff; e[3] = v.y >> 16;
              e[4] = v.z & 0xffff; e[5] = v.z >> 16; e[6] = v.w & 0xffff; e[7] = v.w >> 16;
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int pj = p + j;
            if (pj < prow_lim) {
              const int t = pj / a.cin, ci = pj - t * a.cin;
              const int64_t src = a.geo == kUp ? m : gather_at(a.g, z, y, x, t);
              if (src >= 0) e[j] = a.x[src * a.cin + ci];
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) sA[rc + j][mm] = e[j];
    }
    // B: 16*NB channels x 32 voxels of gy
    for (int i = tid; i < 2 * NB * kBK; i += 256) {
      const int nc = (i % (2 * NB)) * 8, mm = i / (2 * NB);
      const int64_t m = m0 + mm;
      uint16_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = 0;
      if (m < me) {
        int64_t gi = m;
        if (a.geo == kUp) {
          const int x = static_cast<int>(m % a.w);
          const int y = static_cast<int>((m / a.w) % a.h);
          const int z = static_cast<int>(m / (static_cast<int64_t>(a.w) * a.h));
          gi = (static_cast<int64_t>(2 * z + (t_up >> 2)) * (2 * a.h) + 2 * y + ((t_up >> 1) & 1)) *
                   (2 * a.w) + 2 * x + (t_up & 1);
        }
        const uint16_t* row = a.gy + gi * a.cout + n0 + nc;
        if (a.cout % 8 == 0 && n0 + nc + 8 <= a.cout) {
          const uint4 v = *reinterpret_cast<const uint4*>(row);
          e[0] = v.x & 0xffff; e[1] = v.x >> 16; e[2] = v.y & 0xffff; e[3] = v.y >> 16;
          e[4] = v.z & 0xffff; e[5] = v.z >> 16; e[6] = v.w & 0xffff; e[7] = v.w >> 16;
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = (n0 + nc + j < a.cout) ? row[j] : 0;
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) sB[nc + j][mm] = e[j];
    }
    __syncthreads();
    const bf16x8 af = *reinterpret_cast<const bf16x8*>(&sA[wave * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bf16x8 bf = *reinterpret_cast<const bf16x8*>(&sB[j * 16 + (lane & 15)][(lane >> 4) * 8]);
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int n = n0 + j * 16 + (lane & 15);
    if (n >= a.cout) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = p0 + wave * 16 + (lane >> 4) * 4 + i;
      if (p < prow_lim && acc[j][i] != 0.f)
        unsafeAtomicAdd(a.gw + static_cast<int64_t>(p) * a.cout + n, acc[j][i]);
    }
  }
}

// ---------------------------------------- 3x3x3 weight gradient from a slab
// kConv3 layers with cin a multiple of 32.  A workgroup owns one chunk of 32
// input channels (blockIdx.y % chunks), one plane dz = blockIdx.y / chunks
// of taps (the 9 taps t = 9 dz + 3 dy + dx) and 32 NBW output channels
// (blockIdx.z), and walks the 4 x 4 x kSlabTZ voxel tiles blockIdx.x,
// blockIdx.x + gridDim.x, ...  Per tile it stages the kSlabTZ x 6 x 6 slab of x
// the plane's taps read (zero outside the volume), transposed to channel
// rows in three copies, one per tap column dx, each holding the 4 x
// positions dx .. dx + 3 of every (z, y) row of the slab -- so that an A
// fragment (8 voxels: two rows of 4 in x) is two aligned 8-byte reads --
// and the tile's gy transposed to [n][m]; wave w then accumulates the 16
// input channels 16 (w & 1).. and 16 NBW output channels of its half
// (w >> 1) for all 9 taps, with the tile's 16 kSlabTZ voxels on the MFMA's
// reduction axis (kSlabTZ / 2 steps of 32: tiles of 8 z-slices halve the
// staging round trips -- global loads, the transpose, two barriers -- per
// matrix instruction against 4).  The sums are stored to
// part[blockIdx.x][t][ci][n] and wgrad_reduce_kernel adds them to gw in a
// fixed order.
constexpr int kSlabTZ = 8;                     // z-slices per tile
constexpr int kSlabRow = kSlabTZ * 6 * 4 + 4;  // one channel's (z, y, 4 x) of a copy, padded
template <int NBW>
__global__ void __launch_bounds__(256) wgrad_slab_kernel(WgradArgs a) {
  __shared__ __align__(16) uint16_t sXT[3][32][kSlabRow];  // copy dx, channel, (z, y, x - dx)
  __shared__ uint16_t sG[32 * NBW][16 * kSlabTZ + kPadK];  // output channel, tile voxel
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int chunks = a.cin / kBK;
  const int c0 = static_cast<int>(blockIdx.y % chunks) * kBK;
  const int dz = static_cast<int>(blockIdx.y / chunks);
  const int n0 = static_cast<int>(blockIdx.z) * 32 * NBW;
  const int cb = wave & 1;
  const int nw = (wave >> 1) * 16 * NBW;  // this wave's first channel within the group
  const int tx_n = (a.w + 3) >> 2, ty_n = (a.h + 3) >> 2, tz_n = (a.d + kSlabTZ - 1) / kSlabTZ;
  const int tiles = tx_n * ty_n * tz_n;
  const int P = a.taps * a.cin;

  floatx4 acc[9][NBW];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < NBW; ++j) acc[t][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // This thread's staging loads of one tile, held in registers so that the
  // next tile's loads are in flight while the current one is computed:
  // slab item tid (< kSlabTZ * 6 * 4): one (z, y) row of the slab and
  // 8-channel chunk, its 6 voxels; output-gradient items tid + 256 u: one
  // voxel of the tile and 8 output channels.
  constexpr int kXI = kSlabTZ * 6 * 4;
  constexpr int kGI = 16 * kSlabTZ * 4 * NBW / 256;
  static_assert(kXI <= 256 && kGI * 256 == 16 * kSlabTZ * 4 * NBW, "staging items per thread");
  uint4 xv[6], gv[kGI];
  auto load = [&](int tile) {
    const int bx = (tile % tx_n) * 4;
    const int by = ((tile / tx_n) % ty_n) * 4;
    const int bz = (tile / (tx_n * ty_n)) * kSlabTZ;
    if (tid < kXI) {
      const int oc = tid & 3, yy = (tid >> 2) % 6, zz = (tid >> 2) / 6;
      const int gy = by + yy - 1, gz = bz + zz + dz - 1;
      const bool row_in = gy >= 0 && gz >= 0 && gy < a.g.in_h && gz < a.g.in_d;
#pragma unroll
      for (int xx = 0; xx < 6; ++xx) {
        const int gx = bx + xx - 1;
        xv[xx] = make_uint4(0u, 0u, 0u, 0u);
        if (row_in && gx >= 0 && gx < a.g.in_w)
          xv[xx] = *reinterpret_cast<const uint4*>(
              a.x + ((static_cast<int64_t>(gz) * a.g.in_h + gy) * a.g.in_w + gx) * a.cin + c0 +
              oc * 8);
      }
    }
#pragma unroll
    for (int u = 0; u < kGI; ++u) {
      const int i = tid + 256 * u;
      const int m = i / (4 * NBW), nc = (i % (4 * NBW)) * 8;
      const int x = bx + (m & 3), y = by + ((m >> 2) & 3), z = bz + (m >> 4);
      gv[u] = make_uint4(0u, 0u, 0u, 0u);
      if (x < a.w && y < a.h && z < a.d) {
        const uint16_t* row =
            a.gy + ((static_cast<int64_t>(z) * a.h + y) * a.w + x) * a.cout + n0 + nc;
        if (a.cout % 8 == 0 && n0 + nc + 8 <= a.cout) {
          gv[u] = *reinterpret_cast<const uint4*>(row);
        } else {
          uint32_t h[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) h[j] = (n0 + nc + j < a.cout) ? row[j] : 0u;
          gv[u] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                             h[6] | (h[7] << 16));
        }
      }
    }
  };
  // the registers into LDS: each channel of the slab row as its 4-voxel runs
  // starting at x = 0, 1, 2; the output gradient transposed to [n][m]
  auto store = [&]() {
    if (tid < kXI) {
      const int oc = tid & 3, yy = (tid >> 2) % 6, zz = (tid >> 2) / 6;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        uint32_t e[6];  // channel oc * 8 + c of the row's 6 voxels
#pragma unroll
        for (int xx = 0; xx < 6; ++xx) {
          const uint32_t w32 = (&xv[xx].x)[c >> 1];
          e[xx] = (c & 1) ? (w32 >> 16) : (w32 & 0xffffu);
        }
#pragma unroll
        for (int d0 = 0; d0 < 3; ++d0)
          *reinterpret_cast<uint2*>(&sXT[d0][oc * 8 + c][(zz * 6 + yy) * 4]) =
              make_uint2(e[d0] | (e[d0 + 1] << 16), e[d0 + 2] | (e[d0 + 3] << 16));
      }
    }
#pragma unroll
    for (int u = 0; u < kGI; ++u) {
      const int i = tid + 256 * u;
      const int m = i / (4 * NBW), nc = (i % (4 * NBW)) * 8;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t w32 = (&gv[u].x)[j >> 1];
        sG[nc + j][m] = static_cast<uint16_t>((j & 1) ? (w32 >> 16) : (w32 & 0xffffu));
      }
    }
  };

  if (static_cast<int>(blockIdx.x) < tiles) load(blockIdx.x);
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    __syncthreads();  // the previous tile's fragments have been read
    store();
    __syncthreads();
    if (tile + static_cast<int>(gridDim.x) < tiles) load(tile + gridDim.x);
    // B fragments: voxels 32 ks + 8 g .. + 7 of output channel nw + 16 j + r
    bf16x8 bf[kSlabTZ / 2][NBW];
#pragma unroll
    for (int ks = 0; ks < kSlabTZ / 2; ++ks)
#pragma unroll
      for (int j = 0; j < NBW; ++j)
        bf[ks][j] = *reinterpret_cast<const bf16x8*>(&sG[nw + 16 * j + r][32 * ks + 8 * g]);
    // A fragments: channel 16 cb + r of the slab at voxel m + tap offset,
    // m = 32 ks + 8 g + j: x = j & 3, y = 2 (g & 1) + (j >> 2), z = 2 ks + (g >> 1);
    // slab rows y0 + dy and y0 + dy + 1 of copy dx
    const int ci = cb * 16 + r;
#pragma unroll
    for (int ks = 0; ks < kSlabTZ / 2; ++ks) {
      const int zz = 2 * ks + (g >> 1);
      const int y0 = 2 * (g & 1);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int dy = t / 3, dx = t % 3;
        const uint16_t* row = &sXT[dx][ci][(zz * 6 + y0 + dy) * 4];
        const uint2 lo = *reinterpret_cast<const uint2*>(row);
        const uint2 hi = *reinterpret_cast<const uint2*>(row + 4);
        const bf16x8 af = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
#pragma unroll
        for (int j = 0; j < NBW; ++j)
          acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[ks][j], acc[t][j], 0, 0, 0);
      }
    }
  }
  // lane (r, g) holds D[4 g + i][r]: input channel c0 + 16 cb + 4 g + i, output channel
  float* out = a.part + static_cast<int64_t>(blockIdx.x) * P * a.cout;
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
      const int n = n0 + nw + 16 * j + r;
      if (n >= a.cout) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = (9 * dz + t) * a.cin + c0 + 16 * cb + 4 * g + i;
        out[static_cast<int64_t>(p) * a.cout + n] = acc[t][j][i];
      }
    }
}

// ------------------------------------- 3x3x3 weight gradients with one channel
// Taps as a matrix axis (27 of 32 used).  kConv3 layers with cin == 1:
// gw[t][n] = sum_m x[m + d(t)] gy[m][n], rows t, columns n; with cout == 1:
// gw[t][ci] = sum_m x[m][ci] gy[m - d(t)], rows ci, columns t (the same sum
// with m shifted; x and gy are zero outside the volume).  A workgroup
// walks 4 x 4 x 4 tiles blockIdx.x, + gridDim.x, ... and owns 32 columns
// (cin == 1: output channels 32 blockIdx.z ..) or 32 rows (cout == 1: input
// channels 32 blockIdx.z ..); wave w computes the 16 x 16 block (w & 1,
// w >> 1).  Per tile the single-channel side is staged as a 6 x 6 x 6
// brick and the other side transposed to [channel][voxel]; sums go to
// part[blockIdx.x][t][ci][n] for wgrad_reduce_kernel.
template <bool kCin1>
__global__ void __launch_bounds__(256) wgrad_onechannel_kernel(WgradArgs a) {
  __shared__ uint16_t sB[216];                 // brick of the one-channel side
  __shared__ uint16_t sT[32][64 + kPadK];      // [channel][tile voxel] of the other side
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int rb = wave & 1, cb = wave >> 1;     // row block, column block
  const int c0 = static_cast<int>(blockIdx.z) * 32;  // first channel of the many-channel side
  const int cmany = kCin1 ? a.cout : a.cin;
  const int tx_n = (a.w + 3) >> 2, ty_n = (a.h + 3) >> 2, tz_n = (a.d + 3) >> 2;
  const int tiles = tx_n * ty_n * tz_n;
  const int sgn = kCin1 ? 1 : -1;  // brick offset of tap t: x at m + d(t), or gy at m - d(t)
  floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int bx = (tile % tx_n) * 4;
    const int by = ((tile / tx_n) % ty_n) * 4;
    const int bz = (tile / (tx_n * ty_n)) * 4;
    __syncthreads();
    if (tid < 216) {
      const int v = tid;
      const int gx = bx + v % 6 - 1, gy = by + (v / 6) % 6 - 1, gz = bz + v / 36 - 1;
      uint16_t val = 0;
      if (gx >= 0 && gy >= 0 && gz >= 0 && gx < a.w && gy < a.h && gz < a.d) {
        const int64_t o = (static_cast<int64_t>(gz) * a.h + gy) * a.w + gx;
        val = kCin1 ? a.x[o] : a.gy[o];
      }
      sB[v] = val;
    }
    for (int i = tid; i < 64 * 4; i += 256) {
      const int m = i >> 2, cc = (i & 3) * 8;
      const int x = bx + (m & 3), y = by + ((m >> 2) & 3), z = bz + (m >> 4);
      uint16_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = 0;
      if (x < a.w && y < a.h && z < a.d) {
        const int64_t o = (static_cast<int64_t>(z) * a.h + y) * a.w + x;
        const uint16_t* row = (kCin1 ? a.gy : a.x) + o * cmany + c0 + cc;
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = (c0 + cc + j < cmany) ? row[j] : 0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) sT[cc + j][m] = e[j];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      // voxels m = 32 ks + 8 g + j: x = j & 3, y = 2 (g & 1) + (j >> 2), z = 2 ks + (g >> 1)
      const int zz = 2 * ks + (g >> 1), y0 = 2 * (g & 1);
      // brick side: tap t = 16 (kCin1 ? rb : cb) + r at the 8 voxels
      const int t = 16 * (kCin1 ? rb : cb) + r;
      bf16x8 br;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        uint16_t e = 0;
        if (t < 27) {
          const int dz = sgn * (t / 9 - 1), dy = sgn * ((t / 3) % 3 - 1), dx = sgn * (t % 3 - 1);
          e = sB[((zz + 1 + dz) * 6 + (y0 + (j >> 2) + 1 + dy)) * 6 + ((j & 3) + 1 + dx)];
        }
        br[j] = __builtin_bit_cast(__bf16, e);
      }
      // channel side: channel 16 (kCin1 ? cb : rb) + r at the 8 voxels
      const bf16x8 ch = *reinterpret_cast<const bf16x8*>(
          &sT[16 * (kCin1 ? cb : rb) + r][32 * ks + 8 * g]);
      acc = kCin1 ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, ch, acc, 0, 0, 0)
                  : __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, br, acc, 0, 0, 0);
    }
  }
  // lane (r, g) holds D[4 g + i][r] of block (rb, cb)
  float* out = a.part + static_cast<int64_t>(blockIdx.x) * 27 * a.cin * a.cout;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = 16 * rb + 4 * g + i, col = 16 * cb + r;
    const int t = kCin1 ? row : col;
    const int c = c0 + (kCin1 ? col : row);
    if (t < 27 && c < cmany) out[static_cast<int64_t>(t) * cmany + c] = acc[i];
  }
}

// the same for fewer than 8 workgroups: one thread per i
__global__ void wgrad_reduce_few_kernel(const float* part, int groups, int64_t n, float* gw) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float v = part[i];
    for (int k = 1; k < groups; ++k) v += part[k * n + i];
    gw[i] += v;
  }
}

// gw[i] += sum over the workgroups k < groups of part[k][i]: a workgroup
// takes E = 256 / KL consecutive i; thread (q, il) sums k = q, q + KL, ...
// for i = E blockIdx.x + il, and the KL sums of each i are added in q order
template <int KL>
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* part, int groups,
                                                           int64_t n, float* gw) {
  constexpr int E = 256 / KL;
  __shared__ float sh[KL][E + 1];
  const int il = threadIdx.x % E, q = threadIdx.x / E;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * E + il;
  float v = 0.f;
  if (i < n)
    for (int k = q; k < groups; k += KL) v += part[k * n + i];
  sh[q][il] = v;
  __syncthreads();
  if (q == 0 && i < n) {
    float t = sh[0][il];
#pragma unroll
    for (int k = 1; k < KL; ++k) t += sh[k][il];
    gw[i] += t;
  }
}

// ------------------------------------------------------------ element-wise

// Bt[n][koff(t) + ci] from w[t][ci][n] (forward packing) or
// Bt[ci][t * cout + n] from w[t][ci][n] (transposed packing); rows and
// columns beyond the matrix stay zero (the buffer is cleared first).
__global__ void pack_kernel(const float* w, int taps, int cin, int cout, int kpad, int transposed,
                            uint16_t* bt) {
  const int64_t total = static_cast<int64_t>(taps) * cin * cout;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int n = static_cast<int>(i % cout);
    const int ci = static_cast<int>((i / cout) % cin);
    const int t = static_cast<int>(i / (static_cast<int64_t>(cout) * cin));
    const uint16_t v = to_bf16(w[i]);
    if (transposed)
      bt[static_cast<int64_t>(ci) * kpad + t * cout + n] = v;
    else
      bt[static_cast<int64_t>(n) * kpad + t * cin + ci] = v;
  }
}

__global__ void fill_u16_kernel(uint16_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

__global__ void zero2_kernel(double* acc, float* fmax) {
  acc[0] = 0.0;
  acc[1] = 0.0;
  fmax[0] = 0.f;
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// u = (ln max(phi, eps) - shift) / scale, in FP32 and as BF16
__global__ void to_log_kernel(const float* phi, int64_t n, float eps, float shift, float inv_scale,
                              float* u, uint16_t* u16) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float v = (logf(fmaxf(phi[i], eps)) - shift) * inv_scale;
    if (u) u[i] = v;
    if (u16) u16[i] = to_bf16(v);
  }
}

// out[z][y][x] = in[z][y'][x'], (x', y') = (op & 4 ? (y, x) : (x, y)) with
// x' mirrored when op & 1 and y' when op & 2: the eight symmetries of a
// square cross-section (the swap needs nx == ny)
__global__ void mirror_xy_kernel(const float* in, float* out, int nx, int ny, int64_t n, int op) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(i % nx);
    const int64_t r = i / nx;
    const int y = static_cast<int>(r % ny);
    const int64_t z = r / ny;
    int sx = (op & 4) ? y : x;
    int sy = (op & 4) ? x : y;
    if (op & 1) sx = nx - 1 - sx;
    if (op & 2) sy = ny - 1 - sy;
    out[i] = in[(z * ny + sy) * nx + sx];
  }
}

// acc[i] (= when first, else +=) in[src(i)]: the gather of mirror_xy_kernel
// for the symmetry op, accumulated
__global__ void mirror_acc_kernel(const float* in, float* acc, int nx, int ny, int64_t n, int op,
                                  int first) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(i % nx);
    const int64_t r = i / nx;
    const int y = static_cast<int>(r % ny);
    const int64_t z = r / ny;
    int sx = (op & 4) ? y : x;
    int sy = (op & 4) ? x : y;
    if (op & 1) sx = nx - 1 - sx;
    if (op & 2) sy = ny - 1 - sy;
    const float v = in[(z * ny + sy) * nx + sx];
    acc[i] = first ? v : acc[i] + v;
  }
}

// the mean of nsym outputs in u space and its fluence
__global__ void sym_finish_kernel(const float* acc, int64_t n, float inv_nsym, float scale,
                                  float shift, float* out_u, float* phi) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float v = acc[i] * inv_nsym;
    if (out_u) out_u[i] = v;
    if (phi) phi[i] = expf(v * scale + shift);
  }
}

// phi_out = exp((r + u) * scale + shift): output of the residual network
__global__ void from_log_kernel(const float* r, const float* u, int64_t n, float scale, float shift,
                                float* out_u, float* phi) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float v = r[i] + u[i];
    if (out_u) out_u[i] = v;
    if (phi) phi[i] = expf(v * scale + shift);
  }
}

// g16 = bf16((g + skip16) * (y16 > 0)); g may be FP32 or absent (skip
// only).  With `partial` set (and 256 a multiple of cout, so that a thread
// sees one channel in every grid-stride step) each block also writes its
// per-channel sums of g16 to partial[block][cout] for bias_sum_kernel.
__global__ void __launch_bounds__(256) relu_grad_kernel(const float* g, const uint16_t* skip16,
                                                        const uint16_t* y16, int64_t n, int cout,
                                                        uint16_t* g16, float* partial) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float v = g ? g[i] : 0.f;
    if (skip16) v += from_bf16(skip16[i]);
    if (y16 && !(from_bf16(y16[i]) > 0.f)) v = 0.f;
    const uint16_t h = to_bf16(v);
    g16[i] = h;
    s += from_bf16(h);
  }
  if (!partial) return;
  // thread j's sums are of channel j % cout (cout a power of two dividing
  // 256): halve the block's 256 sums down to cout, pairing threads of one
  // channel (a tree, not one thread adding 256 / cout values in a row)
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off >= cout; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (static_cast<int>(threadIdx.x) < cout)
    partial[static_cast<int64_t>(blockIdx.x) * cout + threadIdx.x] = sh[threadIdx.x];
}

// gb[c] += sum over blocks of partial[block][c]; one workgroup per channel
__global__ void __launch_bounds__(256) bias_sum_kernel(const float* partial, int blocks, int cout,
                                                       float* gb) {
  __shared__ float sh[4];
  const int c = blockIdx.x;
  float t = 0.f;
  for (int b = threadIdx.x; b < blocks; b += blockDim.x)
    t += partial[static_cast<int64_t>(b) * cout + c];
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) gb[c] += sh[0] + sh[1] + sh[2] + sh[3];
}

// the bias_sum_kernel sums of several layers in one launch: workgroup x
// takes channel x of the concatenated channels of `jobs`
__global__ void __launch_bounds__(256) bias_sums_kernel(const BiasJob* jobs, int njobs,
                                                        const float* partial, float* grads) {
  __shared__ float sh[4];
  int c = blockIdx.x, j = 0;
  while (j + 1 < njobs && c >= jobs[j].cout) c -= jobs[j++].cout;
  const BiasJob J = jobs[j];
  const float* p = partial + J.partial_off;
  float t = 0.f;
  for (int b = threadIdx.x; b < J.blocks; b += blockDim.x)
    t += p[static_cast<int64_t>(b) * J.cout + c];
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) grads[J.gb_off + c] += sh[0] + sh[1] + sh[2] + sh[3];
}

// block-wide sum of one double per thread (256 threads), returned to thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// masked squared error of out against target (both in u space): sum and
// count into acc[0..1] (FP64, one atomic per block), and the unnormalised
// gradient 2 (out - t) per masked voxel (zero elsewhere)
__global__ void __launch_bounds__(256) mse_kernel(const float* out, const float* target_u,
                                                  const float* target_phi, float rel_floor,
                                                  const float* phi_max, int64_t n, float* grad,
                                                  double* acc) {
  __shared__ double sh[4];
  double s = 0.0, c = 0.0;
  const float thr = rel_floor * phi_max[0];
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const bool on = target_phi[i] >= thr;
    const float d = on ? out[i] - target_u[i] : 0.f;
    grad[i] = 2.f * d;
    s += static_cast<double>(d) * d;
    c += on ? 1.0 : 0.0;
  }
  s = block_sum(s, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(acc, s);
    unsafeAtomicAdd(acc + 1, c);
  }
}

__global__ void __launch_bounds__(256) max_kernel(const float* x, int64_t n, float* out) {
  __shared__ float sh[4];
  float m = 0.f;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    m = fmaxf(m, x[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) m = fmaxf(m, sh[w]);
    atomicMax(reinterpret_cast<int*>(out), __float_as_int(m));  // m >= 0
  }
}

// grad *= 1 / count (count from acc[1])
__global__ void scale_grad_kernel(float* g, int64_t n, const double* acc) {
  const float s = acc[1] > 0.0 ? static_cast<float>(1.0 / acc[1]) : 0.f;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    g[i] *= s;
}

// gb[n] += sum over voxels of gy[m][n]: each block sums a range of rows,
// its threads split as (channel, row phase), then one atomic per channel
__global__ void __launch_bounds__(256) bias_grad_kernel(const uint16_t* gy, int64_t m, int cout,
                                                        int64_t rows_per_block, float* gb) {
  __shared__ float sh[256];
  const int lanes_c = cout < 256 ? cout : 256;       // threads per row
  const int phases = 256 / lanes_c;                  // rows in flight
  const int tid = threadIdx.x;
  const int64_t r0 = blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < m ? r0 + rows_per_block : m;
  for (int c0 = 0; c0 < cout; c0 += lanes_c) {
    float s = 0.f;
    const int c = c0 + tid % lanes_c;
    const int ph = tid / lanes_c;
    if (ph < phases && c < cout)
      for (int64_t r = r0 + ph; r < r1; r += phases) s += from_bf16(gy[r * cout + c]);
    sh[tid] = s;
    __syncthreads();
    if (tid < lanes_c && c0 + tid < cout) {
      float t = 0.f;
      for (int p = 0; p < phases; ++p) t += sh[p * lanes_c + tid];
      unsafeAtomicAdd(gb + c0 + tid, t);
    }
    __syncthreads();
  }
}

// per-block sums of squares of g (for the global gradient norm)
__global__ void __launch_bounds__(256) sumsq_kernel(const float* g, int64_t n, double* partial) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    s += static_cast<double>(g[i]) * g[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Adam with bias-corrected moments on g * scale, where scale also clips
// the global norm: scale = gs * min(1, max_norm / (gs * |g|)) when
// max_norm > 0 (|g|^2 = sum of the `blocks` partial sums)
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2, float gs,
                            float max_norm, const double* partial, int blocks) {
  __shared__ float s_scale;
  if (threadIdx.x == 0) {
    float sc = gs;
    if (max_norm > 0.f) {
      double ss = 0.0;
      for (int b = 0; b < blocks; ++b) ss += partial[b];
      const double norm = gs * sqrt(ss);
      if (norm > max_norm) sc = static_cast<float>(gs * (max_norm / norm));
    }
    s_scale = sc;
  }
  __syncthreads();
  const float scale = s_scale;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float gi = g[i] * scale;
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

int blocks_for(int64_t n, int per = 256, int cap = 8192) {
  const int64_t b = (n + per - 1) / per;
  return static_cast<int>(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

// --------------------------------------------------------------- launchers

namespace {

constexpr int64_t kSplitTargetGroups = 1024;  // about four workgroups per CU
constexpr int64_t kSplitBelowGroups = 512;    // split only launches smaller than this
constexpr int64_t kDeepTileGroups = 1024;     // 4 x 4 x 8 tiles when at least this many

int conv_nb(const ConvArgs& a) { return a.cout > 32 ? 4 : (a.cout > 16 ? 2 : 1); }

bool uses_brick(const ConvArgs& a) {
  return (a.geo == kConv3 || a.geo == kConv3T) && a.cin % kBK == 0;
}

// The resident-weights kernel: 3x3x3 layers gathering exactly 32 channels,
// without a skip input, on grids of at least kResidentTiles 4 x 4 x 8 tiles
// (the full-resolution layers; smaller grids keep the brick kernel, whose
// split reductions fill the chip).
constexpr int64_t kResidentTiles = 1024;
int64_t brick_tiles(const ConvArgs& a, int mz);
bool uses_resident(const ConvArgs& a) {
  return (a.geo == kConv3 || a.geo == kConv3T) && a.cin == 32 && !a.skip &&
         brick_tiles(a, 2) >= kResidentTiles;
}

// 4 x 4 columns of the grid, each a workgroup's unit of work
int64_t resident_columns(const ConvArgs& a) {
  return static_cast<int64_t>((a.w + 3) / 4) * ((a.h + 3) / 4);
}

// compute units of the current device (queried once)
int device_cus() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    return n;
  }();
  return cus;
}

int64_t brick_tiles(const ConvArgs& a, int mz) {
  return static_cast<int64_t>((a.w + 3) / 4) * ((a.h + 3) / 4) * ((a.d + 4 * mz - 1) / (4 * mz));
}

int64_t brick_ngroups(const ConvArgs& a) {
  const int nb = conv_nb(a);
  return (a.cout + 16 * nb - 1) / (16 * nb);
}

// z-slices per wave: two when the launch keeps at least kDeepTileGroups
// workgroups with them
int brick_mz(const ConvArgs& a) {
  return brick_tiles(a, 2) * brick_ngroups(a) >= kDeepTileGroups ? 2 : 1;
}

// splits of the brick kernel's input-channel chunks: for launches of fewer
// than two workgroups per CU, enough to fill the chip, a divisor of the
// chunk count, within `cap` floats (measured: on 8^3 and 16^3 grids the
// split runs 6x and 1.8x faster; at 512 workgroups it gains nothing)
int brick_splits(const ConvArgs& a, int64_t cap) {
  const int64_t groups = brick_tiles(a, brick_mz(a)) * brick_ngroups(a);
  if (groups >= kSplitBelowGroups) return 1;
  const int chunks = a.cin / kBK;
  int sp = static_cast<int>(std::min<int64_t>(chunks, (kSplitTargetGroups + groups - 1) / groups));
  const int64_t per = static_cast<int64_t>(a.d) * a.h * a.w * a.cout;
  while (sp > 1 && (chunks % sp != 0 || sp * per > cap)) --sp;
  return sp < 1 ? 1 : sp;
}

}  // namespace

// the folded input gradient: resident-weights kConv3T products of 32
// channels to 32, without bias or ReLU of their own
bool conv_folds_grad(const ConvArgs& a) {
  return a.geo == kConv3T && uses_resident(a) && a.cout == 32 && !a.bias && !a.relu && !a.y_f32;
}

int conv_fold_rows(const ConvArgs& a) {
  return static_cast<int>(std::min<int64_t>(resident_columns(a), device_cus()));
}

// splits of the generic kernel's reduction for kDown products (the other
// geometries are not split): for launches of fewer than two workgroups per
// CU, enough to fill the chip, at least one stage of 128 per split, within
// `cap` floats
int generic_splits(const ConvArgs& a, int64_t cap) {
  if (a.geo != kDown || a.cin % 8 != 0) return 1;
  const int64_t M = static_cast<int64_t>(a.d) * a.h * a.w;
  const int64_t groups = (M + kBM - 1) / kBM * ((a.cout + 16 * conv_nb(a) - 1) / (16 * conv_nb(a)));
  if (groups >= kSplitBelowGroups) return 1;
  int sp = static_cast<int>(std::min<int64_t>(a.k / (4 * kBK), (kSplitTargetGroups + groups - 1) / groups));
  while (sp > 1 && sp * M * a.cout > cap) --sp;
  return sp < 1 ? 1 : sp;
}

int64_t conv_workspace_floats(const ConvArgs& a) {
  const int64_t per = static_cast<int64_t>(a.d) * a.h * a.w * a.cout;
  if (!uses_brick(a)) {
    const int sp = generic_splits(a, INT64_MAX);
    return sp > 1 ? sp * per : 0;
  }
  const int sp = brick_splits(a, INT64_MAX);
  return sp > 1 ? sp * per : 0;
}

hipError_t launch_conv(const ConvArgs& a, hipStream_t s) {
  const int64_t M = static_cast<int64_t>(a.d) * a.h * a.w;
  const int nb = conv_nb(a);
  if ((a.geo == kConv3 || a.geo == kConv3T) && a.cin == 1) {
    const dim3 grid(static_cast<unsigned>(brick_tiles(a, 1)),
                    static_cast<unsigned>(brick_ngroups(a)), 1);
    if (nb == 4)
      conv3_scalar_kernel<4><<<grid, 256, 0, s>>>(a);
    else if (nb == 2)
      conv3_scalar_kernel<2><<<grid, 256, 0, s>>>(a);
    else
      conv3_scalar_kernel<1><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
  }
  if (a.gmask && (!conv_folds_grad(a) || !a.gpart)) return hipErrorInvalidValue;
  if (uses_resident(a)) {
    const int nbr = a.cout > 16 ? 2 : 1;
    const dim3 grid(static_cast<unsigned>(std::min<int64_t>(resident_columns(a), device_cus())),
                    static_cast<unsigned>((a.cout + 16 * nbr - 1) / (16 * nbr)), 1);
    if (a.gmask)  // conv_folds_grad: 32 output channels, BF16
      conv3_resident_kernel<2, false, true><<<grid, 448, 0, s>>>(a);
    else if (nbr == 2 && a.y_f32)
      conv3_resident_kernel<2, true, false><<<grid, 448, 0, s>>>(a);
    else if (nbr == 2)
      conv3_resident_kernel<2, false, false><<<grid, 448, 0, s>>>(a);
    else if (a.y_f32)
      conv3_resident_kernel<1, true, false><<<grid, 448, 0, s>>>(a);
    else
      conv3_resident_kernel<1, false, false><<<grid, 448, 0, s>>>(a);
    return hipGetLastError();
  }
  if (uses_brick(a)) {
    const int mz = brick_mz(a);
    const int sp = a.part ? brick_splits(a, a.part_cap) : 1;
    const dim3 grid(static_cast<unsigned>(brick_tiles(a, mz)),
                    static_cast<unsigned>(brick_ngroups(a)), static_cast<unsigned>(sp));
#define MCX_BRICK(NB)                                                  \
  if (mz == 2)                                                         \
    conv3_brick_kernel<NB, 2><<<grid, 256, 0, s>>>(a);                 \
  else                                                                 \
    conv3_brick_kernel<NB, 1><<<grid, 256, 0, s>>>(a);
    if (nb == 4) { MCX_BRICK(4) } else if (nb == 2) { MCX_BRICK(2) } else { MCX_BRICK(1) }
#undef MCX_BRICK
    if (sp > 1) split_reduce_kernel<<<blocks_for(M * a.cout), 256, 0, s>>>(a, sp);
    return hipGetLastError();
  }
  const int sp = a.part ? generic_splits(a, a.part_cap) : 1;
  const dim3 grid(static_cast<unsigned>((M + kBM - 1) / kBM),
                  static_cast<unsigned>((a.cout + 16 * nb - 1) / (16 * nb)),
                  a.geo == kUp ? 8 : static_cast<unsigned>(sp));
  const bool vec = a.cin % 8 == 0;
  const bool deep = a.k >= 4 * kBK;  // four reduction steps per stage
#define MCX_CONV(NB)                                                   \
  if (vec && deep)                                                     \
    conv_kernel<NB, true, 4><<<grid, 256, 0, s>>>(a);                  \
  else if (vec)                                                        \
    conv_kernel<NB, true, 1><<<grid, 256, 0, s>>>(a);                  \
  else                                                                 \
    conv_kernel<NB, false, 1><<<grid, 256, 0, s>>>(a);
  if (nb == 4) { MCX_CONV(4) } else if (nb == 2) { MCX_CONV(2) } else { MCX_CONV(1) }
#undef MCX_CONV
  if (sp > 1) split_reduce_kernel<<<blocks_for(M * a.cout), 256, 0, s>>>(a, sp);
  return hipGetLastError();
}

namespace {

constexpr int64_t kSlabTargetGroups = 512;
constexpr int64_t kSlabMaxPart = int64_t(8) << 20;  // floats of partial sums at most

bool uses_onechannel(const WgradArgs& a) {
  return a.geo == kConv3 && (a.cin == 1 || (a.cout == 1 && a.cin > 1));
}
bool uses_slab(const WgradArgs& a) {
  return a.geo == kConv3 && a.cin % kBK == 0 && !uses_onechannel(a);
}

// tile groups of the one-channel kernels: about kSlabTargetGroups in all
int onechannel_groups(const WgradArgs& a, int64_t cap) {
  const int64_t tiles = static_cast<int64_t>((a.w + 3) / 4) * ((a.h + 3) / 4) * ((a.d + 3) / 4);
  const int cmany = a.cin == 1 ? a.cout : a.cin;
  const int64_t other = (cmany + 31) / 32;
  int64_t G = std::min<int64_t>(tiles, (kSlabTargetGroups + other - 1) / other);
  const int64_t per = static_cast<int64_t>(a.taps) * a.cin * a.cout;
  while (G > 1 && G * per > cap) G = (G + 1) / 2;
  return static_cast<int>(G < 1 ? 1 : G);
}
int slab_nbw(const WgradArgs& a) { return a.cout > 32 ? 2 : 1; }

// workgroups along the voxel tiles: about kSlabKernelGroups in all (three
// per CU: the slab kernel's loads are latency-bound), at most one per tile,
// with the partial sums within `cap` floats
constexpr int64_t kSlabKernelGroups = 768;
int slab_groups(const WgradArgs& a, int64_t cap) {
  const int64_t tiles =
      static_cast<int64_t>((a.w + 3) / 4) * ((a.h + 3) / 4) * ((a.d + kSlabTZ - 1) / kSlabTZ);
  const int nbw = slab_nbw(a);
  const int64_t other = static_cast<int64_t>(a.cin / kBK) * 3 * ((a.cout + 32 * nbw - 1) / (32 * nbw));
  int64_t G = std::min<int64_t>(tiles, (kSlabKernelGroups + other - 1) / other);
  const int64_t per = static_cast<int64_t>(a.taps) * a.cin * a.cout;
  while (G > 1 && G * per > cap) G = (G + 1) / 2;
  return static_cast<int>(G < 1 ? 1 : G);
}

}  // namespace

namespace {

// the reduction of G partial sums of n floats into gw
hipError_t launch_wgrad_reduce(const float* part, int G, int64_t n, float* gw, hipStream_t s) {
  if (G < 8)
    wgrad_reduce_few_kernel<<<blocks_for(n), 256, 0, s>>>(part, G, n, gw);
  else if (G >= 64 && n < 8192)  // fewer than 256 workgroups with 8 lanes per i
    wgrad_reduce_kernel<32><<<static_cast<unsigned>((n + 7) / 8), 256, 0, s>>>(part, G, n, gw);
  else
    wgrad_reduce_kernel<8><<<static_cast<unsigned>((n + 31) / 32), 256, 0, s>>>(part, G, n, gw);
  return hipGetLastError();
}

}  // namespace

int64_t wgrad_workspace_floats(const WgradArgs& a) {
  if (uses_onechannel(a))
    return onechannel_groups(a, kSlabMaxPart) * static_cast<int64_t>(a.taps) * a.cin * a.cout;
  if (!uses_slab(a)) return 0;
  return slab_groups(a, kSlabMaxPart) * static_cast<int64_t>(a.taps) * a.cin * a.cout;
}

hipError_t launch_wgrad(const WgradArgs& a, hipStream_t s) {
  if (uses_onechannel(a) && a.part) {
    const int64_t per = static_cast<int64_t>(a.taps) * a.cin * a.cout;
    const int G = onechannel_groups(a, a.part_cap);
    if (static_cast<int64_t>(G) * per <= a.part_cap) {
      const int cmany = a.cin == 1 ? a.cout : a.cin;
      const dim3 grid(static_cast<unsigned>(G), 1, static_cast<unsigned>((cmany + 31) / 32));
      if (a.cin == 1)
        wgrad_onechannel_kernel<true><<<grid, 256, 0, s>>>(a);
      else
        wgrad_onechannel_kernel<false><<<grid, 256, 0, s>>>(a);
      return launch_wgrad_reduce(a.part, G, per, a.gw, s);
    }
  }
  if (uses_slab(a) && a.part) {
    const int64_t per = static_cast<int64_t>(a.taps) * a.cin * a.cout;
    const int G = slab_groups(a, a.part_cap);
    if (static_cast<int64_t>(G) * per <= a.part_cap) {
      const int nbw = slab_nbw(a);
      const dim3 grid(static_cast<unsigned>(G), static_cast<unsigned>(a.cin / kBK * 3),
                      static_cast<unsigned>((a.cout + 32 * nbw - 1) / (32 * nbw)));
      if (nbw == 2)
        wgrad_slab_kernel<2><<<grid, 256, 0, s>>>(a);
      else
        wgrad_slab_kernel<1><<<grid, 256, 0, s>>>(a);
      return launch_wgrad_reduce(a.part, G, per, a.gw, s);
    }
  }
  const int64_t M = static_cast<int64_t>(a.d) * a.h * a.w;
  const int nb = a.cout > 32 ? 4 : (a.cout > 16 ? 2 : 1);
  const int P = a.taps * a.cin;
  const int ptiles = a.geo == kUp ? a.taps * ((a.cin + kBM - 1) / kBM) : (P + kBM - 1) / kBM;
  const dim3 grid(static_cast<unsigned>((M + a.m_per_block - 1) / a.m_per_block),
                  static_cast<unsigned>(ptiles),
                  static_cast<unsigned>((a.cout + 16 * nb - 1) / (16 * nb)));
  const bool vec = a.cin % 8 == 0;
#define MCX_WG(NB)                                                     \
  if (vec)                                                             \
    wgrad_kernel<NB, true><<<grid, 256, 0, s>>>(a);                    \
  else                                                                 \
    wgrad_kernel<NB, false><<<grid, 256, 0, s>>>(a);
  if (nb == 4) { MCX_WG(4) } else if (nb == 2) { MCX_WG(2) } else { MCX_WG(1) }
#undef MCX_WG
  return hipGetLastError();
}

hipError_t launch_pack(const float* w, int taps, int cin, int cout, int rows, int kpad,
                       bool transposed, uint16_t* bt, hipStream_t s, bool clear) {
  if (clear)
    fill_u16_kernel<<<blocks_for(static_cast<int64_t>(rows) * kpad), 256, 0, s>>>(
        bt, static_cast<int64_t>(rows) * kpad);
  pack_kernel<<<blocks_for(static_cast<int64_t>(taps) * cin * cout), 256, 0, s>>>(
      w, taps, cin, cout, kpad, transposed ? 1 : 0, bt);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  fill_f32_kernel<<<blocks_for(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_to_log(const float* phi, int64_t n, float* u, uint16_t* u16, hipStream_t s) {
  to_log_kernel<<<blocks_for(n), 256, 0, s>>>(phi, n, kEps, kLogShift, 1.f / kLogScale, u, u16);
  return hipGetLastError();
}

hipError_t launch_mirror_xy(const float* in, float* out, int nx, int ny, int nz, int op,
                            hipStream_t s) {
  const int64_t n = static_cast<int64_t>(nx) * ny * nz;
  mirror_xy_kernel<<<blocks_for(n), 256, 0, s>>>(in, out, nx, ny, n, op);
  return hipGetLastError();
}

hipError_t launch_mirror_acc(const float* in, float* acc, int nx, int ny, int nz, int op,
                             bool first, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(nx) * ny * nz;
  mirror_acc_kernel<<<blocks_for(n), 256, 0, s>>>(in, acc, nx, ny, n, op, first ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_sym_finish(const float* acc, int64_t n, int nsym, float* out_u, float* phi,
                             hipStream_t s) {
  sym_finish_kernel<<<blocks_for(n), 256, 0, s>>>(acc, n, 1.f / static_cast<float>(nsym),
                                                  kLogScale, kLogShift, out_u, phi);
  return hipGetLastError();
}

hipError_t launch_from_log(const float* r, const float* u, int64_t n, float* out_u, float* phi,
                           hipStream_t s) {
  from_log_kernel<<<blocks_for(n), 256, 0, s>>>(r, u, n, kLogScale, kLogShift, out_u, phi);
  return hipGetLastError();
}

hipError_t launch_mse(const float* out, const float* target_u, const float* target_phi,
                      float rel_floor, int64_t n, float* grad, double* acc, float* phi_max,
                      hipStream_t s) {
  // at most 128 blocks: each ends with atomics on one address (one per
  // block for the maximum, two for the sums), which the memory side takes
  // one at a time
  zero2_kernel<<<1, 1, 0, s>>>(acc, phi_max);
  max_kernel<<<blocks_for(n, 256, 128), 256, 0, s>>>(target_phi, n, phi_max);
  mse_kernel<<<blocks_for(n, 256, 128), 256, 0, s>>>(out, target_u, target_phi, rel_floor,
                                                    phi_max, n, grad, acc);
  scale_grad_kernel<<<blocks_for(n), 256, 0, s>>>(grad, n, acc);
  return hipGetLastError();
}

hipError_t launch_bias_grad(const uint16_t* gy, int64_t m, int cout, float* gb, hipStream_t s) {
  const int64_t blocks = m < 512 ? 1 : (m / 256 < 1024 ? m / 256 : 1024);
  const int64_t per = (m + blocks - 1) / blocks;
  bias_grad_kernel<<<static_cast<int>(blocks), 256, 0, s>>>(gy, m, cout, per, gb);
  return hipGetLastError();
}

hipError_t launch_relu_grad(const float* g, const uint16_t* skip16, const uint16_t* y16, int64_t n,
                            int cout, uint16_t* g16, float* gb, float* partial, hipStream_t s) {
  const int blocks = blocks_for(n, 256, kBiasBlocks);
  const bool fused = gb && partial && cout <= 256 && 256 % cout == 0;
  relu_grad_kernel<<<blocks, 256, 0, s>>>(g, skip16, y16, n, cout, g16,
                                          fused ? partial : nullptr);
  if (fused) {
    bias_sum_kernel<<<cout, 256, 0, s>>>(partial, blocks, cout, gb);
    return hipGetLastError();
  }
  if (gb) return launch_bias_grad(g16, n / cout, cout, gb, s);
  return hipGetLastError();
}

bool relu_grad_defers(int cout) { return cout <= 256 && 256 % cout == 0; }

int relu_grad_blocks(int64_t n) { return blocks_for(n, 256, kBiasBlocks); }

hipError_t launch_relu_grad_deferred(const float* g, const uint16_t* skip16, const uint16_t* y16,
                                     int64_t n, int cout, uint16_t* g16, float* gb, float* partial,
                                     hipStream_t s) {
  if (!relu_grad_defers(cout)) return launch_relu_grad(g, skip16, y16, n, cout, g16, gb, nullptr, s);
  relu_grad_kernel<<<relu_grad_blocks(n), 256, 0, s>>>(g, skip16, y16, n, cout, g16, partial);
  return hipGetLastError();
}

hipError_t launch_bias_sums(const BiasJob* jobs, int njobs, int channels, const float* partial,
                            float* grads, hipStream_t s) {
  if (njobs > 0 && channels > 0)
    bias_sums_kernel<<<channels, 256, 0, s>>>(jobs, njobs, partial, grads);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, int step,
                       float grad_scale, float max_norm, double* partial, hipStream_t s) {
  const double c1 = 1.0 - std::pow(0.9, step), c2 = 1.0 - std::pow(0.999, step);
  int blocks = 0;
  if (max_norm > 0.f) {
    blocks = blocks_for(n, 256, kNormBlocks);
    sumsq_kernel<<<blocks, 256, 0, s>>>(g, n, partial);
  }
  adam_kernel<<<blocks_for(n), 256, 0, s>>>(p, g, m, v, n, lr, 0.9f, 0.999f, 1e-8f,
                                            static_cast<float>(c1), static_cast<float>(c2),
                                            grad_scale, max_norm, partial, blocks);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace mcx
