// Internal interfaces of the denoiser kernels (nn_kernels.hip) used by the
// denoiser runtime (nn_runtime.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcx {
namespace nn {

// log-space input transform u = (ln max(phi, kEps) - kLogShift) / kLogScale
constexpr float kEps = 1e-12f;
constexpr float kLogShift = -16.f;
constexpr float kLogScale = 4.f;

enum Geometry : int32_t { kConv3 = 0, kConv3T = 1, kDown = 2, kUp = 3 };

// One implicit-GEMM convolution.  Rows m run over the d x h x w grid
// (kConv3/kConv3T: the output grid = input grid; kDown: the output grid;
// kUp: the input grid, the output being twice as large per axis).
struct ConvArgs {
  int32_t geo;
  int32_t d, h, w;            // grid of rows
  int32_t in_d, in_h, in_w;   // grid of x (for bounds of kConv3/kConv3T)
  int32_t cin, cout;          // channels of x and of y
  int32_t k;                  // reduction length: taps * cin (kUp: cin)
  int32_t kpad;               // row length of bt
  const uint16_t* x;          // BF16 [voxel][cin]
  const uint16_t* bt;         // BF16 [>= cout rounded to 64][kpad]
  const float* bias;          // [cout] or null
  const uint16_t* skip;       // BF16 [out voxel][cout] added before ReLU, or null
  void* y;                    // BF16 or FP32 [out voxel][cout]
  int32_t y_f32, relu;
  float* part;                // FP32 workspace for split reductions, or null (no split)
  int64_t part_cap;           // its size in floats
  // An input gradient with the next step of the backward pass folded in
  // (conv_folds_grad): when gmask is set, y receives the BF16 gradient of
  // the layer below's pre-activation, bf16(sum * (gmask > 0)), and
  // gpart[workgroup][cout] the per-workgroup channel sums of those BF16
  // values (its bias gradient, for launch_bias_sums).
  const uint16_t* gmask = nullptr;  // BF16 [out voxel][cout]: the layer below's output
  float* gpart = nullptr;
};

// Whether launch_conv can fold the ReLU mask, BF16 rounding and bias sums
// into this input-gradient product (see ConvArgs::gmask), and
// the number of channel-sum rows it then writes to gpart.
bool conv_folds_grad(const ConvArgs& a);
int conv_fold_rows(const ConvArgs& a);

// Weight gradient gw[t][ci][n] += sum_m A(m, t, ci) gy(m, n) (FP32 atomics).
struct WgradArgs {
  int32_t geo;                // kConv3, kDown or kUp (the layer's forward geometry)
  int32_t d, h, w;            // grid of m: the output grid (kConv3, kDown), the input grid (kUp)
  int32_t taps, cin, cout;
  int64_t m_per_block;        // voxels per workgroup (multiple of 32)
  ConvArgs g;                 // geometry fields for the gather (geo, in_d, in_h, in_w)
  const uint16_t* x;          // BF16 [voxel][cin], the layer input
  const uint16_t* gy;         // BF16 [voxel][cout], gradient of the layer output
  float* gw;                  // FP32 [taps][cin][cout], accumulated
  float* part;                // FP32 workspace for per-workgroup partial sums, or null
  int64_t part_cap;           // its size in floats
};

hipError_t launch_conv(const ConvArgs& a, hipStream_t s);
// floats of split-reduction workspace launch_conv would use for `a` given an
// unlimited workspace (0: it does not split this product)
int64_t conv_workspace_floats(const ConvArgs& a);
hipError_t launch_wgrad(const WgradArgs& a, hipStream_t s);
// floats of workspace launch_wgrad uses for `a` (0: it needs none)
int64_t wgrad_workspace_floats(const WgradArgs& a);
// pack w[taps][cin][cout] (FP32) into BF16 rows: forward Bt[n][t * cin + ci]
// (rows >= cout) or transposed Bt[ci][t * cout + n] (rows >= cin); with
// `clear` the rows x kpad buffer is zeroed first (the padding outside the
// weights never changes, so later packs of the same buffer skip it)
hipError_t launch_pack(const float* w, int taps, int cin, int cout, int rows, int kpad,
                       bool transposed, uint16_t* bt, hipStream_t s, bool clear = true);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_to_log(const float* phi, int64_t n, float* u, uint16_t* u16, hipStream_t s);
hipError_t launch_mirror_xy(const float* in, float* out, int nx, int ny, int nz, int op,
                            hipStream_t s);
// acc (= when first, else +=) the symmetry op of in (as launch_mirror_xy)
hipError_t launch_mirror_acc(const float* in, float* acc, int nx, int ny, int nz, int op,
                             bool first, hipStream_t s);
// out_u = acc / nsym and phi = its fluence (either may be null)
hipError_t launch_sym_finish(const float* acc, int64_t n, int nsym, float* out_u, float* phi,
                             hipStream_t s);
hipError_t launch_from_log(const float* r, const float* u, int64_t n, float* out_u, float* phi,
                           hipStream_t s);
// g16 = bf16((g + skip16) * (y16 > 0)) over n = voxels * cout values;
// with gb set, also gb[c] += sum over voxels of g16[.][c] (through
// `partial`, kBiasBlocks * cout floats of scratch)
constexpr int kBiasBlocks = 2048;
hipError_t launch_relu_grad(const float* g, const uint16_t* skip16, const uint16_t* y16, int64_t n,
                            int cout, uint16_t* g16, float* gb, float* partial, hipStream_t s);
// The same with the bias sums deferred: when relu_grad_defers(cout), the
// per-block channel sums go to partial[relu_grad_blocks(n)][cout] and a
// later launch_bias_sums adds them to the gradients; otherwise the bias
// gradient is added at once, as launch_relu_grad does.
bool relu_grad_defers(int cout);
int relu_grad_blocks(int64_t n);
hipError_t launch_relu_grad_deferred(const float* g, const uint16_t* skip16, const uint16_t* y16,
                                     int64_t n, int cout, uint16_t* g16, float* gb, float* partial,
                                     hipStream_t s);
// One deferred bias sum: grads[gb_off + c] += sum over b < blocks of
// partial[partial_off + b * cout + c], c < cout.
struct BiasJob {
  int64_t partial_off;
  int64_t gb_off;
  int32_t blocks;
  int32_t cout;
};
// all jobs (a device array) in one launch; channels = sum of their couts
hipError_t launch_bias_sums(const BiasJob* jobs, int njobs, int channels, const float* partial,
                            float* grads, hipStream_t s);
// masked MSE in u space; target voxels with phi >= rel_floor * max(phi)
// count; grad = 2 (out - t) / count there.  acc[0] = sum of squares,
// acc[1] = count (FP64); phi_max: one float of scratch
hipError_t launch_mse(const float* out, const float* target_u, const float* target_phi,
                      float rel_floor, int64_t n, float* grad, double* acc, float* phi_max,
                      hipStream_t s);
hipError_t launch_bias_grad(const uint16_t* gy, int64_t m, int cout, float* gb, hipStream_t s);
// Adam step on grad_scale * g, clipped to global norm max_norm (> 0);
// partial: kNormBlocks doubles of scratch
constexpr int kNormBlocks = 1024;
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, int step,
                       float grad_scale, float max_norm, double* partial, hipStream_t s);

}  // namespace nn
}  // namespace mcx
