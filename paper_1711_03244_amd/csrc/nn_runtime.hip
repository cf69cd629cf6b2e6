// Host runtime of the fluence denoiser (see include/mcx_nn.h): the U-Net
// graph over the BF16 MFMA convolution kernels, its buffers, the backward
// pass and the optimiser, all enqueued on one stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/mcx_nn.h"
#include "mcx_internal.hpp"
#include "nn_internal.hpp"

namespace {

using namespace mcx::nn;

mcx_status nfail(mcx_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return mcx::report(st, buf);
}

#define NN_HIP(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return nfail(e_ == hipErrorOutOfMemory ? MCX_ENOMEM : MCX_EDEVICE, "%s: %s", \
                   #expr, hipGetErrorString(e_));                                  \
  } while (0)

#define NN_TRY(expr)             \
  do {                           \
    mcx_status s_ = (expr);      \
    if (s_ != MCX_OK) return s_; \
  } while (0)

constexpr float kMaskFloor = 1e-8f;  // loss voxels: target >= 1e-8 of its maximum

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Grid {
  int d, h, w;
  int64_t vox() const { return static_cast<int64_t>(d) * h * w; }
};

struct Layer {
  int kind = MCX_NN_CONV3;
  int taps = 27, cin = 0, cout = 0;
  Grid in{}, out{};
  uint64_t woff = 0, boff = 0;       // offsets into the parameter array
  int fwd_rows = 0, fwd_kpad = 0;    // packed Bt[n][k]
  int bwd_rows = 0, bwd_kpad = 0;    // packed transposed Bt[ci][t * cout + n]
  uint16_t* fwd = nullptr;
  uint16_t* bwd = nullptr;
  uint16_t* act = nullptr;           // BF16 output [out voxel][cout] (null for the output layer)
  int skip_level = -1;               // conv3 whose output is a skip (level), or -1
  int up_level = -1;                 // up layer adding the skip of this level, or -1
};

void describe_layer(Layer& L, int kind, int cin, int cout, Grid in) {
  L.kind = kind;
  L.taps = kind == MCX_NN_CONV3 ? 27 : 8;
  L.cin = cin;
  L.cout = cout;
  L.in = in;
  if (kind == MCX_NN_CONV3)
    L.out = in;
  else if (kind == MCX_NN_DOWN)
    L.out = Grid{in.d / 2, in.h / 2, in.w / 2};
  else
    L.out = Grid{in.d * 2, in.h * 2, in.w * 2};
  L.fwd_rows = round_up(cout, 64);
  L.fwd_kpad = round_up(L.taps * cin, 32);
  L.bwd_rows = round_up(cin, 64);
  L.bwd_kpad = round_up(L.taps * cout, 32);
}

// y = [relu](layer(x) + b [+ skip]); x BF16 with cin channels on L.in
ConvArgs forward_args(const Layer& L, const uint16_t* x, const float* b, const uint16_t* skip,
                      bool relu, bool y_f32, void* y) {
  ConvArgs a{};
  a.cin = L.cin;
  a.cout = L.cout;
  a.in_d = L.in.d;
  a.in_h = L.in.h;
  a.in_w = L.in.w;
  if (L.kind == MCX_NN_CONV3) {
    a.geo = kConv3;
    a.d = L.in.d; a.h = L.in.h; a.w = L.in.w;
    a.k = 27 * L.cin;
  } else if (L.kind == MCX_NN_DOWN) {
    a.geo = kDown;
    a.d = L.out.d; a.h = L.out.h; a.w = L.out.w;
    a.k = 8 * L.cin;
  } else {
    a.geo = kUp;
    a.d = L.in.d; a.h = L.in.h; a.w = L.in.w;
    a.k = L.cin;
  }
  a.kpad = L.fwd_kpad;
  a.x = x;
  a.bt = L.fwd;
  a.bias = b;
  a.skip = skip;
  a.y = y;
  a.y_f32 = y_f32 ? 1 : 0;
  a.relu = relu ? 1 : 0;
  return a;
}

// gx (FP32, cin channels on L.in) from gy (BF16, cout channels on L.out)
ConvArgs dgrad_args(const Layer& L, const uint16_t* gy, float* gx) {
  ConvArgs a{};
  a.cin = L.cout;   // channels of the gathered operand (gy)
  a.cout = L.cin;   // channels produced (gx)
  a.in_d = L.out.d;
  a.in_h = L.out.h;
  a.in_w = L.out.w;
  if (L.kind == MCX_NN_CONV3) {
    a.geo = kConv3T;
    a.d = L.in.d; a.h = L.in.h; a.w = L.in.w;
    a.k = 27 * L.cout;
  } else if (L.kind == MCX_NN_DOWN) {
    // gx[2v + e(c)] = gy[v] W[c]^T: rows over the small (output) grid
    a.geo = kUp;
    a.d = L.out.d; a.h = L.out.h; a.w = L.out.w;
    a.k = L.cout;
  } else {
    // gx[v] = sum_t gy[2v + e(t)] W[t]^T: rows over the small (input) grid
    a.geo = kDown;
    a.d = L.in.d; a.h = L.in.h; a.w = L.in.w;
    a.k = 8 * L.cout;
  }
  a.kpad = L.bwd_kpad;
  a.x = gy;
  a.bt = L.bwd;
  a.y = gx;
  a.y_f32 = 1;
  return a;
}

WgradArgs wgrad_args(const Layer& L, const uint16_t* x, const uint16_t* gy, float* gw) {
  WgradArgs a{};
  a.taps = L.taps;
  a.cin = L.cin;
  a.cout = L.cout;
  a.x = x;
  a.gy = gy;
  a.gw = gw;
  a.g.in_d = L.in.d;
  a.g.in_h = L.in.h;
  a.g.in_w = L.in.w;
  Grid m;
  if (L.kind == MCX_NN_CONV3) {
    a.geo = a.g.geo = kConv3;
    m = L.in;
  } else if (L.kind == MCX_NN_DOWN) {
    a.geo = a.g.geo = kDown;
    m = L.out;
  } else {
    a.geo = a.g.geo = kUp;
    m = L.in;
  }
  a.d = m.d;
  a.h = m.h;
  a.w = m.w;
  // split the voxel reduction so that the launch has about 2048 workgroups
  const int64_t M = m.vox();
  const int nb = L.cout > 32 ? 64 : (L.cout > 16 ? 32 : 16);
  const int64_t tiles = static_cast<int64_t>(L.kind == MCX_NN_UP ? L.taps * ((L.cin + 63) / 64)
                                                                 : (L.taps * L.cin + 63) / 64) *
                        ((L.cout + nb - 1) / nb);
  int64_t blocks = std::max<int64_t>(1, 2048 / std::max<int64_t>(1, tiles));
  blocks = std::min<int64_t>(blocks, (M + 31) / 32);
  int64_t per = (M + blocks - 1) / blocks;
  a.m_per_block = std::max<int64_t>(32, (per + 31) / 32 * 32);
  return a;
}

mcx_status check_kind(int32_t kind, int32_t nx, int32_t ny, int32_t nz, int32_t cin,
                      int32_t cout) {
  if (kind < MCX_NN_CONV3 || kind > MCX_NN_UP) return nfail(MCX_EINVAL, "unknown layer kind %d", kind);
  if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
    return nfail(MCX_EINVAL, "grid %d x %d x %d out of range", nx, ny, nz);
  if (static_cast<int64_t>(nx) * ny * nz * 8 > (1ll << 31))
    return nfail(MCX_EINVAL, "grid too large");
  if (kind == MCX_NN_DOWN && (nx % 2 || ny % 2 || nz % 2))
    return nfail(MCX_EINVAL, "a down layer needs even grid sides");
  if (cin < 1 || cout < 1 || cin > 1024 || cout > 1024)
    return nfail(MCX_EINVAL, "channels %d -> %d out of range", cin, cout);
  return MCX_OK;
}

}  // namespace

struct mcx_nn {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<int> ch;
  int L = 0;
  Grid g0{};
  std::vector<Layer> layers;
  uint64_t nparam = 0;
  float* params = nullptr;
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int step = 0;
  bool packed = false;       // packs hold the current parameters
  bool pads_clear = false;   // pack padding has been zeroed once
  float* u = nullptr;        // input in u space (FP32)
  uint16_t* u16 = nullptr;   // and as BF16
  float* r = nullptr;        // output layer result (FP32)
  float* out_u = nullptr;    // network output u + r
  float* tgt_u = nullptr;    // target in u space
  float* gout = nullptr;     // loss gradient
  float* gx = nullptr;       // FP32 input-gradient scratch
  uint16_t* g16 = nullptr;   // BF16 gradient scratch
  uint16_t* g16b = nullptr;  // and a second one, for folded input gradients
  std::vector<uint16_t*> skip_grad;  // per level 0..L-2
  double* acc = nullptr;
  float* phimax = nullptr;
  float* bias_partial = nullptr;  // per-block channel sums of the bias gradients, per layer
  std::vector<int64_t> bias_off;  // each layer's region of bias_partial
  BiasJob* bias_jobs = nullptr;   // device table of the deferred bias sums
  BiasJob* bias_jobs_fold = nullptr;  // the same with the folded layers' sums
  int nbias_jobs = 0, bias_channels = 0;
  // fold[i]: layer i's output gradient comes from layer i + 1's input-gradient
  // product with the ReLU mask and bias sums folded in
  std::vector<char> fold;
  bool fuse = true;                // use the folds
  double* norm_partial = nullptr; // per-block sums of squares of the gradients
  float* part = nullptr;          // split-reduction workspace of the convolutions
  int64_t part_cap = 0;           // its size in floats
  std::vector<void*> owned;
};

namespace {

template <typename T>
mcx_status nn_alloc(mcx_nn* nn, T** p, size_t count) {
  void* q = nullptr;
  NN_HIP(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
  nn->owned.push_back(q);
  *p = static_cast<T*>(q);
  return MCX_OK;
}

void nn_release(mcx_nn* nn) {
  if (!nn) return;
  (void)hipSetDevice(nn->device);
  if (nn->stream) (void)hipStreamSynchronize(nn->stream);
  for (void* p : nn->owned) (void)hipFree(p);
  if (nn->stream) (void)hipStreamDestroy(nn->stream);
  delete nn;
}

// NULL is the null stream, as for any HIP call (and torch's default stream)
hipStream_t pick(mcx_nn*, void* s) { return static_cast<hipStream_t>(s); }

mcx_status pack_all(mcx_nn* nn, hipStream_t s) {
  if (nn->packed) return MCX_OK;
  for (Layer& L : nn->layers) {
    NN_HIP(launch_pack(nn->params + L.woff, L.taps, L.cin, L.cout, L.fwd_rows, L.fwd_kpad, false,
                       L.fwd, s, !nn->pads_clear));
    NN_HIP(launch_pack(nn->params + L.woff, L.taps, L.cin, L.cout, L.bwd_rows, L.bwd_kpad, true,
                       L.bwd, s, !nn->pads_clear));
  }
  nn->packed = true;
  nn->pads_clear = true;
  return MCX_OK;
}

const uint16_t* layer_input(const mcx_nn* nn, size_t i) {
  return i == 0 ? nn->u16 : nn->layers[i - 1].act;
}

mcx_status run_forward(mcx_nn* nn, const float* phi_in, hipStream_t s) {
  NN_TRY(pack_all(nn, s));
  const int64_t n0 = nn->g0.vox();
  NN_HIP(launch_to_log(phi_in, n0, nn->u, nn->u16, s));
  const size_t last = nn->layers.size() - 1;
  for (size_t i = 0; i <= last; ++i) {
    const Layer& L = nn->layers[i];
    const uint16_t* skip = nullptr;
    if (L.kind == MCX_NN_UP) {
      for (const Layer& S : nn->layers)
        if (S.skip_level == L.up_level) skip = S.act;
    }
    const bool out = i == last;
    ConvArgs a = forward_args(L, layer_input(nn, i), nn->params + L.boff, skip, !out, out,
                              out ? static_cast<void*>(nn->r) : static_cast<void*>(L.act));
    a.part = nn->part;
    a.part_cap = nn->part_cap;
    NN_HIP(launch_conv(a, s));
  }
  return MCX_OK;
}

// the gradient of layer i's output skip connection, or null
const uint16_t* skip_gradient(const mcx_nn* nn, const Layer& L) {
  return (L.skip_level >= 0 && L.skip_level < nn->L - 1) ? nn->skip_grad[L.skip_level] : nullptr;
}

// layer i + 1's input-gradient product with layer i's output-gradient step
// folded in (mcx_nn::fold), from gy of layer i + 1 into gy of layer i
ConvArgs fold_args(const mcx_nn* nn, size_t i, const uint16_t* gy_next, uint16_t* gy) {
  ConvArgs a = dgrad_args(nn->layers[i + 1], gy_next, nullptr);
  a.y = gy;
  a.y_f32 = 0;
  a.gmask = nn->layers[i].act;
  a.gpart = nn->bias_partial + nn->bias_off[i];
  return a;
}

mcx_status run_backward(mcx_nn* nn, bool accumulate, hipStream_t s) {
  const size_t last = nn->layers.size() - 1;
  if (!accumulate) NN_HIP(launch_fill(nn->grads, static_cast<int64_t>(nn->nparam), 0.f, s));
  const float* g = nn->gout;
  uint16_t* gy_folded = nullptr;  // the gradient the last product folded, or null
  for (size_t k = 0; k <= last; ++k) {
    const size_t i = last - k;
    const Layer& L = nn->layers[i];
    const int64_t nout = L.out.vox() * L.cout;
    // gradient of this layer's output, masked by its ReLU, as BF16
    uint16_t* gy = nn->g16;
    if (gy_folded) {
      gy = gy_folded;
    } else {
      if (L.kind == MCX_NN_UP) gy = nn->skip_grad[L.up_level];  // also the skip's gradient
      NN_HIP(launch_relu_grad_deferred(g, skip_gradient(nn, L), i == last ? nullptr : L.act, nout,
                                       L.cout, gy, nn->grads + L.boff,
                                       nn->bias_partial + nn->bias_off[i], s));
    }
    WgradArgs wa = wgrad_args(L, layer_input(nn, i), gy, nn->grads + L.woff);
    wa.part = nn->part;
    wa.part_cap = nn->part_cap;
    NN_HIP(launch_wgrad(wa, s));
    gy_folded = nullptr;
    if (i > 0 && nn->fuse && nn->fold[i - 1]) {
      // into the up layer's skip gradient, or the BF16 buffer gy is not in
      const Layer& B = nn->layers[i - 1];
      uint16_t* dst = B.kind == MCX_NN_UP ? nn->skip_grad[B.up_level]
                                          : (gy == nn->g16 ? nn->g16b : nn->g16);
      ConvArgs a = fold_args(nn, i - 1, gy, dst);
      NN_HIP(launch_conv(a, s));
      gy_folded = dst;
    } else if (i > 0) {
      ConvArgs a = dgrad_args(L, gy, nn->gx);
      a.part = nn->part;
      a.part_cap = nn->part_cap;
      NN_HIP(launch_conv(a, s));
      g = nn->gx;
    }
  }
  // the bias gradients of every layer whose sums were deferred, in one launch
  NN_HIP(launch_bias_sums(nn->fuse ? nn->bias_jobs_fold : nn->bias_jobs, nn->nbias_jobs,
                          nn->bias_channels, nn->bias_partial, nn->grads, s));
  return MCX_OK;
}

}  // namespace

extern "C" {

mcx_status mcx_nn_create(const int32_t* channels, int32_t nlevels, int32_t nx, int32_t ny,
                         int32_t nz, int32_t device, mcx_nn** out) {
  if (!out || !channels) return nfail(MCX_EINVAL, "channels and out are required");
  if (nlevels < 1 || nlevels > 6) return nfail(MCX_EINVAL, "nlevels must be in [1, 6]");
  for (int i = 0; i < nlevels; ++i)
    if (channels[i] < 1 || channels[i] > 1024)
      return nfail(MCX_EINVAL, "channels[%d] = %d out of range", i, channels[i]);
  const int f = 1 << (nlevels - 1);
  if (nx < f || ny < f || nz < f || nx % f || ny % f || nz % f)
    return nfail(MCX_EINVAL, "grid sides must be positive multiples of %d", f);
  if (static_cast<int64_t>(nx) * ny * nz * 1024 > (1ll << 40))
    return nfail(MCX_EINVAL, "grid too large");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return nfail(MCX_ENODEV, "no HIP device available");
  if (device < 0 || device >= ndev) return nfail(MCX_ENODEV, "device %d not present", device);

  mcx_nn* nn = new (std::nothrow) mcx_nn();
  if (!nn) return nfail(MCX_ENOMEM, "host allocation failed");
  nn->device = device;
  nn->ch.assign(channels, channels + nlevels);
  nn->L = nlevels;
  nn->g0 = Grid{nz, ny, nx};
  auto level = [&](int l) { return Grid{nz >> l, ny >> l, nx >> l}; };
  const int L = nlevels;
  const std::vector<int>& c = nn->ch;
  auto add = [&](int kind, int cin, int cout, int lin) -> Layer& {
    nn->layers.emplace_back();
    describe_layer(nn->layers.back(), kind, cin, cout, level(lin));
    return nn->layers.back();
  };
  add(MCX_NN_CONV3, 1, c[0], 0);
  add(MCX_NN_CONV3, c[0], c[0], 0).skip_level = 0;
  for (int l = 1; l < L; ++l) {
    add(MCX_NN_DOWN, c[l - 1], c[l], l - 1);
    add(MCX_NN_CONV3, c[l], c[l], l).skip_level = l;
  }
  add(MCX_NN_CONV3, c[L - 1], c[L - 1], L - 1);
  for (int l = L - 2; l >= 0; --l) {
    add(MCX_NN_UP, c[l + 1], c[l], l + 1).up_level = l;
    add(MCX_NN_CONV3, c[l], c[l], l);
  }
  add(MCX_NN_CONV3, c[0], 1, 0);
  for (Layer& Ly : nn->layers) {
    Ly.woff = nn->nparam;
    nn->nparam += static_cast<uint64_t>(Ly.taps) * Ly.cin * Ly.cout;
    Ly.boff = nn->nparam;
    nn->nparam += Ly.cout;
  }

  auto setup = [&]() -> mcx_status {
    NN_HIP(hipSetDevice(device));
    NN_HIP(hipStreamCreateWithFlags(&nn->stream, hipStreamNonBlocking));
    const int64_t n0 = nn->g0.vox();
    NN_TRY(nn_alloc(nn, &nn->params, nn->nparam));
    NN_TRY(nn_alloc(nn, &nn->grads, nn->nparam));
    NN_TRY(nn_alloc(nn, &nn->adam_m, nn->nparam));
    NN_TRY(nn_alloc(nn, &nn->adam_v, nn->nparam));
    int64_t max_act = 0, max_in = 0;
    for (size_t i = 0; i < nn->layers.size(); ++i) {
      Layer& Ly = nn->layers[i];
      NN_TRY(nn_alloc(nn, &Ly.fwd, static_cast<size_t>(Ly.fwd_rows) * Ly.fwd_kpad));
      NN_TRY(nn_alloc(nn, &Ly.bwd, static_cast<size_t>(Ly.bwd_rows) * Ly.bwd_kpad));
      if (i + 1 < nn->layers.size())
        NN_TRY(nn_alloc(nn, &Ly.act, static_cast<size_t>(Ly.out.vox() * Ly.cout)));
      max_act = std::max(max_act, Ly.out.vox() * Ly.cout);
      max_in = std::max(max_in, Ly.in.vox() * Ly.cin);
    }
    NN_TRY(nn_alloc(nn, &nn->u, n0));
    NN_TRY(nn_alloc(nn, &nn->u16, n0));
    NN_TRY(nn_alloc(nn, &nn->r, n0));
    NN_TRY(nn_alloc(nn, &nn->out_u, n0));
    NN_TRY(nn_alloc(nn, &nn->tgt_u, n0));
    NN_TRY(nn_alloc(nn, &nn->gout, n0));
    NN_TRY(nn_alloc(nn, &nn->gx, max_in));
    NN_TRY(nn_alloc(nn, &nn->g16, max_act));
    nn->skip_grad.assign(std::max(0, L - 1), nullptr);
    for (int l = 0; l + 1 < L; ++l)
      NN_TRY(nn_alloc(nn, &nn->skip_grad[l], static_cast<size_t>(level(l).vox() * c[l])));
    NN_TRY(nn_alloc(nn, &nn->acc, 2));
    // the folds: layers with a deferred bias sum and no skip gradient whose
    // output gradient the next layer's input-gradient product can produce
    const size_t nl = nn->layers.size();
    nn->fold.assign(nl, 0);
    bool any_fold = false;
    for (size_t i = 0; i + 1 < nl; ++i) {
      if (!relu_grad_defers(nn->layers[i].cout) || skip_gradient(nn, nn->layers[i])) continue;
      ConvArgs a = dgrad_args(nn->layers[i + 1], nullptr, nullptr);
      a.y_f32 = 0;
      nn->fold[i] = conv_folds_grad(a) ? 1 : 0;
      any_fold = any_fold || nn->fold[i];
    }
    if (any_fold) NN_TRY(nn_alloc(nn, &nn->g16b, max_act));
    // each layer's partial sums take the rows of either producer
    std::vector<BiasJob> jobs, jobs_fold;
    int64_t bias_floats = 0;
    for (size_t i = 0; i < nl; ++i) {
      const Layer& Ly = nn->layers[i];
      nn->bias_off.push_back(bias_floats);
      if (!relu_grad_defers(Ly.cout)) continue;
      const int blocks = relu_grad_blocks(Ly.out.vox() * Ly.cout);
      const int fblocks = nn->fold[i] ? conv_fold_rows(dgrad_args(nn->layers[i + 1], nullptr, nullptr))
                                      : blocks;
      jobs.push_back(BiasJob{bias_floats, static_cast<int64_t>(Ly.boff), blocks, Ly.cout});
      jobs_fold.push_back(BiasJob{bias_floats, static_cast<int64_t>(Ly.boff), fblocks, Ly.cout});
      bias_floats += static_cast<int64_t>(std::max(blocks, fblocks)) * Ly.cout;
      nn->bias_channels += Ly.cout;
    }
    NN_TRY(nn_alloc(nn, &nn->bias_partial, static_cast<size_t>(std::max<int64_t>(bias_floats, 1))));
    nn->nbias_jobs = static_cast<int>(jobs.size());
    NN_TRY(nn_alloc(nn, &nn->bias_jobs, jobs.size()));
    NN_TRY(nn_alloc(nn, &nn->bias_jobs_fold, jobs.size()));
    if (!jobs.empty()) {
      NN_HIP(hipMemcpy(nn->bias_jobs, jobs.data(), jobs.size() * sizeof(BiasJob),
                       hipMemcpyHostToDevice));
      NN_HIP(hipMemcpy(nn->bias_jobs_fold, jobs_fold.data(), jobs.size() * sizeof(BiasJob),
                       hipMemcpyHostToDevice));
    }
    NN_TRY(nn_alloc(nn, &nn->norm_partial, static_cast<size_t>(kNormBlocks)));
    NN_TRY(nn_alloc(nn, &nn->phimax, 1));
    for (const Layer& Ly : nn->layers) {
      nn->part_cap = std::max(nn->part_cap, conv_workspace_floats(
                                                forward_args(Ly, nullptr, nullptr, nullptr, false,
                                                             false, nullptr)));
      nn->part_cap = std::max(nn->part_cap, conv_workspace_floats(dgrad_args(Ly, nullptr, nullptr)));
      nn->part_cap =
          std::max(nn->part_cap, wgrad_workspace_floats(wgrad_args(Ly, nullptr, nullptr, nullptr)));
    }
    if (nn->part_cap > 0) NN_TRY(nn_alloc(nn, &nn->part, static_cast<size_t>(nn->part_cap)));
    NN_HIP(launch_fill(nn->params, static_cast<int64_t>(nn->nparam), 0.f, nn->stream));
    NN_HIP(launch_fill(nn->adam_m, static_cast<int64_t>(nn->nparam), 0.f, nn->stream));
    NN_HIP(launch_fill(nn->adam_v, static_cast<int64_t>(nn->nparam), 0.f, nn->stream));
    NN_HIP(hipStreamSynchronize(nn->stream));
    return MCX_OK;
  };
  const mcx_status st = setup();
  if (st != MCX_OK) {
    const std::string keep = mcx_last_error();
    nn_release(nn);
    return mcx::report(st, keep.c_str());
  }
  *out = nn;
  return MCX_OK;
}

void mcx_nn_destroy(mcx_nn* nn) { nn_release(nn); }

uint64_t mcx_nn_param_count(const mcx_nn* nn) { return nn ? nn->nparam : 0; }

static mcx_status copy_params(mcx_nn* nn, float* dev, void* host, uint64_t n, bool to_dev) {
  if (!nn || !host) return nfail(MCX_EINVAL, "network and host array are required");
  if (n != nn->nparam)
    return nfail(MCX_ERANGE, "%llu values given, the network has %llu",
                 static_cast<unsigned long long>(n), static_cast<unsigned long long>(nn->nparam));
  NN_HIP(hipSetDevice(nn->device));
  NN_HIP(hipDeviceSynchronize());  // the network's work may be on any stream
  if (to_dev)
    NN_HIP(hipMemcpy(dev, host, n * sizeof(float), hipMemcpyHostToDevice));
  else
    NN_HIP(hipMemcpy(host, dev, n * sizeof(float), hipMemcpyDeviceToHost));
  return MCX_OK;
}

mcx_status mcx_nn_set_params(mcx_nn* nn, const float* host, uint64_t n) {
  NN_TRY(copy_params(nn, nn ? nn->params : nullptr, const_cast<float*>(host), n, true));
  NN_HIP(launch_fill(nn->adam_m, static_cast<int64_t>(nn->nparam), 0.f, nn->stream));
  NN_HIP(launch_fill(nn->adam_v, static_cast<int64_t>(nn->nparam), 0.f, nn->stream));
  NN_HIP(hipStreamSynchronize(nn->stream));
  nn->step = 0;
  nn->packed = false;
  return MCX_OK;
}

mcx_status mcx_nn_get_params(mcx_nn* nn, float* host, uint64_t n) {
  return copy_params(nn, nn ? nn->params : nullptr, host, n, false);
}

mcx_status mcx_nn_get_grads(mcx_nn* nn, float* host, uint64_t n) {
  return copy_params(nn, nn ? nn->grads : nullptr, host, n, false);
}

mcx_status mcx_nn_get_adam(mcx_nn* nn, float* m, float* v, uint64_t n, int32_t* step) {
  if (!m || !v || !step) return nfail(MCX_EINVAL, "m, v and step are required");
  NN_TRY(copy_params(nn, nn ? nn->adam_m : nullptr, m, n, false));
  NN_TRY(copy_params(nn, nn->adam_v, v, n, false));
  *step = nn->step;
  return MCX_OK;
}

mcx_status mcx_nn_set_adam(mcx_nn* nn, const float* m, const float* v, uint64_t n, int32_t step) {
  if (!m || !v) return nfail(MCX_EINVAL, "m and v are required");
  if (step < 0) return nfail(MCX_EINVAL, "step must be >= 0");
  NN_TRY(copy_params(nn, nn ? nn->adam_m : nullptr, const_cast<float*>(m), n, true));
  NN_TRY(copy_params(nn, nn->adam_v, const_cast<float*>(v), n, true));
  nn->step = step;
  return MCX_OK;
}

mcx_status mcx_nn_forward(mcx_nn* nn, const float* phi_in, float* phi_out, float* u_out,
                          void* stream) {
  if (!nn || !phi_in) return nfail(MCX_EINVAL, "network and input are required");
  NN_HIP(hipSetDevice(nn->device));
  hipStream_t s = pick(nn, stream);
  NN_TRY(run_forward(nn, phi_in, s));
  NN_HIP(launch_from_log(nn->r, nn->u, nn->g0.vox(), u_out ? u_out : nn->out_u, phi_out, s));
  return MCX_OK;
}

mcx_status mcx_nn_forward_sym(mcx_nn* nn, const float* phi_in, float* phi_out, float* u_out,
                              int32_t nsym, void* stream) {
  if (!nn || !phi_in) return nfail(MCX_EINVAL, "network and input are required");
  if (nsym != 1 && nsym != 2 && nsym != 4 && nsym != 8)
    return nfail(MCX_EINVAL, "nsym must be 1, 2, 4 or 8");
  const Grid& g = nn->g0;
  if (nsym == 8 && g.w != g.h) return nfail(MCX_EINVAL, "8 symmetries need nx == ny");
  if (nsym == 1) return mcx_nn_forward(nn, phi_in, phi_out, u_out, stream);
  NN_HIP(hipSetDevice(nn->device));
  hipStream_t s = pick(nn, stream);
  // the loss buffers are idle outside mcx_nn_loss_grad: tgt_u holds the
  // transformed input, gout the sum of the outputs mapped back
  for (int op = 0; op < nsym; ++op) {
    const float* x = phi_in;
    if (op > 0) {
      NN_HIP(launch_mirror_xy(phi_in, nn->tgt_u, g.w, g.h, g.d, op, s));
      x = nn->tgt_u;
    }
    NN_TRY(run_forward(nn, x, s));
    NN_HIP(launch_from_log(nn->r, nn->u, g.vox(), nn->out_u, nullptr, s));
    // the inverse of op: a flip is its own inverse; with the swap, the flips
    // of x and y exchange
    const int inv = (op & 4) ? (4 | ((op & 1) << 1) | ((op & 2) >> 1)) : op;
    NN_HIP(launch_mirror_acc(nn->out_u, nn->gout, g.w, g.h, g.d, inv, op == 0, s));
  }
  NN_HIP(launch_sym_finish(nn->gout, g.vox(), nsym, u_out, phi_out, s));
  return MCX_OK;
}

mcx_status mcx_nn_loss_grad(mcx_nn* nn, const float* phi_in, const float* phi_target,
                            int32_t accumulate, double* loss, void* stream) {
  if (!nn || !phi_in || !phi_target)
    return nfail(MCX_EINVAL, "network, input and target are required");
  NN_HIP(hipSetDevice(nn->device));
  hipStream_t s = pick(nn, stream);
  const int64_t n0 = nn->g0.vox();
  NN_TRY(run_forward(nn, phi_in, s));
  NN_HIP(launch_from_log(nn->r, nn->u, n0, nn->out_u, nullptr, s));
  NN_HIP(launch_to_log(phi_target, n0, nn->tgt_u, nullptr, s));
  NN_HIP(launch_mse(nn->out_u, nn->tgt_u, phi_target, kMaskFloor, n0, nn->gout, nn->acc,
                    nn->phimax, s));
  NN_TRY(run_backward(nn, accumulate != 0, s));
  if (loss) {
    double acc[2];
    NN_HIP(hipMemcpyAsync(acc, nn->acc, sizeof(acc), hipMemcpyDeviceToHost, s));
    NN_HIP(hipStreamSynchronize(s));
    *loss = acc[1] > 0 ? acc[0] / acc[1] : 0.0;
  }
  return MCX_OK;
}

mcx_status mcx_nn_set_fused_backward(mcx_nn* nn, int32_t on, int32_t* nfolded) {
  if (!nn) return nfail(MCX_EINVAL, "network is NULL");
  nn->fuse = on != 0;
  if (nfolded) {
    int32_t n = 0;
    for (char f : nn->fold) n += f ? 1 : 0;
    *nfolded = nn->fuse ? n : 0;
  }
  return MCX_OK;
}

mcx_status mcx_nn_adam(mcx_nn* nn, float lr, float grad_scale, float max_norm, void* stream) {
  if (!nn) return nfail(MCX_EINVAL, "network is NULL");
  if (!(lr >= 0.f)) return nfail(MCX_EINVAL, "learning rate must be >= 0");
  if (!(grad_scale > 0.f)) return nfail(MCX_EINVAL, "grad_scale must be > 0");
  if (!(max_norm == max_norm)) return nfail(MCX_EINVAL, "max_norm is NaN");
  NN_HIP(hipSetDevice(nn->device));
  nn->step += 1;
  NN_HIP(launch_adam(nn->params, nn->grads, nn->adam_m, nn->adam_v,
                     static_cast<int64_t>(nn->nparam), lr, nn->step, grad_scale, max_norm,
                     nn->norm_partial, pick(nn, stream)));
  nn->packed = false;
  return MCX_OK;
}

mcx_status mcx_nn_train_step(mcx_nn* nn, const float* phi_in, const float* phi_target, float lr,
                             double* loss, void* stream) {
  NN_TRY(mcx_nn_loss_grad(nn, phi_in, phi_target, 0, loss, stream));
  return mcx_nn_adam(nn, lr, 1.f, 0.f, stream);
}

mcx_status mcx_nn_mirror_xy(const float* in, float* out, int32_t nx, int32_t ny, int32_t nz,
                            int32_t op, void* stream) {
  if (!in || !out || in == out) return nfail(MCX_EINVAL, "in and out are required and distinct");
  if (nx <= 0 || ny <= 0 || nz <= 0) return nfail(MCX_EINVAL, "grid sizes must be positive");
  if (op < 0 || op > 7) return nfail(MCX_EINVAL, "op must be in 0..7");
  if ((op & 4) && nx != ny) return nfail(MCX_EINVAL, "swapping x and y needs nx == ny");
  NN_HIP(launch_mirror_xy(in, out, nx, ny, nz, op, static_cast<hipStream_t>(stream)));
  return MCX_OK;
}

mcx_status mcx_nn_layer_forward(int32_t kind, int32_t nx, int32_t ny, int32_t nz, int32_t cin,
                                int32_t cout, const uint16_t* x, const float* w, const float* b,
                                const uint16_t* skip, int32_t relu, int32_t y_f32, void* y,
                                void* stream) {
  NN_TRY(check_kind(kind, nx, ny, nz, cin, cout));
  if (!x || !w || !y) return nfail(MCX_EINVAL, "x, w and y are required");
  Layer L;
  describe_layer(L, kind, cin, cout, Grid{nz, ny, nx});
  hipStream_t s = static_cast<hipStream_t>(stream);
  NN_HIP(hipMalloc(&L.fwd, static_cast<size_t>(L.fwd_rows) * L.fwd_kpad * sizeof(uint16_t)));
  ConvArgs a = forward_args(L, x, b, skip, relu != 0, y_f32 != 0, y);
  a.part_cap = conv_workspace_floats(a);
  hipError_t e = hipSuccess;
  if (a.part_cap > 0) e = hipMalloc(&a.part, static_cast<size_t>(a.part_cap) * sizeof(float));
  mcx_status st = MCX_OK;
  if (e == hipSuccess)
    e = launch_pack(w, L.taps, cin, cout, L.fwd_rows, L.fwd_kpad, false, L.fwd, s);
  if (e == hipSuccess) e = launch_conv(a, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) st = nfail(MCX_EDEVICE, "layer forward: %s", hipGetErrorString(e));
  (void)hipFree(L.fwd);
  if (a.part) (void)hipFree(a.part);
  return st;
}

mcx_status mcx_nn_layer_backward(int32_t kind, int32_t nx, int32_t ny, int32_t nz, int32_t cin,
                                 int32_t cout, const uint16_t* x, const float* w,
                                 const uint16_t* gy, float* gx, float* gw, float* gb,
                                 void* stream) {
  NN_TRY(check_kind(kind, nx, ny, nz, cin, cout));
  if (!x || !w || !gy || !gw) return nfail(MCX_EINVAL, "x, w, gy and gw are required");
  Layer L;
  describe_layer(L, kind, cin, cout, Grid{nz, ny, nx});
  hipStream_t s = static_cast<hipStream_t>(stream);
  NN_HIP(hipMalloc(&L.bwd, static_cast<size_t>(L.bwd_rows) * L.bwd_kpad * sizeof(uint16_t)));
  mcx_status st = MCX_OK;
  hipError_t e = launch_fill(gw, static_cast<int64_t>(L.taps) * cin * cout, 0.f, s);
  if (e == hipSuccess && gb) e = launch_fill(gb, cout, 0.f, s);
  WgradArgs wa = wgrad_args(L, x, gy, gw);
  wa.part_cap = wgrad_workspace_floats(wa);
  if (e == hipSuccess && wa.part_cap > 0)
    e = hipMalloc(&wa.part, static_cast<size_t>(wa.part_cap) * sizeof(float));
  if (e == hipSuccess) e = launch_wgrad(wa, s);
  if (e == hipSuccess && gb) e = launch_bias_grad(gy, L.out.vox(), cout, gb, s);
  if (e == hipSuccess && gx)
    e = launch_pack(w, L.taps, cin, cout, L.bwd_rows, L.bwd_kpad, true, L.bwd, s);
  ConvArgs da = dgrad_args(L, gy, gx);
  da.part_cap = gx ? conv_workspace_floats(da) : 0;
  if (e == hipSuccess && da.part_cap > 0)
    e = hipMalloc(&da.part, static_cast<size_t>(da.part_cap) * sizeof(float));
  if (e == hipSuccess && gx) e = launch_conv(da, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) st = nfail(MCX_EDEVICE, "layer backward: %s", hipGetErrorString(e));
  (void)hipFree(L.bwd);
  if (da.part) (void)hipFree(da.part);
  if (wa.part) (void)hipFree(wa.part);
  return st;
}

}  // extern "C"
