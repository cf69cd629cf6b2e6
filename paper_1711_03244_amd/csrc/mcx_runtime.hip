// Host runtime and C ABI of libmcx (see include/mcx.h for the contract).
//
// The host side of the paper's workflow (Fig. 1): take the user's domain,
// optical properties, source, detectors and gates, validate them, derive the
// per-medium constants the kernel needs, upload once, launch the photon
// kernel, reduce and normalise the read-back maps.  One context owns one
// device's buffers and one stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/mcx.h"
#include "mcx_internal.hpp"

namespace {

constexpr double kCmmPerNs = 299.792458;  // speed of light in vacuum, mm/ns
constexpr int kDefaultChunk = 256;
constexpr int kParamSlots = 32;  // device copies of launch parameters, used round-robin
constexpr int kDefaultWindow = 4096;  // FP64 cells, 32 KB of LDS

thread_local std::string g_error;

mcx_status fail(mcx_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(e_ == hipErrorOutOfMemory ? MCX_ENOMEM : MCX_EDEVICE, "%s: %s",  \
                  #expr, hipGetErrorString(e_));                                   \
  } while (0)

bool finite(float x) { return std::isfinite(x); }

}  // namespace

struct mcx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int nx = 0, ny = 0, nz = 0;
  uint32_t nvox = 0;
  float h = 1.f;
  int nmedia = 0, ndet = 0, ngates = 0;
  float t0 = 0.f, dt = 1.f;
  mcx_options opt{};
  std::vector<float4> table;  // 3 * nmedia + ndet rows, see TransportParams::media
  int src_i[3] = {0, 0, 0};
  float src_f[3] = {0, 0, 0};
  int src_label = 0;
  float src_dir[3] = {0, 0, 1};
  bool detect = false, diag = false;
  int block = 256, grid = 0, cus = 0;
  int win[7] = {0, 0, 0, 0, 0, 0, 0};  // x0, y0, z0, nx, ny, nz, ngates
  int rec_len = 0;

  uint8_t* d_labels = nullptr;
  float4* d_table = nullptr;
  double* d_tally = nullptr;
  unsigned long long* d_counter = nullptr;
  mcx::TransportParams* d_params = nullptr;  // kParamSlots slots
  uint64_t launches = 0;
  double* d_ledger = nullptr;
  unsigned long long* d_counts = nullptr;
  unsigned long long* d_det_count = nullptr;
  double* d_reduce = nullptr;
  float* d_rec = nullptr;
  unsigned long long* d_rec_photon = nullptr;
  double* d_digest = nullptr;
  float* d_stage32 = nullptr;
  double* d_stage64 = nullptr;
  hipEvent_t ev_begin = nullptr, ev_k0 = nullptr, ev_k1 = nullptr, ev_end = nullptr;

  uint64_t photons = 0;  // photons accumulated since the last reset
  bool have_timing = false;

  uint64_t ncells() const { return static_cast<uint64_t>(nvox) * ngates; }
};

extern "C" {

void mcx_default_options(mcx_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->reflect = 0;
  o->n_outside = 1.0f;
  o->rr_threshold = 1e-4f;
  o->rr_m = 10.f;
  o->max_detected = 1ull << 20;
  o->max_events = 100000000ull;
  o->device = 0;
  o->block_size = 0;
  o->blocks_per_cu = 0;
  o->refill_chunk = 0;
  o->ndigest = 0;
  o->lds_window_cells = 0;
  o->accurate_math = 0;
}

const char* mcx_last_error(void) { return g_error.c_str(); }

static mcx_status validate(const mcx_volume* vol, const mcx_source* src, const mcx_detector* det,
                           int32_t ndet, const mcx_gates* gates, const mcx_options* o) {
  if (!vol || !src || !gates) return fail(MCX_EINVAL, "volume, source and gates are required");
  if (vol->nx <= 0 || vol->ny <= 0 || vol->nz <= 0)
    return fail(MCX_EINVAL, "grid dimensions must be positive (got %d x %d x %d)", vol->nx,
                vol->ny, vol->nz);
  const uint64_t nvox = static_cast<uint64_t>(vol->nx) * vol->ny * vol->nz;
  if (gates->ngates <= 0) return fail(MCX_EINVAL, "ngates must be positive");
  if (nvox * static_cast<uint64_t>(gates->ngates) > (1ull << 31))
    return fail(MCX_EINVAL, "ngates * voxels must be <= 2^31 (got %llu)",
                static_cast<unsigned long long>(nvox * gates->ngates));
  if (!(vol->voxel_mm > 0.f) || !finite(vol->voxel_mm))
    return fail(MCX_EINVAL, "voxel size must be positive and finite");
  if (!vol->labels || !vol->media) return fail(MCX_EINVAL, "labels and media are required");
  if (vol->nmedia < 2 || vol->nmedia > 256)
    return fail(MCX_EINVAL, "nmedia must be in [2, 256] (row 0 is the outside)");
  for (int m = 1; m < vol->nmedia; ++m) {
    const mcx_medium& md = vol->media[m];
    if (!(md.mua >= 0.f) || !finite(md.mua) || !(md.mus >= 0.f) || !finite(md.mus))
      return fail(MCX_EINVAL, "medium %d: mua and mus must be finite and >= 0", m);
    if (!(md.g >= -1.f && md.g <= 1.f)) return fail(MCX_EINVAL, "medium %d: g must be in [-1, 1]", m);
    if (!(md.n >= 1.f) || !finite(md.n)) return fail(MCX_EINVAL, "medium %d: n must be >= 1", m);
  }
  for (uint64_t i = 0; i < nvox; ++i)
    if (vol->labels[i] >= vol->nmedia)
      return fail(MCX_EINVAL, "label %d at voxel %llu is >= nmedia %d", vol->labels[i],
                  static_cast<unsigned long long>(i), vol->nmedia);
  if (!(gates->dt_ns > 0.f) || !finite(gates->dt_ns) || !finite(gates->t0_ns))
    return fail(MCX_EINVAL, "gate width must be positive and t0 finite");
  const double dn = std::sqrt(static_cast<double>(src->dir[0]) * src->dir[0] +
                              static_cast<double>(src->dir[1]) * src->dir[1] +
                              static_cast<double>(src->dir[2]) * src->dir[2]);
  if (!(std::fabs(dn - 1.0) <= 1e-5)) return fail(MCX_EINVAL, "source direction must be a unit vector");
  const int dim[3] = {vol->nx, vol->ny, vol->nz};
  int64_t iv[3];
  for (int a = 0; a < 3; ++a) {
    const double x = static_cast<double>(src->pos[a]) / vol->voxel_mm;
    if (!(x >= 0.0) || !(x < dim[a]))
      return fail(MCX_EINVAL, "source position lies outside the grid (axis %d)", a);
    iv[a] = static_cast<int64_t>(std::floor(x));
  }
  if (vol->labels[iv[0] + vol->nx * (iv[1] + static_cast<int64_t>(vol->ny) * iv[2])] == 0)
    return fail(MCX_EINVAL, "source voxel has label 0 (outside)");
  if (ndet < 0 || ndet > 4096) return fail(MCX_EINVAL, "ndet must be in [0, 4096]");
  if (ndet > 0 && !det) return fail(MCX_EINVAL, "detector array is NULL");
  for (int d = 0; d < ndet; ++d)
    if (!(det[d].radius > 0.f) || !finite(det[d].radius) || !finite(det[d].pos[0]) ||
        !finite(det[d].pos[1]) || !finite(det[d].pos[2]))
      return fail(MCX_EINVAL, "detector %d: radius must be positive and the centre finite", d);
  if (o) {
    if (!(o->n_outside >= 1.f) || !finite(o->n_outside))
      return fail(MCX_EINVAL, "n_outside must be >= 1");
    if (!(o->rr_m > 1.f) || !finite(o->rr_m)) return fail(MCX_EINVAL, "rr_m must be > 1");
    if (!(o->rr_threshold >= 0.f) || !finite(o->rr_threshold))
      return fail(MCX_EINVAL, "rr_threshold must be >= 0");
    if (o->block_size != 0 && (o->block_size < 64 || o->block_size > 1024 || o->block_size % 64))
      return fail(MCX_EINVAL, "block_size must be a multiple of 64 in [64, 1024]");
    if (o->blocks_per_cu < 0 || o->refill_chunk < 0 || o->device < 0)
      return fail(MCX_EINVAL, "blocks_per_cu, refill_chunk and device must be >= 0");
    if (o->refill_chunk != 0 && o->refill_chunk < 64)
      return fail(MCX_EINVAL, "refill_chunk must be 0 or >= 64");
    if (o->max_events == 0 || o->max_events > 0xffffffffull)
      return fail(MCX_EINVAL, "max_events must be in [1, 2^32-1]");
    if (o->lds_window_cells > 8192)
      return fail(MCX_EINVAL, "lds_window_cells must be <= 8192 (64 KB of LDS)");
  }
  return MCX_OK;
}

static void release(mcx_ctx* c) {
  if (!c) return;
  void* bufs[] = {c->d_labels,  c->d_table, c->d_tally, c->d_counter, c->d_params, c->d_ledger,
                  c->d_counts,  c->d_det_count, c->d_reduce, c->d_rec, c->d_rec_photon,
                  c->d_digest,  c->d_stage32, c->d_stage64};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  hipEvent_t evs[] = {c->ev_begin, c->ev_k0, c->ev_k1, c->ev_end};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

static mcx_status setup(mcx_ctx* c, const mcx_volume* vol) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(MCX_ENODEV, "no HIP device available");
  if (c->device >= ndev) return fail(MCX_ENODEV, "device %d not present (%d devices)", c->device, ndev);
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device));
  HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreate(&c->ev_begin));
  HIP_TRY(hipEventCreate(&c->ev_k0));
  HIP_TRY(hipEventCreate(&c->ev_k1));
  HIP_TRY(hipEventCreate(&c->ev_end));

  const uint64_t ncells = c->ncells();
  HIP_TRY(hipMalloc(&c->d_labels, c->nvox));
  HIP_TRY(hipMalloc(&c->d_table, c->table.size() * sizeof(float4)));
  HIP_TRY(hipMalloc(&c->d_tally, ncells * sizeof(double)));
  HIP_TRY(hipMalloc(&c->d_counter, sizeof(unsigned long long)));
  HIP_TRY(hipMalloc(&c->d_params, kParamSlots * sizeof(mcx::TransportParams)));
  HIP_TRY(hipMalloc(&c->d_ledger, mcx::kLedgerN * sizeof(double)));
  HIP_TRY(hipMalloc(&c->d_counts, mcx::kCountN * sizeof(unsigned long long)));
  HIP_TRY(hipMalloc(&c->d_det_count, sizeof(unsigned long long)));
  HIP_TRY(hipMalloc(&c->d_reduce, 2 * sizeof(double)));
  if (c->detect && c->opt.max_detected > 0) {
    HIP_TRY(hipMalloc(&c->d_rec, c->opt.max_detected * c->rec_len * sizeof(float)));
    HIP_TRY(hipMalloc(&c->d_rec_photon, c->opt.max_detected * sizeof(unsigned long long)));
  }
  if (c->diag) HIP_TRY(hipMalloc(&c->d_digest, c->opt.ndigest * mcx::kDigestN * sizeof(double)));
  HIP_TRY(hipMemcpyAsync(c->d_labels, vol->labels, c->nvox, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_table, c->table.data(), c->table.size() * sizeof(float4),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(mcx::launch_clear(c->d_tally, ncells, c->d_ledger, c->d_counts, c->d_det_count,
                            c->d_reduce, c->stream));
  if (c->diag)
    HIP_TRY(hipMemsetAsync(c->d_digest, 0, c->opt.ndigest * mcx::kDigestN * sizeof(double),
                           c->stream));

  // Launch shape: the requested block size, or the one of the candidates
  // that keeps the most waves resident per CU once LDS is counted.
  const int wcells = c->win[3] * c->win[4] * c->win[5] * c->win[6];
  const int candidates[] = {256, 448, 512, 768, 1024};
  int best_block = 0, best_occ = 0, best_waves = -1;
  for (int b : candidates) {
    if (c->opt.block_size > 0 && b != candidates[0]) break;
    const int blk = c->opt.block_size > 0 ? c->opt.block_size : b;
    const size_t smem = mcx::transport_smem_bytes(c->nmedia, c->ndet, blk, c->detect, wcells);
    int occ = 0;
    HIP_TRY(mcx::transport_occupancy(&occ, blk, smem, c->detect, c->diag, c->opt.accurate_math != 0));
    if (occ * blk / 64 > best_waves) {
      best_waves = occ * blk / 64;
      best_block = blk;
      best_occ = occ;
    }
  }
  if (best_occ <= 0) return fail(MCX_EINVAL, "launch shape does not fit (block %d)", best_block);
  c->block = best_block;
  const int per_cu = c->opt.blocks_per_cu > 0 && c->opt.blocks_per_cu < best_occ
                         ? c->opt.blocks_per_cu : best_occ;
  c->grid = per_cu * c->cus;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MCX_OK;
}

mcx_status mcx_create(const mcx_volume* vol, const mcx_source* src, const mcx_detector* det,
                      int32_t ndet, const mcx_gates* gates, const mcx_options* opt,
                      mcx_ctx** out) {
  if (!out) return fail(MCX_EINVAL, "out pointer is NULL");
  mcx_status st = validate(vol, src, det, ndet, gates, opt);
  if (st != MCX_OK) return st;

  mcx_ctx* c = new (std::nothrow) mcx_ctx();
  if (!c) return fail(MCX_ENOMEM, "host allocation failed");
  if (opt)
    c->opt = *opt;
  else
    mcx_default_options(&c->opt);
  c->device = c->opt.device;
  c->nx = vol->nx;
  c->ny = vol->ny;
  c->nz = vol->nz;
  c->nvox = static_cast<uint32_t>(static_cast<uint64_t>(vol->nx) * vol->ny * vol->nz);
  c->h = vol->voxel_mm;
  c->nmedia = vol->nmedia;
  c->ndet = ndet;
  c->ngates = gates->ngates;
  c->t0 = gates->t0_ns;
  c->dt = gates->dt_ns;
  c->detect = ndet > 0;
  c->diag = c->opt.ndigest > 0;
  c->rec_len = 4 + (c->nmedia - 1);

  // per-medium tables: properties, derived reciprocals, HG constants
  c->table.assign(3 * c->nmedia + ndet, make_float4(0.f, 0.f, 0.f, 0.f));
  for (int m = 0; m < c->nmedia; ++m) {
    mcx_medium md = vol->media[m];
    if (m == 0) md = mcx_medium{0.f, 0.f, 0.f, c->opt.n_outside};
    const double mua = md.mua, mus = md.mus, g = md.g, n = md.n;
    c->table[m] = make_float4(md.mua, md.mus, md.g, md.n);
    c->table[c->nmedia + m] = make_float4(
        mus > 0 ? static_cast<float>(1.0 / mus) : __builtin_huge_valf(),
        static_cast<float>(n / kCmmPerNs), static_cast<float>(kCmmPerNs / n),
        mua > 0 ? static_cast<float>(1.0 / mua) : 0.f);
    c->table[2 * c->nmedia + m] =
        make_float4(static_cast<float>(1.0 - g), static_cast<float>(2.0 * g),
                    static_cast<float>(2.0 * (1.0 + g * g)), static_cast<float>((1.0 - g) * (1.0 - g)));
  }
  for (int d = 0; d < ndet; ++d) {
    const double r = det[d].radius;
    c->table[3 * c->nmedia + d] =
        make_float4(det[d].pos[0], det[d].pos[1], det[d].pos[2], static_cast<float>(r * r));
  }
  for (int a = 0; a < 3; ++a) {
    const double x = static_cast<double>(src->pos[a]) / c->h;
    const double fl = std::floor(x);
    c->src_i[a] = static_cast<int>(fl);
    c->src_f[a] = static_cast<float>(x - fl);
    c->src_dir[a] = src->dir[a];
  }
  c->src_label = vol->labels[c->src_i[0] + c->nx * (c->src_i[1] + static_cast<int64_t>(c->ny) * c->src_i[2])];

  // LDS window: a box of cells centred on the source voxel (shifted to stay
  // inside the grid) over the first gate, or the first two when there are
  // several, holding at most `budget` cells.
  const int budget = c->opt.lds_window_cells == 0 ? kDefaultWindow : c->opt.lds_window_cells;
  if (budget > 0) {
    const int wg = c->ngates > 1 ? 2 : 1;
    const int per_gate = budget / wg;
    int side = 1;
    while ((side + 1) * (side + 1) * (side + 1) <= per_gate) ++side;
    const int dims[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
      const int n = side < dims[a] ? side : dims[a];
      int lo = c->src_i[a] - n / 2;
      if (lo > dims[a] - n) lo = dims[a] - n;
      if (lo < 0) lo = 0;
      c->win[a] = lo;
      c->win[3 + a] = n;
    }
    c->win[6] = wg;
  }
  st = setup(c, vol);
  if (st != MCX_OK) {
    std::string keep = g_error;
    release(c);
    g_error = keep;
    return st;
  }
  *out = c;
  return MCX_OK;
}

void mcx_destroy(mcx_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  release(c);
}

uint64_t mcx_ncells(const mcx_ctx* c) { return c ? c->ncells() : 0; }

static hipStream_t pick_stream(mcx_ctx* c, void* s) {
  return s ? static_cast<hipStream_t>(s) : c->stream;
}

mcx_status mcx_reset(mcx_ctx* c, void* stream) {
  if (!c) return fail(MCX_EINVAL, "context is NULL");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  HIP_TRY(mcx::launch_clear(c->d_tally, c->ncells(), c->d_ledger, c->d_counts, c->d_det_count,
                            c->d_reduce, st));
  if (c->diag)
    HIP_TRY(hipMemsetAsync(c->d_digest, 0, c->opt.ndigest * mcx::kDigestN * sizeof(double), st));
  c->photons = 0;
  c->have_timing = false;
  return MCX_OK;
}

static mcx_status enqueue(mcx_ctx* c, uint64_t first, uint64_t n, uint64_t seed, hipStream_t st) {
  mcx::TransportParams p{};
  p.labels = c->d_labels;
  p.nx = c->nx;
  p.ny = c->ny;
  p.nz = c->nz;
  p.nvox = c->nvox;
  p.h = c->h;
  p.inv_h = static_cast<float>(1.0 / c->h);
  p.media = c->d_table;
  p.nmedia = c->nmedia;
  p.ndet = c->ndet;
  p.src_ix = c->src_i[0];
  p.src_iy = c->src_i[1];
  p.src_iz = c->src_i[2];
  p.src_label = c->src_label;
  p.src_fx = c->src_f[0];
  p.src_fy = c->src_f[1];
  p.src_fz = c->src_f[2];
  p.src_vx = c->src_dir[0];
  p.src_vy = c->src_dir[1];
  p.src_vz = c->src_dir[2];
  p.t0 = c->t0;
  p.inv_dt = static_cast<float>(1.0 / c->dt);
  p.t_end = static_cast<float>(static_cast<double>(c->t0) + static_cast<double>(c->ngates) * c->dt);
  p.ngates = c->ngates;
  p.reflect = c->opt.reflect ? 1 : 0;
  p.n_out = c->opt.n_outside;
  p.rr_threshold = c->opt.rr_threshold;
  p.rr_p = static_cast<float>(1.0 / c->opt.rr_m);
  p.rr_m = c->opt.rr_m;
  p.max_events = static_cast<uint32_t>(c->opt.max_events);
  p.first = first;
  p.nphoton = n;
  p.key0 = static_cast<uint32_t>(seed);
  p.key1 = static_cast<uint32_t>(seed >> 32);
  p.chunk = c->opt.refill_chunk > 0 ? static_cast<uint32_t>(c->opt.refill_chunk) : kDefaultChunk;
  p.wx0 = c->win[0];
  p.wy0 = c->win[1];
  p.wz0 = c->win[2];
  p.wnx = c->win[3];
  p.wny = c->win[4];
  p.wnz = c->win[5];
  p.wng = c->win[6];
  p.tally = c->d_tally;
  p.photon_counter = c->d_counter;
  p.ledger = c->d_ledger;
  p.counts = c->d_counts;
  p.det_rec = c->d_rec;
  p.det_photon = c->d_rec_photon;
  p.det_count = c->d_det_count;
  p.det_cap = c->d_rec ? c->opt.max_detected : 0;
  p.rec_len = c->rec_len;
  p.digest = c->d_digest;
  p.ndigest = c->diag ? c->opt.ndigest : 0;

  // Each launch reads its parameters from its own device slot, so launches
  // queued back to back (even on different streams, up to kParamSlots deep)
  // never see each other's parameters.
  mcx::TransportParams* slot = c->d_params + (c->launches++ % kParamSlots);
  HIP_TRY(hipMemcpyAsync(slot, &p, sizeof(p), hipMemcpyHostToDevice, st));
  HIP_TRY(mcx::launch_reset_counter(c->d_counter, st));
  HIP_TRY(hipEventRecord(c->ev_k0, st));
  HIP_TRY(mcx::launch_transport(p, slot, c->grid, c->block, st, c->detect, c->diag,
                                c->opt.accurate_math != 0));
  HIP_TRY(hipEventRecord(c->ev_k1, st));
  HIP_TRY(hipMemsetAsync(c->d_reduce, 0, 2 * sizeof(double), st));
  HIP_TRY(mcx::launch_reduce(c->d_tally, c->d_labels, c->d_table, c->nvox, c->ngates,
                             c->d_reduce, st));
  HIP_TRY(hipEventRecord(c->ev_end, st));
  c->photons += n;
  c->have_timing = true;
  return MCX_OK;
}

mcx_status mcx_run_range(mcx_ctx* c, uint64_t first, uint64_t n, uint64_t seed, void* stream) {
  if (!c) return fail(MCX_EINVAL, "context is NULL");
  if (n > (1ull << 62) || first > (1ull << 62)) return fail(MCX_EINVAL, "photon range too large");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  HIP_TRY(hipEventRecord(c->ev_begin, st));
  return enqueue(c, first, n, seed, st);
}

mcx_status mcx_run(mcx_ctx* c, uint64_t nphoton, uint64_t seed) {
  if (!c) return fail(MCX_EINVAL, "context is NULL");
  if (nphoton > (1ull << 62)) return fail(MCX_EINVAL, "photon count too large");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipEventRecord(c->ev_begin, c->stream));
  mcx_status st = mcx_reset(c, c->stream);
  if (st != MCX_OK) return st;
  st = enqueue(c, 0, nphoton, seed, c->stream);
  if (st != MCX_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MCX_OK;
}

mcx_status mcx_sync(mcx_ctx* c) {
  if (!c) return fail(MCX_EINVAL, "context is NULL");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MCX_OK;
}

static mcx_status scale_for(mcx_ctx* c, int32_t kind, double* scale) {
  if (kind == MCX_RAW) {
    *scale = 1.0;
    return MCX_OK;
  }
  if (kind != MCX_FLUENCE && kind != MCX_FLUENCE_RATE)
    return fail(MCX_EINVAL, "kind must be 0 (raw), 1 (fluence) or 2 (fluence rate)");
  if (c->photons == 0) return fail(MCX_ESTATE, "no photons simulated since the last reset");
  const double hv = static_cast<double>(c->h);
  double s = 1.0 / (static_cast<double>(c->photons) * hv * hv * hv);
  if (kind == MCX_FLUENCE_RATE) s /= static_cast<double>(c->dt);
  *scale = s;
  return MCX_OK;
}

mcx_status mcx_fluence_device(mcx_ctx* c, int32_t kind, float* dev_out, uint64_t ncells,
                              void* stream) {
  if (!c || !dev_out) return fail(MCX_EINVAL, "context and output are required");
  if (ncells < c->ncells()) return fail(MCX_ERANGE, "output holds %llu cells, need %llu",
                                        static_cast<unsigned long long>(ncells),
                                        static_cast<unsigned long long>(c->ncells()));
  double scale = 1.0;
  mcx_status st = scale_for(c, kind, &scale);
  if (st != MCX_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(mcx::launch_normalise_f32(c->d_tally, c->ncells(), scale, dev_out,
                                    pick_stream(c, stream)));
  return MCX_OK;
}

mcx_status mcx_fluence(mcx_ctx* c, int32_t kind, float* host_out, uint64_t ncells) {
  if (!c || !host_out) return fail(MCX_EINVAL, "context and output are required");
  if (ncells < c->ncells()) return fail(MCX_ERANGE, "output holds %llu cells, need %llu",
                                        static_cast<unsigned long long>(ncells),
                                        static_cast<unsigned long long>(c->ncells()));
  double scale = 1.0;
  mcx_status st = scale_for(c, kind, &scale);
  if (st != MCX_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  if (!c->d_stage32) HIP_TRY(hipMalloc(&c->d_stage32, c->ncells() * sizeof(float)));
  HIP_TRY(mcx::launch_normalise_f32(c->d_tally, c->ncells(), scale, c->d_stage32, c->stream));
  HIP_TRY(hipMemcpyAsync(host_out, c->d_stage32, c->ncells() * sizeof(float),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MCX_OK;
}

mcx_status mcx_fluence_f64(mcx_ctx* c, int32_t kind, double* host_out, uint64_t ncells) {
  if (!c || !host_out) return fail(MCX_EINVAL, "context and output are required");
  if (ncells < c->ncells()) return fail(MCX_ERANGE, "output holds %llu cells, need %llu",
                                        static_cast<unsigned long long>(ncells),
                                        static_cast<unsigned long long>(c->ncells()));
  double scale = 1.0;
  mcx_status st = scale_for(c, kind, &scale);
  if (st != MCX_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  if (!c->d_stage64) HIP_TRY(hipMalloc(&c->d_stage64, c->ncells() * sizeof(double)));
  HIP_TRY(mcx::launch_normalise_f64(c->d_tally, c->ncells(), scale, c->d_stage64, c->stream));
  HIP_TRY(hipMemcpyAsync(host_out, c->d_stage64, c->ncells() * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MCX_OK;
}

mcx_status mcx_detected(mcx_ctx* c, float* host_rec, uint64_t* host_photon, uint64_t cap,
                        uint64_t* nrec, uint64_t* ndropped) {
  if (!c) return fail(MCX_EINVAL, "context is NULL");
  if (cap > 0 && !host_rec) return fail(MCX_EINVAL, "record buffer is NULL");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  unsigned long long total = 0;
  HIP_TRY(hipMemcpy(&total, c->d_det_count, sizeof(total), hipMemcpyDeviceToHost));
  const uint64_t stored = c->d_rec ? (total < c->opt.max_detected ? total : c->opt.max_detected) : 0;
  const uint64_t copy = stored < cap ? stored : cap;
  if (copy > 0) {
    HIP_TRY(hipMemcpy(host_rec, c->d_rec, copy * c->rec_len * sizeof(float), hipMemcpyDeviceToHost));
    if (host_photon)
      HIP_TRY(hipMemcpy(host_photon, c->d_rec_photon, copy * sizeof(uint64_t), hipMemcpyDeviceToHost));
  }
  if (nrec) *nrec = copy;
  if (ndropped) *ndropped = total - stored;
  return MCX_OK;
}

mcx_status mcx_stats(mcx_ctx* c, mcx_run_stats* o) {
  if (!c || !o) return fail(MCX_EINVAL, "context and output are required");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double led[mcx::kLedgerN];
  unsigned long long cnt[mcx::kCountN];
  unsigned long long det_total = 0;
  double red[2];
  HIP_TRY(hipMemcpy(led, c->d_ledger, sizeof(led), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(cnt, c->d_counts, sizeof(cnt), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(&det_total, c->d_det_count, sizeof(det_total), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(red, c->d_reduce, sizeof(red), hipMemcpyDeviceToHost));
  memset(o, 0, sizeof(*o));
  o->launched = cnt[mcx::kCntLaunched];
  o->escaped = cnt[mcx::kCntEscaped];
  o->detected = cnt[mcx::kCntDetected];
  o->timeout = cnt[mcx::kCntTimeout];
  o->rr_dead = cnt[mcx::kCntRrDead];
  o->capped = cnt[mcx::kCntCapped];
  o->scatters = cnt[mcx::kCntScatters];
  o->face_events = cnt[mcx::kCntFaceEvents];
  o->fresnel_draws = cnt[mcx::kCntFresnel];
  o->reflections = cnt[mcx::kCntReflections];
  o->rr_tests = cnt[mcx::kCntRrTests];
  o->rr_survived = cnt[mcx::kCntRrSurvived];
  o->events = cnt[mcx::kCntEvents];
  o->lane_slots = cnt[mcx::kCntLaneSlots];
  o->flushes = cnt[mcx::kCntFlushes];
  const uint64_t cap = c->d_rec ? c->opt.max_detected : 0;
  o->det_records = det_total < cap ? det_total : cap;
  o->det_dropped = det_total - o->det_records;
  o->w_launched = static_cast<double>(cnt[mcx::kCntLaunched]);
  o->w_escaped = led[mcx::kLedEscaped];
  o->w_detected = led[mcx::kLedDetected];
  o->w_timeout = led[mcx::kLedTimeout];
  o->w_rr_gain = led[mcx::kLedRrGain];
  o->w_rr_loss = led[mcx::kLedRrLoss];
  o->w_capped = led[mcx::kLedCapped];
  o->tally_sum = red[0];
  o->absorbed_grid = red[1];
  if (c->have_timing) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_k0, c->ev_k1) == hipSuccess) o->kernel_ms = ms;
    if (hipEventElapsedTime(&ms, c->ev_begin, c->ev_end) == hipSuccess) o->run_ms = ms;
  }
  o->grid_blocks = c->grid;
  o->block_size = c->block;
  return MCX_OK;
}

mcx_status mcx_digest(mcx_ctx* c, double* host_out, uint64_t nrows) {
  if (!c || !host_out) return fail(MCX_EINVAL, "context and output are required");
  if (!c->diag) return fail(MCX_ESTATE, "context was created with ndigest = 0");
  if (nrows > c->opt.ndigest) return fail(MCX_ERANGE, "only %llu digest rows are kept",
                                          static_cast<unsigned long long>(c->opt.ndigest));
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(host_out, c->d_digest, nrows * mcx::kDigestN * sizeof(double),
                    hipMemcpyDeviceToHost));
  return MCX_OK;
}

}  // extern "C"
