// Persistent photon-transport kernel for gfx950 (MI355X).
//
// One lane carries one photon at a time through the paper's per-thread
// simulation loop (problem statement and Fig. 1 workflow): launch, free
// path, voxel hops, absorption deposits into a time-gated fluence map,
// Henyey-Greenstein scattering, Fresnel reflection/refraction or escape,
// Russian roulette and detector capture.  The paper's in-workgroup dynamic
// load balancing (a shared photon quota that threads decrement to start
// their next photon) becomes wave-level refill: whenever lanes of a wave
// finish, the wave hands them the next photon indices from a job (a chunk of
// photons of one simulation) it took from that simulation's 64-bit job
// counter, so a wave keeps its 64 lanes busy until the supply runs out.  One
// launch can serve many independent simulations of different grids and
// photon counts: a wave works on one simulation at a time (its descriptor is
// read with scalar loads), starting on a home simulation chosen so that
// waves are spread over simulations in proportion to their work, and moves
// on to the next simulation with jobs left -- after its lanes have finished
// -- only when the current one is exhausted.
//
// Per-lane state stays in registers; each wave keeps its simulation's media
// table and detectors, an FP64 energy ledger and rare-event counters in its
// own slice of LDS, and the lanes' partial pathlengths in LDS.
// Deposits made while a photon stays in one tally cell are summed in a
// register and flushed once when it leaves the cell.  Flushes into the
// densest cells of the workgroup's window simulation (the home simulation
// of its first wave) -- per early gate a box of cells, the "window" -- go to
// integer partial sums in LDS (visit sums are rounded to a fixed deposit
// unit, see deposit()), added to the map once when the workgroup finishes
// (or earlier, by the lane whose addition takes a sum past 2^31 units).  All
// other flushes are one atomic add to the map's integer counts (map_add).
// Device-memory atomics on gfx950 execute at the memory side at a fixed
// aggregate rate, which binds this kernel wherever photons spread out, so
// the window is what keeps the cells that most photons of a workgroup visit
// -- next to a pencil beam, early in the photons' lives -- off that path.
#include <math.h>

#include "mcx_internal.hpp"

namespace mcx {
namespace {

constexpr float kInf = __builtin_huge_valf();

// ----------------------------------------------------------- random numbers
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds; each
// multiplies counter words 0 and 2 by the round constants and rebuilds the
// counter from the high halves xored with the other words and the key and
// from the low halves; the key advances by the Weyl constants per round.
struct Words {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c1 = static_cast<uint32_t>(p1);
    c3 = static_cast<uint32_t>(p0);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// Odd multiple of 2^-24 in (0, 1); exact in FP32.
__device__ __forceinline__ float unit_open(uint32_t x) {
  return static_cast<float>((x >> 8) | 1u) * 0x1p-24f;
}

// ------------------------------------------------------------- wave helpers
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), lane);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), lane);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Pointers read from the descriptors are generic; these casts tell the
// compiler where they point, so that descriptor fields are read with scalar
// loads from the constant space and labels / tallies with global (not flat)
// instructions.
#define MCX_CONST __attribute__((address_space(4)))
#define MCX_GLOBAL __attribute__((address_space(1)))
using CSim = const MCX_CONST SimDesc;

template <typename T>
__device__ __forceinline__ const MCX_CONST T* as_const(const T* p) {
  return (const MCX_CONST T*)(p);
}
template <typename T>
__device__ __forceinline__ MCX_GLOBAL T* as_global(T* p) {
  return (MCX_GLOBAL T*)(p);
}

// A descriptor pointer every lane holds the same value of, kept in scalar
// registers.
__device__ __forceinline__ CSim* uniform_sim(CSim* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<CSim*>((static_cast<uint64_t>(hi) << 32) | lo);
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint32_t wave_count(bool p) {
  return static_cast<uint32_t>(__popcll(__ballot(p)));
}

// ------------------------------------------------------------------ physics
// Distance along the direction to the face a velocity component points at;
// `face` is the local coordinate gap, `r` = h/|v| (only used when v != 0).
__device__ __forceinline__ float face_dist(float f, float v, float r) {
  const float gap = fmaxf(v > 0.f ? 1.f - f : f, 0.f);
  return v != 0.f ? gap * r : kInf;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Transcendentals in two flavours: the hardware instructions (the paper's
// "native math", within ~1 ulp on gfx950; sin/cos take revolutions, so
// 2*pi*u needs no scaling) or the device math library.
template <bool kNative>
__device__ __forceinline__ float neg_log(float u) {  // -ln u, u in (0, 1)
  if constexpr (kNative)
    return __builtin_amdgcn_logf(u) * -0.69314718055994531f;
  else
    return -logf(u);
}

template <bool kNative>
__device__ __forceinline__ void sincos_turn(float u, float* s, float* c) {  // of 2*pi*u
  if constexpr (kNative) {
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
  } else {
    sincospif(2.f * u, s, c);
  }
}

template <bool kNative>
__device__ __forceinline__ float fsqrt(float x) {
  if constexpr (kNative)
    return __builtin_amdgcn_sqrtf(x);
  else
    return sqrtf(x);
}

// 1 - exp(-x) for x >= 0 without cancellation: its alternating series to the
// x^7 term below 0.25 (truncation < 2e-9 relative), 1 - exp(-x) above.
template <bool kNative>
__device__ __forceinline__ float one_minus_exp(float x) {
  if constexpr (kNative) {
    if (x < 0.25f) {
      float r = fmaf(x, 1.f / 5040.f, -1.f / 720.f);
      r = fmaf(x, r, 1.f / 120.f);
      r = fmaf(x, r, -1.f / 24.f);
      r = fmaf(x, r, 1.f / 6.f);
      r = fmaf(x, r, -0.5f);
      r = fmaf(x, r, 1.f);
      return x * r;
    }
    return 1.f - __builtin_amdgcn_exp2f(x * -1.4426950408889634f);
  } else {
    return -expm1f(-x);
  }
}

__device__ __forceinline__ float inv_speed(float h, float v) {
  return v != 0.f ? h * rcp(fabsf(v)) : kInf;
}

// Cosine of the Henyey-Greenstein deflection from its inverse CDF, written
// over a common denominator so that g = 0 needs no special case:
// cos = (2u(1+g^2)(1-g+gu) - (1-g)^2) / (1-g+2gu)^2.
// hg = (1-g, 2g, 2(1+g^2), (1-g)^2).
__device__ __forceinline__ float hg_cos(float g, float4 hg, float u) {
  const float a = fmaf(hg.y, u, hg.x);
  const float num = hg.z * u * fmaf(g, u, hg.x) - hg.w;
  const float c = num * rcp(a * a);
  return fminf(1.f, fmaxf(-1.f, c));
}

// Turn v by polar cosine ct and azimuth 2*pi*u, the azimuth measured in the
// branchless orthonormal basis of Duff et al., JCGT 6(1) 2017, then
// renormalise.
template <bool kNative>
__device__ __forceinline__ void scatter_dir(float& vx, float& vy, float& vz, float ct, float u) {
  const float st = fsqrt<kNative>((1.f - ct) * (1.f + ct));
  float sp, cp;
  sincos_turn<kNative>(u, &sp, &cp);
  const float sg = copysignf(1.f, vz);
  const float a = -rcp(sg + vz);
  const float b = vx * vy * a;
  const float t1x = 1.f + sg * vx * vx * a, t1y = sg * b, t1z = -sg * vx;
  const float t2x = b, t2y = sg + vy * vy * a, t2z = -vy;
  const float nx = ct * vx + st * (cp * t1x + sp * t2x);
  const float ny = ct * vy + st * (cp * t1y + sp * t2y);
  const float nz = ct * vz + st * (cp * t1z + sp * t2z);
  const float inv = __builtin_amdgcn_rsqf(nx * nx + ny * ny + nz * nz);
  vx = nx * inv;
  vy = ny * inv;
  vz = nz * inv;
}

// Unpolarised Fresnel reflectance (mean of the s and p terms).
__device__ __forceinline__ float fresnel_r(float n1, float n2, float ci, float ct) {
  const float rs = (n1 * ci - n2 * ct) * rcp(n1 * ci + n2 * ct);
  const float rp = (n1 * ct - n2 * ci) * rcp(n1 * ct + n2 * ci);
  return 0.5f * (rs * rs + rp * rp);
}

// A visit sum of more than 2^28 deposit units (256 voxel sizes of path in
// one cell) goes to the map directly, and a window sum that reaches 2^31
// units is moved to the map by the lane whose addition took it there, so
// the 32-bit window sums cannot wrap.
constexpr uint32_t kWinMaxAdd = 268435456u;
constexpr uint32_t kWinMove = 0x80000000u;

// Add q deposit units to map cell p, exactly.  The map holds 64-bit integer
// sums of units.  map32: a returning 32-bit add to the cell's low word, and
// when that add carries out of it (the returned old value plus q wraps), a
// second add of 1 to the high word -- every carry is seen by exactly the
// add that caused it, so the 64-bit sum is exact once the launch ends, and
// 32-bit adds execute faster at the memory side than 64-bit ones (the wave
// waits for the returned value, which pays only when enough waves are
// resident to cover that latency).  Otherwise one 64-bit add without a
// return value.
__device__ __forceinline__ void map_add(MCX_GLOBAL uint64_t* p, uint32_t q, bool map32) {
  if (map32) {
    MCX_GLOBAL uint32_t* w = reinterpret_cast<MCX_GLOBAL uint32_t*>(p);
    const uint32_t old = __hip_atomic_fetch_add(w, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + q < old) __hip_atomic_fetch_add(w + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_fetch_add(p, static_cast<uint64_t>(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Add a finished cell visit to the map; returns the number of global
// atomics issued (0 or 1).  The visit's sum v is first rounded to a whole
// number q of the simulation's deposit unit u (a power of two, 2^-20 of the
// voxel size or just below): the map holds integer counts of u, so every
// sum is exact and the map does not depend on the order of the additions
// -- any launch shape, batch or photon split gives the same bits.  A visit
// into the workgroup's LDS window adds q to that cell's 32-bit integer sum
// (the lane that takes it to 2^31 or more exchanges it with zero and adds
// what it took to the map); any other is added to the map by map_add.
// kRacy: a plain read, add and write of the map cell instead of the atomic
// -- the paper's non-atomic benchmark variant (B2), where concurrent updates
// of one cell can be lost.  kCensus: 1 per visit instead (the flush census).
template <bool kRacy, bool kCensus = false>
__device__ __forceinline__ int deposit(CSim* D, uint32_t* s_win, uint32_t cell, int slot,
                                      float v, bool map32) {
  MCX_GLOBAL uint64_t* p = as_global(D->tally) + cell;
  if constexpr (kCensus) {
    map_add(p, 1u, false);
    return 1;
  }
  const float qf = rintf(v * D->q_inv);  // an exact scaling by a power of two
  if (qf >= 4294967296.f) {  // 2^32 units or more in one visit: one 64-bit add
    if constexpr (kRacy)
      *p = *p + static_cast<uint64_t>(qf);
    else
      __hip_atomic_fetch_add(p, static_cast<uint64_t>(qf), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    return 1;
  }
  const uint32_t q = static_cast<uint32_t>(qf);
  if (slot >= 0 && q <= kWinMaxAdd) {
    if (atomicAdd(s_win + slot, q) + q < kWinMove) return 0;
    map_add(p, atomicExch(s_win + slot, 0u), map32);
    return 1;
  }
  if constexpr (kRacy)
    *p = *p + q;
  else
    map_add(p, q, map32);
  return 1;
}

enum : int { kEvTime = 0, kEvScat = 1, kEvCross = 2 };
enum : int { kAlive = 0, kEndEscape = 1, kEndTime = 2, kEndRoulette = 3, kEndCapped = 4 };

// Event-loop variants (the paper's benchmark study, Fig. 2): the default
// loop; map deposits without atomics (B2); the branch-reduced loop (Opt3),
// where every lane computes both the scattering and the face-crossing
// updates and keeps its own by selection instead of branching on its event.
enum : int { kVarDefault = 0, kVarRacy = 1, kVarFlat = 2, kVarCensus = kVariantCensus };

// Window slot of cell (gate, ix, iy, iz) from the per-gate boxes, or -1.
__device__ __forceinline__ int window_slot(const int4* s_wbox, int wng, int gate, int ix, int iy,
                                           int iz) {
  if (gate >= wng) return -1;
  const int4 a = s_wbox[2 * gate], b = s_wbox[2 * gate + 1];
  const uint32_t ux = static_cast<uint32_t>(ix - a.x);
  const uint32_t uy = static_cast<uint32_t>(iy - a.y);
  const uint32_t uz = static_cast<uint32_t>(iz - a.z);
  if (ux < static_cast<uint32_t>(b.x) && uy < static_cast<uint32_t>(b.y) &&
      uz < static_cast<uint32_t>(b.z))
    return a.w + static_cast<int>((uz * b.y + uy) * b.x + ux);
  return -1;
}

// Map cell of window slot i (0 <= i < the window's slot count).
__device__ __forceinline__ uint32_t window_cell(const int4* s_wbox, int wng, CSim* DW, int i) {
  int g = 0;
  while (g + 1 < wng && s_wbox[2 * (g + 1)].w <= i) ++g;
  const int4 a = s_wbox[2 * g], b = s_wbox[2 * g + 1];
  int r = i - a.w;
  const int x = r % b.x;
  r /= b.x;
  const int y = r % b.y;
  const int z = r / b.y;
  return static_cast<uint32_t>(g) * DW->nvox + static_cast<uint32_t>(a.x + x) +
         DW->stride_y * static_cast<uint32_t>(a.y + y) +
         DW->stride_z * static_cast<uint32_t>(a.z + z);
}

template <bool kDetect, bool kDiag, bool kNative, int kVar>
__global__ void __launch_bounds__(1024) transport_kernel(const LaunchParams* params) {
  constexpr bool kRacy = kVar == kVarRacy;
  constexpr bool kCensus = kVar == kVarCensus;
  // Launch and simulation parameters live in device memory and are read
  // where used (scalar loads that hit the scalar cache) rather than held in
  // scalar registers for the whole persistent loop.
  const LaunchParams& L = *params;
  extern __shared__ float4 s_dyn[];
  __shared__ double s_led[kMaxWavesPerBlock][kLedgerN];
  __shared__ unsigned long long s_cnt[kMaxWavesPerBlock][kCountN];
  __shared__ int4 s_wbox[2 * kMaxWinGates];

  const uint32_t lane = __lane_id();
  const int wid = static_cast<int>(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));  // wave-uniform
  const uint32_t bdim = blockDim.x;
  const int rows = L.table_rows;
  float4* s_tab = s_dyn + wid * rows;  // this wave's copy of its simulation's tables
  const int wcells = kCensus ? 0 : L.window_cells;
  const bool map32 = L.map32 != 0;  // how map cells are added to (map_add)
  uint32_t* s_win = reinterpret_cast<uint32_t*>(s_dyn + (bdim >> 6) * rows);
  float* s_len = reinterpret_cast<float*>(s_win + wcells) + threadIdx.x;  // [m * blockDim]

  // Home simulation: the one whose share of home_start holds point
  // ((2 v + 1) / 2) * nhome / nwaves -- shares are the simulations' job
  // counts, or their estimated work (device-level balancing by throughput)
  // -- where v numbers the waves so that the workgroups of one XCD
  // (dispatched round-robin over the 8 XCDs) are consecutive; the waves of a
  // simulation then share an XCD and its L2 as far as the shares allow.
  const MCX_CONST uint64_t* js = as_const(L.job_start);
  const MCX_CONST uint64_t* hs = as_const(L.home_start);
  const uint32_t nb = gridDim.x;
  const uint32_t vb = (nb % 8u == 0u) ? (blockIdx.x % 8u) * (nb / 8u) + blockIdx.x / 8u
                                      : blockIdx.x;
  const uint64_t wpb = bdim >> 6;
  auto home_of = [&](uint64_t v) -> int {
    const uint64_t target = ((2 * v + 1) * L.nhome) / (2 * nb * wpb);
    int lo = 0, hi = L.nsims;  // home_start[lo] <= target < home_start[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (hs[mid] <= target) lo = mid; else hi = mid;
    }
    return lo;
  };
  int scan = home_of(vb * wpb + static_cast<uint64_t>(wid));  // where the wave takes jobs
  // the workgroup's window belongs to the home simulation of its first wave
  const int wsim = home_of(vb * wpb);
  CSim* DW = uniform_sim(as_const(L.sims) + wsim);
  const int wng = wcells ? DW->wng : 0;
  const int wcount = wcells ? DW->wcount : 0;

  for (int i = threadIdx.x; i < wcount; i += bdim) s_win[i] = 0u;
  if (static_cast<int>(threadIdx.x) < 2 * wng) s_wbox[threadIdx.x] = DW->wbox[threadIdx.x];
  if (lane < kLedgerN) s_led[wid][lane] = 0.0;
  if (lane < kCountN) s_cnt[wid][lane] = 0ull;
  __syncthreads();
  const float4* s_med = s_tab;  // (mua, mus, g, n); the other tables follow at nmedia offsets

  // photon state
  bool alive = false;
  int ix = 0, iy = 0, iz = 0, m = 0;
  uint32_t lin = 0;
  float fx = 0.f, fy = 0.f, fz = 0.f, vx = 0.f, vy = 0.f, vz = 1.f;
  float rx = kInf, ry = kInf, rz = kInf;
  float w = 0.f, t = 0.f, s = 0.f;
  uint32_t klo = 0, khi = 0, blk = 0, nev = 0, nscat = 0;
  // two most recent tally cells of this photon, most recent first
  uint32_t acc_cell = 0xffffffffu, old_cell = 0xffffffffu;
  int acc_slot = -1, old_slot = -1;
  float acc = 0.f, old_acc = 0.f;

  // wave-uniform state: current simulation, its photon pool [pool_next,
  // pool_end) (offsets from its first photon), and a job taken but not yet
  // started because the wave was still busy with another simulation
  int cur = -1;
  CSim* D = as_const(L.sims);
  uint64_t pool_next = 0, pool_end = 0;
  bool has_pend = false, dry = false;
  int pend_sim = 0;
  uint64_t pend_first = 0, pend_end = 0;
  // per-wave counts of frequent events (scalar registers); rare events are
  // counted in the wave's LDS slice by the lanes they happen to
  uint32_t c_launch = 0, c_scat = 0, c_face = 0, c_fres = 0, c_ev = 0, c_slots = 0, c_flush = 0;

  // add the wave's tallies of simulation `cur` to its totals and clear them
  // move the 32-bit register counts to the wave's 64-bit LDS counters
  auto spill_counts = [&]() {
    if (lane == 0) {
      s_cnt[wid][kCntLaunched] += c_launch;
      s_cnt[wid][kCntScatters] += c_scat;
      s_cnt[wid][kCntFaceEvents] += c_face;
      s_cnt[wid][kCntFresnel] += c_fres;
      s_cnt[wid][kCntEvents] += c_ev;
      s_cnt[wid][kCntLaneSlots] += c_slots;
      s_cnt[wid][kCntFlushes] += c_flush;
    }
    c_launch = c_scat = c_face = c_fres = c_ev = c_slots = c_flush = 0;
  };
  auto flush_wave = [&]() {
    spill_counts();
    if (cur >= 0) {
      if (lane == 0) {
        unsigned long long* C = D->counts;
        for (int i = 0; i < kCountN; ++i)
          if (s_cnt[wid][i]) atomicAdd(C + i, s_cnt[wid][i]);
        for (int i = 0; i < kLedgerN; ++i)
          if (s_led[wid][i] != 0.0) unsafeAtomicAdd(D->ledger + i, s_led[wid][i]);
      }
    }
    if (lane < kLedgerN) s_led[wid][lane] = 0.0;
    if (lane < kCountN) s_cnt[wid][lane] = 0ull;
  };

  for (;;) {
    // The current simulation is the same for the whole wave; say so, so that
    // its descriptor is read with scalar loads.
    D = uniform_sim(D);
    // ---------------------------------------------------------------- refill
    bool launched = false;
    const uint64_t dead = __ballot(!alive);
    if (dead != 0 && !dry) {
      if (pool_next == pool_end && !has_pend) {
        // next job of simulation `scan`; when it has none left, try the
        // following simulations (cyclically) until one has, or all are done
        const int leader = __ffsll(static_cast<long long>(dead)) - 1;
        for (int tried = 0;; ++tried) {
          if (tried >= L.nsims) {
            dry = true;
            break;
          }
          const uint64_t njob = js[scan + 1] - js[scan];
          unsigned long long* ctr = L.job_counters + scan;
          unsigned long long got = njob;
          if (static_cast<int>(lane) == leader) {
            // a relaxed read first, so that finished simulations cost no atomic
            got = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (got < njob) got = atomicAdd(ctr, 1ull);
          }
          const uint64_t j = readlane_u64(got, leader);
          if (j < njob) {
            const uint64_t off = j * L.chunk;
            const uint64_t n = as_const(L.sims)[scan].nphoton;
            pend_sim = scan;
            pend_first = off;
            pend_end = off + L.chunk < n ? off + L.chunk : n;
            has_pend = true;
            break;
          }
          scan = scan + 1 == L.nsims ? 0 : scan + 1;
        }
      }
      if (pool_next == pool_end && has_pend && (pend_sim == cur || dead == ~0ull)) {
        if (pend_sim != cur) {
          // every lane is idle: move the wave to the job's simulation
          flush_wave();
          cur = pend_sim;
          D = uniform_sim(as_const(L.sims) + cur);
          const int nrow = 3 * D->nmedia + D->ndet;
          for (int i = lane; i < nrow; i += 64) s_tab[i] = D->tables[i];
          __builtin_amdgcn_wave_barrier();
        }
        pool_next = pend_first;
        pool_end = pend_end;
        has_pend = false;
      }
      const uint64_t rem = pool_end - pool_next;
      const uint64_t need = static_cast<uint64_t>(__popcll(dead));
      const uint64_t give = rem < need ? rem : need;
      if (!alive) {
        const uint64_t rank = rank_below(dead);
        if (rank < give) {
          const uint64_t k = D->first + pool_next + rank;
          klo = static_cast<uint32_t>(k);
          khi = static_cast<uint32_t>(k >> 32);
          const Words r = philox4x32_10(klo, khi, 0u, 0u, D->key0, D->key1);
          s = neg_log<kNative>(unit_open(r.x));
          blk = 1;
          ix = D->src_ix;
          iy = D->src_iy;
          iz = D->src_iz;
          lin = D->src_lin;
          m = D->src_label;
          fx = D->src_fx;
          fy = D->src_fy;
          fz = D->src_fz;
          vx = D->src_vx;
          vy = D->src_vy;
          vz = D->src_vz;
          rx = inv_speed(D->h, vx);
          ry = inv_speed(D->h, vy);
          rz = inv_speed(D->h, vz);
          w = 1.f;
          t = D->t0;
          nev = 0;
          nscat = 0;
          acc_cell = 0xffffffffu;
          acc_slot = -1;
          acc = 0.f;
          old_cell = 0xffffffffu;
          old_slot = -1;
          old_acc = 0.f;
          if constexpr (kDetect) {
            for (int mm = 0; mm < L.nmedia_max; ++mm) s_len[mm * bdim] = 0.f;
          }
          alive = true;
          launched = true;
        }
      }
      pool_next += give;
    }
    c_launch += wave_count(launched);
    if (__ballot(alive) == 0) {
      if (dry) break;
      continue;  // the wave's lanes just finished: take the pending job next
    }
    D = uniform_sim(D);
    if (c_slots >= (1u << 30)) spill_counts();  // keeps every 32-bit count from wrapping
    c_slots += 64;
    c_ev += wave_count(alive);

    // ----------------------------------------------------------------- event
    int end = kAlive;
    int det_hit = -1;
    bool f_scat = false, f_face = false, f_fres = false;
    int n_flush = 0;  // global atomics this lane issued in this iteration (at most 3)
    if (alive) {
      if (nev >= L.max_events) {
        end = kEndCapped;
      } else {
        ++nev;
        const int nm = D->nmedia;
        const float4 md = s_med[m];        // mua, mus, g, n
        const float4 dd = s_med[nm + m];   // 1/mus, n/c, c/n, 1/mua
        const float ds = md.y > 0.f ? s * dd.x : kInf;
        const float dx = face_dist(fx, vx, rx), dy = face_dist(fy, vy, ry),
                    dz = face_dist(fz, vz, rz);
        int ax;
        float dv;
        if (dx <= dy && dx <= dz) {
          ax = 0;
          dv = dx;
        } else if (dy <= dz) {
          ax = 1;
          dv = dy;
        } else {
          ax = 2;
          dv = dz;
        }
        const float dtime = fmaxf((D->t_end - t) * dd.z, 0.f);
        int ev;
        float l;
        if (dtime < fminf(ds, dv)) {
          ev = kEvTime;
          l = dtime;
        } else if (ds <= dv) {
          ev = kEvScat;
          l = ds;
        } else {
          ev = kEvCross;
          l = dv;
        }

        // absorption along the segment, booked at the segment-start gate
        int gate = static_cast<int>(floorf((t - D->t0) * D->inv_dt));
        gate = min(max(gate, 0), D->ngates - 1);
        const uint32_t cell = static_cast<uint32_t>(gate) * D->nvox + lin;
        const float q = one_minus_exp<kNative>(md.x * l);  // 1 - exp(-mua l)
        const float dep = md.x > 0.f ? w * q * dd.w : w * l;
        if constexpr (kVar == kVarFlat) {
          // the same two-entry update by selection: a hit on the current
          // entry adds to it; a hit on the previous one swaps the entries;
          // a miss flushes the previous entry and shifts the current one
          const bool hit_a = cell == acc_cell;
          const bool hit_o = !hit_a && cell == old_cell;
          const bool miss = !hit_a && !hit_o;
          if (miss && old_cell != 0xffffffffu && old_acc != 0.f) {
            n_flush += deposit<kRacy, kCensus>(D, s_win, old_cell, old_slot, old_acc, map32);
          }
          const int slot = cur == wsim ? window_slot(s_wbox, wng, gate, ix, iy, iz) : -1;
          const float a_new = hit_a ? acc : (hit_o ? old_acc : 0.f);
          const int s_new = hit_a ? acc_slot : (hit_o ? old_slot : slot);
          old_acc = hit_a ? old_acc : acc;
          old_slot = hit_a ? old_slot : acc_slot;
          old_cell = hit_a ? old_cell : acc_cell;
          acc = miss ? dep : a_new + dep;
          acc_slot = s_new;
          acc_cell = cell;
        } else if (cell == acc_cell) {
          acc += dep;
        } else if (cell == old_cell) {
          // back in the previous cell: swap the two entries
          const float ta = acc;
          const int ts = acc_slot;
          acc = old_acc + dep;
          acc_slot = old_slot;
          old_acc = ta;
          old_slot = ts;
          old_cell = acc_cell;
          acc_cell = cell;
        } else {
          if (old_cell != 0xffffffffu && old_acc != 0.f) {
            n_flush += deposit<kRacy, kCensus>(D, s_win, old_cell, old_slot, old_acc, map32);
          }
          old_cell = acc_cell;
          old_slot = acc_slot;
          old_acc = acc;
          const int slot = cur == wsim ? window_slot(s_wbox, wng, gate, ix, iy, iz) : -1;
          acc_slot = slot;
          acc_cell = cell;
          acc = dep;
        }
        w = w - w * q;

        // move
        const float lh = l * D->inv_h;
        fx = __builtin_amdgcn_fmed3f(fmaf(lh, vx, fx), 0.f, 1.f);
        fy = __builtin_amdgcn_fmed3f(fmaf(lh, vy, fy), 0.f, 1.f);
        fz = __builtin_amdgcn_fmed3f(fmaf(lh, vz, fz), 0.f, 1.f);
        t = fmaf(l, dd.y, t);
        s = ev == kEvScat ? 0.f : fmaxf(fmaf(-md.y, l, s), 0.f);
        if constexpr (kDetect) s_len[m * bdim] += l;

        if constexpr (kVar == kVarFlat) {
          // Every lane that did not time out runs the same instructions:
          // the face-crossing set-up, one Philox block, the scattering
          // direction and the crossing outcome; each keeps the updates of
          // its own event by selection.  Only the label read of the
          // neighbour, the counters of rare events and the bookkeeping of a
          // photon's end stay conditional.
          const bool is_scat = ev == kEvScat, is_cross = ev == kEvCross;
          if (ev == kEvTime) end = kEndTime;
          const float va = ax == 0 ? vx : (ax == 1 ? vy : vz);
          const float vb1 = ax == 0 ? vy : (ax == 1 ? vz : vx);
          const float vb2 = ax == 0 ? vz : (ax == 1 ? vx : vy);
          const int step = va > 0.f ? 1 : -1;
          const int qa = (ax == 0 ? ix : (ax == 1 ? iy : iz)) + step;
          const int na = ax == 0 ? D->nx : (ax == 1 ? D->ny : D->nz);
          const uint32_t stride = ax == 0 ? 1u : (ax == 1 ? D->stride_y : D->stride_z);
          const uint32_t qlin = step > 0 ? lin + stride : lin - stride;
          int m2 = 0;
          if (is_cross && qa >= 0 && qa < na) m2 = as_global(D->labels)[qlin];
          const float n1 = md.w;
          const float n2 = m2 != 0 ? s_med[m2].w : D->n_out;
          const bool fres = is_cross && D->reflect && n2 != n1;
          const float eta = fres ? n1 * rcp(n2) : 1.f;
          const float st2 = eta * eta * (vb1 * vb1 + vb2 * vb2);
          const bool tir = fres && st2 >= 1.f;
          const float cos_t = fsqrt<kNative>(fmaxf(1.f - st2, 0.f));
          const float refl_p = fresnel_r(n1, n2, fabsf(va), cos_t);
          const bool need_rng = is_scat || (fres && !tir);
          const Words r = philox4x32_10(klo, khi, blk, 0u, D->key0, D->key1);
          blk += need_rng ? 1u : 0u;

          // scattering candidate
          float sx = vx, sy = vy, sz = vz;
          const float ct = hg_cos(md.z, s_med[2 * nm + m], unit_open(r.x));
          scatter_dir<kNative>(sx, sy, sz, ct, unit_open(r.y));
          const float s_scat = neg_log<kNative>(unit_open(r.z));
          const bool rr_test = is_scat && w < L.rr_threshold;
          const bool rr_live = rr_test && unit_open(r.w) < L.rr_p;
          if (rr_test) {
            atomicAdd(&s_cnt[wid][kCntRrTests], 1ull);
            if (rr_live) {
              atomicAdd(&s_cnt[wid][kCntRrSurvived], 1ull);
              atomicAdd(&s_led[wid][kLedRrGain], static_cast<double>((L.rr_m - 1.f) * w));
            } else {
              end = kEndRoulette;
            }
          }
          w = rr_live ? w * L.rr_m : w;

          // crossing outcome
          const bool refl = is_cross && (tir || (need_rng && unit_open(r.x) < refl_p));
          const bool enter = is_cross && !refl && m2 != 0;
          if (is_cross && !refl && m2 == 0) end = kEndEscape;
          if (refl) atomicAdd(&s_cnt[wid][kCntReflections], 1ull);
          const bool refr = enter && fres;
          const float vna = static_cast<float>(step) * cos_t;
          const float face = step > 0 ? 1.f : 0.f, entry = step > 0 ? 0.f : 1.f;
          const float fa = enter ? entry : face;
          const float va2 = refl ? -va : (refr ? vna : va);
          const float vb1b = refr ? vb1 * eta : vb1, vb2b = refr ? vb2 * eta : vb2;
          // back to x, y, z: axis ax holds va2, the next ones vb1b, vb2b
          float cx = ax == 0 ? va2 : (ax == 1 ? vb2b : vb1b);
          float cy = ax == 0 ? vb1b : (ax == 1 ? va2 : vb2b);
          float cz = ax == 0 ? vb2b : (ax == 1 ? vb1b : va2);
          if (is_cross) {
            if (ax == 0) fx = fa; else if (ax == 1) fy = fa; else fz = fa;
          }
          const int di = enter ? step : 0;
          ix += ax == 0 ? di : 0;
          iy += ax == 1 ? di : 0;
          iz += ax == 2 ? di : 0;
          lin = enter ? qlin : lin;
          m = enter ? m2 : m;
          // the new direction of each event and its h/|v|
          const bool newdir = is_scat || refr;
          vx = is_scat ? sx : (is_cross ? cx : vx);
          vy = is_scat ? sy : (is_cross ? cy : vy);
          vz = is_scat ? sz : (is_cross ? cz : vz);
          if (newdir) {
            rx = inv_speed(D->h, vx);
            ry = inv_speed(D->h, vy);
            rz = inv_speed(D->h, vz);
          }
          s = is_scat ? s_scat : s;
          nscat += is_scat ? 1u : 0u;
          f_scat = is_scat;
          f_face = is_cross;
          f_fres = is_cross && need_rng;
        } else if (ev == kEvTime) {
          end = kEndTime;
        } else {
          // crossing set-up: neighbour voxel, its medium, Fresnel terms
          bool need_rng = ev == kEvScat;
          bool tir = false, fres = false;
          float va = 0.f, vb1 = 0.f, vb2 = 0.f, eta = 1.f, cos_t = 0.f, refl_p = 0.f;
          int step = 0, m2 = 0;
          uint32_t qlin = 0;
          if (ev == kEvCross) {
            va = ax == 0 ? vx : (ax == 1 ? vy : vz);
            vb1 = ax == 0 ? vy : (ax == 1 ? vz : vx);
            vb2 = ax == 0 ? vz : (ax == 1 ? vx : vy);
            step = va > 0.f ? 1 : -1;
            const int qa = (ax == 0 ? ix : (ax == 1 ? iy : iz)) + step;
            const int na = ax == 0 ? D->nx : (ax == 1 ? D->ny : D->nz);
            const uint32_t stride = ax == 0 ? 1u : (ax == 1 ? D->stride_y : D->stride_z);
            qlin = step > 0 ? lin + stride : lin - stride;
            m2 = (qa >= 0 && qa < na) ? as_global(D->labels)[qlin] : 0;
            const float n1 = md.w;
            const float n2 = m2 != 0 ? s_med[m2].w : D->n_out;
            fres = D->reflect && n2 != n1;
            if (fres) {
              eta = n1 * rcp(n2);
              const float st2 = eta * eta * (vb1 * vb1 + vb2 * vb2);
              if (st2 >= 1.f) {
                tir = true;
              } else {
                cos_t = fsqrt<kNative>(1.f - st2);
                refl_p = fresnel_r(n1, n2, fabsf(va), cos_t);
                need_rng = true;
              }
            }
          }
          Words r = {0u, 0u, 0u, 0u};
          if (need_rng) {
            r = philox4x32_10(klo, khi, blk, 0u, D->key0, D->key1);
            ++blk;
          }

          if (ev == kEvScat) {
            f_scat = true;
            ++nscat;
            const float ct = hg_cos(md.z, s_med[2 * nm + m], unit_open(r.x));
            scatter_dir<kNative>(vx, vy, vz, ct, unit_open(r.y));
            rx = inv_speed(D->h, vx);
            ry = inv_speed(D->h, vy);
            rz = inv_speed(D->h, vz);
            s = neg_log<kNative>(unit_open(r.z));
            if (w < L.rr_threshold) {
              atomicAdd(&s_cnt[wid][kCntRrTests], 1ull);
              if (unit_open(r.w) < L.rr_p) {
                atomicAdd(&s_cnt[wid][kCntRrSurvived], 1ull);
                atomicAdd(&s_led[wid][kLedRrGain], static_cast<double>((L.rr_m - 1.f) * w));
                w *= L.rr_m;
              } else {
                end = kEndRoulette;
              }
            }
          } else {
            // CROSS on axis ax: the photon sits on the face
            f_face = true;
            f_fres = need_rng;
            const float face = step > 0 ? 1.f : 0.f;
            if (ax == 0) fx = face; else if (ax == 1) fy = face; else fz = face;
            const bool reflect = tir || (need_rng && unit_open(r.x) < refl_p);
            if (reflect) {
              atomicAdd(&s_cnt[wid][kCntReflections], 1ull);
              if (ax == 0) vx = -vx; else if (ax == 1) vy = -vy; else vz = -vz;
            } else if (m2 == 0) {
              end = kEndEscape;
            } else {
              if (fres) {
                // refraction: tangential components scale by n1/n2
                const float na_ = static_cast<float>(step) * cos_t;
                if (ax == 0) {
                  vy *= eta; vz *= eta; vx = na_;
                } else if (ax == 1) {
                  vz *= eta; vx *= eta; vy = na_;
                } else {
                  vx *= eta; vy *= eta; vz = na_;
                }
                rx = inv_speed(D->h, vx);
                ry = inv_speed(D->h, vy);
                rz = inv_speed(D->h, vz);
              }
              const float enter = step > 0 ? 0.f : 1.f;
              if (ax == 0) {
                ix += step; fx = enter;
              } else if (ax == 1) {
                iy += step; fy = enter;
              } else {
                iz += step; fz = enter;
              }
              lin = qlin;
              m = m2;
            }
          }
        }
      }

      if (end != kAlive) {
        if (acc != 0.f && acc_cell != 0xffffffffu) {
          n_flush += deposit<kRacy, kCensus>(D, s_win, acc_cell, acc_slot, acc, map32);
        }
        if (old_acc != 0.f && old_cell != 0xffffffffu) {
          n_flush += deposit<kRacy, kCensus>(D, s_win, old_cell, old_slot, old_acc, map32);
        }
        const double wd = static_cast<double>(w);
        const int end_slot = end == kEndEscape ? kCntEscaped
                             : end == kEndTime ? kCntTimeout
                             : end == kEndRoulette ? kCntRrDead : kCntCapped;
        atomicAdd(&s_cnt[wid][end_slot], 1ull);
        if (end == kEndEscape) {
          atomicAdd(&s_led[wid][kLedEscaped], wd);
          if constexpr (kDetect) {
            const float h = D->h;
            const float px = h * (static_cast<float>(ix) + fx);
            const float py = h * (static_cast<float>(iy) + fy);
            const float pz = h * (static_cast<float>(iz) + fz);
            const float4* s_det = s_med + 3 * D->nmedia;
            for (int d = 0; d < D->ndet; ++d) {
              const float4 Dt = s_det[d];
              const float ex = px - Dt.x, ey = py - Dt.y, ez = pz - Dt.z;
              if (ex * ex + ey * ey + ez * ez <= Dt.w) {
                det_hit = d;
                break;
              }
            }
            if (det_hit >= 0) {
              atomicAdd(&s_cnt[wid][kCntDetected], 1ull);
              atomicAdd(&s_led[wid][kLedDetected], wd);
              const unsigned long long slot = atomicAdd(D->det_count, 1ull);
              if (slot < D->det_cap) {
                float* rec = D->det_rec + slot * static_cast<uint64_t>(D->rec_len);
                rec[0] = static_cast<float>(det_hit);
                rec[1] = static_cast<float>(nscat);
                rec[2] = w;
                rec[3] = t;
                for (int mm = 1; mm < D->nmedia; ++mm) rec[3 + mm] = s_len[mm * bdim];
                D->det_photon[slot] = (static_cast<uint64_t>(khi) << 32) | klo;
              }
            }
          }
        } else if (end == kEndTime) {
          atomicAdd(&s_led[wid][kLedTimeout], wd);
        } else if (end == kEndRoulette) {
          atomicAdd(&s_led[wid][kLedRrLoss], wd);
        } else {
          atomicAdd(&s_led[wid][kLedCapped], wd);
        }
        if constexpr (kDiag) {
          const uint64_t k = (static_cast<uint64_t>(khi) << 32) | klo;
          if (k >= D->first && k - D->first < D->ndigest) {
            double* row = D->digest + (k - D->first) * kDigestN;
            row[0] = end;
            row[1] = nscat;
            row[2] = nev;
            row[3] = lin;
            row[4] = w;
            row[5] = t;
            row[6] = blk;
            row[7] = det_hit;
          }
        }
        alive = false;
      }
    }

    c_scat += wave_count(f_scat);
    c_face += wave_count(f_face);
    c_fres += wave_count(f_fres);
    c_flush += wave_count(n_flush >= 1) + wave_count(n_flush >= 2) +
               wave_count(n_flush >= 3);
  }
  flush_wave();

  __syncthreads();
  // add the workgroup's window sums to the map of its window's simulation
  for (int i = threadIdx.x; i < wcount; i += bdim) {
    const uint32_t v = s_win[i];
    if (v != 0u) map_add(as_global(DW->tally) + window_cell(s_wbox, wng, DW, i), v, map32);
  }
}

}  // namespace

size_t transport_smem_bytes(int table_rows, int nmedia_max, int block, bool detect,
                            int window_cells) {
  size_t b = static_cast<size_t>(block / 64) * table_rows * sizeof(float4);
  b += static_cast<size_t>(window_cells) * sizeof(uint32_t);
  if (detect) b += static_cast<size_t>(nmedia_max) * block * sizeof(float);
  return b;
}

template <bool D, bool G, bool N, int V>
static const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&transport_kernel<D, G, N, V>);
}

// The instantiated kernels: every (detect, diag, math) combination of the
// default loop; the ablation loops with hardware math only, the non-atomic
// one also without digests.
static const void* pick(bool detect, bool diag, bool accurate, int variant) {
  if (variant == kVarCensus) {
    if (accurate || diag) return nullptr;
    return detect ? kernel_ptr<true, false, true, kVarCensus>()
                  : kernel_ptr<false, false, true, kVarCensus>();
  }
  if (variant == kVarRacy) {
    if (accurate || diag) return nullptr;
    return detect ? kernel_ptr<true, false, true, kVarRacy>()
                  : kernel_ptr<false, false, true, kVarRacy>();
  }
  if (variant == kVarFlat) {
    if (accurate) return nullptr;
    if (detect)
      return diag ? kernel_ptr<true, true, true, kVarFlat>()
                  : kernel_ptr<true, false, true, kVarFlat>();
    return diag ? kernel_ptr<false, true, true, kVarFlat>()
                : kernel_ptr<false, false, true, kVarFlat>();
  }
  if (variant != kVarDefault) return nullptr;
  if (accurate) {
    if (detect)
      return diag ? kernel_ptr<true, true, false, kVarDefault>()
                  : kernel_ptr<true, false, false, kVarDefault>();
    return diag ? kernel_ptr<false, true, false, kVarDefault>()
                : kernel_ptr<false, false, false, kVarDefault>();
  }
  if (detect)
    return diag ? kernel_ptr<true, true, true, kVarDefault>()
                : kernel_ptr<true, false, true, kVarDefault>();
  return diag ? kernel_ptr<false, true, true, kVarDefault>()
              : kernel_ptr<false, false, true, kVarDefault>();
}

bool transport_variant_available(bool detect, bool diag, bool accurate, int variant) {
  return pick(detect, diag, accurate, variant) != nullptr;
}

hipError_t transport_occupancy(int* blocks_per_cu, int block, size_t smem, bool detect,
                               bool diag, bool accurate, int variant) {
  const void* fn = pick(detect, diag, accurate, variant);
  if (!fn) return hipErrorInvalidDeviceFunction;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, smem);
}

hipError_t launch_transport(const LaunchParams& host, const LaunchParams* dev, int grid,
                            int block, hipStream_t st, bool detect, bool diag, bool accurate,
                            int variant) {
  const int wcells = host.window_cells;
  const size_t smem =
      transport_smem_bytes(host.table_rows, host.nmedia_max, block, detect, wcells);
  const void* fn = pick(detect, diag, accurate, variant);
  if (!fn) return hipErrorInvalidDeviceFunction;
  void* args[] = {const_cast<LaunchParams**>(&dev)};
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, smem, st);
}

}  // namespace mcx
