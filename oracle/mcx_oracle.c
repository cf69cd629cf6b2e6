/*
 * mcx_oracle.c -- plain FP64 CPU oracle of voxel Monte Carlo photon transport.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  Scalar C99,
 * double precision, glibc libm, no fast-math, no blocking or reordering of
 * the per-photon steps.  Threads only split the photon index range; their
 * private tallies are summed in thread order.
 *
 * The paper describes its simulation as a per-thread photon loop (problem
 * statement paragraph and Fig. 1) and defers the loop body to the authors'
 * earlier CUDA paper.  The body below is the standard voxel-based,
 * continuous-absorption Monte Carlo of that line of work, with every open
 * choice frozen as follows (the same choices the GPU path implements on its
 * own):
 *
 *  Random numbers (the paper: independent seeds per thread).  Counter-based
 *  Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).  For photon k and
 *  run seed S: key = (S mod 2^32, S div 2^32), counter = (k mod 2^32,
 *  k div 2^32, b, 0).  Block b = 0 is the launch; every later random event
 *  (a scattering, a Fresnel test) takes the next b.  A 32-bit word x becomes
 *  u = ((x >> 8) | 1) * 2^-24, an odd multiple of 2^-24 in (0,1), exact in
 *  both float and double.
 *
 *  Launch.  The photon starts at the source point (voxel = floor(p/h),
 *  local offset f = p/h - voxel in [0,1]^3), with the source direction,
 *  weight 1, time t0 and a dimensionless free path s = -ln u0 (block 0,
 *  word 0).  No specular loss at entry.
 *
 *  Segment.  With the medium (mua, mus, g, n) of the current voxel:
 *  d_s = s/mus (infinite if mus = 0); d_a = h*(v_a > 0 ? 1-f_a : f_a)/|v_a|
 *  per axis with v_a != 0, d_v = min (lowest axis on ties);
 *  d_t = (t_end - t)*c/n with t_end = t0 + ngates*dt.  The event is TIME if
 *  d_t < min(d_s, d_v), else SCATTER if d_s <= d_v, else CROSS; l is its
 *  distance.  The segment deposits A = w*(1 - exp(-mua l))/mua (w*l if
 *  mua = 0) into gate min(floor((t-t0)/dt), ngates-1) of the current voxel,
 *  w becomes w*exp(-mua l), f += l v/h, t += l n/c, the partial pathlength
 *  of the medium grows by l, and s becomes 0 (SCATTER) or s - mus*l.
 *
 *  TIME: the remaining weight is booked as timed out; the photon ends.
 *
 *  SCATTER: next block; word 0 -> cos(theta) by inverting the
 *  Henyey-Greenstein distribution, word 1 -> azimuth 2*pi*u about the old
 *  direction using the orthonormal basis of Duff et al. (JCGT 2017), then
 *  renormalise; word 2 -> new s = -ln u.  If w < rr_threshold, word 3 plays
 *  Russian roulette: survive if u < 1/M (w *= M), else the photon ends.
 *
 *  CROSS on axis a: the photon sits on the face; the neighbour's medium is
 *  its label, or 0 off the grid.  With reflection on and a different
 *  refractive index: total internal reflection when sin^2(t) >= 1 (no
 *  draw), else the unpolarised Fresnel coefficient R and the next block's
 *  word 0 decide reflect (u < R) or transmit.  Reflection flips v_a and
 *  keeps the voxel; transmission into medium 0 is escape; transmission into
 *  tissue refracts (tangential components times n/n', normal component the
 *  transmitted cosine) and enters the neighbour.  Without reflection or with
 *  equal indices the photon enters unchanged or escapes.  At escape, the
 *  first detector (index order) whose centre lies within its radius of the
 *  exit point records {det, nscat, w, t, L[1..M]}.
 *
 *  Speed of light c = 299.792458 mm/ns.
 */
#define _GNU_SOURCE
#include "mcx_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define C_MM_PER_NS 299.792458

/* ---------------------------------------------------------------- Philox */

/* Philox4x32-10 as published: each round multiplies counter words 0 and 2
 * by the two round constants, forms the 64-bit products, and rebuilds the
 * counter from the high halves xored with the other words and the key, and
 * the low halves; the key is bumped by the two Weyl constants between
 * rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_uniform(uint32_t word) {
  return (double)((word >> 8) | 1u) * (1.0 / 16777216.0);
}

static void photon_block(uint64_t k, uint32_t b, const uint32_t key[2], double u[4]) {
  uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), b, 0u};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  for (int i = 0; i < 4; i++) u[i] = orc_uniform(out[i]);
}

/* ------------------------------------------------------------- physics */

/* Inverse CDF of the Henyey-Greenstein phase function,
 * cos = (1 + g^2 - ((1 - g^2)/(1 - g + 2 g u))^2) / (2 g),
 * multiplied out over the common denominator so that g = 0 needs no special
 * case: cos = (2u(1+g^2)(1-g+gu) - (1-g)^2) / (1-g+2gu)^2. */
double orc_hg_cos(double g, double u) {
  double a = 1.0 - g + 2.0 * g * u;
  double c = (2.0 * u * (1.0 + g * g) * (1.0 - g + g * u) - (1.0 - g) * (1.0 - g)) / (a * a);
  if (c > 1.0) c = 1.0;
  if (c < -1.0) c = -1.0;
  return c;
}

/* New direction at polar cosine cos_theta and azimuth 2*pi*u_phi about v.
 * The azimuth is measured in the basis (t1, t2) of Duff et al., "Building
 * an Orthonormal Basis, Revisited", JCGT 6(1), 2017. */
void orc_scatter_dir(const double v[3], double cos_theta, double u_phi, double out[3]) {
  double st = sqrt((1.0 - cos_theta) * (1.0 + cos_theta));
  double phi = 2.0 * M_PI * u_phi;
  double cp = cos(phi), sp = sin(phi);
  double sg = copysign(1.0, v[2]);
  double a = -1.0 / (sg + v[2]);
  double b = v[0] * v[1] * a;
  double t1[3] = {1.0 + sg * v[0] * v[0] * a, sg * b, -sg * v[0]};
  double t2[3] = {b, sg + v[1] * v[1] * a, -v[1]};
  double nv[3];
  for (int i = 0; i < 3; i++)
    nv[i] = cos_theta * v[i] + st * (cp * t1[i] + sp * t2[i]);
  double norm = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  for (int i = 0; i < 3; i++) out[i] = nv[i] / norm;
}

/* Unpolarised Fresnel reflectance for incidence cosine cos_i and
 * transmitted cosine cos_t from n1 into n2 (mean of the s and p terms). */
static double fresnel_r(double n1, double n2, double ci, double ct) {
  double rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct);
  double rp = (n1 * ct - n2 * ci) / (n1 * ct + n2 * ci);
  return 0.5 * (rs * rs + rp * rp);
}

double orc_fresnel(double n1, double n2, double cos_i) {
  double st2 = (n1 / n2) * (n1 / n2) * (1.0 - cos_i * cos_i);
  if (st2 >= 1.0) return 1.0;
  return fresnel_r(n1, n2, cos_i, sqrt(1.0 - st2));
}

/* ------------------------------------------------------------- problem */

typedef struct {
  int64_t nvox;
  int64_t src_vox[3];
  double src_f[3];
  double t_end;
  int rec_len;
} derived_t;

int orc_validate(const orc_problem *p) {
  if (!p || p->nx <= 0 || p->ny <= 0 || p->nz <= 0 || !(p->h > 0)) return ORC_EINVAL;
  if (!p->labels || !p->media || p->nmedia < 2 || p->nmedia > 256) return ORC_EINVAL;
  if (p->ngates <= 0 || !(p->dt > 0) || !isfinite(p->t0)) return ORC_EINVAL;
  if (p->ndet < 0 || (p->ndet > 0 && !p->det)) return ORC_EINVAL;
  if (!(p->n_out >= 1.0) || !(p->rr_m > 1.0) || !(p->rr_threshold >= 0)) return ORC_EINVAL;
  for (int m = 1; m < p->nmedia; m++) {
    const double *md = p->media + 4 * m;
    if (!(md[0] >= 0) || !(md[1] >= 0) || !(md[2] >= -1 && md[2] <= 1) || !(md[3] >= 1) ||
        !isfinite(md[0]) || !isfinite(md[1]))
      return ORC_EINVAL;
  }
  int64_t nvox = (int64_t)p->nx * p->ny * p->nz;
  for (int64_t i = 0; i < nvox; i++)
    if (p->labels[i] >= p->nmedia) return ORC_EINVAL;
  double dn = sqrt(p->src_dir[0] * p->src_dir[0] + p->src_dir[1] * p->src_dir[1] +
                   p->src_dir[2] * p->src_dir[2]);
  if (!(fabs(dn - 1.0) <= 1e-5)) return ORC_EINVAL;
  int32_t dim[3] = {p->nx, p->ny, p->nz};
  int64_t iv[3];
  for (int a = 0; a < 3; a++) {
    double x = p->src_pos[a] / p->h;
    if (!(x >= 0) || !(x < dim[a])) return ORC_EINVAL;
    iv[a] = (int64_t)floor(x);
  }
  if (p->labels[iv[0] + p->nx * (iv[1] + (int64_t)p->ny * iv[2])] == 0) return ORC_EINVAL;
  for (int d = 0; d < p->ndet; d++)
    if (!(p->det[4 * d + 3] > 0)) return ORC_EINVAL;
  return ORC_OK;
}

static void derive(const orc_problem *p, derived_t *dp) {
  dp->nvox = (int64_t)p->nx * p->ny * p->nz;
  for (int a = 0; a < 3; a++) {
    double x = p->src_pos[a] / p->h;
    double fl = floor(x);
    dp->src_vox[a] = (int64_t)fl;
    dp->src_f[a] = x - fl;
  }
  dp->t_end = p->t0 + p->ngates * p->dt;
  dp->rec_len = 4 + (p->nmedia - 1);
}

/* ---------------------------------------------------------- per thread */

typedef struct {
  const orc_problem *p;
  const derived_t *dp;
  uint64_t first, n, seed;
  double *tally;
  int64_t *deposits;
  int64_t *visits;     /* may be NULL */
  double ledger[ORC_LEDGER_N];
  int64_t counts[ORC_CNT_N];
  float *rec;          /* growable */
  uint64_t *rec_photon;
  uint64_t nrec, rec_capacity;
  double *digest;      /* rows for photons [digest_first, digest_first+ndigest) */
  uint64_t digest_first, ndigest;
  int failed;
} worker_t;

enum { EV_TIME = 0, EV_SCAT = 1, EV_CROSS = 2 };
enum { END_ESCAPE = 1, END_TIMEOUT = 2, END_ROULETTE = 3, END_CAPPED = 4 };

static int push_record(worker_t *wk, uint64_t k, const float *row) {
  int rl = wk->dp->rec_len;
  if (wk->nrec == wk->rec_capacity) {
    uint64_t cap = wk->rec_capacity ? 2 * wk->rec_capacity : 1024;
    float *r = realloc(wk->rec, cap * rl * sizeof(float));
    if (!r) return -1;
    wk->rec = r;
    uint64_t *q = realloc(wk->rec_photon, cap * sizeof(uint64_t));
    if (!q) return -1;
    wk->rec_photon = q;
    wk->rec_capacity = cap;
  }
  memcpy(wk->rec + wk->nrec * rl, row, rl * sizeof(float));
  wk->rec_photon[wk->nrec] = k;
  wk->nrec++;
  return 0;
}

static void simulate_photon(worker_t *wk, uint64_t k, const uint32_t key[2], double *L) {
  const orc_problem *p = wk->p;
  const derived_t *dp = wk->dp;
  const double h = p->h;
  const int64_t dim[3] = {p->nx, p->ny, p->nz};
  double u[4];

  /* launch */
  photon_block(k, 0, key, u);
  uint32_t b = 1;
  double s = -log(u[0]);
  int64_t vox[3] = {dp->src_vox[0], dp->src_vox[1], dp->src_vox[2]};
  double f[3] = {dp->src_f[0], dp->src_f[1], dp->src_f[2]};
  double v[3] = {p->src_dir[0], p->src_dir[1], p->src_dir[2]};
  double w = 1.0, t = p->t0;
  int64_t nscat = 0, events = 0;
  int64_t last_cell = -1; /* cell of the photon's previous deposit (visit count) */
  int reason = 0, det_hit = -1;
  for (int m = 0; m < p->nmedia; m++) L[m] = 0.0;
  wk->counts[ORC_CNT_LAUNCHED]++;
  wk->ledger[ORC_LEDGER_LAUNCHED] += 1.0;

  for (;;) {
    if (p->max_events && (uint64_t)events >= p->max_events) {
      wk->ledger[ORC_LEDGER_CAPPED] += w;
      wk->counts[ORC_CNT_CAPPED]++;
      reason = END_CAPPED;
      break;
    }
    events++;
    int64_t lin = vox[0] + dim[0] * (vox[1] + dim[1] * vox[2]);
    int m = p->labels[lin];
    const double mua = p->media[4 * m + 0], mus = p->media[4 * m + 1];
    const double g = p->media[4 * m + 2], n = p->media[4 * m + 3];

    /* distances to the three possible events */
    double ds = mus > 0 ? s / mus : INFINITY;
    double dv = INFINITY;
    int ax = -1;
    for (int a = 0; a < 3; a++) {
      if (v[a] == 0.0) continue;
      double face = v[a] > 0 ? 1.0 - f[a] : f[a];
      if (face < 0) face = 0;
      double d = h * face / fabs(v[a]);
      if (d < dv) {
        dv = d;
        ax = a;
      }
    }
    double dtime = (dp->t_end - t) * C_MM_PER_NS / n;
    if (dtime < 0) dtime = 0;
    int ev;
    double l;
    if (dtime < fmin(ds, dv)) {
      ev = EV_TIME;
      l = dtime;
    } else if (ds <= dv) {
      ev = EV_SCAT;
      l = ds;
    } else {
      ev = EV_CROSS;
      l = dv;
    }

    /* absorption along the segment, booked at the segment-start gate */
    int64_t gate = (int64_t)floor((t - p->t0) / p->dt);
    if (gate >= p->ngates) gate = p->ngates - 1;
    if (gate < 0) gate = 0;
    double wn = w * exp(-mua * l);
    double dep = mua > 0 ? w * (-expm1(-mua * l)) / mua : w * l;
    wk->tally[gate * dp->nvox + lin] += dep;
    if (dep > 0) {
      const int64_t cell = gate * dp->nvox + lin;
      wk->counts[ORC_CNT_DEPOSITS]++;
      if (wk->deposits) wk->deposits[cell]++;
      if (wk->visits && cell != last_cell) wk->visits[cell]++;
      last_cell = cell;
    }
    wk->ledger[ORC_LEDGER_ABSORBED] += w - wn;
    w = wn;

    /* move */
    for (int a = 0; a < 3; a++) {
      f[a] += l * v[a] / h;
      if (f[a] < 0) f[a] = 0;
      if (f[a] > 1) f[a] = 1;
    }
    t += l * n / C_MM_PER_NS;
    L[m] += l;
    if (ev == EV_SCAT) {
      s = 0;
    } else {
      s -= mus * l;
      if (s < 0) s = 0;
    }

    if (ev == EV_TIME) {
      wk->ledger[ORC_LEDGER_TIMEOUT] += w;
      wk->counts[ORC_CNT_TIMEOUT]++;
      reason = END_TIMEOUT;
      break;
    }

    if (ev == EV_SCAT) {
      nscat++;
      wk->counts[ORC_CNT_SCATTERS]++;
      photon_block(k, b++, key, u);
      double ct = orc_hg_cos(g, u[0]);
      double nv[3];
      orc_scatter_dir(v, ct, u[1], nv);
      v[0] = nv[0]; v[1] = nv[1]; v[2] = nv[2];
      s = -log(u[2]);
      if (w < p->rr_threshold) {
        wk->counts[ORC_CNT_RR_TESTS]++;
        if (u[3] < 1.0 / p->rr_m) {
          wk->counts[ORC_CNT_RR_SURVIVED]++;
          wk->ledger[ORC_LEDGER_RR_GAIN] += (p->rr_m - 1.0) * w;
          w *= p->rr_m;
        } else {
          wk->ledger[ORC_LEDGER_RR_LOSS] += w;
          wk->counts[ORC_CNT_RR_DEAD]++;
          reason = END_ROULETTE;
          break;
        }
      }
      continue;
    }

    /* CROSS on axis ax */
    wk->counts[ORC_CNT_FACE_EVENTS]++;
    const int a = ax;
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    const int sg = v[a] > 0 ? 1 : -1;
    f[a] = sg > 0 ? 1.0 : 0.0;
    int64_t q[3] = {vox[0], vox[1], vox[2]};
    q[a] += sg;
    int m2 = 0;
    if (q[a] >= 0 && q[a] < dim[a]) m2 = p->labels[q[0] + dim[0] * (q[1] + dim[1] * q[2])];
    const double n2 = m2 ? p->media[4 * m2 + 3] : p->n_out;
    int reflect = 0, refract = 0;
    double cos_t = 0.0, eta = 1.0;
    if (p->reflect && n2 != n) {
      double ci = fabs(v[a]);
      eta = n / n2;
      double st2 = eta * eta * (v[b1] * v[b1] + v[b2] * v[b2]);
      if (st2 >= 1.0) {
        reflect = 1;
        wk->counts[ORC_CNT_TIR]++;
      } else {
        cos_t = sqrt(1.0 - st2);
        double R = fresnel_r(n, n2, ci, cos_t);
        photon_block(k, b++, key, u);
        wk->counts[ORC_CNT_FRESNEL_DRAWS]++;
        if (u[0] < R)
          reflect = 1;
        else
          refract = 1;
      }
    }
    if (reflect) {
      v[a] = -v[a];
      wk->counts[ORC_CNT_REFLECTIONS]++;
      continue;
    }
    if (m2 == 0) {
      /* escape through the face; check the detectors at the exit point */
      double pos[3];
      for (int i = 0; i < 3; i++) pos[i] = h * ((double)vox[i] + f[i]);
      for (int d = 0; d < p->ndet; d++) {
        const double *dd = p->det + 4 * d;
        double dx = pos[0] - dd[0], dy = pos[1] - dd[1], dz = pos[2] - dd[2];
        if (dx * dx + dy * dy + dz * dz <= dd[3] * dd[3]) {
          det_hit = d;
          break;
        }
      }
      wk->ledger[ORC_LEDGER_ESCAPED] += w;
      wk->counts[ORC_CNT_ESCAPED]++;
      if (det_hit >= 0) {
        wk->ledger[ORC_LEDGER_DETECTED] += w;
        wk->counts[ORC_CNT_DETECTED]++;
        float row[4 + 256];
        row[0] = (float)det_hit;
        row[1] = (float)nscat;
        row[2] = (float)w;
        row[3] = (float)t;
        for (int mm = 1; mm < p->nmedia; mm++) row[3 + mm] = (float)L[mm];
        if (push_record(wk, k, row)) wk->failed = 1;
      }
      reason = END_ESCAPE;
      break;
    }
    if (refract) {
      v[b1] *= eta;
      v[b2] *= eta;
      v[a] = sg * cos_t;
    }
    vox[0] = q[0]; vox[1] = q[1]; vox[2] = q[2];
    f[a] = sg > 0 ? 0.0 : 1.0;
    wk->counts[ORC_CNT_ENTRIES]++;
  }

  wk->counts[ORC_CNT_EVENTS] += events;
  if (events > wk->counts[ORC_CNT_MAX_EVENTS]) wk->counts[ORC_CNT_MAX_EVENTS] = events;
  if (wk->digest && k >= wk->digest_first && k - wk->digest_first < wk->ndigest) {
    double *row = wk->digest + (k - wk->digest_first) * ORC_DG_N;
    row[ORC_DG_REASON] = reason;
    row[ORC_DG_NSCAT] = (double)nscat;
    row[ORC_DG_EVENTS] = (double)events;
    row[ORC_DG_VOXEL] = (double)(vox[0] + dim[0] * (vox[1] + dim[1] * vox[2]));
    row[ORC_DG_W] = w;
    row[ORC_DG_T] = t;
    row[ORC_DG_BLOCKS] = (double)b;
    row[ORC_DG_DET] = det_hit;
  }
}

static void *worker_main(void *arg) {
  worker_t *wk = (worker_t *)arg;
  uint32_t key[2] = {(uint32_t)wk->seed, (uint32_t)(wk->seed >> 32)};
  double L[256];
  for (uint64_t i = 0; i < wk->n && !wk->failed; i++) simulate_photon(wk, wk->first + i, key, L);
  return NULL;
}

int orc_run(const orc_problem *p, uint64_t first, uint64_t n, uint64_t seed, int nthreads,
            orc_output *out) {
  int rc = orc_validate(p);
  if (rc) return rc;
  if (!out || !out->tally) return ORC_EINVAL;
  derived_t dp;
  derive(p, &dp);
  if (nthreads < 1) nthreads = 1;
  if ((uint64_t)nthreads > n) nthreads = n > 0 ? (int)n : 1;
  const uint64_t cells = (uint64_t)p->ngates * dp.nvox;

  worker_t *wk = calloc(nthreads, sizeof(worker_t));
  pthread_t *th = calloc(nthreads, sizeof(pthread_t));
  if (!wk || !th) {
    free(wk);
    free(th);
    return ORC_ENOMEM;
  }
  uint64_t base = n / nthreads, extra = n % nthreads, start = first;
  for (int i = 0; i < nthreads; i++) {
    wk[i].p = p;
    wk[i].dp = &dp;
    wk[i].seed = seed;
    wk[i].first = start;
    wk[i].n = base + ((uint64_t)i < extra ? 1 : 0);
    start += wk[i].n;
    wk[i].digest = out->digest;
    wk[i].digest_first = first;
    wk[i].ndigest = out->digest ? out->ndigest : 0;
    if (nthreads == 1) {
      wk[i].tally = out->tally;
      wk[i].deposits = out->deposits;
      wk[i].visits = out->visits;
    } else {
      wk[i].tally = calloc(cells, sizeof(double));
      wk[i].deposits = out->deposits ? calloc(cells, sizeof(int64_t)) : NULL;
      wk[i].visits = out->visits ? calloc(cells, sizeof(int64_t)) : NULL;
      if (!wk[i].tally || (out->deposits && !wk[i].deposits) || (out->visits && !wk[i].visits))
        rc = ORC_ENOMEM;
    }
  }
  if (rc == ORC_OK) {
    for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, worker_main, &wk[i]);
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
  }

  memset(out->ledger, 0, sizeof(out->ledger));
  memset(out->counts, 0, sizeof(out->counts));
  out->det_total = 0;
  out->det_written = 0;
  for (int i = 0; i < nthreads && rc == ORC_OK; i++) {
    if (wk[i].failed) rc = ORC_ENOMEM;
    if (nthreads > 1) {
      for (uint64_t c = 0; c < cells; c++) out->tally[c] += wk[i].tally[c];
      if (out->deposits)
        for (uint64_t c = 0; c < cells; c++) out->deposits[c] += wk[i].deposits[c];
      if (out->visits)
        for (uint64_t c = 0; c < cells; c++) out->visits[c] += wk[i].visits[c];
    }
    for (int j = 0; j < ORC_LEDGER_N; j++) out->ledger[j] += wk[i].ledger[j];
    for (int j = 0; j < ORC_CNT_N; j++) {
      if (j == ORC_CNT_MAX_EVENTS) {
        if (wk[i].counts[j] > out->counts[j]) out->counts[j] = wk[i].counts[j];
      } else {
        out->counts[j] += wk[i].counts[j];
      }
    }
    for (uint64_t r = 0; r < wk[i].nrec; r++) {
      if (out->det_written < out->det_cap) {
        if (out->det_rec)
          memcpy(out->det_rec + out->det_written * dp.rec_len, wk[i].rec + r * dp.rec_len,
                 dp.rec_len * sizeof(float));
        if (out->det_photon) out->det_photon[out->det_written] = wk[i].rec_photon[r];
        out->det_written++;
      }
      out->det_total++;
    }
  }
  for (int i = 0; i < nthreads; i++) {
    if (nthreads > 1) {
      free(wk[i].tally);
      free(wk[i].deposits);
      free(wk[i].visits);
    }
    free(wk[i].rec);
    free(wk[i].rec_photon);
  }
  free(wk);
  free(th);
  return rc;
}
