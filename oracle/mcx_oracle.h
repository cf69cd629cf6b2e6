/*
 * mcx_oracle.h -- plain FP64 CPU oracle of voxel Monte Carlo photon transport.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the
 * smoke check and the benchmark's CPU baseline can check the GPU library
 * against an independent, slow, obviously correct implementation.  No
 * product code may link, load or call it.  It shares no source with the GPU
 * path; the only thing both sides have in common is the written contract
 * (random-number layout, event order, units) that each implements on its own.
 *
 * What it computes: the per-photon simulation loop the paper runs in every
 * GPU thread (problem statement paragraph and Fig. 1 workflow: launch,
 * propagate through a voxelised heterogeneous domain, deposit into 3-D
 * time-resolved fluence maps, record detected photons), with the steps the
 * paper leaves to its earlier CUDA work written out from the physics:
 * exponential free paths, voxel-by-voxel hops, continuous Beer-Lambert
 * absorption, Henyey-Greenstein scattering, unpolarised Fresnel reflection
 * or escape at refractive-index mismatches, Russian roulette and disk
 * detectors with per-medium partial pathlengths.
 *
 * Units: mm, ns, 1/mm.  Grids are x-fastest: index = i + nx*(j + ny*k).
 * Tally layout: [gate][k][j][i].
 */
#ifndef MCX_ORACLE_H
#define MCX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_LEDGER_ABSORBED = 0, /* sum of w - w' over all segments */
  ORC_LEDGER_ESCAPED,      /* weight leaving the medium (incl. detected) */
  ORC_LEDGER_DETECTED,     /* weight leaving through a detector */
  ORC_LEDGER_TIMEOUT,      /* weight alive at the end of the last gate */
  ORC_LEDGER_RR_GAIN,      /* (M-1) w added by roulette survivals */
  ORC_LEDGER_RR_LOSS,      /* w removed by roulette deaths */
  ORC_LEDGER_CAPPED,       /* w of photons stopped by the event cap */
  ORC_LEDGER_LAUNCHED,     /* number of photons launched (weight 1 each) */
  ORC_LEDGER_N
};

enum {
  ORC_CNT_LAUNCHED = 0,
  ORC_CNT_ESCAPED,         /* photons ending by escape (incl. detected) */
  ORC_CNT_DETECTED,
  ORC_CNT_TIMEOUT,
  ORC_CNT_RR_DEAD,
  ORC_CNT_CAPPED,
  ORC_CNT_SCATTERS,
  ORC_CNT_FACE_EVENTS,     /* CROSS events: reflections + entries + escapes */
  ORC_CNT_FRESNEL_DRAWS,   /* Fresnel tests that consumed a random block */
  ORC_CNT_TIR,
  ORC_CNT_REFLECTIONS,     /* incl. total internal reflections */
  ORC_CNT_RR_TESTS,
  ORC_CNT_RR_SURVIVED,
  ORC_CNT_DEPOSITS,        /* segments with a positive deposit */
  ORC_CNT_EVENTS,          /* loop iterations (segments) */
  ORC_CNT_MAX_EVENTS,      /* largest segment count of one photon */
  ORC_CNT_ENTRIES,         /* moves into a neighbouring medium voxel */
  ORC_CNT_N
};

enum { /* per-photon digest row */
  ORC_DG_REASON = 0,       /* 1 escaped, 2 timeout, 3 roulette, 4 capped */
  ORC_DG_NSCAT,
  ORC_DG_EVENTS,
  ORC_DG_VOXEL,            /* last voxel (linear index) */
  ORC_DG_W,                /* final weight */
  ORC_DG_T,                /* final time, ns */
  ORC_DG_BLOCKS,           /* random blocks consumed, launch included */
  ORC_DG_DET,              /* detector index or -1 */
  ORC_DG_N
};

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

typedef struct {
  int32_t nx, ny, nz;
  double h;                 /* voxel edge, mm */
  const uint8_t *labels;    /* nx*ny*nz medium indices, 0 = outside */
  int32_t nmedia;           /* rows in media, row 0 (outside) included */
  const double *media;      /* nmedia x {mua, mus, g, n} */
  double src_pos[3];        /* mm from the grid corner */
  double src_dir[3];        /* unit vector */
  int32_t ndet;
  const double *det;        /* ndet x {x, y, z, radius}, mm */
  double t0, dt;            /* first gate start and gate width, ns */
  int32_t ngates;
  int32_t reflect;          /* nonzero: Fresnel reflection at index changes */
  double n_out;             /* refractive index of label 0 and off-grid */
  double rr_threshold;      /* roulette is tested when w < this */
  double rr_m;              /* survive with probability 1/M, then w *= M */
  uint64_t max_events;      /* per-photon segment cap (0 = no cap) */
} orc_problem;

typedef struct {
  double *tally;            /* ngates*nvox, accumulated (+=), required */
  int64_t *deposits;        /* ngates*nvox, accumulated, may be NULL */
  double ledger[ORC_LEDGER_N];   /* overwritten */
  int64_t counts[ORC_CNT_N];     /* overwritten */
  float *det_rec;           /* det_cap rows of (4 + nmedia - 1) floats, may be NULL */
  uint64_t *det_photon;     /* det_cap photon indices, may be NULL */
  uint64_t det_cap;
  uint64_t det_total;       /* out: photons detected */
  uint64_t det_written;     /* out: rows written (<= det_cap) */
  double *digest;           /* ndigest rows of ORC_DG_N, photons first.., may be NULL */
  uint64_t ndigest;
  int64_t *visits;          /* ngates*nvox, accumulated, may be NULL: per cell, the photon
                               visits (maximal runs of one photon's consecutive deposits
                               into that cell) */
} orc_output;

/* Simulate photons [first, first + n) with run seed `seed` on `nthreads`
 * threads.  Results do not depend on nthreads except for FP64 summation
 * order.  Returns ORC_OK, ORC_EINVAL or ORC_ENOMEM. */
int orc_run(const orc_problem *p, uint64_t first, uint64_t n, uint64_t seed,
            int nthreads, orc_output *out);

/* Pieces exposed so that tests can pin them against closed forms. */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t word);
double orc_hg_cos(double g, double u);
void   orc_scatter_dir(const double v[3], double cos_theta, double u_phi, double out[3]);
double orc_fresnel(double n1, double n2, double cos_i);
int    orc_validate(const orc_problem *p);

#ifdef __cplusplus
}
#endif
#endif
