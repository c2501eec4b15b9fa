/*
 * Oracle for the particle-in-cell joint velocity-scalar PDF step.
 *
 * TEST INFRASTRUCTURE ONLY.  A plain, slow CPU implementation of what the
 * particle step computes, used by the tests, the smoke check and the CPU
 * baseline of the benchmark to check the GPU library.  The product path never
 * links, loads or calls it.  It shares no code with the GPU library; the two
 * agree only on the documented array layouts and on the definition of the
 * random numbers (Philox4x32-10 counters, Box-Muller with series log/sincos).
 *
 * State precision: the particle state is held in double ("f64") or in float
 * ("f32").  In f32 mode every state update is carried out in float, so that
 * the oracle follows the same rounding as an f32 implementation; geometric
 * predicates and all statistics are double in both modes.
 *
 * Paper: Bakosi, Franzese & Boybeyi, "Joint PDF modelling of turbulent flow
 * and dispersion in an urban street canyon" -- section 2 with sections 2.1-2.2, eqs. (5)-(13),
 * (19)-(26), section 3.
 */
#ifndef PDF_ORACLE_H
#define PDF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* edge kinds (same numbering as the mesh arrays) */
enum {
  ORC_EDGE_INTERIOR = 0, ORC_EDGE_NOSLIP = 1, ORC_EDGE_SLIP = 2, ORC_EDGE_WALLFN = 3,
  ORC_EDGE_PXP = 4, ORC_EDGE_PXM = 5, ORC_EDGE_PYP = 6, ORC_EDGE_PYM = 7
};

/* per-element statistics record, doubles, in this order */
enum {
  ORC_ST_N = 0,        /* particle count                                   */
  ORC_ST_MEAN = 1,     /* 4: <u>, <v>, <w>, <psi>                          */
  ORC_ST_M2 = 5,       /* 10: central 2nd moments, pairs a<=b of (u,v,w,psi) */
  ORC_ST_BINN = 15,    /* 8: particles per velocity bin                     */
  ORC_ST_BINM = 23,    /* 8: <phi|V> per bin (element mean if empty)        */
  ORC_ST_M3 = 31,      /* 20: central 3rd moments (moments >= 4 only)       */
  ORC_ST_M4 = 51,      /* 35: central 4th moments                           */
  ORC_ST_HIST = 86,    /* hist_bins: scalar histogram counts                */
  ORC_NSTAT_2 = 31,
  ORC_NSTAT_4 = 86
};

/* time-averaged record per element, doubles, in this order; with the
   turbulent frequency two more after the histogram: pooled <omega> and
   <omega'^2> */
enum {
  ORC_AV_STEPS = 0,    /* steps averaged                                    */
  ORC_AV_N = 1,        /* pooled particle count (sum over the steps)        */
  ORC_AV_MEAN = 2,     /* 4: pooled means of u, v, w, psi                   */
  ORC_AV_M2 = 6,       /* 10: pooled central 2nd moments                    */
  ORC_AV_HIST = 16     /* hist_bins: summed scalar histogram counts         */
};

typedef struct orc_params {
  int32_t f32_state;   /* 1: float particle state, 0: double */
  int32_t model;       /* 0 SLM (eq. 19), 1 GLM from wp (eqs. 12-13) */
  int32_t moments;     /* 2 or 4 */
  int32_t hist_bins;   /* 0 or 32 */
  int32_t mix;         /* IECM on */
  int32_t psi_init;    /* 0 zero, 1 psi=1 for x<0.25 */
  int32_t flags;       /* sub-steps: 1 velocity, 2 position and tracking, 4 IECM, 8 source */
  int32_t omega;       /* 1: stochastic turbulent frequency per particle, eqs. (9)-(10), (27)-(28) */
  int32_t vbins;       /* velocity bins per component for <phi|V> in IECM: 2 (signs) or 5 */
  int32_t pad_;
  double dt, nu, C0;   /* time step, viscosity, SLM constant */
  double CT, Cs, Ct;   /* Table 2 */
  double Cmu, kappa, Ewall, yp;  /* wall functions */
  double Lx, Ly;       /* periodic lengths */
  double C3, C4, Cw1, Cw2;  /* Table 2: turbulent frequency model */
} orc_params;

typedef struct orc_ctx orc_ctx;

/* Create from host arrays (copied).  fields: nvert x 20 doubles. */
orc_ctx* orc_create(const orc_params* p, int32_t nvert, const double* vtx, int32_t nelem,
                    const int32_t* tri, const int32_t* nbr, const int32_t* ekind,
                    const double* fields);
void orc_destroy(orc_ctx* c);
/* Add and seed one ensemble.  counts: nelem particles per element. Returns ensemble index. */
int32_t orc_add_ensemble(orc_ctx* c, const int64_t* counts, uint64_t seed, double x0, double y0,
                         double r0);
int32_t orc_nstat(const orc_ctx* c);
int64_t orc_count(const orc_ctx* c, int32_t ens);
/* Advance every ensemble by nsteps. Returns 0, or -5 when a particle is lost. */
int32_t orc_step(orc_ctx* c, int32_t nsteps);
/* Statistics of the current state of one ensemble: nelem x nstat doubles. */
int32_t orc_stats(orc_ctx* c, int32_t ens, double* out);
/* State of one ensemble in particle-id order. */
int32_t orc_get_state(const orc_ctx* c, int32_t ens, double* x, double* y, double* u, double* v,
                      double* w, double* psi, int32_t* elem);
/* Replace the state of one ensemble (values are rounded to the state type). */
int32_t orc_set_state(orc_ctx* c, int32_t ens, const double* x, const double* y, const double* u,
                      const double* v, const double* w, const double* psi, const int32_t* elem);
/* The series exponential the wall condition on the turbulent frequency uses
   (range reduction by ln 2, Taylor series through r^13). */
double orc_exp64(double x);
/* Turbulent frequency per particle of one ensemble, in id order; -1 when the
   context carries none (omega = 0). */
int32_t orc_get_omega(const orc_ctx* c, int32_t ens, double* om);
int32_t orc_set_omega(orc_ctx* c, int32_t ens, const double* om);
/* Per element: frozen <omega> at the centroid (eq. 8 solved) and S_omega
   (eq. 10); per element edge: frozen <omega> at a wall-function edge's
   midpoint (0 elsewhere). */
void orc_omega_fields(const orc_ctx* c, double* om0, double* somega, double* omw);
/* Time averaging: from orc_average_start on, every step's statistics record
   (of the state at the start of the step) joins the average; orc_average
   writes the time-averaged records of one ensemble (nelem x orc_navg). */
int32_t orc_navg(const orc_ctx* c);
void orc_average_start(orc_ctx* c);
void orc_average_stop(orc_ctx* c);
int32_t orc_average(const orc_ctx* c, int32_t ens, double* out);
/* Lowest-index element whose closed triangle contains (x, y), or -1. */
int32_t orc_locate(const orc_ctx* c, double x, double y);
/* Particle steps so far in which a wall-function reflection changed omega. */
int64_t orc_wallfn_hits(const orc_ctx* c);

/* Conditional means <phi|V> used by the IECM step in place of the binned
   estimate of the state (nelem x 8, by velocity bin), until cleared with
   cm = NULL: lets a test feed the step the values another estimator (the
   learned one) produced. */
void orc_set_cond_means(orc_ctx* c, int32_t ens, const double* cm);
int64_t orc_get_step(const orc_ctx* c);
void orc_set_step(orc_ctx* c, int64_t step);
void orc_set_threads(int32_t n);

/* -------- unit-level entry points used by the pins -------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* the 8 normals of one particle step (f32: float arithmetic) */
void orc_normals(uint64_t seed, uint32_t id, uint32_t step, uint32_t ens, int32_t f32, double out[8]);
/* normals of particles 0..n-1: n x 8 */
void orc_normals_batch(uint64_t seed, int64_t n, uint32_t step, uint32_t ens, int32_t f32,
                       double* out);
double orc_log64(double x);
float orc_log32(float x);
void orc_sincos2pi64(double t, double* s, double* c);
void orc_sincos2pi32(float t, float* s, float* c);
double orc_cbrt64(double x);
/* per-vertex coefficient table: nvert x 16 (U V dUdx dUdy dVdx dVdy lapU lapV dPdx dPdy
   G11 G12 G21 G22 G33 C0eps), rounded to the state type */
void orc_coefficients(const orc_ctx* c, double* out);
/* replace G11 G12 G21 G22 G33 C0eps of every vertex (g6: nvert x 6), e.g.
   with the result of the elliptic relaxation, eqs. (12)-(13) */
void orc_set_drift(orc_ctx* c, const double* g6);
/* replace the mean pressure gradient of every vertex (g2: nvert x 2), e.g.
   after a mean-pressure projection */
void orc_set_pressure_gradient(orc_ctx* c, const double* g2);
/* IECM relaxation factor r = min(dt/t_m, 1) per element of one ensemble */
void orc_mix_rate(const orc_ctx* c, int32_t ens, double* out);
/* wall-function alpha per element edge (0 elsewhere): nelem x 3 */
void orc_wall_alpha(const orc_ctx* c, double* out);
/* One straight-line walk from a point in element e to a target, with boundary
   handling.  (sx,sy): start, (tx,ty): target (rounded to the state type);
   vel: 3 velocity components (in/out); om: turbulent frequency (in/out, may
   be NULL: no frequency condition).  Returns the final element, or -1. */
int32_t orc_walk(const orc_ctx* c, int32_t e, double sx, double sy, double* tx, double* ty,
                 double* vel, int32_t* n_reflect, double* om);

#ifdef __cplusplus
}
#endif
#endif
