/*
 * pdfpic -- particle-in-cell Monte Carlo step for the joint PDF of velocity
 * and a passive scalar, for AMD Instinct MI355X (gfx950).
 *
 * Method: Bakosi, Franzese & Boybeyi, "Joint PDF modelling of turbulent flow
 * and dispersion in an urban street canyon".  Particles carry position,
 * velocity and scalar; one step advances them by the explicit Euler-Maruyama
 * scheme (closing summary of section 2.2) of
 *   eq. (5)  position: dX = U dt + (2 nu)^(1/2) dW
 *   eq. (6)  velocity: the generalized Langevin model, with the drift tensor
 *            G and C0 either from the simplified Langevin model, eq. (19),
 *            or from the elliptic-relaxation tensor, eqs. (12)-(13)
 *   eq. (7)  scalar:   IECM relaxation toward <phi|V> over the time scale of
 *            eq. (11)
 *   eq. (9)  optionally, the stochastic turbulent frequency omega, with the
 *            source term of eq. (10) and, at wall-function walls, the
 *            reflection condition of the wall-function section
 * tracks them through an unstructured triangular grid with wall (resolved
 * no-slip, free-slip, wall-function eqs. (20)-(26)) and periodic conditions,
 * applies the street-level source (section 3), and estimates per-element
 * statistics from the particles (section 2, after eq. 7, and section 3).
 *
 * Memory: the caller owns all device memory.  pdf_query_sizes() gives the
 * size of one device arena; the caller allocates it (e.g. a torch uint8
 * tensor) and hands it to pdf_init_mesh().  The library never allocates
 * device memory (the elliptic relaxation keeps two words of pinned host
 * memory per context for its convergence flag).  Host input arrays are
 * copied during the call.
 *
 * Streams: every call enqueues on the HIP stream given to pdf_create() and
 * returns without waiting, except pdf_sync(), the host-copy variants of
 * pdf_estimate_statistics()/pdf_get_state(), and pdf_destroy().
 *
 * Errors: every entry point returns a pdf_status.  Failures found on the
 * device (a particle the walk cannot place, a non-finite value, a full
 * element segment) are recorded in a device error word; the step that raised
 * one completes, later steps do nothing, and pdf_sync() returns the code.
 * pdf_error_string() describes the last error.
 */
#ifndef PDFPIC_H
#define PDFPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pdf_status;
#define PDF_OK 0
#define PDF_E_ARG -1       /* invalid argument                                   */
#define PDF_E_MESH -2      /* degenerate or inconsistent mesh                    */
#define PDF_E_SIZE -3      /* arena too small                                    */
#define PDF_E_HIP -4       /* HIP runtime error                                  */
#define PDF_E_LOST -5      /* tracking could not place a particle                */
#define PDF_E_NAN -6       /* non-finite particle state                          */
#define PDF_E_CAPACITY -7  /* an element segment overflowed between repacks       */
#define PDF_E_STATE -8     /* call out of order (e.g. step before seeding)       */

/* edge kinds of the mesh arrays */
#define PDF_EDGE_INTERIOR 0
#define PDF_EDGE_NOSLIP 1      /* resolved no-slip wall: U -> -U                 */
#define PDF_EDGE_SLIP 2        /* free-slip wall: specular                       */
#define PDF_EDGE_WALLFN 3      /* wall-function wall, eqs. (20)-(21)             */
#define PDF_EDGE_PERIODIC_XP 4 /* crossing adds +Lx to x                         */
#define PDF_EDGE_PERIODIC_XM 5 /* crossing adds -Lx to x                         */
#define PDF_EDGE_PERIODIC_YP 6 /* crossing adds +Ly to y                         */
#define PDF_EDGE_PERIODIC_YM 7 /* crossing adds -Ly to y                         */

/* statistics record per (ensemble, element): doubles in this order */
#define PDF_ST_N 0      /* particle count                                        */
#define PDF_ST_MEAN 1   /* 4: <u> <v> <w> <psi>                                  */
#define PDF_ST_M2 5     /* 10: central 2nd moments, index pairs a<=b of (u,v,w,psi) */
#define PDF_ST_BINN 15  /* 8: particles per velocity bin b = [u'>0]+2[v'>0]+4[w'>0] */
#define PDF_ST_BINM 23  /* 8: <phi|V> per bin, the element mean for an empty bin */
#define PDF_ST_M3 31    /* 20: central 3rd moments, a<=b<=c (moments == 4 only)  */
#define PDF_ST_M4 51    /* 35: central 4th moments, a<=b<=c<=d                   */
#define PDF_NSTAT_2 31  /* record length with moments == 2 (histogram follows)   */
#define PDF_NSTAT_4 86  /* record length with moments == 4 (histogram follows)   */

/* per-vertex frozen Eulerian fields, doubles, in this order (20 per vertex) */
#define PDF_NFIELD 20   /* U V dUdx dUdy dVdx dVdy lapU lapV dPdx dPdy
                           R11 R22 R33 R12 eps wp11 wp12 wp21 wp22 wp33 */

typedef struct pdf_params {
  int32_t f32_state;  /* 1: particle state in float, 0: double                  */
  int32_t model;      /* 0: SLM, eq. (19); 1: G and C0 from wp, eqs. (12)-(13)   */
  int32_t moments;    /* highest central moment order estimated: 2 or 4          */
  int32_t hist_bins;  /* scalar histogram bins on [0,1] per element: 0 or 32;
                         supported (moments, hist_bins): float state (2, 0) and
                         (4, 32), double state (2, 0)                            */
  int32_t mix;        /* 1: IECM mixing on                                       */
  int32_t psi_init;   /* initial scalar: 0 zero; 1 one where x < 0.25            */
  int32_t flags;      /* sub-steps: 1 velocity, 2 position+tracking, 4 IECM,
                         8 source (15 = the full step)                           */
  int32_t omega;      /* 1: particles carry the turbulent frequency of eq. (9):
                         seeded at the element's frozen <omega> (eq. 8 solved
                         at the centroid), advanced with the element's
                         frozen <omega> and the sixth normal of the step,
                         reflected at zero, rescaled at wall-function walls;
                         the velocity keeps the frozen-field coefficients.
                         The record gains <omega>, <omega'^2> and eps =
                         <omega>(k + nu C_T^2 <omega>), k from the record's
                         stresses.  0: off (no memory or work for it).      */
  int32_t vbins;      /* velocity bins per component for <phi|V> in IECM:
                         2: by the sign of each fluctuation (8 bins);
                         5: 5 x 5 x 5 bins of width 1.2 sigma on
                         [-3 sigma, 3 sigma] about the element mean (sigma
                         from its second moments, sigma = 0: the middle bin;
                         bin = k_u + 5 k_v + 25 k_w), float state without
                         omega only.  The record gains 125 counts and 125
                         conditional means (the element mean for an empty
                         bin) after everything else.                        */
  int32_t reserved;
  double dt, nu, C0;  /* time step, kinematic viscosity, SLM constant           */
  double CT, Cs, Ct;  /* Table 2 constants used by eqs. (8) and (11)            */
  double Cmu, kappa, Ewall, yp; /* wall functions: C_mu, Karman constant, E,
                                   distance of the stripped wall y_p            */
  double Lx, Ly;      /* periodic lengths                                        */
  double slack;       /* segment capacity = ceil(slack * initial count) + 32,
                         slack >= 1 (2 leaves room for density fluctuations)     */
  double C3, C4, Cw1, Cw2; /* Table 2, turbulent frequency (used when omega = 1;
                         C3, C4 > 0 and 1/2 + 3/4 C0 + C3 + Cw2 - Cw1 > 0)     */
} pdf_params;

typedef struct pdf_mesh {
  int32_t nvert, nelem;
  const double* vtx;     /* host, nvert x 2                                       */
  const int32_t* tri;    /* host, nelem x 3 vertex ids, counter-clockwise        */
  const int32_t* nbr;    /* host, nelem x 3: element across edge k=(v_k,v_k+1),
                            the periodic partner for periodic edges, -1 on walls */
  const int32_t* ekind;  /* host, nelem x 3: PDF_EDGE_*                          */
  const double* fields;  /* host, nvert x PDF_NFIELD                             */
} pdf_mesh;

typedef struct pdf_sizes {
  /* in */
  int32_t nvert, nelem, nens, reserved;
  int64_t nparticles;    /* total particles over all ensembles                   */
  /* out */
  int64_t arena_bytes;   /* device bytes the caller must provide                  */
  int64_t slots;         /* particle slots per state buffer                       */
} pdf_sizes;

typedef struct pdf_ctx pdf_ctx;

/* Create a context.  hip_stream: a hipStream_t (NULL: the null stream).
   *out receives the context; nothing is allocated on the device. */
pdf_status pdf_create(const pdf_params* p, void* hip_stream, pdf_ctx** out);

/* Fill s->arena_bytes and s->slots from the sizes in s. */
pdf_status pdf_query_sizes(const pdf_ctx* ctx, pdf_sizes* s);

/* The Eulerian grid of the method: the unstructured triangular mesh on which
   the paper tracks particles, estimates statistics and holds the Eulerian
   fields (closing summary of section 2.2; the meshes of section 3).  Copies
   the host arrays of m (layout in pdf_mesh; read during the call only) and
   the frozen per-vertex fields (PDF_NFIELD doubles per vertex) into the
   device arena (caller-owned device memory of arena_bytes, 256-byte aligned,
   sized by pdf_query_sizes; the context keeps the pointer, the caller keeps
   ownership and must keep it alive) and precomputes, per vertex, the drift
   tensor G and C0 eps of eq. (6) from eq. (19) (SLM) or eqs. (12)-(13)
   (from wp), and per wall-function edge alpha of eqs. (22)-(26), and the
   structure of the Eulerian solves on the mesh (the P1 system of
   pdf_elliptic_relaxation and pdf_pressure_projection: unknowns with the
   periodic seam copies joined, sparsity, element matrices).  Waits for
   the stream.  Errors: PDF_E_ARG (null or empty input, unaligned arena),
   PDF_E_MESH (vertex id, neighbour or edge kind out of range; a degenerate or
   clockwise element), PDF_E_SIZE (arena too small for the mesh), PDF_E_HIP. */
pdf_status pdf_init_mesh(pdf_ctx* ctx, const pdf_mesh* m, void* arena, int64_t arena_bytes);

/* The particle representation of the joint PDF (section 2: particles stand
   for fluid elements; section 3: particles per element, the street-level
   source): seed nens independent ensembles.  counts: host, nens x nelem
   int64, particles per element (ensemble-major); seeds: host, nens uint64
   Philox keys; source: host, nens x 3 doubles (x0, y0, r0; r0 = 0: no
   source).  All three are read during the call only.  Particles are placed
   uniformly in their element with the interpolated mean velocity plus
   Gaussian fluctuations with the interpolated Reynolds stress (its Cholesky
   factor); the scalar follows pdf_params.psi_init; particle ids run
   element-major from 0 within each ensemble.  Resets the step counter and
   the device error word.  Waits for the stream.  Errors: PDF_E_STATE
   (before pdf_init_mesh), PDF_E_ARG (bad count, negative r0), PDF_E_SIZE
   (too many cells or particles, or the layout does not fit the arena),
   PDF_E_HIP. */
pdf_status pdf_seed_particles(pdf_ctx* ctx, int32_t nens, const int64_t* counts,
                              const uint64_t* seeds, const double* source);

/* One time step is the explicit Euler-Maruyama step of the particle
   equations (closing summary of section 2.2): IECM, eq. (7), toward the
   binned <phi|V> of the state at the start of the step, with the rate of
   eq. (11); velocity, eq. (6) (and omega, eq. (9), if carried); position,
   eq. (5), with the velocity at the start of the step and the same dW;
   tracking through the grid with the wall and periodic conditions; the
   source of section 3.  The sub-steps taken are pdf_params.flags, fixed at
   pdf_create.  Enqueues nsteps steps of every ensemble on the context's
   stream and returns without waiting (nsteps = 0: nothing); where the order
   is split (cells of at most eight particles taking a launch of their own),
   that launch runs on a second stream of the context, forked from and
   joined back to the context's stream by events within each step, so work
   enqueued on the context's stream afterwards sees whole steps.  After a device
   error the remaining steps do nothing and pdf_sync reports it.  Errors:
   PDF_E_ARG (nsteps < 0), PDF_E_STATE (before pdf_seed_particles),
   PDF_E_HIP (launch failure). */
pdf_status pdf_step(pdf_ctx* ctx, int32_t nsteps);

/* As pdf_step, timing each step's kernels: HIP events recorded on the
   context's stream immediately before and after the kernels of every step
   (the step kernel and, when the order is split, the small cells' launch;
   not the capacity checks, which run every sixth step).  Waits for the stream and writes the summed event time of the
   nsteps steps, in milliseconds, to *kernel_ms (host).  Results are those of
   pdf_step.  Errors as pdf_step, and PDF_E_ARG for a null kernel_ms. */
pdf_status pdf_step_timed(pdf_ctx* ctx, int32_t nsteps, double* kernel_ms);

/* As pdf_step, but replays a HIP graph of six consecutive steps (built on
   first use for the current launch shape, from kernel nodes only); the
   leading and trailing steps that do not fill a graph are launched
   directly.  Results are identical to pdf_step. */
pdf_status pdf_step_graph(pdf_ctx* ctx, int32_t nsteps);

/* Choose the launch shape of the step by timing: lanes per element cell
   (64, 32, 16 or 8; a wavefront then serves 1, 2, 4 or 8 cells; 8 with the
   float state only) and a one-item-per-wavefront grid or a persistent grid
   pulling work from a counter.
   Runs two rounds over the candidates (the second in reverse order), each of
   1 + steps_per_trial real steps per candidate, and scores a candidate by
   its faster trial (the simulation advances by all of them; particle
   trajectories do not depend on the shape).  With the float state and no
   network attached, when the cells of at most 8 particles at seeding and
   the other cells each make up an eighth of the cells or more, the former
   take a launch of their own at 4 lanes per cell and the shape applies to
   the others.  The choice is
   kept in the context and returned in *group, *persist (either may be NULL).
   Synchronizes the stream. */
pdf_status pdf_autotune(pdf_ctx* ctx, int32_t steps_per_trial, int32_t* group, int32_t* persist);

/* Set the launch shape directly (group 8, 16, 32 or 64; persist 0 or 1).
   The double state supports group 64 only; group 8 runs the learned
   conditional means as a separate pass. */
pdf_status pdf_set_launch(pdf_ctx* ctx, int32_t group, int32_t persist);

/* Re-sort by element (the particle-in-cell bookkeeping of the closing summary of section 2.2).
   Each element cell owns a segment of the particle buffers, sized at seeding
   from its initial count: ceil(slack n0) + 32 slots.  Particles stay in
   their cell's segment or are appended to their new cell's segment, so the
   statistics of a cell read one contiguous range (two runs).  When the
   density drifts, a step flags every segment whose free room falls under
   half its count (or under 16) or under twice its arrivals of the last step
   (a step's arrivals may only use the room beyond the current count), and
   every sixth step (the end of the six-step cycle of pdf_step_graph;
   pdf_step checks at the same step counts) a device-side repack gives each
   cell max(initial, floor(g (n + a)) + 32) slots, g = max(3, slack + 1) and
   a its arrivals of the last step (floor(slack n) + 32 if that would not
   fit), copies the particles and continues; no host synchronisation is
   involved.  Particle trajectories do not depend on the layout.
   pdf_query_sizes reserves ceil(1.5 g N) + 32 ncell slots beyond the
   seeding layout for the growth.
   pdf_repack enqueues a repack now (asynchronous); pdf_repack_count waits
   for the stream and returns the repacks done since seeding (-1 on error). */
pdf_status pdf_repack(pdf_ctx* ctx);
int64_t pdf_repack_count(pdf_ctx* ctx);

/* Particle-in-cell estimation (section 2, after eq. 7: Eulerian statistics
   as ensemble averages over the particles of each grid element; section 3:
   the statistics and the <phi|V> bins the paper reports): the statistics of
   the current state into out, nens x nelem x nstat doubles, one record per
   (ensemble, element) in the PDF_ST_* layout (nstat = PDF_NSTAT_2 or
   PDF_NSTAT_4, plus hist_bins, plus 3 with the turbulent frequency: <omega>,
   <omega'^2>, eps, after the histogram, plus 250 with 5 x 5 x 5 velocity
   bins); averages use 1/n, an empty element has count 0 and zero moments.
   out_on_host: 1 -> out is host memory and the call waits; 0 -> out is
   device memory and the call is asynchronous.  out is caller-owned.
   Errors: PDF_E_ARG (null out), PDF_E_STATE (before seeding), PDF_E_HIP. */
pdf_status pdf_estimate_statistics(pdf_ctx* ctx, double* out, int32_t out_on_host);

/* Elliptic relaxation (section 2.1, eqs. 12-18): wp_ij of eq. (14),
     wp_ij - L^2 lap wp_ij = 1/2 (1 - C1) k <omega> delta_ij + k H_ijkl d<U_k>/dx_l,
   with H of eqs. (15)-(17) and L of eq. (18), solved on the mesh from the
   particle statistics of the current state, then G_ij and C0 eps of eqs.
   (12)-(13) per vertex written into the coefficient table the step reads
   (rounded to the state type), so that later steps use them.  Contexts with
   model = 1 only; the records of ensemble 0.  Readings:
   * per element, the Reynolds stress from the record's second moments
     (<u'w'> = <v'w'> = 0), the frozen stress of the centroid where the
     element holds fewer than 10 particles; k = tr R / 2; eps and d<U>/dx
     the frozen fields at the centroid; <omega> from eq. (8); C_xi = 2.3;
   * Galerkin P1 elements on the vertices, the copies of a periodic-seam
     vertex one unknown, L^2 and the right-hand side constant per element,
     zero normal derivative on every wall; the components wp_11, wp_12,
     wp_21, wp_22, wp_33;
   * per vertex, R and k area-weighted over the elements around it, eps the
     frozen field; a negative C0 is set to zero (and counted).
   The linear systems (one matrix, five right-hand sides) are solved by
   Jacobi-preconditioned conjugate gradients (the Chronopoulos-Gear form:
   one reduction per iteration) from the previous solution (the frozen wp
   fields at the first call) until ||r|| <= tol ||b|| for every component
   (tol ||r0|| where b = 0; r of the recurrence), or max_iters iterations
   (1..20000; tol in (0, 1)).
   Outputs, each may be NULL: wp (device, nvert x 5 doubles: wp_11 wp_12
   wp_21 wp_22 wp_33 per vertex); coef (device, nvert x 6 doubles: G_11 G_12
   G_21 G_22 G_33 C0 eps before rounding); info (host, 4 int32: iterations,
   1 if converged, vertices whose C0 was clamped, elements whose stresses came
   from the statistics); resid (host, 5 doubles: ||r|| / ||b|| per component
   at exit).  Waits for the stream.  Errors: PDF_E_ARG, PDF_E_STATE (before
   seeding, or model 0), PDF_E_HIP. */
pdf_status pdf_elliptic_relaxation(pdf_ctx* ctx, int32_t max_iters, double tol, double* wp, double* coef,
                                   int32_t* info, double* resid);

/* Mean-pressure projection (closing summary of section 2.2: the mean
   pressure of eq. (6) by a projection scheme; section 3: the mean-pressure
   Poisson equation solved on the grid by finite elements).  The scheme's
   details are in a work that is not available; this is the reading taken:
   the incremental projection of the particles' mean velocity onto weakly
   divergence-free fields.  From the statistics of the current state (one
   ensemble; per element the particles' mean velocity, the frozen mean
   velocity at the centroid where the element holds fewer than 10
   particles), the pressure increment phi solves lap(phi) = div<U> / T with
   d(phi)/dn = <U>.n / T at walls, in the Galerkin P1 form
     sum_e int_e grad(phi).grad(psi_i) = (1/T) sum_e area_e <U>_e . grad(psi_i)|_e
   on the unknowns of the relaxation system (its right-hand side sums to
   zero: the system is singular and consistent, phi is defined up to a
   constant; the mean the load keeps from rounding is taken off before the
   solve, as the bordered system that fixes phi's mean does).  Then grad(phi), constant per element, averaged by area to the
   vertices, is added to the mean pressure gradient (the device copy of the
   fields and the coefficient table the step reads), and every particle's
   velocity (u, v) loses T grad(phi) of its element (in double, rounded to
   the state type).  T = n dt covers the n steps since the previous applied
   projection (since seeding for the first; n >= 1): grad(phi) is then the
   mean pressure gradient those n steps lacked, so a caller that projects
   every n steps sees the gradient settle (with T = dt at every n > 2 the
   increments would grow about (n - 1)-fold per call, alternating in sign).
   The system is solved by conjugate gradients in the
   form of pdf_elliptic_relaxation (one launch per iteration), preconditioned
   by the inverse diagonal plus a coarse correction on aggregates of 32
   unknowns (the pseudo-inverse of the stiffness matrix projected on them;
   the diagonal alone where pdf_relaxation_size reports no aggregates),
   from phi = 0 until ||r|| <= tol ||b||, or max_iters iterations
   (1..20000; tol in (0, 1)).
   Outputs, each may be NULL: phi (device, nvert doubles, up to a constant);
   grad (device, nvert x 2 doubles: the vertex gradient added); info (host,
   4 int32: iterations, 1 if converged, 1 if the update was applied,
   elements whose velocity came from the particles); resid (host, 5 doubles:
   ||r|| / ||b|| of the increment in the first, 0 in the others).  Waits for
   the stream.  Errors: PDF_E_ARG, PDF_E_STATE (before seeding, or more than
   one ensemble), PDF_E_MESH (the mesh cannot take the Eulerian solves, see
   pdf_relaxation_size), PDF_E_HIP. */
pdf_status pdf_pressure_projection(pdf_ctx* ctx, int32_t max_iters, double tol, double* phi, double* grad,
                                   int32_t* info, double* resid);

/* Size of the relaxation system of the mesh (section 2.1, the Galerkin
   system of eq. 14): out (host, 4 int64) = unknowns (vertices, periodic
   copies joined), nonzeros of the matrix, the padded row length the solver
   stores (the longest row), and the aggregates of the coarse space of the
   mean-pressure projection's preconditioner (32 consecutive unknowns each;
   0: the mesh has more than 192 of them, or a solver block's rows touch
   more than 32, and the projection is preconditioned by the diagonal
   alone); the projection solves on the same unknowns.  Errors: PDF_E_ARG, PDF_E_STATE (before pdf_init_mesh),
   PDF_E_MESH (a row longer than 16 entries, or a vertex in no element: the
   Eulerian solves are unavailable on the mesh). */
pdf_status pdf_relaxation_size(const pdf_ctx* ctx, int64_t* out);

/* Run metrics from the device counters, into out (8 int64, host; waits):
   particles; arrivals written by the last step (particles now in another
   element than before it, 0 right after a repack, which folds them in);
   smallest and largest particle count of a cell; cells filled beyond three
   quarters of their segment; repacks since seeding; the device error word
   (PDF_E_* as bits: 1 lost, 2 non-finite, 4 capacity, 8 overflow area full);
   steps done. */
pdf_status pdf_metrics(pdf_ctx* ctx, int64_t* out);

/* Record length of the statistics. */
int32_t pdf_nstat(const pdf_ctx* ctx);

/* Wait for the stream; return the first device error since seeding. */
pdf_status pdf_sync(pdf_ctx* ctx);

/* Copy the state of ensemble ens in particle-id order into caller device
   memory: xyuvwpsi (6 x n doubles: x, y, u, v, w, psi) and elem (n int32),
   n = pdf_count(ctx, ens).  Asynchronous. */
pdf_status pdf_get_state(pdf_ctx* ctx, int32_t ens, double* xyuvwpsi, int32_t* elem);

/* Checkpoint restore (and a test hook for the device error paths): replace
   the state of ensemble ens with n = pdf_count(ctx, ens) particles given in
   the layout of pdf_get_state (xyuvwpsi 6 x n doubles, elem n int32, om n
   doubles with the turbulent frequency, else NULL; all device memory), in
   id order: particle i gets id i (its Philox counter) and goes to the segment
   of element elem[i]; values are rounded to the state type.  Positions are
   not checked against their elements.  Waits for the stream.  Errors, with
   the state left unchanged: PDF_E_ARG for an element index out of range,
   PDF_E_CAPACITY when an element's particles exceed its segment (create the
   context with a larger slack).  On success the ensemble's counters are
   rebuilt from elem.  After a device error every ensemble's state is void
   (steps that returned early wrote nothing): the device error word is
   cleared, and the context steps again, once every ensemble has been
   restored since the error; until then pdf_sync keeps reporting it. */
pdf_status pdf_set_state(pdf_ctx* ctx, int32_t ens, const double* xyuvwpsi, const int32_t* elem, const double* om);

/* Set the Philox step word of the next step (0 <= step < 2^32 - 1): with
   pdf_set_state, a run resumed from a checkpoint taken after step s draws
   the same numbers as the uninterrupted run.  pdf_steps_done is not
   changed.  Asynchronous. */
pdf_status pdf_set_step(pdf_ctx* ctx, int64_t step);

/* As pdf_get_state, plus the turbulent frequency om (n doubles, device
   memory).  PDF_E_STATE if the context carries none. */
pdf_status pdf_get_omega(pdf_ctx* ctx, int32_t ens, double* xyuvwpsi, int32_t* elem, double* om);

/* The frozen turbulent-frequency fields, into host memory (waits): om0 (nelem:
   <omega> at each centroid, eq. 8), somega (nelem: S_omega of eq. 10 with the
   production of the frozen fields at the centroid), omw (nelem x 3: <omega>
   at the midpoint of each wall-function edge, 0 on other edges).  PDF_E_STATE
   if the context carries no turbulent frequency. */
pdf_status pdf_omega_fields(pdf_ctx* ctx, double* om0, double* somega, double* omw);

/* Time averaging (the statistics the paper collects once the flow is
   stationary).  pdf_average_attach clears acc (device memory, caller-owned:
   nens x nelem x pdf_navg doubles) and from then on every step merges the
   statistics record it computes (of the state at the start of the step) into
   acc, on the stream, also inside graph replays; acc = NULL stops it.  acc
   per cell then holds the statistics of the cell's particles over all merged
   steps taken as one sample:
     PDF_AV_STEPS  steps merged
     PDF_AV_N      pooled particle count (sum of the per-step counts)
     PDF_AV_MEAN   4: pooled <u> <v> <w> <psi>
     PDF_AV_M2     10: pooled central second moments (PDF_ST_M2 pair order)
     PDF_AV_HIST   hist_bins: summed scalar histogram counts
     then, with the turbulent frequency, pooled <omega> and <omega'^2>.
   Means and moments are combined pairwise per step (Chan, Golub & LeVeque),
   so the result equals the law-of-total-variance pooling of the per-step
   records up to rounding.  acc must stay valid while attached. */
#define PDF_AV_STEPS 0
#define PDF_AV_N 1
#define PDF_AV_MEAN 2
#define PDF_AV_M2 6
#define PDF_AV_HIST 16
int32_t pdf_navg(const pdf_ctx* ctx);
pdf_status pdf_average_attach(pdf_ctx* ctx, double* acc);

/* Point location: elem[i] = the lowest-index element whose closed triangle
   contains point i (xy: n x 2 doubles), -1 if none.  Device memory in and
   out, asynchronous.  Used to map sampling locations to elements. */
pdf_status pdf_locate(pdf_ctx* ctx, const double* xy, int32_t n, int32_t* elem);

/* Probe values of ensemble ens from a time average acc at the given elements
   (device memory): out, nprobe x (4 + hist_bins) doubles per probe: steps
   averaged, mean particle count per step, <psi>, <psi'^2>, then the scalar
   CDF of eq. (29) at the upper edge of every histogram bin,
   F((b + 1) / hist_bins) = fraction of the pooled particles with
   psi < (b + 1) / hist_bins (the last bin includes psi = 1).  An element
   index out of range yields NaN entries.  Asynchronous. */
pdf_status pdf_average_probe(pdf_ctx* ctx, const double* acc, int32_t ens, const int32_t* elems, int32_t nprobe,
                             double* out);

/* Number of particles of an ensemble; steps enqueued since seeding. */
int64_t pdf_count(const pdf_ctx* ctx, int32_t ens);
int64_t pdf_steps_done(pdf_ctx* ctx);

/* Text of the last error. */
const char* pdf_error_string(const pdf_ctx* ctx);

/* Release the context (waits for its stream). */
void pdf_destroy(pdf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
