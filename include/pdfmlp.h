/*
 * pdfpic learned conditional means -- C ABI.
 *
 * IECM, eq. (7), relaxes each particle's scalar toward <phi|V>: the mean
 * scalar of the particles of its element whose velocity lies in the same
 * velocity bin (2 x 2 x 2 bins by the sign of each velocity fluctuation
 * about the element mean, statistics of section 2, after eq. 7).  With few particles
 * per element the binned estimate is noisy.  These entry points train and
 * apply a small network that estimates the eight conditional means of an
 * element from its statistics, with the binned estimate as the fallback.
 *
 * Features (32 floats) of an element with statistics record r (pdfpic.h):
 *   0      n / 64
 *   1..4   means of u, v, w, psi
 *   5..14  central second moments (PDF_ST_M2 order)
 *   15..22 bin fractions n_b / n (0 when n = 0)
 *   23..30 binned conditional means (the element mean for an empty bin)
 *   31     standard deviation of psi
 * Normalisation, norm (4 x 32 floats): mean, inverse scale, training
 * minimum, training maximum of each feature; the network input is the
 * bfloat16 rounding of (f - mean) * inverse scale.
 *
 * Network: 32 -> 64 -> 64 -> 64 -> 8, ReLU, bfloat16 weights and biases
 * (w, 16-bit codes), float32 accumulation on the matrix cores, hidden
 * activations rounded to bfloat16.  Parameters, flat, PDF_MLP_NPARAM:
 *   W1 (64 x 32, row-major out x in), b1 (64), W2 (64 x 64), b2, W3 (64 x 64),
 *   b3, W4 (8 x 64), b4 (8).
 * Outputs y_b are standardised conditional means.  Estimate of an element:
 *   p_b = y_b - sum_c (n_c / n) y_c,   m_b = <psi> + sigma_psi p_b,
 * so that sum_b n_b m_b = n <psi> and IECM keeps conserving the element's
 * scalar.  The element takes m_b only if 8 <= n <= 64, every feature lies in
 * [training minimum, training maximum], sigma_psi > 0 and every m_b lies in
 * [0, 1]; otherwise it keeps the binned means.
 *
 * Training rows (PDF_MLP_ROW floats) from a state with many particles per
 * element: in every element a Bernoulli subsample with probability
 * target / n (Philox4x32-10, key = key, counter = (particle id, draw,
 * 0x5EED, ensemble), uniform r 2^-32 + 2^-33 below the probability) plays
 * the few-particle estimator:
 *   0..31  features of the subsample
 *   32..39 targets: (m_ref_b - <psi>_sub) / sigma_sub, clipped to +-8
 *   40..47 loss weights: subsample bin fractions n_b / n_sub
 *   48..55 m_ref_b: mean scalar of all the element's particles in bin b, the
 *          bins split at the subsample's means (the element mean if empty)
 *   56..63 number of all the element's particles in bin b
 * Rows whose subsample has fewer than 2 particles or sigma_sub <= 1e-4 get
 * zero targets and loss weights; an element with an empty subsample gets a
 * zero row.
 *
 * Loss of a batch of B rows: (1/B) sum_rows sum_b lw_b (p_b - t_b)^2 with
 * p the projected output.  Adam (bias-corrected, beta1 0.9, beta2 0.999,
 * eps 1e-8) updates a float32 master copy; w is its bfloat16 rounding.
 *
 * Memory: every pointer is caller-owned device memory (the library
 * allocates nothing).  Work is enqueued on the given HIP stream (NULL: the
 * null stream) and the calls return without waiting.  Errors: PDF_E_ARG for
 * null or inconsistent arguments, PDF_E_HIP for launch failures.
 */
#ifndef PDFMLP_H
#define PDFMLP_H

#include <stdint.h>

#include "pdfpic.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PDF_MLP_NPARAM 10952
#define PDF_MLP_NFEAT 32
#define PDF_MLP_NOUT 8
#define PDF_MLP_ROW 64
#define PDF_MLP_MAX_BATCH 65536

/* Floats of the training workspace for batches up to batch rows:
   ceil(batch / 16) x (PDF_MLP_NPARAM + 1). */
int64_t pdf_mlp_work_floats(int32_t batch);

/* Training rows of the context's current state, one per element cell
   (nens x nelem rows of PDF_MLP_ROW floats, ensemble-major).  target: the
   expected subsample size; key, draw: the Philox key and draw index. */
pdf_status pdf_mlp_dataset(pdf_ctx* ctx, int32_t target, uint64_t key, uint32_t draw, float* rows);

/* Network outputs y (nrows x 8 floats, unprojected) of the features in the
   first 32 floats of each row (row_stride floats apart). */
pdf_status pdf_mlp_forward(const float* rows, int64_t nrows, int32_t row_stride, const float* norm,
                           const uint16_t* w, float* y, void* hip_stream);

/* Loss and gradient (PDF_MLP_NPARAM floats) over training rows 0..batch-1.
   work: pdf_mlp_work_floats(batch) floats.  loss: one float. */
pdf_status pdf_mlp_grad(const float* rows, int32_t batch, const float* norm, const uint16_t* w,
                        float* work, float* grad, float* loss, void* hip_stream);

/* pdf_mlp_grad without a workspace argument, for callers that cannot
   allocate device memory (code under HIP graph capture, serving loops,
   harnesses that forbid allocation).  The gradient partials live in a
   static device array of PDF_MLP_NOALLOC_FLOATS floats (about 2.7 MiB)
   that each device holds until the process ends; the call itself allocates
   nothing.  batch: 1 .. PDF_MLP_NOALLOC_MAX_BATCH, else PDF_E_SIZE.  All
   calls on one device share the array, so calls that overlap on one device
   (different streams, or host threads without ordering) race; calls on one
   stream are ordered and safe.  Results equal pdf_mlp_grad's bit for bit.
   loss: one float (required).  Errors as pdf_mlp_grad, and PDF_E_HIP if the
   array's device address cannot be found. */
#define PDF_MLP_NOALLOC_MAX_BATCH 1024
#define PDF_MLP_NOALLOC_FLOATS (((PDF_MLP_NOALLOC_MAX_BATCH + 15) / 16) * (PDF_MLP_NPARAM + 1))
pdf_status pdf_mlp_grad_noalloc(const float* rows, int32_t batch, const float* norm, const uint16_t* w,
                                float* grad, float* loss, void* hip_stream);

/* iters Adam steps, numbered t0 + 1 ... t0 + iters, each on batch rows drawn
   with replacement from the nrows training rows (Philox4x32-10, key = seed,
   counter = (slot, t, 0x7A11, 0), row = first word mod nrows).  master,
   adam_m, adam_v: PDF_MLP_NPARAM floats; w: the bfloat16 copy, rewritten;
   loss: iters floats, the batch loss before each step. */
pdf_status pdf_mlp_train(const float* rows, int64_t nrows, const float* norm, float* master, float* adam_m,
                         float* adam_v, uint16_t* w, float* work, float* loss, int32_t iters, int32_t batch,
                         float lr, uint64_t seed, int64_t t0, void* hip_stream);

/* Normalisation (4 x 32 floats, layout above) from the training rows whose
   loss weights are not all zero: per feature the mean, the inverse
   population standard deviation (1 where it is below 1e-12) and the
   minimum and maximum. */
pdf_status pdf_mlp_norm(const float* rows, int64_t nrows, float* norm, void* hip_stream);

/* bfloat16 codes w of float32 parameters master (round to nearest even). */
pdf_status pdf_mlp_round(const float* master, uint16_t* w, void* hip_stream);

/* Conditional means per cell (ncell x 8 doubles) from statistics records
   (ncell x nstat doubles) with the fallback rule above; *served (may be
   NULL) is incremented by the cells that took the network's value. */
pdf_status pdf_mlp_infer(const double* stats, int32_t nstat, int32_t ncell, const uint16_t* w,
                         const float* norm, double* cm, uint32_t* served, void* hip_stream);

/* Use the network in the context's steps: each step computes the learned
   conditional means of the state's statistics, writes them to cm (nens x
   nelem x 8 doubles) and relaxes IECM toward them.  With a one-item-per-
   wavefront launch shape this happens inside the step kernel (each block's
   cells form one 16-column network tile; graphs replay it as usual); with a
   persistent shape as a statistics pass and an inference launch before the
   step (pdf_step_graph then launches its steps one by one).  The results are
   the same.  w = NULL returns to the binned means.  The arrays must stay
   valid while attached. */
pdf_status pdf_mlp_attach(pdf_ctx* ctx, const uint16_t* w, const float* norm, double* cm, uint32_t* served);

#ifdef __cplusplus
}
#endif
#endif
