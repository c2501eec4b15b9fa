// Elliptic relaxation (section 2.1): the tensor wp of eq. (14) from the
// particle statistics, by Galerkin P1 finite elements on the mesh and a
// Jacobi-preconditioned conjugate-gradient solve, then G and C0 of eqs.
// (12)-(13) per vertex into the coefficient table the step reads.  The
// mean-pressure projection further down solves its Poisson system with the
// same iteration and a two-level preconditioner.
//
//   wp_ij - L^2 lap wp_ij = 1/2 (1 - C1) k <omega> delta_ij + k H_ijkl d<U_k>/dx_l
//
// H of eq. (15) with A_v of eq. (16) and b of eq. (17); L of eq. (18).  The
// unknowns are the mesh vertices with the two copies of a periodic-seam
// vertex joined; L^2 and the right-hand side are constant per element; every
// wall carries the natural (zero normal derivative) condition.  The five
// components wp_11, wp_12, wp_21, wp_22, wp_33 share the matrix and are
// solved together; vectors are stored component-major (5 x nc doubles), and
// a solver launch runs one block per (BLK unknowns, component).
//
// The iteration is the Chronopoulos-Gear form of preconditioned CG: its two
// inner products come from the same vectors, so one launch per iteration
// does the vector updates, the product with the matrix and the partial inner
// products.  The product needs the new preconditioned residual u = M^-1 r of
// the neighbouring unknowns; each thread recomputes it from their values of
// the previous iteration (r, w = A u, s = A p and the inverse diagonal, one
// 32-byte record per unknown and component, in two buffers by iteration
// parity), with the same operations as their owners, so the product is
// exactly A u.  Every block sums the previous launch's block partials it
// needs (its component's two inner products, every component's residual
// norm) in the same fixed order and derives the iteration's scalars itself,
// so a launch has two dependent rounds of memory accesses (its own
// loads, then the gathers of the neighbours' values), no atomics, and every
// result is reproducible.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdf_kernels.hpp"

namespace pdf {
namespace relax {

constexpr int NC = 5;            // solved components
constexpr int BLK = 128;         // threads of a solver block (one component, BLK unknowns)
constexpr int WPB = BLK / WAVE;  // its wavefronts
constexpr int N_MIN = 10;        // fewer particles: the element takes the frozen stresses
constexpr int ELL_MAX = 16;      // matrix entries per row at most
// Table 2
constexpr double C1 = 1.85, C2 = 0.63, CT = 6.0, CL = 0.134, CETA = 72.0, CV = 1.4, GAMMA5 = 0.1;
constexpr double C_XI = 2.3;     // 1 + 1.3 n_i n_i with a unit normal n

// Scalars of one iteration, written by block (0, 0) of its launch into the
// slot of its parity and read by the next launch.
struct Scal {
  double alpha[NC];             // alpha of the iteration
  double gamma[NC];             // (r, u) of the iteration
  int32_t iter;                 // the next iteration's index
  int32_t done;                 // the solve has stopped
};

// Solver control in device memory.
struct Ctl {
  Scal sc[2];
  double ref[NC];               // (b, b), or (r0, r0) where b = 0
  double rho[NC];               // (r, r) at the stop
  double tol2;
  int32_t iter;                 // iterations done at the stop
  int32_t max_iters;
  int32_t done;                 // converged or out of iterations
  int32_t converged;
  int32_t clamped;              // vertices whose C0 was negative
  int32_t from_stats;           // elements whose stresses came from the particles
  int32_t applied;              // the projection's update has been applied
  int32_t pad_;
};

struct alignas(32) Rec {
  double r, w, s, d;
};

struct Args {
  // mesh (device)
  int32_t ne, nv, nc, nbx, ellw;
  const int32_t* tri;      // ne x 3
  const double* vtx;       // nv x 2
  const double* fields;    // nv x NFIELD (frozen; the projection updates the mean pressure gradient)
  double* fields_rw;       // the same array, written by the projection
  const int32_t* canon;    // nv: unknown of each vertex
  // matrix rows padded to ellw entries, slot t of row i at t * nc + i;
  // padding points at the row itself with a zero entry
  const int32_t* ecol;     // ellw x nc column
  const int32_t* enz;      // ellw x nc nonzero index (-1: padding)
  const int32_t* dpos;     // nc: nonzero index of the diagonal entry of each row
  const int32_t* cptr;     // nnz + 1: contributions of each nonzero
  const int32_t* cidx;     // e * 9 + a * 3 + b
  const int32_t* incptr;   // nc + 1: (element, local vertex) pairs of each unknown
  const int32_t* inc;      // e * 3 + a
  const double* Ke;        // ne x 9: area grad(phi_a) . grad(phi_b)
  const double* area;      // ne
  // statistics records of the state (ensemble 0), nstat doubles per element
  const double* stats;
  int32_t nstat;
  double nu;
  // the system: mass * M + L^2 K; right-hand side 0: relaxation (S per
  // element and component, times a third of the area), 1: projection (S per
  // element and local vertex, component 0 only)
  double mass;
  int32_t rhs_mode;
  double dt;
  // work (device)
  double* S;               // 5 x ne right-hand side per element
  double* L2;              // ne
  double* Rk;              // 4 x ne: R11 R22 R33 R12
  double* aval;            // ellw x nc matrix entries
  double* dinv;            // nc: 1 / diagonal
  double* x;               // 5 x nc (the solution; the previous one is the first guess)
  double* p;               // 5 x nc
  // per (component, unknown), by iteration parity: r_i, w_i, s_{i-1}, 1/diag
  // of iteration i in buffer i & 1
  Rec* rec[2];
  double* part[2];         // 5 x nbx x 3 block partials (r,u) (w,u) (r,r), by parity
  double* pbb;             // 5 x nbx block partials of (b, b)
  Ctl* ctl;
  // the projection's coarse space (na = 0: none, the preconditioner is D^-1)
  int32_t na;
  const float* ep;         // nbx x NEED x NA_MAX: per block, the E^+ rows of the aggregates
                           // whose correction it reads (symmetric, in float; zero past
                           // column na and past the end of its list)
  const int32_t* eneed;    // ellw x nc: position of each row slot's column aggregate in that list
  double* agp[2];          // na x 3 aggregate sums of r_i, w_i, s_{i-1}, by parity
  double* cglob[2];        // na: the coarse correction of r_i, by parity
};

// the projection's coarse space: aggregates of AGG consecutive unknowns (the
// numbering is a recursive bisection, so they are compact patches); a block
// of BLK unknowns owns APB of them and reads the correction of at most NEED
// (its own and those its rows touch), TPE threads per entry of that list,
// each summing JMAX terms of a row of E^+
constexpr int AGG = 32;
constexpr int APB = BLK / AGG;
constexpr int NEED = 32;
constexpr int TPE = BLK / NEED;
constexpr int NA_MAX = 192;
constexpr int JMAX = NA_MAX / TPE;
static_assert(BLK % AGG == 0 && BLK % NEED == 0 && NA_MAX % (4 * TPE) == 0 && NA_MAX == 3 * WAVE, "coarse layout");

// ---------------------------------------------------------------------------
// set-up with the mesh: per element the area and area grad(phi_a).grad(phi_b)
// of the P1 shape functions; the first guess of the solution from the frozen
// wp fields at one vertex of each unknown

__global__ void k_relax_geom(const double* vtx, const int32_t* tri, double* Ke, double* area, int ne) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double x[3], y[3];
  for (int k = 0; k < 3; ++k) {
    x[k] = vtx[2 * tri[3 * e + k]];
    y[k] = vtx[2 * tri[3 * e + k] + 1];
  }
  const double a2 = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
  // 2A grad(phi_a) = (y_{a+1} - y_{a+2}, x_{a+2} - x_{a+1})
  double gx[3], gy[3];
  for (int k = 0; k < 3; ++k) {
    gx[k] = y[(k + 1) % 3] - y[(k + 2) % 3];
    gy[k] = x[(k + 2) % 3] - x[(k + 1) % 3];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ke[9 * e + 3 * i + j] = (gx[i] * gx[j] + gy[i] * gy[j]) / (2.0 * a2);
  area[e] = 0.5 * a2;
}

__global__ void k_relax_warm(const double* fields, const int32_t* rep, double* x, int nc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const double* f = fields + (size_t)rep[i] * NFIELD;
  for (int c = 0; c < NC; ++c) x[(size_t)c * nc + i] = f[F_P11 + c];
}

// ---------------------------------------------------------------------------
// per solve

__global__ void k_relax_reset(Ctl* ctl, int max_iters, double tol2) {
  if (threadIdx.x != 0) return;
  ctl->tol2 = tol2;
  ctl->iter = 0;
  ctl->max_iters = max_iters;
  ctl->done = 0;
  ctl->converged = 0;
  ctl->clamped = 0;
  ctl->from_stats = 0;
  ctl->applied = 0;
  for (int q = 0; q < 2; ++q) {
    for (int c = 0; c < NC; ++c) ctl->sc[q].alpha[c] = ctl->sc[q].gamma[c] = 0.0;
    ctl->sc[q].iter = 0;
    ctl->sc[q].done = 0;
  }
}

// per element: stresses, k, <omega>, L^2 and the right-hand side of eq. (14)
__global__ __launch_bounds__(BLK) void k_relax_inputs(Args a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  bool est = false;
  if (e < a.ne) {
    const double* f0 = a.fields + (size_t)a.tri[3 * e] * NFIELD;
    const double* f1 = a.fields + (size_t)a.tri[3 * e + 1] * NFIELD;
    const double* f2 = a.fields + (size_t)a.tri[3 * e + 2] * NFIELD;
    auto cen = [&](int j) { return (f0[j] + f1[j] + f2[j]) / 3.0; };
    const double* rec = a.stats + (size_t)e * a.nstat;
    double r11, r22, r33, r12;
    est = rec[ST_N] >= (double)N_MIN;
    if (est) {
      // central second moments in pair order (uu uv uw up vv vw vp ww wp pp)
      r11 = rec[ST_M2]; r12 = rec[ST_M2 + 1]; r22 = rec[ST_M2 + 4]; r33 = rec[ST_M2 + 7];
    } else {
      r11 = cen(F_R11); r22 = cen(F_R22); r33 = cen(F_R33); r12 = cen(F_R12);
    }
    const double tr = r11 + r22 + r33;
    const double k = 0.5 * tr;
    const double eps = cen(F_EPS);
    const double om = 2.0 * eps / (k + sqrt(k * k + 4.0 * a.nu * CT * CT * eps));
    // d<U_k>/dx_l for k, l in {x, y}
    const double g[2][2] = {{cen(F_DUDX), cen(F_DUDY)}, {cen(F_DVDX), cen(F_DVDY)}};
    // anisotropy (eq. 17) and A_v (eq. 16); R13 = R23 = 0
    const double b00 = r11 / tr - 1.0 / 3.0, b11 = r22 / tr - 1.0 / 3.0, b01 = r12 / tr;
    const double det = r33 * (r11 * r22 - r12 * r12);
    const double k23 = 2.0 * k / 3.0;
    const double Av = fmin(1.0, CV * det / (k23 * k23 * k23));
    // H_ijkl g_kl (eq. 15); b_ik g_kl sums over k, l in {x, y} (the spanwise
    // row and column of the gradient vanish)
    const double a1 = C2 * Av + GAMMA5 / 3.0;
    const double b[2][2] = {{b00, b01}, {b01, b11}};
    auto hterm = [&](int i, int j) {
      // (C2 Av + g5/3) g_ij - g5/3 g_ji + g5 sum_m b_im g_mj - g5 sum_m b_im g_jm
      double t = a1 * g[i][j] - GAMMA5 / 3.0 * g[j][i];
      double s1 = 0.0, s2 = 0.0;
      for (int m = 0; m < 2; ++m) {
        s1 += b[i][m] * g[m][j];
        s2 += b[i][m] * g[j][m];
      }
      return t + GAMMA5 * s1 - GAMMA5 * s2;
    };
    const double slow = 0.5 * (1.0 - C1) * k * om;
    const int ne = a.ne;
    a.S[0 * ne + e] = k * hterm(0, 0) + slow;
    a.S[1 * ne + e] = k * hterm(0, 1);
    a.S[2 * ne + e] = k * hterm(1, 0);
    a.S[3 * ne + e] = k * hterm(1, 1) + slow;
    a.S[4 * ne + e] = slow;   // H_33kl g_kl = 0: no spanwise gradient
    const double L = CL * fmax(C_XI * k * sqrt(k) / eps, CETA * sqrt(sqrt(a.nu * a.nu * a.nu / eps)));
    a.L2[e] = L * L;
    a.Rk[0 * ne + e] = r11;
    a.Rk[1 * ne + e] = r22;
    a.Rk[2 * ne + e] = r33;
    a.Rk[3 * ne + e] = r12;
  }
  const uint64_t m = __ballot(est);
  if ((threadIdx.x & (WAVE - 1)) == 0 && m) atomicAdd(&a.ctl->from_stats, (int)__popcll(m));
}

// matrix entries (M + L^2 K gathered from the element contributions in
// their fixed order), one thread per padded slot, and the inverse diagonal
__global__ __launch_bounds__(BLK) void k_relax_matrix(Args a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.ellw * a.nc) return;
  const int j = a.enz[q];
  double v = 0.0;
  if (j >= 0) {
    for (int t = a.cptr[j]; t < a.cptr[j + 1]; ++t) {
      const int c = a.cidx[t];
      const int e = c / 9, ab = c - 9 * e, aa = ab / 3, bb = ab - 3 * aa;
      const double m = a.area[e] / 12.0 * (aa == bb ? 2.0 : 1.0);
      v += a.mass * m + a.L2[e] * a.Ke[9 * e + ab];
    }
  }
  a.aval[q] = v;
  const int i = q % a.nc;
  if (j >= 0 && a.dpos[i] == j) a.dinv[i] = 1.0 / v;
}

// ---------------------------------------------------------------------------
// reductions

// One DPP move of a double (both halves with the same lane pattern).
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The sums over the 64 lanes of a wavefront of K values per lane (every lane
// active), the same in every lane: within each row of 16 lanes, partners
// exchange by DPP (lane ^ 1, lane ^ 2, then the mirrored half-row and row),
// so every lane of a row holds the row sum; then the four row sums in order.
// A fixed order, and each pair of partners adds the same two numbers.  The K
// exchanges go step by step side by side, so that they overlap instead of
// waiting on one another.
template <int K> __device__ __forceinline__ void wave_sums(const double (&v)[K], double (&out)[K]) {
  double t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = v[k] + dpp_move<0xB1>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] += dpp_move<0x4E>(t[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] += dpp_move<0x141>(t[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] += dpp_move<0x140>(t[k]);
#pragma unroll
  for (int k = 0; k < K; ++k)
    out[k] = (read_lane(t[k], 0) + read_lane(t[k], 16)) + (read_lane(t[k], 32) + read_lane(t[k], 48));
}

// The block's sums of K values per thread (wavefront sums, then the
// wavefronts in turn), valid in thread 0.
template <int K> __device__ void block_sum(double (&v)[K]) {
  __shared__ double sw[WPB][K];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  double t[K];
  wave_sums<K>(v, t);
  if (lane == 0)
    for (int k = 0; k < K; ++k) sw[wv][k] = t[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) {
      double u = sw[0][k];
      for (int q = 1; q < WPB; ++q) u += sw[q][k];
      v[k] = u;
    }
}

// Sums over the blocks of a launch of K partials per (component, block),
// src[(c * nbx + bx) * K + k], into tot[c][k], computed by every wavefront
// for itself (lane l adds blocks l, l + 64, ... in turn, then wave_sums): a
// fixed order, the same in every block.
template <int K> __device__ void total_partials(const Args& a, const double* src, double (&tot)[NC][K]) {
  const int lane = threadIdx.x & (WAVE - 1);
  double t[NC][K];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int k = 0; k < K; ++k) t[c][k] = 0.0;
  for (int bx = lane; bx < a.nbx; bx += WAVE)
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int k = 0; k < K; ++k) t[c][k] += src[((size_t)c * a.nbx + bx) * K + k];
#pragma unroll
  for (int c = 0; c < NC; ++c) wave_sums<K>(t[c], tot[c]);
}

// the recurrences of one unknown: s = w + beta s, r' = r - alpha s, u' = r' / d;
// neighbours and owners evaluate them with the same operations
__device__ __forceinline__ double s_next(double w, double s, double beta) { return __builtin_fma(beta, s, w); }
__device__ __forceinline__ double r_next(double r, double s, double alpha) { return __builtin_fma(-alpha, s, r); }

// ---------------------------------------------------------------------------
// start: r0 = b - A x0 and (b, b) partials (first launch); w0 = A u0 and the
// partials of iteration 0 (second launch); p and s start at zero

__global__ __launch_bounds__(BLK) void k_relax_start1(Args a) {
  const int i = blockIdx.x * BLK + threadIdx.x, c = blockIdx.y, nc = a.nc;
  double bb[1] = {0.0};
  if (i < nc) {
    double bv = 0.0;
    if (a.rhs_mode == 0) {
      for (int t = a.incptr[i]; t < a.incptr[i + 1]; ++t) {
        const int e = a.inc[t] / 3;
        bv += a.S[(size_t)c * a.ne + e] * (a.area[e] / 3.0);
      }
    } else if (c == 0) {
      for (int t = a.incptr[i]; t < a.incptr[i + 1]; ++t) {
        const int e = a.inc[t] / 3, l = a.inc[t] - 3 * e;
        bv += a.S[(size_t)l * a.ne + e];
      }
    }
    const double* xc = a.x + (size_t)c * nc;
    double ax = 0.0;
    for (int t = 0; t < a.ellw; ++t) ax = __builtin_fma(a.aval[t * nc + i], xc[a.ecol[t * nc + i]], ax);
    const size_t o = (size_t)c * nc + i;
    Rec& q = a.rec[0][o];
    q.r = bv - ax;
    q.s = 0.0;
    q.d = a.dinv[i];
    a.p[o] = 0.0;
    bb[0] = bv * bv;
  }
  block_sum<1>(bb);
  if (threadIdx.x == 0) a.pbb[(size_t)c * a.nbx + blockIdx.x] = bb[0];
}

__global__ __launch_bounds__(BLK) void k_relax_start2(Args a) {
  const int i = blockIdx.x * BLK + threadIdx.x, c = blockIdx.y, nc = a.nc;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < nc) {
    Rec* r0 = a.rec[0] + (size_t)c * nc;
    double acc = 0.0;
    for (int t = 0; t < a.ellw; ++t) {
      const int k = a.ecol[t * nc + i];
      acc = __builtin_fma(a.aval[t * nc + i], r0[k].r * r0[k].d, acc);
    }
    const double ri = r0[i].r, ui = ri * r0[i].d;
    r0[i].w = acc;   // the neighbours read r and d of the record only
    v[0] = ri * ui;
    v[1] = acc * ui;
    v[2] = ri * ri;
  }
  block_sum<3>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) a.part[0][((size_t)c * a.nbx + blockIdx.x) * 3 + k] = v[k];
  if (blockIdx.x != 0 || blockIdx.y != 0) return;
  double tot[NC][1];
  total_partials<1>(a, a.pbb, tot);
  if (threadIdx.x == 0)
    for (int q = 0; q < NC; ++q) a.ctl->ref[q] = tot[q][0];   // (r0, r0) where b = 0: set by iteration 0
}

// ---------------------------------------------------------------------------
// iteration i (parity par): from the partials of the previous launch, gamma_i
// = (r_i, u_i), delta_i = (w_i, u_i), rho_i = (r_i, r_i); stop when every
// component has rho_i <= tol^2 ref or i reaches the limit; else beta_i =
// gamma_i / gamma_{i-1}, alpha_i = gamma_i / (delta_i - beta_i gamma_i /
// alpha_{i-1}), and p = u + beta p, s = w + beta s, x += alpha p,
// r -= alpha s, u = M^-1 r, w = A u with the partials of iteration i + 1.
// W: the padded row length.  Every load is issued before any decision (rows
// past nc read the last row and store nothing): the row's entries, its own
// values, the scalars and the partials in one round, then the neighbours'
// values in a second.

template <int W> __global__ __launch_bounds__(BLK) void k_relax_iter(Args a, int par) {
  const int c = blockIdx.y, nc = a.nc, lane = threadIdx.x & (WAVE - 1);
  const int i = blockIdx.x * BLK + threadIdx.x;
  const bool live = i < nc;
  const int ii = live ? i : nc - 1;
  const Rec* old = a.rec[par] + (size_t)c * nc;
  Rec* nxt = a.rec[par ^ 1] + (size_t)c * nc;
  const size_t o = (size_t)c * nc + ii;
  int cl[W];
  double av[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    cl[t] = a.ecol[t * nc + ii];
    av[t] = a.aval[t * nc + ii];
  }
  const double2 rw_o = *reinterpret_cast<const double2*>(&old[ii].r);
  const double2 sd_o = *reinterpret_cast<const double2*>(&old[ii].s);
  const double r_o = rw_o.x, w_o = rw_o.y, s_o = sd_o.x, d_o = sd_o.y, p_o = a.p[o], x_o = a.x[o];
  const Ctl* ctl = a.ctl;
  const Scal& prev = ctl->sc[par ^ 1];
  const int pdone = prev.done, it = prev.iter, max_iters = ctl->max_iters;
  const double gold = prev.gamma[c], aold = prev.alpha[c], tol2 = ctl->tol2;
  double ref[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) ref[q] = ctl->ref[q];
  // partials of the blocks lane, lane + 64, ... (a fixed order per lane):
  // (r, u) and (w, u) of this block's component, (r, r) of every component
  const double* src = a.part[par];
  double tg[2], tr[NC];
  {
    const int bx = lane < a.nbx ? lane : 0;
    const double keep = lane < a.nbx ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) tg[k] = keep * src[((size_t)c * a.nbx + bx) * 3 + k];
#pragma unroll
    for (int q = 0; q < NC; ++q) tr[q] = keep * src[((size_t)q * a.nbx + bx) * 3 + 2];
  }
  // the neighbours' values
  double2 grw[W], gsd[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const int k = cl[t];
    grw[t] = *reinterpret_cast<const double2*>(&old[k].r);
    gsd[t] = *reinterpret_cast<const double2*>(&old[k].s);
  }
  for (int bx = lane + WAVE; bx < a.nbx; bx += WAVE) {
#pragma unroll
    for (int k = 0; k < 2; ++k) tg[k] += src[((size_t)c * a.nbx + bx) * 3 + k];
#pragma unroll
    for (int q = 0; q < NC; ++q) tr[q] += src[((size_t)q * a.nbx + bx) * 3 + 2];
  }
  if (pdone) return;
  // the two inner products of this component and every component's (r, r)
  double sv[2 + NC], sm[2 + NC];
#pragma unroll
  for (int k = 0; k < 2; ++k) sv[k] = tg[k];
#pragma unroll
  for (int q = 0; q < NC; ++q) sv[2 + q] = tr[q];
  wave_sums<2 + NC>(sv, sm);
  double rho[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) rho[q] = sm[2 + q];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    // where b = 0 the reference is (r0, r0), known from iteration 0 on
    const double rq = ref[q] > 0.0 ? ref[q] : (it == 0 ? rho[q] : ref[q]);
    ok = ok && rho[q] <= tol2 * rq;
  }
  const double g = sm[0], d = sm[1];
  const double beta = gold != 0.0 ? g / gold : 0.0;
  const double den = aold != 0.0 ? d - beta * g / aold : d;
  const double alpha = den != 0.0 ? g / den : 0.0;
  const bool stop = ok || it >= max_iters;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl* cw = a.ctl;
    Scal& cur = cw->sc[par];
    if (blockIdx.y == 0) {
      cur.iter = it + 1;
      cur.done = stop ? 1 : 0;
      if (it == 0)
        for (int q = 0; q < NC; ++q)
          if (!(ref[q] > 0.0)) cw->ref[q] = rho[q];
      if (stop) {
        cw->iter = it;
        cw->done = 1;
        cw->converged = ok ? 1 : 0;
        for (int q = 0; q < NC; ++q) cw->rho[q] = rho[q];
      }
    }
    cur.alpha[c] = alpha;
    cur.gamma[c] = g;
  }
  if (stop) return;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const double un = r_next(grw[t].x, s_next(grw[t].y, gsd[t].x, beta), alpha) * gsd[t].y;
    acc = __builtin_fma(av[t], un, acc);
  }
  const double sn = s_next(w_o, s_o, beta);
  const double pn = __builtin_fma(beta, p_o, r_o * d_o);
  const double rnw = r_next(r_o, sn, alpha);
  const double un = rnw * d_o;
  double v[3] = {0.0, 0.0, 0.0};
  if (live) {
    a.p[o] = pn;
    a.x[o] = __builtin_fma(alpha, pn, x_o);
    *reinterpret_cast<double2*>(&nxt[ii].r) = make_double2(rnw, acc);
    *reinterpret_cast<double2*>(&nxt[ii].s) = make_double2(sn, d_o);
    v[0] = rnw * un;
    v[1] = acc * un;
    v[2] = rnw * rnw;
  }
  block_sum<3>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) a.part[par ^ 1][((size_t)c * a.nbx + blockIdx.x) * 3 + k] = v[k];
}

// the launch of the padded row length w (1..ELL_MAX)
inline const void* relax_iter_kernel(int w) {
  switch (w) {
    case 1: return (const void*)k_relax_iter<1>;
    case 2: return (const void*)k_relax_iter<2>;
    case 3: return (const void*)k_relax_iter<3>;
    case 4: return (const void*)k_relax_iter<4>;
    case 5: return (const void*)k_relax_iter<5>;
    case 6: return (const void*)k_relax_iter<6>;
    case 7: return (const void*)k_relax_iter<7>;
    case 8: return (const void*)k_relax_iter<8>;
    case 9: return (const void*)k_relax_iter<9>;
    case 10: return (const void*)k_relax_iter<10>;
    case 11: return (const void*)k_relax_iter<11>;
    case 12: return (const void*)k_relax_iter<12>;
    case 13: return (const void*)k_relax_iter<13>;
    case 14: return (const void*)k_relax_iter<14>;
    case 15: return (const void*)k_relax_iter<15>;
    case 16: return (const void*)k_relax_iter<16>;
    default: return nullptr;
  }
}

// ---------------------------------------------------------------------------
// The projection's solve: the same iteration for one component, with the
// two-level preconditioner M^-1 = D^-1 + Z E^+ Z^T (Z: the aggregates'
// indicator vectors, E = Z^T K Z; host::build_coarse), so u = D^-1 r + c with
// c = E^+ Z^T r constant on each aggregate.  The aggregate sums of r_{i+1}
// follow the recurrences of the unknowns, Z^T r_{i+1} = Z^T r_i - alpha (Z^T
// w_i + beta Z^T s_{i-1}), from aggregate partials of the previous launch,
// so every block forms them and the correction of the aggregates it needs
// (the same products in the same order in every block, so a neighbour's
// value is exactly its owner's) without another synchronisation; the owner
// keeps its aggregates' correction for the next launch (cglob).

// The sums over the two 32-lane halves of a wavefront (every lane active;
// the same two values in every lane): DPP within rows of 16, then the two
// rows of each half.
__device__ __forceinline__ void half_sums(double v, double& lo, double& hi) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  lo = read_lane(v, 0) + read_lane(v, 16);
  hi = read_lane(v, 32) + read_lane(v, 48);
}

// This thread's share of the E^+ rows of its block's need list: entry
// threadIdx / TPE, the JMAX columns from JMAX (threadIdx % TPE) on, in
// 16-byte loads.  The rows sit in a copy per block, so the addresses need no
// index load first.
constexpr int JV = JMAX / 4;
__device__ __forceinline__ void coarse_rows(const Args& a, float4 (&ev)[JV]) {
  const int e = threadIdx.x / TPE, q = threadIdx.x % TPE;
  const float4* er = reinterpret_cast<const float4*>(a.ep + ((size_t)blockIdx.x * NEED + e) * NA_MAX + JMAX * q);
#pragma unroll
  for (int j = 0; j < JV; ++j) ev[j] = er[j];
}

// c = E^+ v on the need list into csh[NEED] (vw: the wavefront's copy of v
// for every aggregate, zero past na): four running sums per thread, then the
// TPE threads of an entry meet by DPP within a quad, so all of them hold the
// same sum; a fixed order, the same in every block.  Every thread of the
// block calls it; csh is complete after the next block barrier.
__device__ __forceinline__ void coarse_product(const float4 (&ev)[JV], const double* vw, double* csh) {
  const int q = threadIdx.x % TPE;
  const double* v = vw + JMAX * q;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < JV; ++j) {
    const double2 v01 = *reinterpret_cast<const double2*>(v + 4 * j);
    const double2 v23 = *reinterpret_cast<const double2*>(v + 4 * j + 2);
    acc[0] = __builtin_fma((double)ev[j].x, v01.x, acc[0]);
    acc[1] = __builtin_fma((double)ev[j].y, v01.y, acc[1]);
    acc[2] = __builtin_fma((double)ev[j].z, v23.x, acc[2]);
    acc[3] = __builtin_fma((double)ev[j].w, v23.y, acc[3]);
  }
  double t = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  static_assert(TPE == 4, "the quad exchange sums four threads");
  t += dpp_move<0xB1>(t);
  t += dpp_move<0x4E>(t);
  if (q == 0) csh[threadIdx.x / TPE] = t;
}

// The aggregate sums of three values per unknown (zero past nc) into dst
// (na x 3), by lane 0 of each wavefront for its two aggregates.
__device__ __forceinline__ void aggregate_sums(const Args& a, const double (&v)[3], double* dst) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int g0 = (blockIdx.x * BLK + (threadIdx.x - lane)) / AGG;
  // the three exchanges step by step side by side, then the stores
  double t[3], lo[3], hi[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) t[m] = v[m] + dpp_move<0xB1>(v[m]);
#pragma unroll
  for (int m = 0; m < 3; ++m) t[m] += dpp_move<0x4E>(t[m]);
#pragma unroll
  for (int m = 0; m < 3; ++m) t[m] += dpp_move<0x141>(t[m]);
#pragma unroll
  for (int m = 0; m < 3; ++m) t[m] += dpp_move<0x140>(t[m]);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    lo[m] = read_lane(t[m], 0) + read_lane(t[m], 16);
    hi[m] = read_lane(t[m], 32) + read_lane(t[m], 48);
  }
  if (lane == 0) {
    if (g0 < a.na)
      for (int m = 0; m < 3; ++m) dst[(size_t)g0 * 3 + m] = lo[m];
    if (g0 + 1 < a.na)
      for (int m = 0; m < 3; ++m) dst[(size_t)(g0 + 1) * 3 + m] = hi[m];
  }
}

// start: r0 = b - A x0 (component 0), p = 0, s = 0, and the block partials
// of the sum of r0 (in the second component's slots of pbb)
__global__ __launch_bounds__(BLK) void k_proj_start1(Args a) {
  const int i = blockIdx.x * BLK + threadIdx.x, nc = a.nc;
  double sr[1] = {0.0};
  if (i < nc) {
    double bv = 0.0;
    for (int t = a.incptr[i]; t < a.incptr[i + 1]; ++t) {
      const int e = a.inc[t] / 3, l = a.inc[t] - 3 * e;
      bv += a.S[(size_t)l * a.ne + e];
    }
    double ax = 0.0;
    for (int t = 0; t < a.ellw; ++t) ax = __builtin_fma(a.aval[t * nc + i], a.x[a.ecol[t * nc + i]], ax);
    Rec& q = a.rec[0][i];
    q.r = bv - ax;
    q.s = 0.0;
    q.d = a.dinv[i];
    a.p[i] = 0.0;
    sr[0] = bv - ax;
  }
  block_sum<1>(sr);
  if (threadIdx.x == 0) a.pbb[(size_t)a.nbx + blockIdx.x] = sr[0];
}

// start: the mean of r0 taken off.  The system is singular (pure Neumann and
// periodic sides: the constants span its null space) and its range is the
// vectors of zero sum; the load sums to zero only up to rounding, and the
// bordered form that fixes the mean of phi solves with the load's mean
// removed, which is what this does (every block totals the partials in the
// same order, so all take the same mean).  Then the (r0, r0) partials, the
// solve's reference, and the aggregate sums of r0 (and of s_{-1} = 0).
__global__ __launch_bounds__(BLK) void k_proj_center(Args a) {
  const int i = blockIdx.x * BLK + threadIdx.x, nc = a.nc, lane = threadIdx.x & (WAVE - 1);
  double ts[1] = {0.0}, tot[1];
  for (int bx = lane; bx < a.nbx; bx += WAVE) ts[0] += a.pbb[(size_t)a.nbx + bx];
  wave_sums<1>(ts, tot);
  const double mean = tot[0] / nc;
  double bb[1] = {0.0};
  double g[3] = {0.0, 0.0, 0.0};
  if (i < nc) {
    Rec& q = a.rec[0][i];
    const double r = q.r - mean;
    q.r = r;
    bb[0] = r * r;
    g[0] = r;
  }
  if (a.na > 0) aggregate_sums(a, g, a.agp[0]);   // r0, (w0 from the next launch), s_{-1} = 0
  block_sum<1>(bb);
  if (threadIdx.x == 0) a.pbb[blockIdx.x] = bb[0];
}

// start: the coarse correction c0 of r0, u0 = D^-1 r0 + c0, w0 = A u0, the
// partials of iteration 0 and the aggregate sums of w0
__global__ __launch_bounds__(BLK) void k_proj_start2(Args a) {
  __shared__ double vsh[WPB][NA_MAX];
  __shared__ double csh[NEED];
  const int i = blockIdx.x * BLK + threadIdx.x, nc = a.nc, lane = threadIdx.x & (WAVE - 1);
  const bool live = i < nc;
  const int ii = live ? i : nc - 1;
  Rec* r0 = a.rec[0];
  const int own = ii / AGG - blockIdx.x * APB;
  double c0 = 0.0;
  if (a.na > 0) {
    float4 ev[JV];
    coarse_rows(a, ev);
    double* vw = vsh[threadIdx.x / WAVE];
    for (int k = 0; k < NA_MAX / WAVE; ++k) {
      const int g = lane + WAVE * k;
      vw[g] = g < a.na ? a.agp[0][(size_t)g * 3] : 0.0;
    }
    lds_sync_wave();
    coarse_product(ev, vw, csh);
    __syncthreads();
    c0 = csh[own];
  }
  double acc = 0.0;
  for (int t = 0; t < a.ellw; ++t) {
    const int k = a.ecol[t * nc + ii];
    const int e = a.eneed[t * nc + ii] & (NEED - 1);
    const double ck = a.na > 0 ? csh[e] : 0.0;
    acc = __builtin_fma(a.aval[t * nc + ii], __builtin_fma(r0[k].r, r0[k].d, ck), acc);
  }
  const double ri = r0[ii].r, ui = __builtin_fma(ri, r0[ii].d, c0);
  double v[3] = {0.0, 0.0, 0.0};
  double g[3] = {0.0, 0.0, 0.0};
  if (live) {
    r0[ii].w = acc;
    v[0] = ri * ui;
    v[1] = acc * ui;
    v[2] = ri * ri;
    g[1] = acc;
    if (a.na > 0 && ii % AGG == 0) a.cglob[0][ii / AGG] = c0;
  }
  if (a.na > 0) {
    const int lane0 = threadIdx.x - lane;
    const int g0 = (blockIdx.x * BLK + lane0) / AGG;
    double lo, hi;
    half_sums(g[1], lo, hi);
    if (lane == 0) {
      if (g0 < a.na) a.agp[0][(size_t)g0 * 3 + 1] = lo;
      if (g0 + 1 < a.na) a.agp[0][(size_t)(g0 + 1) * 3 + 1] = hi;
    }
  }
  block_sum<3>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) a.part[0][(size_t)blockIdx.x * 3 + k] = v[k];
  if (blockIdx.x != 0) return;
  double tot[NC][1];
  total_partials<1>(a, a.pbb, tot);
  if (threadIdx.x == 0) {
    a.ctl->ref[0] = tot[0][0];   // (r0, r0) where b = 0: set by iteration 0
    for (int q = 1; q < NC; ++q) a.ctl->ref[q] = 0.0;
  }
}

// iteration i of the projection's solve (parity par): as k_relax_iter for
// component 0, with u = D^-1 r + c
template <int W> __global__ __launch_bounds__(BLK) void k_proj_iter(Args a, int par) {
  __shared__ double vsh[WPB][NA_MAX];
  __shared__ double csh[NEED];
  const int nc = a.nc, lane = threadIdx.x & (WAVE - 1);
  const int i = blockIdx.x * BLK + threadIdx.x;
  const bool live = i < nc;
  const int ii = live ? i : nc - 1;
  const bool co = a.na > 0;
  const Rec* old = a.rec[par];
  Rec* nxt = a.rec[par ^ 1];
  int cl[W], en[W];
  double av[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    cl[t] = a.ecol[t * nc + ii];
    av[t] = a.aval[t * nc + ii];
    // loaded whether or not co: the compiler ends a load under a branch with
    // a wait for every load in flight
    en[t] = a.eneed[t * nc + ii] & (NEED - 1);
  }
  const double2 rw_o = *reinterpret_cast<const double2*>(&old[ii].r);
  const double2 sd_o = *reinterpret_cast<const double2*>(&old[ii].s);
  const double r_o = rw_o.x, w_o = rw_o.y, s_o = sd_o.x, d_o = sd_o.y, p_o = a.p[ii], x_o = a.x[ii];
  const int own = ii / AGG - blockIdx.x * APB;
  const double c_o = co ? a.cglob[par][ii / AGG] : 0.0;
  // this thread's share of the E^+ rows: no index load before them, so they
  // go out with the first round
  float4 ev[JV];
  if (co) coarse_rows(a, ev);
  const Ctl* ctl = a.ctl;
  const Scal& prev = ctl->sc[par ^ 1];
  const int pdone = prev.done, it = prev.iter, max_iters = ctl->max_iters;
  const double gold = prev.gamma[0], aold = prev.alpha[0], tol2 = ctl->tol2, ref = ctl->ref[0];
  // partials of the blocks lane, lane + 64, ... (a fixed order per lane)
  const double* src = a.part[par];
  double tp[3];
  {
    const int bx = lane < a.nbx ? lane : 0;
    const double keep = lane < a.nbx ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) tp[k] = keep * src[(size_t)bx * 3 + k];
  }
  // the neighbours' values
  double2 grw[W], gsd[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const int k = cl[t];
    grw[t] = *reinterpret_cast<const double2*>(&old[k].r);
    gsd[t] = *reinterpret_cast<const double2*>(&old[k].s);
  }
  for (int bx = lane + WAVE; bx < a.nbx; bx += WAVE)
#pragma unroll
    for (int k = 0; k < 3; ++k) tp[k] += src[(size_t)bx * 3 + k];
  if (pdone) return;
  // aggregate sums of r_i, w_i, s_{i-1} (aggregates lane + 64 k): issued
  // behind the stop test, so in the second round with the neighbours' values
  // (a wavefront keeps at most 63 loads in flight)
  double ag[NA_MAX / WAVE][3];
  if (co) {
#pragma unroll
    for (int k = 0; k < NA_MAX / WAVE; ++k) {
      const int g = lane + WAVE * k;
      const bool in = g < a.na;
#pragma unroll
      for (int m = 0; m < 3; ++m) ag[k][m] = in ? a.agp[par][(size_t)g * 3 + m] : 0.0;
    }
  }
  double tot[3];
  wave_sums<3>(tp, tot);
  // where b = 0 the reference is (r0, r0), known from iteration 0 on
  const double rq = ref > 0.0 ? ref : (it == 0 ? tot[2] : ref);
  const bool ok = tot[2] <= tol2 * rq;
  const double g = tot[0], d = tot[1];
  const double beta = gold != 0.0 ? g / gold : 0.0;
  const double den = aold != 0.0 ? d - beta * g / aold : d;
  const double alpha = den != 0.0 ? g / den : 0.0;
  const bool stop = ok || it >= max_iters;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl* cw = a.ctl;
    Scal& cur = cw->sc[par];
    cur.iter = it + 1;
    cur.done = stop ? 1 : 0;
    if (it == 0 && !(ref > 0.0)) cw->ref[0] = tot[2];
    if (stop) {
      cw->iter = it;
      cw->done = 1;
      cw->converged = ok ? 1 : 0;
      cw->rho[0] = tot[2];
      for (int q = 1; q < NC; ++q) cw->rho[q] = 0.0;
    }
    cur.alpha[0] = alpha;
    cur.gamma[0] = g;
  }
  if (stop) return;
  // the coarse correction of r_{i+1} on the need list
  double c_n = 0.0;
  if (co) {
    // every wavefront forms Z^T r_{i+1} in its own copy
    double* vw = vsh[threadIdx.x / WAVE];
#pragma unroll
    for (int k = 0; k < NA_MAX / WAVE; ++k) vw[lane + WAVE * k] = r_next(ag[k][0], s_next(ag[k][1], ag[k][2], beta), alpha);
    lds_sync_wave();
    coarse_product(ev, vw, csh);
    __syncthreads();
    c_n = csh[own];
  }
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const double ck = co ? csh[en[t]] : 0.0;
    const double un = __builtin_fma(r_next(grw[t].x, s_next(grw[t].y, gsd[t].x, beta), alpha), gsd[t].y, ck);
    acc = __builtin_fma(av[t], un, acc);
  }
  const double sn = s_next(w_o, s_o, beta);
  const double pn = __builtin_fma(beta, p_o, __builtin_fma(r_o, d_o, c_o));
  const double rnw = r_next(r_o, sn, alpha);
  const double un = __builtin_fma(rnw, d_o, c_n);
  double v[3] = {0.0, 0.0, 0.0};
  double gsum[3] = {0.0, 0.0, 0.0};
  if (live) {
    a.p[ii] = pn;
    a.x[ii] = __builtin_fma(alpha, pn, x_o);
    *reinterpret_cast<double2*>(&nxt[ii].r) = make_double2(rnw, acc);
    *reinterpret_cast<double2*>(&nxt[ii].s) = make_double2(sn, d_o);
    v[0] = rnw * un;
    v[1] = acc * un;
    v[2] = rnw * rnw;
    gsum[0] = rnw;
    gsum[1] = acc;
    gsum[2] = sn;
    if (co && ii % AGG == 0) a.cglob[par ^ 1][ii / AGG] = c_n;
  }
  if (co) aggregate_sums(a, gsum, a.agp[par ^ 1]);
  block_sum<3>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) a.part[par ^ 1][(size_t)blockIdx.x * 3 + k] = v[k];
}

// the projection's launch of the padded row length w (1..ELL_MAX)
inline const void* proj_iter_kernel(int w) {
  switch (w) {
    case 1: return (const void*)k_proj_iter<1>;
    case 2: return (const void*)k_proj_iter<2>;
    case 3: return (const void*)k_proj_iter<3>;
    case 4: return (const void*)k_proj_iter<4>;
    case 5: return (const void*)k_proj_iter<5>;
    case 6: return (const void*)k_proj_iter<6>;
    case 7: return (const void*)k_proj_iter<7>;
    case 8: return (const void*)k_proj_iter<8>;
    case 9: return (const void*)k_proj_iter<9>;
    case 10: return (const void*)k_proj_iter<10>;
    case 11: return (const void*)k_proj_iter<11>;
    case 12: return (const void*)k_proj_iter<12>;
    case 13: return (const void*)k_proj_iter<13>;
    case 14: return (const void*)k_proj_iter<14>;
    case 15: return (const void*)k_proj_iter<15>;
    case 16: return (const void*)k_proj_iter<16>;
    default: return nullptr;
  }
}

// ---------------------------------------------------------------------------
// Mean-pressure projection (closing summary of section 2.2; section 3: the
// mean-pressure Poisson equation on the grid by finite elements).  The
// pressure increment phi solves lap(phi) = div<U> / dt with d(phi)/dn =
// <U>.n / dt at walls, in the Galerkin form K phi = (1/dt) sum_e area_e
// <U>_e . grad(psi_i)|_e (the same unknowns, seams and solver as the
// relaxation, no mass term; the load sums to zero, so the singular system
// is consistent); the mean pressure gradient gains grad(phi) averaged to the
// vertices by area, and every particle's velocity loses dt grad(phi) of its
// element.

// the P1 shape-function gradients of element e (2A grad(psi_k) = (y_{k+1} -
// y_{k+2}, x_{k+2} - x_{k+1})) and its area
__device__ __forceinline__ double shape_grads(const Args& a, int e, double (&gx)[3], double (&gy)[3]) {
  double x[3], y[3];
  for (int k = 0; k < 3; ++k) {
    x[k] = a.vtx[2 * a.tri[3 * e + k]];
    y[k] = a.vtx[2 * a.tri[3 * e + k] + 1];
  }
  const double a2 = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
  for (int k = 0; k < 3; ++k) {
    gx[k] = (y[(k + 1) % 3] - y[(k + 2) % 3]) / a2;
    gy[k] = (x[(k + 2) % 3] - x[(k + 1) % 3]) / a2;
  }
  return 0.5 * a2;
}

// per element: the mean velocity (the particles', the frozen one at the
// centroid under N_MIN particles) and its load on the element's three
// vertices; L^2 = 1
__global__ __launch_bounds__(BLK) void k_proj_inputs(Args a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  bool est = false;
  if (e < a.ne) {
    const double* rec = a.stats + (size_t)e * a.nstat;
    est = rec[ST_N] >= (double)N_MIN;
    double U, V;
    if (est) {
      U = rec[ST_MEAN];
      V = rec[ST_MEAN + 1];
    } else {
      const double* f0 = a.fields + (size_t)a.tri[3 * e] * NFIELD;
      const double* f1 = a.fields + (size_t)a.tri[3 * e + 1] * NFIELD;
      const double* f2 = a.fields + (size_t)a.tri[3 * e + 2] * NFIELD;
      U = (f0[F_U] + f1[F_U] + f2[F_U]) / 3.0;
      V = (f0[F_V] + f1[F_V] + f2[F_V]) / 3.0;
    }
    double gx[3], gy[3];
    const double area = shape_grads(a, e, gx, gy);
    for (int k = 0; k < 3; ++k) a.S[(size_t)k * a.ne + e] = area * (U * gx[k] + V * gy[k]) / a.dt;
    a.L2[e] = 1.0;
  }
  const uint64_t m = __ballot(est);
  if ((threadIdx.x & (WAVE - 1)) == 0 && m) atomicAdd(&a.ctl->from_stats, (int)__popcll(m));
}

// The kernels below do nothing before the stop or after k_proj_done has
// marked the update applied, so the host may enqueue them behind any batch
// of iterations and they act once per solve.

// grad(phi) per element into Rk rows 0 and 1
__global__ __launch_bounds__(BLK) void k_proj_grad(Args a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.ne || !a.ctl->done || a.ctl->applied) return;
  double gx[3], gy[3];
  (void)shape_grads(a, e, gx, gy);
  double px = 0.0, py = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double ph = a.x[a.canon[a.tri[3 * e + k]]];
    px += ph * gx[k];
    py += ph * gy[k];
  }
  a.Rk[e] = px;
  a.Rk[(size_t)a.ne + e] = py;
}

// per vertex: grad(phi) averaged by area over the unknown's elements, added
// to the mean pressure gradient (fields and the coefficient table);
// phi_out (V, may be null): phi (up to a constant); grad_out (V x 2, may be
// null): the vertex gradient
template <typename T>
__global__ __launch_bounds__(BLK) void k_proj_apply(Args a, T* coef, double* phi_out, double* grad_out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.nv || !a.ctl->done || a.ctl->applied) return;
  const int c = a.canon[v];
  double ws = 0.0, gx = 0.0, gy = 0.0;
  for (int t = a.incptr[c]; t < a.incptr[c + 1]; ++t) {
    const int e = a.inc[t] / 3;
    const double w = a.area[e];
    ws += w;
    gx += w * a.Rk[e];
    gy += w * a.Rk[(size_t)a.ne + e];
  }
  gx /= ws;
  gy /= ws;
  double* f = a.fields_rw + (size_t)v * NFIELD;
  f[F_DPDX] += gx;
  f[F_DPDY] += gy;
  coef[(size_t)v * NCOEF + C_DPDX] = (T)f[F_DPDX];
  coef[(size_t)v * NCOEF + C_DPDY] = (T)f[F_DPDY];
  if (phi_out) phi_out[v] = a.x[c];
  if (grad_out) {
    grad_out[2 * (size_t)v] = gx;
    grad_out[2 * (size_t)v + 1] = gy;
  }
}

// every particle of ensemble 0 (one wavefront per element): velocity less
// dt grad(phi) of its element, in double, rounded to the state type
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_proj_particles(Args a, StateDev<T> b0, StateDev<T> b1, CounterSets cs,
                                                          const int32_t* start, const int32_t* cap,
                                                          const pdf::Ctl* sctl, StepIndex si) {
  const int e = blockIdx.x * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
  if (e >= a.ne || !a.ctl->done || a.ctl->applied) return;
  const StateDev<T> st = (si.parity ^ (sctl->flip & 1u)) ? b1 : b0;
  const int capc = cap[e], s0 = start[e];
  const int ns = min(cs.ns[si.rot][e], capc);
  const int nm = min(cs.nm[si.rot][e], capc - ns);
  const double du = a.dt * a.Rk[e], dv = a.dt * a.Rk[(size_t)a.ne + e];
  for (int j = lane_id(); j < ns + nm; j += WAVE) {
    const int s = slot_of(j, s0, ns, nm, capc);
    st.u[s] = (T)((double)st.u[s] - du);
    st.v[s] = (T)((double)st.v[s] - dv);
  }
}

// marks the projection's update applied once the solve has stopped
__global__ void k_proj_done(Ctl* ctl) {
  if (threadIdx.x == 0 && ctl->done) ctl->applied = 1;
}

// ---------------------------------------------------------------------------
// G and C0 per vertex (eqs. 12-13) into the coefficient table.
// wp_out (V x 5, may be null): wp at every vertex; coef_out (V x 6, may be
// null): G_11 G_12 G_21 G_22 G_33 C0 eps before rounding to the table's type

template <typename T>
__global__ __launch_bounds__(BLK) void k_relax_coef(Args a, T* coef, double* wp_out, double* coef_out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  bool neg = false;
  if (v < a.nv) {
    const int c = a.canon[v];
    const int ne = a.ne, nc = a.nc;
    double ws = 0.0, r11 = 0.0, r22 = 0.0, r33 = 0.0, r12 = 0.0;
    for (int t = a.incptr[c]; t < a.incptr[c + 1]; ++t) {
      const int e = a.inc[t] / 3;
      const double w = a.area[e];
      ws += w;
      r11 += w * a.Rk[0 * ne + e];
      r22 += w * a.Rk[1 * ne + e];
      r33 += w * a.Rk[2 * ne + e];
      r12 += w * a.Rk[3 * ne + e];
    }
    r11 /= ws; r22 /= ws; r33 /= ws; r12 /= ws;
    const double k = 0.5 * (r11 + r22 + r33);
    const double eps = a.fields[(size_t)v * NFIELD + F_EPS];
    const double w11 = a.x[0 * (size_t)nc + c], w12 = a.x[1 * (size_t)nc + c], w21 = a.x[2 * (size_t)nc + c];
    const double w22 = a.x[3 * (size_t)nc + c], w33 = a.x[4 * (size_t)nc + c];
    const double k2 = 2.0 * k;
    const double g11 = (2.0 * w11 - eps) / k2, g12 = (2.0 * w12) / k2, g21 = (2.0 * w21) / k2;
    const double g22 = (2.0 * w22 - eps) / k2, g33 = (2.0 * w33 - eps) / k2;
    const double wr = w11 * r11 + w12 * r12 + w21 * r12 + w22 * r22 + w33 * r33;
    double C0 = -2.0 * wr / (3.0 * k * eps);
    if (C0 < 0.0) {
      C0 = 0.0;
      neg = true;
    }
    T* q = coef + (size_t)v * NCOEF;
    q[C_G11] = (T)g11;
    q[C_G12] = (T)g12;
    q[C_G21] = (T)g21;
    q[C_G22] = (T)g22;
    q[C_G33] = (T)g33;
    q[C_C0EPS] = (T)(C0 * eps);
    if (coef_out) {
      double* o = coef_out + 6 * (size_t)v;
      o[0] = g11; o[1] = g12; o[2] = g21; o[3] = g22; o[4] = g33; o[5] = C0 * eps;
    }
    if (wp_out) {
      double* o = wp_out + 5 * (size_t)v;
      o[0] = w11; o[1] = w12; o[2] = w21; o[3] = w22; o[4] = w33;
    }
  }
  const uint64_t m = __ballot(neg);
  if ((threadIdx.x & (WAVE - 1)) == 0 && m) atomicAdd(&a.ctl->clamped, (int)__popcll(m));
}

}  // namespace relax
}  // namespace pdf
