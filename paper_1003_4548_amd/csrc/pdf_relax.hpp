// Elliptic relaxation (section 2.1): the tensor wp of eq. (14) from the
// particle statistics, by Galerkin P1 finite elements on the mesh and a
// Jacobi-preconditioned conjugate-gradient solve, then G and C0 of eqs.
// (12)-(13) per vertex into the coefficient table the step reads.
//
//   wp_ij - L^2 lap wp_ij = 1/2 (1 - C1) k <omega> delta_ij + k H_ijkl d<U_k>/dx_l
//
// H of eq. (15) with A_v of eq. (16) and b of eq. (17); L of eq. (18).  The
// unknowns are the mesh vertices with the two copies of a periodic-seam
// vertex joined; L^2 and the right-hand side are constant per element; every
// wall carries the natural (zero normal derivative) condition.  The five
// components wp_11, wp_12, wp_21, wp_22, wp_33 share the matrix and are
// solved together; vectors are stored component-major (5 x nc doubles).
//
// Determinism: the matrix entries are gathered per nonzero from a fixed list
// of element contributions; every inner product is a fixed-order sum of
// per-block partial sums, which every block of the next kernel recomputes
// identically (no atomics on floating point).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdf_kernels.hpp"

namespace pdf {
namespace relax {

constexpr int NC = 5;            // solved components
constexpr int BLK = 256;         // threads per block of the solver kernels
constexpr int MAX_BLOCKS = 1024; // blocks of a solver launch (nc <= MAX_BLOCKS * BLK)
constexpr int N_MIN = 10;        // fewer particles: the element takes the frozen stresses
// Table 2
constexpr double C1 = 1.85, C2 = 0.63, CT = 6.0, CL = 0.134, CETA = 72.0, CV = 1.4, GAMMA5 = 0.1;
constexpr double C_XI = 2.3;     // 1 + 1.3 n_i n_i with a unit normal n

struct Args {
  // mesh (device)
  int32_t ne, nv, nc;
  const int32_t* tri;      // ne x 3
  const double* fields;    // nv x NFIELD (frozen)
  const int32_t* canon;    // nv: unknown of each vertex
  const int32_t* rowptr;   // nc + 1
  const int32_t* col;      // nnz
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
  // work (device)
  double* S;               // 5 x ne right-hand side per element
  double* L2;              // ne
  double* Rk;              // 5 x ne: R11 R22 R33 R12 and the count of particles used (0: frozen)
  double* aval;            // nnz
  double* diag;            // nc
  double* x;               // 5 x nc (the solution; the previous one is the first guess)
  double* r;               // 5 x nc
  double* z;               // 5 x nc
  double* q;               // 5 x nc
  double* p[2];            // 5 x nc each
  double* part;            // MAX_BLOCKS x 3 x 5 partial sums: p.q, r.z, r.r
  double* hist;            // (max_iters + 2) x 5: r.z of every iteration
  int32_t* flag;           // [0] done, [1] iterations, [2] C0 clamped, [3] elements from statistics
  double* res;             // 10: r.r and b.b per component at exit
  double tol2;             // squared relative residual bound
  int32_t nblk;            // blocks of the solver launches
  int32_t max_iters;
};

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
// per element: stresses, k, <omega>, L^2 and the right-hand side of eq. (14)

__global__ void k_relax_inputs(Args a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.ne) return;
  const double* f0 = a.fields + (size_t)a.tri[3 * e] * NFIELD;
  const double* f1 = a.fields + (size_t)a.tri[3 * e + 1] * NFIELD;
  const double* f2 = a.fields + (size_t)a.tri[3 * e + 2] * NFIELD;
  auto cen = [&](int j) { return (f0[j] + f1[j] + f2[j]) / 3.0; };
  const double* rec = a.stats + (size_t)e * a.nstat;
  double r11, r22, r33, r12;
  const bool est = rec[ST_N] >= (double)N_MIN;
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
  const double g00 = cen(F_DUDX), g01 = cen(F_DUDY), g10 = cen(F_DVDX), g11 = cen(F_DVDY);
  // anisotropy (eq. 17) and A_v (eq. 16); R13 = R23 = 0
  const double b00 = r11 / tr - 1.0 / 3.0, b11 = r22 / tr - 1.0 / 3.0, b01 = r12 / tr;
  const double det = r33 * (r11 * r22 - r12 * r12);
  const double k23 = 2.0 * k / 3.0;
  const double Av = fmin(1.0, CV * det / (k23 * k23 * k23));
  // H_ijkl g_kl (eq. 15) for the five components; b_ik g_kl sums over k, l
  // in {x, y} (the spanwise row and column of the gradient vanish)
  const double a1 = C2 * Av + GAMMA5 / 3.0;
  const double g[2][2] = {{g00, g01}, {g10, g11}};
  const double b[2][2] = {{b00, b01}, {b01, b11}};
  auto hterm = [&](int i, int j) {
    // (C2 Av + g5/3) g_ij - g5/3 g_ji + g5 sum_k b_ik g_kj - g5 sum_l b_il g_jl
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
  a.Rk[4 * ne + e] = est ? rec[ST_N] : 0.0;
}

// ---------------------------------------------------------------------------
// matrix entries per row (M + L^2 K gathered from the element contributions)
// and its diagonal; the right-hand side and the first residual

__global__ void k_relax_matrix(Args a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nc) return;
  for (int j = a.rowptr[i]; j < a.rowptr[i + 1]; ++j) {
    double v = 0.0;
    for (int t = a.cptr[j]; t < a.cptr[j + 1]; ++t) {
      const int c = a.cidx[t];
      const int e = c / 9, ab = c - 9 * e, aa = ab / 3, bb = ab - 3 * aa;
      const double m = a.area[e] / 12.0 * (aa == bb ? 2.0 : 1.0);
      v += m + a.L2[e] * a.Ke[9 * e + ab];
    }
    a.aval[j] = v;
    if (a.col[j] == i) a.diag[i] = v;
  }
}

// block sums of NV values per thread in a fixed tree; thread 0 holds the totals
template <int NV> __device__ void block_sum(double (&v)[NV], double (*sh)[BLK]) {
  const int t = threadIdx.x;
  for (int c = 0; c < NV; ++c) sh[c][t] = v[c];
  __syncthreads();
  for (int s = BLK / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int c = 0; c < NV; ++c) sh[c][t] = sh[c][t] + sh[c][t + s];
    __syncthreads();
  }
  for (int c = 0; c < NV; ++c) v[c] = sh[c][0];
  __syncthreads();
}

// the global sums of one kind of partial (0 p.q, 1 r.z, 2 r.r), the same
// fixed-order sum in every block
__device__ void global_sum(const Args& a, int kind, double (&out)[NC], double (*sh)[BLK]) {
  double v[NC];
  for (int c = 0; c < NC; ++c) v[c] = 0.0;
  for (int b = threadIdx.x; b < a.nblk; b += BLK)
    for (int c = 0; c < NC; ++c) v[c] += a.part[(size_t)(b * 3 + kind) * NC + c];
  block_sum<NC>(v, sh);
  for (int c = 0; c < NC; ++c) out[c] = v[c];
}

// r = b - A x, z = r / diag, partials of r.z and r.r; b.b into hist[0]'s
// neighbour slot (hist row 0 holds b.b, the iterations start at row 1)
__global__ __launch_bounds__(BLK) void k_relax_start(Args a) {
  __shared__ double sh[3 * NC][BLK];
  const int i = blockIdx.x * BLK + threadIdx.x;
  const int nc = a.nc;
  double rz[NC], rr[NC], bb[NC];
  for (int c = 0; c < NC; ++c) rz[c] = rr[c] = bb[c] = 0.0;
  if (i < nc) {
    double bv[NC];
    for (int c = 0; c < NC; ++c) bv[c] = 0.0;
    for (int t = a.incptr[i]; t < a.incptr[i + 1]; ++t) {
      const int e = a.inc[t] / 3;
      const double w = a.area[e] / 3.0;
      for (int c = 0; c < NC; ++c) bv[c] += a.S[(size_t)c * a.ne + e] * w;
    }
    double ax[NC];
    for (int c = 0; c < NC; ++c) ax[c] = 0.0;
    for (int j = a.rowptr[i]; j < a.rowptr[i + 1]; ++j) {
      const double v = a.aval[j];
      const int cj = a.col[j];
      for (int c = 0; c < NC; ++c) ax[c] += v * a.x[(size_t)c * nc + cj];
    }
    const double dinv = 1.0 / a.diag[i];
    for (int c = 0; c < NC; ++c) {
      const double rv = bv[c] - ax[c];
      const double zv = rv * dinv;
      a.r[(size_t)c * nc + i] = rv;
      a.z[(size_t)c * nc + i] = zv;
      rz[c] = rv * zv;
      rr[c] = rv * rv;
      bb[c] = bv[c] * bv[c];
    }
  }
  block_sum<NC>(rz, sh);
  block_sum<NC>(rr, sh + NC);
  block_sum<NC>(bb, sh + 2 * NC);
  if (threadIdx.x == 0) {
    for (int c = 0; c < NC; ++c) {
      a.part[(size_t)(blockIdx.x * 3 + 1) * NC + c] = rz[c];
      a.part[(size_t)(blockIdx.x * 3 + 2) * NC + c] = rr[c];
      a.part[(size_t)(blockIdx.x * 3 + 0) * NC + c] = bb[c];   // b.b, summed once by the next kernel
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) a.flag[k] = 0;
}

// b.b from the start kernel's partials into hist[0] (one block)
__global__ __launch_bounds__(BLK) void k_relax_norm(Args a) {
  __shared__ double sh[NC][BLK];
  double bb[NC];
  global_sum(a, 0, bb, sh);
  if (threadIdx.x == 0)
    for (int c = 0; c < NC; ++c) a.hist[c] = bb[c];
}

// the done flag as one value for the whole block (read by one thread)
__device__ bool block_done(const Args& a) {
  __shared__ int done;
  if (threadIdx.x == 0) done = a.flag[0];
  __syncthreads();
  const bool d = done != 0;
  __syncthreads();
  return d;
}

// converged when r.r <= tol2 b.b for every component (a zero right-hand side
// converges at once)
__device__ bool converged(const Args& a, double (*sh)[BLK]) {
  double rr[NC];
  global_sum(a, 2, rr, sh);
  bool ok = true;
  for (int c = 0; c < NC; ++c) ok = ok && rr[c] <= a.tol2 * a.hist[c];
  return ok;
}

// iteration it, first half: beta from r.z, the new direction p (into the
// other buffer), q = A p, partials of p.q
__global__ __launch_bounds__(BLK) void k_relax_cg_a(Args a, int it) {
  __shared__ double sh[NC][BLK];
  if (block_done(a)) return;
  if (converged(a, sh)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.flag[0] = 1;
      a.flag[1] = it;
    }
    return;
  }
  double rz[NC];
  global_sum(a, 1, rz, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int c = 0; c < NC; ++c) a.hist[(size_t)(it + 1) * NC + c] = rz[c];
  double beta[NC];
  for (int c = 0; c < NC; ++c) {
    const double old = it == 0 ? 0.0 : a.hist[(size_t)it * NC + c];
    beta[c] = old != 0.0 ? rz[c] / old : 0.0;   // a component already at r = 0 keeps p = z
  }
  const double* po = a.p[it & 1];
  double* pn = a.p[(it + 1) & 1];
  const int nc = a.nc;
  const int i = blockIdx.x * BLK + threadIdx.x;
  double pq[NC];
  for (int c = 0; c < NC; ++c) pq[c] = 0.0;
  if (i < nc) {
    double qv[NC];
    for (int c = 0; c < NC; ++c) qv[c] = 0.0;
    for (int j = a.rowptr[i]; j < a.rowptr[i + 1]; ++j) {
      const double v = a.aval[j];
      const int cj = a.col[j];
      for (int c = 0; c < NC; ++c) qv[c] += v * (a.z[(size_t)c * nc + cj] + beta[c] * po[(size_t)c * nc + cj]);
    }
    for (int c = 0; c < NC; ++c) {
      const double pv = a.z[(size_t)c * nc + i] + beta[c] * po[(size_t)c * nc + i];
      pn[(size_t)c * nc + i] = pv;
      a.q[(size_t)c * nc + i] = qv[c];
      pq[c] = pv * qv[c];
    }
  }
  block_sum<NC>(pq, sh);
  if (threadIdx.x == 0)
    for (int c = 0; c < NC; ++c) a.part[(size_t)(blockIdx.x * 3 + 0) * NC + c] = pq[c];
}

// iteration it, second half: alpha, x += alpha p, r -= alpha q, z = r / diag,
// partials of r.z and r.r
__global__ __launch_bounds__(BLK) void k_relax_cg_b(Args a, int it) {
  __shared__ double sh[NC][BLK];
  if (block_done(a)) return;
  double pq[NC];
  global_sum(a, 0, pq, sh);
  double alpha[NC];
  for (int c = 0; c < NC; ++c) {
    const double rz = a.hist[(size_t)(it + 1) * NC + c];
    alpha[c] = pq[c] != 0.0 ? rz / pq[c] : 0.0;
  }
  const double* pn = a.p[(it + 1) & 1];
  const int nc = a.nc;
  const int i = blockIdx.x * BLK + threadIdx.x;
  double rz[NC], rr[NC];
  for (int c = 0; c < NC; ++c) rz[c] = rr[c] = 0.0;
  if (i < nc) {
    const double dinv = 1.0 / a.diag[i];
    for (int c = 0; c < NC; ++c) {
      const size_t o = (size_t)c * nc + i;
      a.x[o] = a.x[o] + alpha[c] * pn[o];
      const double rv = a.r[o] - alpha[c] * a.q[o];
      const double zv = rv * dinv;
      a.r[o] = rv;
      a.z[o] = zv;
      rz[c] = rv * zv;
      rr[c] = rv * rv;
    }
  }
  block_sum<NC>(rz, sh);
  __shared__ double sh2[NC][BLK];
  block_sum<NC>(rr, sh2);
  if (threadIdx.x == 0) {
    for (int c = 0; c < NC; ++c) {
      a.part[(size_t)(blockIdx.x * 3 + 1) * NC + c] = rz[c];
      a.part[(size_t)(blockIdx.x * 3 + 2) * NC + c] = rr[c];
    }
  }
}

// after the iterations the host enqueued (one block): r.r and b.b of every
// component into res; convergence recorded if the loop ran out first
__global__ __launch_bounds__(BLK) void k_relax_finish(Args a, int iters) {
  __shared__ double sh[NC][BLK];
  double rr[NC];
  global_sum(a, 2, rr, sh);
  if (threadIdx.x == 0) {
    bool ok = true;
    for (int c = 0; c < NC; ++c) {
      a.res[c] = rr[c];
      a.res[NC + c] = a.hist[c];
      ok = ok && rr[c] <= a.tol2 * a.hist[c];
    }
    if (!a.flag[0]) {
      a.flag[0] = ok ? 1 : 0;
      a.flag[1] = iters;
    }
  }
}

// ---------------------------------------------------------------------------
// G and C0 per vertex (eqs. 12-13) into the coefficient table

// wp_out (V x 5, may be null): wp at every vertex; coef_out (V x 6, may be
// null): G_11 G_12 G_21 G_22 G_33 C0 eps before rounding to the table's type
template <typename T> __global__ void k_relax_coef(Args a, T* coef, double* wp_out, double* coef_out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.nv) return;
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
  T* q = coef + (size_t)v * NCOEF;
  q[C_G11] = (T)((2.0 * w11 - eps) / k2);
  q[C_G12] = (T)((2.0 * w12) / k2);
  q[C_G21] = (T)((2.0 * w21) / k2);
  q[C_G22] = (T)((2.0 * w22 - eps) / k2);
  q[C_G33] = (T)((2.0 * w33 - eps) / k2);
  const double wr = w11 * r11 + w12 * r12 + w21 * r12 + w22 * r22 + w33 * r33;
  double C0 = -2.0 * wr / (3.0 * k * eps);
  if (C0 < 0.0) {
    C0 = 0.0;
    atomicAdd(&a.flag[2], 1);
  }
  q[C_C0EPS] = (T)(C0 * eps);
  if (coef_out) {
    double* o = coef_out + 6 * (size_t)v;
    o[0] = (2.0 * w11 - eps) / k2;
    o[1] = (2.0 * w12) / k2;
    o[2] = (2.0 * w21) / k2;
    o[3] = (2.0 * w22 - eps) / k2;
    o[4] = (2.0 * w33 - eps) / k2;
    o[5] = C0 * eps;
  }
  if (wp_out) {
    wp_out[5 * (size_t)v + 0] = w11;
    wp_out[5 * (size_t)v + 1] = w12;
    wp_out[5 * (size_t)v + 2] = w21;
    wp_out[5 * (size_t)v + 3] = w22;
    wp_out[5 * (size_t)v + 4] = w33;
  }
}

// elements whose stresses came from the statistics (one block)
__global__ __launch_bounds__(BLK) void k_relax_count(Args a) {
  __shared__ int cnt[BLK];
  int n = 0;
  for (int e = threadIdx.x; e < a.ne; e += BLK) n += a.Rk[4 * a.ne + e] > 0.0 ? 1 : 0;
  cnt[threadIdx.x] = n;
  __syncthreads();
  for (int s = BLK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.flag[3] = cnt[0];
}

}  // namespace relax
}  // namespace pdf
