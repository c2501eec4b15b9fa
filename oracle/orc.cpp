// Oracle for the particle-in-cell joint velocity-scalar PDF step.
//
// TEST INFRASTRUCTURE ONLY: a plain CPU implementation used by the tests, the
// smoke check and the CPU baseline to check the GPU library.  Nothing in the
// product path loads it.  It shares no code with the GPU library.
//
// Paper: Bakosi, Franzese & Boybeyi, "Joint PDF modelling of turbulent flow
// and dispersion in an urban street canyon".  Equation numbers count the
// displayed equations in order: (5) particle position, (6) particle velocity
// (GLM), (7) IECM, (8) dissipation from frequency, (11) micro-mixing time,
// (12)-(13) drift tensor and C0 from the elliptic-relaxation tensor, (19) SLM,
// (20)-(26) wall-function particle conditions.
//
// Readings of points the paper leaves open are listed in the design notes and
// repeated at the place they are used.  Every function below follows its
// definition directly: no blocking, fusion or reordering.  Floating point:
// no contraction by the compiler; a fused multiply-add appears only where
// it is written out (std::fma: the Horner steps of the series, the P1
// interpolation, the IECM, velocity, frequency and position updates), so
// that an implementation in another language can repeat every rounding.
#include "orc.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Counter-based random numbers.  Philox4x32-10 as published by Salmon, Moraes,
// Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten
// rounds of two 32x32->64 multiplications with Weyl-sequence key bumps.

const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Uniform deviates in (0,1), exactly representable: float from the top 23
// bits, double from all 32 bits, each offset by half a grid step.
inline float uniform_f(uint32_t r) { return (float)(r >> 9) * 0x1p-23f + 0x1p-24f; }
inline double uniform_d(uint32_t r) { return (double)r * 0x1p-32 + 0x1p-33; }

// Natural logarithm from its series.  x = m 2^e with m in [sqrt(1/2),
// sqrt(2)); log m = 2 atanh(s), s = (m-1)/(m+1), atanh s = s + s^3/3 + s^5/5
// + ... (Abramowitz & Stegun 4.1.27 / 4.6.22), truncated where the next term
// falls below the type's half ulp: through s^21 in double, s^11 in float.
template <typename T> struct LogTerms;
template <> struct LogTerms<double> { static const int K = 10; };
template <> struct LogTerms<float> { static const int K = 5; };

template <typename T> T series_log(T x) {
  int e0 = 0;
  T f = std::frexp(x, &e0);  // x = f 2^e0, f in [1/2, 1)
  T m;
  int e;
  const T sqrt_half = (T)0.70710678118654752440;
  if (f < sqrt_half) {
    m = f + f;
    e = e0 - 1;
  } else {
    m = f;
    e = e0;
  }
  T s = (m - (T)1) / (m + (T)1);
  T z = s * s;
  const int K = LogTerms<T>::K;
  T p = (T)1 / (T)(2 * K + 1);
  for (int j = K - 1; j >= 1; --j) p = std::fma(p, z, (T)1 / (T)(2 * j + 1));
  T t = std::fma(s, z * p, s);
  T lm = t + t;
  const T ln2 = (T)0.69314718055994530942;
  return std::fma((T)e, ln2, lm);
}

// sin and cos of 2 pi t.  The turn t is split exactly into a quarter-turn
// count q and a remainder r in [-1/8, 1/8]; the remainder angle 2 pi r is
// expanded in Taylor series (through th^15 / th^16 in double, th^9 / th^10 in
// float) and rotated by q quarter turns.
template <typename T> struct TrigTerms;
template <> struct TrigTerms<double> { static const int S = 7, C = 8; };
template <> struct TrigTerms<float> { static const int S = 4, C = 5; };

template <typename T> T inv_factorial(int n) {
  T f = (T)1;
  for (int i = 2; i <= n; ++i) f = f * (T)i;  // exact for the orders used
  return (T)1 / f;
}

template <typename T> void series_sincos2pi(T t, T* s_out, T* c_out) {
  T q = std::floor(t * (T)4 + (T)0.5);
  T r = t - q * (T)0.25;
  const T two_pi = (T)6.28318530717958647692;
  T th = r * two_pi;
  T z = th * th;
  // sin th = th + th z (-1/3! + z (1/5! - z (...)))
  const int NS = TrigTerms<T>::S;
  T ps = ((NS % 2) ? (T)-1 : (T)1) * inv_factorial<T>(2 * NS + 1);
  for (int j = NS - 1; j >= 1; --j) {
    T cj = ((j % 2) ? (T)-1 : (T)1) * inv_factorial<T>(2 * j + 1);
    ps = std::fma(ps, z, cj);
  }
  T sn = std::fma(th, z * ps, th);
  // cos th = 1 + z (-1/2! + z (1/4! - ...))
  const int NC = TrigTerms<T>::C;
  T pc = ((NC % 2) ? (T)-1 : (T)1) * inv_factorial<T>(2 * NC);
  for (int j = NC - 1; j >= 1; --j) {
    T cj = ((j % 2) ? (T)-1 : (T)1) * inv_factorial<T>(2 * j);
    pc = std::fma(pc, z, cj);
  }
  T cs = std::fma(z, pc, (T)1);
  int qi = ((int)q) & 3;
  switch (qi) {
    case 0: *s_out = sn; *c_out = cs; break;
    case 1: *s_out = cs; *c_out = -sn; break;
    case 2: *s_out = -sn; *c_out = -cs; break;
    default: *s_out = -cs; *c_out = sn; break;
  }
}

// Cube root by Newton's method on y^3 = x, twelve fixed iterations from
// 2^(e/3) (x = f 2^e).
double newton_cbrt(double x) {
  int e = 0;
  std::frexp(x, &e);
  double y = std::ldexp(1.0, e / 3);
  for (int i = 0; i < 12; ++i) y = (y + y + x / (y * y)) / 3.0;
  return y;
}

// Normal deviates of one particle step: Philox block b (b = 0, 1) with counter
// (id, step, b, ensemble) and key (seed low, seed high) gives four words; the
// Box-Muller transform (Box & Muller 1958) maps word pairs (0,1), (2,3), (4,5),
// (6,7) to normal pairs.  Arithmetic in the state type.
template <typename T> T uniform_t(uint32_t r);
template <> float uniform_t<float>(uint32_t r) { return uniform_f(r); }
template <> double uniform_t<double>(uint32_t r) { return uniform_d(r); }

template <typename T> void box_muller(uint32_t r1, uint32_t r2, T* z0, T* z1) {
  T u1 = uniform_t<T>(r1), u2 = uniform_t<T>(r2);
  T rad = std::sqrt((T)-2 * series_log<T>(u1));
  T sn, cs;
  series_sincos2pi<T>(u2, &sn, &cs);
  *z0 = rad * cs;
  *z1 = rad * sn;
}

template <typename T> void step_normals(uint64_t seed, uint32_t id, uint32_t step, uint32_t ens,
                                        T xi[8]) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t r[8];
  for (uint32_t b = 0; b < 2; ++b) {
    uint32_t ctr[4] = {id, step, b, ens};
    philox(ctr, key, r + 4 * b);
  }
  for (int p = 0; p < 4; ++p) box_muller<T>(r[2 * p], r[2 * p + 1], &xi[2 * p], &xi[2 * p + 1]);
}

const uint32_t SEED_STEP = 0xFFFFFFFFu;  // step counter word of the initial draw

// ---------------------------------------------------------------------------
// geometry

// (b - a) x (p - a): twice the signed area of (a, b, p), positive when p lies
// to the left of a -> b; one fused multiply-add after the second product.
inline double orient2d(double ax, double ay, double bx, double by, double px, double py) {
  return std::fma(bx - ax, py - ay, -((by - ay) * (px - ax)));
}

enum { NF = 20, NC = 16 };
enum { F_U, F_V, F_DUDX, F_DUDY, F_DVDX, F_DVDY, F_LAPU, F_LAPV, F_DPDX, F_DPDY,
       F_R11, F_R22, F_R33, F_R12, F_EPS, F_P11, F_P12, F_P21, F_P22, F_P33 };
enum { C_U, C_V, C_DUDX, C_DUDY, C_DVDX, C_DVDY, C_LAPU, C_LAPV, C_DPDX, C_DPDY,
       C_G11, C_G12, C_G21, C_G22, C_G33, C_C0EPS };

template <typename T> struct Ens {
  uint64_t seed = 0;
  double x0 = 0, y0 = 0, r0 = 0;
  std::vector<int64_t> counts;
  std::vector<T> x, y, u, v, w, psi;
  std::vector<int32_t> elem;
  std::vector<double> rate;  // IECM relaxation factor per element, min(dt/t_m, 1)
  std::vector<double> cm;    // conditional means from elsewhere (nelem x 8), empty: binned
  std::vector<T> om;         // turbulent frequency (when enabled)
};

}  // namespace

struct orc_ctx {
  orc_params p;
  int32_t nv = 0, ne = 0;
  std::vector<double> vtx;
  std::vector<int32_t> tri, nbr, ekind;
  std::vector<double> fields;
  std::vector<double> inv2a;   // 1 / (2 area) per element
  std::vector<double> coef;    // per-vertex coefficient table, double
  std::vector<double> alpha;   // wall-function alpha per element edge
  std::vector<double> om0;     // frozen <omega> per element (centroid)
  std::vector<double> somega;  // S_omega per element (centroid), eq. (10)
  std::vector<double> omw;     // frozen <omega> at wall-function edge midpoints
  int64_t wf_hits = 0;         // particle steps whose frequency a wall condition changed
  std::vector<Ens<float>> ensF;
  std::vector<Ens<double>> ensD;
  int64_t step = 0;
  // time averaging: the statistics record of every step since the start,
  // per ensemble (kept whole; combined when asked for)
  bool averaging = false;
  std::vector<std::vector<std::vector<double>>> avg_rec;
};

namespace {

double vx(const orc_ctx* c, int v) { return c->vtx[2 * v]; }
double vy(const orc_ctx* c, int v) { return c->vtx[2 * v + 1]; }

// Orientation of point p against edge k of element e (positive inside).  The
// edge is evaluated from its lexicographically smaller endpoint, so the two
// elements that share an edge always get exactly opposite values.
double orient_edge(const orc_ctx* c, int e, int k, double px, double py) {
  int a = c->tri[3 * e + k], b = c->tri[3 * e + (k + 1) % 3];
  double ax = vx(c, a), ay = vy(c, a), bx = vx(c, b), by = vy(c, b);
  bool a_first = (ax < bx) || (ax == bx && ay < by);
  if (a_first) return orient2d(ax, ay, bx, by, px, py);
  return -orient2d(bx, by, ax, ay, px, py);
}

// Barycentric coordinates of p in element e.
void barycentric(const orc_ctx* c, int e, double px, double py, double lam[3]) {
  double ia = c->inv2a[e];
  lam[0] = orient_edge(c, e, 1, px, py) * ia;
  lam[1] = orient_edge(c, e, 2, px, py) * ia;
  lam[2] = orient_edge(c, e, 0, px, py) * ia;
}

// <omega> from eq. (8), eps = <omega>(k + nu C_T^2 <omega>), solved for the
// positive root.
double mean_omega(double k, double eps, double nu, double CT) {
  return 2.0 * eps / (k + std::sqrt(k * k + 4.0 * nu * CT * CT * eps));
}

void build_coefficients(orc_ctx* c) {
  const orc_params& p = c->p;
  c->coef.assign((size_t)c->nv * NC, 0.0);
  for (int i = 0; i < c->nv; ++i) {
    const double* f = &c->fields[(size_t)i * NF];
    double* q = &c->coef[(size_t)i * NC];
    for (int j = 0; j < 10; ++j) q[j] = f[j];  // mean velocity, gradients, Laplacian, pressure gradient
    double k = 0.5 * ((f[F_R11] + f[F_R22]) + f[F_R33]);
    double eps = f[F_EPS];
    if (p.model == 0) {
      // SLM, eq. (19): G_ij = -(1/2 + 3/4 C0) <omega> delta_ij, C0 constant
      double om = mean_omega(k, eps, p.nu, p.CT);
      double g = -(0.5 + 0.75 * p.C0) * om;
      q[C_G11] = g; q[C_G12] = 0.0; q[C_G21] = 0.0; q[C_G22] = g; q[C_G33] = g;
      q[C_C0EPS] = p.C0 * eps;
    } else {
      // eq. (12): G_ij = (2 wp_ij - eps delta_ij) / (2k)
      double k2 = 2.0 * k;
      q[C_G11] = (2.0 * f[F_P11] - eps) / k2;
      q[C_G12] = (2.0 * f[F_P12]) / k2;
      q[C_G21] = (2.0 * f[F_P21]) / k2;
      q[C_G22] = (2.0 * f[F_P22] - eps) / k2;
      q[C_G33] = (2.0 * f[F_P33] - eps) / k2;
      // eq. (13): C0 = -2 wp_ij <u_i u_j> / (3 k eps)
      double wr = f[F_P11] * f[F_R11] + f[F_P12] * f[F_R12];
      wr = wr + f[F_P21] * f[F_R12];
      wr = wr + f[F_P22] * f[F_R22];
      wr = wr + f[F_P33] * f[F_R33];
      double C0 = -2.0 * wr / (3.0 * k * eps);
      q[C_C0EPS] = C0 * eps;
    }
  }
}

// Micro-mixing time scale, eq. (11), evaluated once per element at its
// centroid from the frozen k, eps and <U>; the IECM relaxation factor of one
// Euler step is r = min(dt / t_m, 1).  Without a source (r0 = 0) the first
// argument of the minimum is absent.
void build_rates(const orc_ctx* c, Ens<float>* ef, Ens<double>* ed) {
  const orc_params& p = c->p;
  double x0 = ef ? ef->x0 : ed->x0, y0 = ef ? ef->y0 : ed->y0, r0 = ef ? ef->r0 : ed->r0;
  std::vector<double>& rate = ef ? ef->rate : ed->rate;
  rate.assign(c->ne, 0.0);
  for (int e = 0; e < c->ne; ++e) {
    int v0 = c->tri[3 * e], v1 = c->tri[3 * e + 1], v2 = c->tri[3 * e + 2];
    const double* f0 = &c->fields[(size_t)v0 * NF];
    const double* f1 = &c->fields[(size_t)v1 * NF];
    const double* f2 = &c->fields[(size_t)v2 * NF];
    double xc = ((vx(c, v0) + vx(c, v1)) + vx(c, v2)) / 3.0;
    double yc = ((vy(c, v0) + vy(c, v1)) + vy(c, v2)) / 3.0;
    double k0 = 0.5 * ((f0[F_R11] + f0[F_R22]) + f0[F_R33]);
    double k1 = 0.5 * ((f1[F_R11] + f1[F_R22]) + f1[F_R33]);
    double k2 = 0.5 * ((f2[F_R11] + f2[F_R22]) + f2[F_R33]);
    double k = ((k0 + k1) + k2) / 3.0;
    double eps = ((f0[F_EPS] + f1[F_EPS]) + f2[F_EPS]) / 3.0;
    double U = ((f0[F_U] + f1[F_U]) + f2[F_U]) / 3.0;
    double V = ((f0[F_V] + f1[F_V]) + f2[F_V]) / 3.0;
    double second = std::max(k / eps, p.CT * std::sqrt(p.nu / eps));
    double tm = second;
    if (r0 > 0.0) {
      double Uc = std::sqrt(U * U + V * V);
      double dx = xc - x0, dy = yc - y0;
      double dist = std::sqrt(dx * dx + dy * dy);
      double first = p.Cs * newton_cbrt(r0 * r0 / eps);
      if (Uc >= 1e-12) {
        first = first + p.Ct * dist / Uc;
        tm = std::min(first, second);
      }
      // U_c = 0: the advection term is unbounded and the second argument wins
    }
    rate[e] = std::min(p.dt / tm, 1.0);
  }
}

// Wall-function coefficient alpha, eqs. (22)-(26), per wall-function edge.
// The statistics at the first grid point are the frozen fields at the edge
// midpoint, rotated into the edge frame (tangent t, inward normal n).
void build_alpha(orc_ctx* c) {
  const orc_params& p = c->p;
  c->alpha.assign((size_t)c->ne * 3, 0.0);
  for (int e = 0; e < c->ne; ++e) {
    for (int k = 0; k < 3; ++k) {
      if (c->ekind[3 * e + k] != ORC_EDGE_WALLFN) continue;
      int a = c->tri[3 * e + k], b = c->tri[3 * e + (k + 1) % 3];
      double ex = vx(c, b) - vx(c, a), ey = vy(c, b) - vy(c, a);
      double len = std::sqrt(ex * ex + ey * ey);
      double nx = ey / len, ny = -ex / len;       // outward normal
      double tx = -ny, ty = nx;                   // tangent
      double nix = -nx, niy = -ny;                // inward normal
      const double* fa = &c->fields[(size_t)a * NF];
      const double* fb = &c->fields[(size_t)b * NF];
      double U = (fa[F_U] + fb[F_U]) / 2.0, V = (fa[F_V] + fb[F_V]) / 2.0;
      double R11 = (fa[F_R11] + fb[F_R11]) / 2.0, R22 = (fa[F_R22] + fb[F_R22]) / 2.0;
      double R33 = (fa[F_R33] + fb[F_R33]) / 2.0, R12 = (fa[F_R12] + fb[F_R12]) / 2.0;
      double Px = (fa[F_DPDX] + fb[F_DPDX]) / 2.0, Py = (fa[F_DPDY] + fb[F_DPDY]) / 2.0;
      double Up = U * tx + V * ty;                                       // <U>_p
      double v2 = (nix * R11 + niy * R12) * nix + (nix * R12 + niy * R22) * niy;  // <v^2>_p
      double uv = (tx * R11 + ty * R12) * nix + (tx * R12 + ty * R22) * niy;      // <uv>_p
      double dPdx = Px * tx + Py * ty;                                   // streamwise dP/dx
      double kp = 0.5 * ((R11 + R22) + R33);
      double uhat = std::sqrt(std::sqrt(p.Cmu)) * std::sqrt(kp);         // eq. (23)
      double prod = uv * dPdx;
      double gamma_tau = prod > 0.0 ? 1.0 : 0.0;                         // eq. (26)
      double ustar = std::sqrt(uhat * uhat + gamma_tau * std::fabs(p.yp * dPdx));  // eq. (25)
      double Ue = ustar / p.kappa * series_log<double>(p.Ewall * p.yp * ustar / p.nu);  // eq. (24)
      double al = 2.0 * uhat * uhat * Up * std::fabs(Up) / (v2 * Ue * Ue);           // eq. (22)
      c->alpha[3 * e + k] = al;
    }
  }
}

// exp x = 2^k exp r with k = rint(x / ln 2) and r = x - k ln 2 (ln 2 split in
// a high part with trailing zero bits and a low part, Cody & Waite), exp r
// by its Taylor series through r^13 (|r| <= ln 2 / 2) in Horner form.
double exp_series(double x) {
  const double LN2_HI = 0x1.62e42fefa3800p-1, LN2_LO = 0x1.ef35793c76730p-45;
  const double k = std::rint(x * 0x1.71547652b82fep0);
  const double r = (x - k * LN2_HI) - k * LN2_LO;
  double fact = 1.0;
  for (int j = 2; j <= 13; ++j) fact = fact * (double)j;
  double p = 1.0 / fact;                       // 1/13!
  for (int j = 12; j >= 1; --j) {
    fact = fact / (double)(j + 1);             // j!
    p = p * r + 1.0 / fact;
  }
  p = p * r + 1.0;
  return std::ldexp(p, (int)k);
}

// Turbulent frequency: per element the frozen <omega> at the centroid (eq. 8
// solved) and S_omega = C_w2 - C_w1 P / eps (eq. 10) with the production
// P = -<u_i u_j> d<U_i>/dx_j of the frozen fields at the centroid; per
// wall-function edge the frozen <omega> at its midpoint (y_p), for eq. (27).
void build_omega(orc_ctx* c) {
  const orc_params& p = c->p;
  c->om0.assign(c->ne, 0.0);
  c->somega.assign(c->ne, 0.0);
  c->omw.assign((size_t)c->ne * 3, 0.0);
  for (int e = 0; e < c->ne; ++e) {
    int v0 = c->tri[3 * e], v1 = c->tri[3 * e + 1], v2 = c->tri[3 * e + 2];
    const double* f0 = &c->fields[(size_t)v0 * NF];
    const double* f1 = &c->fields[(size_t)v1 * NF];
    const double* f2 = &c->fields[(size_t)v2 * NF];
    auto cen = [&](int j) { return ((f0[j] + f1[j]) + f2[j]) / 3.0; };
    double k = 0.5 * ((cen(F_R11) + cen(F_R22)) + cen(F_R33));
    double eps = cen(F_EPS);
    double prod = -((cen(F_R11) * cen(F_DUDX) + cen(F_R12) * cen(F_DUDY)) +
                    (cen(F_R12) * cen(F_DVDX) + cen(F_R22) * cen(F_DVDY)));
    c->om0[e] = mean_omega(k, eps, p.nu, p.CT);
    c->somega[e] = p.Cw2 - p.Cw1 * (prod / eps);
    for (int q = 0; q < 3; ++q) {
      if (c->ekind[3 * e + q] != ORC_EDGE_WALLFN) continue;
      int a = c->tri[3 * e + q], b = c->tri[3 * e + (q + 1) % 3];
      const double* fa = &c->fields[(size_t)a * NF];
      const double* fb = &c->fields[(size_t)b * NF];
      double kp = 0.5 * (((fa[F_R11] + fb[F_R11]) / 2.0 + (fa[F_R22] + fb[F_R22]) / 2.0) + (fa[F_R33] + fb[F_R33]) / 2.0);
      double ep = (fa[F_EPS] + fb[F_EPS]) / 2.0;
      c->omw[3 * e + q] = mean_omega(kp, ep, p.nu, p.CT);
    }
  }
}

// ---------------------------------------------------------------------------
// particle tracking (closing summary of section 2.2: the grid is used to track particles)
//
// Straight-line neighbour walk from the start point S (inside the current
// element) toward the target T.  Exit edge: the first edge (lowest local
// index) that T lies outside of and whose endpoints the line S-T separates;
// if rounding leaves none, the edge T is most outside of.  Walls mirror the
// rest of the path about the wall line and reflect the velocity; periodic
// edges move the path by one period into the partner element.

template <typename T> T toward(T x, double dir) {
  return std::nextafter(x, dir > 0 ? std::numeric_limits<T>::infinity()
                                   : -std::numeric_limits<T>::infinity());
}

template <typename T>
int walk(const orc_ctx* c, int e, double Sx, double Sy, T& tx, T& ty, T& u, T& v, T& w, int* nref,
         T* om = nullptr) {
  for (int it = 0; it < 64; ++it) {
    double Tx = (double)tx, Ty = (double)ty;
    double o[3];
    for (int k = 0; k < 3; ++k) o[k] = orient_edge(c, e, k, Tx, Ty);
    if (o[0] >= 0.0 && o[1] >= 0.0 && o[2] >= 0.0) return e;
    int ex = -1;
    for (int k = 0; k < 3 && ex < 0; ++k) {
      if (!(o[k] < 0.0)) continue;
      int a = c->tri[3 * e + k], b = c->tri[3 * e + (k + 1) % 3];
      double sa = orient2d(Sx, Sy, Tx, Ty, vx(c, a), vy(c, a));
      double sb = orient2d(Sx, Sy, Tx, Ty, vx(c, b), vy(c, b));
      if ((sa <= 0.0 && sb >= 0.0) || (sa >= 0.0 && sb <= 0.0)) ex = k;
    }
    if (ex < 0) {
      ex = 0;
      for (int k = 1; k < 3; ++k)
        if (o[k] < o[ex]) ex = k;
    }
    int kind = c->ekind[3 * e + ex];
    if (kind == ORC_EDGE_INTERIOR) {
      e = c->nbr[3 * e + ex];
      continue;
    }
    if (kind >= ORC_EDGE_PXP) {
      double sx = 0.0, sy = 0.0;
      if (kind == ORC_EDGE_PXP) sx = c->p.Lx;
      if (kind == ORC_EDGE_PXM) sx = -c->p.Lx;
      if (kind == ORC_EDGE_PYP) sy = c->p.Ly;
      if (kind == ORC_EDGE_PYM) sy = -c->p.Ly;
      Sx = Sx + sx;
      Sy = Sy + sy;
      tx = tx + (T)sx;
      ty = ty + (T)sy;
      e = c->nbr[3 * e + ex];
      continue;
    }
    // wall: mirror the target about the wall line, restart from the crossing
    int a = c->tri[3 * e + ex], b = c->tri[3 * e + (ex + 1) % 3];
    double ax = vx(c, a), ay = vy(c, a);
    double gx = vx(c, b) - ax, gy = vy(c, b) - ay;
    double len = std::sqrt(gx * gx + gy * gy);
    double nx = gy / len, ny = -gx / len;  // outward unit normal
    double oS = orient_edge(c, e, ex, Sx, Sy), oT = o[ex];
    double den = oS - oT;
    double tpar = den > 0.0 ? oS / den : 0.0;
    double Ix = Sx + tpar * (Tx - Sx), Iy = Sy + tpar * (Ty - Sy);
    double d = (Tx - ax) * nx + (Ty - ay) * ny;
    double Rx = Tx - (2.0 * d) * nx, Ry = Ty - (2.0 * d) * ny;
    tx = (T)Rx;
    ty = (T)Ry;
    for (int j = 0; j < 8; ++j) {  // keep the rounded mirror image inside the wall
      if (!(orient_edge(c, e, ex, (double)tx, (double)ty) < 0.0)) break;
      if (nx != 0.0) tx = toward<T>(tx, -nx);
      if (ny != 0.0) ty = toward<T>(ty, -ny);
    }
    Sx = Ix;
    Sy = Iy;
    T nxT = (T)nx, nyT = (T)ny;
    if (kind == ORC_EDGE_NOSLIP) {
      // resolved no-slip wall: all components reversed
      u = -u; v = -v; w = -w;
    } else if (kind == ORC_EDGE_SLIP) {
      // free-slip wall: specular reflection of the normal component
      T un = u * nxT + v * nyT;
      T un2 = un + un;
      u = u - un2 * nxT;
      v = v - un2 * nyT;
    } else {
      // wall functions, eqs. (20)-(21) in the edge frame
      T tX = -nyT, tY = nxT;          // tangent
      T Vi = -(u * nxT + v * nyT);    // wall-normal component, inward positive
      T Ui = u * tX + v * tY;         // tangential component
      T al = (T)c->alpha[3 * e + ex];
      T Ur = Ui + al * Vi;
      T Vr = -Vi;
      u = Ur * tX + Vr * (-nxT);
      v = Ur * tY + Vr * (-nyT);
      // turbulent frequency, eqs. (27)-(28): omega_R = omega_I exp(beta V_I / (y_p <omega>))
      if (om) {
        const double beta = -2.0 / ((((0.5 + 0.75 * c->p.C0) + c->p.C3) + c->p.Cw2) - c->p.Cw1);
        const double arg = beta * (double)Vi / (c->p.yp * c->omw[3 * e + ex]);
        *om = (T)((double)(*om) * exp_series(arg));
      }
    }
    if (nref) ++(*nref);
  }
  return -1;
}

// ---------------------------------------------------------------------------
// seeding: uniform positions in each element, Gaussian velocities with the
// local mean and Reynolds stress, initial scalar by rule.

template <typename T> void seed_ensemble(orc_ctx* c, Ens<T>& en, uint32_t ens_index) {
  int64_t n = 0;
  for (int e = 0; e < c->ne; ++e) n += en.counts[e];
  en.x.assign(n, 0); en.y.assign(n, 0); en.u.assign(n, 0); en.v.assign(n, 0);
  if (c->p.omega) en.om.assign(n, 0);
  en.w.assign(n, 0); en.psi.assign(n, 0); en.elem.assign(n, 0);
  uint32_t key[2] = {(uint32_t)en.seed, (uint32_t)(en.seed >> 32)};
  int64_t id = 0;
  for (int e = 0; e < c->ne; ++e) {
    int v0 = c->tri[3 * e], v1 = c->tri[3 * e + 1], v2 = c->tri[3 * e + 2];
    double ax = vx(c, v0), ay = vy(c, v0);
    double bx = vx(c, v1) - ax, by = vy(c, v1) - ay;
    double cx = vx(c, v2) - ax, cy = vy(c, v2) - ay;
    double gx = ((vx(c, v0) + vx(c, v1)) + vx(c, v2)) / 3.0;
    double gy = ((vy(c, v0) + vy(c, v1)) + vy(c, v2)) / 3.0;
    for (int64_t j = 0; j < en.counts[e]; ++j, ++id) {
      uint32_t r[8];
      for (uint32_t blk = 0; blk < 2; ++blk) {
        uint32_t ctr[4] = {(uint32_t)id, SEED_STEP, blk, ens_index};
        philox(ctr, key, r + 4 * blk);
      }
      double s1 = uniform_d(r[0]), s2 = uniform_d(r[1]);
      if (s1 + s2 > 1.0) {
        s1 = 1.0 - s1;
        s2 = 1.0 - s2;
      }
      double px = ax + s1 * bx + s2 * cx;
      double py = ay + s1 * by + s2 * cy;
      T tx = (T)px, ty = (T)py;
      for (int it = 0; it < 64; ++it) {  // the rounded point must stay in e
        double qx = (double)tx, qy = (double)ty;
        if (orient_edge(c, e, 0, qx, qy) >= 0.0 && orient_edge(c, e, 1, qx, qy) >= 0.0 &&
            orient_edge(c, e, 2, qx, qy) >= 0.0)
          break;
        tx = (T)((qx + gx) / 2.0);
        ty = (T)((qy + gy) / 2.0);
      }
      double z0, z1, z2, z3;
      box_muller<double>(r[2], r[3], &z0, &z1);
      box_muller<double>(r[4], r[5], &z2, &z3);
      double lam[3];
      barycentric(c, e, (double)tx, (double)ty, lam);
      const double* f0 = &c->fields[(size_t)v0 * NF];
      const double* f1 = &c->fields[(size_t)v1 * NF];
      const double* f2 = &c->fields[(size_t)v2 * NF];
      auto interp = [&](int j2) { return (lam[0] * f0[j2] + lam[1] * f1[j2]) + lam[2] * f2[j2]; };
      double U = interp(F_U), V = interp(F_V);
      double R11 = interp(F_R11), R22 = interp(F_R22), R33 = interp(F_R33), R12 = interp(F_R12);
      // Cholesky factor of the Reynolds stress (the 2x2 block and R33)
      double L11 = std::sqrt(R11);
      double L21 = R12 / L11;
      double L22 = std::sqrt(R22 - L21 * L21);
      double L33 = std::sqrt(R33);
      en.x[id] = tx;
      en.y[id] = ty;
      en.u[id] = (T)(U + L11 * z0);
      en.v[id] = (T)(V + (L21 * z0 + L22 * z1));
      en.w[id] = (T)(L33 * z2);
      en.psi[id] = (T)((c->p.psi_init == 1 && (double)tx < 0.25) ? 1.0 : 0.0);
      if (c->p.omega) en.om[id] = (T)c->om0[e];
      en.elem[id] = e;
    }
  }
}

// ---------------------------------------------------------------------------
// statistics: ensemble averages per element over the particles it contains
// (section 2, the closing summary of section 2.2, section 3): count, means, central moments, velocity-binned
// conditional scalar means and the scalar histogram.  Two passes: means
// first, then moments and bins relative to those means.  Sums run over the
// element's particles in particle-id order.

int nstat_of(const orc_params& p) {
  return (p.moments >= 4 ? ORC_NSTAT_4 : ORC_NSTAT_2) + p.hist_bins + (p.omega ? 3 : 0) + (p.vbins == 5 ? 250 : 0);
}

// Five velocity bins per component: equal widths 1.2 sigma on [-3 sigma,
// 3 sigma] about the element mean (edges at +-0.6 and +-1.8 sigma), the
// outermost bins open; sigma from the element's central second moments; with
// sigma = 0 the middle bin.  Bin = k_u + 5 k_v + 25 k_w.  s: the element's
// record.
int fine_component(double u, double mean, double m2) {
  const double sd = std::sqrt(m2);
  if (!(sd > 0.0)) return 2;
  const double z = (u - mean) / sd;
  const double k = std::floor((z + 3.0) / 1.2);
  return k < 0.0 ? 0 : (k > 4.0 ? 4 : (int)k);
}

int fine_bin(double u, double v, double w, const double* s) {
  return fine_component(u, s[ORC_ST_MEAN], s[ORC_ST_M2 + 0]) + 5 * fine_component(v, s[ORC_ST_MEAN + 1], s[ORC_ST_M2 + 4]) +
         25 * fine_component(w, s[ORC_ST_MEAN + 2], s[ORC_ST_M2 + 7]);
}

// offset of the 125 fine-bin counts in the record (means follow)
int fine_offset(const orc_params& p) {
  return (p.moments >= 4 ? ORC_NSTAT_4 : ORC_NSTAT_2) + p.hist_bins + (p.omega ? 3 : 0);
}

template <typename T> void estimate(const orc_ctx* c, const Ens<T>& en, std::vector<double>& st) {
  const orc_params& p = c->p;
  const int ns = nstat_of(p);
  const int ne = c->ne;
  st.assign((size_t)ne * ns, 0.0);
  const int64_t n = (int64_t)en.x.size();
  // particles of each element in id order
  std::vector<int64_t> start(ne + 1, 0), list(n);
  for (int64_t i = 0; i < n; ++i) start[en.elem[i] + 1]++;
  for (int e = 0; e < ne; ++e) start[e + 1] += start[e];
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i) list[fill[en.elem[i]]++] = i;
  }
  // lexicographic index tuples of the third- and fourth-order moments
  std::vector<int> t3, t4;
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b)
      for (int d = b; d < 4; ++d) { t3.push_back(a); t3.push_back(b); t3.push_back(d); }
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b)
      for (int d = b; d < 4; ++d)
        for (int g = d; g < 4; ++g) { t4.push_back(a); t4.push_back(b); t4.push_back(d); t4.push_back(g); }
#pragma omp parallel for schedule(dynamic, 64)
  for (int e = 0; e < ne; ++e) {
    double* s = &st[(size_t)e * ns];
    int64_t cnt = start[e + 1] - start[e];
    if (cnt == 0) continue;
    double sum[4] = {0, 0, 0, 0};
    for (int64_t j = start[e]; j < start[e + 1]; ++j) {
      int64_t i = list[j];
      sum[0] += (double)en.u[i];
      sum[1] += (double)en.v[i];
      sum[2] += (double)en.w[i];
      sum[3] += (double)en.psi[i];
    }
    double mean[4];
    for (int q = 0; q < 4; ++q) mean[q] = sum[q] / (double)cnt;
    // turbulent frequency: mean and variance; eps from <omega> by eq. (8)
    double om_mean = 0.0, om_var = 0.0;
    if (p.omega) {
      double so = 0.0;
      for (int64_t j = start[e]; j < start[e + 1]; ++j) so += (double)en.om[list[j]];
      om_mean = so / (double)cnt;
      for (int64_t j = start[e]; j < start[e + 1]; ++j) {
        double d = (double)en.om[list[j]] - om_mean;
        om_var += d * d;
      }
      om_var = om_var / (double)cnt;
    }
    double m2[10] = {0}, m3[20] = {0}, m4[35] = {0};
    double binn[8] = {0}, bins[8] = {0};
    std::vector<double> hist(p.hist_bins, 0.0);
    for (int64_t j = start[e]; j < start[e + 1]; ++j) {
      int64_t i = list[j];
      double val[4] = {(double)en.u[i], (double)en.v[i], (double)en.w[i], (double)en.psi[i]};
      double d[4];
      for (int q = 0; q < 4; ++q) d[q] = val[q] - mean[q];
      int idx = 0;
      for (int a = 0; a < 4; ++a)
        for (int b = a; b < 4; ++b) m2[idx++] += d[a] * d[b];
      if (p.moments >= 4) {
        for (int t = 0; t < 20; ++t) m3[t] += (d[t3[3 * t]] * d[t3[3 * t + 1]]) * d[t3[3 * t + 2]];
        for (int t = 0; t < 35; ++t)
          m4[t] += ((d[t4[4 * t]] * d[t4[4 * t + 1]]) * d[t4[4 * t + 2]]) * d[t4[4 * t + 3]];
      }
      // velocity bin: sign of each component's fluctuation (strictly above the mean)
      int bin = (val[0] > mean[0] ? 1 : 0) + (val[1] > mean[1] ? 2 : 0) + (val[2] > mean[2] ? 4 : 0);
      binn[bin] += 1.0;
      bins[bin] += val[3];
      if (p.hist_bins > 0) {
        double hpos = std::floor(val[3] * (double)p.hist_bins);
        int hb = hpos < 0.0 ? 0 : (hpos >= (double)p.hist_bins ? p.hist_bins - 1 : (int)hpos);
        hist[hb] += 1.0;
      }
    }
    double dn = (double)cnt;
    s[ORC_ST_N] = dn;
    for (int q = 0; q < 4; ++q) s[ORC_ST_MEAN + q] = mean[q];
    for (int t = 0; t < 10; ++t) s[ORC_ST_M2 + t] = m2[t] / dn;
    for (int b = 0; b < 8; ++b) {
      s[ORC_ST_BINN + b] = binn[b];
      s[ORC_ST_BINM + b] = binn[b] > 0.0 ? bins[b] / binn[b] : mean[3];
    }
    int off = ORC_NSTAT_2;
    if (p.moments >= 4) {
      for (int t = 0; t < 20; ++t) s[ORC_ST_M3 + t] = m3[t] / dn;
      for (int t = 0; t < 35; ++t) s[ORC_ST_M4 + t] = m4[t] / dn;
      off = ORC_NSTAT_4;
    }
    for (int h = 0; h < p.hist_bins; ++h) s[off + h] = hist[h];
    if (p.omega) {
      double* so = s + off + p.hist_bins;
      double kh = 0.5 * ((s[ORC_ST_M2 + 0] + s[ORC_ST_M2 + 4]) + s[ORC_ST_M2 + 7]);
      so[0] = om_mean;
      so[1] = om_var;
      so[2] = om_mean * (kh + (p.nu * (p.CT * p.CT)) * om_mean);
    }
    if (p.vbins == 5) {
      // <phi|V> on 5 x 5 x 5 bins (bins from this record's means and moments)
      double fn[125] = {0}, fs[125] = {0};
      for (int64_t j = start[e]; j < start[e + 1]; ++j) {
        int64_t i = list[j];
        const int b = fine_bin((double)en.u[i], (double)en.v[i], (double)en.w[i], s);
        fn[b] += 1.0;
        fs[b] += (double)en.psi[i];
      }
      double* sf = s + fine_offset(p);
      for (int b = 0; b < 125; ++b) {
        sf[b] = fn[b];
        sf[125 + b] = fn[b] > 0.0 ? fs[b] / fn[b] : mean[3];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// one time step of one ensemble: explicit Euler-Maruyama (closing summary of section 2.2) of the
// position (eq. 5), velocity (eq. 6) and scalar (eq. 7) equations.  Every
// right-hand side uses the state at the start of the step; the statistics are
// those of that state.

template <typename T> int advance(orc_ctx* c, Ens<T>& en, uint32_t ens_index, uint32_t step,
                                  const std::vector<double>& st) {
  const orc_params& p = c->p;
  const int ns = nstat_of(p);
  const T dt = (T)p.dt;
  const T sdt = std::sqrt(dt);
  const T nu2 = (T)(2.0 * p.nu);
  const T s2nu = std::sqrt(nu2);
  const int64_t n = (int64_t)en.x.size();
  int lost = 0;
  int64_t hits = 0;
#pragma omp parallel for schedule(static) reduction(+ : lost, hits)
  for (int64_t i = 0; i < n; ++i) {
    int e = en.elem[i];
    T xi[8];
    step_normals<T>(en.seed, (uint32_t)i, step, ens_index, xi);
    // Eulerian statistics at the particle location: linear interpolation of
    // the frozen vertex fields (section 2, after eq. 7)
    double lam[3];
    barycentric(c, e, (double)en.x[i], (double)en.y[i], lam);
    T l0 = (T)lam[0], l1 = (T)lam[1], l2 = (T)lam[2];
    const double* q0 = &c->coef[(size_t)c->tri[3 * e] * NC];
    const double* q1 = &c->coef[(size_t)c->tri[3 * e + 1] * NC];
    const double* q2 = &c->coef[(size_t)c->tri[3 * e + 2] * NC];
    T f[NC];
    for (int j = 0; j < NC; ++j) f[j] = std::fma(l2, (T)q2[j], std::fma(l1, (T)q1[j], l0 * (T)q0[j]));
    T x = en.x[i], y = en.y[i], u = en.u[i], v = en.v[i], w = en.w[i], psi = en.psi[i];
    // IECM, eq. (7): relax toward the mean scalar of the particle's velocity bin
    if (p.mix && (p.flags & 4)) {
      const double* s = &st[(size_t)e * ns];
      T m;
      if (p.vbins == 5) {
        m = (T)s[fine_offset(p) + 125 + fine_bin((double)u, (double)v, (double)w, s)];
      } else {
        int bin = ((double)u > s[ORC_ST_MEAN] ? 1 : 0) + ((double)v > s[ORC_ST_MEAN + 1] ? 2 : 0) +
                  ((double)w > s[ORC_ST_MEAN + 2] ? 4 : 0);
        m = en.cm.empty() ? (T)s[ORC_ST_BINM + bin] : (T)en.cm[(size_t)e * 8 + bin];
      }
      T r = (T)en.rate[e];
      psi = std::fma(-r, psi - m, psi);
    }
    // velocity, eq. (6)
    T dW1 = sdt * xi[0], dW2 = sdt * xi[1];
    T dWp1 = sdt * xi[2], dWp2 = sdt * xi[3], dWp3 = sdt * xi[4];
    T uf = u - f[C_U], vf = v - f[C_V];
    T sq = std::sqrt(f[C_C0EPS]);
    T au = std::fma(f[C_G12], vf, std::fma(f[C_G11], uf, std::fma(nu2, f[C_LAPU], -f[C_DPDX])));
    T av = std::fma(f[C_G22], vf, std::fma(f[C_G21], uf, std::fma(nu2, f[C_LAPV], -f[C_DPDY])));
    T gu = std::fma(f[C_DUDY], dW2, f[C_DUDX] * dW1), gv = std::fma(f[C_DVDY], dW2, f[C_DVDX] * dW1);
    T un = std::fma(sq, dWp1, std::fma(s2nu, gu, std::fma(au, dt, u)));
    T vn = std::fma(sq, dWp2, std::fma(s2nu, gv, std::fma(av, dt, v)));
    T wn = std::fma(sq, dWp3, std::fma(f[C_G33] * w, dt, w));
    if (!(p.flags & 1)) {
      un = u; vn = v; wn = w;
    }
    // turbulent frequency, eq. (9), with the sixth normal; Euler-Maruyama,
    // reflected at zero (part of sub-step 1).  <omega> is the element's frozen
    // value, the one the velocity model takes (eq. 19): with the fields frozen
    // one <omega> drives both; the particles' own <omega> is estimated and
    // reported, not fed back
    T omn = p.omega ? en.om[i] : (T)0;
    if (p.omega && (p.flags & 1)) {
      const T om = en.om[i];
      const T mw = (T)c->om0[e];
      const T c3 = (T)p.C3, c34 = (T)(2.0 * p.C3 * p.C4), sw = (T)c->somega[e];
      const T drift = std::fma(sw * mw, om, (c3 * mw) * (om - mw));
      const T diff = std::sqrt((c34 * (mw * mw)) * om);
      omn = std::fma(diff, sdt * xi[5], std::fma(-drift, dt, om));
      omn = std::fabs(omn);
    }
    // position, eq. (5), with the velocity at the start of the step
    T xn = std::fma(s2nu, dW1, std::fma(u, dt, x));
    T yn = std::fma(s2nu, dW2, std::fma(v, dt, y));
    int e2 = e;
    if (p.flags & 2) {
      const T om_before = omn;
      e2 = walk<T>(c, e, (double)x, (double)y, xn, yn, un, vn, wn, nullptr, p.omega ? &omn : nullptr);
      if (omn != om_before) hits += 1;
      if (e2 < 0) {
        lost += 1;
        continue;
      }
    } else {
      xn = x; yn = y;
    }
    // source: particles inside the source disc carry unit scalar (section 3)
    if (en.r0 > 0.0 && (p.flags & 8)) {
      double dx = (double)xn - en.x0, dy = (double)yn - en.y0;
      if (dx * dx + dy * dy <= en.r0 * en.r0) psi = (T)1;
    }
    en.x[i] = xn; en.y[i] = yn; en.u[i] = un; en.v[i] = vn; en.w[i] = wn; en.psi[i] = psi;
    if (p.omega) en.om[i] = omn;
    en.elem[i] = e2;
  }
  c->wf_hits += hits;
  return lost ? -5 : 0;
}

template <typename T> int step_all(orc_ctx* c, std::vector<Ens<T>>& ens) {
  if (c->averaging && c->avg_rec.size() < ens.size()) c->avg_rec.resize(ens.size());
  for (size_t k = 0; k < ens.size(); ++k) {
    std::vector<double> st;
    estimate<T>(c, ens[k], st);
    if (c->averaging) c->avg_rec[k].push_back(st);
    int r = advance<T>(c, ens[k], (uint32_t)k, (uint32_t)c->step, st);
    if (r) return r;
  }
  c->step += 1;
  return 0;
}

template <typename T>
void get_state_t(const Ens<T>& en, double* x, double* y, double* u, double* v, double* w,
                        double* psi, int32_t* elem) {
  for (size_t i = 0; i < en.x.size(); ++i) {
    x[i] = en.x[i]; y[i] = en.y[i]; u[i] = en.u[i]; v[i] = en.v[i]; w[i] = en.w[i];
    psi[i] = en.psi[i]; elem[i] = en.elem[i];
  }
}

template <typename T>
void set_state_t(Ens<T>& en, const double* x, const double* y, const double* u,
                        const double* v, const double* w, const double* psi, const int32_t* elem) {
  for (size_t i = 0; i < en.x.size(); ++i) {
    en.x[i] = (T)x[i]; en.y[i] = (T)y[i]; en.u[i] = (T)u[i]; en.v[i] = (T)v[i]; en.w[i] = (T)w[i];
    en.psi[i] = (T)psi[i]; en.elem[i] = elem[i];
  }
}

template <typename T> void get_om_t(const Ens<T>& en, double* om) {
  for (size_t i = 0; i < en.om.size(); ++i) om[i] = (double)en.om[i];
}
template <typename T> void set_om_t(Ens<T>& en, const double* om) {
  for (size_t i = 0; i < en.om.size(); ++i) en.om[i] = (T)om[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

orc_ctx* orc_create(const orc_params* p, int32_t nvert, const double* vtx, int32_t nelem,
                    const int32_t* tri, const int32_t* nbr, const int32_t* ekind,
                    const double* fields) {
  if (!p || nvert <= 0 || nelem <= 0) return nullptr;
  if (!(p->vbins == 2 || p->vbins == 5)) return nullptr;
  orc_ctx* c = new orc_ctx();
  c->p = *p;
  c->nv = nvert;
  c->ne = nelem;
  c->vtx.assign(vtx, vtx + 2 * (size_t)nvert);
  c->tri.assign(tri, tri + 3 * (size_t)nelem);
  c->nbr.assign(nbr, nbr + 3 * (size_t)nelem);
  c->ekind.assign(ekind, ekind + 3 * (size_t)nelem);
  c->fields.assign(fields, fields + (size_t)NF * nvert);
  c->inv2a.resize(nelem);
  for (int e = 0; e < nelem; ++e) {
    int a = tri[3 * e], b = tri[3 * e + 1], d = tri[3 * e + 2];
    double ar2 = orient2d(vtx[2 * a], vtx[2 * a + 1], vtx[2 * b], vtx[2 * b + 1], vtx[2 * d], vtx[2 * d + 1]);
    if (!(ar2 > 0.0)) {
      delete c;
      return nullptr;
    }
    c->inv2a[e] = 1.0 / ar2;
  }
  build_coefficients(c);
  build_alpha(c);
  build_omega(c);
  return c;
}

void orc_destroy(orc_ctx* c) { delete c; }

int32_t orc_add_ensemble(orc_ctx* c, const int64_t* counts, uint64_t seed, double x0, double y0,
                         double r0) {
  if (c->p.f32_state) {
    c->ensF.emplace_back();
    Ens<float>& en = c->ensF.back();
    en.seed = seed; en.x0 = x0; en.y0 = y0; en.r0 = r0;
    en.counts.assign(counts, counts + c->ne);
    build_rates(c, &en, nullptr);
    seed_ensemble<float>(c, en, (uint32_t)(c->ensF.size() - 1));
    return (int32_t)c->ensF.size() - 1;
  }
  c->ensD.emplace_back();
  Ens<double>& en = c->ensD.back();
  en.seed = seed; en.x0 = x0; en.y0 = y0; en.r0 = r0;
  en.counts.assign(counts, counts + c->ne);
  build_rates(c, nullptr, &en);
  seed_ensemble<double>(c, en, (uint32_t)(c->ensD.size() - 1));
  return (int32_t)c->ensD.size() - 1;
}

int32_t orc_nstat(const orc_ctx* c) { return nstat_of(c->p); }

int64_t orc_count(const orc_ctx* c, int32_t ens) {
  return c->p.f32_state ? (int64_t)c->ensF[ens].x.size() : (int64_t)c->ensD[ens].x.size();
}

int32_t orc_step(orc_ctx* c, int32_t nsteps) {
  for (int s = 0; s < nsteps; ++s) {
    int r = c->p.f32_state ? step_all<float>(c, c->ensF) : step_all<double>(c, c->ensD);
    if (r) return r;
  }
  return 0;
}

int32_t orc_stats(orc_ctx* c, int32_t ens, double* out) {
  std::vector<double> st;
  if (c->p.f32_state) estimate<float>(c, c->ensF[ens], st);
  else estimate<double>(c, c->ensD[ens], st);
  std::memcpy(out, st.data(), st.size() * sizeof(double));
  return 0;
}

int32_t orc_get_state(const orc_ctx* c, int32_t ens, double* x, double* y, double* u, double* v,
                      double* w, double* psi, int32_t* elem) {
  if (c->p.f32_state) get_state_t<float>(c->ensF[ens], x, y, u, v, w, psi, elem);
  else get_state_t<double>(c->ensD[ens], x, y, u, v, w, psi, elem);
  return 0;
}

int32_t orc_set_state(orc_ctx* c, int32_t ens, const double* x, const double* y, const double* u,
                      const double* v, const double* w, const double* psi, const int32_t* elem) {
  if (c->p.f32_state) set_state_t<float>(c->ensF[ens], x, y, u, v, w, psi, elem);
  else set_state_t<double>(c->ensD[ens], x, y, u, v, w, psi, elem);
  return 0;
}

double orc_exp64(double x) { return exp_series(x); }

int32_t orc_navg(const orc_ctx* c) {
  return ORC_AV_HIST + c->p.hist_bins + (c->p.omega ? 2 : 0);
}

void orc_average_start(orc_ctx* c) {
  c->averaging = true;
  c->avg_rec.clear();
}

void orc_average_stop(orc_ctx* c) { c->averaging = false; }

// Time-averaged statistics: the particles of an element over all averaged
// steps taken as one pooled sample.  With n_t, m_t and C_t the count, means
// and central second moments of step t, the pooled count is N = sum n_t, the
// mean M = sum n_t m_t / N and the central moments
// sum n_t (C_t + (m_t - M)(m_t - M)^T) / N (the law of total variance), two
// passes over the stored records; histograms add up.
int32_t orc_average(const orc_ctx* c, int32_t ens, double* out) {
  const orc_params& p = c->p;
  const int ns = nstat_of(p);
  const int na = orc_navg(c);
  const int hoff = p.moments >= 4 ? ORC_NSTAT_4 : ORC_NSTAT_2;
  std::memset(out, 0, sizeof(double) * (size_t)na * c->ne);
  if (ens < 0 || (size_t)ens >= c->avg_rec.size()) return 0;
  const std::vector<std::vector<double>>& recs = c->avg_rec[ens];
  const double T = (double)recs.size();
  for (int e = 0; e < c->ne; ++e) {
    double* o = out + (size_t)e * na;
    o[ORC_AV_STEPS] = T;
    double N = 0.0, sm[4] = {0, 0, 0, 0}, sw = 0.0;
    for (const std::vector<double>& st : recs) {
      const double* r = &st[(size_t)e * ns];
      const double n = r[ORC_ST_N];
      N += n;
      for (int q = 0; q < 4; ++q) sm[q] += n * r[ORC_ST_MEAN + q];
      if (p.omega) sw += n * r[ns - 3];
      for (int h = 0; h < p.hist_bins; ++h) o[ORC_AV_HIST + h] += r[hoff + h];
    }
    o[ORC_AV_N] = N;
    if (N == 0.0) continue;
    double M[4];
    for (int q = 0; q < 4; ++q) M[q] = sm[q] / N;
    const double MW = sw / N;
    double C[10] = {0}, CW = 0.0;
    for (const std::vector<double>& st : recs) {
      const double* r = &st[(size_t)e * ns];
      const double n = r[ORC_ST_N];
      if (n == 0.0) continue;
      double d[4];
      for (int q = 0; q < 4; ++q) d[q] = r[ORC_ST_MEAN + q] - M[q];
      int idx = 0;
      for (int a = 0; a < 4; ++a)
        for (int b = a; b < 4; ++b, ++idx) C[idx] += n * (r[ORC_ST_M2 + idx] + d[a] * d[b]);
      if (p.omega) {
        const double dw = r[ns - 3] - MW;
        CW += n * (r[ns - 2] + dw * dw);
      }
    }
    for (int q = 0; q < 4; ++q) o[ORC_AV_MEAN + q] = M[q];
    for (int t = 0; t < 10; ++t) o[ORC_AV_M2 + t] = C[t] / N;
    if (p.omega) {
      o[ORC_AV_HIST + p.hist_bins] = MW;
      o[ORC_AV_HIST + p.hist_bins + 1] = CW / N;
    }
  }
  return 0;
}

int32_t orc_locate(const orc_ctx* c, double x, double y) {
  for (int e = 0; e < c->ne; ++e)
    if (orient_edge(c, e, 0, x, y) >= 0.0 && orient_edge(c, e, 1, x, y) >= 0.0 && orient_edge(c, e, 2, x, y) >= 0.0)
      return e;
  return -1;
}

int64_t orc_wallfn_hits(const orc_ctx* c) { return c->wf_hits; }

int32_t orc_get_omega(const orc_ctx* c, int32_t ens, double* om) {
  if (!c->p.omega) return -1;
  if (c->p.f32_state) get_om_t<float>(c->ensF[ens], om);
  else get_om_t<double>(c->ensD[ens], om);
  return 0;
}

int32_t orc_set_omega(orc_ctx* c, int32_t ens, const double* om) {
  if (!c->p.omega) return -1;
  if (c->p.f32_state) set_om_t<float>(c->ensF[ens], om);
  else set_om_t<double>(c->ensD[ens], om);
  return 0;
}

void orc_omega_fields(const orc_ctx* c, double* om0, double* somega, double* omw) {
  for (int e = 0; e < c->ne; ++e) {
    om0[e] = c->om0[e];
    somega[e] = c->somega[e];
    for (int q = 0; q < 3; ++q) omw[3 * e + q] = c->omw[3 * e + q];
  }
}

void orc_set_cond_means(orc_ctx* c, int32_t ens, const double* cm) {
  std::vector<double>& dst = c->p.f32_state ? c->ensF[ens].cm : c->ensD[ens].cm;
  if (!cm) {
    dst.clear();
    return;
  }
  dst.assign(cm, cm + (size_t)c->ne * 8);
}

int64_t orc_get_step(const orc_ctx* c) { return c->step; }
void orc_set_step(orc_ctx* c, int64_t step) { c->step = step; }

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(ctr, key, out);
}

void orc_normals(uint64_t seed, uint32_t id, uint32_t step, uint32_t ens, int32_t f32, double out[8]) {
  if (f32) {
    float xi[8];
    step_normals<float>(seed, id, step, ens, xi);
    for (int i = 0; i < 8; ++i) out[i] = xi[i];
  } else {
    double xi[8];
    step_normals<double>(seed, id, step, ens, xi);
    for (int i = 0; i < 8; ++i) out[i] = xi[i];
  }
}

void orc_normals_batch(uint64_t seed, int64_t n, uint32_t step, uint32_t ens, int32_t f32,
                       double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) orc_normals(seed, (uint32_t)i, step, ens, f32, out + 8 * i);
}

double orc_log64(double x) { return series_log<double>(x); }
float orc_log32(float x) { return series_log<float>(x); }
void orc_sincos2pi64(double t, double* s, double* c) { series_sincos2pi<double>(t, s, c); }
void orc_sincos2pi32(float t, float* s, float* c) { series_sincos2pi<float>(t, s, c); }
double orc_cbrt64(double x) { return newton_cbrt(x); }

void orc_coefficients(const orc_ctx* c, double* out) {
  for (size_t i = 0; i < c->coef.size(); ++i)
    out[i] = c->p.f32_state ? (double)(float)c->coef[i] : c->coef[i];
}

void orc_set_pressure_gradient(orc_ctx* c, const double* g2) {
  for (int v = 0; v < c->nv; ++v) {
    c->coef[(size_t)v * NC + C_DPDX] = g2[2 * (size_t)v];
    c->coef[(size_t)v * NC + C_DPDY] = g2[2 * (size_t)v + 1];
  }
}

void orc_set_drift(orc_ctx* c, const double* g6) {
  for (int v = 0; v < c->nv; ++v)
    for (int j = 0; j < 6; ++j) c->coef[(size_t)v * NC + C_G11 + j] = g6[(size_t)v * 6 + j];
}

void orc_mix_rate(const orc_ctx* c, int32_t ens, double* out) {
  const std::vector<double>& r = c->p.f32_state ? c->ensF[ens].rate : c->ensD[ens].rate;
  for (int e = 0; e < c->ne; ++e) out[e] = c->p.f32_state ? (double)(float)r[e] : r[e];
}

void orc_wall_alpha(const orc_ctx* c, double* out) {
  std::memcpy(out, c->alpha.data(), c->alpha.size() * sizeof(double));
}

int32_t orc_walk(const orc_ctx* c, int32_t e, double sx, double sy, double* tx, double* ty,
                 double* vel, int32_t* n_reflect, double* om) {
  int nref = 0;
  int r;
  if (c->p.f32_state) {
    float X = (float)*tx, Y = (float)*ty, u = (float)vel[0], v = (float)vel[1], w = (float)vel[2];
    float o = om ? (float)*om : 0.0f;
    r = walk<float>(c, e, sx, sy, X, Y, u, v, w, &nref, om ? &o : nullptr);
    *tx = X; *ty = Y; vel[0] = u; vel[1] = v; vel[2] = w;
    if (om) *om = o;
  } else {
    double X = *tx, Y = *ty, u = vel[0], v = vel[1], w = vel[2];
    double o = om ? *om : 0.0;
    r = walk<double>(c, e, sx, sy, X, Y, u, v, w, &nref, om ? &o : nullptr);
    *tx = X; *ty = Y; vel[0] = u; vel[1] = v; vel[2] = w;
    if (om) *om = o;
  }
  if (n_reflect) *n_reflect = nref;
  return r;
}

}  // extern "C"
