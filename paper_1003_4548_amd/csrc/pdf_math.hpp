// Device arithmetic of the particle step: counter-based normals, the series
// log / sincos / cube root they and the mixing time need, and the geometric
// predicates of the tracking.  Every routine is a fixed sequence of IEEE
// +, -, *, /, sqrt and fused multiply-adds written out where the definition
// fuses (no other contraction: the library is built with -ffp-contract=off),
// so its result is reproducible bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdf {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  The key words are
// wave-uniform (one seed per ensemble), so the key schedule stays scalar.

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
}

// words 0..3 from counter block 0, 4..7 from block 1: counter (id, step, b, ens)
template <int NBLOCKS>
__device__ __forceinline__ void philox_words(uint32_t id, uint32_t step, uint32_t ens, uint32_t k0,
                                             uint32_t k1, uint32_t* w) {
#pragma unroll
  for (int b = 0; b < NBLOCKS; ++b) {
    uint32_t c0 = id, c1 = step, c2 = (uint32_t)b, c3 = ens;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    w[4 * b + 0] = c0; w[4 * b + 1] = c1; w[4 * b + 2] = c2; w[4 * b + 3] = c3;
  }
}

// Uniform deviates in (0,1), exactly representable: float from the top 23
// bits, double from all 32, each offset by half a grid step.
template <typename T> __device__ __forceinline__ T uniform01(uint32_t r);
template <> __device__ __forceinline__ float uniform01<float>(uint32_t r) {
  return (float)(r >> 9) * 0x1p-23f + 0x1p-24f;
}
template <> __device__ __forceinline__ double uniform01<double>(uint32_t r) {
  return (double)r * 0x1p-32 + 0x1p-33;
}

// ---------------------------------------------------------------------------
// log x = e ln 2 + 2 atanh(s), s = (m-1)/(m+1), x = m 2^e, m in [sqrt(1/2),
// sqrt(2)); the atanh series s + s^3/3 + ... is summed by Horner's rule
// through s^21 (double) or s^11 (float).

template <typename T> struct SeriesTerms;
template <> struct SeriesTerms<double> { static constexpr int LOG = 10, SIN = 7, COS = 8; };
template <> struct SeriesTerms<float> { static constexpr int LOG = 5, SIN = 4, COS = 5; };

__device__ __forceinline__ float frexp_t(float x, int* e) { return frexpf(x, e); }
__device__ __forceinline__ double frexp_t(double x, int* e) { return frexp(x, e); }
__device__ __forceinline__ float floor_t(float x) { return floorf(x); }
__device__ __forceinline__ double floor_t(double x) { return floor(x); }
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
// a * b + c with one rounding (where the step's definition fuses them)
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a / b for b in [1, 4) and a zero or of magnitude at least 2^-30 (no
// operand or quotient near the exponent limits), correctly rounded: the
// reciprocal estimate refined by Newton's step, the quotient by two residual
// corrections (Markstein).  These are the steps the compiler emits for a
// float division, without the operand rescaling and special-case fix-up that
// such operands never need.
__device__ __forceinline__ float div_moderate(float a, float b) {
  float y = __builtin_amdgcn_rcpf(b);
  const float e = __builtin_fmaf(-b, y, 1.0f);
  y = __builtin_fmaf(e, y, y);
  float q = a * y;
  float r = __builtin_fmaf(-b, q, a);
  q = __builtin_fmaf(r, y, q);
  r = __builtin_fmaf(-b, q, a);
  return __builtin_fmaf(r, y, q);
}
// (m - 1) / (m + 1) for m in [sqrt(1/2), sqrt(2)): m - 1 is zero or at least
// 2^-24 in magnitude
__device__ __forceinline__ float atanh_arg(float m) { return div_moderate(m - 1.0f, m + 1.0f); }
__device__ __forceinline__ double atanh_arg(double m) { return (m - 1.0) / (m + 1.0); }

template <typename T> __device__ __forceinline__ T series_log(T x) {
  int e0 = 0;
  const T f = frexp_t(x, &e0);
  T m;
  int e;
  if (f < (T)0.70710678118654752440) {
    m = f + f;
    e = e0 - 1;
  } else {
    m = f;
    e = e0;
  }
  const T s = atanh_arg(m);
  const T z = s * s;
  constexpr int K = SeriesTerms<T>::LOG;
  T p = (T)1 / (T)(2 * K + 1);
#pragma unroll
  for (int j = K - 1; j >= 1; --j) p = fma_t(p, z, (T)1 / (T)(2 * j + 1));
  const T t = fma_t(s, z * p, s);
  return fma_t((T)e, (T)0.69314718055994530942, t + t);
}

template <typename T> __device__ __forceinline__ constexpr T inv_fact(int n) {
  T f = (T)1;
  for (int i = 2; i <= n; ++i) f = f * (T)i;
  return (T)1 / f;
}

// sin and cos of 2 pi t: t = q/4 + r exactly, |r| <= 1/8; Taylor series of
// the remainder angle by Horner's rule, then q quarter turns.
template <typename T> __device__ __forceinline__ void series_sincos2pi(T t, T* sn_out, T* cs_out) {
  const T q = floor_t(t * (T)4 + (T)0.5);
  const T r = t - q * (T)0.25;
  const T th = r * (T)6.28318530717958647692;
  const T z = th * th;
  constexpr int NS = SeriesTerms<T>::SIN;
  T ps = ((NS % 2) ? (T)-1 : (T)1) * inv_fact<T>(2 * NS + 1);
#pragma unroll
  for (int j = NS - 1; j >= 1; --j) ps = fma_t(ps, z, ((j % 2) ? (T)-1 : (T)1) * inv_fact<T>(2 * j + 1));
  const T sn = fma_t(th, z * ps, th);
  constexpr int NC = SeriesTerms<T>::COS;
  T pc = ((NC % 2) ? (T)-1 : (T)1) * inv_fact<T>(2 * NC);
#pragma unroll
  for (int j = NC - 1; j >= 1; --j) pc = fma_t(pc, z, ((j % 2) ? (T)-1 : (T)1) * inv_fact<T>(2 * j));
  const T cs = fma_t(z, pc, (T)1);
  const int qi = ((int)q) & 3;
  T so = sn, co = cs;
  if (qi == 1) { so = cs; co = -sn; }
  if (qi == 2) { so = -sn; co = -cs; }
  if (qi == 3) { so = -cs; co = sn; }
  *sn_out = so;
  *cs_out = co;
}

// exp x = 2^k exp r: k the nearest integer to x / ln 2, r = x - k ln 2 with
// ln 2 split into a high part whose trailing bits are zero (so k times it is
// exact) and a low part (Cody & Waite); exp r by its Taylor series through
// r^13 (|r| <= ln 2 / 2, truncation below 2^-60) in Horner form; then the
// exact scaling by 2^k.
__device__ __forceinline__ double series_exp(double x) {
  const double k = rint(x * 0x1.71547652b82fep0);
  const double r = (x - k * 0x1.62e42fefa3800p-1) - k * 0x1.ef35793c76730p-45;
  double p = inv_fact<double>(13);
#pragma unroll
  for (int j = 12; j >= 1; --j) p = p * r + inv_fact<double>(j);
  p = p * r + 1.0;
  return ldexp(p, (int)k);
}

// Square root of a positive normal float (at least 2^-96), correctly
// rounded: the hardware estimate, then the one-ulp neighbour that the fma
// residuals select.  These are the steps the compiler emits for sqrtf on
// such inputs, without its rescaling of tiny inputs and its special-value
// cases, which the Box-Muller radius (-2 log u1 in [1.2e-7, 34]) never takes.
__device__ __forceinline__ float sqrt_pos_normal(float x) {
  float s = __builtin_amdgcn_sqrtf(x);
  const float sdn = __uint_as_float(__float_as_uint(s) - 1u);
  const float sup = __uint_as_float(__float_as_uint(s) + 1u);
  const float rdn = __builtin_fmaf(-sdn, s, x);
  const float rup = __builtin_fmaf(-sup, s, x);
  if (rdn <= 0.0f) s = sdn;
  if (rup > 0.0f) s = sup;
  return s;
}
__device__ __forceinline__ float sqrt_radius(float x) { return sqrt_pos_normal(x); }
__device__ __forceinline__ double sqrt_radius(double x) { return sqrt(x); }

// Box-Muller (Box & Muller 1958) on two words.
template <typename T> __device__ __forceinline__ void box_muller(uint32_t r1, uint32_t r2, T* z0, T* z1) {
  const T u1 = uniform01<T>(r1), u2 = uniform01<T>(r2);
  const T rad = sqrt_radius((T)-2 * series_log<T>(u1));
  T sn, cs;
  series_sincos2pi<T>(u2, &sn, &cs);
  *z0 = rad * cs;
  *z1 = rad * sn;
}

// Cube root by Newton's method on y^3 = x, twelve iterations from 2^(e/3).
__device__ __forceinline__ double newton_cbrt(double x) {
  int e = 0;
  frexp(x, &e);
  double y = ldexp(1.0, e / 3);
#pragma unroll 1
  for (int i = 0; i < 12; ++i) y = (y + y + x / (y * y)) / 3.0;
  return y;
}

// ---------------------------------------------------------------------------
// geometry

__device__ __forceinline__ double orient2d(double ax, double ay, double bx, double by, double px,
                                           double py) {
  return __builtin_fma(bx - ax, py - ay, -((by - ay) * (px - ax)));
}

// Orientation of p against the edge a->b of a counter-clockwise element,
// evaluated from the lexicographically smaller endpoint so that the two
// elements sharing an edge get exactly opposite values.
__device__ __forceinline__ double orient_edge(double ax, double ay, double bx, double by, double px,
                                              double py) {
  const bool a_first = (ax < bx) || (ax == bx && ay < by);
  return a_first ? orient2d(ax, ay, bx, by, px, py) : -orient2d(bx, by, ax, ay, px, py);
}

__device__ __forceinline__ float next_toward(float x, double dir) {
  return nextafterf(x, dir > 0.0 ? __builtin_huge_valf() : -__builtin_huge_valf());
}
__device__ __forceinline__ double next_toward(double x, double dir) {
  return nextafter(x, dir > 0.0 ? __builtin_huge_val() : -__builtin_huge_val());
}

}  // namespace pdf
