// Kernels of the particle-in-cell joint velocity-scalar PDF step.
//
// Data layout in HBM (structure of arrays):
//   particles  x y u v w psi (state type T) and id (u32), in two buffers.
//              Each (ensemble, element) pair -- a "cell" -- owns a segment of
//              fixed capacity; its particles sit densely at the front.  A
//              particle's element is implied by the segment that holds it.
//   cells      segment start, capacity, particle count per buffer, IECM rate.
//   mesh       vertex coordinates (f64), element vertices / neighbours / edge
//              kinds (i32), 1/(2 area) (f64), wall-function alpha per edge.
//   vertices   16 drift/diffusion coefficients per vertex (T), row-major.
//
// One wavefront (64 lanes) owns one cell per step.  It reads the segment,
// estimates the cell's statistics with lane-strided FP64 accumulators and
// cross-lane butterflies (no atomics), uses them for IECM, advances every
// particle, tracks it through the mesh, and appends it to the segment of its
// new cell in the other buffer.  Appends are counted per wavefront: lanes with
// the same destination share one atomic add on that cell's counter.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdf_math.hpp"

namespace pdf {

enum { NFIELD = 20, NCOEF = 16 };
enum { F_U, F_V, F_DUDX, F_DUDY, F_DVDX, F_DVDY, F_LAPU, F_LAPV, F_DPDX, F_DPDY,
       F_R11, F_R22, F_R33, F_R12, F_EPS, F_P11, F_P12, F_P21, F_P22, F_P33 };
enum { C_U, C_V, C_DUDX, C_DUDY, C_DVDX, C_DVDY, C_LAPU, C_LAPV, C_DPDX, C_DPDY,
       C_G11, C_G12, C_G21, C_G22, C_G33, C_C0EPS };
enum { EDGE_INTERIOR = 0, EDGE_NOSLIP = 1, EDGE_SLIP = 2, EDGE_WALLFN = 3, EDGE_PXP = 4,
       EDGE_PXM = 5, EDGE_PYP = 6, EDGE_PYM = 7 };
enum { ST_N = 0, ST_MEAN = 1, ST_M2 = 5, ST_BINN = 15, ST_BINM = 23, ST_M3 = 31, ST_M4 = 51,
       NSTAT2 = 31, NSTAT4 = 86 };
enum { ERR_LOST = 1, ERR_NAN = 2, ERR_CAPACITY = 4, ERR_OVERFLOW_FULL = 8 };
enum { FLAG_VEL = 1, FLAG_POS = 2, FLAG_MIX = 4, FLAG_SRC = 8 };

constexpr uint32_t SEED_STEP = 0xFFFFFFFFu;  // step counter word of the initial draw
constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;

// Control block in device memory.
struct Ctl {
  uint32_t step;      // Philox step word of the next step
  uint32_t parity;    // buffer holding the current state
  int32_t error;      // OR of ERR_* raised since seeding
  int32_t halt;       // set at the end of a step that raised an error
  uint32_t done;      // workgroups finished in the running launch
  uint32_t ovf;       // particles written to the overflow area
  int64_t steps_done; // steps completed since seeding
  uint32_t lost;      // particles the walk could not place
  uint32_t pad[9];
};

struct MeshDev {
  const double* vtx;
  const int32_t* tri;
  const int32_t* nbr;
  const int32_t* ekind;
  const double* inv2a;
  const double* alpha;
  int32_t ne;
  int32_t nv;
  double Lx, Ly;
};

template <typename T> struct StateDev {
  T* x; T* y; T* u; T* v; T* w; T* psi;
  uint32_t* id;
};

template <typename T> struct StepArgs {
  MeshDev mesh;
  const T* coef;          // nv x 16
  const T* rate;          // ncell
  const int32_t* start;   // ncell
  const int32_t* cap;     // ncell
  int32_t* cnt[2];        // ncell each
  StateDev<T> buf[2];
  StateDev<T> ovf;        // overflow area
  int32_t* ovf_cell;
  uint32_t ovf_cap;
  double* stats;          // ncell x nstat
  const uint64_t* seed;   // nens
  const double* src;      // nens x 3
  Ctl* ctl;
  int32_t ncell;
  int32_t nstat;
  int32_t flags;
  int32_t mix;
  T dt, sdt, nu2, s2nu;
};

// Logical block index that gives each XCD a contiguous range of cells:
// hardware dispatches consecutive workgroups round-robin over the 8 XCDs.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int NX = 8;
  const int q = G / NX, r = G % NX, x = b % NX, i = b / NX;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ---------------------------------------------------------------------------
// tracking: straight-line neighbour walk with wall and periodic conditions.
// Exit edge: the first edge (lowest local index) the target lies outside of
// whose endpoints the line start->target separates; if rounding leaves none,
// the edge the target is most outside of.  Walls mirror the rest of the path
// about the wall line and reflect the velocity; periodic edges shift the path
// by one period into the partner element.

template <typename T>
__device__ int walk(const MeshDev& M, int e, double Sx, double Sy, T& tx, T& ty, T& u, T& v, T& w) {
#pragma unroll 1
  for (int it = 0; it < 64; ++it) {
    const double Tx = (double)tx, Ty = (double)ty;
    const int i0 = M.tri[3 * e], i1 = M.tri[3 * e + 1], i2 = M.tri[3 * e + 2];
    double px[3], py[3];
    px[0] = M.vtx[2 * i0]; py[0] = M.vtx[2 * i0 + 1];
    px[1] = M.vtx[2 * i1]; py[1] = M.vtx[2 * i1 + 1];
    px[2] = M.vtx[2 * i2]; py[2] = M.vtx[2 * i2 + 1];
    double o[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = k == 2 ? 0 : k + 1;
      o[k] = orient_edge(px[k], py[k], px[k1], py[k1], Tx, Ty);
    }
    if (o[0] >= 0.0 && o[1] >= 0.0 && o[2] >= 0.0) return e;
    int ex = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = k == 2 ? 0 : k + 1;
      if (ex < 0 && o[k] < 0.0) {
        const double sa = orient2d(Sx, Sy, Tx, Ty, px[k], py[k]);
        const double sb = orient2d(Sx, Sy, Tx, Ty, px[k1], py[k1]);
        if ((sa <= 0.0 && sb >= 0.0) || (sa >= 0.0 && sb <= 0.0)) ex = k;
      }
    }
    if (ex < 0) {
      ex = 0;
      if (o[1] < o[ex]) ex = 1;
      if (o[2] < o[ex]) ex = 2;
    }
    const int kind = M.ekind[3 * e + ex];
    if (kind == EDGE_INTERIOR) {
      e = M.nbr[3 * e + ex];
      continue;
    }
    if (kind >= EDGE_PXP) {
      double sx = 0.0, sy = 0.0;
      if (kind == EDGE_PXP) sx = M.Lx;
      if (kind == EDGE_PXM) sx = -M.Lx;
      if (kind == EDGE_PYP) sy = M.Ly;
      if (kind == EDGE_PYM) sy = -M.Ly;
      Sx = Sx + sx;
      Sy = Sy + sy;
      tx = tx + (T)sx;
      ty = ty + (T)sy;
      e = M.nbr[3 * e + ex];
      continue;
    }
    const int ex1 = ex == 2 ? 0 : ex + 1;
    const double ax = px[ex], ay = py[ex];
    const double gx = px[ex1] - ax, gy = py[ex1] - ay;
    const double len = sqrt(gx * gx + gy * gy);
    const double nx = gy / len, ny = -gx / len;  // outward unit normal
    const double oS = orient_edge(ax, ay, px[ex1], py[ex1], Sx, Sy), oT = o[ex];
    const double den = oS - oT;
    const double tpar = den > 0.0 ? oS / den : 0.0;
    const double Ix = Sx + tpar * (Tx - Sx), Iy = Sy + tpar * (Ty - Sy);
    const double d = (Tx - ax) * nx + (Ty - ay) * ny;
    tx = (T)(Tx - (2.0 * d) * nx);
    ty = (T)(Ty - (2.0 * d) * ny);
#pragma unroll 1
    for (int j = 0; j < 8; ++j) {
      if (!(orient_edge(ax, ay, px[ex1], py[ex1], (double)tx, (double)ty) < 0.0)) break;
      if (nx != 0.0) tx = next_toward(tx, -nx);
      if (ny != 0.0) ty = next_toward(ty, -ny);
    }
    Sx = Ix;
    Sy = Iy;
    const T nxT = (T)nx, nyT = (T)ny;
    if (kind == EDGE_NOSLIP) {
      u = -u; v = -v; w = -w;
    } else if (kind == EDGE_SLIP) {
      const T un = u * nxT + v * nyT;
      const T un2 = un + un;
      u = u - un2 * nxT;
      v = v - un2 * nyT;
    } else {
      const T tX = -nyT, tY = nxT;
      const T Vi = -(u * nxT + v * nyT);
      const T Ui = u * tX + v * tY;
      const T al = (T)M.alpha[3 * e + ex];
      const T Ur = Ui + al * Vi;
      const T Vr = -Vi;
      u = Ur * tX + Vr * (-nxT);
      v = Ur * tY + Vr * (-nyT);
    }
  }
  return -1;
}

// ---------------------------------------------------------------------------
// the fused step: statistics of the cell, then IECM, velocity, position,
// tracking, source and append.  ADVANCE = false only estimates statistics.

template <int MOM> struct MomCount { static constexpr int M3 = 0, M4 = 0; };

// position of (x, y), x <= y, in the lexicographic list of index pairs of (u, v, w, psi)
__host__ __device__ constexpr int pair_index(int x, int y) { return x * 4 - (x * (x - 1)) / 2 + (y - x); }

// position of (x, y, z), x <= y <= z, in the lexicographic list of index triples
__host__ __device__ constexpr int triple_index(int x, int y, int z) {
  int it = 0;
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b)
      for (int c = b; c < 4; ++c)
        if (a < x || (a == x && (b < y || (b == y && c < z)))) ++it;
  return it;
}
template <> struct MomCount<4> { static constexpr int M3 = 20, M4 = 35; };

template <typename T, int MOM, int HIST, bool ADVANCE>
__global__ __launch_bounds__(BLOCK) void k_step(StepArgs<T> a) {
  __shared__ int hist_lds[WAVES_PER_BLOCK][HIST > 0 ? HIST : 1];
  Ctl* ctl = a.ctl;
  if (ADVANCE && ctl->halt) return;
  const uint32_t step = ctl->step;
  const uint32_t par = ctl->parity;
  const int lane = lane_id();
  const int wid = threadIdx.x / WAVE;
  const int cell = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + wid;
  const StateDev<T> src = a.buf[par];
  const StateDev<T> dst = a.buf[par ^ 1u];
  int32_t* cnt_src = a.cnt[par];
  int32_t* cnt_dst = a.cnt[par ^ 1u];

  if (cell < a.ncell) {
    const int ne = a.mesh.ne;
    const int ens = cell / ne;
    const int e = cell - ens * ne;
    const int start = a.start[cell];
    int n = cnt_src[cell];
    const int capc = a.cap[cell];
    if (n > capc) n = capc;

    // pass 1: means
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = lane; j < n; j += WAVE) {
      s0 += (double)src.u[start + j];
      s1 += (double)src.v[start + j];
      s2 += (double)src.w[start + j];
      s3 += (double)src.psi[start + j];
    }
    const double dn = (double)n;
    double mean[4];
    mean[0] = n > 0 ? wave_sum(s0) / dn : 0.0;
    mean[1] = n > 0 ? wave_sum(s1) / dn : 0.0;
    mean[2] = n > 0 ? wave_sum(s2) / dn : 0.0;
    mean[3] = n > 0 ? wave_sum(s3) / dn : 0.0;

    // pass 2: central moments, velocity bins, histogram
    constexpr int NM3 = MomCount<MOM>::M3, NM4 = MomCount<MOM>::M4;
    double m2[10], m3[NM3 > 0 ? NM3 : 1], m4[NM4 > 0 ? NM4 : 1];
    double bn[8], bs[8];
#pragma unroll
    for (int q = 0; q < 10; ++q) m2[q] = 0.0;
#pragma unroll
    for (int q = 0; q < (NM3 > 0 ? NM3 : 1); ++q) m3[q] = 0.0;
#pragma unroll
    for (int q = 0; q < (NM4 > 0 ? NM4 : 1); ++q) m4[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) { bn[q] = 0.0; bs[q] = 0.0; }
    if (HIST > 0) {
      for (int h = lane; h < HIST; h += WAVE) hist_lds[wid][h] = 0;
    }
    for (int j = lane; j < n; j += WAVE) {
      double val[4];
      val[0] = (double)src.u[start + j];
      val[1] = (double)src.v[start + j];
      val[2] = (double)src.w[start + j];
      val[3] = (double)src.psi[start + j];
      double d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = val[q] - mean[q];
      double p2[10];
      {
        int idx = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = x; y < 4; ++y) { p2[idx] = d[x] * d[y]; m2[idx] += p2[idx]; ++idx; }
      }
      if constexpr (MOM >= 4) {
        double p3[20];
        int i3 = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = x; y < 4; ++y)
#pragma unroll
            for (int z = y; z < 4; ++z) {
              p3[i3] = p2[pair_index(x, y)] * d[z];
              m3[i3] += p3[i3];
              ++i3;
            }
        int i4 = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = x; y < 4; ++y)
#pragma unroll
            for (int z = y; z < 4; ++z)
#pragma unroll
              for (int g = z; g < 4; ++g) {
                m4[i4] += p3[triple_index(x, y, z)] * d[g];
                ++i4;
              }
      }
      const int bin = (val[0] > mean[0] ? 1 : 0) + (val[1] > mean[1] ? 2 : 0) + (val[2] > mean[2] ? 4 : 0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        bn[q] += (bin == q) ? 1.0 : 0.0;
        bs[q] += (bin == q) ? val[3] : 0.0;
      }
      if (HIST > 0) {
        const double hpos = floor(val[3] * (double)HIST);
        const int hb = hpos < 0.0 ? 0 : (hpos >= (double)HIST ? HIST - 1 : (int)hpos);
        atomicAdd(&hist_lds[wid][hb], 1);
      }
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) m2[q] = wave_sum(m2[q]);
    if constexpr (MOM >= 4) {
#pragma unroll
      for (int q = 0; q < (NM3 > 0 ? NM3 : 1); ++q) m3[q] = wave_sum(m3[q]);
#pragma unroll
      for (int q = 0; q < (NM4 > 0 ? NM4 : 1); ++q) m4[q] = wave_sum(m4[q]);
    }
    double bm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      bn[q] = wave_sum(bn[q]);
      bs[q] = wave_sum(bs[q]);
      bm[q] = bn[q] > 0.0 ? bs[q] / bn[q] : mean[3];
    }
    double* rec = a.stats + (size_t)cell * a.nstat;
    if (lane == 0) {
      if (n > 0) {
        rec[ST_N] = dn;
#pragma unroll
        for (int q = 0; q < 4; ++q) rec[ST_MEAN + q] = mean[q];
#pragma unroll
        for (int q = 0; q < 10; ++q) rec[ST_M2 + q] = m2[q] / dn;
#pragma unroll
        for (int q = 0; q < 8; ++q) { rec[ST_BINN + q] = bn[q]; rec[ST_BINM + q] = bm[q]; }
        if constexpr (MOM >= 4) {
#pragma unroll
          for (int q = 0; q < (NM3 > 0 ? NM3 : 1); ++q) rec[ST_M3 + q] = m3[q] / dn;
#pragma unroll
          for (int q = 0; q < (NM4 > 0 ? NM4 : 1); ++q) rec[ST_M4 + q] = m4[q] / dn;
        }
      } else {
        for (int q = 0; q < (MOM >= 4 ? NSTAT4 : NSTAT2); ++q) rec[q] = 0.0;
      }
    }
    if (HIST > 0) {
      __builtin_amdgcn_wave_barrier();
      const int off = MOM >= 4 ? NSTAT4 : NSTAT2;
      for (int h = lane; h < HIST; h += WAVE) rec[off + h] = (double)hist_lds[wid][h];
    }

    if (ADVANCE) {
      // ---- per-cell constants (wave-uniform) ----
      const MeshDev& M = a.mesh;
      const int v0 = M.tri[3 * e], v1 = M.tri[3 * e + 1], v2 = M.tri[3 * e + 2];
      const double ax = M.vtx[2 * v0], ay = M.vtx[2 * v0 + 1];
      const double bx = M.vtx[2 * v1], by = M.vtx[2 * v1 + 1];
      const double cx = M.vtx[2 * v2], cy = M.vtx[2 * v2 + 1];
      const double ia = M.inv2a[e];
      const T* q0 = a.coef + (size_t)v0 * NCOEF;
      const T* q1 = a.coef + (size_t)v1 * NCOEF;
      const T* q2 = a.coef + (size_t)v2 * NCOEF;
      const T rate = a.rate[cell];
      const uint64_t seed = a.seed[ens];
      const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
      const double sx0 = a.src[3 * ens], sy0 = a.src[3 * ens + 1], sr0 = a.src[3 * ens + 2];
      const bool do_mix = a.mix && (a.flags & FLAG_MIX);
      int err = 0;
      for (int base = 0; base < n; base += WAVE) {
        const int j = base + lane;
        const bool act = j < n;
        int tgt = -1;
        T xn = 0, yn = 0, un = 0, vn = 0, wn = 0, psi = 0;
        uint32_t id = 0;
        if (act) {
          const int s = start + j;
          const T x = src.x[s], y = src.y[s], u = src.u[s], v = src.v[s], w = src.w[s];
          psi = src.psi[s];
          id = src.id[s];
          uint32_t rw[8];
          philox_words(id, step, (uint32_t)ens, k0, k1, rw, 2);
          T xi0, xi1, xi2, xi3, xi4, xi5;
          box_muller<T>(rw[0], rw[1], &xi0, &xi1);
          box_muller<T>(rw[2], rw[3], &xi2, &xi3);
          box_muller<T>(rw[4], rw[5], &xi4, &xi5);
          (void)xi5;
          const double X = (double)x, Y = (double)y;
          const T l0 = (T)(orient_edge(bx, by, cx, cy, X, Y) * ia);
          const T l1 = (T)(orient_edge(cx, cy, ax, ay, X, Y) * ia);
          const T l2 = (T)(orient_edge(ax, ay, bx, by, X, Y) * ia);
          T f[NCOEF];
#pragma unroll
          for (int q = 0; q < NCOEF; ++q) f[q] = (l0 * q0[q] + l1 * q1[q]) + l2 * q2[q];
          if (do_mix) {
            const int bin = ((double)u > mean[0] ? 1 : 0) + ((double)v > mean[1] ? 2 : 0) +
                            ((double)w > mean[2] ? 4 : 0);
            double mb = bm[0];
#pragma unroll
            for (int q = 1; q < 8; ++q) mb = (bin == q) ? bm[q] : mb;
            const T m = (T)mb;
            psi = psi - rate * (psi - m);
          }
          const T dW1 = a.sdt * xi0, dW2 = a.sdt * xi1;
          const T dWp1 = a.sdt * xi2, dWp2 = a.sdt * xi3, dWp3 = a.sdt * xi4;
          const T uf = u - f[C_U], vf = v - f[C_V];
          const T sq = sqrt_t(f[C_C0EPS]);
          const T au = (-f[C_DPDX] + a.nu2 * f[C_LAPU]) + (f[C_G11] * uf + f[C_G12] * vf);
          const T av = (-f[C_DPDY] + a.nu2 * f[C_LAPV]) + (f[C_G21] * uf + f[C_G22] * vf);
          un = ((u + au * a.dt) + a.s2nu * (f[C_DUDX] * dW1 + f[C_DUDY] * dW2)) + sq * dWp1;
          vn = ((v + av * a.dt) + a.s2nu * (f[C_DVDX] * dW1 + f[C_DVDY] * dW2)) + sq * dWp2;
          wn = (w + (f[C_G33] * w) * a.dt) + sq * dWp3;
          if (!(a.flags & FLAG_VEL)) { un = u; vn = v; wn = w; }
          xn = (x + u * a.dt) + a.s2nu * dW1;
          yn = (y + v * a.dt) + a.s2nu * dW2;
          int e2 = e;
          if (a.flags & FLAG_POS) {
            e2 = walk<T>(M, e, X, Y, xn, yn, un, vn, wn);
          } else {
            xn = x; yn = y;
          }
          if (e2 < 0) {
            err |= ERR_LOST;
          } else {
            if ((a.flags & FLAG_SRC) && sr0 > 0.0) {
              const double ddx = (double)xn - sx0, ddy = (double)yn - sy0;
              if (ddx * ddx + ddy * ddy <= sr0 * sr0) psi = (T)1;
            }
            if (!(isfinite(un) && isfinite(vn) && isfinite(wn) && isfinite(psi) && isfinite(xn) && isfinite(yn)))
              err |= ERR_NAN;
            tgt = ens * ne + e2;
          }
        }
        // append to the destination cells, one atomic per distinct cell
        uint64_t pending = __ballot(tgt >= 0);
        while (pending) {
          const int leader = __ffsll((unsigned long long)pending) - 1;
          const int t = __shfl(tgt, leader, WAVE);
          const uint64_t mask = __ballot(tgt == t) & pending;
          int basei = 0;
          if (lane == leader) basei = atomicAdd(&cnt_dst[t], (int)__popcll(mask));
          basei = __shfl(basei, leader, WAVE);
          if ((mask >> lane) & 1ull) {
            const int rank = basei + (int)__popcll(mask & lanemask_lt());
            if (rank < a.cap[t]) {
              const int s = a.start[t] + rank;
              dst.x[s] = xn; dst.y[s] = yn; dst.u[s] = un; dst.v[s] = vn; dst.w[s] = wn;
              dst.psi[s] = psi; dst.id[s] = id;
            } else {
              err |= ERR_CAPACITY;
              const uint32_t k = atomicAdd(&ctl->ovf, 1u);
              if (k < a.ovf_cap) {
                a.ovf.x[k] = xn; a.ovf.y[k] = yn; a.ovf.u[k] = un; a.ovf.v[k] = vn; a.ovf.w[k] = wn;
                a.ovf.psi[k] = psi; a.ovf.id[k] = id;
                a.ovf_cell[k] = t;
              } else {
                err |= ERR_OVERFLOW_FULL;
              }
            }
          }
          pending &= ~mask;
        }
      }
      if (lane == 0) cnt_src[cell] = 0;
      // wave-level OR of the error bits, one atomic per wave
      int werr = err;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) werr |= __shfl_xor(werr, off, WAVE);
      if (lane == 0 && werr) atomicOr(&ctl->error, werr);
    }
  }
  if (ADVANCE) {
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const uint32_t prev = atomicAdd(&ctl->done, 1u);
      if (prev == gridDim.x - 1) {
        // last workgroup of the step
        __threadfence();
        ctl->done = 0;
        ctl->step = step + 1;
        ctl->parity = par ^ 1u;
        ctl->steps_done = ctl->steps_done + 1;
        if (atomicAdd(&ctl->error, 0) != 0) ctl->halt = 1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// initialisation kernels

// Per-vertex drift and diffusion coefficients.  SLM, eq. (19):
// G_ij = -(1/2 + 3/4 C0) <omega> delta_ij with <omega> from eq. (8);
// otherwise eqs. (12)-(13) from the elliptic-relaxation tensor wp.
template <typename T>
__global__ void k_coefficients(const double* fields, T* coef, int nv, int model, double C0, double nu,
                               double CT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const double* f = fields + (size_t)i * NFIELD;
  T* q = coef + (size_t)i * NCOEF;
  for (int j = 0; j < 10; ++j) q[j] = (T)f[j];
  const double k = 0.5 * ((f[F_R11] + f[F_R22]) + f[F_R33]);
  const double eps = f[F_EPS];
  if (model == 0) {
    const double om = 2.0 * eps / (k + sqrt(k * k + 4.0 * nu * CT * CT * eps));
    const double g = -(0.5 + 0.75 * C0) * om;
    q[C_G11] = (T)g; q[C_G12] = (T)0.0; q[C_G21] = (T)0.0; q[C_G22] = (T)g; q[C_G33] = (T)g;
    q[C_C0EPS] = (T)(C0 * eps);
  } else {
    const double k2 = 2.0 * k;
    q[C_G11] = (T)((2.0 * f[F_P11] - eps) / k2);
    q[C_G12] = (T)((2.0 * f[F_P12]) / k2);
    q[C_G21] = (T)((2.0 * f[F_P21]) / k2);
    q[C_G22] = (T)((2.0 * f[F_P22] - eps) / k2);
    q[C_G33] = (T)((2.0 * f[F_P33] - eps) / k2);
    double wr = f[F_P11] * f[F_R11] + f[F_P12] * f[F_R12];
    wr = wr + f[F_P21] * f[F_R12];
    wr = wr + f[F_P22] * f[F_R22];
    wr = wr + f[F_P33] * f[F_R33];
    const double c0 = -2.0 * wr / (3.0 * k * eps);
    q[C_C0EPS] = (T)(c0 * eps);
  }
}

__global__ void k_inv2a(const double* vtx, const int32_t* tri, double* inv2a, int32_t* bad, int ne) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int a = tri[3 * e], b = tri[3 * e + 1], c = tri[3 * e + 2];
  const double ar2 = orient2d(vtx[2 * a], vtx[2 * a + 1], vtx[2 * b], vtx[2 * b + 1], vtx[2 * c], vtx[2 * c + 1]);
  if (!(ar2 > 0.0)) atomicOr(bad, 1);
  inv2a[e] = 1.0 / ar2;
}

// IECM relaxation factor of one step, r = min(dt / t_m, 1), with the
// micro-mixing time scale of eq. (11) at the element centroid.
template <typename T>
__global__ void k_rate(const double* vtx, const int32_t* tri, const double* fields, const double* src,
                       T* rate, int ne, int ncell, double dt, double nu, double CT, double Cs, double Ct) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= ncell) return;
  const int ens = cell / ne, e = cell - ens * ne;
  const int v0 = tri[3 * e], v1 = tri[3 * e + 1], v2 = tri[3 * e + 2];
  const double* f0 = fields + (size_t)v0 * NFIELD;
  const double* f1 = fields + (size_t)v1 * NFIELD;
  const double* f2 = fields + (size_t)v2 * NFIELD;
  const double xc = ((vtx[2 * v0] + vtx[2 * v1]) + vtx[2 * v2]) / 3.0;
  const double yc = ((vtx[2 * v0 + 1] + vtx[2 * v1 + 1]) + vtx[2 * v2 + 1]) / 3.0;
  const double k0 = 0.5 * ((f0[F_R11] + f0[F_R22]) + f0[F_R33]);
  const double k1 = 0.5 * ((f1[F_R11] + f1[F_R22]) + f1[F_R33]);
  const double k2 = 0.5 * ((f2[F_R11] + f2[F_R22]) + f2[F_R33]);
  const double k = ((k0 + k1) + k2) / 3.0;
  const double eps = ((f0[F_EPS] + f1[F_EPS]) + f2[F_EPS]) / 3.0;
  const double U = ((f0[F_U] + f1[F_U]) + f2[F_U]) / 3.0;
  const double V = ((f0[F_V] + f1[F_V]) + f2[F_V]) / 3.0;
  const double x0 = src[3 * ens], y0 = src[3 * ens + 1], r0 = src[3 * ens + 2];
  const double second = fmax(k / eps, CT * sqrt(nu / eps));
  double tm = second;
  if (r0 > 0.0) {
    const double Uc = sqrt(U * U + V * V);
    const double dx = xc - x0, dy = yc - y0;
    const double dist = sqrt(dx * dx + dy * dy);
    double first = Cs * newton_cbrt(r0 * r0 / eps);
    if (Uc >= 1e-12) {
      first = first + Ct * dist / Uc;
      tm = fmin(first, second);
    }
  }
  rate[cell] = (T)fmin(dt / tm, 1.0);
}

// Wall-function alpha, eqs. (22)-(26), per wall-function edge: frozen fields
// at the edge midpoint in the edge frame (tangent t, inward normal n).
__global__ void k_alpha(const double* vtx, const int32_t* tri, const int32_t* ekind, const double* fields,
                        double* alpha, int ne, double Cmu, double kappa, double Ewall, double yp, double nu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * ne) return;
  alpha[i] = 0.0;
  if (ekind[i] != EDGE_WALLFN) return;
  const int e = i / 3, k = i - 3 * e;
  const int a = tri[3 * e + k], b = tri[3 * e + (k == 2 ? 0 : k + 1)];
  const double ex = vtx[2 * b] - vtx[2 * a], ey = vtx[2 * b + 1] - vtx[2 * a + 1];
  const double len = sqrt(ex * ex + ey * ey);
  const double nx = ey / len, ny = -ex / len;
  const double tx = -ny, ty = nx;
  const double nix = -nx, niy = -ny;
  const double* fa = fields + (size_t)a * NFIELD;
  const double* fb = fields + (size_t)b * NFIELD;
  const double U = (fa[F_U] + fb[F_U]) / 2.0, V = (fa[F_V] + fb[F_V]) / 2.0;
  const double R11 = (fa[F_R11] + fb[F_R11]) / 2.0, R22 = (fa[F_R22] + fb[F_R22]) / 2.0;
  const double R33 = (fa[F_R33] + fb[F_R33]) / 2.0, R12 = (fa[F_R12] + fb[F_R12]) / 2.0;
  const double Px = (fa[F_DPDX] + fb[F_DPDX]) / 2.0, Py = (fa[F_DPDY] + fb[F_DPDY]) / 2.0;
  const double Up = U * tx + V * ty;
  const double v2 = (nix * R11 + niy * R12) * nix + (nix * R12 + niy * R22) * niy;
  const double uv = (tx * R11 + ty * R12) * nix + (tx * R12 + ty * R22) * niy;
  const double dPdx = Px * tx + Py * ty;
  const double kp = 0.5 * ((R11 + R22) + R33);
  const double uhat = sqrt(sqrt(Cmu)) * sqrt(kp);
  const double prod = uv * dPdx;
  const double gamma_tau = prod > 0.0 ? 1.0 : 0.0;
  const double ustar = sqrt(uhat * uhat + gamma_tau * fabs(yp * dPdx));
  const double Ue = ustar / kappa * series_log<double>(Ewall * yp * ustar / nu);
  alpha[i] = 2.0 * uhat * uhat * Up * fabs(Up) / (v2 * Ue * Ue);
}

// Initial particles: uniform in the element, velocity = local mean plus the
// Cholesky factor of the local Reynolds stress times normals, scalar by rule.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_seed(MeshDev M, const double* fields, StateDev<T> st,
                                                const int32_t* start, const int32_t* count,
                                                const int32_t* idoff, const uint64_t* seeds, int ncell,
                                                int psi_init) {
  const int lane = lane_id();
  const int cell = blockIdx.x * WAVES_PER_BLOCK + threadIdx.x / WAVE;
  if (cell >= ncell) return;
  const int ne = M.ne;
  const int ens = cell / ne, e = cell - ens * ne;
  const int v0 = M.tri[3 * e], v1 = M.tri[3 * e + 1], v2 = M.tri[3 * e + 2];
  const double ax = M.vtx[2 * v0], ay = M.vtx[2 * v0 + 1];
  const double bx = M.vtx[2 * v1] - ax, by = M.vtx[2 * v1 + 1] - ay;
  const double cx = M.vtx[2 * v2] - ax, cy = M.vtx[2 * v2 + 1] - ay;
  const double gx = ((M.vtx[2 * v0] + M.vtx[2 * v1]) + M.vtx[2 * v2]) / 3.0;
  const double gy = ((M.vtx[2 * v0 + 1] + M.vtx[2 * v1 + 1]) + M.vtx[2 * v2 + 1]) / 3.0;
  const double Ax = M.vtx[2 * v0], Ay = M.vtx[2 * v0 + 1];
  const double Bx = M.vtx[2 * v1], By = M.vtx[2 * v1 + 1];
  const double Cx = M.vtx[2 * v2], Cy = M.vtx[2 * v2 + 1];
  const double ia = M.inv2a[e];
  const double* f0 = fields + (size_t)v0 * NFIELD;
  const double* f1 = fields + (size_t)v1 * NFIELD;
  const double* f2 = fields + (size_t)v2 * NFIELD;
  const uint64_t seed = seeds[ens];
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int n = count[cell], s0 = start[cell], id0 = idoff[cell];
  for (int j = lane; j < n; j += WAVE) {
    const uint32_t id = (uint32_t)(id0 + j);
    uint32_t r[8];
    philox_words(id, SEED_STEP, (uint32_t)ens, k0, k1, r, 2);
    double s1 = uniform01<double>(r[0]), s2 = uniform01<double>(r[1]);
    if (s1 + s2 > 1.0) {
      s1 = 1.0 - s1;
      s2 = 1.0 - s2;
    }
    const double px = ax + s1 * bx + s2 * cx;
    const double py = ay + s1 * by + s2 * cy;
    T tx = (T)px, ty = (T)py;
#pragma unroll 1
    for (int it = 0; it < 64; ++it) {
      const double qx = (double)tx, qy = (double)ty;
      if (orient_edge(Ax, Ay, Bx, By, qx, qy) >= 0.0 && orient_edge(Bx, By, Cx, Cy, qx, qy) >= 0.0 &&
          orient_edge(Cx, Cy, Ax, Ay, qx, qy) >= 0.0)
        break;
      tx = (T)((qx + gx) / 2.0);
      ty = (T)((qy + gy) / 2.0);
    }
    double z0, z1, z2, z3;
    box_muller<double>(r[2], r[3], &z0, &z1);
    box_muller<double>(r[4], r[5], &z2, &z3);
    const double X = (double)tx, Y = (double)ty;
    const double l0 = orient_edge(Bx, By, Cx, Cy, X, Y) * ia;
    const double l1 = orient_edge(Cx, Cy, Ax, Ay, X, Y) * ia;
    const double l2 = orient_edge(Ax, Ay, Bx, By, X, Y) * ia;
#define PDF_INTERP(j2) ((l0 * f0[j2] + l1 * f1[j2]) + l2 * f2[j2])
    const double U = PDF_INTERP(F_U), V = PDF_INTERP(F_V);
    const double R11 = PDF_INTERP(F_R11), R22 = PDF_INTERP(F_R22), R33 = PDF_INTERP(F_R33);
    const double R12 = PDF_INTERP(F_R12);
#undef PDF_INTERP
    const double L11 = sqrt(R11);
    const double L21 = R12 / L11;
    const double L22 = sqrt(R22 - L21 * L21);
    const double L33 = sqrt(R33);
    const int s = s0 + j;
    st.x[s] = tx;
    st.y[s] = ty;
    st.u[s] = (T)(U + L11 * z0);
    st.v[s] = (T)(V + (L21 * z0 + L22 * z1));
    st.w[s] = (T)(L33 * z2);
    st.psi[s] = (T)((psi_init == 1 && X < 0.25) ? 1.0 : 0.0);
    st.id[s] = id;
  }
}

// State of one ensemble in particle-id order (doubles) plus element index.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gather(StateDev<T> b0, StateDev<T> b1, const int32_t* cnt0,
                                                  const int32_t* cnt1, const int32_t* start,
                                                  const int32_t* cap, const Ctl* ctl, int ens, int ne,
                                                  int64_t n, double* out, int32_t* elem) {
  const int lane = lane_id();
  const int e = blockIdx.x * WAVES_PER_BLOCK + threadIdx.x / WAVE;
  if (e >= ne) return;
  const uint32_t par = ctl->parity;
  const StateDev<T> st = par ? b1 : b0;
  const int cell = ens * ne + e;
  int c = (par ? cnt1 : cnt0)[cell];
  if (c > cap[cell]) c = cap[cell];
  const int s0 = start[cell];
  for (int j = lane; j < c; j += WAVE) {
    const int s = s0 + j;
    const int64_t id = st.id[s];
    if (id < 0 || id >= n) continue;
    out[id] = (double)st.x[s];
    out[n + id] = (double)st.y[s];
    out[2 * n + id] = (double)st.u[s];
    out[3 * n + id] = (double)st.v[s];
    out[4 * n + id] = (double)st.w[s];
    out[5 * n + id] = (double)st.psi[s];
    elem[id] = e;
  }
}

__global__ void k_reset_ctl(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->step = 0; ctl->parity = 0; ctl->error = 0; ctl->halt = 0; ctl->done = 0; ctl->ovf = 0;
    ctl->steps_done = 0; ctl->lost = 0;
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace pdf
