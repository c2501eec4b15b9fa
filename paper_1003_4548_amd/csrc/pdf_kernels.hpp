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
// One wavefront (64 lanes) owns one cell per step.  It reads the segment once
// into LDS, estimates the cell's statistics with lane-strided FP64
// accumulators and DPP row reductions (no atomics), uses them for IECM,
// advances every particle, tracks it through the mesh, writes the particles
// that stay back to its own segment in order, and appends the ones that move
// to their new cell's segment with one atomic per particle.
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
  uint32_t parity;    // particle buffer holding the current state
  uint32_t crot;      // counter set holding the current counts (0..2)
  int32_t error;      // OR of ERR_* raised since seeding
  int32_t halt;       // set at the end of a step that raised an error
  uint32_t spare;
  uint32_t ovf;       // particles written to the overflow area
  uint32_t lost;
  int64_t steps_done; // steps completed since seeding
  uint32_t pad[6];
};

// Element record for tracking: vertex coordinates and, per edge k
// (v_k -> v_k+1), code = kind | (neighbour + 1) << 4.  64 bytes, one
// vector-load group per walk step.
struct alignas(64) ERec {
  double x[3];
  double y[3];
  int32_t code[3];
  int32_t pad;
};
static_assert(sizeof(ERec) == 64, "element record must be 64 bytes");

template <typename T> struct StateDev {
  T* x; T* y; T* u; T* v; T* w; T* psi;
  uint32_t* id;
};

// A cell's particles sit in two runs of its segment: the ones that stayed in
// the element, written by the cell's own wavefront from the bottom
// (count ns), and the ones that arrived from other elements, appended from the
// top with an atomic counter (count nm).  Counter sets rotate over three
// buffers: the current counts (read only), the next counts (being written),
// and the set two steps back, cleared for the step after.
template <typename T> struct StepArgs {
  const ERec* erec;       // ne
  const int32_t* tri;     // ne x 3
  const double* inv2a;    // ne
  const double* alpha;    // ne x 3
  double Lx, Ly;
  int32_t ne;
  int32_t ncell;
  const T* coef;          // nv x 16
  const T* rate;          // ncell
  const int32_t* start;   // ncell
  const int32_t* cap;     // ncell
  int32_t* ns[3];         // ncell each
  int32_t* nm[3];         // ncell each
  StateDev<T> buf[2];
  StateDev<T> ovf;        // overflow area
  int32_t* ovf_cell;
  uint32_t ovf_cap;
  double* stats;          // ncell x nstat
  const uint64_t* seed;   // nens
  const double* src;      // nens x 3
  Ctl* ctl;
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

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <int CTRL> __device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Sum over the 64 lanes, returned wave-uniform.  Rows of 16 lanes are reduced
// with DPP (quad swaps, half-row and row mirrors: every lane of a row ends with
// the same row sum), then the four row sums are combined in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
  const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
  return (r0 + r1) + (r2 + r3);
}

// Sums of K per-lane values, delivered transposed: lane q (q < K) receives
// the wave sum of value q, other lanes 0.  Quads are reduced with DPP, the 16
// quad sums of each value go through LDS (row stride 17 doubles against bank
// conflicts), and lane q adds its 16 quad sums in order.  The order of every
// addition is fixed, so the result does not depend on timing.
constexpr int RED_STRIDE = 17;

template <int K>
__device__ __forceinline__ double wave_sums_to_lanes(const double (&vals)[K], double* red) {
  const int lane = lane_id();
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double v = vals[q];
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if ((lane & 3) == 0) red[q * RED_STRIDE + (lane >> 2)] = v;
  }
  double s = 0.0;
  if (lane < K) {
#pragma unroll
    for (int r = 0; r < 16; ++r) s += red[lane * RED_STRIDE + r];
  }
  return s;
}

template <typename T> __device__ __forceinline__ T pick3(const T* a, int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}

__device__ __forceinline__ int slot_of(int j, int start, int ns, int nm, int capc) {
  return j < ns ? start + j : start + capc - nm + (j - ns);
}

// ---------------------------------------------------------------------------
// tracking: straight-line neighbour walk with wall and periodic conditions.
// Exit edge: the first edge (lowest local index) the target lies outside of
// whose endpoints the line start->target separates; if rounding leaves none,
// the edge the target is most outside of.  Walls mirror the rest of the path
// about the wall line and reflect the velocity; periodic edges shift the path
// by one period into the partner element.  R holds the record of element e.

template <typename T>
__device__ int walk(const StepArgs<T>& a, ERec R, int e, double Sx, double Sy, T& tx, T& ty, T& u, T& v,
                    T& w) {
#pragma unroll 1
  for (int it = 0; it < 64; ++it) {
    const double Tx = (double)tx, Ty = (double)ty;
    const double o0 = orient_edge(R.x[0], R.y[0], R.x[1], R.y[1], Tx, Ty);
    const double o1 = orient_edge(R.x[1], R.y[1], R.x[2], R.y[2], Tx, Ty);
    const double o2 = orient_edge(R.x[2], R.y[2], R.x[0], R.y[0], Tx, Ty);
    if (o0 >= 0.0 && o1 >= 0.0 && o2 >= 0.0) return e;
    int ex = -1;
    {
      const double o[3] = {o0, o1, o2};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        if (ex < 0 && o[k] < 0.0) {
          const double sa = orient2d(Sx, Sy, Tx, Ty, R.x[k], R.y[k]);
          const double sb = orient2d(Sx, Sy, Tx, Ty, R.x[k1], R.y[k1]);
          if ((sa <= 0.0 && sb >= 0.0) || (sa >= 0.0 && sb <= 0.0)) ex = k;
        }
      }
      if (ex < 0) {
        ex = 0;
        if (o1 < o0) ex = 1;
        if (o2 < (ex == 0 ? o0 : o1)) ex = 2;
      }
    }
    const int code = pick3(R.code, ex);
    const int kind = code & 15;
    const int nb = (code >> 4) - 1;
    if (kind == EDGE_INTERIOR) {
      e = nb;
      R = a.erec[e];
      continue;
    }
    if (kind >= EDGE_PXP) {
      double sx = 0.0, sy = 0.0;
      if (kind == EDGE_PXP) sx = a.Lx;
      if (kind == EDGE_PXM) sx = -a.Lx;
      if (kind == EDGE_PYP) sy = a.Ly;
      if (kind == EDGE_PYM) sy = -a.Ly;
      Sx = Sx + sx;
      Sy = Sy + sy;
      tx = tx + (T)sx;
      ty = ty + (T)sy;
      e = nb;
      R = a.erec[e];
      continue;
    }
    const int ex1 = ex == 2 ? 0 : ex + 1;
    const double ax = pick3(R.x, ex), ay = pick3(R.y, ex);
    const double bx = pick3(R.x, ex1), by = pick3(R.y, ex1);
    const double gx = bx - ax, gy = by - ay;
    const double len = sqrt(gx * gx + gy * gy);
    const double nx = gy / len, ny = -gx / len;  // outward unit normal
    const double oS = orient_edge(ax, ay, bx, by, Sx, Sy);
    const double oT = ex == 0 ? o0 : (ex == 1 ? o1 : o2);
    const double den = oS - oT;
    const double tpar = den > 0.0 ? oS / den : 0.0;
    const double Ix = Sx + tpar * (Tx - Sx), Iy = Sy + tpar * (Ty - Sy);
    const double d = (Tx - ax) * nx + (Ty - ay) * ny;
    tx = (T)(Tx - (2.0 * d) * nx);
    ty = (T)(Ty - (2.0 * d) * ny);
#pragma unroll 1
    for (int j = 0; j < 8; ++j) {
      if (!(orient_edge(ax, ay, bx, by, (double)tx, (double)ty) < 0.0)) break;
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
      const T al = (T)a.alpha[3 * e + ex];
      const T Ur = Ui + al * Vi;
      const T Vr = -Vi;
      u = Ur * tX + Vr * (-nxT);
      v = Ur * tY + Vr * (-nyT);
    }
  }
  return -1;
}

// ---------------------------------------------------------------------------
// the fused step.  One wavefront per cell:
//   A  read the cell's particles once from HBM into an LDS tile (the first
//      TILE of them; a larger cell re-reads the rest from L2) and sum the
//      velocity and scalar: the means;
//   B  central moments, velocity-bin counts and scalar sums, histogram: the
//      statistics record of the cell;
//   C  IECM with those statistics, velocity, position, tracking, source;
//      stayers are written back in order without atomics, movers are
//      appended to their new cell.
// ADVANCE = false stops after B.

template <int MOM> struct MomCount { static constexpr int M3 = 0, M4 = 0; };
template <> struct MomCount<4> { static constexpr int M3 = 20, M4 = 35; };

// position of (x, y), x <= y, in the lexicographic list of index pairs of (u, v, w, psi)
__host__ __device__ constexpr int pair_index(int x, int y) { return x * 4 - (x * (x - 1)) / 2 + (y - x); }

// position of (x, y, z), x <= y <= z, in the lexicographic list of index triples
__host__ __device__ constexpr int triple_index(int x, int y, int z) {
  int it = 0;
  for (int p = 0; p < 4; ++p)
    for (int q = p; q < 4; ++q)
      for (int r = q; r < 4; ++r)
        if (p < x || (p == x && (q < y || (q == y && r < z)))) ++it;
  return it;
}

constexpr int TILE = 256;  // particles of a cell staged in LDS
constexpr int RED_MAX = 20; // values reduced together

template <typename T> struct Tile {
  T x[TILE], y[TILE], u[TILE], v[TILE], w[TILE], psi[TILE];
  uint32_t id[TILE];
};

template <typename T, int MOM, int HIST, bool ADVANCE>
__global__ __launch_bounds__(BLOCK) void k_step(StepArgs<T> a) {
  __shared__ Tile<T> tiles[WAVES_PER_BLOCK];
  __shared__ double red_lds[WAVES_PER_BLOCK][RED_MAX * RED_STRIDE];
  __shared__ int hist_lds[WAVES_PER_BLOCK][HIST > 0 ? HIST : 1];
  Ctl* ctl = a.ctl;
  if (ADVANCE && ctl->halt) return;
  const uint32_t step = ctl->step;
  const uint32_t par = ctl->parity;
  const uint32_t rot = ctl->crot;
  const int lane = lane_id();
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int cell = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + wid;
  const int rc = (int)rot, rn = (int)(rot == 2 ? 0 : rot + 1), rz = (int)(rot == 0 ? 2 : rot - 1);

  if (cell < a.ncell) {
    const StateDev<T> src = a.buf[par];
    const StateDev<T> dst = a.buf[par ^ 1u];
    Tile<T>& L = tiles[wid];
    const int ne = a.ne;
    const int ens = cell / ne;
    const int e = cell - ens * ne;
    const int start = a.start[cell];
    const int capc = a.cap[cell];
    // counts are clamped to the segment so that even the step after an
    // overflow (whose results are void) reads inside the segment
    const int ns = min(a.ns[rc][cell], capc);
    const int nm = min(a.nm[rc][cell], capc - ns);
    const int n = ns + nm;
    const double dn = (double)n;

    // ---- A: load, stage, means ----
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    {
      // the staged part: all TILE/WAVE loads in flight together
      T tx_[TILE / WAVE], ty_[TILE / WAVE], tu_[TILE / WAVE], tv_[TILE / WAVE], tw_[TILE / WAVE], tp_[TILE / WAVE];
      uint32_t ti_[TILE / WAVE];
#pragma unroll
      for (int c = 0; c < TILE / WAVE; ++c) {
        const int j = c * WAVE + lane;
        if (j < n) {
          const int s = slot_of(j, start, ns, nm, capc);
          tx_[c] = src.x[s]; ty_[c] = src.y[s]; tu_[c] = src.u[s]; tv_[c] = src.v[s]; tw_[c] = src.w[s];
          tp_[c] = src.psi[s]; ti_[c] = src.id[s];
        }
      }
#pragma unroll
      for (int c = 0; c < TILE / WAVE; ++c) {
        const int j = c * WAVE + lane;
        if (j < n) {
          L.x[j] = tx_[c]; L.y[j] = ty_[c]; L.u[j] = tu_[c]; L.v[j] = tv_[c]; L.w[j] = tw_[c]; L.psi[j] = tp_[c];
          L.id[j] = ti_[c];
          s0 += (double)tu_[c];
          s1 += (double)tv_[c];
          s2 += (double)tw_[c];
          s3 += (double)tp_[c];
        }
      }
    }
    for (int base = TILE; base < n; base += WAVE) {
      const int j = base + lane;
      if (j < n) {
        const int s = slot_of(j, start, ns, nm, capc);
        const T u = src.u[s], v = src.v[s], w = src.w[s], p = src.psi[s];
        s0 += (double)u;
        s1 += (double)v;
        s2 += (double)w;
        s3 += (double)p;
      }
    }
    double* red = red_lds[wid];
    const double inv_n = n > 0 ? 1.0 / dn : 0.0;
    double mean[4];
    {
      const double sums[4] = {s0, s1, s2, s3};
      const double mean_l = wave_sums_to_lanes<4>(sums, red) * inv_n;
#pragma unroll
      for (int q = 0; q < 4; ++q) mean[q] = readlane_f64(mean_l, q);
    }

    auto load4 = [&](int j, double* val) {
      if (j < TILE) {
        val[0] = (double)L.u[j]; val[1] = (double)L.v[j]; val[2] = (double)L.w[j]; val[3] = (double)L.psi[j];
      } else {
        const int s = slot_of(j, start, ns, nm, capc);
        val[0] = (double)src.u[s]; val[1] = (double)src.v[s]; val[2] = (double)src.w[s]; val[3] = (double)src.psi[s];
      }
    };

    // ---- B: second moments, bins, histogram ----
    double acc[18];  // 10 second moments, 8 per-bin scalar sums
#pragma unroll
    for (int q = 0; q < 18; ++q) acc[q] = 0.0;
    int bcount[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) bcount[q] = 0;
    if (HIST > 0) {
      for (int h = lane; h < HIST; h += WAVE) hist_lds[wid][h] = 0;
    }
    for (int base = 0; base < n; base += WAVE) {
      const int j = base + lane;
      const bool act = j < n;
      int bin = -1;
      if (act) {
        double val[4];
        load4(j, val);
        double d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = val[q] - mean[q];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = x; y < 4; ++y) acc[pair_index(x, y)] += d[x] * d[y];
        bin = (val[0] > mean[0] ? 1 : 0) + (val[1] > mean[1] ? 2 : 0) + (val[2] > mean[2] ? 4 : 0);
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[10 + q] += (bin == q) ? val[3] : 0.0;
        if (HIST > 0) {
          const double hpos = floor(val[3] * (double)HIST);
          const int hb = hpos < 0.0 ? 0 : (hpos >= (double)HIST ? HIST - 1 : (int)hpos);
          atomicAdd(&hist_lds[wid][hb], 1);
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) bcount[q] += (int)__popcll(__ballot(bin == q));
    }
    const double sumB = wave_sums_to_lanes<18>(acc, red);
    // lane q < 10: second moment q; lane 10 + b: scalar sum of bin b
    double cnt_l = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) cnt_l = (lane == 10 + q) ? (double)bcount[q] : cnt_l;
    const double bm_l = cnt_l > 0.0 ? sumB / cnt_l : mean[3];
    double bm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) bm[q] = readlane_f64(bm_l, 10 + q);
    double* rec = a.stats + (size_t)cell * a.nstat;
    {
      // one store per lane: lanes 0-9 second moments, 10-17 bin means,
      // 18-25 bin counts, 26 count, 27-30 means
      int idx = -1;
      double val = 0.0;
      if (lane < 10) { idx = ST_M2 + lane; val = sumB * inv_n; }
      else if (lane < 18) { idx = ST_BINM + (lane - 10); val = bm_l; }
      else if (lane < 26) {
        idx = ST_BINN + (lane - 18);
        double c = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) c = (lane == 18 + q) ? (double)bcount[q] : c;
        val = c;
      } else if (lane == 26) { idx = ST_N; val = dn; }
      else if (lane < 31) {
        idx = ST_MEAN + (lane - 27);
        double mq = mean[0];
#pragma unroll
        for (int q = 1; q < 4; ++q) mq = (lane == 27 + q) ? mean[q] : mq;
        val = mq;
      }
      if (n == 0) val = 0.0;
      if (idx >= 0) rec[idx] = val;
    }
    if constexpr (MOM >= 4) {
      // third-order moments
      double m3[20];
#pragma unroll
      for (int q = 0; q < 20; ++q) m3[q] = 0.0;
      for (int base = 0; base < n; base += WAVE) {
        const int j = base + lane;
        if (j < n) {
          double val[4], d[4];
          load4(j, val);
#pragma unroll
          for (int q = 0; q < 4; ++q) d[q] = val[q] - mean[q];
          int i3 = 0;
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = x; y < 4; ++y)
#pragma unroll
              for (int z = y; z < 4; ++z) { m3[i3] += (d[x] * d[y]) * d[z]; ++i3; }
        }
      }
      const double s3l = wave_sums_to_lanes<20>(m3, red);
      if (lane < 20) rec[ST_M3 + lane] = s3l * inv_n;
      // fourth-order moments, in two groups to bound the accumulator count
#pragma unroll
      for (int grp = 0; grp < 2; ++grp) {
        constexpr int G0 = 18;
        const int lo = grp == 0 ? 0 : G0, hi = grp == 0 ? G0 : 35;
        double m4[G0];
#pragma unroll
        for (int q = 0; q < G0; ++q) m4[q] = 0.0;
        for (int base = 0; base < n; base += WAVE) {
          const int j = base + lane;
          if (j < n) {
            double val[4], d[4];
            load4(j, val);
#pragma unroll
            for (int q = 0; q < 4; ++q) d[q] = val[q] - mean[q];
            int i4 = 0;
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = x; y < 4; ++y)
#pragma unroll
                for (int z = y; z < 4; ++z)
#pragma unroll
                  for (int g = z; g < 4; ++g) {
                    if (i4 >= lo && i4 < hi) m4[i4 - lo] += ((d[x] * d[y]) * d[z]) * d[g];
                    ++i4;
                  }
          }
        }
        const double s4l = wave_sums_to_lanes<G0>(m4, red);
        if (lane < hi - lo) rec[ST_M4 + lo + lane] = s4l * inv_n;
      }
    }
    if (HIST > 0) {
      const int off = MOM >= 4 ? NSTAT4 : NSTAT2;
      for (int h = lane; h < HIST; h += WAVE) rec[off + h] = (double)hist_lds[wid][h];
    }

    if (ADVANCE) {
      // ---- C: advance ----
      const ERec R0 = a.erec[e];
      const int v0 = a.tri[3 * e], v1 = a.tri[3 * e + 1], v2 = a.tri[3 * e + 2];
      const double ia = a.inv2a[e];
      const T* q0 = a.coef + (size_t)v0 * NCOEF;
      const T* q1 = a.coef + (size_t)v1 * NCOEF;
      const T* q2 = a.coef + (size_t)v2 * NCOEF;
      const T rate = a.rate[cell];
      const uint64_t seed = a.seed[ens];
      const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
      const double sx0 = a.src[3 * ens], sy0 = a.src[3 * ens + 1], sr0 = a.src[3 * ens + 2];
      const bool do_mix = a.mix && (a.flags & FLAG_MIX);
      int err = 0;
      int stay_count = 0;
      for (int base = 0; base < n; base += WAVE) {
        const int j = base + lane;
        const bool act = j < n;
        int e2 = -1;
        T xn = 0, yn = 0, un = 0, vn = 0, wn = 0, psi = 0;
        uint32_t id = 0;
        if (act) {
          T x, y, u, v, w;
          if (j < TILE) {
            x = L.x[j]; y = L.y[j]; u = L.u[j]; v = L.v[j]; w = L.w[j]; psi = L.psi[j]; id = L.id[j];
          } else {
            const int s = slot_of(j, start, ns, nm, capc);
            x = src.x[s]; y = src.y[s]; u = src.u[s]; v = src.v[s]; w = src.w[s]; psi = src.psi[s]; id = src.id[s];
          }
          uint32_t rw[8];
          philox_words<2>(id, step, (uint32_t)ens, k0, k1, rw);
          T xi0, xi1, xi2, xi3, xi4, xi5;
          box_muller<T>(rw[0], rw[1], &xi0, &xi1);
          box_muller<T>(rw[2], rw[3], &xi2, &xi3);
          box_muller<T>(rw[4], rw[5], &xi4, &xi5);
          (void)xi5;
          const double X = (double)x, Y = (double)y;
          const T l0 = (T)(orient_edge(R0.x[1], R0.y[1], R0.x[2], R0.y[2], X, Y) * ia);
          const T l1 = (T)(orient_edge(R0.x[2], R0.y[2], R0.x[0], R0.y[0], X, Y) * ia);
          const T l2 = (T)(orient_edge(R0.x[0], R0.y[0], R0.x[1], R0.y[1], X, Y) * ia);
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
          e2 = e;
          if (a.flags & FLAG_POS) {
            e2 = walk<T>(a, R0, e, X, Y, xn, yn, un, vn, wn);
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
          }
        }
        // stayers: own segment, bottom run, in lane order, no atomics
        const bool stay = act && e2 == e;
        const uint64_t smask = __ballot(stay);
        if (stay) {
          const int s = start + stay_count + (int)__popcll(smask & lanemask_lt());
          dst.x[s] = xn; dst.y[s] = yn; dst.u[s] = un; dst.v[s] = vn; dst.w[s] = wn; dst.psi[s] = psi;
          dst.id[s] = id;
        }
        stay_count += (int)__popcll(smask);
        // movers: top run of the new cell's segment
        if (act && e2 >= 0 && e2 != e) {
          const int t = ens * ne + e2;
          const int k = atomicAdd(&a.nm[rn][t], 1);
          const int capt = a.cap[t];
          const int limit = capt - (a.ns[rc][t] + a.nm[rc][t]);
          if (k < limit) {
            const int s = a.start[t] + capt - 1 - k;
            dst.x[s] = xn; dst.y[s] = yn; dst.u[s] = un; dst.v[s] = vn; dst.w[s] = wn; dst.psi[s] = psi;
            dst.id[s] = id;
          } else {
            err |= ERR_CAPACITY;
            const uint32_t kk = atomicAdd(&ctl->ovf, 1u);
            if (kk < a.ovf_cap) {
              a.ovf.x[kk] = xn; a.ovf.y[kk] = yn; a.ovf.u[kk] = un; a.ovf.v[kk] = vn; a.ovf.w[kk] = wn;
              a.ovf.psi[kk] = psi; a.ovf.id[kk] = id;
              a.ovf_cell[kk] = t;
            } else {
              err |= ERR_OVERFLOW_FULL;
            }
          }
        }
      }
      if (lane == 0) {
        a.ns[rn][cell] = stay_count;
        a.ns[rz][cell] = 0;
        a.nm[rz][cell] = 0;
      }
      int werr = 0;
#pragma unroll
      for (int bit = 0; bit < 4; ++bit)
        if (__ballot((err >> bit) & 1)) werr |= 1 << bit;
      if (lane == 0 && werr) atomicOr(&ctl->error, werr);
    }
  }
}

// End of a step: advance the step counter, swap the particle buffers, rotate
// the counter sets, and stop further steps once an error was raised.  A
// separate one-thread launch: the kernel boundary orders it after every
// workgroup of the step without any device-wide fence in the step itself.
__global__ void k_step_end(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && !ctl->halt) {
    ctl->step = ctl->step + 1;
    ctl->parity = ctl->parity ^ 1u;
    ctl->crot = ctl->crot == 2 ? 0 : ctl->crot + 1;
    ctl->steps_done = ctl->steps_done + 1;
    if (ctl->error != 0) ctl->halt = 1;
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

// Per-element tracking records.
__global__ void k_erec(const double* vtx, const int32_t* tri, const int32_t* nbr, const int32_t* ekind,
                       ERec* erec, int ne) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  ERec r;
  for (int k = 0; k < 3; ++k) {
    const int v = tri[3 * e + k];
    r.x[k] = vtx[2 * v];
    r.y[k] = vtx[2 * v + 1];
    r.code[k] = ekind[3 * e + k] | ((nbr[3 * e + k] + 1) << 4);
  }
  r.pad = 0;
  erec[e] = r;
}

// Initial particles: uniform in the element, velocity = local mean plus the
// Cholesky factor of the local Reynolds stress times normals, scalar by rule.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_seed(const ERec* erec, const int32_t* tri, const double* inv2a,
                                                const double* fields, StateDev<T> st, const int32_t* start,
                                                const int32_t* count, const int32_t* idoff,
                                                const uint64_t* seeds, int ne, int ncell, int psi_init) {
  const int lane = lane_id();
  const int cell = blockIdx.x * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
  if (cell >= ncell) return;
  const int ens = cell / ne, e = cell - ens * ne;
  const ERec R = erec[e];
  const int v0 = tri[3 * e], v1 = tri[3 * e + 1], v2 = tri[3 * e + 2];
  const double Ax = R.x[0], Ay = R.y[0], Bx = R.x[1], By = R.y[1], Cx = R.x[2], Cy = R.y[2];
  const double ax = Ax, ay = Ay;
  const double bx = Bx - ax, by = By - ay;
  const double cx = Cx - ax, cy = Cy - ay;
  const double gx = ((Ax + Bx) + Cx) / 3.0;
  const double gy = ((Ay + By) + Cy) / 3.0;
  const double ia = inv2a[e];
  const double* f0 = fields + (size_t)v0 * NFIELD;
  const double* f1 = fields + (size_t)v1 * NFIELD;
  const double* f2 = fields + (size_t)v2 * NFIELD;
  const uint64_t seed = seeds[ens];
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int n = count[cell], s0 = start[cell], id0 = idoff[cell];
  for (int j = lane; j < n; j += WAVE) {
    const uint32_t id = (uint32_t)(id0 + j);
    uint32_t r[8];
    philox_words<2>(id, SEED_STEP, (uint32_t)ens, k0, k1, r);
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
struct CounterSets {
  int32_t* ns[3];
  int32_t* nm[3];
};

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gather(StateDev<T> b0, StateDev<T> b1, CounterSets cs,
                                                  const int32_t* start, const int32_t* cap, const Ctl* ctl,
                                                  int ens, int ne, int64_t n, double* out, int32_t* elem) {
  const int lane = lane_id();
  const int e = blockIdx.x * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
  if (e >= ne) return;
  const uint32_t par = ctl->parity, rot = ctl->crot;
  const StateDev<T> st = par ? b1 : b0;
  const int cell = ens * ne + e;
  const int capc = cap[cell], s0 = start[cell];
  const int ns = min(cs.ns[rot][cell], capc);
  const int nm = min(cs.nm[rot][cell], capc - ns);
  const int c = ns + nm;
  for (int j = lane; j < c; j += WAVE) {
    const int s = slot_of(j, s0, ns, nm, capc);
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
    ctl->step = 0; ctl->parity = 0; ctl->crot = 0; ctl->error = 0; ctl->halt = 0; ctl->spare = 0;
    ctl->ovf = 0; ctl->lost = 0; ctl->steps_done = 0;
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace pdf
