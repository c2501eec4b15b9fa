// Kernels of the particle-in-cell joint velocity-scalar PDF step.
//
// Data layout in HBM (structure of arrays):
//   particles  x y u v w psi (state type T), id (u32) and, with the
//              stochastic turbulent frequency, omega (T), in two buffers.
//              Each (ensemble, element) pair -- a "cell" -- owns a segment of
//              fixed capacity (resized by the device-side repack): the
//              particles that stayed in the element sit densely at its
//              bottom, those that arrived in the last step at its top.  A
//              particle's element is implied by the segment that holds it.
//   cells      segment start, capacity, particle count per buffer, IECM rate.
//   mesh       vertex coordinates (f64), element vertices / neighbours / edge
//              kinds (i32), 1/(2 area) (f64), wall-function alpha per edge.
//   vertices   16 drift/diffusion coefficients per vertex (T), row-major.
//
// A group of G lanes (4 to 64) owns one cell per step.  It reads the
// segment once into LDS, estimates the cell's statistics (per-lane FP64
// partial sums, then a fixed-order cross-lane tree, compensated for the
// fourth-order statistics; bin counts, bin scalar sums and the histogram by
// LDS atomics of the group's own wavefront, in its program order), uses them
// for IECM, advances every particle, tracks it through the mesh, writes the
// particles that stay back to its own segment in order, and appends the ones
// that move to their new cell's segment (one atomic per target cell and
// wavefront).  The order of arrivals from different wavefronts is not fixed,
// so sums over a cell's particles can differ in their last bits from run to
// run; trajectories do not depend on it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pdf_math.hpp"
#include "pdf_mlp_core.hpp"

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
  uint32_t step_base;  // Philox step word of the first step of the running pdf_step call
  int32_t error;       // OR of ERR_* raised since seeding
  uint32_t ovf;        // particles written to the overflow area
  uint32_t next[2];    // work counters of the persistent scheduler, by step parity
  uint32_t repack;     // set by a step that found a segment near its capacity
  uint32_t active;     // the repack in progress (copied from repack by the planner)
  uint32_t flip;       // XOR applied to the step parity to select the particle buffer
  uint32_t repacks;    // repacks done since seeding
  uint32_t pad[7];
};
static_assert(sizeof(Ctl) == 64, "control block is 64 bytes");

// A segment needs a repack when its free room is under half its count (or
// under 16 slots), or under twice the arrivals of the last step: the
// arrivals of a step may only use the room beyond the current count, and a
// cell whose particles turn over quickly (near walls many cross every step)
// needs that room every step until the repack.  nm: arrivals of the last step.
__device__ __forceinline__ bool repack_due(int n, int nm, int cap) {
  const int room = cap - n;
  return 2 * room < max(32, n) || room < 2 * nm;
}

// Per-launch step indices, passed by value: the Philox step word is
// step_base + step_off; parity selects the particle buffer holding the
// current state; rot the counter set holding its counts.
struct StepIndex {
  uint32_t step_off;
  uint32_t parity;
  uint32_t rot;
  uint32_t pad;
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
  T* om;  // turbulent frequency, null when the state carries none
};

// A cell's particles sit in two runs of its segment: the ones that stayed in
// the element, written by the cell's own lane group from the bottom (count
// ns), and the ones that arrived from other elements, appended from the top
// with an atomic counter (count nm).  Counter sets rotate over three buffers:
// the current counts (read only), the next counts (being written), and the
// set two steps back, cleared for the step after.
template <typename T> struct StepArgs {
  const ERec* erec;       // ne
  const int32_t* tri;     // ne x 3
  const double* inv2a;    // ne
  const double* alpha;    // ne x 3
  const double* wnorm;    // ne x 3 x 2: outward unit normal of each element edge
  double Lx, Ly;
  int32_t ne;
  int32_t ncell;
  const int32_t* order;   // ncell: processing order of the cells
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
  const double* cmean;    // ncell x 8 conditional means for IECM from elsewhere, or null
  // learned conditional means computed inside the step (one-item-per-wavefront
  // grids only): network weights, normalisation, output and served count
  const uint16_t* mlp_w;  // null: not used
  const float* mlp_norm;
  double* mlp_cm;
  uint32_t* mlp_served;
  // stochastic turbulent frequency, eqs. (9)-(10) and the wall condition:
  // frozen <omega> and S_omega per element, frozen <omega> at the
  // wall-function edges (ne x 3), beta, y_p, nu C_T^2 (for the dissipation
  // estimate, eq. 8), C3, 2 C3 C4
  const double* om0;
  const double* somega;
  const double* omw;
  double om_beta, om_yp, om_nuct2;
  T om_c3, om_c34;
  Ctl* ctl;
  int32_t nstat;
  int32_t flags;
  int32_t mix;
  int32_t nitems;         // work items (wavefronts' worth of cells)
  int32_t pchunk;         // work items a persistent wavefront claims per atomic
  // one item per wavefront: the work items XCD x runs are [xcd[x], xcd[x+1]),
  // ranges of equal estimated cost (blocks reach the XCDs round-robin)
  int32_t xcd[9];
  T dt, sdt, nu2, s2nu;
};


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

__device__ __forceinline__ double shfl_xor_f64(double v, int m) {
  const long long b = __double_as_longlong(v);
  const int lo = __shfl_xor((int)(unsigned)(b & 0xffffffffll), m, WAVE);
  const int hi = __shfl_xor((int)(b >> 32), m, WAVE);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Sum over a group of G consecutive lanes, returned to every lane of the
// group.  A butterfly in a fixed order: quad swaps, half-row and row mirrors
// (DPP), then lane swaps across rows; every lane of a group gets the same bits.
template <int G> __device__ __forceinline__ double group_sum(double v) {
  v += dpp_f64<0xB1>(v);                      // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);                      // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
  if constexpr (G >= 16) v += dpp_f64<0x140>(v);  // row_mirror
  if constexpr (G >= 32) v += shfl_xor_f64(v, 16);
  if constexpr (G >= 64) v += shfl_xor_f64(v, 32);
  return v;
}

__device__ __forceinline__ double lo_hi_f64(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)lo | ((long long)hi << 32));
}

// Sums of K values over a group of G consecutive lanes by a transposing
// butterfly: at the stage of lane bit d, lanes with the bit clear keep the
// first ceil(Kc/2) of the Kc values the stage starts with, lanes with it set
// the rest, each adding its partner's copy of the ones it keeps, so the
// values per lane halve at every stage (a value without a partner in the
// second half is summed by both).  Bits 32 and 16 pair by the gfx950 lane
// swaps (the first value's upper half against the second's lower half),
// bits 8, 4, 2, 1 by DPP row rotation, half-row mirror and quad swaps.  Each
// sum ends in the lanes whose bits select it, which store it to out[index]
// (scaled by f) unless store is false; a caller that reads it from other
// lanes orders the two.  All lanes of the wavefront take part.  COMP: every
// addition of the tree is an error-free transformation (Knuth's TwoSum), the
// rounding errors travel with the values and are added once at the end, so
// the tree adds no rounding of its own beyond that last addition.
__device__ __forceinline__ double two_sum_err(double a, double b, double s) {
  const double bp = s - a;
  const double ap = s - bp;
  return (a - ap) + (b - bp);
}

template <int G, int K, bool COMP = false>
__device__ __forceinline__ void group_sum_many(double (&v)[K], double* out, double f = 1.0, bool store = true) {
  const int li = lane_id() & (G - 1);
  int off = 0, cnt = K;  // this lane's first index and count of valid values
  double c[COMP ? K : 1];
#pragma unroll
  for (int i = 0; i < (COMP ? K : 1); ++i) c[i] = 0.0;
  auto swap_pair = [&](auto dtag, double a, double b, double& x, double& y) {
    constexpr int D = decltype(dtag)::value;
    const long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
    const auto l = D == 32 ? __builtin_amdgcn_permlane32_swap((unsigned)ab, (unsigned)bb, false, false)
                           : __builtin_amdgcn_permlane16_swap((unsigned)ab, (unsigned)bb, false, false);
    const auto h = D == 32 ? __builtin_amdgcn_permlane32_swap((unsigned)(ab >> 32), (unsigned)(bb >> 32), false, false)
                           : __builtin_amdgcn_permlane16_swap((unsigned)(ab >> 32), (unsigned)(bb >> 32), false, false);
    x = lo_hi_f64(l[0], h[0]);
    y = lo_hi_f64(l[1], h[1]);
  };
  auto stage = [&](auto dtag, auto kctag) {
    constexpr int D = decltype(dtag)::value, KC = decltype(kctag)::value, KN = (KC + 1) / 2;
    const bool hi = (li & D) != 0;
#pragma unroll
    for (int i = 0; i < KN; ++i) {
      const double a = v[i], b = (i + KN < KC) ? v[i + KN] : a;
      double x, y;   // the kept value and the partner's copy of it
      if constexpr (D >= 16) {
        swap_pair(dtag, a, b, x, y);
      } else {
        constexpr int CTRL = D == 8 ? 0x128 : (D == 4 ? 0x141 : (D == 2 ? 0x4E : 0xB1));
        x = hi ? b : a;
        y = dpp_f64<CTRL>(hi ? a : b);
      }
      v[i] = x + y;
      if constexpr (COMP) {
        const double ca = c[i], cb = (i + KN < KC) ? c[i + KN] : ca;
        double cx, cy;
        if constexpr (D >= 16) {
          swap_pair(dtag, ca, cb, cx, cy);
        } else {
          constexpr int CTRL = D == 8 ? 0x128 : (D == 4 ? 0x141 : (D == 2 ? 0x4E : 0xB1));
          cx = hi ? cb : ca;
          cy = dpp_f64<CTRL>(hi ? ca : cb);
        }
        c[i] = (cx + cy) + two_sum_err(x, y, v[i]);
      }
    }
    if (hi) {
      off += KN;
      cnt = cnt > KN ? cnt - KN : 0;
    } else {
      cnt = cnt < KN ? cnt : KN;
    }
  };
  using I = int;
  constexpr int K1 = (K + 1) / 2, K2 = (K1 + 1) / 2, K3 = (K2 + 1) / 2, K4 = (K3 + 1) / 2, K5 = (K4 + 1) / 2;
  // stages from the highest lane bit of the group down, the value count
  // halving from K as they go
  if constexpr (G == 64) {
    stage(std::integral_constant<I, 32>{}, std::integral_constant<I, K>{});
    stage(std::integral_constant<I, 16>{}, std::integral_constant<I, K1>{});
    stage(std::integral_constant<I, 8>{}, std::integral_constant<I, K2>{});
    stage(std::integral_constant<I, 4>{}, std::integral_constant<I, K3>{});
    stage(std::integral_constant<I, 2>{}, std::integral_constant<I, K4>{});
    stage(std::integral_constant<I, 1>{}, std::integral_constant<I, K5>{});
  } else if constexpr (G == 32) {
    stage(std::integral_constant<I, 16>{}, std::integral_constant<I, K>{});
    stage(std::integral_constant<I, 8>{}, std::integral_constant<I, K1>{});
    stage(std::integral_constant<I, 4>{}, std::integral_constant<I, K2>{});
    stage(std::integral_constant<I, 2>{}, std::integral_constant<I, K3>{});
    stage(std::integral_constant<I, 1>{}, std::integral_constant<I, K4>{});
  } else if constexpr (G == 16) {
    stage(std::integral_constant<I, 8>{}, std::integral_constant<I, K>{});
    stage(std::integral_constant<I, 4>{}, std::integral_constant<I, K1>{});
    stage(std::integral_constant<I, 2>{}, std::integral_constant<I, K2>{});
    stage(std::integral_constant<I, 1>{}, std::integral_constant<I, K3>{});
  } else if constexpr (G == 8) {
    stage(std::integral_constant<I, 4>{}, std::integral_constant<I, K>{});
    stage(std::integral_constant<I, 2>{}, std::integral_constant<I, K1>{});
    stage(std::integral_constant<I, 1>{}, std::integral_constant<I, K2>{});
  } else {
    static_assert(G == 4, "groups of 4, 8, 16, 32 or 64 lanes");
    stage(std::integral_constant<I, 2>{}, std::integral_constant<I, K>{});
    stage(std::integral_constant<I, 1>{}, std::integral_constant<I, K1>{});
  }
  constexpr int KF = G == 64 ? (K5 + 1) / 2 : (G == 32 ? K5 : (G == 16 ? K4 : (G == 8 ? K3 : K2)));
#pragma unroll
  for (int i = 0; i < KF; ++i) {
    double r = v[i];
    if constexpr (COMP) r = r + c[i];
    if (store && i < cnt) out[off + i] = r * f;
  }
}

// f(q) for each of the eight velocity bins q, by lane q of a group of 8 or
// more lanes, by lanes q mod 4 of a group of 4
template <int G, typename F> __device__ __forceinline__ void per_bin(int li, F&& f) {
  if constexpr (G >= 8) {
    if (li < 8) f(li);
  } else {
#pragma unroll
    for (int q = li; q < 8; q += G) f(q);
  }
}

template <int G> __device__ __forceinline__ uint64_t group_mask(int grp) {
  if constexpr (G == 64) return ~0ull;
  else return ((1ull << G) - 1ull) << (grp * G);
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

// (f0, f1, f2): the target's orientations against the edges of element e,
// known to the caller for the first iteration.  OMG: the particle carries a
// turbulent frequency om, which a wall-function reflection rescales.
template <typename T, bool OMG>
__device__ int walk(const StepArgs<T>& a, ERec R, int e, double Sx, double Sy, T& tx, T& ty, T& u, T& v,
                    T& w, T& om, double f0, double f1, double f2) {
#pragma unroll 1
  for (int it = 0; it < 64; ++it) {
    const double Tx = (double)tx, Ty = (double)ty;
    double o0 = f0, o1 = f1, o2 = f2;
    if (it > 0) {
      o0 = orient_edge(R.x[0], R.y[0], R.x[1], R.y[1], Tx, Ty);
      o1 = orient_edge(R.x[1], R.y[1], R.x[2], R.y[2], Tx, Ty);
      o2 = orient_edge(R.x[2], R.y[2], R.x[0], R.y[0], Tx, Ty);
    }
    if (o0 >= 0.0 && o1 >= 0.0 && o2 >= 0.0) return e;
    int ex = -1;
    const int nneg = (o0 < 0.0 ? 1 : 0) + (o1 < 0.0 ? 1 : 0) + (o2 < 0.0 ? 1 : 0);
    if (nneg == 1) {
      // one edge has the target outside: the separation test below either
      // picks it or finds none, and then the most-outside edge is that one
      ex = o0 < 0.0 ? 0 : (o1 < 0.0 ? 1 : 2);
    } else {
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
    // outward unit normal (g_y, -g_x) / |g| of the edge g = b - a, precomputed
    const double nx = a.wnorm[6 * e + 2 * ex], ny = a.wnorm[6 * e + 2 * ex + 1];
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
      if constexpr (OMG) {
        // omega_R = omega_I exp(beta V_I / (y_p <omega>)), <omega> frozen at the
        // edge midpoint; V_I < 0 toward the wall, beta < 0: omega grows
        const double arg = a.om_beta * (double)Vi / (a.om_yp * a.omw[3 * e + ex]);
        om = (T)((double)om * series_exp(arg));
      }
    }
  }
  return -1;
}

// ---------------------------------------------------------------------------
// the fused step.  A group of G consecutive lanes owns one cell (64/G cells
// per wavefront, taken from a list ordered so that the cells of a wavefront
// have similar particle counts):
//   A  read the cell's particles once from HBM into an LDS tile (the first
//      4G to 6G of them; a larger cell re-reads the rest from L2) and sum the
//      velocity and scalar: the means;
//   B  central moments, velocity-bin scalar sums and counts, histogram: the
//      statistics record of the cell;
//   C  IECM with those statistics, velocity, position, tracking, source;
//      stayers are written back in order without atomics, movers take one
//      atomic slot at the top of their new cell's segment.
// ADVANCE = false stops after B.  PERSIST: a grid sized to the machine pulls
// wavefront work items from a counter instead of one item per wavefront.

template <int MOM> struct MomCount { static constexpr int M3 = 0, M4 = 0; };
template <> struct MomCount<4> { static constexpr int M3 = 20, M4 = 35; };

// position of (x, y), x <= y, in the lexicographic list of index pairs of (u, v, w, psi)
__host__ __device__ constexpr int pair_index(int x, int y) { return x * 4 - (x * (x - 1)) / 2 + (y - x); }

// A cell's first TILEN particles; in the advance, the slots of particles
// already read also hold the queue of particles whose end point left the
// element (start x y, end point tx ty, new u v w psi, id).
template <typename T, int TILEN> struct Tile {
  T x[TILEN], y[TILEN], u[TILEN], v[TILEN], w[TILEN], psi[TILEN];
  uint32_t id[TILEN];
  T tx[TILEN], ty[TILEN];
};

// LDS written by some lanes of a wavefront and read by others.  A wavefront's
// LDS instructions execute in order, so a wavefront-scope fence (which keeps
// the compiler from moving memory operations across it and adds no wait on
// outstanding global memory) is enough.
__device__ __forceinline__ void lds_sync_wave() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Per-cell constants of the advance, kept in LDS rather than in registers
// across the particle loop: the element's vertices, the interpolation
// coefficients of its three vertices, the velocity means that define the
// bins and the conditional means IECM relaxes toward.
template <typename T> struct CellConst {
  T coef[3 * NCOEF];
  // edge k (vertex k -> k+1) from its lexicographically smaller endpoint:
  // origin, and direction times the sign that turns the result into the
  // orientation against the element's own edge (orient_edge; the sign is
  // exact, so the product is the same number as orient_edge's)
  double ox[3], oy[3], dx[3], dy[3];
  double mean[3];
  double cm[8];
  double om_mean, sw;  // turbulent frequency: the element's frozen <omega> and S_omega
  double fsd[3];       // 5 x 5 x 5 bins: standard deviations of u, v, w
};

// orient_edge of (px, py) against edge k of a cell, from its CellConst data:
// the sign carried by the direction flips the result exactly (the rounding
// of a fused multiply-add is symmetric), so it is orient_edge's number.
template <typename T>
__device__ __forceinline__ double orient_cc(const CellConst<T>& C, int k, double px, double py) {
  return __builtin_fma(C.dx[k], py - C.oy[k], -(C.dy[k] * (px - C.ox[k])));
}

// SCHED: 0 one work item per wavefront; 1 persistent grid; 2 one item per
// wavefront with the learned conditional means computed inside the step.
// XV, an extension of the model: XV_OMEGA, the particles carry the stochastic
// turbulent frequency of eq. (9) and the record gains its mean, variance and
// the dissipation estimate of eq. (8); XV_BINS5, <phi|V> on 5 x 5 x 5
// velocity bins (the record gains their counts and means).
enum { XV_NONE = 0, XV_OMEGA = 1, XV_BINS5 = 2 };

// Five bins per velocity component: widths 1.2 sigma on [-3 sigma, 3 sigma]
// about the element mean, the outermost bins open; sigma = 0: the middle bin.
__device__ __forceinline__ int fine_component(double u, double mean, double sd) {
  if (!(sd > 0.0)) return 2;
  const double z = (u - mean) / sd;
  const double k = floor((z + 3.0) / 1.2);
  return k < 0.0 ? 0 : (k > 4.0 ? 4 : (int)k);
}

// Threads per block of the step: one wavefront (a block's LDS is freed as
// soon as its cells are done), four with the learned means inside the step,
// where each wavefront computes one output tile of a hidden layer.
template <int SCHED> __host__ __device__ constexpr int step_block() { return SCHED == 2 ? 256 : WAVE; }

// Wavefronts per SIMD the compiler must leave room for: four for the float
// second-moment steps at 64 lanes per cell (their LDS allows four; one
// register more than four wavefronts' 128 made them 10 % slower).
template <typename T, int MOM, int G, bool ADVANCE, int SCHED, int XV>
__host__ __device__ constexpr int step_waves_per_eu() {
  return (sizeof(T) == 4 && MOM == 2 && G == 64 && ADVANCE && SCHED == 0 && XV == XV_NONE) ? 4 : 1;
}

template <typename T, int MOM, int HIST, int G, bool ADVANCE, int SCHED, int XV>
__global__ __launch_bounds__(step_block<SCHED>())
__attribute__((amdgpu_waves_per_eu(step_waves_per_eu<T, MOM, G, ADVANCE, SCHED, XV>())))
void k_step(StepArgs<T> a, StepIndex si) {
  constexpr bool OMG = XV == XV_OMEGA;
  constexpr bool VB5 = XV == XV_BINS5;
  // the fourth-order statistics (the large canyon) reduce across lanes with
  // compensated additions
  constexpr bool CMP = MOM >= 4;
  static_assert(!(XV != XV_NONE && SCHED == 2), "model extensions run with the separate learned-means pass");
  static_assert(!(SCHED == 2 && G < 16), "the learned means inside the step need at most 16 cells per block");
  constexpr bool PERSIST = SCHED == 1;
  constexpr int GPW = WAVE / G;             // cells per wavefront
  // particles per cell staged in LDS: four per lane; deeper where registers
  // already set the blocks per CU and the deeper tile still fits their LDS
  // (it saves re-reads of larger cells in each pass): five for the
  // fourth-order float kernels of 32 or 64 lanes per cell (three blocks),
  // six at 8 lanes per cell (two blocks)
  constexpr int TILEN = ((MOM >= 4 && XV == XV_NONE && sizeof(T) == 4 && G >= 32) ? 5 : (G == 8 ? 6 : 4)) * G;
  constexpr int SWPB = step_block<SCHED>() / WAVE;  // wavefronts per block
  constexpr int CPB = SWPB * GPW;
  __shared__ Tile<T, TILEN> tiles[CPB];
  __shared__ int hist_lds[HIST > 0 ? CPB : 1][HIST > 0 ? HIST : 1];
  __shared__ CellConst<T> ccs[ADVANCE ? CPB : 1];
  __shared__ T otile[OMG ? CPB : 1][OMG ? TILEN : 1];
  __shared__ double fsum[VB5 ? CPB : 1][VB5 ? 125 : 1];
  __shared__ int fcnt[VB5 ? CPB : 1][VB5 ? 125 : 1];
  __shared__ T fcm[VB5 && ADVANCE ? CPB : 1][VB5 && ADVANCE ? 125 : 1];
  constexpr int NRED = OMG ? 11 : 10;       // group sums of pass B (A takes the first 4 or 5)
  __shared__ double red[CPB][NRED];
  __shared__ double bsum_lds[CPB][8];       // per-bin scalar sums, then bin means
  __shared__ int bcnt_lds[CPB][8];          // per-bin counts
  Ctl* ctl = a.ctl;
  // after an error the state is void: later steps do nothing
  // (with the learned means inside the step every wavefront of a block must
  // reach its barriers: the step then runs on, on a state that is void anyway)
  constexpr bool fused_mlp = ADVANCE && SCHED == 2;
  if (ADVANCE && !fused_mlp && ctl->error != 0) return;
  const uint32_t step = ctl->step_base + si.step_off;
  const uint32_t par = si.parity;
  const uint32_t bpar = par ^ (ctl->flip & 1u);
  const int rc = (int)si.rot, rn = rc == 2 ? 0 : rc + 1, rz = rc == 0 ? 2 : rc - 1;
  const int lane = lane_id();
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int grp = lane / G;
  const int li = lane - grp * G;
  const int slot_id = wid * GPW + grp;
  const uint64_t gmask = group_mask<G>(grp);
  if (ADVANCE && blockIdx.x == 0 && threadIdx.x == 0) ctl->next[par ^ 1u] = 0;
  const StateDev<T> src = a.buf[bpar];
  const StateDev<T> dst = a.buf[bpar ^ 1u];
  Tile<T, TILEN>& L = tiles[slot_id];
  T* LO = otile[OMG ? slot_id : 0];

  // persistent grid: a wavefront claims a.pchunk consecutive work items per
  // atomic on the shared counter (one address: its atomics serialise in L2)
  int item = 0;
  if (!PERSIST) {
    // block b runs on XCD b mod 8; each XCD walks its own contiguous range of
    // the order (neighbouring cells share the XCD's L2), the ranges balanced
    // by estimated cost rather than by length
    const int x = (int)(blockIdx.x % 8u), i = (int)(blockIdx.x / 8u);
    item = a.xcd[x] + i * SWPB + wid;
    if (item >= a.xcd[x + 1]) item = a.nitems;
  }
  int chunk_end = 0;
  for (;;) {
    if (PERSIST) {
      if (item + 1 < chunk_end) {
        ++item;
      } else {
        int it = 0;
        if (lane == 0) it = (int)atomicAdd(&ctl->next[par], (uint32_t)a.pchunk);
        item = __builtin_amdgcn_readfirstlane(it);
        chunk_end = item + a.pchunk;
      }
    }
    if (item >= a.nitems && !fused_mlp) break;
    const int idx = item * GPW + grp;
    const int cell_l = idx < a.ncell ? a.order[idx] : -1;
    const int cell = (G == WAVE) ? __builtin_amdgcn_readfirstlane(cell_l) : cell_l;
    const bool has = cell >= 0;
    const int ne = a.ne;
    const int ens = has ? cell / ne : 0;
    const int e = has ? cell - ens * ne : 0;
    int start = 0, capc = 0, ns = 0, nm = 0;
    if (has) {
      start = a.start[cell];
      capc = a.cap[cell];
      // counts are clamped to the segment so that reads stay inside it
      ns = min(a.ns[rc][cell], capc);
      nm = min(a.nm[rc][cell], capc - ns);
      if (ADVANCE && li == 0 && repack_due(ns + nm, nm, capc)) ctl->repack = 1u;
    }
    const int n = ns + nm;
    const double dn = (double)n;
    // The cell's constants for the advance (vertex coefficients, edge
    // geometry, 1/(2A), rate, seed), issued here, ahead of the statistics
    // passes, where groups of 32 lanes or fewer take several cells per
    // wavefront or the 5 x 5 x 5 bins make the passes long: 8 % shorter
    // batched steps, 2 % with the bins, 4-6 % on the canyons at 32 lanes.
    // With the turbulent frequency all but the edge geometry (6 % shorter
    // steps; with it: no gain).  The plain 64-lane steps take 2 % longer
    // with any of them issued early.
    constexpr bool PRE = ADVANCE && (G <= 32 || VB5);
    constexpr bool PRE_SC = PRE || (ADVANCE && OMG);
    constexpr int NPRE = PRE_SC ? (3 * NCOEF + G - 1) / G : 1;
    T pre_coef[NPRE];
    double pre_ax = 0.0, pre_ay = 0.0, pre_bx = 0.0, pre_by = 0.0, pre_ia = 0.0;
    T pre_rate = (T)0;
    uint64_t pre_seed = 0;
    if constexpr (PRE_SC) {
      const int vtx[3] = {a.tri[3 * e], a.tri[3 * e + 1], a.tri[3 * e + 2]};
#pragma unroll
      for (int i = 0; i < NPRE; ++i) {
        const int q = li + i * G;
        if (q < 3 * NCOEF) {
          const int k = q / NCOEF;
          const int vk = k == 0 ? vtx[0] : (k == 1 ? vtx[1] : vtx[2]);
          pre_coef[i] = a.coef[(size_t)vk * NCOEF + (q - k * NCOEF)];
        }
      }
    }
    if constexpr (PRE) {
      if (li < 3) {
        const int k = li, k1 = k == 2 ? 0 : k + 1;
        const ERec& R = a.erec[e];
        pre_ax = R.x[k];
        pre_ay = R.y[k];
        pre_bx = R.x[k1];
        pre_by = R.y[k1];
      }
    }
    // (after the edge geometry: the 5 x 5 x 5 bin steps took 4 % longer
    // with these before it)
    if constexpr (PRE_SC) {
      pre_ia = a.inv2a[e];
      pre_rate = has ? a.rate[cell] : (T)0;
      pre_seed = a.seed[ens];
    }

    // ---- A: load, stage, means ----
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    {
      T tx_[TILEN / G], ty_[TILEN / G], tu_[TILEN / G], tv_[TILEN / G], tw_[TILEN / G], tp_[TILEN / G];
      T to_[OMG ? TILEN / G : 1];
      uint32_t ti_[TILEN / G];
#pragma unroll
      for (int c = 0; c < TILEN / G; ++c) {
        const int j = c * G + li;
        if (j < n) {
          const int s = slot_of(j, start, ns, nm, capc);
          tx_[c] = src.x[s]; ty_[c] = src.y[s]; tu_[c] = src.u[s]; tv_[c] = src.v[s]; tw_[c] = src.w[s];
          tp_[c] = src.psi[s]; ti_[c] = src.id[s];
          if constexpr (OMG) to_[c] = src.om[s];
        }
      }
#pragma unroll
      for (int c = 0; c < TILEN / G; ++c) {
        const int j = c * G + li;
        if (j < n) {
          L.x[j] = tx_[c]; L.y[j] = ty_[c]; L.u[j] = tu_[c]; L.v[j] = tv_[c]; L.w[j] = tw_[c]; L.psi[j] = tp_[c];
          L.id[j] = ti_[c];
          s0 += (double)tu_[c];
          s1 += (double)tv_[c];
          s2 += (double)tw_[c];
          s3 += (double)tp_[c];
          if constexpr (OMG) {
            LO[j] = to_[c];
            s4 += (double)to_[c];
          }
        }
      }
    }
    for (int base = TILEN; __ballot(base < n) != 0; base += G) {
      const int j = base + li;
      if (j < n) {
        const int s = slot_of(j, start, ns, nm, capc);
        s0 += (double)src.u[s];
        s1 += (double)src.v[s];
        s2 += (double)src.w[s];
        s3 += (double)src.psi[s];
        if constexpr (OMG) s4 += (double)src.om[s];
      }
    }
    const double inv_n = n > 0 ? 1.0 / dn : 0.0;
    double* redc = red[slot_id];
    double mean[4];
    double om_mean = 0.0;
    {
      double sa[OMG ? 5 : 4];
      sa[0] = s0; sa[1] = s1; sa[2] = s2; sa[3] = s3;
      if constexpr (OMG) sa[4] = s4;
      lds_sync_wave();  // the previous item's sums are read before these are written
      group_sum_many<G, OMG ? 5 : 4, CMP>(sa, redc);
      lds_sync_wave();
#pragma unroll
      for (int q = 0; q < 4; ++q) mean[q] = redc[q] * inv_n;
      if constexpr (OMG) om_mean = redc[4] * inv_n;
    }

    auto load4 = [&](int j, double* val) {
      if (j < TILEN) {
        val[0] = (double)L.u[j]; val[1] = (double)L.v[j]; val[2] = (double)L.w[j]; val[3] = (double)L.psi[j];
      } else {
        const int s = slot_of(j, start, ns, nm, capc);
        val[0] = (double)src.u[s]; val[1] = (double)src.v[s]; val[2] = (double)src.w[s]; val[3] = (double)src.psi[s];
      }
    };

    // ---- B: second moments, bins, histogram ----
    double acc[10];  // second moments
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.0;
    double accw = 0.0;  // turbulent frequency: sum of squared fluctuations
    // bin counts and scalar sums by LDS atomics (the order of the FP64 sums
    // is free, their rounding that of any FP64 sum of the bin's values)
    double* bsum = bsum_lds[slot_id];
    int* bcnt = bcnt_lds[slot_id];
    per_bin<G>(li, [&](int q) {
      bsum[q] = 0.0;
      bcnt[q] = 0;
    });
    if (HIST > 0) {
      for (int h = li; h < HIST; h += G) hist_lds[slot_id][h] = 0;
    }
    lds_sync_wave();
    for (int base = 0; __ballot(base < n) != 0; base += G) {
      const int j = base + li;
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
          for (int y = x; y < 4; ++y) acc[pair_index(x, y)] = __builtin_fma(d[x], d[y], acc[pair_index(x, y)]);
        bin = (val[0] > mean[0] ? 1 : 0) + (val[1] > mean[1] ? 2 : 0) + (val[2] > mean[2] ? 4 : 0);
        atomicAdd(&bcnt[bin], 1);
        atomicAdd(&bsum[bin], val[3]);
        if constexpr (OMG) {
          const double dw = (double)(j < TILEN ? LO[j] : src.om[slot_of(j, start, ns, nm, capc)]) - om_mean;
          accw += dw * dw;
        }
        if (HIST > 0) {
          const double hpos = floor(val[3] * (double)HIST);
          const int hb = hpos < 0.0 ? 0 : (hpos >= (double)HIST ? HIST - 1 : (int)hpos);
          atomicAdd(&hist_lds[slot_id][hb], 1);
        }
      }
    }
    double om_var = 0.0;
    {
      double sb[NRED];
#pragma unroll
      for (int q = 0; q < 10; ++q) sb[q] = acc[q];
      if constexpr (OMG) sb[10] = accw;
      lds_sync_wave();  // the means above are read before the sums below are written
      group_sum_many<G, NRED, CMP>(sb, redc);
      lds_sync_wave();
#pragma unroll
      for (int q = 0; q < 10; ++q) acc[q] = redc[q];
      if constexpr (OMG) om_var = redc[10] * inv_n;
    }
    // bin means, one lane of the group per bin
    per_bin<G>(li, [&](int q) {
      const int c = bcnt[q];
      bsum[q] = c > 0 ? bsum[q] / (double)c : mean[3];
    });
    lds_sync_wave();
    int bcount[8];
    double bm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      bcount[q] = bcnt[q];
      bm[q] = bsum[q];
    }
    double cm[8];
    if constexpr (fused_mlp) {
      // learned conditional means: the block's cells form one 16-column tile
      // of the network (columns beyond the block's cells are padding)
      __shared__ uint16_t mxs[16][mlp::NFEAT];
      __shared__ float mys[16][mlp::NOUT];
      __shared__ int minbox[16];
      const double z = n > 0 ? 1.0 : 0.0;
      double binn[8], binm[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        binn[q] = (double)bcount[q];
        binm[q] = bm[q] * z;
      }
      if (li == 0) {
        double meanr[4], m2r[10];
#pragma unroll
        for (int q = 0; q < 4; ++q) meanr[q] = mean[q] * z;
#pragma unroll
        for (int q = 0; q < 10; ++q) m2r[q] = acc[q] * inv_n;
        float f[mlp::NFEAT];
        mlp::features_from(dn, meanr, m2r, binn, binm, f);
        int ok = has ? 1 : 0;
#pragma unroll
        for (int k = 0; k < mlp::NFEAT; ++k) {
          ok &= (f[k] >= a.mlp_norm[2 * mlp::NFEAT + k] && f[k] <= a.mlp_norm[3 * mlp::NFEAT + k]) ? 1 : 0;
          mxs[slot_id][k] = mlp::f2bf((f[k] - a.mlp_norm[k]) * a.mlp_norm[mlp::NFEAT + k]);
        }
        minbox[slot_id] = ok;
      }
      __syncthreads();
      // the 16-column tile: each wavefront computes output tile wid of a
      // hidden layer (the B operand of k-step wid of the next layer) and
      // leaves it in LDS; wavefront 0 computes the output layer
      __shared__ mlp::bf16x4 hb[2][4][WAVE];
      {
        const int r = lane & 15;
        mlp::f32x4 acc = mlp::zero4();
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const mlp::bf16x4 xb = r < CPB ? *(const mlp::bf16x4*)&mxs[r][16 * ks + 4 * (lane >> 4)] : mlp::bf16x4{0, 0, 0, 0};
          acc = mlp::mfma16(mlp::load_w(a.mlp_w + mlp::OFF_W1, mlp::NFEAT, wid, ks, lane), xb, acc);
        }
        hb[0][wid][lane] = mlp::bias_relu_bf16(acc, a.mlp_w + mlp::OFF_B1, wid, lane);
      }
      __syncthreads();
      {
        mlp::f32x4 acc = mlp::zero4();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          acc = mlp::mfma16(mlp::load_w(a.mlp_w + mlp::OFF_W2, mlp::NHID, wid, ks, lane), hb[0][ks][lane], acc);
        hb[1][wid][lane] = mlp::bias_relu_bf16(acc, a.mlp_w + mlp::OFF_B2, wid, lane);
      }
      __syncthreads();
      {
        mlp::f32x4 acc = mlp::zero4();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          acc = mlp::mfma16(mlp::load_w(a.mlp_w + mlp::OFF_W3, mlp::NHID, wid, ks, lane), hb[1][ks][lane], acc);
        // hb[0] was last read before the previous barrier
        hb[0][wid][lane] = mlp::bias_relu_bf16(acc, a.mlp_w + mlp::OFF_B3, wid, lane);
      }
      __syncthreads();
      if (wid == 0) {
        const int r = lane & 15;
        mlp::f32x4 y = mlp::zero4();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) y = mlp::mfma16(mlp::load_w4(a.mlp_w + mlp::OFF_W4, ks, lane), hb[0][ks][lane], y);
        if (lane < 32 && r < CPB) {
#pragma unroll
          for (int i = 0; i < 4; ++i) mys[r][4 * (lane >> 4) + i] = y[i] + mlp::bf2f(a.mlp_w[mlp::OFF_B4 + 4 * (lane >> 4) + i]);
        }
      }
      __syncthreads();
      float yv[mlp::NOUT];
#pragma unroll
      for (int b = 0; b < mlp::NOUT; ++b) yv[b] = mys[slot_id][b];
      const bool took = mlp::learned_estimate(dn, mean[3] * z, acc[9] * inv_n, binn, binm, yv, minbox[slot_id] != 0, cm);
      if (has && li == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a.mlp_cm[(size_t)cell * 8 + q] = cm[q];
        if (took && a.mlp_served) atomicAdd(a.mlp_served, 1u);
      }
    } else if (ADVANCE && a.cmean != nullptr && has) {
#pragma unroll
      for (int q = 0; q < 8; ++q) cm[q] = a.cmean[(size_t)cell * 8 + q];
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) cm[q] = bm[q];
    }
    double* rec = a.stats + (size_t)(has ? cell : 0) * a.nstat;
    // the record: count and means by the group's first lane, second moments
    // and bins by one lane each from the group sums in LDS
    if (has) {
      const double z = n > 0 ? 1.0 : 0.0;
      for (int q = li; q < 10; q += G) rec[ST_M2 + q] = redc[q] * inv_n;
      per_bin<G>(li, [&](int q) {
        rec[ST_BINN + q] = (double)bcnt[q];
        rec[ST_BINM + q] = bsum[q] * z;
      });
    }
    if (has && li == 0) {
      const double z = n > 0 ? 1.0 : 0.0;
      rec[ST_N] = dn;
#pragma unroll
      for (int q = 0; q < 4; ++q) rec[ST_MEAN + q] = mean[q] * z;
      if constexpr (OMG) {
        // after the moments and the histogram: <omega>, its variance, and
        // eps = <omega>(k + nu C_T^2 <omega>) with k from the estimated stresses
        constexpr int OFF = (MOM >= 4 ? NSTAT4 : NSTAT2) + HIST;
        const double kh = 0.5 * ((acc[0] * inv_n + acc[4] * inv_n) + acc[7] * inv_n);
        rec[OFF] = om_mean;
        rec[OFF + 1] = om_var;
        rec[OFF + 2] = om_mean * (kh + a.om_nuct2 * om_mean);
      }
    }
    if constexpr (MOM >= 4) {
      // third- and fourth-order central moments: the 20 + 35 index combinations
      // in lexicographic order, each product built from the ten pairwise
      // products d_x d_y and accumulated with a fused multiply-add; two passes
      // over the particles bound the number of live accumulators
      constexpr int NM = 55, SPLIT = 28;
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        const int lo = part == 0 ? 0 : SPLIT, hi = part == 0 ? SPLIT : NM;
        double acc3[NM - SPLIT > SPLIT ? NM - SPLIT : SPLIT];
#pragma unroll
        for (int q = 0; q < (NM - SPLIT > SPLIT ? NM - SPLIT : SPLIT); ++q) acc3[q] = 0.0;
        for (int base = 0; __ballot(base < n) != 0; base += G) {
          const int j = base + li;
          if (j < n) {
            double val[4], d[4], pr[10];
            load4(j, val);
#pragma unroll
            for (int q = 0; q < 4; ++q) d[q] = val[q] - mean[q];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = x; y < 4; ++y) pr[pair_index(x, y)] = d[x] * d[y];
            int k = 0;
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = x; y < 4; ++y)
#pragma unroll
                for (int z = y; z < 4; ++z) {
                  if (k >= lo && k < hi) acc3[k - lo] = __builtin_fma(pr[pair_index(x, y)], d[z], acc3[k - lo]);
                  ++k;
                }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = x; y < 4; ++y)
#pragma unroll
                for (int z = y; z < 4; ++z)
#pragma unroll
                  for (int g = z; g < 4; ++g) {
                    if (k >= lo && k < hi)
                      acc3[k - lo] = __builtin_fma(pr[pair_index(x, y)], pr[pair_index(z, g)], acc3[k - lo]);
                    ++k;
                  }
          }
        }
        // M3 (20 entries) and M4 (35) are contiguous in the record; the
        // lanes that end with a sum store it
        if (part == 0) {
          double t[SPLIT];
#pragma unroll
          for (int q = 0; q < SPLIT; ++q) t[q] = acc3[q];
          group_sum_many<G, SPLIT, CMP>(t, rec + ST_M3, inv_n, has);
        } else {
          double t[NM - SPLIT];
#pragma unroll
          for (int q = 0; q < NM - SPLIT; ++q) t[q] = acc3[q];
          group_sum_many<G, NM - SPLIT, CMP>(t, rec + ST_M3 + SPLIT, inv_n, has);
        }
      }
    }
    if (HIST > 0) {
      const int off = MOM >= 4 ? NSTAT4 : NSTAT2;
      lds_sync_wave();
      for (int h = li; h < HIST; h += G)
        if (has) rec[off + h] = (double)hist_lds[slot_id][h];
    }
    if constexpr (VB5) {
      // <phi|V> on 5 x 5 x 5 bins: one more pass over the particles, bins from
      // this record's means and second moments, per-bin counts and FP64
      // scalar sums by LDS atomics (the order of the sums is not fixed; their
      // rounding is that of any FP64 sum, relative to each bin's own values)
      constexpr int FOFF = (MOM >= 4 ? NSTAT4 : NSTAT2) + HIST;
      const double sdu = sqrt(acc[0] * inv_n), sdv = sqrt(acc[4] * inv_n), sdw = sqrt(acc[7] * inv_n);
      for (int b = li; b < 125; b += G) {
        fsum[slot_id][b] = 0.0;
        fcnt[slot_id][b] = 0;
      }
      lds_sync_wave();
      for (int base = 0; __ballot(base < n) != 0; base += G) {
        const int j = base + li;
        if (j < n) {
          double val[4];
          load4(j, val);
          const int b = fine_component(val[0], mean[0], sdu) + 5 * fine_component(val[1], mean[1], sdv) +
                        25 * fine_component(val[2], mean[2], sdw);
          atomicAdd(&fcnt[slot_id][b], 1);
          atomicAdd(&fsum[slot_id][b], val[3]);
        }
      }
      lds_sync_wave();
      for (int b = li; b < 125; b += G) {
        const int cn = fcnt[slot_id][b];
        const double fm = cn > 0 ? fsum[slot_id][b] / (double)cn : mean[3];
        if (has) {
          rec[FOFF + b] = (double)cn;
          rec[FOFF + 125 + b] = fm;
        }
        if constexpr (ADVANCE) fcm[slot_id][b] = (T)fm;
      }
      if constexpr (ADVANCE) {
        if (li == 0) {
          ccs[slot_id].fsd[0] = sdu;
          ccs[slot_id].fsd[1] = sdv;
          ccs[slot_id].fsd[2] = sdw;
        }
      }
    }

    if (ADVANCE) {
      // ---- C: advance ----
      CellConst<T>& CC = ccs[ADVANCE ? slot_id : 0];
      {
        if constexpr (PRE_SC) {
#pragma unroll
          for (int i = 0; i < NPRE; ++i) {
            const int q = li + i * G;
            if (q < 3 * NCOEF) CC.coef[q] = pre_coef[i];
          }
        } else {
          const int vtx[3] = {a.tri[3 * e], a.tri[3 * e + 1], a.tri[3 * e + 2]};
          for (int q = li; q < 3 * NCOEF; q += G) {
            const int k = q / NCOEF;
            const int vk = k == 0 ? vtx[0] : (k == 1 ? vtx[1] : vtx[2]);
            CC.coef[q] = a.coef[(size_t)vk * NCOEF + (q - k * NCOEF)];
          }
        }
        // edge k by lane k
        if (li < 3) {
          const int k = li, k1 = k == 2 ? 0 : k + 1;
          const ERec& R = a.erec[e];
          const double ax = PRE ? pre_ax : R.x[k], ay = PRE ? pre_ay : R.y[k];
          const double bx = PRE ? pre_bx : R.x[k1], by = PRE ? pre_by : R.y[k1];
          const bool a_first = (ax < bx) || (ax == bx && ay < by);
          CC.ox[k] = a_first ? ax : bx;
          CC.oy[k] = a_first ? ay : by;
          CC.dx[k] = a_first ? bx - ax : -(ax - bx);
          CC.dy[k] = a_first ? by - ay : -(ay - by);
        }
        // conditional mean of each bin by one lane
        if constexpr (fused_mlp) {
          if (li == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) CC.cm[q] = cm[q];
          }
        } else {
          per_bin<G>(li, [&](int q) { CC.cm[q] = (a.cmean != nullptr && has) ? a.cmean[(size_t)cell * 8 + q] : bsum[q]; });
        }
        if (li == 0) {
#pragma unroll
          for (int q = 0; q < 3; ++q) CC.mean[q] = mean[q];
          if constexpr (OMG) {
            CC.om_mean = a.om0[e];
            CC.sw = a.somega[e];
          }
        }
        lds_sync_wave();
      }
      const double ia = PRE_SC ? pre_ia : a.inv2a[e];
      const T rate = PRE_SC ? pre_rate : (has ? a.rate[cell] : (T)0);
      const uint64_t seed = PRE_SC ? pre_seed : a.seed[ens];
      const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
      const bool do_mix = a.mix && (a.flags & FLAG_MIX);
      int err = 0;
      int stay_count = 0;

      // Writes a particle that ended in element e2 of ensemble qens: its own
      // cell's bottom run at index k, or the top run of the new cell.
      // Writes a particle that moved to cell t into slot k of that cell's
      // arrivals (counted from the top of its segment), or, when the segment
      // is full, into the overflow area.
      auto put_mover = [&](int t, int k, T xn, T yn, T un, T vn, T wn, T psi, uint32_t id, T omv) {
        const int capt = a.cap[t];
        const int limit = capt - (a.ns[rc][t] + a.nm[rc][t]);
        if (k < limit) {
          const int s = a.start[t] + capt - 1 - k;
          dst.x[s] = xn; dst.y[s] = yn; dst.u[s] = un; dst.v[s] = vn; dst.w[s] = wn; dst.psi[s] = psi;
          dst.id[s] = id;
          if constexpr (OMG) dst.om[s] = omv;
        } else {
          err |= ERR_CAPACITY;
          const uint32_t kk = atomicAdd(&ctl->ovf, 1u);
          if (kk < a.ovf_cap) {
            a.ovf.x[kk] = xn; a.ovf.y[kk] = yn; a.ovf.u[kk] = un; a.ovf.v[kk] = vn; a.ovf.w[kk] = wn;
            a.ovf.psi[kk] = psi; a.ovf.id[kk] = id;
            if constexpr (OMG) a.ovf.om[kk] = omv;
            a.ovf_cell[kk] = t;
          } else {
            err |= ERR_OVERFLOW_FULL;
          }
        }
      };
      // the source, section 3: a particle ending within r0 of x0 takes scalar 1
      auto finish = [&](int qens, T xn, T yn, T& psi) {
        const double qsr = a.src[3 * qens + 2];
        if ((a.flags & FLAG_SRC) && qsr > 0.0) {
          const double ddx = (double)xn - a.src[3 * qens], ddy = (double)yn - a.src[3 * qens + 1];
          if (ddx * ddx + ddy * ddy <= qsr * qsr) psi = (T)1;
        }
      };
      // Particles whose end point leaves the element wait in a queue held in
      // slots of the cell's LDS tile that have already been read (entry q of
      // the queue is never beyond the particle that fills it) and are walked
      // together after the batches, or when the queue fills, so that the walk
      // runs once for all the cell's crossing particles instead of once for
      // the few crossing lanes of every batch.  Those that come back to the
      // element join the stayers after the ones of the batches before.
      int qn = 0;  // queued crossing particles (group-uniform)
      // walks the queue of the groups with go set
      auto walk_queue = [&](bool go) {
        lds_sync_wave();
        const int nq = go ? qn : 0;
        for (int qb = 0; __ballot(qb < nq) != 0; qb += G) {
          const int k = qb + li;
          bool st = false, mv = false;
          int t = 0;
          T tx = 0, ty = 0, un = 0, vn = 0, wn = 0, psi = 0, omv = 0;
          uint32_t id = 0;
          if (k < nq) {
            const double Sx = (double)L.x[k], Sy = (double)L.y[k];
            tx = L.tx[k]; ty = L.ty[k]; un = L.u[k]; vn = L.v[k]; wn = L.w[k]; psi = L.psi[k]; id = L.id[k];
            if constexpr (OMG) omv = LO[k];
            const double Tx = (double)tx, Ty = (double)ty;
            const int e2 = walk<T, OMG>(a, a.erec[e], e, Sx, Sy, tx, ty, un, vn, wn, omv, orient_cc(CC, 0, Tx, Ty),
                                        orient_cc(CC, 1, Tx, Ty), orient_cc(CC, 2, Tx, Ty));
            if (e2 < 0) {
              err |= ERR_LOST;
            } else {
              finish(ens, tx, ty, psi);
              if (!(isfinite(un) && isfinite(vn) && isfinite(wn) && isfinite(psi) && isfinite(tx) && isfinite(ty)) ||
                  (OMG && !isfinite(omv)))
                err |= ERR_NAN;
              if (e2 == e) {
                st = true;
              } else {
                mv = true;
                t = ens * ne + e2;
              }
            }
          }
          // arrival slots: the movers of the wavefront are grouped by target
          // cell (movers of a cell tend to cross the same edge, and
          // same-address atomics of one instruction serialise); the lowest
          // lane of each group takes the group's slots with one atomic, all
          // groups' atomics in one instruction
          uint64_t pend = __ballot(mv);
          int leader = 0, rank = 0, cnt = 0;
          while (pend) {
            const int ld = __builtin_ctzll(pend);
            const int tl = __builtin_amdgcn_readlane(t, ld);
            const uint64_t same = __ballot(mv && t == tl);
            if (mv && t == tl) {
              leader = ld;
              rank = (int)__popcll(same & lanemask_lt());
            }
            if (lane == ld) cnt = (int)__popcll(same);
            pend &= ~same;
          }
          int kb = 0;
          if (mv && lane == leader) kb = atomicAdd(&a.nm[rn][t], cnt);
          kb = __shfl(kb, leader, WAVE);
          if (mv) put_mover(t, kb + rank, tx, ty, un, vn, wn, psi, id, omv);
          const uint64_t smask = __ballot(st) & gmask;
          if (st) {
            const int s = start + stay_count + (int)__popcll(smask & lanemask_lt());
            dst.x[s] = tx; dst.y[s] = ty; dst.u[s] = un; dst.v[s] = vn; dst.w[s] = wn; dst.psi[s] = psi;
            dst.id[s] = id;
            if constexpr (OMG) dst.om[s] = omv;
          }
          stay_count += (int)__popcll(smask);
        }
        if (go) qn = 0;
        lds_sync_wave();
      };
      // one loop with one walk site: a pass either walks the queues that are
      // due (full enough to overflow the tile in the next batch, or final) or
      // advances the next batch
      for (int base = 0;;) {
        const bool more = base < n;
        const bool due = qn > 0 && (qn > TILEN - G || !more);
        if (__ballot(due) != 0) {
          walk_queue(due);
          continue;
        }
        if (__ballot(more) == 0) break;
        const int j = base + li;
        base += G;
        const bool act = j < n;
        bool cross = false;
        T x = 0, y = 0, xn = 0, yn = 0, un = 0, vn = 0, wn = 0, psi = 0, omn = 0;
        uint32_t id = 0;
        if (act) {
          T u, v, w, om = 0;
          if (j < TILEN) {
            x = L.x[j]; y = L.y[j]; u = L.u[j]; v = L.v[j]; w = L.w[j]; psi = L.psi[j]; id = L.id[j];
            if constexpr (OMG) om = LO[j];
          } else {
            const int s = slot_of(j, start, ns, nm, capc);
            x = src.x[s]; y = src.y[s]; u = src.u[s]; v = src.v[s]; w = src.w[s]; psi = src.psi[s]; id = src.id[s];
            if constexpr (OMG) om = src.om[s];
          }
          uint32_t rw[8];
          uint32_t kk0 = k0, kk1 = k1, st = step, en = (uint32_t)ens;
          if constexpr (G == WAVE) {
            // wavefront-uniform key and counter words: rebuilt from four
            // scalars each batch (scalar adds) rather than twenty round
            // keys held across the loop
            kk0 = __builtin_amdgcn_readfirstlane(kk0);
            kk1 = __builtin_amdgcn_readfirstlane(kk1);
            st = __builtin_amdgcn_readfirstlane(st);
            en = __builtin_amdgcn_readfirstlane(en);
            asm volatile("" : "+s"(kk0), "+s"(kk1), "+s"(st), "+s"(en));
          }
          philox_words<2>(id, st, en, kk0, kk1, rw);
          T xi0, xi1, xi2, xi3, xi4, xi5;
          box_muller<T>(rw[0], rw[1], &xi0, &xi1);
          box_muller<T>(rw[2], rw[3], &xi2, &xi3);
          box_muller<T>(rw[4], rw[5], &xi4, &xi5);
          if constexpr (!OMG) (void)xi5;
          const double X = (double)x, Y = (double)y;
          const T l0 = (T)(orient_cc(CC, 1, X, Y) * ia);
          const T l1 = (T)(orient_cc(CC, 2, X, Y) * ia);
          const T l2 = (T)(orient_cc(CC, 0, X, Y) * ia);
          T f[NCOEF];
#pragma unroll
          for (int q = 0; q < NCOEF; ++q) f[q] = fma_t(l2, CC.coef[2 * NCOEF + q], fma_t(l1, CC.coef[NCOEF + q], l0 * CC.coef[q]));
          if (do_mix) {
            T m;
            if constexpr (VB5) {
              const int b = fine_component((double)u, CC.mean[0], CC.fsd[0]) +
                            5 * fine_component((double)v, CC.mean[1], CC.fsd[1]) +
                            25 * fine_component((double)w, CC.mean[2], CC.fsd[2]);
              m = fcm[slot_id][b];
            } else {
              const int bin = ((double)u > CC.mean[0] ? 1 : 0) + ((double)v > CC.mean[1] ? 2 : 0) +
                              ((double)w > CC.mean[2] ? 4 : 0);
              m = (T)CC.cm[bin];
            }
            psi = fma_t(-rate, psi - m, psi);
          }
          const T dW1 = a.sdt * xi0, dW2 = a.sdt * xi1;
          const T dWp1 = a.sdt * xi2, dWp2 = a.sdt * xi3, dWp3 = a.sdt * xi4;
          const T uf = u - f[C_U], vf = v - f[C_V];
          const T sq = sqrt_t(f[C_C0EPS]);
          const T au = fma_t(f[C_G12], vf, fma_t(f[C_G11], uf, fma_t(a.nu2, f[C_LAPU], -f[C_DPDX])));
          const T av = fma_t(f[C_G22], vf, fma_t(f[C_G21], uf, fma_t(a.nu2, f[C_LAPV], -f[C_DPDY])));
          const T gu = fma_t(f[C_DUDY], dW2, f[C_DUDX] * dW1), gv = fma_t(f[C_DVDY], dW2, f[C_DVDX] * dW1);
          un = fma_t(sq, dWp1, fma_t(a.s2nu, gu, fma_t(au, a.dt, u)));
          vn = fma_t(sq, dWp2, fma_t(a.s2nu, gv, fma_t(av, a.dt, v)));
          wn = fma_t(sq, dWp3, fma_t(f[C_G33] * w, a.dt, w));
          if (!(a.flags & FLAG_VEL)) { un = u; vn = v; wn = w; }
          if constexpr (OMG) {
            // turbulent frequency, eq. (9), with the sixth normal; reflected
            // at zero.  <omega>: the element's frozen value, the one the
            // velocity model takes (the particles' own is estimated for the
            // record, not fed back)
            omn = om;
            if (a.flags & FLAG_VEL) {
              const T mw = (T)CC.om_mean, sw = (T)CC.sw;
              const T drift = fma_t(sw * mw, om, (a.om_c3 * mw) * (om - mw));
              const T diff = sqrt_t((a.om_c34 * (mw * mw)) * om);
              omn = fma_t(diff, a.sdt * xi5, fma_t(-drift, a.dt, om));
              omn = fabs(omn);
            }
          }
          if (a.flags & FLAG_POS) {
            xn = fma_t(a.s2nu, dW1, fma_t(u, a.dt, x));
            yn = fma_t(a.s2nu, dW2, fma_t(v, a.dt, y));
            // the walk's first test: is the end point still in the element?
            const double Tx = (double)xn, Ty = (double)yn;
            cross = !(orient_cc(CC, 0, Tx, Ty) >= 0.0 && orient_cc(CC, 1, Tx, Ty) >= 0.0 &&
                      orient_cc(CC, 2, Tx, Ty) >= 0.0);
          } else {
            xn = x; yn = y;
          }
          if (!cross) {
            finish(ens, xn, yn, psi);
            if (!(isfinite(un) && isfinite(vn) && isfinite(wn) && isfinite(psi) && isfinite(xn) && isfinite(yn)) ||
                (OMG && !isfinite(omn)))
              err |= ERR_NAN;
          }
        }
        // stayers: own segment, bottom run, in lane order, no atomics
        const bool stay = act && !cross;
        const uint64_t smask = __ballot(stay) & gmask;
        if (stay) {
          const int s = start + stay_count + (int)__popcll(smask & lanemask_lt());
          dst.x[s] = xn; dst.y[s] = yn; dst.u[s] = un; dst.v[s] = vn; dst.w[s] = wn; dst.psi[s] = psi;
          dst.id[s] = id;
          if constexpr (OMG) dst.om[s] = omn;
        }
        stay_count += (int)__popcll(smask);
        // crossing particles: into the queue
        const uint64_t xmask = __ballot(cross) & gmask;
        if (cross) {
          const int q = qn + (int)__popcll(xmask & lanemask_lt());
          L.x[q] = x; L.y[q] = y; L.tx[q] = xn; L.ty[q] = yn; L.u[q] = un; L.v[q] = vn; L.w[q] = wn; L.psi[q] = psi;
          L.id[q] = id;
          if constexpr (OMG) LO[q] = omn;
        }
        qn += (int)__popcll(xmask);
      }
      if (has && li == 0) {
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
    if (!PERSIST) break;
  }
}

// Adds the steps of one call to the Philox step base (after the call's steps).
__global__ void k_advance_base(Ctl* ctl, uint32_t nsteps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step_base = ctl->step_base + nsteps;
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

// Outward unit normal of every element edge: g = v_k+1 - v_k, n = (g_y, -g_x) / |g|.
__global__ void k_wnorm(const double* vtx, const int32_t* tri, double* wn, int ne) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * ne) return;
  const int e = i / 3, k = i - 3 * e, k1 = k == 2 ? 0 : k + 1;
  const int va = tri[3 * e + k], vb = tri[3 * e + k1];
  const double gx = vtx[2 * vb] - vtx[2 * va], gy = vtx[2 * vb + 1] - vtx[2 * va + 1];
  const double len = sqrt(gx * gx + gy * gy);
  wn[2 * i] = gy / len;
  wn[2 * i + 1] = -gx / len;
}

// Initial particles: uniform in the element, velocity = local mean plus the
// Cholesky factor of the local Reynolds stress times normals, scalar by rule,
// turbulent frequency (if carried) the element's frozen <omega> (om0).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_seed(const ERec* erec, const int32_t* tri, const double* inv2a,
                                                const double* fields, StateDev<T> st, const int32_t* start,
                                                const int32_t* count, const int32_t* idoff,
                                                const uint64_t* seeds, int ne, int ncell, int psi_init,
                                                const double* om0) {
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
    if (st.om) st.om[s] = (T)om0[e];
  }
}

// Turbulent frequency fields per element: the frozen <omega> at the centroid
// (eq. 8 solved for its positive root) and S_omega = C_w2 - C_w1 P / eps
// (eq. 10) with P = -<u_i u_j> d<U_i>/dx_j from the centroid values; per
// wall-function edge the frozen <omega> at its midpoint (0 on other edges).
__device__ __forceinline__ double frozen_omega(double k, double eps, double nu, double CT) {
  return 2.0 * eps / (k + sqrt(k * k + 4.0 * nu * CT * CT * eps));
}

__global__ void k_omega_fields(const int32_t* tri, const int32_t* ekind, const double* fields, double* om0,
                               double* somega, double* omw, int ne, double nu, double CT, double Cw1,
                               double Cw2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double* f0 = fields + (size_t)tri[3 * e] * NFIELD;
  const double* f1 = fields + (size_t)tri[3 * e + 1] * NFIELD;
  const double* f2 = fields + (size_t)tri[3 * e + 2] * NFIELD;
  double c[NFIELD];
  for (int j = 0; j < NFIELD; ++j) c[j] = ((f0[j] + f1[j]) + f2[j]) / 3.0;
  const double k = 0.5 * ((c[F_R11] + c[F_R22]) + c[F_R33]);
  const double eps = c[F_EPS];
  const double prod = -((c[F_R11] * c[F_DUDX] + c[F_R12] * c[F_DUDY]) + (c[F_R12] * c[F_DVDX] + c[F_R22] * c[F_DVDY]));
  om0[e] = frozen_omega(k, eps, nu, CT);
  somega[e] = Cw2 - Cw1 * (prod / eps);
  for (int q = 0; q < 3; ++q) {
    double w = 0.0;
    if (ekind[3 * e + q] == EDGE_WALLFN) {
      const double* fa = fields + (size_t)tri[3 * e + q] * NFIELD;
      const double* fb = fields + (size_t)tri[3 * e + (q == 2 ? 0 : q + 1)] * NFIELD;
      const double kp = 0.5 * (((fa[F_R11] + fb[F_R11]) / 2.0 + (fa[F_R22] + fb[F_R22]) / 2.0) +
                               (fa[F_R33] + fb[F_R33]) / 2.0);
      w = frozen_omega(kp, (fa[F_EPS] + fb[F_EPS]) / 2.0, nu, CT);
    }
    omw[3 * e + q] = w;
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
                                                  StepIndex si, int ens, int ne, int64_t n, double* out,
                                                  int32_t* elem, double* om_out) {
  const int lane = lane_id();
  const int e = blockIdx.x * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
  if (e >= ne) return;
  const StateDev<T> st = (si.parity ^ (ctl->flip & 1u)) ? b1 : b0;
  const int cell = ens * ne + e;
  const int capc = cap[cell], s0 = start[cell];
  const int ns = min(cs.ns[si.rot][cell], capc);
  const int nm = min(cs.nm[si.rot][cell], capc - ns);
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
    if (om_out) om_out[id] = (double)st.om[s];
  }
}

// ---------------------------------------------------------------------------
// run metrics from the cell counters

// One block over the cells of the current counter set: out[0] particles,
// out[1] arrivals written by the last step (particles now in another element
// than before it; 0 right after a repack, which folds them in), out[2] and
// out[3] the smallest and largest count of a cell, out[4] cells filled beyond
// three quarters of their segment.
constexpr int METRIC_THREADS = 1024;
__global__ __launch_bounds__(METRIC_THREADS) void k_metrics(const int32_t* ns, const int32_t* nm, const int32_t* cap,
                                                            int ncell, int64_t* out) {
  __shared__ long long red[5][METRIC_THREADS / WAVE];
  long long tot = 0, arr = 0, mn = 0x7fffffffffffll, mx = 0, full = 0;
  for (int c = threadIdx.x; c < ncell; c += METRIC_THREADS) {
    const long long k = (long long)ns[c] + nm[c];
    tot += k;
    arr += nm[c];
    mn = k < mn ? k : mn;
    mx = k > mx ? k : mx;
    full += (4 * k > 3 * (long long)cap[c]) ? 1 : 0;
  }
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    tot += __shfl_xor(tot, off, WAVE);
    arr += __shfl_xor(arr, off, WAVE);
    const long long omn = __shfl_xor(mn, off, WAVE), omx = __shfl_xor(mx, off, WAVE);
    mn = omn < mn ? omn : mn;
    mx = omx > mx ? omx : mx;
    full += __shfl_xor(full, off, WAVE);
  }
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    red[0][w] = tot; red[1][w] = arr; red[2][w] = mn; red[3][w] = mx; red[4][w] = full;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < METRIC_THREADS / WAVE; ++i) {
      red[0][0] += red[0][i];
      red[1][0] += red[1][i];
      red[2][0] = red[2][i] < red[2][0] ? red[2][i] : red[2][0];
      red[3][0] = red[3][i] > red[3][0] ? red[3][i] : red[3][0];
      red[4][0] += red[4][i];
    }
    out[0] = red[0][0];
    out[1] = red[1][0];
    out[2] = ncell > 0 ? red[2][0] : 0;
    out[3] = red[3][0];
    out[4] = red[4][0];
  }
}

// ---------------------------------------------------------------------------
// replacing the state of one ensemble (checkpoint restore)

// Particles of ensemble ens per element (cnt: the cells' scratch counters,
// zero on entry); flag bit 1: an element index out of range.
__global__ void k_set_count(const int32_t* elem, int64_t n, int ne, int ens, int32_t* cnt, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e = elem[i];
  if (e < 0 || e >= ne) {
    atomicOr(flag, 1);
    return;
  }
  atomicAdd(&cnt[(size_t)ens * ne + e], 1);
}

// flag bit 2: a cell whose segment cannot hold its particles.
__global__ void k_set_check(const int32_t* cnt, const int32_t* cap, int ne, int ens, int32_t* flag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int c = ens * ne + e;
  if (cnt[c] > cap[c]) atomicOr(flag, 2);
}

// Installs the counts as the cells' current stayers (no arrivals) and clears
// the scratch counters, which then number the particles of each cell.
__global__ void k_set_counts(int32_t* cnt, int32_t* ns, int32_t* nm, int ne, int ens) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int c = ens * ne + e;
  ns[c] = cnt[c];
  nm[c] = 0;
  cnt[c] = 0;
}

// Writes particle i (id i) of the caller's arrays into its cell's segment of
// the buffer holding the current state.
template <typename T>
__global__ void k_set_place(StateDev<T> b0, StateDev<T> b1, const Ctl* ctl, StepIndex si, const double* v,
                            const int32_t* elem, const double* om, int64_t n, int ne, int ens, const int32_t* start,
                            int32_t* pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const StateDev<T> st = (si.parity ^ (ctl->flip & 1u)) ? b1 : b0;
  const int c = ens * ne + elem[i];
  const int s = start[c] + atomicAdd(&pos[c], 1);
  st.x[s] = (T)v[i];
  st.y[s] = (T)v[n + i];
  st.u[s] = (T)v[2 * n + i];
  st.v[s] = (T)v[3 * n + i];
  st.w[s] = (T)v[4 * n + i];
  st.psi[s] = (T)v[5 * n + i];
  st.id[s] = (uint32_t)i;
  if (st.om) st.om[s] = (T)om[i];
}

__global__ void k_set_step(Ctl* ctl, uint32_t step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step_base = step;
}

// After a restore: the persistent scheduler's work counters start over (a
// step that returned early after an error left them unreset) and, once
// every ensemble has been restored, the error word and the overflow count.
__global__ void k_restore_ctl(Ctl* ctl, int clear_error) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->next[0] = 0;
    ctl->next[1] = 0;
    if (clear_error) {
      ctl->error = 0;
      ctl->ovf = 0;
    }
  }
}

__global__ void k_reset_ctl(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->step_base = 0; ctl->error = 0; ctl->ovf = 0; ctl->next[0] = 0; ctl->next[1] = 0;
    ctl->repack = 0; ctl->active = 0; ctl->flip = 0; ctl->repacks = 0;
  }
}

// ---------------------------------------------------------------------------
// repack: new segment layout from the current counts
//
// Segments are sized at seeding from the initial counts.  When the particle
// density drifts, a step flags the segments that run short of room
// (repack_due) and, at the next check, the planner gives every cell
// capacity max(initial, floor(grow (n + a)) + pad), a the cell's arrivals of
// the last step (or floor(slack n) + pad if that does not fit the slots), the
// mover copies each cell's particles, in their
// logical order, into the other buffer at the new offsets, and the buffer
// parity flips.  Without the flag both kernels return at once.

struct RepackPlan {
  const int32_t* cap;     // ncell: current capacities
  const int32_t* cap0;    // ncell: capacities at seeding
  const int32_t* ns;      // ncell: current counter set
  const int32_t* nm;
  int32_t* nstart;        // ncell: new offsets (out)
  int32_t* ncap;          // ncell: new capacities (out)
  Ctl* ctl;
  int32_t ncell;
  int32_t pad;
  int64_t slots;
  double grow, slack;
  uint32_t advance;       // steps to add to the Philox step base first (0: none)
  uint32_t unused;
};

constexpr int PLAN_THREADS = 1024;

__device__ __forceinline__ int64_t plan_cap(const RepackPlan& p, int c, bool fallback) {
  const int capc = p.cap[c];
  const int ns = min(p.ns[c], capc);
  const int nm = min(p.nm[c], capc - ns);
  const double n = (double)(ns + nm);
  if (fallback) return (int64_t)floor(p.slack * n) + p.pad;
  // room for the count to grow and for a step's arrivals (nm: the last step's)
  return max((int64_t)p.cap0[c], (int64_t)floor(p.grow * (n + (double)nm)) + p.pad);
}

// One block: capacities, then an exclusive scan over the cells.  Each
// wavefront owns a contiguous range of cells and reads it in runs of 64
// consecutive cells (coalesced, one cell per lane): first the range's sum,
// then, after a block scan of the wavefronts' sums, the offsets, by a
// wavefront scan of each run carried from run to run.
__global__ __launch_bounds__(PLAN_THREADS) void k_repack_plan(RepackPlan p) {
  constexpr int NW = PLAN_THREADS / WAVE;
  __shared__ int64_t wsum[NW];
  __shared__ int64_t total_s;
  Ctl* ctl = p.ctl;
  // a graph cycle ends here: its steps join the step base (no other thread
  // of this launch reads it)
  if (p.advance != 0u && threadIdx.x == 0) ctl->step_base = ctl->step_base + p.advance;
  if (ctl->repack == 0u || ctl->error != 0) {
    if (threadIdx.x == 0) ctl->active = 0u;
    return;
  }
  const int t = threadIdx.x;
  const int lane = lane_id(), wv = t / WAVE;
  // the wavefront's cells [c0, c1), a whole number of runs of 64
  const int per = (p.ncell + NW * WAVE - 1) / (NW * WAVE) * WAVE;
  const int c0 = min(p.ncell, wv * per), c1 = min(p.ncell, c0 + per);
  bool fallback = false;
  int64_t woff = 0;
  for (int pass = 0; pass < 2; ++pass) {
    int64_t mine = 0;
#pragma unroll 4
    for (int c = c0 + lane; c < c1; c += WAVE) mine += plan_cap(p, c, fallback);
    // the wavefront's sum, then the block's exclusive scan of those sums
    for (int off = WAVE / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off, WAVE);
    if (lane == 0) wsum[wv] = mine;
    __syncthreads();
    if (t == 0) {
      int64_t acc = 0;
      for (int w = 0; w < NW; ++w) {
        const int64_t v = wsum[w];
        wsum[w] = acc;
        acc += v;
      }
      total_s = acc;
    }
    __syncthreads();
    woff = wsum[wv];
    const int64_t total = total_s;
    __syncthreads();
    if (total <= p.slots) break;
    if (fallback) {
      // cannot happen while the particle count is conserved
      if (t == 0) {
        atomicOr(&ctl->error, ERR_CAPACITY);
        ctl->active = 0u;
        ctl->repack = 0u;
      }
      return;
    }
    fallback = true;
  }
  // offsets: an inclusive scan of each run of 64 cells, carried over the runs
  int64_t run = woff;
  for (int b = c0; b < c1; b += WAVE) {
    const int c = b + lane;
    const int64_t cp = c < c1 ? plan_cap(p, c, fallback) : 0;
    int64_t incl = cp;
    for (int off = 1; off < WAVE; off <<= 1) {
      const int64_t o = __shfl_up(incl, off, WAVE);
      if (lane >= off) incl += o;
    }
    if (c < c1) {
      p.nstart[c] = (int32_t)(run + incl - cp);
      p.ncap[c] = (int32_t)cp;
    }
    run += __shfl(incl, WAVE - 1, WAVE);
  }
  if (t == 0) {
    ctl->active = 1u;
    ctl->repack = 0u;
    ctl->flip = ctl->flip ^ 1u;
    ctl->repacks = ctl->repacks + 1u;
  }
}

template <typename T> struct RepackMove {
  StateDev<T> buf[2];
  int32_t* start;
  int32_t* cap;
  int32_t* ns;            // current counter set
  int32_t* nm;
  const int32_t* nstart;
  const int32_t* ncap;
  const Ctl* ctl;
  int32_t ncell;
};

// One wavefront per cell: copy the particles to the new segment (all in the
// bottom run) and install the new offsets, capacity and counts.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_repack_move(RepackMove<T> m, StepIndex si) {
  if (m.ctl->active == 0u) return;
  const int lane = lane_id();
  // the planner has flipped the parity: the current state is in the other buffer
  const uint32_t bnew = si.parity ^ (m.ctl->flip & 1u);
  const StateDev<T> src = m.buf[bnew ^ 1u];
  const StateDev<T> dst = m.buf[bnew];
  // one wavefront per cell, the grid's wavefronts striding over the cells
  // (a grid of bounded size: it is launched at every capacity check and
  // mostly returns at once)
  for (int cell = blockIdx.x * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE); cell < m.ncell;
       cell += gridDim.x * WAVES_PER_BLOCK) {
    const int capc = m.cap[cell], s0 = m.start[cell];
    const int ns = min(m.ns[cell], capc);
    const int nm = min(m.nm[cell], capc - ns);
    const int n = ns + nm;
    const int d0 = m.nstart[cell];
    for (int j = lane; j < n; j += WAVE) {
      const int s = slot_of(j, s0, ns, nm, capc);
      const int d = d0 + j;
      dst.x[d] = src.x[s]; dst.y[d] = src.y[s]; dst.u[d] = src.u[s]; dst.v[d] = src.v[s]; dst.w[d] = src.w[s];
      dst.psi[d] = src.psi[s]; dst.id[d] = src.id[s];
      if (src.om) dst.om[d] = src.om[s];
    }
    if (lane == 0) {
      m.start[cell] = d0;
      m.cap[cell] = m.ncap[cell];
      m.ns[cell] = n;
      m.nm[cell] = 0;
    }
  }
}

// Host-requested repack: raise the flag for the next planner.
__global__ void k_request_repack(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->repack = 1u;
}

// ---------------------------------------------------------------------------
// time averaging, point location, probes

// Time-averaged record per cell (doubles): steps averaged, pooled particle
// count, pooled means of u v w psi, pooled central second moments (pairs a<=b),
// summed histogram, then (with the turbulent frequency) pooled <omega> and
// <omega'^2>.
enum { AV_STEPS = 0, AV_N = 1, AV_MEAN = 2, AV_M2 = 6, AV_HIST = 16 };

// Merges each cell's statistics record of one step into its time average:
// the pooled sample of all the cell's particles over the averaged steps.
// Means and central moments are combined pairwise (Chan, Golub & LeVeque):
// with counts na, nb and mean difference d, M' = M_a + d nb / n and
// C' = (na C_a + nb C_b + d d^T na nb / n) / n.
// A block takes MERGE_CELLS consecutive cells: the record fields it needs
// (count, means, second moments, histogram, frequency statistics) and the
// averages are staged through LDS with coalesced loads, one thread merges
// each cell, and the averages go back coalesced.
constexpr int MERGE_CELLS = 64;
constexpr int MERGE_MAXAV = AV_HIST + 32 + 2;   // largest time-averaged record

__global__ __launch_bounds__(BLOCK) void k_average_merge(const double* stats, int nstat, int hoff, int hist,
                                                         int omega, double* acc, int navg, int ncell) {
  __shared__ double rs[MERGE_CELLS][MERGE_MAXAV];   // record fields, in the average's order
  __shared__ double as[MERGE_CELLS * MERGE_MAXAV];  // the averages, as stored
  const int c0 = blockIdx.x * MERGE_CELLS;
  const int nc = min(MERGE_CELLS, ncell - c0);
  if (nc <= 0) return;
  const int nrf = AV_HIST + hist + (omega ? 2 : 0);   // = navg
  // record field f of the average's layout: 0 count, 1..14 means and moments,
  // then histogram and frequency entries
  for (int i = threadIdx.x; i < nc * nrf; i += BLOCK) {
    const int c = i / nrf, f = i - c * nrf;
    int src;
    if (f < AV_HIST - 1) src = f;                       // ST_N, ST_MEAN.., ST_M2..
    else if (f < AV_HIST) src = -1;                     // no record field
    else if (f < AV_HIST + hist) src = hoff + (f - AV_HIST);
    else src = nstat - 3 + (f - AV_HIST - hist);
    rs[c][f] = src >= 0 ? stats[(size_t)(c0 + c) * nstat + src] : 0.0;
  }
  double* A0 = acc + (size_t)c0 * navg;
  for (int i = threadIdx.x; i < nc * navg; i += BLOCK) as[i] = A0[i];
  __syncthreads();
  const int c = threadIdx.x;
  if (c < nc) {
    const double* r = rs[c];
    double* A = as + c * navg;
    A[AV_STEPS] = A[AV_STEPS] + 1.0;
    const double nb = r[ST_N];
    if (nb > 0.0) {
      const double na = A[AV_N], nn = na + nb;
      const double fb = nb / nn, wab = na * fb;
      double d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = r[ST_MEAN + q] - A[AV_MEAN + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) A[AV_MEAN + q] = A[AV_MEAN + q] + d[q] * fb;
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = x; y < 4; ++y) {
          const int t = pair_index(x, y);
          A[AV_M2 + t] = ((na * A[AV_M2 + t] + nb * r[ST_M2 + t]) + wab * (d[x] * d[y])) / nn;
        }
      for (int h = 0; h < hist; ++h) A[AV_HIST + h] = A[AV_HIST + h] + r[AV_HIST + h];
      if (omega) {
        double* W = A + AV_HIST + hist;
        const double* rw = r + AV_HIST + hist;
        const double dw = rw[0] - W[0];
        W[0] = W[0] + dw * fb;
        W[1] = ((na * W[1] + nb * rw[1]) + wab * (dw * dw)) / nn;
      }
      A[AV_N] = nn;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nc * navg; i += BLOCK) A0[i] = as[i];
}

// Lowest-index element whose closed triangle contains each point (-1: none);
// one block per point.
__global__ __launch_bounds__(BLOCK) void k_locate(const ERec* erec, int ne, const double* xy, int npt,
                                                  int32_t* out) {
  __shared__ int best;
  const int p = blockIdx.x;
  if (p >= npt) return;
  if (threadIdx.x == 0) best = 0x7fffffff;
  __syncthreads();
  const double px = xy[2 * p], py = xy[2 * p + 1];
  for (int e = threadIdx.x; e < ne; e += BLOCK) {
    const ERec R = erec[e];
    if (orient_edge(R.x[0], R.y[0], R.x[1], R.y[1], px, py) >= 0.0 &&
        orient_edge(R.x[1], R.y[1], R.x[2], R.y[2], px, py) >= 0.0 &&
        orient_edge(R.x[2], R.y[2], R.x[0], R.y[0], px, py) >= 0.0) {
      atomicMin(&best, e);
      break;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) out[p] = best == 0x7fffffff ? -1 : best;
}

// Probe values from the time average of ensemble ens at the given elements,
// 4 + hist doubles each: steps averaged, mean particle count per step, <psi>,
// <psi'^2>, then the CDF of psi (eq. 29) at the upper edge of each histogram
// bin, F((b + 1) / hist) = (particles with psi < (b + 1) / hist) / count, from
// the summed histogram.  An element index out of range gives NaN.
__global__ void k_probe(const double* acc, int navg, int ne, int ens, const int32_t* elems, int nprobe, int hist,
                        double* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprobe) return;
  double* o = out + (size_t)p * (4 + hist);
  const int e = elems[p];
  if (e < 0 || e >= ne) {
    for (int q = 0; q < 4 + hist; ++q) o[q] = __builtin_nan("");
    return;
  }
  const double* A = acc + ((size_t)ens * ne + e) * navg;
  const double T = A[AV_STEPS], N = A[AV_N];
  o[0] = T;
  o[1] = T > 0.0 ? N / T : 0.0;
  o[2] = A[AV_MEAN + 3];
  o[3] = A[AV_M2 + 9];
  double cum = 0.0;
  for (int b = 0; b < hist; ++b) {
    cum = cum + A[AV_HIST + b];
    o[4 + b] = N > 0.0 ? cum / N : 0.0;
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace pdf
