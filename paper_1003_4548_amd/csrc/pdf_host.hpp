// Host bookkeeping of the elliptic relaxation (section 2.1): the structure of
// the Galerkin system of eq. (14) on the mesh, in plain C++ (no HIP), so that
// it can also be built and checked on the CPU under the sanitizers.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <string>
#include <vector>

namespace pdf {
namespace host {

// The structure of the relaxation system:
// * unknowns: the vertices, with the copies of one point of the periodic
//   domain joined (across a periodic edge, the partner element's vertex that
//   equals an edge vertex shifted by the edge's period); rep[i] is the lowest
//   vertex index of unknown i; numbered by recursive coordinate bisection of
//   the rep vertices (the longer side of the bounding box halved at a
//   multiple of agg unknowns, ties by vertex index), so that every run of
//   agg consecutive unknowns (an aggregate of the projection's coarse space)
//   is a compact patch of the mesh;
// * the matrix rows in CSR form (rowptr, col), each nonzero with its element
//   contributions e * 9 + a * 3 + b (element, local row, local column) in
//   increasing order (cptr, cidx), so that a gather assembles every entry in
//   a fixed order;
// * the rows padded to the longest, ellw entries (ecol, enz: slot t of row i
//   at t * nc + i; padding points at the row itself with nonzero index -1),
//   and dpos[i], the nonzero index of row i's diagonal entry;
// * the (element, local vertex) pairs e * 3 + a of every unknown in
//   increasing order (incptr, inc).
struct RelaxStructure {
  int32_t nc = 0, ellw = 0;
  int64_t nnz = 0;
  std::vector<int32_t> canon, rep, rowptr, col, cptr, cidx, ecol, enz, dpos, incptr, inc;
};

enum RelaxStatus { RELAX_OK = 0, RELAX_ROW_TOO_LONG = 1, RELAX_LONE_VERTEX = 2 };

// Edge kinds 4..7 are periodic: crossing adds +Lx, -Lx, +Ly, -Ly.
// The unknowns' classes (by their lowest vertex) in recursive coordinate
// bisection order into runs of agg.
inline void bisection_order(const double* vtx, std::vector<int32_t>& ord, size_t lo, size_t hi, int32_t agg) {
  const size_t n = hi - lo;
  if (n <= (size_t)agg) return;
  double x0 = vtx[2 * ord[lo]], x1 = x0, y0 = vtx[2 * ord[lo] + 1], y1 = y0;
  for (size_t k = lo; k < hi; ++k) {
    x0 = std::min(x0, vtx[2 * ord[k]]);
    x1 = std::max(x1, vtx[2 * ord[k]]);
    y0 = std::min(y0, vtx[2 * ord[k] + 1]);
    y1 = std::max(y1, vtx[2 * ord[k] + 1]);
  }
  const int ax = (x1 - x0) >= (y1 - y0) ? 0 : 1;
  std::sort(ord.begin() + (std::ptrdiff_t)lo, ord.begin() + (std::ptrdiff_t)hi, [&](int32_t a, int32_t b) {
    const double ca = vtx[2 * a + ax], cb = vtx[2 * b + ax];
    return ca != cb ? ca < cb : a < b;
  });
  const size_t half = ((n + agg - 1) / agg / 2) * (size_t)agg;
  bisection_order(vtx, ord, lo, lo + half, agg);
  bisection_order(vtx, ord, lo + half, hi, agg);
}

inline RelaxStatus build_relax_structure(int32_t nv, int32_t ne, const double* vtx, const int32_t* tri,
                                         const int32_t* nbr, const int32_t* ekind, double Lx, double Ly,
                                         int32_t ell_max, int32_t agg, RelaxStructure& s) {
  std::vector<int32_t> root(nv);
  for (int32_t v = 0; v < nv; ++v) root[v] = v;
  auto find = [&](int32_t v) {
    while (root[v] != v) {
      root[v] = root[root[v]];
      v = root[v];
    }
    return v;
  };
  for (int32_t e = 0; e < ne; ++e) {
    for (int k = 0; k < 3; ++k) {
      const int32_t kind = ekind[3 * e + k];
      if (kind < 4 || kind > 7) continue;
      const double sx = kind == 4 ? Lx : (kind == 5 ? -Lx : 0.0);
      const double sy = kind == 6 ? Ly : (kind == 7 ? -Ly : 0.0);
      const int32_t nb = nbr[3 * e + k];
      for (int j = 0; j < 2; ++j) {
        const int32_t v = tri[3 * e + (k + j) % 3];
        const double px = vtx[2 * v] + sx, py = vtx[2 * v + 1] + sy;
        for (int t = 0; t < 3; ++t) {
          const int32_t w = tri[3 * nb + t];
          if (vtx[2 * w] != px || vtx[2 * w + 1] != py) continue;
          const int32_t a = find(v), b = find(w);
          if (a != b) root[std::max(a, b)] = std::min(a, b);   // a class's root is its lowest vertex
        }
      }
    }
  }
  s = RelaxStructure{};
  s.canon.assign(nv, 0);
  for (int32_t v = 0; v < nv; ++v)
    if (find(v) == v) s.rep.push_back(v);
  bisection_order(vtx, s.rep, 0, s.rep.size(), std::max(1, agg));
  std::vector<int32_t> id_of(nv, -1);
  for (size_t i = 0; i < s.rep.size(); ++i) id_of[s.rep[i]] = (int32_t)i;
  for (int32_t v = 0; v < nv; ++v) s.canon[v] = id_of[find(v)];
  const int32_t nc = (int32_t)s.rep.size();
  s.nc = nc;
  struct Ent {
    int32_t row, col, cid;
  };
  std::vector<Ent> ent((size_t)9 * ne);
  for (int32_t e = 0; e < ne; ++e)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        ent[(size_t)9 * e + 3 * a + b] = Ent{s.canon[tri[3 * e + a]], s.canon[tri[3 * e + b]], 9 * e + 3 * a + b};
  std::sort(ent.begin(), ent.end(), [](const Ent& x, const Ent& y) {
    if (x.row != y.row) return x.row < y.row;
    if (x.col != y.col) return x.col < y.col;
    return x.cid < y.cid;
  });
  s.rowptr.assign((size_t)nc + 1, 0);
  s.cidx.resize(ent.size());
  for (size_t i = 0; i < ent.size(); ++i) {
    s.cidx[i] = ent[i].cid;
    if (i == 0 || ent[i].row != ent[i - 1].row || ent[i].col != ent[i - 1].col) {
      s.col.push_back(ent[i].col);
      s.cptr.push_back((int32_t)i);
      ++s.rowptr[ent[i].row + 1];
    }
  }
  s.cptr.push_back((int32_t)ent.size());
  for (int32_t i = 0; i < nc; ++i) s.rowptr[i + 1] += s.rowptr[i];
  s.nnz = (int64_t)s.col.size();
  s.incptr.assign((size_t)nc + 1, 0);
  s.inc.resize((size_t)3 * ne);
  for (int32_t e = 0; e < ne; ++e)
    for (int a = 0; a < 3; ++a) ++s.incptr[s.canon[tri[3 * e + a]] + 1];
  for (int32_t i = 0; i < nc; ++i) {
    if (s.incptr[i + 1] == 0) return RELAX_LONE_VERTEX;
    s.incptr[i + 1] += s.incptr[i];
  }
  std::vector<int32_t> fill(s.incptr.begin(), s.incptr.end() - 1);
  for (int32_t e = 0; e < ne; ++e)
    for (int a = 0; a < 3; ++a) s.inc[fill[s.canon[tri[3 * e + a]]]++] = 3 * e + a;
  // rows padded to the longest
  int32_t ellw = 0;
  for (int32_t i = 0; i < nc; ++i) ellw = std::max(ellw, s.rowptr[i + 1] - s.rowptr[i]);
  if (ellw > ell_max) return RELAX_ROW_TOO_LONG;
  s.ellw = ellw;
  s.dpos.assign((size_t)nc, -1);
  s.ecol.resize((size_t)ellw * nc);
  s.enz.resize((size_t)ellw * nc);
  for (int32_t i = 0; i < nc; ++i)
    for (int32_t t = 0; t < ellw; ++t) {
      const int32_t j = s.rowptr[i] + t;
      const bool has = j < s.rowptr[i + 1];
      s.ecol[(size_t)t * nc + i] = has ? s.col[j] : i;
      s.enz[(size_t)t * nc + i] = has ? j : -1;
      if (has && s.col[j] == i) s.dpos[i] = j;
    }
  return RELAX_OK;
}

// The coarse space of the projection's preconditioner M^-1 = D^-1 + Z E^+ Z^T:
// Z has one column per aggregate (agg consecutive unknowns, the last one
// possibly shorter), E = Z^T K Z with K the P1 stiffness matrix (the
// projection's system); K and E are singular (constants), so E^+ is the
// inverse of E + sigma 1 1^T (sigma = trace(E) / na^2), which maps every v
// with zero sum to the solution of E y = v with zero sum.  A solver block of
// blk unknowns reads the correction of the aggregates its rows touch: need
// lists of need_max entries per block (its own aggregates first, then the
// others in increasing order, -1 padding), and for every padded row slot the
// position of its column's aggregate in its row's list.
struct CoarseStructure {
  int32_t na = 0;
  std::vector<double> ep;        // na x na
  std::vector<int32_t> need;     // nbx x need_max
  std::vector<int32_t> eneed;    // ellw x nc
};

enum CoarseStatus { COARSE_OK = 0, COARSE_TOO_LARGE = 1, COARSE_NEED = 2, COARSE_SINGULAR = 3 };

inline CoarseStatus build_coarse(const RelaxStructure& s, int32_t ne, const double* vtx, const int32_t* tri,
                                 int32_t agg, int32_t blk, int32_t need_max, int32_t na_max, CoarseStructure& cs) {
  cs = CoarseStructure{};
  const int32_t nc = s.nc, na = (nc + agg - 1) / agg, apb = blk / agg, nbx = (nc + blk - 1) / blk;
  if (na > na_max || na < 1) return COARSE_TOO_LARGE;
  // E from the element stiffness matrices: 4|A| Ke_ab = b_a b_b + c_a c_b with
  // b_k = y_{k+1} - y_{k+2}, c_k = x_{k+2} - x_{k+1}
  std::vector<double> E((size_t)na * na, 0.0);
  for (int32_t e = 0; e < ne; ++e) {
    double x[3], y[3], b[3], c[3];
    int32_t g[3];
    for (int k = 0; k < 3; ++k) {
      x[k] = vtx[2 * tri[3 * e + k]];
      y[k] = vtx[2 * tri[3 * e + k] + 1];
      g[k] = s.canon[tri[3 * e + k]] / agg;
    }
    for (int k = 0; k < 3; ++k) {
      b[k] = y[(k + 1) % 3] - y[(k + 2) % 3];
      c[k] = x[(k + 2) % 3] - x[(k + 1) % 3];
    }
    const double a4 = 2.0 * std::fabs((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]));
    if (!(a4 > 0.0)) continue;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) E[(size_t)g[i] * na + g[j]] += (b[i] * b[j] + c[i] * c[j]) / a4;
  }
  double tr = 0.0;
  for (int32_t i = 0; i < na; ++i) tr += E[(size_t)i * na + i];
  if (!(tr > 0.0)) return COARSE_SINGULAR;
  const double sigma = tr / ((double)na * na);
  for (double& v : E) v += sigma;
  // Gauss-Jordan with partial pivoting
  std::vector<double> inv((size_t)na * na, 0.0);
  for (int32_t i = 0; i < na; ++i) inv[(size_t)i * na + i] = 1.0;
  for (int32_t k = 0; k < na; ++k) {
    int32_t pr = k;
    for (int32_t i = k + 1; i < na; ++i)
      if (std::fabs(E[(size_t)i * na + k]) > std::fabs(E[(size_t)pr * na + k])) pr = i;
    const double pv = E[(size_t)pr * na + k];
    if (!(std::fabs(pv) > 1e-300)) return COARSE_SINGULAR;
    if (pr != k)
      for (int32_t j = 0; j < na; ++j) {
        std::swap(E[(size_t)pr * na + j], E[(size_t)k * na + j]);
        std::swap(inv[(size_t)pr * na + j], inv[(size_t)k * na + j]);
      }
    for (int32_t j = 0; j < na; ++j) {
      E[(size_t)k * na + j] /= pv;
      inv[(size_t)k * na + j] /= pv;
    }
    for (int32_t i = 0; i < na; ++i) {
      if (i == k) continue;
      const double f = E[(size_t)i * na + k];
      if (f == 0.0) continue;
      for (int32_t j = 0; j < na; ++j) {
        E[(size_t)i * na + j] -= f * E[(size_t)k * na + j];
        inv[(size_t)i * na + j] -= f * inv[(size_t)k * na + j];
      }
    }
  }
  for (double v : inv)
    if (!std::isfinite(v)) return COARSE_SINGULAR;
  // need lists and the slots' positions in them
  cs.need.assign((size_t)nbx * need_max, -1);
  cs.eneed.assign((size_t)s.ellw * nc, 0);
  for (int32_t bx = 0; bx < nbx; ++bx) {
    std::vector<int32_t> own, other;
    for (int32_t k = 0; k < apb; ++k)
      if (bx * apb + k < na) own.push_back(bx * apb + k);
    const int32_t i0 = bx * blk, i1 = std::min(nc, i0 + blk);
    for (int32_t i = i0; i < i1; ++i)
      for (int32_t t = 0; t < s.ellw; ++t) {
        const int32_t ag = s.ecol[(size_t)t * nc + i] / agg;
        if (ag / apb != bx) other.push_back(ag);
      }
    std::sort(other.begin(), other.end());
    other.erase(std::unique(other.begin(), other.end()), other.end());
    if ((int32_t)(own.size() + other.size()) > need_max) return COARSE_NEED;
    std::vector<int32_t> list = own;
    list.insert(list.end(), other.begin(), other.end());
    for (size_t k = 0; k < list.size(); ++k) cs.need[(size_t)bx * need_max + k] = list[k];
    for (int32_t i = i0; i < i1; ++i)
      for (int32_t t = 0; t < s.ellw; ++t) {
        const int32_t ag = s.ecol[(size_t)t * nc + i] / agg;
        cs.eneed[(size_t)t * nc + i] = (int32_t)(std::find(list.begin(), list.end(), ag) - list.begin());
      }
  }
  cs.na = na;
  cs.ep = std::move(inv);
  return COARSE_OK;
}

}  // namespace host
}  // namespace pdf
