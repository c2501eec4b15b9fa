// Host bookkeeping of the elliptic relaxation (section 2.1): the structure of
// the Galerkin system of eq. (14) on the mesh, in plain C++ (no HIP), so that
// it can also be built and checked on the CPU under the sanitizers.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace pdf {
namespace host {

// The structure of the relaxation system:
// * unknowns: the vertices, with the copies of one point of the periodic
//   domain joined (across a periodic edge, the partner element's vertex that
//   equals an edge vertex shifted by the edge's period), numbered by their
//   lowest vertex index; rep[i] is that vertex;
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
inline RelaxStatus build_relax_structure(int32_t nv, int32_t ne, const double* vtx, const int32_t* tri,
                                         const int32_t* nbr, const int32_t* ekind, double Lx, double Ly,
                                         int32_t ell_max, RelaxStructure& s) {
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
  std::vector<int32_t> id_of(nv, -1);
  for (int32_t v = 0; v < nv; ++v) {
    const int32_t r = find(v);
    if (r == v) {
      id_of[v] = (int32_t)s.rep.size();
      s.rep.push_back(v);
    }
    s.canon[v] = id_of[r];
  }
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

}  // namespace host
}  // namespace pdf
