// Runs the oracle's C interface on a workload read from a file, for the
// sanitizer builds (address and undefined-behaviour checks): create, seed
// every ensemble, average, step, and write the statistics, states, averages,
// omega and point locations of every ensemble to the output file.
//
// input: orc_params bytes; nvert, nelem (int32); vtx, tri, nbr, ekind,
// fields; nens (int32); per ensemble counts (nelem int64), seed (uint64),
// x0, y0, r0 (double); nsteps (int32); npoints (int32), points (2 doubles each)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "orc.h"

static FILE* in_file;
template <typename T> static void get(T* p, size_t n) {
  if (fread(p, sizeof(T), n, in_file) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
}
template <typename T> static void put(FILE* f, const T* p, size_t n) {
  if (fwrite(p, sizeof(T), n, f) != n) {
    fprintf(stderr, "short output\n");
    exit(2);
  }
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  in_file = fopen(argv[1], "rb");
  FILE* out = fopen(argv[2], "wb");
  if (!in_file || !out) return 2;
  orc_params p;
  get(&p, 1);
  int32_t nv, ne;
  get(&nv, 1);
  get(&ne, 1);
  std::vector<double> vtx(2 * (size_t)nv), fields(20 * (size_t)nv);
  std::vector<int32_t> tri(3 * (size_t)ne), nbr(3 * (size_t)ne), ekind(3 * (size_t)ne);
  get(vtx.data(), vtx.size());
  get(tri.data(), tri.size());
  get(nbr.data(), nbr.size());
  get(ekind.data(), ekind.size());
  get(fields.data(), fields.size());
  orc_set_threads(2);
  orc_ctx* c = orc_create(&p, nv, vtx.data(), ne, tri.data(), nbr.data(), ekind.data(), fields.data());
  if (!c) return 3;
  int32_t nens;
  get(&nens, 1);
  for (int32_t e = 0; e < nens; ++e) {
    std::vector<int64_t> counts(ne);
    uint64_t seed;
    double x0, y0, r0;
    get(counts.data(), counts.size());
    get(&seed, 1);
    get(&x0, 1);
    get(&y0, 1);
    get(&r0, 1);
    orc_add_ensemble(c, counts.data(), seed, x0, y0, r0);
  }
  int32_t nsteps, npts;
  get(&nsteps, 1);
  get(&npts, 1);
  std::vector<double> pts(2 * (size_t)npts);
  get(pts.data(), pts.size());
  orc_average_start(c);
  if (orc_step(c, nsteps) != 0) return 4;
  const int32_t ns = orc_nstat(c), na = orc_navg(c);
  for (int32_t e = 0; e < nens; ++e) {
    std::vector<double> st((size_t)ne * ns), av((size_t)ne * na);
    orc_stats(c, e, st.data());
    put(out, st.data(), st.size());
    const int64_t n = orc_count(c, e);
    std::vector<double> x(n), y(n), u(n), v(n), w(n), psi(n), om(n);
    std::vector<int32_t> el(n);
    orc_get_state(c, e, x.data(), y.data(), u.data(), v.data(), w.data(), psi.data(), el.data());
    for (auto* a : {&x, &y, &u, &v, &w, &psi}) put(out, a->data(), a->size());
    put(out, el.data(), el.size());
    if (p.omega) {
      orc_get_omega(c, e, om.data());
      put(out, om.data(), om.size());
    }
    orc_average(c, e, av.data());
    put(out, av.data(), av.size());
    // a restore of the same state leaves the statistics unchanged
    orc_set_state(c, e, x.data(), y.data(), u.data(), v.data(), w.data(), psi.data(), el.data());
    std::vector<double> st2((size_t)ne * ns);
    orc_stats(c, e, st2.data());
    put(out, st2.data(), st2.size());
  }
  std::vector<int32_t> loc(npts);
  for (int32_t q = 0; q < npts; ++q) loc[q] = orc_locate(c, pts[2 * q], pts[2 * q + 1]);
  put(out, loc.data(), loc.size());
  orc_destroy(c);
  fclose(out);
  fclose(in_file);
  return 0;
}
