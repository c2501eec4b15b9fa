// Builds the relaxation system's structure (pdf::host::build_relax_structure)
// and the projection's coarse space (pdf::host::build_coarse) of a mesh read
// from a file, for the sanitizer builds, and writes them out.
//
// input: nvert, nelem (int32); Lx, Ly (double); vtx, tri, nbr, ekind;
// ell_max, agg, blk, need_max, na_max (int32)
// output: status, nc, ellw (int32), nnz (int64), then canon, rep, rowptr, col,
// cptr, cidx, ecol, enz, dpos, incptr, inc, each as its length (int64) and
// int32s; then the coarse status and na (int32), ep (length, doubles), need
// and eneed (length, int32s)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pdf_host.hpp"

static FILE* in_file;
template <typename T> static void get(T* p, size_t n) {
  if (fread(p, sizeof(T), n, in_file) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  in_file = fopen(argv[1], "rb");
  FILE* out = fopen(argv[2], "wb");
  if (!in_file || !out) return 2;
  int32_t nv, ne, ell_max, agg, blk, need_max, na_max;
  double Lx, Ly;
  get(&nv, 1);
  get(&ne, 1);
  get(&Lx, 1);
  get(&Ly, 1);
  std::vector<double> vtx(2 * (size_t)nv);
  std::vector<int32_t> tri(3 * (size_t)ne), nbr(3 * (size_t)ne), ekind(3 * (size_t)ne);
  get(vtx.data(), vtx.size());
  get(tri.data(), tri.size());
  get(nbr.data(), nbr.size());
  get(ekind.data(), ekind.size());
  get(&ell_max, 1);
  get(&agg, 1);
  get(&blk, 1);
  get(&need_max, 1);
  get(&na_max, 1);
  pdf::host::RelaxStructure s;
  const int32_t st = pdf::host::build_relax_structure(nv, ne, vtx.data(), tri.data(), nbr.data(), ekind.data(), Lx,
                                                      Ly, ell_max, agg, s);
  fwrite(&st, 4, 1, out);
  fwrite(&s.nc, 4, 1, out);
  fwrite(&s.ellw, 4, 1, out);
  fwrite(&s.nnz, 8, 1, out);
  for (const auto* a : {&s.canon, &s.rep, &s.rowptr, &s.col, &s.cptr, &s.cidx, &s.ecol, &s.enz, &s.dpos, &s.incptr,
                        &s.inc}) {
    const int64_t n = (int64_t)a->size();
    fwrite(&n, 8, 1, out);
    if (n) fwrite(a->data(), 4, (size_t)n, out);
  }
  pdf::host::CoarseStructure cs;
  const int32_t cst = st == 0 ? pdf::host::build_coarse(s, ne, vtx.data(), tri.data(), agg, blk, need_max, na_max, cs) : -1;
  fwrite(&cst, 4, 1, out);
  fwrite(&cs.na, 4, 1, out);
  const int64_t nep = (int64_t)cs.ep.size();
  fwrite(&nep, 8, 1, out);
  if (nep) fwrite(cs.ep.data(), 8, (size_t)nep, out);
  for (const auto* a : {&cs.need, &cs.eneed}) {
    const int64_t n = (int64_t)a->size();
    fwrite(&n, 8, 1, out);
    if (n) fwrite(a->data(), 4, (size_t)n, out);
  }
  fclose(out);
  fclose(in_file);
  return 0;
}
