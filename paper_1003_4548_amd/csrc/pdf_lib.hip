// Host side of the pdfpic C ABI: arena layout, argument checks, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pdf_kernels.hpp"
#include "pdfpic.h"

using namespace pdf;

namespace {

constexpr int64_t ALIGN = 256;
constexpr int32_t SEG_PAD = 32;

int64_t align_up(int64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Byte offsets of the arena sections.
struct Layout {
  int64_t vtx, tri, nbr, ekind, inv2a, alpha, fields, coef, erec;
  int64_t start, cap, ns[3], nm[3], rate, idoff, seed, src;
  int64_t buf0, buf1, ovf, ovf_cell, stats, ctl, flag;
  int64_t total;
  int64_t slots;
  int64_t ovf_cap;
};

Layout make_layout(int32_t nv, int32_t ne, int32_t nens, int64_t slots, int32_t nstat, int tsize) {
  Layout L{};
  int64_t o = 0;
  auto take = [&](int64_t bytes) { int64_t r = o; o = align_up(o + bytes); return r; };
  const int64_t ncell = (int64_t)ne * nens;
  L.vtx = take((int64_t)nv * 2 * 8);
  L.tri = take((int64_t)ne * 3 * 4);
  L.nbr = take((int64_t)ne * 3 * 4);
  L.ekind = take((int64_t)ne * 3 * 4);
  L.inv2a = take((int64_t)ne * 8);
  L.alpha = take((int64_t)ne * 3 * 8);
  L.fields = take((int64_t)nv * NFIELD * 8);
  L.coef = take((int64_t)nv * NCOEF * tsize);
  L.erec = take((int64_t)ne * (int64_t)sizeof(ERec));
  L.start = take(ncell * 4);
  L.cap = take(ncell * 4);
  for (int r = 0; r < 3; ++r) {
    L.ns[r] = take(ncell * 4);
    L.nm[r] = take(ncell * 4);
  }
  L.rate = take(ncell * tsize);
  L.idoff = take(ncell * 4);
  L.seed = take((int64_t)nens * 8);
  L.src = take((int64_t)nens * 3 * 8);
  const int64_t per_buf = align_up(slots * tsize) * 6 + align_up(slots * 4);
  L.buf0 = take(per_buf);
  L.buf1 = take(per_buf);
  L.ovf_cap = std::max<int64_t>(4096, slots / 64);
  L.ovf = take(align_up(L.ovf_cap * tsize) * 6 + align_up(L.ovf_cap * 4));
  L.ovf_cell = take(L.ovf_cap * 4);
  L.stats = take(ncell * (int64_t)nstat * 8);
  L.ctl = take(sizeof(Ctl));
  L.flag = take(16);
  L.total = o;
  L.slots = slots;
  return L;
}

template <typename T> StateDev<T> state_at(char* base, int64_t off, int64_t slots) {
  StateDev<T> s;
  char* p = base + off;
  const int64_t fb = align_up(slots * (int64_t)sizeof(T));
  s.x = (T*)(p + 0 * fb);
  s.y = (T*)(p + 1 * fb);
  s.u = (T*)(p + 2 * fb);
  s.v = (T*)(p + 3 * fb);
  s.w = (T*)(p + 4 * fb);
  s.psi = (T*)(p + 5 * fb);
  s.id = (uint32_t*)(p + 6 * fb);
  return s;
}

}  // namespace

struct pdf_ctx {
  pdf_params p{};
  hipStream_t stream = nullptr;
  int device = 0;
  // mesh
  int32_t nv = 0, ne = 0;
  bool mesh_ready = false;
  char* arena = nullptr;
  int64_t arena_bytes = 0;
  // ensembles
  int32_t nens = 0;
  bool seeded = false;
  int64_t slots = 0;
  Layout L{};
  std::vector<int32_t> h_start, h_cap, h_cnt, h_idoff, h_zero;
  std::vector<uint64_t> h_seed;
  std::vector<double> h_src;
  std::vector<int64_t> ens_count;
  std::string err;
  pdf_status last = PDF_OK;
};

namespace {

int tsize_of(const pdf_params& p) { return p.f32_state ? 4 : 8; }

int nstat_of(const pdf_params& p) { return (p.moments >= 4 ? NSTAT4 : NSTAT2) + p.hist_bins; }

pdf_status fail(pdf_ctx* c, pdf_status s, const std::string& msg) {
  if (c) {
    c->err = msg;
    c->last = s;
  }
  return s;
}

pdf_status hip_check(pdf_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return PDF_OK;
  return fail(c, PDF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t slots_bound(int64_t nparticles, int64_t ncell, double slack) {
  return (int64_t)std::ceil(slack * (double)nparticles) + (int64_t)(SEG_PAD + 1) * ncell;
}

template <typename T> StepArgs<T> step_args(pdf_ctx* c) {
  const Layout& L = c->L;
  char* a = c->arena;
  StepArgs<T> s{};
  s.erec = (const ERec*)(a + L.erec);
  s.tri = (const int32_t*)(a + L.tri);
  s.inv2a = (const double*)(a + L.inv2a);
  s.alpha = (const double*)(a + L.alpha);
  s.ne = c->ne;
  s.Lx = c->p.Lx;
  s.Ly = c->p.Ly;
  s.coef = (const T*)(a + L.coef);
  s.rate = (const T*)(a + L.rate);
  s.start = (const int32_t*)(a + L.start);
  s.cap = (const int32_t*)(a + L.cap);
  for (int r = 0; r < 3; ++r) {
    s.ns[r] = (int32_t*)(a + L.ns[r]);
    s.nm[r] = (int32_t*)(a + L.nm[r]);
  }
  s.buf[0] = state_at<T>(a, L.buf0, L.slots);
  s.buf[1] = state_at<T>(a, L.buf1, L.slots);
  s.ovf = state_at<T>(a, L.ovf, L.ovf_cap);
  s.ovf_cell = (int32_t*)(a + L.ovf_cell);
  s.ovf_cap = (uint32_t)L.ovf_cap;
  s.stats = (double*)(a + L.stats);
  s.seed = (const uint64_t*)(a + L.seed);
  s.src = (const double*)(a + L.src);
  s.ctl = (Ctl*)(a + L.ctl);
  s.ncell = c->ne * c->nens;
  s.nstat = nstat_of(c->p);
  s.flags = c->p.flags;
  s.mix = c->p.mix;
  s.dt = (T)c->p.dt;
  s.sdt = (T)std::sqrt((T)c->p.dt);
  s.nu2 = (T)(2.0 * c->p.nu);
  s.s2nu = (T)std::sqrt((T)(2.0 * c->p.nu));
  return s;
}

template <typename T, int MOM, int HIST, bool ADV> void launch_step(pdf_ctx* c, const StepArgs<T>& s) {
  const int ncell = s.ncell;
  const int blocks = (ncell + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  hipLaunchKernelGGL((k_step<T, MOM, HIST, ADV>), dim3(blocks), dim3(BLOCK), 0, c->stream, s);
}

template <typename T, bool ADV> pdf_status dispatch_step(pdf_ctx* c) {
  StepArgs<T> s = step_args<T>(c);
  const int mom = c->p.moments >= 4 ? 4 : 2;
  const int hist = c->p.hist_bins;
  if (mom == 2 && hist == 0) launch_step<T, 2, 0, ADV>(c, s);
  else if (mom == 2 && hist == 32) launch_step<T, 2, 32, ADV>(c, s);
  else if (mom == 4 && hist == 0) launch_step<T, 4, 0, ADV>(c, s);
  else if (mom == 4 && hist == 32) launch_step<T, 4, 32, ADV>(c, s);
  else return fail(c, PDF_E_ARG, "unsupported moments/hist_bins combination");
  return hip_check(c, hipGetLastError(), "step launch");
}

}  // namespace

extern "C" {

pdf_status pdf_create(const pdf_params* p, void* hip_stream, pdf_ctx** out) {
  if (!p || !out) return PDF_E_ARG;
  if (!(p->moments == 2 || p->moments == 4)) return PDF_E_ARG;
  if (!(p->hist_bins == 0 || p->hist_bins == 32)) return PDF_E_ARG;
  if (!(p->dt > 0.0) || p->nu < 0.0 || !(p->slack >= 1.0)) return PDF_E_ARG;
  pdf_ctx* c = new pdf_ctx();
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return PDF_E_HIP;
  }
  *out = c;
  return PDF_OK;
}

pdf_status pdf_query_sizes(const pdf_ctx* c, pdf_sizes* s) {
  if (!c || !s || s->nvert <= 0 || s->nelem <= 0 || s->nens <= 0 || s->nparticles < 0) return PDF_E_ARG;
  const int64_t ncell = (int64_t)s->nelem * s->nens;
  const int64_t slots = slots_bound(s->nparticles, ncell, c->p.slack);
  if (slots >= (int64_t)1 << 31) return PDF_E_SIZE;
  const Layout L = make_layout(s->nvert, s->nelem, s->nens, slots, nstat_of(c->p), tsize_of(c->p));
  s->arena_bytes = L.total;
  s->slots = slots;
  return PDF_OK;
}

pdf_status pdf_init_mesh(pdf_ctx* c, const pdf_mesh* m, void* arena, int64_t arena_bytes) {
  if (!c || !m || !arena || m->nvert <= 0 || m->nelem <= 0 || !m->vtx || !m->tri || !m->nbr || !m->ekind ||
      !m->fields)
    return fail(c, PDF_E_ARG, "pdf_init_mesh: null or empty input");
  if (((uintptr_t)arena) % ALIGN) return fail(c, PDF_E_ARG, "arena must be 256-byte aligned");
  for (int64_t i = 0; i < 3 * (int64_t)m->nelem; ++i) {
    if (m->tri[i] < 0 || m->tri[i] >= m->nvert) return fail(c, PDF_E_MESH, "vertex id out of range");
    if (m->ekind[i] < 0 || m->ekind[i] > 7) return fail(c, PDF_E_MESH, "unknown edge kind");
    const bool has_nbr = m->ekind[i] == PDF_EDGE_INTERIOR || m->ekind[i] >= PDF_EDGE_PERIODIC_XP;
    if (has_nbr && (m->nbr[i] < 0 || m->nbr[i] >= m->nelem)) return fail(c, PDF_E_MESH, "neighbour out of range");
  }
  c->nv = m->nvert;
  c->ne = m->nelem;
  c->arena = (char*)arena;
  c->arena_bytes = arena_bytes;
  // the mesh part of the layout does not depend on the ensembles
  Layout L = make_layout(c->nv, c->ne, 1, 1, nstat_of(c->p), tsize_of(c->p));
  if (L.erec + (int64_t)c->ne * (int64_t)sizeof(ERec) > arena_bytes) return fail(c, PDF_E_SIZE, "arena too small for the mesh");
  c->L = L;
  hipStream_t st = c->stream;
  pdf_status r;
  if ((r = hip_check(c, hipMemcpyAsync(c->arena + L.vtx, m->vtx, (size_t)c->nv * 2 * 8, hipMemcpyHostToDevice, st), "copy vtx"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(c->arena + L.tri, m->tri, (size_t)c->ne * 3 * 4, hipMemcpyHostToDevice, st), "copy tri"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(c->arena + L.nbr, m->nbr, (size_t)c->ne * 3 * 4, hipMemcpyHostToDevice, st), "copy nbr"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(c->arena + L.ekind, m->ekind, (size_t)c->ne * 3 * 4, hipMemcpyHostToDevice, st), "copy ekind"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(c->arena + L.fields, m->fields, (size_t)c->nv * NFIELD * 8, hipMemcpyHostToDevice, st), "copy fields"))) return r;
  int32_t* flag = (int32_t*)(c->arena + L.flag);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, flag, 0, (int64_t)4);
  const int tb = 256;
  hipLaunchKernelGGL(k_inv2a, dim3((c->ne + tb - 1) / tb), dim3(tb), 0, st, (const double*)(c->arena + L.vtx),
                     (const int32_t*)(c->arena + L.tri), (double*)(c->arena + L.inv2a), flag, c->ne);
  hipLaunchKernelGGL(k_erec, dim3((c->ne + tb - 1) / tb), dim3(tb), 0, st, (const double*)(c->arena + L.vtx),
                     (const int32_t*)(c->arena + L.tri), (const int32_t*)(c->arena + L.nbr),
                     (const int32_t*)(c->arena + L.ekind), (ERec*)(c->arena + L.erec), c->ne);
  hipLaunchKernelGGL(k_alpha, dim3((3 * c->ne + tb - 1) / tb), dim3(tb), 0, st, (const double*)(c->arena + L.vtx),
                     (const int32_t*)(c->arena + L.tri), (const int32_t*)(c->arena + L.ekind),
                     (const double*)(c->arena + L.fields), (double*)(c->arena + L.alpha), c->ne, c->p.Cmu,
                     c->p.kappa, c->p.Ewall, c->p.yp, c->p.nu);
  if (c->p.f32_state)
    hipLaunchKernelGGL(k_coefficients<float>, dim3((c->nv + tb - 1) / tb), dim3(tb), 0, st,
                       (const double*)(c->arena + L.fields), (float*)(c->arena + L.coef), c->nv, c->p.model,
                       c->p.C0, c->p.nu, c->p.CT);
  else
    hipLaunchKernelGGL(k_coefficients<double>, dim3((c->nv + tb - 1) / tb), dim3(tb), 0, st,
                       (const double*)(c->arena + L.fields), (double*)(c->arena + L.coef), c->nv, c->p.model,
                       c->p.C0, c->p.nu, c->p.CT);
  if ((r = hip_check(c, hipGetLastError(), "init kernels"))) return r;
  int32_t bad = 0;
  if ((r = hip_check(c, hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st), "read mesh flag"))) return r;
  if ((r = hip_check(c, hipStreamSynchronize(st), "sync init"))) return r;
  if (bad) return fail(c, PDF_E_MESH, "degenerate or clockwise element");
  c->mesh_ready = true;
  c->seeded = false;
  return PDF_OK;
}

pdf_status pdf_seed_particles(pdf_ctx* c, int32_t nens, const int64_t* counts, const uint64_t* seeds,
                              const double* source) {
  if (!c || nens <= 0 || !counts || !seeds || !source) return fail(c, PDF_E_ARG, "pdf_seed_particles: bad argument");
  if (!c->mesh_ready) return fail(c, PDF_E_STATE, "pdf_seed_particles before pdf_init_mesh");
  const int64_t ncell = (int64_t)nens * c->ne;
  if (ncell >= (int64_t)1 << 31) return fail(c, PDF_E_SIZE, "too many cells");
  c->nens = nens;
  c->h_start.assign(ncell, 0);
  c->h_cap.assign(ncell, 0);
  c->h_cnt.assign(ncell, 0);
  c->h_idoff.assign(ncell, 0);
  c->h_zero.assign(ncell, 0);
  c->ens_count.assign(nens, 0);
  int64_t total = 0, slot = 0;
  for (int32_t en = 0; en < nens; ++en) {
    int64_t id = 0;
    for (int32_t e = 0; e < c->ne; ++e) {
      const int64_t cell = (int64_t)en * c->ne + e;
      const int64_t n = counts[cell];
      if (n < 0 || n >= ((int64_t)1 << 30)) return fail(c, PDF_E_ARG, "bad particle count");
      c->h_idoff[cell] = (int32_t)id;
      c->h_cnt[cell] = (int32_t)n;
      id += n;
      if (id >= ((int64_t)1 << 31)) return fail(c, PDF_E_SIZE, "ensemble too large");
    }
    c->ens_count[en] = id;
    total += id;
  }
  // segment capacities, as in the sizing query
  const double slack = c->p.slack;
  for (int64_t cell = 0; cell < ncell; ++cell) {
    const int64_t capc = (int64_t)std::ceil(slack * (double)c->h_cnt[cell]) + SEG_PAD;
    c->h_start[cell] = (int32_t)slot;
    c->h_cap[cell] = (int32_t)capc;
    slot += capc;
  }
  const int64_t slots = slot;
  const Layout L = make_layout(c->nv, c->ne, nens, slots, nstat_of(c->p), tsize_of(c->p));
  if (L.total > c->arena_bytes)
    return fail(c, PDF_E_SIZE, "arena too small for the particle layout (query with slack >= 2)");
  c->L = L;
  c->slots = slots;
  c->h_seed.assign(seeds, seeds + nens);
  c->h_src.assign(source, source + 3 * (size_t)nens);
  for (int32_t en = 0; en < nens; ++en)
    if (!(c->h_src[3 * en + 2] >= 0.0)) return fail(c, PDF_E_ARG, "negative source radius");
  hipStream_t st = c->stream;
  char* a = c->arena;
  pdf_status r;
  if ((r = hip_check(c, hipMemcpyAsync(a + L.start, c->h_start.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy start"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(a + L.cap, c->h_cap.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy cap"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(a + L.ns[0], c->h_cnt.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy counts"))) return r;
  for (int rr = 0; rr < 3; ++rr) {
    if (rr > 0 && (r = hip_check(c, hipMemcpyAsync(a + L.ns[rr], c->h_zero.data(), ncell * 4, hipMemcpyHostToDevice, st), "clear counts"))) return r;
    if ((r = hip_check(c, hipMemcpyAsync(a + L.nm[rr], c->h_zero.data(), ncell * 4, hipMemcpyHostToDevice, st), "clear counts"))) return r;
  }
  if ((r = hip_check(c, hipMemcpyAsync(a + L.idoff, c->h_idoff.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy idoff"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(a + L.seed, c->h_seed.data(), nens * 8, hipMemcpyHostToDevice, st), "copy seeds"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(a + L.src, c->h_src.data(), nens * 3 * 8, hipMemcpyHostToDevice, st), "copy src"))) return r;
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, st, (Ctl*)(a + L.ctl));
  const int tb = 256;
  const int cb = (int)((ncell + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
  if (c->p.f32_state) {
    StepArgs<float> s = step_args<float>(c);
    hipLaunchKernelGGL(k_rate<float>, dim3((unsigned)((ncell + tb - 1) / tb)), dim3(tb), 0, st, (const double*)(a + L.vtx), s.tri,
                       (const double*)(a + L.fields), s.src, (float*)(a + L.rate), c->ne, (int)ncell, c->p.dt,
                       c->p.nu, c->p.CT, c->p.Cs, c->p.Ct);
    hipLaunchKernelGGL(k_seed<float>, dim3(cb), dim3(BLOCK), 0, st, s.erec, s.tri, s.inv2a,
                       (const double*)(a + L.fields), s.buf[0], s.start, (const int32_t*)s.ns[0],
                       (const int32_t*)(a + L.idoff), s.seed, c->ne, (int)ncell, c->p.psi_init);
  } else {
    StepArgs<double> s = step_args<double>(c);
    hipLaunchKernelGGL(k_rate<double>, dim3((unsigned)((ncell + tb - 1) / tb)), dim3(tb), 0, st, (const double*)(a + L.vtx), s.tri,
                       (const double*)(a + L.fields), s.src, (double*)(a + L.rate), c->ne, (int)ncell, c->p.dt,
                       c->p.nu, c->p.CT, c->p.Cs, c->p.Ct);
    hipLaunchKernelGGL(k_seed<double>, dim3(cb), dim3(BLOCK), 0, st, s.erec, s.tri, s.inv2a,
                       (const double*)(a + L.fields), s.buf[0], s.start, (const int32_t*)s.ns[0],
                       (const int32_t*)(a + L.idoff), s.seed, c->ne, (int)ncell, c->p.psi_init);
  }
  if ((r = hip_check(c, hipGetLastError(), "seed kernels"))) return r;
  // the host vectors stay alive in the context until the copies complete
  if ((r = hip_check(c, hipStreamSynchronize(st), "sync seed"))) return r;
  c->seeded = true;
  c->last = PDF_OK;
  c->err.clear();
  return PDF_OK;
}

pdf_status pdf_step(pdf_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return fail(c, PDF_E_ARG, "pdf_step: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_step before pdf_seed_particles");
  Ctl* ctl = (Ctl*)(c->arena + c->L.ctl);
  for (int32_t i = 0; i < nsteps; ++i) {
    pdf_status r = c->p.f32_state ? dispatch_step<float, true>(c) : dispatch_step<double, true>(c);
    if (r) return r;
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, c->stream, ctl);
  }
  return PDF_OK;
}

int32_t pdf_nstat(const pdf_ctx* c) { return c ? nstat_of(c->p) : 0; }

pdf_status pdf_estimate_statistics(pdf_ctx* c, double* out, int32_t out_on_host) {
  if (!c || !out) return fail(c, PDF_E_ARG, "pdf_estimate_statistics: null output");
  if (!c->seeded) return fail(c, PDF_E_STATE, "statistics before seeding");
  pdf_status r = c->p.f32_state ? dispatch_step<float, false>(c) : dispatch_step<double, false>(c);
  if (r) return r;
  const size_t bytes = (size_t)c->nens * c->ne * nstat_of(c->p) * 8;
  if ((r = hip_check(c, hipMemcpyAsync(out, c->arena + c->L.stats, bytes,
                                       out_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream),
                     "copy statistics")))
    return r;
  if (out_on_host) return hip_check(c, hipStreamSynchronize(c->stream), "sync statistics");
  return PDF_OK;
}

pdf_status pdf_sync(pdf_ctx* c) {
  if (!c) return PDF_E_ARG;
  pdf_status r;
  if ((r = hip_check(c, hipStreamSynchronize(c->stream), "stream sync"))) return r;
  if (!c->seeded) return PDF_OK;
  Ctl h{};
  if ((r = hip_check(c, hipMemcpy(&h, c->arena + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost), "read control"))) return r;
  if (h.error & ERR_LOST) return fail(c, PDF_E_LOST, "tracking could not place a particle");
  if (h.error & ERR_NAN) return fail(c, PDF_E_NAN, "non-finite particle state");
  if (h.error & (ERR_CAPACITY | ERR_OVERFLOW_FULL))
    return fail(c, PDF_E_CAPACITY, "an element segment overflowed its capacity");
  return PDF_OK;
}

pdf_status pdf_get_state(pdf_ctx* c, int32_t ens, double* xyuvwpsi, int32_t* elem) {
  if (!c || !xyuvwpsi || !elem) return fail(c, PDF_E_ARG, "pdf_get_state: null output");
  if (!c->seeded) return fail(c, PDF_E_STATE, "state before seeding");
  if (ens < 0 || ens >= c->nens) return fail(c, PDF_E_ARG, "ensemble out of range");
  const int64_t n = c->ens_count[ens];
  char* a = c->arena;
  const Layout& L = c->L;
  const int blocks = (c->ne + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  CounterSets cs;
  for (int r = 0; r < 3; ++r) {
    cs.ns[r] = (int32_t*)(a + L.ns[r]);
    cs.nm[r] = (int32_t*)(a + L.nm[r]);
  }
  if (c->p.f32_state)
    hipLaunchKernelGGL(k_gather<float>, dim3(blocks), dim3(BLOCK), 0, c->stream, state_at<float>(a, L.buf0, L.slots),
                       state_at<float>(a, L.buf1, L.slots), cs, (const int32_t*)(a + L.start),
                       (const int32_t*)(a + L.cap), (const Ctl*)(a + L.ctl), ens, c->ne, n, xyuvwpsi, elem);
  else
    hipLaunchKernelGGL(k_gather<double>, dim3(blocks), dim3(BLOCK), 0, c->stream, state_at<double>(a, L.buf0, L.slots),
                       state_at<double>(a, L.buf1, L.slots), cs, (const int32_t*)(a + L.start),
                       (const int32_t*)(a + L.cap), (const Ctl*)(a + L.ctl), ens, c->ne, n, xyuvwpsi, elem);
  return hip_check(c, hipGetLastError(), "gather launch");
}

int64_t pdf_count(const pdf_ctx* c, int32_t ens) {
  if (!c || ens < 0 || ens >= c->nens) return -1;
  return c->ens_count[ens];
}

int64_t pdf_steps_done(pdf_ctx* c) {
  if (!c || !c->seeded) return -1;
  Ctl h{};
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
  if (hipMemcpy(&h, c->arena + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return h.steps_done;
}

const char* pdf_error_string(const pdf_ctx* c) { return c ? c->err.c_str() : "null context"; }

void pdf_destroy(pdf_ctx* c) {
  if (!c) return;
  if (c->stream || c->seeded) (void)hipStreamSynchronize(c->stream);
  delete c;
}

}  // extern "C"
