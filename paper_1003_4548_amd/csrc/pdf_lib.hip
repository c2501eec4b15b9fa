// Host side of the pdfpic C ABI: arena layout, argument checks, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "pdf_host.hpp"
#include "pdf_kernels.hpp"
#include "pdf_mlp.hpp"
#include "pdf_relax.hpp"
#include "pdfmlp.h"
#include "pdfpic.h"

using namespace pdf;

namespace {

constexpr int64_t ALIGN = 256;
constexpr int32_t SEG_PAD = 32;
// cells of at most SMALL_COUNT particles at seeding may take a step launch of
// their own at SMALL_GROUP lanes per cell (see pdf_seed_particles): 16 cells
// per wavefront share its per-cell work (batched steps 4 % shorter than at 8
// lanes per cell, 0.7 % shorter than with only cells of at most 4 there)
constexpr int32_t SMALL_GROUP = 4;
constexpr int32_t SMALL_COUNT = 8;

int64_t align_up(int64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Byte offsets of the arena sections.
struct Layout {
  int64_t vtx, tri, nbr, ekind, inv2a, alpha, wnorm, fields, coef, erec, om0, somega, omw;
  // the Eulerian solves (elliptic relaxation, mean-pressure projection): sparsity, element data, solver vectors
  int64_t rx_canon, rx_rep, rx_ecol, rx_enz, rx_dpos, rx_cptr, rx_cidx, rx_incptr, rx_inc, rx_Ke, rx_area;
  int64_t rx_S, rx_L2, rx_Rk, rx_aval, rx_dinv, rx_x, rx_px, rx_p, rx_rec[2], rx_part[2], rx_pbb, rx_ctl;
  int64_t rx_ep, rx_eneed, rx_agp[2], rx_cglob[2];   // the projection's coarse space
  int64_t start, cap, cap0, nstart, ncap, ns[3], nm[3], rate, idoff, order, seed, src;
  int64_t buf0, buf1, ovf, ovf_cell, stats, ctl, flag, metrics;
  int64_t total;
  int64_t slots;
  int64_t ovf_cap;
  bool omega;  // the particle buffers carry the turbulent frequency
};

// Iterations of one relaxation solve at most.
constexpr int32_t RELAX_MAX_ITERS = 20000;
// Iterations of the two replayed relaxation graphs (even: the parity of an
// iteration continues across replays).
constexpr int32_t RELAX_LONG = 32, RELAX_SHORT = 8;
// Nonzeros of the relaxation matrix at most: the diagonal and the six
// ordered vertex pairs of every element.
int64_t relax_nnz_bound(int32_t nv, int32_t ne) { return (int64_t)nv + 6 * (int64_t)ne; }
int32_t relax_blocks(int32_t nv) { return std::max(1, (nv + relax::BLK - 1) / relax::BLK); }

Layout make_layout(int32_t nv, int32_t ne, int32_t nens, int64_t slots, int32_t nstat, int tsize, bool omega) {
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
  L.wnorm = take((int64_t)ne * 6 * 8);
  L.fields = take((int64_t)nv * NFIELD * 8);
  L.coef = take((int64_t)nv * NCOEF * tsize);
  L.erec = take((int64_t)ne * (int64_t)sizeof(ERec));
  L.om0 = take(omega ? (int64_t)ne * 8 : 0);
  L.somega = take(omega ? (int64_t)ne * 8 : 0);
  L.omw = take(omega ? (int64_t)ne * 3 * 8 : 0);
  {
    const int64_t nnz = relax_nnz_bound(nv, ne), nc = nv, E = ne, vec = relax::NC * nc * 8;
    const int64_t ell = (int64_t)relax::ELL_MAX * nc, nbx = relax_blocks(nv);
    L.rx_canon = take(nv * 4);
    L.rx_rep = take(nc * 4);
    L.rx_ecol = take(ell * 4);
    L.rx_enz = take(ell * 4);
    L.rx_dpos = take(nc * 4);
    L.rx_cptr = take((nnz + 1) * 4);
    L.rx_cidx = take(9 * E * 4);
    L.rx_incptr = take((nc + 1) * 4);
    L.rx_inc = take(3 * E * 4);
    L.rx_Ke = take(9 * E * 8);
    L.rx_area = take(E * 8);
    L.rx_S = take(relax::NC * E * 8);
    L.rx_L2 = take(E * 8);
    L.rx_Rk = take(4 * E * 8);
    L.rx_aval = take(ell * 8);
    L.rx_dinv = take(nc * 8);
    L.rx_x = take(vec);
    L.rx_px = take(vec);
    L.rx_p = take(vec);
    for (int b = 0; b < 2; ++b) {
      L.rx_rec[b] = take(relax::NC * nc * (int64_t)sizeof(relax::Rec));
      L.rx_part[b] = take(relax::NC * nbx * 3 * 8);
    }
    L.rx_pbb = take(relax::NC * nbx * 8);
    L.rx_ctl = take((int64_t)sizeof(relax::Ctl));
    const int64_t na = std::min<int64_t>((nc + relax::AGG - 1) / relax::AGG, relax::NA_MAX);
    const int64_t nbc = (na + relax::APB - 1) / relax::APB;   // blocks that can hold a coarse space
    L.rx_ep = take(nbc * relax::NEED * relax::NA_MAX * 4);
    L.rx_eneed = take(ell * 4);
    for (int b = 0; b < 2; ++b) {
      L.rx_agp[b] = take(relax::NA_MAX * 3 * 8);
      L.rx_cglob[b] = take(relax::NA_MAX * 8);
    }
  }
  L.start = take(ncell * 4);
  L.cap = take(ncell * 4);
  L.cap0 = take(ncell * 4);
  L.nstart = take(ncell * 4);
  L.ncap = take(ncell * 4);
  for (int r = 0; r < 3; ++r) {
    L.ns[r] = take(ncell * 4);
    L.nm[r] = take(ncell * 4);
  }
  L.rate = take(ncell * tsize);
  L.idoff = take(ncell * 4);
  L.order = take(ncell * 4);
  L.seed = take((int64_t)nens * 8);
  L.src = take((int64_t)nens * 3 * 8);
  const int64_t per_buf = align_up(slots * tsize) * (omega ? 7 : 6) + align_up(slots * 4);
  L.buf0 = take(per_buf);
  L.buf1 = take(per_buf);
  L.ovf_cap = std::max<int64_t>(4096, slots / 64);
  L.ovf = take(align_up(L.ovf_cap * tsize) * (omega ? 7 : 6) + align_up(L.ovf_cap * 4));
  L.ovf_cell = take(L.ovf_cap * 4);
  L.stats = take(ncell * (int64_t)nstat * 8);
  L.ctl = take(sizeof(Ctl));
  L.flag = take(16);
  L.metrics = take(64);
  L.total = o;
  L.slots = slots;
  L.omega = omega;
  return L;
}

// x y u v w psi, id, then omega when carried
template <typename T> StateDev<T> state_at(char* base, int64_t off, int64_t slots, bool omega) {
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
  s.om = omega ? (T*)(p + 6 * fb + align_up(slots * 4)) : nullptr;
  return s;
}

}  // namespace

// Replayable graphs of RELAX_LONG and RELAX_SHORT iteration launches of one
// solve (built for its kernel arguments: pointers of the mesh part of the
// arena), and the iteration count of its last run.
struct SolveGraphs {
  hipGraph_t g[2] = {nullptr, nullptr};
  hipGraphExec_t ex[2] = {nullptr, nullptr};
  bool ok = false;
  int32_t last_iters = 0;
  void release() {
    for (int i = 0; i < 2; ++i) {
      if (ex[i]) (void)hipGraphExecDestroy(ex[i]);
      if (g[i]) (void)hipGraphDestroy(g[i]);
      ex[i] = nullptr;
      g[i] = nullptr;
    }
    ok = false;
  }
};

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
  std::vector<int32_t> h_start, h_cap, h_cnt, h_idoff, h_zero, h_order;
  // host-side step state: the launch arguments of the next step
  int64_t steps_done = 0;
  int64_t proj_mark = 0;   // steps_done at the last applied projection
  uint32_t parity = 0, rot = 0;
  // launch configuration (set by pdf_autotune; defaults below)
  int32_t group = 64;     // lanes per cell
  int32_t persist = 0;    // persistent scheduler
  int32_t persist_blocks = 0;
  // cells of the order's first part (the rest are small cells, stepped by a
  // launch of their own at SMALL_GROUP lanes per cell); 0: one launch
  int64_t nsplit = 0;
  // per lanes-per-cell (64, 32, 16, 8, 4) and order part: the XCD ranges of
  // work items and the cell count they were cut for (-1: none since seeding)
  int32_t xcd[5][2][9] = {};
  int64_t xcd_n[5][2] = {{-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}};
  // replayable graph of GRAPH_STEPS steps (built for one launch shape)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int32_t graph_group = 0, graph_persist = -1;
  // learned conditional means in the step (null: binned means)
  const uint16_t* mlp_w = nullptr;
  const float* mlp_norm = nullptr;
  double* mlp_cm = nullptr;
  uint32_t* mlp_served = nullptr;
  // time-averaged statistics (caller-owned, null: not averaging)
  double* avg = nullptr;
  std::vector<uint64_t> h_seed;
  std::vector<double> h_src;
  std::vector<int64_t> ens_count;
  // after a device error: the ensembles not yet restored (the error word
  // stays set until every one is, since the steps that returned early left
  // every ensemble's particles and counters void)
  std::vector<uint8_t> restore_pending;
  // elliptic relaxation (model 1): unknowns and nonzeros of its matrix
  int32_t rx_nc = 0, rx_ellw = 0;
  int32_t rx_na = 0;           // aggregates of the projection's coarse space (0: none)
  int64_t rx_nnz = 0;
  std::string rx_err;          // why the relaxation is unavailable on this mesh
  // the solver control after each batch of replays, copied to pinned host
  // memory behind it
  relax::Ctl* rx_pin = nullptr;
  hipEvent_t rx_ev[2] = {nullptr, nullptr};
  // a split order's small cells run on a second stream beside the other
  // cells' launch (fork and join by events; created at the first such step)
  hipStream_t side = nullptr;
  hipEvent_t side_ev[2] = {nullptr, nullptr};
  // the iteration graphs of the relaxation and of the projection solves
  SolveGraphs rx_sg, px_sg;
  std::string err;
  pdf_status last = PDF_OK;
};

namespace {

int tsize_of(const pdf_params& p) { return p.f32_state ? 4 : 8; }

int nstat_of(const pdf_params& p) {
  return (p.moments >= 4 ? NSTAT4 : NSTAT2) + p.hist_bins + (p.omega ? 3 : 0) + (p.vbins == 5 ? 250 : 0);
}

int navg_of(const pdf_params& p) { return AV_HIST + p.hist_bins + (p.omega ? 2 : 0); }

// The learned conditional means run as a statistics pass and an inference
// launch before each step on persistent grids, with the turbulent frequency
// and with 8 lanes per cell (a block's cells then exceed one 16-column
// network tile); otherwise inside the step.
bool mlp_separate(const pdf_ctx* c) { return c->mlp_w && (c->persist || c->p.omega || c->group < 16); }

pdf_status fail(pdf_ctx* c, pdf_status s, const std::string& msg) {
  if (c) {
    c->err = msg;
    c->last = s;
  }
  return s;
}

// beta of the wall condition on the turbulent frequency (SLM wall functions)
double omega_beta(const pdf_params& p) {
  return -2.0 / ((((0.5 + 0.75 * p.C0) + p.C3) + p.Cw2) - p.Cw1);
}

pdf_status hip_check(pdf_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return PDF_OK;
  return fail(c, PDF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// The relaxation system's structure from the mesh (host::build_relax_structure:
// joined seam vertices, CSR rows with their element contributions, padded
// rows, incidence), copied to the arena; then the element matrices and the
// first guess (the frozen wp at each unknown's lowest vertex) on the device.
// Waits for the stream.
pdf_status relax_setup(pdf_ctx* c, const pdf_mesh* m) {
  const int32_t nv = m->nvert, ne = m->nelem;
  host::RelaxStructure S;
  const host::RelaxStatus hs =
      host::build_relax_structure(nv, ne, m->vtx, m->tri, m->nbr, m->ekind, c->p.Lx, c->p.Ly, relax::ELL_MAX,
                                  relax::AGG, S);
  // a mesh the Eulerian solves cannot take still steps particles
  if (hs != host::RELAX_OK) {
    c->rx_nc = 0;
    c->rx_err = hs == host::RELAX_LONE_VERTEX
                    ? std::string("Eulerian solves: a vertex belongs to no element")
                    : "Eulerian solves: a matrix row has more than " + std::to_string(relax::ELL_MAX) +
                          " entries (a vertex with more than " + std::to_string(relax::ELL_MAX - 1) + " neighbours)";
    return PDF_OK;
  }
  if (S.nnz > relax_nnz_bound(nv, ne)) return fail(c, PDF_E_MESH, "relaxation: more nonzeros than the layout holds");
  const int32_t nc = S.nc, ellw = S.ellw;
  const int64_t nnz = S.nnz;
  const std::vector<int32_t>&canon = S.canon, &rep = S.rep, &ecol = S.ecol, &enz = S.enz, &dpos = S.dpos,
                             &cptr = S.cptr, &cidx = S.cidx, &incptr = S.incptr, &inc = S.inc;
  const Layout& L = c->L;
  char* d = c->arena;
  hipStream_t st = c->stream;
  pdf_status r;
  auto put = [&](int64_t off, const std::vector<int32_t>& h, const char* what) {
    return hip_check(c, hipMemcpyAsync(d + off, h.data(), h.size() * 4, hipMemcpyHostToDevice, st), what);
  };
  if ((r = put(L.rx_canon, canon, "copy relaxation unknowns"))) return r;
  if ((r = put(L.rx_rep, rep, "copy relaxation unknowns"))) return r;
  if ((r = put(L.rx_ecol, ecol, "copy relaxation columns"))) return r;
  if ((r = put(L.rx_enz, enz, "copy relaxation nonzeros"))) return r;
  if ((r = put(L.rx_dpos, dpos, "copy relaxation diagonal"))) return r;
  if ((r = put(L.rx_cptr, cptr, "copy relaxation contributions"))) return r;
  if ((r = put(L.rx_cidx, cidx, "copy relaxation contributions"))) return r;
  if ((r = put(L.rx_incptr, incptr, "copy relaxation incidence"))) return r;
  if ((r = put(L.rx_inc, inc, "copy relaxation incidence"))) return r;
  // the projection's coarse space, where the mesh allows one (else its
  // preconditioner is the diagonal alone)
  host::CoarseStructure CS;
  const bool coarse = host::build_coarse(S, ne, m->vtx, m->tri, relax::AGG, relax::BLK, relax::NEED, relax::NA_MAX,
                                         CS) == host::COARSE_OK;
  // E^+ on the device, symmetric in float: per block, the rows of its need
  // list, NA_MAX wide (zero past na and past the end of the list)
  std::vector<float> epf;
  if (coarse) {
    const int32_t na = CS.na;
    const size_t nk = CS.need.size();   // blocks x NEED
    if ((int64_t)(nk * relax::NA_MAX * 4) > L.rx_eneed - L.rx_ep)   // the layout's bound on the blocks
      return fail(c, PDF_E_SIZE, "relaxation: coarse rows exceed their layout");
    epf.assign(nk * relax::NA_MAX, 0.0f);
    for (size_t k = 0; k < nk; ++k) {
      const int32_t i = CS.need[k];
      if (i < 0) continue;
      for (int32_t j = 0; j < na; ++j)
        epf[(size_t)k * relax::NA_MAX + j] = (float)(0.5 * (CS.ep[(size_t)i * na + j] + CS.ep[(size_t)j * na + i]));
    }
    if ((r = hip_check(c, hipMemcpyAsync(d + L.rx_ep, epf.data(), epf.size() * 4, hipMemcpyHostToDevice, st),
                       "copy coarse operator"))) return r;
    if ((r = put(L.rx_eneed, CS.eneed, "copy coarse need lists"))) return r;
  }
  const int tb = 256;
  hipLaunchKernelGGL(relax::k_relax_geom, dim3((ne + tb - 1) / tb), dim3(tb), 0, st, (const double*)(d + L.vtx),
                     (const int32_t*)(d + L.tri), (double*)(d + L.rx_Ke), (double*)(d + L.rx_area), ne);
  hipLaunchKernelGGL(relax::k_relax_warm, dim3((nc + tb - 1) / tb), dim3(tb), 0, st, (const double*)(d + L.fields),
                     (const int32_t*)(d + L.rx_rep), (double*)(d + L.rx_x), nc);
  if ((r = hip_check(c, hipGetLastError(), "relaxation set-up kernels"))) return r;
  // the host vectors stay alive until the copies complete
  if ((r = hip_check(c, hipStreamSynchronize(st), "sync relaxation set-up"))) return r;
  c->rx_nc = nc;
  c->rx_nnz = nnz;
  c->rx_ellw = ellw;
  c->rx_na = coarse ? CS.na : 0;
  c->rx_err.clear();
  c->rx_sg.ok = c->px_sg.ok = false;
  c->rx_sg.last_iters = c->px_sg.last_iters = 0;
  return PDF_OK;
}

// Capacity factor of segments that a repack grows: room for the count to
// double again before the next repack.
double grow_factor(double slack) { return std::max(3.0, slack + 1.0); }

// Slots beyond the seeding layout, kept for segments that grow at a repack.
// A repack gives a cell max(initial, grow (n + a) + pad) slots, a its last
// arrivals; the reserve covers that sum while the arrivals of a step stay
// under half the particles.
int64_t growth_reserve(int64_t nparticles, int64_t ncell, double slack) {
  return (int64_t)std::ceil(1.5 * grow_factor(slack) * (double)nparticles) + (int64_t)SEG_PAD * ncell;
}

int64_t slots_bound(int64_t nparticles, int64_t ncell, double slack) {
  return (int64_t)std::ceil(slack * (double)nparticles) + (int64_t)(SEG_PAD + 1) * ncell +
         growth_reserve(nparticles, ncell, slack);
}


template <typename T> StepArgs<T> step_args(pdf_ctx* c) {
  const Layout& L = c->L;
  char* a = c->arena;
  StepArgs<T> s{};
  s.erec = (const ERec*)(a + L.erec);
  s.order = (const int32_t*)(a + L.order);
  s.tri = (const int32_t*)(a + L.tri);
  s.inv2a = (const double*)(a + L.inv2a);
  s.alpha = (const double*)(a + L.alpha);
  s.wnorm = (const double*)(a + L.wnorm);
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
  s.buf[0] = state_at<T>(a, L.buf0, L.slots, L.omega);
  s.buf[1] = state_at<T>(a, L.buf1, L.slots, L.omega);
  s.ovf = state_at<T>(a, L.ovf, L.ovf_cap, L.omega);
  s.ovf_cell = (int32_t*)(a + L.ovf_cell);
  s.ovf_cap = (uint32_t)L.ovf_cap;
  s.stats = (double*)(a + L.stats);
  s.seed = (const uint64_t*)(a + L.seed);
  s.src = (const double*)(a + L.src);
  s.ctl = (Ctl*)(a + L.ctl);
  // the learned means run inside the step on one-item-per-wavefront grids
  if (c->mlp_w && !mlp_separate(c)) {
    s.mlp_w = c->mlp_w;
    s.mlp_norm = c->mlp_norm;
    s.mlp_cm = c->mlp_cm;
    s.mlp_served = c->mlp_served;
  }
  s.ncell = c->ne * c->nens;
  s.nstat = nstat_of(c->p);
  s.flags = c->p.flags;
  s.mix = c->p.mix;
  s.dt = (T)c->p.dt;
  s.sdt = (T)std::sqrt((T)c->p.dt);
  s.nu2 = (T)(2.0 * c->p.nu);
  s.s2nu = (T)std::sqrt((T)(2.0 * c->p.nu));
  if (c->p.omega) {
    s.om0 = (const double*)(a + L.om0);
    s.somega = (const double*)(a + L.somega);
    s.omw = (const double*)(a + L.omw);
    s.om_beta = omega_beta(c->p);
    s.om_yp = c->p.yp;
    s.om_nuct2 = c->p.nu * (c->p.CT * c->p.CT);
    s.om_c3 = (T)c->p.C3;
    s.om_c34 = (T)(2.0 * c->p.C3 * c->p.C4);
  }
  return s;
}

// Work items per claim of a persistent wavefront: about a sixteenth of its
// fair share, between 1 and 16.
// Work items of a one-item-per-wavefront launch over the order cells [off,
// off + n) at G lanes per cell, split into 8 contiguous ranges of equal
// estimated cost, one per XCD.  A wavefront's cost: two units for its cells'
// set-up, statistics and crossing particles, one per batch of its largest
// cell (counts at seeding; the flow keeps the particle density near its
// initial one).  Weights measured best among 1-4 units per wavefront and a
// cost proportional to the count.  A launch of at most 16384 cells keeps
// ranges of equal length, the eighths its order is sorted within.
const int32_t* xcd_ranges(pdf_ctx* c, int G, int64_t off, int64_t n) {
  const int gi = G == 64 ? 0 : (G == 32 ? 1 : (G == 16 ? 2 : (G == 8 ? 3 : 4)));
  const int part = off == 0 ? 0 : 1;
  int32_t* r = c->xcd[gi][part];
  if (c->xcd_n[gi][part] == n) return r;
  const int gpw = WAVE / G;
  const int64_t items = (n + gpw - 1) / gpw;
  r[0] = 0;
  if (n <= 16384) {
    for (int x = 1; x <= 8; ++x) r[x] = (int32_t)(items * x / 8);
    c->xcd_n[gi][part] = n;
    return r;
  }
  std::vector<double> pre((size_t)items + 1, 0.0);
  for (int64_t it = 0; it < items; ++it) {
    int32_t mx = 0;
    for (int j = 0; j < gpw; ++j) {
      const int64_t k = it * gpw + j;
      if (k < n) mx = std::max(mx, c->h_cnt[c->h_order[off + k]]);
    }
    pre[it + 1] = pre[it] + 2.0 + (double)((mx + G - 1) / G);
  }
  int64_t it = 0;
  for (int x = 1; x < 8; ++x) {
    const double target = pre[items] * x / 8.0;
    while (it < items && pre[it + 1] <= target) ++it;
    r[x] = (int32_t)std::max<int64_t>(it, r[x - 1]);
  }
  r[8] = (int32_t)items;
  c->xcd_n[gi][part] = n;
  return r;
}

// Blocks of a launch over those ranges: each XCD's blocks cover its longest
// range (the others' surplus blocks return at once).
int xcd_blocks(const int32_t* r, int wpb) {
  int m = 0;
  for (int x = 0; x < 8; ++x) m = std::max(m, r[x + 1] - r[x]);
  return 8 * std::max(1, (m + wpb - 1) / wpb);
}

int persist_chunk(int nitems, int waves) {
  waves = std::max(1, waves);
  return std::max(1, std::min(16, nitems / (16 * waves)));
}

template <typename T, int MOM, int HIST, int G, bool ADV, int SCHED, int XV>
void launch_step(pdf_ctx* c, StepArgs<T> s, StepIndex si) {
  constexpr int GPW = WAVE / G;
  constexpr int TB = step_block<SCHED>(), WPB = TB / WAVE;
  s.nitems = (s.ncell + GPW - 1) / GPW;
  int blocks = (s.nitems + WPB - 1) / WPB;
  if (SCHED != 1) {
    const int32_t* r = xcd_ranges(c, G, s.order - (const int32_t*)(c->arena + c->L.order), s.ncell);
    for (int x = 0; x < 9; ++x) s.xcd[x] = r[x];
    blocks = xcd_blocks(r, WPB);
  }
  if (SCHED == 1) {
    int per_cu = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step<T, MOM, HIST, G, ADV, SCHED, XV>, TB, 0);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    const int cap_blocks = std::max(1, per_cu) * std::max(1, cus);
    blocks = std::min(blocks, cap_blocks);
    c->persist_blocks = blocks;
  }
  s.pchunk = persist_chunk(s.nitems, blocks * WPB);
  hipLaunchKernelGGL((k_step<T, MOM, HIST, G, ADV, SCHED, XV>), dim3(blocks), dim3(TB), 0, c->stream, s, si);
}

// Scheduling variant of a step launch: persistent grid, or one work item per
// wavefront with or without the learned means inside the step.
int sched_of(const pdf_ctx* c, bool adv) {
  if (!adv) return 0;
  if (c->persist) return 1;
  return (c->mlp_w && !mlp_separate(c)) ? 2 : 0;
}

template <typename T, int MOM, int HIST, bool ADV, int XV, int G>
void launch_shape(pdf_ctx* c, const StepArgs<T>& s, StepIndex si, int sc) {
  if (!ADV || sc == 0) launch_step<T, MOM, HIST, G, ADV, 0, XV>(c, s, si);
  else if (sc == 1) launch_step<T, MOM, HIST, G, ADV, ADV ? 1 : 0, XV>(c, s, si);
  else if constexpr (XV == XV_NONE && G >= 16) launch_step<T, MOM, HIST, G, ADV, ADV ? 2 : 0, XV>(c, s, si);
}

template <typename T, int MOM, int HIST, bool ADV, int XV>
void launch_group(pdf_ctx* c, const StepArgs<T>& s, StepIndex si) {
  const int sc = sched_of(c, ADV);
  switch (c->group) {
    case 4:
      if constexpr (std::is_same<T, float>::value) launch_shape<T, MOM, HIST, ADV, XV, 4>(c, s, si, sc);
      break;
    case 8:
      if constexpr (std::is_same<T, float>::value) launch_shape<T, MOM, HIST, ADV, XV, 8>(c, s, si, sc);
      break;
    case 16: launch_shape<T, MOM, HIST, ADV, XV, 16>(c, s, si, sc); break;
    case 32: launch_shape<T, MOM, HIST, ADV, XV, 32>(c, s, si, sc); break;
    default: launch_shape<T, MOM, HIST, ADV, XV, 64>(c, s, si, sc); break;
  }
}

// The float state supports (moments, histogram) = (2, 0) and (4, 32); the
// double state (2, 0); velocity bins 2 (signs) or 5 per component.
bool supported(const pdf_params& p) {
  if (!(p.vbins == 2 || p.vbins == 5)) return false;
  // the 5 x 5 x 5 bins: float state, without the turbulent frequency
  if (p.vbins == 5 && (!p.f32_state || p.omega)) return false;
  if (p.f32_state) return (p.moments == 2 && p.hist_bins == 0) || (p.moments == 4 && p.hist_bins == 32);
  return p.moments == 2 && p.hist_bins == 0;
}

// The model extension of a context: turbulent frequency, 5 x 5 x 5 velocity
// bins (float state only), or none.
template <typename T, int MOM, int HIST, bool ADV>
void launch_ext(pdf_ctx* c, const StepArgs<T>& s, StepIndex si) {
  if (c->p.omega) {
    launch_group<T, MOM, HIST, ADV, XV_OMEGA>(c, s, si);
  } else if (c->p.vbins == 5) {
    if constexpr (std::is_same<T, float>::value) launch_group<T, MOM, HIST, ADV, XV_BINS5>(c, s, si);
  } else {
    launch_group<T, MOM, HIST, ADV, XV_NONE>(c, s, si);
  }
}

// The small cells' launch of a split order (nsplit > 0), not with a
// network attached (its means inside the step need 16 or more lanes per cell).
bool split_launch(const pdf_ctx* c) { return c->nsplit > 0 && !c->mlp_w && c->p.f32_state; }

// The side stream of a split order and its fork and join events.
pdf_status side_stream(pdf_ctx* c) {
  pdf_status r = PDF_OK;
  if (!c->side && (r = hip_check(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "side stream")))
    return r;
  for (auto& e : c->side_ev)
    if (!e && (r = hip_check(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "side event"))) return r;
  return r;
}

template <bool ADV> pdf_status dispatch_step(pdf_ctx* c, StepIndex si) {
  if (c->p.f32_state) {
    StepArgs<float> s = step_args<float>(c);
    if (ADV) s.cmean = mlp_separate(c) ? c->mlp_cm : nullptr;
    if (!ADV) s.mlp_w = nullptr;
    const bool split = split_launch(c);
    const int32_t ncell = s.ncell;
    pdf_status r;
    if (split) {
      // the small cells (at the end of the order) on the side stream, at the
      // same time as the others: the two launches touch disjoint cells, as
      // the wavefronts of one launch do
      if ((r = side_stream(c))) return r;
      if ((r = hip_check(c, hipEventRecord(c->side_ev[0], c->stream), "fork"))) return r;
      if ((r = hip_check(c, hipStreamWaitEvent(c->side, c->side_ev[0], 0), "fork"))) return r;
      StepArgs<float> sm = s;
      sm.order = s.order + c->nsplit;
      sm.ncell = ncell - (int32_t)c->nsplit;
      const int32_t g = c->group, pe = c->persist;
      hipStream_t main = c->stream;
      c->group = SMALL_GROUP;
      c->persist = 0;
      c->stream = c->side;
      if (c->p.moments == 2) launch_ext<float, 2, 0, ADV>(c, sm, si);
      else launch_ext<float, 4, 32, ADV>(c, sm, si);
      c->group = g;
      c->persist = pe;
      c->stream = main;
      if ((r = hip_check(c, hipGetLastError(), "step launch"))) return r;
      s.ncell = (int32_t)c->nsplit;
    }
    if (c->p.moments == 2) launch_ext<float, 2, 0, ADV>(c, s, si);
    else launch_ext<float, 4, 32, ADV>(c, s, si);
    if (split) {
      if ((r = hip_check(c, hipEventRecord(c->side_ev[1], c->side), "join"))) return r;
      if ((r = hip_check(c, hipStreamWaitEvent(c->stream, c->side_ev[1], 0), "join"))) return r;
    }
  } else {
    StepArgs<double> s = step_args<double>(c);
    if (ADV) s.cmean = mlp_separate(c) ? c->mlp_cm : nullptr;
    if (!ADV) s.mlp_w = nullptr;
    launch_ext<double, 2, 0, ADV>(c, s, si);
  }
  return hip_check(c, hipGetLastError(), "step launch");
}

// The learned conditional means of the current state: its statistics, then
// the network over every cell.
pdf_status enqueue_mlp_means(pdf_ctx* c, StepIndex si) {
  pdf_status r = dispatch_step<false>(c, si);
  if (r) return r;
  mlp::InferArgs ia{};
  ia.stats = (const double*)(c->arena + c->L.stats);
  ia.nstat = nstat_of(c->p);
  ia.ncell = c->ne * c->nens;
  ia.w = c->mlp_w;
  ia.norm = c->mlp_norm;
  ia.cm = c->mlp_cm;
  ia.served = c->mlp_served;
  const int tiles = (ia.ncell + mlp::TILE - 1) / mlp::TILE;
  hipLaunchKernelGGL(mlp::k_mlp_infer, dim3((tiles + mlp::MLP_WAVES - 1) / mlp::MLP_WAVES), dim3(64 * mlp::MLP_WAVES),
                     0, c->stream, ia);
  return hip_check(c, hipGetLastError(), "inference launch");
}

// Arguments of the time-average merge of one step's statistics.
struct MergeArgs {
  const double* stats;
  int nstat, hoff, hist, omega;
  double* acc;
  int navg, ncell;
};

MergeArgs merge_args(pdf_ctx* c) {
  MergeArgs m{};
  m.stats = (const double*)(c->arena + c->L.stats);
  m.nstat = nstat_of(c->p);
  m.hoff = c->p.moments >= 4 ? NSTAT4 : NSTAT2;
  m.hist = c->p.hist_bins;
  m.omega = c->p.omega;
  m.acc = c->avg;
  m.navg = navg_of(c->p);
  m.ncell = c->ne * c->nens;
  return m;
}

int merge_blocks(const MergeArgs& m) { return (m.ncell + MERGE_CELLS - 1) / MERGE_CELLS; }

pdf_status enqueue_merge(pdf_ctx* c) {
  const MergeArgs m = merge_args(c);
  hipLaunchKernelGGL(k_average_merge, dim3(merge_blocks(m)), dim3(BLOCK), 0,
                     c->stream, m.stats, m.nstat, m.hoff, m.hist, m.omega, m.acc, m.navg, m.ncell);
  return hip_check(c, hipGetLastError(), "average launch");
}

RepackPlan repack_plan_args(pdf_ctx* c, uint32_t rot) {
  const Layout& L = c->L;
  char* a = c->arena;
  RepackPlan p{};
  p.cap = (const int32_t*)(a + L.cap);
  p.cap0 = (const int32_t*)(a + L.cap0);
  p.ns = (const int32_t*)(a + L.ns[rot]);
  p.nm = (const int32_t*)(a + L.nm[rot]);
  p.nstart = (int32_t*)(a + L.nstart);
  p.ncap = (int32_t*)(a + L.ncap);
  p.ctl = (Ctl*)(a + L.ctl);
  p.ncell = c->ne * c->nens;
  p.pad = SEG_PAD;
  p.slots = L.slots;
  p.grow = grow_factor(c->p.slack);
  p.slack = c->p.slack;
  return p;
}

template <typename T> RepackMove<T> repack_move_args(pdf_ctx* c, uint32_t rot) {
  const Layout& L = c->L;
  char* a = c->arena;
  RepackMove<T> m{};
  m.buf[0] = state_at<T>(a, L.buf0, L.slots, L.omega);
  m.buf[1] = state_at<T>(a, L.buf1, L.slots, L.omega);
  m.start = (int32_t*)(a + L.start);
  m.cap = (int32_t*)(a + L.cap);
  m.ns = (int32_t*)(a + L.ns[rot]);
  m.nm = (int32_t*)(a + L.nm[rot]);
  m.nstart = (const int32_t*)(a + L.nstart);
  m.ncap = (const int32_t*)(a + L.ncap);
  m.ctl = (const Ctl*)(a + L.ctl);
  m.ncell = c->ne * c->nens;
  return m;
}

// the mover's grid: one wavefront per cell up to 2048 blocks, beyond that the
// wavefronts stride over the cells
int repack_move_blocks(const pdf_ctx* c) {
  return std::min(2048, (c->ne * c->nens + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
}

// The planner and the mover at a step boundary; both return at once unless a
// repack was requested.
pdf_status enqueue_repack(pdf_ctx* c) {
  const StepIndex si{0, c->parity, c->rot, 0};
  hipLaunchKernelGGL(k_repack_plan, dim3(1), dim3(PLAN_THREADS), 0, c->stream, repack_plan_args(c, c->rot));
  if (c->p.f32_state)
    hipLaunchKernelGGL(k_repack_move<float>, dim3(repack_move_blocks(c)), dim3(BLOCK), 0, c->stream,
                       repack_move_args<float>(c, c->rot), si);
  else
    hipLaunchKernelGGL(k_repack_move<double>, dim3(repack_move_blocks(c)), dim3(BLOCK), 0, c->stream,
                       repack_move_args<double>(c, c->rot), si);
  return hip_check(c, hipGetLastError(), "repack launch");
}

// One step's kernel, its grid and its arguments, for graph construction.
struct StepLaunch {
  const void* func = nullptr;
  int blocks = 0;
  int threads = 0;
};

template <typename T, int MOM, int HIST, int G, int SCHED, int XV>
StepLaunch step_launch_of(pdf_ctx* c, StepArgs<T>& s) {
  constexpr int GPW = WAVE / G;
  constexpr int TB = step_block<SCHED>(), WPB = TB / WAVE;
  s.nitems = (s.ncell + GPW - 1) / GPW;
  int blocks = (s.nitems + WPB - 1) / WPB;
  if (SCHED != 1) {
    const int32_t* r = xcd_ranges(c, G, s.order - (const int32_t*)(c->arena + c->L.order), s.ncell);
    for (int x = 0; x < 9; ++x) s.xcd[x] = r[x];
    blocks = xcd_blocks(r, WPB);
  }
  if (SCHED == 1) {
    int per_cu = 0, cus = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step<T, MOM, HIST, G, true, SCHED, XV>, TB, 0);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    blocks = std::min(blocks, std::max(1, per_cu) * std::max(1, cus));
  }
  s.pchunk = persist_chunk(s.nitems, blocks * WPB);
  StepLaunch l;
  l.func = reinterpret_cast<const void*>(&k_step<T, MOM, HIST, G, true, SCHED, XV>);
  l.blocks = blocks;
  l.threads = TB;
  return l;
}

template <typename T, int MOM, int HIST, int XV, int G>
StepLaunch step_launch_shape(pdf_ctx* c, StepArgs<T>& s, int sc) {
  if (sc == 1) return step_launch_of<T, MOM, HIST, G, 1, XV>(c, s);
  if constexpr (XV == XV_NONE && G >= 16) {
    if (sc == 2) return step_launch_of<T, MOM, HIST, G, 2, XV>(c, s);
  }
  return step_launch_of<T, MOM, HIST, G, 0, XV>(c, s);
}

template <typename T, int MOM, int HIST, int XV>
StepLaunch step_launch_group(pdf_ctx* c, StepArgs<T>& s) {
  const int sc = sched_of(c, true);
  switch (c->group) {
    case 4:
      if constexpr (std::is_same<T, float>::value) return step_launch_shape<T, MOM, HIST, XV, 4>(c, s, sc);
      return StepLaunch{};
    case 8:
      if constexpr (std::is_same<T, float>::value) return step_launch_shape<T, MOM, HIST, XV, 8>(c, s, sc);
      return StepLaunch{};
    case 16: return step_launch_shape<T, MOM, HIST, XV, 16>(c, s, sc);
    case 32: return step_launch_shape<T, MOM, HIST, XV, 32>(c, s, sc);
    default: return step_launch_shape<T, MOM, HIST, XV, 64>(c, s, sc);
  }
}

template <typename T, int MOM, int HIST>
StepLaunch step_launch_ext(pdf_ctx* c, StepArgs<T>& s) {
  if (c->p.omega) return step_launch_group<T, MOM, HIST, XV_OMEGA>(c, s);
  if constexpr (std::is_same<T, float>::value) {
    if (c->p.vbins == 5) return step_launch_group<T, MOM, HIST, XV_BINS5>(c, s);
  }
  return step_launch_group<T, MOM, HIST, XV_NONE>(c, s);
}

constexpr int GRAPH_STEPS = 6;  // parity repeats every 2 steps, the counter sets every 3

// Builds a graph of GRAPH_STEPS consecutive steps (and the capacity check,
// whose planner also advances the step base)
// for the current launch shape.  Nodes are added explicitly, so no stream
// capture is involved and nothing but kernel nodes is recorded.
template <typename T> pdf_status build_graph_t(pdf_ctx* c) {
  // the runtime copies kernel arguments into each node when it is added
  StepArgs<T> args_store = step_args<T>(c);
  // with a split order, a second node per step for the small cells
  const bool split = split_launch(c);
  StepArgs<T> args_small = args_store;
  StepLaunch l, ls;
  if (split) {
    args_store.ncell = (int32_t)c->nsplit;
    args_small.order = args_small.order + c->nsplit;
    args_small.ncell = args_small.ncell - (int32_t)c->nsplit;
  }
  if (c->p.moments == 2) l = step_launch_ext<T, 2, 0>(c, args_store);
  else l = step_launch_ext<T, 4, 32>(c, args_store);
  if (split) {
    const int32_t g = c->group, pe = c->persist;
    c->group = SMALL_GROUP;
    c->persist = 0;
    if (c->p.moments == 2) ls = step_launch_ext<T, 2, 0>(c, args_small);
    else ls = step_launch_ext<T, 4, 32>(c, args_small);
    c->group = g;
    c->persist = pe;
  }
  pdf_status r;
  hipGraph_t g = nullptr;
  if ((r = hip_check(c, hipGraphCreate(&g, 0), "graph create"))) return r;
  // the nodes the next one depends on (none before the first step)
  hipGraphNode_t deps[2] = {nullptr, nullptr};
  size_t ndep = 0;
  StepIndex sis[GRAPH_STEPS];
  void* params[GRAPH_STEPS][2];
  void* params_small[GRAPH_STEPS][2];
  MergeArgs margs = merge_args(c);
  void* mparams8[8] = {&margs.stats, &margs.nstat, &margs.hoff, &margs.hist, &margs.omega, &margs.acc, &margs.navg,
                       &margs.ncell};
  for (int i = 0; i < GRAPH_STEPS; ++i) {
    sis[i] = StepIndex{(uint32_t)i, (uint32_t)(i % 2), (uint32_t)(i % 3), 0};
    params[i][0] = &args_store;
    params[i][1] = &sis[i];
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(l.func);
    kp.gridDim = dim3(l.blocks);
    kp.blockDim = dim3(l.threads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = params[i];
    kp.extra = nullptr;
    hipGraphNode_t node;
    if ((r = hip_check(c, hipGraphAddKernelNode(&node, g, deps, ndep, &kp), "graph node"))) return r;
    if (split) {
      // the small cells' launch is a parallel branch of the same step: the two
      // launches touch disjoint cells, as the wavefronts of one launch do
      params_small[i][0] = &args_small;
      params_small[i][1] = &sis[i];
      hipKernelNodeParams ks = kp;
      ks.func = const_cast<void*>(ls.func);
      ks.gridDim = dim3(ls.blocks);
      ks.blockDim = dim3(ls.threads);
      ks.kernelParams = params_small[i];
      hipGraphNode_t sn;
      if ((r = hip_check(c, hipGraphAddKernelNode(&sn, g, deps, ndep, &ks), "graph node"))) return r;
      deps[1] = sn;
      ndep = 2;
    } else {
      ndep = 1;
    }
    deps[0] = node;
    if (c->avg) {
      hipKernelNodeParams km{};
      km.func = reinterpret_cast<void*>(&k_average_merge);
      km.gridDim = dim3(merge_blocks(margs));
      km.blockDim = dim3(BLOCK);
      km.kernelParams = mparams8;
      hipGraphNode_t mn;
      if ((r = hip_check(c, hipGraphAddKernelNode(&mn, g, deps, ndep, &km), "graph node"))) return r;
      deps[0] = mn;
      ndep = 1;
    }
  }
  // capacity check at the end of the cycle (parity 0, counter set 0); the
  // planner also adds the cycle's steps to the step base
  RepackPlan plan = repack_plan_args(c, 0);
  plan.advance = GRAPH_STEPS;
  void* pparams[1] = {&plan};
  hipKernelNodeParams kpl{};
  kpl.func = reinterpret_cast<void*>(&k_repack_plan);
  kpl.gridDim = dim3(1);
  kpl.blockDim = dim3(PLAN_THREADS);
  kpl.kernelParams = pparams;
  hipGraphNode_t pnode;
  if ((r = hip_check(c, hipGraphAddKernelNode(&pnode, g, deps, ndep, &kpl), "graph node"))) return r;
  RepackMove<T> mv = repack_move_args<T>(c, 0);
  StepIndex si0{0, 0, 0, 0};
  void* mparams[2] = {&mv, &si0};
  hipKernelNodeParams kmv{};
  kmv.func = reinterpret_cast<void*>(&k_repack_move<T>);
  kmv.gridDim = dim3(repack_move_blocks(c));
  kmv.blockDim = dim3(BLOCK);
  kmv.kernelParams = mparams;
  hipGraphNode_t mnode;
  if ((r = hip_check(c, hipGraphAddKernelNode(&mnode, g, &pnode, 1, &kmv), "graph node"))) return r;
  hipGraphExec_t ex = nullptr;
  if ((r = hip_check(c, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate"))) return r;
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph = g;
  c->graph_exec = ex;
  c->graph_group = c->group;
  c->graph_persist = c->persist;
  return PDF_OK;
}

// ev: null, or 2 nsteps events recorded on the stream just before and just
// after each step's kernels (the timed-step entry point)
pdf_status enqueue_steps(pdf_ctx* c, int32_t nsteps, hipEvent_t* ev = nullptr) {
  Ctl* ctl = (Ctl*)(c->arena + c->L.ctl);
  for (int32_t i = 0; i < nsteps; ++i) {
    StepIndex si{(uint32_t)i, c->parity, c->rot, 0};
    pdf_status r;
    // persistent grids (and steps with the turbulent frequency) take the
    // learned means from a separate statistics pass and inference launch; the
    // other grids compute them inside the step
    if (mlp_separate(c) && (r = enqueue_mlp_means(c, si))) return r;
    if (ev && (r = hip_check(c, hipEventRecord(ev[2 * i], c->stream), "event record"))) return r;
    if ((r = dispatch_step<true>(c, si))) return r;
    if (ev && (r = hip_check(c, hipEventRecord(ev[2 * i + 1], c->stream), "event record"))) return r;
    // the step's statistics (of the state it started from) join the time average
    if (c->avg && (r = enqueue_merge(c))) return r;
    c->parity ^= 1u;
    c->rot = c->rot == 2 ? 0 : c->rot + 1;
    // the capacity check runs every GRAPH_STEPS steps, where the graph runs it
    if ((c->steps_done + i + 1) % GRAPH_STEPS == 0 && (r = enqueue_repack(c))) return r;
  }
  hipLaunchKernelGGL(k_advance_base, dim3(1), dim3(64), 0, c->stream, ctl, (uint32_t)nsteps);
  c->steps_done += nsteps;
  return hip_check(c, hipGetLastError(), "step base launch");
}

}  // namespace

extern "C" {

pdf_status pdf_create(const pdf_params* p, void* hip_stream, pdf_ctx** out) {
  if (!p || !out) return PDF_E_ARG;
  if (!(p->moments == 2 || p->moments == 4)) return PDF_E_ARG;
  if (!(p->hist_bins == 0 || p->hist_bins == 32)) return PDF_E_ARG;
  if (!(p->dt > 0.0) || p->nu < 0.0 || !(p->slack >= 1.0)) return PDF_E_ARG;
  if (!(p->omega == 0 || p->omega == 1)) return PDF_E_ARG;
  if (p->omega && (!(p->C3 > 0.0) || !(p->C4 > 0.0) || !(((((0.5 + 0.75 * p->C0) + p->C3) + p->Cw2) - p->Cw1) > 0.0)))
    return PDF_E_ARG;
  if (!supported(*p)) return PDF_E_ARG;
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
  const Layout L = make_layout(s->nvert, s->nelem, s->nens, slots, nstat_of(c->p), tsize_of(c->p), c->p.omega != 0);
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
  Layout L = make_layout(c->nv, c->ne, 1, 1, nstat_of(c->p), tsize_of(c->p), c->p.omega != 0);
  if (L.start > arena_bytes) return fail(c, PDF_E_SIZE, "arena too small for the mesh");
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
  hipLaunchKernelGGL(k_wnorm, dim3((3 * c->ne + tb - 1) / tb), dim3(tb), 0, st, (const double*)(c->arena + L.vtx),
                     (const int32_t*)(c->arena + L.tri), (double*)(c->arena + L.wnorm), c->ne);
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
  if (c->p.omega)
    hipLaunchKernelGGL(k_omega_fields, dim3((c->ne + tb - 1) / tb), dim3(tb), 0, st, (const int32_t*)(c->arena + L.tri),
                       (const int32_t*)(c->arena + L.ekind), (const double*)(c->arena + L.fields),
                       (double*)(c->arena + L.om0), (double*)(c->arena + L.somega), (double*)(c->arena + L.omw), c->ne,
                       c->p.nu, c->p.CT, c->p.Cw1, c->p.Cw2);
  if ((r = hip_check(c, hipGetLastError(), "init kernels"))) return r;
  if ((r = relax_setup(c, m))) return r;
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
  // processing order: within windows of consecutive cells (neighbouring
  // elements), cells by decreasing particle count, so that the cells sharing
  // a wavefront have similar counts and the larger cells start first.
  // Windows of 256 keep the mesh data of a stretch of wavefronts in L2.  A
  // launch of at most 16384 cells (a few wavefronts per slot of the chip)
  // sorts each eighth of the order as a whole instead: the XCDs take equal
  // contiguous eighths (see xcd_ranges), so every XCD starts with its largest
  // cells and ends with its smallest (12 % shorter steps on a 10k-element
  // canyon than windows of 256; windows of 2048, not aligned with the
  // eighths: 6 %; larger windows on a 50k-element canyon: 1-7 % longer).
  // With the float state, when both the cells of at most SMALL_COUNT
  // particles and the others make up at least an eighth of the cells, the
  // small ones go to the end of the order and take a launch of their own at
  // SMALL_GROUP lanes per cell (the batched ensembles of very different
  // sizes); each part is ordered as above.
  c->h_order.clear();
  c->h_order.reserve(ncell);
  int64_t nsmall = 0;
  for (int64_t i = 0; i < ncell; ++i) nsmall += c->h_cnt[i] <= SMALL_COUNT ? 1 : 0;
  const bool split = c->p.f32_state && 8 * nsmall >= ncell && 8 * (ncell - nsmall) >= ncell;
  for (int part = 0; part < (split ? 2 : 1); ++part) {
    const int64_t b = (int64_t)c->h_order.size();
    for (int64_t i = 0; i < ncell; ++i)
      if (!split || (c->h_cnt[i] <= SMALL_COUNT) == (part == 1)) c->h_order.push_back((int32_t)i);
    const int64_t e = (int64_t)c->h_order.size();
    auto sort_window = [&](int64_t w0, int64_t w1) {
      std::stable_sort(c->h_order.begin() + w0, c->h_order.begin() + w1,
                       [&](int32_t x, int32_t y) { return c->h_cnt[x] > c->h_cnt[y]; });
    };
    if (ncell <= 16384) {
      for (int x = 0; x < 8; ++x) sort_window(b + (e - b) * x / 8, b + (e - b) * (x + 1) / 8);
    } else {
      for (int64_t w0 = b; w0 < e; w0 += 256) sort_window(w0, std::min<int64_t>(e, w0 + 256));
      // and the last fifth of each XCD's range (cut as xcd_ranges cuts them
      // at 64 lanes per cell) largest-first, so that the XCDs end with their
      // smallest cells: 1.5 % shorter steps on a 50k-element canyon (a third
      // or all of the range: less)
      std::vector<double> pre((size_t)(e - b) + 1, 0.0);
      for (int64_t k = b; k < e; ++k)
        pre[k - b + 1] = pre[k - b] + 2.0 + (double)((c->h_cnt[c->h_order[k]] + WAVE - 1) / WAVE);
      int64_t it = 0, prev = 0;
      for (int x = 1; x <= 8; ++x) {
        int64_t bx = e - b;
        if (x < 8) {
          const double target = pre[e - b] * x / 8.0;
          while (it < e - b && pre[it + 1] <= target) ++it;
          bx = std::max(it, prev);
        }
        const int64_t tail = (bx - prev) / 5;
        if (tail > 1) sort_window(b + bx - tail, b + bx);
        prev = bx;
      }
    }
  }
  c->nsplit = split ? ncell - nsmall : 0;
  for (int gi = 0; gi < 5; ++gi) c->xcd_n[gi][0] = c->xcd_n[gi][1] = -1;
  const int64_t slots = slot + growth_reserve(total, ncell, slack);
  const Layout L = make_layout(c->nv, c->ne, nens, slots, nstat_of(c->p), tsize_of(c->p), c->p.omega != 0);
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
  if ((r = hip_check(c, hipMemcpyAsync(a + L.cap0, c->h_cap.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy cap"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(a + L.ns[0], c->h_cnt.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy counts"))) return r;
  for (int rr = 0; rr < 3; ++rr) {
    if (rr > 0 && (r = hip_check(c, hipMemcpyAsync(a + L.ns[rr], c->h_zero.data(), ncell * 4, hipMemcpyHostToDevice, st), "clear counts"))) return r;
    if ((r = hip_check(c, hipMemcpyAsync(a + L.nm[rr], c->h_zero.data(), ncell * 4, hipMemcpyHostToDevice, st), "clear counts"))) return r;
  }
  if ((r = hip_check(c, hipMemcpyAsync(a + L.idoff, c->h_idoff.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy idoff"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(a + L.order, c->h_order.data(), ncell * 4, hipMemcpyHostToDevice, st), "copy order"))) return r;
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
                       (const int32_t*)(a + L.idoff), s.seed, c->ne, (int)ncell, c->p.psi_init,
                       (const double*)(a + L.om0));
  } else {
    StepArgs<double> s = step_args<double>(c);
    hipLaunchKernelGGL(k_rate<double>, dim3((unsigned)((ncell + tb - 1) / tb)), dim3(tb), 0, st, (const double*)(a + L.vtx), s.tri,
                       (const double*)(a + L.fields), s.src, (double*)(a + L.rate), c->ne, (int)ncell, c->p.dt,
                       c->p.nu, c->p.CT, c->p.Cs, c->p.Ct);
    hipLaunchKernelGGL(k_seed<double>, dim3(cb), dim3(BLOCK), 0, st, s.erec, s.tri, s.inv2a,
                       (const double*)(a + L.fields), s.buf[0], s.start, (const int32_t*)s.ns[0],
                       (const int32_t*)(a + L.idoff), s.seed, c->ne, (int)ncell, c->p.psi_init,
                       (const double*)(a + L.om0));
  }
  if ((r = hip_check(c, hipGetLastError(), "seed kernels"))) return r;
  // the host vectors stay alive in the context until the copies complete
  if ((r = hip_check(c, hipStreamSynchronize(st), "sync seed"))) return r;
  c->seeded = true;
  c->restore_pending.clear();
  c->graph_group = 0;  // a graph built for an earlier layout is stale
  c->steps_done = 0;
  c->proj_mark = 0;
  c->parity = 0;
  c->rot = 0;
  c->last = PDF_OK;
  c->err.clear();
  return PDF_OK;
}

pdf_status pdf_step(pdf_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return fail(c, PDF_E_ARG, "pdf_step: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_step before pdf_seed_particles");
  if (nsteps == 0) return PDF_OK;
  return enqueue_steps(c, nsteps);
}

pdf_status pdf_step_timed(pdf_ctx* c, int32_t nsteps, double* kernel_ms) {
  if (!c || nsteps < 0 || !kernel_ms) return fail(c, PDF_E_ARG, "pdf_step_timed: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_step_timed before pdf_seed_particles");
  *kernel_ms = 0.0;
  if (nsteps == 0) return PDF_OK;
  std::vector<hipEvent_t> ev((size_t)2 * nsteps, nullptr);
  pdf_status r = PDF_OK;
  for (auto& e : ev)
    if ((r = hip_check(c, hipEventCreate(&e), "event create"))) break;
  if (!r) r = enqueue_steps(c, nsteps, ev.data());
  if (!r) r = hip_check(c, hipStreamSynchronize(c->stream), "sync timed steps");
  double tot = 0.0;
  for (int32_t i = 0; !r && i < nsteps; ++i) {
    float ms = 0.0f;
    r = hip_check(c, hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]), "event time");
    tot += ms;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (!r) *kernel_ms = tot;
  return r;
}

pdf_status pdf_step_graph(pdf_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return fail(c, PDF_E_ARG, "pdf_step_graph: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_step_graph before pdf_seed_particles");
  pdf_status r;
  // with the learned conditional means as a separate pass every step is
  // launched directly
  if (mlp_separate(c)) return enqueue_steps(c, nsteps);
  // align to the start of a parity / counter-set cycle with ordinary launches
  int32_t lead = (int32_t)((GRAPH_STEPS - c->steps_done % GRAPH_STEPS) % GRAPH_STEPS);
  lead = std::min(lead, nsteps);
  if (lead > 0 && (r = enqueue_steps(c, lead))) return r;
  int32_t left = nsteps - lead;
  if (left >= GRAPH_STEPS) {
    if (!c->graph_exec || c->graph_group != c->group || c->graph_persist != c->persist) {
      r = c->p.f32_state ? build_graph_t<float>(c) : build_graph_t<double>(c);
      if (r) return r;
    }
    while (left >= GRAPH_STEPS) {
      if ((r = hip_check(c, hipGraphLaunch(c->graph_exec, c->stream), "graph launch"))) return r;
      c->steps_done += GRAPH_STEPS;
      left -= GRAPH_STEPS;
    }
  }
  if (left > 0 && (r = enqueue_steps(c, left))) return r;
  return PDF_OK;
}

pdf_status pdf_autotune(pdf_ctx* c, int32_t steps_per_trial, int32_t* group, int32_t* persist) {
  if (!c || steps_per_trial <= 0) return fail(c, PDF_E_ARG, "pdf_autotune: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_autotune before pdf_seed_particles");
  const int groups[4] = {64, 32, 16, 8};
  // two rounds over the candidates, the second in reverse order, each
  // candidate scored by its faster trial: the state drifts as the trials
  // advance it (cells fill, a repack may fall into one trial)
  float score[8];
  for (int i = 0; i < 8; ++i) score[i] = 1e30f;
  hipEvent_t e0, e1;
  pdf_status r;
  if ((r = hip_check(c, hipEventCreate(&e0), "event"))) return r;
  if ((r = hip_check(c, hipEventCreate(&e1), "event"))) {
    (void)hipEventDestroy(e0);
    return r;
  }
  for (int round = 0; round < 2; ++round) {
    for (int t = 0; t < 8; ++t) {
      const int i = round == 0 ? t : 7 - t;
      const int gi = i / 2, pe = i % 2;
      if (!c->p.f32_state && groups[gi] != 64) continue;
      c->group = groups[gi];
      c->persist = pe;
      // one untimed step with this shape, then the timed trial
      r = enqueue_steps(c, 1);
      if (!r) {
        (void)hipEventRecord(e0, c->stream);
        r = enqueue_steps(c, steps_per_trial);
      }
      if (!r) {
        (void)hipEventRecord(e1, c->stream);
        r = hip_check(c, hipEventSynchronize(e1), "autotune sync");
      }
      if (r) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return r;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      score[i] = std::min(score[i], ms);
    }
  }
  int bg = 64, bp = 0;
  float best = 1e30f;
  for (int i = 0; i < 8; ++i) {
    if (score[i] < best) {
      best = score[i];
      bg = groups[i / 2];
      bp = i % 2;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->group = bg;
  c->persist = bp;
  if (group) *group = bg;
  if (persist) *persist = bp;
  return PDF_OK;
}

pdf_status pdf_set_launch(pdf_ctx* c, int32_t group, int32_t persist) {
  if (!c || !(group == 8 || group == 16 || group == 32 || group == 64) || persist < 0 || persist > 1)
    return fail(c, PDF_E_ARG, "pdf_set_launch: group must be 8, 16, 32 or 64, persist 0 or 1");
  if (!c->p.f32_state && group != 64) return fail(c, PDF_E_ARG, "pdf_set_launch: double state runs with group 64");
  c->group = group;
  c->persist = persist;
  return PDF_OK;
}

pdf_status pdf_repack(pdf_ctx* c) {
  if (!c) return PDF_E_ARG;
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_repack before pdf_seed_particles");
  hipLaunchKernelGGL(k_request_repack, dim3(1), dim3(64), 0, c->stream, (Ctl*)(c->arena + c->L.ctl));
  pdf_status r = hip_check(c, hipGetLastError(), "repack request");
  if (r) return r;
  return enqueue_repack(c);
}

int64_t pdf_repack_count(pdf_ctx* c) {
  if (!c || !c->seeded) return -1;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
  Ctl h{};
  if (hipMemcpy(&h, c->arena + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return (int64_t)h.repacks;
}

pdf_status pdf_metrics(pdf_ctx* c, int64_t* out) {
  if (!c || !out) return fail(c, PDF_E_ARG, "pdf_metrics: null output");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_metrics before pdf_seed_particles");
  char* a = c->arena;
  int64_t* m = (int64_t*)(a + c->L.metrics);
  hipLaunchKernelGGL(k_metrics, dim3(1), dim3(METRIC_THREADS), 0, c->stream, (const int32_t*)(a + c->L.ns[c->rot]),
                     (const int32_t*)(a + c->L.nm[c->rot]), (const int32_t*)(a + c->L.cap), c->ne * c->nens, m);
  pdf_status r;
  if ((r = hip_check(c, hipGetLastError(), "metrics launch"))) return r;
  int64_t h[5];
  Ctl ctl{};
  if ((r = hip_check(c, hipMemcpyAsync(h, m, sizeof(h), hipMemcpyDeviceToHost, c->stream), "copy metrics"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(&ctl, a + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream), "copy control"))) return r;
  if ((r = hip_check(c, hipStreamSynchronize(c->stream), "sync metrics"))) return r;
  for (int i = 0; i < 5; ++i) out[i] = h[i];
  out[5] = ctl.repacks;
  out[6] = ctl.error;
  out[7] = c->steps_done;
  return PDF_OK;
}

int32_t pdf_nstat(const pdf_ctx* c) { return c ? nstat_of(c->p) : 0; }

pdf_status pdf_estimate_statistics(pdf_ctx* c, double* out, int32_t out_on_host) {
  if (!c || !out) return fail(c, PDF_E_ARG, "pdf_estimate_statistics: null output");
  if (!c->seeded) return fail(c, PDF_E_STATE, "statistics before seeding");
  pdf_status r = dispatch_step<false>(c, StepIndex{0, c->parity, c->rot, 0});
  if (r) return r;
  const size_t bytes = (size_t)c->nens * c->ne * nstat_of(c->p) * 8;
  if ((r = hip_check(c, hipMemcpyAsync(out, c->arena + c->L.stats, bytes,
                                       out_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream),
                     "copy statistics")))
    return r;
  if (out_on_host) return hip_check(c, hipStreamSynchronize(c->stream), "sync statistics");
  return PDF_OK;
}

// Kernel arguments of the relaxation solve, statistics of ensemble 0.
static relax::Args relax_args(pdf_ctx* c) {
  const Layout& L = c->L;
  char* d = c->arena;
  relax::Args a{};
  a.ne = c->ne;
  a.nv = c->nv;
  a.nc = c->rx_nc;
  a.nbx = relax_blocks(c->rx_nc);
  a.ellw = c->rx_ellw;
  a.tri = (const int32_t*)(d + L.tri);
  a.vtx = (const double*)(d + L.vtx);
  a.fields = (const double*)(d + L.fields);
  a.fields_rw = (double*)(d + L.fields);
  a.canon = (const int32_t*)(d + L.rx_canon);
  a.ecol = (const int32_t*)(d + L.rx_ecol);
  a.enz = (const int32_t*)(d + L.rx_enz);
  a.dpos = (const int32_t*)(d + L.rx_dpos);
  a.cptr = (const int32_t*)(d + L.rx_cptr);
  a.cidx = (const int32_t*)(d + L.rx_cidx);
  a.incptr = (const int32_t*)(d + L.rx_incptr);
  a.inc = (const int32_t*)(d + L.rx_inc);
  a.Ke = (const double*)(d + L.rx_Ke);
  a.area = (const double*)(d + L.rx_area);
  a.stats = (const double*)(d + L.stats);
  a.nstat = nstat_of(c->p);
  a.nu = c->p.nu;
  a.mass = 1.0;
  a.rhs_mode = 0;
  a.dt = c->p.dt;
  a.S = (double*)(d + L.rx_S);
  a.L2 = (double*)(d + L.rx_L2);
  a.Rk = (double*)(d + L.rx_Rk);
  a.aval = (double*)(d + L.rx_aval);
  a.dinv = (double*)(d + L.rx_dinv);
  a.x = (double*)(d + L.rx_x);
  a.p = (double*)(d + L.rx_p);
  for (int b = 0; b < 2; ++b) a.rec[b] = (relax::Rec*)(d + L.rx_rec[b]);
  a.part[0] = (double*)(d + L.rx_part[0]);
  a.part[1] = (double*)(d + L.rx_part[1]);
  a.pbb = (double*)(d + L.rx_pbb);
  a.ctl = (relax::Ctl*)(d + L.rx_ctl);
  a.na = 0;   // the projection sets its coarse space
  a.ep = (const float*)(d + L.rx_ep);
  a.eneed = (const int32_t*)(d + L.rx_eneed);
  for (int b = 0; b < 2; ++b) {
    a.agp[b] = (double*)(d + L.rx_agp[b]);
    a.cglob[b] = (double*)(d + L.rx_cglob[b]);
  }
  return a;
}

// The graphs of RELAX_LONG and RELAX_SHORT iteration launches of a solve
// (kernel nodes only; every launch after the stop returns at once): the
// relaxation's five components, or the projection's one.
static pdf_status build_solve_graphs(pdf_ctx* c, const relax::Args& a, SolveGraphs& sg, bool proj) {
  if (sg.ok) return PDF_OK;
  static_assert(RELAX_LONG % 2 == 0 && RELAX_SHORT % 2 == 0, "iteration parity continues across replays");
  sg.release();
  pdf_status r;
  for (int gi = 0; gi < 2; ++gi) {
    hipGraph_t g = nullptr;
    if ((r = hip_check(c, hipGraphCreate(&g, 0), "solver graph create"))) return r;
    relax::Args store = a;   // kernel parameters are copied into the nodes at creation
    int32_t pars[2] = {0, 1};
    hipGraphNode_t prev = nullptr;
    const int n = gi == 0 ? RELAX_LONG : RELAX_SHORT;
    for (int i = 0; i < n; ++i) {
      void* params[2] = {&store, &pars[i & 1]};
      hipKernelNodeParams kp{};
      kp.func = const_cast<void*>(proj ? relax::proj_iter_kernel(a.ellw) : relax::relax_iter_kernel(a.ellw));
      kp.gridDim = dim3((unsigned)a.nbx, proj ? 1 : relax::NC);
      kp.blockDim = dim3(relax::BLK);
      kp.sharedMemBytes = 0;
      kp.kernelParams = params;
      kp.extra = nullptr;
      hipGraphNode_t node;
      if ((r = hip_check(c, hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp),
                         "solver graph node"))) {
        (void)hipGraphDestroy(g);
        return r;
      }
      prev = node;
    }
    hipGraphExec_t ex = nullptr;
    if ((r = hip_check(c, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "solver graph instantiate"))) {
      (void)hipGraphDestroy(g);
      return r;
    }
    sg.g[gi] = g;
    sg.ex[gi] = ex;
  }
  sg.ok = true;
  return PDF_OK;
}

// The iterations of a solve whose start kernels are enqueued, in graph
// replays until the device reports the stop (launch i checks the stop after
// i iterations, so up to max_iters + 1 launches run; launches after the stop
// return at once).  The first batch covers the iteration count of the last
// run; finish(again) enqueues the kernels that use the solution, then a copy
// of the solver control into pinned host memory follows, and the host waits
// once.  If the solve has not stopped, batches of RELAX_SHORT follow, each
// with its control copy and event, the next one enqueued before the host
// waits for the previous one, and finish(true) runs again.  *out: the
// control at the end (pinned host memory of the context).
static pdf_status run_solve(pdf_ctx* c, const relax::Args& a, SolveGraphs& sg, bool proj, int32_t max_iters,
                            const std::function<pdf_status(bool)>& finish, const relax::Ctl** out) {
  pdf_status r;
  if ((r = build_solve_graphs(c, a, sg, proj))) return r;
  hipStream_t st = c->stream;
  if (!c->rx_pin) {
    if ((r = hip_check(c, hipHostMalloc((void**)&c->rx_pin, 2 * sizeof(relax::Ctl), hipHostMallocDefault), "pinned control"))) return r;
    for (auto& e : c->rx_ev)
      if ((r = hip_check(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "solver event"))) return r;
  }
  int32_t launched = 0;
  auto replay = [&](int gi) -> pdf_status {
    launched += gi == 0 ? RELAX_LONG : RELAX_SHORT;
    return hip_check(c, hipGraphLaunch(sg.ex[gi], st), "solver graph launch");
  };
  auto mark = [&](int slot) -> pdf_status {
    pdf_status q;
    if ((q = hip_check(c, hipMemcpyAsync(c->rx_pin + slot, a.ctl, sizeof(relax::Ctl), hipMemcpyDeviceToHost, st), "read solver control"))) return q;
    return hip_check(c, hipEventRecord(c->rx_ev[slot], st), "solver event");
  };
  const int32_t first = std::max(1, std::min(sg.last_iters, max_iters) + 1);
  while (launched + RELAX_LONG <= first)
    if ((r = replay(0))) return r;
  while (launched < first)
    if ((r = replay(1))) return r;
  int slot = 0;
  if ((r = finish(false)) || (r = mark(slot))) return r;
  if ((r = hip_check(c, hipEventSynchronize(c->rx_ev[slot]), "sync solver"))) return r;
  if (!c->rx_pin[slot].done && launched <= max_iters) {
    if ((r = replay(1)) || (r = mark(slot))) return r;
    for (;;) {
      const bool more = launched <= max_iters;
      if (more && ((r = replay(1)) || (r = mark(slot ^ 1)))) return r;
      if ((r = hip_check(c, hipEventSynchronize(c->rx_ev[slot]), "sync solver"))) return r;
      if (c->rx_pin[slot].done || !more) break;
      slot ^= 1;
    }
    if ((r = finish(true)) || (r = mark(slot))) return r;
    if ((r = hip_check(c, hipEventSynchronize(c->rx_ev[slot]), "sync solver"))) return r;
  }
  sg.last_iters = c->rx_pin[slot].iter;
  *out = c->rx_pin + slot;
  return PDF_OK;
}

static void report_solve(const relax::Ctl& h, int32_t* info, double* resid, int32_t extra) {
  if (info) {
    info[0] = h.iter;
    info[1] = h.converged;
    info[2] = extra;
    info[3] = h.from_stats;
  }
  if (resid)
    for (int q = 0; q < relax::NC; ++q) resid[q] = h.ref[q] > 0.0 ? std::sqrt(h.rho[q] / h.ref[q]) : 0.0;
}

pdf_status pdf_elliptic_relaxation(pdf_ctx* c, int32_t max_iters, double tol, double* wp, double* coef,
                                   int32_t* info, double* resid) {
  if (!c || max_iters < 1 || max_iters > RELAX_MAX_ITERS || !(tol > 0.0) || !(tol < 1.0))
    return fail(c, PDF_E_ARG, "pdf_elliptic_relaxation: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_elliptic_relaxation before pdf_seed_particles");
  if (c->p.model != 1) return fail(c, PDF_E_STATE, "pdf_elliptic_relaxation: the context uses the SLM (model 0)");
  if (c->rx_nc == 0) return fail(c, PDF_E_MESH, c->rx_err);
  // the statistics of the current state
  pdf_status r = dispatch_step<false>(c, StepIndex{0, c->parity, c->rot, 0});
  if (r) return r;
  const relax::Args a = relax_args(c);
  hipStream_t st = c->stream;
  const int tb = relax::BLK;
  const unsigned eb = (unsigned)((c->ne + tb - 1) / tb), vb = (unsigned)((c->nv + tb - 1) / tb);
  const unsigned zb = (unsigned)(((int64_t)c->rx_ellw * c->rx_nc + tb - 1) / tb);
  const dim3 grid((unsigned)a.nbx, relax::NC);
  hipLaunchKernelGGL(relax::k_relax_reset, dim3(1), dim3(64), 0, st, a.ctl, max_iters, tol * tol);
  hipLaunchKernelGGL(relax::k_relax_inputs, dim3(eb), dim3(tb), 0, st, a);
  hipLaunchKernelGGL(relax::k_relax_matrix, dim3(zb), dim3(tb), 0, st, a);
  hipLaunchKernelGGL(relax::k_relax_start1, grid, dim3(tb), 0, st, a);
  hipLaunchKernelGGL(relax::k_relax_start2, grid, dim3(tb), 0, st, a);
  if ((r = hip_check(c, hipGetLastError(), "relaxation launch"))) return r;
  // G and C0 from the solution; run again after further iterations (the
  // count of clamped C0 anew)
  auto update = [&](bool again) -> pdf_status {
    if (again) hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, &a.ctl->clamped, 0, (int64_t)1);
    if (c->p.f32_state)
      hipLaunchKernelGGL(relax::k_relax_coef<float>, dim3(vb), dim3(tb), 0, st, a, (float*)(c->arena + c->L.coef), wp, coef);
    else
      hipLaunchKernelGGL(relax::k_relax_coef<double>, dim3(vb), dim3(tb), 0, st, a, (double*)(c->arena + c->L.coef), wp, coef);
    return hip_check(c, hipGetLastError(), "relaxation launch");
  };
  const relax::Ctl* h = nullptr;
  if ((r = run_solve(c, a, c->rx_sg, false, max_iters, update, &h))) return r;
  report_solve(*h, info, resid, h->clamped);
  return PDF_OK;
}

pdf_status pdf_pressure_projection(pdf_ctx* c, int32_t max_iters, double tol, double* phi, double* grad,
                                   int32_t* info, double* resid) {
  if (!c || max_iters < 1 || max_iters > RELAX_MAX_ITERS || !(tol > 0.0) || !(tol < 1.0))
    return fail(c, PDF_E_ARG, "pdf_pressure_projection: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_pressure_projection before pdf_seed_particles");
  if (c->nens != 1) return fail(c, PDF_E_STATE, "pdf_pressure_projection: one ensemble only");
  if (c->rx_nc == 0) return fail(c, PDF_E_MESH, c->rx_err);
  pdf_status r = dispatch_step<false>(c, StepIndex{0, c->parity, c->rot, 0});
  if (r) return r;
  relax::Args a = relax_args(c);
  a.x = (double*)(c->arena + c->L.rx_px);
  a.mass = 0.0;
  a.rhs_mode = 1;
  a.na = c->rx_na;
  // the span the correction covers: the steps since the last applied
  // projection (at least one)
  const int64_t span = std::max<int64_t>(1, c->steps_done - c->proj_mark);
  a.dt = (double)span * c->p.dt;
  hipStream_t st = c->stream;
  const int tb = relax::BLK;
  const unsigned eb = (unsigned)((c->ne + tb - 1) / tb), vb = (unsigned)((c->nv + tb - 1) / tb);
  const unsigned zb = (unsigned)(((int64_t)c->rx_ellw * c->rx_nc + tb - 1) / tb);
  const int64_t xwords = 2 * (int64_t)relax::NC * c->rx_nc;
  hipLaunchKernelGGL(relax::k_relax_reset, dim3(1), dim3(64), 0, st, a.ctl, max_iters, tol * tol);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((xwords + 255) / 256)), dim3(256), 0, st, (int32_t*)a.x, 0, xwords);
  hipLaunchKernelGGL(relax::k_proj_inputs, dim3(eb), dim3(tb), 0, st, a);
  hipLaunchKernelGGL(relax::k_relax_matrix, dim3(zb), dim3(tb), 0, st, a);
  hipLaunchKernelGGL(relax::k_proj_start1, dim3((unsigned)a.nbx), dim3(tb), 0, st, a);
  hipLaunchKernelGGL(relax::k_proj_center, dim3((unsigned)a.nbx), dim3(tb), 0, st, a);
  hipLaunchKernelGGL(relax::k_proj_start2, dim3((unsigned)a.nbx), dim3(tb), 0, st, a);
  if ((r = hip_check(c, hipGetLastError(), "projection launch"))) return r;
  // the update, once the solve has stopped (the kernels check the device's
  // stop and applied flags, so a launch behind an unfinished batch does nothing)
  char* d = c->arena;
  const Layout& L = c->L;
  CounterSets cs;
  for (int q = 0; q < 3; ++q) {
    cs.ns[q] = (int32_t*)(d + L.ns[q]);
    cs.nm[q] = (int32_t*)(d + L.nm[q]);
  }
  const StepIndex si{0, c->parity, c->rot, 0};
  const unsigned pb = (unsigned)((c->ne + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
  auto apply = [&](bool) -> pdf_status {
    hipLaunchKernelGGL(relax::k_proj_grad, dim3(eb), dim3(tb), 0, st, a);
    if (c->p.f32_state) {
      hipLaunchKernelGGL(relax::k_proj_apply<float>, dim3(vb), dim3(tb), 0, st, a, (float*)(d + L.coef), phi, grad);
      hipLaunchKernelGGL(relax::k_proj_particles<float>, dim3(pb), dim3(BLOCK), 0, st, a,
                         state_at<float>(d, L.buf0, L.slots, L.omega), state_at<float>(d, L.buf1, L.slots, L.omega), cs,
                         (const int32_t*)(d + L.start), (const int32_t*)(d + L.cap), (const Ctl*)(d + L.ctl), si);
    } else {
      hipLaunchKernelGGL(relax::k_proj_apply<double>, dim3(vb), dim3(tb), 0, st, a, (double*)(d + L.coef), phi, grad);
      hipLaunchKernelGGL(relax::k_proj_particles<double>, dim3(pb), dim3(BLOCK), 0, st, a,
                         state_at<double>(d, L.buf0, L.slots, L.omega), state_at<double>(d, L.buf1, L.slots, L.omega), cs,
                         (const int32_t*)(d + L.start), (const int32_t*)(d + L.cap), (const Ctl*)(d + L.ctl), si);
    }
    hipLaunchKernelGGL(relax::k_proj_done, dim3(1), dim3(64), 0, st, a.ctl);
    return hip_check(c, hipGetLastError(), "projection launch");
  };
  const relax::Ctl* h = nullptr;
  if ((r = run_solve(c, a, c->px_sg, true, max_iters, apply, &h))) return r;
  if (h->applied) c->proj_mark = c->steps_done;
  report_solve(*h, info, resid, h->applied);
  return PDF_OK;
}

pdf_status pdf_relaxation_size(const pdf_ctx* c, int64_t* out) {
  if (!c || !out) return PDF_E_ARG;
  if (!c->mesh_ready) return PDF_E_STATE;
  if (c->rx_nc == 0) return PDF_E_MESH;
  out[0] = c->rx_nc;
  out[1] = c->rx_nnz;
  out[2] = c->rx_ellw;
  out[3] = c->rx_na;
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
  if (h.error & (ERR_CAPACITY | ERR_OVERFLOW_FULL)) {
    // name the first overflowing cell: its capacity and counter sets
    std::string msg = "an element segment overflowed its capacity";
    int32_t cell = -1;
    if (h.ovf > 0 && hipMemcpy(&cell, c->arena + c->L.ovf_cell, 4, hipMemcpyDeviceToHost) == hipSuccess &&
        cell >= 0 && cell < c->ne * c->nens) {
      int32_t v[6] = {0, 0, 0, 0, 0, 0};
      int32_t capd = 0;
      (void)hipMemcpy(&capd, c->arena + c->L.cap + 4 * (int64_t)cell, 4, hipMemcpyDeviceToHost);
      for (int rr = 0; rr < 3; ++rr) {
        (void)hipMemcpy(&v[rr], c->arena + c->L.ns[rr] + 4 * (int64_t)cell, 4, hipMemcpyDeviceToHost);
        (void)hipMemcpy(&v[3 + rr], c->arena + c->L.nm[rr] + 4 * (int64_t)cell, 4, hipMemcpyDeviceToHost);
      }
      msg += " (" + std::to_string(h.ovf) + " particles; first cell " + std::to_string(cell) + ", capacity " +
             std::to_string(capd) + ", initial count " + std::to_string(c->h_cnt[cell]) +
             ", counter sets ns " + std::to_string(v[0]) + "/" + std::to_string(v[1]) + "/" + std::to_string(v[2]) +
             " nm " + std::to_string(v[3]) + "/" + std::to_string(v[4]) + "/" + std::to_string(v[5]) +
             ", current set " + std::to_string(c->rot) + ", repacks " + std::to_string(h.repacks) + ")";
    }
    return fail(c, PDF_E_CAPACITY, msg);
  }
  return PDF_OK;
}

// State of one ensemble in id order; om (may be null) receives the turbulent
// frequency.
static pdf_status gather_state(pdf_ctx* c, int32_t ens, double* xyuvwpsi, int32_t* elem, double* om) {
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
    hipLaunchKernelGGL(k_gather<float>, dim3(blocks), dim3(BLOCK), 0, c->stream, state_at<float>(a, L.buf0, L.slots, L.omega),
                       state_at<float>(a, L.buf1, L.slots, L.omega), cs, (const int32_t*)(a + L.start),
                       (const int32_t*)(a + L.cap), (const Ctl*)(a + L.ctl), StepIndex{0, c->parity, c->rot, 0}, ens, c->ne, n, xyuvwpsi,
                       elem, om);
  else
    hipLaunchKernelGGL(k_gather<double>, dim3(blocks), dim3(BLOCK), 0, c->stream, state_at<double>(a, L.buf0, L.slots, L.omega),
                       state_at<double>(a, L.buf1, L.slots, L.omega), cs, (const int32_t*)(a + L.start),
                       (const int32_t*)(a + L.cap), (const Ctl*)(a + L.ctl), StepIndex{0, c->parity, c->rot, 0}, ens, c->ne, n, xyuvwpsi,
                       elem, om);
  return hip_check(c, hipGetLastError(), "gather launch");
}

pdf_status pdf_set_state(pdf_ctx* c, int32_t ens, const double* xyuvwpsi, const int32_t* elem, const double* om) {
  if (!c || !xyuvwpsi || !elem) return fail(c, PDF_E_ARG, "pdf_set_state: null input");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_set_state before pdf_seed_particles");
  if (ens < 0 || ens >= c->nens) return fail(c, PDF_E_ARG, "ensemble out of range");
  if (c->p.omega && !om) return fail(c, PDF_E_ARG, "pdf_set_state: the context carries the turbulent frequency");
  const int64_t n = c->ens_count[ens];
  char* a = c->arena;
  const Layout& L = c->L;
  const int ne = c->ne;
  const uint32_t rz = c->rot == 0 ? 2u : c->rot - 1u;   // counter set not read by the next step
  int32_t* scratch = (int32_t*)(a + L.ns[rz]);
  int32_t* flag = (int32_t*)(a + L.flag) + 1;
  hipStream_t st = c->stream;
  const int tb = 256;
  const unsigned pb = (unsigned)std::max<int64_t>(1, (n + tb - 1) / tb), eb = (unsigned)((ne + tb - 1) / tb);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, flag, 0, (int64_t)1);
  hipLaunchKernelGGL(k_fill_i32, dim3(eb), dim3(tb), 0, st, scratch + (size_t)ens * ne, 0, (int64_t)ne);
  hipLaunchKernelGGL(k_set_count, dim3(pb), dim3(tb), 0, st, elem, n, ne, ens, scratch, flag);
  hipLaunchKernelGGL(k_set_check, dim3(eb), dim3(tb), 0, st, scratch, (const int32_t*)(a + L.cap), ne, ens, flag);
  pdf_status r;
  if ((r = hip_check(c, hipGetLastError(), "set-state launch"))) return r;
  int32_t bad = 0;
  if ((r = hip_check(c, hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st), "read flag"))) return r;
  if ((r = hip_check(c, hipStreamSynchronize(st), "sync set-state"))) return r;
  if (bad) {
    hipLaunchKernelGGL(k_fill_i32, dim3(eb), dim3(tb), 0, st, scratch + (size_t)ens * ne, 0, (int64_t)ne);
    (void)hipStreamSynchronize(st);
    if (bad & 1) return fail(c, PDF_E_ARG, "pdf_set_state: element index out of range (state unchanged)");
    return fail(c, PDF_E_CAPACITY, "pdf_set_state: an element segment cannot hold its particles (state unchanged)");
  }
  // a device error since the last restore: every ensemble must be restored
  // before the error word clears
  Ctl hctl{};
  if ((r = hip_check(c, hipMemcpy(&hctl, a + L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost), "read control"))) return r;
  if (hctl.error != 0 && c->restore_pending.empty()) c->restore_pending.assign(c->nens, 1);
  if (!c->restore_pending.empty()) c->restore_pending[ens] = 0;
  const bool all_restored =
      std::find(c->restore_pending.begin(), c->restore_pending.end(), (uint8_t)1) == c->restore_pending.end();
  if (all_restored) c->restore_pending.clear();
  // the other counter sets of the ensemble start from zero: the next step
  // appends its arrivals to nm[rn] and later steps rotate through all three
  // (steps that returned early after an error left them stale)
  const uint32_t rn = c->rot == 2 ? 0u : c->rot + 1u;
  hipLaunchKernelGGL(k_fill_i32, dim3(eb), dim3(tb), 0, st, (int32_t*)(a + L.nm[rz]) + (size_t)ens * ne, 0, (int64_t)ne);
  hipLaunchKernelGGL(k_fill_i32, dim3(eb), dim3(tb), 0, st, (int32_t*)(a + L.ns[rn]) + (size_t)ens * ne, 0, (int64_t)ne);
  hipLaunchKernelGGL(k_fill_i32, dim3(eb), dim3(tb), 0, st, (int32_t*)(a + L.nm[rn]) + (size_t)ens * ne, 0, (int64_t)ne);
  hipLaunchKernelGGL(k_set_counts, dim3(eb), dim3(tb), 0, st, scratch, (int32_t*)(a + L.ns[c->rot]),
                     (int32_t*)(a + L.nm[c->rot]), ne, ens);
  const StepIndex si{0, c->parity, c->rot, 0};
  if (c->p.f32_state)
    hipLaunchKernelGGL(k_set_place<float>, dim3(pb), dim3(tb), 0, st, state_at<float>(a, L.buf0, L.slots, L.omega),
                       state_at<float>(a, L.buf1, L.slots, L.omega), (const Ctl*)(a + L.ctl), si, xyuvwpsi, elem, om,
                       n, ne, ens, (const int32_t*)(a + L.start), scratch);
  else
    hipLaunchKernelGGL(k_set_place<double>, dim3(pb), dim3(tb), 0, st, state_at<double>(a, L.buf0, L.slots, L.omega),
                       state_at<double>(a, L.buf1, L.slots, L.omega), (const Ctl*)(a + L.ctl), si, xyuvwpsi, elem, om,
                       n, ne, ens, (const int32_t*)(a + L.start), scratch);
  hipLaunchKernelGGL(k_fill_i32, dim3(eb), dim3(tb), 0, st, scratch + (size_t)ens * ne, 0, (int64_t)ne);
  hipLaunchKernelGGL(k_restore_ctl, dim3(1), dim3(64), 0, st, (Ctl*)(a + L.ctl), all_restored ? 1 : 0);
  if ((r = hip_check(c, hipGetLastError(), "set-state launch"))) return r;
  return hip_check(c, hipStreamSynchronize(st), "sync set-state");
}

pdf_status pdf_set_step(pdf_ctx* c, int64_t step) {
  if (!c || step < 0 || step > 0xFFFFFFFEll) return fail(c, PDF_E_ARG, "pdf_set_step: bad step");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_set_step before pdf_seed_particles");
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, c->stream, (Ctl*)(c->arena + c->L.ctl), (uint32_t)step);
  return hip_check(c, hipGetLastError(), "set-step launch");
}

pdf_status pdf_get_state(pdf_ctx* c, int32_t ens, double* xyuvwpsi, int32_t* elem) {
  if (!c || !xyuvwpsi || !elem) return fail(c, PDF_E_ARG, "pdf_get_state: null output");
  return gather_state(c, ens, xyuvwpsi, elem, nullptr);
}

pdf_status pdf_get_omega(pdf_ctx* c, int32_t ens, double* xyuvwpsi, int32_t* elem, double* om) {
  if (!c || !xyuvwpsi || !elem || !om) return fail(c, PDF_E_ARG, "pdf_get_omega: null output");
  if (!c->p.omega) return fail(c, PDF_E_STATE, "pdf_get_omega: the context carries no turbulent frequency");
  return gather_state(c, ens, xyuvwpsi, elem, om);
}

pdf_status pdf_omega_fields(pdf_ctx* c, double* om0, double* somega, double* omw) {
  if (!c || !om0 || !somega || !omw) return fail(c, PDF_E_ARG, "pdf_omega_fields: null output");
  if (!c->mesh_ready) return fail(c, PDF_E_STATE, "pdf_omega_fields before pdf_init_mesh");
  if (!c->p.omega) return fail(c, PDF_E_STATE, "pdf_omega_fields: the context carries no turbulent frequency");
  pdf_status r;
  const char* a = c->arena;
  if ((r = hip_check(c, hipMemcpyAsync(om0, a + c->L.om0, (size_t)c->ne * 8, hipMemcpyDeviceToHost, c->stream), "copy om0"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(somega, a + c->L.somega, (size_t)c->ne * 8, hipMemcpyDeviceToHost, c->stream), "copy somega"))) return r;
  if ((r = hip_check(c, hipMemcpyAsync(omw, a + c->L.omw, (size_t)c->ne * 24, hipMemcpyDeviceToHost, c->stream), "copy omw"))) return r;
  return hip_check(c, hipStreamSynchronize(c->stream), "sync omega fields");
}

int32_t pdf_navg(const pdf_ctx* c) { return c ? navg_of(c->p) : 0; }

pdf_status pdf_average_attach(pdf_ctx* c, double* acc) {
  if (!c) return PDF_E_ARG;
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_average_attach before pdf_seed_particles");
  c->avg = acc;
  c->graph_group = 0;  // graphs carry the merge only when averaging
  if (!acc) return PDF_OK;
  const int64_t words = 2 * (int64_t)c->nens * c->ne * navg_of(c->p);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, c->stream, (int32_t*)acc, 0, words);
  return hip_check(c, hipGetLastError(), "average clear");
}

pdf_status pdf_locate(pdf_ctx* c, const double* xy, int32_t n, int32_t* elem) {
  if (!c || n < 0 || (n > 0 && (!xy || !elem))) return fail(c, PDF_E_ARG, "pdf_locate: bad argument");
  if (!c->mesh_ready) return fail(c, PDF_E_STATE, "pdf_locate before pdf_init_mesh");
  if (n == 0) return PDF_OK;
  hipLaunchKernelGGL(k_locate, dim3(n), dim3(BLOCK), 0, c->stream, (const ERec*)(c->arena + c->L.erec), c->ne, xy, n, elem);
  return hip_check(c, hipGetLastError(), "locate launch");
}

pdf_status pdf_average_probe(pdf_ctx* c, const double* acc, int32_t ens, const int32_t* elems, int32_t nprobe,
                             double* out) {
  if (!c || !acc || nprobe < 0 || (nprobe > 0 && (!elems || !out))) return fail(c, PDF_E_ARG, "pdf_average_probe: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_average_probe before pdf_seed_particles");
  if (ens < 0 || ens >= c->nens) return fail(c, PDF_E_ARG, "ensemble out of range");
  if (nprobe == 0) return PDF_OK;
  hipLaunchKernelGGL(k_probe, dim3((nprobe + 63) / 64), dim3(64), 0, c->stream, acc, navg_of(c->p), c->ne, ens, elems,
                     nprobe, c->p.hist_bins, out);
  return hip_check(c, hipGetLastError(), "probe launch");
}

int64_t pdf_count(const pdf_ctx* c, int32_t ens) {
  if (!c || ens < 0 || ens >= c->nens) return -1;
  return c->ens_count[ens];
}

int64_t pdf_steps_done(pdf_ctx* c) {
  if (!c || !c->seeded) return -1;
  return c->steps_done;
}

const char* pdf_error_string(const pdf_ctx* c) { return c ? c->err.c_str() : "null context"; }

void pdf_destroy(pdf_ctx* c) {
  if (!c) return;
  if (c->stream || c->seeded) (void)hipStreamSynchronize(c->stream);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->rx_sg.release();
  c->px_sg.release();
  for (auto& e : c->rx_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  for (auto& e : c->side_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->rx_pin) (void)hipHostFree(c->rx_pin);
  delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned conditional means

namespace {

int mlp_blocks(int64_t tiles) { return (int)((tiles + mlp::MLP_WAVES - 1) / mlp::MLP_WAVES); }

pdf_status mlp_hip(hipError_t e) { return e == hipSuccess ? PDF_OK : PDF_E_HIP; }

// One gradient pass over a batch, then the reduction (and, with update, the
// Adam step numbered t).
pdf_status mlp_grad_step(const float* rows, int64_t nrows, int32_t batch, int32_t draw, uint64_t seed, uint32_t t,
                         const float* norm, uint16_t* w, float* work, float* grad, float* loss, int update,
                         float* master, float* am, float* av, float lr, hipStream_t st) {
  const int ntiles = (batch + mlp::TILE - 1) / mlp::TILE;
  mlp::GradArgs g{};
  g.rows = rows;
  g.nrows = nrows;
  g.batch = batch;
  g.draw = draw;
  g.k0 = (uint32_t)seed;
  g.k1 = (uint32_t)(seed >> 32);
  g.iter = t;
  g.norm = norm;
  g.w = w;
  g.partial = work;
  g.loss_partial = work + (size_t)ntiles * mlp::NPARAM;
  hipLaunchKernelGGL(mlp::k_mlp_grad, dim3(mlp_blocks(ntiles)), dim3(64 * mlp::MLP_WAVES), 0, st, g);
  mlp::AdamArgs a{};
  a.partial = g.partial;
  a.loss_partial = g.loss_partial;
  a.ntiles = ntiles;
  a.inv_batch = 1.0f / (float)batch;
  a.loss_out = loss;
  a.grad_out = grad;
  a.update = update;
  a.master = master;
  a.m = am;
  a.v = av;
  a.w = w;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.bc1 = (float)(1.0 - std::pow(0.9, (double)t));
  a.bc2 = (float)(1.0 - std::pow(0.999, (double)t));
  hipLaunchKernelGGL(mlp::k_mlp_adam, dim3((mlp::NPARAM + 255) / 256), dim3(256), 0, st, a);
  return mlp_hip(hipGetLastError());
}

template <typename T> void launch_dataset(pdf_ctx* c, int32_t target, uint64_t key, uint32_t draw, float* rows) {
  const Layout& L = c->L;
  char* a = c->arena;
  mlp::DatasetArgs<T> d{};
  d.buf[0] = state_at<T>(a, L.buf0, L.slots, L.omega);
  d.buf[1] = state_at<T>(a, L.buf1, L.slots, L.omega);
  d.ctl = (const Ctl*)(a + L.ctl);
  d.parity = c->parity;
  d.start = (const int32_t*)(a + L.start);
  d.cap = (const int32_t*)(a + L.cap);
  d.ns = (const int32_t*)(a + L.ns[c->rot]);
  d.nm = (const int32_t*)(a + L.nm[c->rot]);
  d.ne = c->ne;
  d.ncell = c->ne * c->nens;
  d.target = target;
  d.k0 = (uint32_t)key;
  d.k1 = (uint32_t)(key >> 32);
  d.draw = draw;
  d.rows = rows;
  hipLaunchKernelGGL(mlp::k_mlp_dataset<T>, dim3((d.ncell + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK), dim3(BLOCK), 0,
                     c->stream, d);
}

// Gradient partials of pdf_mlp_grad_noalloc: one row of PDF_MLP_NPARAM floats
// per 16-row tile of the largest batch, then one loss partial per tile.  The
// gradient kernel writes every word of the tiles a call uses before the
// reduction reads it, so nothing needs clearing between calls.  Each device
// holds its own copy until the process ends; in host code the array's name
// is not a device address, so kernels receive the address that
// hipGetSymbolAddress returns for the current device.
constexpr int64_t NOALLOC_TILES = (PDF_MLP_NOALLOC_MAX_BATCH + mlp::TILE - 1) / mlp::TILE;
static __device__ __align__(256) float scratch[NOALLOC_TILES * (mlp::NPARAM + 1)];
static_assert(NOALLOC_TILES * (mlp::NPARAM + 1) == PDF_MLP_NOALLOC_FLOATS, "scratch size of the header");

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
float* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of the current device's scratch array, looked up once
// per device.
pdf_status noalloc_scratch(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PDF_E_HIP;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return PDF_E_ARG;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PDF_E_HIP;
    noalloc_ptr[dev] = (float*)ptr;
  }
  *out = noalloc_ptr[dev];
  return PDF_OK;
}

}  // namespace

extern "C" {

int64_t pdf_mlp_work_floats(int32_t batch) {
  if (batch <= 0) return 0;
  const int64_t tiles = (batch + mlp::TILE - 1) / mlp::TILE;
  return tiles * (mlp::NPARAM + 1);
}

pdf_status pdf_mlp_dataset(pdf_ctx* c, int32_t target, uint64_t key, uint32_t draw, float* rows) {
  if (!c || !rows || target <= 0) return fail(c, PDF_E_ARG, "pdf_mlp_dataset: bad argument");
  if (!c->seeded) return fail(c, PDF_E_STATE, "pdf_mlp_dataset before pdf_seed_particles");
  if (c->p.f32_state) launch_dataset<float>(c, target, key, draw, rows);
  else launch_dataset<double>(c, target, key, draw, rows);
  return hip_check(c, hipGetLastError(), "dataset launch");
}

pdf_status pdf_mlp_forward(const float* rows, int64_t nrows, int32_t row_stride, const float* norm,
                           const uint16_t* w, float* y, void* hip_stream) {
  if (!rows || !norm || !w || !y || nrows < 0 || row_stride < mlp::NFEAT) return PDF_E_ARG;
  if (nrows == 0) return PDF_OK;
  mlp::ForwardArgs f{rows, nrows, row_stride, norm, w, y};
  const int64_t tiles = (nrows + mlp::TILE - 1) / mlp::TILE;
  if (tiles > (int64_t)1 << 30) return PDF_E_SIZE;
  hipLaunchKernelGGL(mlp::k_mlp_forward, dim3(mlp_blocks(tiles)), dim3(64 * mlp::MLP_WAVES), 0,
                     (hipStream_t)hip_stream, f);
  return mlp_hip(hipGetLastError());
}

pdf_status pdf_mlp_grad(const float* rows, int32_t batch, const float* norm, const uint16_t* w, float* work,
                        float* grad, float* loss, void* hip_stream) {
  if (!rows || !norm || !w || !work || !grad || batch <= 0 || batch > PDF_MLP_MAX_BATCH) return PDF_E_ARG;
  return mlp_grad_step(rows, batch, batch, 0, 0, 0, norm, const_cast<uint16_t*>(w), work, grad, loss, 0, nullptr,
                       nullptr, nullptr, 0.0f, (hipStream_t)hip_stream);
}

pdf_status pdf_mlp_grad_noalloc(const float* rows, int32_t batch, const float* norm, const uint16_t* w, float* grad,
                                float* loss, void* hip_stream) {
  if (!rows || !norm || !w || !grad || !loss || batch <= 0) return PDF_E_ARG;
  if (batch > PDF_MLP_NOALLOC_MAX_BATCH) return PDF_E_SIZE;
  float* work = nullptr;
  const pdf_status r = noalloc_scratch(&work);
  if (r) return r;
  return mlp_grad_step(rows, batch, batch, 0, 0, 0, norm, const_cast<uint16_t*>(w), work, grad, loss, 0, nullptr,
                       nullptr, nullptr, 0.0f, (hipStream_t)hip_stream);
}

pdf_status pdf_mlp_train(const float* rows, int64_t nrows, const float* norm, float* master, float* adam_m,
                         float* adam_v, uint16_t* w, float* work, float* loss, int32_t iters, int32_t batch,
                         float lr, uint64_t seed, int64_t t0, void* hip_stream) {
  if (!rows || !norm || !master || !adam_m || !adam_v || !w || !work || nrows <= 0 || nrows > 0xFFFFFFFFll ||
      iters < 0 || batch <= 0 || batch > PDF_MLP_MAX_BATCH || t0 < 0 || t0 + iters > 0xFFFFFFFFll || !(lr > 0.0f))
    return PDF_E_ARG;
  for (int32_t i = 0; i < iters; ++i) {
    const uint32_t t = (uint32_t)(t0 + i + 1);
    pdf_status r = mlp_grad_step(rows, nrows, batch, 1, seed, t, norm, w, work, nullptr, loss ? loss + i : nullptr, 1,
                                 master, adam_m, adam_v, lr, (hipStream_t)hip_stream);
    if (r) return r;
  }
  return PDF_OK;
}

pdf_status pdf_mlp_norm(const float* rows, int64_t nrows, float* norm, void* hip_stream) {
  if (!rows || !norm || nrows < 0) return PDF_E_ARG;
  hipLaunchKernelGGL(mlp::k_mlp_norm, dim3(mlp::NFEAT), dim3(256), 0, (hipStream_t)hip_stream, rows, nrows, norm);
  return mlp_hip(hipGetLastError());
}

pdf_status pdf_mlp_round(const float* master, uint16_t* w, void* hip_stream) {
  if (!master || !w) return PDF_E_ARG;
  hipLaunchKernelGGL(mlp::k_mlp_to_bf16, dim3((mlp::NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream,
                     master, w, (int)mlp::NPARAM);
  return mlp_hip(hipGetLastError());
}

pdf_status pdf_mlp_infer(const double* stats, int32_t nstat, int32_t ncell, const uint16_t* w, const float* norm,
                         double* cm, uint32_t* served, void* hip_stream) {
  if (!stats || !w || !norm || !cm || ncell < 0 || nstat < NSTAT2) return PDF_E_ARG;
  if (ncell == 0) return PDF_OK;
  mlp::InferArgs ia{stats, nstat, ncell, w, norm, cm, served};
  const int tiles = (ncell + mlp::TILE - 1) / mlp::TILE;
  hipLaunchKernelGGL(mlp::k_mlp_infer, dim3(mlp_blocks(tiles)), dim3(64 * mlp::MLP_WAVES), 0, (hipStream_t)hip_stream,
                     ia);
  return mlp_hip(hipGetLastError());
}

pdf_status pdf_mlp_attach(pdf_ctx* c, const uint16_t* w, const float* norm, double* cm, uint32_t* served) {
  if (!c) return PDF_E_ARG;
  c->graph_group = 0;  // a graph holds the step arguments it was built with
  if (!w) {
    c->mlp_w = nullptr;
    c->mlp_norm = nullptr;
    c->mlp_cm = nullptr;
    c->mlp_served = nullptr;
    return PDF_OK;
  }
  if (!norm || !cm) return fail(c, PDF_E_ARG, "pdf_mlp_attach: null normalisation or output");
  if (c->p.vbins != 2) return fail(c, PDF_E_STATE, "pdf_mlp_attach: the network estimates the eight sign bins only");
  c->mlp_w = w;
  c->mlp_norm = norm;
  c->mlp_cm = cm;
  c->mlp_served = served;
  return PDF_OK;
}

}  // extern "C"
