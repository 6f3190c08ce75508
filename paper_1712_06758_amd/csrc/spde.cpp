// C interface and host orchestration of the SPDE field sampler.
//
// The solve of eq. linsys for a batch of noise vectors runs as a loop of
// MINRES iterations on the device; the host only replays iteration blocks
// (captured HIP graphs, or plain launches) and polls per-sample convergence
// flags between blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/spde.h"
#include "spde_internal.h"

namespace spde {
int build_transfer_csr(int n, int64_t n_vert, const double* xyz, int64_t n_tet, const int32_t* tets,
                       std::vector<int64_t>& row_ptr, std::vector<int32_t>& cols, std::vector<double>& vals,
                       char* err, size_t errlen);
int coarsen_transfer_csr(int n_fine, int64_t n_rows, const int64_t* rp, const int32_t* ci, const double* cv,
                         std::vector<int64_t>& rp_c, std::vector<int32_t>& ci_c, std::vector<double>& cv_c,
                         char* err, size_t errlen);
}

using namespace spde;

namespace {

thread_local std::string g_err;

spde_status fail(spde_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
spde_status fail(spde_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(SPDE_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

const char* kKernelNames[KID_COUNT] = {
    "init", "mg_down_fine", "mg_down", "mg_coarse", "mg_up", "mg_up_fine",
    "scalar", "operator", "output", "flux", "resid", "spmm", "restrict_noise", "spmm_stage"};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace spde {

struct LaunchRec {
  int kid;
  int iter;          // MINRES iteration of the launch (0 outside the loop)
  int level;         // multigrid level of a level kernel
  int s0, nslots;    // slots of the launch (nslots < 0: the whole batch)
  hipEvent_t e0, e1;
  double bytes;      // algorithmic bytes of the whole launch, or < 0: per slot from slot_bytes
};

struct Ctx {
  // problem
  int n = 0;
  double kappa = 0, g = 0;
  double kappa_pre = 0;         // kappa of the multigrid preconditioner (the constant kappa, or
                                // the reference kappa of cell-wise coefficients)
  Box box{};
  // configuration
  int prec = SPDE_FP64;
  double rtol = 1e-10;
  int max_iter = 1000;
  int max_batch = 1;
  bool configured = false;
  // hierarchy
  int nlev = 0;                 // levels 0..nlev-1 (m = n >> l, down to 1)
  Level lv[kMaxLevels];
  int top = 1;                  // first level handled by the persistent kernel
  size_t coarse_lds = 0;
  CoarseParams cp{};
  int shape_down[kMaxLevels];
  int shape_up[kMaxLevels];
  int nb_up0 = 0, nb_pb = 0;
  // device
  int device = -1;
  int lds_limit = 65536;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Fields F{};
  void* mgb[kMaxLevels] = {};   // restricted right-hand sides per level (l >= 1)
  void* mge[kMaxLevels] = {};   // level corrections (l >= 1)
  void* mgd[kMaxLevels] = {};   // cell-wise diagonal of S~ per level (shared by the slots)
  void* mgdi[kMaxLevels] = {};  // and its reciprocal
  void* cinv = nullptr;         // inverse of the 4^3 level's S~ (exact solve of the persistent kernel)
  bool cinv_dirty = true;       // cinv must be rebuilt before the next solve
  bool mg_cellwise = false;     // the kappa field enters the multigrid (Galerkin coarse kappa^2)
  bool mg_dirty = false;        // the level diagonals must be rebuilt before the next solve
  double* resid_out = nullptr;  // [max_batch]
  hipStream_t own_stream = nullptr;
  hipStream_t aux_stream = nullptr;   // second half of a split batch
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  Scalars* host_sc = nullptr;   // pinned
  double* host_res = nullptr;   // pinned
  // transfer
  int64_t n_tet = 0, nnz = 0;
  const int64_t* rp = nullptr;
  const int32_t* ci = nullptr;
  const double* cv = nullptr;
  const int32_t* order = nullptr;   // optional chunk visiting order of the SpMM
  // optional row units of the LDS-staged SpMM (spde_set_transfer_units)
  const int64_t* uptr = nullptr;
  const int32_t* ucells = nullptr;
  const uint16_t* lcol = nullptr;
  int u_max_cells = 0, u_max_entries = 0;
  int64_t u_cells = 0;   // listed cells over all units
  // execution
  bool use_graphs = true;
  int poll = 8;
  std::map<int64_t, hipGraphExec_t> graphs;   // (first slot, half-iterations, batch) -> graph
  int split = 1;                 // 2: batches of 8+ run as two halves on two streams
  int expect_iters = 0;          // iterations (incl. the finishing pass) the last call needed
  double refine_target = 0.0;     // > 0: refine until ||F - A U|| / ||F|| <= target (float64 residuals)
  int refine_max = 0;             // at most this many refinement passes
  bool tuned = false;
  bool autotune = true;
  int face_precond = 1;          // 0 diag(M)^-1, 1 truncated Neumann series of M^-1
  // timing: 0 off; 1 every kernel class, plain launches; 2 the operator pass
  // only: every third operator launch runs on its own between graph replays,
  // bracketed by an event pair
  int timing = 0;
  bool capturing = false;                       // no event pairs inside a captured graph
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<LaunchRec> recs;
  double t_ms[KID_COUNT] = {};
  int64_t t_n[KID_COUNT] = {};
  double t_bytes[KID_COUNT] = {};

  bool fp64() const { return prec == SPDE_FP64; }
  size_t szm() const { return fp64() ? 8 : 4; }
};

}  // namespace spde

namespace {

// Chebyshev degree-2 smoother coefficients on [lmax/4, lmax] of D^-1 S~, with
// lmax the Gershgorin bound (k2 + 12 a) / (k2 + 6 a) (capped at 2).
void set_level(Level& L, int m, double kappa) {
  const double H = 1.0 / m;
  L.m = m;
  L.nc = (int64_t)m * m * m;
  L.k2 = kappa * kappa * H * H * H;
  L.a = 1.5 * H;
  const double lmax = std::min(2.0, (L.k2 + 12.0 * L.a) / (L.k2 + 6.0 * L.a));
  const double lmin = lmax / 4.0;
  const double th = 0.5 * (lmax + lmin), dl = 0.5 * (lmax - lmin);
  const double sig = th / dl, rho0 = 1.0 / sig, rho1 = 1.0 / (2.0 * sig - rho0);
  L.c0 = 1.0 / th;
  L.c1 = 1.0 + rho1 * rho0;
  L.c2 = 2.0 * rho1 / dl;
  L.cA = L.c1 * L.c0 + L.c2 * (1.0 - L.c0);
  L.cB = L.c2 * L.a * L.c0;
  L.dg = nullptr;
  L.dgi = nullptr;
}

// The persistent kernel solves the 4^3 level exactly when its top level is
// 4^3 or larger.
bool coarse_dense(const Ctx* c) { return c->lv[c->top].m >= 4; }

size_t coarse_bytes(const Ctx* c, int top) {
  size_t tot = 0;
  for (int l = top; l < c->nlev; ++l) tot += 4 * (size_t)c->lv[l].nc * c->szm();
  return tot;
}

void plan_hierarchy(Ctx* c) {
  c->nlev = 0;
  for (int m = c->n; m >= 1; m >>= 1) set_level(c->lv[c->nlev++], m, c->kappa_pre);
  c->mg_dirty = c->mg_cellwise;   // level diagonals (if any) are rebuilt before the next solve
  c->cinv_dirty = true;
  // persistent kernel: the largest levels (below the finest) that fit in LDS, at most 16^3
  int top = c->nlev - 1;
  for (int l = 1; l < c->nlev; ++l) {
    if (c->lv[l].m <= 16 && coarse_bytes(c, l) + kCoarseStaticLds <= (size_t)c->lds_limit) { top = l; break; }
  }
  c->top = top;
  c->coarse_lds = coarse_bytes(c, top);
  c->cp.nl = c->nlev - top;
  int64_t off = 0;
  for (int l = top; l < c->nlev; ++l) {
    c->cp.lv[l - top] = c->lv[l];
    c->cp.off[l - top] = off;
    off += 4 * c->lv[l].nc;
  }
  for (int l = 0; l < c->nlev; ++l) {
    c->shape_down[l] = 0;
    c->shape_up[l] = c->fp64() ? 1 : 0;
  }
  int mx = 0;
  for (int s = 0; s < kNumShapes; ++s) mx = std::max(mx, tiles_for(s, c->n));
  c->nb_up0 = mx;   // capacity; the partial count used is tiles_for(shape_up[0], n)
  c->nb_pb = operator_blocks(c->box);
}

size_t layout(Ctx* c, char* base) {
  const int64_t nc = c->box.nc;
  const size_t B = (size_t)c->max_batch;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  for (int p = 0; p < 2; ++p) c->F.vs[p] = (double*)take(B * 3 * nc * 8);
  for (int p = 0; p < 2; ++p) c->F.vu[p] = (double*)take(B * nc * 8);
  for (int p = 0; p < 2; ++p) c->F.z[p] = (void*)take(B * nc * c->szm());
  for (int p = 0; p < 2; ++p) c->F.w[p] = (double*)take(B * nc * 8);
  c->F.x = (double*)take(B * nc * 8);
  for (int l = 1; l <= c->top && l < c->nlev; ++l) {
    c->mgb[l] = take(B * c->lv[l].nc * c->szm());
    c->mge[l] = take(B * c->lv[l].nc * c->szm());
  }
  for (int l = 0; l < c->nlev; ++l) {
    c->mgd[l] = take(c->lv[l].nc * c->szm());
    c->mgdi[l] = take(c->lv[l].nc * c->szm());
  }
  c->cinv = take((size_t)64 * 64 * c->szm());
  c->cp.cinv = c->cinv;
  if (base) c->cinv_dirty = true;   // new memory: the inverse is built again
  c->F.part_up = (double*)take(B * (size_t)c->nb_up0 * 2 * 8);
  c->F.part_pb = (double*)take(B * (size_t)c->nb_pb * 2 * 8);
  c->F.sc = (Scalars*)take(B * sizeof(Scalars));
  c->resid_out = (double*)take(B * 8);
  return off;
}

// ---- timing -----------------------------------------------------------------

hipEvent_t next_event(Ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

struct Timed {
  Ctx* c;
  int kid, iter, level, s0, nslots;
  hipStream_t st;
  double bytes;
  hipEvent_t e0 = nullptr;
  bool on = false;
  Timed(Ctx* c_, int kid_, int iter_, hipStream_t st_, int level_ = 0, int s0_ = 0, int nslots_ = -1,
        double bytes_ = -1.0)
      : c(c_), kid(kid_), iter(iter_), level(level_), s0(s0_), nslots(nslots_), st(st_), bytes(bytes_) {
    on = !c->capturing && (c->timing == 1 || (c->timing == 2 && kid == KID_OPERATOR));
    if (!on) return;
    e0 = next_event(c);
    if (e0) hipEventRecord(e0, st);
  }
  ~Timed() {
    if (!on || !e0) return;
    hipEvent_t e1 = next_event(c);
    if (e1) {
      hipEventRecord(e1, st);
      c->recs.push_back({kid, iter, level, s0, nslots, e0, e1, bytes});
    }
  }
};

// Algorithmic bytes of one launch for one slot (compulsory HBM traffic of the
// method's data: every input read once, every output written once).
double slot_bytes(const Ctx* c, int kid, int level, int iter, int wmode_active) {
  const double nc = (double)c->box.nc, sz = (double)c->szm();
  switch (kid) {
    case KID_OPERATOR: {
      // v update (iterations 1..J): read v_j (faces 24, cell 8), v_{j-1} (32, from j = 2), zhat_j;
      // write v_{j+1} (32).  Direction update (iterations 1..J): read W_j (j >= 2) and W_{j-1}
      // (j >= 3), write W_{j+1}.  x: written alone at j = 2, read and written on later even passes
      // and on the finishing pass J + 1, which reads W_J and W_{J-1} and writes nothing else.
      double b = 0;
      const bool fin = (wmode_active & 4) != 0;
      if (wmode_active & 1) b += nc * ((iter > 1 ? 64.0 : 32.0) + sz + 32.0 + (c->box.kap ? 8.0 : 0.0));
      if ((wmode_active & 2) && !fin) b += nc * (8.0 + (iter >= 2 ? 8.0 : 0.0) + (iter >= 3 ? 8.0 : 0.0));
      if (fin) b += nc * (8.0 + (iter >= 4 ? 8.0 : 0.0));
      if ((wmode_active & 2) && iter >= 2) {
        if (iter == 2) b += nc * 8.0;
        else if ((iter % 2) == 0 || fin) b += nc * 16.0;
      }
      return b;
    }
    case KID_MG_UP_FINE: return nc * (8.0 + sz / 8.0 + 24.0 + sz + (c->box.kap ? 8.0 : 0.0));
    case KID_MG_DOWN_FINE: return nc * (8.0 + sz / 8.0);
    case KID_MG_DOWN: { const double m = (double)c->lv[level].nc; return m * (sz + sz / 8.0); }
    case KID_MG_UP: { const double m = (double)c->lv[level].nc; return m * (sz + sz / 8.0 + sz); }
    case KID_MG_COARSE: return 2.0 * (double)c->lv[c->top].nc * sz;
    default: return 0.0;
  }
}

// Tile shapes a level's kernels run with: the tuned ones, except that the
// cell-wise-diagonal kernels exist only in the pipelined column shapes (10-17).
int eff_down(const Ctx* c, int l) {
  const int s = c->shape_down[l];
  return (c->lv[l].dg && s < 10) ? 16 : s;
}
int eff_up(const Ctx* c, int l) {
  const int s = c->shape_up[l];
  return (c->lv[l].dg && s < 10) ? 17 : s;
}

// ---- one MINRES iteration (all kernels), enqueued on st ------------------------

// The slots [s0, s0 + batch) of the context: device pointers advanced to slot
// s0, so that every kernel sees its sub-batch as slots 0 .. batch-1.
struct View {
  int s0 = 0;
  Fields F{};
  void* mgb[kMaxLevels] = {};
  void* mge[kMaxLevels] = {};
};

View make_view(const Ctx* c, int s0) {
  View V;
  V.s0 = s0;
  V.F = c->F;
  const int64_t nc = c->box.nc;
  const size_t sz = c->szm();
  for (int p = 0; p < 2; ++p) {
    V.F.vs[p] += (int64_t)s0 * 3 * nc;
    V.F.vu[p] += (int64_t)s0 * nc;
    V.F.z[p] = (char*)c->F.z[p] + (size_t)s0 * nc * sz;
    V.F.w[p] += (int64_t)s0 * nc;
  }
  V.F.x += (int64_t)s0 * nc;
  V.F.part_up += (int64_t)s0 * tiles_for(eff_up(c, 0), c->n) * 2;
  V.F.part_pb += (int64_t)s0 * c->nb_pb;
  V.F.sc += s0;
  for (int l = 1; l < c->nlev; ++l) {
    if (c->mgb[l]) V.mgb[l] = (char*)c->mgb[l] + (size_t)s0 * c->lv[l].nc * sz;
    if (c->mge[l]) V.mge[l] = (char*)c->mge[l] + (size_t)s0 * c->lv[l].nc * sz;
  }
  return V;
}

spde_status enqueue_vcycle(Ctx* c, const View& V, int batch, hipStream_t st, int iter, const void* b0,
                           const void* b1, void* o0, void* o1, const Scalars* sc, double* part) {
  const bool f64 = c->fp64();
  const int s0 = V.s0;
  {
    Timed t(c, KID_MG_DOWN_FINE, iter, st, 0, s0, batch);
    HIPCHK(launch_mg_down(f64, eff_down(c, 0), true, b0, b1, V.mgb[1], c->lv[0], batch, sc, st));
  }
  for (int l = 1; l < c->top; ++l) {
    Timed t(c, KID_MG_DOWN, iter, st, l, s0, batch);
    HIPCHK(launch_mg_down(f64, eff_down(c, l), false, V.mgb[l], V.mgb[l], V.mgb[l + 1], c->lv[l], batch, sc, st));
  }
  if (c->cinv_dirty && coarse_dense(c))
    return fail(SPDE_EINVAL, "the exact 4^3 coarse solve was not prepared before the V-cycle");
  {
    Timed t(c, KID_MG_COARSE, iter, st, 0, s0, batch);
    HIPCHK(launch_mg_coarse(f64, V.mgb[c->top], V.mge[c->top], c->cp, c->coarse_lds, batch, sc, st));
  }
  for (int l = c->top - 1; l >= 1; --l) {
    Timed t(c, KID_MG_UP, iter, st, l, s0, batch);
    HIPCHK(launch_mg_up(f64, eff_up(c, l), false, V.mgb[l], V.mgb[l], V.mge[l + 1], V.mge[l], V.mge[l],
                        c->lv[l], batch, sc, nullptr, nullptr, nullptr, c->box, st));
  }
  {
    Timed t(c, KID_MG_UP_FINE, iter, st, 0, s0, batch);
    HIPCHK(launch_mg_up(f64, eff_up(c, 0), true, b0, b1, V.mge[1], o0, o1, c->lv[0], batch, sc,
                        V.F.vs[0], V.F.vs[1], part, c->box, st));
  }
  return SPDE_OK;
}

// One MINRES iteration without its operator pass: V-cycle and scalars.
spde_status enqueue_vpart(Ctx* c, const View& V, int batch, hipStream_t st, int iter) {
  spde_status s = enqueue_vcycle(c, V, batch, st, iter, V.F.vu[0], V.F.vu[1], V.F.z[0], V.F.z[1], V.F.sc,
                                 V.F.part_up);
  if (s != SPDE_OK) return s;
  Timed t(c, KID_SCALAR, iter, st, 0, V.s0, batch);
  HIPCHK(launch_scalar(V.F, tiles_for(eff_up(c, 0), c->n), c->nb_pb, batch, st));
  return SPDE_OK;
}

spde_status enqueue_operator(Ctx* c, const View& V, int batch, hipStream_t st, int iter) {
  Timed t(c, KID_OPERATOR, iter, st, 0, V.s0, batch);
  HIPCHK(launch_operator(c->fp64(), V.F, c->box, batch, st));
  return SPDE_OK;
}

spde_status enqueue_iteration(Ctx* c, const View& V, int batch, hipStream_t st, int iter) {
  spde_status s = enqueue_vpart(c, V, batch, st, iter);
  if (s != SPDE_OK) return s;
  return enqueue_operator(c, V, batch, st, iter);
}

// Graph of L half-iterations for the slots of V, captured on first use:
// V-part, operator, V-part, ... (L = 2 K is K whole iterations; L odd ends
// with a V-part).  The iteration numbers inside a graph are irrelevant: the
// kernels take their state from the per-slot scalars.
spde_status get_graph(Ctx* c, const View& V, int batch, hipStream_t st, hipGraphExec_t* out, int L) {
  const int64_t key = ((int64_t)V.s0 << 40) | ((int64_t)L << 24) | (int64_t)batch;
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) { *out = it->second; return SPDE_OK; }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  spde_status s = SPDE_OK;
  for (int h = 0; h < L && s == SPDE_OK; ++h)
    s = (h & 1) ? enqueue_operator(c, V, batch, st, 0) : enqueue_vpart(c, V, batch, st, 0);
  c->capturing = false;
  hipError_t e = hipStreamEndCapture(st, &g);
  if (s != SPDE_OK) { if (g) hipGraphDestroy(g); return s; }
  if (e != hipSuccess) return fail(SPDE_EHIP, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return fail(SPDE_EHIP, "graph instantiate: %s", hipGetErrorString(e));
  c->graphs[key] = ex;
  *out = ex;
  return SPDE_OK;
}

// Launch the graph of L half-iterations; false if graphs are not available.
bool launch_graph(Ctx* c, const View& V, int batch, hipStream_t st, int L) {
  hipGraphExec_t ex = nullptr;
  if (get_graph(c, V, batch, st, &ex, L) != SPDE_OK || !ex) {
    hipGetLastError();
    c->use_graphs = false;
    return false;
  }
  return hipGraphLaunch(ex, st) == hipSuccess;
}

// Operator passes timed in mode 2: every kTimedStride-th iteration of a block
// (both parities of the iteration number occur).
constexpr int kTimedStride = 3;

// `count` iterations for the slots of V: a captured graph if graphs are on
// and count is the poll interval, else plain launches.  In timing mode 2 the
// operator passes k = 0, 3, 6, ... of the block are launched on their own,
// bracketed by an event pair, and everything between them replays as graphs.
spde_status enqueue_block(Ctx* c, const View& V, int batch, hipStream_t st, bool graphs, int iter0, int count) {
  if (graphs && c->timing == 2) {
    bool ok = launch_graph(c, V, batch, st, 1);   // V-part of iteration 0
    for (int k = 0; ok && k < count; k += kTimedStride) {
      spde_status s = enqueue_operator(c, V, batch, st, iter0 + k + 1);
      if (s != SPDE_OK) return s;
      const int next = k + kTimedStride;
      // iterations k+1 .. next-1 whole, then the V-part of `next` (or the rest of the block)
      const int L = next < count ? 2 * (kTimedStride - 1) + 1 : 2 * (count - 1 - k);
      if (L > 0) ok = launch_graph(c, V, batch, st, L);
    }
    if (ok) return SPDE_OK;
    return fail(SPDE_EHIP, "graph launch failed in timing mode 2");
  }
  if (graphs && c->timing == 0 && count == c->poll) {
    if (launch_graph(c, V, batch, st, 2 * c->poll)) return SPDE_OK;
  }
  for (int k = 0; k < count; ++k) {
    spde_status s = enqueue_iteration(c, V, batch, st, iter0 + k + 1);
    if (s != SPDE_OK) return s;
  }
  return SPDE_OK;
}

void drop_graphs(Ctx* c) {
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

spde_status check_ready(Ctx* c) {
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!c->configured) return fail(SPDE_EINVAL, "spde_configure has not been called");
  if (!c->ws) return fail(SPDE_EINVAL, "no workspace bound (spde_bind_workspace)");
  return SPDE_OK;
}

hipStream_t pick_stream(Ctx* c, void* stream) {
  return stream ? (hipStream_t)stream : c->own_stream;
}

// Close the timing records of a sample: per-launch bytes from the final
// per-slot iteration counts, elapsed times from the event pairs.
void close_timing(Ctx* c, int batch) {
  if (!c->timing) return;
  std::vector<int> iters(batch);
  std::vector<int> states(batch);
  for (int s = 0; s < batch; ++s) { iters[s] = c->host_sc[s].iters; states[s] = c->host_sc[s].state; }
  for (const LaunchRec& r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) continue;
    double bytes = r.bytes >= 0.0 ? r.bytes : 0.0;
    const int s_end = r.bytes >= 0.0 ? r.s0 : (r.nslots < 0 ? batch : std::min(batch, r.s0 + r.nslots));
    for (int s = r.s0; s < s_end; ++s) {
      const bool done = states[s] == ST_DONE || states[s] == ST_FINISH;
      const int J = done ? iters[s] : (1 << 30);
      if (r.kid == KID_OPERATOR) {
        int mode = 0;
        if (r.iter <= J) mode |= 1;
        if (r.iter >= 1 && r.iter <= J + 1) mode |= 2;
        if (r.iter == J + 1) mode |= 4;
        bytes += slot_bytes(c, r.kid, 0, r.iter, mode);
      } else if (r.iter >= 1 && r.iter <= J + 1) {
        bytes += slot_bytes(c, r.kid, r.level, r.iter, 0);
      }
    }
    c->t_ms[r.kid] += ms;
    c->t_n[r.kid] += 1;
    c->t_bytes[r.kid] += bytes;
  }
  c->recs.clear();
  c->ev_used = 0;
}

// ---- autotuner -----------------------------------------------------------------
//
// Chooses the tile shape of every per-level multigrid kernel by timing each
// admissible shape at the context's largest batch.  The choice is keyed by
// (device architecture, n, precision, batch class of max_batch: 1, 2-15, 16+),
// never by the batch of a call, so that every call of a context uses the same
// tiles and the per-block partial sums (hence the results) do not depend on
// how many samples share a launch.
// Choices are kept for the process and, if SPDE_TUNE_CACHE names a file,
// appended there as lines "key level down up".

std::map<std::string, std::vector<std::pair<int, int>>>& tune_table() {
  static std::map<std::string, std::vector<std::pair<int, int>>> t;
  return t;
}

std::string tune_key(Ctx* c) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
  const size_t cut = arch.find(':');
  if (cut != std::string::npos) arch = arch.substr(0, cut);
  // batch class of the context's largest batch: 1, 2..15, 16+
  const char* cls = c->max_batch == 1 ? "b1" : (c->max_batch < 16 ? "b2" : "b16");
  char buf[128];
  // t2: the finest up kernel is timed together with the operator pass that reads its output
  snprintf(buf, sizeof buf, "%s:n%d:%s:%s:t2", arch.c_str(), c->n, c->fp64() ? "fp64" : "mixed", cls);
  return buf;
}

void load_tune_file(const std::string& key) {
  const char* path = getenv("SPDE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char k[128];
  int l, d, u;
  std::vector<std::pair<int, int>> v;
  while (fscanf(f, "%127s %d %d %d", k, &l, &d, &u) == 4) {
    if (key != k || l < 0 || l >= kMaxLevels) continue;
    if ((int)v.size() <= l) v.resize(l + 1, {-1, -1});
    v[l] = {d, u};
  }
  fclose(f);
  if (!v.empty()) tune_table()[key] = v;
}

void save_tune_file(const std::string& key, const std::vector<std::pair<int, int>>& v) {
  const char* path = getenv("SPDE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  for (size_t l = 0; l < v.size(); ++l) fprintf(f, "%s %zu %d %d\n", key.c_str(), l, v[l].first, v[l].second);
  fclose(f);
}

spde_status time_launches(Ctx* c, hipStream_t st, const std::function<hipError_t()>& fn, float* ms) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t err = fn();
  if (err == hipSuccess) err = hipEventRecord(e0, st);
  for (int k = 0; k < 3 && err == hipSuccess; ++k) err = fn();
  if (err == hipSuccess) err = hipEventRecord(e1, st);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err != hipSuccess) return fail(SPDE_EHIP, "autotune: %s", hipGetErrorString(err));
  *ms /= 3.0f;
  return SPDE_OK;
}

spde_status autotune(Ctx* c, hipStream_t st) {
  if (c->tuned) return SPDE_OK;
  const std::string key = tune_key(c);
  auto& tab = tune_table();
  if (!tab.count(key)) load_tune_file(key);
  const bool f64 = c->fp64();
  auto it = tab.find(key);
  bool complete = it != tab.end() && (int)it->second.size() >= c->top;
  if (complete)
    for (int l = 0; l < c->top; ++l)
      if (!shape_ok_down(it->second[l].first, f64) || !shape_ok_up(it->second[l].second, f64)) complete = false;
  if (!complete && c->autotune) {
    const int B = c->max_batch;
    const int64_t nc = c->box.nc;
    // defined contents for the timing launches
    HIPCHK(hipMemsetAsync(c->F.vu[0], 0, (size_t)B * nc * 8, st));
    HIPCHK(hipMemsetAsync(c->F.vs[0], 0, (size_t)B * 3 * nc * 8, st));
    for (int l = 1; l <= c->top && l < c->nlev; ++l) {
      HIPCHK(hipMemsetAsync(c->mgb[l], 0, (size_t)B * c->lv[l].nc * c->szm(), st));
      HIPCHK(hipMemsetAsync(c->mge[l], 0, (size_t)B * c->lv[l].nc * c->szm(), st));
    }
    // the operator pass in the finest level's up timing runs on steady-state scalars
    HIPCHK(launch_tune_scalars(c->F.sc, B, st));
    std::vector<std::pair<int, int>> v(c->top, {0, f64 ? 1 : 0});
    const char* verbose = getenv("SPDE_TUNE_VERBOSE");
    const bool say = verbose && *verbose && *verbose != '0';
    for (int l = 0; l < c->top; ++l) {
      const bool fine = l == 0;
      const void* bsrc = fine ? (const void*)c->F.vu[0] : c->mgb[l];
      void* osrc = fine ? c->F.z[0] : c->mge[l];
      float best = 1e30f;
      for (int sh = 0; sh < kNumShapes; ++sh) {
        if (!shape_ok_down(sh, f64)) continue;
        float ms = 0.f;
        spde_status s = time_launches(c, st, [&] {
          return launch_mg_down(f64, sh, fine, bsrc, bsrc, c->mgb[l + 1], c->lv[l], B, nullptr, st);
        }, &ms);
        if (s != SPDE_OK) return s;
        if (say) fprintf(stderr, "spde autotune %s level %d down shape %2d: %.4f ms\n", key.c_str(), l, sh, ms);
        if (ms < best) { best = ms; v[l].first = sh; }
      }
      best = 1e30f;
      for (int sh = 0; sh < kNumShapes; ++sh) {
        if (!shape_ok_up(sh, f64)) continue;
        float ms = 0.f;
        // On the finest level the operator pass follows and reads the kernel's
        // output; how much of it is still in the caches depends on the tile
        // order, so the two are timed together.
        spde_status s = time_launches(c, st, [&] {
          hipError_t e = launch_mg_up(f64, sh, fine, bsrc, bsrc, c->mge[l + 1], osrc, osrc, c->lv[l], B, nullptr,
                                      c->F.vs[0], c->F.vs[0], fine ? c->F.part_up : nullptr, c->box, st);
          if (e == hipSuccess && fine) e = launch_operator(f64, c->F, c->box, B, st);
          return e;
        }, &ms);
        if (s != SPDE_OK) return s;
        if (say) fprintf(stderr, "spde autotune %s level %d up shape %2d: %.4f ms\n", key.c_str(), l, sh, ms);
        if (ms < best) { best = ms; v[l].second = sh; }
      }
    }
    tab[key] = v;
    save_tune_file(key, v);
    it = tab.find(key);
    complete = true;
  }
  if (complete) {
    for (int l = 0; l < c->top; ++l) {
      c->shape_down[l] = it->second[l].first;
      c->shape_up[l] = it->second[l].second;
    }
  }
  c->tuned = true;
  drop_graphs(c);
  return SPDE_OK;
}

// Cell-wise kappa in the multigrid preconditioner: the reaction diagonal of
// every level (k2 = (kappa kappa) h^3 on the finest, the Galerkin sum of the 8
// children on the coarser ones), each level's diagonal D = K + a nn and D^-1
// in the level precision, and the Chebyshev intervals from kappa_min (the
// Gershgorin bound (k2 + 12 a) / (k2 + 6 a) of D^-1 S~ is largest where k2 is
// smallest, and every level's k2 is at least kappa_min^2 H^3).  The float64
// chain is built in a Lanczos buffer that no solve uses between calls.
spde_status prepare_mg_diag(Ctx* c, hipStream_t st) {
  if (!c->mg_dirty) return SPDE_OK;
  if (!c->mg_cellwise || !c->box.kap) { c->mg_dirty = false; return SPDE_OK; }
  const int64_t nc = c->box.nc;
  double* k2 = c->F.vs[0];                       // [sum of the level sizes] float64 scratch
  double* k2l[kMaxLevels];
  int64_t off = 0;
  for (int l = 0; l < c->nlev; ++l) { k2l[l] = k2 + off; off += c->lv[l].nc; }
  double* mins = k2 + off;                       // block minima of kappa (the chain needs < 8/7 nc)
  HIPCHK(launch_mg_k2_fine(c->box.kap, c->box.h3, k2l[0], nc, st));
  for (int l = 1; l < c->nlev; ++l) HIPCHK(launch_mg_k2_coarsen(k2l[l - 1], k2l[l], c->lv[l - 1].m, st));
  // kappa_min by repeated block minima until at most 4096 values remain
  const double* src = c->box.kap;
  int64_t cnt = nc;
  double* dst = mins;
  while (true) {
    HIPCHK(launch_block_min(src, cnt, dst, st));
    cnt = (cnt + kBlock - 1) / kBlock;
    src = dst;
    if (cnt <= 4096) break;
    dst = dst + cnt;
  }
  HIPCHK(hipMemcpyAsync(c->host_res, src, cnt * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double kmin = c->host_res[0];
  for (int64_t i = 1; i < cnt; ++i) kmin = std::min(kmin, c->host_res[i]);
  if (!(kmin > 0.0) || !std::isfinite(kmin))
    return fail(SPDE_EINVAL, "the kappa field must be positive and finite (minimum %g)", kmin);
  for (int l = 0; l < c->nlev; ++l) {
    set_level(c->lv[l], c->lv[l].m, kmin);
    HIPCHK(launch_mg_diag(c->fp64(), k2l[l], c->lv[l].m, c->lv[l].a, c->mgd[l], c->mgdi[l], st));
    c->lv[l].dg = c->mgd[l];
    c->lv[l].dgi = c->mgdi[l];
  }
  for (int l = c->top; l < c->nlev; ++l) c->cp.lv[l - c->top] = c->lv[l];
  c->kappa_pre = kmin;
  c->mg_dirty = false;
  c->cinv_dirty = true;
  drop_graphs(c);
  return SPDE_OK;
}

// The multigrid coefficients of the next solve: the level diagonals (cell-wise
// kappa) and the inverse of the 4^3 level's operator, both on the stream.
spde_status prepare_mg_coeffs(Ctx* c, hipStream_t st) {
  spde_status s = prepare_mg_diag(c, st);
  if (s != SPDE_OK) return s;
  if (c->cinv_dirty) {
    if (coarse_dense(c)) {
      int l4 = -1;
      for (int l = c->top; l < c->nlev; ++l)
        if (c->lv[l].m == 4) l4 = l;
      if (l4 < 0 || !c->cinv) return fail(SPDE_EINVAL, "no 4^3 level for the exact coarse solve");
      HIPCHK(launch_coarse_inverse(c->fp64(), c->lv[l4], c->cinv, st));
    }
    c->cinv_dirty = false;
  }
  return SPDE_OK;
}

}  // namespace

// =============================================================================
// C interface

extern "C" {

spde_status spde_setup_box(int n, double kappa, double g, spde_handle* out) {
  if (!out) return fail(SPDE_EINVAL, "out is null");
  *out = nullptr;
  if (n < 4 || n > 1024 || (n & (n - 1))) return fail(SPDE_EINVAL, "n must be a power of two in [4, 1024], got %d", n);
  if (!(kappa > 0.0) || !std::isfinite(kappa)) return fail(SPDE_EINVAL, "kappa must be positive and finite");
  if (!(g > 0.0) || !std::isfinite(g)) return fail(SPDE_EINVAL, "g must be positive and finite");
  Ctx* c = new Ctx();
  c->n = n;
  c->kappa = kappa;
  c->kappa_pre = kappa;
  c->g = g;
  Box& b = c->box;
  b.n = n;
  b.n2 = (int64_t)n * n;
  b.nc = b.n2 * n;
  b.h = 1.0 / n;
  b.h2 = b.h * b.h;
  b.h3 = b.h2 * b.h;
  b.kappa = kappa;
  b.g = g;
  b.q = 1.5 / b.h3;
  b.k2h3 = kappa * kappa * b.h3;
  b.h15 = std::pow(b.h, 1.5);
  b.kap = nullptr;
  b.gfld = nullptr;
  b.h2q = b.h2 * b.q;
  *out = reinterpret_cast<spde_handle>(c);
  return SPDE_OK;
}

spde_status spde_configure(spde_handle h, spde_precision prec, double rtol, int max_iter, int max_batch) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (prec != SPDE_FP64 && prec != SPDE_MIXED) return fail(SPDE_EINVAL, "unknown precision %d", (int)prec);
  if (!(rtol > 0.0 && rtol < 1.0)) return fail(SPDE_EINVAL, "rtol must lie in (0, 1)");
  if (max_iter < 1 || max_iter > 100000) return fail(SPDE_EINVAL, "max_iter must lie in [1, 100000]");
  if (max_batch < 1 || max_batch > 4096) return fail(SPDE_EINVAL, "max_batch must lie in [1, 4096]");
  drop_graphs(c);
  c->prec = prec;
  c->rtol = rtol;
  c->max_iter = max_iter;
  c->max_batch = max_batch;
  c->configured = true;
  c->box.poly = c->face_precond;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->tuned = false;
  plan_hierarchy(c);
  return SPDE_OK;
}

spde_status spde_set_coefficients(spde_handle h, const double* kappa_dev, const double* g_dev, double kappa_ref) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (kappa_ref != 0.0 && !(kappa_ref > 0.0 && std::isfinite(kappa_ref)))
    return fail(SPDE_EINVAL, "kappa_ref must be 0 or positive and finite");
  drop_graphs(c);   // kernel arguments change
  c->box.kap = kappa_dev;
  c->box.gfld = g_dev;
  // kappa field with kappa_ref = 0: the multigrid takes the cell-wise kappa
  // (its level diagonals are built before the next solve); otherwise one
  // constant kappa
  c->mg_cellwise = kappa_dev && kappa_ref == 0.0;
  c->mg_dirty = c->mg_cellwise;
  c->kappa_pre = kappa_ref > 0.0 ? kappa_ref : c->kappa;
  // new level coefficients of the preconditioner; shapes, tiles and layout stay
  for (int l = 0; l < c->nlev; ++l) set_level(c->lv[l], c->lv[l].m, c->kappa_pre);
  for (int l = c->top; l < c->nlev; ++l) c->cp.lv[l - c->top] = c->lv[l];
  c->cinv_dirty = true;
  return SPDE_OK;
}

// Bytes the layout needs, leaving the handle's bound pointers as they are
// (a size-only layout sets every pointer it lays out to null).
size_t workspace_size(Ctx* c) {
  const Fields F = c->F;
  void* mgb[kMaxLevels];
  void* mge[kMaxLevels];
  void* mgd[kMaxLevels];
  void* mgdi[kMaxLevels];
  std::copy(c->mgb, c->mgb + kMaxLevels, mgb);
  std::copy(c->mge, c->mge + kMaxLevels, mge);
  std::copy(c->mgd, c->mgd + kMaxLevels, mgd);
  std::copy(c->mgdi, c->mgdi + kMaxLevels, mgdi);
  void* cinv = c->cinv;
  const void* cp_cinv = c->cp.cinv;
  double* resid_out = c->resid_out;
  const size_t need = layout(c, nullptr);
  c->F = F;
  std::copy(mgb, mgb + kMaxLevels, c->mgb);
  std::copy(mge, mge + kMaxLevels, c->mge);
  std::copy(mgd, mgd + kMaxLevels, c->mgd);
  std::copy(mgdi, mgdi + kMaxLevels, c->mgdi);
  c->cinv = cinv;
  c->cp.cinv = cp_cinv;
  c->resid_out = resid_out;
  return need;
}

size_t spde_workspace_bytes(spde_handle h) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c || !c->configured) return 0;
  return workspace_size(c);
}

spde_status spde_bind_workspace(spde_handle h, void* dev_ptr, size_t bytes) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!c->configured) return fail(SPDE_EINVAL, "spde_configure has not been called");
  if (!dev_ptr) return fail(SPDE_EINVAL, "workspace pointer is null");
  if ((uintptr_t)dev_ptr & 255) return fail(SPDE_EINVAL, "workspace must be 256-byte aligned");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (c->device != dev) {
    if (c->own_stream) { hipStreamDestroy(c->own_stream); c->own_stream = nullptr; }
    if (c->aux_stream) { hipStreamDestroy(c->aux_stream); c->aux_stream = nullptr; }
    if (c->ev_fork) { hipEventDestroy(c->ev_fork); c->ev_fork = nullptr; }
    if (c->ev_join) { hipEventDestroy(c->ev_join); c->ev_join = nullptr; }
    c->device = dev;
    int lds = 65536;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
      c->lds_limit = lds;
    HIPCHK(hipStreamCreate(&c->own_stream));
    // default priority, like every stream of the library
    HIPCHK(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    if (!c->host_sc) HIPCHK(hipHostMalloc((void**)&c->host_sc, 4096 * sizeof(Scalars), hipHostMallocDefault));
    if (!c->host_res) HIPCHK(hipHostMalloc((void**)&c->host_res, 4096 * sizeof(double), hipHostMallocDefault));
  }
  drop_graphs(c);
  plan_hierarchy(c);
  const size_t need = workspace_size(c);
  if (bytes < need) return fail(SPDE_ENOMEM, "workspace has %zu bytes, %zu needed", bytes, need);
  layout(c, (char*)dev_ptr);
  c->ws = (char*)dev_ptr;
  c->ws_bytes = bytes;
  HIPCHK(prepare_coarse(c->fp64(), c->coarse_lds));
  return SPDE_OK;
}

spde_status spde_build_transfer(spde_handle h, int64_t n_vert, const double* xyz_host, int64_t n_tet,
                                const int32_t* tet_host, int64_t** row_ptr_host, int32_t** col_host,
                                double** val_host, int64_t* nnz) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!xyz_host || !tet_host || !row_ptr_host || !col_host || !val_host || !nnz)
    return fail(SPDE_EINVAL, "null argument");
  if (n_vert < 4 || n_tet < 1) return fail(SPDE_EINVAL, "empty mesh");
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> cv;
  char err[256] = {0};
  if (build_transfer_csr(c->n, n_vert, xyz_host, n_tet, tet_host, rp, ci, cv, err, sizeof err) != 0)
    return fail(SPDE_EINVAL, "%s", err);
  *row_ptr_host = (int64_t*)malloc(rp.size() * sizeof(int64_t));
  *col_host = (int32_t*)malloc(std::max<size_t>(1, ci.size()) * sizeof(int32_t));
  *val_host = (double*)malloc(std::max<size_t>(1, cv.size()) * sizeof(double));
  if (!*row_ptr_host || !*col_host || !*val_host) return fail(SPDE_ENOMEM, "host allocation failed");
  memcpy(*row_ptr_host, rp.data(), rp.size() * sizeof(int64_t));
  memcpy(*col_host, ci.data(), ci.size() * sizeof(int32_t));
  memcpy(*val_host, cv.data(), cv.size() * sizeof(double));
  *nnz = (int64_t)ci.size();
  return SPDE_OK;
}

spde_status spde_transfer_coarsen(int n_fine, int64_t n_rows, const int64_t* row_ptr_host, const int32_t* col_host,
                                  const double* val_host, int64_t** row_ptr_c, int32_t** col_c, double** val_c,
                                  int64_t* nnz_c) {
  if (n_fine < 2 || n_fine > 1024 || (n_fine & 1)) return fail(SPDE_EINVAL, "n_fine must be even in [2, 1024]");
  if (n_rows < 1 || !row_ptr_host || !row_ptr_c || !col_c || !val_c || !nnz_c)
    return fail(SPDE_EINVAL, "null argument or empty matrix");
  if (row_ptr_host[n_rows] > 0 && (!col_host || !val_host)) return fail(SPDE_EINVAL, "null column or value array");
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> cv;
  char err[256] = {0};
  if (coarsen_transfer_csr(n_fine, n_rows, row_ptr_host, col_host, val_host, rp, ci, cv, err, sizeof err) != 0)
    return fail(SPDE_EINVAL, "%s", err);
  *row_ptr_c = (int64_t*)malloc(rp.size() * sizeof(int64_t));
  *col_c = (int32_t*)malloc(std::max<size_t>(1, ci.size()) * sizeof(int32_t));
  *val_c = (double*)malloc(std::max<size_t>(1, cv.size()) * sizeof(double));
  if (!*row_ptr_c || !*col_c || !*val_c) return fail(SPDE_ENOMEM, "host allocation failed");
  memcpy(*row_ptr_c, rp.data(), rp.size() * sizeof(int64_t));
  memcpy(*col_c, ci.data(), ci.size() * sizeof(int32_t));
  memcpy(*val_c, cv.data(), cv.size() * sizeof(double));
  *nnz_c = (int64_t)ci.size();
  return SPDE_OK;
}

namespace {

spde_status check_device_mesh(int n, int64_t n_vert, const double* xyz_dev, int64_t n_tet, const int32_t* tet_dev) {
  if (n < 2 || n > 1024) return fail(SPDE_EINVAL, "n must lie in [2, 1024], got %d", n);
  if (n_vert < 4 || n_vert > INT32_MAX || n_tet < 1 || n_tet > INT32_MAX)
    return fail(SPDE_EINVAL, "mesh sizes out of range (n_vert %lld, n_tet %lld)", (long long)n_vert, (long long)n_tet);
  if (!xyz_dev || !tet_dev) return fail(SPDE_EINVAL, "null mesh array");
  return SPDE_OK;
}

}  // namespace

spde_status spde_build_transfer_device_rows(int n, int64_t n_vert, const double* xyz_dev, int64_t n_tet,
                                            const int32_t* tet_dev, int64_t* row_ptr_dev, int64_t* nnz,
                                            void* stream) {
  spde_status s = check_device_mesh(n, n_vert, xyz_dev, n_tet, tet_dev);
  if (s != SPDE_OK) return s;
  if (!row_ptr_dev || !nnz) return fail(SPDE_EINVAL, "null row_ptr or nnz");
  const hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_transfer_rows(n, xyz_dev, n_vert, tet_dev, n_tet, row_ptr_dev, st));
  int64_t last = 0;
  HIPCHK(hipMemcpyAsync(&last, row_ptr_dev + n_tet, sizeof last, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (last < 0) {
    const int64_t b = -last - 1, t = b / 4;
    const int code = (int)(b % 4);
    const char* what = code == 1 ? "references a vertex out of range"
                       : code == 2 ? "has a vertex outside [0,1]^3" : "is degenerate (zero volume)";
    return fail(SPDE_EINVAL, "tet %lld %s", (long long)t, what);
  }
  *nnz = last;
  return SPDE_OK;
}

spde_status spde_build_transfer_device_fill(int n, int64_t n_vert, const double* xyz_dev, int64_t n_tet,
                                            const int32_t* tet_dev, const int64_t* row_ptr_dev, int32_t* col_dev,
                                            double* val_dev, void* stream) {
  spde_status s = check_device_mesh(n, n_vert, xyz_dev, n_tet, tet_dev);
  if (s != SPDE_OK) return s;
  if (!row_ptr_dev || !col_dev || !val_dev) return fail(SPDE_EINVAL, "null row_ptr, col or val");
  HIPCHK(launch_transfer_fill(n, xyz_dev, n_vert, tet_dev, n_tet, row_ptr_dev, col_dev, val_dev, (hipStream_t)stream));
  return SPDE_OK;
}

spde_status spde_set_transfer(spde_handle h, int64_t n_tet, int64_t nnz, const int64_t* row_ptr_dev,
                              const int32_t* col_dev, const double* val_dev) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (n_tet < 1 || nnz < 0 || !row_ptr_dev || (nnz > 0 && (!col_dev || !val_dev)))
    return fail(SPDE_EINVAL, "invalid transfer matrix");
  c->n_tet = n_tet;
  c->nnz = nnz;
  c->order = nullptr;
  c->uptr = nullptr;
  c->ucells = nullptr;
  c->lcol = nullptr;
  c->rp = row_ptr_dev;
  c->ci = col_dev;
  c->cv = val_dev;
  return SPDE_OK;
}

namespace {

// Where a sample's noise comes from: device memory, or the counter-based
// generator (events event0, event0 + 1, ... of `seed`; coupled = the
// restriction of each event's (2n)^3 field).
struct NoiseSrc {
  const double* xi = nullptr;
  uint64_t seed = 0, event0 = 0;
  int coupled = 0;
};

spde_status check_noise_grid(const Ctx* c, int coupled) {
  if (!coupled && (c->n % 4)) return fail(SPDE_EINVAL, "generated noise needs n divisible by 4, got %d", c->n);
  if (coupled && (c->n % 2)) return fail(SPDE_EINVAL, "coupled noise needs an even n, got %d", c->n);
  return SPDE_OK;
}

// u_tet = Pi u for a batch of box fields, the samples staged sample-minor in
// the second Lanczos face buffer (free between solves; 3 batch n^3 doubles
// hold any sample block), with the algorithmic bytes of each launch:
// staging reads the block's fields and writes the staged block, the gather
// reads the CSR once per sample block, the staged fields and writes u_tet.
spde_status enqueue_transfer(Ctx* c, int batch, const double* u, double* u_tet, hipStream_t st) {
  const int bp = spmm_block(batch);
  const double nc = (double)c->box.nc, nt = (double)c->n_tet;
  const double csr = 8.0 * (nt + 1.0) + 12.0 * (double)c->nnz;
  double* scratch = c->F.vs[1];
  for (int s0 = 0; s0 < batch; s0 += bp) {
    const int nb = std::min(bp, batch - s0);
    if (bp > 1) {
      Timed t(c, KID_SPMM_STAGE, 0, st, 0, s0, nb, 8.0 * nc * (nb + bp));
      HIPCHK(launch_spmm_stage(u, scratch, c->box.nc, batch, s0, st));
    }
    if (c->uptr && (bp == 32 || bp == 64) &&
        spmm_units_lds(bp, c->u_max_cells, c->u_max_entries) <= kSpmmUnitLds) {
      // the unit lists replace the column indices: 2 B per entry, 4 B per listed cell
      const double units = 8.0 * (nt + 1.0) + 10.0 * (double)c->nnz + 4.0 * (double)c->u_cells;
      Timed t(c, KID_SPMM, 0, st, 0, s0, nb, units + 8.0 * nb * (nc + nt));
      HIPCHK(launch_spmm_units(c->rp, c->cv, c->uptr, c->ucells, c->lcol, scratch, u_tet, c->n_tet, c->nnz,
                               c->box.nc, batch, s0, c->order, c->u_max_cells, c->u_max_entries, st));
      continue;
    }
    Timed t(c, KID_SPMM, 0, st, 0, s0, nb, csr + 8.0 * nb * (nc + nt));
    HIPCHK(launch_spmm_gather(c->rp, c->ci, c->cv, u, scratch, u_tet, c->n_tet, c->nnz, c->box.nc, batch, s0,
                              c->order, st));
  }
  return SPDE_OK;
}

spde_status sample_impl(Ctx* c, int batch, const NoiseSrc& src, double* u_tet_dev, double* u_box_dev,
                        double* sigma_dev, void* stream, int* iters_host, double* relres_host,
                        const double* warm_uc = nullptr) {
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (batch < 1) return fail(SPDE_EINVAL, "batch must be >= 1");
  if (batch > c->max_batch) return fail(SPDE_ENOMEM, "batch %d exceeds max_batch %d", batch, c->max_batch);
  if (u_tet_dev && !c->rp) return fail(SPDE_EINVAL, "u_tet requested but no transfer set");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  const Box& bx = c->box;
  const double scale = -c->g * std::pow(bx.h, 1.5);
  s = autotune(c, st);
  if (s != SPDE_OK) return s;
  s = prepare_mg_coeffs(c, st);
  if (s != SPDE_OK) return s;
  // the load F_u: the caller's noise, or the generated noise drawn again into
  // a Lanczos buffer that no running solve uses
  const double* xi_res = src.xi;
  auto load_for_residual = [&]() -> spde_status {
    if (!src.xi) {
      HIPCHK(launch_noise(bx.n, src.coupled, src.seed, src.event0, batch, c->F.vu[0], st));
      xi_res = c->F.vu[0];
    }
    return SPDE_OK;
  };
  // True residual r = F - A U of the current U = x, with the flux recovered
  // from U (so only the cell row is nonzero): ||r|| / ||F|| into host_res, and
  // r into vu[1], the load of a correction solve.
  auto residual = [&]() -> spde_status {
    spde_status s2 = load_for_residual();
    if (s2 != SPDE_OK) return s2;
    {
      Timed t(c, KID_FLUX, 0, st);
      HIPCHK(launch_flux(c->F.x, c->F.vs[0], nullptr, bx, batch, st));
    }
    {
      Timed t(c, KID_RESID, 0, st);
      HIPCHK(launch_resid(c->F.vs[0], c->F.x, xi_res, scale, bx, batch, c->F.part_pb, c->resid_out, c->F.vu[1],
                          st));
    }
    HIPCHK(hipMemcpyAsync(c->host_res, c->resid_out, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return SPDE_OK;
  };
  if (!warm_uc) {
    // the noise read (none when drawn), three face arrays and the cell array written
    Timed t(c, KID_INIT, 0, st, 0, 0, batch, (src.xi ? 40.0 : 32.0) * (double)bx.nc * batch);
    if (src.xi) HIPCHK(launch_init(c->F, bx, src.xi, scale, batch, c->rtol, c->max_iter, 0, st));
    else
      HIPCHK(launch_init_gen(c->F, bx, src.seed, src.event0, src.coupled, scale, batch, c->rtol, c->max_iter, 0,
                             st));
  } else {
    // Warm start from the coupled coarse solution: U0 = P u_c, then one
    // correction solve on r0 = F - A U0 that adds to x, stopped where the cold
    // solve would stop relative to F: its tolerance is rtol ||F|| / ||r0||.
    HIPCHK(launch_inject_coarse(warm_uc, c->F.x, bx.n, batch, st));
    s = residual();
    if (s != SPDE_OK) return s;
    // each sample's own tolerance, so that its result does not depend on the batch
    for (int b = 0; b < batch; ++b) {
      const double r0 = c->host_res[b];
      c->host_res[b] = std::isfinite(r0) && r0 > 0.0 ? std::min(0.5, std::max(c->rtol, c->rtol / r0)) : c->rtol;
    }
    HIPCHK(hipMemcpyAsync(c->resid_out, c->host_res, batch * sizeof(double), hipMemcpyHostToDevice, st));
    // three face arrays of v_1 cleared (the cell part was written by the residual pass)
    Timed t(c, KID_INIT, 0, st, 0, 0, batch, 24.0 * (double)bx.nc * batch);
    HIPCHK(launch_init_correction(c->F, bx, batch, c->resid_out, c->max_iter, st));
  }
  const bool graphs = c->use_graphs && c->timing != 1 && st != nullptr;
  // A batch of 8 or more runs as two halves on two streams, so that the
  // memory-bound operator pass of one half can overlap the compute-bound
  // V-cycle of the other and each fills the other's launch tails.  The halves
  // are independent samples; they meet at every convergence poll.
  const bool split = c->split >= 2 && batch >= 8 && c->aux_stream && st != nullptr;
  const int b1 = split ? (batch + 1) / 2 : batch;
  const View V0 = make_view(c, 0), V1 = make_view(c, b1);
  if (split) {
    HIPCHK(hipEventRecord(c->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(c->aux_stream, c->ev_fork, 0));
  }
  // MINRES iterations in blocks of the poll interval until no sample is active.
  // expect: iterations the previous call needed (0: unknown); the block that
  // would pass it stops there, so that a batch like the last one is not
  // carried through idle iterations.
  auto iterate = [&](int expect, int& launched) -> spde_status {
    launched = 0;
    const int cap = c->max_iter + 2;
    bool all_done = false;
    while (!all_done && launched < cap + c->poll) {
      int count = c->poll;
      if (expect > launched) count = std::min(count, expect - launched);
      spde_status s2 = enqueue_block(c, V0, b1, st, graphs, launched, count);
      if (s2 != SPDE_OK) return s2;
      if (split) {
        s2 = enqueue_block(c, V1, batch - b1, c->aux_stream, graphs, launched, count);
        if (s2 != SPDE_OK) return s2;
        HIPCHK(hipEventRecord(c->ev_join, c->aux_stream));
        HIPCHK(hipStreamWaitEvent(st, c->ev_join, 0));
      }
      launched += count;
      HIPCHK(hipMemcpyAsync(c->host_sc, c->F.sc, batch * sizeof(Scalars), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      all_done = true;
      for (int b = 0; b < batch; ++b) {
        if (c->host_sc[b].state == ST_ACTIVE) { all_done = false; break; }
      }
    }
    return SPDE_OK;
  };
  int launched = 0;
  s = iterate(c->expect_iters, launched);
  if (s != SPDE_OK) return s;
  bool notconv = false, failed = false;
  int most = 0;
  std::vector<int> total(batch, 0);
  std::vector<char> bad(batch, 0);   // samples that failed: excluded from refinement
  for (int b = 0; b < batch; ++b) {
    const Scalars& sc = c->host_sc[b];
    if (sc.state == ST_FAILED) { failed = true; bad[b] = 1; }
    if (sc.state == ST_ACTIVE || (sc.flags & FL_NOTCONV)) notconv = true;
    total[b] = sc.state == ST_ACTIVE ? launched : sc.iters;
    if (sc.state == ST_FINISH || sc.state == ST_DONE) most = std::max(most, sc.iters);
  }
  // a converged sample needs its iterations plus the finishing pass
  c->expect_iters = (!notconv && !failed && most > 0) ? most + 1 : 0;
  HIPCHK(launch_fix_solution(c->F, bx, batch, 0, st));
  // Iterative refinement in float64: with r = F - A U (flux recovered from U,
  // so only the cell row is nonzero), solve A d = r by the same MINRES and set
  // U += d, for the samples whose relative true residual exceeds the target.
  // A failed sample (its field is NaN) is left out of every pass; the others
  // are refined as if it were not in the batch.
  bool res_final = false;   // host_res holds the residual of the current U
  if (c->refine_target > 0.0) {
    for (int pass = 0;; ++pass) {
      s = residual();
      if (s != SPDE_OK) return s;
      res_final = true;
      std::vector<char> refine(batch, 0);
      bool need_any = false;
      for (int b = 0; b < batch; ++b) {
        if (bad[b] || c->host_res[b] <= c->refine_target) continue;
        refine[b] = 1;
        need_any = true;
      }
      if (!need_any || pass >= c->refine_max) break;
      // A sample's pass has to reduce its residual by target / residual only (a
      // factor of 2 to spare: the true residual of a pass ends a few times
      // below its MINRES estimate, and a sample left above the target takes
      // another pass of its own), never tighter than the configured rtol, which
      // the preconditioned MINRES is known to reach.  Each sample takes its own
      // tolerance, so that its result does not depend on the batch.
      std::vector<double> tols(batch);
      for (int b = 0; b < batch; ++b) {
        const double r = c->host_res[b];
        tols[b] = refine[b] && std::isfinite(r) && r > 0.0
                      ? std::min(0.5, std::max(c->rtol, 0.5 * c->refine_target / r))
                      : c->rtol;
      }
      std::copy(tols.begin(), tols.end(), c->host_res);
      HIPCHK(hipMemcpyAsync(c->resid_out, c->host_res, batch * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(launch_init_correction(c->F, bx, batch, c->resid_out, c->max_iter, st));
      for (int b = 0; b < batch; ++b)
        if (!refine[b]) HIPCHK(launch_set_state(c->F.sc, b, 1, ST_DONE, st));
      if (split) {   // the second stream's half starts after the pass's set-up
        HIPCHK(hipEventRecord(c->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(c->aux_stream, c->ev_fork, 0));
      }
      int lp = 0;
      s = iterate(0, lp);
      if (s != SPDE_OK) return s;
      bool more = false;
      for (int b = 0; b < batch; ++b) {
        if (!refine[b]) continue;   // not refined in this pass
        const Scalars& sc = c->host_sc[b];
        if (sc.state == ST_FAILED) { failed = true; bad[b] = 1; }
        else more = true;
        if (sc.state == ST_ACTIVE || (sc.flags & FL_NOTCONV)) notconv = true;
        total[b] += sc.state == ST_ACTIVE ? lp : sc.iters;
      }
      // samples that failed in this pass get a NaN field; the others keep
      // their refined iterate
      HIPCHK(launch_fix_solution(c->F, bx, batch, 0, st));
      res_final = false;
      if (!more) break;
    }
  }
  if (iters_host)
    for (int b = 0; b < batch; ++b) iters_host[b] = total[b];
  if (u_box_dev) HIPCHK(hipMemcpyAsync(u_box_dev, c->F.x, (size_t)batch * bx.nc * 8, hipMemcpyDeviceToDevice, st));
  // (after refinement host_res already holds the residual of the final U)
  const bool need_res = relres_host && !res_final;
  if (sigma_dev || need_res) {
    double* sig_int = need_res ? c->F.vs[0] : nullptr;
    {
      Timed t(c, KID_FLUX, 0, st);
      HIPCHK(launch_flux(c->F.x, sig_int, sigma_dev, bx, batch, st));
    }
    if (need_res) {
      s = load_for_residual();
      if (s != SPDE_OK) return s;
      {
        Timed t(c, KID_RESID, 0, st);
        HIPCHK(launch_resid(sig_int, c->F.x, xi_res, scale, bx, batch, c->F.part_pb, c->resid_out, nullptr, st));
      }
      HIPCHK(hipMemcpyAsync(c->host_res, c->resid_out, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    }
  }
  if (u_tet_dev) {
    s = enqueue_transfer(c, batch, c->F.x, u_tet_dev, st);
    if (s != SPDE_OK) return s;
  }
  if (relres_host || c->timing) {
    HIPCHK(hipStreamSynchronize(st));
    if (relres_host) for (int b = 0; b < batch; ++b) relres_host[b] = c->host_res[b];
  }
  close_timing(c, batch);
  if (failed) return fail(SPDE_EFAILED, "breakdown or non-finite value in some sample");
  if (notconv) return fail(SPDE_ENOTCONV, "max_iter reached for some sample");
  return SPDE_OK;
}

}  // namespace

spde_status spde_sample(spde_handle h, int batch, const double* xi_dev, double* u_tet_dev, double* u_box_dev,
                        double* sigma_dev, void* stream, int* iters_host, double* relres_host) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!xi_dev) return fail(SPDE_EINVAL, "xi is null");
  NoiseSrc src;
  src.xi = xi_dev;
  return sample_impl(c, batch, src, u_tet_dev, u_box_dev, sigma_dev, stream, iters_host, relres_host);
}

spde_status spde_sample_warm(spde_handle h, int batch, const double* xi_dev, const double* u_coarse_dev,
                             int64_t u_coarse_count, double* u_tet_dev, double* u_box_dev, double* sigma_dev,
                             void* stream, int* iters_host, double* relres_host) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!xi_dev || !u_coarse_dev) return fail(SPDE_EINVAL, "xi or u_coarse is null");
  const int64_t mc = c->n / 2;
  if (batch >= 1 && u_coarse_count != (int64_t)batch * mc * mc * mc)
    return fail(SPDE_EINVAL, "u_coarse holds %lld values, %d samples of (n/2)^3 = %lld need %lld",
                (long long)u_coarse_count, batch, (long long)(mc * mc * mc), (long long)(batch * mc * mc * mc));
  NoiseSrc src;
  src.xi = xi_dev;
  return sample_impl(c, batch, src, u_tet_dev, u_box_dev, sigma_dev, stream, iters_host, relres_host, u_coarse_dev);
}

spde_status spde_sample_seeded(spde_handle h, int batch, uint64_t seed, uint64_t event0, int coupled,
                               double* u_tet_dev, double* u_box_dev, double* sigma_dev, void* stream,
                               int* iters_host, double* relres_host) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (coupled != 0 && coupled != 1) return fail(SPDE_EINVAL, "coupled must be 0 or 1");
  spde_status s = check_noise_grid(c, coupled);
  if (s != SPDE_OK) return s;
  NoiseSrc src;
  src.seed = seed;
  src.event0 = event0;
  src.coupled = coupled;
  return sample_impl(c, batch, src, u_tet_dev, u_box_dev, sigma_dev, stream, iters_host, relres_host);
}

spde_status spde_noise(int n, int coupled, uint64_t seed, uint64_t event0, int batch, double* xi_dev,
                       void* stream) {
  if (coupled != 0 && coupled != 1) return fail(SPDE_EINVAL, "coupled must be 0 or 1");
  if (n < 2 || n > 1024) return fail(SPDE_EINVAL, "n must lie in [2, 1024], got %d", n);
  if (!coupled && (n % 4)) return fail(SPDE_EINVAL, "generated noise needs n divisible by 4, got %d", n);
  if (coupled && (n % 2)) return fail(SPDE_EINVAL, "coupled noise needs an even n, got %d", n);
  if (batch < 1 || batch > 65535) return fail(SPDE_EINVAL, "batch must lie in [1, 65535]");
  if (!xi_dev) return fail(SPDE_EINVAL, "xi is null");
  HIPCHK(launch_noise(n, coupled, seed, event0, batch, xi_dev, (hipStream_t)stream));
  return SPDE_OK;
}

spde_status spde_philox4x64(uint64_t seed, uint64_t event, uint64_t ctr0, uint64_t ctr1, int64_t nblocks,
                            uint64_t* out_dev, void* stream) {
  if (nblocks < 1 || nblocks > ((int64_t)1 << 36)) return fail(SPDE_EINVAL, "nblocks out of range");
  if (!out_dev) return fail(SPDE_EINVAL, "out is null");
  HIPCHK(launch_philox_raw(seed, event, ctr0, ctr1, nblocks, out_dev, (hipStream_t)stream));
  return SPDE_OK;
}

// ---- continuous batching ----------------------------------------------------

spde_status spde_slots_reset(spde_handle h, int nslots, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (nslots < 1 || nslots > c->max_batch) return fail(SPDE_EINVAL, "nslots out of range");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  s = autotune(c, st);
  if (s != SPDE_OK) return s;
  s = prepare_mg_coeffs(c, st);
  if (s != SPDE_OK) return s;
  HIPCHK(launch_set_state(c->F.sc, 0, nslots, ST_IDLE, st));
  return SPDE_OK;
}

spde_status spde_slot_start(spde_handle h, int slot, const double* xi_dev, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (slot < 0 || slot >= c->max_batch) return fail(SPDE_EINVAL, "slot out of range");
  if (!xi_dev) return fail(SPDE_EINVAL, "xi is null");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  const double scale = -c->g * std::pow(c->box.h, 1.5);
  HIPCHK(launch_init(c->F, c->box, xi_dev, scale, 1, c->rtol, c->max_iter, slot, st));
  return SPDE_OK;
}

spde_status spde_slot_start_seeded(spde_handle h, int slot, uint64_t seed, uint64_t event, int coupled,
                                   void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (slot < 0 || slot >= c->max_batch) return fail(SPDE_EINVAL, "slot out of range");
  if (coupled != 0 && coupled != 1) return fail(SPDE_EINVAL, "coupled must be 0 or 1");
  s = check_noise_grid(c, coupled);
  if (s != SPDE_OK) return s;
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  const double scale = -c->g * std::pow(c->box.h, 1.5);
  HIPCHK(launch_init_gen(c->F, c->box, seed, event, coupled, scale, 1, c->rtol, c->max_iter, slot, st));
  return SPDE_OK;
}

spde_status spde_slots_step(spde_handle h, int nslots, int iters, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (nslots < 1 || nslots > c->max_batch) return fail(SPDE_EINVAL, "nslots out of range");
  if (iters < 1) return fail(SPDE_EINVAL, "iters must be >= 1");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  const bool graphs = c->use_graphs && c->timing != 1 && st != nullptr;
  int done = 0;
  const View V0 = make_view(c, 0);
  while (done < iters) {
    hipGraphExec_t ex = nullptr;
    if (graphs && iters - done >= c->poll && get_graph(c, V0, nslots, st, &ex, 2 * c->poll) != SPDE_OK) {
      hipGetLastError();
      c->use_graphs = false;
      ex = nullptr;
    }
    if (ex) {
      HIPCHK(hipGraphLaunch(ex, st));
      done += c->poll;
    } else {
      s = enqueue_iteration(c, V0, nslots, st, 0);
      if (s != SPDE_OK) return s;
      done += 1;
    }
  }
  return SPDE_OK;
}

spde_status spde_slots_poll(spde_handle h, int nslots, int* state_host, int* iters_host, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (nslots < 1 || nslots > c->max_batch) return fail(SPDE_EINVAL, "nslots out of range");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  HIPCHK(hipMemcpyAsync(c->host_sc, c->F.sc, nslots * sizeof(Scalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < nslots; ++i) {
    const Scalars& v = c->host_sc[i];
    int code;
    switch (v.state) {
      case ST_ACTIVE: code = 0; break;
      case ST_FINISH:
      case ST_DONE: code = (v.flags & FL_NOTCONV) ? 2 : 1; break;
      case ST_FAILED: code = 3; break;
      default: code = 4;
    }
    if (state_host) state_host[i] = code;
    if (iters_host) iters_host[i] = v.iters;
  }
  return SPDE_OK;
}

spde_status spde_slot_finish(spde_handle h, int slot, double* u_box_dev, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (slot < 0 || slot >= c->max_batch) return fail(SPDE_EINVAL, "slot out of range");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  HIPCHK(launch_fix_solution(c->F, c->box, 1, slot, st));
  if (u_box_dev)
    HIPCHK(hipMemcpyAsync(u_box_dev, c->F.x + cell_off(slot, c->box.nc), c->box.nc * 8, hipMemcpyDeviceToDevice,
                          st));
  HIPCHK(launch_set_state(c->F.sc, slot, 1, ST_IDLE, st));
  return SPDE_OK;
}

size_t spde_csr_apply_work_bytes(int64_t n_cols, int batch) {
  if (n_cols < 1 || batch < 1) return 0;
  return spmm_scratch_bytes(n_cols, batch);
}

spde_status spde_csr_apply(int64_t n_rows, int64_t nnz, const int64_t* rp, const int32_t* ci, const double* cv,
                           int64_t n_cols, int batch, const double* x_dev, double* y_dev,
                           const int32_t* chunk_order_dev, void* work_dev, size_t work_bytes, void* stream) {
  if (n_rows < 1 || nnz < 0 || n_cols < 1 || batch < 1) return fail(SPDE_EINVAL, "invalid sizes");
  if (!rp || !x_dev || !y_dev || (nnz > 0 && (!ci || !cv))) return fail(SPDE_EINVAL, "null pointer");
  const size_t need = spmm_scratch_bytes(n_cols, batch);
  if (need && (!work_dev || work_bytes < need))
    return fail(SPDE_EINVAL, "work buffer has %zu bytes, %zu needed for batch %d", work_dev ? work_bytes : 0, need,
                batch);
  if (need && ((uintptr_t)work_dev & 255)) return fail(SPDE_EINVAL, "work buffer must be 256-byte aligned");
  HIPCHK(launch_spmm(rp, ci, cv, x_dev, y_dev, n_rows, nnz, n_cols, batch, chunk_order_dev, (double*)work_dev,
                     (hipStream_t)stream));
  return SPDE_OK;
}

spde_status spde_csr_apply_noalloc(int64_t n_rows, int64_t nnz, const int64_t* rp, const int32_t* ci,
                                   const double* cv, int64_t n_cols, int batch, const double* x_dev, double* y_dev,
                                   const int32_t* chunk_order_dev, void* stream) {
  if (n_rows < 1 || nnz < 0 || n_cols < 1 || batch < 1) return fail(SPDE_EINVAL, "invalid sizes");
  if (!rp || !x_dev || !y_dev || (nnz > 0 && (!ci || !cv))) return fail(SPDE_EINVAL, "null pointer");
  const size_t need = spmm_scratch_bytes(n_cols, batch);
  if (need > kStaticScratchBytes)
    return fail(SPDE_EINVAL,
                "the staged sample block needs %zu bytes (%d samples x %lld columns), the static scratch holds %zu; "
                "use spde_csr_apply with a work buffer", need, spmm_block(batch), (long long)n_cols,
                kStaticScratchBytes);
  double* scratch_dev = nullptr;
  if (need) HIPCHK(static_scratch_ptr(&scratch_dev));
  HIPCHK(launch_spmm(rp, ci, cv, x_dev, y_dev, n_rows, nnz, n_cols, batch, chunk_order_dev, scratch_dev,
                     (hipStream_t)stream));
  return SPDE_OK;
}

size_t spde_csr_apply_noalloc_max_bytes(void) { return kStaticScratchBytes; }

spde_status spde_restrict_noise(int n_fine, int batch, const double* xi_f_dev, double* xi_c_dev, void* stream) {
  if (n_fine < 2 || (n_fine & 1)) return fail(SPDE_EINVAL, "n_fine must be even and >= 2");
  if (batch < 1) return fail(SPDE_EINVAL, "batch must be >= 1");
  if (!xi_f_dev || !xi_c_dev) return fail(SPDE_EINVAL, "null pointer");
  HIPCHK(launch_restrict_noise(xi_f_dev, xi_c_dev, n_fine, batch, (hipStream_t)stream));
  return SPDE_OK;
}

spde_status spde_apply_operator(spde_handle h, int batch, const double* x_sigma_dev, const double* x_u_dev,
                                double* y_sigma_dev, double* y_u_dev, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (batch < 1 || batch > c->max_batch) return fail(SPDE_EINVAL, "batch out of range");
  if (!x_sigma_dev || !x_u_dev || !y_sigma_dev || !y_u_dev) return fail(SPDE_EINVAL, "null pointer");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  Fields G = c->F;
  G.z[0] = G.w[0];            // a float64 cell buffer for zhat = x_u
  Box bd = c->box;
  bd.poly = 0;                // face block diag(M)^-1: the pass then computes A x itself
  HIPCHK(launch_ext_to_int(x_sigma_dev, x_u_dev, G, bd, batch, st));
  HIPCHK(launch_probe_scalars(G.sc, batch, st));
  HIPCHK(launch_operator(true, G, bd, batch, st));
  HIPCHK(launch_int_to_ext(G, y_sigma_dev, y_u_dev, bd, batch, st));
  return SPDE_OK;
}

spde_status spde_apply_operator_precond(spde_handle h, int batch, const double* x_sigma_dev, const double* x_u_dev,
                                        double* y_sigma_dev, double* y_u_dev, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (batch < 1 || batch > c->max_batch) return fail(SPDE_EINVAL, "batch out of range");
  if (!x_sigma_dev || !x_u_dev || !y_sigma_dev || !y_u_dev) return fail(SPDE_EINVAL, "null pointer");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  // v_sigma = diag(M) x_sigma and zhat = x_u in the solver's own buffers, so
  // that the pass forms z_sigma = P_f v_sigma with the handle's face block
  HIPCHK(launch_ext_to_int_zhat(x_sigma_dev, x_u_dev, c->F, c->box, batch, c->fp64(), st));
  HIPCHK(launch_probe_scalars(c->F.sc, batch, st));
  HIPCHK(launch_operator(c->fp64(), c->F, c->box, batch, st));
  HIPCHK(launch_int_to_ext(c->F, y_sigma_dev, y_u_dev, c->box, batch, st));
  return SPDE_OK;
}

spde_status spde_apply_vcycle(spde_handle h, int batch, const double* r_dev, double* z_dev, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (batch < 1 || batch > c->max_batch) return fail(SPDE_EINVAL, "batch out of range");
  if (!r_dev || !z_dev) return fail(SPDE_EINVAL, "null pointer");
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = pick_stream(c, stream);
  void* out = c->fp64() ? (void*)z_dev : c->F.z[0];
  s = autotune(c, st);
  if (s != SPDE_OK) return s;
  s = prepare_mg_coeffs(c, st);
  if (s != SPDE_OK) return s;
  // the finest up kernel always writes partial sums: give it the solver's buffer
  s = enqueue_vcycle(c, make_view(c, 0), batch, st, 0, r_dev, r_dev, out, out, nullptr, c->F.part_up);
  if (s != SPDE_OK) return s;
  if (!c->fp64()) HIPCHK(launch_f32_to_f64((const float*)c->F.z[0], z_dev, (int64_t)batch * c->box.nc, st));
  return SPDE_OK;
}

spde_status spde_apply_transfer(spde_handle h, int batch, const double* u_box_dev, double* u_tet_dev, void* stream) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  spde_status s = check_ready(c);
  if (s != SPDE_OK) return s;
  if (!c->rp) return fail(SPDE_EINVAL, "no transfer set");
  if (batch < 1 || batch > c->max_batch || !u_box_dev || !u_tet_dev) return fail(SPDE_EINVAL, "invalid argument");
  HIPCHK(hipSetDevice(c->device));
  return enqueue_transfer(c, batch, u_box_dev, u_tet_dev, pick_stream(c, stream));
}

int spde_transfer_chunk_rows(void) { return kSpmmChunk; }

spde_status spde_transfer_chunk_order(int n, int64_t n_rows, const int64_t* row_ptr_host, const int32_t* col_host,
                                      int32_t* order_host) {
  if (n < 1 || n > 1024) return fail(SPDE_EINVAL, "n must lie in [1, 1024]");
  if (n_rows < 1 || !row_ptr_host || !order_host) return fail(SPDE_EINVAL, "invalid argument");
  const int64_t nchunk = (n_rows + kSpmmChunk - 1) / kSpmmChunk;
  if (nchunk > INT32_MAX) return fail(SPDE_EINVAL, "too many rows");
  // key of a chunk: the cell of its first entry, ordered by 16 x 16 tile of
  // (x, y), then z, then y, then x; chunks without entries last
  const int64_t tiles = (n + 15) / 16;
  std::vector<std::pair<uint64_t, int32_t>> key(nchunk);
  for (int64_t q = 0; q < nchunk; ++q) {
    uint64_t k = UINT64_MAX;
    const int64_t r1 = std::min(n_rows, (q + 1) * kSpmmChunk);
    for (int64_t r = q * kSpmmChunk; r < r1 && col_host; ++r) {
      if (row_ptr_host[r + 1] > row_ptr_host[r]) {
        const int64_t c = col_host[row_ptr_host[r]];
        if (c < 0 || c >= (int64_t)n * n * n) break;
        const uint64_t i = c % n, j = (c / n) % n, kz = c / ((int64_t)n * n);
        const uint64_t tile = (i / 16) * tiles + j / 16;
        k = (tile << 30) | (kz << 20) | (j << 10) | i;
        break;
      }
    }
    key[q] = {k, (int32_t)q};
  }
  std::stable_sort(key.begin(), key.end());
  for (int64_t q = 0; q < nchunk; ++q) order_host[q] = key[q].second;
  return SPDE_OK;
}

spde_status spde_set_transfer_chunk_order(spde_handle h, const int32_t* order_dev) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!c->rp) return fail(SPDE_EINVAL, "no transfer set");
  c->order = order_dev;
  return SPDE_OK;
}

int spde_transfer_unit_rows(void) { return kSpmmUnit; }

spde_status spde_transfer_units(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr_host,
                                const int32_t* col_host, int64_t* unit_ptr_host, int32_t* unit_cells_host,
                                uint16_t* local_col_host, int32_t* max_cells, int32_t* max_entries) {
  if (n_rows < 1 || n_cols < 1 || !row_ptr_host || !unit_ptr_host || !max_cells || !max_entries)
    return fail(SPDE_EINVAL, "invalid argument");
  const bool fill = unit_cells_host != nullptr;
  if (fill != (local_col_host != nullptr)) return fail(SPDE_EINVAL, "unit_cells and local_col go together");
  const int64_t nnz = row_ptr_host[n_rows];
  if (row_ptr_host[0] != 0 || nnz < 0) return fail(SPDE_EINVAL, "row pointers must start at 0 and end at nnz");
  for (int64_t r = 0; r < n_rows; ++r)
    if (row_ptr_host[r + 1] < row_ptr_host[r]) return fail(SPDE_EINVAL, "row pointers decrease at row %lld", (long long)r);
  if (nnz > 0 && !col_host) return fail(SPDE_EINVAL, "null column array");
  const int64_t nunit = (n_rows + kSpmmUnit - 1) / kSpmmUnit;
  // units in parallel ranges; the first call counts, the second writes
  std::vector<int64_t> count(fill ? 0 : nunit);
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (nunit < 4096) nth = 1;
  std::vector<int32_t> mcs(nth, 0), mes(nth, 0);
  std::vector<int64_t> bad(nth, -1);
  std::vector<char> oom(nth, 0);
  auto work = [&](unsigned t) {
    try {
    std::vector<int32_t> cells;
    const int64_t u0 = nunit * t / nth, u1 = nunit * (t + 1) / nth;
    for (int64_t u = u0; u < u1; ++u) {
      const int64_t e0 = row_ptr_host[u * kSpmmUnit], e1 = row_ptr_host[std::min(n_rows, (u + 1) * kSpmmUnit)];
      cells.clear();
      for (int64_t k = e0; k < e1; ++k)
        if (col_host[k] >= 0 && col_host[k] < n_cols) cells.push_back(col_host[k]);
      std::sort(cells.begin(), cells.end());
      cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
      mcs[t] = std::max(mcs[t], (int32_t)cells.size());
      mes[t] = std::max(mes[t], (int32_t)(e1 - e0));
      if (!fill) {
        count[u] = (int64_t)cells.size();
        continue;
      }
      const int64_t off = unit_ptr_host[u];
      if (unit_ptr_host[u + 1] - off != (int64_t)cells.size()) {
        if (bad[t] < 0) bad[t] = u;
        continue;
      }
      std::copy(cells.begin(), cells.end(), unit_cells_host + off);
      for (int64_t k = e0; k < e1; ++k) {
        const int32_t col = col_host[k];
        local_col_host[k] = (col >= 0 && col < n_cols)
                                ? (uint16_t)(std::lower_bound(cells.begin(), cells.end(), col) - cells.begin())
                                : (uint16_t)65535;
      }
    }
    } catch (...) {
      oom[t] = 1;
    }
  };
  std::vector<std::thread> th;
  try {
    for (unsigned t = 1; t < nth; ++t) th.emplace_back(work, t);
  } catch (...) {
    // no more threads: the ranges not started run on this one
    for (unsigned t = (unsigned)th.size() + 1; t < nth; ++t) work(t);
  }
  work(0);
  for (auto& x : th) x.join();
  int32_t mc = 0, me = 0;
  for (unsigned t = 0; t < nth; ++t) {
    if (oom[t]) return fail(SPDE_ENOMEM, "out of host memory building the transfer units");
    mc = std::max(mc, mcs[t]);
    me = std::max(me, mes[t]);
    if (bad[t] >= 0) return fail(SPDE_EINVAL, "unit_ptr does not match the matrix (unit %lld)", (long long)bad[t]);
  }
  if (mc >= 65535) return fail(SPDE_EINVAL, "a unit references more than 65534 cells");
  if (!fill) {
    unit_ptr_host[0] = 0;
    for (int64_t u = 0; u < nunit; ++u) unit_ptr_host[u + 1] = unit_ptr_host[u] + count[u];
  }
  *max_cells = mc;
  *max_entries = me;
  return SPDE_OK;
}

spde_status spde_set_transfer_units(spde_handle h, const int64_t* unit_ptr_dev, const int32_t* unit_cells_dev,
                                    const uint16_t* local_col_dev, int32_t max_cells, int32_t max_entries) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!unit_ptr_dev || !unit_cells_dev || !local_col_dev) {
    c->uptr = nullptr;
    c->ucells = nullptr;
    c->lcol = nullptr;
    return SPDE_OK;
  }
  if (!c->rp) return fail(SPDE_EINVAL, "no transfer set");
  if (max_cells < 0 || max_entries < 0 || max_cells >= 65535)
    return fail(SPDE_EINVAL, "invalid unit maxima (%d cells, %d entries)", max_cells, max_entries);
  // the total of listed cells (for the byte model): the last unit pointer
  const int64_t nunit = (c->n_tet + kSpmmUnit - 1) / kSpmmUnit;
  int64_t total = 0;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpy(&total, unit_ptr_dev + nunit, sizeof(int64_t), hipMemcpyDeviceToHost));
  c->uptr = unit_ptr_dev;
  c->ucells = unit_cells_dev;
  c->lcol = local_col_dev;
  c->u_max_cells = max_cells;
  c->u_max_entries = max_entries;
  c->u_cells = total;
  return SPDE_OK;
}

spde_status spde_stream_create_cu_mask(int n_words, const uint32_t* mask, void** stream_out) {
  if (n_words < 1 || n_words > 64 || !mask || !stream_out) return fail(SPDE_EINVAL, "invalid CU mask");
  uint32_t any = 0;
  for (int w = 0; w < n_words; ++w) any |= mask[w];
  if (!any) return fail(SPDE_EINVAL, "the CU mask selects no compute unit");
  hipStream_t st = nullptr;
  HIPCHK(hipExtStreamCreateWithCUMask(&st, (uint32_t)n_words, mask));
  *stream_out = (void*)st;
  return SPDE_OK;
}

spde_status spde_stream_destroy(void* stream) {
  if (!stream) return fail(SPDE_EINVAL, "null stream");
  HIPCHK(hipStreamDestroy((hipStream_t)stream));
  return SPDE_OK;
}

spde_status spde_set_split(spde_handle h, int ways) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (ways != 1 && ways != 2) return fail(SPDE_EINVAL, "split must be 1 or 2");
  c->split = ways;
  return SPDE_OK;
}

spde_status spde_set_graphs(spde_handle h, int enable) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  c->use_graphs = enable != 0;
  return SPDE_OK;
}

spde_status spde_set_refinement(spde_handle h, double target, int max_passes) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (!(target >= 0.0 && target < 1.0)) return fail(SPDE_EINVAL, "refinement target must lie in [0, 1)");
  if (max_passes < 0 || max_passes > 16) return fail(SPDE_EINVAL, "refinement passes must lie in [0, 16]");
  c->refine_target = target;
  c->refine_max = target > 0.0 ? max_passes : 0;
  return SPDE_OK;
}

spde_status spde_set_face_preconditioner(spde_handle h, int kind) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (kind != 0 && kind != 1) return fail(SPDE_EINVAL, "face preconditioner must be 0 or 1");
  c->face_precond = kind;
  c->box.poly = kind;
  drop_graphs(c);
  return SPDE_OK;
}

spde_status spde_set_autotune(spde_handle h, int enable) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  c->autotune = enable != 0;
  c->tuned = false;
  if (c->configured) plan_hierarchy(c);
  drop_graphs(c);
  return SPDE_OK;
}

spde_status spde_set_tiles(spde_handle h, int level, int down_shape, int up_shape) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c || !c->configured) return fail(SPDE_EINVAL, "handle not configured");
  if (level < -1 || level >= c->top) return fail(SPDE_EINVAL, "level %d has no per-level kernels", level);
  if (!shape_ok_down(down_shape, c->fp64()) || !shape_ok_up(up_shape, c->fp64()))
    return fail(SPDE_EINVAL, "tile shape not available for this precision");
  for (int l = 0; l < c->top; ++l) {
    if (level == -1 || level == l) {
      c->shape_down[l] = down_shape;
      c->shape_up[l] = up_shape;
    }
  }
  c->autotune = false;
  c->tuned = true;
  drop_graphs(c);
  return SPDE_OK;
}

spde_status spde_get_tiles(spde_handle h, int level, int* down_shape, int* up_shape) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c || !c->configured) return fail(SPDE_EINVAL, "handle not configured");
  if (level < 0 || level >= c->top) return fail(SPDE_EINVAL, "level %d has no per-level kernels", level);
  if (down_shape) *down_shape = c->shape_down[level];
  if (up_shape) *up_shape = c->shape_up[level];
  return SPDE_OK;
}

spde_status spde_set_poll_interval(spde_handle h, int iters) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (iters < 1 || iters > 256) return fail(SPDE_EINVAL, "poll interval must lie in [1, 256]");
  if (iters != c->poll) drop_graphs(c);
  c->poll = iters;
  return SPDE_OK;
}

spde_status spde_timing(spde_handle h, int enable) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (enable < -1 || enable > 2) return fail(SPDE_EINVAL, "timing mode must be -1, 0, 1 or 2");
  if (enable < 0) {   // clear the totals, keep the mode
    for (int k = 0; k < KID_COUNT; ++k) { c->t_ms[k] = 0; c->t_n[k] = 0; c->t_bytes[k] = 0; }
    return SPDE_OK;
  }
  c->timing = enable;
  return SPDE_OK;
}

int spde_kernel_count(void) { return KID_COUNT; }

const char* spde_kernel_name(int id) { return (id >= 0 && id < KID_COUNT) ? kKernelNames[id] : nullptr; }

spde_status spde_timing_get(spde_handle h, int id, double* total_ms, int64_t* launches, double* bytes_per_launch) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return fail(SPDE_EINVAL, "null handle");
  if (id < 0 || id >= KID_COUNT) return fail(SPDE_EINVAL, "kernel id out of range");
  if (total_ms) *total_ms = c->t_ms[id];
  if (launches) *launches = c->t_n[id];
  if (bytes_per_launch) *bytes_per_launch = c->t_n[id] ? c->t_bytes[id] / (double)c->t_n[id] : 0.0;
  return SPDE_OK;
}

spde_status spde_info(spde_handle h, int* levels, int* persistent_top_n, int* device_lds_bytes) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c || !c->configured) return fail(SPDE_EINVAL, "handle not configured");
  if (levels) *levels = c->nlev;
  if (persistent_top_n) *persistent_top_n = c->lv[c->top].m;
  if (device_lds_bytes) *device_lds_bytes = c->lds_limit;
  return SPDE_OK;
}

void spde_free_host(void* p) { free(p); }

void spde_destroy(spde_handle h) {
  Ctx* c = reinterpret_cast<Ctx*>(h);
  if (!c) return;
  drop_graphs(c);
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  if (c->own_stream) hipStreamDestroy(c->own_stream);
  if (c->aux_stream) hipStreamDestroy(c->aux_stream);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  if (c->host_sc) hipHostFree(c->host_sc);
  if (c->host_res) hipHostFree(c->host_res);
  delete c;
}

const char* spde_last_error(void) { return g_err.c_str(); }

}  // extern "C"
