// Internal types shared by the HIP kernels and the host orchestration.
//
// Storage (all device, inside the caller's workspace), batch-outermost:
//   a cell array of one sample is n^3 values in cell order c = i + n (j + n k);
//   a face field of one sample is 3 such arrays, entry c of array d holding
//   the face on the low side of cell c in direction d (the face at i_d = 0 is
//   on the box boundary and always 0; the high boundary face of the last cell
//   is not stored).  All face arrays therefore share the cell indexing.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace spde {

constexpr int kMaxLevels = 12;
// static LDS of the persistent coarse kernel (a table of 8 reciprocals per level)
constexpr size_t kCoarseStaticLds = kMaxLevels * 8 * sizeof(double);
constexpr int kBlock = 256;          // threads per block of the streaming kernels

// Per-sample solver state (one per batch slot).
enum SlotState : int {
  ST_ACTIVE = 0,   // iterating
  ST_FINISH = 1,   // converged or capped: the operator pass applies the last x update
  ST_DONE   = 2,   // solution final in x
  ST_FAILED = 3,   // breakdown / non-finite
  ST_IDLE   = 4    // slot not in use
};

enum SlotFlags : int {
  FL_ZERO    = 1,  // right-hand side was exactly zero: solution is 0
  FL_NOTCONV = 2,  // stopped at max_iter
  FL_ACCUM   = 4   // refinement pass: the solve adds its solution to x (which holds the
                   // previous iterate) instead of overwriting it
};

// MINRES scalars of one sample.  Notation: iteration j works on the Lanczos
// vector v_j and its preconditioned image zhat_j = P^-1 v_j (not yet
// normalised); gamma_j^2 = <zhat_j, v_j>, delta_j = <A z_j, z_j> with
// z_j = zhat_j / gamma_j.
struct alignas(16) Scalars {
  double gamma, gamma_prev;   // gamma_j, gamma_{j-1}
  double delta;               // delta_j
  double c, s, c_prev, s_prev;
  double eta, eta0;
  // coefficients consumed by the operator pass of iteration `pit`
  double zs;                  // 1 / gamma_j
  double a_v;                 // delta_j / gamma_j
  double b_v;                 // gamma_j / gamma_{j-1}
  // Directions are stored unnormalised, W_{j+1} = alpha1_j w_{j+1}, so that the
  // operator pass of iteration j can form W_{j+1} from zhat_j before alpha1_j
  // (which needs gamma_{j+1}) is known:
  //   W_{j+1} = zs zhat_j + ww W_j + ww_prev W_{j-1};  x += xw W_j (+ xpend W_{j-1})
  double ww, ww_prev;
  double xw;                  // coefficient of W_j in the solution update
  double xpend;               // coefficient of W_{j-1} whose x update was deferred (0 if none)
  double al1_prev;            // alpha1 of the previous Givens step
  double tol;                 // relative stopping tolerance on |eta| / eta0
  int it;                     // iteration the V-cycle and the scalar step work on
  int pit;                    // iteration the operator pass works on
  int state;
  int flags;
  int wmode;                  // -1 no w/x update, 0 first (no reads), 1 no W_{j-1}, 2 full
  int iters;                  // iterations when finished
  int max_iter;
  int pad;
};

// Box constants.
struct Box {
  int n;
  int64_t n2;
  int64_t nc;        // n^3
  double h, h2, h3;
  double kappa, g;
  double q;          // 3 / (2 h^3): inverse of the face diagonal of M
  double k2h3;       // kappa^2 h^3
  double h2q;        // h^2 q
  int poly;          // face block of the preconditioner: 0 diag(M)^-1, 1 q (I - S + S^2)
  // Cell-wise coefficients (caller-owned device arrays [n^3], null: the
  // constants above): the operator's reaction term is kap_c^2 h^3 and the load
  // factor -g_c h^{3/2}; the multigrid preconditioner keeps a constant kappa.
  const double* kap;
  const double* gfld;
  double h15;        // h^{3/2}
};

#ifdef __HIPCC__
// Byte-offset load from a uniform base (global_load with a scalar base and a
// 32-bit lane offset).
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
// Streaming accesses for vectors that a pass reads once and writes once.  With
// NT they carry the nontemporal hint: at sizes far beyond the caches the lines
// they bring in then need not displace the ones that other streams of the pass
// still reuse.  Without it they are plain accesses, which keeps a working set
// that fits the last-level cache there between passes.  Values are the same.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
#endif

// kappa^2 h^3 of cell c (same rounding as the host's kappa * kappa * h^3).
// VAR: cell-wise kappa (a compile-time choice in the hot kernels, so that the
// constant path carries no branch); the run-time form serves the others.
template <bool VAR>
__host__ __device__ inline double cell_k2h3(const Box& b, int64_t c) {
  if constexpr (VAR) return (b.kap[c] * b.kap[c]) * b.h3;
  else return b.k2h3;
}
__host__ __device__ inline double cell_k2h3(const Box& b, int64_t c) {
  return b.kap ? cell_k2h3<true>(b, c) : b.k2h3;
}

// One multigrid level: operator S~ = K + a L (L the Neumann graph Laplacian,
// K = k2 I, or with cell-wise kappa the diagonal of the level's kappa_c^2 H^3),
// Chebyshev smoother coefficients of the degree-2 polynomial.
struct Level {
  int m;             // cells per edge
  int64_t nc;        // m^3
  double k2;         // kappa^2 H^3 (cell-wise kappa: kappa_min^2 H^3, which bounds the spectrum)
  double a;          // 3 H / 2
  double c0, c1, c2; // y = c0 D^-1 r ; x = c1 y + c2 D^-1 (r - A y)
  double cA, cB;     // pre-smoothing from zero in terms of bhat = D^-1 b:
                     // x = cA bhat + (cB / d) * sum_nbr bhat
  // Cell-wise diagonal D = K + a diag(neighbour count) of the level and its
  // reciprocal ([m^3] in the level precision, shared by all samples), or null
  // when kappa is constant.  The coarse K is the Galerkin one: each coarse
  // cell's k2 is the sum of its 8 children's.
  const void* dg;
  const void* dgi;
};

struct CoarseParams {
  int nl;                      // levels handled (top first, last is 1^3 or the coarsest)
  Level lv[kMaxLevels];
  int64_t off[kMaxLevels];     // element offset of each level's 4 arrays in LDS
  const void* cinv;            // 64 x 64 inverse of the 4^3 level's operator (level precision),
                               // row-major; read when the top level is 4^3 or larger
};

// Device pointers of the MINRES state.  Index [p] is the buffer parity.
struct Fields {
  double* vs[2];     // face Lanczos vectors: vs[p] + (slot*3 + d) * nc
  double* vu[2];     // cell Lanczos vectors
  void*   z[2];      // preconditioned cell vectors (float or double)
  double* w[2];      // MINRES direction vectors (cell part)
  double* x;         // solution (cell part)
  double* part_up;   // [slot][nb_up][2] partial sums of <zhat, v_u>, zhat^T A zhat
  double* part_pb;   // [slot][nb_pb]    partial sums of q |v_sigma|^2
  Scalars* sc;       // [slot]
};

// Per-sample offsets.
__host__ __device__ inline int64_t cell_off(int slot, int64_t nc) { return (int64_t)slot * nc; }
__host__ __device__ inline int64_t face_off(int slot, int d, int64_t nc) { return ((int64_t)slot * 3 + d) * nc; }

// Kernel classes (for timing and names).
enum KernelId : int {
  KID_INIT = 0, KID_MG_DOWN_FINE, KID_MG_DOWN, KID_MG_COARSE, KID_MG_UP, KID_MG_UP_FINE,
  KID_SCALAR, KID_OPERATOR, KID_OUTPUT, KID_FLUX, KID_RESID, KID_SPMM, KID_RESTRICT, KID_SPMM_STAGE,
  KID_COUNT
};

}  // namespace spde

// ---------------------------------------------------------------------------
// host launchers (defined in spde_kernels.hip)
namespace spde {
constexpr int kNumShapes = 18;
extern const int kShapes[kNumShapes][3];
bool shape_ok_up(int shape, bool fp64);
bool shape_ok_down(int shape, bool fp64);
int tiles_for(int shape, int m);
int operator_blocks(const Box& bx);

hipError_t launch_init(const Fields& F, const Box& bx, const double* xi, double scale, int batch, double tol,
                       int max_iter, int slot0, hipStream_t st);
hipError_t launch_init_gen(const Fields& F, const Box& bx, uint64_t seed, uint64_t event0, int coupled,
                           double scale, int batch, double tol, int max_iter, int slot0, hipStream_t st);
hipError_t launch_noise(int m, int coupled, uint64_t seed, uint64_t event0, int batch, double* out,
                        hipStream_t st);
hipError_t launch_philox_raw(uint64_t seed, uint64_t event, uint64_t ctr0, uint64_t ctr1, int64_t nblocks,
                             uint64_t* out, hipStream_t st);
// Device construction of the transfer: row lengths and pointers (rp[n_tet] < 0
// flags the first invalid tet), then the entries.
hipError_t launch_transfer_rows(int n, const double* xyz, int64_t n_vert, const int32_t* tets, int64_t n_tet,
                                int64_t* rp, hipStream_t st);
hipError_t launch_transfer_fill(int n, const double* xyz, int64_t n_vert, const int32_t* tets, int64_t n_tet,
                                const int64_t* rp, int32_t* col, double* val, hipStream_t st);
hipError_t launch_set_state(Scalars* sc, int slot0, int count, int state, hipStream_t st);
// Per-sample scalars of a steady-state operator pass (autotuner timing).
hipError_t launch_tune_scalars(Scalars* sc, int batch, hipStream_t st);
hipError_t launch_mg_down(bool fp64, int shape, bool fine, const void* b0, const void* b1, void* rH,
                          const Level& L, int batch, const Scalars* sc, hipStream_t st);
hipError_t launch_mg_up(bool fp64, int shape, bool fine, const void* b0, const void* b1, const void* eH, void* o0,
                        void* o1, const Level& L, int batch, const Scalars* sc, const double* vs0,
                        const double* vs1, double* part, const Box& bx, hipStream_t st);
hipError_t prepare_coarse(bool fp64, size_t lds_bytes);
// the same per level precision (spde_mg_f32.hip / spde_mg_f64.hip)
#define SPDE_MG_DECL(NAME)                                                                                      \
  hipError_t launch_mg_down_##NAME(int shape, bool fine, const void* b0, const void* b1, void* rH,            \
                                   const Level& L, int batch, const Scalars* sc, hipStream_t st);             \
  hipError_t launch_mg_up_##NAME(int shape, bool fine, const void* b0, const void* b1, const void* eH,        \
                                 void* o0, void* o1, const Level& L, int batch, const Scalars* sc,            \
                                 const double* vs0, const double* vs1, double* part, const Box& bx,           \
                                 hipStream_t st);                                                             \
  hipError_t prepare_coarse_##NAME(size_t lds_bytes);                                                         \
  hipError_t launch_mg_coarse_##NAME(const void* btop, void* etop, const CoarseParams& P, size_t lds_bytes,   \
                                     int batch, const Scalars* sc, hipStream_t st);                          \
  hipError_t launch_coarse_inverse_##NAME(const Level& L, void* out, hipStream_t st);
SPDE_MG_DECL(f32)
SPDE_MG_DECL(f64)
#undef SPDE_MG_DECL
hipError_t launch_mg_coarse(bool fp64, const void* btop, void* etop, const CoarseParams& P, size_t lds_bytes,
                            int batch, const Scalars* sc, hipStream_t st);
// Inverse of the 4^3 level's operator S~ (L.m must be 4) into out (64 x 64, level precision).
hipError_t launch_coarse_inverse(bool fp64, const Level& L, void* out, hipStream_t st);
hipError_t launch_scalar(const Fields& F, int nb_up, int nb_pb, int batch, hipStream_t st);
hipError_t launch_operator(bool z_fp64, const Fields& F, const Box& bx, int batch, hipStream_t st);
hipError_t launch_fix_solution(const Fields& F, const Box& bx, int batch, int slot0, hipStream_t st);
hipError_t launch_flux(const double* u, double* sig_int, double* sig_ext, const Box& bx, int batch,
                       hipStream_t st);
hipError_t launch_resid(const double* sig, const double* u, const double* xi, double scale, const Box& bx,
                        int batch, double* part, double* out, double* rhs, hipStream_t st);
// Warm start: x[slot] = the (n/2)^3 field uc[slot] injected into its children.
hipError_t launch_inject_coarse(const double* uc, double* x, int n, int batch, hipStream_t st);
// Refinement pass: v_1 = [0; the load already in vu[1]], scalars reset with FL_ACCUM.
// The tolerance of slot b is tols[b] (device array [batch]).
hipError_t launch_init_correction(const Fields& F, const Box& bx, int batch, const double* tols, int max_iter,
                                  hipStream_t st);
// Transfer SpMM out[s][row] = (Pi u[s])[row]: samples in blocks of
// spmm_block(batch), each staged sample-minor into `scratch`
// (spmm_scratch_bytes(nc, batch) bytes; unused for batch 1), then gathered,
// rows in chunks of kSpmmChunk visited in the chunk order corder (nullable).
constexpr int kSpmmChunk = 64;
// Rows per unit of the LDS-staged product (a chunk holds kSpmmChunk / kSpmmUnit
// units), and its LDS budget per block.
constexpr int kSpmmUnit = 16;
constexpr size_t kSpmmUnitLds = 60 << 10;
// Loads per thread of the unit kernel's stage: a unit's cells (x lanes per
// cell) and entries must fit them.
constexpr int kSpmmUnitCellIt = 8, kSpmmUnitEntIt = 2;
// Entries the unit kernel's LDS entry buffers hold beyond a unit's own.
constexpr int kSpmmUnitPad = 4;
// Static device scratch of the no-allocation transfer product (per device).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch_ptr(double** out);
int spmm_block(int batch);
size_t spmm_scratch_bytes(int64_t nc, int batch);
hipError_t launch_spmm_stage(const double* u, double* xt, int64_t nc, int batch, int s0, hipStream_t st);
hipError_t launch_spmm_gather(const int64_t* rp, const int32_t* ci, const double* cv, const double* u,
                              const double* xt, double* out, int64_t ntet, int64_t nnz, int64_t nc, int batch,
                              int s0, const int32_t* corder, hipStream_t st);
// The LDS-staged product for sample blocks of 32 or 64 (spmm_units_lds bytes of
// LDS per block; usable when that is at most kSpmmUnitLds): unit u's cells
// ucells[uptr[u] .. uptr[u + 1]) and each entry's index lcol in that list.
size_t spmm_units_lds(int bp, int max_cells, int max_entries);
hipError_t launch_spmm_units(const int64_t* rp, const double* cv, const int64_t* uptr, const int32_t* ucells,
                             const uint16_t* lcol, const double* xt, double* out, int64_t ntet, int64_t nnz,
                             int64_t nc, int batch, int s0, const int32_t* corder, int max_cells, int max_entries,
                             hipStream_t st);
hipError_t launch_spmm(const int64_t* rp, const int32_t* ci, const double* cv, const double* u, double* out,
                       int64_t ntet, int64_t nnz, int64_t nc, int batch, const int32_t* corder, double* scratch,
                       hipStream_t st);
hipError_t launch_restrict_noise(const double* xf, double* xc, int nf, int batch, hipStream_t st);
hipError_t launch_ext_to_int(const double* xs, const double* xu, const Fields& F, const Box& bx, int batch,
                             hipStream_t st);
// Same, with zhat = x_u written to the solver's own z buffer in the multigrid
// precision (float32 unless z_fp64).
hipError_t launch_ext_to_int_zhat(const double* xs, const double* xu, const Fields& F, const Box& bx, int batch,
                                  bool z_fp64, hipStream_t st);
hipError_t launch_int_to_ext(const Fields& F, double* ys, double* yu, const Box& bx, int batch, hipStream_t st);
hipError_t launch_probe_scalars(Scalars* sc, int batch, hipStream_t st);
// Cell-wise multigrid coefficients: k2 = (kappa kappa) h^3 on the finest level,
// the sum of the 8 children on each coarser one (float64), then the level's
// diagonal k2 + a nn and its reciprocal in the level precision.
hipError_t launch_mg_k2_fine(const double* kap, double h3, double* k2, int64_t nc, hipStream_t st);
hipError_t launch_mg_k2_coarsen(const double* k2f, double* k2c, int mf, hipStream_t st);
hipError_t launch_mg_diag(bool fp64, const double* k2, int m, double a, void* dg, void* dgi, hipStream_t st);
// Per-block minima of v[0, n) into out[(n + 255) / 256].
hipError_t launch_block_min(const double* v, int64_t n, double* out, hipStream_t st);
hipError_t launch_f32_to_f64(const float* s, double* d, int64_t count, hipStream_t st);
}  // namespace spde
