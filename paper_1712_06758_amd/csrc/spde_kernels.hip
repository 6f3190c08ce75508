// HIP kernels (gfx950) of the SPDE field sampler.
//
// The solve is MINRES on the RT0/P0 saddle-point system of eq. linsys,
// preconditioned by blkdiag(diag(M), V) where V is one V-cycle of geometric
// multigrid on S~ = kappa^2 W + B diag(M)^-1 B^T (eq. ldu's approximate Schur
// complement with the kappa^2 W block).  Only the cell part of the MINRES
// iterate is stored ("u-only" MINRES): the face parts of x and w never feed
// back into the recurrence, and the face part of z = P^-1 v is diag(M)^-1 v,
// applied on the fly.
//
// Per iteration j (all launches cover every slot of the batch; each block
// reads its slot's state and exits unless the slot is iterating):
//   mg_down (fine, then per level)  : smooth from zero, restrict the residual
//   mg_coarse                        : the levels that fit in LDS, one block per slot
//   mg_up (per level, then fine)     : prolong, correct, smooth; the fine launch
//                                      writes zhat_j and the partial sums of
//                                      <zhat_j, v_j> and zhat_j^T A zhat_j
//   scalar                           : per-slot reductions, Givens rotation,
//                                      convergence test
//   operator                         : v_{j+1} = A z_j - (delta/gamma) v_j - (gamma/gamma_prev) v_{j-1}
//                                      and the delayed w/x update of step j-1
#include <mutex>

#include "spde_common.inc"

namespace spde {

// ---------------------------------------------------------------------------
// initialisation: v_1 = F = [0; scale * xi], state reset

__device__ __forceinline__ void init_scalars(const Fields& F, int slot, double tol, int max_iter) {
  Scalars s{};
  s.it = 1; s.pit = 0; s.state = ST_ACTIVE; s.flags = 0; s.wmode = -1;
  s.c = s.c_prev = 1.0; s.s = s.s_prev = 0.0;
  s.gamma_prev = 1.0; s.tol = tol; s.max_iter = max_iter; s.iters = 0;
  F.sc[slot] = s;
}

__global__ __launch_bounds__(kBlock) void k_init(Fields F, Box bx, const double* __restrict__ xi,
                                                 double scale, int nb, double tol, int max_iter, int slot0) {
  const int rel = blockIdx.x / nb;
  const int slot = slot0 + rel;
  const int blk = blockIdx.x - rel * nb;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c < bx.nc) {
    const double sc_c = bx.gfld ? -bx.gfld[c] * bx.h15 : scale;
    F.vu[1][cell_off(slot, bx.nc) + c] = sc_c * xi[cell_off(rel, bx.nc) + c];
    F.vs[1][face_off(slot, 0, bx.nc) + c] = 0.0;
    F.vs[1][face_off(slot, 1, bx.nc) + c] = 0.0;
    F.vs[1][face_off(slot, 2, bx.nc) + c] = 0.0;
  }
  if (blk == 0 && threadIdx.x == 0) init_scalars(F, slot, tol, max_iter);
}

// Refinement pass (iterative refinement in float64 around the whole solve):
// v_1 = [0; r] with r = F - A U already in vu[1], MINRES state reset with the
// slot's own tolerance tols[slot], and FL_ACCUM so that the pass adds its
// correction to x = U.
__global__ __launch_bounds__(kBlock) void k_init_correction(Fields F, Box bx, int nb, const double* __restrict__ tols,
                                                            int max_iter) {
  const int slot = blockIdx.x / nb;
  const int blk = blockIdx.x - slot * nb;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c < bx.nc) {
    F.vs[1][face_off(slot, 0, bx.nc) + c] = 0.0;
    F.vs[1][face_off(slot, 1, bx.nc) + c] = 0.0;
    F.vs[1][face_off(slot, 2, bx.nc) + c] = 0.0;
  }
  if (blk == 0 && threadIdx.x == 0) {
    init_scalars(F, slot, tols[slot], max_iter);
    F.sc[slot].flags = FL_ACCUM;
  }
}

// ---------------------------------------------------------------------------
// scalar step of iteration j (one block per slot)

__global__ __launch_bounds__(kBlock) void k_scalar(Fields F, int nb_up, int nb_pb) {
  __shared__ double red[kBlock / 64];
  const int slot = blockIdx.x;
  Scalars* S = F.sc + slot;
  const int state = S->state;
  if (state == ST_FINISH) {
    if (threadIdx.x == 0) S->state = ST_DONE;
    return;
  }
  if (state != ST_ACTIVE) return;
  const int j = S->it;
  double a0 = 0.0, a1 = 0.0;
  const double* pu = F.part_up + (int64_t)slot * nb_up * 2;
  for (int i = threadIdx.x; i < nb_up; i += kBlock) { a0 += pu[2 * i]; a1 += pu[2 * i + 1]; }
  a0 = block_sum(a0, red);
  a1 = block_sum(a1, red);
  if (threadIdx.x != 0) return;
  (void)nb_pb;

  Scalars s = *S;
  const double gg = a0;               // gamma_j^2
  if (!(gg >= 0.0) || !isfinite(gg) || !isfinite(a1)) {
    s.state = ST_FAILED; s.iters = j - 1; *S = s; return;
  }
  if (gg == 0.0 && j == 1) {           // zero right-hand side: the solution is 0
    s.state = ST_DONE; s.flags |= FL_ZERO; s.iters = 0; *S = s; return;
  }
  const double gam = sqrt(gg);
  const double del = gg > 0.0 ? a1 / gg : 0.0;
  if (j == 1) {
    s.eta = gam; s.eta0 = gam;
    s.c = s.c_prev = 1.0; s.s = s.s_prev = 0.0;
    s.wmode = 0;                       // W_2 = z_1
    s.ww = s.ww_prev = 0.0;
    s.xw = s.xpend = 0.0;
    s.al1_prev = 1.0;
    s.b_v = 0.0;
  } else {
    // complete the Givens rotation of step j-1 now that gamma_j is known
    const double dp = s.delta, gp = s.gamma;
    const double al0 = s.c * dp - s.c_prev * s.s * gp;
    const double al1 = sqrt(al0 * al0 + gg);
    if (!(al1 > 0.0) || !isfinite(al1)) { s.state = ST_FAILED; s.iters = j - 1; *S = s; return; }
    const double cn = al0 / al1, sn = gam / al1;
    // x_{j-1} = x_{j-2} + c_j eta w_j with w_j = W_j / alpha1_{j-1}.  The
    // operator pass of an odd iteration >= 3 defers its solution update to the
    // next pass (x absorbs two directions every other iteration).
    s.xpend = ((j - 1) % 2 == 1 && j - 1 >= 3) ? s.xw : 0.0;
    s.xw = cn * s.eta / al1;
    s.eta = -sn * s.eta;
    // W_{j+1} = z_j - alpha3_j w_{j-1} - alpha2_j w_j, with
    // alpha2_j = s_j delta_j + c_{j-1} c_j gamma_j and alpha3_j = s_{j-1} gamma_j
    const double a2 = sn * del + s.c * cn * gam;
    const double a3 = s.s * gam;
    s.ww = -a2 / al1;
    s.ww_prev = -a3 / s.al1_prev;
    s.al1_prev = al1;
    s.c_prev = s.c; s.s_prev = s.s;
    s.c = cn; s.s = sn;
    s.wmode = (j == 2) ? 1 : 2;
    s.b_v = gam / gp;
    if (fabs(s.eta) <= s.tol * s.eta0 || gg == 0.0) {
      s.state = ST_FINISH; s.iters = j - 1;
    } else if (j - 1 >= s.max_iter) {
      s.state = ST_FINISH; s.iters = j - 1; s.flags |= FL_NOTCONV;
    }
  }
  s.gamma_prev = (j == 1) ? 1.0 : s.gamma;
  s.gamma = gam;
  s.delta = del;
  s.zs = gam > 0.0 ? 1.0 / gam : 0.0;
  s.a_v = gam > 0.0 ? del / gam : 0.0;
  s.pit = j;
  s.it = j + 1;
  *S = s;
}

// ---------------------------------------------------------------------------
// finishing

// Slot states for continuous batching: set [slot0, slot0 + count) to `state`.
__global__ void k_set_state(Scalars* sc, int slot0, int count, int state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) sc[slot0 + i].state = state;
}

// Zero / NaN the solution of slots that finished with FL_ZERO / ST_FAILED (a
// refinement pass with a zero load leaves the previous iterate in place).
__global__ __launch_bounds__(kBlock) void k_fix_solution(Fields F, Box bx, int nb, int slot0) {
  const int rel = blockIdx.x / nb, blk = blockIdx.x - rel * nb;
  const int slot = slot0 + rel;
  const Scalars* S = F.sc + slot;
  const bool fail = S->state == ST_FAILED;
  const bool zero = (S->flags & FL_ZERO) && !(S->flags & FL_ACCUM);
  if (!zero && !fail) return;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c < bx.nc) F.x[cell_off(slot, bx.nc) + c] = zero ? 0.0 : __builtin_nan("");
}

// Flux recovery sigma = -M^-1 B^T u (first block row of eq. linsys): along
// each grid line, tridiag(1/6, 2/3, 1/6) sigma = (u_c - u_{c-1}) / h over the
// n-1 interior faces (Thomas algorithm; one thread per line).  Writes the
// internal face layout (sig_int [slot][3][n^3], may be null) and the external
// layout (sig_ext [slot][3 n^2 (n+1)], may be null).
__global__ __launch_bounds__(kBlock) void k_flux(const double* __restrict__ u, double* __restrict__ sig_int,
                                                 double* __restrict__ sig_ext, Box bx, int batch) {
  __shared__ double cp[1024];
  const int n = bx.n;
  // c'_i of the forward sweep (identical for every line)
  if (threadIdx.x == 0) {
    double cprev = 0.0;
    for (int i = 1; i < n; ++i) {
      const double mdiag = (2.0 / 3.0) - (1.0 / 6.0) * cprev;
      cprev = (1.0 / 6.0) / mdiag;
      cp[i] = cprev;
    }
  }
  __syncthreads();
  const int64_t lines = 3 * bx.n2;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= lines * batch) return;
  const int slot = (int)(gid / lines);
  const int64_t l = gid - (int64_t)slot * lines;
  const int d = (int)(l / bx.n2);
  const int64_t rest = l - (int64_t)d * bx.n2;
  const int64_t nc = bx.nc;
  const double* us = u + cell_off(slot, nc);
  // line coordinates: the two indices other than d, fastest first
  const int a = (int)(rest % n), b = (int)(rest / n);
  int64_t base, stride;
  if (d == 0) { base = (int64_t)n * (a + (int64_t)n * b); stride = 1; }
  else if (d == 1) { base = a + (int64_t)n * n * b; stride = n; }
  else { base = a + (int64_t)n * b; stride = bx.n2; }
  const double inv_h = 1.0 / bx.h;
  double* si = sig_int ? sig_int + face_off(slot, d, nc) : nullptr;
  double* se = nullptr;
  int64_t ebase = 0, estride = 0;
  if (sig_ext) {
    const int64_t nf = bx.n2 * (n + 1);
    se = sig_ext + (int64_t)slot * 3 * nf + (int64_t)d * nf;
    if (d == 0) { ebase = (int64_t)(n + 1) * (a + (int64_t)n * b); estride = 1; }
    else if (d == 1) { ebase = a + (int64_t)n * (n + 1) * b; estride = n; }
    else { ebase = a + (int64_t)n * b; estride = bx.n2; }
  }
  // forward sweep: store d'_i in the output (internal if present, else external)
  double dprev = 0.0;
  double* tmp = si ? si : se;
  const int64_t tb = si ? base : ebase;
  const int64_t ts = si ? stride : estride;
  for (int i = 1; i < n; ++i) {
    const double rhs = (us[base + (int64_t)i * stride] - us[base + (int64_t)(i - 1) * stride]) * inv_h;
    const double mdiag = (2.0 / 3.0) - (1.0 / 6.0) * (i > 1 ? cp[i - 1] : 0.0);
    dprev = (rhs - (1.0 / 6.0) * dprev) / mdiag;
    tmp[tb + (int64_t)i * ts] = dprev;
  }
  double snext = 0.0;
  for (int i = n - 1; i >= 1; --i) {
    const double sv = tmp[tb + (int64_t)i * ts] - (i < n - 1 ? cp[i] * snext : 0.0);
    snext = sv;
    if (si) si[base + (int64_t)i * stride] = sv;
    if (se) se[ebase + (int64_t)i * estride] = sv;
  }
  if (si) si[base] = 0.0;
  if (se) { se[ebase] = 0.0; se[ebase + (int64_t)n * estride] = 0.0; }
}

// True residual of the cell row with the recovered flux:
//   r = F_u - (B sigma - kappa^2 h^3 u),  F_u = -g h^{3/2} xi.
// Per-block partial sums of |r|^2 and |F_u|^2; r itself into rhs (if not null),
// the load of a refinement pass.  (The face row of the residual vanishes up
// to rounding: sigma = -M^-1 B^T u solves it.)
__global__ __launch_bounds__(kBlock) void k_resid(const double* __restrict__ sig, const double* __restrict__ u,
                                                  const double* __restrict__ xi, double scale, Box bx,
                                                  int nb, double* __restrict__ part, double* __restrict__ rhs) {
  __shared__ double red[kBlock / 64];
  const int slot = blockIdx.x / nb, blk = blockIdx.x - slot * nb;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  const int64_t nc = bx.nc;
  const int n = bx.n;
  double rr = 0.0, ff = 0.0;
  if (c < nc) {
    const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / bx.n2);
    const double* sx = sig + face_off(slot, 0, nc);
    const double* sy = sig + face_off(slot, 1, nc);
    const double* sz = sig + face_off(slot, 2, nc);
    const double div = ((i < n - 1 ? sx[c + 1] : 0.0) - sx[c]) + ((j < n - 1 ? sy[c + n] : 0.0) - sy[c]) +
                       ((k < n - 1 ? sz[c + bx.n2] : 0.0) - sz[c]);
    const double uc = u[cell_off(slot, nc) + c];
    const double sc_c = bx.gfld ? -bx.gfld[c] * bx.h15 : scale;
    const double fu = sc_c * xi[cell_off(slot, nc) + c];
    const double r = fu - (bx.h2 * div - cell_k2h3(bx, c) * uc);
    if (rhs) rhs[cell_off(slot, nc) + c] = r;
    rr = r * r;
    ff = fu * fu;
  }
  rr = block_sum(rr, red);
  ff = block_sum(ff, red);
  if (threadIdx.x == 0) {
    part[((int64_t)slot * nb + blk) * 2 + 0] = rr;
    part[((int64_t)slot * nb + blk) * 2 + 1] = ff;
  }
}

__global__ __launch_bounds__(kBlock) void k_resid_reduce(const double* __restrict__ part, int nb,
                                                         double* __restrict__ out) {
  __shared__ double red[kBlock / 64];
  const int slot = blockIdx.x;
  double rr = 0.0, ff = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    rr += part[((int64_t)slot * nb + i) * 2];
    ff += part[((int64_t)slot * nb + i) * 2 + 1];
  }
  rr = block_sum(rr, red);
  ff = block_sum(ff, red);
  if (threadIdx.x == 0) out[slot] = ff > 0.0 ? sqrt(rr / ff) : sqrt(rr);
}

// ---------------------------------------------------------------------------
// transfer: u_tet = Pi u (CSR rows = tets, eq. proj_op)
//
// The box fields are first staged sample-minor, xt[c][s] for a block of BP
// samples (BP a power of two <= 64, the padding zero), so that the gather of
// one cell brings every sample of the block in one coalesced access of BP x 8
// bytes instead of BP separate lines.  Lanes then own samples: a wave works
// on 64 / BP rows at a time, reading each row's entries once per sample block,
// and a block's results leave through an LDS tile, so that each sample's rows
// are written contiguously.  Entries are summed in column order, as a plain
// CSR product does.

// x [batch][nc] -> xt [nc][BP] for the samples s0 .. s0 + BP - 1 (zero past
// batch), through an LDS tile of TC cells x BP samples.
template <int BP>
__global__ __launch_bounds__(kBlock) void k_spmm_stage(const double* __restrict__ x, double* __restrict__ xt,
                                                       int64_t nc, int batch, int s0) {
  constexpr int TC = 4096 / BP;            // cells per tile
  constexpr int LD = BP + 1;               // padded tile row
  __shared__ double tile[TC * LD];
  const int64_t c0 = (int64_t)blockIdx.x * TC;
#pragma unroll 4
  for (int idx = threadIdx.x; idx < TC * BP; idx += kBlock) {
    const int sl = idx / TC, cl = idx - sl * TC;    // consecutive threads: consecutive cells of one sample
    const int64_t c = c0 + cl;
    const int smp = s0 + sl;
    tile[cl * LD + sl] = (c < nc && smp < batch) ? x[(int64_t)smp * nc + c] : 0.0;
  }
  __syncthreads();
#pragma unroll 4
  for (int idx = threadIdx.x; idx < TC * BP; idx += kBlock) {
    const int cl = idx / BP, sl = idx - cl * BP;    // consecutive threads: the samples of one cell
    const int64_t c = c0 + cl;
    if (c < nc) xt[c * BP + sl] = tile[cl * LD + sl];
  }
}

// Rows are taken in chunks of kSpmmChunk consecutive rows, so that each
// sample's stores stay contiguous; corder (nullable) gives the order in which
// the chunks are visited (logical chunk q is chunk corder[q]), which decides
// how much of the staged field is still in cache when a neighbouring chunk
// needs it.

// out[s0 + s][row] = sum_k Pi[row, col_k] x[s0 + s][col_k] for s < min(BP, batch - s0),
// from the staged xt, for blocks of BP >= 16 samples.  Each lane carries two
// samples (one 16-byte load per entry), so a wave's lanes form G = 128 / BP
// groups of BP / 2 lanes; a group owns 8 consecutive rows of a chunk and works
// through them one after the other.  For each row the group first holds up to
// U = 12 of its entries (column, value) in its lanes, then issues their U
// gathers at once; while those are in flight it loads the row pointers and
// entries of the next row, so a row (9 entries on average for the workload
// meshes) costs one memory round trip and a wave keeps G x U gathers of
// BP x 8 bytes in flight.  Measured at 128^3 x 64: U = 12 at 3 waves per SIMD
// runs as fast as U = 8 at 4 (1.28 ms) and fetches 3.8 instead of 6.2 GB from
// memory (counter bytes); U = 16 fits only 2 waves per SIMD and is slower
// (1.7 ms).  Each row's sum runs over its entries in order.  The block's results (its chunks' rows x BP samples) go through an
// LDS tile and leave row-contiguous per sample.  Row pointers must not
// decrease; if they do, no memory outside the arrays is touched, but the sums
// are undefined.
template <int BP, int UM = 12, int WPS = 3>
__global__ __launch_bounds__(kBlock, WPS) void k_spmm_gather(const int64_t* __restrict__ rp,
                                                             const int32_t* __restrict__ ci,
                                                             const double* __restrict__ cv,
                                                             const double* __restrict__ xt, double* __restrict__ out,
                                                             int64_t ntet, int64_t nnz, int64_t nc, int batch, int s0,
                                                             const int32_t* __restrict__ corder, int64_t nchunk) {
  static_assert(BP >= 16 && BP <= 64, "sample block");
  constexpr int LG = BP / 2;               // lanes per group (two samples each)
  constexpr int G = 64 / LG;               // row groups per wave
  constexpr int RG = 8;                    // consecutive rows per group
  constexpr int R = 4 * G * RG;            // rows per block
  constexpr int CPB = R / kSpmmChunk;      // chunks per block
  constexpr int GPC = kSpmmChunk / RG;     // groups per chunk
  constexpr int LD = BP + 2;               // padded tile row (16-byte aligned pairs)
  constexpr int U = LG < UM ? LG : UM;     // entries held per row chunk
  static_assert(R % kSpmmChunk == 0, "whole chunks per block");
  __shared__ double tile[R * LD];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int sl = lane % LG, g = lane / LG;
  const int s = 2 * sl;                    // the lane's first sample
  const int gbase = g * LG;                // the group's first lane
  const int nb = min(BP, batch - s0);
  const int gi = wv * G + g;               // group index within the block
  const int lr0 = gi * RG;                 // its first row within the block's tile
  const int64_t q = (int64_t)lb * CPB + gi / GPC;
  const int64_t chunk = q < nchunk ? (corder ? (int64_t)corder[q] : q) : nchunk;
  const int64_t ra = chunk * kSpmmChunk + (gi % GPC) * RG;
  const int64_t rb = min(ra + RG, ntet);
  auto clampk = [&](int64_t k) { return max((int64_t)0, min(k, nnz)); };
  // entries [k, kend) into the group's lanes (lane sl holds entry k + sl, sl < U)
  auto load_chunk = [&](int64_t k, int64_t kend, int32_t& cc, double& vv) {
    const bool in = sl < U && k + sl < kend;
    cc = in ? ci[k + sl] : -1;
    vv = in ? cv[k + sl] : 0.0;
  };
  if (ra < rb) {
    int64_t k0 = clampk(rp[ra]);
    int64_t k1 = max(k0, clampk(rp[ra + 1]));
    int32_t cc;
    double vv;
    load_chunk(k0, k1, cc, vv);
    for (int64_t row = ra; row < rb; ++row) {
      // pointer of the row after next, loaded while this row's gathers run
      const int64_t k2 = row + 1 < rb ? clampk(rp[row + 2]) : k1;
      double acc0 = 0.0, acc1 = 0.0;
      int64_t kc = k0;
      while (true) {
        const int cnt = (int)min((int64_t)U, k1 - kc);
        int32_t c[U];
        double v[U];
        double2 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          c[u] = __shfl(cc, gbase + u, 64);
          v[u] = __shfl(vv, gbase + u, 64);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool ok = u < cnt && c[u] >= 0 && c[u] < nc;
          x[u] = *reinterpret_cast<const double2*>(xt + (ok ? (int64_t)c[u] : 0) * BP + s);
        }
        // the next chunk of this row, or the first chunk of the next row
        const int64_t kn = kc + U;
        const bool more = kn < k1;
        load_chunk(more ? kn : k1, more ? k1 : max(k1, k2), cc, vv);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (u < cnt && c[u] >= 0 && c[u] < nc) {
            acc0 += v[u] * x[u].x;
            acc1 += v[u] * x[u].y;
          }
        }
        if (!more) break;
        kc = kn;
      }
      *reinterpret_cast<double2*>(&tile[(lr0 + (int)(row - ra)) * LD + s]) = make_double2(acc0, acc1);
      k0 = k1;
      k1 = max(k0, k2);
    }
  }
  __syncthreads();
  // consecutive threads store consecutive rows of one sample and chunk
  for (int idx = threadIdx.x; idx < R * BP; idx += kBlock) {
    const int ss = idx / R, li = idx - ss * R;
    const int64_t qq = (int64_t)lb * CPB + li / kSpmmChunk;
    if (ss >= nb || qq >= nchunk) continue;
    const int64_t row = (corder ? (int64_t)corder[qq] : qq) * kSpmmChunk + li % kSpmmChunk;
    if (row < ntet) out[(int64_t)(s0 + ss) * ntet + row] = tile[li * LD + ss];
  }
}

// The same product with each row unit's cells staged in LDS (blocks of BP = 32
// or 64 samples).  Units of kSpmmUnit rows are taken in the chunk visiting
// order; block b handles logical units b, b + G, b + 2G, ... (G blocks).  Per
// unit it loads the staged sample rows xt[cell][0 .. BP) of the unit's distinct
// cells (ucells[uptr[u] .. uptr[u + 1]), ascending) and the unit's entries
// (value, index lcol of the column in that list) into LDS, forms the unit's
// rows from LDS in the groups and entry order of k_spmm_gather (so the sums are
// bitwise the same), and stores through an LDS tile that reuses the cell
// buffer.  Each cell of a unit is read from memory once instead of once per
// entry, and the next unit's cell indices are loaded while this unit computes,
// so a unit costs one memory round trip.  Lists that do not fit the sizes the
// launch was given are cut at them (no access outside the LDS buffers; the
// sums are then wrong), which cannot happen for lists built from the
// registered matrix.
template <int BP>
__global__ __launch_bounds__(kBlock) void k_spmm_units(const int64_t* __restrict__ rp, const double* __restrict__ cv,
                                                       const int64_t* __restrict__ uptr,
                                                       const int32_t* __restrict__ ucells,
                                                       const uint16_t* __restrict__ lcol,
                                                       const double* __restrict__ xt, double* __restrict__ out,
                                                       int64_t ntet, int64_t nnz, int64_t nc, int batch, int s0,
                                                       const int32_t* __restrict__ corder, int64_t nunit,
                                                       int cells_cap, int entries_cap) {
  static_assert(BP == 32 || BP == 64, "sample block");
  constexpr int LG = BP / 2;                 // lanes per group (two samples each)
  constexpr int NG = kBlock / LG;            // groups per block
  constexpr int RPG = kSpmmUnit / NG;        // rows per group
  constexpr int LD = BP + 2;                 // padded row of a staged cell (16-byte aligned pairs)
  constexpr int UPC = kSpmmChunk / kSpmmUnit;
  static_assert(RPG >= 1 && RPG * NG == kSpmmUnit && kSpmmChunk % kSpmmUnit == 0, "unit split");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sx = reinterpret_cast<double*>(smem_raw);              // [cells_cap][LD], then the output tile
  double* sv = sx + (size_t)cells_cap * LD;                       // [entries_cap] entry values
  uint16_t* sl = reinterpret_cast<uint16_t*>(sv + entries_cap);   // [entries_cap] entry cells
  __shared__ int srp[kSpmmUnit + 1];
  const int tid = threadIdx.x;
  const int64_t nlog = ((ntet + kSpmmChunk - 1) / kSpmmChunk) * UPC;   // logical units
  const int64_t G = gridDim.x;
  auto clampk = [&](int64_t k) { return max((int64_t)0, min(k, nnz)); };
  auto unit_of = [&](int64_t lu) {
    const int64_t lq = lu / UPC;
    return (corder ? (int64_t)corder[lq] : lq) * UPC + (lu - lq * UPC);
  };
  // cell indices of a unit's stage items (the launcher keeps ncell * LG <=
  // kSpmmUnitCellIt * kBlock and ne <= kSpmmUnitEntIt * kBlock)
  int32_t cellv[kSpmmUnitCellIt];
  auto load_cells = [&](int64_t unit) {
    const int64_t c0 = unit < nunit ? uptr[unit] : 0;
    const int ncell = unit < nunit ? (int)min((int64_t)cells_cap, max((int64_t)0, uptr[unit + 1] - c0)) : 0;
#pragma unroll
    for (int it = 0; it < kSpmmUnitCellIt; ++it) {
      const int cl = (tid + it * kBlock) / LG;
      cellv[it] = cl < ncell ? ucells[c0 + cl] : -1;
    }
    return ncell;
  };
  int64_t lu = xcd_remap(blockIdx.x, gridDim.x);
  int64_t unit = lu < nlog ? unit_of(lu) : nunit;
  int ncell = load_cells(unit);
  const int nb = min(BP, batch - s0);
  const int lane = tid & 63;
  const int g = lane / LG, s = 2 * (lane % LG);
  const int gi = (tid >> 6) * (64 / LG) + g;   // group index within the block
  for (; lu < nlog; lu += G) {
    const bool live = unit < nunit;
    const int64_t r0 = unit * kSpmmUnit;
    const int nr = live ? (int)min((int64_t)kSpmmUnit, ntet - r0) : 0;
    const int64_t e0 = live ? clampk(rp[r0]) : 0;
    const int ne = live ? (int)min((int64_t)(entries_cap - kSpmmUnitPad), max((int64_t)0, clampk(rp[r0 + nr]) - e0)) : 0;
    if (tid <= nr && live) srp[tid] = (int)max((int64_t)0, min(clampk(rp[r0 + tid]) - e0, (int64_t)ne));
    // this unit's entries and cell rows (all issued before any is consumed)
    double ev[kSpmmUnitEntIt];
    uint16_t el[kSpmmUnitEntIt];
#pragma unroll
    for (int it = 0; it < kSpmmUnitEntIt; ++it) {
      const int k = tid + it * kBlock;
      ev[it] = k < ne ? cv[e0 + k] : 0.0;
      el[it] = k < ne ? lcol[e0 + k] : (uint16_t)65535;
    }
    double2 xv[kSpmmUnitCellIt];
#pragma unroll
    for (int it = 0; it < kSpmmUnitCellIt; ++it) {
      const int p = (tid + it * kBlock) % LG;
      const bool ok = cellv[it] >= 0 && cellv[it] < nc;
      xv[it] = *reinterpret_cast<const double2*>(xt + (ok ? (int64_t)cellv[it] : 0) * BP + 2 * p);
    }
    // the next unit's cell indices, in flight while this unit computes
    const int64_t lun = lu + G;
    const int64_t unext = lun < nlog ? unit_of(lun) : nunit;
    int32_t cur[kSpmmUnitCellIt];
#pragma unroll
    for (int it = 0; it < kSpmmUnitCellIt; ++it) cur[it] = cellv[it];
    const int ncur = ncell;
    ncell = load_cells(unext);
#pragma unroll
    for (int it = 0; it < kSpmmUnitEntIt; ++it) {
      const int k = tid + it * kBlock;
      if (k < ne) {
        sv[k] = ev[it];
        sl[k] = el[it];
      }
    }
#pragma unroll
    for (int it = 0; it < kSpmmUnitCellIt; ++it) {
      const int idx = tid + it * kBlock, cl = idx / LG, p = idx - cl * LG;
      const bool ok = cur[it] >= 0 && cur[it] < nc;
      if (cl < ncur) *reinterpret_cast<double2*>(sx + cl * LD + 2 * p) = ok ? xv[it] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double a0[RPG], a1[RPG];
#pragma unroll
    for (int rr = 0; rr < RPG; ++rr) {
      const int lr = gi * RPG + rr;
      double acc0 = 0.0, acc1 = 0.0;
      if (lr < nr) {
        const int ka = srp[lr], kb = max(ka, srp[lr + 1]);
        // four entries at a time, their LDS reads issued before the sums; the
        // entry buffers are padded by kSpmmUnitPad, so the reads past the row
        // stay inside them.  A slot past the row or with a skipped column adds
        // 0 * x (x a staged value, finite unless the sample itself is not),
        // which leaves the sum's bits unchanged.
        for (int k = ka; k < kb; k += 4) {
          int l[4];
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            l[u] = sl[k + u];
            v[u] = sv[k + u];
          }
          double2 x[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const bool ok = k + u < kb && l[u] < ncur;
            x[u] = *reinterpret_cast<const double2*>(sx + (ok ? l[u] : 0) * LD + s);
            v[u] = ok ? v[u] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            acc0 = fma(v[u], x[u].x, acc0);
            acc1 = fma(v[u], x[u].y, acc1);
          }
        }
      }
      a0[rr] = acc0;
      a1[rr] = acc1;
    }
    __syncthreads();   // the cells are read; the tile reuses their buffer
#pragma unroll
    for (int rr = 0; rr < RPG; ++rr)
      *reinterpret_cast<double2*>(sx + (gi * RPG + rr) * LD + s) = make_double2(a0[rr], a1[rr]);
    __syncthreads();
    // consecutive threads store consecutive rows of one sample
    for (int idx = tid; idx < kSpmmUnit * BP; idx += kBlock) {
      const int ss = idx / kSpmmUnit, li = idx - ss * kSpmmUnit;
      if (ss < nb && li < nr) out[(int64_t)(s0 + ss) * ntet + r0 + li] = sx[li * LD + ss];
    }
    __syncthreads();   // the tile is read before the next unit's stage overwrites it
    unit = unext;
  }
}

// The same product for blocks of BP <= 8 samples: one row per lane, its BP
// samples contiguous in xt (one load of BP x 8 bytes per entry), a wave on the
// 64 rows of one chunk, so that the entries it reads and the values it stores
// are contiguous.  For BP = 1 xt is the sample's own field.  A row's entries
// are taken U at a time: their columns and values are all loaded before the
// gathers, and the gathers before the sums, so that a lane has U loads in
// flight; the sums keep the entry order.
template <int BP>
__global__ __launch_bounds__(kBlock) void k_spmm_rows(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                      const double* __restrict__ cv, const double* __restrict__ xt,
                                                      double* __restrict__ out, int64_t ntet, int64_t nnz, int64_t nc,
                                                      int batch, int s0,
                                                      const int32_t* __restrict__ corder, int64_t nchunk) {
  static_assert(BP >= 1 && BP <= 8 && kSpmmChunk == 64, "sample block; a wave per chunk");
  constexpr int U = BP >= 8 ? 2 : 16 / BP;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t q = (int64_t)lb * (kBlock / 64) + (threadIdx.x >> 6);
  if (q >= nchunk) return;
  const int64_t row = (corder ? (int64_t)corder[q] : q) * kSpmmChunk + (threadIdx.x & 63);
  if (row >= ntet) return;
  const int nb = min(BP, batch - s0);
  const int64_t k0 = max((int64_t)0, min(rp[row], nnz)), k1 = max(k0, min(rp[row + 1], nnz));
  double acc[BP];
#pragma unroll
  for (int q2 = 0; q2 < BP; ++q2) acc[q2] = 0.0;
  for (int64_t k = k0; k < k1; k += U) {
    int64_t col[U];
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = k + u < k1;
      col[u] = in ? (int64_t)ci[k + u] : -1;
      v[u] = in ? cv[k + u] : 0.0;
    }
    double xv[U][BP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double* px = xt + ((col[u] >= 0 && col[u] < nc) ? col[u] : 0) * BP;
#pragma unroll
      for (int q2 = 0; q2 < BP; ++q2) xv[u][q2] = px[q2];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (col[u] >= 0 && col[u] < nc) {
#pragma unroll
        for (int q2 = 0; q2 < BP; ++q2) acc[q2] += v[u] * xv[u][q2];
      }
    }
  }
#pragma unroll
  for (int q2 = 0; q2 < BP; ++q2)
    if (q2 < nb) out[(int64_t)(s0 + q2) * ntet + row] = acc[q2];
}

// ---------------------------------------------------------------------------
// warm start of a coupled fine solve: x = P u_c, the coarse cell field of the
// (n/2)^3 box injected into its 8 children (P0 prolongation, the nested
// piecewise-constant interpolation of the box hierarchy)

__global__ __launch_bounds__(kBlock) void k_inject_coarse(const double* __restrict__ uc, double* __restrict__ x,
                                                          int n, int batch) {
  const int64_t nc = (int64_t)n * n * n;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= nc * batch) return;
  const int slot = (int)(gid / nc);
  const int64_t c = gid - (int64_t)slot * nc;
  const int m = n >> 1;
  const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / ((int64_t)n * n));
  x[gid] = uc[(int64_t)slot * m * m * m + (i >> 1) + (int64_t)m * ((j >> 1) + (int64_t)m * (k >> 1))];
}

// ---------------------------------------------------------------------------
// noise restriction (eq. ml-linsys): xi_c[I] = 8^{-1/2} sum of the 8 children

__global__ __launch_bounds__(kBlock) void k_restrict_noise(const double* __restrict__ xf, double* __restrict__ xc,
                                                           int nf, int batch) {
  const int ncx = nf >> 1;
  const int64_t ncc = (int64_t)ncx * ncx * ncx;
  const int64_t nff = (int64_t)nf * nf * nf;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= ncc * batch) return;
  const int slot = (int)(gid / ncc);
  const int64_t C = gid - (int64_t)slot * ncc;
  const int I = (int)(C % ncx), J = (int)((C / ncx) % ncx), K = (int)(C / ((int64_t)ncx * ncx));
  const double* f = xf + (int64_t)slot * nff;
  double acc = 0.0;
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    const int i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
    acc += f[i + (int64_t)nf * (j + (int64_t)nf * k)];
  }
  xc[gid] = acc * 0.35355339059327376220;   // 1 / sqrt(8)
}

// ---------------------------------------------------------------------------
// layout conversions for the operator check: external -> internal Lanczos form
// (v_sigma = x_sigma / q so that q v_sigma = x_sigma, zhat = x_u), and back.

// zhat = x_u into the solver's z[0] in the multigrid precision TZ, v_sigma =
// x_sigma / q as above (the check of the production operator instances).
template <typename TZ>
__global__ __launch_bounds__(kBlock) void k_ext_to_int_zhat(const double* __restrict__ xs,
                                                            const double* __restrict__ xu, Fields F, Box bx, int nb) {
  const int slot = blockIdx.x / nb, blk = blockIdx.x - slot * nb;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  const int64_t nc = bx.nc;
  const int n = bx.n;
  if (c >= nc) return;
  const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / bx.n2);
  const int64_t nf = bx.n2 * (n + 1);
  const double* e = xs + (int64_t)slot * 3 * nf;
  const double iq = 1.0 / bx.q;
  F.vs[0][face_off(slot, 0, nc) + c] = i > 0 ? e[i + (int64_t)(n + 1) * (j + (int64_t)n * k)] * iq : 0.0;
  F.vs[0][face_off(slot, 1, nc) + c] = j > 0 ? e[nf + i + (int64_t)n * (j + (int64_t)(n + 1) * k)] * iq : 0.0;
  F.vs[0][face_off(slot, 2, nc) + c] = k > 0 ? e[2 * nf + i + (int64_t)n * (j + (int64_t)n * k)] * iq : 0.0;
  reinterpret_cast<TZ*>(F.z[0])[cell_off(slot, nc) + c] = (TZ)xu[cell_off(slot, nc) + c];
  F.vu[0][cell_off(slot, nc) + c] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_ext_to_int(const double* __restrict__ xs, const double* __restrict__ xu,
                                                       Fields F, Box bx, int nb) {
  const int slot = blockIdx.x / nb, blk = blockIdx.x - slot * nb;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  const int64_t nc = bx.nc;
  const int n = bx.n;
  if (c >= nc) return;
  const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / bx.n2);
  const int64_t nf = bx.n2 * (n + 1);
  const double* e = xs + (int64_t)slot * 3 * nf;
  const double iq = 1.0 / bx.q;
  F.vs[0][face_off(slot, 0, nc) + c] = i > 0 ? e[i + (int64_t)(n + 1) * (j + (int64_t)n * k)] * iq : 0.0;
  F.vs[0][face_off(slot, 1, nc) + c] = j > 0 ? e[nf + i + (int64_t)n * (j + (int64_t)(n + 1) * k)] * iq : 0.0;
  F.vs[0][face_off(slot, 2, nc) + c] = k > 0 ? e[2 * nf + i + (int64_t)n * (j + (int64_t)n * k)] * iq : 0.0;
  reinterpret_cast<double*>(F.z[0])[cell_off(slot, nc) + c] = xu[cell_off(slot, nc) + c];
  F.vu[0][cell_off(slot, nc) + c] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_int_to_ext(Fields F, double* __restrict__ ys, double* __restrict__ yu,
                                                       Box bx, int nb) {
  const int slot = blockIdx.x / nb, blk = blockIdx.x - slot * nb;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  const int64_t nc = bx.nc;
  const int n = bx.n;
  if (c >= nc) return;
  const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / bx.n2);
  const int64_t nf = bx.n2 * (n + 1);
  double* e = ys + (int64_t)slot * 3 * nf;
  e[i + (int64_t)(n + 1) * (j + (int64_t)n * k)] = F.vs[1][face_off(slot, 0, nc) + c];
  e[nf + i + (int64_t)n * (j + (int64_t)(n + 1) * k)] = F.vs[1][face_off(slot, 1, nc) + c];
  e[2 * nf + i + (int64_t)n * (j + (int64_t)n * k)] = F.vs[1][face_off(slot, 2, nc) + c];
  if (i == n - 1) e[n + (int64_t)(n + 1) * (j + (int64_t)n * k)] = 0.0;
  if (j == n - 1) e[nf + i + (int64_t)n * (n + (int64_t)(n + 1) * k)] = 0.0;
  if (k == n - 1) e[2 * nf + i + (int64_t)n * (j + (int64_t)n * n)] = 0.0;
  yu[cell_off(slot, nc) + c] = F.vu[1][cell_off(slot, nc) + c];
}

// Scalars of the operator check: z = (q v, zhat) / 1, no recurrence terms.
__global__ void k_probe_scalars(Scalars* sc, int batch) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch) return;
  Scalars v{};
  v.state = ST_ACTIVE; v.pit = 0; v.it = 0; v.zs = 1.0; v.a_v = 0.0; v.b_v = 0.0; v.wmode = -1; v.xpend = 0.0;
  sc[s] = v;
}

// Scalars of a steady-state iteration (an even pass with the previous vectors
// and the solution update) for timing the operator pass; the coefficients are
// zero, so whatever the vectors hold, nothing is read at a data-dependent place.
__global__ void k_tune_scalars(Scalars* sc, int batch) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch) return;
  Scalars v{};
  v.state = ST_ACTIVE; v.pit = 4; v.it = 4; v.wmode = 2; v.zs = 1.0;
  sc[s] = v;
}

// ---------------------------------------------------------------------------
// cell-wise kappa in the multigrid hierarchy (set-up, once per coefficient field)

// Finest level: k2_c = (kappa_c kappa_c) h^3, the reaction term of the cell row
// with the operator's rounding.
__global__ __launch_bounds__(kBlock) void k_mg_k2_fine(const double* __restrict__ kap, double h3,
                                                       double* __restrict__ k2, int64_t nc) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c < nc) k2[c] = (kap[c] * kap[c]) * h3;
}

// Galerkin reaction term of the next coarser level: P^T diag(k2_f) P with the
// P0 injection P is diagonal, each coarse cell holding the sum of its 8
// children (the coarse kappa^2 is the children's mean, eq. ml-linsys).
__global__ __launch_bounds__(kBlock) void k_mg_k2_coarsen(const double* __restrict__ k2f,
                                                          double* __restrict__ k2c, int mf) {
  const int mc = mf >> 1;
  const int64_t C = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (C >= (int64_t)mc * mc * mc) return;
  const int I = (int)(C % mc), J = (int)((C / mc) % mc), K = (int)(C / ((int64_t)mc * mc));
  double acc = 0.0;
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    const int i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
    acc += k2f[i + (int64_t)mf * (j + (int64_t)mf * k)];
  }
  k2c[C] = acc;
}

// Diagonal of S~ = K + a L on an m^3 level and its reciprocal, formed in
// float64 and rounded once to the level precision.
template <typename TM>
__global__ __launch_bounds__(kBlock) void k_mg_diag(const double* __restrict__ k2, int m, double a,
                                                    TM* __restrict__ dg, TM* __restrict__ dgi) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (int64_t)m * m * m) return;
  const int i = (int)(c % m), j = (int)((c / m) % m), k = (int)(c / ((int64_t)m * m));
  const double d = k2[c] + a * (double)nnbr(i, j, k, m);
  dg[c] = (TM)d;
  dgi[c] = (TM)(1.0 / d);
}

// Per-block minimum.
__global__ __launch_bounds__(kBlock) void k_block_min(const double* __restrict__ v, int64_t n,
                                                      double* __restrict__ out) {
  __shared__ double red[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double x = i < n ? v[i] : INFINITY;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < kBlock / 64; ++w) r = fmin(r, red[w]);
    out[blockIdx.x] = r;
  }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(kBlock) void k_convert(const TS* __restrict__ s, TD* __restrict__ d, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) d[i] = (TD)s[i];
}

}  // namespace spde

#include "spde_rng.inc"
#include "spde_transfer.inc"
#include "spde_launch.inc"
