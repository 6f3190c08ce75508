// Operator pass of the MINRES iteration (fused Lanczos recurrence, direction
// and solution updates), one-cell-per-thread and column forms.
#include "spde_common.inc"

namespace spde {

// ---------------------------------------------------------------------------
// operator pass of iteration j:
//   v_{j+1} = A z_j - a_v v_j - b_v v_{j-1},  z_j = (P_sigma^-1 v_sigma, zhat_u) / gamma_j
// and the delayed direction/solution update of step j-1.  One thread per
// cell: the cell value and the three low faces of the cell.
//   (M z)_face = (M P_sigma^-1 v)_f / gamma              (line_terms)
//   (B^T z_u)_face = h^2 (zhat[c - e_d] - zhat[c]) / gamma
//   (A z)_cell = (h^2 q sum_d (z_hi - z_lo) / q - kappa^2 h^3 zhat) / gamma

// UNI: every wave lies in one grid row (n >= 64), so the y and z line
// positions, and with them the y- and z-window offsets, are wave-uniform.
// POLY: face block of the preconditioner (0 diag(M)^-1, 1 Neumann series), a
// template parameter so that no window load sits behind a branch on it.
// VAR: cell-wise kappa (the reaction term kappa_c^2 h^3 of the cell row).
template <typename TZ, bool UNI, int POLY, bool VAR>
__global__ __launch_bounds__(kBlock) void k_operator(Fields F, Box bx, int nb) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = lb / nb, blk = lb - slot * nb;
  const Scalars* S = F.sc + slot;
  const int state = S->state;
  if (state != ST_ACTIVE && state != ST_FINISH) return;
  const int j = S->pit;
  const int p = j & 1, pq = p ^ 1;
  const int64_t nc = bx.nc;
  const int n = bx.n;
  const int64_t n2 = bx.n2;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c >= nc) return;
  const int i = (int)(c % n);
  int jj = (int)((c / n) % n), k = (int)(c / n2);
  if constexpr (UNI) {
    jj = __builtin_amdgcn_readfirstlane(jj);
    k = __builtin_amdgcn_readfirstlane(k);
  }
  const int64_t co = cell_off(slot, nc);
  const bool active = state == ST_ACTIVE;
  const bool has_prev = j > 1;
  const int wm = S->wmode;
  // x is written on even iterations and on the finishing pass; an odd
  // iteration leaves its term to the next pass (coefficient xpend of W_{j-1})
  const bool upd_x = wm >= 1 && ((j & 1) == 0 || state == ST_FINISH);
  const int idx[3] = {i, jj, k};
  const int64_t str[3] = {1, n, n2};
  // scalars before any store (after a store they could no longer be scalar loads)
  const double zs = S->zs, av = S->a_v, bv = S->b_v;
  const double sww = S->ww, swwp = S->ww_prev, sxw = S->xw, sxp = S->xpend;
  const bool acc = S->flags & FL_ACCUM;   // refinement pass: x holds the previous iterate

  // Direction and solution updates (unnormalised directions, see Scalars):
  //   W_{j+1} = zs zhat_j + ww W_j + ww_prev W_{j-1}      (W_j in w[pq], W_{j-1} in w[p])
  //   x += xpend W_{j-1} + xw W_j                          (even passes, the finishing pass)
  // The W store is unconditional (a pass without update writes back the old
  // value) so that the loads it needs stay ahead of the other stores.
  auto x_update = [&](double wj, double wjm1) {
    if (upd_x) {
      const double inc = sxp * wjm1 + sxw * wj;
      F.x[co + c] = (j == 2 && !acc) ? inc : F.x[co + c] + inc;
    }
  };
  if (!active) {   // the finishing pass only applies the last solution update
    x_update(F.w[pq][co + c], wm >= 2 ? F.w[p][co + c] : 0.0);
    return;
  }
  // All loads first, unconditionally (the addresses are valid in every state;
  // values that a state does not need are discarded).  The stores go through
  // pointers that may alias the loads, so a load after a store, or inside a
  // branch the compiler may sink below the stores, would cost the wave another
  // memory round trip.
  const TZ* z = reinterpret_cast<const TZ*>(F.z[p]) + co;
  double w[3][7], vo[3], zlo[3];
  const double zc = (double)z[c];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // radius 3 in either face-block mode (a branch here would split the
    // loads into groups that each wait for their own data)
    line_load_ext<3>(F.vs[p] + face_off(slot, d, nc), c, str[d], idx[d], n, w[d]);
    zlo[d] = (double)z[idx[d] > 0 ? c - str[d] : c];
    vo[d] = F.vs[pq][face_off(slot, d, nc) + c];
  }
  const double vuc = F.vu[p][co + c], vuo = F.vu[pq][co + c];
  const double wj = F.w[pq][co + c], wjm1 = F.w[p][co + c];
  // VAR: cell-wise kappa (shared by the slots), read with the other loads
  const double kc = VAR ? bx.kap[c] : 0.0;

  double dv = 0.0, nf[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double mz, zf, zh;
    line_terms_ext(w[d], POLY, mz, zf, zh);
    dv += zh - zf;
    const double a = zs * (mz + bx.h2 * (zlo[d] - zc));
    const double nv = a - av * w[d][3];
    nf[d] = idx[d] > 0 ? (has_prev ? nv - bv * vo[d] : nv) : 0.0;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) F.vs[pq][face_off(slot, d, nc) + c] = nf[d];
  const double k2 = VAR ? (kc * kc) * bx.h3 : bx.k2h3;
  const double Au = zs * (bx.h2q * dv - k2 * zc);
  const double nu = Au - av * vuc;
  F.vu[pq][co + c] = has_prev ? nu - bv * vuo : nu;
  double wn = zs * zc;
  if (wm >= 1) wn += sww * wj;
  if (wm >= 2) wn += swwp * wjm1;
  F.w[p][co + c] = wm >= 0 ? wn : wjm1;
  if (wm >= 1) x_update(wj, wm >= 2 ? wjm1 : 0.0);
}

// Column form of the operator pass for n a multiple of 64.  A block owns
// 64 x 4 cell columns (one grid row per wave) and walks ZC planes up z.  The
// z-window of the z faces slides in registers (one new plane per step), the z
// neighbour of zhat is the previous step's value, and each step stages the x
// faces of its 4 rows (with a 3-face halo along x) and the y faces of rows
// -3 .. +6 in LDS, from which the x and y windows are read.  Same arithmetic,
// in the same order, as k_operator.
// NT: the Lanczos, direction and solution vectors are streamed with the
// nontemporal hint (chosen by the launcher from the launch's working set).
template <typename TZ, int POLY, bool VAR, int ZC, bool NT>
__global__ __launch_bounds__(kBlock) void k_operator_col(Fields F, Box bx, int nb) {
  constexpr int XW = 64 + 6, AXF = XW * 4, RXF = (AXF + kBlock - 1) / kBlock;   // x faces, halo 3 in x
  constexpr int AYF = 64 * (4 + 6), RYF = (AYF + kBlock - 1) / kBlock;           // y faces, halo 3 in y
  __shared__ double sxf[2][AXF];
  __shared__ double syf[2][AYF];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = lb / nb, t = lb - slot * nb;
  const Scalars* S = F.sc + slot;
  const int state = S->state;
  if (state != ST_ACTIVE && state != ST_FINISH) return;
  const int j = S->pit;
  const int p = j & 1, pq = p ^ 1;
  const int64_t nc = bx.nc;
  const int n = bx.n;
  const int64_t n2 = bx.n2;
  const int tpx = n >> 6, tpy = n >> 2;
  const int x0 = (t % tpx) << 6, y0 = ((t / tpx) % tpy) << 2, z0 = (t / (tpx * tpy)) * ZC;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = x0 + lane;
  const int jj = __builtin_amdgcn_readfirstlane(y0 + wv);
  const int64_t col = i + (int64_t)n * jj;
  const int64_t co = cell_off(slot, nc);
  const bool active = state == ST_ACTIVE;
  const bool has_prev = j > 1;
  const int wm = S->wmode;
  const bool upd_x = wm >= 1 && ((j & 1) == 0 || state == ST_FINISH);
  const double zs = S->zs, av = S->a_v, bv = S->b_v;
  const double sww = S->ww, swwp = S->ww_prev, sxw = S->xw, sxp = S->xpend;
  const bool acc = S->flags & FL_ACCUM;   // refinement pass: x holds the previous iterate
  auto x_update = [&](int64_t c, double wj, double wjm1) {
    if (upd_x) {
      const double inc = sxp * wjm1 + sxw * wj;
      st_stream<NT>((j == 2 && !acc) ? inc : ld_stream<NT>(&F.x[co + c]) + inc, &F.x[co + c]);
    }
  };
  if (!active) {
    for (int kk = 0; kk < ZC; ++kk) {
      const int64_t c = col + n2 * (z0 + kk);
      x_update(c, F.w[pq][co + c], wm >= 2 ? F.w[p][co + c] : 0.0);
    }
    return;
  }
  // staged items: byte offset within a plane and the odd-reflection factor
  uint32_t xo[RXF], yo[RYF];
  double xf[RXF], yf[RYF];
#pragma unroll
  for (int r = 0; r < RXF; ++r) {
    const int q = tid + r * kBlock;
    const int gx = x0 + q % XW - 3, gy = y0 + q / XW;
    const bool neg = gx < 0 || gx > n;
    const int src = gx < 0 ? -gx : (gx > n ? 2 * n - gx : gx);
    xo[r] = q < AXF ? (uint32_t)(min(src, n - 1) + n * gy) * 8u : 0u;
    xf[r] = (q >= AXF || src == n) ? 0.0 : (neg ? -1.0 : 1.0);
  }
#pragma unroll
  for (int r = 0; r < RYF; ++r) {
    const int q = tid + r * kBlock;
    const int gx = x0 + q % 64, gy = y0 + q / 64 - 3;
    const bool neg = gy < 0 || gy > n;
    const int src = gy < 0 ? -gy : (gy > n ? 2 * n - gy : gy);
    yo[r] = q < AYF ? (uint32_t)(gx + n * min(src, n - 1)) * 8u : 0u;
    yf[r] = (q >= AYF || src == n) ? 0.0 : (neg ? -1.0 : 1.0);
  }
  const TZ* z = reinterpret_cast<const TZ*>(F.z[p]) + co;
  const double* vs0 = F.vs[p] + face_off(slot, 0, nc);
  const double* vs1 = F.vs[p] + face_off(slot, 1, nc);
  const double* vz = F.vs[p] + face_off(slot, 2, nc) + col;
  // z face of plane g of this column, odd reflection about the boundary faces
  // 0 and n (the plane index is block-uniform, so the reflection is scalar)
  auto face_z = [&](int g) {
    const bool neg = g < 0 || g > n;
    const int src = g < 0 ? -g : (g > n ? 2 * n - g : g);
    const double x = vz[n2 * min(src, n - 1)];
    return x * (src == n ? 0.0 : (neg ? -1.0 : 1.0));
  };
  double wz[7];
#pragma unroll
  for (int q = 0; q < 6; ++q) wz[q] = face_z(z0 - 3 + q);
  double zprev = (double)z[col + n2 * max(z0 - 1, 0)];
  for (int kk = 0; kk < ZC; ++kk) {
    const int k = z0 + kk;
    const int64_t pk = n2 * k;
    const int64_t c = col + pk;
    const int b = kk & 1;
    // stage this plane's x and y faces (the buffer written two steps ago has
    // been read by everyone: the previous step's barrier lies between)
    const double* px = vs0 + pk;
    const double* py = vs1 + pk;
#pragma unroll
    for (int r = 0; r < RXF; ++r) {
      const int q = tid + r * kBlock;
      if ((r + 1) * kBlock <= AXF || q < AXF) sxf[b][q] = ld_off(px, xo[r]) * xf[r];
    }
#pragma unroll
    for (int r = 0; r < RYF; ++r) {
      const int q = tid + r * kBlock;
      if ((r + 1) * kBlock <= AYF || q < AYF) syf[b][q] = ld_off(py, yo[r]) * yf[r];
    }
    wz[6] = face_z(k + 3);
    double vo[3];
    const double zc = (double)z[c];
    const double zlo[3] = {(double)z[i > 0 ? c - 1 : c], (double)z[jj > 0 ? c - n : c], k > 0 ? zprev : zc};
#pragma unroll
    for (int d = 0; d < 3; ++d) vo[d] = ld_stream<NT>(&F.vs[pq][face_off(slot, d, nc) + c]);
    const double vuc = ld_stream<NT>(&F.vu[p][co + c]), vuo = ld_stream<NT>(&F.vu[pq][co + c]);
    const double wj = ld_stream<NT>(&F.w[pq][co + c]), wjm1 = ld_stream<NT>(&F.w[p][co + c]);
    const double kc = VAR ? bx.kap[c] : 0.0;
    __syncthreads();
    double w[2][7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      w[0][q] = sxf[b][lane + q + XW * wv];
      w[1][q] = syf[b][lane + 64 * (wv + q)];
    }
    const int idx[3] = {i, jj, k};
    double dv = 0.0, nf[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* wd = d == 2 ? wz : w[d];
      double mz, zf, zh;
      line_terms_ext(wd, POLY, mz, zf, zh);
      dv += zh - zf;
      const double a = zs * (mz + bx.h2 * (zlo[d] - zc));
      const double nv = a - av * wd[3];
      nf[d] = idx[d] > 0 ? (has_prev ? nv - bv * vo[d] : nv) : 0.0;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) st_stream<NT>(nf[d], &F.vs[pq][face_off(slot, d, nc) + c]);
    const double k2 = VAR ? (kc * kc) * bx.h3 : bx.k2h3;
    const double Au = zs * (bx.h2q * dv - k2 * zc);
    const double nu = Au - av * vuc;
    st_stream<NT>(has_prev ? nu - bv * vuo : nu, &F.vu[pq][co + c]);
    double wn = zs * zc;
    if (wm >= 1) wn += sww * wj;
    if (wm >= 2) wn += swwp * wjm1;
    st_stream<NT>(wm >= 0 ? wn : wjm1, &F.w[p][co + c]);
    if (wm >= 1) x_update(c, wj, wm >= 2 ? wjm1 : 0.0);
#pragma unroll
    for (int q = 0; q < 6; ++q) wz[q] = wz[q + 1];
    zprev = zc;
  }
}


// planes per block of the column form of the operator pass
constexpr int kOpZC = 16;
// The column pass streams its vectors with the nontemporal hint when the
// launch's vectors (about 128 bytes per cell and sample) exceed this size.
// MI355X has a 256 MB last-level cache: one 128^3 sample (about 265 MB) still
// runs faster without the hint (its vectors largely stay cached between
// passes), two or more run faster with it.
constexpr double kOpStreamBytes = 384.0 * 1024 * 1024;

hipError_t launch_operator(bool z_fp64, const Fields& F, const Box& bx, int batch, hipStream_t st) {
  if (bx.n % 64 == 0 && bx.n % kOpZC == 0) {
    // 64 x 4 columns of kOpZC planes per block
    const int nbc = (bx.n / 64) * (bx.n / 4) * (bx.n / kOpZC);
    const dim3 gridc(nbc * batch), blkc(kBlock);
    const bool nt = 128.0 * (double)bx.nc * (double)batch > kOpStreamBytes;
#define SPDE_OPC(TZ, NT)                                                                                        \
  do {                                                                                                          \
    if (bx.kap) {                                                                                               \
      if (bx.poly) hipLaunchKernelGGL((k_operator_col<TZ, 1, true, kOpZC, NT>), gridc, blkc, 0, st, F, bx, nbc);  \
      else hipLaunchKernelGGL((k_operator_col<TZ, 0, true, kOpZC, NT>), gridc, blkc, 0, st, F, bx, nbc);          \
    } else {                                                                                                    \
      if (bx.poly) hipLaunchKernelGGL((k_operator_col<TZ, 1, false, kOpZC, NT>), gridc, blkc, 0, st, F, bx, nbc); \
      else hipLaunchKernelGGL((k_operator_col<TZ, 0, false, kOpZC, NT>), gridc, blkc, 0, st, F, bx, nbc);         \
    }                                                                                                           \
  } while (0)
    if (z_fp64) {
      if (nt) SPDE_OPC(double, true);
      else SPDE_OPC(double, false);
    } else {
      if (nt) SPDE_OPC(float, true);
      else SPDE_OPC(float, false);
    }
#undef SPDE_OPC
    return hipGetLastError();
  }
  const int nb = operator_blocks(bx);
  const dim3 grid(nb * batch), blk(kBlock);
  // with n >= 64 every 64-lane wave lies in one grid row
#define SPDE_OP(TZ, UNI)                                                                             \
  do {                                                                                               \
    if (bx.kap) {                                                                                    \
      if (bx.poly) hipLaunchKernelGGL((k_operator<TZ, UNI, 1, true>), grid, blk, 0, st, F, bx, nb);  \
      else hipLaunchKernelGGL((k_operator<TZ, UNI, 0, true>), grid, blk, 0, st, F, bx, nb);          \
    } else {                                                                                         \
      if (bx.poly) hipLaunchKernelGGL((k_operator<TZ, UNI, 1, false>), grid, blk, 0, st, F, bx, nb); \
      else hipLaunchKernelGGL((k_operator<TZ, UNI, 0, false>), grid, blk, 0, st, F, bx, nb);         \
    }                                                                                                \
  } while (0)
  if (bx.n >= 64) {
    if (z_fp64) SPDE_OP(double, true);
    else SPDE_OP(float, true);
  } else {
    if (z_fp64) SPDE_OP(double, false);
    else SPDE_OP(float, false);
  }
#undef SPDE_OP
  return hipGetLastError();
}

}  // namespace spde
