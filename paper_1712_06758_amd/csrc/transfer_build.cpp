// Host construction of the L2 projection Pi = W_h^-1 G between the structured
// box and a non-matching tetrahedral mesh (Sec. "L2-Projection", eq. proj_op,
// and Sec. "Implementation details of the L2-projection operator").
//
// With piecewise-constant spaces on both meshes G[t, c] = vol(t intersect c)
// and W_h = diag(vol t), so Pi[t, c] = vol(t intersect c) / vol(t).  The paper
// meshes each intersection into simplices and integrates with quadrature; for
// a constant integrand that is the intersection volume, computed here exactly
// (up to rounding) by clipping.
//
// The box grid is implicit, so no search structure is needed: the candidate
// cells of a tet are the cells met by its bounding box.  The tet is first cut
// into x-slabs of the grid, each slab piece into y-slabs, each of those into
// z-slabs; every cut keeps a list of tetrahedra (a tet cut by a plane leaves
// 1, 2 or 3 tets on each side).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace spde {

namespace {

struct V3 { double x[3]; };
struct Tet { V3 p[4]; };

inline V3 lerp(const V3& a, const V3& b, double t) {
  V3 r;
  for (int d = 0; d < 3; ++d) r.x[d] = a.x[d] + t * (b.x[d] - a.x[d]);
  return r;
}

inline double tet_vol(const Tet& t) {
  double e[3][3];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) e[i][d] = t.p[i + 1].x[d] - t.p[0].x[d];
  const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                     e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                     e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
  return std::fabs(det) / 6.0;
}

// Keep the part of `t` with sign * (x_d - c) <= 0, appending tets to `out`.
// A wedge (two triangles joined by three edges) is split into the 3 tets
// (a0 a1 a2 b0), (a1 a2 b0 b1), (a2 b0 b1 b2).
void clip_keep(const Tet& t, int d, double c, double sign, std::vector<Tet>& out) {
  double s[4];
  int in[4], ni = 0, outi[4], no = 0;
  for (int i = 0; i < 4; ++i) {
    s[i] = sign * (t.p[i].x[d] - c);
    if (s[i] <= 0.0) in[ni++] = i; else outi[no++] = i;
  }
  if (ni == 0) return;
  if (no == 0) { out.push_back(t); return; }
  auto cut = [&](int a, int b) {  // a inside (s <= 0), b outside (s > 0)
    const double tt = s[a] / (s[a] - s[b]);
    V3 r = lerp(t.p[a], t.p[b], tt);
    r.x[d] = c;
    return r;
  };
  if (ni == 1) {
    const int a = in[0];
    Tet r{{t.p[a], cut(a, outi[0]), cut(a, outi[1]), cut(a, outi[2])}};
    out.push_back(r);
  } else if (ni == 3) {
    const int o = outi[0];
    const V3 a0 = t.p[in[0]], a1 = t.p[in[1]], a2 = t.p[in[2]];
    const V3 b0 = cut(in[0], o), b1 = cut(in[1], o), b2 = cut(in[2], o);
    out.push_back(Tet{{a0, a1, a2, b0}});
    out.push_back(Tet{{a1, a2, b0, b1}});
    out.push_back(Tet{{a2, b0, b1, b2}});
  } else {  // two inside (a, b), two outside (c, e): wedge with ends (a, ac, ae), (b, bc, be)
    const int a = in[0], b = in[1], c1 = outi[0], e = outi[1];
    const V3 A0 = t.p[a], A1 = cut(a, c1), A2 = cut(a, e);
    const V3 B0 = t.p[b], B1 = cut(b, c1), B2 = cut(b, e);
    out.push_back(Tet{{A0, A1, A2, B0}});
    out.push_back(Tet{{A1, A2, B0, B1}});
    out.push_back(Tet{{A2, B0, B1, B2}});
  }
}

// Part of the tet list inside the slab lo <= x_d <= hi.
void slab(const std::vector<Tet>& in, int d, double lo, double hi, std::vector<Tet>& tmp,
          std::vector<Tet>& out) {
  tmp.clear();
  out.clear();
  for (const Tet& t : in) clip_keep(t, d, hi, 1.0, tmp);     // x_d <= hi
  for (const Tet& t : tmp) clip_keep(t, d, lo, -1.0, out);   // x_d >= lo
}

struct RowBuf {
  std::vector<int64_t> len;     // entries per row (rows of this chunk)
  std::vector<int32_t> col;
  std::vector<double> val;
};

}  // namespace

// Returns 0 on success, -1 on invalid input (message in err).
int build_transfer_csr(int n, int64_t n_vert, const double* xyz, int64_t n_tet, const int32_t* tets,
                       std::vector<int64_t>& row_ptr, std::vector<int32_t>& cols, std::vector<double>& vals,
                       char* err, size_t errlen) {
  for (int64_t v = 0; v < n_vert * 3; ++v) {
    if (!(xyz[v] >= 0.0 && xyz[v] <= 1.0)) {
      snprintf(err, errlen, "vertex %lld lies outside [0,1]^3", (long long)(v / 3));
      return -1;
    }
  }
  for (int64_t t = 0; t < n_tet * 4; ++t) {
    if (tets[t] < 0 || tets[t] >= n_vert) {
      snprintf(err, errlen, "tet %lld references vertex %d out of range", (long long)(t / 4), tets[t]);
      return -1;
    }
  }
  const double h = 1.0 / n;
  unsigned nth = std::thread::hardware_concurrency();
  if (nth == 0) nth = 1;
  if (nth > 64) nth = 64;
  const int64_t chunk = 4096;
  const int64_t nchunks = (n_tet + chunk - 1) / chunk;
  std::vector<RowBuf> bufs(nchunks);
  std::atomic<int64_t> next{0};
  std::atomic<int64_t> bad{-1};

  auto worker = [&]() {
    std::vector<Tet> a, b, c, tmp, leaf;
    for (;;) {
      const int64_t ch = next.fetch_add(1);
      if (ch >= nchunks) break;
      RowBuf& rb = bufs[ch];
      const int64_t t0 = ch * chunk, t1 = std::min(n_tet, t0 + chunk);
      rb.len.assign(t1 - t0, 0);
      for (int64_t t = t0; t < t1; ++t) {
        Tet T;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int v = 0; v < 4; ++v) {
          const int64_t vi = tets[t * 4 + v];
          for (int d = 0; d < 3; ++d) {
            T.p[v].x[d] = xyz[vi * 3 + d];
            lo[d] = std::min(lo[d], T.p[v].x[d]);
            hi[d] = std::max(hi[d], T.p[v].x[d]);
          }
        }
        const double vol = tet_vol(T);
        if (!(vol > 0.0)) {
          int64_t expect = -1;
          bad.compare_exchange_strong(expect, t);
          continue;
        }
        int i0[3], i1[3];
        for (int d = 0; d < 3; ++d) {
          i0[d] = std::max(0, std::min(n - 1, (int)std::floor(lo[d] / h)));
          i1[d] = std::max(0, std::min(n - 1, (int)std::floor(hi[d] / h)));
        }
        const size_t before = rb.col.size();
        a.assign(1, T);
        for (int k = i0[2]; k <= i1[2]; ++k) {
          slab(a, 2, k * h, (k + 1) * h, tmp, b);
          if (b.empty()) continue;
          for (int j = i0[1]; j <= i1[1]; ++j) {
            slab(b, 1, j * h, (j + 1) * h, tmp, c);
            if (c.empty()) continue;
            for (int i = i0[0]; i <= i1[0]; ++i) {
              slab(c, 0, i * h, (i + 1) * h, tmp, leaf);
              double v = 0.0;
              for (const Tet& q : leaf) v += tet_vol(q);
              if (v > 1e-15 * vol) {
                rb.col.push_back((int32_t)(i + n * (j + n * k)));
                rb.val.push_back(v / vol);
              }
            }
          }
        }
        // columns in ascending order (cell index grows with k, then j, then i)
        rb.len[t - t0] = (int64_t)(rb.col.size() - before);
      }
    }
  };
  std::vector<std::thread> th;
  for (unsigned i = 0; i < nth; ++i) th.emplace_back(worker);
  for (auto& x : th) x.join();
  if (bad.load() >= 0) {
    snprintf(err, errlen, "tet %lld is degenerate (zero volume)", (long long)bad.load());
    return -1;
  }
  row_ptr.assign(n_tet + 1, 0);
  int64_t nnz = 0;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int64_t t0 = ch * chunk;
    for (size_t r = 0; r < bufs[ch].len.size(); ++r) {
      row_ptr[t0 + r] = nnz;
      nnz += bufs[ch].len[r];
    }
  }
  row_ptr[n_tet] = nnz;
  cols.resize(nnz);
  vals.resize(nnz);
  int64_t pos = 0;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    std::memcpy(cols.data() + pos, bufs[ch].col.data(), bufs[ch].col.size() * sizeof(int32_t));
    std::memcpy(vals.data() + pos, bufs[ch].val.data(), bufs[ch].val.size() * sizeof(double));
    pos += (int64_t)bufs[ch].col.size();
    RowBuf().len.swap(bufs[ch].len);
  }
  return 0;
}

// Pi of the (n_fine/2)^3 box onto the same tet mesh from Pi of the n_fine^3
// box (eq. recursive_l2_projection with the box hierarchy's P0 injection and
// the tet mesh kept): the overlap of a tet with a coarse cell is the sum of its
// overlaps with the 8 children, so Pi_c[t, I] = sum over the children c of I of
// Pi_f[t, c].  Each row's children are summed in the order of the fine row;
// the coarse columns come out ascending.  Returns 0, or -1 on invalid input.
int coarsen_transfer_csr(int n_fine, int64_t n_rows, const int64_t* rp, const int32_t* ci, const double* cv,
                         std::vector<int64_t>& rp_c, std::vector<int32_t>& ci_c, std::vector<double>& cv_c,
                         char* err, size_t errlen) {
  const int m = n_fine / 2;
  const int64_t ncf = (int64_t)n_fine * n_fine * n_fine;
  if (rp[0] != 0) {
    snprintf(err, errlen, "row_ptr[0] must be 0");
    return -1;
  }
  for (int64_t r = 0; r < n_rows; ++r) {
    if (rp[r + 1] < rp[r]) {
      snprintf(err, errlen, "row_ptr decreases at row %lld", (long long)r);
      return -1;
    }
  }
  for (int64_t k = 0; k < rp[n_rows]; ++k) {
    if (ci[k] < 0 || ci[k] >= ncf) {
      snprintf(err, errlen, "column %d at entry %lld lies outside the %d^3 box", ci[k], (long long)k, n_fine);
      return -1;
    }
  }
  rp_c.assign(n_rows + 1, 0);
  std::vector<int32_t> pc(rp[n_rows]);
  std::vector<double> pv(rp[n_rows]);
  // rows are independent: map, stable-sort by parent, merge (in place within the row's fine range)
  unsigned nth = std::thread::hardware_concurrency();
  if (nth == 0) nth = 1;
  if (nth > 64) nth = 64;
  std::vector<int64_t> len(n_rows, 0);
  std::atomic<int64_t> next{0};
  const int64_t chunk = 16384;
  auto worker = [&]() {
    std::vector<std::pair<int32_t, int32_t>> key;   // (parent, position in the row)
    for (;;) {
      const int64_t r0 = next.fetch_add(chunk);
      if (r0 >= n_rows) break;
      const int64_t r1 = std::min(n_rows, r0 + chunk);
      for (int64_t r = r0; r < r1; ++r) {
        const int64_t k0 = rp[r], k1 = rp[r + 1];
        key.clear();
        for (int64_t k = k0; k < k1; ++k) {
          const int32_t c = ci[k];
          const int i = c % n_fine, j = (c / n_fine) % n_fine, kk = c / (n_fine * n_fine);
          key.push_back({(int32_t)((i >> 1) + m * ((j >> 1) + m * (kk >> 1))), (int32_t)(k - k0)});
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                           return a.first < b.first;
                         });
        int64_t out = k0;
        for (size_t e = 0; e < key.size(); ++e) {
          const double v = cv[k0 + key[e].second];
          if (e > 0 && key[e].first == key[e - 1].first) {
            pv[out - 1] += v;
          } else {
            pc[out] = key[e].first;
            pv[out] = v;
            ++out;
          }
        }
        len[r] = out - k0;
      }
    }
  };
  std::vector<std::thread> th;
  for (unsigned i = 0; i < nth; ++i) th.emplace_back(worker);
  for (auto& x : th) x.join();
  int64_t nnz = 0;
  for (int64_t r = 0; r < n_rows; ++r) {
    rp_c[r] = nnz;
    nnz += len[r];
  }
  rp_c[n_rows] = nnz;
  ci_c.resize(nnz);
  cv_c.resize(nnz);
  for (int64_t r = 0; r < n_rows; ++r) {
    std::memcpy(ci_c.data() + rp_c[r], pc.data() + rp[r], len[r] * sizeof(int32_t));
    std::memcpy(cv_c.data() + rp_c[r], pv.data() + rp[r], len[r] * sizeof(double));
  }
  return 0;
}

}  // namespace spde
