// Seeded input generator: builds the serialized H^2 representation of a kernel
// matrix K_ij = kappa(p_i, p_j) on a point set, by the construction the paper
// uses for its test matrices (Section 6.1 and Section 6.4): a k-d tree over the
// points, a geometric admissibility condition
//     eta * |C_t - C_s| >= (D_t + D_s) / 2
// (C = centre, D = diagonal length of the cluster's bounding box), low-rank
// blocks from tensor Chebyshev interpolation of the kernel on the bounding
// boxes, and dense blocks by direct kernel evaluation.
//
// This file produces inputs only.  It holds no part of the matrix-vector
// product; the layout it writes is described in h2gen/fmt.py.
//
// Readings of points the paper leaves open (k-d split rule, Chebyshev node
// family, box choice, degenerate boxes, the singular kernel at r = 0) are the
// ones listed in the design notes: uniform-depth tree, longest-extent split,
// first-kind Chebyshev nodes on the tight box, widening of degenerate extents,
// and kappa = 0 for the Laplace kernel at r = 0.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include <omp.h>

namespace {

enum KernelId { K_EXP = 1, K_LAPLACE = 2, K_POLY2 = 3, K_ONE = 4, K_GAUSS = 5 };

constexpr int64_t kHeader = 128;
constexpr int64_t kAlign = 64;

inline int64_t align64(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline double kernel_eval(int id, double par, const double* x, const double* y, int dim) {
  double r2 = 0.0, dot = 0.0;
  for (int d = 0; d < dim; ++d) {
    double t = x[d] - y[d];
    r2 += t * t;
    dot += x[d] * y[d];
  }
  switch (id) {
    case K_EXP: return std::exp(-std::sqrt(r2) / par);
    case K_LAPLACE: return r2 == 0.0 ? 0.0 : 1.0 / (4.0 * M_PI * std::sqrt(r2));
    case K_POLY2: return (1.0 + dot) * (1.0 + dot);
    case K_ONE: return 1.0;
    case K_GAUSS: return std::exp(-r2 / (par * par));
    default: return 0.0;
  }
}

struct Box {
  double lo[3], hi[3];
};

// Lagrange basis polynomial j on nodes xi[0..p) evaluated at x.
inline double lagrange(const double* xi, int p, int j, double x) {
  double v = 1.0;
  for (int i = 0; i < p; ++i)
    if (i != j) v *= (x - xi[i]) / (xi[j] - xi[i]);
  return v;
}

}  // namespace

extern "C" {

// Build the representation.  pts: n x dim, point-major, original order.
// Returns 0 on success and a malloc'd buffer in *out (free with h2gen_free).
// Error codes: -1 bad arguments, -4 out of memory.
int h2gen_build(const double* pts, int64_t n, int64_t dim, int64_t leaf, int64_t p,
                double eta, int kernel_id, double kparam, int store_points,
                uint8_t** out, int64_t* out_len) {
  if (!pts || !out || !out_len || n < 1 || dim < 1 || dim > 3 || leaf < 1 || p < 1 || p > 16)
    return -1;
  int64_t k = 1;
  for (int d = 0; d < dim; ++d) k *= p;

  // ---- k-d tree of uniform depth q: smallest q with ceil(n / 2^q) <= leaf ----
  int q = 0;
  while (((n + (int64_t(1) << q) - 1) >> q) > leaf) ++q;
  const int64_t nnodes = (int64_t(2) << q) - 1;
  std::vector<int64_t> lo(nnodes), hi(nnodes), parent(nnodes);
  std::vector<Box> box(nnodes);
  std::vector<int64_t> idx(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  lo[0] = 0; hi[0] = n; parent[0] = -1;

  double rootdiag = 0.0;
  for (int l = 0; l <= q; ++l) {
    const int64_t first = (int64_t(1) << l) - 1, cnt = int64_t(1) << l;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < cnt; ++j) {
      const int64_t t = first + j;
      Box b;
      for (int d = 0; d < 3; ++d) { b.lo[d] = 0.0; b.hi[d] = 0.0; }
      if (hi[t] > lo[t]) {
        for (int d = 0; d < dim; ++d) { b.lo[d] = INFINITY; b.hi[d] = -INFINITY; }
        for (int64_t i = lo[t]; i < hi[t]; ++i)
          for (int d = 0; d < dim; ++d) {
            double v = pts[idx[i] * dim + d];
            b.lo[d] = std::min(b.lo[d], v);
            b.hi[d] = std::max(b.hi[d], v);
          }
      } else if (t > 0) {
        b = box[parent[t]];  // empty node: inherit the parent's box
      }
      box[t] = b;
      if (l < q) {
        int sd = 0;
        double best = -1.0;
        for (int d = 0; d < dim; ++d)
          if (b.hi[d] - b.lo[d] > best) { best = b.hi[d] - b.lo[d]; sd = d; }
        std::sort(idx.begin() + lo[t], idx.begin() + hi[t], [&](int64_t a, int64_t c) {
          double va = pts[a * dim + sd], vc = pts[c * dim + sd];
          return va < vc || (va == vc && a < c);
        });
        const int64_t len = hi[t] - lo[t];
        const int64_t mid = lo[t] + (len + 1) / 2;
        const int64_t c0 = 2 * t + 1, c1 = 2 * t + 2;
        lo[c0] = lo[t]; hi[c0] = mid; parent[c0] = t;
        lo[c1] = mid; hi[c1] = hi[t]; parent[c1] = t;
      }
    }
    if (l == 0) {
      double s = 0.0;
      for (int d = 0; d < dim; ++d) s += (box[0].hi[d] - box[0].lo[d]) * (box[0].hi[d] - box[0].lo[d]);
      rootdiag = std::sqrt(s);
      if (rootdiag == 0.0) rootdiag = 1.0;
    }
  }
  // Widen degenerate extents so the Chebyshev grids are well defined.
  const double minh = 1e-12 * rootdiag;
  std::vector<double> cen(nnodes * 3), half(nnodes * 3), diag(nnodes);
  for (int64_t t = 0; t < nnodes; ++t) {
    double s = 0.0;
    for (int d = 0; d < dim; ++d) {
      double c = 0.5 * (box[t].lo[d] + box[t].hi[d]);
      double h = std::max(0.5 * (box[t].hi[d] - box[t].lo[d]), minh);
      cen[t * 3 + d] = c; half[t * 3 + d] = h;
      s += 4.0 * h * h;
    }
    diag[t] = std::sqrt(s);
  }

  // ---- dual-tree traversal: admissible pairs per level, dense leaf pairs ----
  std::vector<std::vector<std::pair<int64_t, int64_t>>> adm(q + 1);
  std::vector<std::pair<int64_t, int64_t>> dense, cur{{0, 0}}, next;
  for (int l = 0; l <= q; ++l) {
    next.clear();
    for (auto& ts : cur) {
      const int64_t t = ts.first, s = ts.second;
      double dist2 = 0.0;
      for (int d = 0; d < dim; ++d) {
        double v = cen[t * 3 + d] - cen[s * 3 + d];
        dist2 += v * v;
      }
      const bool admissible = t != s && eta * std::sqrt(dist2) >= 0.5 * (diag[t] + diag[s]);
      if (admissible) {
        adm[l].push_back(ts);
      } else if (l == q) {
        dense.push_back(ts);
      } else {
        for (int64_t a = 1; a <= 2; ++a)
          for (int64_t b = 1; b <= 2; ++b) next.push_back({2 * t + a, 2 * s + b});
      }
    }
    std::sort(adm[l].begin(), adm[l].end());
    std::swap(cur, next);
  }
  std::sort(dense.begin(), dense.end());
  const int64_t leaf0 = (int64_t(1) << q) - 1, nleaves = int64_t(1) << q;

  // ---- section sizes and offsets (layout of h2gen/fmt.py) ----
  const int64_t nsec = 19;
  int64_t cnt[nsec];
  int64_t nadm_tot = 0;
  for (int l = 0; l <= q; ++l) nadm_tot += (int64_t)adm[l].size();
  int64_t e_sz = 0;
  for (int l = 1; l <= q; ++l) e_sz += (int64_t(1) << l) * k * k;
  std::vector<int64_t> d_off(dense.size() + 1, 0);
  for (size_t b = 0; b < dense.size(); ++b) {
    int64_t t = dense[b].first, s = dense[b].second;
    d_off[b + 1] = d_off[b] + (hi[t] - lo[t]) * (hi[s] - lo[s]);
  }
  cnt[0] = q + 2; cnt[1] = q + 1; cnt[2] = q + 1; cnt[3] = q + 1;
  cnt[4] = n; cnt[5] = nnodes; cnt[6] = nnodes; cnt[7] = nnodes;
  cnt[8] = nnodes + q + 1; cnt[9] = nadm_tot;
  cnt[10] = nleaves + 1; cnt[11] = (int64_t)dense.size();
  cnt[12] = n * k; cnt[13] = e_sz; cnt[14] = 0; cnt[15] = 0;
  cnt[16] = nadm_tot * k * k; cnt[17] = d_off.back();
  cnt[18] = store_points ? n * dim : 0;
  int64_t off[nsec];
  int64_t pos = kHeader;
  for (int s = 0; s < nsec; ++s) {
    pos = align64(pos);
    off[s] = pos;
    pos += 8 * cnt[s];
  }
  const int64_t total = align64(pos);
  uint8_t* buf = static_cast<uint8_t*>(std::malloc(total));
  if (!buf) return -4;
  // zero header and the padding gaps; data sections are overwritten below
  std::memset(buf, 0, kHeader);
  for (int s = 0; s < nsec; ++s) {
    int64_t end = off[s] + 8 * cnt[s];
    int64_t nxt = s + 1 < nsec ? off[s + 1] : total;
    std::memset(buf + end, 0, nxt - end);
  }
  auto I = [&](int s) { return reinterpret_cast<int64_t*>(buf + off[s]); };
  auto F = [&](int s) { return reinterpret_cast<double*>(buf + off[s]); };

  std::memcpy(buf, "H2MATV01", 8);
  uint32_t ver = 1, flags = store_points ? 2u : 0u;
  std::memcpy(buf + 8, &ver, 4);
  std::memcpy(buf + 12, &flags, 4);
  int64_t hd[4] = {n, q, nnodes, store_points ? dim : 0};
  std::memcpy(buf + 16, hd, 32);
  int64_t kid = kernel_id;
  std::memcpy(buf + 48, &kid, 8);
  double hf[2] = {kparam, eta};
  std::memcpy(buf + 56, hf, 16);
  int64_t ht[4] = {p, leaf, (int64_t)dense.size(), total};
  std::memcpy(buf + 72, ht, 32);

  for (int l = 0; l <= q + 1; ++l) I(0)[l] = (int64_t(1) << l) - 1;
  for (int l = 0; l <= q; ++l) { I(1)[l] = k; I(2)[l] = k; I(3)[l] = (int64_t)adm[l].size(); }
  std::memcpy(I(4), idx.data(), 8 * n);
  std::memcpy(I(5), lo.data(), 8 * nnodes);
  std::memcpy(I(6), hi.data(), 8 * nnodes);
  std::memcpy(I(7), parent.data(), 8 * nnodes);
  {
    int64_t* rp = I(8);
    int64_t* cl = I(9);
    int64_t rpos = 0, cpos = 0;
    for (int l = 0; l <= q; ++l) {
      const int64_t first = (int64_t(1) << l) - 1, nl = int64_t(1) << l;
      int64_t b = 0;
      for (int64_t r = 0; r < nl; ++r) {
        rp[rpos++] = b;
        while (b < (int64_t)adm[l].size() && adm[l][b].first == first + r) {
          cl[cpos++] = adm[l][b].second - first;
          ++b;
        }
      }
      rp[rpos++] = b;
    }
    int64_t* drp = I(10);
    int64_t* dcl = I(11);
    int64_t b = 0;
    for (int64_t r = 0; r < nleaves; ++r) {
      drp[r] = b;
      while (b < (int64_t)dense.size() && dense[b].first == leaf0 + r) {
        dcl[b] = dense[b].second - leaf0;
        ++b;
      }
    }
    drp[nleaves] = b;
  }

  // ---- Chebyshev grids: per node, per dimension, p first-kind nodes ----
  std::vector<double> grid(nnodes * 3 * p);
  for (int64_t t = 0; t < nnodes; ++t)
    for (int d = 0; d < dim; ++d)
      for (int j = 0; j < p; ++j)
        grid[(t * 3 + d) * p + j] =
            cen[t * 3 + d] + half[t * 3 + d] * std::cos((2.0 * j + 1.0) * M_PI / (2.0 * p));
  // tensor index alpha = a0 + p*a1 + p^2*a2
  auto tensor_point = [&](int64_t t, int64_t alpha, double* xo) {
    for (int d = 0; d < dim; ++d) {
      xo[d] = grid[(t * 3 + d) * p + alpha % p];
      alpha /= p;
    }
  };

  // ---- leaf bases U_t[i, alpha] = prod_d L^t_{alpha_d}(x_{i,d}) ----
  double* U = F(12);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < nleaves; ++j) {
    const int64_t t = leaf0 + j, m = hi[t] - lo[t];
    std::vector<double> L(3 * p);
    double* Ut = U + lo[t] * k;
    for (int64_t i = 0; i < m; ++i) {
      const double* x = pts + idx[lo[t] + i] * dim;
      for (int d = 0; d < dim; ++d)
        for (int a = 0; a < p; ++a) L[d * p + a] = lagrange(&grid[(t * 3 + d) * p], (int)p, a, x[d]);
      for (int64_t alpha = 0; alpha < k; ++alpha) {
        int64_t r = alpha;
        double v = 1.0;
        for (int d = 0; d < dim; ++d) { v *= L[d * p + r % p]; r /= p; }
        Ut[i + m * alpha] = v;
      }
    }
  }
  // ---- transfers E_c[alpha', alpha] = prod_d L^{parent}_{alpha_d}(xi^c_{alpha'_d}) ----
  double* E = F(13);
#pragma omp parallel for schedule(static)
  for (int64_t c = 1; c < nnodes; ++c) {
    const int64_t par = parent[c];
    double* Ec = E + (c - 1) * k * k;  // every level has k x k transfers, node order
    double xc[3];
    for (int64_t a1 = 0; a1 < k; ++a1) {
      tensor_point(c, a1, xc);
      for (int64_t a = 0; a < k; ++a) {
        int64_t r = a;
        double v = 1.0;
        for (int d = 0; d < dim; ++d) {
          v *= lagrange(&grid[(par * 3 + d) * p], (int)p, (int)(r % p), xc[d]);
          r /= p;
        }
        Ec[a1 + k * a] = v;
      }
    }
  }
  // ---- coupling S_ts[alpha, beta] = kappa(xi^t_alpha, xi^s_beta) ----
  {
    std::vector<std::pair<int64_t, int64_t>> all;
    all.reserve(nadm_tot);
    for (int l = 0; l <= q; ++l) all.insert(all.end(), adm[l].begin(), adm[l].end());
    double* S = F(16);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nadm_tot; ++b) {
      const int64_t t = all[b].first, s = all[b].second;
      double* Sb = S + b * k * k;
      std::vector<double> xs(k * 3), xt(k * 3);
      for (int64_t a = 0; a < k; ++a) { tensor_point(t, a, &xt[a * 3]); tensor_point(s, a, &xs[a * 3]); }
      for (int64_t be = 0; be < k; ++be)
        for (int64_t a = 0; a < k; ++a)
          Sb[a + k * be] = kernel_eval(kernel_id, kparam, &xt[a * 3], &xs[be * 3], (int)dim);
    }
  }
  // ---- dense blocks D_ts[i, j] = kappa(p_i, p_j), tree order ----
  {
    double* D = F(17);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < (int64_t)dense.size(); ++b) {
      const int64_t t = dense[b].first, s = dense[b].second;
      const int64_t mt = hi[t] - lo[t], ms = hi[s] - lo[s];
      double* Db = D + d_off[b];
      for (int64_t j = 0; j < ms; ++j) {
        const double* y = pts + idx[lo[s] + j] * dim;
        for (int64_t i = 0; i < mt; ++i)
          Db[i + mt * j] = kernel_eval(kernel_id, kparam, pts + idx[lo[t] + i] * dim, y, (int)dim);
      }
    }
  }
  if (store_points) std::memcpy(F(18), pts, 8 * n * dim);
  *out = buf;
  *out_len = total;
  return 0;
}

void h2gen_free(void* p) { std::free(p); }

}  // extern "C"
