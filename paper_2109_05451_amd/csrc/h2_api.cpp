// C ABI of libh2gemv: loading (validation, launch schedules built once --
// the role the paper gives to its per-level marshaling kernels, Algorithm 3,
// done here at load time because the structure is static), the product
// h2_gemv, and the helpers declared in include/h2.h.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "h2_internal.h"

namespace {
thread_local std::string g_err;
}

namespace h2 {

void set_error(const std::string& msg) { g_err = msg; }

namespace {

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? H2_ENOMEM : H2_EHIP;
}

#define HIP_TRY(expr, what)                       \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <class T>
int upload(const std::vector<T>& v, T** dst, int64_t* bytes) {
  *dst = nullptr;
  if (v.empty()) return H2_OK;
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(dst), v.size() * sizeof(T)), "hipMalloc(index)");
  HIP_TRY(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy(index)");
  *bytes += (int64_t)(v.size() * sizeof(T));
  return H2_OK;
}

// Streaming schedule (op 'N') over block rows: `rows_of` yields, for each
// output row, its blocks in memory order.
struct BlockRef {
  int64_t data;    // element offset of the stored block
  int64_t in_off;  // input row offset
  int32_t width;   // columns of the stored block
};

void add_stream_row(StreamSched& sc, int64_t out_off, int32_t nrows, int64_t out_ld, int64_t in_ld,
                    const std::vector<BlockRef>& blks) {
  RowDesc R{};
  R.data_off = blks.empty() ? 0 : blks[0].data;
  R.out_off = out_off;
  R.nrows = nrows;
  R.blk_begin = (int32_t)sc.colend.size();
  int32_t col = 0;
  for (const BlockRef& b : blks) {
    col += b.width;
    sc.colend.push_back(col);
    sc.in_off.push_back(b.in_off);
  }
  R.blk_end = (int32_t)sc.colend.size();
  R.out_ld = out_ld;
  R.in_ld = in_ld;
  sc.rows.push_back(R);
}

void add_gather_row(GatherSched& sc, int64_t out_off, int32_t nrows, int64_t out_ld, int64_t in_ld,
                    const std::vector<BlockRef>& blks, const std::vector<int32_t>& mr) {
  RowDesc R{};
  R.out_off = out_off;
  R.nrows = nrows;
  R.blk_begin = (int32_t)sc.data.size();
  for (size_t i = 0; i < blks.size(); ++i) {
    sc.data.push_back(blks[i].data);
    sc.in_off.push_back(blks[i].in_off);
    sc.mr.push_back(mr[i]);
  }
  R.blk_end = (int32_t)sc.data.size();
  R.out_ld = out_ld;
  R.in_ld = in_ld;
  sc.rows.push_back(R);
}

void free_device(h2_op_s* h) {
  auto F = [](void* p) { if (p) (void)hipFree(p); };
  F(h->d_mat); F(h->d_perm); F(h->d_lo); F(h->d_m); F(h->d_parent); F(h->d_cptr); F(h->d_hoff);
  F(h->coupleN.d_rows); F(h->coupleN.d_colend); F(h->coupleN.d_in_off);
  F(h->denseN.d_rows); F(h->denseN.d_colend); F(h->denseN.d_in_off);
  F(h->coupleT.d_rows); F(h->coupleT.d_data); F(h->coupleT.d_mr); F(h->coupleT.d_in_off);
  F(h->denseT.d_rows); F(h->denseT.d_data); F(h->denseT.d_mr); F(h->denseT.d_in_off);
  F(h->d_xt); F(h->d_xh); F(h->d_yh); F(h->d_zn);
  for (auto& set : h->ev_pool)
    for (hipEvent_t e : set)
      if (e) (void)hipEventDestroy(e);
  h->ev_pool.clear();
}

// Build schedules, upload; `h` has its device set current.
int build_handle(const uint8_t* buf, const Parsed& P, h2_op_s* h) {
  const int64_t q = P.q, n = P.n;
  h->n = n; h->q = q; h->nnodes = P.nnodes; h->nleaves = P.nleaves; h->leaf0 = P.leaf0;
  h->shared = !(P.flags & 1u);
  // ---- levels, node offsets into the vector trees
  h->lv.resize(q + 1);
  const int64_t mat0 = P.off_U;  // device matrix array keeps the section layout from U on
  for (int64_t l = 0; l <= q; ++l) {
    LevelInfo& L = h->lv[l];
    L.begin = P.level_ptr[l];
    L.count = P.level_ptr[l + 1] - P.level_ptr[l];
    L.krow = P.krow[l];
    L.kcol = P.kcol[l];
    L.kmax = std::max(L.krow, L.kcol);
    L.e_off = (P.off_E - mat0) / 8 + P.ebase[l];
    L.f_off = ((h->shared ? P.off_E : P.off_F) - mat0) / 8 + P.fbase[l];
  }
  h->u_off = 0;
  h->v_off = ((h->shared ? P.off_U : P.off_V) - mat0) / 8;
  h->s_off = (P.off_S - mat0) / 8;
  h->d_off = (P.off_D - mat0) / 8;
  std::vector<int64_t> hoff(P.nnodes);
  int64_t H = 0;
  for (int64_t l = 0; l <= q; ++l)
    for (int64_t c = P.level_ptr[l]; c < P.level_ptr[l + 1]; ++c) {
      hoff[c] = H;
      H += h->lv[l].kmax;
    }
  h->H = H;
  std::vector<int32_t> perm(n), lo(P.nnodes), msz(P.nnodes), parent(P.nnodes), cptr(P.nnodes + 1, 0);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)P.perm[i];
  for (int64_t c = 0; c < P.nnodes; ++c) {
    lo[c] = (int32_t)P.lo[c];
    msz[c] = (int32_t)(P.hi[c] - P.lo[c]);
    parent[c] = (int32_t)P.parent[c];
  }
  // children of p are consecutive: cptr[p] = first child, cptr[p+1] = one past the last
  {
    int64_t next_child = 1;
    for (int64_t p = 0; p < P.nnodes; ++p) {
      cptr[p] = (int32_t)next_child;
      while (next_child < P.nnodes && P.parent[next_child] == p) ++next_child;
    }
    cptr[P.nnodes] = (int32_t)next_child;
  }
  // ---- coupling schedules: op 'N' rows (CSR), op 'T' columns (CSC)
  int64_t csp = 0, csp_dense = 0;
  {
    std::vector<BlockRef> blks;
    std::vector<std::vector<int64_t>> by_col;  // per node of the level: global block ids
    for (int64_t l = 0; l <= q; ++l) {
      const LevelInfo& L = h->lv[l];
      const int64_t* rp = P.s_rowptr + P.rp_base[l];
      const int64_t bsz = L.krow * L.kcol;
      by_col.assign(L.count, {});
      for (int64_t t = 0; t < L.count; ++t) {
        blks.clear();
        for (int64_t b = rp[t]; b < rp[t + 1]; ++b) {
          const int64_t g = P.blk_base[l] + b, s = P.s_col[g];
          blks.push_back({h->s_off + P.sdat[l] + b * bsz, hoff[L.begin + s], (int32_t)L.kcol});
          by_col[s].push_back(b);
        }
        csp = std::max<int64_t>(csp, (int64_t)blks.size());
        add_stream_row(h->coupleN, hoff[L.begin + t], (int32_t)L.krow, H, H, blks);
      }
      // op 'T': output node s gets sum_t S_ts^T x^_t
      std::vector<int32_t> mr;
      for (int64_t s = 0; s < L.count; ++s) {
        blks.clear();
        mr.clear();
        // row node of block b: search the CSR (b is increasing with t)
        for (int64_t b : by_col[s]) {
          const int64_t t = std::upper_bound(rp, rp + L.count + 1, b) - rp - 1;
          blks.push_back({h->s_off + P.sdat[l] + b * bsz, hoff[L.begin + t], (int32_t)L.kcol});
          mr.push_back((int32_t)L.krow);
        }
        csp = std::max<int64_t>(csp, (int64_t)blks.size());
        add_gather_row(h->coupleT, hoff[L.begin + s], (int32_t)L.kcol, H, H, blks, mr);
      }
    }
  }
  // ---- dense schedules over leaves
  {
    std::vector<BlockRef> blks;
    std::vector<std::vector<int64_t>> by_col(P.nleaves);
    for (int64_t t = 0; t < P.nleaves; ++t) {
      blks.clear();
      for (int64_t b = P.d_rowptr[t]; b < P.d_rowptr[t + 1]; ++b) {
        const int64_t s = P.d_col[b];
        blks.push_back({h->d_off + P.ddat[b], P.lo[P.leaf0 + s], (int32_t)(P.hi[P.leaf0 + s] - P.lo[P.leaf0 + s])});
        by_col[s].push_back(b);
      }
      csp_dense = std::max<int64_t>(csp_dense, (int64_t)blks.size());
      add_stream_row(h->denseN, P.lo[P.leaf0 + t], msz[P.leaf0 + t], n, n, blks);
    }
    std::vector<int32_t> mr;
    for (int64_t s = 0; s < P.nleaves; ++s) {
      blks.clear();
      mr.clear();
      for (int64_t b : by_col[s]) {
        const int64_t t = std::upper_bound(P.d_rowptr, P.d_rowptr + P.nleaves + 1, b) - P.d_rowptr - 1;
        blks.push_back({h->d_off + P.ddat[b], P.lo[P.leaf0 + t], msz[P.leaf0 + s]});
        mr.push_back(msz[P.leaf0 + t]);
      }
      csp_dense = std::max<int64_t>(csp_dense, (int64_t)blks.size());
      add_gather_row(h->denseT, P.lo[P.leaf0 + s], msz[P.leaf0 + s], n, n, blks, mr);
    }
  }
  // ---- stats
  h2_stats_t& st = h->stats;
  st = h2_stats_t{};
  st.n = n; st.depth = q; st.nnodes = P.nnodes; st.nleaves = P.nleaves;
  st.ncoupling = P.nadm_tot; st.ndense = P.ndense; st.csp = csp; st.csp_dense = csp_dense;
  st.entries_U = n * P.krow[q];
  st.entries_V = n * P.kcol[q];
  st.entries_E = P.ebase[q + 1];
  st.entries_F = P.fbase[q + 1];
  st.entries_S = P.sdat[q + 1];
  st.entries_D = P.ddat[P.ndense];
  int64_t tree_rows = 0;
  for (int64_t l = 0; l <= q; ++l) tree_rows += h->lv[l].count * h->lv[l].kmax;
  st.tree_rows = tree_rows;
  st.shared_basis = h->shared ? 1 : 0;
  for (int64_t l = 0; l <= q; ++l) st.max_rank = std::max(st.max_rank, h->lv[l].kmax);
  for (int64_t t = P.leaf0; t < P.nnodes; ++t) st.max_leaf = std::max<int64_t>(st.max_leaf, msz[t]);
  // ---- upload
  const int64_t mat_bytes = P.off_end - P.off_U;
  if (mat_bytes > 0) {
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&h->d_mat), mat_bytes), "hipMalloc(matrix data)");
    HIP_TRY(hipMemcpy(h->d_mat, buf + P.off_U, mat_bytes, hipMemcpyHostToDevice), "hipMemcpy(matrix data)");
  }
  int64_t ib = 0;
  int rc;
  std::vector<int64_t> hoff64(hoff);
  if ((rc = upload(perm, &h->d_perm, &ib)) || (rc = upload(lo, &h->d_lo, &ib)) || (rc = upload(msz, &h->d_m, &ib)) ||
      (rc = upload(parent, &h->d_parent, &ib)) || (rc = upload(cptr, &h->d_cptr, &ib)) ||
      (rc = upload(hoff64, &h->d_hoff, &ib)) ||
      (rc = upload(h->coupleN.rows, &h->coupleN.d_rows, &ib)) ||
      (rc = upload(h->coupleN.colend, &h->coupleN.d_colend, &ib)) ||
      (rc = upload(h->coupleN.in_off, &h->coupleN.d_in_off, &ib)) ||
      (rc = upload(h->denseN.rows, &h->denseN.d_rows, &ib)) ||
      (rc = upload(h->denseN.colend, &h->denseN.d_colend, &ib)) ||
      (rc = upload(h->denseN.in_off, &h->denseN.d_in_off, &ib)) ||
      (rc = upload(h->coupleT.rows, &h->coupleT.d_rows, &ib)) ||
      (rc = upload(h->coupleT.data, &h->coupleT.d_data, &ib)) ||
      (rc = upload(h->coupleT.mr, &h->coupleT.d_mr, &ib)) ||
      (rc = upload(h->coupleT.in_off, &h->coupleT.d_in_off, &ib)) ||
      (rc = upload(h->denseT.rows, &h->denseT.d_rows, &ib)) ||
      (rc = upload(h->denseT.data, &h->denseT.d_data, &ib)) ||
      (rc = upload(h->denseT.mr, &h->denseT.d_mr, &ib)) ||
      (rc = upload(h->denseT.in_off, &h->denseT.d_in_off, &ib)))
    return rc;
  h->index_bytes = ib;
  h->stats.device_bytes = mat_bytes + ib;
  return H2_OK;
}

int ensure_workspace(h2_op_s* h, int64_t nv) {
  const int64_t want = std::min<int64_t>(std::max<int64_t>(nv, 1), kNvChunk);
  if (want <= h->cap) return H2_OK;
  double *xt = nullptr, *xh = nullptr, *yh = nullptr, *zn = nullptr;
  auto cleanup = [&]() {
    if (xt) (void)hipFree(xt);
    if (xh) (void)hipFree(xh);
    if (yh) (void)hipFree(yh);
    if (zn) (void)hipFree(zn);
  };
  hipError_t e;
  if ((e = hipMalloc(reinterpret_cast<void**>(&xt), sizeof(double) * h->n * want)) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&xh), sizeof(double) * std::max<int64_t>(h->H, 1) * want)) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&yh), sizeof(double) * std::max<int64_t>(h->H, 1) * want)) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&zn), sizeof(double) * h->n * want)) != hipSuccess) {
    cleanup();
    return hip_fail(e, "hipMalloc(workspace)");
  }
  // the old workspace may still be in use by queued work
  if (h->cap > 0) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize(workspace growth)");
    (void)hipFree(h->d_xt); (void)hipFree(h->d_xh); (void)hipFree(h->d_yh); (void)hipFree(h->d_zn);
  }
  h->d_xt = xt; h->d_xh = xh; h->d_yh = yh; h->d_zn = zn;
  h->stats.device_bytes += (int64_t)sizeof(double) * (2 * h->n + 2 * std::max<int64_t>(h->H, 1)) * (want - h->cap);
  h->cap = want;
  return H2_OK;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int load_common(const uint8_t* buf, int64_t len, int device, h2_handle* out) {
  if (!out) { set_error("null output handle"); return H2_EINVAL; }
  *out = nullptr;
  Parsed P;
  int rc = parse(buf, len, &P);
  if (rc != H2_OK) return rc;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) { set_error("device ordinal out of range"); return H2_EINVAL; }
  DeviceGuard guard(device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  h2_op_s* h = new (std::nothrow) h2_op_s();
  if (!h) { set_error("out of host memory"); return H2_ENOMEM; }
  h->device = device;
  rc = build_handle(buf, P, h);
  if (rc != H2_OK) {
    free_device(h);
    delete h;
    return rc;
  }
  *out = h;
  return H2_OK;
}

// One pass of the product over nv <= cap vectors (X, Y already offset).
int gemv_pass(h2_op_s* h, bool trans, double alpha, const double* X, int64_t ldx, int nv, double beta, double* Y,
              int64_t ldy, hipStream_t s) {
  const int64_t q = h->q, n = h->n, H = h->H;
  std::array<hipEvent_t, 7>* ev = nullptr;
  if (h->profiling) {
    if (h->ev_used == h->ev_pool.size()) {
      std::array<hipEvent_t, 7> set{};
      for (auto& e : set) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
      h->ev_pool.push_back(set);
    }
    ev = &h->ev_pool[h->ev_used++];
  }
  auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord((*ev)[i], s) : hipSuccess; };
  const double* mat = h->d_mat;
  // the operator's column basis (input side) and row basis (output side)
  const double* Bcol = mat + (trans ? h->u_off : h->v_off);
  const double* Brow = mat + (trans ? h->v_off : h->u_off);
  auto Tcol = [&](int64_t l) { return mat + (trans ? h->lv[l].e_off : h->lv[l].f_off); };
  auto Trow = [&](int64_t l) { return mat + (trans ? h->lv[l].f_off : h->lv[l].e_off); };
  auto kcol = [&](int64_t l) { return (int)(trans ? h->lv[l].krow : h->lv[l].kcol); };
  auto krow = [&](int64_t l) { return (int)(trans ? h->lv[l].kcol : h->lv[l].krow); };

  HIP_TRY(mark(0), "hipEventRecord");
  HIP_TRY(launch_permute_in(X, ldx, h->d_perm, h->d_xt, n, nv, s), "permute");
  HIP_TRY(mark(1), "hipEventRecord");
  HIP_TRY(launch_leaf_up(Bcol, kcol(q), h->leaf0, h->nleaves, h->d_lo, h->d_m, h->d_hoff, h->d_xt, n, h->d_xh, H,
                         nv, s), "leaf upsweep");
  for (int64_t l = q; l >= 1; --l)
    HIP_TRY(launch_transfer_up(Tcol(l), kcol(l), kcol(l - 1), h->lv[l - 1].begin, h->lv[l - 1].count,
                               h->lv[l].begin, h->d_cptr, h->d_hoff, h->d_xh, H, nv, s), "transfer upsweep");
  HIP_TRY(mark(2), "hipEventRecord");
  if (!trans)
    HIP_TRY(launch_stream_rows(h->coupleN, mat, h->d_xh, h->d_yh, nv, s), "coupling");
  else
    HIP_TRY(launch_gather_rows(h->coupleT, mat, h->d_xh, h->d_yh, nv, s), "coupling");
  HIP_TRY(mark(3), "hipEventRecord");
  for (int64_t l = 1; l <= q; ++l)
    HIP_TRY(launch_transfer_down(Trow(l), krow(l), krow(l - 1), h->lv[l].begin, h->lv[l].count, h->d_parent,
                                 h->d_hoff, h->d_yh, H, nv, s), "transfer downsweep");
  HIP_TRY(mark(4), "hipEventRecord");
  if (!trans)
    HIP_TRY(launch_stream_rows(h->denseN, mat, h->d_xt, h->d_zn, nv, s), "dense");
  else
    HIP_TRY(launch_gather_rows(h->denseT, mat, h->d_xt, h->d_zn, nv, s), "dense");
  HIP_TRY(mark(5), "hipEventRecord");
  HIP_TRY(launch_leaf_down(Brow, krow(q), h->leaf0, h->nleaves, h->d_lo, h->d_m, h->d_hoff, h->d_yh, H, h->d_zn, n,
                           h->d_perm, alpha, beta, Y, ldy, nv, s), "leaf expansion");
  HIP_TRY(mark(6), "hipEventRecord");
  return H2_OK;
}

}  // namespace
}  // namespace h2

using namespace h2;

extern "C" {

const char* h2_last_error(void) { return g_err.c_str(); }

int h2_validate(const void* buf, size_t len) {
  Parsed P;
  return parse(static_cast<const uint8_t*>(buf), (int64_t)len, &P);
}

int h2_load_mem(const void* buf, size_t len, int device, h2_handle* out) {
  if (!buf) { set_error("null buffer"); return H2_EINVAL; }
  return load_common(static_cast<const uint8_t*>(buf), (int64_t)len, device, out);
}

int h2_load(const char* path, int device, h2_handle* out) {
  if (!path || !out) { set_error("null path or handle"); return H2_EINVAL; }
  FILE* f = std::fopen(path, "rb");
  if (!f) { set_error(std::string("cannot open ") + path); return H2_EIO; }
  std::fseek(f, 0, SEEK_END);
  const long long len = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  if (len < 0) { std::fclose(f); set_error("cannot size file"); return H2_EIO; }
  // 64-byte aligned host copy
  std::vector<uint64_t> storage(((size_t)len + 7) / 8);
  const size_t got = std::fread(storage.data(), 1, (size_t)len, f);
  std::fclose(f);
  if (got != (size_t)len) { set_error("short read"); return H2_EIO; }
  return load_common(reinterpret_cast<const uint8_t*>(storage.data()), len, device, out);
}

int h2_reserve(h2_handle h, int64_t nv_max) {
  if (!h || nv_max < 0) { set_error("bad handle or nv_max"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  return ensure_workspace(h, nv_max);
}

int h2_gemv(h2_handle h, char op, double alpha, const double* X, int64_t ldx, int64_t nv, double beta, double* Y,
            int64_t ldy, void* stream) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  const bool trans = op == 'T' || op == 't';
  if (!trans && op != 'N' && op != 'n') { set_error("op must be 'N' or 'T'"); return H2_EINVAL; }
  if (nv < 0) { set_error("nv < 0"); return H2_EINVAL; }
  if (nv == 0) return H2_OK;
  if (!Y || ldy < h->n) { set_error("bad Y or ldy"); return H2_EINVAL; }
  if (alpha != 0.0) {
    if (!X || ldx < h->n) { set_error("bad X or ldx"); return H2_EINVAL; }
    const char* xb = reinterpret_cast<const char*>(X);
    const char* xe = reinterpret_cast<const char*>(X + ldx * (nv - 1) + h->n);
    const char* yb = reinterpret_cast<const char*>(Y);
    const char* ye = reinterpret_cast<const char*>(Y + ldy * (nv - 1) + h->n);
    if (xb < ye && yb < xe) { set_error("X and Y overlap"); return H2_EINVAL; }
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (alpha == 0.0) {
    HIP_TRY(launch_scale(Y, ldy, h->n, nv, beta, s), "scale");
    return H2_OK;
  }
  int rc = ensure_workspace(h, nv);
  if (rc != H2_OK) return rc;
  for (int64_t v0 = 0; v0 < nv; v0 += h->cap) {
    const int nvc = (int)std::min<int64_t>(h->cap, nv - v0);
    rc = gemv_pass(h, trans, alpha, X + ldx * v0, ldx, nvc, beta, Y + ldy * v0, ldy, s);
    if (rc != H2_OK) return rc;
  }
  if (h->profiling) ++h->prof.calls;
  return H2_OK;
}

int h2_stats(h2_handle h, h2_stats_t* st) {
  if (!h || !st) { set_error("null handle or output"); return H2_EINVAL; }
  *st = h->stats;
  return H2_OK;
}

int64_t h2_n(h2_handle h) { return h ? h->n : -1; }

int h2_profile(h2_handle h, int enable) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize(profile)");
  h->profiling = enable != 0;
  h->ev_used = 0;
  h->prof = h2_profile_t{};
  return H2_OK;
}

int h2_profile_read(h2_handle h, h2_profile_t* out) {
  if (!h || !out) { set_error("null handle or output"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  for (size_t i = 0; i < h->ev_used; ++i) {
    auto& e = h->ev_pool[i];
    HIP_TRY(hipEventSynchronize(e[6]), "hipEventSynchronize");
    float t[6];
    for (int k = 0; k < 6; ++k) HIP_TRY(hipEventElapsedTime(&t[k], e[k], e[k + 1]), "hipEventElapsedTime");
    float tot;
    HIP_TRY(hipEventElapsedTime(&tot, e[0], e[6]), "hipEventElapsedTime");
    h->prof.ms_permute += t[0];
    h->prof.ms_upsweep += t[1];
    h->prof.ms_coupling += t[2];
    h->prof.ms_downsweep += t[3];
    h->prof.ms_dense += t[4];
    h->prof.ms_leaf_out += t[5];
    h->prof.ms_total += tot;
  }
  h->ev_used = 0;
  *out = h->prof;
  return H2_OK;
}

int h2_free(h2_handle h) {
  if (!h) return H2_OK;
  {
    DeviceGuard guard(h->device);
    (void)hipDeviceSynchronize();
    free_device(h);
  }
  delete h;
  return H2_OK;
}

}  // extern "C"
