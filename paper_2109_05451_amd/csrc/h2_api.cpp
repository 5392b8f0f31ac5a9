// C ABI of libh2gemv: loading (validation; launch plans built once -- the
// role the paper gives to its per-level marshaling kernels, Algorithm 3,
// done here at load time because the structure is static), the product
// h2_gemv, and the helpers declared in include/h2.h.
#include <algorithm>
#include <cmath>
#include <array>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
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

#define HIP_TRY(expr, what)                          \
  do {                                               \
    hipError_t e_ = (expr);                          \
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

void append_gather(GatherTables& t, const RowSpec& r) {
  RowDesc R{};
  R.out_off = r.out_off;
  R.nrows = r.nrows;
  R.blk_begin = (int32_t)t.data.size();
  for (const BlockRef& b : r.blks) {
    t.data.push_back(b.data);
    t.in_off.push_back(b.in_off);
    t.mr.push_back(b.mr);
  }
  R.blk_end = (int32_t)t.data.size();
  R.out_ld = r.out_ld;
  R.in_ld = r.in_ld;
  t.rows.push_back(R);
}

// Row indices, most work (columns x outputs) first; ties keep their order.
std::vector<size_t> order_by_work(const std::vector<RowSpec>& rows) {
  std::vector<int64_t> w(rows.size());
  for (size_t i = 0; i < rows.size(); ++i) w[i] = row_work(rows[i]);
  std::vector<size_t> o(rows.size());
  std::iota(o.begin(), o.end(), 0);
  std::stable_sort(o.begin(), o.end(), [&](size_t a, size_t b) { return w[a] > w[b]; });
  return o;
}

// Row indices in output position order (tree order).
std::vector<size_t> order_by_position(const std::vector<RowSpec>& rows) {
  std::vector<size_t> o(rows.size());
  std::iota(o.begin(), o.end(), 0);
  std::stable_sort(o.begin(), o.end(), [&](size_t a, size_t b) { return rows[a].out_off < rows[b].out_off; });
  return o;
}

// Append a phase of streaming rows taken in the given order (narrow rows to
// the tabled kernel, wide ones to the fallback).
void add_stream_rows(h2_op_s* h, const std::vector<RowSpec>& rows, const size_t* order, size_t count, int arr,
                     int in, int out, int mode, std::vector<Launch>& dst) {
  Launch narrow, wide;
  narrow.kind = KIND_STREAM; wide.kind = KIND_WIDE;
  narrow.arr = wide.arr = arr;
  narrow.in = wide.in = in;
  narrow.out = wide.out = out;
  narrow.mode = wide.mode = mode;
  narrow.row_begin = (int64_t)h->rt.rows.size();
  wide.row_begin = (int64_t)h->wide.rows.size();
  for (size_t i = 0; i < count; ++i) {
    const RowSpec& r = rows[order ? order[i] : i];
    if ((int64_t)r.blks.size() <= kNbMax) {
      append_row(h->rt, r);
      narrow.max_rows = std::max(narrow.max_rows, r.nrows);
    } else {
      append_row(h->wide, r);
      wide.max_rows = std::max(wide.max_rows, r.nrows);
    }
  }
  narrow.row_count = (int64_t)h->rt.rows.size() - narrow.row_begin;
  wide.row_count = (int64_t)h->wide.rows.size() - wide.row_begin;
  if (narrow.row_count) dst.push_back(narrow);
  if (wide.row_count) dst.push_back(wide);
}

// A phase of streaming rows in emission order, or longest rows first for
// load balance.
void add_stream_phase(h2_op_s* h, const std::vector<RowSpec>& rows, int arr, int in, int out, int mode, bool sort,
                      std::vector<Launch>& dst) {
  if (!sort) {
    add_stream_rows(h, rows, nullptr, rows.size(), arr, in, out, mode, dst);
    return;
  }
  const std::vector<size_t> o = order_by_work(rows);
  add_stream_rows(h, rows, o.data(), o.size(), arr, in, out, mode, dst);
}

// Rows first, first + step, ... of `rows` as one launch of the transposed kernel.
void add_gather_phase(h2_op_s* h, const std::vector<RowSpec>& rows, int in, int out, std::vector<Launch>& dst,
                      size_t first = 0, size_t step = 1) {
  Launch L;
  L.kind = KIND_GATHER;
  L.arr = ARR_MAT;
  L.in = in;
  L.out = out;
  L.mode = MODE_STORE;
  L.row_begin = (int64_t)h->gt.rows.size();
  for (size_t i = first; i < rows.size(); i += step) append_gather(h->gt, rows[i]);
  L.row_count = (int64_t)h->gt.rows.size() - L.row_begin;
  if (L.row_count) dst.push_back(L);
}

// Destroy the captured graphs of h2_gemv (their launch parameters are stale
// after retuning); the device must be idle or the graphs finished.
void drop_graphs(h2_op_s* h) {
  for (GraphEntry& g : h->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

void free_device(h2_op_s* h) {
  drop_graphs(h);
  auto F = [](void* p) { if (p) (void)hipFree(p); };
  F(h->d_mat); F(h->d_trans); F(h->d_perm); F(h->d_pinv); F(h->d_mat32); F(h->d_trans32);
  F(h->d_mat16); F(h->d_trans16); F(h->d_fl); F(h->d_fl32);
  F(h->rt.d_rows); F(h->rt.d_colend); F(h->rt.d_in_off);
  F(h->wide.d_rows); F(h->wide.d_colend); F(h->wide.d_in_off);
  F(h->gt.d_rows); F(h->gt.d_data); F(h->gt.d_mr); F(h->gt.d_in_off); F(h->d_tree_ranges);
  for (auto& set : h->ev_pool)
    for (hipEvent_t e : set)
      if (e) (void)hipEventDestroy(e);
  h->ev_pool.clear();
  ws_destroy(&h->ws);
  ws_destroy(&h->na);
}

// Fused sweeps of the op-'N' multi-vector path.  Level boundaries
// 0 = b_0 < ... < b_k = q, the last interval four levels deep (its subtree
// roots are the nodes of level q - 4: 1024 of them for 2^14 leaves) and the
// others five.  Upsweep group i (i = k .. 1, run in that order) has a
// workgroup per node of level b_(i-1) and runs, bottom-up, the leaf products
// (last interval only) and the transfer rows of the parents on levels
// b_i - 1 .. b_(i-1); downsweep group i (i = 1 .. k) runs, top-down, the rows
// of the children on levels b_(i-1) + 1 .. b_i and, in the last interval,
// the leaf expansion.  A workgroup's rows on a level are the node range its
// subtree covers there.  Leaves true when every launch of the plan is one
// narrow row list in node order and every row has at most 64 outputs.
bool build_tree_groups(h2_op_s* h, const Parsed& P, const OpLayout& lay, std::vector<int2>* ranges) {
  const int64_t q = P.q;
  const int64_t* lp = P.level_ptr;
  const Plan& plan = h->planN;
  if ((int64_t)plan.up.size() != q + 1 || (int64_t)plan.down.size() != q) return false;
  auto narrow_of = [](const Launch& L, int64_t rows) { return L.kind == KIND_STREAM && L.row_count == rows; };
  if (!narrow_of(plan.up[0], P.nleaves) || !narrow_of(plan.out, P.nleaves)) return false;
  for (int64_t l = 1; l <= q; ++l)
    if (!narrow_of(plan.up[q - l + 1], lp[l] - lp[l - 1]) || !narrow_of(plan.down[l - 1], lp[l + 1] - lp[l]))
      return false;
  std::vector<int64_t> bnd;  // increasing boundaries
  {
    int64_t b = q;
    bnd.push_back(b);
    if (q > 0) {
      b = std::max<int64_t>(0, q - 4);
      bnd.push_back(b);
      while (b > 0) {
        b = std::max<int64_t>(0, b - 5);
        bnd.push_back(b);
      }
    } else {
      bnd.push_back(0);
    }
    std::reverse(bnd.begin(), bnd.end());
  }
  const int64_t k = (int64_t)bnd.size() - 1;
  // descendants of node r on level l (l >= level of r): one node range
  auto desc = [&](int64_t r, int64_t lr, int64_t l) {
    int64_t lo = r, hi = r + 1;
    for (int64_t x = lr; x < l; ++x) {
      lo = lay.cbeg[lo];
      hi = lay.cbeg[hi];
    }
    return std::make_pair(lo, hi);
  };
  // one level entry of a group: the rows of launch L for the nodes [lo, hi)
  // of a level whose first node is `first`
  struct Entry { const Launch* L; int64_t level; int64_t first; int in, out, mode; };
  auto add_group = [&](std::vector<TreeGroup>& dst, int64_t root_level, const std::vector<Entry>& ent, bool up) {
    TreeGroup G;
    G.lv.nlev = (int)ent.size();
    G.nwg = lp[root_level + 1] - lp[root_level];
    G.range_off = (int64_t)ranges->size();
    G.trans_data = up;
    for (size_t j = 0; j < ent.size(); ++j) {
      G.lv.in[j] = ent[j].in;
      G.lv.out[j] = ent[j].out;
      G.lv.mode[j] = ent[j].mode;
      G.max_rows = std::max(G.max_rows, ent[j].L->max_rows);
    }
    for (int64_t r = lp[root_level]; r < lp[root_level + 1]; ++r)
      for (const Entry& e : ent) {
        const auto d = desc(r, root_level, e.level);
        const int64_t b = e.L->row_begin + (d.first - e.first), c = e.L->row_begin + (d.second - e.first);
        ranges->push_back(int2{(int)b, (int)c});
      }
    dst.push_back(G);
  };
  if ((int64_t)h->rt.rows.size() >= (int64_t)1 << 31) return false;
  for (int64_t i = k; i >= 1; --i) {
    std::vector<Entry> ent;
    if (i == k) ent.push_back({&plan.up[0], q, lp[q], BUF_XT, BUF_XH, MODE_STORE});
    for (int64_t l = bnd[i]; l > bnd[i - 1]; --l)  // parents on level l - 1
      ent.push_back({&plan.up[q - l + 1], l - 1, lp[l - 1], BUF_XH, BUF_XH, MODE_STORE});
    if (ent.empty()) continue;
    if ((int)ent.size() > kMaxTreeLevels) return false;
    add_group(h->tree_up, bnd[i - 1], ent, true);
  }
  for (int64_t i = 1; i <= k; ++i) {
    std::vector<Entry> ent;
    for (int64_t l = bnd[i - 1] + 1; l <= bnd[i]; ++l)
      ent.push_back({&plan.down[l - 1], l, lp[l], BUF_YH, BUF_YH, MODE_ACCUM});
    if (i == k) ent.push_back({&plan.out, q, lp[q], BUF_YH, 3, MODE_STORE});
    if (ent.empty()) continue;
    if ((int)ent.size() > kMaxTreeLevels) return false;
    add_group(h->tree_down, bnd[i - 1], ent, false);
  }
  for (const auto* v : {&h->tree_up, &h->tree_down})
    for (const TreeGroup& G : *v)
      if (G.max_rows > 64) return false;
  return true;
}

// Build plans and upload; the handle's device is current.
int build_handle(const uint8_t* buf, const Parsed& P, h2_op_s* h, const double* d_dense) {
  const int64_t q = P.q, n = P.n;
  const int64_t* lp = P.level_ptr;
  h->n = n; h->q = q; h->nnodes = P.nnodes; h->nleaves = P.nleaves; h->leaf0 = P.leaf0;
  h->lmin = first_coupling_level(P);
  h->shared = !(P.flags & 1u);
  h->lv.resize(q + 1);
  for (int64_t l = 0; l <= q; ++l) {
    LevelInfo& L = h->lv[l];
    L.begin = lp[l];
    L.count = lp[l + 1] - lp[l];
    L.krow = P.krow[l];
    L.kcol = P.kcol[l];
    L.kmax = std::max(L.krow, L.kcol);
  }
  OpLayout lay;
  int rc0 = make_layout(P, &lay);
  if (rc0 != H2_OK) return rc0;
  const int64_t oU = lay.oU, oE = lay.oE, oV = lay.oV, oF = lay.oF, oS = lay.oS, oD = lay.oD;
  const int64_t tUT = lay.tUT, tET = lay.tET;
  const int64_t nU = n * P.krow[q], nE = P.ebase[q + 1], nV = n * P.kcol[q], nF = P.fbase[q + 1];
  const int64_t ntrans = lay.ntrans;
  h->n_trans = ntrans;
  h->n_lowrank = oD;
  const std::vector<int64_t>& hoff = lay.hoff;
  const int64_t H = lay.H;
  h->H = H;
  auto msz = [&](int64_t c) { return (int32_t)(P.hi[c] - P.lo[c]); };

  // ---- plan for op 'N': rows from the shared emitter (column-major layout)
  {
    RowsN R;
    RowBases B;
    B.ld_x = n;
    B.ld_h = H;
    emit_rows_N(lay, B, &R);
    {
      // room for every row the plans append: the sweeps of both ops, three
      // orders of the coupling rows, two of the dense rows
      size_t nr = 0, nb = 0;
      auto count = [&](const std::vector<RowSpec>& v, size_t copies) {
        for (const RowSpec& r : v) {
          nr += copies;
          nb += copies * r.blks.size();
        }
      };
      for (const auto& v : R.up) count(v, 2);
      for (const auto& v : R.down) count(v, 2);
      count(R.out, 2);
      count(R.couple, 3);
      count(R.dense, 2);
      h->rt.rows.reserve(nr);
      h->rt.colend.reserve(nb);
      h->rt.in_off.reserve(nb);
    }
    Plan& plan = h->planN;
    add_stream_phase(h, R.up[0], ARR_TRANS, BUF_XT, BUF_XH, MODE_STORE, false, plan.up);
    for (int64_t hh = 1; hh <= q; ++hh) {
      add_stream_phase(h, R.up[hh], ARR_TRANS, BUF_XH, BUF_XH, MODE_STORE, false, plan.up);
      plan.up.back().level = q - hh;
    }
    add_stream_phase(h, R.couple, ARR_MAT, BUF_XH, BUF_YH, MODE_STORE, true, plan.couple);
    {
      // the leaf level's coupling rows are the last ones emitted
      const size_t nq = (size_t)(lp[q + 1] - lp[q]);
      const std::vector<RowSpec> rest(R.couple.begin(), R.couple.end() - (long)nq),
          deep(R.couple.end() - (long)nq, R.couple.end());
      add_stream_phase(h, deep, ARR_MAT, BUF_XH, BUF_YH, MODE_STORE, true, plan.couple_deep);
      add_stream_phase(h, rest, ARR_MAT, BUF_XH, BUF_YH, MODE_STORE, true, plan.couple_rest);
    }
    {
      // the same rows in tree order; the dense rows in two halves of the domain
      const std::vector<size_t> oc = order_by_position(R.couple);
      add_stream_rows(h, R.couple, oc.data(), oc.size(), ARR_MAT, BUF_XH, BUF_YH, MODE_STORE, plan.couple_loc);
      const std::vector<size_t> od = order_by_position(R.dense);
      const size_t half = od.size() / 2;
      add_stream_rows(h, R.dense, od.data(), half, ARR_MAT, BUF_XT, BUF_ZN, MODE_STORE, plan.dense_loc);
      add_stream_rows(h, R.dense, od.data() + half, od.size() - half, ARR_MAT, BUF_XT, BUF_ZN, MODE_STORE,
                      plan.dense2_loc);
      for (auto* v : {&plan.dense_loc, &plan.dense2_loc})
        for (Launch& L : *v) L.lowrank = false;
    }
    for (int64_t l = 1; l <= q; ++l) {
      add_stream_phase(h, R.down[l - 1], ARR_MAT, BUF_YH, BUF_YH, MODE_ACCUM, false, plan.down);
      plan.down.back().level = l - 1;
    }
    {
      // two halves with the same mix of long and short rows (longest first in each)
      const std::vector<size_t> o = order_by_work(R.dense);
      std::vector<size_t> o1, o2;
      for (size_t i = 0; i < o.size(); ++i) (i % 2 ? o2 : o1).push_back(o[i]);
      add_stream_rows(h, R.dense, o1.data(), o1.size(), ARR_MAT, BUF_XT, BUF_ZN, MODE_STORE, plan.dense);
      add_stream_rows(h, R.dense, o2.data(), o2.size(), ARR_MAT, BUF_XT, BUF_ZN, MODE_STORE, plan.dense2);
      for (Launch& L : plan.dense) L.lowrank = false;
      for (Launch& L : plan.dense2) L.lowrank = false;
    }
    std::vector<Launch> outl;
    add_stream_phase(h, R.out, ARR_MAT, BUF_YH, BUF_ZN, MODE_FINAL, false, outl);
    if (outl.size() != 1) {
      set_error("internal: leaf expansion schedule");
      return H2_EUNSUPPORTED;
    }
    plan.out = outl[0];
  }
  std::vector<int2> tree_ranges;
  h->tree_ok = build_tree_groups(h, P, lay, &tree_ranges);
  if (!h->tree_ok) {
    h->tree_up.clear();
    h->tree_down.clear();
    tree_ranges.clear();
  }
  // ---- plan for op 'T' (A^T = D^T + V S^T U^T): upsweep with U, E; coupling
  // and dense blocks read transposed; downsweep with V, F
  {
    const int64_t* lp = P.level_ptr;
    Plan& plan = h->planT;
    const int64_t* kc = P.krow;  // ranks of the input side
    const int64_t* kr = P.kcol;  // ranks of the output side
    std::vector<RowSpec> rows;
    for (int64_t t = P.leaf0; t < P.nnodes; ++t)
      rows.push_back({tUT + P.lo[t] * kc[q], hoff[t], H, n, (int32_t)kc[q], {BlockRef{0, P.lo[t], msz(t), 0}}});
    add_stream_phase(h, rows, ARR_TRANS, BUF_XT, BUF_XH, MODE_STORE, false, plan.up);
    for (int64_t l = q; l >= 1; --l) {
      rows.clear();
      for (int64_t p = lp[l - 1]; p < lp[l]; ++p) {
        RowSpec r{tET + lay.eoff(lay.cbeg[p], l), hoff[p], H, H, (int32_t)kc[l - 1], {}};
        for (int64_t c = lay.cbeg[p]; c < lay.cbeg[p + 1]; ++c) r.blks.push_back({0, hoff[c], (int32_t)kc[l], 0});
        rows.push_back(std::move(r));
      }
      add_stream_phase(h, rows, ARR_TRANS, BUF_XH, BUF_XH, MODE_STORE, false, plan.up);
      plan.up.back().level = l - 1;
    }
    rows.clear();
    for (int64_t l = 0; l <= q; ++l) {
      const int64_t* rp = P.s_rowptr + P.rp_base[l];
      const int64_t nl = lp[l + 1] - lp[l], bsz = P.krow[l] * P.kcol[l];
      std::vector<std::vector<BlockRef>> by_col(nl);
      for (int64_t t = 0; t < nl; ++t)
        for (int64_t b = rp[t]; b < rp[t + 1]; ++b)
          by_col[P.s_col[P.blk_base[l] + b]].push_back({oS + P.sdat[l] + b * bsz, hoff[lp[l] + t], 0, (int32_t)P.krow[l]});
      for (int64_t s = 0; s < nl; ++s)
        rows.push_back({0, hoff[lp[l] + s], H, H, (int32_t)P.kcol[l], std::move(by_col[s])});
    }
    add_gather_phase(h, rows, BUF_XH, BUF_YH, plan.couple);
    for (int64_t l = 1; l <= q; ++l) {
      rows.clear();
      for (int64_t c = lp[l]; c < lp[l + 1]; ++c)
        rows.push_back({oF + lay.foff(c, l), hoff[c], H, H, (int32_t)kr[l],
                        {BlockRef{0, hoff[P.parent[c]], (int32_t)kr[l - 1], 0}}});
      add_stream_phase(h, rows, ARR_MAT, BUF_YH, BUF_YH, MODE_ACCUM, false, plan.down);
      plan.down.back().level = l - 1;
    }
    rows.clear();
    std::vector<std::vector<BlockRef>> by_col(P.nleaves);
    for (int64_t t = 0; t < P.nleaves; ++t)
      for (int64_t b = P.d_rowptr[t]; b < P.d_rowptr[t + 1]; ++b)
        by_col[P.d_col[b]].push_back({oD + P.ddat[b], P.lo[P.leaf0 + t], 0, msz(P.leaf0 + t)});
    for (int64_t s = 0; s < P.nleaves; ++s)
      rows.push_back({0, P.lo[P.leaf0 + s], n, n, msz(P.leaf0 + s), std::move(by_col[s])});
    add_gather_phase(h, rows, BUF_XT, BUF_ZN, plan.dense, 0, 2);
    add_gather_phase(h, rows, BUF_XT, BUF_ZN, plan.dense2, 1, 2);
    for (Launch& L : plan.dense) L.lowrank = false;
    for (Launch& L : plan.dense2) L.lowrank = false;
    rows.clear();
    for (int64_t t = P.leaf0; t < P.nnodes; ++t)
      rows.push_back({oV + P.lo[t] * kr[q], P.lo[t], n, H, msz(t), {BlockRef{0, hoff[t], (int32_t)kr[q], 0}}});
    std::vector<Launch> outl;
    add_stream_phase(h, rows, ARR_MAT, BUF_YH, BUF_ZN, MODE_FINAL, false, outl);
    if (outl.size() != 1) {
      set_error("internal: leaf expansion schedule");
      return H2_EUNSUPPORTED;
    }
    plan.out = outl[0];
  }
  (void)oU; (void)oE;

  // ---- stats
  int64_t csp = 0, csp_dense = 0;
  h->level_stats.assign(q + 1, h2_level_stats_t{});
  for (int64_t l = 0; l <= q; ++l) {
    const int64_t* rp = P.s_rowptr + P.rp_base[l];
    const int64_t nl = lp[l + 1] - lp[l];
    int64_t lcsp = 0;
    std::vector<int64_t> colcnt(nl, 0);
    for (int64_t t = 0; t < nl; ++t) {
      lcsp = std::max(lcsp, rp[t + 1] - rp[t]);
      for (int64_t b = rp[t]; b < rp[t + 1]; ++b) ++colcnt[P.s_col[P.blk_base[l] + b]];
    }
    for (int64_t c : colcnt) lcsp = std::max(lcsp, c);
    csp = std::max(csp, lcsp);
    h2_level_stats_t& ls = h->level_stats[l];
    ls.nodes = nl;
    ls.krow = P.krow[l];
    ls.kcol = P.kcol[l];
    ls.coupling_blocks = P.blk_base[l + 1] - P.blk_base[l];
    ls.csp = lcsp;
    ls.entries_S = P.sdat[l + 1] - P.sdat[l];
    ls.entries_E = l > 0 ? nl * P.krow[l] * P.krow[l - 1] : 0;
    ls.entries_F = l > 0 ? nl * P.kcol[l] * P.kcol[l - 1] : 0;
  }
  {
    std::vector<int64_t> colcnt(P.nleaves, 0);
    for (int64_t t = 0; t < P.nleaves; ++t) {
      csp_dense = std::max(csp_dense, P.d_rowptr[t + 1] - P.d_rowptr[t]);
      for (int64_t b = P.d_rowptr[t]; b < P.d_rowptr[t + 1]; ++b) ++colcnt[P.d_col[b]];
    }
    for (int64_t c : colcnt) csp_dense = std::max(csp_dense, c);
  }
  h2_stats_t& st = h->stats;
  st = h2_stats_t{};
  st.n = n; st.depth = q; st.nnodes = P.nnodes; st.nleaves = P.nleaves;
  st.ncoupling = P.nadm_tot; st.ndense = P.ndense; st.csp = csp; st.csp_dense = csp_dense;
  st.entries_U = nU; st.entries_V = nV; st.entries_E = nE; st.entries_F = nF;
  st.entries_S = P.sdat[q + 1];
  st.entries_D = P.ddat[P.ndense];
  for (int64_t l = 0; l <= q; ++l) st.tree_rows += h->lv[l].count * h->lv[l].kmax;
  st.shared_basis = h->shared ? 1 : 0;
  for (int64_t l = 0; l <= q; ++l) st.max_rank = std::max(st.max_rank, h->lv[l].kmax);
  for (int64_t t = P.leaf0; t < P.nnodes; ++t) st.max_leaf = std::max<int64_t>(st.max_leaf, msz(t));
  {
    const double entries = (double)(st.entries_U + st.entries_V + st.entries_E + st.entries_F + st.entries_S +
                                    st.entries_D);
    st.alg_flops_per_vector = 2.0 * entries + (double)n;
    st.alg_bytes_matrix = 8.0 * entries;
    st.alg_bytes_per_vector = 8.0 * (2.0 * (double)n + 4.0 * (double)st.tree_rows);
  }

  // ---- upload
  const int64_t mat_bytes = P.off_end - P.off_U;
  if (mat_bytes > 0) {
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&h->d_mat), mat_bytes), "hipMalloc(matrix data)");
    const int64_t host_bytes = d_dense ? P.off_D - P.off_U : mat_bytes;
    if (host_bytes > 0)
      HIP_TRY(hipMemcpy(h->d_mat, buf + P.off_U, host_bytes, hipMemcpyHostToDevice), "hipMemcpy(matrix data)");
    if (d_dense && P.off_end > P.off_D)
      HIP_TRY(hipMemcpy(reinterpret_cast<uint8_t*>(h->d_mat) + (P.off_D - P.off_U), d_dense, P.off_end - P.off_D,
                        hipMemcpyDeviceToDevice),
              "hipMemcpy(dense blocks)");
  }
  // ---- transposed copies of the bases (for the upsweep products), made on
  // the device from the uploaded matrix data
  if (ntrans > 0) {
    std::vector<TransTask> tasks;
    transpose_tasks(lay, &tasks);
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&h->d_trans), ntrans * sizeof(double)), "hipMalloc(trans)");
    HIP_TRY(hipMemset(h->d_trans, 0, ntrans * sizeof(double)), "hipMemset(trans)");
    if (!tasks.empty()) {
      TransTask* d_tasks = nullptr;
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&d_tasks), sizeof(TransTask) * tasks.size()), "hipMalloc(tasks)");
      hipError_t e = hipMemcpy(d_tasks, tasks.data(), sizeof(TransTask) * tasks.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = launch_transpose_tasks(d_tasks, (int64_t)tasks.size(), h->d_mat, h->d_trans, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
      (void)hipFree(d_tasks);
      if (e != hipSuccess) return hip_fail(e, "transposed basis copies");
    }
  }
  h->prefix.assign((size_t)(P.off_U + 7) / 8, 0);
  std::memcpy(h->prefix.data(), buf, (size_t)P.off_U);
  h->prefix_len = P.off_U;
  std::vector<int32_t> perm(n), pinv(n);
  for (int64_t i = 0; i < n; ++i) {
    perm[i] = (int32_t)P.perm[i];
    pinv[P.perm[i]] = (int32_t)i;
  }
  for (const auto* v : {&h->planN.up, &h->planN.couple, &h->planN.down, &h->planN.dense, &h->planN.dense2,
                        &h->planN.couple_loc, &h->planN.dense_loc, &h->planN.dense2_loc, &h->planN.couple_deep,
                        &h->planN.couple_rest})
    for (const Launch& L : *v)
      if (L.kind != KIND_STREAM) h->mfma_ok = false;
  int64_t ib = 0;
  int rc;
  if ((rc = upload(perm, &h->d_perm, &ib)) || (rc = upload(pinv, &h->d_pinv, &ib)) || (rc = upload(h->rt.rows, &h->rt.d_rows, &ib)) ||
      (rc = upload(h->rt.colend, &h->rt.d_colend, &ib)) || (rc = upload(h->rt.in_off, &h->rt.d_in_off, &ib)) ||
      (rc = upload(h->wide.rows, &h->wide.d_rows, &ib)) ||
      (rc = upload(h->wide.colend, &h->wide.d_colend, &ib)) ||
      (rc = upload(h->wide.in_off, &h->wide.d_in_off, &ib)) || (rc = upload(h->gt.rows, &h->gt.d_rows, &ib)) ||
      (rc = upload(h->gt.data, &h->gt.d_data, &ib)) || (rc = upload(h->gt.mr, &h->gt.d_mr, &ib)) ||
      (rc = upload(h->gt.in_off, &h->gt.d_in_off, &ib)) || (rc = upload(tree_ranges, &h->d_tree_ranges, &ib)))
    return rc;
  h->index_bytes = ib;
  h->stats.device_bytes = mat_bytes + ntrans * (int64_t)sizeof(double) + ib;
  return H2_OK;
}

int ensure_workspace(h2_op_s* h, int64_t nv) {
  const int64_t want = (nv > kPassVectors && h->mfma_ok) ? kPassVectorsMfma : kPassVectors;
  if (h->ws.cap >= want) return H2_OK;
  if (h->ws.cap > 0) {  // grow: the old buffers may still be in use by queued work
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize(workspace growth)");
    h->stats.device_bytes -= ws_bytes(h->ws.n, h->ws.H, h->ws.cap);
    ws_destroy(&h->ws);
  }
  const int rc = ws_create(&h->ws, h->n, h->H, want);
  if (rc == H2_OK) h->stats.device_bytes += ws_bytes(h->ws.n, h->ws.H, h->ws.cap);
  return rc;
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

int load_common(const uint8_t* buf, int64_t len, int device, h2_handle* out, const double* d_dense = nullptr) {
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
  int ncu = 0;
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
  h2_op_s* h = new (std::nothrow) h2_op_s();
  if (!h) { set_error("out of host memory"); return H2_ENOMEM; }
  h->device = device;
  h->dense_stream_grid = 2 * (int64_t)std::max(ncu, 1);
  try {
    rc = build_handle(buf, P, h, d_dense);
    h->file_len = len;
  } catch (const std::bad_alloc&) {
    set_error("out of host memory while building schedules");
    rc = H2_ENOMEM;
  }
  // the no-allocation product's stream and events, and the device address
  // of its scratch array on this device
  if (rc == H2_OK) {
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&h->na.side, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->na.ev_fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->na.ev_join, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->na.ev_mid, hipEventDisableTiming)) != hipSuccess)
      rc = hip_fail(e, "stream and events of the no-allocation product");
  }
  if (rc == H2_OK) rc = scratch_attach(device);
  if (rc != H2_OK) {
    free_device(h);
    delete h;
    return rc;
  }
  *out = h;
  return H2_OK;
}

// nvp > 0: MFMA path with nvp vectors per row (row-major workspace).
// FP32: the low-rank launches read the FP32 copy of the data (the dense
// phase never does); x32: a coupling launch that may gather x^ from its FP32
// copy (w.xh32, converted from w.xh after the upsweep).
// out_ptr: an output buffer in place of the launch's own (the multi-vector
// leaf expansion into w.zx).
// A sweep transfer launch above the first level with coupling blocks: its
// parents' x^ is never read (upsweep) or their y^ is zero (downsweep), so it
// adds only exact zeros and does not run.
bool skipped(const h2_op_s* h, const Launch& L) { return L.level >= 0 && L.level < h->lmin; }

int run_launch(h2_op_s* h, const Workspace& w, const Launch& L, int nv, const Epilogue& ep, hipStream_t s,
               int nvp = 0, int mode_override = -1, int prec = H2_PREC_FP64, bool x32 = false,
               double* out_ptr = nullptr) {
  double* bufs[4] = {w.xt, w.xh, w.yh, w.zn};
  const bool lowp = prec == H2_PREC_FP32 && L.lowrank && L.kind != KIND_WIDE;
  if (prec == H2_PREC_BF16 && L.lowrank && nvp > 0) {
    // x^ lives as BF16 column-major [vector][ld16] in the x^ buffer's memory
    // (H * cap doubles hold ld16 * nvp BF16 values)
    const int64_t ld16 = (h->H + 7) / 8 * 8;
    const bool in16 = L.in == BUF_XH, out16 = mode_override < 0 && L.out == BUF_XH;
    const hipError_t eb = launch_rows_mfma_bf16(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend,
                                                h->rt.d_in_off, L.arr == ARR_TRANS ? h->d_trans16 : h->d_mat16,
                                                bufs[L.in], in16, ld16,
                                                out_ptr ? out_ptr : bufs[mode_override >= 0 ? BUF_ZN : L.out],
                                                out16, ld16, nvp, mode_override >= 0 ? mode_override : L.mode,
                                                L.max_rows, s, L.gridp[H2_PREC_BF16], L.remapp[H2_PREC_BF16]);
    if (eb != hipSuccess) return hip_fail(eb, "kernel launch");
    return H2_OK;
  }
  const double* data = L.arr == ARR_TRANS ? h->d_trans : h->d_mat;
  const float* data32 = L.arr == ARR_TRANS ? h->d_trans32 : h->d_mat32;
  double* out = out_ptr ? out_ptr : bufs[mode_override >= 0 ? BUF_ZN : L.out];
  const int mode = mode_override >= 0 ? mode_override : L.mode;
  hipError_t e = hipSuccess;
  // the dense rows' grid on the multi-vector path: the tuned one, or the
  // handle's override (h2_set_dense_grid)
  const int64_t grid_of = [&](int pi) {
    return (!L.lowrank && h->dense_grid_mv >= 0) ? h->dense_grid_mv : L.gridp[pi];
  }(lowp ? H2_PREC_FP32 : H2_PREC_FP64);
  const int kcw = L.kcp[lowp ? H2_PREC_FP32 : H2_PREC_FP64];
  if (nvp > 0 && (kcw == kWaveRows || kcw == kWaveTiles) && L.max_rows <= 64) {
    const bool narrow = kcw == kWaveTiles;
    const int rm = L.remapp[lowp ? H2_PREC_FP32 : H2_PREC_FP64];
    const bool fl = L.flp[lowp ? H2_PREC_FP32 : H2_PREC_FP64] != 0;
    const int occ = L.occp[lowp ? H2_PREC_FP32 : H2_PREC_FP64];
    e = lowp ? launch_wave_rows<float>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend, h->rt.d_in_off,
                                       data32, bufs[L.in], out, nvp, mode, L.max_rows, s, grid_of, narrow, rm,
                                       fl ? h->d_fl32 : nullptr, occ)
             : launch_wave_rows<double>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend, h->rt.d_in_off,
                                        data, bufs[L.in], out, nvp, mode, L.max_rows, s, grid_of, narrow, rm,
                                        fl ? h->d_fl : nullptr, occ);
  } else if (nvp > 0) {
    const int pi = lowp ? H2_PREC_FP32 : H2_PREC_FP64;
    const float* in32 = lowp && x32 && nvp == kPassVectorsMfma && L.in == BUF_XH ? w.xh32 : nullptr;
    e = lowp ? launch_rows_mfma<float>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend, h->rt.d_in_off,
                                       data32, bufs[L.in], out, nvp, mode, L.max_rows, s, L.kcp[pi], grid_of,
                                       L.remapp[pi], in32)
             : launch_rows_mfma<double>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend, h->rt.d_in_off,
                                        data, bufs[L.in], out, nvp, mode, L.max_rows, s, L.kcp[pi], grid_of,
                                        L.remapp[pi]);
  } else if (L.kind == KIND_STREAM) {
    // the dense rows (beside the sweeps) hold two workgroup slots per CU, so
    // the sweeps' small launches find free slots at once
    const int64_t sg = L.lowrank ? 0 : h->dense_stream_grid;
    e = lowp ? launch_rows<float>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend, h->rt.d_in_off, data32,
                                  bufs[L.in], out, nv, mode, ep, s, sg)
             : launch_rows<double>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend, h->rt.d_in_off, data,
                                   bufs[L.in], out, nv, mode, ep, s, sg);
  } else if (L.kind == KIND_WIDE) {
    e = launch_rows_wide(h->wide.d_rows + L.row_begin, L.row_count, h->wide.d_colend, h->wide.d_in_off, data,
                         bufs[L.in], out, nv, s);
  } else {
    e = lowp ? launch_gather<float>(h->gt.d_rows + L.row_begin, L.row_count, h->gt.d_data, h->gt.d_mr,
                                    h->gt.d_in_off, data32, bufs[L.in], out, nv, s)
             : launch_gather<double>(h->gt.d_rows + L.row_begin, L.row_count, h->gt.d_data, h->gt.d_mr,
                                     h->gt.d_in_off, data, bufs[L.in], out, nv, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return H2_OK;
}

int prepare_f32(h2_op_s* h) {
  std::lock_guard<std::mutex> lock(h->prep_mu);  // a concurrent call may be preparing it
  if (h->d_mat32 || h->n_lowrank + h->n_trans == 0) return H2_OK;
  float *m32 = nullptr, *t32 = nullptr;
  hipError_t e;
  if ((e = hipMalloc(reinterpret_cast<void**>(&m32), sizeof(float) * std::max<int64_t>(h->n_lowrank, 1))) !=
          hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&t32), sizeof(float) * std::max<int64_t>(h->n_trans, 1))) !=
          hipSuccess) {
    if (m32) (void)hipFree(m32);
    return hip_fail(e, "hipMalloc(FP32 copy)");
  }
  h->d_mat32 = m32;
  h->d_trans32 = t32;
  HIP_TRY(launch_to_f32(h->d_mat, m32, h->n_lowrank, nullptr), "FP32 copy");
  HIP_TRY(launch_to_f32(h->d_trans, t32, h->n_trans, nullptr), "FP32 copy");
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize(FP32 copy)");
  h->stats.device_bytes += (int64_t)sizeof(float) * (h->n_lowrank + h->n_trans);
  return H2_OK;
}

// The fragment-ordered copies of the op-'N' rows for the wave-row kernels:
// FP64 of every row, and for FP32 (after prepare_f32) of the low-rank rows.
int prepare_fl(h2_op_s* h, int prec) {
  std::lock_guard<std::mutex> lock(h->prep_mu);
  if (!h->mfma_ok) return H2_OK;
  const Plan& p = h->planN;
  if (!h->fl_placed) {
    // the copies' regions, in the rows' fl_off (the device row table is
    // rewritten; nothing runs on the handle meanwhile)
    FlKeys keys;
    keys.reserve(2 * h->rt.rows.size());
    int64_t n_fl = 0;
    for (const auto* v : {&p.up, &p.couple, &p.down, &p.dense, &p.dense2, &p.couple_loc, &p.dense_loc,
                          &p.dense2_loc, &p.couple_deep, &p.couple_rest})
      for (const Launch& L : *v)
        if (L.kind == KIND_STREAM) place_fl(h->rt, L.row_begin, L.row_begin + L.row_count, L.arr, &keys, &n_fl);
    place_fl(h->rt, p.out.row_begin, p.out.row_begin + p.out.row_count, p.out.arr, &keys, &n_fl);
    if (!h->rt.rows.empty())
      HIP_TRY(hipMemcpy(h->rt.d_rows, h->rt.rows.data(), sizeof(RowDesc) * h->rt.rows.size(), hipMemcpyHostToDevice),
              "hipMemcpy(row table)");
    h->n_fl = n_fl;
    h->fl_placed = true;
  }
  if (h->n_fl == 0) return H2_OK;
  // one copy: every launch's rows (FP64), or the low-rank ones (FP32); the
  // handle keeps it only when every relayout ran
  auto make = [&](void* d, bool fp32) -> hipError_t {
    hipError_t e = hipSuccess;
    auto one = [&](const Launch& L) {
      if (e != hipSuccess || (fp32 && !L.lowrank)) return;  // the dense rows stay FP64
      if (fp32)
        e = launch_rows_to_fl<float>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend,
                                     L.arr == ARR_TRANS ? h->d_trans32 : h->d_mat32, static_cast<float*>(d), nullptr);
      else
        e = launch_rows_to_fl<double>(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend,
                                      L.arr == ARR_TRANS ? h->d_trans : h->d_mat, static_cast<double*>(d), nullptr);
    };
    for (const auto* v : {&p.up, &p.couple, &p.down, &p.dense, &p.dense2, &p.couple_loc, &p.dense_loc,
                          &p.dense2_loc, &p.couple_deep, &p.couple_rest})
      for (const Launch& L : *v) one(L);
    one(p.out);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
  };
  if (!h->d_fl) {
    double* d = nullptr;
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&d), sizeof(double) * h->n_fl), "hipMalloc(fragment-ordered copy)");
    const hipError_t e = make(d, false);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return hip_fail(e, "fragment-ordered copy");
    }
    h->d_fl = d;
    h->stats.device_bytes += (int64_t)sizeof(double) * h->n_fl;
  }
  if (prec == H2_PREC_FP32 && h->d_mat32 && !h->d_fl32) {
    float* d = nullptr;
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&d), sizeof(float) * h->n_fl), "hipMalloc(fragment-ordered copy)");
    const hipError_t e = make(d, true);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return hip_fail(e, "fragment-ordered copy");
    }
    h->d_fl32 = d;
    h->stats.device_bytes += (int64_t)sizeof(float) * h->n_fl;
  }
  return H2_OK;
}

// Frees a fragment-ordered copy that no tuned launch reads (the FP64 copy
// serves every precision's dense rows through their FP64 entry).
int drop_unused_fl(h2_op_s* h) {
  std::lock_guard<std::mutex> lock(h->prep_mu);
  bool use64 = false, use32 = false;
  auto look = [&](const Launch& L) {
    auto reads = [&](int p) { return (L.kcp[p] == kWaveRows || L.kcp[p] == kWaveTiles) && L.flp[p] != 0; };
    use64 = use64 || reads(H2_PREC_FP64);
    use32 = use32 || (L.lowrank && reads(H2_PREC_FP32));
  };
  const Plan& p = h->planN;
  for (const auto* v : {&p.up, &p.couple, &p.down, &p.dense, &p.dense2, &p.couple_loc, &p.dense_loc,
                        &p.dense2_loc, &p.couple_deep, &p.couple_rest})
    for (const Launch& L : *v) look(L);
  look(p.out);
  if (!use64 && h->d_fl) {
    HIP_TRY(hipFree(h->d_fl), "hipFree(fragment-ordered copy)");
    h->d_fl = nullptr;
    h->stats.device_bytes -= (int64_t)sizeof(double) * h->n_fl;
  }
  if (!use32 && h->d_fl32) {
    HIP_TRY(hipFree(h->d_fl32), "hipFree(fragment-ordered copy)");
    h->d_fl32 = nullptr;
    h->stats.device_bytes -= (int64_t)sizeof(float) * h->n_fl;
  }
  return H2_OK;
}

int prepare_bf16(h2_op_s* h) {
  std::lock_guard<std::mutex> lock(h->prep_mu);
  if (h->d_mat16 || h->n_lowrank + h->n_trans == 0) return H2_OK;
  void *m16 = nullptr, *t16 = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&m16, 2 * std::max<int64_t>(h->n_lowrank, 1))) != hipSuccess ||
      (e = hipMalloc(&t16, 2 * std::max<int64_t>(h->n_trans, 1))) != hipSuccess) {
    if (m16) (void)hipFree(m16);
    return hip_fail(e, "hipMalloc(BF16 copy)");
  }
  h->d_mat16 = m16;
  h->d_trans16 = t16;
  const Plan& p = h->planN;
  for (const auto* v : {&p.up, &p.couple, &p.down})
    for (const Launch& L : *v)
      HIP_TRY(launch_rows_to_bf16(h->rt.d_rows + L.row_begin, L.row_count, h->rt.d_colend,
                                  L.arr == ARR_TRANS ? h->d_trans : h->d_mat, L.arr == ARR_TRANS ? t16 : m16, nullptr),
              "BF16 copy");
  HIP_TRY(launch_rows_to_bf16(h->rt.d_rows + p.out.row_begin, p.out.row_count, h->rt.d_colend, h->d_mat, m16, nullptr),
          "BF16 copy");
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize(BF16 copy)");
  h->stats.device_bytes += 2 * (h->n_lowrank + h->n_trans);
  return H2_OK;
}

// The fused sweep launches of one direction (multi-vector path, FP64/FP32).
int run_tree(h2_op_s* h, const Workspace& w, const std::vector<TreeGroup>& groups, int nvp, int prec,
             hipStream_t s) {
  double* const bufs[4] = {w.xt, w.xh, w.yh, w.zx};
  for (const TreeGroup& G : groups) {
    const hipError_t e =
        prec == H2_PREC_FP32
            ? launch_tree<float>(h->d_tree_ranges + G.range_off, G.nwg, G.lv, h->rt.d_rows, h->rt.d_colend,
                                 h->rt.d_in_off, G.trans_data ? h->d_trans32 : h->d_mat32, bufs, nvp, G.max_rows, s)
            : launch_tree<double>(h->d_tree_ranges + G.range_off, G.nwg, G.lv, h->rt.d_rows, h->rt.d_colend,
                                  h->rt.d_in_off, G.trans_data ? h->d_trans : h->d_mat, bufs, nvp, G.max_rows, s);
    if (e != hipSuccess) return hip_fail(e, "fused sweep launch");
  }
  return H2_OK;
}

// Whether a multi-vector pass runs the fused sweeps.
bool use_tree(const h2_op_s* h, const Workspace& w, bool trans, int nvp, int prec) {
  const int pidx = prec == H2_PREC_FP32 ? 1 : prec == H2_PREC_BF16 ? 2 : 0;
  return nvp > 0 && !trans && prec != H2_PREC_BF16 && h->tree_ok && w.zx != nullptr && h->sweep_fused[pidx] != 0;
}

// One pass of the product: nv <= kPassVectors vectors on the streaming path
// (nvp == 0), or nv <= kPassVectorsMfma vectors padded to nvp on the MFMA path.
int gemv_pass(h2_op_s* h, const Workspace& w, bool trans, double alpha, const double* X, int64_t ldx, int nv,
              double beta, double* Y, int64_t ldy, hipStream_t s, int nvp, int prec) {
  const Plan& plan = trans ? h->planT : h->planN;
  // tree-ordered coupling / dense rows on the multi-vector path when tuned so
  const int pidx = prec == H2_PREC_FP32 ? 1 : prec == H2_PREC_BF16 ? 2 : 0;
  const int cm = (!trans && nvp > 0) ? h->couple_mode[pidx] : 0;
  const int dm = (!trans && nvp > 0) ? h->dense_mode[pidx] : 0;
  const std::vector<Launch>& couple = cm == 1 ? plan.couple_loc : plan.couple;
  const std::vector<Launch>& dense1 = dm == 1 ? plan.dense_loc : plan.dense;
  const std::vector<Launch>& dense2 = dm == 1 ? plan.dense2_loc : plan.dense2;
  std::array<hipEvent_t, 13>* ev = nullptr;
  if (h->profiling && &w == &h->ws) {
    if (h->ev_used == h->ev_pool.size()) {
      std::array<hipEvent_t, 13> set{};
      for (auto& e : set) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
      h->ev_pool.push_back(set);
    }
    ev = &h->ev_pool[h->ev_used++];
  }
  auto mark = [&](int i, hipStream_t st) -> int {
    if (ev) HIP_TRY(hipEventRecord((*ev)[i], st), "hipEventRecord");
    return H2_OK;
  };
  Epilogue ep{w.zn, h->d_perm, alpha, beta, Y, ldy, h->n};
  int rc;
#define STEP(x) do { if ((rc = (x)) != H2_OK) return rc; } while (0)
  STEP(mark(0, s));
  if (nvp) HIP_TRY(launch_permute_in_rm(X, ldx, h->d_pinv, w.xt, h->n, nv, nvp, s), "permute");
  else HIP_TRY(launch_permute_in(X, ldx, h->d_perm, w.xt, h->n, nv, s), "permute");
  STEP(mark(1, s));
  // dense near field on the side stream, concurrent with the low-rank phases.
  // Schedule (multi-vector path, per precision, h2_tune): 0 the first half
  // beside the upsweep, the second beside the downsweep; 1 the first half
  // beside the coupling launch instead; 2 both halves from the start; 3 as 2,
  // and the leaf level's coupling rows on a third stream as soon as the leaf
  // products are done, beside the upper upsweep, the other levels' coupling
  // rows and the upper downsweep (the last downsweep level waits for them).
  const int sched = trans ? 0 : nvp > 0 ? h->sched[pidx] : h->sched1[pidx];
  const bool fused = use_tree(h, w, trans, nvp, prec);
  // FP32 at 64 vectors: the coupling launches gather x^ from an FP32 copy
  const bool x32 = prec == H2_PREC_FP32 && nvp == kPassVectorsMfma && w.xh32;
  // (a workspace without the third stream, such as the no-allocation
  // product's views, takes schedule 2's order instead)
  const bool split = sched == 3 && !fused && !x32 && !plan.down.empty() && !plan.couple_deep.empty() &&
                     !plan.up.empty() && w.side2 && w.ev_deep && w.ev_deep_done;
  auto fork_dense1 = [&]() -> int {
    HIP_TRY(hipEventRecord(w.ev_fork, s), "hipEventRecord(fork)");
    HIP_TRY(hipStreamWaitEvent(w.side, w.ev_fork, 0), "hipStreamWaitEvent(fork)");
    STEP(mark(5, w.side));
    for (const Launch& L : dense1) STEP(run_launch(h, w, L, nv, ep, w.side, nvp));
    STEP(mark(9, w.side));
    return H2_OK;
  };
  if (sched != 1) STEP(fork_dense1());
  if (fused) {
    STEP(run_tree(h, w, h->tree_up, nvp, prec, s));
  } else {
    for (size_t i = 0; i < plan.up.size(); ++i) {
      if (!skipped(h, plan.up[i])) STEP(run_launch(h, w, plan.up[i], nv, ep, s, nvp, -1, prec));
      if (split && i == 0) {  // the leaf level's x^ is complete
        HIP_TRY(hipEventRecord(w.ev_deep, s), "hipEventRecord(deep)");
        HIP_TRY(hipStreamWaitEvent(w.side2, w.ev_deep, 0), "hipStreamWaitEvent(deep)");
        STEP(mark(11, w.side2));
        for (const Launch& L : plan.couple_deep) STEP(run_launch(h, w, L, nv, ep, w.side2, nvp, -1, prec));
        STEP(mark(12, w.side2));
        HIP_TRY(hipEventRecord(w.ev_deep_done, w.side2), "hipEventRecord(deep done)");
      }
    }
  }
  if (x32) HIP_TRY(launch_to_f32(w.xh, w.xh32, h->H * (int64_t)nvp, s), "x^ to FP32");
  if (sched == 1) STEP(fork_dense1());
  STEP(mark(2, s));
  for (const Launch& L : (split ? plan.couple_rest : couple)) STEP(run_launch(h, w, L, nv, ep, s, nvp, -1, prec, x32));
  STEP(mark(3, s));
  if (!split) {  // no third-stream interval: a zero one
    STEP(mark(11, s));
    STEP(mark(12, s));
  }
  // second half of the dense rows, beside the downsweep and the leaf expansion
  if (sched != 2 && sched != 3) {
    HIP_TRY(hipEventRecord(w.ev_mid, s), "hipEventRecord(mid)");
    HIP_TRY(hipStreamWaitEvent(w.side, w.ev_mid, 0), "hipStreamWaitEvent(mid)");
  }
  STEP(mark(10, w.side));
  for (const Launch& L : dense2) STEP(run_launch(h, w, L, nv, ep, w.side, nvp));
  STEP(mark(6, w.side));
  HIP_TRY(hipEventRecord(w.ev_join, w.side), "hipEventRecord(join)");
  // Multi-vector path: the leaf expansion U y^ goes to its own buffer w.zx,
  // beside the dense rows (the fused downsweep ends with it); the output
  // permutation adds the dense partial, the same Z + U y^ addition.
  const bool zx = nvp > 0 && w.zx != nullptr;
  if (fused) {
    STEP(run_tree(h, w, h->tree_down, nvp, prec, s));
  } else {
    for (size_t i = 0; i < plan.down.size(); ++i) {
      if (split && i + 1 == plan.down.size())  // the leaf level's y^ needs its coupling rows
        HIP_TRY(hipStreamWaitEvent(s, w.ev_deep_done, 0), "hipStreamWaitEvent(deep done)");
      if (!skipped(h, plan.down[i])) STEP(run_launch(h, w, plan.down[i], nv, ep, s, nvp, -1, prec));
    }
  }
  if (zx && !fused) STEP(run_launch(h, w, plan.out, nv, ep, s, nvp, MODE_STORE, prec, false, w.zx));
  STEP(mark(4, s));
  HIP_TRY(hipStreamWaitEvent(s, w.ev_join, 0), "hipStreamWaitEvent(join)");
  STEP(mark(7, s));
  if (zx) {
    // Y = alpha (Z + U y^)[pinv] + beta Y
    HIP_TRY(launch_permute_out_rm2(w.zn, w.zx, h->d_pinv, alpha, beta, Y, ldy, h->n, nv, nvp, s), "permute out");
  } else if (nvp) {
    // Z += U y^ (into the dense partial), then Y = alpha Z[pinv] + beta Y
    STEP(run_launch(h, w, plan.out, nv, ep, s, nvp, MODE_ACCUM, prec));
    HIP_TRY(launch_permute_out_rm(w.zn, h->d_pinv, alpha, beta, Y, ldy, h->n, nv, nvp, s), "permute out");
  } else {
    STEP(run_launch(h, w, plan.out, nv, ep, s, 0, -1, prec));
  }
  STEP(mark(8, s));
#undef STEP
  return H2_OK;
}

}  // namespace

int load_handle(const uint8_t* buf, int64_t len, int device, const double* d_dense, h2_handle* out) {
  return load_common(buf, len, device, out, d_dense);
}

bool prepared(h2_op_s* h, int prec) {
  if (prec == H2_PREC_FP64) return true;
  std::lock_guard<std::mutex> lock(h->prep_mu);
  const bool empty = h->n_lowrank + h->n_trans == 0;
  if (prec == H2_PREC_FP32) return empty || h->d_mat32 != nullptr;
  return h->mfma_ok && (empty || h->d_mat16 != nullptr);
}
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
  std::vector<uint64_t> storage;
  try {
    storage.resize(((size_t)len + 7) / 8);
  } catch (const std::bad_alloc&) {
    std::fclose(f);
    set_error("out of host memory");
    return H2_ENOMEM;
  }
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

}  // extern "C"

namespace h2 {
int64_t ws_bytes(int64_t n, int64_t H, int64_t cap) {
  return (int64_t)sizeof(double) *
             (2 * std::max<int64_t>(n, 1) + std::max<int64_t>(H, 8) + std::max<int64_t>(H, 1)) * cap +
         (cap >= kPassVectorsMfma ? (int64_t)sizeof(float) * std::max<int64_t>(H, 1) * cap +
                                        (int64_t)sizeof(double) * std::max<int64_t>(n, 1) * cap
                                  : 0);
}

int ws_create(Workspace* w, int64_t n, int64_t H, int64_t cap) {
  *w = Workspace();
  w->n = n;
  w->H = H;
  const int64_t nn = std::max<int64_t>(n, 1), Hs = std::max<int64_t>(H, 1);
  hipError_t e;
  if ((e = hipMalloc(reinterpret_cast<void**>(&w->xt), sizeof(double) * nn * cap)) != hipSuccess ||
      // at least 8 rows: the BF16 path keeps x^ as BF16 [nvp][round_up(H, 8)] in this memory
      (e = hipMalloc(reinterpret_cast<void**>(&w->xh), sizeof(double) * std::max<int64_t>(Hs, 8) * cap)) !=
          hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&w->yh), sizeof(double) * Hs * cap)) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void**>(&w->zn), sizeof(double) * nn * cap)) != hipSuccess ||
      (cap >= kPassVectorsMfma &&
       (e = hipMalloc(reinterpret_cast<void**>(&w->xh32), sizeof(float) * Hs * cap)) != hipSuccess) ||
      (cap >= kPassVectorsMfma &&
       (e = hipMalloc(reinterpret_cast<void**>(&w->zx), sizeof(double) * nn * cap)) != hipSuccess) ||
      (e = hipStreamCreateWithFlags(&w->side, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev_fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev_join, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev_mid, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&w->side2, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev_deep, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev_deep_done, hipEventDisableTiming)) != hipSuccess) {
    ws_destroy(w);
    return hip_fail(e, "workspace allocation");
  }
  w->cap = cap;
  return H2_OK;
}

void ws_destroy(Workspace* w) {
  for (double* p : {w->xt, w->xh, w->yh, w->zn})
    if (p) (void)hipFree(p);
  if (w->xh32) (void)hipFree(w->xh32);
  if (w->zx) (void)hipFree(w->zx);
  if (w->ev_fork) (void)hipEventDestroy(w->ev_fork);
  if (w->ev_join) (void)hipEventDestroy(w->ev_join);
  if (w->ev_mid) (void)hipEventDestroy(w->ev_mid);
  if (w->side) (void)hipStreamDestroy(w->side);
  if (w->ev_deep) (void)hipEventDestroy(w->ev_deep);
  if (w->ev_deep_done) (void)hipEventDestroy(w->ev_deep_done);
  if (w->side2) (void)hipStreamDestroy(w->side2);
  *w = Workspace();
}

// The product on an explicit workspace (sized for this operator); used by
// h2_gemv_ex with the handle's workspace and by the server with a slot's.
int gemv_ws(h2_op_s* h, const Workspace& w, bool trans, double alpha, const double* X, int64_t ldx, int64_t nv,
            double beta, double* Y, int64_t ldy, int prec, hipStream_t s) {
  int rc;
  if (prec == H2_PREC_FP32 && (rc = prepare_f32(h)) != H2_OK) return rc;
  if (prec == H2_PREC_BF16) {
    if (trans || !h->mfma_ok || w.cap < kPassVectorsMfma) {
      set_error("BF16 needs op 'N' and the MFMA path");
      return H2_EUNSUPPORTED;
    }
    if ((rc = prepare_bf16(h)) != H2_OK) return rc;
  }
  // multi-vector products of op 'N' (and every BF16 product) go to the MFMA kernels
  const bool mfma = !trans && h->mfma_ok && w.cap >= kPassVectorsMfma && (nv > kPassVectors || prec == H2_PREC_BF16);
  // (a workspace with fewer than kPassVectors columns takes passes of its width)
  const int64_t pass = mfma ? kPassVectorsMfma : std::min<int64_t>(kPassVectors, w.cap);
  for (int64_t v0 = 0; v0 < nv; v0 += pass) {
    const int nvc = (int)std::min<int64_t>(pass, nv - v0);
    rc = gemv_pass(h, w, trans, alpha, X + ldx * v0, ldx, nvc, beta, Y + ldy * v0, ldy, s,
                   mfma ? (nvc + 15) / 16 * 16 : 0, prec);
    if (rc != H2_OK) return rc;
  }
  return H2_OK;
}

int check_gemv_args(h2_op_s* h, char op, double alpha, const double* X, int64_t ldx, int64_t nv, double* Y,
                    int64_t ldy, int prec, bool* trans) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  if (prec != H2_PREC_FP64 && prec != H2_PREC_FP32 && prec != H2_PREC_BF16) {
    set_error("unknown precision");
    return H2_EINVAL;
  }
  *trans = op == 'T' || op == 't';
  if (!*trans && op != 'N' && op != 'n') { set_error("op must be 'N' or 'T'"); return H2_EINVAL; }
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
  return H2_OK;
}
}  // namespace h2

namespace {
// Streaming products (nv <= kPassVectors): the four schedules of
// h2_set_schedule timed on whole products (a warm-up, then three runs each)
// on zeroed buffers; the fastest is kept.
// A schedule later in the list replaces the best so far only when it is at
// least 1% faster: schedules differ by a few per cent at most, and a choice
// made on timing noise would move the launches' overlap from run to run.
constexpr float kScheduleGain = 0.99f;

int tune_stream_schedule(h2_op_s* h, int64_t nv, int prec, void* stream) {
  if (nv == 0) return H2_OK;
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);
  int rc;
  if ((rc = h2_prepare(h, prec)) != H2_OK) return rc;
  if ((rc = ensure_workspace(h, nv)) != H2_OK) return rc;
  const int nvc = (int)std::min<int64_t>(nv, kPassVectors);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *X = nullptr, *Y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t vb = sizeof(double) * (size_t)std::max<int64_t>(h->n, 1) * nvc;
  auto done = [&](int r) {
    if (X) (void)hipFree(X);
    if (Y) (void)hipFree(Y);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return r;
  };
  if (hipMalloc(reinterpret_cast<void**>(&X), vb) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&Y), vb) != hipSuccess || hipMemsetAsync(X, 0, vb, s) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("tuning buffers");
    return done(H2_ENOMEM);
  }
  // each schedule: two warm-up products, then products one at a time (each
  // waited for) for about 4 ms, 3 to 63 of them, and the median time: a
  // product of ~0.1 ms varies by more than the schedules differ when timed
  // a few times, and the latency of one product is what a schedule changes
  const int orig = h->sched1[prec];
  auto timed = [&](float* ms) -> int {
    if (hipEventRecord(e0, s) != hipSuccess) return H2_EHIP;
    const int rr = gemv_ws(h, h->ws, false, 1.0, X, h->n, nvc, 0.0, Y, h->n, prec, s);
    if (rr != H2_OK) return rr;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess) {
      set_error("timing the streaming schedules failed");
      return H2_EHIP;
    }
    return H2_OK;
  };
  float best = 1e30f;
  int best_s = orig;
  for (int sc = 0; sc < 4; ++sc) {
    h->sched1[prec] = sc;
    float t1 = 0.0f;
    if ((rc = timed(&t1)) != H2_OK || (rc = timed(&t1)) != H2_OK) {
      h->sched1[prec] = orig;
      return done(rc);
    }
    const int reps = (int)std::min(63.0f, std::max(3.0f, std::ceil(4.0f / std::max(t1, 1e-3f))));
    std::vector<float> ts((size_t)reps);
    for (int r = 0; r < reps; ++r)
      if ((rc = timed(&ts[(size_t)r])) != H2_OK) {
        h->sched1[prec] = orig;
        return done(rc);
      }
    std::nth_element(ts.begin(), ts.begin() + reps / 2, ts.end());
    const float t = ts[(size_t)reps / 2];
    h->sched1_ms[prec][sc] = t;
    if (t < best * kScheduleGain) {
      best = t;
      best_s = sc;
    }
  }
  h->sched1[prec] = best_s;
  return done(H2_OK);
}
}  // namespace

extern "C" {
int h2_gemv_ex(h2_handle h, char op, double alpha, const double* X, int64_t ldx, int64_t nv, double beta,
               double* Y, int64_t ldy, int prec, void* stream) {
  bool trans = false;
  int rc = check_gemv_args(h, op, alpha, X, ldx, nv, Y, ldy, prec, &trans);
  if (rc != H2_OK || nv == 0) return rc;
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (alpha == 0.0) {
    HIP_TRY(launch_scale(Y, ldy, h->n, nv, beta, s), "scale");
    return H2_OK;
  }
  if ((rc = ensure_workspace(h, prec == H2_PREC_BF16 ? kPassVectorsMfma : nv)) != H2_OK) return rc;
  if (h->use_graph && s != nullptr && !h->profiling) {
    // replay the call's captured launch sequence, or capture it now (the
    // reduced-precision copy is made first: its allocation and
    // synchronization cannot be captured)
    if (prec == H2_PREC_FP32 && (rc = prepare_f32(h)) != H2_OK) return rc;
    if (prec == H2_PREC_BF16 && (rc = prepare_bf16(h)) != H2_OK) return rc;
    const GraphKey key{trans, prec, X, ldx, nv, alpha, beta, Y, ldy, s};
    for (GraphEntry& g : h->graphs)
      if (g.key == key) {
        g.last_use = ++h->graph_clock;
        HIP_TRY(hipGraphLaunch(g.exec, s), "hipGraphLaunch");
        return H2_OK;
      }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    rc = gemv_ws(h, h->ws, trans, alpha, X, ldx, nv, beta, Y, ldy, prec, s);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc != H2_OK || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != H2_OK) return rc;
      return hip_fail(ec, "hipStreamEndCapture");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
    if (h->graphs.size() >= kMaxGraphs) {  // drop the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < h->graphs.size(); ++i)
        if (h->graphs[i].last_use < h->graphs[lru].last_use) lru = i;
      HIP_TRY(hipStreamSynchronize(h->graphs[lru].key.s), "hipStreamSynchronize(graph)");
      (void)hipGraphExecDestroy(h->graphs[lru].exec);
      h->graphs.erase(h->graphs.begin() + (long)lru);
    }
    h->graphs.push_back(GraphEntry{key, exec, ++h->graph_clock});
    HIP_TRY(hipGraphLaunch(exec, s), "hipGraphLaunch");
    return H2_OK;
  }
  if ((rc = gemv_ws(h, h->ws, trans, alpha, X, ldx, nv, beta, Y, ldy, prec, s)) != H2_OK) return rc;
  if (h->profiling) ++h->prof.calls;
  return H2_OK;
}

int h2_graph(h2_handle h, int enable) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);
  h->use_graph = enable != 0;
  return H2_OK;
}

int h2_gemv(h2_handle h, char op, double alpha, const double* X, int64_t ldx, int64_t nv, double beta, double* Y,
            int64_t ldy, void* stream) {
  return h2_gemv_ex(h, op, alpha, X, ldx, nv, beta, Y, ldy, H2_PREC_FP64, stream);
}

int h2_prepare(h2_handle h, int prec) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  if (prec == H2_PREC_FP64) return H2_OK;
  if (prec != H2_PREC_FP32 && prec != H2_PREC_BF16) { set_error("unknown precision"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  return prec == H2_PREC_FP32 ? prepare_f32(h) : prepare_bf16(h);
}

int h2_tune(h2_handle h, int64_t nv, int prec, void* stream) {
  if (!h || nv < 0) { set_error("bad handle or nv"); return H2_EINVAL; }
  if (prec != H2_PREC_FP64 && prec != H2_PREC_FP32 && prec != H2_PREC_BF16) {
    set_error("unknown precision");
    return H2_EINVAL;
  }
  if (nv <= kPassVectors && prec != H2_PREC_BF16) return tune_stream_schedule(h, nv, prec, stream);
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);  // captured with the old launch parameters
  int rc;
  if ((rc = h2_prepare(h, prec)) != H2_OK) return rc;
  if ((rc = ensure_workspace(h, prec == H2_PREC_BF16 ? kPassVectorsMfma : nv)) != H2_OK) return rc;
  if (!h->mfma_ok) return H2_OK;
  if (prec != H2_PREC_BF16 && (rc = prepare_fl(h, prec)) != H2_OK) return rc;
  const int nvp = (int)std::min<int64_t>((nv + 15) / 16 * 16, kPassVectorsMfma);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Workspace& w = h->ws;
  // the candidates run on zeroed buffers (their timing does not depend on the values)
  HIP_TRY(hipMemsetAsync(w.xt, 0, sizeof(double) * std::max<int64_t>(w.n, 1) * w.cap, s), "hipMemsetAsync");
  HIP_TRY(hipMemsetAsync(w.xh, 0, sizeof(double) * std::max<int64_t>(w.H, 8) * w.cap, s), "hipMemsetAsync");
  HIP_TRY(hipMemsetAsync(w.yh, 0, sizeof(double) * std::max<int64_t>(w.H, 1) * w.cap, s), "hipMemsetAsync");
  HIP_TRY(hipMemsetAsync(w.zn, 0, sizeof(double) * std::max<int64_t>(w.n, 1) * w.cap, s), "hipMemsetAsync");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return H2_EHIP;
  }
  const Epilogue ep{w.zn, h->d_perm, 1.0, 0.0, nullptr, 0, h->n};
  if (w.xh32)
    HIP_TRY(hipMemsetAsync(w.xh32, 0, sizeof(float) * std::max<int64_t>(w.H, 1) * w.cap, s), "hipMemsetAsync");
  // FP32 at 64 vectors: the coupling candidates gather from the FP32 copy of x^
  const bool x32 = prec == H2_PREC_FP32 && nvp == kPassVectorsMfma && w.xh32;
  // best candidate of one launch; its time (ms, two timed runs) in *tbest
  auto tune_one = [&](Launch& L, int mode_override, float* tbest, bool couple = false) -> int {
    const int pi = L.lowrank ? prec : H2_PREC_FP64;
    // 0: pipelined, 1-8: balanced (64 vectors only), kWaveRows / kWaveTiles: a wave per row / per
    // 16-vector tile (rows of <= 64 outputs)
    const int kcs[13] = {32, 64, 0, 1, 2, 3, 4, 5, 6, 7, 8, kWaveRows, kWaveTiles};
    const int64_t grids[4] = {0, 1024, 2048, 4096};
    float best = 1e30f;
    int best_kc = L.kcp[pi], best_remap = L.remapp[pi], best_fl = L.flp[pi], best_occ = L.occp[pi];
    int64_t best_grid = L.gridp[pi];
    // the wave-row kernels also without the fragment-ordered copy
    const bool has_fl = pi == H2_PREC_FP32 ? h->d_fl32 != nullptr : h->d_fl != nullptr;
    for (int kc : kcs) {
      if (pi == H2_PREC_BF16 && kc != 64) continue;  // the BF16 kernel has one chunk width
      if (kc >= 0 && kc <= 8 && nvp != 64) continue;
      if (kc >= 1 && kc <= 8 && L.max_rows > 64) continue;
      if ((kc == kWaveRows || kc == kWaveTiles) && L.max_rows > 64) continue;
      if (kc == kWaveTiles && nvp != 32 && nvp != 64) continue;
      const bool wave = kc == kWaveRows || kc == kWaveTiles;
      for (int64_t g : grids)
        for (int cand = 0; cand < (wave ? 8 : 2); ++cand) {
          // wave-row forms: also without the copy, and the five-waves-per-SIMD form
          const int remap = cand & 1, fl = wave && has_fl ? (cand >> 1) & 1 : 1, occ = cand >> 2 ? 5 : 0;
          if (wave && !has_fl && (cand >> 1) & 1) continue;
          if (occ && !wave_occ5(nvp, L.max_rows, kc == kWaveTiles)) continue;
          if (g != 0 && g >= L.row_count) continue;
          // the dense rows run beside the sweeps: a persistent grid would hold
          // every CU slot and starve them, so they keep one workgroup per row
          if (g != 0 && !L.lowrank) continue;
          Launch T = L;
          T.kcp[pi] = kc;
          T.gridp[pi] = g;
          T.remapp[pi] = remap;
          T.flp[pi] = fl;
          T.occp[pi] = occ;
          float tsum = 0.0f;
          for (int rep = 0; rep < 3; ++rep) {
            HIP_TRY(hipEventRecord(e0, s), "hipEventRecord");
            int r = run_launch(h, w, T, nvp, ep, s, nvp, mode_override, L.lowrank ? prec : H2_PREC_FP64,
                               couple && x32);
            if (r != H2_OK) return r;
            HIP_TRY(hipEventRecord(e1, s), "hipEventRecord");
            HIP_TRY(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (rep > 0) tsum += ms;  // the first repetition warms up
          }
          if (tsum < best) {
            best = tsum;
            best_kc = kc;
            best_grid = g;
            best_remap = remap;
            best_fl = fl;
            best_occ = occ;
          }
        }
    }
    L.kcp[pi] = best_kc;
    L.gridp[pi] = best_grid;
    L.remapp[pi] = best_remap;
    L.flp[pi] = best_fl;
    L.occp[pi] = best_occ;
    L.tuned_ms[pi] = best / 2;
    if (tbest) *tbest = best;
    return H2_OK;
  };
  Plan& plan = h->planN;
  auto tune_list = [&](std::vector<Launch>& v, float* total, bool couple = false) -> int {
    *total = 0.0f;
    for (Launch& L : v) {
      if (skipped(h, L)) continue;  // never runs
      float t = 0.0f;
      const int r = tune_one(L, -1, &t, couple);
      if (r != H2_OK) return r;
      *total += t;
    }
    return H2_OK;
  };
  float t_up = 0, t_down = 0, t_out = 0, tc = 0, tcl = 0, td1 = 0, td2 = 0, tl1 = 0, tl2 = 0;
  rc = tune_list(plan.up, &t_up);
  if (rc == H2_OK) rc = tune_list(plan.down, &t_down);
  if (rc == H2_OK) rc = tune_list(plan.couple, &tc, true);
  if (rc == H2_OK) rc = tune_list(plan.couple_loc, &tcl, true);
  // the split coupling rows of schedule 3 (their times are not compared)
  for (auto* v : {&plan.couple_deep, &plan.couple_rest})
    for (Launch& L : *v)
      if (rc == H2_OK) rc = tune_one(L, -1, nullptr, true);
  if (rc == H2_OK) rc = tune_list(plan.dense, &td1);
  if (rc == H2_OK) rc = tune_list(plan.dense2, &td2);
  if (rc == H2_OK) rc = tune_list(plan.dense_loc, &tl1);
  if (rc == H2_OK) rc = tune_list(plan.dense2_loc, &tl2);
  if (rc == H2_OK) rc = tune_one(plan.out, w.zx ? MODE_STORE : MODE_ACCUM, &t_out);  // as the product runs it
  if (rc == H2_OK) {
    h->couple_mode[prec] = tcl < tc ? 1 : 0;
    h->dense_mode[prec] = tl1 + tl2 < td1 + td2 ? 1 : 0;
  }
  // fused sweeps (both directions, leaf expansion included) against the tuned
  // per-level launches, two timed runs each after a warm-up
  if (rc == H2_OK && prec != H2_PREC_BF16 && h->tree_ok && w.zx) {
    float tf = 0.0f;
    for (int rep = 0; rep < 3 && rc == H2_OK; ++rep) {
      HIP_TRY(hipEventRecord(e0, s), "hipEventRecord");
      rc = run_tree(h, w, h->tree_up, nvp, prec, s);
      if (rc == H2_OK) rc = run_tree(h, w, h->tree_down, nvp, prec, s);
      HIP_TRY(hipEventRecord(e1, s), "hipEventRecord");
      HIP_TRY(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (rep > 0) tf += ms;
    }
    const float tl = t_up + t_down + t_out;
    if (rc == H2_OK) {
      h->sweep_fused[prec] = tf < tl ? 1 : 0;
      h->sweep_ms[prec][0] = tl / 2;
      h->sweep_ms[prec][1] = tf / 2;
    }
  }
  // the dense rows' schedule, timed on whole products (three runs each after
  // a warm-up) on zeroed input and output buffers
  if (rc == H2_OK) {
    double *X = nullptr, *Y = nullptr;
    const size_t vb = sizeof(double) * (size_t)std::max<int64_t>(h->n, 1) * nvp;
    if (hipMalloc(reinterpret_cast<void**>(&X), vb) == hipSuccess &&
        hipMalloc(reinterpret_cast<void**>(&Y), vb) == hipSuccess && hipMemsetAsync(X, 0, vb, s) == hipSuccess) {
      float best = 1e30f;
      int best_s = h->sched[prec];
      for (int sc = 0; sc < 4 && rc == H2_OK; ++sc) {
        h->sched[prec] = sc;
        float t = 0.0f;
        for (int rep = 0; rep < 4 && rc == H2_OK; ++rep) {
          if (hipEventRecord(e0, s) != hipSuccess) { rc = H2_EHIP; break; }
          rc = gemv_ws(h, w, false, 1.0, X, h->n, nvp, 0.0, Y, h->n, prec, s);
          float ms = 0.0f;
          if (rc == H2_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = H2_EHIP;
          if (rep > 0) t += ms;
        }
        h->sched_ms[prec][sc] = t / 3;
        if (t < best * kScheduleGain) {
          best = t;
          best_s = sc;
        }
      }
      h->sched[prec] = best_s;
      if (rc == H2_EHIP) set_error("timing the dense schedules failed");
    }
    if (X) (void)hipFree(X);
    if (Y) (void)hipFree(Y);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == H2_OK) rc = drop_unused_fl(h);
  return rc;
}

int h2_tune_set(h2_handle h, int prec, int kc, int64_t grid, int xcd, int tree_order) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  if (prec != H2_PREC_FP64 && prec != H2_PREC_FP32 && prec != H2_PREC_BF16) {
    set_error("unknown precision");
    return H2_EINVAL;
  }
  if (!(kc >= 0 && kc <= kWaveTiles + 2) && kc != 32 && kc != 64) {
    set_error("kc must be 0-12, 32 or 64");
    return H2_EINVAL;
  }
  // 11, 12: the wave-row forms compiled for five waves per SIMD
  const int occ = kc == kWaveTiles + 1 || kc == kWaveTiles + 2 ? 5 : 0;
  if (occ) kc -= 2;
  if (prec == H2_PREC_BF16 && kc != 64) { set_error("the BF16 kernel has kc 64 only"); return H2_EINVAL; }
  if (grid < 0) { set_error("grid < 0"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);
  Plan& P = h->planN;
  for (auto* v : {&P.up, &P.couple, &P.down, &P.couple_loc, &P.couple_deep, &P.couple_rest})
    for (Launch& L : *v) {
      L.kcp[prec] = kc;
      L.gridp[prec] = grid;
      L.remapp[prec] = xcd ? 1 : 0;
      L.flp[prec] = 1;
      L.occp[prec] = occ;
    }
  P.out.kcp[prec] = kc;
  P.out.gridp[prec] = grid;
  P.out.remapp[prec] = xcd ? 1 : 0;
  P.out.flp[prec] = 1;
  P.out.occp[prec] = occ;
  if (prec == H2_PREC_FP64 || kc != 0)  // the dense rows are always FP64
    for (auto* v : {&P.dense, &P.dense2, &P.dense_loc, &P.dense2_loc})
      for (Launch& L : *v) {
        L.kcp[H2_PREC_FP64] = prec == H2_PREC_BF16 ? 64 : kc;
        L.gridp[H2_PREC_FP64] = grid;
        L.remapp[H2_PREC_FP64] = xcd ? 1 : 0;
        L.flp[H2_PREC_FP64] = 1;
        L.occp[H2_PREC_FP64] = occ;
      }
  h->couple_mode[prec] = tree_order != 0 ? 1 : 0;
  h->dense_mode[prec] = tree_order != 0 ? 1 : 0;
  return H2_OK;
}

int h2_set_dense_grid(h2_handle h, int64_t workgroups) {
  if (!h || workgroups < -1) { set_error("bad handle or workgroups"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);
  h->dense_grid_mv = workgroups;
  return H2_OK;
}

int h2_set_schedule(h2_handle h, int prec, int schedule) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  if (prec != H2_PREC_FP64 && prec != H2_PREC_FP32 && prec != H2_PREC_BF16) {
    set_error("unknown precision");
    return H2_EINVAL;
  }
  if (schedule < 0 || schedule > 3) { set_error("schedule must be 0-3"); return H2_EINVAL; }
  DeviceGuard guard(h->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);
  h->sched[prec] = schedule;
  h->sched1[prec] = schedule;
  return H2_OK;
}

int h2_set_sweeps(h2_handle h, int prec, int fused) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  if (prec != H2_PREC_FP64 && prec != H2_PREC_FP32) { set_error("sweeps are chosen for FP64 and FP32"); return H2_EINVAL; }
  if (fused && !h->tree_ok) {
    set_error("this operator has rows that the fused sweeps do not take (more than 64 outputs)");
    return H2_EUNSUPPORTED;
  }
  DeviceGuard guard(h->device);
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);
  h->sweep_fused[prec] = fused ? 1 : 0;
  return H2_OK;
}

int h2_set_fragment_order(h2_handle h, int prec, int enable) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  if (prec != H2_PREC_FP64 && prec != H2_PREC_FP32) {
    set_error("the fragment-ordered copies exist for FP64 and FP32");
    return H2_EINVAL;
  }
  DeviceGuard guard(h->device);
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  drop_graphs(h);
  int rc;
  if (enable) {
    if ((rc = h2_prepare(h, prec)) != H2_OK || (rc = prepare_fl(h, prec)) != H2_OK) return rc;
  }
  Plan& P = h->planN;
  for (auto* v : {&P.up, &P.couple, &P.down, &P.couple_loc, &P.couple_deep, &P.couple_rest})
    for (Launch& L : *v) L.flp[prec] = enable ? 1 : 0;
  P.out.flp[prec] = enable ? 1 : 0;
  for (auto* v : {&P.dense, &P.dense2, &P.dense_loc, &P.dense2_loc})  // always FP64
    for (Launch& L : *v) L.flp[H2_PREC_FP64] = enable ? 1 : 0;
  return enable ? H2_OK : drop_unused_fl(h);
}

int h2_plan_info(h2_handle h, char* buf, size_t cap, size_t* needed) {
  if (!h || !needed) { set_error("null handle or size output"); return H2_EINVAL; }
  std::string t;
  char line[256];
  const char* pn[3] = {"fp64", "fp32", "bf16"};
  std::snprintf(line, sizeof line, "first level with coupling blocks: %lld (sweep transfers above it skipped)\n",
                (long long)h->lmin);
  t += line;
  for (int p = 0; p < 3; ++p) {
    const char* cmn[2] = {"longest first", "tree order"};
    std::snprintf(line, sizeof line, "%s: coupling rows %s, dense rows %s\n", pn[p], cmn[h->couple_mode[p]],
                  cmn[h->dense_mode[p]]);
    t += line;
  }
  auto dump = [&](const char* phase, const std::vector<Launch>& v) {
    for (const Launch& L : v) {
      std::snprintf(line, sizeof line, "%s rows=%lld max_rows=%d kind=%d", phase, (long long)L.row_count, L.max_rows,
                    L.kind);
      t += line;
      for (int p = 0; p < 3; ++p) {
        std::snprintf(line, sizeof line, " | %s kc=%d grid=%lld xcd=%d fl=%d occ=%d %.3fms", pn[p], L.kcp[p],
                      (long long)L.gridp[p], L.remapp[p], L.flp[p], L.occp[p], L.tuned_ms[p]);
        t += line;
      }
      if (skipped(h, L)) t += " | skipped (above the first coupling level)";
      t += "\n";
    }
  };
  for (int p = 0; p < 2; ++p) {
    std::snprintf(line, sizeof line, "%s: sweeps %s (per-level %.3fms, fused %.3fms when tuned)\n", pn[p],
                  h->tree_ok && h->sweep_fused[p] ? "fused" : "per level", h->sweep_ms[p][0], h->sweep_ms[p][1]);
    t += line;
  }
  for (int p = 0; p < 3; ++p) {
    std::snprintf(line, sizeof line, "%s: dense schedule %d (tuned products %.3f / %.3f / %.3f / %.3f ms)\n",
                  pn[p], h->sched[p], h->sched_ms[p][0], h->sched_ms[p][1], h->sched_ms[p][2], h->sched_ms[p][3]);
    t += line;
    std::snprintf(line, sizeof line,
                  "%s: streaming dense schedule %d (tuned products %.3f / %.3f / %.3f / %.3f ms)\n", pn[p],
                  h->sched1[p], h->sched1_ms[p][0], h->sched1_ms[p][1], h->sched1_ms[p][2], h->sched1_ms[p][3]);
    t += line;
  }
  for (const auto* v : {&h->tree_up, &h->tree_down})
    for (const TreeGroup& G : *v) {
      std::snprintf(line, sizeof line, "%s tree workgroups=%lld levels=%d max_rows=%d\n",
                    v == &h->tree_up ? "up" : "down", (long long)G.nwg, G.lv.nlev, G.max_rows);
      t += line;
    }
  const Plan& P = h->planN;
  dump("up", P.up);
  dump("couple", P.couple);
  dump("couple_deep", P.couple_deep);
  dump("couple_rest", P.couple_rest);
  dump("couple_tree", P.couple_loc);
  dump("down", P.down);
  dump("dense1", P.dense);
  dump("dense2", P.dense2);
  dump("dense1_tree", P.dense_loc);
  dump("dense2_tree", P.dense2_loc);
  dump("out", std::vector<Launch>{P.out});
  *needed = t.size() + 1;
  if (buf && cap > 0) {
    const size_t c = std::min(cap - 1, t.size());
    std::memcpy(buf, t.data(), c);
    buf[c] = 0;
  }
  return H2_OK;
}

int h2_stats(h2_handle h, h2_stats_t* st) {
  if (!h || !st) { set_error("null handle or output"); return H2_EINVAL; }
  *st = h->stats;
  return H2_OK;
}

int h2_level_stats(h2_handle h, int64_t level, h2_level_stats_t* out) {
  if (!h || !out) { set_error("null handle or output"); return H2_EINVAL; }
  if (level < 0 || level >= (int64_t)h->level_stats.size()) { set_error("level out of range"); return H2_EINVAL; }
  *out = h->level_stats[level];
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
    HIP_TRY(hipEventSynchronize(e[8]), "hipEventSynchronize");
    HIP_TRY(hipEventSynchronize(e[6]), "hipEventSynchronize");
    float t[9];
    const int from[9] = {0, 1, 2, 3, 5, 7, 0, 10, 11}, to[9] = {1, 2, 3, 4, 9, 8, 8, 6, 12};
    for (int k = 0; k < 9; ++k) HIP_TRY(hipEventElapsedTime(&t[k], e[from[k]], e[to[k]]), "hipEventElapsedTime");
    h->prof.ms_permute += t[0];
    h->prof.ms_upsweep += t[1];
    h->prof.ms_coupling += t[2] + t[8];
    h->prof.ms_downsweep += t[3];
    h->prof.ms_dense += t[4] + t[7];
    h->prof.ms_leaf_out += t[5];
    h->prof.ms_total += t[6];
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
