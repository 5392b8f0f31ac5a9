// Launch-plan construction shared by the single-operator handle and the
// multi-operator batch: the per-operator layout (vector-tree offsets,
// section offsets, transposed basis copies) and the rows of every op-'N'
// phase, each row a block row whose stored blocks are contiguous.
//
// The paper marshals, per call and per level, pointer arrays for batched
// kernels (Algorithm 3, Section 3.1).  The structure is static, so here the
// same information is produced once, at load time, as row lists.
#include <algorithm>
#include <vector>

#include "h2_internal.h"

namespace h2 {

int make_layout(const Parsed& P, OpLayout* L) {
  const int64_t q = P.q, n = P.n;
  const int64_t* lp = P.level_ptr;
  L->P = &P;
  L->shared = !(P.flags & 1u);
  L->kmax.assign(q + 1, 0);
  for (int64_t l = 0; l <= q; ++l) L->kmax[l] = std::max(P.krow[l], P.kcol[l]);
  const int64_t mat0 = P.off_U;
  L->oU = 0;
  L->oE = (P.off_E - mat0) / 8;
  L->oV = L->shared ? L->oU : (P.off_V - mat0) / 8;
  L->oF = L->shared ? L->oE : (P.off_F - mat0) / 8;
  L->oS = (P.off_S - mat0) / 8;
  L->oD = (P.off_D - mat0) / 8;
  L->nmat = (P.off_end - mat0) / 8;
  auto up32 = [](int64_t x) { return (x + 31) / 32 * 32; };
  const int64_t nU = n * P.krow[q], nE = P.ebase[q + 1], nV = n * P.kcol[q], nF = P.fbase[q + 1];
  L->tUT = 0;
  L->tET = up32(nU);
  L->tVT = L->shared ? L->tUT : up32(L->tET + nE);
  L->tFT = L->shared ? L->tET : up32(L->tVT + nV);
  L->ntrans = L->shared ? up32(L->tET + nE) : up32(L->tFT + nF);
  L->hoff.assign(P.nnodes, 0);
  int64_t H = 0;
  for (int64_t l = 0; l <= q; ++l)
    for (int64_t c = lp[l]; c < lp[l + 1]; ++c) {
      L->hoff[c] = H;
      H += L->kmax[l];
    }
  L->H = H;
  L->cbeg.assign(P.nnodes + 1, P.nnodes);
  int64_t next = 1;
  for (int64_t p = 0; p < P.nnodes; ++p) {
    L->cbeg[p] = next;
    while (next < P.nnodes && P.parent[next] == p) ++next;
    if (next - L->cbeg[p] > kMaxChildren) {
      set_error("h2 representation: node with more than 512 children");
      return H2_EUNSUPPORTED;
    }
  }
  L->cbeg[P.nnodes] = next;
  return H2_OK;
}

int64_t OpLayout::eoff(int64_t c, int64_t l) const {
  return P->ebase[l] + (c - P->level_ptr[l]) * P->krow[l] * P->krow[l - 1];
}
int64_t OpLayout::foff(int64_t c, int64_t l) const {
  return P->fbase[l] + (c - P->level_ptr[l]) * P->kcol[l] * P->kcol[l - 1];
}

void transpose_tasks(const OpLayout& L, std::vector<TransTask>* out) {
  const Parsed& P = *L.P;
  const int64_t q = P.q;
  out->clear();
  for (int pass = 0; pass < (L.shared ? 1 : 2); ++pass) {
    const int64_t* k = pass ? P.kcol : P.krow;
    const int64_t ob = pass ? L.oV : L.oU, ot = pass ? L.oF : L.oE;
    const int64_t tb = pass ? L.tVT : L.tUT, tt = pass ? L.tFT : L.tET;
    for (int64_t t = P.leaf0; t < P.nnodes; ++t) {  // leaf basis: m x k
      const int64_t m = P.hi[t] - P.lo[t], base = P.lo[t] * k[q];
      out->push_back({ob + base, tb + base, (int32_t)m, (int32_t)k[q]});
    }
    for (int64_t l = 1; l <= q; ++l)
      for (int64_t c = P.level_ptr[l]; c < P.level_ptr[l + 1]; ++c) {  // transfer: k[l] x k[l-1]
        const int64_t base = pass ? L.foff(c, l) : L.eoff(c, l);
        out->push_back({ot + base, tt + base, (int32_t)k[l], (int32_t)k[l - 1]});
      }
  }
}

void build_transposed(const uint8_t* buf, const OpLayout& L, double* tr) {
  std::fill(tr, tr + L.ntrans, 0.0);
  const double* M = reinterpret_cast<const double*>(buf + L.P->off_U);  // the matrix array
  std::vector<TransTask> tasks;
  transpose_tasks(L, &tasks);
  for (const TransTask& T : tasks)
    for (int64_t c = 0; c < T.cols; ++c)
      for (int64_t r = 0; r < T.rows; ++r) tr[T.dst + c + T.cols * r] = M[T.src + r + T.rows * c];
}

void emit_rows_N(const OpLayout& L, const RowBases& B, RowsN* R) {
  const Parsed& P = *L.P;
  const int64_t q = P.q;
  const int64_t* lp = P.level_ptr;
  const int64_t* kc = P.kcol;
  const int64_t* kr = P.krow;
  auto msz = [&](int64_t c) { return (int32_t)(P.hi[c] - P.lo[c]); };
  const std::vector<int64_t>& hoff = L.hoff;
  R->up.assign(q + 1, {});
  R->down.assign(q, {});
  R->couple.clear();
  R->dense.clear();
  R->out.clear();
  // leaf products x^_t = V_t^T x~_t (transposed leaf basis, contiguous rows)
  for (int64_t t = P.leaf0; t < P.nnodes; ++t)
    R->up[0].push_back({B.trans + L.tVT + P.lo[t] * kc[q], B.xh + hoff[t], B.ld_h, B.ld_x, (int32_t)kc[q],
                        {BlockRef{0, B.xt + P.lo[t], msz(t), 0}}});
  // transfer level l (h = q - l + 1 from the leaves): x^_p = [F_c1^T F_c2^T ..] [x^_c1; x^_c2; ..]
  for (int64_t l = q; l >= 1; --l) {
    std::vector<RowSpec>& rows = R->up[q - l + 1];
    for (int64_t p = lp[l - 1]; p < lp[l]; ++p) {
      RowSpec r{B.trans + L.tFT + L.foff(L.cbeg[p], l), B.xh + hoff[p], B.ld_h, B.ld_h, (int32_t)kc[l - 1], {}};
      for (int64_t c = L.cbeg[p]; c < L.cbeg[p + 1]; ++c) r.blks.push_back({0, B.xh + hoff[c], (int32_t)kc[l], 0});
      rows.push_back(std::move(r));
    }
  }
  // coupling rows of every level (Algorithm 4)
  for (int64_t l = 0; l <= q; ++l) {
    const int64_t* rp = P.s_rowptr + P.rp_base[l];
    const int64_t nl = lp[l + 1] - lp[l], bsz = P.krow[l] * P.kcol[l];
    for (int64_t t = 0; t < nl; ++t) {
      RowSpec r{B.mat + L.oS + P.sdat[l] + rp[t] * bsz, B.yh + hoff[lp[l] + t], B.ld_h, B.ld_h,
                (int32_t)P.krow[l], {}};
      for (int64_t b = rp[t]; b < rp[t + 1]; ++b)
        r.blks.push_back({0, B.xh + hoff[lp[l] + P.s_col[P.blk_base[l] + b]], (int32_t)P.kcol[l], 0});
      R->couple.push_back(std::move(r));
    }
  }
  // transfer downsweep level l: y^_c += E_c y^_parent
  for (int64_t l = 1; l <= q; ++l)
    for (int64_t c = lp[l]; c < lp[l + 1]; ++c)
      R->down[l - 1].push_back({B.mat + L.oE + L.eoff(c, l), B.yh + hoff[c], B.ld_h, B.ld_h, (int32_t)kr[l],
                                {BlockRef{0, B.yh + hoff[P.parent[c]], (int32_t)kr[l - 1], 0}}});
  // dense leaf rows: Z_t = sum_s D_ts x~_s
  for (int64_t t = 0; t < P.nleaves; ++t) {
    RowSpec r{B.mat + L.oD + P.ddat[P.d_rowptr[t]], B.zn + P.lo[P.leaf0 + t], B.ld_x, B.ld_x, msz(P.leaf0 + t), {}};
    for (int64_t b = P.d_rowptr[t]; b < P.d_rowptr[t + 1]; ++b)
      r.blks.push_back({0, B.xt + P.lo[P.leaf0 + P.d_col[b]], msz(P.leaf0 + P.d_col[b]), 0});
    R->dense.push_back(std::move(r));
  }
  // leaf expansion U_t y^_t (the caller picks the epilogue)
  for (int64_t t = P.leaf0; t < P.nnodes; ++t)
    R->out.push_back({B.mat + L.oU + P.lo[t] * kr[q], B.zn + P.lo[t], B.ld_x, B.ld_h, msz(t),
                      {BlockRef{0, B.yh + hoff[t], (int32_t)kr[q], 0}}});
}

void append_row(RowTables& t, const RowSpec& r) {
  RowDesc R{};
  R.data_off = r.data_off;
  R.out_off = r.out_off;
  R.nrows = r.nrows;
  R.blk_begin = (int32_t)t.colend.size();
  int32_t col = 0;
  for (const BlockRef& b : r.blks) {
    col += b.width;
    t.colend.push_back(col);
    t.in_off.push_back(b.in_off);
  }
  R.blk_end = (int32_t)t.colend.size();
  R.out_ld = r.out_ld;
  R.in_ld = r.in_ld;
  t.rows.push_back(R);
}

void place_fl(RowTables& t, int64_t begin, int64_t end, int arr, FlKeys* keys, int64_t* n_fl) {
  for (int64_t i = begin; i < end; ++i) {
    RowDesc& R = t.rows[i];
    const int32_t ncols = R.blk_end > R.blk_begin ? t.colend[R.blk_end - 1] : 0;
    const int64_t size = ((int64_t)R.nrows * ncols + 1) / 2 * 2;
    const auto ins = keys->emplace(2 * R.data_off + arr, FlRegion{*n_fl, R.nrows, ncols});
    if (!ins.second && (ins.first->second.nrows != R.nrows || ins.first->second.ncols != ncols)) {
      R.fl_off = *n_fl;  // the same offset with another shape: a region of its own
      *n_fl += size;
      continue;
    }
    R.fl_off = ins.first->second.fl_off;
    if (ins.second) *n_fl += size;
  }
}

int64_t row_work(const RowSpec& r) {
  int64_t c = 0;
  for (const BlockRef& b : r.blks) c += b.width;
  return c * r.nrows;
}

}  // namespace h2
