/*
 * h2_oracle.c -- reference H^2 matrix-vector product on the CPU, in FP64.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this code.  The GPU library never links
 * it, and the two share no code: this file has its own reader of the
 * serialized representation and its own arithmetic, in plain loops.
 *
 * What it computes is the plain definition of the product with an H^2 matrix
 * (Section 2.1 of the paper, "Hierarchy of Blocks" / "Hierarchy of Bases"):
 *
 *     A = A_de + sum over levels l, over coupling blocks (t,s) of level l,
 *                of  Uhat_t S_ts Vhat_s^T,
 *
 * where the explicit basis of an inner node is given by the nested-basis
 * identity  Uhat_parent = [Uhat_c1 E_c1 ; Uhat_c2 E_c2 ; ...]  (rows stacked in
 * child order; Section 2.1, the equation for U^{l-1}_i), and Vhat likewise
 * with the transfers F.  The matrix acts in original point order through the
 * permutation stored with the representation (tree position i holds original
 * index perm[i]; sub-vectors are taken in tree order, Section 3).
 *
 *   op 'N':  Y <- alpha * A   X + beta * Y
 *   op 'T':  Y <- alpha * A^T X + beta * Y      (BLAS semantics; beta == 0
 *                                                means Y is not read)
 *
 * Evaluation order: every coupling block contributes Uhat_t (S_ts (Vhat_s^T x_s))
 * where the rows of Uhat_t and Vhat_s are formed explicitly by the nested
 * recursion above, one row chain per leaf; Vhat_s^T x_s is summed leaf by leaf
 * in tree order.  There is no transfer recursion applied to vectors (that is
 * the fast algorithm of Sections 3.1-3.3, which the oracle is meant to check).
 *
 * With absval != 0 every stored entry, every input entry, alpha and beta are
 * replaced by their absolute values.  The result bounds the magnitude of every
 * partial sum of any evaluation order of the product, which is the scale used
 * for elementwise rounding tolerances.
 *
 * Parallelism: OpenMP only over independent leaves or nodes; every output
 * entry is summed sequentially in a fixed order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define H2O_OK 0
#define H2O_EINVAL (-1)
#define H2O_EFORMAT (-3)
#define H2O_ENOMEM (-4)

typedef struct h2o_rep {
  int64_t n, q, nnodes, nleaves, leaf0, ndense, dim;
  uint32_t flags;
  const int64_t *level_ptr, *krow, *kcol, *nadm, *perm, *lo, *hi, *parent;
  const int64_t *s_rowptr, *s_col, *d_rowptr, *d_col;
  const double *U, *E, *V, *F, *S, *D, *points;
  /* derived, owned */
  int64_t *level_of;  /* level of each node */
  int64_t *rp_base;   /* per level: index of its first entry in s_rowptr */
  int64_t *blk_base;  /* per level: global index of its first coupling block */
  int64_t *sdat;      /* per level: offset in S of its first block */
  int64_t *ebase;     /* per level: offset in E of node level_ptr[l] */
  int64_t *fbase;     /* per level: offset in F of node level_ptr[l] */
  int64_t *ddat;      /* per dense block: offset in D (ndense+1 entries) */
  int64_t *leaf_at;   /* tree position -> leaf index */
  int64_t *leafbeg, *leafend; /* per node: leaf index range below it */
  int64_t *blk_row;   /* per coupling block: row node (global id) */
  int64_t *blk_colg;  /* per coupling block: column node (global id) */
  int64_t *sc_ptr, *sc_blk; /* per node: coupling blocks whose column is that node */
  int64_t *drow;      /* per dense block: row leaf index */
  int64_t *dc_ptr, *dc_blk; /* per leaf: dense blocks whose column is that leaf */
} h2o_rep;

/* ------------------------------------------------------------------------ */
/* reader                                                                   */
/* ------------------------------------------------------------------------ */

static int64_t al64(int64_t x) { return (x + 63) / 64 * 64; }

static int64_t rd_i64(const uint8_t* p) { int64_t v; memcpy(&v, p, 8); return v; }
static double rd_f64(const uint8_t* p) { double v; memcpy(&v, p, 8); return v; }

void h2o_close(h2o_rep* r) {
  if (!r) return;
  free(r->level_of); free(r->rp_base); free(r->blk_base); free(r->sdat);
  free(r->ebase); free(r->fbase); free(r->ddat); free(r->leaf_at);
  free(r->leafbeg); free(r->leafend); free(r->blk_row); free(r->blk_colg);
  free(r->sc_ptr); free(r->sc_blk); free(r->drow); free(r->dc_ptr); free(r->dc_blk);
  free(r);
}

/* Parse and validate a serialized representation held in memory.  The buffer
 * must outlive the returned object (arrays point into it) and be 8-byte
 * aligned.  Returns 0, H2O_EFORMAT or H2O_ENOMEM. */
int h2o_open(const uint8_t* buf, int64_t len, h2o_rep** out) {
  if (!buf || !out || len < 128 || ((uintptr_t)buf & 7)) return H2O_EINVAL;
  *out = NULL;
  if (memcmp(buf, "H2MATV01", 8) != 0) return H2O_EFORMAT;
  uint32_t version, flags;
  memcpy(&version, buf + 8, 4);
  memcpy(&flags, buf + 12, 4);
  if (version != 1 || (flags & ~3u)) return H2O_EFORMAT;
  const int64_t n = rd_i64(buf + 16), q = rd_i64(buf + 24), nnodes = rd_i64(buf + 32);
  const int64_t dim = rd_i64(buf + 40), ndense = rd_i64(buf + 88), total = rd_i64(buf + 96);
  (void)rd_f64;
  if (n < 1 || q < 0 || q > 62 || nnodes < 1 || dim < 0 || ndense < 0 || total != len) return H2O_EFORMAT;
  if (!(flags & 2u) && dim != 0) return H2O_EFORMAT;
  h2o_rep* r = (h2o_rep*)calloc(1, sizeof(h2o_rep));
  if (!r) return H2O_ENOMEM;
  r->n = n; r->q = q; r->nnodes = nnodes; r->ndense = ndense; r->dim = dim; r->flags = flags;

  int64_t pos = 128;
  int rc = H2O_EFORMAT;
#define TAKE(ptr, type, count)                                             \
  do {                                                                     \
    int64_t c_ = (count);                                                  \
    pos = al64(pos);                                                       \
    if (c_ < 0 || c_ > (len - pos) / 8) goto fail;                         \
    ptr = (const type*)(buf + pos);                                        \
    pos += 8 * c_;                                                         \
  } while (0)

  TAKE(r->level_ptr, int64_t, q + 2);
  TAKE(r->krow, int64_t, q + 1);
  TAKE(r->kcol, int64_t, q + 1);
  TAKE(r->nadm, int64_t, q + 1);
  TAKE(r->perm, int64_t, n);
  TAKE(r->lo, int64_t, nnodes);
  TAKE(r->hi, int64_t, nnodes);
  TAKE(r->parent, int64_t, nnodes);
  const int64_t* lp = r->level_ptr;
  if (lp[0] != 0 || lp[q + 1] != nnodes || (nnodes >= 1 && q >= 0 && lp[1] != 1)) goto fail;
  for (int64_t l = 0; l <= q; ++l)
    if (lp[l + 1] <= lp[l]) goto fail;
  int64_t nadm_tot = 0;
  for (int64_t l = 0; l <= q; ++l) {
    if (r->krow[l] < 0 || r->kcol[l] < 0 || r->nadm[l] < 0) goto fail;
    if (r->krow[l] > 4096 || r->kcol[l] > 4096) goto fail;
    if (!(flags & 1u) && r->krow[l] != r->kcol[l]) goto fail;
    nadm_tot += r->nadm[l];
    if (nadm_tot > ((int64_t)1 << 40)) goto fail;
  }
  r->leaf0 = lp[q];
  r->nleaves = nnodes - lp[q];
  TAKE(r->s_rowptr, int64_t, nnodes + q + 1);
  TAKE(r->s_col, int64_t, nadm_tot);
  TAKE(r->d_rowptr, int64_t, r->nleaves + 1);
  TAKE(r->d_col, int64_t, ndense);

  /* permutation */
  {
    uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
    if (!seen) { rc = H2O_ENOMEM; goto fail; }
    int ok = 1;
    for (int64_t i = 0; i < n && ok; ++i) {
      int64_t p = r->perm[i];
      if (p < 0 || p >= n || seen[p]) ok = 0; else seen[p] = 1;
    }
    free(seen);
    if (!ok) goto fail;
  }
  /* tree: root covers [0,n); children of each parent are consecutive, in
   * parent order, and tile the parent's range; every non-leaf has a child */
  if (r->lo[0] != 0 || r->hi[0] != n || r->parent[0] != -1) goto fail;
  r->level_of = (int64_t*)malloc(sizeof(int64_t) * nnodes);
  if (!r->level_of) { rc = H2O_ENOMEM; goto fail; }
  r->level_of[0] = 0;
  for (int64_t l = 1; l <= q; ++l) {
    int64_t prev_par = lp[l - 1] - 1;
    for (int64_t c = lp[l]; c < lp[l + 1]; ++c) {
      int64_t p = r->parent[c];
      r->level_of[c] = l;
      if (r->lo[c] > r->hi[c]) goto fail;
      if (p == prev_par) {
        if (r->lo[c] != r->hi[c - 1]) goto fail;
      } else {
        if (p != prev_par + 1) goto fail;           /* no parent skipped */
        if (prev_par >= lp[l - 1] && r->hi[c - 1] != r->hi[prev_par]) goto fail;
        if (r->lo[c] != r->lo[p]) goto fail;
        prev_par = p;
      }
    }
    if (prev_par != lp[l] - 1) goto fail;           /* last parent reached */
    if (r->hi[lp[l + 1] - 1] != r->hi[prev_par]) goto fail;
  }
  /* coupling CSR per level */
  r->rp_base = (int64_t*)malloc(sizeof(int64_t) * (q + 1));
  r->blk_base = (int64_t*)malloc(sizeof(int64_t) * (q + 2));
  r->sdat = (int64_t*)malloc(sizeof(int64_t) * (q + 2));
  if (!r->rp_base || !r->blk_base || !r->sdat) { rc = H2O_ENOMEM; goto fail; }
  {
    int64_t rb = 0, bb = 0, sd = 0;
    for (int64_t l = 0; l <= q; ++l) {
      const int64_t nl = lp[l + 1] - lp[l];
      const int64_t* rp = r->s_rowptr + rb;
      r->rp_base[l] = rb; r->blk_base[l] = bb; r->sdat[l] = sd;
      if (rp[0] != 0 || rp[nl] != r->nadm[l]) goto fail;
      for (int64_t t = 0; t < nl; ++t) {
        if (rp[t + 1] < rp[t]) goto fail;
        for (int64_t b = rp[t]; b < rp[t + 1]; ++b) {
          int64_t s = r->s_col[bb + b];
          if (s < 0 || s >= nl) goto fail;
          if (b > rp[t] && s <= r->s_col[bb + b - 1]) goto fail;
        }
      }
      rb += nl + 1; bb += r->nadm[l]; sd += r->nadm[l] * r->krow[l] * r->kcol[l];
    }
    r->blk_base[q + 1] = bb; r->sdat[q + 1] = sd;
  }
  /* dense CSR over leaves */
  r->ddat = (int64_t*)malloc(sizeof(int64_t) * (ndense + 1));
  if (!r->ddat) { rc = H2O_ENOMEM; goto fail; }
  {
    const int64_t* rp = r->d_rowptr;
    if (rp[0] != 0 || rp[r->nleaves] != ndense) goto fail;
    r->ddat[0] = 0;
    for (int64_t t = 0; t < r->nleaves; ++t) {
      if (rp[t + 1] < rp[t]) goto fail;
      for (int64_t b = rp[t]; b < rp[t + 1]; ++b) {
        int64_t s = r->d_col[b];
        if (s < 0 || s >= r->nleaves) goto fail;
        if (b > rp[t] && s <= r->d_col[b - 1]) goto fail;
        int64_t mt = r->hi[r->leaf0 + t] - r->lo[r->leaf0 + t];
        int64_t ms = r->hi[r->leaf0 + s] - r->lo[r->leaf0 + s];
        if (mt > ((int64_t)1 << 31) || ms > ((int64_t)1 << 31)) goto fail;
        r->ddat[b + 1] = r->ddat[b] + mt * ms;
        if (r->ddat[b + 1] > len / 8) goto fail;
      }
    }
  }
  /* transfer offsets */
  r->ebase = (int64_t*)calloc((size_t)(q + 2), sizeof(int64_t));
  r->fbase = (int64_t*)calloc((size_t)(q + 2), sizeof(int64_t));
  if (!r->ebase || !r->fbase) { rc = H2O_ENOMEM; goto fail; }
  for (int64_t l = 1; l <= q; ++l) {
    int64_t nl = lp[l + 1] - lp[l];
    r->ebase[l + 1] = r->ebase[l] + nl * r->krow[l] * r->krow[l - 1];
    r->fbase[l + 1] = r->fbase[l] + nl * r->kcol[l] * r->kcol[l - 1];
  }
  {
    const int sep = (flags & 1u) != 0;
    TAKE(r->U, double, n * r->krow[q]);
    TAKE(r->E, double, r->ebase[q + 1]);
    if (sep) {
      TAKE(r->V, double, n * r->kcol[q]);
      TAKE(r->F, double, r->fbase[q + 1]);
    } else {
      TAKE(r->V, double, 0);
      TAKE(r->F, double, 0);
      r->V = r->U; r->F = r->E;
    }
    TAKE(r->S, double, r->sdat[q + 1]);
    TAKE(r->D, double, r->ddat[ndense]);
    TAKE(r->points, double, (flags & 2u) ? n * dim : 0);
    if (al64(pos) != len) goto fail;
  }
  /* derived maps */
  r->leaf_at = (int64_t*)malloc(sizeof(int64_t) * n);
  r->leafbeg = (int64_t*)malloc(sizeof(int64_t) * nnodes);
  r->leafend = (int64_t*)malloc(sizeof(int64_t) * nnodes);
  r->blk_row = (int64_t*)malloc(sizeof(int64_t) * (nadm_tot + 1));
  r->blk_colg = (int64_t*)malloc(sizeof(int64_t) * (nadm_tot + 1));
  r->sc_ptr = (int64_t*)calloc((size_t)(nnodes + 1), sizeof(int64_t));
  r->sc_blk = (int64_t*)malloc(sizeof(int64_t) * (nadm_tot + 1));
  r->drow = (int64_t*)malloc(sizeof(int64_t) * (ndense + 1));
  r->dc_ptr = (int64_t*)calloc((size_t)(r->nleaves + 1), sizeof(int64_t));
  r->dc_blk = (int64_t*)malloc(sizeof(int64_t) * (ndense + 1));
  if (!r->leaf_at || !r->leafbeg || !r->leafend || !r->blk_row || !r->blk_colg || !r->sc_ptr ||
      !r->sc_blk || !r->drow || !r->dc_ptr || !r->dc_blk) { rc = H2O_ENOMEM; goto fail; }
  for (int64_t j = 0; j < r->nleaves; ++j) {
    int64_t t = r->leaf0 + j;
    for (int64_t i = r->lo[t]; i < r->hi[t]; ++i) r->leaf_at[i] = j;
    r->leafbeg[t] = j; r->leafend[t] = j + 1;
  }
  for (int64_t l = q - 1; l >= 0; --l)
    for (int64_t t = lp[l]; t < lp[l + 1]; ++t) { r->leafbeg[t] = INT64_MAX; r->leafend[t] = -1; }
  for (int64_t c = nnodes - 1; c >= 1; --c) {
    int64_t p = r->parent[c];
    if (r->leafbeg[c] < r->leafbeg[p]) r->leafbeg[p] = r->leafbeg[c];
    if (r->leafend[c] > r->leafend[p]) r->leafend[p] = r->leafend[c];
  }
  for (int64_t l = 0; l <= q; ++l) {
    const int64_t* rp = r->s_rowptr + r->rp_base[l];
    for (int64_t t = 0; t < lp[l + 1] - lp[l]; ++t)
      for (int64_t b = rp[t]; b < rp[t + 1]; ++b) {
        int64_t g = r->blk_base[l] + b;
        r->blk_row[g] = lp[l] + t;
        r->blk_colg[g] = lp[l] + r->s_col[g];
        r->sc_ptr[r->blk_colg[g] + 1]++;
      }
  }
  for (int64_t c = 0; c < nnodes; ++c) r->sc_ptr[c + 1] += r->sc_ptr[c];
  {
    int64_t* fill = (int64_t*)calloc((size_t)nnodes, sizeof(int64_t));
    if (!fill) { rc = H2O_ENOMEM; goto fail; }
    for (int64_t g = 0; g < nadm_tot; ++g) {  /* increasing g: rows in order */
      int64_t c = r->blk_colg[g];
      r->sc_blk[r->sc_ptr[c] + fill[c]++] = g;
    }
    free(fill);
  }
  for (int64_t t = 0; t < r->nleaves; ++t)
    for (int64_t b = r->d_rowptr[t]; b < r->d_rowptr[t + 1]; ++b) {
      r->drow[b] = t;
      r->dc_ptr[r->d_col[b] + 1]++;
    }
  for (int64_t s = 0; s < r->nleaves; ++s) r->dc_ptr[s + 1] += r->dc_ptr[s];
  {
    int64_t* fill = (int64_t*)calloc((size_t)r->nleaves + 1, sizeof(int64_t));
    if (!fill) { rc = H2O_ENOMEM; goto fail; }
    for (int64_t b = 0; b < ndense; ++b) {
      int64_t s = r->d_col[b];
      r->dc_blk[r->dc_ptr[s] + fill[s]++] = b;
    }
    free(fill);
  }
#undef TAKE
  *out = r;
  return H2O_OK;
fail:
  h2o_close(r);
  return rc;
}

int64_t h2o_n(const h2o_rep* r) { return r ? r->n : -1; }

/* Threads the oracle's parallel loops use. */
int h2o_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the threads of later parallel loops (t >= 1; a serial build ignores it). */
void h2o_set_threads(int t) {
#ifdef _OPENMP
  if (t >= 1) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* the product                                                              */
/* ------------------------------------------------------------------------ */

/* The two bases seen from the operator being applied: the output ("row")
 * basis and the input ("column") basis.  For op 'T' the roles swap, and the
 * coupling and dense blocks are read transposed. */
typedef struct {
  const double *Brow, *Trow, *Bcol, *Tcol;
  const int64_t *krow, *kcol, *tbrow, *tbcol;
  int trans;
} view_t;

static view_t make_view(const h2o_rep* r, int trans) {
  view_t w;
  w.trans = trans;
  if (!trans) {
    w.Brow = r->U; w.Trow = r->E; w.krow = r->krow; w.tbrow = r->ebase;
    w.Bcol = r->V; w.Tcol = r->F; w.kcol = r->kcol; w.tbcol = r->fbase;
  } else {
    w.Brow = r->V; w.Trow = r->F; w.krow = r->kcol; w.tbrow = r->fbase;
    w.Bcol = r->U; w.Tcol = r->E; w.kcol = r->krow; w.tbcol = r->ebase;
  }
  return w;
}

static inline double A(double v, int absval) { return absval ? fabs(v) : v; }

/* Rows of the explicit basis of every ancestor of leaf j, by the nested
 * recursion: W_q = B_leaf (m x k_q); W_{l-1} = W_l * T_{anc_l} (m x k_{l-1}).
 * chain[l] receives W_l (column-major m x k_l); returns 0 or -1 (no memory). */
static void leaf_chain(const h2o_rep* r, const double* B, const double* T, const int64_t* k,
                       const int64_t* tb, int64_t j, double** chain, int absval) {
  const int64_t q = r->q, t = r->leaf0 + j, m = r->hi[t] - r->lo[t];
  const double* Bt = B + r->lo[t] * k[q];
  for (int64_t a = 0; a < k[q]; ++a)
    for (int64_t i = 0; i < m; ++i) chain[q][i + m * a] = A(Bt[i + m * a], absval);
  int64_t c = t;
  for (int64_t l = q; l >= 1; --l) {
    /* T_c is k[l] x k[l-1], column-major, node c on level l */
    const double* Tc = T + tb[l] + (c - r->level_ptr[l]) * k[l] * k[l - 1];
    for (int64_t b = 0; b < k[l - 1]; ++b)
      for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t a = 0; a < k[l]; ++a) s += chain[l][i + m * a] * A(Tc[a + k[l] * b], absval);
        chain[l - 1][i + m * b] = s;
      }
    c = r->parent[c];
  }
}

/* Core: xh_s = Vhat_s^T xt_s for every node s; yh_t = sum_s S_ts xh_s for the
 * nodes with need_node[t]; Z rows of the leaves with need_leaf[j].
 * xt: tree-ordered input, n x nv column-major.  Z: n x nv (only needed leaves
 * written). */
static int core(const h2o_rep* r, int trans, const double* xt, int64_t nv, const uint8_t* need_node,
                const uint8_t* need_leaf, double* Z, int absval) {
  const int64_t q = r->q, nn = r->nnodes, nl = r->nleaves;
  const view_t w = make_view(r, trans);
  int64_t kmax = 0, mmax = 0;
  for (int64_t l = 0; l <= q; ++l) {
    if (w.krow[l] > kmax) kmax = w.krow[l];
    if (w.kcol[l] > kmax) kmax = w.kcol[l];
  }
  for (int64_t j = 0; j < nl; ++j) {
    int64_t m = r->hi[r->leaf0 + j] - r->lo[r->leaf0 + j];
    if (m > mmax) mmax = m;
  }
  /* per-leaf, per-level contributions Vhat_anc[rows of leaf]^T xt[rows] */
  int64_t* cbase = (int64_t*)malloc(sizeof(int64_t) * (q + 2));
  int64_t* xoff = (int64_t*)malloc(sizeof(int64_t) * (nn + 1));
  int64_t* yoff = (int64_t*)malloc(sizeof(int64_t) * (nn + 1));
  if (!cbase || !xoff || !yoff) { free(cbase); free(xoff); free(yoff); return H2O_ENOMEM; }
  cbase[0] = 0;
  for (int64_t l = 0; l <= q; ++l) cbase[l + 1] = cbase[l] + nl * w.kcol[l] * nv;
  xoff[0] = 0; yoff[0] = 0;
  for (int64_t c = 0; c < nn; ++c) {
    xoff[c + 1] = xoff[c] + w.kcol[r->level_of[c]] * nv;
    yoff[c + 1] = yoff[c] + w.krow[r->level_of[c]] * nv;
  }
  double* contrib = (double*)calloc((size_t)(cbase[q + 1] + 1), sizeof(double));
  double* xh = (double*)calloc((size_t)(xoff[nn] + 1), sizeof(double));
  double* yh = (double*)calloc((size_t)(yoff[nn] + 1), sizeof(double));
  int rc = H2O_OK;
  if (!contrib || !xh || !yh) { rc = H2O_ENOMEM; goto done; }

#pragma omp parallel
  {
    double** chain = (double**)malloc(sizeof(double*) * (q + 1));
    double* store = (double*)malloc(sizeof(double) * (size_t)((q + 1) * (mmax * kmax + 1)));
    int ok = chain && store;
    if (ok)
      for (int64_t l = 0; l <= q; ++l) chain[l] = store + l * (mmax * kmax + 1);
#pragma omp for schedule(dynamic, 4)
    for (int64_t j = 0; j < nl; ++j) {
      if (!ok) continue;
      const int64_t t = r->leaf0 + j, m = r->hi[t] - r->lo[t];
      leaf_chain(r, w.Bcol, w.Tcol, w.kcol, w.tbcol, j, chain, absval);
      for (int64_t l = 0; l <= q; ++l) {
        const int64_t k = w.kcol[l];
        double* cj = contrib + cbase[l] + j * k * nv;
        for (int64_t v = 0; v < nv; ++v)
          for (int64_t a = 0; a < k; ++a) {
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += chain[l][i + m * a] * A(xt[r->lo[t] + i + r->n * v], absval);
            cj[a + k * v] = s;
          }
      }
    }
    free(chain);
    free(store);
    if (!ok) {
#pragma omp atomic write
      rc = H2O_ENOMEM;
    }
  }
  if (rc) goto done;

  /* xh_s = sum over the leaves below s, in tree order */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < nn; ++s) {
    const int64_t l = r->level_of[s], k = w.kcol[l];
    double* xs = xh + xoff[s];
    for (int64_t j = r->leafbeg[s]; j < r->leafend[s]; ++j) {
      const double* cj = contrib + cbase[l] + j * k * nv;
      for (int64_t e = 0; e < k * nv; ++e) xs[e] += cj[e];
    }
  }

  /* yh_t = sum over the blocks of row t (op 'N': CSR; op 'T': the blocks of
   * column t, transposed) */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nn; ++t) {
    if (!need_node[t]) continue;
    const int64_t l = r->level_of[t];
    const int64_t kr = w.krow[l], kc = w.kcol[l];
    double* yt = yh + yoff[t];
    int64_t bbeg, bend;
    if (!trans) {
      const int64_t* rp = r->s_rowptr + r->rp_base[l];
      bbeg = r->blk_base[l] + rp[t - r->level_ptr[l]];
      bend = r->blk_base[l] + rp[t - r->level_ptr[l] + 1];
    } else {
      bbeg = r->sc_ptr[t];
      bend = r->sc_ptr[t + 1];
    }
    for (int64_t bi = bbeg; bi < bend; ++bi) {
      const int64_t g = trans ? r->sc_blk[bi] : bi;
      const int64_t s = trans ? r->blk_row[g] : r->blk_colg[g];
      /* stored block is krow[l] x kcol[l] (untransposed sizes) */
      const double* Sg = r->S + r->sdat[l] + (g - r->blk_base[l]) * r->krow[l] * r->kcol[l];
      const double* xs = xh + xoff[s];
      for (int64_t v = 0; v < nv; ++v)
        for (int64_t a = 0; a < kr; ++a) {
          double acc = 0.0;
          for (int64_t b = 0; b < kc; ++b) {
            double sab = trans ? Sg[b + r->krow[l] * a] : Sg[a + r->krow[l] * b];
            acc += A(sab, absval) * xs[b + kc * v];
          }
          yt[a + kr * v] += acc;
        }
    }
  }

  /* Z rows of leaf j: sum over its ancestors of Uhat_anc[rows] yh_anc, then
   * the dense blocks of its row */
#pragma omp parallel
  {
    double** chain = (double**)malloc(sizeof(double*) * (q + 1));
    double* store = (double*)malloc(sizeof(double) * (size_t)((q + 1) * (mmax * kmax + 1)));
    int ok = chain && store;
    if (ok)
      for (int64_t l = 0; l <= q; ++l) chain[l] = store + l * (mmax * kmax + 1);
#pragma omp for schedule(dynamic, 4)
    for (int64_t j = 0; j < nl; ++j) {
      if (!ok || !need_leaf[j]) continue;
      const int64_t t = r->leaf0 + j, m = r->hi[t] - r->lo[t], lo = r->lo[t];
      leaf_chain(r, w.Brow, w.Trow, w.krow, w.tbrow, j, chain, absval);
      for (int64_t v = 0; v < nv; ++v)
        for (int64_t i = 0; i < m; ++i) Z[lo + i + r->n * v] = 0.0;
      int64_t anc = t;
      for (int64_t l = q; l >= 0; --l) {
        const int64_t k = w.krow[l];
        const double* ya = yh + yoff[anc];
        for (int64_t v = 0; v < nv; ++v)
          for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t a = 0; a < k; ++a) s += chain[l][i + m * a] * ya[a + k * v];
            Z[lo + i + r->n * v] += s;
          }
        anc = r->parent[anc];
      }
      const int64_t bbeg = trans ? r->dc_ptr[j] : r->d_rowptr[j];
      const int64_t bend = trans ? r->dc_ptr[j + 1] : r->d_rowptr[j + 1];
      for (int64_t bi = bbeg; bi < bend; ++bi) {
        const int64_t b = trans ? r->dc_blk[bi] : bi;
        const int64_t rl = r->leaf0 + r->drow[b], cl = r->leaf0 + r->d_col[b];
        const int64_t mt = r->hi[rl] - r->lo[rl], ms = r->hi[cl] - r->lo[cl];
        const double* Db = r->D + r->ddat[b];
        const int64_t other = trans ? rl : cl; /* leaf whose input rows are read */
        const int64_t mo = trans ? mt : ms;
        for (int64_t v = 0; v < nv; ++v)
          for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t jj = 0; jj < mo; ++jj) {
              double d = trans ? Db[jj + mt * i] : Db[i + mt * jj];
              s += A(d, absval) * A(xt[r->lo[other] + jj + r->n * v], absval);
            }
            Z[lo + i + r->n * v] += s;
          }
      }
    }
    free(chain);
    free(store);
    if (!ok) {
#pragma omp atomic write
      rc = H2O_ENOMEM;
    }
  }
done:
  free(cbase); free(xoff); free(yoff); free(contrib); free(xh); free(yh);
  return rc;
}

static int op_trans(char op) {
  if (op == 'N' || op == 'n') return 0;
  if (op == 'T' || op == 't') return 1;
  return -1;
}

/* Y <- alpha op(A) X + beta Y.  X: n x nv column-major with leading dimension
 * ldx, original order; Y likewise (ldy).  Returns 0 or a negative code. */
int h2o_gemv(const h2o_rep* r, char op, double alpha, const double* X, int64_t ldx, int64_t nv,
             double beta, double* Y, int64_t ldy, int absval) {
  const int trans = op_trans(op);
  if (!r || trans < 0 || nv < 0) return H2O_EINVAL;
  if (nv == 0) return H2O_OK;
  if (!Y || ldy < r->n || (alpha != 0.0 && (!X || ldx < r->n))) return H2O_EINVAL;
  const int64_t n = r->n;
  const double al = A(alpha, absval), be = A(beta, absval);
  if (alpha == 0.0) {
    for (int64_t v = 0; v < nv; ++v)
      for (int64_t i = 0; i < n; ++i)
        Y[i + ldy * v] = beta == 0.0 ? 0.0 : be * A(Y[i + ldy * v], absval);
    return H2O_OK;
  }
  double* xt = (double*)malloc(sizeof(double) * (size_t)(n * nv));
  double* Z = (double*)malloc(sizeof(double) * (size_t)(n * nv));
  uint8_t* need_node = (uint8_t*)malloc((size_t)r->nnodes);
  uint8_t* need_leaf = (uint8_t*)malloc((size_t)r->nleaves + 1);
  int rc = H2O_ENOMEM;
  if (xt && Z && need_node && need_leaf) {
    memset(need_node, 1, (size_t)r->nnodes);
    memset(need_leaf, 1, (size_t)r->nleaves + 1);
    for (int64_t v = 0; v < nv; ++v)
      for (int64_t i = 0; i < n; ++i) xt[i + n * v] = X[r->perm[i] + ldx * v];
    rc = core(r, trans, xt, nv, need_node, need_leaf, Z, absval);
    if (rc == H2O_OK)
      for (int64_t v = 0; v < nv; ++v)
        for (int64_t i = 0; i < n; ++i) {
          double* y = &Y[r->perm[i] + ldy * v];
          *y = al * Z[i + n * v] + (beta == 0.0 ? 0.0 : be * A(*y, absval));
        }
  }
  free(xt); free(Z); free(need_node); free(need_leaf);
  return rc;
}

/* Selected rows of  alpha op(A) X + beta Y0:  out[k + nrows*v] for the
 * original row index rows[k].  Y0 (ldy) is read only where beta != 0.
 * Only the coupling rows on the paths from those rows' leaves to the root are
 * evaluated, which makes single rows cheap at any size. */
int h2o_gemv_rows(const h2o_rep* r, char op, double alpha, const double* X, int64_t ldx, int64_t nv,
                  double beta, const double* Y0, int64_t ldy, const int64_t* rows, int64_t nrows,
                  double* out, int absval) {
  const int trans = op_trans(op);
  if (!r || trans < 0 || nv < 0 || nrows < 0 || (nrows && (!rows || !out))) return H2O_EINVAL;
  if (nv == 0 || nrows == 0) return H2O_OK;
  if ((alpha != 0.0 && (!X || ldx < r->n)) || (beta != 0.0 && (!Y0 || ldy < r->n))) return H2O_EINVAL;
  const int64_t n = r->n;
  int64_t* pinv = (int64_t*)malloc(sizeof(int64_t) * n);
  double* xt = (double*)malloc(sizeof(double) * (size_t)(n * nv));
  double* Z = (double*)calloc((size_t)(n * nv), sizeof(double));
  uint8_t* need_node = (uint8_t*)calloc((size_t)r->nnodes, 1);
  uint8_t* need_leaf = (uint8_t*)calloc((size_t)r->nleaves + 1, 1);
  int rc = H2O_ENOMEM;
  if (pinv && xt && Z && need_node && need_leaf) {
    rc = H2O_OK;
    for (int64_t i = 0; i < n; ++i) pinv[r->perm[i]] = i;
    for (int64_t k = 0; k < nrows; ++k) {
      if (rows[k] < 0 || rows[k] >= n) { rc = H2O_EINVAL; break; }
      int64_t j = r->leaf_at[pinv[rows[k]]];
      need_leaf[j] = 1;
      for (int64_t c = r->leaf0 + j; c >= 0; c = r->parent[c]) need_node[c] = 1;
    }
    if (rc == H2O_OK && alpha != 0.0) {
      for (int64_t v = 0; v < nv; ++v)
        for (int64_t i = 0; i < n; ++i) xt[i + n * v] = X[r->perm[i] + ldx * v];
      rc = core(r, trans, xt, nv, need_node, need_leaf, Z, absval);
    }
    if (rc == H2O_OK) {
      const double al = A(alpha, absval), be = A(beta, absval);
      for (int64_t v = 0; v < nv; ++v)
        for (int64_t k = 0; k < nrows; ++k) {
          const int64_t i = pinv[rows[k]];
          double y = alpha == 0.0 ? 0.0 : al * Z[i + n * v];
          if (beta != 0.0) y += be * A(Y0[rows[k] + ldy * v], absval);
          out[k + nrows * v] = y;
        }
    }
  }
  free(pinv); free(xt); free(Z); free(need_node); free(need_leaf);
  return rc;
}

/* Dense expansion of op(A) (n x n, column-major, original order), block by
 * block: every coupling block is formed as Uhat_t S_ts Vhat_s^T from the
 * explicit bases, every dense block is copied.  For small n only. */
int h2o_dense(const h2o_rep* r, char op, double* Aout) {
  const int trans = op_trans(op);
  if (!r || trans < 0 || !Aout) return H2O_EINVAL;
  const int64_t n = r->n, q = r->q;
  /* explicit basis rows per level: Uex[l] is n x krow[l], row i = row of
   * Uhat_{anc_l(leaf(i))} at position i; Vex likewise */
  int64_t ku = 0, kv = 0;
  for (int64_t l = 0; l <= q; ++l) { ku += r->krow[l]; kv += r->kcol[l]; }
  double* Uex = (double*)calloc((size_t)(n * ku + 1), sizeof(double));
  double* Vex = (double*)calloc((size_t)(n * kv + 1), sizeof(double));
  int64_t* ub = (int64_t*)malloc(sizeof(int64_t) * (q + 1));
  int64_t* vb = (int64_t*)malloc(sizeof(int64_t) * (q + 1));
  int64_t kmax = 1, mmax = 1;
  for (int64_t l = 0; l <= q; ++l) {
    if (r->krow[l] > kmax) kmax = r->krow[l];
    if (r->kcol[l] > kmax) kmax = r->kcol[l];
  }
  for (int64_t j = 0; j < r->nleaves; ++j)
    if (r->hi[r->leaf0 + j] - r->lo[r->leaf0 + j] > mmax) mmax = r->hi[r->leaf0 + j] - r->lo[r->leaf0 + j];
  double** chain = (double**)malloc(sizeof(double*) * (q + 1));
  double* store = (double*)malloc(sizeof(double) * (size_t)((q + 1) * mmax * kmax));
  if (!Uex || !Vex || !ub || !vb || !chain || !store) {
    free(Uex); free(Vex); free(ub); free(vb); free(chain); free(store);
    return H2O_ENOMEM;
  }
  for (int64_t l = 0; l <= q; ++l) chain[l] = store + l * mmax * kmax;
  {
    int64_t a = 0, b = 0;
    for (int64_t l = 0; l <= q; ++l) { ub[l] = a; vb[l] = b; a += n * r->krow[l]; b += n * r->kcol[l]; }
  }
  for (int pass = 0; pass < 2; ++pass) {
    const double* B = pass ? r->V : r->U;
    const double* T = pass ? r->F : r->E;
    const int64_t* k = pass ? r->kcol : r->krow;
    const int64_t* tb = pass ? r->fbase : r->ebase;
    double* ex = pass ? Vex : Uex;
    const int64_t* base = pass ? vb : ub;
    for (int64_t j = 0; j < r->nleaves; ++j) {
      const int64_t t = r->leaf0 + j, m = r->hi[t] - r->lo[t];
      leaf_chain(r, B, T, k, tb, j, chain, 0);
      for (int64_t l = 0; l <= q; ++l)
        for (int64_t a = 0; a < k[l]; ++a)
          for (int64_t i = 0; i < m; ++i) ex[base[l] + (r->lo[t] + i) + n * a] = chain[l][i + m * a];
    }
  }
  for (int64_t e = 0; e < n * n; ++e) Aout[e] = 0.0;
  /* tree-ordered entry (i, j) of A goes to (perm[i], perm[j]), or transposed */
#define PUT(i, j, val)                                                        \
  do {                                                                        \
    int64_t pi_ = r->perm[i], pj_ = r->perm[j];                               \
    if (trans) Aout[pj_ + n * pi_] += (val); else Aout[pi_ + n * pj_] += (val); \
  } while (0)
  for (int64_t l = 0; l <= q; ++l) {
    const int64_t kr = r->krow[l], kc = r->kcol[l];
    for (int64_t g = r->blk_base[l]; g < r->blk_base[l + 1]; ++g) {
      const int64_t t = r->blk_row[g], s = r->blk_colg[g];
      const double* Sg = r->S + r->sdat[l] + (g - r->blk_base[l]) * kr * kc;
      for (int64_t j = r->lo[s]; j < r->hi[s]; ++j)
        for (int64_t i = r->lo[t]; i < r->hi[t]; ++i) {
          double val = 0.0;
          for (int64_t a = 0; a < kr; ++a) {
            double inner = 0.0;
            for (int64_t b = 0; b < kc; ++b) inner += Sg[a + kr * b] * Vex[vb[l] + j + n * b];
            val += Uex[ub[l] + i + n * a] * inner;
          }
          PUT(i, j, val);
        }
    }
  }
  for (int64_t b = 0; b < r->ndense; ++b) {
    const int64_t t = r->leaf0 + r->drow[b], s = r->leaf0 + r->d_col[b];
    const int64_t mt = r->hi[t] - r->lo[t];
    const double* Db = r->D + r->ddat[b];
    for (int64_t j = r->lo[s]; j < r->hi[s]; ++j)
      for (int64_t i = r->lo[t]; i < r->hi[t]; ++i) PUT(i, j, Db[(i - r->lo[t]) + mt * (j - r->lo[s])]);
  }
#undef PUT
  free(Uex); free(Vex); free(ub); free(vb); free(chain); free(store);
  return H2O_OK;
}
