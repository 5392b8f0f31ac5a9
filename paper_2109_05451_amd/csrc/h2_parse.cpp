// Reader and validator of the serialized H^2 representation ("H2MATV01").
//
// Sections (8-byte elements, each starting on a 64-byte boundary after a
// 128-byte header): level_ptr, krow, kcol, nadm, perm, lo, hi, parent,
// s_rowptr, s_col, d_rowptr, d_col, U, E, V, F, S, D, points.  V and F are
// empty when the column basis is shared with the row basis (flags bit 0
// clear); points are empty unless flags bit 1 is set.
//
// Validation establishes everything the kernels rely on: a single root
// covering [0, n); children of each parent consecutive, in parent order, and
// tiling its range; every inner node with a child; perm a permutation; CSR
// row pointers monotone with in-range, strictly increasing columns; section
// sizes consistent with the structure; and the limits of this build.
#include <cstring>
#include <string>
#include <vector>

#include "h2_internal.h"

namespace h2 {
namespace {

struct Cursor {
  const uint8_t* buf;
  int64_t len;
  int64_t pos;
  bool take(int64_t count, int64_t* at) {
    pos = (pos + 63) / 64 * 64;
    if (count < 0 || pos > len || count > (len - pos) / 8) return false;
    *at = pos;
    pos += 8 * count;
    return true;
  }
};

int fail(int code, const std::string& msg) {
  set_error("h2 representation: " + msg);
  return code;
}

}  // namespace

int parse(const uint8_t* buf, int64_t len, Parsed* p) {
  if (!buf || !p) return fail(H2_EINVAL, "null buffer");
  if (reinterpret_cast<uintptr_t>(buf) % 8) return fail(H2_EINVAL, "buffer is not 8-byte aligned");
  if (len < 128) return fail(H2_EFORMAT, "shorter than the header");
  if (std::memcmp(buf, "H2MATV01", 8) != 0) return fail(H2_EFORMAT, "bad magic");
  uint32_t version, flags;
  std::memcpy(&version, buf + 8, 4);
  std::memcpy(&flags, buf + 12, 4);
  if (version != 1) return fail(H2_EFORMAT, "unsupported version");
  if (flags & ~3u) return fail(H2_EFORMAT, "unknown flags");
  int64_t hd[4], tail[2];
  std::memcpy(hd, buf + 16, 32);
  std::memcpy(tail, buf + 88, 16);
  const int64_t n = hd[0], q = hd[1], nnodes = hd[2], dim = hd[3];
  const int64_t ndense = tail[0], total = tail[1];
  if (total != len) return fail(H2_EFORMAT, "size in header differs from buffer size");
  if (n < 1 || q < 0 || q > 40 || nnodes < 1 || dim < 0 || dim > 64 || ndense < 0)
    return fail(H2_EFORMAT, "bad header counts");
  if (!(flags & 2u) && dim != 0) return fail(H2_EFORMAT, "dimension set without points");
  if (n >= (int64_t(1) << 31) || nnodes >= (int64_t(1) << 31) || ndense >= (int64_t(1) << 31))
    return fail(H2_EUNSUPPORTED, "n, nodes and dense blocks must be below 2^31");

  Parsed& P = *p;
  P = Parsed();
  P.n = n; P.q = q; P.nnodes = nnodes; P.ndense = ndense; P.flags = flags;
  Cursor c{buf, len, 128};
  int64_t at;
  auto I = [&](int64_t off) { return reinterpret_cast<const int64_t*>(buf + off); };
#define SECTION(dst, count) \
  do { if (!c.take((count), &at)) return fail(H2_EFORMAT, "truncated section " #dst); dst = I(at); } while (0)
  SECTION(P.level_ptr, q + 2);
  SECTION(P.krow, q + 1);
  SECTION(P.kcol, q + 1);
  SECTION(P.nadm, q + 1);
  const int64_t* lp = P.level_ptr;
  if (lp[0] != 0 || lp[1] != 1 || lp[q + 1] != nnodes) return fail(H2_EFORMAT, "bad level pointers");
  for (int64_t l = 0; l <= q; ++l) {
    if (lp[l + 1] <= lp[l]) return fail(H2_EFORMAT, "empty level");
    if (P.krow[l] < 0 || P.kcol[l] < 0 || P.nadm[l] < 0) return fail(H2_EFORMAT, "negative rank or count");
    if (P.krow[l] > kMaxDim || P.kcol[l] > kMaxDim) return fail(H2_EUNSUPPORTED, "rank above 256");
    if (!(flags & 1u) && P.krow[l] != P.kcol[l]) return fail(H2_EFORMAT, "shared basis with unequal ranks");
    if (P.nadm[l] > (len / 8)) return fail(H2_EFORMAT, "block count exceeds buffer");
    P.nadm_tot += P.nadm[l];
  }
  if (P.nadm_tot >= (int64_t(1) << 31)) return fail(H2_EUNSUPPORTED, "more than 2^31 coupling blocks");
  P.leaf0 = lp[q];
  P.nleaves = nnodes - lp[q];
  SECTION(P.perm, n);
  SECTION(P.lo, nnodes);
  SECTION(P.hi, nnodes);
  SECTION(P.parent, nnodes);
  SECTION(P.s_rowptr, nnodes + q + 1);
  SECTION(P.s_col, P.nadm_tot);
  SECTION(P.d_rowptr, P.nleaves + 1);
  SECTION(P.d_col, ndense);

  {  // permutation
    std::vector<uint8_t> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t v = P.perm[i];
      if (v < 0 || v >= n || seen[v]) return fail(H2_EFORMAT, "perm is not a permutation");
      seen[v] = 1;
    }
  }
  // tree
  if (P.lo[0] != 0 || P.hi[0] != n || P.parent[0] != -1) return fail(H2_EFORMAT, "root must cover [0, n)");
  for (int64_t l = 1; l <= q; ++l) {
    int64_t expect_parent = lp[l - 1];  // parents must appear in order, none skipped
    for (int64_t cnode = lp[l]; cnode < lp[l + 1]; ++cnode) {
      const int64_t par = P.parent[cnode];
      if (P.lo[cnode] > P.hi[cnode]) return fail(H2_EFORMAT, "node with lo > hi");
      const bool first_child = cnode == lp[l] || par != P.parent[cnode - 1];
      if (first_child) {
        if (par != expect_parent) return fail(H2_EFORMAT, "parents out of order or childless inner node");
        if (P.lo[cnode] != P.lo[par]) return fail(H2_EFORMAT, "first child does not start at parent lo");
        if (cnode > lp[l] && P.hi[cnode - 1] != P.hi[P.parent[cnode - 1]])
          return fail(H2_EFORMAT, "last child does not end at parent hi");
        ++expect_parent;
      } else if (P.lo[cnode] != P.hi[cnode - 1]) {
        return fail(H2_EFORMAT, "sibling ranges do not tile the parent");
      }
    }
    if (expect_parent != lp[l]) return fail(H2_EFORMAT, "inner node without children");
    if (P.hi[lp[l + 1] - 1] != P.hi[P.parent[lp[l + 1] - 1]])
      return fail(H2_EFORMAT, "last child does not end at parent hi");
  }
  for (int64_t t = P.leaf0; t < nnodes; ++t)
    if (P.hi[t] - P.lo[t] > kMaxDim) return fail(H2_EUNSUPPORTED, "leaf larger than 256");
  // coupling CSR, per level
  P.rp_base.assign(q + 1, 0);
  P.blk_base.assign(q + 2, 0);
  P.sdat.assign(q + 2, 0);
  {
    int64_t rb = 0, bb = 0, sd = 0;
    for (int64_t l = 0; l <= q; ++l) {
      const int64_t nl = lp[l + 1] - lp[l];
      const int64_t* rp = P.s_rowptr + rb;
      P.rp_base[l] = rb; P.blk_base[l] = bb; P.sdat[l] = sd;
      if (rp[0] != 0 || rp[nl] != P.nadm[l]) return fail(H2_EFORMAT, "coupling row pointer ends");
      // the whole pointer array first, so that no row's range runs past the level's columns
      for (int64_t t = 0; t < nl; ++t)
        if (rp[t + 1] < rp[t]) return fail(H2_EFORMAT, "coupling row pointer decreases");
      for (int64_t t = 0; t < nl; ++t) {
        for (int64_t b = rp[t]; b < rp[t + 1]; ++b) {
          const int64_t s = P.s_col[bb + b];
          if (s < 0 || s >= nl) return fail(H2_EFORMAT, "coupling column out of range");
          if (b > rp[t] && s <= P.s_col[bb + b - 1]) return fail(H2_EFORMAT, "coupling columns not increasing");
        }
      }
      rb += nl + 1;
      bb += P.nadm[l];
      sd += P.nadm[l] * P.krow[l] * P.kcol[l];
    }
    P.blk_base[q + 1] = bb;
    P.sdat[q + 1] = sd;
  }
  // dense CSR over leaves
  P.ddat.assign(ndense + 1, 0);
  {
    const int64_t* rp = P.d_rowptr;
    if (rp[0] != 0 || rp[P.nleaves] != ndense) return fail(H2_EFORMAT, "dense row pointer ends");
    for (int64_t t = 0; t < P.nleaves; ++t)
      if (rp[t + 1] < rp[t]) return fail(H2_EFORMAT, "dense row pointer decreases");
    for (int64_t t = 0; t < P.nleaves; ++t) {
      const int64_t mt = P.hi[P.leaf0 + t] - P.lo[P.leaf0 + t];
      for (int64_t b = rp[t]; b < rp[t + 1]; ++b) {
        const int64_t s = P.d_col[b];
        if (s < 0 || s >= P.nleaves) return fail(H2_EFORMAT, "dense column out of range");
        if (b > rp[t] && s <= P.d_col[b - 1]) return fail(H2_EFORMAT, "dense columns not increasing");
        P.ddat[b + 1] = P.ddat[b] + mt * (P.hi[P.leaf0 + s] - P.lo[P.leaf0 + s]);
      }
    }
  }
  // transfers
  P.ebase.assign(q + 2, 0);
  P.fbase.assign(q + 2, 0);
  for (int64_t l = 1; l <= q; ++l) {
    const int64_t nl = lp[l + 1] - lp[l];
    P.ebase[l + 1] = P.ebase[l] + nl * P.krow[l] * P.krow[l - 1];
    P.fbase[l + 1] = P.fbase[l] + nl * P.kcol[l] * P.kcol[l - 1];
  }
  const bool sep = (flags & 1u) != 0;
  if (!c.take(n * P.krow[q], &P.off_U)) return fail(H2_EFORMAT, "truncated U");
  if (!c.take(P.ebase[q + 1], &P.off_E)) return fail(H2_EFORMAT, "truncated E");
  if (!c.take(sep ? n * P.kcol[q] : 0, &P.off_V)) return fail(H2_EFORMAT, "truncated V");
  if (!c.take(sep ? P.fbase[q + 1] : 0, &P.off_F)) return fail(H2_EFORMAT, "truncated F");
  if (!c.take(P.sdat[q + 1], &P.off_S)) return fail(H2_EFORMAT, "truncated S");
  if (!c.take(P.ddat[ndense], &P.off_D)) return fail(H2_EFORMAT, "truncated D");
  P.off_end = c.pos;
  if (!c.take((flags & 2u) ? n * dim : 0, &at)) return fail(H2_EFORMAT, "truncated points");
  if ((c.pos + 63) / 64 * 64 != len) return fail(H2_EFORMAT, "trailing bytes after the last section");
#undef SECTION
  return H2_OK;
}

}  // namespace h2
