// Host-side check of the representation reader and the launch-plan builder
// (h2_parse.cpp, h2_plan.cpp), compiled with g++ and AddressSanitizer +
// UndefinedBehaviorSanitizer by tests/test_host_sanitize.py.
//
// For each representation file given on the command line:
//  1. the file parses, and the plan built from it stays inside its sections:
//     every row's matrix slice lies in the section its phase reads, every
//     gathered input segment and every output range lies in its vector tree
//     or point array, and the transposed basis copy is written in bounds;
//  2. seeded mutations of the file (an index entry overwritten with an
//     extreme or neighbouring value, a byte flipped, a row pointer run past
//     the end of its column array, the buffer cut short)
//     are parsed from an allocation of exactly the mutated length; a mutation
//     the reader accepts goes through the same plan construction and bounds
//     checks.  Any read or write outside a buffer, or signed overflow, stops
//     the program with a sanitizer report.
//
// Output: one line per file, "<file> ok <accepted> <rejected>", or a line
// starting with "FAIL" and exit status 1.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "h2_internal.h"

namespace h2 {
void set_error(const std::string&) {}
}  // namespace h2

namespace {

using namespace h2;

uint64_t g_state = 0x9e3779b97f4a7c15ull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

bool g_fail = false;
void fail(const char* what, long long a, long long b) {
  std::printf("FAIL %s (%lld, %lld)\n", what, a, b);
  g_fail = true;
}

// Every row of one phase: matrix slice in [sec_lo, sec_hi), inputs of the
// given length, outputs of the given length.
void check_rows(const char* phase, const std::vector<RowSpec>& rows, int64_t sec_lo, int64_t sec_hi,
                int64_t in_len, int64_t out_len) {
  for (const RowSpec& r : rows) {
    int64_t cols = 0;
    for (const BlockRef& b : r.blks) {
      if (b.width < 0 || b.in_off < 0 || b.in_off + b.width > in_len) {
        fail(phase, b.in_off, b.width);
        return;
      }
      cols += b.width;
    }
    if (r.nrows < 0 || r.out_off < 0 || r.out_off + r.nrows > out_len) {
      fail(phase, r.out_off, r.nrows);
      return;
    }
    if (r.data_off < sec_lo || r.data_off + int64_t(r.nrows) * cols > sec_hi) {
      fail(phase, r.data_off, int64_t(r.nrows) * cols);
      return;
    }
  }
}

// Builds everything h2_load builds on the host and checks its bounds.
void plan_and_check(const uint8_t* buf, const Parsed& P) {
  OpLayout L;
  if (make_layout(P, &L) != H2_OK) return;
  const int64_t q = P.q, n = P.n;
  // transposed copy into an allocation of exactly ntrans doubles
  double* tr = static_cast<double*>(std::malloc(sizeof(double) * std::max<int64_t>(L.ntrans, 1)));
  build_transposed(buf, L, tr);
  std::free(tr);
  RowBases B;
  B.ld_x = n;
  B.ld_h = L.H;
  RowsN R;
  emit_rows_N(L, B, &R);
  const int64_t nU = n * P.krow[q], nV = n * P.kcol[q];
  check_rows("leaf products", R.up[0], L.tVT, L.tVT + nV, n, L.H);
  for (size_t h = 1; h < R.up.size(); ++h) check_rows("upsweep transfers", R.up[h], L.tFT, L.tFT + P.fbase[q + 1], L.H, L.H);
  check_rows("coupling", R.couple, L.oS, L.oS + P.sdat[q + 1], L.H, L.H);
  for (const auto& lv : R.down) check_rows("downsweep transfers", lv, L.oE, L.oE + P.ebase[q + 1], L.H, L.H);
  check_rows("dense", R.dense, L.oD, L.oD + P.ddat[P.ndense], n, n);
  check_rows("leaf expansion", R.out, L.oU, L.oU + nU, L.H, n);
  if (L.nmat * 8 != P.off_end - P.off_U) fail("matrix array length", L.nmat, P.off_end - P.off_U);
  // the tables the kernels read
  RowTables t;
  for (const RowSpec& r : R.couple) append_row(t, r);
  for (const RowSpec& r : R.dense) append_row(t, r);
  for (const RowDesc& d : t.rows) {
    if (d.blk_begin < 0 || d.blk_end < d.blk_begin || d.blk_end > int64_t(t.colend.size())) {
      fail("row table", d.blk_begin, d.blk_end);
      break;
    }
    for (int32_t b = d.blk_begin + 1; b < d.blk_end; ++b)
      if (t.colend[b] < t.colend[b - 1]) fail("column ends decrease", b, t.colend[b]);
  }
}

bool load(const char* path, std::vector<uint8_t>* out) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  std::fseek(f, 0, SEEK_END);
  const long len = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  out->resize(len);
  const bool ok = std::fread(out->data(), 1, len, f) == size_t(len);
  std::fclose(f);
  return ok;
}

// Parses a copy of `bytes` held in an allocation of exactly its length.
int parse_exact(const std::vector<uint8_t>& bytes, bool plan) {
  uint8_t* b = static_cast<uint8_t*>(std::malloc(std::max<size_t>(bytes.size(), 1)));
  std::memcpy(b, bytes.data(), bytes.size());
  Parsed P;
  const int rc = parse(b, int64_t(bytes.size()), &P);
  if (rc == H2_OK && plan) plan_and_check(b, P);
  std::free(b);
  return rc;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 3) {
    std::printf("usage: host_check MUTATIONS FILE...\n");
    return 2;
  }
  const int mutations = std::atoi(argv[1]);
  for (int fi = 2; fi < argc; ++fi) {
    std::vector<uint8_t> base;
    if (!load(argv[fi], &base)) {
      std::printf("FAIL cannot read %s\n", argv[fi]);
      return 1;
    }
    if (parse_exact(base, true) != H2_OK) {
      std::printf("FAIL %s does not parse\n", argv[fi]);
      return 1;
    }
    Parsed P0;
    parse(base.data(), int64_t(base.size()), &P0);
    const int64_t idx_end = P0.off_U;  // header and index sections
    int accepted = 0, rejected = 0;
    g_state = 0x243f6a8885a308d3ull + uint64_t(fi);
    for (int it = 0; it < mutations && !g_fail; ++it) {
      std::vector<uint8_t> m = base;
      const uint64_t kind = next_u64() % 5;
      if (kind <= 1) {  // one index entry (8-byte aligned, after the magic) overwritten
        const int64_t slots = (idx_end - 16) / 8;
        const int64_t at = 16 + 8 * int64_t(next_u64() % uint64_t(slots));
        int64_t v;
        std::memcpy(&v, m.data() + at, 8);
        static const int64_t extremes[] = {0, -1, 1, 2, 255, 256, 257, int64_t(1) << 31, int64_t(1) << 40,
                                           INT64_MAX, INT64_MIN, INT64_MAX / 8};
        if (kind == 0) v = extremes[next_u64() % (sizeof(extremes) / sizeof(extremes[0]))];
        else v += int64_t(next_u64() % 7) - 3;
        std::memcpy(m.data() + at, &v, 8);
      } else if (kind == 2) {  // one byte flipped anywhere before the matrix data
        const int64_t at = int64_t(next_u64() % uint64_t(idx_end));
        m[at] ^= uint8_t(1u << (next_u64() % 8));
      } else if (kind == 3) {  // a row pointer run past its array's end: rp[t] = end, rp[t+1] > end
        const bool dense = P0.ndense > 0 && (next_u64() & 1);
        const int64_t l = int64_t(next_u64() % uint64_t(P0.q + 1));
        const int64_t* rp = dense ? P0.d_rowptr : P0.s_rowptr + P0.rp_base[l];
        const int64_t rows = dense ? P0.nleaves : P0.level_ptr[l + 1] - P0.level_ptr[l];
        const int64_t end = dense ? P0.ndense : P0.nadm[l];
        if (rows >= 2) {
          const int64_t t = int64_t(next_u64() % uint64_t(rows - 1));
          const int64_t at = reinterpret_cast<const uint8_t*>(rp + t) - base.data();
          const int64_t v0 = end, v1 = end + 1 + int64_t(next_u64() % 3);
          std::memcpy(m.data() + at, &v0, 8);
          std::memcpy(m.data() + at + 8, &v1, 8);
        }
      } else {  // cut short (the header's size field kept consistent half of the time)
        const int64_t len = 8 * int64_t(next_u64() % uint64_t(base.size() / 8));
        m.resize(len);
        if (len >= 104 && (next_u64() & 1)) std::memcpy(m.data() + 96, &len, 8);
      }
      if (parse_exact(m, true) == H2_OK) ++accepted;
      else ++rejected;
    }
    if (g_fail) {
      std::printf("FAIL %s\n", argv[fi]);
      return 1;
    }
    std::printf("%s ok %d %d\n", argv[fi], accepted, rejected);
  }
  return 0;
}
