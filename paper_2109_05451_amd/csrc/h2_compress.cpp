// Algebraic recompression of a loaded operator (Section 5 of the paper) and
// export of a handle to the serialized format.
//
// The steps follow the paper: orthogonalize each basis tree (QR upsweep,
// Sec. 5 "orthogonalize"), compute for every node the reweighting of its
// basis by everything its block row holds (downsweep, Sec. 5.1), truncate
// the reweighed bases bottom-up (Sec. 5.2) and project the coupling blocks on
// the new bases.  Two departures, both exact in exact arithmetic:
//  * the reweighting downsweep carries the Gram matrix G_i = R_i^T R_i of
//    each node's stack instead of its R factor,
//      G_i = E_i G_parent E_i^T + sum over own blocks S S^T (block columns:
//      S^T S),
//    which turns the paper's batched QR of tall stacks into batched GEMMs;
//  * the truncation SVDs become symmetric eigenproblems of the same singular
//    structure: at a leaf the reweighed basis U_t R_t^T has left singular
//    vectors U_t z and singular values sqrt(lambda) for the eigenpairs of
//    G_t; at an inner node the stack M = [T_c E_c] R^T (R any square root of
//    G, here diag(sqrt(lambda)) Z^T) has right singular vectors from the
//    eigenpairs of M^T M and left ones M y / sigma.
// Singular values enter through their squares, so kept counts are decided
// reliably for thresholds well above sqrt(machine epsilon) (tau >= 1e-7).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "h2_compress.h"
#include "h2_internal.h"

namespace h2 {
namespace {

int hfail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? H2_ENOMEM : H2_EHIP;
}
#define CK(call, what)                            \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hfail(e_, what); \
  } while (0)
#define RC(x)                         \
  do {                                \
    int r_ = (x);                     \
    if (r_ != H2_OK) return r_;       \
  } while (0)

// Device allocations of one compression, with a bounds registry: every task
// operand is checked to lie inside one allocation before its launch.
class Arena {
 public:
  ~Arena() {
    (void)hipDeviceSynchronize();  // the uploads read host_ until they ran
    for (void* p : ptrs_) (void)hipFree(p);
  }
  template <class T>
  int alloc(T** out, int64_t count, hipStream_t s) {
    *out = nullptr;
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(out), bytes);
    if (e != hipSuccess) return hfail(e, "hipMalloc(compression)");
    ptrs_.push_back(*out);
    reg(*out, bytes);
    CK(hipMemsetAsync(*out, 0, bytes, s), "hipMemsetAsync(compression)");
    return H2_OK;
  }
  // asynchronous upload of a copy of v that the arena keeps until it is
  // destroyed; small uploads are carved from 16 MiB device chunks
  template <class T>
  int upload(const std::vector<T>& v, T** out, hipStream_t s) {
    const size_t bytes = (sizeof(T) * std::max<size_t>(v.size(), 1) + 255) / 256 * 256;
    if (bytes > kChunk) {
      RC(alloc(out, (int64_t)v.size(), s));
    } else {
      if (!chunk_ || used_ + bytes > kChunk) {
        uint8_t* c = nullptr;
        RC(alloc(&c, (int64_t)kChunk, s));
        chunk_ = c;
        used_ = 0;
      }
      *out = reinterpret_cast<T*>(chunk_ + used_);
      used_ += bytes;
    }
    if (v.empty()) return H2_OK;
    host_.emplace_back(reinterpret_cast<const uint8_t*>(v.data()),
                       reinterpret_cast<const uint8_t*>(v.data()) + sizeof(T) * v.size());
    CK(hipMemcpyAsync(*out, host_.back().data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s), "upload");
    return H2_OK;
  }
  void reg(const void* p, size_t bytes) {
    regions_.push_back({reinterpret_cast<uintptr_t>(p), reinterpret_cast<uintptr_t>(p) + bytes});
  }
  // a column-major rows x cols matrix at p with leading dimension ld
  bool inside(const double* p, int64_t rows, int64_t cols, int64_t ld) const {
    if (rows <= 0 || cols <= 0) return true;
    if (!p || ld < rows) return false;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    const uintptr_t b = reinterpret_cast<uintptr_t>(p + (rows - 1) + (cols - 1) * ld) + sizeof(double);
    for (const auto& r : regions_)
      if (a >= r.first && b <= r.second) return true;
    return false;
  }

 private:
  std::vector<void*> ptrs_;
  std::vector<std::pair<uintptr_t, uintptr_t>> regions_;
  std::vector<std::vector<uint8_t>> host_;
  static constexpr size_t kChunk = size_t(16) << 20;
  uint8_t* chunk_ = nullptr;
  size_t used_ = 0;
};

int oob(const char* what) {
  set_error(std::string("recompression: internal operand out of bounds (") + what + ")");
  return H2_EINVAL;
}

// Structure of one basis tree on the device.
struct Tree {
  const int64_t* k = nullptr;  // rank per level
  const double* B = nullptr;   // leaf bases (U or V section)
  const double* T = nullptr;   // transfers (E or F section)
  const std::vector<int64_t>* tbase = nullptr;  // per level: first transfer's element offset
  // results
  double *Bo = nullptr, *To = nullptr;  // orthogonal bases
  double* R = nullptr;                  // per node k x k: orthogonalization factor, later sqrt(G)
  double* G = nullptr;                  // per node k x k: reweighting Gram matrix
  double* W = nullptr;                  // per node k x k: scratch (masked Gram, K = M^T M)
  double* Z = nullptr;                  // per node k x k: eigenvectors
  double* Y = nullptr;                  // per node k x k: second eigenvectors (inner nodes)
  double* lam = nullptr;                // per node k: eigenvalues
  double* lam2 = nullptr;               // per node k: second eigenvalues
  double* Tt = nullptr;                 // per node k' x k: T_i = U'_i^T U_i
  double* stack = nullptr;              // per parent: QR stacks, then N_p
  double* Mb = nullptr;                 // per parent: M_p
  double* Et = nullptr;                 // new transfers, in the old transfers' slots (ld k'_l)
  double* Bn = nullptr;                 // new leaf bases (n x k'_q, final layout)
  int32_t* counts = nullptr;            // per node kept count
  double* sref2 = nullptr;              // largest leaf eigenvalue
  std::vector<int64_t> knew;            // new rank per level
  double sigma_ref = 0.0;
};

struct Ctx {
  h2_op_s* h = nullptr;
  Parsed P;
  hipStream_t s = nullptr;
  Arena ar;
  std::vector<int64_t> lvl;      // level of each node
  std::vector<int64_t> nk2;      // per node: offset of its k x k slot (k of its level)
  std::vector<int64_t> nk;       // per node: offset of its length-k slot
  std::vector<int64_t> stoff;    // per node (as parent): offset of its stack (nch*k_l x k_{l-1})
  std::vector<std::vector<int64_t>> kids;
  int64_t tot_k2 = 0, tot_k = 0, tot_stack = 0;
  std::vector<int64_t> bl_t, bl_s, bl_lvl, bl_soff;  // per coupling block
  const double* S = nullptr;     // coupling blocks (device)
  double* So = nullptr;          // orthogonalized coupling blocks
  int64_t m(int64_t c) const { return P.hi[c] - P.lo[c]; }
};

int launch_eigs(Ctx& C, const std::vector<EigTask>& tasks) {
  if (tasks.empty()) return H2_OK;
  int nmax = 0;
  for (const EigTask& t : tasks) nmax = std::max(nmax, t.n);
  EigTask* d = nullptr;
  RC(C.ar.upload(tasks, &d, C.s));
  CK(launch_eig(d, (int64_t)tasks.size(), nmax, C.s), "eigensolver");
  return H2_OK;
}

template <class T>
int launch_tasks(Ctx& C, const std::vector<T>& tasks, hipError_t (*fn)(const T*, int64_t, hipStream_t)) {
  if (tasks.empty()) return H2_OK;
  T* d = nullptr;
  RC(C.ar.upload(tasks, &d, C.s));
  CK(fn(d, (int64_t)tasks.size(), C.s), "compression kernel");
  return H2_OK;
}

int launch_gemm_tasks(Ctx& C, const std::vector<GemmTask>& tasks, const std::vector<GemmPair>& pairs) {
  if (tasks.empty()) return H2_OK;
  int md = 1;
  for (const GemmTask& t : tasks) md = std::max(md, std::max(t.m, t.n));
  GemmTask* dt = nullptr;
  GemmPair* dp = nullptr;
  RC(C.ar.upload(tasks, &dt, C.s));
  RC(C.ar.upload(pairs, &dp, C.s));
  CK(launch_gemm(dt, (int64_t)tasks.size(), dp, C.s, md), "compression GEMM");
  return H2_OK;
}

int launch_triple_tasks(Ctx& C, const std::vector<TripleTask>& tasks) {
  if (tasks.empty()) return H2_OK;
  int md = 1;
  for (const TripleTask& t : tasks) md = std::max(md, std::max(std::max(t.a, t.b), t.k2));
  TripleTask* d = nullptr;
  RC(C.ar.upload(tasks, &d, C.s));
  CK(launch_triple(d, (int64_t)tasks.size(), C.s, md), "compression triple product");
  return H2_OK;
}

// checked task builders
int add_gemm(Ctx& C, std::vector<GemmTask>& tasks, double* Cm, int64_t ldc, int m, int n, double beta,
             const std::vector<GemmPair>& prs, std::vector<GemmPair>& pairs) {
  if (m > 64 || n > 64) return oob("GEMM tile");
  if (!C.ar.inside(Cm, m, n, ldc)) return oob("GEMM output");
  for (const GemmPair& p : prs) {
    const int64_t ar = (p.flags & 1) ? p.k : m, ac = (p.flags & 1) ? m : p.k;
    const int64_t br = (p.flags & 2) ? n : p.k, bc = (p.flags & 2) ? p.k : n;
    if (!C.ar.inside(p.A, ar, ac, p.lda) || !C.ar.inside(p.B, br, bc, p.ldb)) return oob("GEMM operand");
  }
  GemmTask t{Cm, ldc, 1.0, beta, m, n, (int32_t)pairs.size(), (int32_t)(pairs.size() + prs.size())};
  pairs.insert(pairs.end(), prs.begin(), prs.end());
  tasks.push_back(t);
  return H2_OK;
}

int add_triple(Ctx& C, std::vector<TripleTask>& tasks, const TripleTask& t) {
  if (t.a > 64 || t.b > 64 || t.k1 > 64 || t.k2 > 64) return oob("triple tile");
  if (!C.ar.inside(t.L, t.a, t.k1, t.ldl) || !C.ar.inside(t.M, t.k1, t.k2, t.ldm) ||
      !C.ar.inside(t.R, t.b, t.k2, t.ldr) || !C.ar.inside(t.C, t.a, t.b, t.ldc))
    return oob("triple operand");
  tasks.push_back(t);
  return H2_OK;
}

int add_eig(Ctx& C, std::vector<EigTask>& tasks, const double* G, int64_t ldg, double* lam, double* Z,
            int64_t ldz, int n) {
  if (n > kMaxCompressRank) return oob("eigenproblem order");
  if (!C.ar.inside(G, n, n, ldg) || !C.ar.inside(lam, n, 1, n) || !C.ar.inside(Z, n, n, ldz)) return oob("eig");
  tasks.push_back(EigTask{G, ldg, lam, Z, ldz, n, 0});
  return H2_OK;
}

int add_copy(Ctx& C, std::vector<CopyTask>& tasks, const double* src, int64_t lds, double* dst, int64_t ldd,
             int rows, int cols, bool trans) {
  if (!C.ar.inside(dst, rows, cols, ldd) ||
      !C.ar.inside(src, trans ? cols : rows, trans ? rows : cols, lds))
    return oob("copy");
  tasks.push_back(CopyTask{src, dst, lds, ldd, rows, cols, trans ? 1 : 0, 0});
  return H2_OK;
}

const double* transfer(const Ctx& C, const Tree& X, const double* base, int64_t c) {
  const int64_t l = C.lvl[c];
  return base + (*X.tbase)[l] + (c - C.P.level_ptr[l]) * X.k[l] * X.k[l - 1];
}

// ---- step 1: orthogonalization (QR upsweep) of one basis tree
int orthogonalize(Ctx& C, Tree& X) {
  const Parsed& P = C.P;
  const int64_t q = P.q, kq = X.k[q];
  std::vector<QrTask> qr;
  for (int64_t t = P.leaf0; t < P.nnodes; ++t) {
    const int64_t mt = C.m(t);
    if (mt * kq > kQrMaxElems) { set_error("recompression: leaf size times rank above 8192"); return H2_EUNSUPPORTED; }
    const double* A = X.B + P.lo[t] * kq;
    double* Q = X.Bo + P.lo[t] * kq;
    double* R = X.R + C.nk2[t];
    if (!C.ar.inside(A, mt, kq, std::max<int64_t>(mt, 1)) || !C.ar.inside(Q, mt, kq, std::max<int64_t>(mt, 1)) ||
        !C.ar.inside(R, kq, kq, kq))
      return oob("leaf QR");
    qr.push_back(QrTask{A, std::max<int64_t>(mt, 1), Q, std::max<int64_t>(mt, 1), R, std::max<int64_t>(kq, 1),
                        (int32_t)mt, (int32_t)kq});
  }
  RC(launch_tasks(C, qr, launch_qr));
  for (int64_t l = q; l >= 1; --l) {
    const int64_t kl = X.k[l], kp = X.k[l - 1];
    std::vector<GemmTask> gt;
    std::vector<GemmPair> gp;
    std::vector<QrTask> qt;
    std::vector<CopyTask> ct;
    for (int64_t p = P.level_ptr[l - 1]; p < P.level_ptr[l]; ++p) {
      const auto& ch = C.kids[p];
      const int64_t rows = (int64_t)ch.size() * kl;
      if (rows * kp > kQrMaxElems) { set_error("recompression: transfer stack above 8192 elements"); return H2_EUNSUPPORTED; }
      double* st = X.stack + C.stoff[p];
      const int64_t ld = std::max<int64_t>(rows, 1);
      for (size_t i = 0; i < ch.size(); ++i) {
        if (kl == 0 || kp == 0) break;
        const int64_t c = ch[i];
        RC(add_gemm(C, gt, st + i * kl, ld, (int)kl, (int)kp, 0.0,
                    {GemmPair{X.R + C.nk2[c], transfer(C, X, X.T, c), kl, kl, (int32_t)kl, 0}}, gp));
        RC(add_copy(C, ct, st + i * kl, ld, const_cast<double*>(transfer(C, X, X.To, c)), kl, (int)kl, (int)kp,
                    false));
      }
      if (!C.ar.inside(st, rows, kp, ld) || !C.ar.inside(X.R + C.nk2[p], kp, kp, std::max<int64_t>(kp, 1)))
        return oob("stack QR");
      qt.push_back(QrTask{st, ld, st, ld, X.R + C.nk2[p], std::max<int64_t>(kp, 1), (int32_t)rows, (int32_t)kp});
    }
    RC(launch_gemm_tasks(C, gt, gp));
    RC(launch_tasks(C, qt, launch_qr));
    RC(launch_tasks(C, ct, launch_copy));
  }
  return H2_OK;
}

// ---- So = R_t S R_s^T for every coupling block
int transform_coupling(Ctx& C, const Tree& Xr, const Tree& Xc) {
  std::vector<TripleTask> tt;
  tt.reserve(C.bl_t.size());
  for (size_t b = 0; b < C.bl_t.size(); ++b) {
    const int64_t l = C.bl_lvl[b], kr = Xr.k[l], kc = Xc.k[l];
    if (kr == 0 || kc == 0) continue;
    TripleTask t{};
    t.L = Xr.R + C.nk2[C.bl_t[b]]; t.ldl = kr;
    t.M = C.S + C.bl_soff[b]; t.ldm = kr;
    t.R = Xc.R + C.nk2[C.bl_s[b]]; t.ldr = kc;
    t.C = C.So + C.bl_soff[b]; t.ldc = kr;
    t.a = (int32_t)kr; t.k1 = (int32_t)kr; t.k2 = (int32_t)kc; t.b = (int32_t)kc;
    t.beta = 0.0;
    RC(add_triple(C, tt, t));
  }
  return launch_triple_tasks(C, tt);
}

// ---- step 2: Gram matrices of the block rows (own blocks), then the downsweep
int reweight(Ctx& C, Tree& X, bool rows, bool cols) {
  const Parsed& P = C.P;
  std::vector<std::vector<GemmPair>> own(P.nnodes);
  for (size_t b = 0; b < C.bl_t.size(); ++b) {
    const int64_t l = C.bl_lvl[b];
    const int64_t kr = P.krow[l], kc = P.kcol[l];
    if (kr == 0 || kc == 0) continue;
    const double* Sb = C.So + C.bl_soff[b];
    if (rows) own[C.bl_t[b]].push_back(GemmPair{Sb, Sb, kr, kr, (int32_t)kc, 2});  // S S^T
    if (cols) own[C.bl_s[b]].push_back(GemmPair{Sb, Sb, kr, kr, (int32_t)kr, 1});  // S^T S
  }
  std::vector<GemmTask> gt;
  std::vector<GemmPair> gp;
  for (int64_t i = 0; i < P.nnodes; ++i) {
    const int64_t k = X.k[C.lvl[i]];
    if (k == 0) continue;
    RC(add_gemm(C, gt, X.G + C.nk2[i], k, (int)k, (int)k, 0.0, own[i], gp));
  }
  RC(launch_gemm_tasks(C, gt, gp));
  for (int64_t l = 1; l <= P.q; ++l) {
    const int64_t kl = X.k[l], kp = X.k[l - 1];
    if (kl == 0 || kp == 0) continue;
    std::vector<TripleTask> tt;
    for (int64_t i = P.level_ptr[l]; i < P.level_ptr[l + 1]; ++i) {
      const double* E = transfer(C, X, X.To, i);
      TripleTask t{};
      t.L = E; t.ldl = kl;
      t.M = X.G + C.nk2[P.parent[i]]; t.ldm = kp;
      t.R = E; t.ldr = kl;
      t.C = X.G + C.nk2[i]; t.ldc = kl;
      t.a = (int32_t)kl; t.k1 = (int32_t)kp; t.k2 = (int32_t)kp; t.b = (int32_t)kl;
      t.beta = 1.0;
      RC(add_triple(C, tt, t));
    }
    RC(launch_triple_tasks(C, tt));
  }
  return H2_OK;
}

int read_counts(Ctx& C, const Tree& X, int64_t l, int64_t* kmax) {
  const int64_t b = C.P.level_ptr[l], e = C.P.level_ptr[l + 1];
  std::vector<int32_t> cnt((size_t)(e - b));
  if (e > b)
    CK(hipMemcpyAsync(cnt.data(), X.counts + b, sizeof(int32_t) * (e - b), hipMemcpyDeviceToHost, C.s),
       "download counts");
  CK(hipStreamSynchronize(C.s), "hipStreamSynchronize");
  *kmax = 0;
  for (int32_t c : cnt) *kmax = std::max<int64_t>(*kmax, c);
  return H2_OK;
}

// ---- step 3, one level of parents (level l-1) when every stacked rank
// n_p = children * k'_l is at most 64: the left singular vectors of
// M = N_p R_p^T are the eigenvectors of M M^T = N_p G_p N_p^T (order n_p)
int truncate_level_direct(Ctx& C, Tree& X, int64_t l, double thr2) {
  const Parsed& P = C.P;
  const int64_t kl = X.k[l], kp = X.k[l - 1], kln = X.knew[l];
  const int64_t b0 = P.level_ptr[l - 1], b1 = P.level_ptr[l];
  // per parent: n_p x n_p Gram matrix and eigenvectors, n_p eigenvalues
  std::vector<int64_t> off(b1 - b0 + 1, 0);
  for (int64_t p = b0; p < b1; ++p) {
    const int64_t np = (int64_t)C.kids[p].size() * kln;
    off[p - b0 + 1] = off[p - b0] + np * np;
  }
  double *Dg = nullptr, *Dz = nullptr, *Dl = nullptr;
  RC(C.ar.alloc(&Dg, off.back(), C.s));
  RC(C.ar.alloc(&Dz, off.back(), C.s));
  RC(C.ar.alloc(&Dl, (b1 - b0) * kMaxCompressRank, C.s));
  std::vector<GemmTask> g1;
  std::vector<GemmPair> p1;
  std::vector<TripleTask> tt;
  std::vector<EigTask> et;
  std::vector<CountTask> cnt;
  std::vector<ScaleTask> sc;
  for (int64_t p = b0; p < b1; ++p) {
    const auto& ch = C.kids[p];
    const int64_t np = (int64_t)ch.size() * kln, ldn = std::max<int64_t>(np, 1);
    if (np == 0) continue;
    double* N = X.stack + C.stoff[p];
    // N_p = [T_c E_c] (np x kp)
    for (size_t i = 0; i < ch.size() && kl > 0; ++i) {
      const int64_t c = ch[i];
      RC(add_gemm(C, g1, N + i * kln, ldn, (int)kln, (int)kp, 0.0,
                  {GemmPair{X.Tt + C.nk2[c], transfer(C, X, X.To, c), kln, kl, (int32_t)kl, 0}}, p1));
    }
    // N_p G_p N_p^T
    TripleTask t{};
    t.L = N; t.ldl = ldn;
    t.M = X.G + C.nk2[p]; t.ldm = kp;
    t.R = N; t.ldr = ldn;
    t.C = Dg + off[p - b0]; t.ldc = np;
    t.a = (int32_t)np; t.k1 = (int32_t)kp; t.k2 = (int32_t)kp; t.b = (int32_t)np;
    t.beta = 0.0;
    RC(add_triple(C, tt, t));
    double* lam = Dl + (p - b0) * kMaxCompressRank;
    RC(add_eig(C, et, Dg + off[p - b0], np, lam, Dz + off[p - b0], np, (int)np));
    // N G N^T has rank at most kp: only its kp leading eigenvalues can be kept
    cnt.push_back(CountTask{lam, (int32_t)std::min(np, kp), (int32_t)p});
    sc.push_back(ScaleTask{Dz + off[p - b0], np, lam, (int32_t)np, (int32_t)np, (int32_t)p, 0});
  }
  RC(launch_gemm_tasks(C, g1, p1));
  RC(launch_triple_tasks(C, tt));
  RC(launch_eigs(C, et));
  if (!cnt.empty()) {
    CountTask* d = nullptr;
    RC(C.ar.upload(cnt, &d, C.s));
    CK(launch_count(d, (int64_t)cnt.size(), thr2, X.counts, C.s), "count");
  }
  RC(read_counts(C, X, l - 1, &X.knew[l - 1]));
  const int64_t kpn = X.knew[l - 1];
  if (!sc.empty()) {
    ScaleTask* d = nullptr;
    RC(C.ar.upload(sc, &d, C.s));
    CK(launch_scale_cols(d, (int64_t)sc.size(), X.counts, 0, C.s), "scale");
  }
  if (kpn == 0) return H2_OK;
  // E'_c = rows of child c of W[:, :kpn]; T_p = W[:, :kpn]^T N_p (kpn x kp).
  // W has only n_p columns: where n_p < kpn the rest of E'_c and of T_p are
  // the zero padding the arena starts with.
  std::vector<CopyTask> ct;
  std::vector<GemmTask> g2;
  std::vector<GemmPair> p2;
  for (int64_t p = b0; p < b1; ++p) {
    const auto& ch = C.kids[p];
    const int64_t np = (int64_t)ch.size() * kln, ldn = std::max<int64_t>(np, 1);
    if (np == 0) continue;
    const int64_t kw = std::min(kpn, np);
    const double* W = Dz + off[p - b0];
    for (size_t i = 0; i < ch.size(); ++i)
      RC(add_copy(C, ct, W + i * kln, np, const_cast<double*>(transfer(C, X, X.Et, ch[i])), kln, (int)kln, (int)kw,
                  false));
    RC(add_gemm(C, g2, X.Tt + C.nk2[p], kpn, (int)kw, (int)kp, 0.0,
                {GemmPair{W, X.stack + C.stoff[p], np, ldn, (int32_t)np, 1}}, p2));
  }
  RC(launch_tasks(C, ct, launch_copy));
  RC(launch_gemm_tasks(C, g2, p2));
  return H2_OK;
}

// ---- step 3: truncation upsweep of one tree
int truncate(Ctx& C, Tree& X, double tau) {
  const Parsed& P = C.P;
  const int64_t q = P.q, kq = X.k[q];
  X.knew.assign(q + 1, 0);
  std::vector<CountTask> leaf_counts;
  // leaves: eigenpairs of P G P
  {
    std::vector<MaskTask> mt;
    std::vector<EigTask> et;
    for (int64_t t = P.leaf0; t < P.nnodes; ++t) {
      if (kq == 0) break;
      const int64_t mtt = C.m(t);
      const double* U = X.Bo + P.lo[t] * kq;
      if (!C.ar.inside(U, mtt, kq, std::max<int64_t>(mtt, 1)) || !C.ar.inside(X.G + C.nk2[t], kq, kq, kq) ||
          !C.ar.inside(X.W + C.nk2[t], kq, kq, kq))
        return oob("mask");
      mt.push_back(MaskTask{U, std::max<int64_t>(mtt, 1), X.G + C.nk2[t], kq, X.W + C.nk2[t], (int32_t)mtt,
                            (int32_t)kq});
      RC(add_eig(C, et, X.W + C.nk2[t], kq, X.lam + C.nk[t], X.Z + C.nk2[t], kq, (int)kq));
      leaf_counts.push_back(CountTask{X.lam + C.nk[t], (int32_t)kq, (int32_t)t});
    }
    RC(launch_tasks(C, mt, launch_mask_gram));
    RC(launch_eigs(C, et));
  }
  double sref2 = 0.0;
  if (!leaf_counts.empty()) {
    CountTask* d = nullptr;
    RC(C.ar.upload(leaf_counts, &d, C.s));
    CK(launch_max_lead(d, (int64_t)leaf_counts.size(), X.sref2, C.s), "max eigenvalue");
    CK(hipMemcpyAsync(&sref2, X.sref2, sizeof(double), hipMemcpyDeviceToHost, C.s), "download");
    CK(hipStreamSynchronize(C.s), "hipStreamSynchronize");
  }
  X.sigma_ref = std::sqrt(std::max(sref2, 0.0));
  const double thr2 = tau * tau * std::max(sref2, 0.0);
  if (!leaf_counts.empty()) {
    CountTask* d = nullptr;
    RC(C.ar.upload(leaf_counts, &d, C.s));
    CK(launch_count(d, (int64_t)leaf_counts.size(), thr2, X.counts, C.s), "count");
  }
  RC(read_counts(C, X, q, &X.knew[q]));
  const int64_t kn = X.knew[q];
  {
    std::vector<ScaleTask> sc;
    std::vector<GemmTask> gt;
    std::vector<GemmPair> gp;
    std::vector<CopyTask> ct;
    for (int64_t t = P.leaf0; t < P.nnodes && kq > 0 && kn > 0; ++t) {
      const int64_t mtt = C.m(t);
      double* Z = X.Z + C.nk2[t];
      sc.push_back(ScaleTask{Z, kq, X.lam + C.nk[t], (int32_t)kq, (int32_t)kq, (int32_t)t, 0});
      for (int64_t r0 = 0; r0 < mtt; r0 += 64) {
        const int rows = (int)std::min<int64_t>(64, mtt - r0);
        RC(add_gemm(C, gt, X.Bn + P.lo[t] * kn + r0, mtt, rows, (int)kn, 0.0,
                    {GemmPair{X.Bo + P.lo[t] * kq + r0, Z, mtt, kq, (int32_t)kq, 0}}, gp));
      }
      RC(add_copy(C, ct, Z, kq, X.Tt + C.nk2[t], kn, (int)kn, (int)kq, true));
    }
    if (!sc.empty()) {
      ScaleTask* d = nullptr;
      RC(C.ar.upload(sc, &d, C.s));
      CK(launch_scale_cols(d, (int64_t)sc.size(), X.counts, 0, C.s), "scale");
    }
    RC(launch_gemm_tasks(C, gt, gp));
    RC(launch_tasks(C, ct, launch_copy));
  }
  // inner levels, parents on level l-1
  for (int64_t l = q; l >= 1; --l) {
    const int64_t kl = X.k[l], kp = X.k[l - 1], kln = X.knew[l];
    int64_t npmax = 0;
    for (int64_t p = P.level_ptr[l - 1]; p < P.level_ptr[l]; ++p)
      npmax = std::max<int64_t>(npmax, (int64_t)C.kids[p].size() * kln);
    if (kp > 0 && npmax <= kMaxCompressRank) {
      RC(truncate_level_direct(C, X, l, thr2));
      continue;
    }
    std::vector<GemmTask> g1, g2, g3;
    std::vector<GemmPair> p1, p2, p3;
    std::vector<EigTask> e1, e2;
    std::vector<double*> sq_out;
    std::vector<int64_t> sq_ld;
    std::vector<CountTask> cnt;
    std::vector<ScaleTask> sc;
    for (int64_t p = P.level_ptr[l - 1]; p < P.level_ptr[l]; ++p) {
      if (kp == 0) continue;
      const auto& ch = C.kids[p];
      const int64_t np = (int64_t)ch.size() * kln, ldn = std::max<int64_t>(np, 1);
      double* N = X.stack + C.stoff[p];
      double* M = X.Mb + C.stoff[p];
      // N_p = [T_c E_c] (np x kp)
      for (size_t i = 0; i < ch.size() && kln > 0 && kl > 0; ++i) {
        const int64_t c = ch[i];
        RC(add_gemm(C, g1, N + i * kln, ldn, (int)kln, (int)kp, 0.0,
                    {GemmPair{X.Tt + C.nk2[c], transfer(C, X, X.To, c), kln, kl, (int32_t)kl, 0}}, p1));
      }
      // eig(G_p) -> R_p = diag(sqrt(lam)) Z^T (in X.R)
      RC(add_eig(C, e1, X.G + C.nk2[p], kp, X.lam2 + C.nk[p], X.Y + C.nk2[p], kp, (int)kp));
      sq_out.push_back(X.R + C.nk2[p]);
      sq_ld.push_back(kp);
      // M_p = N_p R_p^T, K_p = M_p^T M_p (in X.W)
      for (int64_t r0 = 0; r0 < np; r0 += 64) {
        const int rows = (int)std::min<int64_t>(64, np - r0);
        RC(add_gemm(C, g2, M + r0, ldn, rows, (int)kp, 0.0,
                    {GemmPair{N + r0, X.R + C.nk2[p], ldn, kp, (int32_t)kp, 2}}, p2));
      }
      std::vector<GemmPair> kp_pairs;
      if (np > 0) kp_pairs.push_back(GemmPair{M, M, ldn, ldn, (int32_t)np, 1});
      RC(add_gemm(C, g3, X.W + C.nk2[p], kp, (int)kp, (int)kp, 0.0, kp_pairs, p3));
      RC(add_eig(C, e2, X.W + C.nk2[p], kp, X.lam + C.nk[p], X.Z + C.nk2[p], kp, (int)kp));
      cnt.push_back(CountTask{X.lam + C.nk[p], (int32_t)kp, (int32_t)p});
      sc.push_back(ScaleTask{X.Z + C.nk2[p], kp, X.lam + C.nk[p], (int32_t)kp, (int32_t)kp, (int32_t)p, 0});
    }
    RC(launch_gemm_tasks(C, g1, p1));
    RC(launch_eigs(C, e1));
    if (!e1.empty()) {
      EigTask* de = nullptr;
      double** dout = nullptr;
      int64_t* dld = nullptr;
      RC(C.ar.upload(e1, &de, C.s));
      RC(C.ar.upload(sq_out, &dout, C.s));
      RC(C.ar.upload(sq_ld, &dld, C.s));
      CK(launch_sqrt_factor(de, (int64_t)e1.size(), dout, dld, C.s), "square-root factor");
    }
    RC(launch_gemm_tasks(C, g2, p2));
    RC(launch_gemm_tasks(C, g3, p3));
    RC(launch_eigs(C, e2));
    if (!cnt.empty()) {
      CountTask* d = nullptr;
      RC(C.ar.upload(cnt, &d, C.s));
      CK(launch_count(d, (int64_t)cnt.size(), thr2, X.counts, C.s), "count");
    }
    RC(read_counts(C, X, l - 1, &X.knew[l - 1]));
    const int64_t kpn = X.knew[l - 1];
    if (!sc.empty()) {
      ScaleTask* d = nullptr;
      RC(C.ar.upload(sc, &d, C.s));
      CK(launch_scale_cols(d, (int64_t)sc.size(), X.counts, 1, C.s), "scale");
    }
    // E'_c = M_p[rows of c] Y_p[:, :kpn]  (in the old slot of E_c, ld kln)
    // T_p = sum_c E'_c^T N_p[rows of c]  (kpn x kp)
    std::vector<GemmTask> g4, g5;
    std::vector<GemmPair> p4, p5;
    for (int64_t p = P.level_ptr[l - 1]; p < P.level_ptr[l] && kp > 0 && kpn > 0; ++p) {
      const auto& ch = C.kids[p];
      const int64_t np = (int64_t)ch.size() * kln, ldn = std::max<int64_t>(np, 1);
      const double* N = X.stack + C.stoff[p];
      const double* M = X.Mb + C.stoff[p];
      std::vector<GemmPair> tp;
      for (size_t i = 0; i < ch.size() && kln > 0; ++i) {
        const int64_t c = ch[i];
        double* Ec = const_cast<double*>(transfer(C, X, X.Et, c));
        RC(add_gemm(C, g4, Ec, kln, (int)kln, (int)kpn, 0.0,
                    {GemmPair{M + i * kln, X.Z + C.nk2[p], ldn, kp, (int32_t)kp, 0}}, p4));
        tp.push_back(GemmPair{Ec, N + i * kln, kln, ldn, (int32_t)kln, 1});
      }
      RC(add_gemm(C, g5, X.Tt + C.nk2[p], kpn, (int)kpn, (int)kp, 0.0, tp, p5));
    }
    RC(launch_gemm_tasks(C, g4, p4));
    RC(launch_gemm_tasks(C, g5, p5));
  }
  return H2_OK;
}

void align64(int64_t* pos) { *pos = (*pos + 63) / 64 * 64; }

// section sizes (elements) of a representation with ranks kr, kc
struct Sizes {
  int64_t U, E, V, F, S;
};
Sizes sizes_of(const Parsed& P, const std::vector<int64_t>& kr, const std::vector<int64_t>& kc, bool sep) {
  Sizes z{0, 0, 0, 0, 0};
  z.U = P.n * kr[P.q];
  z.V = sep ? P.n * kc[P.q] : 0;
  for (int64_t l = 1; l <= P.q; ++l) {
    const int64_t nl = P.level_ptr[l + 1] - P.level_ptr[l];
    z.E += nl * kr[l] * kr[l - 1];
    if (sep) z.F += nl * kc[l] * kc[l - 1];
  }
  for (int64_t l = 0; l <= P.q; ++l) z.S += P.nadm[l] * kr[l] * kc[l];
  return z;
}

int compress_impl(h2_op_s* h, double tau, hipStream_t s, h2_handle* out, h2_compress_info_t* info) {
  hipEvent_t ev[6] = {};
  for (auto& e : ev) CK(hipEventCreate(&e), "hipEventCreate");
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 6; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } eg{ev};
  Ctx C;
  C.h = h;
  C.s = s;
  {
    const int prc = parse(reinterpret_cast<const uint8_t*>(h->prefix.data()), h->file_len, &C.P);
    if (prc != H2_OK) {
      set_error("recompression: the operator's stored structure does not parse (" + std::string(h2_last_error()) +
                ")");
      return prc;
    }
  }
  const Parsed& P = C.P;
  const int64_t q = P.q;
  const bool sep = (P.flags & 1u) != 0;
  for (int64_t l = 0; l <= q; ++l)
    if (P.krow[l] > kMaxCompressRank || P.kcol[l] > kMaxCompressRank) {
      set_error("recompression: ranks above 64 are not supported");
      return H2_EUNSUPPORTED;
    }
  // structure
  C.lvl.resize(P.nnodes);
  for (int64_t l = 0; l <= q; ++l)
    for (int64_t c = P.level_ptr[l]; c < P.level_ptr[l + 1]; ++c) C.lvl[c] = l;
  C.kids.assign(P.nnodes, {});
  for (int64_t c = 1; c < P.nnodes; ++c) C.kids[P.parent[c]].push_back(c);
  const int64_t kmaxl = *std::max_element(P.krow, P.krow + q + 1);
  const int64_t kmaxc = *std::max_element(P.kcol, P.kcol + q + 1);
  const int64_t kmx = std::max(kmaxl, kmaxc);
  C.nk2.resize(P.nnodes);
  C.nk.resize(P.nnodes);
  C.stoff.assign(P.nnodes, 0);
  for (int64_t c = 0; c < P.nnodes; ++c) {
    const int64_t k = std::max(P.krow[C.lvl[c]], P.kcol[C.lvl[c]]);
    C.nk2[c] = C.tot_k2;
    C.tot_k2 += k * k;
    C.nk[c] = C.tot_k;
    C.tot_k += k;
    if (C.lvl[c] < q) {
      const int64_t rows = (int64_t)C.kids[c].size() * kmx;
      C.stoff[c] = C.tot_stack;
      C.tot_stack += rows * kmx;
    }
  }
  for (int64_t l = 0; l <= q; ++l) {
    const int64_t nl = P.level_ptr[l + 1] - P.level_ptr[l];
    const int64_t sz = P.krow[l] * P.kcol[l];
    for (int64_t ti = 0; ti < nl; ++ti)
      for (int64_t b = P.s_rowptr[P.rp_base[l] + ti]; b < P.s_rowptr[P.rp_base[l] + ti + 1]; ++b) {
        const int64_t gb = P.blk_base[l] + b;
        C.bl_t.push_back(P.level_ptr[l] + ti);
        C.bl_s.push_back(P.level_ptr[l] + P.s_col[gb]);
        C.bl_lvl.push_back(l);
        C.bl_soff.push_back(P.sdat[l] + b * sz);
      }
  }
  // device views of the operator's data
  const double* base = h->d_mat;
  const int64_t oE = (P.off_E - P.off_U) / 8, oV = (P.off_V - P.off_U) / 8, oF = (P.off_F - P.off_U) / 8,
                oS = (P.off_S - P.off_U) / 8;
  C.ar.reg(h->d_mat, (size_t)(P.off_end - P.off_U));
  C.S = base + oS;
  Sizes old = sizes_of(P, std::vector<int64_t>(P.krow, P.krow + q + 1), std::vector<int64_t>(P.kcol, P.kcol + q + 1),
                       sep);
  RC(C.ar.alloc(&C.So, old.S, s));
  Tree Xr, Xc;
  Xr.k = P.krow; Xr.B = base; Xr.T = base + oE; Xr.tbase = &P.ebase;
  Xc.k = P.kcol; Xc.B = base + oV; Xc.T = base + oF; Xc.tbase = &P.fbase;
  auto alloc_tree = [&](Tree& X, int64_t nB, int64_t nT) -> int {
    RC(C.ar.alloc(&X.Bo, nB, s)); RC(C.ar.alloc(&X.To, nT, s)); RC(C.ar.alloc(&X.Et, nT, s));
    RC(C.ar.alloc(&X.R, C.tot_k2, s)); RC(C.ar.alloc(&X.G, C.tot_k2, s)); RC(C.ar.alloc(&X.W, C.tot_k2, s));
    RC(C.ar.alloc(&X.Z, C.tot_k2, s)); RC(C.ar.alloc(&X.Y, C.tot_k2, s)); RC(C.ar.alloc(&X.Tt, C.tot_k2, s));
    RC(C.ar.alloc(&X.lam, C.tot_k, s)); RC(C.ar.alloc(&X.lam2, C.tot_k, s));
    RC(C.ar.alloc(&X.stack, C.tot_stack, s)); RC(C.ar.alloc(&X.Mb, C.tot_stack, s));
    RC(C.ar.alloc(&X.counts, P.nnodes, s)); RC(C.ar.alloc(&X.sref2, 1, s));
    return H2_OK;
  };
  RC(alloc_tree(Xr, old.U, old.E));
  if (sep) RC(alloc_tree(Xc, old.V, old.F));
  Tree& Xcol = sep ? Xc : Xr;
  CK(hipEventRecord(ev[0], s), "hipEventRecord");
  // 1. orthogonalize, transform the coupling blocks
  RC(orthogonalize(C, Xr));
  if (sep) RC(orthogonalize(C, Xc));
  RC(transform_coupling(C, Xr, Xcol));
  CK(hipEventRecord(ev[1], s), "hipEventRecord");
  // 2. reweighting
  RC(reweight(C, Xr, true, !sep));
  if (sep) RC(reweight(C, Xc, false, true));
  CK(hipEventRecord(ev[2], s), "hipEventRecord");
  // 3. truncation (leaf bases go straight to their final arrays)
  // new leaf bases need k'_q: allocated inside truncate's first step
  {
    // upper bound allocation for the new leaf bases (k' <= k)
    RC(C.ar.alloc(&Xr.Bn, old.U, s));
    if (sep) RC(C.ar.alloc(&Xc.Bn, old.V, s));
  }
  RC(truncate(C, Xr, tau));
  if (sep) RC(truncate(C, Xc, tau));
  CK(hipEventRecord(ev[3], s), "hipEventRecord");
  // 4. projection S'_ts = T_t So_ts T_s^T and packing of the transfers
  std::vector<int64_t> kr = Xr.knew, kc = sep ? Xc.knew : Xr.knew;
  Sizes nw = sizes_of(P, kr, kc, sep);
  double *Sn = nullptr, *En = nullptr, *Fn = nullptr;
  RC(C.ar.alloc(&Sn, nw.S, s));
  RC(C.ar.alloc(&En, nw.E, s));
  if (sep) RC(C.ar.alloc(&Fn, nw.F, s));
  std::vector<int64_t> sdn(q + 2, 0), ebn(q + 2, 0), fbn(q + 2, 0);
  for (int64_t l = 0; l <= q; ++l) {
    sdn[l + 1] = sdn[l] + P.nadm[l] * kr[l] * kc[l];
    const int64_t nl = P.level_ptr[l + 1] - P.level_ptr[l];
    ebn[l + 1] = ebn[l] + (l >= 1 ? nl * kr[l] * kr[l - 1] : 0);
    fbn[l + 1] = fbn[l] + (l >= 1 ? nl * kc[l] * kc[l - 1] : 0);
  }
  {
    std::vector<TripleTask> tt;
    for (size_t b = 0; b < C.bl_t.size(); ++b) {
      const int64_t l = C.bl_lvl[b];
      if (kr[l] == 0 || kc[l] == 0) continue;
      const int64_t i = (C.bl_soff[b] - P.sdat[l]) / (P.krow[l] * P.kcol[l]);
      TripleTask t{};
      t.L = Xr.Tt + C.nk2[C.bl_t[b]]; t.ldl = kr[l];
      t.M = C.So + C.bl_soff[b]; t.ldm = P.krow[l];
      t.R = Xcol.Tt + C.nk2[C.bl_s[b]]; t.ldr = kc[l];
      t.C = Sn + sdn[l] + i * kr[l] * kc[l]; t.ldc = kr[l];
      t.a = (int32_t)kr[l]; t.k1 = (int32_t)P.krow[l]; t.k2 = (int32_t)P.kcol[l]; t.b = (int32_t)kc[l];
      t.beta = 0.0;
      RC(add_triple(C, tt, t));
    }
    RC(launch_triple_tasks(C, tt));
    std::vector<CopyTask> ct;
    for (int64_t l = 1; l <= q; ++l) {
      for (int64_t c = P.level_ptr[l]; c < P.level_ptr[l + 1]; ++c) {
        const int64_t j = c - P.level_ptr[l];
        if (kr[l] > 0 && kr[l - 1] > 0)
          RC(add_copy(C, ct, transfer(C, Xr, Xr.Et, c), kr[l], En + ebn[l] + j * kr[l] * kr[l - 1], kr[l],
                      (int)kr[l], (int)kr[l - 1], false));
        if (sep && kc[l] > 0 && kc[l - 1] > 0)
          RC(add_copy(C, ct, transfer(C, Xc, Xc.Et, c), kc[l], Fn + fbn[l] + j * kc[l] * kc[l - 1], kc[l],
                      (int)kc[l], (int)kc[l - 1], false));
      }
    }
    RC(launch_tasks(C, ct, launch_copy));
  }
  CK(hipEventRecord(ev[4], s), "hipEventRecord");
  CK(hipStreamSynchronize(s), "hipStreamSynchronize");
  // 5. the new representation: header and index sections with the new
  // ranks, low-rank sections downloaded, dense blocks copied on the device
  const int64_t pre = h->prefix_len;
  std::vector<int64_t> offs(6, 0);  // U E V F S D
  int64_t pos = pre;
  const int64_t cnts[5] = {nw.U, nw.E, nw.V, nw.F, nw.S};
  for (int i = 0; i < 5; ++i) {
    align64(&pos);
    offs[i] = pos;
    pos += 8 * cnts[i];
  }
  align64(&pos);
  offs[5] = pos;
  const int64_t dbytes = P.off_end - P.off_D;
  int64_t total = pos + dbytes;
  align64(&total);
  std::vector<uint64_t> hb((size_t)(offs[5] + 7) / 8, 0);
  uint8_t* hbp = reinterpret_cast<uint8_t*>(hb.data());
  std::memcpy(hbp, h->prefix.data(), (size_t)pre);
  uint32_t flags = P.flags & ~2u;
  std::memcpy(hbp + 12, &flags, 4);
  const int64_t zero = 0;
  std::memcpy(hbp + 40, &zero, 8);   // dim: points are not carried over
  std::memcpy(hbp + 96, &total, 8);
  const uint8_t* pfx = reinterpret_cast<const uint8_t*>(h->prefix.data());
  std::memcpy(hbp + (reinterpret_cast<const uint8_t*>(P.krow) - pfx), kr.data(), 8 * (q + 1));
  std::memcpy(hbp + (reinterpret_cast<const uint8_t*>(P.kcol) - pfx), kc.data(), 8 * (q + 1));
  const double* srcs[5] = {Xr.Bn, En, sep ? Xc.Bn : nullptr, Fn, Sn};
  for (int i = 0; i < 5; ++i)
    if (cnts[i] > 0)
      CK(hipMemcpy(hbp + offs[i], srcs[i], 8 * cnts[i], hipMemcpyDeviceToHost), "download new representation");
  const double* d_dense = reinterpret_cast<const double*>(reinterpret_cast<const uint8_t*>(h->d_mat) +
                                                          (P.off_D - P.off_U));
  h2_handle nh = nullptr;
  const int rc = load_handle(hbp, total, h->device, d_dense, &nh);
  if (rc != H2_OK) {
    std::string msg = "recompression: the new representation does not load (" + std::string(h2_last_error()) +
                      "); ranks";
    for (int64_t l = 0; l <= q; ++l) msg += " " + std::to_string(kr[l]) + "/" + std::to_string(kc[l]);
    msg += "; level_ptr";
    for (int64_t l = 0; l <= q + 1 && l < 6; ++l) msg += " " + std::to_string(reinterpret_cast<const int64_t*>(hbp + 128)[l]);
    msg += "; sizes U " + std::to_string(nw.U) + " E " + std::to_string(nw.E) + " S " + std::to_string(nw.S) +
           " total " + std::to_string(total) + " prefix " + std::to_string(pre);
    set_error(msg);
    return rc;
  }
  CK(hipEventRecord(ev[5], nullptr), "hipEventRecord");
  CK(hipEventSynchronize(ev[5]), "hipEventSynchronize");
  if (info) {
    float t[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) CK(hipEventElapsedTime(&t[i], ev[i], ev[i + 1]), "hipEventElapsedTime");
    CK(hipEventElapsedTime(&t[4], ev[4], ev[5]), "hipEventElapsedTime");
    *info = h2_compress_info_t{};
    info->ms_orthogonalize = t[0];
    info->ms_reweight = t[1];
    info->ms_truncate = t[2];
    info->ms_project = t[3];
    info->ms_assemble = t[4];
    info->lowrank_entries_before = old.U + old.E + old.V + old.F + old.S;
    info->lowrank_entries_after = nw.U + nw.E + nw.V + nw.F + nw.S;
    info->sigma_ref_row = Xr.sigma_ref;
    info->sigma_ref_col = Xcol.sigma_ref;
  }
  *out = nh;
  return H2_OK;
}

}  // namespace
}  // namespace h2

using namespace h2;

extern "C" {

int h2_compress(h2_handle h, double tau, h2_handle* out, h2_compress_info_t* info, void* stream) {
  if (!h || !out) { set_error("null handle or output"); return H2_EINVAL; }
  *out = nullptr;
  if (!(tau >= 0.0 && tau < 1.0)) { set_error("tau must be in [0, 1)"); return H2_EINVAL; }
  if (h->prefix.empty()) { set_error("handle has no structure"); return H2_EINVAL; }
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(h->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return H2_EHIP;
  }
  int rc;
  try {
    rc = compress_impl(h, tau, static_cast<hipStream_t>(stream), out, info);
  } catch (const std::bad_alloc&) {
    set_error("out of host memory in recompression");
    rc = H2_ENOMEM;
  }
  (void)hipSetDevice(prev);
  return rc;
}

int h2_export(h2_handle h, void* buf, size_t cap, size_t* needed) {
  if (!h || !needed) { set_error("null handle or size output"); return H2_EINVAL; }
  Parsed P;
  int rc = parse(reinterpret_cast<const uint8_t*>(h->prefix.data()), h->file_len, &P);
  if (rc != H2_OK) return rc;
  int64_t total = P.off_end;
  total = (total + 63) / 64 * 64;
  *needed = (size_t)total;
  if (!buf) return H2_OK;
  if (cap < (size_t)total) { set_error("export buffer too small"); return H2_EINVAL; }
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(h->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return H2_EHIP;
  }
  uint8_t* b = static_cast<uint8_t*>(buf);
  std::memset(b, 0, (size_t)total);
  std::memcpy(b, h->prefix.data(), (size_t)h->prefix_len);
  uint32_t flags = P.flags & ~2u;
  std::memcpy(b + 12, &flags, 4);
  const int64_t zero = 0;
  std::memcpy(b + 40, &zero, 8);
  std::memcpy(b + 96, &total, 8);
  hipError_t e = hipSuccess;
  if (P.off_end > P.off_U) e = hipMemcpy(b + P.off_U, h->d_mat, P.off_end - P.off_U, hipMemcpyDeviceToHost);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return hfail(e, "hipMemcpy(export)");
  return H2_OK;
}

int h2_ranks(h2_handle h, int64_t* krow, int64_t* kcol, int64_t cap) {
  if (!h) { set_error("null handle"); return H2_EINVAL; }
  if (cap < h->q + 1 || !krow || !kcol) { set_error("rank arrays shorter than depth + 1"); return H2_EINVAL; }
  for (int64_t l = 0; l <= h->q; ++l) {
    krow[l] = h->lv[l].krow;
    kcol[l] = h->lv[l].kcol;
  }
  return H2_OK;
}

}  // extern "C"
