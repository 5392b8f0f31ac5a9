// h2_gemv_noalloc: the FP64 product of h2_gemv for callers that cannot
// allocate device memory.  Its scratch -- the tree-ordered input X~, the
// vector trees x^ and y^, and the dense partial Z, column-major with up to
// kPassVectors columns -- is a view of one fixed device array per GPU,
// declared below.  The array lives as long as the process; every call on a
// GPU reuses that GPU's copy, so calls that overlap on one GPU race.
//
// Host code never passes the array's name to a kernel or a copy: its device
// address is looked up once per device (scratch_attach, called by every
// h2_load on that device, with the device current) and only that address is
// used.
#include <mutex>
#include <string>
#include <vector>

#include "h2_internal.h"

namespace h2 {
namespace {

// 64 MiB: a pass of one vector needs 8 * (2 n + 2 H) bytes (n points, H
// tree rows), so operators with n + H up to 4 Mi rows fit (2^20 points at
// rank 36, H = 1.18 Mi, take passes of one vector).
constexpr int64_t kScratchBytes = int64_t(64) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
std::vector<double*> g_ptr;  // per device ordinal: device address of `scratch`

double* scratch_ptr(int device) {
  std::lock_guard<std::mutex> g(g_mu);
  return device >= 0 && device < (int)g_ptr.size() ? g_ptr[device] : nullptr;
}

// Bytes of one vector's pass: X~ and Z (n rows each), x^ (at least 8 rows)
// and y^ (H rows).
int64_t bytes_per_vector(int64_t n, int64_t H) {
  return (int64_t)sizeof(double) *
         (2 * std::max<int64_t>(n, 1) + std::max<int64_t>(H, 8) + std::max<int64_t>(H, 1));
}

}  // namespace

int scratch_attach(int device) {
  std::lock_guard<std::mutex> g(g_mu);
  if (device < 0) {
    set_error("scratch_attach: bad device");
    return H2_EINVAL;
  }
  if (device < (int)g_ptr.size() && g_ptr[device]) return H2_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return H2_EHIP;
  }
  if ((int)g_ptr.size() <= device) g_ptr.resize(device + 1, nullptr);
  g_ptr[device] = static_cast<double*>(p);
  return H2_OK;
}

}  // namespace h2

using namespace h2;

extern "C" int h2_gemv_noalloc(h2_handle h, char op, double alpha, const double* X, int64_t ldx, int64_t nv,
                               double beta, double* Y, int64_t ldy, void* stream) {
  bool trans = false;
  int rc = check_gemv_args(h, op, alpha, X, ldx, nv, Y, ldy, H2_PREC_FP64, &trans);
  if (rc != H2_OK || nv == 0) return rc;
  const int64_t per = bytes_per_vector(h->n, h->H);
  if (per > kScratchBytes) {
    set_error("h2_gemv_noalloc: one vector needs " + std::to_string(per) + " bytes of scratch (n = " +
              std::to_string(h->n) + ", tree rows = " + std::to_string(h->H) + "); the fixed array holds " +
              std::to_string(kScratchBytes));
    return H2_EUNSUPPORTED;
  }
  double* base = scratch_ptr(h->device);
  if (!base || !h->na.side) {
    set_error("h2_gemv_noalloc: scratch or stream not set up for this device");
    return H2_EHIP;
  }
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(h->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return H2_EHIP;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (alpha == 0.0) {
    const hipError_t e = launch_scale(Y, ldy, h->n, nv, beta, s);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
      set_error(std::string("scale: ") + hipGetErrorString(e));
      return H2_EHIP;
    }
    return H2_OK;
  }
  // views of the array: as many columns (<= kPassVectors) as fit
  Workspace w = h->na;  // side stream and events
  w.n = h->n;
  w.H = h->H;
  w.cap = std::min<int64_t>(kPassVectors, kScratchBytes / per);
  const int64_t nn = std::max<int64_t>(h->n, 1), Hs = std::max<int64_t>(h->H, 1);
  w.xt = base;
  w.zn = w.xt + nn * w.cap;
  w.xh = w.zn + nn * w.cap;
  w.yh = w.xh + std::max<int64_t>(Hs, 8) * w.cap;
  w.xh32 = nullptr;
  rc = gemv_ws(h, w, trans, alpha, X, ldx, nv, beta, Y, ldy, H2_PREC_FP64, s);
  (void)hipSetDevice(prev);
  return rc;
}
