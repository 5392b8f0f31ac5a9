// Library-private declarations of libh2gemv: the host view of a serialized
// representation, the launch schedules built at load time, the handle, and
// the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "h2.h"

namespace h2 {

// Largest rank and leaf size the kernels accept (one output entry per
// thread of a 256-thread workgroup along the row dimension).
constexpr int kMaxDim = 256;
// Vectors per pass of the workspace; larger nv is processed in chunks.
constexpr int kNvChunk = 64;

void set_error(const std::string& msg);

// Host view of a representation; arrays point into the caller's buffer.
struct Parsed {
  int64_t n = 0, q = 0, nnodes = 0, nleaves = 0, leaf0 = 0, ndense = 0, nadm_tot = 0;
  uint32_t flags = 0;
  const int64_t *level_ptr = nullptr, *krow = nullptr, *kcol = nullptr, *nadm = nullptr;
  const int64_t *perm = nullptr, *lo = nullptr, *hi = nullptr, *parent = nullptr;
  const int64_t *s_rowptr = nullptr, *s_col = nullptr, *d_rowptr = nullptr, *d_col = nullptr;
  // byte offsets of the FP64 sections in the buffer
  int64_t off_U = 0, off_E = 0, off_V = 0, off_F = 0, off_S = 0, off_D = 0, off_end = 0;
  std::vector<int64_t> ebase, fbase;  // per level: element offset of level's first transfer
  std::vector<int64_t> rp_base;       // per level: first entry in s_rowptr
  std::vector<int64_t> blk_base;      // per level: first global coupling block (q+2 entries)
  std::vector<int64_t> sdat;          // per level: element offset of level's first block in S
  std::vector<int64_t> ddat;          // per dense block: element offset in D (ndense+1)
};

// Parse and validate; returns H2_OK, H2_EFORMAT, H2_EUNSUPPORTED, H2_ENOMEM.
int parse(const uint8_t* buf, int64_t len, Parsed* p);

// A block row (or, transposed, a block column) processed by one workgroup.
struct RowDesc {
  int64_t data_off;  // streaming kernel: element offset of the row's first block
  int64_t out_off;   // row offset of the output (element (a, v) at out_off + a + out_ld*v)
  int32_t nrows;     // output length (rows of the stored blocks, or columns when transposed)
  int32_t blk_begin; // blocks [blk_begin, blk_end) in the per-block arrays
  int32_t blk_end;
  int32_t pad;
  int64_t out_ld;    // output stride between vectors
  int64_t in_ld;     // input stride between vectors
};

// Schedule for the streaming kernel (op 'N'): the blocks of a row are
// contiguous in memory and form one column-major nrows x ncols matrix.
struct StreamSched {
  std::vector<RowDesc> rows;
  std::vector<int32_t> colend;   // per block: cumulative end column within its row
  std::vector<int64_t> in_off;   // per block: input row offset of its first column
  RowDesc* d_rows = nullptr;
  int32_t* d_colend = nullptr;
  int64_t* d_in_off = nullptr;
};

// Schedule for the transposed product (op 'T'): the blocks of a block
// column, each read transposed.
struct GatherSched {
  std::vector<RowDesc> rows;
  std::vector<int64_t> data;     // per block: element offset of the stored block
  std::vector<int32_t> mr;       // per block: rows of the stored block
  std::vector<int64_t> in_off;   // per block: input row offset
  RowDesc* d_rows = nullptr;
  int64_t* d_data = nullptr;
  int32_t* d_mr = nullptr;
  int64_t* d_in_off = nullptr;
};

struct LevelInfo {
  int64_t begin, count;  // nodes [begin, begin+count)
  int64_t krow, kcol, kmax;
  int64_t e_off, f_off;  // element offsets (in the device matrix array) of the level's transfers
};

}  // namespace h2

struct h2_op_s {
  int device = 0;
  int64_t n = 0, q = 0, nnodes = 0, nleaves = 0, leaf0 = 0;
  int64_t H = 0;  // rows of the vector trees (sum of per-node max rank)
  bool shared = true;
  std::vector<h2::LevelInfo> lv;
  h2_stats_t stats{};
  // device data
  double* d_mat = nullptr;   // U, E, V, F, S, D (one allocation, section layout kept)
  int64_t u_off = 0, v_off = 0, s_off = 0, d_off = 0;  // element offsets into d_mat
  int32_t* d_perm = nullptr;
  int32_t* d_lo = nullptr;
  int32_t* d_m = nullptr;
  int32_t* d_parent = nullptr;
  int32_t* d_cptr = nullptr;   // children of p: [cptr[p], cptr[p+1])
  int64_t* d_hoff = nullptr;   // per node: first row in the vector trees
  h2::StreamSched coupleN, denseN;
  h2::GatherSched coupleT, denseT;
  int64_t index_bytes = 0;
  // workspace (n x cap, H x cap, H x cap, n x cap)
  int64_t cap = 0;
  double *d_xt = nullptr, *d_xh = nullptr, *d_yh = nullptr, *d_zn = nullptr;
  // profiling
  bool profiling = false;
  std::vector<std::array<hipEvent_t, 7>> ev_pool;
  size_t ev_used = 0;
  h2_profile_t prof{};
};

namespace h2 {

// kernel launchers (h2_kernels.hip); all asynchronous on `s`
hipError_t launch_permute_in(const double* X, int64_t ldx, const int32_t* perm, double* xt, int64_t n,
                             int nv, hipStream_t s);
hipError_t launch_scale(double* Y, int64_t ldy, int64_t n, int64_t nv, double beta, hipStream_t s);
hipError_t launch_leaf_up(const double* B, int k, int64_t leaf0, int64_t nleaves, const int32_t* lo,
                          const int32_t* m, const int64_t* hoff, const double* xt, int64_t n, double* xh,
                          int64_t H, int nv, hipStream_t s);
hipError_t launch_transfer_up(const double* T, int kc, int kp, int64_t pbegin, int64_t pcount,
                              int64_t cbegin, const int32_t* cptr, const int64_t* hoff, double* xh,
                              int64_t H, int nv, hipStream_t s);
hipError_t launch_transfer_down(const double* T, int kc, int kp, int64_t cbegin, int64_t ccount,
                                const int32_t* parent, const int64_t* hoff, double* yh, int64_t H, int nv,
                                hipStream_t s);
hipError_t launch_leaf_down(const double* B, int k, int64_t leaf0, int64_t nleaves, const int32_t* lo,
                            const int32_t* m, const int64_t* hoff, const double* yh, int64_t H,
                            const double* zn, int64_t n, const int32_t* perm, double alpha, double beta,
                            double* Y, int64_t ldy, int nv, hipStream_t s);
hipError_t launch_stream_rows(const StreamSched& sc, const double* data, const double* in, double* out,
                              int nv, hipStream_t s);
hipError_t launch_gather_rows(const GatherSched& sc, const double* data, const double* in, double* out,
                              int nv, hipStream_t s);

}  // namespace h2
