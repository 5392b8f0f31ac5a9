// Library-private declarations of libh2gemv: the host view of a serialized
// representation, the launch plans built at load time, the handle, and the
// kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "h2.h"

struct h2_op_s;

namespace h2 {

// Largest rank and leaf size the kernels accept (one output entry per
// thread of a 256-thread workgroup along the row dimension).
constexpr int kMaxDim = 256;
// Largest number of blocks in one row handled by the LDS-tabled streaming
// kernel; wider rows (never produced by the builder) take a simpler kernel.
constexpr int kNbMax = 512;
// Largest number of children of one node.
constexpr int kMaxChildren = kNbMax;
// Vectors per pass of the streaming path (one thread keeps them in registers).
constexpr int kPassVectors = 4;
// Vectors per pass of the MFMA path (four 16-wide tiles).
constexpr int kPassVectorsMfma = 64;

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
// Reads the header and the index sections only (bytes before U).
int parse(const uint8_t* buf, int64_t len, Parsed* p);

// One output row-block processed by one workgroup: out[out_off + a + out_ld*v]
// (a < nrows) from the column-major nrows x ncols matrix at data + data_off
// (its blocks are contiguous) times the input gathered block by block.
struct RowDesc {
  int64_t data_off;  // element offset of the row's first stored block (streaming)
  int64_t out_off;   // output row offset
  int32_t nrows;     // output length
  int32_t blk_begin; // blocks [blk_begin, blk_end) in the per-block tables
  int32_t blk_end;
  int32_t pad;
  int64_t out_ld;    // output stride between vectors
  int64_t in_ld;     // input stride between vectors
  int64_t fl_off;    // element offset of the row's fragment-ordered copy (wave-row kernels), even
};

// Row schedules of the streaming kernel: per block, the cumulative end
// column within its row and the input row offset of its first column.
struct RowTables {
  std::vector<RowDesc> rows;
  std::vector<int32_t> colend;
  std::vector<int64_t> in_off;
  RowDesc* d_rows = nullptr;
  int32_t* d_colend = nullptr;
  int64_t* d_in_off = nullptr;
};

// Row schedules of the transposed (gather) kernel: the blocks of a block
// column, each read transposed.
struct GatherTables {
  std::vector<RowDesc> rows;
  std::vector<int64_t> data;     // per block: element offset of the stored block
  std::vector<int32_t> mr;       // per block: rows of the stored block
  std::vector<int64_t> in_off;   // per block: input row offset
  RowDesc* d_rows = nullptr;
  int64_t* d_data = nullptr;
  int32_t* d_mr = nullptr;
  int64_t* d_in_off = nullptr;
};

// Where a launch reads and writes.
enum Buf { BUF_XT = 0, BUF_XH = 1, BUF_YH = 2, BUF_ZN = 3 };
enum Arr { ARR_MAT = 0, ARR_TRANS = 1 };
enum Mode { MODE_STORE = 0, MODE_ACCUM = 1, MODE_FINAL = 2 };
enum Kind { KIND_STREAM = 0, KIND_GATHER = 1, KIND_WIDE = 2 };

struct Launch {
  int kind = KIND_STREAM;
  int arr = ARR_MAT;
  int in = BUF_XT, out = BUF_XH;
  int mode = MODE_STORE;
  int64_t row_begin = 0, row_count = 0;  // slice of the kind's row table
  int32_t max_rows = 0;                   // largest output length of its rows
  bool lowrank = true;                    // false for the dense near-field phase (always FP64)
  int kc = 64;                            // MFMA path: columns per LDS chunk (tuned in batches)
  int64_t grid = 0;                       // MFMA path: workgroups (0 = one per row; fewer = persistent)
  // single-operator MFMA path, per precision of the launch (H2_PREC_*; the
  // dense rows always use the FP64 entry): chunk columns and workgroups, set
  // by h2_tune
  int kcp[3] = {64, 64, 64};
  int64_t gridp[3] = {0, 0, 0};
  int remapp[3] = {0, 0, 0};  // XCD-aware row ranges
  int flp[3] = {1, 1, 1};     // wave-row kernels: read the fragment-ordered copy when there is one
  int occp[3] = {0, 0, 0};    // wave-row kernels: 5 = the form compiled for five waves per SIMD
  float tuned_ms[3] = {0, 0, 0};  // time of the chosen setting when tuned (two runs)
  // sweep transfer launches: the level of the parent nodes (upsweep: whose
  // x^ it computes; downsweep: whose y^ it pushes down); -1 for other launches
  int64_t level = -1;
};

// The launch sequence of one operation (op 'N' or 'T').
struct Plan {
  std::vector<Launch> up;      // leaf products, then transfer levels q..1
  std::vector<Launch> couple;  // all levels at once (plus wide rows, if any)
  std::vector<Launch> down;    // transfer levels 1..q
  std::vector<Launch> dense;   // dense leaf blocks, first half (side stream, beside the upsweep)
  std::vector<Launch> dense2;  // second half (side stream, beside the downsweep and leaf expansion)
  // the same rows in tree order (neighbouring rows share input segments), for
  // the multi-vector path when the tuner finds it faster
  std::vector<Launch> couple_loc, dense_loc, dense2_loc;
  // the coupling rows split: the leaf level's (they need only the leaf
  // products of the upsweep) and the other levels', longest first in each
  std::vector<Launch> couple_deep, couple_rest;
  Launch out;                  // leaf expansion + dense partial + alpha/beta update
};

// Fused sweeps of the multi-vector path (h2_tree_kernels.hip): the levels
// one launch runs, in order, with their input and output buffers (0 X~, 1 x^,
// 2 y^, 3 the leaf-expansion output) and epilogue (MODE_STORE / MODE_ACCUM).
constexpr int kMaxTreeLevels = 8;
struct TreeLevels {
  int nlev = 0;
  int in[kMaxTreeLevels] = {};
  int out[kMaxTreeLevels] = {};
  int mode[kMaxTreeLevels] = {};
};
// One fused launch: workgroup w owns the subtree of the w-th node of its
// root level; ranges [range_off + w * nlev + lev] are its rows on each level.
struct TreeGroup {
  TreeLevels lv;
  int64_t nwg = 0;
  int64_t range_off = 0;
  int max_rows = 0;
  bool trans_data = false;  // rows read the transposed basis copies (upsweep)
};

// A captured h2_gemv call (HIP graph replay): every argument that the
// launch sequence bakes in.
struct GraphKey {
  bool trans;
  int prec;
  const double* X;
  int64_t ldx, nv;
  double alpha, beta;
  double* Y;
  int64_t ldy;
  hipStream_t s;
  bool operator==(const GraphKey& o) const {
    return trans == o.trans && prec == o.prec && X == o.X && ldx == o.ldx && nv == o.nv && alpha == o.alpha &&
           beta == o.beta && Y == o.Y && ldy == o.ldy && s == o.s;
  }
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};
constexpr size_t kMaxGraphs = 8;

struct Epilogue {
  const double* zn;     // dense partial, n x nv (ld n)
  const int32_t* perm;  // tree position -> original index
  double alpha, beta;
  double* Y;
  int64_t ldy;
  int64_t n;
};

struct LevelInfo {
  int64_t begin, count;  // nodes [begin, begin+count)
  int64_t krow, kcol, kmax;
};

// ---- plan construction (h2_plan.cpp)

struct BlockRef {
  int64_t data;    // element offset of the stored block (gather rows)
  int64_t in_off;  // input row offset
  int32_t width;   // columns of the stored block
  int32_t mr;      // rows of the stored block (gather rows)
};

struct RowSpec {
  int64_t data_off, out_off, out_ld, in_ld;
  int32_t nrows;
  std::vector<BlockRef> blks;
};

// First level with coupling blocks, q + 1 if there is none.
inline int64_t first_coupling_level(const Parsed& P) {
  for (int64_t l = 0; l <= P.q; ++l)
    if (P.nadm[l] > 0) return l;
  return P.q + 1;
}

// Per-operator offsets used to emit rows.
struct OpLayout {
  const Parsed* P = nullptr;
  bool shared = true;
  std::vector<int64_t> kmax;   // per level
  std::vector<int64_t> hoff;   // per node: first row in the vector trees
  std::vector<int64_t> cbeg;   // per node: first child (children contiguous); nnodes+1 entries
  int64_t H = 0;               // rows of the vector trees
  int64_t oU = 0, oE = 0, oV = 0, oF = 0, oS = 0, oD = 0, nmat = 0;  // matrix array (elements)
  int64_t tUT = 0, tET = 0, tVT = 0, tFT = 0, ntrans = 0;            // transposed array (elements)
  int64_t eoff(int64_t c, int64_t l) const;  // offset of E_c within the E section
  int64_t foff(int64_t c, int64_t l) const;  // offset of F_c within the F section
};

// Where an operator's data and workspace sit: element offsets of its matrix
// and transposed arrays, row offsets of its X~, x^, y^ and dense-partial
// regions, and the vector strides of the column-major streaming layout.
struct RowBases {
  int64_t mat = 0, trans = 0;
  int64_t xt = 0, xh = 0, yh = 0, zn = 0;
  int64_t ld_x = 0, ld_h = 0;
};

// Rows of every op-'N' phase of one operator.
struct RowsN {
  std::vector<std::vector<RowSpec>> up;    // up[0]: leaf products; up[h]: transfer level q-h+1 -> q-h
  std::vector<RowSpec> couple;             // all levels
  std::vector<std::vector<RowSpec>> down;  // down[l-1]: transfer level l
  std::vector<RowSpec> dense;
  std::vector<RowSpec> out;                // leaf expansion
};

int make_layout(const Parsed& P, OpLayout* L);
// The transposed copies of the bases as a list of blocks: the column-major
// rows x cols block at element src of the matrix array goes, transposed
// (cols x rows, column-major), to element dst of the transposed array
// (leaf bases, then transfers; both bases when they are separate).
struct TransTask {
  int64_t src, dst;
  int32_t rows, cols;
};
void transpose_tasks(const OpLayout& L, std::vector<TransTask>* out);
// The transposed array on the host (zeros where no block lands).
void build_transposed(const uint8_t* buf, const OpLayout& L, double* tr);
void emit_rows_N(const OpLayout& L, const RowBases& B, RowsN* R);
void append_row(RowTables& t, const RowSpec& r);
int64_t row_work(const RowSpec& r);
// Places the fragment-ordered copy of rows [begin, end) of t: rows with the
// same matrix (array, offset and shape) share one region; regions start at
// even offsets.  *n_fl grows by the elements placed.  `keys` carries the
// placed regions between calls.
struct FlRegion {
  int64_t fl_off;
  int32_t nrows, ncols;
};
using FlKeys = std::unordered_map<int64_t, FlRegion>;  // key: 2 * data_off + array
void place_fl(RowTables& t, int64_t begin, int64_t end, int arr, FlKeys* keys, int64_t* n_fl);

// Per-product scratch: X~ and the dense partial (n x cap), x^ and y^
// (H x cap) in doubles; the streaming path uses them column-major with up
// to 4 columns, the MFMA path row-major with up to 64.  The side stream and
// events fork and join the dense phase.  One workspace serves one product at
// a time; concurrent products need one each.
struct Workspace {
  int64_t n = 0, H = 0, cap = 0;
  double *xt = nullptr, *xh = nullptr, *yh = nullptr, *zn = nullptr;
  // leaf-expansion output of the fused sweeps (n * cap; cap >= kPassVectorsMfma only)
  double* zx = nullptr;
  // FP32 copy of x^ (H * cap floats; cap >= kPassVectorsMfma only) that the
  // FP32 variant's 64-vector coupling launches gather from
  float* xh32 = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_mid = nullptr;
  // third stream of the multi-vector schedule 3: the leaf level's coupling
  // rows beside the rest of the sweeps
  hipStream_t side2 = nullptr;
  hipEvent_t ev_deep = nullptr, ev_deep_done = nullptr;
};
int ws_create(Workspace* w, int64_t n, int64_t H, int64_t cap);
// The product of h2_gemv_ex on an explicit workspace (w.n >= n, w.H >= H),
// after check_gemv_args; alpha != 0 and nv > 0.
int gemv_ws(h2_op_s* h, const Workspace& w, bool trans, double alpha, const double* X, int64_t ldx, int64_t nv,
            double beta, double* Y, int64_t ldy, int prec, hipStream_t s);
int check_gemv_args(h2_op_s* h, char op, double alpha, const double* X, int64_t ldx, int64_t nv, double* Y,
                    int64_t ldy, int prec, bool* trans);
void ws_destroy(Workspace* w);
int64_t ws_bytes(int64_t n, int64_t H, int64_t cap);
// A new handle on `device` from a representation of `len` bytes whose first
// bytes are at `buf`.  With d_dense == nullptr the whole representation is in
// `buf`; otherwise `buf` holds the bytes before the dense section only and
// the dense blocks are copied from device memory at d_dense (same device).
int load_handle(const uint8_t* buf, int64_t len, int device, const double* d_dense, h2_handle* out);
// Look up, once per device, the device address of the fixed scratch array of
// h2_gemv_noalloc (h2_noalloc.hip); `device` is current.  Called by every load.
int scratch_attach(int device);
// True when products in precision `prec` need no preparation (allocation)
// on this handle.
bool prepared(h2_op_s* h, int prec);

}  // namespace h2

struct h2_op_s {
  int device = 0;
  int64_t n = 0, q = 0, nnodes = 0, nleaves = 0, leaf0 = 0;
  // first level with coupling blocks (q + 1 if none): above it x^ is never
  // read and y^ is zero, so the per-level sweeps skip those transfer levels
  int64_t lmin = 0;
  int64_t H = 0;  // rows of the vector trees (sum of per-node max rank)
  bool shared = true;
  std::vector<h2::LevelInfo> lv;
  h2_stats_t stats{};
  std::vector<h2_level_stats_t> level_stats;
  // device data
  double* d_mat = nullptr;    // U, E, V, F, S, D (section layout of the buffer kept)
  double* d_trans = nullptr;  // transposed copies: U^T, E^T (and V^T, F^T)
  int64_t n_lowrank = 0;      // elements of d_mat before the dense section (U, E, V, F, S)
  int64_t n_trans = 0;        // elements of d_trans
  float* d_mat32 = nullptr;   // FP32 copies of d_mat[0, n_lowrank) and of d_trans
  float* d_trans32 = nullptr;
  void* d_mat16 = nullptr;    // BF16 copies of the op-'N' low-rank rows, row-major per row
  void* d_trans16 = nullptr;
  // fragment-ordered copies of the op-'N' rows (FP64 every row, FP32 the
  // low-rank rows) at the rows' fl_off, read by the wave-row kernels; made by
  // h2_tune on the multi-vector path (the regions are placed then too)
  bool fl_placed = false;
  int64_t n_fl = 0;
  double* d_fl = nullptr;
  float* d_fl32 = nullptr;
  std::mutex prep_mu;         // guards the lazy creation of the FP32 and BF16 copies
  int32_t* d_perm = nullptr;
  int32_t* d_pinv = nullptr;  // original index -> tree position
  bool mfma_ok = true;        // every op-'N' launch fits the MFMA row kernel
  // workgroups of the dense launches on the streaming path (nv <= 4): two per
  // CU, a persistent grid that leaves the other slots to the sweeps beside it
  int64_t dense_stream_grid = 0;
  // workgroups of the dense launches on the multi-vector path: -1 the tuned
  // grid, 0 one per row, else a persistent grid (h2_set_dense_grid)
  int64_t dense_grid_mv = -1;
  int couple_mode[3] = {0, 0, 0};  // per precision: 0 longest first, 1 tree order (h2_tune)
  int dense_mode[3] = {0, 0, 0};   // per precision: 0 longest first, 1 tree order (h2_tune)
  h2::RowTables rt;           // streaming rows of both plans
  h2::RowTables wide;         // rows too wide for the tabled kernel
  h2::GatherTables gt;        // transposed rows of the 'T' plan
  h2::Plan planN, planT;
  // fused sweeps of the op-'N' multi-vector path: upsweep groups (deepest
  // first) and downsweep groups (the last one ends with the leaf expansion)
  std::vector<h2::TreeGroup> tree_up, tree_down;
  int2* d_tree_ranges = nullptr;
  bool tree_ok = false;              // every group fits the fused kernel
  int sweep_fused[3] = {0, 0, 0};    // per precision (FP64, FP32; BF16 has none): use the fused sweeps
  float sweep_ms[3][2] = {};         // tuned times of the sweeps: per level, fused
  // multi-vector path, per precision: where the dense rows run (h2_tune):
  // 0 halves beside the upsweep and the downsweep, 1 the first half beside the
  // coupling launch instead, 2 both halves from the start, 3 both halves from
  // the start and the leaf level's coupling rows on a third stream, beside
  // the upsweep above the leaves, the other levels' coupling rows and the
  // downsweep above the leaves
  int sched[3] = {0, 0, 0};
  float sched_ms[3][4] = {};
  // the same choice for the streaming path (at most 4 vectors per pass; FP64
  // and FP32), tuned separately
  int sched1[3] = {0, 0, 0};
  float sched1_ms[3][4] = {};
  int64_t index_bytes = 0;
  // the serialized header and index sections (bytes before U), 8-byte aligned,
  // and the representation's total size: the host view of the structure
  // (export, recompression)
  std::vector<uint64_t> prefix;
  int64_t prefix_len = 0, file_len = 0;
  h2::Workspace ws;  // the handle's own workspace (h2_gemv), allocated on first use
  // captured calls of h2_gemv / h2_gemv_ex (h2_graph), least recently used dropped first
  bool use_graph = false;
  std::vector<h2::GraphEntry> graphs;
  uint64_t graph_clock = 0;
  // side stream and fork/join events of h2_gemv_noalloc, created at load
  // (its buffers are views of the fixed scratch array)
  h2::Workspace na;
  // profiling
  bool profiling = false;
  std::vector<std::array<hipEvent_t, 13>> ev_pool;
  size_t ev_used = 0;
  h2_profile_t prof{};
};

namespace h2 {

// kernel launchers (h2_kernels.hip); all asynchronous on `s`
hipError_t launch_permute_in(const double* X, int64_t ldx, const int32_t* perm, double* xt, int64_t n, int nv,
                             hipStream_t s);
hipError_t launch_scale(double* Y, int64_t ldy, int64_t n, int64_t nv, double beta, hipStream_t s);
template <typename T>
hipError_t launch_rows(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                       const T* data, const double* in, double* out, int nv, int mode, const Epilogue& ep,
                       hipStream_t s, int64_t grid = 0);
template <typename T>
hipError_t launch_rows_mfma(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                            const T* data, const double* in, double* out, int nvp, int mode, int max_rows,
                            hipStream_t s, int kc = 64, int64_t grid = 0, int remap = 0,
                            const float* in32 = nullptr);

// One operator's part of a batched call, as the batched permutation kernels see it.
struct BatchItem {
  const double* X;
  double* Y;
  int64_t ldx, ldy, nv;
  double alpha, beta;
  int64_t n;         // operator order
  int64_t pinv_off;  // its inverse permutation in the concatenated array
  int64_t xt_row;    // its X~ rows in the workspace arena
  int64_t zn_row;    // its dense-partial rows in the workspace arena
};
// tiles of kPermTile original rows: tile b is rows tile_j0[b] .. + 63 of operator tile_op[b]
constexpr int kPermTile = 64;
hipError_t launch_batch_permute(const BatchItem* items, const int32_t* tile_op, const int32_t* tile_j0,
                                int64_t ntiles, const int32_t* pinv, double* ws, int nvp, bool out, hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);
// The transposed basis copies on the device (h2_load_kernels.hip): every
// task's block of `mat` transposed into `trans` (which the caller zeroed).
hipError_t launch_transpose_tasks(const TransTask* tasks, int64_t ntasks, const double* mat, double* trans,
                                  hipStream_t s);
// BF16 path (data: __bf16, rows stored row-major; see the kernel file)
hipError_t launch_rows_mfma_bf16(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                                 const void* data, const void* in, bool in16, int64_t ldb, void* out, bool out16,
                                 int64_t ldo, int nvp, int mode, int max_rows, hipStream_t s, int64_t grid = 0,
                                 int remap = 0);
hipError_t launch_rows_to_bf16(const RowDesc* rows, int64_t nrows, const int32_t* colend, const double* src,
                               void* dst, hipStream_t s);
hipError_t launch_permute_in_rm(const double* X, int64_t ldx, const int32_t* pinv, double* xt, int64_t n, int nv,
                                int nvp, hipStream_t s);
hipError_t launch_permute_out_rm(const double* Z, const int32_t* pinv, double alpha, double beta, double* Y,
                                 int64_t ldy, int64_t n, int nv, int nvp, hipStream_t s);
// The multi-vector row product with one wave per row (kc code kWaveRows of
// the tuner), or one wave per 16-vector tile of a row (kWaveTiles); grid =
// workgroups (0: enough for every row at once); remap: XCD-aware row ranges
constexpr int kWaveRows = 9, kWaveTiles = 10;
// fl: the fragment-ordered copy of the rows' matrices (rows' fl_off), read
// instead of `data` when not null; occ 5: the form compiled for five waves
// per SIMD where one exists (one 16-vector tile per wave, rows of at most 48
// outputs), else the default; the results are bitwise the same
template <typename T>
hipError_t launch_wave_rows(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                            const T* data, const double* in, double* out, int nvp, int mode, int max_rows,
                            hipStream_t s, int64_t grid, bool narrow = false, int remap = 0, const T* fl = nullptr,
                            int occ = 0);
// True when launch_wave_rows has a five-waves-per-SIMD form for this pass
// width, row length and kernel (one 16-vector tile per wave, at most three
// 16-row tiles)
inline bool wave_occ5(int nvp, int max_rows, bool narrow) {
  return max_rows <= 48 && (nvp == 16 || (narrow && (nvp == 32 || nvp == 64)));
}
// dst[R.fl_off ...] = the fragment-ordered copy of every row's matrix at src[R.data_off ...]
template <typename T>
hipError_t launch_rows_to_fl(const RowDesc* rows, int64_t nrows, const int32_t* colend, const T* src, T* dst,
                             hipStream_t s);
template <typename T>
hipError_t launch_tree(const int2* ranges, int64_t nwg, const TreeLevels& L, const RowDesc* rows,
                       const int32_t* colend, const int64_t* in_off, const T* data, double* const bufs[4], int nvp,
                       int max_rows, hipStream_t s);
// Y[j, v] = alpha * (Z[pinv[j], v] + Z2[pinv[j], v]) + beta * Y[j, v] (Z, Z2 row-major nvp, tree order)
hipError_t launch_permute_out_rm2(const double* Z, const double* Z2, const int32_t* pinv, double alpha, double beta,
                                  double* Y, int64_t ldy, int64_t n, int nv, int nvp, hipStream_t s);
hipError_t launch_rows_wide(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                            const double* data, const double* in, double* out, int nv, hipStream_t s);
template <typename T>
hipError_t launch_gather(const RowDesc* rows, int64_t nrows, const int64_t* bdata, const int32_t* bmr,
                         const int64_t* bin, const T* data, const double* in, double* out, int nv,
                         hipStream_t s);

}  // namespace h2
