// Cross-operator batching: several H^2 operators in one device arena, all
// applied by one sequence of merged launches (declarations in include/h2.h).
//
// Every operator contributes the rows of each op-'N' phase (h2_plan.cpp)
// with its own arena offsets, so rows of different operators mix freely in
// one launch.  Uneven trees are merged level by level: upsweep launch h holds
// transfer level q_i - h + 1 of every operator with q_i >= h (aligned by
// height from the leaves), downsweep launch l holds level l of every operator
// with q_i >= l (aligned by depth from the root).
//
// Operators are grouped by vector width: operator i's rows carry
// nvp_i = nv_max_i rounded up to 16 vectors (the MFMA tile width), so an
// operator that never takes more than 16 vectors does not pay for 32.  Each
// width has its own workspace arena and its own merged launches; the launches
// of the groups follow each other, interleaved level by level.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "h2_internal.h"

namespace h2 {
namespace {

int hip_fail_b(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? H2_ENOMEM : H2_EHIP;
}

#define HIP_TRYB(expr, what)                            \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail_b(e_, what);  \
  } while (0)

struct DevGuard {
  int prev = -1;
  bool ok = false;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// The operators of one vector width: their workspace arena (row-major, nvp
// doubles per row), merged launches and permutation tiles.
struct Group {
  int nvp = 16;
  double* d_ws = nullptr;
  int64_t ws_rows = 0;
  std::vector<Launch> up, couple, down, dense, out;  // up[h] / down[d]: merged level h / d (may be absent)
  std::vector<int64_t> up_level, down_level;         // the merged level of each launch
  int32_t *d_tile_op = nullptr, *d_tile_j0 = nullptr;
  int64_t ntiles = 0;
  // groups after the first: their own stream for the sweeps and coupling
  // rows when the groups run side by side (h2_batch_s::par)
  hipStream_t st = nullptr;
  hipEvent_t ev_go = nullptr, ev_done = nullptr;
};

}  // namespace
}  // namespace h2

struct h2_batch_s {
  int device = 0;
  int64_t count = 0, nmax = 0, total_n = 0, maxq = 0;
  double flops_per_vector = 0.0;
  std::vector<int64_t> n, nv_max, pinv_off, xt_row, zn_row;
  double* d_mat = nullptr;
  double* d_trans = nullptr;
  int32_t* d_pinv = nullptr;
  h2::RowTables rt;
  std::vector<h2::Group> groups;
  h2::BatchItem* h_items = nullptr;  // pinned
  h2::BatchItem* d_items = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_items = nullptr;
  bool items_pending = false;
  // where the dense rows run (h2_batch_tune): 0 on the second stream from the
  // start, beside the upsweep; 1 on the second stream after the upsweep,
  // beside the coupling launches
  int sched = 0;
  // par: each vector-width group's sweeps and coupling rows on a stream of
  // its own (the groups are independent operators), the dense rows beside
  // them from the start; else the groups' launches interleaved on one stream
  bool par = false;
  float sched_ms[3] = {0.0f, 0.0f, 0.0f};
  bool use_graph = false;
  hipGraphExec_t graph = nullptr;
  hipStream_t graph_stream = nullptr;
};

namespace h2 {
namespace {

void free_batch(h2_batch_s* b) {
  auto F = [](void* p) { if (p) (void)hipFree(p); };
  F(b->d_mat); F(b->d_trans); F(b->d_pinv); F(b->d_items);
  for (Group& g : b->groups) {
    if (g.ev_go) (void)hipEventDestroy(g.ev_go);
    if (g.ev_done) (void)hipEventDestroy(g.ev_done);
    if (g.st) (void)hipStreamDestroy(g.st);
    F(g.d_ws); F(g.d_tile_op); F(g.d_tile_j0);
  }
  F(b->rt.d_rows); F(b->rt.d_colend); F(b->rt.d_in_off);
  if (b->h_items) (void)hipHostFree(b->h_items);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->ev_items) (void)hipEventDestroy(b->ev_items);
  if (b->side) (void)hipStreamDestroy(b->side);
}

bool add_phase(h2_batch_s* b, std::vector<RowSpec>& rows, int arr, int mode, bool sort, bool lowrank,
               std::vector<Launch>& dst) {
  if (rows.empty()) return false;
  if (sort)
    std::stable_sort(rows.begin(), rows.end(),
                     [](const RowSpec& x, const RowSpec& y) { return row_work(x) > row_work(y); });
  Launch L;
  L.kind = KIND_STREAM;
  L.arr = arr;
  L.mode = mode;
  L.lowrank = lowrank;
  L.row_begin = (int64_t)b->rt.rows.size();
  for (const RowSpec& r : rows) {
    append_row(b->rt, r);
    L.max_rows = std::max(L.max_rows, r.nrows);
  }
  L.row_count = (int64_t)b->rt.rows.size() - L.row_begin;
  dst.push_back(L);
  return true;
}

int batch_build(const void* const* bufs, const size_t* lens, int64_t count, h2_batch_s* b) {
  std::vector<Parsed> P(count);
  std::vector<OpLayout> lay(count);
  for (int64_t i = 0; i < count; ++i) {
    int rc = parse(static_cast<const uint8_t*>(bufs[i]), (int64_t)lens[i], &P[i]);
    if (rc != H2_OK) {
      set_error("batch operator " + std::to_string(i) + ": " + h2_last_error());
      return rc;
    }
    if ((rc = make_layout(P[i], &lay[i])) != H2_OK) return rc;
  }
  // groups by vector width
  std::map<int, size_t> gidx;
  std::vector<size_t> op_group(count);
  for (int64_t i = 0; i < count; ++i) {
    const int nvp = (int)((b->nv_max[i] + 15) / 16 * 16);
    auto it = gidx.find(nvp);
    if (it == gidx.end()) {
      it = gidx.emplace(nvp, b->groups.size()).first;
      b->groups.emplace_back();
      b->groups.back().nvp = nvp;
    }
    op_group[i] = it->second;
  }
  // arena offsets: matrix data and transposed bases shared, workspace rows per group
  auto up32 = [](int64_t x) { return (x + 31) / 32 * 32; };
  std::vector<RowBases> base(count);
  int64_t mat = 0, trans = 0, pin = 0;
  b->n.resize(count); b->pinv_off.resize(count); b->xt_row.resize(count); b->zn_row.resize(count);
  for (int64_t i = 0; i < count; ++i) {
    RowBases& B = base[i];
    int64_t& row = b->groups[op_group[i]].ws_rows;
    B.mat = mat;
    B.trans = trans;
    mat = up32(mat + lay[i].nmat);
    trans = up32(trans + lay[i].ntrans);
    B.xt = row; row += P[i].n;
    B.xh = row; row += lay[i].H;
    B.yh = row; row += lay[i].H;
    B.zn = row; row += P[i].n;
    b->n[i] = P[i].n;
    b->pinv_off[i] = pin;
    pin += P[i].n;
    b->xt_row[i] = B.xt;
    b->zn_row[i] = B.zn;
    b->nmax = std::max(b->nmax, P[i].n);
    b->total_n += P[i].n;
    const int64_t q = P[i].q;
    b->maxq = std::max(b->maxq, q);
    b->flops_per_vector += 2.0 * (double)(P[i].n * P[i].krow[q] + P[i].n * P[i].kcol[q] + P[i].ebase[q + 1] +
                                          P[i].fbase[q + 1] + P[i].sdat[q + 1] + P[i].ddat[P[i].ndense]);
  }
  // rows of every operator, merged level by level within each group
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& G = b->groups[gi];
    std::vector<std::vector<RowSpec>> up(b->maxq + 1), down(b->maxq);
    std::vector<RowSpec> couple, dense, outr;
    for (int64_t i = 0; i < count; ++i) {
      if (op_group[i] != gi) continue;
      RowsN R;
      emit_rows_N(lay[i], base[i], &R);
      // transfer levels above the operator's first level with coupling blocks
      // are left out (x^ there is never read, y^ there is zero)
      const int64_t lmin = first_coupling_level(P[i]), qi = P[i].q;
      for (size_t h = 0; h < R.up.size(); ++h)
        if (h == 0 || qi - (int64_t)h >= lmin) up[h].insert(up[h].end(), R.up[h].begin(), R.up[h].end());
      for (size_t d = 0; d < R.down.size(); ++d)
        if ((int64_t)d >= lmin) down[d].insert(down[d].end(), R.down[d].begin(), R.down[d].end());
      couple.insert(couple.end(), R.couple.begin(), R.couple.end());
      dense.insert(dense.end(), R.dense.begin(), R.dense.end());
      outr.insert(outr.end(), R.out.begin(), R.out.end());
    }
    for (const auto* v : {&couple, &dense})
      for (const RowSpec& r : *v)
        if ((int64_t)r.blks.size() > kNbMax) {
          set_error("batch: a row with more than 512 blocks");
          return H2_EUNSUPPORTED;
        }
    for (int64_t h = 0; h <= b->maxq; ++h)
      if (add_phase(b, up[h], ARR_TRANS, MODE_STORE, false, true, G.up)) G.up_level.push_back(h);
    add_phase(b, couple, ARR_MAT, MODE_STORE, false, true, G.couple);
    for (int64_t d = 0; d < b->maxq; ++d)
      if (add_phase(b, down[d], ARR_MAT, MODE_ACCUM, false, true, G.down)) G.down_level.push_back(d);
    add_phase(b, dense, ARR_MAT, MODE_STORE, false, false, G.dense);
    add_phase(b, outr, ARR_MAT, MODE_ACCUM, false, true, G.out);
  }

  // device arena: matrix data, transposed bases, inverse permutations
  HIP_TRYB(hipMalloc(reinterpret_cast<void**>(&b->d_mat), sizeof(double) * std::max<int64_t>(mat, 1)), "hipMalloc(arena)");
  HIP_TRYB(hipMalloc(reinterpret_cast<void**>(&b->d_trans), sizeof(double) * std::max<int64_t>(trans, 1)), "hipMalloc(arena)");
  std::vector<int32_t> pinv(std::max<int64_t>(pin, 1));
  // the transposed bases are made on the device from the uploaded matrix
  // data: every operator's blocks, at its arena offsets
  std::vector<TransTask> tasks, ti;
  for (int64_t i = 0; i < count; ++i) {
    const uint8_t* bi = static_cast<const uint8_t*>(bufs[i]);
    if (lay[i].nmat)
      HIP_TRYB(hipMemcpy(b->d_mat + base[i].mat, bi + P[i].off_U, sizeof(double) * lay[i].nmat,
                         hipMemcpyHostToDevice), "hipMemcpy(arena)");
    if (lay[i].ntrans) {
      transpose_tasks(lay[i], &ti);
      for (TransTask& t : ti) {
        t.src += base[i].mat;
        t.dst += base[i].trans;
        tasks.push_back(t);
      }
    }
    for (int64_t j = 0; j < P[i].n; ++j) pinv[b->pinv_off[i] + P[i].perm[j]] = (int32_t)j;
  }
  HIP_TRYB(hipMemset(b->d_trans, 0, sizeof(double) * std::max<int64_t>(trans, 1)), "hipMemset(arena)");
  if (!tasks.empty()) {
    TransTask* d_tasks = nullptr;
    HIP_TRYB(hipMalloc(reinterpret_cast<void**>(&d_tasks), sizeof(TransTask) * tasks.size()), "hipMalloc(tasks)");
    hipError_t e = hipMemcpy(d_tasks, tasks.data(), sizeof(TransTask) * tasks.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_transpose_tasks(d_tasks, (int64_t)tasks.size(), b->d_mat, b->d_trans, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(d_tasks);
    if (e != hipSuccess) return hip_fail_b(e, "transposed basis copies");
  }
  HIP_TRYB(hipMalloc(reinterpret_cast<void**>(&b->d_pinv), sizeof(int32_t) * pinv.size()), "hipMalloc(pinv)");
  HIP_TRYB(hipMemcpy(b->d_pinv, pinv.data(), sizeof(int32_t) * pinv.size(), hipMemcpyHostToDevice), "hipMemcpy");
  // schedules
  auto up_tab = [&](auto& v, auto** d) -> int {
    if (v.empty()) return H2_OK;
    HIP_TRYB(hipMalloc(reinterpret_cast<void**>(d), sizeof(v[0]) * v.size()), "hipMalloc(schedule)");
    HIP_TRYB(hipMemcpy(*d, v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice), "hipMemcpy(schedule)");
    return H2_OK;
  };
  int rc;
  if ((rc = up_tab(b->rt.rows, &b->rt.d_rows)) || (rc = up_tab(b->rt.colend, &b->rt.d_colend)) ||
      (rc = up_tab(b->rt.in_off, &b->rt.d_in_off)))
    return rc;

  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& G = b->groups[gi];
    // permutation tiles: kPermTile original rows of one operator each
    std::vector<int32_t> tile_op, tile_j0;
    for (int64_t i = 0; i < count; ++i)
      if (op_group[i] == gi)
        for (int64_t j0 = 0; j0 < P[i].n; j0 += kPermTile) {
          tile_op.push_back((int32_t)i);
          tile_j0.push_back((int32_t)j0);
        }
    G.ntiles = (int64_t)tile_op.size();
    if ((rc = up_tab(tile_op, &G.d_tile_op)) || (rc = up_tab(tile_j0, &G.d_tile_j0))) return rc;
    // workspace (row-major, nvp per row), zeroed once
    const size_t wsb = sizeof(double) * std::max<int64_t>(G.ws_rows, 1) * G.nvp;
    HIP_TRYB(hipMalloc(reinterpret_cast<void**>(&G.d_ws), wsb), "hipMalloc(workspace)");
    HIP_TRYB(hipMemset(G.d_ws, 0, wsb), "hipMemset(workspace)");
  }
  HIP_TRYB(hipHostMalloc(reinterpret_cast<void**>(&b->h_items), sizeof(BatchItem) * count, hipHostMallocDefault),
           "hipHostMalloc(items)");
  HIP_TRYB(hipMalloc(reinterpret_cast<void**>(&b->d_items), sizeof(BatchItem) * count), "hipMalloc(items)");
  HIP_TRYB(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking), "hipStreamCreate");
  for (size_t gi = 1; gi < b->groups.size(); ++gi) {
    Group& G = b->groups[gi];
    HIP_TRYB(hipStreamCreateWithFlags(&G.st, hipStreamNonBlocking), "hipStreamCreate");
    HIP_TRYB(hipEventCreateWithFlags(&G.ev_go, hipEventDisableTiming), "hipEventCreate");
    HIP_TRYB(hipEventCreateWithFlags(&G.ev_done, hipEventDisableTiming), "hipEventCreate");
  }
  HIP_TRYB(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "hipEventCreate");
  HIP_TRYB(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming), "hipEventCreate");
  HIP_TRYB(hipEventCreateWithFlags(&b->ev_items, hipEventDisableTiming), "hipEventCreate");
  HIP_TRYB(hipDeviceSynchronize(), "hipDeviceSynchronize(batch load)");
  return H2_OK;
}

int run_blaunch(h2_batch_s* b, const Group& G, const Launch& L, hipStream_t s) {
  const double* data = L.arr == ARR_TRANS ? b->d_trans : b->d_mat;
  if ((L.kc == kWaveRows || L.kc == kWaveTiles) && L.max_rows <= 64) {
    const hipError_t e = launch_wave_rows<double>(b->rt.d_rows + L.row_begin, L.row_count, b->rt.d_colend,
                                                  b->rt.d_in_off, data, G.d_ws, G.d_ws, G.nvp, L.mode,
                                                  L.max_rows, s, L.grid, L.kc == kWaveTiles, L.remapp[0], nullptr,
                                                  L.occp[0]);
    if (e != hipSuccess) return hip_fail_b(e, "batch kernel launch");
    return H2_OK;
  }
  hipError_t e = launch_rows_mfma<double>(b->rt.d_rows + L.row_begin, L.row_count, b->rt.d_colend, b->rt.d_in_off,
                                          data, G.d_ws, G.d_ws, G.nvp, L.mode, L.max_rows, s, L.kc, L.grid);
  if (e != hipSuccess) return hip_fail_b(e, "batch kernel launch");
  return H2_OK;
}

// Launches of one phase of every group, merged level `lev` (or all, lev < 0).
int run_phase(h2_batch_s* b, std::vector<Launch> Group::*ph, const std::vector<int64_t> Group::*lv, int64_t lev,
              hipStream_t s) {
  int rc;
  for (const Group& G : b->groups) {
    const std::vector<Launch>& v = G.*ph;
    for (size_t k = 0; k < v.size(); ++k) {
      if (lv && (G.*lv)[k] != lev) continue;
      if ((rc = run_blaunch(b, G, v[k], s))) return rc;
    }
  }
  return H2_OK;
}

// The launch sequence after the items are on the device.
int batch_sequence(h2_batch_s* b, hipStream_t s) {
  int rc;
  for (const Group& G : b->groups)
    HIP_TRYB(launch_batch_permute(b->d_items, G.d_tile_op, G.d_tile_j0, G.ntiles, b->d_pinv, G.d_ws, G.nvp, false, s),
             "batch permute");
  auto fork_dense = [&]() -> int {
    HIP_TRYB(hipEventRecord(b->ev_fork, s), "hipEventRecord");
    HIP_TRYB(hipStreamWaitEvent(b->side, b->ev_fork, 0), "hipStreamWaitEvent");
    int r = run_phase(b, &Group::dense, nullptr, -1, b->side);
    if (r != H2_OK) return r;
    HIP_TRYB(hipEventRecord(b->ev_join, b->side), "hipEventRecord");
    return H2_OK;
  };
  if (b->par && b->groups.size() > 1) {
    if ((rc = fork_dense())) return rc;
    // one stream per group: its upsweep, coupling rows and downsweep; every
    // group's stream forks from this point of the main stream, before the
    // first group's launches are queued on it
    for (size_t gi = 1; gi < b->groups.size(); ++gi) {
      HIP_TRYB(hipEventRecord(b->groups[gi].ev_go, s), "hipEventRecord");
      HIP_TRYB(hipStreamWaitEvent(b->groups[gi].st, b->groups[gi].ev_go, 0), "hipStreamWaitEvent");
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const Group& G = b->groups[gi];
      hipStream_t gs = gi == 0 ? s : G.st;
      for (int64_t h = 0; h <= b->maxq; ++h)
        for (size_t k = 0; k < G.up.size(); ++k)
          if (G.up_level[k] == h && (rc = run_blaunch(b, G, G.up[k], gs))) return rc;
      for (const Launch& L : G.couple)
        if ((rc = run_blaunch(b, G, L, gs))) return rc;
      for (int64_t d = 0; d < b->maxq; ++d)
        for (size_t k = 0; k < G.down.size(); ++k)
          if (G.down_level[k] == d && (rc = run_blaunch(b, G, G.down[k], gs))) return rc;
      if (gi > 0) HIP_TRYB(hipEventRecord(G.ev_done, gs), "hipEventRecord");
    }
    for (size_t gi = 1; gi < b->groups.size(); ++gi)
      HIP_TRYB(hipStreamWaitEvent(s, b->groups[gi].ev_done, 0), "hipStreamWaitEvent");
  } else {
    if (b->sched == 0 && (rc = fork_dense())) return rc;
    for (int64_t h = 0; h <= b->maxq; ++h)
      if ((rc = run_phase(b, &Group::up, &Group::up_level, h, s))) return rc;
    if (b->sched == 1 && (rc = fork_dense())) return rc;
    if ((rc = run_phase(b, &Group::couple, nullptr, -1, s))) return rc;
    for (int64_t d = 0; d < b->maxq; ++d)
      if ((rc = run_phase(b, &Group::down, &Group::down_level, d, s))) return rc;
  }
  HIP_TRYB(hipStreamWaitEvent(s, b->ev_join, 0), "hipStreamWaitEvent");
  if ((rc = run_phase(b, &Group::out, nullptr, -1, s))) return rc;
  for (const Group& G : b->groups)
    HIP_TRYB(launch_batch_permute(b->d_items, G.d_tile_op, G.d_tile_j0, G.ntiles, b->d_pinv, G.d_ws, G.nvp, true, s),
             "batch permute out");
  return H2_OK;
}

int fill_items(h2_batch_s* b, const h2_batch_item* items) {
  // the previous call's copy of the items must have left the pinned buffer
  if (b->items_pending) HIP_TRYB(hipEventSynchronize(b->ev_items), "hipEventSynchronize(items)");
  for (int64_t i = 0; i < b->count; ++i) {
    const h2_batch_item& it = items[i];
    if (it.nv < 0 || it.nv > b->nv_max[i]) {
      set_error("batch item " + std::to_string(i) + ": nv outside [0, the operator's nv_max]");
      return H2_EINVAL;
    }
    if (it.nv > 0) {
      if (!it.Y || it.ldy < b->n[i] || (it.alpha != 0.0 && (!it.X || it.ldx < b->n[i]))) {
        set_error("batch item " + std::to_string(i) + ": bad pointer or leading dimension");
        return H2_EINVAL;
      }
    }
    BatchItem& d = b->h_items[i];
    d.X = it.X; d.Y = it.Y; d.ldx = it.ldx; d.ldy = it.ldy; d.nv = it.nv;
    d.alpha = it.alpha; d.beta = it.beta; d.n = b->n[i];
    d.pinv_off = b->pinv_off[i]; d.xt_row = b->xt_row[i]; d.zn_row = b->zn_row[i];
  }
  return H2_OK;
}

int64_t launch_count(const h2_batch_s* b) {
  int64_t l = 0;
  for (const Group& G : b->groups)
    l += 2 + (int64_t)(G.up.size() + G.couple.size() + G.down.size() + G.dense.size() + G.out.size());
  return l;
}

}  // namespace
}  // namespace h2

using namespace h2;

extern "C" {

int h2_batch_load_ex(const void* const* bufs, const size_t* lens, int64_t count, const int64_t* nv_max, int device,
                     h2_batch* out) {
  if (!out || !bufs || !lens || !nv_max || count < 1) {
    set_error("h2_batch_load: bad arguments");
    return H2_EINVAL;
  }
  *out = nullptr;
  for (int64_t i = 0; i < count; ++i) {
    if (!bufs[i]) { set_error("h2_batch_load: null buffer"); return H2_EINVAL; }
    if (nv_max[i] < 1 || nv_max[i] > kPassVectorsMfma) {
      set_error("h2_batch_load: nv_max of operator " + std::to_string(i) + " outside [1, 64]");
      return H2_EINVAL;
    }
  }
  int ndev = 0;
  HIP_TRYB(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) { set_error("device ordinal out of range"); return H2_EINVAL; }
  DevGuard guard(device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  h2_batch_s* b = new (std::nothrow) h2_batch_s();
  if (!b) { set_error("out of host memory"); return H2_ENOMEM; }
  b->device = device;
  b->count = count;
  int rc;
  try {
    b->nv_max.assign(nv_max, nv_max + count);
    rc = batch_build(bufs, lens, count, b);
  } catch (const std::bad_alloc&) {
    set_error("out of host memory while building the batch");
    rc = H2_ENOMEM;
  }
  if (rc != H2_OK) {
    (void)hipDeviceSynchronize();
    free_batch(b);
    delete b;
    return rc;
  }
  *out = b;
  return H2_OK;
}

int h2_batch_load(const void* const* bufs, const size_t* lens, int64_t count, int64_t nv_max, int device,
                  h2_batch* out) {
  if (count < 1) {
    set_error("h2_batch_load: bad arguments");
    return H2_EINVAL;
  }
  std::vector<int64_t> v;
  try {
    v.assign((size_t)count, nv_max);
  } catch (const std::bad_alloc&) {
    set_error("out of host memory");
    return H2_ENOMEM;
  }
  return h2_batch_load_ex(bufs, lens, count, v.data(), device, out);
}

int h2_batch_gemv(h2_batch b, const h2_batch_item* items, void* stream) {
  if (!b || !items) { set_error("null batch or items"); return H2_EINVAL; }
  DevGuard guard(b->device);
  if (!guard.ok) { set_error("hipSetDevice failed"); return H2_EHIP; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = fill_items(b, items);
  if (rc != H2_OK) return rc;
  if (b->use_graph && b->graph && b->graph_stream == s) {
    HIP_TRYB(hipGraphLaunch(b->graph, s), "hipGraphLaunch");
    // the next call may refill the pinned items once this replay has run
    HIP_TRYB(hipEventRecord(b->ev_items, s), "hipEventRecord(items)");
    b->items_pending = true;
    return H2_OK;
  }
  const bool capture = b->use_graph && s != nullptr;
  if (capture) HIP_TRYB(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  auto body = [&]() -> int {
    HIP_TRYB(hipMemcpyAsync(b->d_items, b->h_items, sizeof(BatchItem) * b->count, hipMemcpyHostToDevice, s),
             "hipMemcpyAsync(items)");
    HIP_TRYB(hipEventRecord(b->ev_items, s), "hipEventRecord(items)");
    return batch_sequence(b, s);
  };
  rc = body();
  if (capture) {
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != H2_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail_b(e, "hipStreamEndCapture");
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    const hipError_t ei = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return hip_fail_b(ei, "hipGraphInstantiate");
    b->graph_stream = s;
    HIP_TRYB(hipGraphLaunch(b->graph, s), "hipGraphLaunch");
    HIP_TRYB(hipEventRecord(b->ev_items, s), "hipEventRecord(items)");
  } else if (rc != H2_OK) {
    return rc;
  }
  b->items_pending = true;
  return H2_OK;
}

int h2_batch_tune(h2_batch b, const h2_batch_item* items, void* stream) {
  if (!b || !items) { set_error("null batch or items"); return H2_EINVAL; }
  DevGuard guard(b->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool graph_was = b->use_graph;
  b->use_graph = false;
  if (b->graph) { (void)hipGraphExecDestroy(b->graph); b->graph = nullptr; }
  int rc = h2_batch_gemv(b, items, stream);  // fills the workspace with this call's data
  if (rc != H2_OK) { b->use_graph = graph_was; return rc; }
  HIP_TRYB(hipStreamSynchronize(s), "hipStreamSynchronize");
  hipEvent_t e0, e1;
  HIP_TRYB(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRYB(hipEventCreate(&e1), "hipEventCreate");
  // chunk widths of the LDS-staged kernel; a wave per row; a wave per 16-vector tile
  const int kcs[4] = {32, 64, kWaveRows, kWaveTiles};
  const int64_t grids[4] = {0, 1024, 2048, 4096};
  for (Group& G : b->groups)
    for (auto* v : {&G.up, &G.couple, &G.down, &G.dense, &G.out})
      for (Launch& L : *v) {
        float best = 1e30f;
        int best_kc = L.kc, best_remap = L.remapp[0], best_occ = L.occp[0];
        int64_t best_grid = L.grid;
        for (int kc : kcs)
          for (int64_t gsz : grids)
            for (int cand = 0; cand < 4; ++cand) {
            // XCD ranges and the five-waves-per-SIMD form: wave-row kernels only
            const int remap = cand & 1, occ = cand >> 1 ? 5 : 0;
            const bool wave = kc == kWaveRows || kc == kWaveTiles;
            if (gsz != 0 && gsz >= L.row_count) continue;
            if (wave && L.max_rows > 64) continue;
            if (kc == kWaveTiles && G.nvp != 32 && G.nvp != 64) continue;
            if ((remap || occ) && !wave) continue;
            if (occ && !wave_occ5(G.nvp, L.max_rows, kc == kWaveTiles)) continue;
            Launch T = L;
            T.kc = kc;
            T.grid = gsz;
            T.remapp[0] = remap;
            T.occp[0] = occ;
            float tsum = 0.0f;
            for (int rep = 0; rep < 3; ++rep) {
              HIP_TRYB(hipEventRecord(e0, s), "hipEventRecord");
              if ((rc = run_blaunch(b, G, T, s))) return rc;
              HIP_TRYB(hipEventRecord(e1, s), "hipEventRecord");
              HIP_TRYB(hipEventSynchronize(e1), "hipEventSynchronize");
              float ms = 0.0f;
              HIP_TRYB(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
              if (rep > 0) tsum += ms;  // first repetition warms up
            }
            if (tsum < best) {
              best = tsum;
              best_kc = kc;
              best_grid = gsz;
              best_remap = remap;
              best_occ = occ;
            }
          }
        L.kc = best_kc;
        L.grid = best_grid;
        L.remapp[0] = best_remap;
        L.occp[0] = best_occ;
        L.tuned_ms[0] = best / 2;
      }
  // the dense rows' schedule, on whole launch sequences (a warm-up, then two
  // timed runs each)
  for (int sc = 0; sc < 3; ++sc) {  // dense from the start; after the upsweep; groups side by side
    b->sched = sc == 1 ? 1 : 0;
    b->par = sc == 2;
    float t = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
      HIP_TRYB(hipEventRecord(e0, s), "hipEventRecord");
      if ((rc = batch_sequence(b, s))) return rc;
      HIP_TRYB(hipEventRecord(e1, s), "hipEventRecord");
      HIP_TRYB(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.0f;
      HIP_TRYB(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (rep > 0) t += ms;
    }
    b->sched_ms[sc] = t / 2;
  }
  int best = 0;
  for (int sc = 1; sc < 3; ++sc)
    if (b->sched_ms[sc] < 0.99f * b->sched_ms[best]) best = sc;  // a later form only when 1% faster
  b->sched = best == 1 ? 1 : 0;
  b->par = best == 2;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->use_graph = graph_was;
  return H2_OK;
}

int h2_batch_graph(h2_batch b, int enable) {
  if (!b) { set_error("null batch"); return H2_EINVAL; }
  DevGuard guard(b->device);
  HIP_TRYB(hipDeviceSynchronize(), "hipDeviceSynchronize");
  b->use_graph = enable != 0;
  if (b->graph) { (void)hipGraphExecDestroy(b->graph); b->graph = nullptr; }
  return H2_OK;
}

int h2_batch_info(h2_batch b, int64_t* count, int64_t* total_n, double* flops_per_vector, int64_t* launches) {
  if (!b) { set_error("null batch"); return H2_EINVAL; }
  if (count) *count = b->count;
  if (total_n) *total_n = b->total_n;
  if (flops_per_vector) *flops_per_vector = b->flops_per_vector;
  if (launches) *launches = launch_count(b);
  return H2_OK;
}

int h2_batch_plan_info(h2_batch b, char* buf, size_t cap, size_t* needed) {
  if (!b || !needed) { set_error("null batch or size output"); return H2_EINVAL; }
  std::string t;
  char line[256];
  std::snprintf(line, sizeof line, "schedule %s (tuned calls %.3f / %.3f / %.3f ms)\n",
                b->par ? "groups side by side" : b->sched == 1 ? "dense after the upsweep" : "dense from the start",
                b->sched_ms[0], b->sched_ms[1], b->sched_ms[2]);
  t += line;
  for (const Group& G : b->groups) {
    std::snprintf(line, sizeof line, "group nvp=%d\n", G.nvp);
    t += line;
    const char* names[5] = {"up", "couple", "down", "dense", "out"};
    int k = 0;
    for (const auto* v : {&G.up, &G.couple, &G.down, &G.dense, &G.out}) {
      for (const Launch& L : *v) {
        std::snprintf(line, sizeof line, "%s rows=%lld max_rows=%d kc=%d grid=%lld xcd=%d occ=%d %.3fms\n",
                      names[k], (long long)L.row_count, L.max_rows, L.kc, (long long)L.grid, L.remapp[0], L.occp[0],
                      L.tuned_ms[0]);
        t += line;
      }
      ++k;
    }
  }
  *needed = t.size() + 1;
  if (buf && cap > 0) {
    const size_t c = std::min(cap - 1, t.size());
    std::memcpy(buf, t.data(), c);
    buf[c] = 0;
  }
  return H2_OK;
}

int h2_batch_free(h2_batch b) {
  if (!b) return H2_OK;
  {
    DevGuard guard(b->device);
    (void)hipDeviceSynchronize();
    free_batch(b);
  }
  delete b;
  return H2_OK;
}

}  // extern "C"
