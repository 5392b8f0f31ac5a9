/*
 * h2.h -- C ABI of the MI355X H^2 matrix-vector product library (libh2gemv.so).
 *
 * The library applies one H^2 matrix
 *     A = A_de + <U, S, V^T>                      (Section 2.1 of the paper)
 * to a block of nv vectors on one GPU:
 *     Y <- alpha * op(A) * X + beta * Y,   op(A) = A or A^T,
 * by the three phases of Section 3 -- the upsweep of the column basis tree
 * (x^ = V^T x, Section 3.1 / Algorithm 1), the level-wise coupling product
 * (y^ = S x^, Section 3.2 / Algorithm 4), the downsweep of the row basis
 * tree (y = U y^, Section 3.3 / Algorithm 6) -- plus the block-sparse product
 * with the dense leaf blocks A_de (Section 3).  The operator's data comes
 * from the serialized representation "H2MATV01" (layout documented in the
 * design notes and in h2gen/fmt.py): cluster tree, permutation, per-level
 * ranks, leaf bases U (and V), transfers E (and F), coupling blocks S in CSR
 * per level, dense blocks D in CSR over leaves, all FP64, column-major.
 *
 * Conventions for every entry point
 *   - Return value: H2_OK (0) or a negative H2_E* code; on error a message is
 *     available from h2_last_error() in the calling thread.
 *   - No entry point throws or aborts; HIP errors are reported as H2_EHIP.
 *   - Handles own all device memory they allocate; callers own X and Y.
 */
#ifndef H2_H_
#define H2_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2_op_s* h2_handle;

enum {
  H2_OK = 0,
  H2_EINVAL = -1,      /* bad argument: NULL handle or pointer, bad op, nv < 0,
                          leading dimension < n, X and Y overlap */
  H2_EIO = -2,         /* file could not be read */
  H2_EFORMAT = -3,     /* not a valid representation (magic, version, sizes,
                          tree, permutation, CSR structure, a point
                          dimension above 64) */
  H2_ENOMEM = -4,      /* host or device allocation failed */
  H2_EHIP = -5,        /* other HIP runtime error (message has the HIP text) */
  H2_EUNSUPPORTED = -6 /* valid, but outside this build's limits (a rank or a
                          leaf size above 256, n >= 2^31) */
};

/* Precision of the low-rank phases (leaf and transfer sweeps, coupling
 * products, leaf expansion) in h2_gemv_ex.  The dense near-field products
 * and the final Y update always run in FP64. */
enum {
  H2_PREC_FP64 = 0, /* everything in FP64 */
  H2_PREC_FP32 = 1, /* low-rank data stored and multiplied in FP32, FP32 accumulation */
  H2_PREC_BF16 = 2  /* low-rank data in BF16 on the BF16 matrix cores, FP32 accumulation;
                       op 'N' only (vectors are padded to multiples of 16) */
};

/* Structure and algorithmic work of a loaded operator.  "entries" count the
 * stored FP64 values of each part; when V, F are shared with U, E they are
 * still counted, because the product reads them in both sweeps. */
typedef struct {
  int64_t n;              /* matrix order */
  int64_t depth;          /* leaf level q (root is level 0) */
  int64_t nnodes;         /* cluster-tree nodes */
  int64_t nleaves;        /* leaves (nodes of level q) */
  int64_t ncoupling;      /* coupling blocks, all levels */
  int64_t ndense;         /* dense leaf blocks */
  int64_t csp;            /* largest number of coupling blocks in a block row
                             or column of any level (sparsity constant) */
  int64_t csp_dense;      /* largest number of dense blocks in a leaf row/column */
  int64_t entries_U, entries_V, entries_E, entries_F, entries_S, entries_D;
  int64_t tree_rows;      /* sum over nodes of the node's rank: the length of
                             the vector trees x^ and y^ for one vector */
  int64_t shared_basis;   /* 1 when V = U and F = E */
  int64_t device_bytes;   /* device memory held by the handle now */
  int64_t max_rank;       /* largest rank of any level */
  int64_t max_leaf;       /* largest leaf size */
  /* Algorithmic work of one FP64 product with nv vectors (every stored entry
   * read once, the vector trees x^ and y^ written once and read once):
   *   flops = alg_flops_per_vector * nv + 2 n nv if beta != 0
   *   bytes = alg_bytes_matrix + alg_bytes_per_vector * nv + 8 n nv if beta != 0 */
  double alg_flops_per_vector;  /* 2 * (all stored entries) + n (the alpha scaling) */
  double alg_bytes_matrix;      /* 8 * (all stored entries) */
  double alg_bytes_per_vector;  /* 8 * (2 n + 4 tree_rows): X read, Y written, x^ and y^ */
} h2_stats_t;

/* Structure of one level of the cluster tree (root = level 0). */
typedef struct {
  int64_t nodes;            /* nodes of the level */
  int64_t krow, kcol;       /* ranks of the row and column bases on the level */
  int64_t coupling_blocks;  /* coupling blocks S_ts with t, s on the level */
  int64_t csp;              /* largest number of coupling blocks in a block row or column of the level */
  int64_t entries_S;        /* stored entries of those blocks */
  int64_t entries_E;        /* stored entries of the level's transfers E (0 on the root level) */
  int64_t entries_F;        /* the same for F (counted even when F = E) */
} h2_level_stats_t;

/* Per-phase GPU time accumulated over the h2_gemv calls made while profiling
 * was on (h2_profile), measured with HIP events recorded on the stream each
 * phase runs on.  Times in milliseconds. */
typedef struct {
  int64_t calls;          /* h2_gemv calls profiled */
  double ms_permute;      /* input permutation into tree order */
  double ms_upsweep;      /* leaf products V^T x and transfer upsweep */
  double ms_coupling;     /* coupling products, all levels */
  double ms_downsweep;    /* transfer downsweep (on the multi-vector path, with the leaf
                             expansion U y^, which runs beside the dense rows there) */
  double ms_dense;        /* dense near-field blocks: the sum of the durations of its two
                             halves on the side stream (the first runs beside the upsweep,
                             the second beside the downsweep and the leaf expansion) */
  double ms_leaf_out;     /* leaf expansion U y^ and the alpha/beta update (the output
                             permutation and update only, on the multi-vector path) */
  double ms_total;        /* first to last event of each call, summed */
} h2_profile_t;

/* Load the representation stored in the file at `path` onto GPU `device`
 * (a HIP device ordinal) and build the launch schedules.  On success *out
 * receives a handle that owns all device memory.  Errors: H2_EINVAL,
 * H2_EIO, H2_EFORMAT, H2_ENOMEM, H2_EHIP, H2_EUNSUPPORTED. */
int h2_load(const char* path, int device, h2_handle* out);

/* As h2_load, from a host buffer of `len` bytes holding the serialized
 * representation (8-byte aligned).  The buffer is only read during the
 * call; the caller keeps ownership. */
int h2_load_mem(const void* buf, size_t len, int device, h2_handle* out);

/* Validate a serialized representation on the host only (no GPU is
 * touched).  Returns H2_OK, H2_EINVAL, H2_EFORMAT or H2_EUNSUPPORTED. */
int h2_validate(const void* buf, size_t len);

/* Y <- alpha * op(A) * X + beta * Y on the handle's GPU.
 *   op      'N' (A) or 'T' (A^T), either case.
 *   X, Y    DEVICE pointers, caller-owned, FP64, column-major n x nv with
 *           leading dimensions ldx, ldy >= n, rows in the ORIGINAL point
 *           order (the library applies the tree permutation).  X is read
 *           only; X and Y must not overlap.
 *   nv      number of vectors, >= 0; nv == 0 returns H2_OK with no work.
 *   alpha   alpha == 0 means Y <- beta * Y and X is not read.
 *   beta    beta == 0 means Y is overwritten and not read (NaN-safe).
 *   stream  hipStream_t to enqueue on (NULL = the device's null stream).
 * Asynchronous: returns after enqueueing.  The dense near-field phase runs
 * on a second stream owned by the handle, forked from and joined back to
 * `stream` with events, so the call is ordered on `stream` like a single
 * kernel.  Results are deterministic (no floating-point atomics).  A
 * handle's workspace is shared: calls on one handle must not run
 * concurrently on different streams.  The workspace is allocated on the
 * first call unless h2_reserve allocated it first; vectors are processed
 * in passes of up to 4.
 * Errors: H2_EINVAL, H2_ENOMEM, H2_EHIP. */
int h2_gemv(h2_handle h, char op, double alpha, const double* X, int64_t ldx, int64_t nv,
            double beta, double* Y, int64_t ldy, void* stream);

/* As h2_gemv, with the low-rank phases in precision `prec` (H2_PREC_*).
 * The reduced-precision copy of the low-rank data is made on the device by
 * h2_prepare, or by the first call that needs it (device allocation).  The
 * result differs from the FP64 product by the rounding of the low-rank data
 * and arithmetic to that precision (about 1e-7 relative for FP32, 1e-3 for
 * BF16 data with FP32 accumulation).
 * Errors: as h2_gemv, plus H2_EINVAL for an unknown precision and
 * H2_EUNSUPPORTED for BF16 with op 'T'. */
int h2_gemv_ex(h2_handle h, char op, double alpha, const double* X, int64_t ldx, int64_t nv,
               double beta, double* Y, int64_t ldy, int prec, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * product of h2_gemv, same arguments and semantics, with its scratch (the
 * tree-ordered input, the vector trees x^ and y^, the dense partial) in one
 * fixed device array of 64 MiB per GPU that the library holds until the
 * process ends, instead of the handle's workspace.  The call allocates no
 * memory and creates no stream or event (those are made by h2_load).
 * Vectors go in passes of up to 4 columns, as many as fit; one column needs
 * 8 * (2 n + 2 H) bytes, n the matrix order and H = tree_rows of h2_stats,
 * so operators with n + H above 4 Mi rows are refused.  The array is shared
 * by every call on its GPU, whatever the handle, and keeps the last call's
 * contents (no call relies on its initial contents): calls that overlap on
 * one GPU -- on different streams, or from different host threads -- race
 * and give wrong results; calls in order on one stream do not.
 * Errors: as h2_gemv, plus H2_EUNSUPPORTED when one column of scratch does
 * not fit the array. */
int h2_gemv_noalloc(h2_handle h, char op, double alpha, const double* X, int64_t ldx, int64_t nv,
                    double beta, double* Y, int64_t ldy, void* stream);

/* Graph replay of h2_gemv / h2_gemv_ex (enable != 0): the first call with a
 * given set of arguments (op, precision, X, ldx, nv, alpha, beta, Y, ldy and
 * a non-null stream) captures its launch sequence into a HIP graph, and
 * later calls with the same arguments replay it with one launch (X is read
 * afresh at every replay).  Up to 8 graphs are kept per handle, the least
 * recently used dropped first; retuning (h2_tune, h2_tune_set,
 * h2_set_sweeps, h2_set_dense_grid) drops them all.  For repeated products on
 * the same buffers, where launching the sequence costs more than the GPU
 * work (small operators).  Calls on the null stream, or while profiling, are
 * not captured.  No memset nodes are captured.  Disabling drops the graphs.
 * Synchronizes the device.  Errors: H2_EINVAL, H2_EHIP. */
int h2_graph(h2_handle h, int enable);

/* Build the device copy of the low-rank data in precision `prec` now
 * (no-op for H2_PREC_FP64 or when it exists).  Synchronous. */
int h2_prepare(h2_handle h, int prec);

/* Allocate the workspace now (it serves any nv), so that later h2_gemv
 * calls allocate nothing.  nv_max >= 0 is the largest nv the caller plans
 * to pass. */
int h2_reserve(h2_handle h, int64_t nv_max);

/* Autotune the multi-vector (MFMA) path of op 'N' for `nv` vectors in
 * precision `prec`: first it makes the fragment-ordered copy of the op-'N'
 * rows' matrices (FP64 for every row; for FP32 also of the low-rank rows, in
 * FP32; device memory about the size of the matrix data, once per handle):
 * each row's matrix reordered so that a wave of the wave-row kernels reads
 * its MFMA operands of two four-column steps as whole 128-byte lines.  Then,
 * for every launch of the product, each candidate kernel form (the
 * h2_tune_set codes; the wave-row forms with and without the copy; BF16 has
 * one form) and grid (one workgroup per row, or a persistent grid of 1024,
 * 2048 or 4096 workgroups) is timed with
 * HIP events on `stream` (three runs, the first discarded) on zeroed
 * workspace buffers, and the fastest is kept for later calls in that
 * precision (the dense rows, always FP64, keep theirs in the FP64 entry);
 * then the fused sweeps are timed against the tuned per-level sweeps and the
 * faster form is kept (h2_set_sweeps), and the four schedules of
 * h2_set_schedule are timed on whole products (zeroed input) and the
 * fastest is kept (a later schedule in the list only when it is at least 1%
 * faster than the best before it, so that timing noise does not decide).
 * Results do not depend on the choice: every candidate sums each output in
 * the same order, so they are bitwise identical.  For nv <= 4 outside BF16
 * (the streaming path) it times the four schedules of h2_set_schedule on
 * whole products (the median of 3 to 63 products timed one at a time, for
 * about 4 ms per schedule) and keeps the fastest (by the same 1% rule).
 * Synchronous;
 * must not run concurrently with other calls on the handle (it uses the
 * handle's workspace).
 * Errors: H2_EINVAL (null handle, nv < 0, unknown precision), H2_ENOMEM,
 * H2_EHIP. */
int h2_tune(h2_handle h, int64_t nv, int prec, void* stream);

/* Timings and sizes of one recompression (h2_compress). */
typedef struct {
  double ms_orthogonalize;  /* QR upsweeps and the transform of the coupling blocks */
  double ms_reweight;       /* Gram matrices of the block rows and their downsweep */
  double ms_truncate;       /* eigenproblems, new bases and transfers, bottom-up */
  double ms_project;        /* projection of the coupling blocks on the new bases */
  double ms_assemble;       /* building the new handle (downloads, schedules, uploads) */
  int64_t lowrank_entries_before;  /* stored entries of U, E, V, F, S */
  int64_t lowrank_entries_after;
  double sigma_ref_row;     /* reference singular value of the row (and column) tree */
  double sigma_ref_col;
} h2_compress_info_t;

/* Algebraic recompression (Section 5 of the paper): a new handle on the same
 * device holding an H^2 representation of h's matrix with nested orthogonal
 * bases of lower rank.  Steps, on the device: orthogonalize each basis tree
 * (QR upsweep), weight every node by the block row its basis represents (own
 * and ancestors' coupling blocks; block columns too for a shared basis),
 * truncate bottom-up keeping the singular values above tau * sigma_ref
 * (sigma_ref: the largest leaf value of the tree, the 2-norm of the largest
 * low-rank block row), and project the coupling blocks on the new bases.
 * Each level keeps one rank, the largest count its nodes keep.  Dense blocks
 * are copied unchanged; stored points are not carried over.
 *   tau     in [0, 1); values below about 1e-7 reach the rounding of the
 *           squared singular values and keep more vectors than needed
 *   out     receives the new handle (free it with h2_free)
 *   info    optional timings and sizes (may be NULL)
 *   stream  hipStream_t for the device work (NULL = null stream)
 * Synchronous.  h is not modified.  Supported: ranks <= 64, leaf size times
 * rank <= 8192, children times rank times parent rank <= 8192.
 * Errors: H2_EINVAL (null arguments, tau outside [0, 1)), H2_EUNSUPPORTED
 * (limits), H2_ENOMEM, H2_EHIP. */
int h2_compress(h2_handle h, double tau, h2_handle* out, h2_compress_info_t* info, void* stream);

/* Serialize a handle's representation into host memory `buf` of `cap`
 * bytes (the format h2_load_mem reads; points are not included).  *needed
 * receives the size; with buf == NULL only the size is returned.
 * Errors: H2_EINVAL (null handle or size pointer, cap too small), H2_EHIP. */
int h2_export(h2_handle h, void* buf, size_t cap, size_t* needed);

/* Ranks per level of the row and column bases (arrays of at least depth + 1
 * entries, `cap` their length).  Errors: H2_EINVAL. */
int h2_ranks(h2_handle h, int64_t* krow, int64_t* kcol, int64_t cap);

/* Set the multi-vector launch parameters that h2_tune would pick, the same
 * for every launch of precision `prec`: kc = 32 or 64 columns per chunk, 0
 * for the software-pipelined kernel, 1 or 2 for the balanced kernel with 32
 * or 16 columns, 3 or 4 for the balanced kernel with 16 or 32 columns and
 * loads issued two chunks ahead, 5 or 6 for the balanced kernel with 16
 * columns (loads one or two chunks ahead) compiled for four workgroups per
 * CU, 7 or 8 the same with 8 columns and five workgroups per CU (0-8 take
 * passes of 64 vectors, 1-8 rows of at most 64 outputs; other launches use
 * 64 columns), 9 for one wave per row with no LDS staging (rows of at most
 * 64 outputs, any pass width), 10 the same with one wave per 16-vector tile
 * (passes of 32 or 64 vectors), 11 and 12 the forms of 9 and 10 compiled for
 * five waves per SIMD (where one wave holds one 16-vector tile of rows of at
 * most 48 outputs; else the forms of 9 and 10); grid = workgroups (0 = one per
 * row); xcd != 0 for XCD-aware row ranges; tree_order != 0 for tree-ordered
 * coupling and dense rows.  Results do not change (same summation order).  For
 * reproducible timing and for tests.  Errors: H2_EINVAL. */
int h2_tune_set(h2_handle h, int prec, int kc, int64_t grid, int xcd, int tree_order);

/* Workgroups of the dense near-field launches on the multi-vector path
 * (more than 4 vectors): -1 (the default) the grid h2_tune picked, 0 one
 * workgroup per row, a positive count a persistent grid of that many.  The
 * dense rows run on a second stream beside the latency-bound sweeps; a
 * persistent grid holds fewer CU slots, so the sweeps' small launches start
 * sooner.  Results do not change.  Synchronizes the device.
 * Errors: H2_EINVAL. */
int h2_set_dense_grid(h2_handle h, int64_t workgroups);

/* Where the product of op 'N' runs its dense near-field rows and its
 * coupling rows, for precision `prec` (on the multi-vector path, more than 4
 * vectors or BF16, and on the streaming path; h2_tune tunes each path on
 * its own):
 *   0  the dense rows' first half on a second stream beside the upsweep, the
 *      second half beside the downsweep and the leaf expansion
 *   1  the first half beside the coupling launch instead
 *   2  both halves from the start
 *   3  both halves from the start, and the coupling rows of the leaf level
 *      (they need only the leaf products of the upsweep) on a third stream
 *      beside the upper upsweep, the other levels' coupling rows and the
 *      upper downsweep; the last downsweep level waits for them (not with
 *      the fused sweeps, nor for FP32 passes of 64 vectors, which take
 *      schedule 2 instead)
 * Results are bitwise the same; h2_tune keeps the fastest.  Synchronizes the
 * device.  Errors: H2_EINVAL. */
int h2_set_schedule(h2_handle h, int prec, int schedule);

/* How the multi-vector path (op 'N', 64-vector passes or fewer, FP64 and
 * FP32) runs the upsweep, the downsweep and the leaf expansion: fused != 0
 * in a few launches in which each workgroup runs several levels of one
 * subtree (operators whose rows have at most 64 outputs), 0 one launch per
 * level (the default).  Results are bitwise the same; h2_tune keeps the
 * faster.
 * Errors: H2_EINVAL (null handle, precision other than FP64 or FP32),
 * H2_EUNSUPPORTED (fused asked for, but the operator has longer rows). */
int h2_set_sweeps(h2_handle h, int prec, int fused);

/* enable != 0: make the fragment-ordered copy of the rows' matrices for
 * precision `prec` now (see h2_tune) and let every wave-row launch of that
 * precision read it (the dense rows' FP64 entries too); enable == 0: read
 * the column-major data, and free copies that no launch reads any more.
 * Results are bitwise the same either way; h2_tune chooses per launch.
 * Synchronizes the device and drops the captured graphs; must not run
 * concurrently with other calls on the handle.
 * Errors: H2_EINVAL (null handle, precision other than FP64 or FP32),
 * H2_ENOMEM, H2_EHIP. */
int h2_set_fragment_order(h2_handle h, int prec, int enable);

/* A text description of the op-'N' launch plan and its tuned parameters
 * (row order per precision; per launch: rows, chunk width, grid, XCD mapping,
 * fragment-ordered copy and tuned time per precision), NUL-terminated,
 * truncated to `cap` bytes; *needed receives the full size.
 * Errors: H2_EINVAL. */
int h2_plan_info(h2_handle h, char* buf, size_t cap, size_t* needed);

/* Fill *st with the operator's structure and stored-entry counts. */
int h2_stats(h2_handle h, h2_stats_t* st);

/* Fill *out with the structure of level `level` (0 <= level <= depth).
 * Errors: H2_EINVAL (null arguments, level out of range). */
int h2_level_stats(h2_handle h, int64_t level, h2_level_stats_t* out);

/* Matrix order n of a loaded operator, or -1 for a NULL handle. */
int64_t h2_n(h2_handle h);

/* Turn per-phase event timing of h2_gemv on (enable != 0) or off, and reset
 * the accumulated times.  Off by default. */
int h2_profile(h2_handle h, int enable);

/* Synchronize on the recorded events and return the accumulated per-phase
 * times since profiling was last enabled. */
int h2_profile_read(h2_handle h, h2_profile_t* out);

/* Release the handle and its device memory (synchronizes the device first).
 * h2_free(NULL) is a no-op returning H2_OK. */
int h2_free(h2_handle h);

/* ---- Cross-operator batching ------------------------------------------
 * A batch holds several operators in one device arena and applies all of
 * them in one sequence of launches: the leaf products of every operator in
 * one launch, then each transfer level of the upsweep aligned by height from
 * the leaves (Section 3.1, Algorithm 1: uneven trees merge level by level),
 * the coupling products of every level of every operator in one launch
 * (Algorithm 4), the downsweep aligned by depth from the root (Algorithm 6),
 * the dense leaf rows (second stream) and the leaf expansion.  Products run
 * on the FP64 MFMA row kernels with nv_max vectors per row, rounded up to 16
 * (padding vectors are zero); op 'N' only. */
typedef struct h2_batch_s* h2_batch;

/* One operator's product in a batched call:
 * Y <- alpha * A_i * X + beta * Y, X and Y device pointers, column-major
 * n_i x nv in original point order (leading dimensions >= n_i), nv at most
 * the operator's nv_max.  nv == 0 skips the operator; alpha == 0 does not
 * read X; beta == 0 does not read Y. */
typedef struct {
  const double* X;
  int64_t ldx;
  double* Y;
  int64_t ldy;
  int64_t nv;       /* 0 <= nv <= the batch's nv_max */
  double alpha, beta;
} h2_batch_item;

/* Load `count` serialized representations (bufs[i], lens[i] bytes, host
 * memory, only read during the call) onto `device` as one batch whose calls
 * carry at most nv_max (1..64) vectors per operator.  Allocates the arena,
 * the workspace (sum of 2*(n_i + tree rows_i) * roundup16(nv_max) doubles)
 * and the merged schedules.  Errors: as h2_load_mem. */
int h2_batch_load(const void* const* bufs, const size_t* lens, int64_t count, int64_t nv_max, int device,
                  h2_batch* out);

/* As h2_batch_load with a vector bound per operator: operator i's calls
 * carry at most nv_max[i] (1..64) vectors.  Operators are grouped by
 * nv_max rounded up to 16 (the matrix-core tile width): each group has its
 * own workspace and merged launches, so an operator bounded by 16 vectors
 * costs the work of 16, not of the batch's widest operator. */
int h2_batch_load_ex(const void* const* bufs, const size_t* lens, int64_t count, const int64_t* nv_max, int device,
                     h2_batch* out);

/* All products of one call: items[i] belongs to operator i (count items).
 * Asynchronous on `stream`; the items array is copied during the call.
 * Errors: H2_EINVAL (bad item), H2_EHIP. */
int h2_batch_gemv(h2_batch b, const h2_batch_item* items, void* stream);

/* Autotuner: for every merged launch, time each candidate shape (columns
 * staged per LDS chunk: 32 or 64, or one wave per row or per 16-vector tile
 * with no LDS staging, the latter two also with XCD-aware row ranges;
 * workgroups: one per row (four rows for the wave form) or a persistent grid
 * of 1024, 2048 or 4096) on these items and keep the fastest; then time
 * whole calls with the dense rows on the second stream from the start
 * (beside the upsweep) or from the end of the upsweep (beside the coupling
 * launches), and with each vector-width group's sweeps and coupling rows on
 * a stream of its own, and keep the fastest (a later form only when at
 * least 1% faster than the best before it).  Results do not depend on the
 * choices.
 * Synchronous; the workspace content afterwards is unspecified. */
int h2_batch_tune(h2_batch b, const h2_batch_item* items, void* stream);

/* enable != 0: capture the batch's launch sequence into a HIP graph on the
 * next h2_batch_gemv and replay it on later calls (the item array is still
 * read afresh every call).  A later h2_batch_tune drops the graph. */
int h2_batch_graph(h2_batch b, int enable);

/* Number of operators, total order sum n_i, algorithmic flops per vector
 * (2 * stored entries of all parts) and merged launches per call. */
int h2_batch_info(h2_batch b, int64_t* count, int64_t* total_n, double* flops_per_vector, int64_t* launches);

/* A text description of the batch's launch plan: the whole-call schedule
 * with the tuned call times, then per vector-width group and merged launch
 * the phase, rows, largest row, kernel form, grid, XCD mapping and tuned
 * time.  NUL-terminated, truncated to `cap` bytes; *needed receives the full
 * size.  Errors: H2_EINVAL. */
int h2_batch_plan_info(h2_batch b, char* buf, size_t cap, size_t* needed);

/* Release the batch (synchronizes the device first); NULL is a no-op. */
int h2_batch_free(h2_batch b);

/* ---- Serving loop -------------------------------------------------------
 * A server keeps several loaded operators resident and serves matvec
 * requests on them.  A scheduler thread admits work while a slot (a stream
 * with its own workspace) is free and the device-memory budget has room for
 * the call's input/output buffers; requests waiting for the same operator and
 * precision are fused into one multi-vector product (up to max_fuse_nv
 * vectors), so requests arriving while others run join the next call
 * (continuous batching) and calls on different slots overlap on the GPU.
 * Requests hold device pointers (column-major n x nv, leading dimension n,
 * original point order) that must stay valid until the request completes.
 * Nothing in the scheduler allocates device memory or synchronizes the
 * device: the budget is one region allocated at creation, and a precision
 * other than FP64 must have been prepared on an operator (h2_prepare) before
 * requests use it. */
typedef struct h2_server_s* h2_server;

typedef struct {
  int64_t submitted, completed;   /* requests */
  int64_t calls;                  /* fused products issued */
  int64_t vectors;                /* vectors served */
  int64_t max_inflight_calls;     /* largest number of calls running at once */
  int64_t slots;                  /* slots */
  int64_t budget_bytes;           /* device memory for call buffers */
  int64_t hbm_free_at_create;     /* free HBM (hipMemGetInfo) when the budget was taken */
  double alg_bytes;               /* algorithmic bytes of the calls issued: low-rank data at the
                                     call's precision, dense blocks and vectors in FP64 */
  double alg_flops;               /* algorithmic flops of the calls issued (2 per stored entry
                                     and vector, plus n per vector) */
} h2_server_stats_t;

/* Create a server over `nops` loaded handles (all on one device; the server
 * does not own them).  `slots` concurrent calls at most, each slot with a
 * workspace sized for the largest operator; `budget_bytes` of device memory
 * for the calls' fused input/output buffers, taken from the HBM that is free
 * after the slots' workspaces (hipMemGetInfo): budget_bytes <= 0 takes a
 * quarter of it, and a budget above 90% of it is refused (H2_ENOMEM).
 * Admission waits while the budget is exhausted.  `max_fuse_nv` (1..64)
 * vectors per fused call.
 * Errors: H2_EINVAL, H2_ENOMEM, H2_EHIP. */
int h2_server_create(const h2_handle* ops, int64_t nops, int64_t slots, int64_t budget_bytes,
                     int64_t max_fuse_nv, h2_server* out);

/* Queue Y <- op(A_op) X (op 'N', alpha 1, beta 0) in precision `prec`;
 * nv <= max_fuse_nv.  `stream` (a hipStream_t, NULL = the null stream) is
 * the stream whose work produces X: an event recorded on it now orders the
 * server's read of X after that work, so the caller need not synchronize.
 * Y is written by the server's own streams; read it after h2_server_wait.
 * Returns at once with the request id in *id.
 * Errors: H2_EINVAL (bad arguments, a request larger than the budget, a
 * precision not prepared on the operator), H2_EHIP. */
int h2_server_submit(h2_server s, int64_t op, int prec, int64_t nv, const double* X, double* Y, void* stream,
                     int64_t* id);

/* Block until request `id` has completed; *latency_ms (optional) receives
 * the time from submission to completion as seen by the scheduler. */
int h2_server_wait(h2_server s, int64_t id, double* latency_ms);

/* Counters since creation. */
int h2_server_stats(h2_server s, h2_server_stats_t* st);

/* Finish all queued requests, stop the scheduler, release the server. */
int h2_server_free(h2_server s);

/* Message of the last error in the calling thread ("" if none).  The string
 * is owned by the library and valid until the next call in that thread. */
const char* h2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* H2_H_ */
