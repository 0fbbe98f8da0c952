/*
 * hm.h -- C-ABI of the MI355X H-matrix-vector product library (libhm.so).
 *
 * The operation (Kriemann, "Hierarchical Lowrank Arithmetic with Binary
 * Compression"):
 *
 *   y := y + alpha * A x,   A = sum_{b=(tau,sigma) in L(T)} E_tau M_b E_sigma^T
 *
 * over the leaves L(T) of a block tree (Sec. 2.1, Definition "Block Tree").
 * Inadmissible leaves hold a dense block M_b = D_b; admissible leaves hold a
 * low-rank block M_b = U_b V_b^T of fixed accuracy (Eq. (1), Definition
 * "H-Matrix"), optionally in the form W_b diag(s_b) X_b^T whose columns are
 * split into groups stored in different floating-point formats (Sec. 3.3).
 * U and V are stored independently of each other (Sec. 3).  The product only
 * needs the blocks decoded from their storage formats (Sec. 1, Sec. 5.4);
 * here the decoding happens in registers inside the GPU kernels.
 *
 * All index ranges and vectors are in cluster order (the order in which the
 * cluster tree's leaves enumerate the index set).
 *
 * Conventions for every entry point:
 *  - Return value: HM_OK (0) or a negative hm_status.  No C++ exception
 *    crosses this boundary.  hm_last_error() gives a text for the last
 *    failure on the calling thread.
 *  - Arguments, shapes and the partition are validated synchronously before
 *    anything is enqueued; on error nothing is enqueued and outputs are
 *    untouched.
 *  - Device memory (store, vectors, workspace, server arena) is allocated by
 *    the caller and borrowed; it must outlive the handles that use it.
 *  - Streams are hipStream_t passed as void* (NULL = the null stream).
 *    Compute calls are stream-ordered and return after enqueueing.
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hm_status;
#define HM_OK 0
#define HM_EINVAL (-1)      /* bad argument (NULL pointer, negative size, bad option) */
#define HM_EPARTITION (-2)  /* blocks do not tile [0,n_rows) x [0,n_cols) exactly once */
#define HM_ESHAPE (-3)      /* inconsistent block shape, rank or column groups */
#define HM_EDTYPE (-4)      /* unsupported storage / accumulation / vector dtype combination */
#define HM_ENOMEM (-5)      /* caller buffer (store, workspace, arena) too small, or host allocation failed */
#define HM_EDEVICE (-6)     /* HIP runtime error (text via hm_last_error) */
#define HM_EBUSY (-7)       /* server queue full */
#define HM_ESTATE (-8)      /* object in the wrong state (e.g. server stopped, unknown ticket) */
#define HM_ETIMEOUT (-9)    /* hm_wait timed out */

/* Storage formats.  F64, F32, F16, BF16: the IEEE-754 binary formats of
 * Table 1.  DFL16 ... DFL48: the byte-aligned truncated formats with the 11
 * exponent bits of FP64 (DFL, Sec. 3.2): the leading 2, 3, 4, 5 or 6 bytes
 * of the FP64 encoding (sign, exponent, 4 / 12 / 20 / 28 / 36 mantissa
 * bits), rounded to nearest even from FP64; they decode exactly to FP64.
 * AFLP16 ... AFLP48: the byte-aligned adaptive formats of Sec. 3.2 in 2 ..
 * 6 bytes, per data block (a dense block, or the columns of one column
 * group of U_b, or of V_b): values scaled by 2^-k (2^k the power of two at
 * or below the block's smallest nonzero magnitude) and shifted by 1, so
 * d = |v| 2^-k + 1 >= 2; the code holds the sign, the e exponent bits the
 * block's range of d needs (its binary exponents 1 .. 2^e - 1; 0 codes
 * zero) and 8 B - 1 - e mantissa bits of d rounded to nearest even; the
 * stored value sign(v) (d - 1) 2^k.  hm_upload derives k and e from the
 * data.  BFL24, BFL40, BFL48: the byte-aligned formats with FP32's 8
 * exponent bits (BFL, Sec. 3.2) in 3, 5 or 6 bytes (15 / 31 / 39 mantissa
 * bits), rounded to nearest even from FP64; magnitudes below 2^-126 are
 * stored as zero, and hm_upload rejects values that round beyond FP32's
 * range.  BFL in 2 and 4 bytes is BF16 and FP32.  The DFL, AFLP and BFL
 * formats need HM_F64 accumulation.
 * The number of formats is HM_NUM_DTYPES. */
typedef enum {
  HM_F64 = 0, HM_F32 = 1, HM_F16 = 2, HM_BF16 = 3,
  HM_DFL32 = 4, HM_DFL40 = 5, HM_DFL48 = 6, HM_DFL16 = 7, HM_DFL24 = 8,
  HM_AFLP16 = 9, HM_AFLP24 = 10, HM_AFLP32 = 11, HM_AFLP40 = 12, HM_AFLP48 = 13,
  HM_BFL24 = 14, HM_BFL40 = 15, HM_BFL48 = 16
} hm_dtype;
#define HM_NUM_DTYPES 17
typedef enum { HM_DENSE = 0, HM_LOWRANK = 1 } hm_kind;

/* One leaf block b = tau x sigma of the block tree (Sec. 2.1).
 * Ranges are half-open, in cluster order.
 * DENSE:   rank = 0, ngroups = 1, group_dtype[0] = storage dtype of D_b.
 * LOWRANK: rank = k >= 0 (0 = zero block, contributes nothing);
 *          columns 0..k-1 are split into ngroups (1..4) consecutive groups of
 *          group_cols[g] columns stored in group_dtype[g] (Sec. 3.3);
 *          sum(group_cols) == k.  has_sigma = 1: M_b = W diag(s) X^T with
 *          s applied in the accumulation dtype; 0: M_b = U V^T. */
typedef struct {
  int64_t row_begin, row_end, col_begin, col_end;
  int32_t kind, rank;
  int32_t ngroups, group_cols[4], group_dtype[4];
  int32_t has_sigma;
} hm_block_desc;

/* acc_dtype: HM_F64 or HM_F32, the accumulation type of every sum.
 * vec_dtype: must equal acc_dtype (x, y, X, Y are stored in it).
 * Storage dtypes allowed: any with HM_F64 accumulation; F32/F16/BF16 with
 * HM_F32 accumulation (DFL, AFLP and BFL formats need HM_F64 accumulation).
 * max_nrhs: largest nrhs passed to hm_mvm_batch (>= 1); sizes the workspace.
 * tune: 0 = built-in launch parameters; 1 = read tune_cache, a text file
 * written by the tuner with one "key params" line per kind of matrix (see
 * hm_matrix_tune_key and hm_matrix_set_launch); a key that is missing
 * falls back to the built-ins.  tune_cache may be NULL when tune = 0.
 * chunk_rows, tile_groups: the column-tile shape.  The rows of every V_b
 * are cut into chunks of at most chunk_rows rows (64 .. 512), and a chunk's
 * columns into tiles of at most tile_groups 16-byte groups (8 .. 64).  0
 * takes the value from the tune cache line of this kind of matrix (keys
 * "chunk" and "tile"), else the built-ins 512 and 64.  tile_mix: 1 gives
 * every tile one storage format (a chunk's columns of another format start
 * a new tile), 2 lets a tile hold columns of up to four formats, 0 takes
 * the tune cache's "tmix" (0 or 1 there), else the built-in one format per
 * tile.  Results depend on the shape only by rounding (the partial sums are
 * cut differently). */
typedef struct {
  int32_t acc_dtype, vec_dtype, max_nrhs, tune;
  const char* tune_cache;
  int32_t chunk_rows, tile_groups;
  int32_t tile_mix;
} hm_plan_opts;

/* Sizes and byte accounting of a plan (all counts exact).
 * store_bytes: device bytes hm_upload needs (factors + descriptors).
 * work_bytes_per_rhs: workspace bytes hm_mvm needs (hm_mvm_batch: see there).
 * alg_bytes: algorithmic bytes of one single-RHS product: stored factor
 *   elements at their storage width, s_b values, x read once, y read and
 *   written once.  alg_flops: 2 (sum_dense m n + sum_lowrank (m + n) k).
 * overhead_bytes: index/descriptor bytes and padding streamed per product
 *   beyond alg_bytes (reported separately; not counted as algorithmic).
 * bytes_by_dtype: stored factor bytes per storage dtype (index = hm_dtype). */
typedef struct {
  size_t store_bytes, work_bytes_per_rhs;
  double alg_bytes, alg_flops, overhead_bytes;
  int64_t n_dense, n_lowrank, n_row_panels, n_col_tiles, n_partials, n_t;
  size_t bytes_by_dtype[HM_NUM_DTYPES];
} hm_plan_info_t;

typedef struct hm_plan hm_plan;
typedef struct hm_matrix hm_matrix;
typedef struct hm_server hm_server;

/* Block scheduler (host only).  Validates the block table -- shapes, ranks,
 * groups, dtypes, and that the leaves tile [0,n_rows) x [0,n_cols) exactly
 * once, the defining property of the block tree's leaf set (Sec. 2.1) --
 * then lays out the store: every block's rows, cut by elementary row
 * interval (<= 64 rows), form row panels with sections by kind and storage
 * format; the columns of the low-rank blocks, cut by column chunk (the
 * sub-clusters of <= 512 rows recovered from the nested block ranges), form
 * column panels whose 16-byte groups of all formats are cut into tiles of
 * 64 groups; plus work orders and reduction tables.  Copies what it needs
 * from `blocks`.  opts may be NULL (F64, 1 RHS).  Errors: HM_EINVAL,
 * HM_ESHAPE, HM_EDTYPE (the table), HM_EPARTITION (the leaves do not tile
 * the matrix exactly once), HM_ENOMEM (sizes beyond 32-bit indices). */
hm_status hm_build_plan(int64_t n_rows, int64_t n_cols, const hm_block_desc* blocks,
                        int64_t n_blocks, const hm_plan_opts* opts, hm_plan** out);
hm_status hm_plan_info(const hm_plan* p, hm_plan_info_t* out);
void hm_plan_destroy(hm_plan* p);

/* Where entry (i, j) of a block's first factor (which = 0: D_b or U_b / W_b,
 * j < n_b resp. k) or second factor (which = 1: V_b / X_b, i < n_b, j < k)
 * lives in the store: byte offset and storage dtype.  For DFL formats the
 * offset is that of the value's leading 4 bytes (DFL32 / 40 / 48: a
 * little-endian 32-bit word) or 2 bytes (DFL16 / 24: a 16-bit word); for
 * DFL40 / DFL48 / DFL24 its remaining 1 / 2 / 1 bytes (bits 31..24 /
 * 31..16 / 47..40 of the FP64 encoding) are at lo_offset, else lo_offset =
 * 0.  AFLP and BFL values sit like the DFL values of the same byte count (their
 * left-aligned code in place of the FP64 encoding).  lo_offset may be NULL.
 * For tests of the packing and conversion done by hm_upload. */
hm_status hm_plan_locate(const hm_plan* p, int64_t block, int32_t which, int64_t i, int64_t j,
                         size_t* byte_offset, int32_t* dtype, size_t* lo_offset);

/* Device block store.  Converts every factor from FP64 to its storage dtype
 * with round-to-nearest-even (rounded once, directly from FP64), packs it
 * into the plan's panel layout with its descriptors, and copies the result
 * to d_store (device, >= store_bytes, 256-byte aligned, on the current
 * device) on `stream`; the call returns after the copy has completed.  Per
 * block b (host, FP64, column-major): a[b] = D_b (m x n_b) or U_b / W_b
 * (m x k); bf[b] = NULL or V_b / X_b (n_b x k); s[b] = NULL or s_b (k
 * values, when has_sigma).  The factor data is packed and copied in windows
 * (256 MiB; the environment variable HM_UPLOAD_WINDOW_BYTES, >= 4096,
 * overrides) through two pinned host buffers, so the host memory used
 * beyond the caller's factors is the descriptor tables plus two windows.
 * Converting each block after assembly follows Sec. 5.3.  Errors: HM_EINVAL
 * (NULL or missing factor pointers, alignment, an AFLP data block with a
 * value that is not finite or a range whose exponents need more than 10
 * bits or leave no mantissa bit; a BFL value that is not finite or rounds
 * beyond FP32's range), HM_ENOMEM (store too small,
 * pinned staging), HM_EDEVICE (no usable device, copy failure). */
hm_status hm_upload(const hm_plan* p, const double* const* a, const double* const* bf,
                    const double* const* s, void* d_store, size_t store_bytes, void* stream,
                    hm_matrix** out);
void hm_matrix_destroy(hm_matrix* A);

/* The packing half of hm_upload into host memory h_buf (>= store_bytes),
 * with no device involved; the bytes are exactly what hm_upload copies to
 * the device.  For inspection and tests of the store layout. */
hm_status hm_pack_host(const hm_plan* p, const double* const* a, const double* const* bf,
                       const double* const* s, void* h_buf, size_t buf_bytes);

/* y := y + alpha A x (single right-hand side).  d_x: n_cols vector, d_y:
 * n_rows vector, both device memory in vec_dtype; x must not alias y.
 * d_work: device workspace of >= work_bytes_per_rhs bytes, 256-byte aligned;
 * concurrent calls on one matrix need distinct workspaces.  The result is
 * deterministic: every sum has a fixed order independent of timing. */
hm_status hm_mvm(const hm_matrix* A, double alpha, const void* d_x, void* d_y, void* d_work,
                 size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): hm_mvm
 * with the workspace taken from a fixed array of HM_NOALLOC_SCRATCH_BYTES in
 * device memory that the library holds, one copy per GPU, until the process
 * ends.  Same arguments, kernels and result (bit for bit) as hm_mvm.  The
 * call allocates nothing: no hipMalloc, hipFree or allocating library call;
 * on the first call on a device it looks up that device's copy of the array.
 * The current device must be the matrix's (else HM_EINVAL).  A matrix whose
 * work_bytes_per_rhs exceeds HM_NOALLOC_SCRATCH_BYTES is rejected with
 * HM_ENOMEM before anything is launched.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (two streams, or two host
 * threads without stream ordering between them) race and give undefined
 * results; calls ordered on one stream are safe.  The array keeps the last
 * call's contents; the product writes every workspace entry it reads within
 * the call, so nothing needs clearing. */
#define HM_NOALLOC_SCRATCH_BYTES (64u << 20)
hm_status hm_mvm_noalloc(const hm_matrix* A, double alpha, const void* d_x, void* d_y, void* stream);

/* Y := Y + alpha A X for nrhs right-hand sides (1 <= nrhs <= max_nrhs).
 * X is n_cols x nrhs, Y is n_rows x nrhs, column-major with leading
 * dimensions ldx >= n_cols, ldy >= n_rows; X must not overlap Y.
 * Workspace: at least slots * work_bytes_per_rhs bytes, where slots = 32 for
 * nrhs <= 32 and 64 otherwise with HM_F32 accumulation (right-hand sides run
 * in groups of up to 64 on the matrix cores), and slots = 1 with HM_F64
 * accumulation (right-hand sides run one after another).
 * HM_F32: every result column depends only on its own right-hand side, so a
 * column's result is bitwise the same whatever else is in the batch; it
 * agrees with hm_mvm up to the rounding of the accumulation order.
 * HM_F64: each column is computed exactly as hm_mvm computes it. */
hm_status hm_mvm_batch(const hm_matrix* A, int32_t nrhs, double alpha, const void* d_X,
                       int64_t ldx, void* d_Y, int64_t ldy, void* d_work, size_t work_bytes,
                       void* stream);

/* HIP graph of one product.  hm_graph_create records into a graph the
 * kernel launches that hm_mvm (nrhs == 1; ldx and ldy are ignored) or
 * hm_mvm_batch (nrhs > 1) would enqueue with these arguments and the
 * matrix's current launch parameters, checks the arguments as those calls
 * do, and instantiates the graph on the current device (which must be the
 * matrix's).  hm_graph_launch enqueues one replay on `stream`: the same
 * product, y += alpha A x, on the same buffers, bit for bit what the eager
 * call gives.  The graph holds the device addresses of A's store, x, y and
 * the workspace: they must stay allocated until hm_graph_destroy; their
 * contents may change between replays.  Replays that overlap in time (on
 * different streams) race on y and the workspace.  The graph contains
 * kernels only (no memory set, copy or allocation nodes).  Later changes
 * of the launch parameters do not affect an existing graph.  Errors:
 * HM_EINVAL (arguments, wrong device), HM_ENOMEM (workspace), HM_EDEVICE
 * (capture or instantiation failed; text via hm_last_error). */
typedef struct hm_graph hm_graph;
hm_status hm_graph_create(const hm_matrix* A, int32_t nrhs, double alpha, const void* d_X, int64_t ldx,
                          void* d_Y, int64_t ldy, void* d_work, size_t work_bytes, hm_graph** out);
hm_status hm_graph_launch(hm_graph* g, void* stream);
void hm_graph_destroy(hm_graph* g);

/* Kernel timing for measurement.  While enabled, each hm_mvm / hm_mvm_batch
 * call on A records HIP events around each of its kernels on the call's
 * stream, for up to max_calls calls (later calls are not recorded).
 * hm_profile_end waits for the recorded events, returns the summed
 * milliseconds per kernel -- ms[0] column tiles (far field, phase 1), ms[1]
 * partial reduction, ms[2] row panels (near field and far field, phase 2) --
 * and the number of calls recorded, and stops recording.  Events are owned
 * by the library. */
hm_status hm_profile_begin(hm_matrix* A, int32_t max_calls);
hm_status hm_profile_end(hm_matrix* A, double* ms, int64_t* calls);

/* Launch parameters of one matrix, as text
 * "schedule=S unroll=U order=O persist=P" (any subset of the keys; the
 * built-in choice is schedule=0 unroll=8 order=1 persist=0; the text
 * hm_matrix_get_launch writes, and a tune cache line, also name the plan's
 * tile shape, "chunk=C tile=G tmix=M", which hm_matrix_set_launch accepts
 * only with the plan's own values; tmix 0, the built-in, gives every column
 * tile one storage format, tmix 1 lets a tile hold up to four; the
 * batched column-tile variant "colb=B" (0 .. 3) is set the same way):
 *   schedule 0: column tiles, partial reduction, whole row panels;
 *   schedule 1: one grouped launch of the dense row-panel sections with the
 *               column tiles, the reduction, then the U sections;
 *   unroll 4 or 8: 16-byte groups each wave keeps in flight in row panels;
 *   order 0: row panels largest first; order 1: row panels in cluster order,
 *            cut into 8 contiguous ranges, one per XCD, so that neighbouring
 *            panels share one L2 (whole-panel kernels: schedule 0 and the
 *            batched path);
 *   persist 0: one workgroup per work item (row panel, column tile);
 *   persist 1, 2, 4 or 8: single-right-hand-side kernels run persistent
 *            grids of at most that many workgroups per compute unit, each
 *            looping over work items in the same order;
 *   colw 0: single-right-hand-side column tiles (schedule 0) run a
 *            workgroup per tile, its four waves taking turns over the tile's
 *            rows; colw 2: a wave per tile; colw 1 (built in): a wave per tile
 *            in the launch classes of small tiles (where a workgroup would
 *            leave more than a quarter of its waves' turns idle).
 * Unroll depth, order and persistence do not change any sum's order (results
 * are identical bit for bit); schedule 1 adds the near-field and far-field parts
 * to y in two steps, so it differs from schedule 0 by rounding only; colw
 * changes the order in which a column tile's rows are added.  Each
 * choice is deterministic.  hm_matrix_tune_key writes the key under which the
 * tuner stores the best choice for matrices of this kind (accumulation type,
 * storage formats present, size class, rank class = floor(log2) of the mean
 * rank of the low-rank blocks, and whether the plan was made for several
 * right-hand sides) into buf (NUL-terminated, <= len). */
hm_status hm_matrix_set_launch(hm_matrix* A, const char* params);
hm_status hm_matrix_get_launch(const hm_matrix* A, char* buf, size_t len);
hm_status hm_matrix_tune_key(const hm_matrix* A, char* buf, size_t len);

/* Reorders vectors between the caller's index order and the cluster order
 * every product uses (the cluster tree orders the index set, Sec. 2.1; the
 * block table's ranges are in cluster order).  Not part of a product.
 * d_perm: device int64[n], perm[i] = caller index of cluster position i (a
 * permutation of [0, n)).  direction 0: out[i] = in[perm[i]] (into cluster
 * order); 1: out[perm[i]] = in[i] (back).  nvec vectors, column-major with
 * leading dimensions ld_in, ld_out >= n; dtype HM_F64 or HM_F32 (in and out
 * alike).  in and out must not overlap.  A perm entry outside [0, n) is
 * never dereferenced: direction 0 writes NaN at that position, direction 1
 * writes nothing for it.  Stream-ordered; returns after enqueueing.
 * Errors: HM_EINVAL (NULL pointers, n < 1, nvec < 1, ld < n, direction),
 * HM_EDTYPE (dtype), HM_EDEVICE (launch failure). */
hm_status hm_permute(const int64_t* d_perm, int64_t n, int32_t dtype, int32_t direction, int32_t nvec,
                     const void* d_in, int64_t ld_in, void* d_out, int64_t ld_out, void* stream);

/* Streaming-read probe for measurement: reads `bytes` (a multiple of 16) of
 * device memory at d_buf with the 16-byte loads the kernels use, on stream.
 * d_out: device memory of >= 4 bytes (written only in a case that does not
 * occur for real data; it keeps the reads from being removed). */
hm_status hm_stream_read(const void* d_buf, size_t bytes, void* d_out, void* stream);

/* Request loop with continuous batching over device-resident matrices:
 * requests of one matrix are batched into hm_mvm_batch calls, so a
 * request's result does not depend on the batch it lands in (FP32: bitwise
 * by construction; FP64: each column is computed as hm_mvm computes it).
 * mats: matrices to serve (borrowed; all on the current device).  d_arena:
 * device memory (arena_bytes, 256-byte aligned) from which each batch's
 * vectors and workspace are carved by a first-fit allocator; a batch is
 * admitted when its footprint fits in the free part of the arena (HBM-budget
 * admission) and otherwise waits; a request that can never fit completes
 * with HM_ENOMEM.  streams: n_streams HIP streams (borrowed), one per slot.
 * A dispatcher thread batches queued requests of the same matrix (FIFO, up
 * to its max_nrhs) and hands each batch to an idle slot; the slot's worker
 * thread gathers the right-hand sides into pinned host memory, runs copy,
 * product and copy-back on its stream, scatters the results and completes
 * the tickets.  Test hook: the environment variable HM_SERVER_FAULT_EVERY=N
 * (read here) fails every N-th batch with HM_EDEVICE before it is enqueued.
 * Errors: HM_EINVAL (arguments, alignment). */
hm_status hm_server_create(hm_matrix* const* mats, int32_t n_mats, void* d_arena,
                           size_t arena_bytes, void* const* streams, int32_t n_streams,
                           hm_server** out);
/* Queue Y := A_mat X (Y overwritten) for host buffers X (n_cols x nrhs,
 * leading dimension ldx) and Y (n_rows x nrhs, ldy) in the matrix's
 * vec_dtype; both must stay valid until the ticket completes.  Thread-safe.
 * Errors: HM_EINVAL (arguments), HM_ESTATE (server stopping), HM_EBUSY
 * (queue full). */
hm_status hm_submit(hm_server* s, int32_t mat, int32_t nrhs, const void* h_X, int64_t ldx,
                    void* h_Y, int64_t ldy, uint64_t* ticket);
/* Whether a ticket has completed and with which status (HM_ESTATE for an
 * unknown ticket); hm_wait blocks up to timeout_us (< 0: no limit) and
 * returns HM_ETIMEOUT if the ticket is still running.  Once either call has
 * reported a ticket done (hm_poll with *done = 1, or hm_wait returning
 * HM_OK), the server forgets the ticket: later calls on it return
 * HM_ESTATE.  A completed ticket that is never reported stays until the
 * server is destroyed. */
hm_status hm_poll(hm_server* s, uint64_t ticket, int32_t* done, hm_status* result);
hm_status hm_wait(hm_server* s, uint64_t ticket, int64_t timeout_us, hm_status* result);
/* Latency percentiles (microseconds, completion minus submission) over the
 * most recent 2^20 completed requests, and throughput (right-hand sides
 * completed per second, from the first submission to the last completion)
 * since creation. */
hm_status hm_server_stats(hm_server* s, double* p50_us, double* p99_us, double* matvecs_per_s);
/* Serves every queued request, then stops the threads and frees the
 * server's pinned memory (the arena and streams stay the caller's). */
void hm_server_destroy(hm_server* s);

/* Text of the last error on the calling thread (valid until the next hm_*
 * call on this thread); "" when the last call succeeded. */
const char* hm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
