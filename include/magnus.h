/*
 * magnus.h -- C ABI of a gfx950 (MI355X) sparse matrix-matrix product
 * C = A * B in CSR, by Gustavson's row-wise method with the intermediate
 * products of long rows reordered into column chunks whose accumulators fit
 * the 160 KiB of LDS of a compute unit (MAGNUS, ICS '25).
 *
 * Problem statement (Section 2.1, Eq. 1): row i of C is the sum over the
 * stored entries (i, j) of A of A_ij times row j of B.  Matrices are CSR
 * (Section 2.1): rowptr (n + 1 entries), col and val (nnz entries each).
 *
 * Conventions for every call:
 *   - Every pointer inside a magnus_csr_t / magnus_csr_out_t is a DEVICE
 *     pointer on the handle's device.  Host pointers are named as such.
 *   - The caller owns A, B and C's buffers; the library never frees them.
 *     Device memory the library needs for a plan is obtained through the
 *     handle's allocator (magnus_set_allocator; default hipMalloc/hipFree)
 *     and released by magnus_plan_destroy.
 *   - Work is ordered on the stream passed in.  magnus_plan and
 *     magnus_execute synchronise that stream once each (to read back sizes).
 *   - Nothing throws across the ABI; each call returns a magnus_status_t.
 *     On MAGNUS_ERR_HIP, magnus_last_error(h) holds the HIP error text.
 *   - A handle is not thread safe; use one handle per host thread.
 *
 * Semantics of C (readings of the paper recorded with the implementation):
 *   - C's rows list strictly ascending columns;
 *   - a column present in the structure of a row is kept even when its
 *     value sums to zero (the structure is that of the dense accumulator's
 *     bitmap, Algorithm 1); stored zeros of A or B count as structure;
 *   - every sum starts at +0.0, so no entry of C is -0.0;
 *   - B's rows must list strictly ascending columns (validated only when
 *     magnus_options_t.validate is set);
 *   - C.val has A's and B's value type; C.col has B's column type; C's row
 *     pointer type is the caller's choice (int64 is required once nnz(C) or a
 *     row offset reaches 2^31).
 */
#ifndef MAGNUS_H
#define MAGNUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MAGNUS_OK = 0,
  MAGNUS_ERR_INVALID_ARG = 1,    /* null pointer, negative size, bad enum */
  MAGNUS_ERR_SHAPE = 2,          /* A.ncols != B.nrows, or C's shape wrong */
  MAGNUS_ERR_DTYPE = 3,          /* mixed value / index types */
  MAGNUS_ERR_INVALID_CSR = 4,    /* only with options.validate */
  MAGNUS_ERR_INDEX_OVERFLOW = 5, /* nnz(C) does not fit C's row pointer type */
  MAGNUS_ERR_CAPACITY = 6,       /* C.capacity < nnz(C); *nnz_out = nnz(C) */
  MAGNUS_ERR_WORKSPACE = 7,      /* a fixed scratch array too small for the request */
  MAGNUS_ERR_OOM = 8,            /* the allocator returned null */
  MAGNUS_ERR_REJECTED = 9,       /* server: request can never fit */
  MAGNUS_ERR_HIP = 10,           /* a HIP call failed; see magnus_last_error */
  MAGNUS_ERR_NOT_READY = 11,     /* server: result not complete yet */
  MAGNUS_ERR_INTERNAL = 12       /* a device-side consistency check failed */
} magnus_status_t;

typedef enum { MAGNUS_I32 = 0, MAGNUS_I64 = 1 } magnus_itype_t;
typedef enum { MAGNUS_F32 = 0, MAGNUS_F64 = 1 } magnus_vtype_t;

/* Row categories (Section 3.1): SORT rows are accumulated by sorting their
 * intermediate product (expand-sort-compress, Algorithm 2), DENSE rows by a
 * dense accumulator over the row's column range (Algorithm 1), CHUNKED rows
 * by reordering into column chunks first (Algorithm 3) then accumulating each
 * chunk.  EMPTY rows form no product. */
typedef enum {
  MAGNUS_CAT_AUTO = -1,
  MAGNUS_CAT_SORT = 0,
  MAGNUS_CAT_DENSE = 1,
  MAGNUS_CAT_CHUNKED = 2,
  MAGNUS_CAT_EMPTY = 3
} magnus_category_t;

/* Input CSR descriptor (device pointers, read only). */
typedef struct {
  int64_t nrows, ncols, nnz;
  int32_t rowptr_type; /* magnus_itype_t */
  int32_t col_type;    /* magnus_itype_t */
  int32_t val_type;    /* magnus_vtype_t */
  int32_t _pad;
  const void* rowptr;
  const void* col;
  const void* val;
} magnus_csr_t;

/* Output CSR descriptor (device pointers, caller-allocated).  rowptr holds
 * nrows + 1 entries of rowptr_type; col/val hold capacity entries. */
typedef struct {
  int64_t nrows, ncols, capacity;
  int32_t rowptr_type;
  int32_t col_type;
  int32_t val_type;
  int32_t _pad;
  void* rowptr;
  void* col;
  void* val;
} magnus_csr_out_t;

/* Tuning and behaviour.  magnus_options_default() fills the defaults; a zero
 * or negative field means "chosen by the chunk-count model". */
typedef struct {
  int32_t force_category; /* MAGNUS_CAT_AUTO or a category for all non-empty rows */
  int32_t sort_max;       /* rows with ip < sort_max are SORT rows (<= 1024) */
  int32_t chunk_shift;    /* log2 of the chunk length of CHUNKED rows (<= 16) */
  int32_t bin_dense_min;  /* a chunk with >= this many products uses the dense accumulator */
  int32_t tile_products;  /* products per binning tile (power of two, 512..8192) */
  int32_t dense_block;    /* threads per dense-accumulator workgroup (256, 512, 1024) */
  int64_t batch_products; /* products per row batch of CHUNKED rows (0: from workspace cap) */
  int64_t max_workspace_bytes; /* cap on the plan's device memory (0: 40% of free memory) */
  int32_t validate;       /* 1: check CSR invariants of A and B (one extra pass) */
  int32_t lds_bytes;      /* LDS budget per workgroup (0: device maximum) */
  int32_t sort_group_max; /* products per packed sort group of small chunks (<= 1024; 0: 512);
                           * a chunk below bin_dense_min but above this is sorted alone */
  int32_t stream_hints;   /* non-temporal accesses: 1 workspace stores, 2 workspace loads, 4 C stores */
  int32_t coarse_chunks;  /* chunks per coarse chunk (power of two, Section 3.3): CHUNKED rows
                           * wider than one coarse chunk are reordered into coarse chunks first.
                           * 0: the widest coarse chunk whose symbolic bitmap fits the LDS
                           * budget; < 0: no coarse level */
  int32_t deterministic;  /* 1: every value is the row-wise sum of Eq. 1 taken in stored order
                           * (for each entry of A's row in order, each entry of the B row in
                           * order, from +0.0, products rounded to the value type), the same
                           * bits on every run.  All non-empty rows go through the CHUNKED
                           * path without the coarse level (so a row may span at most 65535
                           * chunks), with chunks a quarter of the usual length unless
                           * chunk_shift is set; force_category and coarse_chunks are ignored.  Single
                           * products only: batch plans and the server reject it. */
  int32_t chunk_runs;     /* how CHUNKED rows are reordered into chunks (Algorithm 3): by
                           * single products (-1), or by runs, i.e. the part of one B row
                           * in one chunk, which B's ascending columns keep contiguous, so
                           * each chunk's accumulator reads its products from B through
                           * its list of runs (1); 0: by runs when the rows' products
                           * number at least 8 per run and the run lists fit the
                           * workspace cap.  Deterministic mode always reorders products. */
  int32_t _reserved;
} magnus_options_t;

/* Sizes the plan reports (host struct). */
typedef struct {
  int64_t ip_total;        /* intermediate products, sum over (i,j) in A of nnz(B_j) */
  int64_t flops;           /* 2 * ip_total */
  int64_t nnz_c;           /* exact nnz of C (precise symbolic phase) */
  int64_t max_row_ip;
  int64_t rows_by_category[4]; /* SORT, DENSE, CHUNKED, EMPTY */
  int64_t ip_by_category[4];
  int64_t nnz_by_category[4];  /* nnz of C in the rows of each category */
  int64_t n_batches;       /* row batches of CHUNKED rows */
  int64_t n_bins;          /* chunks (bins) over all CHUNKED rows */
  int64_t n_dense_chunks;  /* chunks accumulated by the dense LDS accumulator */
  int64_t n_sort_groups;   /* packed sort work items of small chunks */
  int64_t plan_bytes;      /* device memory held by the plan */
  int32_t chunk_shift;     /* chosen chunk length = 2^chunk_shift */
  int32_t sort_max;
  int32_t bin_dense_min;
  int32_t tile_products;
  double symbolic_ms;      /* device time of the symbolic phase (events) */
  int64_t coarse_rows;     /* CHUNKED rows taken through the coarse level */
  int64_t coarse_chunks;   /* their coarse chunks (2^coarse_shift columns each) */
  int64_t coarse_fine_chunks; /* chunks of 2^chunk_shift columns inside the coarse chunks */
  int32_t coarse_shift;
  int32_t run_binned;      /* 1: CHUNKED rows were reordered by runs (options.chunk_runs) */
  int64_t n_runs;          /* runs of those rows (0 otherwise) */
} magnus_plan_info_t;

typedef struct magnus_handle_s* magnus_handle_t;
typedef struct magnus_plan_s* magnus_plan_t;

/* Allocator: alloc(bytes, stream, ctx) returns device memory or NULL;
 * free(ptr, bytes, stream, ctx) releases it. */
typedef void* (*magnus_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*magnus_free_fn)(void* ptr, size_t bytes, void* stream, void* ctx);

const char* magnus_status_string(magnus_status_t s);
const char* magnus_last_error(magnus_handle_t h);
void magnus_options_default(magnus_options_t* opts);

/* Lifecycle.  device: HIP device ordinal; opts may be NULL (defaults). */
magnus_status_t magnus_create(magnus_handle_t* h, int device, const magnus_options_t* opts);
magnus_status_t magnus_destroy(magnus_handle_t h);
magnus_status_t magnus_set_options(magnus_handle_t h, const magnus_options_t* opts);
magnus_status_t magnus_set_allocator(magnus_handle_t h, magnus_alloc_fn alloc, magnus_free_fn free_,
                                     void* ctx);

/* Plan: the setup phase (chunk-count model, intermediate-product count per
 * row, categorisation; Section 3.1) and the precise symbolic phase (exact
 * nnz of every row of C followed by a prefix sum; Section 2.1).  Synchronises
 * `stream` (a few times: sizes are read back between passes).  On success
 * *plan owns device memory until magnus_plan_destroy; A and B must stay
 * unchanged until then.  info may be NULL.
 * With options.validate, A and B are checked first and the result read back
 * before any pass indexes B by A's columns: MAGNUS_ERR_INVALID_CSR for
 * rowptr[0] != 0, decreasing row pointers, rowptr[n] != nnz, a column
 * outside [0, ncols), or a B row whose columns are not strictly ascending.
 * When an allocation fails and some row batch of CHUNKED rows (Section 3.3's
 * batching) was wider than the longest row, the plan is made again with
 * batches half as wide, up to four times, before MAGNUS_ERR_OOM. */
magnus_status_t magnus_plan(magnus_handle_t h, const magnus_csr_t* A, const magnus_csr_t* B,
                            void* stream, magnus_plan_t* plan, magnus_plan_info_t* info);

/* Numeric phase: writes C.rowptr, C.col, C.val (C.capacity >= info.nnz_c,
 * C.nrows == A.nrows, C.ncols == B.ncols).  *nnz_out (host) receives nnz(C).
 * Checked before anything is launched, in this order:
 * MAGNUS_ERR_INDEX_OVERFLOW when C.rowptr_type is MAGNUS_I32 and nnz(C)
 * >= 2^31, then MAGNUS_ERR_CAPACITY when C.capacity < nnz(C).
 * Does not synchronise the stream. */
magnus_status_t magnus_execute(magnus_handle_t h, magnus_plan_t plan, const magnus_csr_t* A,
                               const magnus_csr_t* B, const magnus_csr_out_t* C, int64_t* nnz_out,
                               void* stream);

magnus_status_t magnus_plan_destroy(magnus_plan_t plan);
magnus_status_t magnus_plan_get_info(magnus_plan_t plan, magnus_plan_info_t* info);

/* The whole product in one call (Section 2.1's problem statement: CSR A and
 * B in, CSR C out): magnus_plan, then C's three arrays from the handle's
 * allocator (exactly nnz(C) entries, known from the precise symbolic phase),
 * then magnus_execute, then magnus_plan_destroy.
 *   c_rowptr_type: MAGNUS_I32 or MAGNUS_I64, the type of C's row pointers.
 *   C (host struct, out): on success every field is set: device pointers to
 *     rowptr (nrows + 1 entries), col and val (capacity = nnz(C) entries),
 *     C.col_type = B's, C.val_type = A's.  On failure it is zeroed and
 *     nothing stays allocated.  The caller owns C's memory and returns it
 *     with magnus_csr_free.
 * Synchronises `stream` as magnus_plan does; the numeric phase is still in
 * flight on `stream` when the call returns.  Errors: those of magnus_plan
 * and magnus_execute; MAGNUS_ERR_INDEX_OVERFLOW when nnz(C) needs 64-bit
 * row pointers but c_rowptr_type is MAGNUS_I32 (no numeric launch);
 * MAGNUS_ERR_OOM when the allocator fails (a plan whose allocations fail is
 * retried with row batches half as wide, up to four times). */
magnus_status_t magnus_spgemm(magnus_handle_t h, const magnus_csr_t* A, const magnus_csr_t* B,
                              int32_t c_rowptr_type, magnus_csr_out_t* C, void* stream);
/* Returns the three arrays of a C made by magnus_spgemm to the handle's
 * allocator (in stream order on `stream`) and clears its pointers. */
magnus_status_t magnus_csr_free(magnus_handle_t h, magnus_csr_out_t* C, void* stream);

/* Intermediate-product count per row (the setup phase's per-row count,
 * Section 3.1 / n_interProd of Section 4.3).  ip_out: device int64[A.nrows];
 * *ip_total (host) receives the sum.  Synchronises the stream. */
magnus_status_t magnus_row_ip(magnus_handle_t h, const magnus_csr_t* A, const magnus_csr_t* B,
                              int64_t* ip_out, int64_t* ip_total, void* stream);

/* Chunk-count model (Section 3.5, Eqs. 2-7) evaluated as printed, for any
 * cache size: m_c columns, s_cache the cache the fine-level structures must
 * fit, s_line the cache line, s_dense_accum bytes per accumulator column.
 * Host only.  Outputs: fine chunk count, coarse chunk count, m_CmaxL2. */
magnus_status_t magnus_paper_chunk_model(int64_t m_c, int64_t s_cache, int64_t s_line,
                                         double s_dense_accum, int64_t* n_chunks_fine,
                                         int64_t* n_chunks_coarse, int64_t* m_cmax);

/* The gfx950 chunk length: the largest power-of-two column range whose dense
 * accumulator (values plus one bitmap bit per column) fits lds_bytes, capped
 * at 2^16 so chunk-local columns fit 16 bits.  Host only. */
magnus_status_t magnus_gpu_chunk_shift(int32_t val_type, int64_t lds_bytes, int32_t* shift);

/* Per-kernel timing.  While enabled, the library brackets each launch of its
 * main kernels with HIP events on the launch stream and records the
 * algorithmic bytes the launch must move (its inputs read once and outputs
 * written once, counted from the sizes it processes).  magnus_profile_read
 * waits for the recorded events, returns up to max entries aggregated by
 * kernel name (*n receives the count) and clears the records. */
typedef struct {
  char name[40];
  int64_t launches;
  double ms;     /* summed event time */
  double bytes;  /* summed algorithmic bytes */
} magnus_kernel_stat_t;
magnus_status_t magnus_profile_enable(magnus_handle_t h, int on);
magnus_status_t magnus_profile_read(magnus_handle_t h, magnus_kernel_stat_t* out, int max, int* n);

/* Plain device-to-device copy of `bytes` bytes (16-byte vectors): the
 * streaming reference of Section 4.3 for the achievable bandwidth, and the
 * known-size kernel that memory counters are scaled against.  Does not
 * synchronise. */
magnus_status_t magnus_stream_copy(magnus_handle_t h, void* dst, const void* src, size_t bytes,
                                   void* stream);

/* Building block: exclusive prefix sum of n int64 values (device in/out, may
 * alias).  *total (host, may be NULL) receives the sum; synchronises only
 * when total is requested. */
magnus_status_t magnus_exclusive_scan_i64(magnus_handle_t h, const int64_t* in, int64_t* out,
                                          int64_t n, int64_t* total, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * exclusive prefix sum of magnus_exclusive_scan_i64 without any allocation.
 * Its block partial sums live in a fixed array of the library in device
 * memory (8.5 MiB on every device the library runs on, held until the process
 * ends; its address is looked up once per device by magnus_create).
 *   in, out: device int64[n] (may alias); n <= 2^31, else
 *     MAGNUS_ERR_WORKSPACE with nothing launched.
 *   total: DEVICE pointer receiving the sum (may be NULL).
 * Never synchronises and calls no allocator.  Every call on one device uses
 * the same array and leaves in it what the last call wrote: calls whose
 * execution overlaps on one device (other streams, threads or handles) race,
 * so the caller orders them. */
magnus_status_t magnus_exclusive_scan_i64_noalloc(magnus_handle_t h, const int64_t* in,
                                                  int64_t* out, int64_t n, int64_t* total,
                                                  void* stream);

/* Building blocks on one stream of intermediate products (the reordering
 * and accumulation microbenchmarks of Section 4.1, Figs. 4-6): the n
 * products (cols[i], vals[i]) of one row are cut into chunks of
 * 2^chunk_shift columns by a histogram, a prefix sum and a reorder
 * (Algorithm 3); each chunk is then accumulated, by the dense accumulator
 * (Algorithm 1) when it holds at least dense_min products and otherwise by
 * sorting (Algorithm 2, consecutive small chunks packed into one sort),
 * first counting its distinct columns (the precise symbolic phase) and then
 * summing.  The same kernels run for CHUNKED rows.
 *   cols: device uint32[n], each < m; vals: device, n values of val_type
 *     (read only).
 *   m: columns (m < 2^31; m >> chunk_shift chunks, at most 8191).
 *   chunk_shift: log2 of the chunk length, 1..16, and its dense accumulator
 *     must fit the LDS (magnus_gpu_chunk_shift gives the largest).
 *   dense_min: 1..1025 (1025: every chunk of <= 1024 products is sorted; a
 *     bigger one is always dense); 0: the library default.
 *   out_cols (device int32[n]), out_vals (device, n values): the distinct
 *     columns in ascending order with their sums; *nnz (host) receives how
 *     many.  Workspace comes from the handle's allocator.
 *   times (host, may be NULL): event milliseconds of each block.
 * Synchronises the stream.  Errors: MAGNUS_ERR_INVALID_ARG for sizes out of
 * range, MAGNUS_ERR_OOM. */
typedef struct {
  double histogram_ms, scan_ms, reorder_ms, group_ms, count_ms, accumulate_ms;
  int64_t chunks, dense_chunks, sort_groups;
} magnus_stream_times_t;
magnus_status_t magnus_stream_chunks(magnus_handle_t h, const uint32_t* cols, const void* vals,
                                     int32_t val_type, int64_t n, int64_t m, int32_t chunk_shift,
                                     int32_t dense_min, int32_t* out_cols, void* out_vals,
                                     int64_t* nnz, void* stream, magnus_stream_times_t* times);

/* ------------------------------------------------------------------------
 * Batches of independent products C_b = A_b * B_b (b = 0 .. count-1).
 *
 * The rows of all products are numbered one after another and every phase
 * of Sections 3.1 and 2.1 (setup, categorisation, precise symbolic count,
 * prefix sum, numeric accumulation, row pointers of C) runs as one set of
 * launches over the whole batch, with a per-row product index.  Products
 * with CHUNKED rows (Algorithm 3) are planned and executed on their own
 * inside the batch calls.  All products of a batch share the value type and
 * the index types.
 * ---------------------------------------------------------------------- */
typedef struct magnus_batch_plan_s* magnus_batch_plan_t;

/* Plans the batch.  A and B: host arrays of `count` descriptors (device
 * pointers inside, as everywhere).  sort_max: host array of `count`
 * per-product SORT thresholds (rows with ip < sort_max[b] are SORT rows;
 * <= 1025), or NULL for the handle's option.  nnz_out: host int64[count]
 * receiving nnz(C_b).  info (may be NULL) receives totals over the batch.
 * Synchronises `stream` twice (sizes, then nnz per product) plus once per
 * product planned on its own.  A_b and B_b must stay unchanged until the
 * plan is destroyed. */
magnus_status_t magnus_batch_plan(magnus_handle_t h, int32_t count, const magnus_csr_t* A,
                                  const magnus_csr_t* B, const int32_t* sort_max, void* stream,
                                  magnus_batch_plan_t* plan, int64_t* nnz_out,
                                  magnus_plan_info_t* info);

/* Execution modes of magnus_batch_execute. */
#define MAGNUS_BATCH_GRAPH 0 /* numeric launches captured once into a HIP graph, then replayed */
#define MAGNUS_BATCH_EAGER 1 /* the same launches issued one by one */
/* OR-ed with either mode: each numeric stage (one SORT size class, or the
 * DENSE rows) runs as one persistent kernel whose waves (SORT) or workgroups
 * (DENSE) take runs of row tiles from a device counter, instead of one grid
 * with a wave or workgroup per tile.  Same results; on gfx950 the plain
 * grids are faster, so this is off unless asked for. */
#define MAGNUS_BATCH_PERSISTENT 2

/* Numeric phase of every product: writes C[b].rowptr/col/val (host array of
 * `count` output descriptors; C[b].capacity >= nnz_out[b] of the plan).  The
 * descriptors of A, B and C may point to other buffers of the same shapes on
 * every call: a small table of pointers is copied to the device first and the
 * captured graph reads it.  Does not synchronise the stream (it waits, on the
 * host, for the previous call's table copy to finish).  Returns
 * MAGNUS_ERR_CAPACITY (nothing launched) when any capacity is short. */
magnus_status_t magnus_batch_execute(magnus_handle_t h, magnus_batch_plan_t plan, int32_t count,
                                     const magnus_csr_t* A, const magnus_csr_t* B,
                                     const magnus_csr_out_t* C, int32_t mode, void* stream);

magnus_status_t magnus_batch_plan_destroy(magnus_batch_plan_t plan);

/* Upper bound of nnz(C_b) for every product of a batch, from the setup
 * phase's per-row count alone (Section 3.1): row i of C has at most
 * min(ip_i, columns of C) entries.  ip_out and nnz_bound_out: host
 * int64[count], receiving the intermediate products and the bound of each
 * product.  One pass over A's entries and B's row pointers; synchronises the
 * stream once.  Device scratch comes from the handle's allocator and is
 * released before returning. */
magnus_status_t magnus_batch_bound(magnus_handle_t h, int32_t count, const magnus_csr_t* A,
                                   const magnus_csr_t* B, void* stream, int64_t* ip_out,
                                   int64_t* nnz_bound_out);

/* ------------------------------------------------------------------------
 * Serving: products of registered, device-resident operands submitted as
 * requests.  A scheduler thread owned by the server bounds each request's
 * memory from the setup phase's per-row count (magnus_batch_bound: C bytes
 * <= sum_i min(ip_i, columns) * (col + value bytes) + (n + 1) * 8, plus an
 * estimate of its planning memory), admits requests in arrival order while
 * that reservation fits the unreserved budget and a slot is free (a request
 * that does not fit may be passed by at most max_bypass later ones), runs
 * each admitted group as one batch (magnus_batch_plan / magnus_batch_execute)
 * on its own stream, so that a group is planned while earlier groups
 * execute, and stamps completion from a host function enqueued behind the
 * group.  A group's planning may allocate only its requests' planning
 * estimates (allocations past that fail, and the plan retries with narrower
 * row batches); a group that still does not fit goes back to the head of the
 * queue with doubled estimates.  So the plans and results of admitted
 * requests never hold more than the budget (the stats report the peak).  A
 * request whose reservation exceeds exact_above_pct of the budget is
 * planned exactly first (the precise symbolic phase; the plan is kept for
 * its run), capped at the unreserved budget, and then reserves its exact C;
 * it is rejected (MAGNUS_ERR_REJECTED) only if it does not fit that way
 * with nothing else running.  All
 * operands of a server share value and index types.  The server's calls are
 * thread safe; its results stay valid until released.
 * ---------------------------------------------------------------------- */
typedef struct magnus_server_s* magnus_server_t;

typedef struct {
  int64_t memory_budget_bytes; /* device memory for admitted requests' C and plans (0: half the free memory) */
  int64_t workspace_cap_bytes; /* CHUNKED-row workspace of one request (0: budget / 16) */
  int32_t max_inflight;        /* admitted, unfinished requests at most (0: 64) */
  int32_t max_batch;           /* requests per group (0: 32) */
  int32_t streams;             /* groups on the device at once (0: 2, at most 8) */
  int32_t max_bypass;          /* see above (0: 8) */
  int32_t plan_estimate_pct;   /* scale of the planning-memory estimate, percent (0: 100): lower
                                * admits more requests per group, and more groups are deferred */
  int32_t exact_above_pct;     /* requests whose reservation exceeds this percentage of the
                                * budget are sized exactly before admission (0: 25) */
} magnus_server_config_t;

typedef enum {
  MAGNUS_REQ_QUEUED = 0,
  MAGNUS_REQ_RUNNING = 1,
  MAGNUS_REQ_DONE = 2,
  MAGNUS_REQ_REJECTED = 3,
  MAGNUS_REQ_FAILED = 4
} magnus_req_state_t;

typedef struct {
  int32_t state;        /* magnus_req_state_t */
  int32_t batch_size;   /* requests in the group it ran in */
  int64_t nnz;          /* nnz(C), once running */
  int64_t bound_bytes;  /* admission estimate */
  int64_t exact_bytes;  /* bytes of C allocated */
  double queue_ms;      /* submit -> admitted (-1 before) */
  double latency_ms;    /* submit -> C complete on the device (-1 before) */
  int32_t status;       /* magnus_status_t of a failed or rejected request */
  int32_t _pad;
} magnus_request_info_t;

typedef struct {
  int64_t submitted, completed, rejected, failed;
  int64_t batches, batched_requests, exact_probes;
  int64_t reserved_bytes, budget_bytes, queued, running;
  /* the largest reserved_bytes so far (never above budget_bytes), and the
   * groups put back into the queue because their planning did not fit the
   * memory reserved for it */
  int64_t peak_reserved_bytes, deferred;
} magnus_server_stats_t;

void magnus_server_config_default(magnus_server_config_t* cfg);
/* Creates a server with its own handle on `device` (opts may be NULL) and
 * starts its scheduler thread. */
magnus_status_t magnus_server_create(int device, const magnus_options_t* opts,
                                     const magnus_server_config_t* cfg, magnus_server_t* server);
/* Drops queued requests, waits for running ones, frees every result. */
magnus_status_t magnus_server_destroy(magnus_server_t server);
/* Registers a device-resident CSR operand (the caller keeps its buffers
 * unchanged and alive until the server is destroyed); *id is its handle. */
magnus_status_t magnus_server_register(magnus_server_t server, const magnus_csr_t* X, int32_t* id);
/* Queues C = X[a_id] * X[b_id]; returns at once with *request_id. */
magnus_status_t magnus_server_submit(magnus_server_t server, int32_t a_id, int32_t b_id,
                                     int64_t* request_id);
magnus_status_t magnus_server_query(magnus_server_t server, int64_t request_id,
                                    magnus_request_info_t* info);
/* Device view of a finished request's C (int64 row pointers); NOT_READY
 * before, REJECTED or the failure's status otherwise. */
magnus_status_t magnus_server_result(magnus_server_t server, int64_t request_id,
                                     magnus_csr_out_t* C);
/* Frees a finished request's C and forgets the request. */
magnus_status_t magnus_server_release(magnus_server_t server, int64_t request_id);
magnus_status_t magnus_server_get_stats(magnus_server_t server, magnus_server_stats_t* stats);

/* A request that reached a final state (done, rejected or failed). */
typedef struct {
  int64_t request_id;
  int32_t state;       /* MAGNUS_REQ_DONE, MAGNUS_REQ_REJECTED or MAGNUS_REQ_FAILED */
  int32_t status;      /* magnus_status_t: MAGNUS_OK when done */
  int64_t nnz;         /* nnz(C) when done */
  double latency_ms;   /* submit -> C complete on the device; -1 unless done */
} magnus_completion_t;

/* Takes, without waiting, up to max completions in the order the scheduler
 * saw them finish; *n (host) receives how many were written to out (host
 * array).  Each request is reported once.  A completion is queued for every
 * submitted request, whether or not its state was also read by
 * magnus_server_query, until the request is released or the server is
 * destroyed; a request released before it is polled is not reported. */
magnus_status_t magnus_server_poll(magnus_server_t server, magnus_completion_t* out, int32_t max,
                                   int32_t* n);

#ifdef __cplusplus
}
#endif

#endif /* MAGNUS_H */
