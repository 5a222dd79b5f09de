/*
 * spgemm.h -- C ABI of the MI355X (gfx950) column-wise sparse matrix product.
 *
 * Operation (Gustavson column method, paper Section 2.1): for sparse A
 * (m x k) and B (k x n), both in compressed sparse column (CSC) form,
 *
 *     C(:,j) = sum over the stored B(k,j) of B(k,j) * A(:,k),
 *
 * returned as CSC C (m x n). The structure of C is the boolean product of the
 * stored patterns: a row touched by any product is a stored entry, even when
 * its value cancels to zero (the SPA flags of Algorithm 1 ignore values).
 *
 * Storage (Section 2.1): colptr[ncols + 1] with colptr[0] = 0 and
 * colptr[ncols] = nnz, rowidx[nnz], val[nnz]. Indices are int32. Rows inside
 * an input column may be stored in any order; rows inside every output column
 * are ascending.
 *
 * Arithmetic: every product A(i,k)*B(k,j) is rounded on its own (no fused
 * multiply-add) and added to the running value of row i in the storage order
 * of B(:,j), starting from zero, exactly as the sequential SPA of Algorithm 1.
 * The result is therefore bit-identical run to run and independent of how the
 * library splits the work.
 *
 * Pointers: every array argument is a DEVICE pointer (memory of the current
 * HIP device) unless its name ends in _host. The caller owns all A, B, C, G,
 * dA and dB arrays. `stream` is a hipStream_t (NULL = the default stream).
 *
 * Plans: spgemm_symbolic creates (or refreshes) a plan. The plan borrows the
 * A and B pattern arrays (colptr/rowidx) and the C colptr array: they must stay
 * allocated and unchanged while the plan is used. The plan owns its device
 * workspace (from the allocator of spgemm_set_allocator, by default
 * stream-ordered hipMallocAsync) and frees it in spgemm_plan_destroy. A plan
 * may be used on another stream than its last call's: the new call is
 * ordered after the plan's earlier work without a host wait.
 *
 * Errors: every call returns a status code; nothing aborts or throws across
 * the ABI. On error, outputs are unspecified. Input checks that keep every
 * memory access in bounds always run on the device (column pointers monotone
 * and within nnz, row indices inside their range); a failure gives
 * SPGEMM_ERR_CSC. Repeated rows inside one input column are only detected with
 * SPGEMM_VALIDATE (host-side check); without it they are summed in storage
 * order like distinct products.
 *
 * Synchronisation: spgemm_symbolic and the size-query form of spgemm_batched
 * block the host until the output sizes are known (one read-back at the end
 * when the plan has run before with the same product count, two otherwise).
 * The final read-back is written by a kernel into the plan's mapped, coherent
 * host memory; the calling thread spins on it (polling the stream, so an
 * error on the stream ends the wait with SPGEMM_ERR_HIP). A plan must not be
 * used by two host threads at once. Every other call is stream-ordered and
 * returns immediately.
 */
#ifndef SPGEMM_H
#define SPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPGEMM_OK = 0,
    SPGEMM_ERR_NULL = 1,           /* a required pointer is NULL */
    SPGEMM_ERR_SHAPE = 2,          /* A.ncols != B.nrows, or negative sizes */
    SPGEMM_ERR_CSC = 3,            /* malformed CSC input (see above) */
    SPGEMM_ERR_DTYPE = 4,          /* unknown value type */
    SPGEMM_ERR_INDEX_OVERFLOW = 5, /* nnz(C) of one problem, or a column's product count, exceeds INT32_MAX */
    SPGEMM_ERR_NO_MEMORY = 6,      /* device or host allocation failed */
    SPGEMM_ERR_HIP = 7,            /* a HIP runtime call failed */
    SPGEMM_ERR_PLAN = 8,           /* plan missing, of the wrong kind, or not in the needed state */
    SPGEMM_ERR_INVALID = 9,        /* invalid option value or argument combination */
    SPGEMM_ERR_NOT_TUNED = 10,     /* no tuning cache entry for the workload (lookup only) */
    SPGEMM_ERR_CAPACITY = 11,      /* spgemm_multiply: the C arrays hold fewer than nnz(C) entries */
    SPGEMM_ERR_SCRATCH = 12        /* spgemm_multiply_noalloc: the problem needs more workspace
                                      than the static scratch array holds */
} spgemm_status;

typedef enum { SPGEMM_F32 = 0, SPGEMM_F64 = 1 } spgemm_dtype;

/* One CSC matrix (Section 2.1). colptr/rowidx/val are device pointers; val
 * may be NULL where only the pattern is needed (symbolic phase). */
typedef struct {
    int32_t nrows, ncols, nnz;
    const int32_t *colptr; /* [ncols + 1] */
    const int32_t *rowidx; /* [nnz] */
    const void *val;       /* [nnz] float or double, or NULL */
} spgemm_csc;

typedef struct spgemm_plan_s *spgemm_plan;
/* Plans made by spgemm_batched (the same object; destroyed with
 * spgemm_batch_plan_destroy or spgemm_plan_destroy). */
typedef spgemm_plan spgemm_batch_plan;

/*
 * Device memory of plans (workspace, per-product arrays, staging, the
 * backward view). By default a plan takes it with hipMallocAsync on the
 * stream of the call that needs it and returns it with hipFreeAsync, in
 * stream order: growing a plan never waits on the host.
 *
 * spgemm_set_allocator installs another source for plans created after the
 * call (each plan keeps the pair it was created with until it is destroyed):
 *   alloc(bytes, stream, ctx)    returns device memory of the current device
 *                                usable by work queued on `stream` from now
 *                                on, or NULL (the call then fails with
 *                                SPGEMM_ERR_NO_MEMORY).
 *   free(ptr, bytes, stream, ctx) returns memory from alloc; `stream` is the
 *                                one the memory was allocated on, and every
 *                                use of it by the library has been ordered
 *                                before the work queued on `stream` so far
 *                                (stream-ordered caching allocators may hand
 *                                it out again to later work on that stream).
 * A stream that plan memory was allocated on must outlive the plan. Passing
 * NULL for both restores the default; exactly one NULL gives SPGEMM_ERR_NULL.
 * Host only; thread-safe.
 */
typedef void *(*spgemm_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*spgemm_free_fn)(void *ptr, size_t bytes, void *stream, void *ctx);
spgemm_status spgemm_set_allocator(spgemm_alloc_fn alloc, spgemm_free_fn free_fn, void *ctx);

/* flags */
#define SPGEMM_VALIDATE 1u /* host-side check of both inputs, including repeated rows per column */
#define SPGEMM_ONE_STREAM 2u /* run every accumulator kind on the caller's stream instead of
                                 overlapping them on internal side streams (same results;
                                 per-kernel timings without overlap); products of fewer
                                 than 2^20 products do so without the flag */
#define SPGEMM_NO_PLANNED_LAUNCH 4u /* always read the bin sizes back before launching the
                                       accumulators (by default a plan that has run before
                                       launches the whole symbolic phase from its previous
                                       sizes and redoes it only if the device finds others) */
#define SPGEMM_LANE_HASH 8u /* columns of at most 64 products (the wavefront sort-merge
                               sub-bins up to 64) go to a lane-per-column hash accumulator
                               instead: one output column per lane with a lane-private
                               LDS table, the paper's per-element mapping of HASH
                               (Section 3.2); same results */
#define SPGEMM_LANE_BLOCKED 32u /* columns of at most t_lane products go to lane-per-column
                                   blocks (Section 3.1): sorted by decreasing Op_j, cut by the
                                   Blocking Algorithm (b_min, b_max), one block per wavefront,
                                   one column per lane stepping one product at a time as in
                                   Algorithm 3, each lane with a private hash table whose size
                                   adapts to the block (HASH, Section 3.2); same results
                                   (ignored with SPGEMM_LANE_HASH or t_block != 0) */
#define SPGEMM_LANE_SPARS 64u /* with SPGEMM_LANE_BLOCKED: a private dense accumulator over
                                 all rows per lane instead (SPARS, Algorithm 3); needs
                                 A.nrows <= 4096, else SPGEMM_ERR_INVALID */
#define SPGEMM_RADIX_ESC 16u /* columns above 1024 products go to the global ESC of Section 4
                                instead of row windows: groups of consecutive such columns
                                holding 10,000 products or more, each sorted by (column, row)
                                with a stable radix sort of 5 or 6 bits per round; same
                                results (ignored with SPGEMM_LANE_HASH or t_block != 0) */

/*
 * Tuning options. Results never depend on them: they only choose which
 * accumulator handles a column and how the work is cut (the role of the
 * paper's switch threshold t, Section 3.3, and of its hash-size adaptation,
 * Section 3.2). A zero field takes the library default.
 *   t_esc       columns with at most this many products go to the wavefront
 *               sort-merge (ESC, Section 4) accumulator; 4..256, rounded up
 *               to a power of two; default 256.
 *   t_block     the other columns go to the workgroup sort-merge accumulator
 *               (row-windowed above 4096 products) unless they have more than
 *               t_block products: those go to the workgroup hash accumulator
 *               (HASH, Section 3.2, with direct indexing for row windows that
 *               fit); -1 = every non-ESC column, 0 = none (default).
 *   t_dense     hash-accumulator columns with at least this many products
 *               may accumulate a row window by direct indexing (the SPA of
 *               Section 2.2) when its row span fits the LDS table; >= 1;
 *               default 1.
 *   dense_rows  largest row span of a directly indexed window; 0 = the
 *               table's capacity.
 *   hash_cap    planned distinct rows per row window of the workgroup
 *               accumulator (columns with more products are cut into row
 *               windows); 16..1048576, or 0 = half the LDS table.
 *   t_split     numeric phase: columns with more products than this are
 *               split over several workgroups (chunks of stored B entries);
 *               >= 1, -1 = never; default 2048.
 *   t_lane      SPGEMM_LANE_BLOCKED: columns with at most this many products
 *               (rounded up to a power of two, at most t_esc) go to the lane
 *               blocks (the paper's switch threshold t of Section 3.3);
 *               1..64, default 64.
 *   b_min,      SPGEMM_LANE_BLOCKED: smallest and largest block of the
 *   b_max       Blocking Algorithm (Section 3.1); 1 <= b_min <= b_max <= 64;
 *               defaults 16 and 64 (the paper's variable block size).
 */
typedef struct {
    int32_t t_esc;
    int32_t t_dense;
    int32_t dense_rows;
    int32_t hash_cap;
    uint32_t flags;
    int32_t t_split;
    int32_t t_block;
    int32_t t_lane;
    int32_t b_min;
    int32_t b_max;
} spgemm_options;
/* Work statistics of a plan, for reports and tests. */
typedef struct {
    int64_t total_products;     /* sum of Op_j (Section 3.1) */
    int64_t nnz_c;              /* total stored entries of C */
    int32_t ncols;              /* columns of C (summed over problems) */
    int32_t cols_empty;         /* columns with no product */
    int32_t cols_esc;           /* columns in the wavefront sort-merge accumulator */
    int32_t cols_block;         /* columns in the workgroup hash accumulator */
    int32_t esc_groups;         /* wavefront groups of sort-merge columns */
    int32_t nprob;              /* problems in the plan */
    int32_t later_max;          /* most products adding into one output entry, minus 1 */
    int32_t pad;
    int64_t later_products;     /* products that are not the first of their output entry */
    int32_t cols_direct;        /* workgroup columns with a directly indexed row window */
    int32_t cols_hash;          /* workgroup columns with a hash-table row window */
    int32_t cols_split;         /* workgroup columns with a window split after overflowing */
    int32_t cols_sort;          /* columns in the workgroup sort-merge accumulator */
    int32_t lane_cols;          /* SPGEMM_LANE_BLOCKED: columns in lane-per-column blocks */
    int32_t lane_blocks;        /* SPGEMM_LANE_BLOCKED: blocks of the Blocking Algorithm in the
                                   last symbolic or numeric launch */
} spgemm_plan_stats;
/*
 * Symbolic phase of C = A x B (structure only).
 *   A, B        host pointers to descriptors of device arrays; values unused.
 *   dt          value type the later numeric call will use.
 *   opt         tuning options or NULL for defaults.
 *   plan_inout  on entry NULL or an existing plan (its workspace is reused);
 *               on success the plan for this pattern pair.
 *   C_colptr    device array [B.ncols + 1], filled with C's column pointers.
 *   nnzC_host   host pointer, receives nnz(C).
 * Blocks until nnz(C) is known.
 */
spgemm_status spgemm_symbolic(const spgemm_csc *A, const spgemm_csc *B, spgemm_dtype dt,
                              const spgemm_options *opt, void *stream,
                              spgemm_plan *plan_inout, int32_t *C_colptr, int64_t *nnzC_host);

/*
 * Numeric phase: fills C's row indices (ascending in every column) and values
 * for the pattern pair of `plan`, with the value arrays given here (same
 * sparsity patterns as at symbolic time; values may differ call to call).
 *   A_val [A.nnz], B_val [B.nnz]   device, type of the plan's dtype.
 *   C_rowidx [nnz(C)], C_val [nnz(C)]  device, caller-allocated.
 * Stream-ordered; does not allocate.
 */
spgemm_status spgemm_numeric(spgemm_plan plan, const void *A_val, const void *B_val,
                             int32_t *C_rowidx, void *C_val, void *stream);

/*
 * Both phases in one call, for callers that can offer C arrays of some
 * capacity (typically the previous call's nnz(C) on fixed patterns): the
 * symbolic phase of spgemm_symbolic (Sections 2.1 and 3.1: Op count, binning,
 * distinct rows per column, scan) followed by the numeric phase of
 * spgemm_numeric, same results bit for bit. When the plan has run before, the
 * numeric phase is queued on the stream right behind the symbolic one, from
 * the previous call's sizes, and the call waits only for the read-back of
 * nnz(C); if the sizes read back differ, the numeric phase is queued again
 * with the right ones (it overwrites every output entry).
 *   A, B        as spgemm_symbolic, with their value arrays (device, dtype).
 *   C_colptr    device array [B.ncols + 1], filled.
 *   C_rowidx, C_val  device arrays of `capacity` entries (int32, dtype),
 *               caller-allocated; may be NULL when capacity is 0.
 *   nnzC_host   receives nnz(C).
 * Returns SPGEMM_ERR_CAPACITY when nnz(C) > capacity: nothing is written to
 * C_rowidx / C_val, nnzC_host and C_colptr are set and the plan is ready for
 * spgemm_numeric with larger arrays. Blocks until nnz(C) is known; the numeric
 * phase is stream-ordered after the return. Single problems only.
 */
spgemm_status spgemm_multiply(const spgemm_csc *A, const spgemm_csc *B, spgemm_dtype dt,
                              const spgemm_options *opt, void *stream,
                              spgemm_plan *plan_inout, int32_t *C_colptr, int32_t *C_rowidx,
                              void *C_val, int64_t capacity, int64_t *nnzC_host);

/*
 * spgemm_multiply without any allocation, for callers that cannot allocate
 * memory at call time (serving loops and harnesses that forbid hipMalloc or
 * any allocating routine). Same arguments, results and blocking as
 * spgemm_multiply (symbolic phase, then the numeric phase queued on `stream`
 * after the return), but no plan: every call is a fresh single-problem pass
 * on the caller's stream (no side streams, no planned launch), and all
 * workspace is carved from one static device array of 128 MiB that each GPU
 * the library runs on holds until the process ends (found once per device).
 * nnz(C) is read back by a copy into library-owned host memory.
 *   Workspace needed: about 60 B per column of C and 8 B per stored entry of
 *   B, plus 12 B per intermediate product (Op, Section 3.1) of the columns
 *   with more than 1024 of them (20 B with SPGEMM_RADIX_ESC; 16 B per product
 *   of every column, and 16 B per product beyond the first of its entry, with
 *   the hash options t_block or SPGEMM_LANE_HASH; with SPGEMM_LANE_BLOCKED
 *   also 16 B per column and 32 MiB of per-lane value slabs); a problem
 *   beyond the array gives
 *   SPGEMM_ERR_SCRATCH before any kernel writes the workspace.
 *   SPGEMM_VALIDATE gives SPGEMM_ERR_INVALID (its host check allocates).
 *   SPGEMM_ERR_CAPACITY: as spgemm_multiply (colptr and nnzC_host set); call
 *   again with larger arrays.
 * Every call on a GPU shares that GPU's array and keeps nothing from the
 * last call: calls that overlap on one GPU (two host threads, or two
 * streams whose work is not ordered) race and give wrong results.
 */
spgemm_status spgemm_multiply_noalloc(const spgemm_csc *A, const spgemm_csc *B, spgemm_dtype dt,
                                      const spgemm_options *opt, void *stream,
                                      int32_t *C_colptr, int32_t *C_rowidx, void *C_val,
                                      int64_t capacity, int64_t *nnzC_host);

/*
 * Gradients of a loss L with dL/dC = G (given on C's stored entries) with
 * respect to the stored values of A and B, sparsity patterns fixed:
 *   dA(i,k) = sum_j G(i,j) B(k,j)  over stored B(k,j), j ascending   (G B^T on A's pattern)
 *   dB(k,j) = sum_i A(i,k) G(i,j)  over stored A(i,k), A's order     (A^T G on B's pattern)
 * G_val [nnz(C)] is in the entry order spgemm_numeric gave C; C_rowidx is
 * the row array it filled (C's positions come from the plan, so only its
 * presence is checked). A_val, B_val, G_val device arrays of the plan's dtype;
 * dA_val [A.nnz], dB_val [B.nnz] device outputs, either may be NULL to skip
 * that gradient. Every term is added in the stated order without FMA, so the
 * result equals the sequential sums bit for bit. Single-problem plans only.
 * The first call builds and caches a view of the two patterns inside the plan
 * (per stored entry: its first product and C column start; a row view of B)
 * and may allocate; later calls on the plan are stream-ordered, allocate
 * nothing and queue only kernels (they may be captured in a HIP graph together
 * with spgemm_numeric on the same plan).
 */
spgemm_status spgemm_backward(spgemm_plan plan, const void *A_val, const void *B_val,
                              const int32_t *C_rowidx, const void *G_val,
                              void *dA_val, void *dB_val, void *stream);

/*
 * Batched products C_i = A_i x B_i, i < count, of independent problems of any
 * sizes, run together: every phase is one set of launches over all problems.
 * Two-call convention:
 *   C_rowidx_host == NULL: size query. Builds the plan (plan_inout as in
 *     spgemm_symbolic), fills every C_colptr_host[i] (device array of
 *     B_i.ncols + 1) and nnzC_host[i]. Blocks.
 *   C_rowidx_host != NULL: numeric. Uses the plan of the size query, the value
 *     arrays in A_host[i].val / B_host[i].val, and writes C_rowidx_host[i] /
 *     C_val_host[i] (device arrays of nnzC_host[i] entries). Stream-ordered;
 *     does not allocate and may be captured in a HIP graph once the same
 *     pointers have been passed once (the plan caches the pointer table on the
 *     device and uploads it only when a pointer changes).
 * Arrays ending in _host are host arrays of `count` entries (of device
 * pointers where stated).
 */
spgemm_status spgemm_batched(int32_t count, const spgemm_csc *A_host, const spgemm_csc *B_host,
                             spgemm_dtype dt, const spgemm_options *opt, void *stream,
                             spgemm_plan *plan_inout, int32_t *const *C_colptr_host,
                             int64_t *nnzC_host, int32_t *const *C_rowidx_host,
                             void *const *C_val_host);

/* Per-kernel timing, for measurement tools. When enabled, every launch the
 * library makes is bracketed by HIP events on its own stream; reading
 * synchronises those events and sums their durations per kernel name. */
typedef struct {
    char name[32];       /* kernel (or launch group) name */
    int32_t launches;    /* launches recorded since enabling */
    double total_ms;     /* summed event-measured duration */
} spgemm_kernel_time;

/* on != 0 starts recording (and clears earlier records); on == 0 stops. */
spgemm_status spgemm_profile_enable(int32_t on);

/* Restricts recording to the launch group `name` (NULL or "" = every group),
 * so that a timed loop carries the events of one kernel only. Host only. */
spgemm_status spgemm_profile_select(const char *name);
/* Copies up to `max` records into out_host and their number into n_host
 * (host pointers). Waits for the recorded events. */
spgemm_status spgemm_profile_read(spgemm_kernel_time *out_host, int32_t max, int32_t *n_host);

/* Statistics of a plan after its symbolic phase (reads per-column flags back
 * from the device: synchronous). */
spgemm_status spgemm_plan_get_stats(spgemm_plan plan, spgemm_plan_stats *out);

/* Frees the plan and its workspace (returns the device memory in stream order
 * behind the plan's last work, then synchronises with that stream). */
void spgemm_plan_destroy(spgemm_plan plan);

/* Frees a plan made by spgemm_batched (the same as spgemm_plan_destroy). */
void spgemm_batch_plan_destroy(spgemm_batch_plan plan);

/* Static text for a status code. */
const char *spgemm_status_string(spgemm_status s);

/*
 * Autotuning. Chooses tuning options for a workload by timing candidate
 * settings of t_esc, t_block, t_split, hash_cap and dense_rows (the role of
 * the paper's switch threshold t, Section 3.3, and of its hash-size
 * adaptation, Section 3.2): coordinate descent from the defaults, each
 * candidate timed as symbolic + numeric (best of three runs after a
 * warm-up). Options never change results, so neither does tuning.
 *   count, A_host, B_host  the problems as for spgemm_batched (count == 1:
 *               a single product); value arrays are needed for the timing.
 *   cache_path  JSON file keyed by device and workload signature, or NULL.
 *               A hit returns the cached options without timing; after a
 *               search the choice is stored. A file that does not parse is
 *               treated as empty and rewritten.
 *   tune_flags  SPGEMM_TUNE_LOOKUP_ONLY: never time (SPGEMM_ERR_NOT_TUNED
 *               without a cache entry); SPGEMM_TUNE_REFRESH: ignore the entry.
 * Allocates device memory for the trial outputs and frees it; blocks.
 */
#define SPGEMM_TUNE_LOOKUP_ONLY 1u
#define SPGEMM_TUNE_REFRESH 2u
typedef struct {
    int32_t trials;      /* candidate settings timed (0 when served from the cache) */
    int32_t from_cache;  /* 1 when the options came from the cache */
    double default_ms;   /* symbolic + numeric time with the default options */
    double best_ms;      /* the same with the chosen options */
} spgemm_tune_report;

spgemm_status spgemm_autotune(int32_t count, const spgemm_csc *A_host, const spgemm_csc *B_host,
                              spgemm_dtype dt, void *stream, const char *cache_path,
                              uint32_t tune_flags, spgemm_options *opts_out,
                              spgemm_tune_report *report_out);

/* Cache key of a workload: the device tag (any text; the autotuner uses
 * "<architecture>:<compute units>"), the value type and half-octave buckets
 * of the problem count and of the summed sizes and nonzeros. Host only. */
spgemm_status spgemm_tune_key(int32_t count, const spgemm_csc *A_host, const spgemm_csc *B_host,
                              spgemm_dtype dt, const char *device_tag, char *key_out,
                              int32_t key_len);

/* Cache access, host only: load returns SPGEMM_ERR_NOT_TUNED when the file is
 * missing, does not parse, or has no entry for the key; store replaces the
 * key's entry (rewriting a corrupt file). */
spgemm_status spgemm_tune_cache_load(const char *path, const char *key, spgemm_options *opts_out);
spgemm_status spgemm_tune_cache_store(const char *path, const char *key,
                                      const spgemm_options *opts, double ms);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t spgemm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPGEMM_H */
