/*
 * spmm.h -- C ABI of the MI355X (gfx950) hybrid MFMA / vector SpMM library.
 *
 * The library computes C = A * B for a sparse A (M x K, CSR) and a dense B
 * (K x N), the operation of NeutronSparse Sec. 5.1 ("SpMM"): C[i][j] is the
 * sum over the stored entries p of row i of v_p * B[col_p][j].  Following the
 * paper's workflow (Sec. 4, Fig. 7) the work is split in two stages:
 *
 *   spmm_plan  -- integer preprocessing on the host: the two-stage row/column
 *                 extraction of Sec. 5.2.2 (Eq. 4-5) per row window (Sec. 6.1),
 *                 column compaction, K-tiles kept for the matrix cores when
 *                 their density reaches alpha (Sec. 5.2.1), bitmap packing of
 *                 the kept tiles and index/value lists for the remainder, then
 *                 a balanced list of work items (Sec. 7, row-window lists).
 *                 The plan is uploaded to the device once.
 *   spmm_run   -- one asynchronous execution on a HIP stream: MFMA over the
 *                 kept tiles with B staged in LDS, FP32 gather-FMA for the
 *                 remainder, one write of every C row.
 *
 * Conventions for every entry point:
 *   - Return value is an spmm_status; no C++ exception crosses the ABI.  On
 *     failure spmm_last_error() (thread-local) holds a message.
 *   - "host" pointers point to CPU memory, "device" pointers to memory on the
 *     current HIP device (e.g. torch tensors' data_ptr()).
 *   - Streams are hipStream_t values passed as void* (NULL = the null stream).
 *   - Dense matrices are row-major with a leading dimension in elements.
 */
#ifndef SPMM_H
#define SPMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPMM_ABI_VERSION 1

typedef int32_t spmm_status;
#define SPMM_OK 0
#define SPMM_ERR_INVALID 1     /* malformed CSR, null pointer, bad size or leading dimension */
#define SPMM_ERR_OOM 2         /* host or device allocation failed */
#define SPMM_ERR_DEVICE 3      /* a HIP call failed (message in spmm_last_error) */
#define SPMM_ERR_UNSUPPORTED 4 /* dtype combination, option value or size not supported */
#define SPMM_ERR_BUDGET 5      /* request exceeds a memory budget */
#define SPMM_ERR_BUSY 6        /* object still referenced by unfinished work */

/* precision classes of a plan (spmm_plan_stats_t.tol_class) and the error bound each is
 * held to, max |C - C*| / sum_p |v_p| |B[col_p][j]| against the FP64 result C* */
#define SPMM_TOL_FP32 0       /* 1e-5 */
#define SPMM_TOL_ROUNDED16 1  /* 2e-2 */

/* element types */
#define SPMM_F32 0
#define SPMM_BF16 1
#define SPMM_F16 2

/* execution modes (Sec. 8.3 ablation: vector-only, matrix-only, coordinated) */
#define SPMM_MODE_AUTO 0       /* the tuned profile of this sparsity pattern, else MIXED defaults when
                                  tiles would hold most entries, else PLAIN_F32.  AUTO keeps the
                                  precision class of the inputs: with f32 B (the FP32 path) it
                                  always plans PLAIN_F32 (a tuned profile keeps its other options);
                                  with 16-bit B tiles may round f32 values to bf16 (tol_class) */
#define SPMM_MODE_PLAIN_F32 1  /* every entry on the FP32 vector path */
#define SPMM_MODE_MIXED 2      /* dense-enough tiles on MFMA, the rest on the vector path */
#define SPMM_MODE_MFMA_ONLY 3  /* every row in a window, every column in a tile (alpha = 0) */

/* how rows that pass the row stage are grouped into windows (Sec. 6.1) */
#define SPMM_ORDER_AUTO 0
#define SPMM_ORDER_ORIGINAL_RANGES 1 /* fixed ranges [wH, wH+H); rows failing the row stage leave holes */
#define SPMM_ORDER_COMPACTED 2       /* passing rows in original order, cut into groups of H */
#define SPMM_ORDER_LENGTH_SORTED 3   /* passing rows by length descending (ties: row id), groups of H */
#define SPMM_ORDER_CLUSTERED 4       /* passing rows in the global clustering order (Sec. 6.1 global
                                        stage: Rabbit Order -- incremental modularity aggregation,
                                        then a depth-first walk of the merge dendrogram -- on the
                                        bipartite row-column graph of A), groups of H */

#define SPMM_AUTO_INT (-2147483647 - 1) /* "choose for me" for integer options that accept -1 */

/* Sparse A in CSR.  Arrays are host memory and are only read during
 * spmm_plan / spmm_plan_build; the caller may free them afterwards.
 * rowptr: m+1 entries, rowptr[0] = 0, non-decreasing, rowptr[m] = nnz.
 * colidx: nnz entries in [0, k); order within a row is free; duplicates add.
 * vals:   nnz entries of type val_type; explicit zeros are ordinary entries. */
typedef struct {
    int64_t m, k, nnz;
    const int64_t *rowptr;
    const int32_t *colidx;
    const void *vals;
    int32_t val_type;
    int32_t reserved;
} spmm_csr;

/* Planning options.  spmm_opts_default() fills every field with "auto". */
typedef struct {
    int32_t mode;      /* SPMM_MODE_* */
    int32_t window_h;  /* H: 16, 32 or 64 rows per window; <= 0: auto */
    int32_t t_row;     /* row stage: Len(row) <= t_row stays on the vector path (Eq. 5); SPMM_AUTO_INT: auto */
    int32_t kt;        /* compacted columns per K-tile: 32; <= 0: auto */
    int32_t n_panel;   /* columns of B/C per pass over A; <= 0: auto (whole N when it fits) */
    int32_t row_order; /* SPMM_ORDER_* */
    int32_t seg_len;   /* remainder entries per segment; longer rows are split; <= 0: auto */
    int32_t item_cost; /* target work per vector work item, in entries; <= 0: auto */
    int32_t xcd_remap; /* 1: consecutive items on one XCD, 0: dispatch order, < 0: auto */
    int32_t hot_cols;  /* with cold_policy != 0: the most-gathered columns (at most this many)
                          keep the default cache policy, the others use cold_policy (Sec. 6.2.1,
                          hot B rows cached, the rest bypassing).  < 0: auto (80% of one XCD's
                          4 MiB L2 in B-panel rows, or 0 when cold_policy is 0); 0: none */
    float alpha_c;     /* column stage: a window column is a tile column iff its count > floor(alpha_c*H); < 0: auto */
    float alpha;       /* a K-tile is kept iff nnz / (H*kt) >= alpha (Sec. 5.2.1); < 0: auto */
    int32_t cold_policy; /* cache-policy bits of gathers of non-hot B rows (gfx950 buffer-load aux:
                            2 = nt, 16 = sc1, 18 = nt|sc1, 0 = default); < 0: auto (0: measured
                            fastest on gfx950).  Non-zero needs pipeline 0 (auto picks it) and
                            applies to the segment and vector kernels; window rows' remainders
                            gather with the default policy. */
    int32_t pipeline;  /* vector kernel variant: 0 = row by row; 1 = prefetch the next row during
                          the current row's gathers (bitwise identical to 0); 2 = short rows (at
                          most two unrolled batches) packed one per lane group, each summed in
                          entry order (a different, equally fixed order); 3 = rows packed by size
                          class: a row of remainder length len is summed by S lane groups, S the
                          least power of two with len <= 2*U*S (at most all groups), entry p of
                          the row by group p mod S in entry order, then the groups' sums by an
                          xor butterfly (classes 1 and all-groups sum as in variant 2); < 0: auto */
    int32_t win_sched; /* launch order of windows: 0 = by window id (neighbouring windows, which
                          tend to gather the same B rows, run together on one XCD); 1 = heaviest
                          first (LPT, Sec. 7 row-window lists); < 0: auto */
    int32_t local_reorder; /* Sec. 6.1 local reordering: > 0 = rows per cluster (rounded up to a
                              multiple of H) of the compacted or length-sorted row list, inside
                              which windows are rebuilt: the longest unassigned row of each
                              current window becomes an anchor and takes the H-1 unassigned rows
                              of the cluster most similar to it (Jaccard over distinct column
                              sets, ties: earlier row in the list), leftover rows form windows in
                              list order; 0 = off; < 0: auto (off).  UNSUPPORTED with the
                              original-ranges order. */
    int32_t exec;      /* how a run launches its items (Sec. 5.3, the two engines side by side):
                          1 = one kernel per item kind in dependency order (segments, window partials,
                          vector items, windows); 2 = co-scheduled: the vector path (segments and
                          vector items) and the MFMA path (window partials and owners) as two grids that
                          run concurrently on the run's stream and a second stream of it (fork and join
                          by events, so a graph capture of the run records both); 3 = co-scheduled in one
                          grid.  In 2 and 3 a result needing several items (a split row, a window with
                          partial tiles or split rows) is finished by its last contributor, through
                          integer counters in the workspace; C is bitwise the same in all three.  A cold
                          policy needs 1.  <= 0: auto */
} spmm_opts;

typedef struct spmm_plan_s spmm_plan_t;

/* Summary of a plan (all counts are of the built plan). */
typedef struct {
    int64_t m, k, nnz, n;
    int32_t val_type, b_type, c_type, tile_type;
    spmm_opts opts;             /* options after resolving "auto" */
    int64_t windows;            /* kept windows (each owns at least one tile) */
    int64_t tiles;              /* kept K-tiles */
    int64_t nnz_tiles;          /* entries placed in tiles */
    int64_t nnz_remainder;      /* entries on the vector path */
    int64_t vector_rows;        /* rows not covered by a window */
    int64_t segments;           /* remainder segments computed as separate partial sums */
    int64_t vector_items;       /* vector work items (one wavefront each) */
    int64_t k_ref;              /* distinct columns referenced by A */
    int64_t hot_cols;           /* columns gathered with the cacheable policy */
    double mean_tile_density;   /* nnz_tiles / (tiles * H * kt) */
    double zero_fraction_tiles; /* 1 - mean_tile_density: zeros computed by MFMA (Table 1 measure) */
    int64_t device_bytes;       /* bytes of the uploaded plan */
    int64_t workspace_bytes;    /* per-run scratch for segment partial sums */
    double algorithmic_bytes;   /* 4(M+1) + nnz(4+s_A) + k_ref*N*s_B + M*N*s_C */
    double flops;               /* 2 * nnz * N */
    double plan_ms;             /* host time spent building the plan */
    int32_t uploaded;           /* 1 after spmm_plan_upload */
    int32_t tol_class;          /* precision class of the plan's results: SPMM_TOL_FP32 when every
                                   product is formed from the operands as given (FP32 FMAs, or
                                   16-bit operands widened exactly) and summed in FP32;
                                   SPMM_TOL_ROUNDED16 when MFMA tiles round f32 values or f32 B
                                   to bf16 (round to nearest even) */
    double work_vec;            /* entries gathered by the segment and vector kernels */
    double work_tile;           /* tile slots: tiles * H * kt */
    double work_winrem;         /* remainder entries of window rows (gathered in the window kernels) */
} spmm_plan_stats_t;

/* Host views of the plan's arrays (valid until spmm_plan_destroy).  Used by
 * tests to check the partition against an independent reference. */
typedef struct {
    int64_t m, nnz;
    int32_t window_h, kt;
    int64_t n_windows;          /* windows: int32 [n_windows * H], original row per slot, -1 = empty */
    const int32_t *windows;
    int64_t n_tiles;
    const int32_t *tile_window; /* int32 [n_tiles] */
    const int32_t *tile_cols;   /* int32 [n_tiles * kt], -1 = padding */
    const uint32_t *tile_bitmap;/* uint32 [n_tiles * H], bit j of word s <-> (slot s, column j), LSB first */
    const int64_t *tile_val_ptr;/* int64 [n_tiles + 1] */
    const uint16_t *tile_vals;  /* bf16 / f16 bit patterns, row-major over set bits */
    const int64_t *tile_src;    /* CSR entry index of every packed value */
    const int64_t *rem_ptr;     /* int64 [m + 1] */
    const int64_t *rem_src;     /* CSR entry index of every remainder entry, CSR order per row */
    int64_t n_vector_rows;
    const int32_t *vector_rows; /* rows not in a window, ascending */
    const int32_t *nseg;        /* int32 [m]: segments of the row's remainder (0: not split) */
    int64_t n_vitems;
    const int32_t *vitem_ptr;   /* int32 [n_vitems + 1]: item i covers vexec_rows[ptr[i] .. ptr[i+1]) */
    const int32_t *vitem_seg;   /* int32 [n_vitems]: first segment id used by the item */
    int64_t n_segments;
    const int32_t *seg_row;     /* int32 [n_segments]: row of each segment */
    const int32_t *seg_begin;   /* int32 [n_segments]: first remainder index (into rem arrays) */
    const int32_t *seg_end;     /* int32 [n_segments] */
    const int32_t *win_seg;     /* int32 [n_windows]: first segment id used by the window */
    const int32_t *win_order;   /* int32 [n_windows]: launch order of windows (see win_sched) */
    const int32_t *rem_col_dev; /* int32 [nnz_remainder]: device column array, bit 31 set for hot columns */
    int64_t n_wparts;           /* window partial items: tiles of a window beyond its first 16 */
    const int32_t *win_part;    /* int32 [n_windows + 1]: partial items of window w */
    const int32_t *wpart_win;   /* int32 [n_wparts] */
    const int32_t *wpart_t0;    /* int32 [n_wparts]: first tile */
    const int32_t *wpart_t1;    /* int32 [n_wparts]: end tile */
    const int32_t *vexec_rows;  /* int32 [n_vector_rows]: the vector rows in the order the vector
                                   kernel takes them, item by item (equal to vector_rows except
                                   with pipeline 3, which orders each item's rows by remainder
                                   length, longest first, and split rows last) */
    /* tables of co-scheduled runs (exec 2, 3) */
    int64_t n_dep;              /* windows whose result needs other items' parts */
    const int32_t *seg_win;     /* int32 [n_segments] (or NULL without windows): window of the
                                   segment's row, -1 for a vector row */
    const int32_t *win_dep;     /* int32 [n_windows]: slot of such a window, else -1 */
    const int32_t *win_nsseg;   /* int32 [n_windows]: segments of the window's split rows */
} spmm_plan_dump_t;

/* One matrix of a batched submission (device pointers). */
typedef struct {
    const spmm_plan_t *plan;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
} spmm_work;

typedef uint64_t spmm_ticket;
typedef struct spmm_timer_s spmm_timer_t;

int32_t spmm_abi_version(void);
/* sizeof of the ABI structs, for bindings to check their mirrors:
 * 0 spmm_csr, 1 spmm_opts, 2 spmm_plan_stats_t, 3 spmm_plan_dump_t, 4 spmm_work,
 * 5 spmm_adapt_state;
 * -1 for any other value. */
int64_t spmm_sizeof(int32_t which);
const char *spmm_status_string(spmm_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char *spmm_last_error(void);
void spmm_opts_default(spmm_opts *o);

/* Build a plan on the host only (no device call).  Errors: INVALID for a
 * malformed CSR or n < 1; UNSUPPORTED for nnz, m or k >= 2^31, a dtype
 * combination other than (vals, B) = (f32, f32), (f32, bf16), (bf16, bf16),
 * (f16, f16), c_type other than f32, or an option outside its range.
 * *out is owned by the caller and released with spmm_plan_destroy. */
spmm_status spmm_plan_build(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                            const spmm_opts *opts, spmm_plan_t **out);
/* Copy a host-built plan to the current device (one allocation, one copy). */
spmm_status spmm_plan_upload(spmm_plan_t *p);
/* spmm_plan_build followed by spmm_plan_upload. */
spmm_status spmm_plan(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                      const spmm_opts *opts, spmm_plan_t **out);
/* Release a plan.  BUSY while batched submissions that use it are unfinished. */
spmm_status spmm_plan_destroy(spmm_plan_t *p);
/* A plan built on the device from a CSR whose rowptr, colidx and vals are
 * device pointers (sizes as in spmm_csr), work enqueued on `stream` (which
 * is synchronised); AUTO means PLAIN_F32 here.  Plain plans: the CSR checks,
 * row lengths (Eq. 4), the item cut, the launch order and the segments run
 * as kernels, and A's entries are copied device to device; only O(m)
 * schedule arrays are read back.  Mixed and MFMA-only plans (Sec. 5.2.2,
 * Sec. 6.1): the row stage (Eq. 5), the window slots (original ranges, or
 * the passing rows compacted, or those stably sorted by decreasing length),
 * the column stage, the K-tile density test, the remainder, the bitmaps and
 * the packed values run as kernels; O(m + windows + tiles) arrays come back
 * for the schedule.  The result equals spmm_plan's plan of the same matrix
 * and options array for array.  UNSUPPORTED for clustered windows or local
 * reordering (built on the host), a cold policy, kt other than 32, or (plain)
 * item_cost > 4096; INVALID for a malformed CSR (found on the device, before
 * anything is indexed by it). */
spmm_status spmm_plan_device(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                             const spmm_opts *opts, void *stream, spmm_plan_t **out);
/* Plan images, so that a plan is built once and loaded by later processes
 * (Sec. 5.2.2 preprocessing is amortised over many runs).  serialize writes a
 * versioned, checksummed image of the host plan into buf (cap bytes) and its
 * size into *size; with buf = NULL only *size is set; INVALID if cap is too
 * small.  deserialize reads an image written by the same library version,
 * checks the checksum and every index invariant the kernels rely on (row,
 * column, tile, segment and item ranges), and returns a new plan, uploaded
 * when `upload` is non-zero.  INVALID for a malformed or corrupted image,
 * UNSUPPORTED for another format version.  The image holds the plan's host
 * arrays, including the packed values: the caller's copy of A is not needed. */
spmm_status spmm_plan_serialize(const spmm_plan_t *p, void *buf, int64_t cap, int64_t *size);
spmm_status spmm_plan_deserialize(const void *buf, int64_t size, int32_t upload,
                                  spmm_plan_t **out);
spmm_status spmm_plan_stats(const spmm_plan_t *p, spmm_plan_stats_t *out);
spmm_status spmm_plan_export(const spmm_plan_t *p, spmm_plan_dump_t *out);

/* C = A * B on `stream`, asynchronously.  B: device, K x N of the plan's
 * b_type with row stride ldb >= N; C: device f32, M x N with ldc >= N, fully
 * overwritten (no scaling, no accumulation).  B and C must not overlap.  A
 * plan may be used by concurrent runs on different streams; scratch space is
 * per stream.  Errors: INVALID (null plan/pointer, ld < N), UNSUPPORTED (plan
 * not uploaded), DEVICE. */
spmm_status spmm_run(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc,
                     void *stream);

/* Device memory one execution of a plan occupies besides the plan itself
 * (admission by HBM budget, as a serving loop does): B (k rows of ldb
 * elements), C (m rows of ldc floats) and the scratch the execution uses --
 * for a batched submission (batched != 0) its share of the submission's
 * workspace, for spmm_run the stream's workspace and arrival counters.  Writes
 * the byte count to *bytes and returns SPMM_ERR_BUDGET when it exceeds
 * `budget` (a budget < 0 is unlimited); INVALID for a null plan or output or
 * ld < n. */
spmm_status spmm_run_bytes(const spmm_plan_t *p, int64_t ldb, int64_t ldc, int32_t batched,
                           int64_t budget, int64_t *bytes);

/* spmm_run for callers that cannot allocate (code under graph capture, tight
 * serving loops, harnesses that forbid allocation): the same kernels and the
 * same C bit for bit, but the workspace and the arrival counters come from a
 * fixed device array of the library (32 MiB per device, held by every device
 * the library runs on until the process ends; 1 MiB of it counters, cleared on
 * the first call on a device), and a co-scheduled run keeps both grids on
 * `stream` (no second stream).  No allocation is made by the call.  BUDGET
 * when the run needs more than 31 MiB of workspace or 1 MiB of counters (the
 * message gives the sizes); other errors as spmm_run.  Every call on a device
 * shares that device's array: calls that overlap in time on one device race
 * and must be serialised by the caller (one stream, or events). */
spmm_status spmm_run_noalloc(const spmm_plan_t *p, const void *B, int64_t ldb, void *C, int64_t ldc,
                             void *stream);

/* Kernel timing: spmm_run_timed records a HIP event pair around every kernel
 * it launches (on `stream`) into the timer; spmm_timer_read waits for them
 * and returns the launches' kernel ids and durations in milliseconds. */
#define SPMM_KERNEL_SEGMENT 0 /* partial sums of long remainder rows */
#define SPMM_KERNEL_VECTOR 1  /* FP32 gather-FMA over vector rows */
#define SPMM_KERNEL_WINDOW 2  /* MFMA windows + their rows' remainders */
#define SPMM_KERNEL_WINDOW_PARTIAL 3 /* MFMA partial results of windows' extra tiles */
#define SPMM_KERNEL_VECTOR_PATH 4 /* co-scheduled: segments and vector items in one grid */
#define SPMM_KERNEL_MFMA_PATH 5   /* co-scheduled: window partials and owners in one grid (second stream) */
#define SPMM_KERNEL_ONE_GRID 6    /* co-scheduled: every item kind in one grid */
spmm_status spmm_timer_create(int32_t capacity, spmm_timer_t **out);
spmm_status spmm_timer_reset(spmm_timer_t *t);
spmm_status spmm_timer_read(spmm_timer_t *t, int32_t *kernel_ids, float *ms, int32_t cap,
                            int32_t *count);
spmm_status spmm_timer_destroy(spmm_timer_t *t);
spmm_status spmm_run_timed(const spmm_plan_t *p, const void *B, int64_t ldb, void *C,
                           int64_t ldc, void *stream, spmm_timer_t *t);

/* Batched execution: the work of `count` matrices in one launch sequence on
 * `stream` (plans must share val_type and b_type).  *out receives a ticket
 * for spmm_poll / spmm_wait. */
spmm_status spmm_submit(const spmm_work *items, int32_t count, void *stream, spmm_ticket *out);
spmm_status spmm_poll(spmm_ticket t, int32_t *done);
spmm_status spmm_wait(spmm_ticket t);

/* Dry-run microbenchmarks of the cost model (Sec. 5.2.1, Eq. 1): measured
 * vector-path throughput (entries*N per second) and MFMA-tile throughput
 * (tile slots*N per second) for this N and B type on the current device. */
spmm_status spmm_dryrun(int32_t n, int32_t b_type, void *stream, double *p_vec, double *p_mfma);
/* Autotuner (Sec. 5.2.1 cost model, Sec. 6.2.2 tile shaping, Sec. 8.3 threshold
 * sensitivity).  Derives alpha = P_vec / P_mfma from the dry run (Eq. 3 with
 * r = 1), then times candidate plans of A on the device (B, C: device buffers
 * of the run's shapes; C is overwritten) in a staged search over mode, window
 * height, row order, column/tile thresholds, segment length and N-panel width,
 * within about budget_ms of wall time, each candidate timed the way the
 * plan will run (context: SPMM_TUNE_RUN or SPMM_TUNE_SUBMIT; anything else is
 * INVALID).  A winner other than the plain plan
 * is timed again against it over 10 runs each and kept only when at least 3%
 * faster (otherwise the plain plan's options are the result).  The options
 * are written to *out and cached under A's sparsity-profile key, so
 * spmm_plan with mode = SPMM_MODE_AUTO reuses them for matrices of the same
 * profile. */
typedef struct {
    int32_t candidates;     /* plans timed */
    int32_t reserved;
    double default_ms;      /* run time of the plain plan (the verification timing when
                               another candidate won the search) */
    double best_ms;         /* run time with *out (the same timing as default_ms when the
                               plain plan is the result) */
    double alpha_cost;      /* alpha from Eq. 3 (r = 1) */
    double p_vec, p_mfma;   /* dry-run throughputs (entries*N/s, slots*N/s) */
    double search_ms;       /* wall time spent */
} spmm_tune_report;

#define SPMM_TUNE_RUN 0    /* candidates timed as spmm_run calls */
#define SPMM_TUNE_SUBMIT 1 /* candidates timed as spmm_submit batches of copies of A (up to
                              64, about 4M entries in all, writing the same C): the batched
                              kernels' throughput, for plans that will run among other
                              matrices in spmm_submit */
spmm_status spmm_autotune(const spmm_csr *A, int32_t n, int32_t b_type, int32_t c_type,
                          const void *B, int64_t ldb, void *C, int64_t ldc, void *stream,
                          double budget_ms, int32_t context, spmm_opts *out,
                          spmm_tune_report *report);
/* Sparsity-profile key of A for N and the B type: log2 sizes, the log2 row-
 * length histogram of the entries and the window co-occurrence share of a
 * sample of 16-row windows, as text.  INVALID if cap is too small. */
spmm_status spmm_profile_key(const spmm_csr *A, int32_t n, int32_t b_type, char *buf, int32_t cap);
/* The tuned-options cache (process-wide).  put/get by key; save/load a text
 * file of "key<TAB>options" lines. */
spmm_status spmm_tune_cache_put(const char *key, const spmm_opts *o);
spmm_status spmm_tune_cache_get(const char *key, spmm_opts *o, int32_t *found);
spmm_status spmm_tune_cache_save(const char *path);
spmm_status spmm_tune_cache_load(const char *path);
void spmm_tune_cache_clear(void);

/* Epoch-level adaptive re-partition (Sec. 5.3, Eq. 6-7), read for one pool of
 * compute units: the vector path (segments and vector items) and the MFMA path
 * (windows) share the same CUs -- one after the other (exec 1) or as two
 * co-resident grids (exec 2), where a grid that finishes first leaves its CUs
 * to the other -- so the split that minimises an epoch is the cost crossover
 * of Eq. 3 with r = 1 rather than equal path times.  Each
 * epoch measures both paths and derives their throughputs (Eq. 1 inverted;
 * the window kernels' remainder entries are charged at the vector rate), the
 * crossover alpha* = P_vec / P_mfma, and Eq. 6's skew between the two paths'
 * times for a tile of the current threshold density, which is
 * max(alpha, alpha*) / min(alpha, alpha*).  Above 1 + eps the plan is rebuilt
 * with the threshold moved towards alpha* (sparser tiles move to the vector
 * path when alpha* > alpha, denser rows are packed into tiles when
 * alpha* < alpha): to the secant estimate of log(alpha*) = log(alpha) from
 * this epoch and the previous one when it lies strictly inside the bracket of
 * earlier thresholds, on alpha*'s side and at most twice as far (in
 * logarithms) as alpha*, else to alpha* but at most to the geometric midpoint
 * towards a known bracket end (after two such cut steps in one direction that
 * bracket end is dropped and the step goes to alpha*); at most 7 rounds.  A path without work in an
 * epoch keeps the throughput measured last (the dry run's before any).
 *
 * Zero the state before the first epoch; alpha <= 0 starts from the plan's
 * own threshold.  All throughputs are entries (or tile slots) * N per second. */
typedef struct {
    double alpha;       /* threshold of the current plan (next plan's after a re-partition) */
    double alpha_star;  /* crossover measured in the last epoch, at most 1 */
    double lo, hi;      /* bracket of the threshold; 0 = open */
    int32_t rounds;     /* re-partitions so far */
    int32_t converged;  /* 1 once skew <= 1 + eps */
    int32_t replanned;  /* 1 if the last epoch rebuilt the plan */
    int32_t capped;     /* +1 / -1: the last step was cut at the bracket midpoint going up / down */
    double skew;        /* Eq. 6 of the last epoch */
    double p_vec, p_mfma;       /* throughputs used for alpha_star */
    double t_vec_ms, t_mfma_ms; /* the last epoch's path times */
    double prev_alpha, prev_alpha_star; /* the epoch before: threshold and crossover (0 = none) */
} spmm_adapt_state;

/* The host part of one epoch: from the two paths' times (ms) and work
 * (w_vec entries*N gathered by the vector path, w_tile tile slots*N, w_winrem
 * remainder entries*N of window rows gathered inside the window kernels) and
 * the dry-run throughputs used for a path without work when *st holds no
 * measured one, update *st (alpha,
 * bracket, rounds, skew, converged, replanned).  INVALID for a null state,
 * negative times or work, or eps < 0. */
spmm_status spmm_adapt_next(spmm_adapt_state *st, double t_vec_ms, double t_mfma_ms,
                            double w_vec, double w_tile, double w_winrem, double p_vec_dry,
                            double p_mfma_dry, float eps);
/* One epoch on the device: C = A*B with *plan (timed on `stream`, which is
 * synchronised; each path's time is that of its kernels, or of its grid when
 * co-scheduled), then spmm_adapt_next, and when it asks for a re-partition,
 * a new mixed plan of A with the same options except the threshold replaces
 * *plan (the old plan is destroyed; BUSY, with *plan kept, if it still has
 * outstanding tickets).  A must be the matrix *plan was built from.
 * UNSUPPORTED for a plan with exec 3 (one grid: the paths' times cannot be
 * told apart). */
spmm_status spmm_adapt_epoch(const spmm_csr *A, spmm_plan_t **plan, const void *B, int64_t ldb,
                             void *C, int64_t ldc, void *stream, float eps,
                             spmm_adapt_state *st);

/* Device copy bandwidth (read + write bytes per second) over `bytes` bytes. */
spmm_status spmm_copy_bandwidth(int64_t bytes, void *stream, double *bytes_per_s);

/* Gather ceiling of a column sequence (the B-row gathers of Eq. 1 with
 * nothing else done): times `reps` launches (after 3 untimed ones) of a
 * kernel that reads, for each of the n row ids in `rows` (device, int32; an
 * id outside [0, k) is clamped), the first n_cols f32 of that row of B
 * (device, k rows of leading dimension ldb f32, 16-byte aligned) and sums
 * them in registers, writing nothing; on `stream`, which is synchronised.
 * *bytes_per_s = n * n_cols * 4 * reps / time.  n_cols a multiple of 4 in
 * [4, 128], ldb a multiple of 4 and >= n_cols, k <= 2^31 - 1; else INVALID.
 * Allocates and frees 256 bytes of device memory. */
spmm_status spmm_gather_bandwidth(const int32_t *rows, int64_t n, const void *B, int64_t k,
                                  int64_t ldb, int32_t n_cols, int32_t reps, void *stream,
                                  double *bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* SPMM_H */
