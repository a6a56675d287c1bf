/*
 * spmm.h -- C ABI of the MI355X semi-external SpMM library (libspmm.so).
 *
 * Computes Y = A X for a sparse n_rows x n_cols matrix A (typically the
 * adjacency matrix of a power-law graph) and a dense n_cols x k matrix X,
 * k = 1..64.  This is the operation SparseMatrixMultiply(spm, inM) -> outM of
 * Algorithm 1 of Zheng et al., "Semi-External Memory Sparse Matrix
 * Multiplication for Billion-Node Graphs": the output starts at zero and
 * every non-zero (r, c, v) of A adds v * X[c, :] to Y[r, :].  SpMV is k = 1.
 *
 * Conventions shared by every entry point
 *   - Return value: SPMM_OK (0) or a negative spmm_status_t.  No exception
 *     crosses the ABI.  spmm_last_error() returns a thread-local message
 *     describing the most recent failure on the calling thread.
 *   - Host pointers are read during the call only and stay owned by the
 *     caller.  Device pointers (X, Y, scales, vectors) are owned by the
 *     caller; the library never frees them.
 *   - Dense matrices are row-major: element (i, j) of X is at
 *     X[i * ldx + j] with ldx >= k; likewise for Y with ldy.
 *   - Device-side entry points are asynchronous on the stream they are given
 *     and return as soon as the work is enqueued, except where noted.
 *   - A handle may be used from one stream at a time.  Calls on the same
 *     handle from different host threads must be serialised by the caller.
 *   - On failure, no output other than Y (then undefined) is modified.
 */
#ifndef SPMM_H
#define SPMM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPMM_OK = 0,
    SPMM_EINVAL = -1,        /* bad argument or malformed CSR                 */
    SPMM_ENOMEM = -2,        /* host or device allocation failed              */
    SPMM_EHIP = -3,          /* a HIP runtime call failed                     */
    SPMM_EUNSUPPORTED = -4,  /* valid request this library does not support   */
    SPMM_ESTATE = -5,        /* handle is in the wrong state for this call    */
    SPMM_ENOTCONV = -6       /* an iterative method stopped before converging */
} spmm_status_t;

/* Element type of X.  Y is always FP32; how the products are summed is
 * described at spmm_run. */
typedef enum {
    SPMM_X_F32 = 0,
    SPMM_X_BF16 = 1,       /* round-to-nearest-even of the FP32 value          */
    SPMM_X_FP8_E4M3 = 2    /* OCP E4M3 of X[i][j] * s_j, per-column scale s_j  */
} spmm_xdtype_t;

/*
 * Kernel variant of a tile.  A tile is the block of A formed by h
 * consecutive rows (a tile row, "slab") and w consecutive columns, with
 * 16-bit row and column indices local to the tile (Section 3.2).  Every
 * variant computes the same product; they differ in how the tile's entries
 * are encoded and mapped onto the 64 lanes of a wavefront:
 *   COO    - every entry as a (row, col) pair, one lane (group) per entry,
 *            pairs in column order inside the tile, so that lanes gathering
 *            the same X row share one memory request.
 *   ROW    - rows with one entry as COO pairs, the other rows in the
 *            paper's SCSR+COO layout (Section 3.2): one lane (group) per row.
 *   HYBRID - rows shorter than 64 entries as COO pairs, longer rows on a
 *            whole wavefront, which splits the row and reduces it with
 *            cross-lane shuffles (the default).
 *   WAVE   - single-entry rows as COO, every other row one wavefront.
 */
typedef enum {
    SPMM_VAR_COO = 0,
    SPMM_VAR_ROW = 1,
    SPMM_VAR_HYBRID = 2,
    SPMM_VAR_WAVE = 3
} spmm_variant_t;
#define SPMM_NUM_VARIANTS 4

/* Number of per-tile features reported by spmm_tile_features. */
#define SPMM_NUM_FEATURES 8

/* Where the encoded tiles live. */
typedef enum {
    SPMM_PLACE_DEVICE = 0,       /* HBM; used by spmm_run                     */
    SPMM_PLACE_PINNED_HOST = 1   /* pinned host DRAM; used by spmm_stream_run */
} spmm_place_t;

/* Build options.  A zero-initialised struct selects every default. */
typedef struct {
    uint32_t tile_rows;      /* h: rows per tile row; 0 -> 32; 1..4096           */
    uint32_t tile_cols;      /* w: columns per tile; 0 -> 65536; power of 2,
                                 <= 65536 (16-bit local column index)           */
    int32_t fixed_variant;   /* variant of every tile; < 0 -> SPMM_VAR_HYBRID    */
    uint32_t item_nnz;       /* target non-zeros per work item (one wavefront);
                                 longer rows are split; 0 -> 16384, <= 131072      */
    uint32_t place;          /* spmm_place_t                                     */
    uint32_t threads;        /* host threads for the build; 0 -> all cores       */
    uint32_t validate;       /* row pointers and column ranges are always
                                 checked; 1 also rejects unsorted or duplicate
                                 columns within a row (duplicates otherwise add) */
    uint32_t max_kc;         /* widest block of X columns one kernel launch
                                 accumulates: 16 or 32; 0 -> 32                   */
    uint32_t keep_order;     /* 0 (default): tiles index columns by descending
                                 in-degree, and spmm_run first gathers X into that
                                 row order (a handle-owned buffer), so the X rows
                                 of hub columns are contiguous and cache-resident;
                                 1: tiles keep the given column and row order     */
    uint32_t stream_kib;     /* streamed mode: payload per host->device transfer
                                 group, KiB; 0 -> 262144 (256 MiB)                 */
    uint32_t ring_depth;     /* streamed mode: device slots in the transfer ring;
                                 0 -> 3; 2..16                                    */
    int32_t x_stage_kib;     /* launches of <= 8 X columns: > 0 stages the
                                 hottest X rows in this many KiB of LDS per
                                 workgroup (a persistent launch, one workgroup
                                 per CU; capped by the device's LDS); <= 0 -> no
                                 staging (the default: measured faster)          */
    uint32_t transpose;      /* 1 -> the handle holds A^T: the given CSR is
                                 transposed on the host first (for PageRank's
                                 in-link matrix and NMF's A^T on a directed
                                 graph); its shape is then n_cols x n_rows       */
    uint32_t keep_row_order; /* 0 (default, unless keep_order = 1): tile rows take
                                 the rows in order of descending out-degree (ties
                                 by row id), so that rows sharing hub columns
                                 share tile rows and gather those X rows once;
                                 Y is still written in the given row order, and
                                 rows without entries are zero-filled.  1 (or
                                 keep_order = 1): tile rows take the given row
                                 order                                           */
    uint32_t format;         /* SPMM_FORMAT_TILES (0, default): the tile store.
                                 SPMM_FORMAT_CSR: the untiled baseline (V-csr) --
                                 rows by descending length, columns in in-degree
                                 order, one lane group, wavefront or several
                                 wavefronts per row by length, FP32 register sums;
                                 binary A, FP32 X, HBM only (spmm_run and the
                                 paths built on it: PageRank, NMF, eigensolver)  */
} spmm_build_opts;

#define SPMM_FORMAT_TILES 0u
#define SPMM_FORMAT_CSR 1u

typedef struct spmm_handle_s* spmm_handle_t;

/*
 * Convert a CSR matrix into the tile store (the CSR -> SCSR conversion of
 * Section 5, Table 3).  Host work only: the device copy is made by the
 * first spmm_run (or the pinned host copy by the first spmm_stream_run).
 *   n_rows, n_cols : matrix shape, 0 <= n <= 2^31 - 1.
 *   row_ptr        : host int64[n_rows + 1], row_ptr[0] = 0, non-decreasing.
 *   col_idx        : host int32[row_ptr[n_rows]], columns of each row sorted
 *                    ascending without duplicates (checked if opts->validate).
 *   values         : host float[nnz] or NULL for a binary (all-ones) A.
 *   opts           : NULL for defaults.
 *   out            : receives the handle, set only on SPMM_OK.
 * The CSR arrays are copied; the caller may free them after the call.
 * Errors: SPMM_EINVAL (bad shape/options/CSR), SPMM_ENOMEM, SPMM_EHIP.
 */
spmm_status_t spmm_build_tiles(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr,
                               const int32_t* col_idx, const float* values,
                               const spmm_build_opts* opts, spmm_handle_t* out);

/*
 * Slab-wise build, for a matrix whose CSR is produced (or held) a block of
 * rows at a time: the same tile store as spmm_build_tiles, without the whole
 * CSR in host memory at once.  The conversion is still one linear pass over
 * the rows (Section 3.2; the conversion cost of Section 5, Table 3).
 *
 * spmm_build_begin: a handle for an n_rows x n_cols matrix, to be filled by
 *   spmm_build_append_rows and completed by spmm_build_end.  Options as for
 *   spmm_build_tiles, except that
 *     - the columns keep the given order (the in-degree order needs every
 *       column's count before the first tile is cut): order the columns
 *       beforehand if hub columns should be contiguous;
 *     - rows are taken by descending out-degree within each appended block
 *       (together with the rows still untiled from the block before), unless
 *       keep_row_order or keep_order is set;
 *     - transpose is not supported (SPMM_EUNSUPPORTED);
 *     - every tile takes fixed_variant (HYBRID if it is -1): the per-tile
 *       selectors (spmm_tile_features, spmm_get_variants, spmm_set_variants,
 *       spmm_selector_collect, spmm_autotune, spmm_select_learned) return
 *       SPMM_EUNSUPPORTED on such a handle, which keeps no per-tile store.
 *   Errors: SPMM_EINVAL (shape, options), SPMM_EUNSUPPORTED, SPMM_ENOMEM.
 *
 * spmm_build_append_rows: rows [row0, row0 + nrows), in order: row0 must be
 *   the first row not yet appended.
 *     row_ptr_local : host int64[nrows + 1], row_ptr_local[0] = 0; row i's
 *                     entries are col_idx[row_ptr_local[i - row0] ..].
 *     col_idx       : host int32, columns sorted ascending without
 *                     duplicates within a row (checked if opts->validate).
 *     values        : host float or NULL; NULL for every block or for none
 *                     (the first call decides).
 *   The arrays are read during the call only; the caller may free them on
 *   return.  Whole tile rows are tiled and encoded at once, and their tiles
 *   released: host memory holds the encoded payload plus one block's tiles,
 *   never a per-tile store of the whole matrix.  Up to tile_rows - 1 rows
 *   are copied and kept for the next call.  On error the handle must be
 *   destroyed.  Errors: SPMM_EINVAL (order, CSR), SPMM_ESTATE (not being
 *   built), SPMM_ENOMEM.
 *
 * spmm_build_end: tiles the rows still kept and encodes the work items; the
 *   handle can then be used like one from spmm_build_tiles.  Every other
 *   entry point rejects a handle between begin and end with SPMM_ESTATE.
 *   Errors: SPMM_ESTATE (rows missing, or not being built), SPMM_ENOMEM.
 */
spmm_status_t spmm_build_begin(int64_t n_rows, int64_t n_cols, const spmm_build_opts* opts, spmm_handle_t* out);
spmm_status_t spmm_build_append_rows(spmm_handle_t h, int64_t row0, int64_t nrows, const int64_t* row_ptr_local,
                                     const int32_t* col_idx, const float* values);
spmm_status_t spmm_build_end(spmm_handle_t h);

/* Release a handle and everything it owns.  NULL is ignored.  Waits for
   work already enqueued on the handle's device buffers to finish. */
void spmm_destroy(spmm_handle_t h);

/* Message for the last failure on this thread ("" if none).  The pointer
   stays valid until the next library call on this thread. */
const char* spmm_last_error(void);

/*
 * Y = A X on the device (A placed in HBM).
 *   X     : device pointer, n_cols x k, element type dt, row stride ldx >= k
 *           (elements).  FP32 rows 16-byte aligned run fastest.
 *   k     : 1..64.
 *   col_scale : device float[k], the FP8 column scales s_j (Y is divided by
 *           s_j at write-out); must be NULL unless dt is SPMM_X_FP8_E4M3.
 *   Y     : device pointer, n_rows x k FP32, row stride ldy >= k; every
 *           element of the n_rows x k block is overwritten.
 *   s     : HIP stream (0 = null stream).
 * The first call on a handle copies the tile payload to HBM and allocates
 * the partial-result buffer of split tile rows (synchronous allocations).
 * Rows without entries of a handle that orders rows by degree are not
 * tiled and are zero-filled: when there are at least 2^26 such values and s
 * is not being captured, on a stream the handle owns, forked from s at the
 * start of the call and joined back into s before it returns (so all of
 * the call's work stays ordered on s).
 *
 * Arithmetic.  X is decoded to FP32 and multiplied by A's value in FP32.
 * The products are summed exactly, in 64-bit fixed point: column j uses the
 * grid 2^-f_j with f_j = 61 - e_j, where 2^e_j is the smallest power of two
 * above (largest row L1 norm of A) * max_i |X[i][j]|, so that no partial
 * sum can overflow.  Each FP32 product -- or the FP32 register sum of a run
 * of one row's products inside one tile, which the ROW, HYBRID and WAVE
 * variants form first -- is rounded once to that grid (to nearest, ties to
 * even); Y[r][j] is the FP32 rounding of the exact sum of those grid
 * values.  So results do not depend on the order of the sums (run to run,
 * streamed or in HBM, any launch width) and integer X is exact.  A product
 * smaller than 2^-(f_j+1) in magnitude, i.e. more than about 2^-62 of the
 * column's bound, rounds to zero.  (This departs from plain FP32
 * accumulation, which rounds every partial sum.)
 * A NaN or an infinity anywhere in column j of X (for FP8, a NaN code)
 * makes Y[r][j] NaN for every row r that has at least one entry; the other
 * columns are unaffected.
 * Errors: SPMM_EINVAL (bad k/ld/pointer/dtype), SPMM_ESTATE (tiles placed in
 * host memory, or a slab-wise build not ended), SPMM_ENOMEM, SPMM_EHIP.
 */
spmm_status_t spmm_run(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                       const float* col_scale, float* Y, int64_t ldy, hipStream_t s);

/*
 * spmm_run for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, arithmetic and result as spmm_run (bit-identical), with
 * two preconditions and no allocation of any kind:
 *   - the handle is built with keep_order = 1 (columns and rows in the given
 *     order), so X is read in place: SPMM_EUNSUPPORTED otherwise;
 *   - its tiles are already on the device, i.e. spmm_run has been called on
 *     the handle once: SPMM_ESTATE otherwise.
 * The launch's scratch (split-row partial sums, their counters, X's column
 * maxima and fixed-point exponents) lives in a static device array of
 * 16 MiB that each GPU the library runs on holds until the process ends; a
 * handle needing more (about n_parts * 32 * 8 bytes, reported by
 * spmm_get_stats) gets SPMM_EINVAL.  All calls on one GPU share that array:
 * calls that overlap on one GPU race (serialise them, e.g. on one stream).
 * Asynchronous on s.  Errors: SPMM_EINVAL, SPMM_ESTATE, SPMM_EUNSUPPORTED,
 * SPMM_EHIP.
 */
spmm_status_t spmm_run_static(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                              const float* col_scale, float* Y, int64_t ldy, hipStream_t s);

/*
 * Quantise X for the reduced-precision SpMM paths (not in the paper; halves
 * or quarters the X bytes every SpMM gathers).
 *   X     : device FP32, n x k, row stride ldx >= k.
 *   dt    : SPMM_X_BF16 -> Xq is uint16 BF16 codes, round to nearest even.
 *           SPMM_X_FP8_E4M3 -> Xq is uint8 OCP E4M3 codes of fp32(X[i][j] * s_j),
 *           nearest with ties to even, saturating at +-448.
 *   Xq    : device, n x k codes, row stride ldq >= k (elements).
 *   col_scale : device float[k]; FP8 only (NULL for BF16).  Unless flags has
 *           SPMM_QUANT_SCALES_GIVEN, it is overwritten with
 *           s_j = 448 / max_i |X[i][j]| (FP32 division; 1 for a zero column);
 *           with the flag it is read as given.  Pass the same array to
 *           spmm_run, which divides Y's column j by s_j.
 *   flags : 0 or SPMM_QUANT_SCALES_GIVEN.
 * Asynchronous on s.  Errors: SPMM_EINVAL, SPMM_EHIP.
 */
#define SPMM_QUANT_SCALES_GIVEN 1u
spmm_status_t spmm_quantize_x(const float* X, int64_t n, int k, int64_t ldx, spmm_xdtype_t dt,
                              void* Xq, int64_t ldq, float* col_scale, uint32_t flags,
                              hipStream_t s);

/*
 * Y = A X with the tile payload in pinned host memory: the semi-external
 * mode of Section 3.1 on one GPU (A in host DRAM instead of on SSDs; X and Y
 * resident in HBM).  Consecutive work items are grouped into transfers of
 * about opts.stream_kib KiB; each group is copied on `copy` into one slot of a
 * ring of opts.ring_depth device buffers while the kernels of the previous
 * groups run on `compute` (events order each copy after the kernels that
 * last read its slot, and each kernel after its copy).
 *   h : built with opts.place = SPMM_PLACE_PINNED_HOST.  Other arguments as
 *       spmm_run.  compute and copy should be different streams for overlap.
 * The result is identical to spmm_run's on the same tiles (same kernels,
 * same work items).  Asynchronous: the copies into a slot wait, on the
 * device, for the kernels that last read it -- also those of an earlier
 * call -- so calls may be queued back to back without host
 * synchronisation.  The first call allocates the ring.
 * Errors: SPMM_EINVAL, SPMM_ESTATE (tiles placed in HBM), SPMM_ENOMEM,
 * SPMM_EHIP.
 */
spmm_status_t spmm_stream_run(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                              const float* col_scale, float* Y, int64_t ldy, hipStream_t compute,
                              hipStream_t copy);

/*
 * Y = A X with the tile payload streamed from pinned host memory (as
 * spmm_stream_run) and Y streamed back to host memory as its tile rows
 * finish: the device analogue of Algorithm 1's asynchronous write of output
 * rows (Section 3.5), so that neither A nor Y has to be resident in HBM.
 * The kernels of each transfer group write its rows of Y into a device slot
 * (one per ring slot); a copy on `out` moves those rows -- one contiguous
 * range per group -- to Y, and the slot is reused once that copy is done.
 *   h   : built with place = SPMM_PLACE_PINNED_HOST and keep_row_order = 1
 *         (or keep_order = 1), so that a group's rows are one range of Y;
 *         SPMM_EUNSUPPORTED otherwise.
 *   X   : device pointer as for spmm_run (resident).
 *   Y   : pinned host memory (hipHostMalloc, or a torch tensor with
 *         pin_memory), n_rows x k FP32, row stride ldy >= k; every element
 *         of the n_rows x k block is written.
 *   compute, copy, out : streams for the kernels, the host-to-device copies
 *         and the device-to-host copies (distinct streams overlap the three).
 * Asynchronous: Y is complete when the work queued on `out` has finished.
 * Consecutive calls need no synchronisation (events order every reuse of a
 * slot).  The Y slots (largest group's rows x k floats per ring slot) belong
 * to the handle; a call with a larger k than before reallocates them after
 * waiting for the earlier copy-outs.  Results are bit-identical to spmm_run
 * and spmm_stream_run on a handle with the same options.
 * Errors: as spmm_stream_run, plus SPMM_EUNSUPPORTED.
 */
spmm_status_t spmm_stream_run_yhost(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                                    const float* col_scale, float* Y, int64_t ldy, hipStream_t compute,
                                    hipStream_t copy, hipStream_t out);


/*
 * Semi-external SpMM with the dense matrices in host memory as well: X and
 * Y stay in (pinned) host DRAM and their columns are processed in blocks of
 * cols_per_block -- the paper's dense matrix partly in memory (Section 3.5's
 * memory and I/O model, Section 3.6).  For each block the library copies
 * that block of X to the device, streams all of A over it (as
 * spmm_stream_run), and copies the block of Y back while the next block
 * starts.  A crosses the host link ceil(k / cols_per_block) times, so fewer
 * columns in memory cost more A traffic: the trade-off the paper measures.
 *   h : built with opts.place = SPMM_PLACE_PINNED_HOST.
 *   X : host FP32, pinned memory for full speed.  Row-major [n_cols][ldx]
 *       (ldx >= k), or with SPMM_HOSTXY_BLOCKED the blocked layout: block b
 *       (columns b*cols_per_block ... up to k) stored contiguously as
 *       [n_cols][width of block b], blocks back to back (ldx ignored).
 *   Y : host FP32 [n_rows][ldy] (ldy >= k), or blocked like X; fully
 *       overwritten.
 *   cols_per_block : 1..k.
 * A block that is contiguous in host memory (blocked layout, or
 * cols_per_block = k = ldx) crosses the link as one copy; strided columns
 * of a row-major X or Y need a 2-D copy, which the copy engines perform far
 * below the link rate for narrow rows.
 * Device memory for two X blocks and two Y blocks (n x cols_per_block FP32)
 * is allocated per call.  Synchronous: returns when Y is in host memory.
 * The result equals spmm_run's on the same tiles up to the FP32 rounding of
 * per-row register partial sums, whose lane order depends on the column
 * width of a launch (bit-identical when cols_per_block equals the launch
 * width spmm_run uses, and for integer-valued X).
 * Errors: SPMM_EINVAL, SPMM_ESTATE (tiles placed in HBM), SPMM_ENOMEM,
 * SPMM_EHIP.
 */
#define SPMM_HOSTXY_BLOCKED 1u
spmm_status_t spmm_stream_run_host(spmm_handle_t h, const float* X, int k, int64_t ldx, float* Y, int64_t ldy,
                                   int cols_per_block, uint32_t flags);

/*
 * PageRank power iteration (Section 4.1):
 *   PR'(u) = (1 - d)/N + d * ( sum_{v in B(u)} PR(v) / L(v)  +  D/N ),
 * B(u) = in-neighbours of u, L(v) = out-degree of v, D = sum of PR over the
 * vertices with L = 0 (dangling mass, spread evenly so that sum PR = 1; the
 * paper's formula without this term is SPMM_PR_NO_REDISTRIBUTE).
 *   h      : handle of the n x n matrix whose row u lists the in-neighbours of
 *            u, i.e. the transpose of the adjacency matrix (for an undirected
 *            graph, the adjacency matrix itself).  L(v) is taken as the number
 *            of entries in column v of this matrix.
 *   pr     : device float[n]; initialised to 1/N unless SPMM_PR_INIT_GIVEN;
 *            holds the result.
 *   resid  : host double[iters] (or NULL): resid[t] = sum_u |PR_{t+1}(u) - PR_t(u)|,
 *            reduced in FP64 (as is D).
 *   flags  : SPMM_PR_INIT_GIVEN | SPMM_PR_NO_REDISTRIBUTE | SPMM_PR_NO_GRAPH
 *            (the default captures all iterations into one HIP graph).
 * Exactly `iters` iterations (no early stop).  Synchronous: returns after the
 * last iteration has finished.  Errors: SPMM_EINVAL, SPMM_ESTATE, SPMM_ENOMEM,
 * SPMM_EHIP.
 */
#define SPMM_PR_INIT_GIVEN 1u
#define SPMM_PR_NO_REDISTRIBUTE 2u
#define SPMM_PR_NO_GRAPH 4u
spmm_status_t spmm_pagerank(spmm_handle_t h, float damping, int iters, uint32_t flags, float* pr,
                            double* resid, hipStream_t s);

/*
 * Non-negative matrix factorisation A ~ W H^T by the multiplicative updates
 * of Section 4.3, H first, then W, every iteration:
 *   H <- H * (A^T W) / (H (W^T W) + eps),   W <- W * (A H) / (W (H^T H) + eps).
 *   hA, hAT : handles of A (n x m) and of A^T (pass hA twice if A is symmetric).
 *   rank    : r, 1..32.   W : device float n x r;  H : device float m x r (the
 *             paper's H transposed), both row-major with stride r, updated in place.
 *   eps     : added to every denominator (rows of isolated vertices go to 0).
 * Gram matrices are accumulated in FP64 (deterministic order), everything
 * else in FP32.  Asynchronous on s: the workspace (max(n, m) x r floats plus
 * the Gram partials) belongs to hA and is kept for later calls; the first
 * call, or one needing a larger workspace, allocates it (and waits for s
 * before releasing a smaller one).  Errors: SPMM_EINVAL, SPMM_ESTATE,
 * SPMM_ENOMEM, SPMM_EHIP.
 */
spmm_status_t spmm_nmf(spmm_handle_t hA, spmm_handle_t hAT, int rank, int iters, float eps, float* W,
                       float* H, hipStream_t s);

/*
 * Rebuild the CSR of A from the encoded work items (host copy of the tile
 * payload), walking them with the same indexing as the kernels.  A check of
 * the encoding: the result equals the CSR given to spmm_build_tiles.
 *   row_ptr : host int64[n_rows + 1] (output);  col_idx : host int32[nnz];
 *   values  : host float[nnz] for a weighted A, else NULL.
 * Errors: SPMM_EINVAL (NULL arguments, values for a binary A), SPMM_ENOMEM.
 */
spmm_status_t spmm_decode_tiles(spmm_handle_t h, int64_t* row_ptr, int32_t* col_idx, float* values);

/*
 * Kernel timing.  Between spmm_timing_begin and spmm_timing_end, every
 * spmm_run on h records a HIP event pair on its stream around its SpMM
 * launches only (not the X reordering or fixed-point exponent kernels),
 * without host synchronisation.  spmm_timing_end waits for the recorded
 * events, returns the summed milliseconds and the number of runs, and stops
 * recording.  Not for use while a stream that runs on h is being captured.
 */
spmm_status_t spmm_timing_begin(spmm_handle_t h);
spmm_status_t spmm_timing_end(spmm_handle_t h, double* total_ms, uint64_t* n_runs);

/*
 * Measurement utility: one streaming read of `bytes` of device memory at
 * `buf` (16-byte aligned, a multiple of 16) with 16-byte loads, asynchronous
 * on s.  `sink` (device float[1]) is written only for a sum no all-ones or
 * all-zeros buffer produces.  Timed by the caller, it gives the HBM read
 * rate a plain kernel attains, the context for the SpMM's roofline.
 * Errors: SPMM_EINVAL (NULL, misaligned), SPMM_EHIP.
 */
spmm_status_t spmm_read_probe(const void* buf, uint64_t bytes, float* sink, hipStream_t s);

/* Shape and storage statistics of a handle. */
typedef struct {
    uint64_t n_rows, n_cols, nnz;
    uint64_t tile_rows, tile_cols;
    uint64_t n_slabs;          /* tile rows                                      */
    uint64_t n_tiles;          /* non-empty tiles                                */
    uint64_t sum_nnr;          /* sum over tiles of non-empty rows               */
    uint64_t sum_nnc;          /* sum over tiles of non-empty columns            */
    uint64_t n_items;          /* work items (one wavefront each)                */
    uint64_t n_parts;          /* items whose tile row is split across items     */
    uint64_t blob_bytes;       /* encoded tile payload                           */
    uint64_t desc_bytes;       /* work-item descriptors and combine lists        */
    uint64_t variant_tiles[SPMM_NUM_VARIANTS];
    uint64_t variant_nnz[SPMM_NUM_VARIANTS];
} spmm_stats_t;

spmm_status_t spmm_get_stats(spmm_handle_t h, spmm_stats_t* out);

/*
 * Byte model of the paper's tile format for t x t tiles (Section 3.2), read
 * straight from a CSR (same argument rules as spmm_build_tiles):
 *   n_tiles = non-empty tiles, sum_nnr / sum_nnc = non-empty rows / columns
 *   summed over tiles.  S_SCSR of the matrix is 2 sum_nnr + (2 + c) nnz.
 */
spmm_status_t spmm_model_tiles(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr,
                               const int32_t* col_idx, int64_t t, uint64_t* n_tiles,
                               uint64_t* sum_nnr, uint64_t* sum_nnc);

/* ------------------------------------------------------------------------
 * Per-tile variant selection.
 *
 * The paper fixes one per-tile layout, SCSR plus COO (Section 3.2).  Here
 * each tile picks one of the SPMM_NUM_VARIANTS encodings, either by timing
 * (an exhaustive autotuner over buckets of similar tiles) or by a learned
 * cost model: an MLP mapping the 8 tile features to a predicted log time
 * per variant, the tile taking the variant of least prediction.  Tiles are
 * numbered in the handle's order (tile rows, then strips), 0..n_tiles-1.
 * ------------------------------------------------------------------------ */

/*
 * Features of every tile, feat[t * 8 + i] (host float[n_tiles * 8]):
 *   0 log2(1 + nnz_t)      1 log2(1 + non-empty rows)
 *   2 log2(1 + non-empty columns)   3 log2(1 + longest row)
 *   4 fraction of non-empty rows with one entry
 *   5 log2(longest row / mean row length)
 *   6 log2(k)              7 log2(bytes per X element of dt)
 * Errors: SPMM_EINVAL (NULL, k outside 1..64, unknown dt).
 */
spmm_status_t spmm_tile_features(spmm_handle_t h, int k, spmm_xdtype_t dt, float* feat);

/* Current variant of every tile (host uint8[n_tiles]). */
spmm_status_t spmm_get_variants(spmm_handle_t h, uint8_t* variant);

/*
 * Set the variant of every tile (host uint8[n_tiles], values <
 * SPMM_NUM_VARIANTS) and re-encode the work items on the host.  Device or
 * pinned copies are released and rebuilt by the next call that needs them,
 * so no work on the handle may be in flight.  The matrix is unchanged.
 * Errors: SPMM_EINVAL (NULL, a value out of range), SPMM_ENOMEM.
 */
spmm_status_t spmm_set_variants(spmm_handle_t h, const uint8_t* variant);

/* Largest number of buckets spmm_selector_collect forms. */
#define SPMM_MAX_BUCKETS 128

typedef struct {
    uint32_t min_tiles;  /* smallest bucket, in tiles; 0 -> 64                */
    uint32_t reps;       /* timed launches per (bucket, variant); 0 -> 5      */
} spmm_tune_opts;

/*
 * Bucketed timing (device placement only).  Tiles are bucketed by features
 * 0, 4 and 5 (size, single-entry fraction, skew); neighbouring feature
 * cells merge until each bucket holds at least min_tiles tiles.  For every
 * bucket and variant, a matrix made of that bucket's tiles alone, all in
 * that variant, is encoded, uploaded and multiplied by an n_cols x k X of
 * type dt (library-owned, zero-filled: timing does not depend on values);
 * the median launch time over reps launches, divided by the bucket's tile
 * count, is the time per tile.  Synchronous on s.
 *   bucket   : host uint32[n_tiles] (output): bucket of each tile
 *   n_buckets: (output) number of buckets, <= SPMM_MAX_BUCKETS
 *   ns       : host float[SPMM_MAX_BUCKETS * SPMM_NUM_VARIANTS] (output):
 *              ns[b * SPMM_NUM_VARIANTS + v], nanoseconds per tile
 * The handle's own variants and device copies are not touched.
 * Errors: SPMM_EINVAL, SPMM_ESTATE (pinned placement), SPMM_ENOMEM, SPMM_EHIP.
 */
spmm_status_t spmm_selector_collect(spmm_handle_t h, int k, spmm_xdtype_t dt, const spmm_tune_opts* opts,
                                    uint32_t* bucket, uint32_t* n_buckets, float* ns, hipStream_t s);

/*
 * Exhaustive autotuner: spmm_selector_collect, then every tile takes the
 * variant of least time in its bucket (the lowest index on ties), then
 * spmm_set_variants.  ns (host float[SPMM_MAX_BUCKETS * SPMM_NUM_VARIANTS]
 * or NULL) receives the timing table, n_buckets (or NULL) its row count.
 */
spmm_status_t spmm_autotune(spmm_handle_t h, int k, spmm_xdtype_t dt, const spmm_tune_opts* opts,
                            uint32_t* n_buckets, float* ns, hipStream_t s);

/*
 * The cost model: an MLP 8 -> 64 -> 64 -> SPMM_NUM_VARIANTS with ReLU after
 * the two hidden layers, FP32.  Its parameters are one float array of
 * SPMM_MLP_PARAMS values, each weight matrix row-major [fan_in][fan_out]
 * (out = in . W + b):  W1 [8][64], b1 [64], W2 [64][64], b2 [64],
 * W3 [64][V], b3 [V], at the offsets below.
 */
#define SPMM_MLP_HIDDEN 64
#define SPMM_MLP_OFF_W1 0
#define SPMM_MLP_OFF_B1 (SPMM_MLP_OFF_W1 + SPMM_NUM_FEATURES * SPMM_MLP_HIDDEN)
#define SPMM_MLP_OFF_W2 (SPMM_MLP_OFF_B1 + SPMM_MLP_HIDDEN)
#define SPMM_MLP_OFF_B2 (SPMM_MLP_OFF_W2 + SPMM_MLP_HIDDEN * SPMM_MLP_HIDDEN)
#define SPMM_MLP_OFF_W3 (SPMM_MLP_OFF_B2 + SPMM_MLP_HIDDEN)
#define SPMM_MLP_OFF_B3 (SPMM_MLP_OFF_W3 + SPMM_MLP_HIDDEN * SPMM_NUM_VARIANTS)
#define SPMM_MLP_PARAMS (SPMM_MLP_OFF_B3 + SPMM_NUM_VARIANTS)

/*
 * He-uniform initial weights, W ~ U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)),
 * zero biases, from SplitMix64 draws keyed by seed (host float[PARAMS]).
 */
spmm_status_t spmm_mlp_init(uint64_t seed, float* params);

/*
 * Inference on the device: out[i * V + v] = predicted log time of variant v
 * for feature row i, choice[i] = argmin_v (lowest index on ties).
 *   params: device float[PARAMS]; feat: device float[n * 8];
 *   out: device float[n * V] or NULL; choice: device uint8[n] or NULL.
 * Asynchronous on s.
 */
spmm_status_t spmm_mlp_predict(const float* params, const float* feat, int64_t n, float* out,
                               uint8_t* choice, hipStream_t s);

/*
 * Loss and gradient on the device.  L = sum_{i,v} m_iv (out_iv - y_iv)^2 /
 * max(1, sum m), m = mask (uint8, non-zero = measured) or all ones when
 * mask is NULL.  grad: device float[PARAMS] (dL/dparams, same layout);
 * loss: device double[1] or NULL.  Reductions run in a fixed order.  The
 * call allocates its workspace and synchronises s before returning.
 */
spmm_status_t spmm_mlp_grad(const float* params, const float* feat, const float* target, const uint8_t* mask,
                            int64_t n, float* grad, double* loss, hipStream_t s);

/*
 * One Adam step (Kingma and Ba, 2015) on device arrays of PARAMS floats:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t >= 1.
 */
spmm_status_t spmm_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t t, float lr,
                            float beta1, float beta2, float eps, hipStream_t s);

typedef struct {
    uint32_t epochs;  /* 0 -> 30                                              */
    uint32_t batch;   /* minibatch rows; 0 -> 1024                            */
    float lr;         /* 0 -> 1e-3 (Adam b1 0.9, b2 0.999, eps 1e-8)          */
    uint64_t seed;    /* shuffling of the rows in every epoch                 */
} spmm_train_opts;

/*
 * Train the cost model on the current device: minibatch Adam on the masked
 * MSE, rows shuffled every epoch (SplitMix64 Fisher-Yates keyed by seed).
 *   feat: host float[n * 8]; target: host float[n * V] (log ns per tile);
 *   mask: host uint8[n * V] or NULL; params: host float[PARAMS], initial
 *   weights in, trained weights out; loss_trace: host double[epochs] (mean
 *   minibatch loss per epoch) or NULL.  Synchronous.
 */
spmm_status_t spmm_selector_train(const float* feat, const float* target, const uint8_t* mask, int64_t n,
                                  const spmm_train_opts* opts, float* params, double* loss_trace);

/*
 * Learned selection: features of every tile (for k and dt), cost-model
 * inference on the device, then spmm_set_variants with the argmin.
 *   params: host float[PARAMS].  Synchronous.
 */
spmm_status_t spmm_select_learned(spmm_handle_t h, const float* params, int k, spmm_xdtype_t dt);

/* ---------------------------------------------------------------------------
 * Eigensolver (Section 4.2): a few eigenpairs of a symmetric sparse matrix
 * by the block Krylov-Schur method, every sparse product an SpMM with k =
 * block columns.
 * ------------------------------------------------------------------------- */
#define SPMM_EIGS_LM 0  /* largest magnitude */
#define SPMM_EIGS_LA 1  /* largest algebraic */
#define SPMM_EIGS_SA 2  /* smallest algebraic */

typedef struct {
    int32_t nev;          /* eigenpairs wanted, >= 1                                   */
    int32_t block;        /* block size b (vectors per SpMM), 1..16; 0 -> 4            */
    int32_t max_dim;      /* basis columns m before a restart: a multiple of b with
                             m >= nev + b, m + b <= n, m * b <= 2048 and
                             m + b <= 512;
                             0 -> the smallest multiple of b >= min(max(6 nev,
                             nev + 4b, 24 b), max(128, 8 nev + 4b)), lowered to
                             the limits                                            */
    int32_t which;        /* SPMM_EIGS_LM / _LA / _SA                                  */
    int32_t max_restarts; /* 0 -> 500                                                  */
    int32_t reserved;     /* 0                                                         */
    double tol;           /* converged when ||A y - theta y|| <= tol |theta|; 0 -> 1e-5 */
    uint64_t seed;        /* starting block (and any replacement block): uniform
                             [-1/2, 1/2) from SplitMix64 of (seed, row, column)       */
} spmm_eigs_opts;

typedef struct {
    int32_t n_converged;  /* wanted pairs whose residual estimate met tol  */
    int32_t restarts;
    int64_t n_spmm;       /* SpMM calls (each with k = block)              */
    double spmm_ms;       /* device time of the SpMM calls (HIP events)    */
    double total_ms;      /* wall-clock time of the whole call             */
    int32_t max_dim;      /* m and b actually used                         */
    int32_t block;
    double dense_ms;      /* device time of the dense basis kernels (events) */
    double dense_bytes;   /* their algorithmic HBM bytes: 4 n (p + q) for
                             C = A^T B, 4 n (p + 2q) for W += A C            */
    int64_t n_orth;       /* blocks projected out of the basis ...          */
    int64_t n_reorth;     /* ... and how many needed the second projection  */
} spmm_eigs_info;

/*
 * Eigenpairs of a symmetric A (handle built from a symmetric CSR; symmetry
 * is not checked) with the block Krylov-Schur method: an orthonormal basis
 * V (n x (m + b) FP32 in HBM) grows one block at a time (W = A V_j by
 * spmm_run, projected out of V in FP64 arithmetic -- a second time where
 * the first projection cancelled a column by more than 1/sqrt(2) -- then
 * made orthonormal by two SVQB passes), T = V^T A V is kept on the host in FP64,
 * and after m columns the Ritz pairs of T (cyclic Jacobi) decide: stop when
 * the nev wanted ones have residual estimates <= tol |theta|, else keep the
 * best p ~ (m + nev) / 2 Ritz vectors and the residual block and expand
 * again (thick restart).  Directions of W lost to cancellation (an invariant
 * subspace) are replaced by random vectors orthogonal to V.
 *   h      : square.  Tiles in HBM (SPMM_PLACE_DEVICE), or in pinned host
 *            memory (SPMM_PLACE_PINNED_HOST): then every product streams
 *            the tiles as spmm_stream_run does -- the semi-external
 *            eigensolver of Section 4.2 with A in host DRAM and the basis in
 *            HBM -- on two streams of the solver's own, after the work
 *            already queued on s.  Both give identical results.
 *   evals  : host double[nev], wanted end first (|theta| descending for LM,
 *            ties by value descending).
 *   evecs  : device float n x nev (row stride ldvec >= nev): unit Ritz
 *            vectors in the order of evals; or NULL.
 *   resid  : host double[nev], residual estimates ||A y - theta y|| / |theta|
 *            (absolute if theta = 0); or NULL.
 *   info   : or NULL.
 * Device workspace: two bases of n x (m + b) FP32 (stored as m / b + 1
 * blocks of b columns, each n x b contiguous) and two n x b FP32 buffers
 * plus 32 MiB, allocated per call (and the handle's ring, for tiles in host
 * memory).  Synchronous (several host
 * round trips per block).  Errors: SPMM_EINVAL, SPMM_ENOMEM, SPMM_EHIP,
 * SPMM_ENOTCONV (max_restarts reached:
 * evals, evecs, resid and info hold the current Ritz pairs; or, with the
 * message saying so, a replacement block came out rank deficient: outputs
 * unspecified).
 */
spmm_status_t spmm_eigs(spmm_handle_t h, const spmm_eigs_opts* opts, double* evals, float* evecs, int64_t ldvec,
                        double* resid, spmm_eigs_info* info, hipStream_t s);

/*
 * The eigensolver's tall-skinny dense products, for FP32 row-major blocks
 * of n rows (Section 4.2 notes that an eigensolver adds many dense matrix
 * operations to the SpMMs):
 *   spmm_dense_tn : C = A^T B.  A n x p (stride lda >= p), B n x q (stride
 *                   ldb >= q), 1 <= p <= 512, 1 <= q <= 16, p q <= 2048.
 *                   C: device double p x q, row-major.  Products and sums
 *                   in FP64, summed in an order fixed by n alone (the same
 *                   bits for the same inputs).  work: device scratch of at
 *                   least spmm_dense_tn_workspace(n, p, q) bytes.
 *   spmm_dense_nn : W = alpha W + beta A C.  A n x p (stride lda >= p), C
 *                   device double p x q row-major, W n x q (stride ldw >= q;
 *                   must not overlap A).  FP64 sums, FP32 store; W is not
 *                   read when alpha = 0.
 * Asynchronous on s.  Errors: SPMM_EINVAL, SPMM_EHIP.
 */
size_t spmm_dense_tn_workspace(int64_t n, int p, int q);
spmm_status_t spmm_dense_tn(const float* A, int64_t lda, int p, const float* B, int64_t ldb, int q, int64_t n,
                            double* C, void* work, size_t work_bytes, hipStream_t s);
spmm_status_t spmm_dense_nn(const float* A, int64_t lda, int p, const double* C, int q, double alpha, double beta,
                            float* W, int64_t ldw, int64_t n, hipStream_t s);

/*
 * Host helper: all eigenpairs of a small dense symmetric matrix by the
 * cyclic Jacobi method, the Rayleigh-Ritz step spmm_eigs applies to T.
 *   a : host double n x n row-major, exactly symmetric (else SPMM_EINVAL).
 *   w : host double[n], ascending.   z : host double n x n row-major,
 *       column j the unit eigenvector of w[j].
 * 1 <= n <= 1024 (each Jacobi sweep costs O(n^3)).  No device work.
 */
spmm_status_t spmm_sym_eig_small(int n, const double* a, double* w, double* z);

#ifdef __cplusplus
}
#endif

#endif /* SPMM_H */
