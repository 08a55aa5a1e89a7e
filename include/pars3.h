/*
 * pars3.h -- C ABI of the MI355X (gfx950) skew-symmetric SpMV library.
 *
 * Problem (Section 1, eq. (1)): products and solves with a sparse
 * skew-symmetric S (S = -S^T) or a shifted skew-symmetric A = alpha*I + S.
 * Only the strictly lower triangle L of S is stored (the SSS idea of keeping
 * one triangle, Sections 1 and 3), so S = L - L^T and every stored l_ij
 * (i > j) contributes y_i += l_ij x_j and y_j -= l_ij x_i (eqs. (2)-(6),
 * Section 3.1.2).  Before multiplying, the matrix is reordered by reverse
 * Cuthill-McKee into a band and the band is split three ways (diagonal/inner,
 * middle, outer) by distance from the diagonal (Sections 1 and 3.1.2).
 *
 * Conventions for every call:
 *  - Return value: pars3_status; PARS3_OK (0) on success.  On failure a
 *    message is available from pars3_last_error() (thread-local).
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory (for example torch tensors' data_ptr()).  The library never
 *    takes ownership of caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it; calls documented as synchronous wait for
 *    it before returning.
 *  - Device faults of asynchronous calls surface as PARS3_EHIP at the next
 *    synchronising call.
 *  - One handle must not be used from two threads at once; distinct handles
 *    are independent.  No C++ exception crosses this interface.
 */
#ifndef PARS3_H
#define PARS3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PARS3_OK = 0,
  PARS3_EINVAL = 1,     /* invalid argument, sizes or row pointers */
  PARS3_ENOTLOWER = 2,  /* an entry outside the strictly lower triangle */
  PARS3_EUNSORTED = 3,  /* unsorted or duplicate columns in a row */
  PARS3_ENOMEM = 4,     /* host or device allocation failed */
  PARS3_EHIP = 5,       /* HIP runtime error */
  PARS3_ESTATE = 6,     /* wrong call order or dtype not available */
  PARS3_ENOCONV = 7,    /* iteration limit reached before the tolerance */
  PARS3_EBREAKDOWN = 8, /* singular recurrence (gamma = 0) */
  PARS3_ENAN = 9,       /* NaN or Inf met in a solver */
  PARS3_EIO = 10        /* file input/output error */
} pars3_status;

typedef enum { PARS3_F64 = 0, PARS3_F32 = 1, PARS3_BF16 = 2 } pars3_dtype;

enum { PARS3_ORDER_RCM = 0, PARS3_ORDER_ORIGINAL = 1 };

/* What the stored triangle L stands for: S = L - L^T (skew-symmetric, the
 * paper's case) or S = L + L^T (symmetric: the SSS format the paper starts
 * from, Section 1, where the same one-triangle storage serves both). */
typedef enum { PARS3_SKEW = 0, PARS3_SYMMETRIC = 1 } pars3_kind;

typedef struct pars3_matrix pars3_matrix;

/* Split and layout parameters of pars3_reorder (Sections 1 and 3.1.2: the
 * band is split into an inner part, a middle part and an outer part whose
 * distance from the diagonal is a user-given bandwidth).  For a stored entry at
 * distance d = i - j (in the reordered matrix):
 *   inner  : d <= w_in            (w_in = 0: only the diagonal, i.e. the shift)
 *   middle : w_in < d <= t_out
 *   outer  : d > t_out
 * The inner part is stored diagonal-major without indices; the middle and
 * outer parts are stored in tile-pair blocks of tile_rows x tile_rows (the
 * outer part in blocks of its own).  Fields set to -1 (or 0 where noted) take
 * the defaults. */
typedef struct {
  int32_t w_in;        /* inner half-width, 0..64; -1 = 0 (the paper's diagonal split) */
  int32_t t_out;       /* middle/outer boundary; -1 = max(beta - 3, 0) ("outer bandwidth 3") */
  int32_t tile_rows;   /* rows per tile: 64, 128, 256, 512 or 1024; 0 = 256 */
  int32_t value_dtype; /* pars3_dtype of the stored values used by pars3_spmv */
  int32_t keep_fp64;   /* also keep FP64 values (needed by the mixed-precision solver) */
  int32_t permute;     /* 1 = reverse Cuthill-McKee (default); 0 = keep the given order */
  int32_t engine;      /* pars3_engine of pars3_spmv's one-right-hand-side products */
} pars3_split_params;

/* Which kernel serves pars3_spmv (and pars3_spmv_noalloc) with one
 * right-hand side.  PARS3_ENGINE_TILES: the skew product over the split
 * (the method).  PARS3_ENGINE_CSR: pars3_reorder also builds the full CSR of
 * the reordered matrix (both triangles; rocSPARSE, as pars3_csr_create with
 * the stored FP64 or FP32 values) and those products run on it, for matrices
 * where the split does not pay (power-law degree distributions, whose
 * reordered bandwidth stays near n); the learned selector can choose it.
 * Products with several right-hand sides, the solvers and batches always use
 * the split.  Not with BF16 values (EINVAL). */
typedef enum { PARS3_ENGINE_TILES = 0, PARS3_ENGINE_CSR = 1 } pars3_engine;

/* Fills `p` with the defaults (RCM, paper split, 256-row tiles, FP64). */
void pars3_split_params_default(pars3_split_params *p);

/* Read-back of the split (pars3_get_split_info). */
typedef struct {
  int64_t n, nnz;
  int32_t beta;        /* max d after reordering (the RCM bandwidth) */
  int32_t w_in, t_out; /* resolved split parameters */
  int32_t tile_rows, value_dtype, permute;
  int64_t nnz_inner, nnz_middle, nnz_outer; /* the three parts, by definition */
  int32_t n_tiles;
  int32_t n_blocks;          /* non-empty tile-pair blocks (middle and outer) */
  int32_t max_blocks;        /* max over tiles of blocks read on one side */
  int32_t n_components;      /* connected components of the graph of S */
  int32_t bfs_levels;        /* levels of the Cuthill-McKee search (max over components) */
  int32_t engine;            /* pars3_engine in use */
  /* LDS bank passes of the product's adds (layout quality, not part of the
   * method).  The product's FP64 LDS adds are served in quarters of a
   * wavefront (16 lanes), so a block's entries are read in aligned runs of
   * 16 from the block start; a run takes as many passes as the most
   * frequent row offset mod 32 among its entries (row side) plus the same
   * for the column offsets (column side).  lds_runs counts the runs of all
   * blocks, lds_passes_sorted sums the passes of the entries sorted by
   * (block, diagonal, row), lds_passes those of the stored order, in which
   * pars3_reorder regroups the entries of blocks where that lowers bank
   * conflicts more than it spreads the x gathers (lds_passes <=
   * lds_passes_sorted; 2 lds_runs is the floor). */
  int64_t lds_runs, lds_passes_sorted, lds_passes;
} pars3_split_info;

/* Host-only validation of a strictly lower CSR (no device use).  Checks, rows
 * in order and entries in order, the first violation deciding the code:
 * EINVAL for n < 0, nnz < 0, n or nnz > INT32_MAX, NULL rowptr (or col when
 * nnz > 0), rowptr[0] != 0, rowptr[n] != nnz, decreasing row pointers;
 * ENOTLOWER for col < 0 or col >= row; EUNSORTED for a column not larger than
 * its predecessor in the row (unsorted or duplicate). */
pars3_status pars3_validate(int64_t n, int64_t nnz_lower, const int32_t *rowptr, const int32_t *col);

/* Creates a handle from host arrays rowptr[n+1], col[nnz], val[nnz] holding
 * the strictly lower triangle L (Sections 1 and 3: one triangle stored).  The
 * arrays are validated (as pars3_validate) and copied to the current HIP
 * device; the caller keeps ownership and may free them on return.  Explicit
 * zeros are kept as structural entries.  n = 0 and nnz = 0 are valid.  On error
 * *out is set to NULL and nothing stays allocated.  Synchronous. */
pars3_status pars3_create(int64_t n, int64_t nnz_lower, const int32_t *rowptr, const int32_t *col,
                          const double *val, pars3_matrix **out);

/* SSS storage (Section 1): the strictly lower triangle as for pars3_create,
 * plus an optional diagonal array diag[n] (host, FP64; NULL: D = 0), and the
 * kind of S.  Products then compute y = shift*x + D x + S x with
 * S = L - L^T (PARS3_SKEW) or L + L^T (PARS3_SYMMETRIC).  A skew matrix
 * without a diagonal is exactly what pars3_create makes.  The diagonal is
 * copied to the device (FP64, and rounded to FP32 for FP32 vectors) and
 * follows the reordering.  The MRS solvers need S skew-symmetric and D = 0
 * (ESTATE otherwise).  Errors: those of pars3_create; EINVAL for another
 * kind. */
pars3_status pars3_create_sss(int64_t n, int64_t nnz_lower, const int32_t *rowptr, const int32_t *col,
                              const double *val, const double *diag, int32_t kind, pars3_matrix **out);

/* *kind receives the handle's pars3_kind, *has_diag 1 when a diagonal array
 * was given (either pointer may be NULL). */
pars3_status pars3_get_kind(const pars3_matrix *A, int32_t *kind, int32_t *has_diag);

/* The diagonal array in the reordered numbering (host, n doubles:
 * out[k] = diag[perm[k]]).  ESTATE before pars3_reorder or without a
 * diagonal.  Synchronous. */
pars3_status pars3_get_diagonal(const pars3_matrix *A, double *out);

/* Shifted skew-symmetric form (Section 1: a system A = J - S with J symmetric
 * positive semi-definite is brought to the alpha*I + S form).  For a skew
 * handle with J = alpha*I + D diagonal and positive definite (D = 0 when the
 * handle has no diagonal array, then alpha > 0), the two-sided scaling
 *   J^(-1/2) (alpha*I + D + S) J^(-1/2) = I + S~,  S~ = J^(-1/2) S J^(-1/2)
 * is exact and S~ is skew.  *out receives a new handle holding S~ (caller
 * owns it; pars3_destroy), with A's structure, permutation and split
 * parameters, already reordered; solve (I + S~) x~ = b~ with b~_i =
 * b_i / sqrt(alpha + d_i) and take x_i = x~_i / sqrt(alpha + d_i).
 * Synchronous.  Errors: ESTATE before pars3_reorder or for a symmetric
 * handle; EINVAL when some alpha + d_i <= 0. */
pars3_status pars3_skew_form(const pars3_matrix *A, double alpha, pars3_matrix **out, void *stream);

/* Frees every device and host resource of the handle.  NULL is allowed. */
void pars3_destroy(pars3_matrix *A);

/* Reorders and splits on the GPU (Section 3.1.2: reverse Cuthill-McKee, then
 * the three-way split; both are integer work and bit-exact against the fixed
 * tie-break definition).  p == NULL: when a network is in use
 * (pars3_model_use), the configuration it selects from the features of the
 * reordered matrix (Section 3.1.2 leaves the outer bandwidth to be chosen from
 * the bandwidth and density of the reordered matrix; as pars3_select with the
 * network's stored grid), else the defaults.  Reverse Cuthill-McKee runs once
 * per handle; later calls with other parameters only re-split and rebuild the
 * layouts.  Also reserves 2 n x 64 bytes of device scratch for products in the
 * caller's numbering (pars3_spmv with PARS3_ORDER_ORIGINAL, up to 8 FP64
 * right-hand sides), so that pars3_spmv never allocates.  Synchronous (reads
 * back the split sizes).  Errors: EINVAL for out-of-range parameters or
 * w_in > t_out; ENOMEM. */
pars3_status pars3_reorder(pars3_matrix *A, const pars3_split_params *p, void *stream);

/* y = shift*x + S*x  (the shifted skew-symmetric product; Section 1 and eqs.
 * (2)-(6)); for a handle from pars3_create_sss, y = shift*x + D x + S x with
 * S of the handle's kind (a symmetric S adds the transposed products instead
 * of subtracting them).  x and y are device arrays of n x k values, row-major (k values of
 * one row are contiguous), k in {1, 2, 4, 8}.  vec_dtype is PARS3_F64 when the
 * stored values are FP64 and PARS3_F32 when they are FP32 or BF16 (products
 * formed in FP32, summed per row in FP64, results rounded to FP32).  order = PARS3_ORDER_RCM: x and y are in the reordered
 * numbering; PARS3_ORDER_ORIGINAL: in the caller's numbering (a gather and a
 * scatter are added).  x and y must not overlap and, when k > 1, must be
 * 16-byte aligned (rows are read and written as 16-byte vectors).  On a
 * handle reordered with engine = PARS3_ENGINE_CSR, products with k = 1 in the
 * values' precision run on its full CSR (rocSPARSE; with shift != 0 a
 * scaled copy of x into y first).
 * Asynchronous: neither allocates nor waits for the stream, so it may be
 * captured in a hipGraph (in both orders).  Errors: ESTATE before
 * pars3_reorder or for a dtype mismatch; EINVAL otherwise. */
pars3_status pars3_spmv(pars3_matrix *A, double shift, const void *x, void *y, int32_t k, int32_t vec_dtype,
                        int32_t order, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * of pars3_spmv with PARS3_ORDER_ORIGINAL (x and y in the caller's numbering,
 * same arguments and kernels, so the same results up to the order in which
 * the product adds its per-row sums, which may vary from call to call in
 * either entry point), whose reordered
 * copies of x and y live in a fixed device array of the library
 * (PARS3_NOALLOC_SCRATCH_BYTES = 64 MiB per GPU, reserved when the library's
 * code is loaded on that GPU and held until the process ends) instead of the
 * handle's scratch, and always on the split's kernel (also on a handle with
 * engine = PARS3_ENGINE_CSR).  Limit: n x k x (8 for FP64, 4 for FP32) <= 32 MiB, half
 * of the array per vector (e.g. n <= 4,194,304 rows for one FP64 right-hand
 * side); larger inputs return EINVAL.  Calls no hipMalloc, hipFree or other
 * allocating routine; the array's device address is looked up once per GPU
 * on the first call there.  Every call on one GPU uses the same array and
 * leaves its contents behind; each call writes every byte it reads first, so
 * nothing needs clearing.  Calls that overlap in time on one GPU (several
 * streams, or host threads) race on the array and give wrong results: order
 * them on one stream.  Asynchronous.  Errors as pars3_spmv, plus ESTATE while
 * per-kernel timing is on (pars3_set_profiling records events). */
#define PARS3_NOALLOC_SCRATCH_BYTES (64ll << 20)
pars3_status pars3_spmv_noalloc(pars3_matrix *A, double shift, const void *x, void *y, int32_t k,
                                int32_t vec_dtype, void *stream);

/* Inspection (host output buffers, caller-allocated; synchronous).
 * perm[n]: new position k holds old node perm[k].  The permuted strictly lower
 * triangle is returned in CSR order (rows, then columns ascending):
 * rowptr[n+1], col[nnz], val[nnz] (FP64, signs fixed by eq. (2)) and part[nnz]
 * (0 inner, 1 middle, 2 outer); any output pointer may be NULL.  Values of the
 * stored precision (pars3_get_values): FP64 as double, FP32 as float, BF16 as
 * uint16 bit patterns, in the same CSR order. */
pars3_status pars3_get_perm(const pars3_matrix *A, int32_t *perm);
pars3_status pars3_get_permuted_lower(const pars3_matrix *A, int32_t *rowptr, int32_t *col, double *val,
                                      int8_t *part);
pars3_status pars3_get_split_info(const pars3_matrix *A, pars3_split_info *info);
pars3_status pars3_get_values(const pars3_matrix *A, int32_t dtype, void *host);

/* Per-kernel timing of products (measurement harness).  While enabled, every
 * kernel that pars3_spmv launches is bracketed by two hipEvents recorded on the
 * launch stream (at most 4096 products between reads; later ones are not
 * timed).  pars3_get_profile waits for the recorded events, returns the summed
 * durations in milliseconds per kernel class (ms_band: the product kernel;
 * ms_fixup: work in the caller's numbering, gather and scatter; ms_other:
 * reserved) and the number of timed products, then resets the counters. */
typedef struct {
  int64_t calls;
  double ms_band, ms_fixup, ms_other;
} pars3_profile;
pars3_status pars3_set_profiling(pars3_matrix *A, int32_t enable);
pars3_status pars3_get_profile(pars3_matrix *A, pars3_profile *out);

/* Conflict map of a block-row distribution (Section 3, Fig. 2): block p owns
 * rows [R_p, R_{p+1}) of the reordered matrix (after pars3_reorder; with
 * permute = 0, of the given numbering) and the stored lower entries of those
 * rows.  An entry (i, j) is safe (R1) when j >= R_p, conflicting (R2) when
 * j < R_p: its transposed product lands in another block's output and it
 * reads that block's x_j.  Block 0 never conflicts.  Per block (host output
 * out[nblocks]):
 *   first_row, rows     R_p and R_{p+1} - R_p
 *   safe[3]             R1 entries of the inner, middle and outer parts
 *   conflict[3]         R2 entries of the three parts
 *   reach               smallest column of an R2 entry (R_p when none)
 *   partners            distinct other blocks owning such columns
 *   halo                distinct such columns: x values to receive and
 *                       partial sums to send back for one product
 * bounds: host array of nblocks + 1 nondecreasing row boundaries from 0 to n
 * (empty blocks allowed), or NULL for R_p = floor(p n / nblocks).  Integer
 * work on the GPU; synchronous.  Errors: ESTATE before pars3_reorder; EINVAL
 * for nblocks < 1, bad bounds or a NULL output. */
typedef struct {
  int64_t first_row, rows;
  int64_t safe[3];
  int64_t conflict[3];
  int64_t reach, partners, halo;
} pars3_block_conflicts;
pars3_status pars3_conflict_map(const pars3_matrix *A, int32_t nblocks, const int64_t *bounds,
                                pars3_block_conflicts *out, void *stream);

/* Three features of the conflict map over nblocks balanced row blocks of the
 * reordered matrix (Section 3, Fig. 2; the closing remarks of Section 4.1
 * propose identifying the data races ahead of time for a given number of
 * processors), the learned selector's inputs 33-35 with nblocks =
 * PARS3_SELECT_BLOCKS, the 8 XCDs whose contiguous tile ranges the product
 * spreads its work over:
 *   feat3[0] = conflicting (R2) entries of all blocks / nnz (0 when nnz = 0)
 *   feat3[1] = max over blocks of halo / rows
 *   feat3[2] = max over blocks of (first_row - reach) / rows
 * (rows of an empty block count as 1).  Ratios of integer counts, so
 * bit-exact against the same definition on the host.  Synchronous.  Errors
 * as pars3_conflict_map. */
#define PARS3_SELECT_BLOCKS 8
pars3_status pars3_conflict_features(const pars3_matrix *A, int32_t nblocks, double *feat3, void *stream);

/* Full-CSR comparison path (the storage that keeps every nonzero, Section 1).
 * pars3_csr_create builds, on the GPU, the full CSR of S (both triangles,
 * 2*nnz entries, columns ascending in every row; with a diagonal array, D + S
 * with an entry d_i at (i, i) for every nonzero d_i, and the transposed
 * entries signed by the handle's kind) in the reordered numbering
 * (order = PARS3_ORDER_RCM, after pars3_reorder) or in the caller's numbering
 * (PARS3_ORDER_ORIGINAL), with FP64 or FP32 values (value_dtype).  Synchronous.
 * pars3_csr_spmv computes y = shift*x + S*x (device vectors of n values of the
 * value precision, x != y) with engine 0 = this library's CSR-vector kernel
 * (a power-of-two group of lanes per row) or engine 1 = rocSPARSE's CSR
 * product (default algorithm; shift must be 0 there).  Asynchronous.
 * pars3_csr_get copies the CSR (FP64 values) to caller-allocated host arrays
 * rowptr[n+1], col[m], val[m] (m from pars3_csr_size: 2*nnz plus the nonzero
 * diagonal entries); NULL outputs are skipped. */
typedef struct pars3_csr pars3_csr;
pars3_status pars3_csr_size(const pars3_csr *C, int64_t *n, int64_t *nnz_full);
pars3_status pars3_csr_create(const pars3_matrix *A, int32_t order, int32_t value_dtype, pars3_csr **out);
pars3_status pars3_csr_spmv(pars3_csr *C, double shift, const void *x, void *y, int32_t engine, void *stream);
pars3_status pars3_csr_get(const pars3_csr *C, int32_t *rowptr, int32_t *col, double *val);
void pars3_csr_destroy(pars3_csr *C);

/* Exhaustive autotuner (Section 3.1.2 leaves the outer bandwidth to the user;
 * on the GPU the choice also covers the inner band width and the tile
 * height).  pars3_tune_grid_default writes the default grid for one value
 * precision into grid[0..cap) and its size into *count (grid may be NULL to
 * query the size): tile_rows in {64, 128, 256, 512, 1024} x w_in in {0, 1, 2, 4} x
 * t_out in {paper (-1: beta - 3), -2: half the RCM bandwidth} (40 entries),
 * then, for FP64 and FP32 values, one entry with engine = PARS3_ENGINE_CSR
 * (the full-CSR product; 41 entries).
 * pars3_autotune applies every configuration of grid[0..ngrid) to A (the
 * reordering is computed once and kept; t_out = -1 and -2 are resolved against
 * beta, and t_out is raised to w_in where it would fall below it), times
 * pars3_spmv-equivalent products with k right-hand sides on a fixed vector
 * (median of three batches of reps products, hipEvents on `stream`, after
 * 3 warm-up products, and before the first configuration products for at
 * least 20 ms so that the GPU clock is steady), writes
 * out[g] = {resolved parameters, microseconds per product}, sets *best (may
 * be NULL) to the fastest index and leaves A split with that configuration.
 * Synchronous.  Timings are of cache-warm repeated products. */
typedef struct {
  pars3_split_params params;
  double us;
} pars3_tune_result;
pars3_status pars3_tune_grid_default(int32_t value_dtype, pars3_split_params *grid, int32_t cap, int32_t *count);
pars3_status pars3_autotune(pars3_matrix *A, const pars3_split_params *grid, int32_t ngrid, int32_t k, int32_t reps,
                            pars3_tune_result *out, int32_t *best, void *stream);

/* 32 sparsity features of the reordered lower triangle (after
 * pars3_reorder): the band profile, spread of distances from the diagonal and
 * row-length mix that Section 3.1.2 reads off the structure of the reordered
 * matrix to place the split, as numbers for the configuration selector.  With
 * b_i = i - first column of row i (0 for an empty row), d = i - j per entry,
 * beta = max d and l_i the row length:
 *   f[0] log2 n   f[1] log2 nnz   f[2] nnz/n   f[3] beta/n   f[4] log2(beta+1)
 *   f[5..9]   nearest-rank p10, p50, p90, p99 and max of b_i, each / beta
 *   f[10]     nnz / sum b_i
 *   f[11..18] share of entries with d <= 1, 2, 4, ..., 128
 *   f[19..21] share of entries with d/beta > 1/2, 3/4, 9/10
 *   f[22..28] share of rows with l = 0, 1, 2, 3-4, 5-8, 9-16, >= 17
 *   f[29] max l / mean l   f[30] std(l) / mean(l) (population)
 *   f[31] share of 256-row tiles whose window (tile end - smallest column of
 *         the tile) holds at most 160 KiB of FP64 x and y (16 bytes a row)
 * Ratios with a zero denominator are 0; n = 0 gives all zeros.  Counts are
 * taken on the GPU, on `stream` (after the work already queued there); f
 * (host, 32 doubles) is written on return (synchronous).  Errors: ESTATE
 * before pars3_reorder; EINVAL for a NULL argument. */
pars3_status pars3_features(const pars3_matrix *A, double *f, void *stream);

/* MRS solver for (alpha*I + S) x = b (Section 1: the minimal-residual method
 * for shifted skew-symmetric systems that motivates the product; each
 * iteration costs one product with S and one inner product).  x_k minimises
 * ||b - A x|| over x_0 + K_k(S, r_0) by a skew Lanczos recurrence with Givens
 * rotations.  Every iteration runs on the device (the product with a fused
 * epilogue that also applies the previous iteration's vector update, and one
 * scalar kernel, replayed from a hipGraph);
 * the host polls the stop flag at most every check_every iterations (rounded
 * down to whole six-iteration replays, at least one), sooner when the
 * observed rate of |eta| says the tolerance is near.
 *
 * precision = PARS3_F64: the whole iteration in FP64 (needs FP64 values).
 * precision = PARS3_F32 / PARS3_BF16: mixed precision; FP64 iterative
 * refinement (residual b - A x with FP64 values and vectors) around inner MRS
 * solves whose matrix values are FP32 / BF16 and vectors FP32, with FP64 inner
 * products and scalars; each inner solve reduces its residual by inner_tol
 * (0 = 1e-6 for FP32, 1e-2 for BF16), or by less when less already meets
 * the outer tolerance; at most max_refine refinements.  Needs a
 * layout built with value_dtype F32 / BF16 and keep_fp64 = 1.
 *
 * Stopping: ||b - A x|| <= tol ||b|| (for FP64, the recurrence's |eta|;
 * maxit bounds the total number of iterations (inner ones for mixed).  b and x
 * (initial guess in, solution out) are device FP64 arrays of n values in the
 * numbering selected by order.  hist (host, hist_len values, may be NULL when
 * hist_len = 0) receives |eta_j|/||b|| of the first iterations.  The stream is
 * the caller's: the solve starts after work already queued on it and is
 * synchronous (returns when x is written).  info (may be NULL) receives
 * iteration counts, the final status and the true relative residual
 * ||b - A x||/||b|| of the returned x computed in FP64.
 * Errors: ESTATE before pars3_reorder or when the needed values are not
 * stored; EINVAL for bad options; ENOCONV when the tolerance was not reached
 * (x holds the last iterate); EBREAKDOWN when gamma = 0 (singular A, e.g.
 * alpha = 0 with n odd); ENAN when a NaN or Inf appears. */
typedef struct {
  double tol;           /* relative residual target (default 1e-10) */
  int32_t maxit;        /* iteration limit (default 10000) */
  int32_t check_every;  /* most iterations between host polls of the stop flag (default 32) */
  int32_t precision;    /* PARS3_F64 (default), PARS3_F32 or PARS3_BF16 */
  double inner_tol;     /* mixed: relative reduction of each inner solve (0 = default) */
  int32_t max_refine;   /* mixed: maximum number of refinements (default 30) */
  int32_t order;        /* PARS3_ORDER_RCM (default) or PARS3_ORDER_ORIGINAL */
  int32_t hist_len;     /* length of hist (0 = no history) */
  double *hist;         /* host array of hist_len values, or NULL */
} pars3_mrs_opts;

typedef struct {
  int32_t iters;       /* total MRS iterations (inner ones for mixed) */
  int32_t refinements; /* mixed: outer refinement steps taken */
  int32_t status;      /* 0 converged, 1 iteration limit, 2 breakdown, 3 NaN/Inf */
  double relres;       /* ||b - A x|| / ||b|| of the returned x (FP64) */
  double eta;          /* FP64: |eta|/||b|| of the recurrence; mixed: relres */
  double time_ms;      /* wall time of the call */
} pars3_mrs_info;

/* The solver needs S skew-symmetric: a handle made by pars3_create_sss with
 * PARS3_SYMMETRIC gives ESTATE.  A skew handle with a diagonal array D is
 * solved for (alpha*I + D + S) x = b through its shifted skew-symmetric form
 * (see pars3_skew_form): MRS on (I + S~) x~ = J^(-1/2) b to the tolerance
 * tol / sqrt(max j / min j), x = J^(-1/2) x~; info->relres is then the
 * original system's residual and hist the scaled system's.  EINVAL when
 * J = alpha*I + D is not positive definite. */
void pars3_mrs_opts_default(pars3_mrs_opts *o);
pars3_status pars3_mrs_solve(pars3_matrix *A, double alpha, const double *b, double *x, const pars3_mrs_opts *opts,
                             pars3_mrs_info *info, void *stream);

/* Batches of matrices (independent systems of uneven sizes), each reordered
 * and split with its own configuration, processed together: one launch per
 * product covers a work list of (matrix, tile) items split into 8 per-XCD
 * queues of equal estimated cost (matrices largest first, tiles ascending),
 * one workgroup per item, the workgroups of an XCD taking its queue in order;
 * each launch is captured in a hipGraph and replayed.
 *  pars3_batch_create: m reordered handles (the batch keeps pointers to them;
 *    they must outlive it).  The work list is fixed from the handles' tiles
 *    at creation: if a handle is split again (pars3_reorder) with another
 *    tile height or tile count, pars3_batch_spmv and pars3_batch_mrs_solve
 *    return ESTATE before any launch; a new split with the same tiles is
 *    used as it is.
 *  pars3_batch_info: number of items, grid size (8 times the longest queue)
 *    and the 9 queue boundaries (host outputs, each may be NULL).
 *  pars3_batch_spmv: y_i = shifts[i] x_i + D_i x_i + S_i x_i for every matrix
 *    i (D_i = 0 and S_i skew unless made by pars3_create_sss), with
 *    host arrays x[m], y[m] of device pointers (n_i x k row-major vectors in
 *    matrix i's reordered numbering, k in {1, 2, 4, 8}); shifts (host, m) may
 *    be NULL (all zero); 16-byte aligned when k > 1; vec_dtype and
 *    value_dtype as in pars3_spmv (every
 *    matrix must store the values used).  The launch is captured once per
 *    distinct (pointers, shifts, k, dtype) and replayed while they repeat.
 *    Asynchronous on `stream`.
 *  pars3_batch_mrs_solve: MRS for (alphas[i] I + S_i) x_i = b_i for every i
 *    (host arrays of m device pointers to FP64 vectors; x holds x0 on entry),
 *    FP64 iterations (opts->precision must be PARS3_F64; FP64 values
 *    needed), all systems advanced together by one batched product per
 *    iteration (the previous iteration's vector update fused into it) and one
 *    scalar kernel (systems that have converged are skipped), six iterations
 *    per graph replay, the work list compacted whenever the number of running
 *    systems halves (ESTATE if a matrix is symmetric or has a diagonal
 *    array).  infos (host, m,
 *    may be NULL) per system; time_ms is the whole batch's.  Returns the worst
 *    status (ENOCONV, EBREAKDOWN, ENAN) if any system fails.  Synchronous. */
typedef struct pars3_batch pars3_batch;
pars3_status pars3_batch_create(int32_t m, pars3_matrix *const *mats, pars3_batch **out);
void pars3_batch_destroy(pars3_batch *B);
pars3_status pars3_batch_info(const pars3_batch *B, int32_t *n_items, int32_t *grid, int32_t *queue_begin9);
pars3_status pars3_batch_spmv(pars3_batch *B, const double *shifts, const void *const *x, void *const *y, int32_t k,
                              int32_t vec_dtype, int32_t value_dtype, void *stream);
pars3_status pars3_batch_mrs_solve(pars3_batch *B, const double *alphas, const double *const *b, double *const *x,
                                   const pars3_mrs_opts *opts, pars3_mrs_info *infos, void *stream);

/* Batch-level autotuner: the tile height shared by a batch, chosen by timing
 * whole batch launches (a batch's work list is one queue per XCD over all its
 * matrices' tiles, so the best height for the batch is not that of each
 * matrix alone; Section 3.1.2 leaves the split to the user).  For each
 * tile_rows[j] (64, 128, 256, 512 or 1024; nt >= 1) every reordered handle
 * mats[0..m) is split again with that height (its reordering and other split
 * parameters kept, engine set to PARS3_ENGINE_TILES), a batch is made over
 * them and `reps` launches of pars3_batch_spmv with k right-hand sides of
 * vec_dtype (fixed vectors the call allocates, zero shifts, the stored
 * values) are timed with hipEvents on `stream` (at least 20 ms of warm-up
 * launches, then the median of three runs of reps launches).  us[j] (host,
 * nt) receives microseconds per launch, *best (may be NULL) the fastest
 * index, and every handle is left
 * split with that height; batches made over the handles before the call
 * must be made again (ESTATE otherwise, as after any re-split).  Errors:
 * EINVAL (NULL or empty arrays, a bad height, k, vec_dtype or reps), ESTATE
 * (a handle not reordered), those of pars3_reorder and pars3_batch_spmv (the
 * handles then stay split with the height being tried).  Synchronous. */
pars3_status pars3_batch_autotune(pars3_matrix *const *mats, int32_t m, const int32_t *tile_rows, int32_t nt,
                                  int32_t k, int32_t vec_dtype, int32_t reps, double *us, int32_t *best,
                                  void *stream);

/* Learned configuration selector: a multilayer perceptron
 *   x -> ReLU(x W1 + b1) -> ReLU(h1 W2 + b2) -> h2 W3 + b3
 * from the standardised features (pars3_features) of a reordered matrix to
 * one predicted log time ratio log(t_g / t_best) per configuration g of a
 * tuning grid; the argmin is the selection (the paper leaves the outer
 * bandwidth to be chosen from the bandwidth and density of the reordered
 * matrix, Section 3.1.2).  FP32 throughout; weights packed W1 [n_in x h1], b1,
 * W2 [h1 x h2], b2, W3 [h2 x n_out], b3 (input-major).  Training minimises
 * sum M (out - T)^2 / sum M with Adam.
 *  create:      He-uniform weights from SplitMix64(seed), zero biases, Adam
 *               state zero, scaler mean 0 / std 1.
 *  sizes:       sizes4 = {n_in, h1, h2, n_out}; *n_params (either may be NULL).
 *  set/get_params, get_grads: host arrays of n_params floats (set_params also
 *               resets the Adam state and step count).
 *  set/get_scaler, fit_scaler: feature mean and standard deviation (host
 *               arrays of n_in floats; fit_scaler computes them from device
 *               rows X [rows x n_in], population std, 1 where it is 0).
 *  forward:     out[rows x n_out] (device) for device rows X; standardize = 1
 *               applies the scaler first.
 *  loss_grad:   forward and backward on device rows X, targets T and mask M
 *               ([rows x n_out]); keeps the gradients; *loss (host, may be
 *               NULL) receives the loss.  Synchronous when loss != NULL.
 *  adam:        one Adam step with the kept gradients (step count + 1).
 *  train:       `epochs` passes over device rows X, T, M (scaler applied),
 *               each over a shuffle (SplitMix64 keys of seed and epoch) cut
 *               into whole mini-batches of `batch` rows, one Adam step (beta1
 *               0.9, beta2 0.999, eps 1e-8) per mini-batch; loss_hist (host,
 *               may be NULL) receives the mean mini-batch loss per epoch.
 *  select_rows: choice[r] (device) = argmin over the outputs of row r whose
 *               valid[r][g] > 0 (valid may be NULL: all valid).
 * pars3_select: features of A on the GPU, the network's choice over grid
 * (n_out must equal ngrid, n_in 32), and A re-split with that configuration
 * (t_out resolved as in pars3_autotune); *choice (host, may be NULL) receives
 * the index.  Synchronous.  The exhaustive pars3_autotune is the fallback when
 * no trained network is available. */
typedef struct pars3_mlp pars3_mlp;
pars3_status pars3_mlp_create(int32_t n_in, int32_t h1, int32_t h2, int32_t n_out, uint64_t seed, pars3_mlp **out);
void pars3_mlp_destroy(pars3_mlp *m);
pars3_status pars3_mlp_sizes(const pars3_mlp *m, int32_t *sizes4, int64_t *n_params);
pars3_status pars3_mlp_set_params(pars3_mlp *m, const float *host);
pars3_status pars3_mlp_get_params(const pars3_mlp *m, float *host);
pars3_status pars3_mlp_get_grads(const pars3_mlp *m, float *host);
pars3_status pars3_mlp_set_scaler(pars3_mlp *m, const float *mean, const float *stdv);
pars3_status pars3_mlp_get_scaler(const pars3_mlp *m, float *mean, float *stdv);
pars3_status pars3_mlp_fit_scaler(pars3_mlp *m, const float *X, int32_t rows, void *stream);
pars3_status pars3_mlp_forward(pars3_mlp *m, const float *X, int32_t rows, int32_t standardize, float *out,
                               void *stream);
pars3_status pars3_mlp_loss_grad(pars3_mlp *m, const float *X, const float *T, const float *M, int32_t rows,
                                 int32_t standardize, double *loss, void *stream);
pars3_status pars3_mlp_adam(pars3_mlp *m, float lr, float beta1, float beta2, float eps, void *stream);
pars3_status pars3_mlp_train(pars3_mlp *m, const float *X, const float *T, const float *M, int32_t rows,
                             int32_t batch, int32_t epochs, float lr, uint64_t seed, double *loss_hist, void *stream);
pars3_status pars3_mlp_select_rows(pars3_mlp *m, const float *X, int32_t rows, const float *valid, int32_t *choice,
                                   void *stream);
pars3_status pars3_select(pars3_matrix *A, pars3_mlp *m, const pars3_split_params *grid, int32_t ngrid,
                          int32_t *choice, void *stream);

/* The configurations the network's outputs stand for (output g predicts
 * grid[g]), kept with the network for pars3_select with grid = NULL, for
 * pars3_model_save and for pars3_reorder(A, NULL) (Section 3.1.2: the split is
 * a choice made from the reordered matrix).  set: ngrid must equal n_out
 * (EINVAL).  get: *count receives the size; grid (may be NULL) receives up to
 * cap entries (EINVAL when cap < size).  Host arrays. */
pars3_status pars3_mlp_set_grid(pars3_mlp *m, const pars3_split_params *grid, int32_t ngrid);
pars3_status pars3_mlp_get_grid(const pars3_mlp *m, pars3_split_params *grid, int32_t cap, int32_t *count);

/* Trained selector on disk (a binary file, little-endian): the magic
 * "PARS3MLP", format version 2 (uint32), int32 n_in, h1, h2, n_out, ngrid,
 * ngrid x 7 int32 split parameters in pars3_split_params field order
 * (version 1 files, which hold the first 6 and no engine, load with engine
 * PARS3_ENGINE_TILES), the
 * scaler (n_in float means, n_in float standard deviations), the packed
 * weights (float, as pars3_mlp_get_params) and a 64-bit FNV-1a hash of every
 * preceding byte.  save: needs a grid (ESTATE otherwise); EIO when the file
 * cannot be written.  load: *out receives a new network (caller owns it;
 * pars3_mlp_destroy) with weights, scaler and grid; Adam state zero; EIO for
 * a missing, truncated or corrupted file, a bad magic, version or size.
 * Synchronous. */
pars3_status pars3_model_save(const pars3_mlp *m, const char *path);
pars3_status pars3_model_load(const char *path, pars3_mlp **out);

/* Sets the network that pars3_reorder(A, NULL, ...) consults, process-wide
 * (NULL: none, the defaults apply).  The caller keeps ownership and keeps the
 * network alive while it is in use; pars3_mlp_destroy of the network in use
 * clears it.  ESTATE when the network has no grid. */
pars3_status pars3_model_use(pars3_mlp *m);

/* Message of the last failing call on this thread ("" if none). */
const char *pars3_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PARS3_H */
