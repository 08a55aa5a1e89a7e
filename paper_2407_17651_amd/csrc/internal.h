// Internal declarations of the pars3 library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <vector>

#include "pars3.h"

namespace p3 {

// ---------------------------------------------------------------- errors
pars3_status fail(pars3_status st, const char *fmt, ...);
void clear_error();

#define P3_HIP(call)                                                                                      \
  do {                                                                                                    \
    hipError_t e_ = (call);                                                                               \
    if (e_ != hipSuccess) {                                                                               \
      (void)hipGetLastError(); /* do not leave the error pending for later checks */                     \
      return ::p3::fail(e_ == hipErrorOutOfMemory ? PARS3_ENOMEM : PARS3_EHIP, "%s: %s (%s:%d)", #call,   \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                       \
    }                                                                                                     \
  } while (0)

#define P3_TRY(...)                      \
  do {                                   \
    pars3_status s_ = (__VA_ARGS__);     \
    if (s_ != PARS3_OK) return s_;       \
  } while (0)

// Launch check: reports launch-configuration errors immediately.
#define P3_LAUNCHED() P3_HIP(hipGetLastError())

// ---------------------------------------------------------------- device buffers
template <class T>
struct dbuf {
  T *p = nullptr;
  size_t n = 0;
  dbuf() = default;
  dbuf(const dbuf &) = delete;
  dbuf &operator=(const dbuf &) = delete;
  ~dbuf() { release(); }
  // On failure the buffer stays empty (p == nullptr, n == 0), so a size check
  // of a later call never mistakes a failed allocation for a usable one.
  hipError_t alloc(size_t m) {
    release();
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, (m ? m : 1) * sizeof(T));
    if (e != hipSuccess) return e;
    p = (T *)q;
    n = m;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int bits_for(uint64_t v) {  // bits needed to hold values 0..v
  int b = 0;
  while (v) {
    b++;
    v >>= 1;
  }
  return b;
}

// ---------------------------------------------------------------- wave-aggregated atomics
// When every valid lane of the wavefront targets the same address, the lanes
// combine their values with shuffles and one lane issues the atomic;
// otherwise each valid lane issues its own.  All 64 lanes must call these
// (lanes without work pass valid = false), so callers must not return early.
__device__ __forceinline__ int wave_uniform_leader(int64_t idx, bool valid, int64_t *i0) {
  const unsigned long long m = __ballot(valid);
  if (m == 0ull) return -1;
  const int l = __ffsll((long long)m) - 1;
  *i0 = __shfl(idx, l, 64);
  return __all(!valid || idx == *i0) ? l : -2;
}
template <class T>
__device__ __forceinline__ void agg_atomic_add(T *base, int64_t idx, T v, bool valid) {
  int64_t i0 = 0;
  const int l = wave_uniform_leader(idx, valid, &i0);
  if (l == -1) return;
  if (l >= 0) {
    T s = valid ? v : (T)0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((int)(threadIdx.x & 63) == l) atomicAdd(&base[i0], s);
  } else if (valid) {
    atomicAdd(&base[idx], v);
  }
}
template <class T>
__device__ __forceinline__ void agg_atomic_min(T *base, int64_t idx, T v, bool valid, T ident) {
  int64_t i0 = 0;
  const int l = wave_uniform_leader(idx, valid, &i0);
  if (l == -1) return;
  if (l >= 0) {
    T s = valid ? v : ident;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      T o = __shfl_xor(s, off, 64);
      s = o < s ? o : s;
    }
    if ((int)(threadIdx.x & 63) == l) atomicMin(&base[i0], s);
  } else if (valid) {
    atomicMin(&base[idx], v);
  }
}
template <class T>
__device__ __forceinline__ void agg_atomic_max(T *base, int64_t idx, T v, bool valid, T ident) {
  int64_t i0 = 0;
  const int l = wave_uniform_leader(idx, valid, &i0);
  if (l == -1) return;
  if (l >= 0) {
    T s = valid ? v : ident;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      T o = __shfl_xor(s, off, 64);
      s = o > s ? o : s;
    }
    if ((int)(threadIdx.x & 63) == l) atomicMax(&base[i0], s);
  } else if (valid) {
    atomicMax(&base[idx], v);
  }
}

// ---------------------------------------------------------------- primitives (util.hip)
// Exclusive prefix sum of in[0..m) into out[0..m]; out[m] = total.  in and
// out must not overlap.  Asynchronous on `s`.
pars3_status scan_i32(const int32_t *in, int32_t *out, int64_t m, hipStream_t s);
pars3_status scan_i64(const int64_t *in, int64_t *out, int64_t m, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on the low `key_bits` bits of
// the keys.  Sorted pairs end in (k0, v0); k1/v1 are scratch of the same size.
pars3_status radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t m, int key_bits,
                              hipStream_t s);
// Integer fill helpers.
pars3_status fill_i32(int32_t *p, int32_t v, int64_t m, hipStream_t s);
pars3_status fill_u64(uint64_t *p, uint64_t v, int64_t m, hipStream_t s);
pars3_status iota_i32(int32_t *p, int64_t m, hipStream_t s);

// ---------------------------------------------------------------- stored layouts
constexpr int CHUNKS_FIXED = 32;          // fixed chunk slots per tile (4 wavefronts x 8)
constexpr uint32_t CHUNK_EMPTY = 0xffffffffu;
constexpr int ENT16_MAX_LGT = 8;          // tiles of at most 256 rows store 16-bit entry words
constexpr size_t ORIG_MAX_ROW_BYTES = 8 * sizeof(double);  // 8 FP64 right-hand sides
// One SpMV layout: the three parts of the split arranged for the kernel.
struct layout {
  int32_t T = 256, lgT = 8, w_in = 0, t_out = 0;
  int32_t ntiles = 0, nblocks = 0, max_blocks = 0;
  int64_t nnz_blocked = 0;  // middle + outer entries
  int32_t vdtype = PARS3_F64;
  // inner band, diagonal-major: value of (i, i-k) at [(k-1)*n + i]
  dbuf<double> in_f64;
  dbuf<float> in_f32;
  dbuf<uint16_t> in_bf16;
  // tile-pair blocks: entries [blk_start[b], blk_start[b+1]) of block b, whose
  // row tile is blk_t[b] and column tile blk_u[b].  Entry word: the row's and
  // the column's offsets in their tiles, (row offset) << 8 | column offset in
  // 16 bits when T <= 256 (ent_rc16), << 16 in 32 bits otherwise (ent_rc);
  // only one of the two is allocated
  dbuf<uint16_t> ent_rc16;
  dbuf<uint32_t> ent_rc;
  dbuf<double> ent_f64;
  dbuf<float> ent_f32;
  dbuf<uint16_t> ent_bf16;
  dbuf<int32_t> blk_start, blk_t, blk_u;
  // row tile t owns blocks [tblk_ptr[t], tblk_ptr[t+1]); column tile u is the
  // column tile of blocks ublk[ublk_ptr[u] .. ublk_ptr[u+1]) (ascending)
  dbuf<int32_t> tblk_ptr, ublk_ptr, ublk;
  // per tile, its chunks: runs of at most 64 consecutive entries of one
  // block, its own blocks (row side) first, then the blocks of its column
  // list (column side); chunk.x = first entry, chunk.y = other tile << 8 |
  // column side << 7 | (length - 1).  The first CHUNKS_FIXED chunks of tile t
  // sit at chunk_fix[t * CHUNKS_FIXED + 8 w + k] for chunk w + 4 k (the 8
  // chunks of wavefront w side by side; CHUNK_EMPTY in .y past the end), so
  // the product finds them without a pointer load; the rest are
  // chunk_ovf[ovf_ptr[t] .. ovf_ptr[t+1]).
  dbuf<uint2> chunk_fix, chunk_ovf;
  dbuf<int32_t> ovf_ptr;
  int32_t nchunks = 0, nchunks_ovf = 0;
  // layout position of every canonical entry (-1 for inner-band entries)
  dbuf<int32_t> pos_of;
  // LDS bank passes of the blocks' aligned runs of 16 entries (row side +
  // column side), in the sorted (diagonal) order and in the stored order
  int64_t lds_runs = 0, lds_passes_sorted = 0, lds_passes = 0;
};

struct mrs_ws;
void mrs_ws_free(mrs_ws *w);

}  // namespace p3

namespace p3 {
struct skew_shadow;  // skewform.hip
void skew_shadow_free(skew_shadow *sh);
}  // namespace p3

struct pars3_matrix {
  int64_t n = 0, nnz = 0;
  int device = 0;
  // PARS3_SKEW (S = L - L^T) or PARS3_SYMMETRIC (S = L + L^T)
  int32_t kind = PARS3_SKEW;
  // input, original numbering; diag: the SSS diagonal array (empty: D = 0)
  p3::dbuf<int32_t> rowptr, col;
  p3::dbuf<double> val, diag;
  // the diagonal in the reordered numbering, FP64 and rounded to FP32, and
  // its smallest and largest entry (host, from the caller's array)
  p3::dbuf<double> pdiag;
  p3::dbuf<float> pdiag32;
  double dmin = 0.0, dmax = 0.0;
  // scaled skew form for the MRS solver (skewform.hip), created on first use
  p3::skew_shadow *shadow = nullptr;
  // reordering
  bool perm_done = false;
  int32_t perm_kind = -1;  // 1 RCM, 0 identity
  int32_t ncomp = 0, nlevels = 0;
  p3::dbuf<int32_t> perm, iperm;
  // permuted strictly lower CSR, FP64, canonical order
  p3::dbuf<int32_t> prow, pcol;
  p3::dbuf<double> pval;
  p3::dbuf<int8_t> part;
  int32_t beta = 0;
  int64_t cnt[3] = {0, 0, 0};
  bool split_done = false;
  pars3_split_params params{};
  p3::layout lay;
  bool has_f64 = false, has_f32 = false, has_bf16 = false;
  // scratch for products in the caller's numbering: x and y in the reordered
  // numbering, n rows of up to ORIG_MAX_ROW_BYTES each, reserved by
  // pars3_reorder so that pars3_spmv never allocates or synchronises
  p3::dbuf<char> xr, yr;
  // full CSR serving one-right-hand-side products (engine PARS3_ENGINE_CSR)
  pars3_csr *csr = nullptr;
  // solver stream and workspace (mrs.hip), created on first use
  hipStream_t solver_stream = nullptr;
  p3::mrs_ws *mrs = nullptr;
  // per-kernel event timing (pars3_set_profiling)
  struct {
    bool on = false;
    int64_t calls = 0;
    int used[3] = {0, 0, 0};
    std::vector<hipEvent_t> ev[3];  // pairs: [2q] start, [2q+1] stop
  } prof;
  ~pars3_matrix();
};

namespace p3 {
// reorder.hip
pars3_status rcm_gpu(pars3_matrix *A, hipStream_t s);
pars3_status identity_perm_gpu(pars3_matrix *A, hipStream_t s);
pars3_status permute_gpu(pars3_matrix *A, hipStream_t s);
// pdiag[k] = diag[perm[k]] and its FP32 rounding
pars3_status permute_diagonal(pars3_matrix *A, hipStream_t s);
// layout.hip
pars3_status split_and_layout(pars3_matrix *A, const pars3_split_params &p, hipStream_t s);
// spmv.hip
enum { PROF_BAND = 0, PROF_FIXUP = 1, PROF_OTHER = 2 };
// Optional epilogue of the product kernel (used by the solvers):
//   y += (*beta) * z                      when z != nullptr,
//   partials[t] = sum over tile t of y^2  when partials != nullptr (FP64),
//   the whole launch is skipped           when done != nullptr and *done != 0.
template <class X>
struct epilogue {
  const X *z = nullptr;
  const double *beta = nullptr;
  double *partials = nullptr;
  const int32_t *done = nullptr;
  // fused MRS iteration (one right-hand side): y = (*scale) (S x) + (*beta) z,
  // and, while *active, the previous iteration's vector update on the
  // tile's rows: p = (z vec[4] - vec[0] p1 - vec[1] p2) / vec[2] written over
  // p2, xs += vec[3] p
  const double *scale = nullptr;
  const double *vec = nullptr;
  const int32_t *active = nullptr;
  const X *p1 = nullptr;
  X *p2 = nullptr;
  X *xs = nullptr;
};
// Device state of one MRS run.  Rotation state is double-buffered by
// iteration parity: iteration j reads slot j&1 and writes slot (j+1)&1.
struct mrs_dev {
  double beta[2], c1[2], s1[2], c2[2], s2[2], eta[2];
  // this iteration's vector update: p = (v - delta p1 - eps p2) / gamma,
  // x += ceta p, with v = (stored Lanczos vector) * vnrm_inv
  double delta, eps, gamma, ceta, vnrm_inv;
  double inv_beta;          // 1 / beta_{j+1} (normalised vectors)
  double scaleS, zcoef;     // next product with unnormalised vectors: scaleS (S w_j) + zcoef w_{j-1}
  double nrm[2];            // norm of the stored vector that represents v_j (slot j&1)
  double bnorm, tol_abs, alpha, minus_one;
  int32_t iter, maxit, done, active, status;  // status: 0 ok, 1 maxit, 2 breakdown, 3 nan
};

// One step of the rotation recurrence from ||w||^2 (see mrs.hip); run by
// one thread.  Sets the coefficients of this iteration's vector update
// (active = 1) or stops the run (done = 1, status).  The state it reads is
// loaded first (mrs_load), all of it before any store, so that the loads go
// out together instead of one memory round trip after another.
struct mrs_in {
  double beta_j, c1, s1, c2, s2, eta, alpha, nrm, bnorm, tol_abs;
  int32_t iter, maxit;
};
__device__ __forceinline__ mrs_in mrs_load(const mrs_dev *d, int par) {
  mrs_in in;
  in.beta_j = d->beta[par];
  in.c1 = d->c1[par];
  in.s1 = d->s1[par];
  in.c2 = d->c2[par];
  in.s2 = d->s2[par];
  in.eta = d->eta[par];
  in.alpha = d->alpha;
  in.nrm = d->nrm[par];
  in.bnorm = d->bnorm;
  in.tol_abs = d->tol_abs;
  in.iter = d->iter;
  in.maxit = d->maxit;
  return in;
}
__device__ __forceinline__ void mrs_apply(mrs_dev *d, int par, double sumsq, double *hist, const mrs_in &in) {
  const double beta_n = sqrt(sumsq);
  const double eps = in.s2 * (-in.beta_j);
  const double dbar = in.c2 * (-in.beta_j);
  const double delta = in.c1 * dbar + in.s1 * in.alpha;
  const double gbar = -in.s1 * dbar + in.c1 * in.alpha;
  const double gamma = sqrt(gbar * gbar + beta_n * beta_n);
  if (!isfinite(beta_n) || !isfinite(gamma)) {
    d->status = 3;
    d->done = 1;
    d->active = 0;
    return;
  }
  if (gamma == 0.0) {
    d->status = 2;
    d->done = 1;
    d->active = 0;
    return;
  }
  const double c = gbar / gamma, s = beta_n / gamma;
  const double inv_beta = beta_n > 0.0 ? 1.0 / beta_n : 0.0;
  const double vnrm_inv = in.nrm > 0.0 ? 1.0 / in.nrm : 0.0;
  const double eta_n = -s * in.eta;
  const int32_t it = in.iter + 1;
  d->delta = delta;
  d->eps = eps;
  d->gamma = gamma;
  d->ceta = c * in.eta;
  d->inv_beta = inv_beta;
  d->vnrm_inv = vnrm_inv;
  d->scaleS = inv_beta;
  d->zcoef = beta_n * vnrm_inv;
  d->nrm[par ^ 1] = beta_n;
  d->active = 1;
  d->iter = it;
  if (hist) hist[it - 1] = fabs(eta_n) / in.bnorm;
  const int q = par ^ 1;
  d->beta[q] = beta_n;
  d->c1[q] = c;
  d->s1[q] = s;
  d->c2[q] = in.c1;
  d->s2[q] = in.s1;
  d->eta[q] = eta_n;
  if (fabs(eta_n) <= in.tol_abs || beta_n == 0.0) {
    d->done = 1;
  } else if (it >= in.maxit) {
    d->done = 1;
    d->status = 1;
  }
}
__device__ __forceinline__ void mrs_update(mrs_dev *d, int par, double sumsq, double *hist) {
  mrs_apply(d, par, sumsq, hist, mrs_load(d, par));
}

// One product task as the product kernels read it: a matrix layout, its
// value arrays (type given separately), the vectors and the epilogue.
struct prod_task {
  const uint2 *chunk_fix;
  const int32_t *ovf_ptr;
  const uint2 *chunk_ovf;
  const void *ent_rc;  // entry words: uint16_t when lgT <= ENT16_MAX_LGT, uint32_t otherwise
  const void *ent_v, *dia;
  int32_t w_in, ntiles, lgT, n;
  int32_t sym;       // 1: S = L + L^T (the transposed update keeps its sign)
  double shift;
  const void *dg;    // diagonal array in the vector type, or nullptr (D = 0)
  const void *x;
  void *y;
  const void *z;
  const double *beta;
  double *partials;
  const int32_t *done;
  const double *scale;   // fused MRS iteration (see epilogue)
  const double *vec;
  const int32_t *active;
  const void *p1;
  void *p2;
  void *xs;
};
// Fills the layout and value fields of a task for products with vectors of
// vec_dtype (value_dtype picks FP32 or BF16 values when both are stored, -1:
// whichever is stored); *vkind receives the value type used.
pars3_status make_task(const pars3_matrix *A, int vec_dtype, int value_dtype, prod_task *a, int *vkind);
// Product over many tasks, one workgroup per item: items (task, tile) in 8
// queues [qbeg[q], qbeg[q+1]), one per XCD; grid = 8 x the longest queue.
// minT, maxT: the smallest and largest tile heights among the tasks (they
// decide the LDS size and the entry word types).  ep: with the solver
// epilogue (k = 1 only).  gen: some task is symmetric or has a diagonal array.
pars3_status launch_batch(int vkind, int k, bool ep, bool gen, const prod_task *tasks, const int2 *items,
                          const int32_t *qbeg, int32_t grid, int32_t minT, int32_t maxT, hipStream_t s);
// skewform.hip: MRS for alpha*I + D + S through its shifted skew form
pars3_status mrs_shifted(pars3_matrix *A, double alpha, const double *b, double *x, const pars3_mrs_opts &o,
                         pars3_mrs_info *info, hipStream_t s);
// csr.hip: y = shift x + S x on a handle's full CSR (rocSPARSE), and the
// precision of its values
pars3_status csr_product(pars3_csr *C, double shift, const void *x, void *y, hipStream_t s);
int32_t csr_vdtype(const pars3_csr *C);
// A symmetric matrix or one with a diagonal array (the general kernels).
inline bool is_general(const pars3_matrix *A) { return A->kind != PARS3_SKEW || A->diag.p != nullptr; }
// Product with an optional epilogue; value_dtype selects FP32 or BF16 values
// when both are stored (-1: whichever is stored).
pars3_status spmv_ex(pars3_matrix *A, double shift, const void *x, void *y, int k, int vec_dtype, int value_dtype,
                     hipStream_t s, const void *ep);
pars3_status prof_mark(pars3_matrix *A, int cls, int stop, hipStream_t s);
pars3_status spmv_rcm(pars3_matrix *A, double shift, const void *x, void *y, int k, int vec_dtype, hipStream_t s);
pars3_status gather_rows(const void *src, void *dst, const int32_t *idx, int64_t n, int k, size_t elem,
                         hipStream_t s);
// mlp.hip / tune.hip: the configuration grid of a network, the process-wide
// selector that pars3_reorder(A, NULL) consults, and its use
const std::vector<pars3_split_params> &mlp_grid(const pars3_mlp *m);
void forget_selector(const pars3_mlp *m);
bool has_selector();
pars3_status reorder_selected(pars3_matrix *A, void *stream);
pars3_status scatter_rows(const void *src, void *dst, const int32_t *idx, int64_t n, int k, size_t elem,
                          hipStream_t s);
}  // namespace p3
