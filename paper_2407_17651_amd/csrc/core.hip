// C ABI entry points: validation, handle life cycle, reorder, product,
// inspection.  Argument checks run on the host before any device work.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"

using p3::fail;

extern "C" void pars3_split_params_default(pars3_split_params *p) {
  if (!p) return;
  p->w_in = -1;
  p->t_out = -1;
  p->tile_rows = 256;
  p->value_dtype = PARS3_F64;
  p->keep_fp64 = 0;
  p->permute = 1;
  p->engine = PARS3_ENGINE_TILES;
}

extern "C" pars3_status pars3_validate(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col) {
  p3::clear_error();
  if (n < 0 || nnz < 0 || n > INT32_MAX || nnz > INT32_MAX) return fail(PARS3_EINVAL, "validate: bad n or nnz");
  if (!rowptr) return fail(PARS3_EINVAL, "validate: rowptr is NULL");
  if (nnz > 0 && !col) return fail(PARS3_EINVAL, "validate: col is NULL");
  if (rowptr[0] != 0) return fail(PARS3_EINVAL, "validate: rowptr[0] = %d", rowptr[0]);
  if ((int64_t)rowptr[n] != nnz) return fail(PARS3_EINVAL, "validate: rowptr[n] = %d, nnz = %lld", rowptr[n], (long long)nnz);
  for (int64_t i = 0; i < n; i++)
    if (rowptr[i + 1] < rowptr[i]) return fail(PARS3_EINVAL, "validate: rowptr decreases at row %lld", (long long)i);
  for (int64_t i = 0; i < n; i++) {
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      if (col[e] < 0 || col[e] >= i)
        return fail(PARS3_ENOTLOWER, "validate: entry (%lld, %d) is not strictly lower", (long long)i, col[e]);
      if (e > rowptr[i] && col[e] <= col[e - 1])
        return fail(PARS3_EUNSORTED, "validate: row %lld has unsorted or duplicate columns", (long long)i);
    }
  }
  return PARS3_OK;
}

extern "C" pars3_status pars3_create(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                                     const double *val, pars3_matrix **out) {
  return pars3_create_sss(n, nnz, rowptr, col, val, nullptr, PARS3_SKEW, out);
}

extern "C" pars3_status pars3_create_sss(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                                         const double *val, const double *diag, int32_t kind, pars3_matrix **out) {
  if (!out) return fail(PARS3_EINVAL, "create: out is NULL");
  *out = nullptr;
  if (kind != PARS3_SKEW && kind != PARS3_SYMMETRIC) return fail(PARS3_EINVAL, "create: bad kind %d", kind);
  pars3_status st = pars3_validate(n, nnz, rowptr, col);
  if (st != PARS3_OK) return st;
  if (nnz > 0 && !val) return fail(PARS3_EINVAL, "create: val is NULL");
  pars3_matrix *A = new (std::nothrow) pars3_matrix();
  if (!A) return fail(PARS3_ENOMEM, "create: host allocation failed");
  auto bail = [&](pars3_status s) {
    delete A;
    return s;
  };
  A->n = n;
  A->nnz = nnz;
  hipError_t e = hipGetDevice(&A->device);
  if (e != hipSuccess) return bail(fail(PARS3_EHIP, "create: hipGetDevice: %s", hipGetErrorString(e)));
  if ((e = A->rowptr.alloc(n + 1)) != hipSuccess || (e = A->col.alloc(nnz)) != hipSuccess ||
      (e = A->val.alloc(nnz)) != hipSuccess)
    return bail(fail(PARS3_ENOMEM, "create: device allocation failed: %s", hipGetErrorString(e)));
  if ((e = hipMemcpy(A->rowptr.p, rowptr, (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (nnz > 0 && (e = hipMemcpy(A->col.p, col, nnz * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) ||
      (nnz > 0 && (e = hipMemcpy(A->val.p, val, nnz * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess))
    return bail(fail(PARS3_EHIP, "create: copy to device failed: %s", hipGetErrorString(e)));
  A->kind = kind;
  if (diag) {
    if ((e = A->diag.alloc(n)) != hipSuccess)
      return bail(fail(PARS3_ENOMEM, "create: device allocation failed: %s", hipGetErrorString(e)));
    if (n > 0 && (e = hipMemcpy(A->diag.p, diag, n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
      return bail(fail(PARS3_EHIP, "create: copy to device failed: %s", hipGetErrorString(e)));
    if (n > 0) {
      A->dmin = A->dmax = diag[0];
      for (int64_t i = 1; i < n; i++) {
        A->dmin = std::min(A->dmin, diag[i]);
        A->dmax = std::max(A->dmax, diag[i]);
      }
    }
  }
  *out = A;
  return PARS3_OK;
}

extern "C" pars3_status pars3_get_kind(const pars3_matrix *A, int32_t *kind, int32_t *has_diag) {
  if (!A) return fail(PARS3_EINVAL, "get_kind: NULL handle");
  if (kind) *kind = A->kind;
  if (has_diag) *has_diag = A->diag.p ? 1 : 0;
  return PARS3_OK;
}

extern "C" pars3_status pars3_get_diagonal(const pars3_matrix *A, double *out) {
  if (!A || !out) return fail(PARS3_EINVAL, "get_diagonal: NULL argument");
  if (!A->perm_done) return fail(PARS3_ESTATE, "get_diagonal: call pars3_reorder first");
  if (!A->diag.p) return fail(PARS3_ESTATE, "get_diagonal: the handle has no diagonal array");
  if (A->n) P3_HIP(hipMemcpy(out, A->pdiag.p, A->n * sizeof(double), hipMemcpyDeviceToHost));
  return PARS3_OK;
}

pars3_matrix::~pars3_matrix() {
  pars3_csr_destroy(csr);
  p3::skew_shadow_free(shadow);
  p3::mrs_ws_free(mrs);
  if (solver_stream) (void)hipStreamDestroy(solver_stream);
  for (auto &v : prof.ev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
}

extern "C" void pars3_destroy(pars3_matrix *A) { delete A; }

extern "C" pars3_status pars3_set_profiling(pars3_matrix *A, int32_t enable) {
  if (!A) return fail(PARS3_EINVAL, "set_profiling: NULL handle");
  A->prof.on = enable != 0;
  A->prof.calls = 0;
  for (int c = 0; c < 3; c++) A->prof.used[c] = 0;
  return PARS3_OK;
}

extern "C" pars3_status pars3_get_profile(pars3_matrix *A, pars3_profile *out) {
  if (!A || !out) return fail(PARS3_EINVAL, "get_profile: NULL argument");
  auto &P = A->prof;
  double ms[3] = {0, 0, 0};
  for (int c = 0; c < 3; c++) {
    for (int q = 0; q < P.used[c]; q++) {
      P3_HIP(hipEventSynchronize(P.ev[c][2 * q + 1]));
      float t = 0.f;
      P3_HIP(hipEventElapsedTime(&t, P.ev[c][2 * q], P.ev[c][2 * q + 1]));
      ms[c] += t;
    }
    P.used[c] = 0;
  }
  out->calls = P.calls;
  out->ms_band = ms[0];
  out->ms_fixup = ms[1];
  out->ms_other = ms[2];
  P.calls = 0;
  return PARS3_OK;
}

static pars3_status check_params(const pars3_split_params &p) {
  if (p.w_in < -1 || p.t_out < -1) return fail(PARS3_EINVAL, "reorder: w_in and t_out must be >= -1");
  if (p.permute != 0 && p.permute != 1) return fail(PARS3_EINVAL, "reorder: permute must be 0 or 1");
  if (p.keep_fp64 != 0 && p.keep_fp64 != 1) return fail(PARS3_EINVAL, "reorder: keep_fp64 must be 0 or 1");
  if (p.engine != PARS3_ENGINE_TILES && p.engine != PARS3_ENGINE_CSR)
    return fail(PARS3_EINVAL, "reorder: engine must be PARS3_ENGINE_TILES or PARS3_ENGINE_CSR");
  if (p.engine == PARS3_ENGINE_CSR && p.value_dtype == PARS3_BF16)
    return fail(PARS3_EINVAL, "reorder: the full-CSR engine takes FP64 or FP32 values");
  return PARS3_OK;
}

extern "C" pars3_status pars3_reorder(pars3_matrix *A, const pars3_split_params *pp, void *stream) {
  p3::clear_error();
  if (!A) return fail(PARS3_EINVAL, "reorder: NULL handle");
  // no parameters: the selector's configuration when a network is in use
  // (pars3_model_use), else the defaults
  if (!pp && p3::has_selector()) return p3::reorder_selected(A, stream);
  pars3_split_params p;
  if (pp) p = *pp;
  else pars3_split_params_default(&p);
  P3_TRY(check_params(p));
  hipStream_t s = (hipStream_t)stream;
  P3_HIP(hipSetDevice(A->device));
  if (!A->perm_done || A->perm_kind != p.permute) {
    A->perm_done = false;
    A->split_done = false;
    if (p.permute) P3_TRY(p3::rcm_gpu(A, s));
    else P3_TRY(p3::identity_perm_gpu(A, s));
    P3_TRY(p3::permute_gpu(A, s));
    if (A->diag.p) P3_TRY(p3::permute_diagonal(A, s));
    A->perm_done = true;
    A->perm_kind = p.permute;
  }
  A->split_done = false;
  p3::skew_shadow_free(A->shadow);  // built for the previous split
  A->shadow = nullptr;
  pars3_csr_destroy(A->csr);  // built for the previous split
  A->csr = nullptr;
  P3_TRY(p3::split_and_layout(A, p, s));
  // scratch of products in the caller's numbering (up to 8 FP64 right-hand
  // sides), reserved here so that pars3_spmv never allocates
  const size_t rbytes = (size_t)A->n * p3::ORIG_MAX_ROW_BYTES;
  if (A->xr.n < rbytes || A->yr.n < rbytes) {
    P3_HIP(hipStreamSynchronize(s));
    P3_HIP(A->xr.alloc(rbytes));
    P3_HIP(A->yr.alloc(rbytes));
  }
  P3_HIP(hipStreamSynchronize(s));
  A->split_done = true;
  if (p.engine == PARS3_ENGINE_CSR && A->n > 0) {
    // the full CSR of the reordered matrix serves the one-right-hand-side
    // products; the split stays for everything else
    pars3_csr *C = nullptr;
    const pars3_status st = pars3_csr_create(A, PARS3_ORDER_RCM, A->lay.vdtype, &C);
    if (st != PARS3_OK) {
      A->split_done = false;
      return st;
    }
    A->csr = C;
  }
  return PARS3_OK;
}

static bool overlap(const void *a, const void *b, size_t bytes) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + bytes && y < x + bytes;
}

extern "C" pars3_status pars3_spmv(pars3_matrix *A, double shift, const void *x, void *y, int32_t k, int32_t vec_dtype,
                                   int32_t order, void *stream) {
  if (!A) return fail(PARS3_EINVAL, "spmv: NULL handle");
  if (!A->split_done) return fail(PARS3_ESTATE, "spmv: call pars3_reorder first");
  if (k != 1 && k != 2 && k != 4 && k != 8) return fail(PARS3_EINVAL, "spmv: k must be 1, 2, 4 or 8");
  if (vec_dtype != PARS3_F64 && vec_dtype != PARS3_F32) return fail(PARS3_EINVAL, "spmv: bad vec_dtype");
  if (order != PARS3_ORDER_RCM && order != PARS3_ORDER_ORIGINAL) return fail(PARS3_EINVAL, "spmv: bad order");
  if (k > 1 && (((uintptr_t)x | (uintptr_t)y) & 15u))
    return fail(PARS3_EINVAL, "spmv: x and y must be 16-byte aligned when k > 1");
  if (A->n == 0) return PARS3_OK;
  if (!x || !y) return fail(PARS3_EINVAL, "spmv: NULL vector");
  const size_t elem = vec_dtype == PARS3_F64 ? 8 : 4;
  const size_t bytes = (size_t)A->n * k * elem;
  if (overlap(x, y, bytes)) return fail(PARS3_EINVAL, "spmv: x and y overlap");
  hipStream_t s = (hipStream_t)stream;
  if (order == PARS3_ORDER_RCM) return p3::spmv_rcm(A, shift, x, y, k, vec_dtype, s);
  // the scratch was reserved by pars3_reorder (no allocation or wait here)
  if (A->xr.n < bytes || A->yr.n < bytes) return fail(PARS3_ESTATE, "spmv: no scratch for the caller's numbering");
  P3_TRY(p3::prof_mark(A, p3::PROF_FIXUP, 0, s));
  P3_TRY(p3::gather_rows(x, A->xr.p, A->perm.p, A->n, k, elem, s));
  P3_TRY(p3::prof_mark(A, p3::PROF_FIXUP, 1, s));
  P3_TRY(p3::spmv_rcm(A, shift, A->xr.p, A->yr.p, k, vec_dtype, s));
  P3_TRY(p3::prof_mark(A, p3::PROF_FIXUP, 0, s));
  P3_TRY(p3::scatter_rows(A->yr.p, y, A->perm.p, A->n, k, elem, s));
  P3_TRY(p3::prof_mark(A, p3::PROF_FIXUP, 1, s));
  return PARS3_OK;
}

// ------------------------------------------------------------ allocation-free caller-order product
// Scratch of pars3_spmv_noalloc: x and y in the reordered numbering, one half
// each, in a file-scope device array (every GPU the library runs on holds its
// own copy until the process ends).  Host code never passes the array's name
// to a kernel or a copy (on the host it only stands in for the symbol): the
// device address of each GPU's copy is looked up once per device, with that
// device current, and kept in noalloc_ptr.
static constexpr size_t NOALLOC_BYTES = (size_t)PARS3_NOALLOC_SCRATCH_BYTES;
static constexpr size_t NOALLOC_HALF = NOALLOC_BYTES / 2;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];
static constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex noalloc_mu;
static char *noalloc_ptr[NOALLOC_MAX_DEVICES];

static pars3_status noalloc_scratch(int dev, char **out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(PARS3_EINVAL, "spmv_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> g(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    int cur = 0;
    P3_HIP(hipGetDevice(&cur));
    if (cur != dev) P3_HIP(hipSetDevice(dev));
    void *q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !q) {
      (void)hipGetLastError();
      return fail(PARS3_EHIP, "spmv_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    }
    noalloc_ptr[dev] = (char *)q;
  }
  *out = noalloc_ptr[dev];
  return PARS3_OK;
}

extern "C" pars3_status pars3_spmv_noalloc(pars3_matrix *A, double shift, const void *x, void *y, int32_t k,
                                           int32_t vec_dtype, void *stream) {
  if (!A) return fail(PARS3_EINVAL, "spmv_noalloc: NULL handle");
  if (!A->split_done) return fail(PARS3_ESTATE, "spmv_noalloc: call pars3_reorder first");
  if (k != 1 && k != 2 && k != 4 && k != 8) return fail(PARS3_EINVAL, "spmv_noalloc: k must be 1, 2, 4 or 8");
  if (vec_dtype != PARS3_F64 && vec_dtype != PARS3_F32) return fail(PARS3_EINVAL, "spmv_noalloc: bad vec_dtype");
  if (k > 1 && (((uintptr_t)x | (uintptr_t)y) & 15u))
    return fail(PARS3_EINVAL, "spmv_noalloc: x and y must be 16-byte aligned when k > 1");
  // per-kernel timing records events, which may allocate
  if (A->prof.on) return fail(PARS3_ESTATE, "spmv_noalloc: switch profiling off (pars3_set_profiling)");
  const size_t elem = vec_dtype == PARS3_F64 ? 8 : 4;
  const size_t bytes = (size_t)A->n * k * elem;
  if (bytes > NOALLOC_HALF)
    return fail(PARS3_EINVAL, "spmv_noalloc: n x k x %zu = %zu bytes per vector exceeds the %zu-byte limit", elem,
                bytes, NOALLOC_HALF);
  if (A->n == 0) return PARS3_OK;
  if (!x || !y) return fail(PARS3_EINVAL, "spmv_noalloc: NULL vector");
  if (overlap(x, y, bytes)) return fail(PARS3_EINVAL, "spmv_noalloc: x and y overlap");
  char *base = nullptr;
  P3_TRY(noalloc_scratch(A->device, &base));
  // every byte of both halves that the product reads is written first in
  // this call (the gather fills x, the product every row of y), so nothing
  // of an earlier call's contents needs clearing
  hipStream_t s = (hipStream_t)stream;
  P3_TRY(p3::gather_rows(x, base, A->perm.p, A->n, k, elem, s));
  // always the split's kernel (the full-CSR engine's library calls may allocate)
  P3_TRY(p3::spmv_ex(A, shift, base, base + NOALLOC_HALF, k, vec_dtype, -1, s, nullptr));
  P3_TRY(p3::scatter_rows(base + NOALLOC_HALF, y, A->perm.p, A->n, k, elem, s));
  return PARS3_OK;
}

// ------------------------------------------------------------ inspection
extern "C" pars3_status pars3_get_perm(const pars3_matrix *A, int32_t *perm) {
  if (!A || !perm) return fail(PARS3_EINVAL, "get_perm: NULL argument");
  if (!A->perm_done) return fail(PARS3_ESTATE, "get_perm: call pars3_reorder first");
  if (A->n) P3_HIP(hipMemcpy(perm, A->perm.p, A->n * sizeof(int32_t), hipMemcpyDeviceToHost));
  return PARS3_OK;
}

extern "C" pars3_status pars3_get_permuted_lower(const pars3_matrix *A, int32_t *rowptr, int32_t *col, double *val,
                                                 int8_t *part) {
  if (!A) return fail(PARS3_EINVAL, "get_permuted_lower: NULL handle");
  if (!A->split_done) return fail(PARS3_ESTATE, "get_permuted_lower: call pars3_reorder first");
  if (rowptr) P3_HIP(hipMemcpy(rowptr, A->prow.p, (A->n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (A->nnz) {
    if (col) P3_HIP(hipMemcpy(col, A->pcol.p, A->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (val) P3_HIP(hipMemcpy(val, A->pval.p, A->nnz * sizeof(double), hipMemcpyDeviceToHost));
    if (part) P3_HIP(hipMemcpy(part, A->part.p, A->nnz * sizeof(int8_t), hipMemcpyDeviceToHost));
  }
  return PARS3_OK;
}

extern "C" pars3_status pars3_get_split_info(const pars3_matrix *A, pars3_split_info *info) {
  if (!A || !info) return fail(PARS3_EINVAL, "get_split_info: NULL argument");
  if (!A->split_done) return fail(PARS3_ESTATE, "get_split_info: call pars3_reorder first");
  const p3::layout &L = A->lay;
  std::memset(info, 0, sizeof(*info));
  info->n = A->n;
  info->nnz = A->nnz;
  info->beta = A->beta;
  info->w_in = L.w_in;
  info->t_out = L.t_out;
  info->tile_rows = L.T;
  info->value_dtype = L.vdtype;
  info->permute = A->perm_kind;
  info->engine = A->csr ? PARS3_ENGINE_CSR : PARS3_ENGINE_TILES;
  info->nnz_inner = A->cnt[0];
  info->nnz_middle = A->cnt[1];
  info->nnz_outer = A->cnt[2];
  info->n_tiles = L.ntiles;
  info->n_blocks = L.nblocks;
  info->max_blocks = L.max_blocks;
  info->n_components = A->ncomp;
  info->bfs_levels = A->nlevels;
  info->lds_runs = L.lds_runs;
  info->lds_passes_sorted = L.lds_passes_sorted;
  info->lds_passes = L.lds_passes;
  return PARS3_OK;
}

// The stored values of one precision, gathered back into canonical CSR order.
namespace p3 {
template <class V>
__global__ void k_collect(const int32_t *__restrict__ prow, const int32_t *__restrict__ pcol,
                          const int32_t *__restrict__ pos_of, int32_t n, const V *__restrict__ ent_v,
                          const V *__restrict__ in_v, V *__restrict__ out) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = prow[i]; e < prow[i + 1]; e++) {
    const int32_t q = pos_of[e];
    out[e] = q >= 0 ? ent_v[q] : in_v[(int64_t)(i - pcol[e] - 1) * n + i];
  }
}
}  // namespace p3

extern "C" pars3_status pars3_get_values(const pars3_matrix *A, int32_t dtype, void *host) {
  if (!A || !host) return fail(PARS3_EINVAL, "get_values: NULL argument");
  if (!A->split_done) return fail(PARS3_ESTATE, "get_values: call pars3_reorder first");
  const p3::layout &L = A->lay;
  const int32_t n = (int32_t)A->n;
  if (A->nnz == 0) return PARS3_OK;
  size_t elem = dtype == PARS3_F64 ? 8 : dtype == PARS3_F32 ? 4 : 2;
  p3::dbuf<char> out;
  P3_HIP(out.alloc(A->nnz * elem));
  unsigned g = (unsigned)p3::cdiv(n, 256);
  if (dtype == PARS3_F64 && A->has_f64)
    p3::k_collect<double><<<g, 256>>>(A->prow.p, A->pcol.p, L.pos_of.p, n, L.ent_f64.p, L.in_f64.p, (double *)out.p);
  else if (dtype == PARS3_F32 && A->has_f32)
    p3::k_collect<float><<<g, 256>>>(A->prow.p, A->pcol.p, L.pos_of.p, n, L.ent_f32.p, L.in_f32.p, (float *)out.p);
  else if (dtype == PARS3_BF16 && A->has_bf16)
    p3::k_collect<uint16_t><<<g, 256>>>(A->prow.p, A->pcol.p, L.pos_of.p, n, L.ent_bf16.p, L.in_bf16.p,
                                        (uint16_t *)out.p);
  else
    return fail(PARS3_ESTATE, "get_values: precision %d is not stored", dtype);
  P3_LAUNCHED();
  P3_HIP(hipMemcpy(host, out.p, A->nnz * elem, hipMemcpyDeviceToHost));
  return PARS3_OK;
}
