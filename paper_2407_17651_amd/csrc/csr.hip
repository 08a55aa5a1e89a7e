// Full-CSR comparison path: the whole of S (both triangles, 2*nnz entries) in
// CSR form (the storage that keeps every nonzero, Section 1), multiplied by a
// plain CSR-vector kernel or by rocSPARSE.  It is the baseline the skew
// product is measured against; it reads every matrix value twice as often.
// A diagonal array adds an entry d_i at (i, i) for every nonzero d_i; the
// transposed entries are -l (skew) or +l (symmetric).
#include <algorithm>

#include <rocsparse/rocsparse.h>

#include "internal.h"

struct pars3_csr {
  int64_t n = 0, nnz = 0;
  int32_t order = PARS3_ORDER_RCM, vdtype = PARS3_F64, lanes = 4;
  p3::dbuf<int32_t> rowptr, col;
  p3::dbuf<double> v64;
  p3::dbuf<float> v32;
  rocsparse_handle rh = nullptr;
  rocsparse_spmat_descr mat = nullptr;
  p3::dbuf<char> buf;
  size_t bufsz = 0;
  bool rs_ready = false;
  ~pars3_csr() {
    if (mat) rocsparse_destroy_spmat_descr(mat);
    if (rh) rocsparse_destroy_handle(rh);
  }
};

namespace p3 {

static constexpr int TB = 256;
static inline unsigned nblk(int64_t m) { return (unsigned)std::max<int64_t>(1, cdiv(m, TB)); }

// entries of row i up to and including its diagonal one
__device__ __forceinline__ int32_t lower_len(const int32_t *__restrict__ rp, const double *__restrict__ dg,
                                             int32_t i) {
  return rp[i + 1] - rp[i] + (dg && dg[i] != 0.0 ? 1 : 0);
}
__global__ void k_full_count(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const double *__restrict__ dg, int32_t n, int32_t *__restrict__ cnt) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&cnt[i], lower_len(rp, dg, i));
  for (int32_t e = rp[i]; e < rp[i + 1]; e++) atomicAdd(&cnt[col[e]], 1);
}
// row i: its lower entries in place (ascending), d_i when nonzero, then
// tsign l_ki for every stored (k, i), k > i, in arbitrary order (sorted by
// k_full_sort_upper)
__global__ void k_full_fill(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const double *__restrict__ dg, double tsign, int32_t n,
                            const int32_t *__restrict__ frow, int32_t *__restrict__ ufill, int32_t *__restrict__ fcol,
                            double *__restrict__ fval) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t f = frow[i];
  for (int32_t e = rp[i]; e < rp[i + 1]; e++) {
    const int32_t j = col[e];
    fcol[f] = j;
    fval[f++] = val[e];
    const int32_t slot = atomicAdd(&ufill[j], 1);
    const int32_t at = frow[j] + lower_len(rp, dg, j) + slot;
    fcol[at] = i;
    fval[at] = tsign * val[e];
  }
  if (dg && dg[i] != 0.0) {
    fcol[f] = i;
    fval[f] = dg[i];
  }
}
__device__ __forceinline__ int32_t row_of_csr(const int32_t *__restrict__ ptr, int32_t n, int64_t e) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
// rank sort of the upper part of every row by column (columns are distinct)
__global__ void k_full_sort_upper(const int32_t *__restrict__ rp, const double *__restrict__ dg,
                                  const int32_t *__restrict__ frow, int32_t n, int64_t m,
                                  const int32_t *__restrict__ fcol_in, const double *__restrict__ fval_in,
                                  int32_t *__restrict__ fcol, double *__restrict__ fval) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t r = row_of_csr(frow, n, e);
  const int32_t ub = frow[r] + lower_len(rp, dg, r);
  if (e < ub) {
    fcol[e] = fcol_in[e];
    fval[e] = fval_in[e];
    return;
  }
  const int32_t c = fcol_in[e];
  int32_t rank = 0;
  for (int32_t t = ub; t < frow[r + 1]; t++) rank += fcol_in[t] < c;
  fcol[ub + rank] = c;
  fval[ub + rank] = fval_in[e];
}
__global__ void k_to_f32(const double *__restrict__ a, float *__restrict__ b, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (float)a[i];
}

// y_i = shift x_i + sum_j a_ij x_j; a group of G lanes per row, ascending
// column order inside each lane, shuffle reduction across the group.
template <class V, class X, int G>
__global__ __launch_bounds__(TB) void k_csr_vector(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                   const V *__restrict__ val, int32_t n, X shift,
                                                   const X *__restrict__ x, X *__restrict__ y) {
  const int64_t g = ((int64_t)blockIdx.x * TB + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  const bool ok = g < n;
  X s = (X)0;
  if (ok) {
    const int32_t b = rp[g], e = rp[g + 1];
    for (int32_t q = b + lane; q < e; q += G) s += (X)__builtin_nontemporal_load(val + q) * x[__builtin_nontemporal_load(col + q)];
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, G);
  if (ok && lane == 0) y[g] = shift * x[g] + s;
}

template <class V, class X>
static pars3_status csr_launch(pars3_csr *C, const V *val, X shift, const X *x, X *y, hipStream_t s) {
  const int32_t n = (int32_t)C->n;
  const unsigned grid = (unsigned)cdiv((int64_t)n * C->lanes, TB);
  switch (C->lanes) {
    case 1: k_csr_vector<V, X, 1><<<grid, TB, 0, s>>>(C->rowptr.p, C->col.p, val, n, shift, x, y); break;
    case 2: k_csr_vector<V, X, 2><<<grid, TB, 0, s>>>(C->rowptr.p, C->col.p, val, n, shift, x, y); break;
    case 4: k_csr_vector<V, X, 4><<<grid, TB, 0, s>>>(C->rowptr.p, C->col.p, val, n, shift, x, y); break;
    case 8: k_csr_vector<V, X, 8><<<grid, TB, 0, s>>>(C->rowptr.p, C->col.p, val, n, shift, x, y); break;
    case 16: k_csr_vector<V, X, 16><<<grid, TB, 0, s>>>(C->rowptr.p, C->col.p, val, n, shift, x, y); break;
    case 32: k_csr_vector<V, X, 32><<<grid, TB, 0, s>>>(C->rowptr.p, C->col.p, val, n, shift, x, y); break;
    default: k_csr_vector<V, X, 64><<<grid, TB, 0, s>>>(C->rowptr.p, C->col.p, val, n, shift, x, y); break;
  }
  P3_LAUNCHED();
  return PARS3_OK;
}

#define P3_RS(call)                                                                          \
  do {                                                                                       \
    rocsparse_status r_ = (call);                                                            \
    if (r_ != rocsparse_status_success) return fail(PARS3_EHIP, "%s: rocsparse status %d", #call, (int)r_); \
  } while (0)

}  // namespace p3

using p3::fail;

static pars3_status rocsparse_prepare(pars3_csr *C, const void *x, void *y, hipStream_t s) {
  const bool f64 = C->vdtype == PARS3_F64;
  const rocsparse_datatype dt = f64 ? rocsparse_datatype_f64_r : rocsparse_datatype_f32_r;
  if (!C->rh) P3_RS(rocsparse_create_handle(&C->rh));
  P3_RS(rocsparse_set_stream(C->rh, s));
  if (!C->mat)
    P3_RS(rocsparse_create_csr_descr(&C->mat, C->n, C->n, C->nnz, C->rowptr.p, C->col.p,
                                     f64 ? (void *)C->v64.p : (void *)C->v32.p, rocsparse_indextype_i32,
                                     rocsparse_indextype_i32, rocsparse_index_base_zero, dt));
  rocsparse_dnvec_descr dx = nullptr, dy = nullptr;
  P3_RS(rocsparse_create_dnvec_descr(&dx, C->n, const_cast<void *>(x), dt));
  P3_RS(rocsparse_create_dnvec_descr(&dy, C->n, y, dt));
  const double one64 = 1.0, zero64 = 0.0;
  const float one32 = 1.f, zero32 = 0.f;
  const void *one = f64 ? (const void *)&one64 : (const void *)&one32;
  const void *zero = f64 ? (const void *)&zero64 : (const void *)&zero32;
  rocsparse_status r = rocsparse_spmv(C->rh, rocsparse_operation_none, one, C->mat, dx, zero, dy, dt,
                                      rocsparse_spmv_alg_default, rocsparse_spmv_stage_buffer_size, &C->bufsz, nullptr);
  if (r == rocsparse_status_success) {
    hipError_t e = C->buf.alloc(C->bufsz ? C->bufsz : 1);
    if (e != hipSuccess) r = rocsparse_status_memory_error;
  }
  if (r == rocsparse_status_success)
    r = rocsparse_spmv(C->rh, rocsparse_operation_none, one, C->mat, dx, zero, dy, dt, rocsparse_spmv_alg_default,
                       rocsparse_spmv_stage_preprocess, &C->bufsz, C->buf.p);
  rocsparse_destroy_dnvec_descr(dx);
  rocsparse_destroy_dnvec_descr(dy);
  if (r != rocsparse_status_success) return fail(PARS3_EHIP, "csr_spmv: rocsparse preprocessing failed (%d)", (int)r);
  C->rs_ready = true;
  return PARS3_OK;
}

extern "C" pars3_status pars3_csr_create(const pars3_matrix *A, int32_t order, int32_t value_dtype, pars3_csr **out) {
  if (!A || !out) return fail(PARS3_EINVAL, "csr_create: NULL argument");
  *out = nullptr;
  if (order != PARS3_ORDER_RCM && order != PARS3_ORDER_ORIGINAL) return fail(PARS3_EINVAL, "csr_create: bad order");
  if (value_dtype != PARS3_F64 && value_dtype != PARS3_F32)
    return fail(PARS3_EINVAL, "csr_create: value_dtype must be PARS3_F64 or PARS3_F32");
  if (order == PARS3_ORDER_RCM && !A->perm_done) return fail(PARS3_ESTATE, "csr_create: call pars3_reorder first");
  pars3_csr *C = new (std::nothrow) pars3_csr();
  if (!C) return fail(PARS3_ENOMEM, "csr_create: host allocation failed");
  auto run = [&]() -> pars3_status {
    const int32_t n = (int32_t)A->n;
    C->n = n;
    C->order = order;
    C->vdtype = value_dtype;
    const int32_t *rp = order == PARS3_ORDER_RCM ? A->prow.p : A->rowptr.p;
    const int32_t *cl = order == PARS3_ORDER_RCM ? A->pcol.p : A->col.p;
    const double *vl = order == PARS3_ORDER_RCM ? A->pval.p : A->val.p;
    const double *dg = order == PARS3_ORDER_RCM ? A->pdiag.p : A->diag.p;
    const double tsign = A->kind == PARS3_SYMMETRIC ? 1.0 : -1.0;
    hipStream_t s = nullptr;
    p3::dbuf<int32_t> cnt, ufill, fcol0;
    p3::dbuf<double> fval0;
    P3_HIP(C->rowptr.alloc(n + 1));
    P3_HIP(cnt.alloc(n));
    P3_HIP(ufill.alloc(n));
    if (n > 0) {
      P3_HIP(hipMemsetAsync(cnt.p, 0, n * sizeof(int32_t), s));
      P3_HIP(hipMemsetAsync(ufill.p, 0, n * sizeof(int32_t), s));
      p3::k_full_count<<<p3::nblk(n), p3::TB, 0, s>>>(rp, cl, dg, n, cnt.p);
      P3_LAUNCHED();
    }
    P3_TRY(p3::scan_i32(cnt.p, C->rowptr.p, n, s));
    int32_t total = 0;
    P3_HIP(hipMemcpyAsync(&total, C->rowptr.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
    const int64_t m = total;
    C->nnz = m;
    P3_HIP(C->col.alloc(m));
    P3_HIP(C->v64.alloc(m));
    P3_HIP(fcol0.alloc(m));
    P3_HIP(fval0.alloc(m));
    if (m > 0) {
      p3::k_full_fill<<<p3::nblk(n), p3::TB, 0, s>>>(rp, cl, vl, dg, tsign, n, C->rowptr.p, ufill.p, fcol0.p,
                                                      fval0.p);
      P3_LAUNCHED();
      p3::k_full_sort_upper<<<p3::nblk(m), p3::TB, 0, s>>>(rp, dg, C->rowptr.p, n, m, fcol0.p, fval0.p, C->col.p,
                                                            C->v64.p);
      P3_LAUNCHED();
    }
    if (value_dtype == PARS3_F32) {
      P3_HIP(C->v32.alloc(m));
      if (m > 0) {
        p3::k_to_f32<<<p3::nblk(m), p3::TB, 0, s>>>(C->v64.p, C->v32.p, m);
        P3_LAUNCHED();
      }
    }
    P3_HIP(hipStreamSynchronize(s));
    // lanes per row: the power of two nearest the mean row length (1..64)
    const double mean = n > 0 ? (double)m / (double)n : 1.0;
    int lanes = 1;
    while (lanes < 64 && lanes * 1.5 < mean) lanes *= 2;
    C->lanes = lanes;
    // rocSPARSE's analysis of the matrix (handle, buffer, preprocessing) is
    // done here, once, so that a product never runs setup work; its vector
    // descriptors point at scratch vectors that are freed afterwards (the
    // analysis depends on the matrix only)
    if (n > 0) {
      p3::dbuf<double> tx, ty;
      P3_HIP(tx.alloc(n));
      P3_HIP(ty.alloc(n));
      P3_TRY(rocsparse_prepare(C, tx.p, ty.p, s));
      P3_HIP(hipStreamSynchronize(s));
    }
    return PARS3_OK;
  };
  pars3_status st = run();
  if (st != PARS3_OK) {
    delete C;
    return st;
  }
  *out = C;
  return PARS3_OK;
}

extern "C" void pars3_csr_destroy(pars3_csr *C) { delete C; }

extern "C" pars3_status pars3_csr_spmv(pars3_csr *C, double shift, const void *x, void *y, int32_t engine,
                                       void *stream) {
  if (!C) return fail(PARS3_EINVAL, "csr_spmv: NULL handle");
  if (engine != 0 && engine != 1) return fail(PARS3_EINVAL, "csr_spmv: engine must be 0 (own) or 1 (rocSPARSE)");
  if (C->n == 0) return PARS3_OK;
  if (!x || !y || x == y) return fail(PARS3_EINVAL, "csr_spmv: bad vectors");
  hipStream_t s = (hipStream_t)stream;
  const bool f64 = C->vdtype == PARS3_F64;
  if (engine == 0) {
    if (f64) return p3::csr_launch<double, double>(C, C->v64.p, shift, (const double *)x, (double *)y, s);
    return p3::csr_launch<float, float>(C, C->v32.p, (float)shift, (const float *)x, (float *)y, s);
  }
  if (shift != 0.0) return fail(PARS3_EINVAL, "csr_spmv: the rocSPARSE engine computes S*x only (shift must be 0)");
  if (!C->rs_ready) return fail(PARS3_ESTATE, "csr_spmv: rocSPARSE was not prepared");
  P3_RS(rocsparse_set_stream(C->rh, s));
  const rocsparse_datatype dt = f64 ? rocsparse_datatype_f64_r : rocsparse_datatype_f32_r;
  rocsparse_dnvec_descr dx = nullptr, dy = nullptr;
  P3_RS(rocsparse_create_dnvec_descr(&dx, C->n, const_cast<void *>(x), dt));
  P3_RS(rocsparse_create_dnvec_descr(&dy, C->n, y, dt));
  const double one64 = 1.0, zero64 = 0.0;
  const float one32 = 1.f, zero32 = 0.f;
  rocsparse_status r = rocsparse_spmv(C->rh, rocsparse_operation_none, f64 ? (const void *)&one64 : (const void *)&one32,
                                      C->mat, dx, f64 ? (const void *)&zero64 : (const void *)&zero32, dy, dt,
                                      rocsparse_spmv_alg_default, rocsparse_spmv_stage_compute, &C->bufsz, C->buf.p);
  rocsparse_destroy_dnvec_descr(dx);
  rocsparse_destroy_dnvec_descr(dy);
  if (r != rocsparse_status_success) return fail(PARS3_EHIP, "csr_spmv: rocsparse_spmv failed (%d)", (int)r);
  return PARS3_OK;
}

namespace p3 {
template <class X>
__global__ void k_scale_copy(const X *__restrict__ x, X *__restrict__ y, X a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// y = shift x + S x with rocSPARSE (the engine of a handle reordered with
// PARS3_ENGINE_CSR): y = shift x first, then y = S x + y (beta = 1); with
// shift = 0 the product alone (beta = 0).
pars3_status csr_product(pars3_csr *C, double shift, const void *x, void *y, hipStream_t s) {
  if (C->n == 0) return PARS3_OK;
  if (!C->rs_ready) return fail(PARS3_ESTATE, "spmv: the full CSR was not prepared");
  const bool f64 = C->vdtype == PARS3_F64;
  if (shift != 0.0) {
    if (f64) k_scale_copy<double><<<nblk(C->n), TB, 0, s>>>((const double *)x, (double *)y, shift, C->n);
    else k_scale_copy<float><<<nblk(C->n), TB, 0, s>>>((const float *)x, (float *)y, (float)shift, C->n);
    P3_LAUNCHED();
  }
  P3_RS(rocsparse_set_stream(C->rh, s));
  const rocsparse_datatype dt = f64 ? rocsparse_datatype_f64_r : rocsparse_datatype_f32_r;
  rocsparse_dnvec_descr dx = nullptr, dy = nullptr;
  P3_RS(rocsparse_create_dnvec_descr(&dx, C->n, const_cast<void *>(x), dt));
  const rocsparse_status ry = rocsparse_create_dnvec_descr(&dy, C->n, y, dt);
  if (ry != rocsparse_status_success) {
    rocsparse_destroy_dnvec_descr(dx);
    return fail(PARS3_EHIP, "spmv: rocsparse_create_dnvec_descr failed (%d)", (int)ry);
  }
  const double one64 = 1.0, b64 = shift != 0.0 ? 1.0 : 0.0;
  const float one32 = 1.f, b32 = shift != 0.0 ? 1.f : 0.f;
  const rocsparse_status r =
      rocsparse_spmv(C->rh, rocsparse_operation_none, f64 ? (const void *)&one64 : (const void *)&one32, C->mat, dx,
                     f64 ? (const void *)&b64 : (const void *)&b32, dy, dt, rocsparse_spmv_alg_default,
                     rocsparse_spmv_stage_compute, &C->bufsz, C->buf.p);
  rocsparse_destroy_dnvec_descr(dx);
  rocsparse_destroy_dnvec_descr(dy);
  if (r != rocsparse_status_success) return fail(PARS3_EHIP, "spmv: rocsparse_spmv failed (%d)", (int)r);
  return PARS3_OK;
}
int32_t csr_vdtype(const pars3_csr *C) { return C->vdtype; }
}  // namespace p3

extern "C" pars3_status pars3_csr_size(const pars3_csr *C, int64_t *n, int64_t *nnz_full) {
  if (!C) return fail(PARS3_EINVAL, "csr_size: NULL handle");
  if (n) *n = C->n;
  if (nnz_full) *nnz_full = C->nnz;
  return PARS3_OK;
}

extern "C" pars3_status pars3_csr_get(const pars3_csr *C, int32_t *rowptr, int32_t *col, double *val) {
  if (!C) return fail(PARS3_EINVAL, "csr_get: NULL handle");
  if (rowptr) P3_HIP(hipMemcpy(rowptr, C->rowptr.p, (C->n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (C->nnz) {
    if (col) P3_HIP(hipMemcpy(col, C->col.p, C->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (val) P3_HIP(hipMemcpy(val, C->v64.p, C->nnz * sizeof(double), hipMemcpyDeviceToHost));
  }
  return PARS3_OK;
}
