// Shifted skew-symmetric form (Section 1): a system A x = b with
// A = J + S, S skew-symmetric and J = alpha*I + D diagonal and positive
// definite (the paper's "J - S" form with a diagonal J), is brought to the
// form the MRS solver takes by the two-sided scaling
//   J^(-1/2) A J^(-1/2) = I + S~,   S~ = J^(-1/2) S J^(-1/2)  (still skew),
// solved as (I + S~) x~ = ds * b with ds = J^(-1/2), x = ds * x~.  Since
// ||b - A x|| <= max(1/ds) ||b~ - A~ x~|| and ||b|| >= min(1/ds) ||b~||, the
// scaled system is solved to tol / sqrt(max j / min j), which bounds the
// original relative residual by tol; the residual reported is the original
// system's, computed with the general product kernel.
//
// S~ is a handle of its own (the same structure, permutation and split as A,
// values scaled on the GPU); pars3_mrs_solve keeps one per handle and alpha.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "internal.h"

namespace p3 {

static constexpr int TB = 256;
static inline unsigned nblk(int64_t m) { return (unsigned)std::max<int64_t>(1, cdiv(m, TB)); }

struct skew_shadow {
  double alpha = 0.0;
  pars3_matrix *B = nullptr;
  dbuf<double> ds_orig, ds_perm, bt, xt, yt, partials;
  ~skew_shadow() { pars3_destroy(B); }
};

void skew_shadow_free(skew_shadow *sh) { delete sh; }

// ds_i = 1 / sqrt(alpha + d_i) (d = nullptr: D = 0)
__global__ void k_inv_sqrt_shift(const double *__restrict__ d, double alpha, int32_t n, double *__restrict__ ds) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ds[i] = 1.0 / sqrt(alpha + (d ? d[i] : 0.0));
}

// out_e = (val_e ds_i) ds_j for the stored (i, j) of every row i
__global__ void k_scale_lower(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                              const double *__restrict__ val, const double *__restrict__ ds, int32_t n,
                              double *__restrict__ out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = ds[i];
  for (int32_t e = rp[i]; e < rp[i + 1]; e++) out[e] = val[e] * di * ds[col[e]];
}

__global__ void k_mul(const double *__restrict__ a, const double *__restrict__ b, int32_t n, double *__restrict__ out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}
__global__ void k_div(const double *__restrict__ a, const double *__restrict__ b, int32_t n, double *__restrict__ out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] / b[i];
}

// per workgroup: sum of (y - b)^2 and of b^2 over a grid-stride range
__global__ void k_resid_partials(const double *__restrict__ y, const double *__restrict__ b, int64_t n,
                                 double *__restrict__ part) {
  __shared__ double s_r[TB / 64], s_b[TB / 64];
  double r2 = 0.0, b2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
    const double r = y[i] - b[i];
    r2 += r * r;
    b2 += b[i] * b[i];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    r2 += __shfl_xor(r2, o, 64);
    b2 += __shfl_xor(b2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_r[threadIdx.x >> 6] = r2;
    s_b[threadIdx.x >> 6] = b2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, tb = 0.0;
    for (int w = 0; w < TB / 64; w++) {
      tr += s_r[w];
      tb += s_b[w];
    }
    part[2 * blockIdx.x] = tr;
    part[2 * blockIdx.x + 1] = tb;
  }
}

// A handle holding S~ = J^(-1/2) S J^(-1/2) with A's structure, permutation
// and split parameters; ds_orig / ds_perm: J^(-1/2) in the caller's and the
// reordered numbering.
static pars3_status make_scaled(const pars3_matrix *A, const double *ds_orig, const double *ds_perm,
                                pars3_matrix **out, hipStream_t s) {
  *out = nullptr;
  pars3_matrix *B = new (std::nothrow) pars3_matrix();
  if (!B) return fail(PARS3_ENOMEM, "skew_form: host allocation failed");
  auto run = [&]() -> pars3_status {
    const int32_t n = (int32_t)A->n;
    const int64_t nnz = A->nnz;
    B->n = n;
    B->nnz = nnz;
    B->device = A->device;
    B->kind = PARS3_SKEW;
    P3_HIP(B->rowptr.alloc(n + 1));
    P3_HIP(B->col.alloc(nnz));
    P3_HIP(B->val.alloc(nnz));
    P3_HIP(B->perm.alloc(n));
    P3_HIP(B->iperm.alloc(n));
    P3_HIP(B->prow.alloc(n + 1));
    P3_HIP(B->pcol.alloc(nnz));
    P3_HIP(B->pval.alloc(nnz));
    P3_HIP(hipMemcpyAsync(B->rowptr.p, A->rowptr.p, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    P3_HIP(hipMemcpyAsync(B->prow.p, A->prow.p, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (n > 0) {
      P3_HIP(hipMemcpyAsync(B->perm.p, A->perm.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      P3_HIP(hipMemcpyAsync(B->iperm.p, A->iperm.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    if (nnz > 0) {
      P3_HIP(hipMemcpyAsync(B->col.p, A->col.p, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      P3_HIP(hipMemcpyAsync(B->pcol.p, A->pcol.p, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      k_scale_lower<<<nblk(n), TB, 0, s>>>(A->rowptr.p, A->col.p, A->val.p, ds_orig, n, B->val.p);
      k_scale_lower<<<nblk(n), TB, 0, s>>>(A->prow.p, A->pcol.p, A->pval.p, ds_perm, n, B->pval.p);
      P3_LAUNCHED();
    }
    B->ncomp = A->ncomp;
    B->nlevels = A->nlevels;
    B->perm_kind = A->perm_kind;
    B->perm_done = true;
    P3_TRY(split_and_layout(B, A->params, s));
    P3_HIP(hipStreamSynchronize(s));
    B->split_done = true;
    return PARS3_OK;
  };
  pars3_status st = run();
  if (st != PARS3_OK) {
    delete B;
    return st;
  }
  *out = B;
  return PARS3_OK;
}

static pars3_status check_definite(const pars3_matrix *A, double alpha) {
  if (!A->split_done) return fail(PARS3_ESTATE, "skew_form: call pars3_reorder first");
  if (A->kind != PARS3_SKEW) return fail(PARS3_ESTATE, "skew_form: S must be skew-symmetric");
  const double jmin = alpha + (A->diag.p ? A->dmin : 0.0);
  if (A->n > 0 && !(jmin > 0.0))
    return fail(PARS3_EINVAL, "skew_form: alpha*I + D is not positive definite (min %.3e)", jmin);
  return PARS3_OK;
}

// the handle's cached S~ for this alpha (rebuilt when alpha changes)
static pars3_status shadow_for(pars3_matrix *A, double alpha, hipStream_t s, skew_shadow **out) {
  if (!A->shadow) A->shadow = new (std::nothrow) skew_shadow();
  skew_shadow *sh = A->shadow;
  if (!sh) return fail(PARS3_ENOMEM, "mrs: host allocation failed");
  const int32_t n = (int32_t)A->n;
  if (!sh->B || sh->alpha != alpha) {
    pars3_destroy(sh->B);
    sh->B = nullptr;
    P3_HIP(sh->ds_orig.alloc(n));
    P3_HIP(sh->ds_perm.alloc(n));
    P3_HIP(sh->bt.alloc(n));
    P3_HIP(sh->xt.alloc(n));
    P3_HIP(sh->yt.alloc(n));
    P3_HIP(sh->partials.alloc(2 * 1024));
    if (n > 0) {
      k_inv_sqrt_shift<<<nblk(n), TB, 0, s>>>(A->diag.p, alpha, n, sh->ds_orig.p);
      k_inv_sqrt_shift<<<nblk(n), TB, 0, s>>>(A->pdiag.p, alpha, n, sh->ds_perm.p);
      P3_LAUNCHED();
    }
    P3_TRY(make_scaled(A, sh->ds_orig.p, sh->ds_perm.p, &sh->B, s));
    sh->alpha = alpha;
  }
  *out = sh;
  return PARS3_OK;
}

pars3_status mrs_shifted(pars3_matrix *A, double alpha, const double *b, double *x, const pars3_mrs_opts &o,
                         pars3_mrs_info *info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  P3_TRY(check_definite(A, alpha));
  const int32_t n = (int32_t)A->n;
  pars3_mrs_info inf{};
  if (n == 0) {
    if (info) *info = inf;
    return PARS3_OK;
  }
  skew_shadow *sh = nullptr;
  P3_TRY(shadow_for(A, alpha, s, &sh));
  const double *ds = o.order == PARS3_ORDER_RCM ? sh->ds_perm.p : sh->ds_orig.p;
  // b~ = ds b, x~0 = x0 / ds
  k_mul<<<nblk(n), TB, 0, s>>>(ds, b, n, sh->bt.p);
  k_div<<<nblk(n), TB, 0, s>>>(x, ds, n, sh->xt.p);
  P3_LAUNCHED();
  pars3_mrs_opts oi = o;
  const double jmin = alpha + A->dmin, jmax = alpha + A->dmax;
  oi.tol = o.tol / std::sqrt(jmax / jmin);
  pars3_mrs_info ii{};
  const pars3_status sti = pars3_mrs_solve(sh->B, 1.0, sh->bt.p, sh->xt.p, &oi, &ii, s);
  if (sti != PARS3_OK && sti != PARS3_ENOCONV && sti != PARS3_EBREAKDOWN && sti != PARS3_ENAN) return sti;
  // x = ds x~ and the original system's residual
  k_mul<<<nblk(n), TB, 0, s>>>(ds, sh->xt.p, n, x);
  P3_LAUNCHED();
  P3_TRY(pars3_spmv(A, alpha, x, sh->yt.p, 1, PARS3_F64, o.order, s));
  const unsigned g = std::min<unsigned>(nblk(n), 1024u);
  k_resid_partials<<<g, TB, 0, s>>>(sh->yt.p, b, n, sh->partials.p);
  P3_LAUNCHED();
  std::vector<double> hp(2 * (size_t)g);
  P3_HIP(hipMemcpyAsync(hp.data(), sh->partials.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  double r2 = 0.0, b2 = 0.0;
  for (unsigned q = 0; q < g; q++) {
    r2 += hp[2 * q];
    b2 += hp[2 * q + 1];
  }
  const double bscale = b2 > 0.0 ? std::sqrt(b2) : 1.0;
  inf = ii;
  inf.relres = std::sqrt(r2) / bscale;
  int32_t status = ii.status;
  if (!std::isfinite(inf.relres)) status = 3;
  else if (inf.relres <= o.tol) status = 0;
  else if (status == 0) status = 1;
  inf.status = status;
  inf.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (status == 3) return fail(PARS3_ENAN, "mrs: NaN or Inf met");
  if (status == 2) return fail(PARS3_EBREAKDOWN, "mrs: breakdown (gamma = 0)");
  if (status == 1)
    return fail(PARS3_ENOCONV, "mrs: relative residual %.3e after %d iterations (tol %.1e)", inf.relres, inf.iters,
                o.tol);
  return PARS3_OK;
}

}  // namespace p3

using p3::fail;

extern "C" pars3_status pars3_skew_form(const pars3_matrix *A, double alpha, pars3_matrix **out, void *stream) {
  using namespace p3;
  if (!A || !out) return fail(PARS3_EINVAL, "skew_form: NULL argument");
  *out = nullptr;
  P3_TRY(check_definite(A, alpha));
  hipStream_t s = (hipStream_t)stream;
  P3_HIP(hipSetDevice(A->device));
  const int32_t n = (int32_t)A->n;
  dbuf<double> dso, dsp;
  P3_HIP(dso.alloc(n));
  P3_HIP(dsp.alloc(n));
  if (n > 0) {
    k_inv_sqrt_shift<<<nblk(n), TB, 0, s>>>(A->diag.p, alpha, n, dso.p);
    k_inv_sqrt_shift<<<nblk(n), TB, 0, s>>>(A->pdiag.p, alpha, n, dsp.p);
    P3_LAUNCHED();
  }
  return make_scaled(A, dso.p, dsp.p, out, s);
}
