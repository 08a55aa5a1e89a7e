// MRS for shifted skew-symmetric systems (alpha*I + S) x = b (Section 1:
// the minimal-residual method for (shifted) skew-symmetric systems needs one
// product with S and one inner product per iteration).
//
// Recurrence.  Skew Lanczos: w = S v_j + beta_j v_{j-1}, beta_{j+1} = ||w||,
// v_{j+1} = w / beta_{j+1}, so (alpha*I + S) V_k = V_{k+1} H_k where column j
// of H_k holds -beta_j (row j-1), alpha (row j) and beta_{j+1} (row j+1).  H_k
// is reduced by Givens rotations as in MINRES; |eta| is the residual norm.
//
// One iteration is two launches on one stream, captured once in a hipGraph
// (six iterations, the period of the buffer roles) and replayed:
//   1. the product kernel with the solver epilogue.  Lanczos vectors are kept
//      unnormalised (W_j = w_j), so the product computes
//      W_{j+1} = (S W_j) / beta_{j+1} + (beta_{j+1} / beta_j) W_{j-1}
//      with per-tile partial sums of W_{j+1}^2 in FP64 (the inner product),
//      and on the same rows applies iteration j's vector update
//      p_j = (v_j - delta p_{j-1} - eps p_{j-2}) / gamma, x += c eta p_j
//      with v_j = W_{j-1} / beta_j;
//   2. k_mrs_scalar, one workgroup: sums the partials in a fixed order,
//      updates the rotations and eta, records |eta|/||b||, decides to stop.
// Scalars live on the device; the host reads the stop flag every
// check_every iterations.  Once stopped, the next product still applies the
// last vector update (or k_mrs_flush does, when no product followed within
// the replay) and every later kernel returns at once.
//
// Mixed precision: iterative refinement in FP64 around an inner MRS whose
// matrix values and vectors are FP32 (or BF16 values with FP32 vectors) while
// its inner products and scalars stay FP64:
//   r = b - A x (FP64 values and vectors); stop when ||r|| <= tol ||b||;
//   solve (alpha*I + S~) d = r to relative tolerance max(inner_tol,
//   0.3 tol ||b|| / ||r||) (no tighter than the outer target needs); x += d.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "internal.h"

namespace p3 {

static constexpr int TB = 256;
static inline unsigned nblk(int64_t m) { return (unsigned)std::max<int64_t>(1, cdiv(m, TB)); }

// Sum of the per-tile partials in a fixed order (deterministic): every
// thread adds a fixed strided subset, then the wavefronts and the workgroup
// combine in a fixed tree.  All loads (the stop flag, the recurrence state
// and the thread's first SU partials) go out before the first result is used.
static constexpr int SB = 256, SU = 32;
__global__ __launch_bounds__(SB) void k_mrs_scalar(mrs_dev *d, int par, const double *__restrict__ partials,
                                                  int32_t np, double *__restrict__ hist) {
  __shared__ double red[SB / 64];
  const int32_t done = d->done;
  const mrs_in in = mrs_load(d, par);
  double v[SU];
#pragma unroll
  for (int u = 0; u < SU; u++) {
    const int32_t q = (int32_t)threadIdx.x + u * SB;
    v[u] = q < np ? partials[q] : 0.0;
  }
  for (int32_t q = threadIdx.x + SU * SB; q < np; q += SB) v[0] += partials[q];
  if (done) {
    if (threadIdx.x == 0) d->active = 0;
    return;
  }
#pragma unroll
  for (int w = SU / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; u++) v[u] += v[u + w];
  double sum = v[0];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot = red[0];
#pragma unroll
  for (int w = 1; w < SB / 64; w++) tot += red[w];
  mrs_apply(d, par, tot, hist, in);
}

// The vector update of the last iteration when no product carried it:
// p = (W vnrm_inv - delta p1 - eps p2) / gamma over p2, x += ceta p.
template <class X>
__global__ __launch_bounds__(TB) void k_mrs_flush(mrs_dev *d, int64_t n, const X *__restrict__ w,
                                                 const X *__restrict__ p1, X *p2, X *x) {
  const double delta = d->delta, eps = d->eps, gamma = d->gamma, ceta = d->ceta, vn = d->vnrm_inv;
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
    const double pn = ((double)w[i] * vn - delta * (double)p1[i] - eps * (double)p2[i]) / gamma;
    p2[i] = (X)pn;
    x[i] = (X)((double)x[i] + ceta * pn);
  }
}

// v = -y * inv (the start vector from y = A x - b), in the inner precision
template <class XI, class XO>
__global__ void k_neg_scale(const XI *__restrict__ y, XO *__restrict__ v, double inv, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) v[i] = (XO)(-(double)y[i] * inv);
}
template <class X>
__global__ void k_zero(X *__restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) a[i] = (X)0;
}
template <class X>
__global__ void k_add_to_f64(double *__restrict__ x, const X *__restrict__ d, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) x[i] += (double)d[i];
}
__global__ void k_sumsq_partials(const double *__restrict__ a, int64_t n, double *__restrict__ partials) {
  __shared__ double red[TB];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) s += a[i] * a[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = TB / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ------------------------------------------------------------ host side
struct mrs_ws {
  dbuf<char> vb0, vb1, w, pb0, pb1, xin;  // inner-precision vectors
  dbuf<double> xr, br, yr;                 // FP64 solution, rhs, residual (reordered numbering)
  dbuf<double> partials, hist;
  dbuf<mrs_dev> dev;
};

static pars3_status sum_partials(const double *partials, int64_t np, hipStream_t s, double *out) {
  std::vector<double> h(std::max<int64_t>(np, 1));
  if (np) P3_HIP(hipMemcpyAsync(h.data(), partials, np * sizeof(double), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (int64_t q = 0; q < np; q++) t += h[q];
  *out = t;
  return PARS3_OK;
}

// y = alpha x + S x - b (FP64); returns ||y||
static pars3_status residual64(pars3_matrix *A, double alpha, const double *x, const double *b, double *y,
                               double *partials, const double *minus_one, hipStream_t s, double *rnorm) {
  epilogue<double> ep;
  ep.z = b;
  ep.beta = minus_one;
  ep.partials = partials;
  P3_TRY(spmv_ex(A, alpha, x, y, 1, PARS3_F64, -1, s, &ep));
  double ss = 0.0;
  P3_TRY(sum_partials(partials, A->lay.ntiles, s, &ss));
  *rnorm = std::sqrt(ss);
  return PARS3_OK;
}

// Runs MRS iterations from the normalized start vector already in vb0 (v_1),
// accumulating into x (inner precision), until |eta| <= tol_abs, maxit, or a
// breakdown.  Iteration counts, status and the last |eta| are returned.
template <class X>
static pars3_status mrs_iterate(pars3_matrix *A, int value_dtype, double alpha, double beta1, double bnorm,
                                double tol_abs, int32_t maxit, int32_t check_every, mrs_ws &ws, X *x, hipStream_t s,
                                int32_t *iters, int32_t *status, double *eta_out, double *hist) {
  const int64_t n = A->n;
  const int vec = sizeof(X) == 8 ? PARS3_F64 : PARS3_F32;
  // Lanczos vectors are kept unnormalised: W_k = w_k (W_0 = v_1 from the
  // caller, in ws.vb0), stored in Wb[(k + 1) % 3]; p_k in P[k & 1].  The
  // product of iteration J computes W_J = scaleS (S W_{J-1}) + zcoef W_{J-2}
  // and applies iteration J-1's vector update on its rows.
  X *Wb[3] = {(X *)ws.w.p, (X *)ws.vb0.p, (X *)ws.vb1.p};
  X *P[2] = {(X *)ws.pb0.p, (X *)ws.pb1.p};
  k_zero<X><<<nblk(n), TB, 0, s>>>(Wb[0], n);
  k_zero<X><<<nblk(n), TB, 0, s>>>(P[0], n);
  k_zero<X><<<nblk(n), TB, 0, s>>>(P[1], n);
  P3_LAUNCHED();
  mrs_dev h{};
  h.beta[0] = 0.0;
  h.c1[0] = 1.0;
  h.s1[0] = 0.0;
  h.c2[0] = 1.0;
  h.s2[0] = 0.0;
  h.eta[0] = beta1;
  h.nrm[0] = 1.0;  // W_0 = v_1 is normalised
  h.scaleS = 1.0;
  h.zcoef = 0.0;
  h.bnorm = bnorm > 0.0 ? bnorm : 1.0;
  h.tol_abs = tol_abs;
  h.alpha = alpha;
  h.minus_one = -1.0;
  h.iter = 0;
  h.maxit = maxit;
  h.done = (beta1 == 0.0 || beta1 <= tol_abs || maxit <= 0) ? 1 : 0;
  h.active = 0;
  h.status = 0;
  P3_HIP(hipMemcpyAsync(ws.dev.p, &h, sizeof(h), hipMemcpyHostToDevice, s));
  const int32_t np = A->lay.ntiles;
  // capture six iterations (buffer roles repeat with period 6)
  const bool prof = A->prof.on;
  A->prof.on = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  pars3_status st = PARS3_OK;
  mrs_dev *dv = ws.dev.p;
  hipError_t ce = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (ce == hipSuccess) {
    for (int J = 1; J <= 6 && st == PARS3_OK; J++) {
      epilogue<X> ep;
      ep.z = Wb[(J + 2) % 3];
      ep.beta = &dv->zcoef;
      ep.scale = &dv->scaleS;
      ep.partials = ws.partials.p;
      ep.done = &dv->done;
      ep.active = &dv->active;
      ep.vec = &dv->delta;
      ep.p1 = P[J & 1];
      ep.p2 = P[(J + 1) & 1];
      ep.xs = x;
      st = spmv_ex(A, 0.0, Wb[J % 3], Wb[(J + 1) % 3], 1, vec, value_dtype, s, &ep);
      if (st != PARS3_OK) break;
      k_mrs_scalar<<<1, SB, 0, s>>>(dv, (J - 1) & 1, ws.partials.p, np, hist);
    }
    hipError_t ee = hipStreamEndCapture(s, &graph);
    if (st == PARS3_OK && ee != hipSuccess) st = fail(PARS3_EHIP, "mrs: stream capture failed: %s", hipGetErrorString(ee));
  } else {
    st = fail(PARS3_EHIP, "mrs: cannot capture the solver stream: %s", hipGetErrorString(ce));
  }
  A->prof.on = prof;
  if (st == PARS3_OK) {
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) st = fail(PARS3_EHIP, "mrs: graph instantiation failed: %s", hipGetErrorString(ie));
  }
  // Replays between stop checks: at most check_every / 6, and once |eta| has
  // been seen to fall, about as many as its observed rate per iteration says
  // are still needed (iterations launched past the stop return at once but
  // still cost two launches each).
  int32_t done = h.done;
  const int32_t chunk_max = std::max(1, check_every / 6);
  int32_t chunk = chunk_max;
  double eta_prev = std::fabs(beta1);
  int32_t iter_prev = 0;
  for (int32_t it = 0; st == PARS3_OK && !done && it < maxit;) {
    for (int32_t c = 0; c < chunk; c++) {
      hipError_t le = hipGraphLaunch(exec, s);
      if (le != hipSuccess) {
        st = fail(PARS3_EHIP, "mrs: graph launch failed: %s", hipGetErrorString(le));
        break;
      }
    }
    if (st != PARS3_OK) break;
    it += 6 * chunk;
    hipError_t me = hipMemcpyAsync(&h, dv, sizeof(h), hipMemcpyDeviceToHost, s);
    if (me == hipSuccess) me = hipStreamSynchronize(s);
    if (me != hipSuccess) st = fail(PARS3_EHIP, "mrs: %s", hipGetErrorString(me));
    done = h.done;
    const double eta_now = std::fabs(h.eta[h.iter & 1]);
    const int32_t di = h.iter - iter_prev;
    chunk = chunk_max;
    if (!done && di > 0 && eta_now > tol_abs && eta_now < eta_prev) {
      const double per_iter = std::log(eta_now / eta_prev) / di;  // < 0
      const double need = std::log(tol_abs / eta_now) / per_iter;  // iterations still needed, > 0
      // with a margin of 10% and one replay: a check that finds the solve
      // still running costs a host round trip, about as much as several
      // iterations past the stop
      chunk = (int32_t)std::min<double>(chunk_max, std::max(1.0, std::ceil((1.1 * need + 6.0) / 6.0)));
    }
    eta_prev = eta_now;
    iter_prev = h.iter;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (st != PARS3_OK) {
    (void)hipGetLastError();
    return st;
  }
  P3_HIP(hipMemcpyAsync(&h, dv, sizeof(h), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  if (h.active) {
    // the last iteration's vector update, when no product followed it
    const int32_t j = h.iter;
    k_mrs_flush<X><<<std::min<unsigned>(nblk(n), 4096u), TB, 0, s>>>(dv, n, Wb[j % 3], P[(j + 1) & 1], P[j & 1], x);
    P3_LAUNCHED();
  }
  *iters = h.iter;
  *status = h.status;
  *eta_out = std::fabs(h.eta[h.iter & 1]);
  return PARS3_OK;
}

template <class T>
static hipError_t fit(dbuf<T> &b, size_t m) {
  return b.p && b.n == m ? hipSuccess : b.alloc(m);
}

// Workspace kept in the handle between solves; resized when n, the inner
// precision or the history length change.
static pars3_status ensure_ws(mrs_ws &ws, int64_t n, int32_t ntiles, size_t inner_elem, int32_t hist_len) {
  const size_t vb = (size_t)std::max<int64_t>(n, 1) * inner_elem;
  const size_t n1 = (size_t)std::max<int64_t>(n, 1);
  P3_HIP(fit(ws.vb0, vb));
  P3_HIP(fit(ws.vb1, vb));
  P3_HIP(fit(ws.w, vb));
  P3_HIP(fit(ws.pb0, vb));
  P3_HIP(fit(ws.pb1, vb));
  P3_HIP(fit(ws.xin, vb));
  P3_HIP(fit(ws.xr, n1));
  P3_HIP(fit(ws.br, n1));
  P3_HIP(fit(ws.yr, n1));
  P3_HIP(fit(ws.partials, (size_t)std::max<int64_t>(std::max(ntiles, 1), 1024)));
  if (hist_len > 0) P3_HIP(fit(ws.hist, (size_t)hist_len));
  P3_HIP(fit(ws.dev, 1));
  return PARS3_OK;
}

void mrs_ws_free(mrs_ws *w) { delete w; }

}  // namespace p3

using p3::fail;

extern "C" void pars3_mrs_opts_default(pars3_mrs_opts *o) {
  if (!o) return;
  o->tol = 1e-10;
  o->maxit = 10000;
  o->check_every = 32;
  o->precision = PARS3_F64;
  o->inner_tol = 0.0;
  o->max_refine = 30;
  o->order = PARS3_ORDER_RCM;
  o->hist_len = 0;
  o->hist = nullptr;
}

extern "C" pars3_status pars3_mrs_solve(pars3_matrix *A, double alpha, const double *b, double *x,
                                        const pars3_mrs_opts *opts, pars3_mrs_info *info, void *stream) {
  using namespace p3;
  if (!A) return fail(PARS3_EINVAL, "mrs: NULL handle");
  if (!A->split_done) return fail(PARS3_ESTATE, "mrs: call pars3_reorder first");
  if (A->kind != PARS3_SKEW) return fail(PARS3_ESTATE, "mrs: the solver needs S skew-symmetric");
  pars3_mrs_opts o;
  if (opts) o = *opts;
  else pars3_mrs_opts_default(&o);
  if (!(o.tol >= 0.0) || o.maxit < 0 || o.check_every < 1 || o.max_refine < 1 || o.hist_len < 0 ||
      (o.hist_len > 0 && !o.hist))
    return fail(PARS3_EINVAL, "mrs: bad options");
  if (o.order != PARS3_ORDER_RCM && o.order != PARS3_ORDER_ORIGINAL) return fail(PARS3_EINVAL, "mrs: bad order");
  if (o.precision != PARS3_F64 && o.precision != PARS3_F32 && o.precision != PARS3_BF16)
    return fail(PARS3_EINVAL, "mrs: bad precision");
  if (!A->has_f64) return fail(PARS3_ESTATE, "mrs: FP64 values are needed (value_dtype F64 or keep_fp64)");
  if (o.precision == PARS3_F32 && !A->has_f32)
    return fail(PARS3_ESTATE, "mrs: FP32 inner solves need value_dtype = PARS3_F32 with keep_fp64");
  if (o.precision == PARS3_BF16 && !A->has_bf16)
    return fail(PARS3_ESTATE, "mrs: BF16 inner solves need value_dtype = PARS3_BF16 with keep_fp64");
  const int64_t n = A->n;
  if (n > 0 && (!b || !x)) return fail(PARS3_EINVAL, "mrs: NULL vector");
  // alpha*I + D + S: through its shifted skew form I + S~
  if (A->diag.p) return mrs_shifted(A, alpha, b, x, o, info, (hipStream_t)stream);
  pars3_mrs_info inf{};
  if (n == 0) {
    if (info) *info = inf;
    return PARS3_OK;
  }
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t caller = (hipStream_t)stream;
  if (!A->solver_stream) {
    P3_HIP(hipStreamCreateWithFlags(&A->solver_stream, hipStreamNonBlocking));
  }
  hipStream_t s = A->solver_stream;
  {
    hipEvent_t ev;
    P3_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    P3_HIP(hipEventRecord(ev, caller));
    P3_HIP(hipStreamWaitEvent(s, ev, 0));
    P3_HIP(hipEventDestroy(ev));
  }
  const bool mixed = o.precision != PARS3_F64;
  if (!A->mrs) A->mrs = new (std::nothrow) mrs_ws;
  if (!A->mrs) return fail(PARS3_ENOMEM, "mrs: out of host memory");
  mrs_ws &ws = *A->mrs;
  const int32_t hist_len = o.hist_len > 0 ? std::max(o.hist_len, o.maxit) : 0;
  P3_TRY(ensure_ws(ws, n, A->lay.ntiles, mixed ? sizeof(float) : sizeof(double), hist_len));
  // b and x0 in the reordered numbering
  if (o.order == PARS3_ORDER_ORIGINAL) {
    P3_TRY(gather_rows(b, ws.br.p, A->perm.p, n, 1, 8, s));
    P3_TRY(gather_rows(x, ws.xr.p, A->perm.p, n, 1, 8, s));
  } else {
    P3_HIP(hipMemcpyAsync(ws.br.p, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    P3_HIP(hipMemcpyAsync(ws.xr.p, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  // ||b||
  const unsigned nbk = std::min<unsigned>(nblk(n), 1024u);
  k_sumsq_partials<<<nbk, TB, 0, s>>>(ws.br.p, n, ws.partials.p);
  P3_LAUNCHED();
  double bb = 0.0;
  P3_TRY(sum_partials(ws.partials.p, nbk, s, &bb));
  const double bnorm = std::sqrt(bb);
  const double bscale = bnorm > 0.0 ? bnorm : 1.0;
  // constant -1 for the residual epilogue
  mrs_dev hd{};
  hd.minus_one = -1.0;
  P3_HIP(hipMemcpyAsync(ws.dev.p, &hd, sizeof(hd), hipMemcpyHostToDevice, s));
  P3_HIP(hipStreamSynchronize(s));
  const double *minus_one = &ws.dev.p->minus_one;
  double rnorm = 0.0;
  int32_t iters = 0, status = 0, refine = 0;
  double eta = 0.0;
  pars3_status st = PARS3_OK;
  if (!mixed) {
    // r0 = b - A x0: y = A x0 - b, v_1 = -y / ||y||
    P3_TRY(residual64(A, alpha, ws.xr.p, ws.br.p, ws.yr.p, ws.partials.p, minus_one, s, &rnorm));
    if (!std::isfinite(rnorm) || !std::isfinite(bnorm)) {
      // a NaN or Inf in b, x0 or the matrix: nothing to iterate on
      status = 3;
    } else {
      if (rnorm > 0.0) {
        k_neg_scale<double, double><<<nblk(n), TB, 0, s>>>(ws.yr.p, (double *)ws.vb0.p, 1.0 / rnorm, n);
        P3_LAUNCHED();
      }
      st = mrs_iterate<double>(A, -1, alpha, rnorm, bscale, o.tol * bnorm, o.maxit, o.check_every, ws, ws.xr.p, s,
                               &iters, &status, &eta, hist_len > 0 ? ws.hist.p : nullptr);
      if (st != PARS3_OK) return st;
    }
  } else {
    const double itol = o.inner_tol > 0.0 ? o.inner_tol : (o.precision == PARS3_F32 ? 1e-6 : 1e-2);
    int32_t budget = o.maxit;
    status = 1;
    for (refine = 0; refine <= o.max_refine; refine++) {
      P3_TRY(residual64(A, alpha, ws.xr.p, ws.br.p, ws.yr.p, ws.partials.p, minus_one, s, &rnorm));
      if (!std::isfinite(rnorm)) {
        status = 3;
        break;
      }
      if (rnorm <= o.tol * bnorm) {
        status = 0;
        break;
      }
      if (budget <= 0 || refine == o.max_refine) {
        status = 1;
        break;
      }
      // inner solve (alpha*I + S~) d = r, r = -y, from d = 0
      k_neg_scale<double, float><<<nblk(n), TB, 0, s>>>(ws.yr.p, (float *)ws.vb0.p, 1.0 / rnorm, n);
      k_zero<float><<<nblk(n), TB, 0, s>>>((float *)ws.xin.p, n);
      P3_LAUNCHED();
      int32_t it = 0, ist = 0;
      double ieta = 0.0;
      // stop the inner solve at the reduction the outer tolerance still
      // needs (with a margin for the difference between the inner estimate
      // and the true FP64 residual), never looser than inner_tol
      const double need = 0.3 * o.tol * bnorm / rnorm;
      const double itol_now = std::max(itol, need);
      st = mrs_iterate<float>(A, o.precision, alpha, rnorm, bscale, itol_now * rnorm, budget, o.check_every, ws,
                              (float *)ws.xin.p, s, &it, &ist, &ieta, hist_len > 0 ? ws.hist.p + iters : nullptr);
      if (st != PARS3_OK) return st;
      iters += it;
      budget -= it;
      k_add_to_f64<float><<<nblk(n), TB, 0, s>>>(ws.xr.p, (const float *)ws.xin.p, n);
      P3_LAUNCHED();
      if (ist == 2 || ist == 3) {
        status = ist;
        break;
      }
      if (it == 0) {  // no progress possible
        status = 1;
        break;
      }
    }
  }
  // true FP64 residual of the returned x
  P3_TRY(residual64(A, alpha, ws.xr.p, ws.br.p, ws.yr.p, ws.partials.p, minus_one, s, &rnorm));
  if (o.order == PARS3_ORDER_ORIGINAL) P3_TRY(scatter_rows(ws.xr.p, x, A->perm.p, n, 1, 8, s));
  else P3_HIP(hipMemcpyAsync(x, ws.xr.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (hist_len > 0 && iters > 0)
    P3_HIP(hipMemcpyAsync(o.hist, ws.hist.p, std::min(iters, o.hist_len) * sizeof(double), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  inf.iters = iters;
  inf.refinements = mixed ? refine : 0;
  inf.relres = rnorm / bscale;
  inf.eta = mixed ? inf.relres : eta / bscale;
  if (!std::isfinite(rnorm)) status = 3;
  else if (inf.relres <= o.tol) status = 0;
  else if (status == 0) status = 1;
  inf.status = status;
  inf.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (status == 3) return fail(PARS3_ENAN, "mrs: NaN or Inf met");
  if (status == 2) return fail(PARS3_EBREAKDOWN, "mrs: breakdown (gamma = 0)");
  if (status == 1)
    return fail(PARS3_ENOCONV, "mrs: relative residual %.3e after %d iterations (tol %.1e)", inf.relres, iters, o.tol);
  return PARS3_OK;
}
