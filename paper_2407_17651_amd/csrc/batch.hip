// Many matrices at once: products with block right-hand sides and MRS solves
// for a batch of independent shifted skew-symmetric systems, each matrix in
// its own configuration, all of them in one launch per product.
//
// Work list.  Every (matrix, tile) pair is an item with an estimated cost
// (the tile's share of the matrix's stored entries plus its rows).  Matrices
// are taken largest first and their tiles in ascending order (so the two
// reads of a tile-pair block stay close in time); the sequence is cut into 8
// contiguous queues of equal cost, one per XCD; the workgroups of XCD q take
// the items of queue q in order, one each (see k_batch_product).
//
// The launch of a product is captured once per set of vector pointers in a
// hipGraph and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "internal.h"

struct pars3_batch {
  std::vector<pars3_matrix *> mats;
  std::vector<int64_t> off;    // vector offsets (prefix of n)
  std::vector<int32_t> poff;   // partial-sum offsets (prefix of tiles)
  std::vector<int32_t> Ts;     // tile height of each matrix when the batch was made
  int32_t minT = 1024, maxT = 64, grid = 0, nitems = 0;
  p3::dbuf<int2> items;
  p3::dbuf<int32_t> qbeg;
  hipStream_t gs = nullptr;  // capture stream
  // product graph cache (one pointer set)
  p3::dbuf<p3::prod_task> tasks;
  std::vector<p3::prod_task> hkey;
  int hk = 0, hv = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~pars3_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gs) (void)hipStreamDestroy(gs);
  }
};

namespace p3 {

static constexpr int BT = 256;

// ---------------------------------------------------------------- MRS kernels
// Block b of a per-element kernel belongs to system bsys[b] and covers its
// elements [bstart[b], bstart[b] + BT * 4).
struct bmrs_ptrs {
  mrs_dev *dev;
  const int64_t *off;
  const int32_t *poff, *ntl;
  const int32_t *bsys;
  const int64_t *bstart;
  double *W0, *W1, *W2, *P0, *P1, *X, *B, *Y, *partials;
};

// sum of squares of each system's segment of a (one workgroup per system)
__global__ __launch_bounds__(BT) void k_bnorm(const double *__restrict__ a, const int64_t *__restrict__ off,
                                             double *__restrict__ out) {
  __shared__ double red[BT / 64];
  const int32_t i = blockIdx.x;
  double s = 0.0;
  for (int64_t e = off[i] + threadIdx.x; e < off[i + 1]; e += BT) s += a[e] * a[e];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[i] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_bmrs_const(mrs_dev *__restrict__ dev, int32_t m) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dev[i].minus_one = -1.0;
}

// start of every system: state from ||b|| and ||r0|| (y = A x0 - b in Y)
__global__ void k_bmrs_init(bmrs_ptrs p, const double *__restrict__ bn2, const double *__restrict__ rn2,
                            const double *__restrict__ alpha, double tol, int32_t maxit, int32_t m) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  mrs_dev &d = p.dev[i];
  const double bnorm = sqrt(bn2[i]), beta1 = sqrt(rn2[i]);
  for (int k = 0; k < 2; k++) d.beta[k] = d.c1[k] = d.s1[k] = d.c2[k] = d.s2[k] = d.eta[k] = d.nrm[k] = 0.0;
  d.c1[0] = 1.0;
  d.c2[0] = 1.0;
  d.eta[0] = beta1;
  d.nrm[0] = 1.0;  // W_0 = v_1 is normalised
  d.delta = d.eps = d.gamma = d.ceta = d.inv_beta = d.vnrm_inv = d.zcoef = 0.0;
  d.scaleS = 1.0;
  d.bnorm = bnorm > 0.0 ? bnorm : 1.0;
  d.tol_abs = tol * bnorm;
  d.alpha = alpha[i];
  d.minus_one = -1.0;
  d.iter = 0;
  d.maxit = maxit;
  d.done = (beta1 == 0.0 || beta1 <= d.tol_abs || maxit <= 0) ? 1 : 0;
  d.active = 0;
  d.status = 0;
  if (!isfinite(beta1) || !isfinite(bnorm)) {  // a NaN or Inf in b, x0 or the matrix
    d.done = 1;
    d.status = 3;
  }
}

// W_0 = v_1 = -y / ||y|| (unnormalised Lanczos vectors W_k live in
// W[(k + 1) % 3]), W_{-1} = p_0 = p_{-1} = 0 for every system
__global__ __launch_bounds__(BT) void k_bmrs_start(bmrs_ptrs p) {
  const int32_t i = p.bsys[blockIdx.x];
  const int64_t e1 = p.off[i + 1];
  const double beta1 = p.dev[i].eta[0];
  const double inv = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
  for (int64_t e = p.bstart[blockIdx.x] + threadIdx.x, q = 0; q < 4 && e < e1; q++, e += BT) {
    p.W1[e] = -p.Y[e] * inv;
    p.W0[e] = 0.0;
    p.P0[e] = 0.0;
    p.P1[e] = 0.0;
  }
}

__global__ __launch_bounds__(1024) void k_bmrs_scalar(bmrs_ptrs p, int par) {
  __shared__ double red[1024 / 64];
  const int32_t i = blockIdx.x;
  mrs_dev *d = &p.dev[i];
  if (d->done) {
    if (threadIdx.x == 0) d->active = 0;
    return;
  }
  const double *pp = p.partials + p.poff[i];
  const int32_t np = p.ntl[i];
  double s = 0.0;
  for (int32_t q = threadIdx.x; q < np; q += 1024) s += pp[q];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x >= 64) return;
  s = threadIdx.x < 16 ? red[threadIdx.x] : 0.0;
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x != 0) return;
  mrs_update(d, par, s, nullptr);
}

// The pending vector update of every finished system whose last iteration
// was not followed by a product: p_j = (W_{j-1} vnrm_inv - delta p_{j-1}
// - eps p_{j-2}) / gamma, x += ceta p_j.  Then k_bmrs_settle clears its flag.
__global__ __launch_bounds__(BT) void k_bmrs_flush(bmrs_ptrs p) {
  const int32_t i = p.bsys[blockIdx.x];
  const mrs_dev *d = &p.dev[i];
  if (!(d->done && d->active)) return;
  const int32_t j = d->iter;
  const double *w = j % 3 == 0 ? p.W0 : (j % 3 == 1 ? p.W1 : p.W2);
  const double *p1 = (j + 1) & 1 ? p.P1 : p.P0;
  double *p2 = j & 1 ? p.P1 : p.P0;
  const double delta = d->delta, eps = d->eps, gamma = d->gamma, ceta = d->ceta, vn = d->vnrm_inv;
  const int64_t e1 = p.off[i + 1];
  for (int64_t e = p.bstart[blockIdx.x] + threadIdx.x, q = 0; q < 4 && e < e1; q++, e += BT) {
    const double pn = (w[e] * vn - delta * p1[e] - eps * p2[e]) / gamma;
    p2[e] = pn;
    p.X[e] += ceta * pn;
  }
}
__global__ void k_bmrs_settle(mrs_dev *__restrict__ dev, int32_t m) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m && dev[i].done) dev[i].active = 0;
}

static inline unsigned g1(int64_t m, int b = BT) { return (unsigned)std::max<int64_t>(1, cdiv(m, b)); }

}  // namespace p3

using p3::fail;

// Work list of the matrices with use[i] != 0 (all when use is NULL):
// matrices largest first, tiles ascending, cut into 8 contiguous queues of
// equal estimated cost (stored entries twice, rows once, inner band).
static void build_queues(const std::vector<pars3_matrix *> &mats, const int32_t *use, std::vector<int2> &it,
                         std::vector<int32_t> &qb) {
  const int32_t m = (int32_t)mats.size();
  std::vector<int32_t> ord;
  for (int32_t i = 0; i < m; i++)
    if (!use || use[i]) ord.push_back(i);
  auto mcost = [&](int32_t i) {
    const pars3_matrix *A = mats[i];
    return 2.0 * (double)A->lay.nnz_blocked + (double)A->n * (1 + A->lay.w_in);
  };
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return mcost(a) > mcost(b); });
  it.clear();
  std::vector<double> cost;
  double total = 0.0;
  for (int32_t i : ord) {
    const int32_t nt = mats[i]->lay.ntiles;
    const double c = nt ? mcost(i) / nt : 0.0;
    for (int32_t t = 0; t < nt; t++) {
      it.push_back(make_int2(i, t));
      cost.push_back(c);
      total += c;
    }
  }
  qb.assign(9, 0);
  double acc = 0.0;
  int q = 1;
  for (size_t k = 0; k < it.size(); k++) {
    acc += cost[k];
    while (q < 8 && acc >= total * q / 8.0) qb[q++] = (int32_t)(k + 1);
  }
  while (q < 8) qb[q++] = (int32_t)it.size();
  qb[8] = (int32_t)it.size();
  for (int k = 1; k <= 8; k++) qb[k] = std::max(qb[k], qb[k - 1]);
}

// one workgroup per item of the longest queue, for each of the 8 queues
static int32_t queue_grid(const std::vector<int32_t> &qb) {
  int32_t longest = 1;
  for (int q = 0; q < 8; q++) longest = std::max(longest, qb[q + 1] - qb[q]);
  return 8 * longest;
}

extern "C" pars3_status pars3_batch_create(int32_t m, pars3_matrix *const *mats, pars3_batch **out) {
  using namespace p3;
  if (!out) return fail(PARS3_EINVAL, "batch: NULL output");
  *out = nullptr;
  if (m < 1 || !mats) return fail(PARS3_EINVAL, "batch: need at least one matrix");
  for (int32_t i = 0; i < m; i++) {
    if (!mats[i]) return fail(PARS3_EINVAL, "batch: matrix %d is NULL", i);
    if (!mats[i]->split_done) return fail(PARS3_ESTATE, "batch: matrix %d is not reordered", i);
  }
  pars3_batch *B = new (std::nothrow) pars3_batch;
  if (!B) return fail(PARS3_ENOMEM, "batch: out of host memory");
  auto bad = [&](pars3_status st) {
    delete B;
    return st;
  };
  B->mats.assign(mats, mats + m);
  B->off.assign(m + 1, 0);
  B->poff.assign(m + 1, 0);
  B->Ts.assign(m, 0);
  for (int32_t i = 0; i < m; i++) {
    B->off[i + 1] = B->off[i] + mats[i]->n;
    B->poff[i + 1] = B->poff[i] + mats[i]->lay.ntiles;
    B->Ts[i] = mats[i]->lay.T;
    B->minT = std::min(B->minT, mats[i]->lay.T);
    B->maxT = std::max(B->maxT, mats[i]->lay.T);
  }
  std::vector<int2> it;
  std::vector<int32_t> qb;
  build_queues(B->mats, nullptr, it, qb);
  B->nitems = (int32_t)it.size();
  B->grid = queue_grid(qb);
  if (B->items.alloc(std::max<size_t>(it.size(), 1)) != hipSuccess || B->qbeg.alloc(9) != hipSuccess || B->tasks.alloc(m) != hipSuccess) {
    (void)hipGetLastError();
    return bad(fail(PARS3_ENOMEM, "batch: device allocation failed"));
  }
  if ((!it.empty() && hipMemcpy(B->items.p, it.data(), it.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(B->qbeg.p, qb.data(), 9 * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamCreateWithFlags(&B->gs, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return bad(fail(PARS3_EHIP, "batch: set-up copy failed"));
  }
  *out = B;
  return PARS3_OK;
}

extern "C" void pars3_batch_destroy(pars3_batch *B) { delete B; }

extern "C" pars3_status pars3_batch_info(const pars3_batch *B, int32_t *n_items, int32_t *grid, int32_t *queue_begin9) {
  if (!B) return fail(PARS3_EINVAL, "batch: NULL handle");
  if (n_items) *n_items = B->nitems;
  if (grid) *grid = B->grid;
  if (queue_begin9) P3_HIP(hipMemcpy(queue_begin9, B->qbeg.p, 9 * sizeof(int32_t), hipMemcpyDeviceToHost));
  return PARS3_OK;
}

// The work list, LDS size and entry word types of a batch were fixed from the
// layouts its matrices had when it was made.
static pars3_status check_layouts(const pars3_batch *B) {
  using namespace p3;
  for (size_t i = 0; i < B->mats.size(); i++) {
    const layout &L = B->mats[i]->lay;
    if (L.T != B->Ts[i] || L.ntiles != B->poff[i + 1] - B->poff[i])
      return fail(PARS3_ESTATE, "batch: matrix %d was split again after the batch was made", (int)i);
  }
  return PARS3_OK;
}

static pars3_status batch_tasks(pars3_batch *B, const double *shifts, const void *const *x, void *const *y,
                                int32_t vec_dtype, int32_t value_dtype, std::vector<p3::prod_task> &t, int *vkind) {
  using namespace p3;
  const int32_t m = (int32_t)B->mats.size();
  t.resize(m);
  int vk0 = -1;
  P3_TRY(check_layouts(B));
  for (int32_t i = 0; i < m; i++) {
    int vk = -1;
    P3_TRY(make_task(B->mats[i], vec_dtype, value_dtype, &t[i], &vk));
    if (vk0 >= 0 && vk != vk0) return fail(PARS3_ESTATE, "batch: matrices store different value types");
    vk0 = vk;
    t[i].shift = shifts ? shifts[i] : 0.0;
    t[i].x = x[i];
    t[i].y = y[i];
  }
  *vkind = vk0;
  return PARS3_OK;
}

static bool same_tasks(const std::vector<p3::prod_task> &a, const std::vector<p3::prod_task> &b) {
  return a.size() == b.size() && std::equal(a.begin(), a.end(), b.begin(), [](const p3::prod_task &u, const p3::prod_task &v) {
           return std::memcmp(&u, &v, sizeof(u)) == 0;
         });
}

extern "C" pars3_status pars3_batch_spmv(pars3_batch *B, const double *shifts, const void *const *x, void *const *y,
                                         int32_t k, int32_t vec_dtype, int32_t value_dtype, void *stream) {
  using namespace p3;
  if (!B || !x || !y) return fail(PARS3_EINVAL, "batch spmv: NULL argument");
  if (k != 1 && k != 2 && k != 4 && k != 8) return fail(PARS3_EINVAL, "batch spmv: k must be 1, 2, 4 or 8");
  if (vec_dtype != PARS3_F64 && vec_dtype != PARS3_F32) return fail(PARS3_EINVAL, "batch spmv: bad vec_dtype");
  const int32_t m = (int32_t)B->mats.size();
  for (int32_t i = 0; i < m; i++) {
    if (B->mats[i]->n > 0 && (!x[i] || !y[i])) return fail(PARS3_EINVAL, "batch spmv: NULL vector of matrix %d", i);
    if (k > 1 && (((uintptr_t)x[i] | (uintptr_t)y[i]) & 15u))
      return fail(PARS3_EINVAL, "batch spmv: vectors of matrix %d must be 16-byte aligned when k > 1", i);
  }
  std::vector<prod_task> t;
  int vk = -1;
  P3_TRY(batch_tasks(B, shifts, x, y, vec_dtype, value_dtype, t, &vk));
  hipStream_t s = (hipStream_t)stream;
  if (!(B->exec && B->hk == k && B->hv == vk && same_tasks(t, B->hkey))) {
    // new pointer set: upload the task table and capture the launch
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    P3_HIP(hipStreamSynchronize(s));
    P3_HIP(hipMemcpy(B->tasks.p, t.data(), m * sizeof(prod_task), hipMemcpyHostToDevice));
    P3_HIP(hipStreamBeginCapture(B->gs, hipStreamCaptureModeThreadLocal));
    bool gen = false;
    for (const pars3_matrix *A : B->mats) gen = gen || is_general(A);
    pars3_status st =
        launch_batch(vk, k, false, gen, B->tasks.p, B->items.p, B->qbeg.p, B->grid, B->minT, B->maxT, B->gs);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(B->gs, &g);
    if (st != PARS3_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ee != hipSuccess) return fail(PARS3_EHIP, "batch spmv: capture failed: %s", hipGetErrorString(ee));
    B->graph = g;
    P3_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->hkey = t;
    B->hk = k;
    B->hv = vk;
  }
  P3_HIP(hipGraphLaunch(B->exec, s));
  return PARS3_OK;
}

extern "C" pars3_status pars3_batch_mrs_solve(pars3_batch *B, const double *alphas, const double *const *b,
                                              double *const *x, const pars3_mrs_opts *opts, pars3_mrs_info *infos,
                                              void *stream) {
  using namespace p3;
  if (!B || !alphas || !b || !x) return fail(PARS3_EINVAL, "batch mrs: NULL argument");
  pars3_mrs_opts o;
  if (opts) o = *opts;
  else pars3_mrs_opts_default(&o);
  if (!(o.tol >= 0.0) || o.maxit < 0 || o.check_every < 1) return fail(PARS3_EINVAL, "batch mrs: bad options");
  if (o.precision != PARS3_F64) return fail(PARS3_EINVAL, "batch mrs: only FP64 iterations are batched");
  if (o.order != PARS3_ORDER_RCM && o.order != PARS3_ORDER_ORIGINAL) return fail(PARS3_EINVAL, "batch mrs: bad order");
  const int32_t m = (int32_t)B->mats.size();
  for (int32_t i = 0; i < m; i++) {
    if (B->mats[i]->n > 0 && (!b[i] || !x[i])) return fail(PARS3_EINVAL, "batch mrs: NULL vector of system %d", i);
    if (B->mats[i]->kind != PARS3_SKEW || B->mats[i]->diag.p)
      return fail(PARS3_ESTATE, "batch mrs: system %d is not alpha*I + S with S skew-symmetric", i);
  }
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t cs = (hipStream_t)stream;
  hipStream_t s = B->gs;
  {
    hipEvent_t ev;
    P3_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    P3_HIP(hipEventRecord(ev, cs));
    P3_HIP(hipStreamWaitEvent(s, ev, 0));
    P3_HIP(hipEventDestroy(ev));
  }
  const int64_t N = B->off[m];
  const int32_t NT = B->poff[m];
  // per-element blocks
  std::vector<int32_t> bsys;
  std::vector<int64_t> bstart;
  for (int32_t i = 0; i < m; i++)
    for (int64_t e = B->off[i]; e < B->off[i + 1]; e += 4 * BT) {
      bsys.push_back(i);
      bstart.push_back(e);
    }
  const int32_t nvb = (int32_t)bsys.size();
  std::vector<int32_t> ntl(m);
  for (int32_t i = 0; i < m; i++) ntl[i] = B->mats[i]->lay.ntiles;
  dbuf<double> W0, W1, W2, P0, P1, X, Bv, Y, part, nb2, nr2, alph;
  dbuf<mrs_dev> dev;
  dbuf<int64_t> doff, dbst;
  dbuf<int32_t> dpoff, dntl, dbsys, dqb;
  dbuf<int2> ditems;
  dbuf<prod_task> tk;
  const size_t n1 = (size_t)std::max<int64_t>(N, 1);
  P3_HIP(W0.alloc(n1));
  P3_HIP(W1.alloc(n1));
  P3_HIP(W2.alloc(n1));
  P3_HIP(P0.alloc(n1));
  P3_HIP(P1.alloc(n1));
  P3_HIP(X.alloc(n1));
  P3_HIP(Bv.alloc(n1));
  P3_HIP(Y.alloc(n1));
  P3_HIP(part.alloc(std::max(NT, 1)));
  P3_HIP(nb2.alloc(m));
  P3_HIP(nr2.alloc(m));
  P3_HIP(alph.alloc(m));
  P3_HIP(dev.alloc(m));
  P3_HIP(doff.alloc(m + 1));
  P3_HIP(dbst.alloc(std::max(nvb, 1)));
  P3_HIP(dpoff.alloc(m + 1));
  P3_HIP(dntl.alloc(m));
  P3_HIP(dbsys.alloc(std::max(nvb, 1)));
  P3_HIP(dqb.alloc(9));
  P3_HIP(ditems.alloc(std::max(B->nitems, 1)));
  P3_HIP(tk.alloc(7 * (size_t)m));
  P3_HIP(hipMemcpyAsync(doff.p, B->off.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  P3_HIP(hipMemcpyAsync(dpoff.p, B->poff.data(), (m + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  P3_HIP(hipMemcpyAsync(dntl.p, ntl.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (nvb) {
    P3_HIP(hipMemcpyAsync(dbsys.p, bsys.data(), nvb * sizeof(int32_t), hipMemcpyHostToDevice, s));
    P3_HIP(hipMemcpyAsync(dbst.p, bstart.data(), nvb * sizeof(int64_t), hipMemcpyHostToDevice, s));
  }
  P3_HIP(hipMemcpyAsync(alph.p, alphas, m * sizeof(double), hipMemcpyHostToDevice, s));
  // inputs into the concatenated (reordered) numbering
  for (int32_t i = 0; i < m; i++) {
    const pars3_matrix *A = B->mats[i];
    if (A->n == 0) continue;
    if (o.order == PARS3_ORDER_ORIGINAL) {
      P3_TRY(gather_rows(b[i], Bv.p + B->off[i], A->perm.p, A->n, 1, 8, s));
      P3_TRY(gather_rows(x[i], X.p + B->off[i], A->perm.p, A->n, 1, 8, s));
    } else {
      P3_HIP(hipMemcpyAsync(Bv.p + B->off[i], b[i], A->n * sizeof(double), hipMemcpyDeviceToDevice, s));
      P3_HIP(hipMemcpyAsync(X.p + B->off[i], x[i], A->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  }
  bmrs_ptrs P{dev.p, doff.p, dpoff.p, dntl.p, dbsys.p, dbst.p, W0.p, W1.p, W2.p, P0.p, P1.p, X.p, Bv.p, Y.p, part.p};
  double *Wb[3] = {W0.p, W1.p, W2.p};
  double *Pb[2] = {P0.p, P1.p};
  // task tables: [0, m) the residual y = alpha x + S x - b; [J m, (J+1) m)
  // for J = 1..6 the fused iterations (buffer roles repeat with period 6):
  // W_J = scaleS (S W_{J-1}) + zcoef W_{J-2}, with iteration J-1's vector
  // update on the same rows
  std::vector<prod_task> ht(7 * (size_t)m);
  int vk = -1;
  P3_TRY(check_layouts(B));
  for (int32_t i = 0; i < m; i++) {
    const int64_t e = B->off[i];
    for (int r = 0; r < 7; r++) {
      prod_task &a = ht[(size_t)r * m + i];
      P3_TRY(make_task(B->mats[i], PARS3_F64, -1, &a, &vk));
      a.partials = part.p + B->poff[i];
      if (r == 0) {
        a.shift = alphas[i];
        a.x = X.p + e;
        a.y = Y.p + e;
        a.z = Bv.p + e;
        a.beta = &dev.p[i].minus_one;
      } else {
        const int J = r;
        a.shift = 0.0;
        a.x = Wb[J % 3] + e;
        a.y = Wb[(J + 1) % 3] + e;
        a.z = Wb[(J + 2) % 3] + e;
        a.beta = &dev.p[i].zcoef;
        a.scale = &dev.p[i].scaleS;
        a.done = &dev.p[i].done;
        a.active = &dev.p[i].active;
        a.vec = &dev.p[i].delta;
        a.p1 = Pb[J & 1] + e;
        a.p2 = Pb[(J + 1) & 1] + e;
        a.xs = X.p + e;
      }
    }
  }
  P3_HIP(hipMemcpyAsync(tk.p, ht.data(), ht.size() * sizeof(prod_task), hipMemcpyHostToDevice, s));
  // the full work list (also used for the residuals)
  std::vector<int2> hit;
  std::vector<int32_t> hqb;
  build_queues(B->mats, nullptr, hit, hqb);
  int32_t grid = queue_grid(hqb);
  if (!hit.empty()) P3_HIP(hipMemcpyAsync(ditems.p, hit.data(), hit.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  P3_HIP(hipMemcpyAsync(dqb.p, hqb.data(), 9 * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // ||b|| and r0 = b - A x0 (y = alpha x0 + S x0 - b)
  k_bmrs_const<<<g1(m), BT, 0, s>>>(dev.p, m);
  k_bnorm<<<m, BT, 0, s>>>(Bv.p, doff.p, nb2.p);
  P3_LAUNCHED();
  P3_TRY(launch_batch(PARS3_F64, 1, true, false, tk.p, ditems.p, dqb.p, grid, B->minT, B->maxT, s));
  k_bnorm<<<m, BT, 0, s>>>(Y.p, doff.p, nr2.p);
  k_bmrs_init<<<g1(m), BT, 0, s>>>(P, nb2.p, nr2.p, alph.p, o.tol, o.maxit, m);
  if (nvb) k_bmrs_start<<<nvb, BT, 0, s>>>(P);
  P3_LAUNCHED();
  // six iterations captured and replayed; the work list is rebuilt from the
  // systems still iterating whenever their number has fallen to 3/4 of those
  // in the list (measured on 256 systems: 56.4 ms, against 58.0 ms when
  // rebuilt at 1/2; 7/8 and every change of the count gave 56.5-56.7 ms)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto capture = [&]() -> pars3_status {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    P3_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    pars3_status st2 = PARS3_OK;
    for (int J = 1; J <= 6 && st2 == PARS3_OK; J++) {
      st2 = launch_batch(PARS3_F64, 1, true, false, tk.p + (size_t)J * m, ditems.p, dqb.p, grid, B->minT, B->maxT,
                         s);
      if (st2 == PARS3_OK) k_bmrs_scalar<<<m, 1024, 0, s>>>(P, (J - 1) & 1);
    }
    const hipError_t ee = hipStreamEndCapture(s, &graph);
    if (st2 != PARS3_OK) return st2;
    if (ee != hipSuccess) return fail(PARS3_EHIP, "batch mrs: capture failed: %s", hipGetErrorString(ee));
    P3_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    return PARS3_OK;
  };
  pars3_status st = capture();
  std::vector<mrs_dev> hd(m);
  std::vector<int32_t> use(m, 1);
  int32_t in_list = m;
  const int32_t chunk = std::max(1, o.check_every / 6);
  for (int32_t it = 0; st == PARS3_OK && it < o.maxit; it += 6 * chunk) {
    for (int32_t c = 0; c < chunk && st == PARS3_OK; c++)
      if (hipGraphLaunch(exec, s) != hipSuccess) st = fail(PARS3_EHIP, "batch mrs: graph launch failed");
    if (st != PARS3_OK) break;
    if (hipMemcpyAsync(hd.data(), dev.p, m * sizeof(mrs_dev), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = fail(PARS3_EHIP, "batch mrs: state read failed");
      break;
    }
    int32_t running = 0;
    for (int32_t i = 0; i < m; i++) running += hd[i].done ? 0 : 1;
    if (running == 0) break;
    if (4 * running <= 3 * in_list) {
      // apply the pending updates of the systems leaving the list, then
      // restrict the work list to the systems still iterating
      if (nvb) k_bmrs_flush<<<nvb, BT, 0, s>>>(P);
      k_bmrs_settle<<<g1(m), BT, 0, s>>>(dev.p, m);
      for (int32_t i = 0; i < m; i++) use[i] = hd[i].done ? 0 : 1;
      build_queues(B->mats, use.data(), hit, hqb);
      grid = queue_grid(hqb);
      if (!hit.empty() && hipMemcpyAsync(ditems.p, hit.data(), hit.size() * sizeof(int2), hipMemcpyHostToDevice, s) != hipSuccess)
        st = fail(PARS3_EHIP, "batch mrs: work list upload failed");
      if (st == PARS3_OK && hipMemcpyAsync(dqb.p, hqb.data(), 9 * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
        st = fail(PARS3_EHIP, "batch mrs: work list upload failed");
      if (st == PARS3_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(PARS3_EHIP, "batch mrs: sync failed");
      if (st == PARS3_OK) st = capture();
      in_list = running;
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (st != PARS3_OK) {
    (void)hipGetLastError();
    return st;
  }
  // pending updates, then the true residuals over the full work list
  if (nvb) k_bmrs_flush<<<nvb, BT, 0, s>>>(P);
  k_bmrs_settle<<<g1(m), BT, 0, s>>>(dev.p, m);
  P3_LAUNCHED();
  build_queues(B->mats, nullptr, hit, hqb);
  grid = queue_grid(hqb);
  if (!hit.empty()) P3_HIP(hipMemcpyAsync(ditems.p, hit.data(), hit.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  P3_HIP(hipMemcpyAsync(dqb.p, hqb.data(), 9 * sizeof(int32_t), hipMemcpyHostToDevice, s));
  P3_TRY(launch_batch(PARS3_F64, 1, true, false, tk.p, ditems.p, dqb.p, grid, B->minT, B->maxT, s));
  k_bnorm<<<m, BT, 0, s>>>(Y.p, doff.p, nr2.p);
  P3_LAUNCHED();
  std::vector<double> hr(m), hb(m);
  P3_HIP(hipMemcpyAsync(hd.data(), dev.p, m * sizeof(mrs_dev), hipMemcpyDeviceToHost, s));
  P3_HIP(hipMemcpyAsync(hr.data(), nr2.p, m * sizeof(double), hipMemcpyDeviceToHost, s));
  P3_HIP(hipMemcpyAsync(hb.data(), nb2.p, m * sizeof(double), hipMemcpyDeviceToHost, s));
  for (int32_t i = 0; i < m; i++) {
    const pars3_matrix *A = B->mats[i];
    if (A->n == 0) continue;
    if (o.order == PARS3_ORDER_ORIGINAL) P3_TRY(scatter_rows(X.p + B->off[i], x[i], A->perm.p, A->n, 1, 8, s));
    else P3_HIP(hipMemcpyAsync(x[i], X.p + B->off[i], A->n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  P3_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int32_t worst = 0;
  for (int32_t i = 0; i < m; i++) {
    const double bn = hb[i] > 0.0 ? std::sqrt(hb[i]) : 1.0;
    const double rel = std::sqrt(hr[i]) / bn;
    int32_t status = hd[i].status;
    if (!std::isfinite(rel)) status = 3;
    else if (rel <= o.tol) status = 0;
    else if (status == 0) status = 1;
    if (infos) {
      infos[i].iters = hd[i].iter;
      infos[i].refinements = 0;
      infos[i].status = status;
      infos[i].relres = rel;
      infos[i].eta = std::fabs(hd[i].eta[hd[i].iter & 1]) / bn;
      infos[i].time_ms = ms;
    }
    // worst first: NaN/Inf (3), then breakdown (2), then the iteration limit (1)
    if (status != 0 && (worst == 0 || status > worst)) worst = status;
  }
  if (worst == 3) return fail(PARS3_ENAN, "batch mrs: NaN or Inf met");
  if (worst == 2) return fail(PARS3_EBREAKDOWN, "batch mrs: breakdown in at least one system");
  if (worst == 1) return fail(PARS3_ENOCONV, "batch mrs: at least one system did not converge");
  return PARS3_OK;
}

// ------------------------------------------------------------ batch-level autotuner
namespace p3 {
// a fixed pattern in [-1, 1) for the timing vectors
__global__ void k_batch_tune_fill(double *__restrict__ a, float *__restrict__ b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t h = (uint32_t)(i * 2654435761u) >> 8;
  const double v = (double)h * (2.0 / 16777216.0) - 1.0;
  if (a) a[i] = v;
  if (b) b[i] = (float)v;
}
}  // namespace p3

extern "C" pars3_status pars3_batch_autotune(pars3_matrix *const *mats, int32_t m, const int32_t *tile_rows,
                                             int32_t nt, int32_t k, int32_t vec_dtype, int32_t reps, double *us,
                                             int32_t *best, void *stream) {
  using namespace p3;
  if (!mats || m < 1 || !tile_rows || nt < 1 || !us)
    return fail(PARS3_EINVAL, "batch autotune: NULL or empty argument");
  if (k != 1 && k != 2 && k != 4 && k != 8) return fail(PARS3_EINVAL, "batch autotune: k must be 1, 2, 4 or 8");
  if (vec_dtype != PARS3_F64 && vec_dtype != PARS3_F32) return fail(PARS3_EINVAL, "batch autotune: bad vec_dtype");
  if (reps < 1) return fail(PARS3_EINVAL, "batch autotune: reps must be >= 1");
  for (int32_t j = 0; j < nt; j++) {
    const int32_t T = tile_rows[j];
    if (T != 64 && T != 128 && T != 256 && T != 512 && T != 1024)
      return fail(PARS3_EINVAL, "batch autotune: tile_rows must be 64, 128, 256, 512 or 1024 (got %d)", T);
  }
  for (int32_t i = 0; i < m; i++) {
    if (!mats[i]) return fail(PARS3_EINVAL, "batch autotune: matrix %d is NULL", i);
    if (!mats[i]->split_done) return fail(PARS3_ESTATE, "batch autotune: matrix %d is not reordered", i);
  }
  hipStream_t s = (hipStream_t)stream;
  // timing vectors: matrix i's x and y at 256-byte aligned offsets
  const size_t elem = vec_dtype == PARS3_F64 ? sizeof(double) : sizeof(float);
  std::vector<size_t> off(m + 1, 0);
  for (int32_t i = 0; i < m; i++) off[i + 1] = off[i] + ((size_t)mats[i]->n * k * elem + 255) / 256 * 256;
  const int64_t total = (int64_t)std::max<size_t>(off[m] / elem, 1);
  dbuf<char> xb, yb;
  P3_HIP(xb.alloc(off[m] + 256));
  P3_HIP(yb.alloc(off[m] + 256));
  k_batch_tune_fill<<<(unsigned)cdiv(total, 256), 256, 0, s>>>(
      vec_dtype == PARS3_F64 ? (double *)xb.p : nullptr, vec_dtype == PARS3_F32 ? (float *)xb.p : nullptr, total);
  P3_LAUNCHED();
  std::vector<const void *> xs(m);
  std::vector<void *> ys(m);
  for (int32_t i = 0; i < m; i++) {
    xs[i] = xb.p + off[i];
    ys[i] = yb.p + off[i];
  }
  hipEvent_t e0, e1;
  P3_HIP(hipEventCreate(&e0));
  P3_HIP(hipEventCreate(&e1));
  pars3_status st = PARS3_OK;
  int32_t ib = -1;
  for (int32_t j = 0; j < nt && st == PARS3_OK; j++) {
    us[j] = -1.0;
    // every matrix re-split with this tile height (its reordering and other
    // split parameters kept), then one batch over them
    for (int32_t i = 0; i < m && st == PARS3_OK; i++) {
      pars3_split_params p = mats[i]->params;
      p.tile_rows = tile_rows[j];
      p.engine = PARS3_ENGINE_TILES;
      st = pars3_reorder(mats[i], &p, stream);
    }
    if (st != PARS3_OK) break;
    pars3_batch *B = nullptr;
    st = pars3_batch_create(m, mats, &B);
    if (st != PARS3_OK) break;
    // warm-up: launches for at least 20 ms of wall time (the first captures
    // the launch; the GPU reaches its steady clock only after some
    // milliseconds of continuous work), then the median of three batches of
    // reps launches
    const auto w0 = std::chrono::steady_clock::now();
    for (int r = 0; st == PARS3_OK; r++) {
      st = pars3_batch_spmv(B, nullptr, xs.data(), ys.data(), k, vec_dtype, -1, stream);
      if (st == PARS3_OK && (r & 3) == 3) {
        if (hipStreamSynchronize(s) != hipSuccess) st = fail(PARS3_EHIP, "batch autotune: sync failed");
        if (std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count() >= 20.0) break;
      }
    }
    double t[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < 3 && st == PARS3_OK; b++) {
      if (hipEventRecord(e0, s) != hipSuccess) st = fail(PARS3_EHIP, "batch autotune: event record failed");
      for (int r = 0; r < reps && st == PARS3_OK; r++)
        st = pars3_batch_spmv(B, nullptr, xs.data(), ys.data(), k, vec_dtype, -1, stream);
      if (st == PARS3_OK && hipEventRecord(e1, s) != hipSuccess)
        st = fail(PARS3_EHIP, "batch autotune: event record failed");
      float ms = 0.f;
      if (st == PARS3_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(PARS3_EHIP, "batch autotune: event timing failed");
      t[b] = 1e3 * (double)ms / reps;
    }
    pars3_batch_destroy(B);
    if (st != PARS3_OK) break;
    std::sort(t, t + 3);
    us[j] = t[1];
    if (ib < 0 || us[j] < us[ib]) ib = j;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PARS3_OK) return st;
  // leave every matrix split with the fastest tile height
  for (int32_t i = 0; i < m; i++) {
    pars3_split_params p = mats[i]->params;
    p.tile_rows = tile_rows[ib];
    p.engine = PARS3_ENGINE_TILES;
    P3_TRY(pars3_reorder(mats[i], &p, stream));
  }
  if (best) *best = ib;
  return PARS3_OK;
}
