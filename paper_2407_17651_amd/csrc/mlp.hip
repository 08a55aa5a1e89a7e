// Learned configuration selector: a multilayer perceptron
//   x -> ReLU(x W1 + b1) -> ReLU(h1 W2 + b2) -> h2 W3 + b3
// mapping the standardised sparsity features of a reordered matrix to one
// predicted log time ratio log(t_config / t_best) per configuration of the
// tuning grid; the selection is the argmin.  Training minimises the masked
// mean squared error  sum M (out - T)^2 / sum M  with Adam (Kingma and Ba,
// 2015).  Forward, backward and the optimiser are the kernels below, in FP32.
// Weights are stored input-major (W has shape [fan_in, fan_out]) and packed
// W1, b1, W2, b2, W3, b3 in one device array.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

struct pars3_mlp {
  int32_t n_in = 0, h1 = 0, h2 = 0, n_out = 0;
  int64_t np = 0;  // number of parameters
  int64_t o[7] = {0, 0, 0, 0, 0, 0, 0};  // offsets of W1, b1, W2, b2, W3, b3, end
  p3::dbuf<float> P, G, Mo, Vo;
  p3::dbuf<float> mean, stdv;  // feature scaler
  int64_t t = 0;                // Adam steps taken
  int32_t cap = 0;              // batch capacity of the workspace
  p3::dbuf<float> Xs, Ts, Ms, Z1, H1, Z2, H2, Out, GOut, GH2, GH1;
  p3::dbuf<double> red;  // loss and mask count
  p3::dbuf<int32_t> idx;
  // the configurations the outputs stand for (output g predicts grid[g]);
  // empty until pars3_mlp_set_grid or pars3_model_load
  std::vector<pars3_split_params> grid;
};

namespace p3 {

static constexpr int GT = 16;  // GEMM tile

// C[M x N] = op(A) op(B) (+ bias) with op(A) of shape [M x K], op(B) [K x N].
// TA: A is stored [K x M] (use its transpose); TB: B is stored [N x K].
// relu_out (optional) receives max(C, 0); gate (optional, [M x N]) zeroes C
// where gate <= 0 (the ReLU derivative of the pre-activation).
template <bool TA, bool TB>
__global__ __launch_bounds__(GT *GT) void k_gemm(const float *__restrict__ A, const float *__restrict__ B,
                                                 const float *__restrict__ bias, const float *__restrict__ gate,
                                                 float *__restrict__ C, float *__restrict__ relu_out, int32_t M,
                                                 int32_t N, int32_t K) {
  __shared__ float sa[GT][GT + 1], sb[GT][GT + 1];
  const int32_t tx = threadIdx.x % GT, ty = threadIdx.x / GT;
  const int32_t row = blockIdx.y * GT + ty, colx = blockIdx.x * GT + tx;
  float acc = 0.f;
  for (int32_t k0 = 0; k0 < K; k0 += GT) {
    // sa[ty][tx] = op(A)[blockIdx.y*GT + ty][k0 + tx]
    {
      const int32_t r = blockIdx.y * GT + ty, k = k0 + tx;
      float v = 0.f;
      if (r < M && k < K) v = TA ? A[(int64_t)k * M + r] : A[(int64_t)r * K + k];
      sa[ty][tx] = v;
    }
    // sb[ty][tx] = op(B)[k0 + ty][blockIdx.x*GT + tx]
    {
      const int32_t k = k0 + ty, c = blockIdx.x * GT + tx;
      float v = 0.f;
      if (k < K && c < N) v = TB ? B[(int64_t)c * K + k] : B[(int64_t)k * N + c];
      sb[ty][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int32_t kk = 0; kk < GT; kk++) acc = fmaf(sa[ty][kk], sb[kk][tx], acc);
    __syncthreads();
  }
  if (row >= M || colx >= N) return;
  if (bias) acc += bias[colx];
  const int64_t q = (int64_t)row * N + colx;
  if (gate && !(gate[q] > 0.f)) acc = 0.f;
  C[q] = acc;
  if (relu_out) relu_out[q] = acc > 0.f ? acc : 0.f;
}

// out[c] = sum over rows of G[r][c]  (bias gradients), fixed order
__global__ void k_colsum(const float *__restrict__ G, int32_t rows, int32_t cols, float *__restrict__ out) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int32_t r = 0; r < rows; r++) s += G[(int64_t)r * cols + c];
  out[c] = s;
}

// red[1] = sum of the mask (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_mask_count(const float *__restrict__ M, int64_t m, double *__restrict__ red) {
  __shared__ double s[256];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) a += (double)M[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[1] = s[0];
}

// GOut = 2 (Out - T) M / cnt; red[0] = sum ((Out - T) M)^2 / cnt (one
// workgroup, fixed order)
__global__ __launch_bounds__(256) void k_loss_grad(const float *__restrict__ Out, const float *__restrict__ T,
                                                   const float *__restrict__ M, int64_t m, float *__restrict__ GOut,
                                                   double *__restrict__ red) {
  __shared__ double s[256];
  const double cnt = red[1];
  const float inv = cnt > 0.0 ? (float)(1.0 / cnt) : 0.f;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const float d = (Out[i] - T[i]) * M[i];
    GOut[i] = 2.f * d * inv;
    a += (double)d * (double)d;
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[0] = cnt > 0.0 ? s[0] / cnt : 0.0;
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ Mo,
                       float *__restrict__ Vo, int64_t m, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float g = G[i];
  const float mo = b1 * Mo[i] + (1.f - b1) * g;
  const float vo = b2 * Vo[i] + (1.f - b2) * g * g;
  Mo[i] = mo;
  Vo[i] = vo;
  const float mh = mo / bc1, vh = vo / bc2;
  P[i] -= lr * mh / (sqrtf(vh) + eps);
}

// rows of X (and T, M) gathered by idx, X standardised on the way
__global__ void k_gather_std(const float *__restrict__ X, const int32_t *__restrict__ idx, int32_t rows, int32_t cols,
                             const float *__restrict__ mean, const float *__restrict__ stdv, float *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)rows * cols) return;
  const int32_t r = (int32_t)(q / cols), c = (int32_t)(q % cols);
  const int32_t src = idx ? idx[r] : r;
  float v = X[(int64_t)src * cols + c];
  if (mean) v = (v - mean[c]) / stdv[c];
  out[q] = v;
}

// per-feature mean and population standard deviation (1 where it is 0)
__global__ void k_scaler(const float *__restrict__ X, int32_t rows, int32_t cols, float *__restrict__ mean,
                         float *__restrict__ stdv) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0, s2 = 0.0;
  for (int32_t r = 0; r < rows; r++) {
    const double v = X[(int64_t)r * cols + c];
    s += v;
    s2 += v * v;
  }
  const double mu = rows ? s / rows : 0.0;
  const double var = rows ? std::max(s2 / rows - mu * mu, 0.0) : 0.0;
  const double sd = sqrt(var);
  mean[c] = (float)mu;
  stdv[c] = sd > 1e-12 ? (float)sd : 1.f;
}

// argmin over the valid outputs of each row (valid: mask == NULL or mask > 0)
__global__ void k_argmin(const float *__restrict__ Out, const float *__restrict__ M, int32_t rows, int32_t cols,
                         int32_t *__restrict__ choice) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  int32_t b = -1;
  float bv = 0.f;
  for (int32_t c = 0; c < cols; c++) {
    const int64_t q = (int64_t)r * cols + c;
    if (M && !(M[q] > 0.f)) continue;
    if (b < 0 || Out[q] < bv) {
      b = c;
      bv = Out[q];
    }
  }
  choice[r] = b;
}

// sort keys of one epoch's shuffle: a SplitMix64 hash of (seed, epoch, i)
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__global__ void k_shuffle_keys(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, int32_t m, uint64_t seed) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  keys[i] = splitmix64(seed ^ ((uint64_t)i * 0x632be59bd9b4e019ull)) >> 32;
  vals[i] = (uint32_t)i;
}

static inline unsigned g1(int64_t m, int b = 256) { return (unsigned)std::max<int64_t>(1, cdiv(m, b)); }

template <bool TA, bool TB>
static pars3_status gemm(const float *A, const float *B, const float *bias, const float *gate, float *C, float *relu,
                         int32_t M, int32_t N, int32_t K, hipStream_t s) {
  if (M == 0 || N == 0) return PARS3_OK;
  dim3 grid((unsigned)cdiv(N, GT), (unsigned)cdiv(M, GT));
  k_gemm<TA, TB><<<grid, GT * GT, 0, s>>>(A, B, bias, gate, C, relu, M, N, K);
  P3_LAUNCHED();
  return PARS3_OK;
}

static pars3_status ensure_cap(pars3_mlp *m, int32_t b) {
  if (b <= m->cap) return PARS3_OK;
  const size_t B = (size_t)b;
  P3_HIP(m->Xs.alloc(B * m->n_in));
  P3_HIP(m->Ts.alloc(B * m->n_out));
  P3_HIP(m->Ms.alloc(B * m->n_out));
  P3_HIP(m->Z1.alloc(B * m->h1));
  P3_HIP(m->H1.alloc(B * m->h1));
  P3_HIP(m->Z2.alloc(B * m->h2));
  P3_HIP(m->H2.alloc(B * m->h2));
  P3_HIP(m->Out.alloc(B * m->n_out));
  P3_HIP(m->GOut.alloc(B * m->n_out));
  P3_HIP(m->GH2.alloc(B * m->h2));
  P3_HIP(m->GH1.alloc(B * m->h1));
  P3_HIP(m->idx.alloc(B));
  m->cap = b;
  return PARS3_OK;
}

// forward on the (already standardised) rows in m->Xs
static pars3_status forward(pars3_mlp *m, int32_t b, hipStream_t s) {
  const float *P = m->P.p;
  P3_TRY(gemm<false, false>(m->Xs.p, P + m->o[0], P + m->o[1], nullptr, m->Z1.p, m->H1.p, b, m->h1, m->n_in, s));
  P3_TRY(gemm<false, false>(m->H1.p, P + m->o[2], P + m->o[3], nullptr, m->Z2.p, m->H2.p, b, m->h2, m->h1, s));
  P3_TRY(gemm<false, false>(m->H2.p, P + m->o[4], P + m->o[5], nullptr, m->Out.p, nullptr, b, m->n_out, m->h2, s));
  return PARS3_OK;
}

// loss and gradients of the rows in m->Xs / Ts / Ms (after forward)
static pars3_status backward(pars3_mlp *m, int32_t b, hipStream_t s) {
  const float *P = m->P.p;
  float *G = m->G.p;
  const int64_t mo = (int64_t)b * m->n_out;
  k_mask_count<<<1, 256, 0, s>>>(m->Ms.p, mo, m->red.p);
  k_loss_grad<<<1, 256, 0, s>>>(m->Out.p, m->Ts.p, m->Ms.p, mo, m->GOut.p, m->red.p);
  P3_LAUNCHED();
  // layer 3: gW3 = H2^T GOut, gb3 = colsum GOut, GH2 = (GOut W3^T) * [Z2 > 0]
  P3_TRY(gemm<true, false>(m->H2.p, m->GOut.p, nullptr, nullptr, G + m->o[4], nullptr, m->h2, m->n_out, b, s));
  k_colsum<<<g1(m->n_out), 256, 0, s>>>(m->GOut.p, b, m->n_out, G + m->o[5]);
  P3_LAUNCHED();
  P3_TRY(gemm<false, true>(m->GOut.p, P + m->o[4], nullptr, m->Z2.p, m->GH2.p, nullptr, b, m->h2, m->n_out, s));
  // layer 2
  P3_TRY(gemm<true, false>(m->H1.p, m->GH2.p, nullptr, nullptr, G + m->o[2], nullptr, m->h1, m->h2, b, s));
  k_colsum<<<g1(m->h2), 256, 0, s>>>(m->GH2.p, b, m->h2, G + m->o[3]);
  P3_LAUNCHED();
  P3_TRY(gemm<false, true>(m->GH2.p, P + m->o[2], nullptr, m->Z1.p, m->GH1.p, nullptr, b, m->h1, m->h2, s));
  // layer 1
  P3_TRY(gemm<true, false>(m->Xs.p, m->GH1.p, nullptr, nullptr, G + m->o[0], nullptr, m->n_in, m->h1, b, s));
  k_colsum<<<g1(m->h1), 256, 0, s>>>(m->GH1.p, b, m->h1, G + m->o[1]);
  P3_LAUNCHED();
  return PARS3_OK;
}

static pars3_status adam(pars3_mlp *m, float lr, float b1, float b2, float eps, hipStream_t s) {
  m->t++;
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)m->t));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)m->t));
  k_adam<<<g1(m->np), 256, 0, s>>>(m->P.p, m->G.p, m->Mo.p, m->Vo.p, m->np, lr, b1, b2, eps, bc1, bc2);
  P3_LAUNCHED();
  return PARS3_OK;
}

static uint64_t host_splitmix(uint64_t &st) {
  uint64_t z = (st += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace p3

using p3::fail;

extern "C" pars3_status pars3_mlp_create(int32_t n_in, int32_t h1, int32_t h2, int32_t n_out, uint64_t seed,
                                         pars3_mlp **out) {
  using namespace p3;
  if (!out) return fail(PARS3_EINVAL, "mlp: NULL output");
  *out = nullptr;
  if (n_in < 1 || h1 < 1 || h2 < 1 || n_out < 1 || n_in > 4096 || h1 > 4096 || h2 > 4096 || n_out > 4096)
    return fail(PARS3_EINVAL, "mlp: layer sizes must be in 1..4096");
  pars3_mlp *m = new (std::nothrow) pars3_mlp;
  if (!m) return fail(PARS3_ENOMEM, "mlp: out of host memory");
  m->n_in = n_in;
  m->h1 = h1;
  m->h2 = h2;
  m->n_out = n_out;
  const int64_t sz[6] = {(int64_t)n_in * h1, h1, (int64_t)h1 * h2, h2, (int64_t)h2 * n_out, n_out};
  m->o[0] = 0;
  for (int k = 0; k < 6; k++) m->o[k + 1] = m->o[k] + sz[k];
  m->np = m->o[6];
  // He-uniform weights (bound sqrt(6 / fan_in)), zero biases, from SplitMix64
  std::vector<float> h(m->np, 0.f);
  uint64_t st = seed;
  const int32_t fan[3] = {n_in, h1, h2};
  for (int L = 0; L < 3; L++) {
    const double bound = std::sqrt(6.0 / fan[L]);
    for (int64_t i = m->o[2 * L]; i < m->o[2 * L + 1]; i++) {
      const double u = (double)(host_splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
      h[i] = (float)((2.0 * u - 1.0) * bound);
    }
  }
  std::vector<float> ones(n_in, 1.f), zeros(n_in, 0.f);
  auto fin = [&](pars3_status st2) {
    if (st2 != PARS3_OK) delete m;
    else *out = m;
    return st2;
  };
  if (m->P.alloc(m->np) != hipSuccess || m->G.alloc(m->np) != hipSuccess || m->Mo.alloc(m->np) != hipSuccess ||
      m->Vo.alloc(m->np) != hipSuccess || m->mean.alloc(n_in) != hipSuccess || m->stdv.alloc(n_in) != hipSuccess ||
      m->red.alloc(2) != hipSuccess) {
    (void)hipGetLastError();
    return fin(fail(PARS3_ENOMEM, "mlp: device allocation failed"));
  }
  if (hipMemcpy(m->P.p, h.data(), m->np * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->G.p, 0, m->np * sizeof(float)) != hipSuccess ||
      hipMemset(m->Mo.p, 0, m->np * sizeof(float)) != hipSuccess ||
      hipMemset(m->Vo.p, 0, m->np * sizeof(float)) != hipSuccess ||
      hipMemcpy(m->mean.p, zeros.data(), n_in * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->stdv.p, ones.data(), n_in * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return fin(fail(PARS3_EHIP, "mlp: initialisation copy failed"));
  }
  return fin(PARS3_OK);
}

extern "C" void pars3_mlp_destroy(pars3_mlp *m) {
  if (!m) return;
  p3::forget_selector(m);
  delete m;
}

extern "C" pars3_status pars3_mlp_sizes(const pars3_mlp *m, int32_t *sizes4, int64_t *n_params) {
  if (!m) return fail(PARS3_EINVAL, "mlp: NULL handle");
  if (sizes4) {
    sizes4[0] = m->n_in;
    sizes4[1] = m->h1;
    sizes4[2] = m->h2;
    sizes4[3] = m->n_out;
  }
  if (n_params) *n_params = m->np;
  return PARS3_OK;
}

static pars3_status copy_host(void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
  if (bytes == 0) return PARS3_OK;
  P3_HIP(hipMemcpy(dst, src, bytes, kind));
  return PARS3_OK;
}

extern "C" pars3_status pars3_mlp_set_params(pars3_mlp *m, const float *host) {
  if (!m || !host) return fail(PARS3_EINVAL, "mlp: NULL argument");
  m->t = 0;
  P3_TRY(copy_host(m->P.p, host, m->np * sizeof(float), hipMemcpyHostToDevice));
  P3_HIP(hipMemset(m->Mo.p, 0, m->np * sizeof(float)));
  P3_HIP(hipMemset(m->Vo.p, 0, m->np * sizeof(float)));
  return PARS3_OK;
}
extern "C" pars3_status pars3_mlp_get_params(const pars3_mlp *m, float *host) {
  if (!m || !host) return fail(PARS3_EINVAL, "mlp: NULL argument");
  return copy_host(host, m->P.p, m->np * sizeof(float), hipMemcpyDeviceToHost);
}
extern "C" pars3_status pars3_mlp_get_grads(const pars3_mlp *m, float *host) {
  if (!m || !host) return fail(PARS3_EINVAL, "mlp: NULL argument");
  return copy_host(host, m->G.p, m->np * sizeof(float), hipMemcpyDeviceToHost);
}
extern "C" pars3_status pars3_mlp_set_scaler(pars3_mlp *m, const float *mean, const float *stdv) {
  if (!m || !mean || !stdv) return fail(PARS3_EINVAL, "mlp: NULL argument");
  P3_TRY(copy_host(m->mean.p, mean, m->n_in * sizeof(float), hipMemcpyHostToDevice));
  return copy_host(m->stdv.p, stdv, m->n_in * sizeof(float), hipMemcpyHostToDevice);
}
extern "C" pars3_status pars3_mlp_get_scaler(const pars3_mlp *m, float *mean, float *stdv) {
  if (!m || !mean || !stdv) return fail(PARS3_EINVAL, "mlp: NULL argument");
  P3_TRY(copy_host(mean, m->mean.p, m->n_in * sizeof(float), hipMemcpyDeviceToHost));
  return copy_host(stdv, m->stdv.p, m->n_in * sizeof(float), hipMemcpyDeviceToHost);
}

extern "C" pars3_status pars3_mlp_fit_scaler(pars3_mlp *m, const float *X, int32_t rows, void *stream) {
  using namespace p3;
  if (!m || (!X && rows > 0) || rows < 0) return fail(PARS3_EINVAL, "mlp: bad scaler input");
  hipStream_t s = (hipStream_t)stream;
  k_scaler<<<g1(m->n_in), 256, 0, s>>>(X, rows, m->n_in, m->mean.p, m->stdv.p);
  P3_LAUNCHED();
  P3_HIP(hipStreamSynchronize(s));
  return PARS3_OK;
}

extern "C" pars3_status pars3_mlp_forward(pars3_mlp *m, const float *X, int32_t rows, int32_t standardize, float *out,
                                          void *stream) {
  using namespace p3;
  if (!m || rows < 0 || (rows > 0 && (!X || !out))) return fail(PARS3_EINVAL, "mlp: bad forward arguments");
  if (rows == 0) return PARS3_OK;
  hipStream_t s = (hipStream_t)stream;
  P3_TRY(ensure_cap(m, rows));
  const int64_t q = (int64_t)rows * m->n_in;
  k_gather_std<<<g1(q), 256, 0, s>>>(X, nullptr, rows, m->n_in, standardize ? m->mean.p : nullptr, m->stdv.p,
                                     m->Xs.p);
  P3_LAUNCHED();
  P3_TRY(forward(m, rows, s));
  P3_HIP(hipMemcpyAsync(out, m->Out.p, (size_t)rows * m->n_out * sizeof(float), hipMemcpyDeviceToDevice, s));
  return PARS3_OK;
}

extern "C" pars3_status pars3_mlp_loss_grad(pars3_mlp *m, const float *X, const float *T, const float *M,
                                            int32_t rows, int32_t standardize, double *loss, void *stream) {
  using namespace p3;
  if (!m || rows < 1 || !X || !T || !M) return fail(PARS3_EINVAL, "mlp: bad loss_grad arguments");
  hipStream_t s = (hipStream_t)stream;
  P3_TRY(ensure_cap(m, rows));
  const int64_t qx = (int64_t)rows * m->n_in, qo = (int64_t)rows * m->n_out;
  k_gather_std<<<g1(qx), 256, 0, s>>>(X, nullptr, rows, m->n_in, standardize ? m->mean.p : nullptr, m->stdv.p,
                                      m->Xs.p);
  k_gather_std<<<g1(qo), 256, 0, s>>>(T, nullptr, rows, m->n_out, nullptr, nullptr, m->Ts.p);
  k_gather_std<<<g1(qo), 256, 0, s>>>(M, nullptr, rows, m->n_out, nullptr, nullptr, m->Ms.p);
  P3_LAUNCHED();
  P3_TRY(forward(m, rows, s));
  P3_TRY(backward(m, rows, s));
  if (loss) {
    P3_HIP(hipMemcpyAsync(loss, m->red.p, sizeof(double), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
  }
  return PARS3_OK;
}

extern "C" pars3_status pars3_mlp_adam(pars3_mlp *m, float lr, float beta1, float beta2, float eps, void *stream) {
  using namespace p3;
  if (!m) return fail(PARS3_EINVAL, "mlp: NULL handle");
  return adam(m, lr, beta1, beta2, eps, (hipStream_t)stream);
}

extern "C" pars3_status pars3_mlp_train(pars3_mlp *m, const float *X, const float *T, const float *M, int32_t rows,
                                        int32_t batch, int32_t epochs, float lr, uint64_t seed, double *loss_hist,
                                        void *stream) {
  using namespace p3;
  if (!m || rows < 1 || !X || !T || !M || batch < 1 || epochs < 0 || !(lr > 0.f))
    return fail(PARS3_EINVAL, "mlp: bad training arguments");
  hipStream_t s = (hipStream_t)stream;
  const int32_t b = std::min(batch, rows);
  P3_TRY(ensure_cap(m, b));
  dbuf<uint64_t> k0, k1;
  dbuf<uint32_t> v0, v1;
  dbuf<double> ep_loss;
  P3_HIP(k0.alloc(rows));
  P3_HIP(k1.alloc(rows));
  P3_HIP(v0.alloc(rows));
  P3_HIP(v1.alloc(rows));
  std::vector<double> hl;
  for (int32_t e = 0; e < epochs; e++) {
    k_shuffle_keys<<<g1(rows), 256, 0, s>>>(k0.p, v0.p, rows, seed * 0x9e3779b97f4a7c15ull + (uint64_t)e);
    P3_LAUNCHED();
    P3_TRY(radix_sort_pairs(k0.p, v0.p, k1.p, v1.p, rows, 32, s));
    double acc = 0.0;
    int32_t steps = 0;
    for (int32_t r0 = 0; r0 + b <= rows; r0 += b, steps++) {  // whole batches only
      const int32_t *idx = (const int32_t *)(v0.p + r0);
      k_gather_std<<<g1((int64_t)b * m->n_in), 256, 0, s>>>(X, idx, b, m->n_in, m->mean.p, m->stdv.p, m->Xs.p);
      k_gather_std<<<g1((int64_t)b * m->n_out), 256, 0, s>>>(T, idx, b, m->n_out, nullptr, nullptr, m->Ts.p);
      k_gather_std<<<g1((int64_t)b * m->n_out), 256, 0, s>>>(M, idx, b, m->n_out, nullptr, nullptr, m->Ms.p);
      P3_LAUNCHED();
      P3_TRY(forward(m, b, s));
      P3_TRY(backward(m, b, s));
      P3_TRY(adam(m, lr, 0.9f, 0.999f, 1e-8f, s));
      if (loss_hist) {
        double l = 0.0;
        P3_HIP(hipMemcpyAsync(&l, m->red.p, sizeof(double), hipMemcpyDeviceToHost, s));
        P3_HIP(hipStreamSynchronize(s));
        acc += l;
      }
    }
    if (loss_hist) loss_hist[e] = steps ? acc / steps : 0.0;
  }
  P3_HIP(hipStreamSynchronize(s));
  return PARS3_OK;
}

extern "C" pars3_status pars3_mlp_select_rows(pars3_mlp *m, const float *X, int32_t rows, const float *valid,
                                              int32_t *choice, void *stream) {
  using namespace p3;
  if (!m || rows < 0 || (rows > 0 && (!X || !choice))) return fail(PARS3_EINVAL, "mlp: bad select arguments");
  if (rows == 0) return PARS3_OK;
  hipStream_t s = (hipStream_t)stream;
  P3_TRY(ensure_cap(m, rows));
  const int64_t q = (int64_t)rows * m->n_in;
  k_gather_std<<<g1(q), 256, 0, s>>>(X, nullptr, rows, m->n_in, m->mean.p, m->stdv.p, m->Xs.p);
  P3_LAUNCHED();
  P3_TRY(forward(m, rows, s));
  k_argmin<<<g1(rows), 256, 0, s>>>(m->Out.p, valid, rows, m->n_out, choice);
  P3_LAUNCHED();
  return PARS3_OK;
}

// ------------------------------------------------------------ grid and files
namespace p3 {
const std::vector<pars3_split_params> &mlp_grid(const pars3_mlp *m) { return m->grid; }
}  // namespace p3

extern "C" pars3_status pars3_mlp_set_grid(pars3_mlp *m, const pars3_split_params *grid, int32_t ngrid) {
  if (!m || !grid) return fail(PARS3_EINVAL, "mlp: NULL argument");
  if (ngrid != m->n_out) return fail(PARS3_EINVAL, "mlp: the grid has %d entries, the network %d outputs", ngrid, m->n_out);
  m->grid.assign(grid, grid + ngrid);
  return PARS3_OK;
}

extern "C" pars3_status pars3_mlp_get_grid(const pars3_mlp *m, pars3_split_params *grid, int32_t cap, int32_t *count) {
  if (!m || !count) return fail(PARS3_EINVAL, "mlp: NULL argument");
  *count = (int32_t)m->grid.size();
  if (!grid) return PARS3_OK;
  if (cap < *count) return fail(PARS3_EINVAL, "mlp: grid capacity %d < %d", cap, *count);
  std::copy(m->grid.begin(), m->grid.end(), grid);
  return PARS3_OK;
}

// Model file: little-endian, in this order
//   char[8]  magic "PARS3MLP"
//   uint32   format version (2; version 1 files load too)
//   int32    n_in, h1, h2, n_out, ngrid (= n_out)
//   int32    ngrid x 7 split parameters (w_in, t_out, tile_rows, value_dtype,
//            keep_fp64, permute, engine); version 1: 6 of them, engine 0
//   float    n_in feature means, n_in feature standard deviations
//   float    n_params weights packed W1, b1, W2, b2, W3, b3
//   uint64   FNV-1a hash of every byte above
namespace {
constexpr char kMagic[8] = {'P', 'A', 'R', 'S', '3', 'M', 'L', 'P'};
constexpr uint32_t kVersion = 2;

struct fnv_writer {
  FILE *f;
  uint64_t h = 1469598103934665603ull;
  bool ok = true;
  void put(const void *p, size_t bytes) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < bytes; i++) h = (h ^ c[i]) * 1099511628211ull;
    ok = ok && fwrite(p, 1, bytes, f) == bytes;
  }
};
struct fnv_reader {
  FILE *f;
  uint64_t h = 1469598103934665603ull;
  bool ok = true;
  void get(void *p, size_t bytes) {
    ok = ok && fread(p, 1, bytes, f) == bytes;
    if (!ok) return;
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < bytes; i++) h = (h ^ c[i]) * 1099511628211ull;
  }
};
}  // namespace

extern "C" pars3_status pars3_model_save(const pars3_mlp *m, const char *path) {
  if (!m || !path) return fail(PARS3_EINVAL, "model_save: NULL argument");
  if ((int32_t)m->grid.size() != m->n_out)
    return fail(PARS3_ESTATE, "model_save: the network has no configuration grid (pars3_mlp_set_grid)");
  std::vector<float> P(m->np), mean(m->n_in), stdv(m->n_in);
  P3_TRY(copy_host(P.data(), m->P.p, m->np * sizeof(float), hipMemcpyDeviceToHost));
  P3_TRY(copy_host(mean.data(), m->mean.p, m->n_in * sizeof(float), hipMemcpyDeviceToHost));
  P3_TRY(copy_host(stdv.data(), m->stdv.p, m->n_in * sizeof(float), hipMemcpyDeviceToHost));
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(PARS3_EIO, "model_save: cannot open %s for writing", path);
  fnv_writer w{f};
  w.put(kMagic, 8);
  w.put(&kVersion, 4);
  const int32_t hdr[5] = {m->n_in, m->h1, m->h2, m->n_out, (int32_t)m->grid.size()};
  w.put(hdr, sizeof(hdr));
  for (const pars3_split_params &g : m->grid) {
    const int32_t v[7] = {g.w_in, g.t_out, g.tile_rows, g.value_dtype, g.keep_fp64, g.permute, g.engine};
    w.put(v, sizeof(v));
  }
  w.put(mean.data(), mean.size() * sizeof(float));
  w.put(stdv.data(), stdv.size() * sizeof(float));
  w.put(P.data(), P.size() * sizeof(float));
  const uint64_t h = w.h;
  const bool ok = w.ok && std::fwrite(&h, 1, 8, f) == 8;
  if (std::fclose(f) != 0 || !ok) return fail(PARS3_EIO, "model_save: write to %s failed", path);
  return PARS3_OK;
}

extern "C" pars3_status pars3_model_load(const char *path, pars3_mlp **out) {
  if (!path || !out) return fail(PARS3_EINVAL, "model_load: NULL argument");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(PARS3_EIO, "model_load: cannot open %s", path);
  fnv_reader r{f};
  char magic[8];
  uint32_t ver = 0;
  int32_t hdr[5] = {0, 0, 0, 0, 0};
  r.get(magic, 8);
  r.get(&ver, 4);
  r.get(hdr, sizeof(hdr));
  auto bad = [&](const char *what) {
    std::fclose(f);
    return fail(PARS3_EIO, "model_load: %s: %s", path, what);
  };
  if (!r.ok) return bad("truncated header");
  if (std::memcmp(magic, kMagic, 8) != 0) return bad("not a model file");
  if (ver != 1 && ver != kVersion) return bad("unknown format version");
  for (int k = 0; k < 4; k++)
    if (hdr[k] < 1 || hdr[k] > 4096) return bad("layer size out of range");
  if (hdr[4] != hdr[3]) return bad("grid size differs from the output count");
  std::vector<pars3_split_params> grid(hdr[4]);
  const size_t nfield = ver == 1 ? 6 : 7;
  for (auto &g : grid) {
    int32_t v[7] = {0, 0, 0, 0, 0, 0, PARS3_ENGINE_TILES};
    r.get(v, nfield * sizeof(int32_t));
    g.w_in = v[0];
    g.t_out = v[1];
    g.tile_rows = v[2];
    g.value_dtype = v[3];
    g.keep_fp64 = v[4];
    g.permute = v[5];
    g.engine = v[6];
  }
  const int64_t np = (int64_t)hdr[0] * hdr[1] + hdr[1] + (int64_t)hdr[1] * hdr[2] + hdr[2] +
                     (int64_t)hdr[2] * hdr[3] + hdr[3];
  std::vector<float> mean(hdr[0]), stdv(hdr[0]), P(np);
  r.get(mean.data(), mean.size() * sizeof(float));
  r.get(stdv.data(), stdv.size() * sizeof(float));
  r.get(P.data(), P.size() * sizeof(float));
  const uint64_t want = r.h;
  uint64_t got = 0;
  const bool tail = r.ok && std::fread(&got, 1, 8, f) == 8;
  char extra;
  const bool at_end = std::fread(&extra, 1, 1, f) == 0;
  std::fclose(f);
  if (!r.ok || !tail) return fail(PARS3_EIO, "model_load: %s: truncated", path);
  if (got != want) return fail(PARS3_EIO, "model_load: %s: checksum mismatch", path);
  if (!at_end) return fail(PARS3_EIO, "model_load: %s: trailing bytes", path);
  pars3_mlp *m = nullptr;
  P3_TRY(pars3_mlp_create(hdr[0], hdr[1], hdr[2], hdr[3], 1, &m));
  pars3_status st = pars3_mlp_set_params(m, P.data());
  if (st == PARS3_OK) st = pars3_mlp_set_scaler(m, mean.data(), stdv.data());
  if (st == PARS3_OK) st = pars3_mlp_set_grid(m, grid.data(), (int32_t)grid.size());
  if (st != PARS3_OK) {
    pars3_mlp_destroy(m);
    return st;
  }
  *out = m;
  return PARS3_OK;
}
