// Sparsity features of the reordered lower triangle (the band profile,
// distance-from-diagonal spread and row-length mix that Section 3.1.2 reads
// off the structure plots to choose the split; here as 32 numbers that feed
// the configuration selector).  Every feature is a ratio of integer counts;
// the counts are taken on the GPU, the ratios formed on the host in FP64.
//
// Definitions (row lower bandwidth b_i = i - first column of row i, 0 for an
// empty row; d = i - j per entry; beta = max d; l_i = row length):
//  f0 log2 n, f1 log2 nnz, f2 nnz/n, f3 beta/n, f4 log2(beta+1),
//  f5..f9 nearest-rank quantiles p10, p50, p90, p99 and the max of b_i over
//  beta, f10 nnz / sum b_i, f11..f18 share of entries with d <= 2^k (k=0..7),
//  f19..f21 share with d/beta > 1/2, 3/4, 9/10, f22..f28 share of rows with
//  length 0, 1, 2, 3-4, 5-8, 9-16, >= 17, f29 max l / mean l, f30 std(l) /
//  mean(l) (population), f31 share of 256-row tiles whose window
//  (tile end - smallest column in the tile) fits 160 KiB of FP64 x and y.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace p3 {

static constexpr int FB = 256;  // one workgroup = one 256-row tile in the row pass

struct feat_counts {
  unsigned long long sumb, maxl, s1, s2, beta, fit;
  unsigned long long lenh[7], dle[8], dfar[3];
};

template <class T>
__device__ __forceinline__ T block_sum(T v, T *red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = 0;
  for (int w = 0; w < FB / 64; w++) t += red[w];
  return t;
}
template <class T>
__device__ __forceinline__ T block_max(T v, T *red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = red[0];
  for (int w = 1; w < FB / 64; w++) t = red[w] > t ? red[w] : t;
  return t;
}

// Row pass: b_i (also as sort key), sums, length histogram, beta, and the
// tile window test (this workgroup's 256 rows are one tile).
__global__ __launch_bounds__(FB) void k_feat_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                  int32_t n, feat_counts *__restrict__ fc,
                                                  uint64_t *__restrict__ bkey) {
  __shared__ unsigned long long red[FB / 64];
  const int32_t i = blockIdx.x * FB + threadIdx.x;
  unsigned long long l = 0, b = 0, lo = (unsigned long long)blockIdx.x * FB;
  if (i < n) {
    l = (unsigned long long)(rp[i + 1] - rp[i]);
    if (l > 0) {
      const int32_t c0 = col[rp[i]];
      b = (unsigned long long)(i - c0);
      lo = (unsigned long long)c0;
    }
    bkey[i] = b;
  }
  const int h = l == 0 ? 0 : l == 1 ? 1 : l == 2 ? 2 : l <= 4 ? 3 : l <= 8 ? 4 : l <= 16 ? 5 : 6;
  const unsigned long long sumb = block_sum<unsigned long long>(b, red);
  const unsigned long long s1 = block_sum<unsigned long long>(l, red);
  const unsigned long long s2 = block_sum<unsigned long long>(l * l, red);
  const unsigned long long maxl = block_max<unsigned long long>(l, red);
  const unsigned long long mb = block_max<unsigned long long>(b, red);
  // smallest column of the tile: the max of (tile start - first column)
  const unsigned long long t0 = (unsigned long long)blockIdx.x * FB;
  const unsigned long long reach = block_max<unsigned long long>(t0 - (lo < t0 ? lo : t0), red);
  unsigned long long hc[7];
  for (int k = 0; k < 7; k++) hc[k] = block_sum<unsigned long long>(i < n && h == k ? 1ull : 0ull, red);
  if (threadIdx.x == 0) {
    atomicAdd(&fc->sumb, sumb);
    atomicAdd(&fc->s1, s1);
    atomicAdd(&fc->s2, s2);
    atomicMax(&fc->maxl, maxl);
    atomicMax(&fc->beta, mb);
    const unsigned long long r1 = min((unsigned long long)n, t0 + FB);
    const unsigned long long lo_t = t0 - reach;
    if ((r1 - lo_t) * 16ull <= 160ull * 1024ull) atomicAdd(&fc->fit, 1ull);
    for (int k = 0; k < 7; k++)
      if (hc[k]) atomicAdd(&fc->lenh[k], hc[k]);
  }
}

// Entry pass: distance thresholds (needs beta from the row pass).
__global__ __launch_bounds__(FB) void k_feat_entries(const int32_t *__restrict__ erow, const int32_t *__restrict__ col,
                                                     int64_t nnz, feat_counts *__restrict__ fc) {
  __shared__ unsigned long long red[FB / 64];
  const unsigned long long beta = fc->beta;
  unsigned long long c[11];
  for (int k = 0; k < 11; k++) c[k] = 0;
  for (int64_t e = (int64_t)blockIdx.x * FB + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * FB) {
    const unsigned long long d = (unsigned long long)(erow[e] - col[e]);
    for (int k = 0; k < 8; k++) c[k] += d <= (1ull << k) ? 1ull : 0ull;
    c[8] += 2 * d > beta ? 1ull : 0ull;
    c[9] += 4 * d > 3 * beta ? 1ull : 0ull;
    c[10] += 10 * d > 9 * beta ? 1ull : 0ull;
  }
  for (int k = 0; k < 11; k++) {
    const unsigned long long s = block_sum<unsigned long long>(c[k], red);
    if (threadIdx.x == 0 && s) atomicAdd(k < 8 ? &fc->dle[k] : &fc->dfar[k - 8], s);
  }
}

__global__ void k_row_of_entry(const int32_t *__restrict__ rp, int32_t n, int32_t *__restrict__ erow) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = rp[i]; e < rp[i + 1]; e++) erow[e] = i;
}

}  // namespace p3

using p3::fail;

extern "C" pars3_status pars3_features(const pars3_matrix *A, double *f, void *stream) {
  using namespace p3;
  if (!A || !f) return fail(PARS3_EINVAL, "features: NULL argument");
  if (!A->perm_done) return fail(PARS3_ESTATE, "features: call pars3_reorder first");
  for (int k = 0; k < 32; k++) f[k] = 0.0;
  const int32_t n = (int32_t)A->n;
  const int64_t nnz = A->nnz;
  if (n <= 0) return PARS3_OK;
  hipStream_t s = (hipStream_t)stream;
  dbuf<feat_counts> dfc;
  dbuf<uint64_t> k0, k1;
  dbuf<uint32_t> v0, v1;
  dbuf<int32_t> erow;
  P3_HIP(dfc.alloc(1));
  P3_HIP(k0.alloc(n));
  P3_HIP(k1.alloc(n));
  P3_HIP(v0.alloc(n));
  P3_HIP(v1.alloc(n));
  P3_HIP(erow.alloc(std::max<int64_t>(nnz, 1)));
  P3_HIP(hipMemsetAsync(dfc.p, 0, sizeof(feat_counts), s));
  const unsigned ntile = (unsigned)cdiv(n, FB);
  k_feat_rows<<<ntile, FB, 0, s>>>(A->prow.p, A->pcol.p, n, dfc.p, k0.p);
  P3_LAUNCHED();
  if (nnz > 0) {
    k_row_of_entry<<<ntile, FB, 0, s>>>(A->prow.p, n, erow.p);
    P3_LAUNCHED();
    const unsigned g = (unsigned)std::min<int64_t>(cdiv(nnz, FB), 8192);
    k_feat_entries<<<g, FB, 0, s>>>(erow.p, A->pcol.p, nnz, dfc.p);
    P3_LAUNCHED();
  }
  // nearest-rank quantiles of b_i: sort the keys (the payload is unused)
  P3_TRY(iota_i32((int32_t *)v0.p, n, s));
  P3_TRY(radix_sort_pairs(k0.p, v0.p, k1.p, v1.p, n, 32, s));
  feat_counts h{};
  P3_HIP(hipMemcpyAsync(&h, dfc.p, sizeof(h), hipMemcpyDeviceToHost, s));
  const int64_t pct[4] = {10, 50, 90, 99};
  uint64_t q[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < 4; k++) {
    const int64_t rank = (pct[k] * (int64_t)n + 99) / 100;
    P3_HIP(hipMemcpyAsync(&q[k], k0.p + rank - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  }
  P3_HIP(hipMemcpyAsync(&q[4], k0.p + n - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  // ratios, in the order and precision of the definitions above
  const double dn = (double)n;
  const int64_t beta = (int64_t)h.beta;
  f[0] = std::log2(dn);
  f[1] = nnz > 0 ? std::log2((double)nnz) : 0.0;
  f[2] = (double)nnz / dn;
  f[3] = (double)beta / dn;
  f[4] = std::log2((double)(beta + 1));
  if (beta > 0) {
    for (int k = 0; k < 5; k++) f[5 + k] = (double)q[k] / (double)beta;
  }
  f[10] = h.sumb > 0 ? (double)nnz / (double)h.sumb : 0.0;
  if (nnz > 0) {
    for (int k = 0; k < 8; k++) f[11 + k] = (double)h.dle[k] / (double)nnz;
    for (int k = 0; k < 3; k++) f[19 + k] = (double)h.dfar[k] / (double)nnz;
  }
  for (int k = 0; k < 7; k++) f[22 + k] = (double)h.lenh[k] / dn;
  const int64_t s1 = (int64_t)h.s1, s2 = (int64_t)h.s2, maxl = (int64_t)h.maxl;
  if (s1 > 0) {
    f[29] = (double)(maxl * (int64_t)n) / (double)s1;
    f[30] = std::sqrt((double)((int64_t)n * s2 - s1 * s1)) / (double)s1;
  }
  f[31] = (double)h.fit / (double)cdiv(n, 256);
  return PARS3_OK;
}
