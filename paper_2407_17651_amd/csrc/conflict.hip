// Conflict map of a block-row distribution (Section 3, Fig. 2).  Block p owns
// rows [R_p, R_{p+1}) of the reordered matrix and the stored lower entries of
// those rows.  An entry (i, j) is safe (R1) when j >= R_p: both products stay
// in the block's outputs; it is conflicting (R2) when j < R_p: its transposed
// product writes y_j of an earlier block and it reads x_j from there.  The
// paper finds these before iterating, by a pass over the stored triangle that
// compares column indices with the owner's range; here that pass runs on the
// GPU and also counts, per block, the distinct columns it touches outside
// itself (the halo of x values it receives and of partial sums it returns)
// and the distinct blocks that own them.
//
// Pass 1, one thread per row: safe and conflicting entries per split part,
// the smallest conflicting column, and the row's number of conflicting
// entries.  Pass 2 writes one key (block, column) per conflicting entry; the
// keys are radix-sorted and pass 3 counts the distinct keys (halo) and the
// distinct owners of their columns (partners) per block.
#include <algorithm>
#include <climits>
#include <vector>

#include "internal.h"

namespace p3 {

static constexpr int TB = 256;
static inline unsigned nblk(int64_t m) { return (unsigned)std::max<int64_t>(1, cdiv(m, TB)); }

// The block owning row i: the largest p with R[p] <= i (empty blocks, where
// R[p] == R[p + 1], are skipped by taking the largest).
__device__ __forceinline__ int32_t owner_of(const int64_t *__restrict__ R, int32_t nb, int64_t i) {
  int32_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (R[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_cf_rows(const int32_t *__restrict__ prow, const int32_t *__restrict__ pcol,
                          const int8_t *__restrict__ part, int32_t n, const int64_t *__restrict__ R, int32_t nb,
                          unsigned long long *__restrict__ cnt, int32_t *__restrict__ reach,
                          int32_t *__restrict__ nconf) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < n;
  int32_t p = 0, mn = INT_MAX, tot = 0;
  unsigned long long c[6] = {0, 0, 0, 0, 0, 0};
  if (ok) {
    p = owner_of(R, nb, i);
    const int64_t lo = R[p];
    for (int32_t e = prow[i]; e < prow[i + 1]; e++) {
      const int32_t j = pcol[e];
      const int k = part[e];
      if (j >= lo) {
        c[k]++;
      } else {
        c[3 + k]++;
        mn = min(mn, j);
        tot++;
      }
    }
    nconf[i] = tot;
  }
#pragma unroll
  for (int k = 0; k < 6; k++) agg_atomic_add<unsigned long long>(cnt, (int64_t)p * 6 + k, c[k], ok && c[k] != 0);
  agg_atomic_min<int32_t>(reach, p, mn, ok && tot > 0, INT_MAX);
}

__global__ void k_cf_keys(const int32_t *__restrict__ prow, const int32_t *__restrict__ pcol, int32_t n,
                          const int64_t *__restrict__ R, int32_t nb, const int32_t *__restrict__ off, int bj,
                          uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t p = owner_of(R, nb, i);
  const int64_t lo = R[p];
  int32_t w = off[i];
  for (int32_t e = prow[i]; e < prow[i + 1]; e++) {
    const int32_t j = pcol[e];
    if (j < lo) {
      keys[w] = ((uint64_t)p << bj) | (uint64_t)j;
      vals[w] = 0u;
      w++;
    }
  }
}

__global__ void k_cf_unique(const uint64_t *__restrict__ keys, int64_t m, int bj, const int64_t *__restrict__ R,
                            int32_t nb, unsigned long long *__restrict__ halo,
                            unsigned long long *__restrict__ partners) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = t < m;
  const uint64_t mask = (1ull << bj) - 1ull;
  int32_t p = 0;
  bool new_col = false, new_owner = false;
  if (ok) {
    const uint64_t k = keys[t];
    p = (int32_t)(k >> bj);
    const int32_t q = owner_of(R, nb, (int64_t)(k & mask));
    if (t == 0 || (keys[t - 1] >> bj) != (uint64_t)p) {
      new_col = new_owner = true;
    } else {
      new_col = keys[t - 1] != k;
      new_owner = owner_of(R, nb, (int64_t)(keys[t - 1] & mask)) != q;
    }
  }
  agg_atomic_add<unsigned long long>(halo, p, 1ull, ok && new_col);
  agg_atomic_add<unsigned long long>(partners, p, 1ull, ok && new_owner);
}

}  // namespace p3

using p3::fail;

extern "C" pars3_status pars3_conflict_map(const pars3_matrix *A, int32_t nblocks, const int64_t *bounds,
                                           pars3_block_conflicts *out, void *stream) {
  using namespace p3;
  if (!A || !out) return fail(PARS3_EINVAL, "conflict_map: NULL argument");
  if (!A->split_done) return fail(PARS3_ESTATE, "conflict_map: call pars3_reorder first");
  if (nblocks < 1) return fail(PARS3_EINVAL, "conflict_map: nblocks must be >= 1");
  const int32_t n = (int32_t)A->n;
  const int32_t nb = nblocks;
  std::vector<int64_t> R((size_t)nb + 1);
  for (int32_t p = 0; p <= nb; p++) R[p] = bounds ? bounds[p] : ((int64_t)p * n) / nb;
  if (R[0] != 0 || R[nb] != n) return fail(PARS3_EINVAL, "conflict_map: bounds must run from 0 to n");
  for (int32_t p = 0; p < nb; p++)
    if (R[p + 1] < R[p]) return fail(PARS3_EINVAL, "conflict_map: bounds decrease at block %d", p);
  hipStream_t s = (hipStream_t)stream;
  P3_HIP(hipSetDevice(A->device));
  dbuf<int64_t> dR;
  dbuf<unsigned long long> cnt, halo, partners;
  dbuf<int32_t> reach, nconf, off;
  P3_HIP(dR.alloc(nb + 1));
  P3_HIP(cnt.alloc((size_t)nb * 6));
  P3_HIP(halo.alloc(nb));
  P3_HIP(partners.alloc(nb));
  P3_HIP(reach.alloc(nb));
  P3_HIP(nconf.alloc(n));
  P3_HIP(off.alloc((size_t)n + 1));
  P3_HIP(hipMemcpyAsync(dR.p, R.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  P3_TRY(fill_u64((uint64_t *)cnt.p, 0, (int64_t)nb * 6, s));
  P3_TRY(fill_u64((uint64_t *)halo.p, 0, nb, s));
  P3_TRY(fill_u64((uint64_t *)partners.p, 0, nb, s));
  P3_TRY(fill_i32(reach.p, INT_MAX, nb, s));
  int64_t m = 0;
  if (n > 0) {
    k_cf_rows<<<nblk(n), TB, 0, s>>>(A->prow.p, A->pcol.p, A->part.p, n, dR.p, nb, cnt.p, reach.p, nconf.p);
    P3_LAUNCHED();
    P3_TRY(scan_i32(nconf.p, off.p, n, s));
    int32_t total = 0;
    P3_HIP(hipMemcpyAsync(&total, off.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
    m = total;
  }
  if (m > 0) {
    const int bj = std::max(1, bits_for((uint64_t)(n - 1)));
    const int key_bits = bj + bits_for((uint64_t)(nb - 1));
    dbuf<uint64_t> k0, k1;
    dbuf<uint32_t> v0, v1;
    P3_HIP(k0.alloc(m));
    P3_HIP(k1.alloc(m));
    P3_HIP(v0.alloc(m));
    P3_HIP(v1.alloc(m));
    k_cf_keys<<<nblk(n), TB, 0, s>>>(A->prow.p, A->pcol.p, n, dR.p, nb, off.p, bj, k0.p, v0.p);
    P3_LAUNCHED();
    P3_TRY(radix_sort_pairs(k0.p, v0.p, k1.p, v1.p, m, key_bits, s));
    k_cf_unique<<<nblk(m), TB, 0, s>>>(k0.p, m, bj, dR.p, nb, halo.p, partners.p);
    P3_LAUNCHED();
    P3_HIP(hipStreamSynchronize(s));
  }
  std::vector<unsigned long long> hc((size_t)nb * 6), hh(nb), hp(nb);
  std::vector<int32_t> hr(nb);
  P3_HIP(hipMemcpyAsync(hc.data(), cnt.p, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  P3_HIP(hipMemcpyAsync(hh.data(), halo.p, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  P3_HIP(hipMemcpyAsync(hp.data(), partners.p, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  P3_HIP(hipMemcpyAsync(hr.data(), reach.p, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  for (int32_t p = 0; p < nb; p++) {
    pars3_block_conflicts &o = out[p];
    o.first_row = R[p];
    o.rows = R[p + 1] - R[p];
    for (int k = 0; k < 3; k++) {
      o.safe[k] = (int64_t)hc[(size_t)p * 6 + k];
      o.conflict[k] = (int64_t)hc[(size_t)p * 6 + 3 + k];
    }
    o.reach = hr[p] == INT_MAX ? R[p] : hr[p];
    o.partners = (int64_t)hp[p];
    o.halo = (int64_t)hh[p];
  }
  return PARS3_OK;
}

extern "C" pars3_status pars3_conflict_features(const pars3_matrix *A, int32_t nblocks, double *feat3, void *stream) {
  using namespace p3;
  if (!A || !feat3) return fail(PARS3_EINVAL, "conflict_features: NULL argument");
  if (nblocks < 1) return fail(PARS3_EINVAL, "conflict_features: nblocks must be >= 1");
  std::vector<pars3_block_conflicts> blk((size_t)nblocks);
  P3_TRY(pars3_conflict_map(A, nblocks, nullptr, blk.data(), stream));
  int64_t conf = 0;
  double halo = 0.0, reach = 0.0;
  for (const pars3_block_conflicts &o : blk) {
    conf += o.conflict[0] + o.conflict[1] + o.conflict[2];
    const int64_t rows = o.rows > 0 ? o.rows : 1;
    halo = std::max(halo, (double)o.halo / (double)rows);
    reach = std::max(reach, (double)(o.first_row - o.reach) / (double)rows);
  }
  feat3[0] = A->nnz > 0 ? (double)conf / (double)A->nnz : 0.0;
  feat3[1] = halo;
  feat3[2] = reach;
  return PARS3_OK;
}
