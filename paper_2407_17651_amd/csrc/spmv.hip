// Skew-symmetric product y = shift*x + S*x, S = L - L^T, from the stored
// lower triangle only: every stored l_ij is read once and gives the two
// products y_i += l_ij x_j and y_j -= l_ij x_i (eqs. (2)-(6), Section 3.1.2).
//
// Launch sequence on one stream (each kernel's writes are visible to the next):
//  1. k_inner : one thread per row.  y_i = shift*x_i plus the whole inner-band
//     contribution, gathered from the diagonal-major band in both directions
//     (the row's own entries and the entries of the rows below that store
//     column i), so no atomics are needed.  This is the only writer of y that
//     does not add, so it also initialises y.
//  2. k_tiles : one workgroup per tile of T rows.  The tile's entries are
//     prefetched into registers, then the x values of the tile's rows and of
//     its back window are staged in LDS; both products of every middle entry
//     accumulate into LDS (ds_add); the tile then adds its LDS sums to y with
//     one global atomic per touched row (consecutive addresses).  Extra
//     workgroups of the same launch take the coordinate list (the outer part
//     and middle entries outside any window), both products by global atomics.
// Values are FP64, FP32 or BF16; vectors and accumulation are FP64 for FP64
// values and FP32 otherwise.  k right-hand sides are stored row-major.
#include <algorithm>

#include "internal.h"

namespace p3 {

static constexpr int TB = 256;
static constexpr int LDS_MAX = 160 * 1024;

template <class V>
struct vload;
template <>
struct vload<double> {
  static __device__ __forceinline__ double get(const double *p, int64_t i) { return __builtin_nontemporal_load(p + i); }
};
template <>
struct vload<float> {
  static __device__ __forceinline__ float get(const float *p, int64_t i) { return __builtin_nontemporal_load(p + i); }
};
template <>
struct vload<uint16_t> {
  static __device__ __forceinline__ float get(const uint16_t *p, int64_t i) {
    return __uint_as_float((uint32_t)__builtin_nontemporal_load(p + i) << 16);
  }
};

template <class V, class X, int K>
__global__ __launch_bounds__(TB) void k_inner(const V *__restrict__ dia, int32_t w_in, int32_t n, X shift,
                                              const X *__restrict__ x, X *__restrict__ y) {
  const int32_t i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  X acc[K];
#pragma unroll
  for (int c = 0; c < K; c++) acc[c] = shift * x[(int64_t)i * K + c];
  for (int32_t k = 1; k <= w_in; k++) {
    const int64_t base = (int64_t)(k - 1) * n;
    if (i - k >= 0) {
      X l = (X)vload<V>::get(dia, base + i);
      if (l != (X)0) {
#pragma unroll
        for (int c = 0; c < K; c++) acc[c] += l * x[(int64_t)(i - k) * K + c];
      }
    }
    if (i + k < n) {
      X l = (X)vload<V>::get(dia, base + i + k);
      if (l != (X)0) {
#pragma unroll
        for (int c = 0; c < K; c++) acc[c] -= l * x[(int64_t)(i + k) * K + c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < K; c++) y[(int64_t)i * K + c] = acc[c];
}

// Entries prefetched into registers per thread before the x window is staged,
// so that the matrix stream is in flight while the window loads.
static constexpr int PRE = 4;
// Coordinate-list entries per thread in the extra workgroups of the launch.
static constexpr int FAR_ITEMS = 8;

template <class X, int K>
__device__ __forceinline__ void tile_entry(uint32_t rc, X v, int32_t la, const X *xs, X *ys) {
  const int32_t si = la + (int32_t)(rc >> 16), sj = (int32_t)(rc & 0xffffu);
#pragma unroll
  for (int c = 0; c < K; c++) {
    const X xi = xs[si * K + c], xj = xs[sj * K + c];
    atomicAdd(&ys[si * K + c], v * xj);
    atomicAdd(&ys[sj * K + c], -(v * xi));
  }
}

// Workgroups [0, tile_grid) process tiles; the remaining ones process the
// coordinate list, FAR_ITEMS entries per thread.
template <class V, class X, int K>
__global__ __launch_bounds__(TB) void k_tiles(const int32_t *__restrict__ tile_ptr, const int32_t *__restrict__ tile_alo,
                                              const int32_t *__restrict__ tile_la, const uint32_t *__restrict__ ent_rc,
                                              const V *__restrict__ ent_v, int32_t ntiles, int32_t T, int32_t n,
                                              int32_t tile_grid, const int32_t *__restrict__ far_row,
                                              const int32_t *__restrict__ far_col, const V *__restrict__ far_v,
                                              int64_t nfar, const X *__restrict__ x, X *__restrict__ y) {
  extern __shared__ unsigned char smem[];
  const int32_t b = blockIdx.x;
  if (b >= tile_grid) {
    const int64_t base = (int64_t)(b - tile_grid) * TB * FAR_ITEMS + threadIdx.x;
#pragma unroll
    for (int q = 0; q < FAR_ITEMS; q++) {
      const int64_t e = base + (int64_t)q * TB;
      if (e >= nfar) break;
      const int32_t i = far_row[e], j = far_col[e];
      const X v = (X)vload<V>::get(far_v, e);
#pragma unroll
      for (int c = 0; c < K; c++) {
        const X xi = x[(int64_t)i * K + c], xj = x[(int64_t)j * K + c];
        unsafeAtomicAdd(&y[(int64_t)i * K + c], v * xj);
        unsafeAtomicAdd(&y[(int64_t)j * K + c], -(v * xi));
      }
    }
    return;
  }
  // Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
  // contiguous range of tiles so that its L2 keeps the x and y lines that the
  // back windows of its later tiles revisit.
  const int32_t per = (ntiles + 7) >> 3;
  const int32_t t = (b & 7) * per + (b >> 3);
  if (t >= ntiles) return;
  const int32_t e0 = tile_ptr[t], e1 = tile_ptr[t + 1];
  if (e0 == e1) return;
  uint32_t prc[PRE];
  X pv[PRE];
#pragma unroll
  for (int q = 0; q < PRE; q++) {
    const int32_t e = e0 + threadIdx.x + q * TB;
    prc[q] = 0u;
    pv[q] = (X)0;
    if (e < e1) {
      prc[q] = __builtin_nontemporal_load(ent_rc + e);
      pv[q] = (X)vload<V>::get(ent_v, e);
    }
  }
  const int32_t la = tile_la[t], alo = tile_alo[t], r0 = t * T;
  const int32_t nslot = la + T;
  X *xs = reinterpret_cast<X *>(smem);
  X *ys = xs + (int64_t)nslot * K;
  for (int32_t s = threadIdx.x; s < nslot; s += TB) {
    const int32_t row = s < la ? alo + s : r0 + (s - la);
#pragma unroll
    for (int c = 0; c < K; c++) {
      xs[s * K + c] = row < n ? x[(int64_t)row * K + c] : (X)0;
      ys[s * K + c] = (X)0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PRE; q++)
    if (e0 + (int32_t)threadIdx.x + q * TB < e1) tile_entry<X, K>(prc[q], pv[q], la, xs, ys);
  for (int32_t e = e0 + threadIdx.x + PRE * TB; e < e1; e += TB)
    tile_entry<X, K>(__builtin_nontemporal_load(ent_rc + e), (X)vload<V>::get(ent_v, e), la, xs, ys);
  __syncthreads();
  for (int32_t s = threadIdx.x; s < nslot; s += TB) {
    const int32_t row = s < la ? alo + s : r0 + (s - la);
    if (row >= n) continue;
#pragma unroll
    for (int c = 0; c < K; c++) {
      const X a = ys[s * K + c];
      if (a != (X)0) unsafeAtomicAdd(&y[(int64_t)row * K + c], a);
    }
  }
}

template <class V, class X, int K>
static pars3_status launch(pars3_matrix *A, const V *in_v, const V *ent_v, const V *far_v, X shift, const X *x, X *y,
                           hipStream_t s) {
  const layout &L = A->lay;
  const int32_t n = (int32_t)A->n;
  if (n == 0) return PARS3_OK;
  P3_TRY(prof_mark(A, PROF_INNER, 0, s));
  k_inner<V, X, K><<<(unsigned)cdiv(n, TB), TB, 0, s>>>(in_v, L.w_in, n, shift, x, y);
  P3_LAUNCHED();
  P3_TRY(prof_mark(A, PROF_INNER, 1, s));
  if (L.nnz_tiled + L.nnz_far > 0) {
    const size_t lds = L.nnz_tiled > 0 ? (size_t)L.max_slots * K * 2 * sizeof(X) : 0;
    if (lds > (size_t)LDS_MAX)
      return fail(PARS3_EINVAL, "spmv: a tile needs %zu bytes of LDS for k=%d; reorder with a smaller window_max", lds,
                  K);
    static bool attr_set = false;
    if (!attr_set) {
      P3_HIP(hipFuncSetAttribute((const void *)k_tiles<V, X, K>, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX));
      attr_set = true;
    }
    const int32_t tile_grid = L.nnz_tiled > 0 ? (int32_t)(8 * cdiv(L.ntiles, 8)) : 0;
    const int64_t far_grid = cdiv(L.nnz_far, (int64_t)TB * FAR_ITEMS);
    P3_TRY(prof_mark(A, PROF_TILES, 0, s));
    k_tiles<V, X, K><<<(unsigned)(tile_grid + far_grid), TB, lds, s>>>(
        L.tile_ptr.p, L.tile_alo.p, L.tile_la.p, L.ent_rc.p, ent_v, L.ntiles, L.T, n, tile_grid, L.far_row.p,
        L.far_col.p, far_v, L.nnz_far, x, y);
    P3_LAUNCHED();
    P3_TRY(prof_mark(A, PROF_TILES, 1, s));
  }
  return PARS3_OK;
}

template <class V, class X>
static pars3_status dispatch_k(pars3_matrix *A, const V *in_v, const V *ent_v, const V *far_v, double shift,
                               const void *x, void *y, int k, hipStream_t s) {
  const X *xx = (const X *)x;
  X *yy = (X *)y;
  switch (k) {
    case 1: return launch<V, X, 1>(A, in_v, ent_v, far_v, (X)shift, xx, yy, s);
    case 2: return launch<V, X, 2>(A, in_v, ent_v, far_v, (X)shift, xx, yy, s);
    case 4: return launch<V, X, 4>(A, in_v, ent_v, far_v, (X)shift, xx, yy, s);
    case 8: return launch<V, X, 8>(A, in_v, ent_v, far_v, (X)shift, xx, yy, s);
    default: return fail(PARS3_EINVAL, "spmv: k must be 1, 2, 4 or 8 (got %d)", k);
  }
}

static constexpr int PROF_MAX = 4096;

pars3_status prof_mark(pars3_matrix *A, int cls, int stop, hipStream_t s) {
  auto &P = A->prof;
  if (!P.on) return PARS3_OK;
  int q = P.used[cls];
  if (q >= PROF_MAX) return PARS3_OK;
  auto &ev = P.ev[cls];
  if ((int)ev.size() < 2 * (q + 1)) {
    hipEvent_t a, b;
    P3_HIP(hipEventCreate(&a));
    P3_HIP(hipEventCreate(&b));
    ev.push_back(a);
    ev.push_back(b);
  }
  P3_HIP(hipEventRecord(ev[2 * q + stop], s));
  if (stop) P.used[cls] = q + 1;
  return PARS3_OK;
}

pars3_status spmv_rcm(pars3_matrix *A, double shift, const void *x, void *y, int k, int vec_dtype, hipStream_t s) {
  const layout &L = A->lay;
  if (A->prof.on && A->prof.calls < PROF_MAX) A->prof.calls++;
  if (vec_dtype == PARS3_F64) {
    if (!A->has_f64) return fail(PARS3_ESTATE, "spmv: FP64 values are not stored (value_dtype/keep_fp64)");
    return dispatch_k<double, double>(A, L.in_f64.p, L.ent_f64.p, L.far_f64.p, shift, x, y, k, s);
  }
  if (vec_dtype == PARS3_F32) {
    if (A->has_f32) return dispatch_k<float, float>(A, L.in_f32.p, L.ent_f32.p, L.far_f32.p, shift, x, y, k, s);
    if (A->has_bf16)
      return dispatch_k<uint16_t, float>(A, L.in_bf16.p, L.ent_bf16.p, L.far_bf16.p, shift, x, y, k, s);
    return fail(PARS3_ESTATE, "spmv: no FP32 or BF16 values are stored for FP32 vectors");
  }
  return fail(PARS3_EINVAL, "spmv: vec_dtype must be PARS3_F64 or PARS3_F32");
}

// ------------------------------------------------------------ numbering changes
template <class T>
__global__ void k_gather(const T *__restrict__ src, T *__restrict__ dst, const int32_t *__restrict__ idx, int64_t n,
                         int k) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  int64_t r = t / k, c = t - r * k;
  dst[t] = src[(int64_t)idx[r] * k + c];
}
template <class T>
__global__ void k_scatter(const T *__restrict__ src, T *__restrict__ dst, const int32_t *__restrict__ idx, int64_t n,
                          int k) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  int64_t r = t / k, c = t - r * k;
  dst[(int64_t)idx[r] * k + c] = src[t];
}

pars3_status gather_rows(const void *src, void *dst, const int32_t *idx, int64_t n, int k, size_t elem,
                         hipStream_t s) {
  if (n * k == 0) return PARS3_OK;
  unsigned g = (unsigned)cdiv(n * k, TB);
  if (elem == 8) k_gather<double><<<g, TB, 0, s>>>((const double *)src, (double *)dst, idx, n, k);
  else k_gather<float><<<g, TB, 0, s>>>((const float *)src, (float *)dst, idx, n, k);
  P3_LAUNCHED();
  return PARS3_OK;
}
pars3_status scatter_rows(const void *src, void *dst, const int32_t *idx, int64_t n, int k, size_t elem,
                          hipStream_t s) {
  if (n * k == 0) return PARS3_OK;
  unsigned g = (unsigned)cdiv(n * k, TB);
  if (elem == 8) k_scatter<double><<<g, TB, 0, s>>>((const double *)src, (double *)dst, idx, n, k);
  else k_scatter<float><<<g, TB, 0, s>>>((const float *)src, (float *)dst, idx, n, k);
  P3_LAUNCHED();
  return PARS3_OK;
}

}  // namespace p3
