// Three-way split of the band and the layouts the product kernels read
// (Sections 1 and 3.1.2: diagonal/inner, middle and outer parts chosen by
// distance from the diagonal, the outer distance set by a user bandwidth).
//
// For a stored entry (i, j) of the reordered matrix, d = i - j:
//   inner  d <= w_in         -> diagonal-major band, no indices, read by the
//                               gather kernel that also applies the shift;
//   middle w_in < d <= t_out -> row tiles of T rows; a tile keeps in LDS the
//                               x and y values of its own rows and of one
//                               contiguous "back" window of columns
//                               [alo, alo + la) holding its targets j < r0;
//   outer  d > t_out         -> coordinate list (rows ascending).
// Middle entries of a tile whose back targets do not fit a window of
// `window_max` columns also go to the coordinate list, which the kernels treat
// exactly like the outer part.  Every placement is a stable compaction by a
// prefix sum in row-major entry order, so the layout is deterministic.
#include <algorithm>

#include "internal.h"

namespace p3 {

static constexpr int TB = 256;
static inline unsigned nblk(int64_t m) { return (unsigned)std::max<int64_t>(1, cdiv(m, TB)); }

__global__ void k_entry_rows(const int32_t *__restrict__ prow, int32_t n, int32_t *__restrict__ erow) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = prow[i]; e < prow[i + 1]; e++) erow[e] = i;
}
__global__ __launch_bounds__(TB) void k_beta(const int32_t *__restrict__ erow, const int32_t *__restrict__ pcol,
                                             int64_t nnz, int32_t *__restrict__ beta) {
  __shared__ int32_t bmax;
  if (threadIdx.x == 0) bmax = 0;
  __syncthreads();
  int32_t d = 0;
  for (int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * TB)
    d = max(d, erow[e] - pcol[e]);
  agg_atomic_max<int32_t>(&bmax, 0, d, true, 0);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(beta, bmax);
}
__global__ __launch_bounds__(TB) void k_classify(const int32_t *__restrict__ erow, const int32_t *__restrict__ pcol,
                                                 int64_t nnz, int32_t w_in, int32_t t_out, int8_t *__restrict__ part,
                                                 unsigned long long *__restrict__ cnt) {
  __shared__ unsigned long long bc[3];
  if (threadIdx.x < 3) bc[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long c[3] = {0, 0, 0};
  for (int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * TB) {
    int32_t d = erow[e] - pcol[e];
    int8_t p = d <= w_in ? 0 : (d <= t_out ? 1 : 2);
    part[e] = p;
    c[p]++;
  }
  for (int q = 0; q < 3; q++) agg_atomic_add<unsigned long long>(bc, q, c[q], true);
  __syncthreads();
  if (threadIdx.x < 3) atomicAdd(&cnt[threadIdx.x], bc[threadIdx.x]);
}
// back-window bounds of each tile: columns j < r0 of its middle entries
__global__ void k_tile_bounds(const int32_t *__restrict__ erow, const int32_t *__restrict__ pcol,
                              const int8_t *__restrict__ part, int64_t nnz, int32_t T, int32_t *__restrict__ tmin,
                              int32_t *__restrict__ tmax) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ok = e < nnz && part[e] == 1;
  int32_t i = ok ? erow[e] : 0, j = ok ? pcol[e] : 0;
  int32_t t = i / T, r0 = t * T;
  ok = ok && j < r0;
  agg_atomic_min<int32_t>(tmin, t, j, ok, 0x7fffffff);
  agg_atomic_max<int32_t>(tmax, t, j, ok, -1);
}
__global__ void k_tile_window(const int32_t *__restrict__ tmin, const int32_t *__restrict__ tmax, int32_t ntiles,
                              int32_t wmax, int32_t use_windows, int32_t *__restrict__ alo, int32_t *__restrict__ la) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int32_t lo = tmin[t], hi = tmax[t];
  if (use_windows && hi >= lo && hi - lo + 1 <= wmax) {
    alo[t] = lo;
    la[t] = hi - lo + 1;
  } else {
    alo[t] = 0;
    la[t] = 0;
  }
}
// placement flags: 1 = tile kernel, 2 = coordinate list, 0 = inner band
__global__ void k_place(const int32_t *__restrict__ erow, const int32_t *__restrict__ pcol,
                        const int8_t *__restrict__ part, int64_t nnz, int32_t T, int32_t use_tiles,
                        const int32_t *__restrict__ la, int32_t *__restrict__ ftile, int32_t *__restrict__ ffar,
                        int32_t *__restrict__ tcount) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = e < nnz;
  int32_t i = ok ? erow[e] : 0, j = ok ? pcol[e] : 0;
  int32_t t = i / T, r0 = t * T;
  int tiled = 0, far = 0;
  if (!ok) {
  } else if (part[e] == 1) {
    if (use_tiles && (j >= r0 || la[t] > 0)) tiled = 1;
    else far = 1;
  } else if (part[e] == 2) {
    far = 1;
  }
  if (ok) {
    ftile[e] = tiled;
    ffar[e] = far;
  }
  agg_atomic_add<int32_t>(tcount, t, 1, tiled);
}

template <class F>
__device__ __forceinline__ void store_vals(int64_t at, double v, double *f64, float *f32, uint16_t *bf16) {
  if (f64) f64[at] = v;
  float f = (float)v;  // round to nearest even
  if (f32) f32[at] = f;
  if (bf16) {
    uint32_t u = __float_as_uint(f);
    uint16_t b;
    if ((u & 0x7fffffffu) > 0x7f800000u) b = (uint16_t)((u >> 16) | 0x0040u);
    else b = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    bf16[at] = b;
  }
}

__global__ void k_fill_layout(const int32_t *__restrict__ erow, const int32_t *__restrict__ pcol,
                              const double *__restrict__ pval, const int8_t *__restrict__ part, int64_t nnz, int32_t n,
                              int32_t T, const int32_t *__restrict__ alo, const int32_t *__restrict__ la,
                              const int32_t *__restrict__ ftile, const int32_t *__restrict__ ptile,
                              const int32_t *__restrict__ ffar, const int32_t *__restrict__ pfar,
                              uint32_t *__restrict__ ent_rc, double *ef64, float *ef32, uint16_t *ebf16,
                              int32_t *__restrict__ far_row, int32_t *__restrict__ far_col, double *ff64, float *ff32,
                              uint16_t *fbf16, double *if64, float *if32, uint16_t *ibf16) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int32_t i = erow[e], j = pcol[e];
  double v = pval[e];
  if (part[e] == 0) {
    int64_t at = (int64_t)(i - j - 1) * n + i;
    store_vals<double>(at, v, if64, if32, ibf16);
    return;
  }
  if (ftile[e]) {
    int32_t t = i / T, r0 = t * T;
    int32_t a = la[t];
    uint32_t slot = j >= r0 ? (uint32_t)(a + (j - r0)) : (uint32_t)(j - alo[t]);
    int64_t at = ptile[e];
    ent_rc[at] = ((uint32_t)(i - r0) << 16) | slot;
    store_vals<double>(at, v, ef64, ef32, ebf16);
  } else if (ffar[e]) {
    int64_t at = pfar[e];
    far_row[at] = i;
    far_col[at] = j;
    store_vals<double>(at, v, ff64, ff32, fbf16);
  }
}
__global__ void k_max_slots(const int32_t *__restrict__ la, int32_t ntiles, int32_t T, int32_t *__restrict__ mx) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntiles) atomicMax(mx, la[t] + T);
}

pars3_status split_and_layout(pars3_matrix *A, const pars3_split_params &p, hipStream_t s) {
  const int32_t n = (int32_t)A->n;
  const int64_t nnz = A->nnz;
  layout &L = A->lay;
  // ---- beta and classes
  dbuf<int32_t> erow, dbeta;
  P3_HIP(erow.alloc(nnz));
  P3_HIP(dbeta.alloc(1));
  P3_HIP(hipMemsetAsync(dbeta.p, 0, sizeof(int32_t), s));
  if (n > 0) {
    k_entry_rows<<<nblk(n), TB, 0, s>>>(A->prow.p, n, erow.p);
    P3_LAUNCHED();
  }
  if (nnz > 0) {
    k_beta<<<std::min<unsigned>(nblk(nnz), 2048u), TB, 0, s>>>(erow.p, A->pcol.p, nnz, dbeta.p);
    P3_LAUNCHED();
  }
  int32_t beta = 0;
  P3_HIP(hipMemcpyAsync(&beta, dbeta.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  int32_t w_in = p.w_in < 0 ? 0 : p.w_in;
  int32_t t_out = p.t_out < 0 ? std::max(beta - 3, 0) : p.t_out;
  if (w_in > t_out) return fail(PARS3_EINVAL, "split: w_in (%d) > t_out (%d)", w_in, t_out);
  int32_t T = p.tile_rows <= 0 ? 256 : p.tile_rows;
  int32_t wmax = p.window_max <= 0 ? 1024 : p.window_max;
  if (T != 64 && T != 128 && T != 256 && T != 512 && T != 1024)
    return fail(PARS3_EINVAL, "split: tile_rows must be 64, 128, 256, 512 or 1024 (got %d)", T);
  if (wmax > 16384) return fail(PARS3_EINVAL, "split: window_max must be <= 16384 (got %d)", wmax);
  if (w_in > 64) return fail(PARS3_EINVAL, "split: w_in must be <= 64 (got %d)", w_in);
  if (p.value_dtype < PARS3_F64 || p.value_dtype > PARS3_BF16) return fail(PARS3_EINVAL, "split: bad value dtype");
  if (p.y_mode < PARS3_Y_AUTO || p.y_mode > PARS3_Y_ATOMIC) return fail(PARS3_EINVAL, "split: bad y_mode");

  P3_HIP(A->part.alloc(nnz));
  dbuf<unsigned long long> dcnt;
  P3_HIP(dcnt.alloc(3));
  P3_HIP(hipMemsetAsync(dcnt.p, 0, 3 * sizeof(unsigned long long), s));
  if (nnz > 0) {
    k_classify<<<std::min<unsigned>(nblk(nnz), 2048u), TB, 0, s>>>(erow.p, A->pcol.p, nnz, w_in, t_out, A->part.p,
                                                                    dcnt.p);
    P3_LAUNCHED();
  }
  unsigned long long hc[3] = {0, 0, 0};
  P3_HIP(hipMemcpyAsync(hc, dcnt.p, sizeof(hc), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));

  // ---- tiles and windows
  const int32_t ntiles = (int32_t)cdiv(n, T);
  const int use_tiles = p.y_mode != PARS3_Y_ATOMIC;
  dbuf<int32_t> tmin, tmax, tcount, ftile, ffar, ptile, pfar, mx;
  P3_HIP(L.tile_alo.alloc(ntiles));
  P3_HIP(L.tile_la.alloc(ntiles));
  P3_HIP(L.tile_ptr.alloc(ntiles + 1));
  P3_HIP(tmin.alloc(ntiles));
  P3_HIP(tmax.alloc(ntiles));
  P3_HIP(tcount.alloc(ntiles));
  P3_HIP(ftile.alloc(nnz));
  P3_HIP(ffar.alloc(nnz));
  P3_HIP(ptile.alloc(nnz + 1));
  P3_HIP(pfar.alloc(nnz + 1));
  P3_HIP(mx.alloc(1));
  P3_TRY(fill_i32(tmin.p, 0x7fffffff, ntiles, s));
  P3_TRY(fill_i32(tmax.p, -1, ntiles, s));
  P3_HIP(hipMemsetAsync(tcount.p, 0, std::max<int64_t>(ntiles, 1) * sizeof(int32_t), s));
  P3_HIP(hipMemsetAsync(mx.p, 0, sizeof(int32_t), s));
  if (nnz > 0) {
    k_tile_bounds<<<nblk(nnz), TB, 0, s>>>(erow.p, A->pcol.p, A->part.p, nnz, T, tmin.p, tmax.p);
    P3_LAUNCHED();
  }
  if (ntiles > 0) {
    k_tile_window<<<nblk(ntiles), TB, 0, s>>>(tmin.p, tmax.p, ntiles, wmax, use_tiles, L.tile_alo.p, L.tile_la.p);
    P3_LAUNCHED();
    k_max_slots<<<nblk(ntiles), TB, 0, s>>>(L.tile_la.p, ntiles, T, mx.p);
    P3_LAUNCHED();
  }
  if (nnz > 0) {
    k_place<<<nblk(nnz), TB, 0, s>>>(erow.p, A->pcol.p, A->part.p, nnz, T, use_tiles, L.tile_la.p, ftile.p, ffar.p,
                                     tcount.p);
    P3_LAUNCHED();
  }
  P3_TRY(scan_i32(ftile.p, ptile.p, nnz, s));
  P3_TRY(scan_i32(ffar.p, pfar.p, nnz, s));
  P3_TRY(scan_i32(tcount.p, L.tile_ptr.p, ntiles, s));
  int32_t ntiled = 0, nfar = 0, maxslots = 0;
  P3_HIP(hipMemcpyAsync(&ntiled, ptile.p + nnz, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipMemcpyAsync(&nfar, pfar.p + nnz, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipMemcpyAsync(&maxslots, mx.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));

  // ---- values of the stored precisions
  const int vd = p.value_dtype;
  const bool want64 = vd == PARS3_F64 || p.keep_fp64;
  const bool want32 = vd == PARS3_F32;
  const bool want16 = vd == PARS3_BF16;
  L.in_f64.release();
  L.in_f32.release();
  L.in_bf16.release();
  L.ent_f64.release();
  L.ent_f32.release();
  L.ent_bf16.release();
  L.far_f64.release();
  L.far_f32.release();
  L.far_bf16.release();
  const int64_t nin = (int64_t)w_in * n;
  if (want64) {
    P3_HIP(L.in_f64.alloc(nin));
    P3_HIP(L.ent_f64.alloc(ntiled));
    P3_HIP(L.far_f64.alloc(nfar));
    if (nin) P3_HIP(hipMemsetAsync(L.in_f64.p, 0, nin * sizeof(double), s));
  }
  if (want32) {
    P3_HIP(L.in_f32.alloc(nin));
    P3_HIP(L.ent_f32.alloc(ntiled));
    P3_HIP(L.far_f32.alloc(nfar));
    if (nin) P3_HIP(hipMemsetAsync(L.in_f32.p, 0, nin * sizeof(float), s));
  }
  if (want16) {
    P3_HIP(L.in_bf16.alloc(nin));
    P3_HIP(L.ent_bf16.alloc(ntiled));
    P3_HIP(L.far_bf16.alloc(nfar));
    if (nin) P3_HIP(hipMemsetAsync(L.in_bf16.p, 0, nin * sizeof(uint16_t), s));
  }
  P3_HIP(L.ent_rc.alloc(ntiled));
  P3_HIP(L.far_row.alloc(nfar));
  P3_HIP(L.far_col.alloc(nfar));
  if (nnz > 0) {
    k_fill_layout<<<nblk(nnz), TB, 0, s>>>(
        erow.p, A->pcol.p, A->pval.p, A->part.p, nnz, n, T, L.tile_alo.p, L.tile_la.p, ftile.p, ptile.p, ffar.p,
        pfar.p, L.ent_rc.p, want64 ? L.ent_f64.p : nullptr, want32 ? L.ent_f32.p : nullptr,
        want16 ? L.ent_bf16.p : nullptr, L.far_row.p, L.far_col.p, want64 ? L.far_f64.p : nullptr,
        want32 ? L.far_f32.p : nullptr, want16 ? L.far_bf16.p : nullptr, want64 ? L.in_f64.p : nullptr,
        want32 ? L.in_f32.p : nullptr, want16 ? L.in_bf16.p : nullptr);
    P3_LAUNCHED();
  }
  // window tiles (for the read-back)
  std::vector<int32_t> hla(ntiles);
  if (ntiles) P3_HIP(hipMemcpyAsync(hla.data(), L.tile_la.p, ntiles * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  int32_t nwin = 0;
  for (int32_t t = 0; t < ntiles; t++) nwin += hla[t] > 0;

  L.T = T;
  L.wmax = wmax;
  L.y_mode = p.y_mode;
  L.w_in = w_in;
  L.t_out = t_out;
  L.ntiles = ntiles;
  L.n_window_tiles = nwin;
  L.max_slots = maxslots;
  L.nnz_tiled = ntiled;
  L.nnz_far = nfar;
  L.vdtype = vd;
  A->beta = beta;
  A->cnt[0] = (int64_t)hc[0];
  A->cnt[1] = (int64_t)hc[1];
  A->cnt[2] = (int64_t)hc[2];
  A->has_f64 = want64;
  A->has_f32 = want32;
  A->has_bf16 = want16;
  A->params = p;
  A->params.w_in = w_in;
  A->params.t_out = t_out;
  A->params.tile_rows = T;
  A->params.window_max = wmax;
  return PARS3_OK;
}

}  // namespace p3
