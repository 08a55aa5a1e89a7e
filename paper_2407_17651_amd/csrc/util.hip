// Primitives: error state, prefix sums, stable radix sort, fills.
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace p3 {

static thread_local char g_err[512] = "";

pars3_status fail(pars3_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}
void clear_error() { g_err[0] = 0; }

}  // namespace p3

extern "C" const char *pars3_last_error(void) { return p3::g_err; }

namespace p3 {

// ------------------------------------------------------------------ scan
// Block of 256 threads scans 1024 items (4 per thread) with wave64 shuffles.
static constexpr int SCAN_THREADS = 256;
static constexpr int SCAN_ITEMS = 4;
static constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

template <class T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile(const T *__restrict__ in, T *__restrict__ out,
                                                             T *__restrict__ bsum, int64_t m) {
  __shared__ T wsum[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T tsum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; k++) {
    v[k] = (base + k < m) ? in[base + k] : (T)0;
    tsum += v[k];
  }
  T incl = wave_incl_scan(tsum);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  T wpre = 0;
  for (int w = 0; w < wave; w++) wpre += wsum[w];
  T run = wpre + incl - tsum;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; k++) {
    if (base + k < m) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == SCAN_THREADS - 1) {
    T tot = 0;
    for (int w = 0; w < SCAN_THREADS / 64; w++) tot += wsum[w];
    bsum[blockIdx.x] = tot;
  }
}

template <class T>
__global__ void k_scan_add(T *__restrict__ out, const T *__restrict__ boff, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] += boff[i / SCAN_TILE];
}

template <class T>
__global__ void k_scan_single_total(T *__restrict__ out, const T *__restrict__ bsum, int64_t m) {
  // one block only: out[m] = bsum[0]
  if (threadIdx.x == 0 && blockIdx.x == 0) out[m] = bsum[0];
}

template <class T>
static pars3_status scan_impl(const T *in, T *out, int64_t m, hipStream_t s) {
  if (m <= 0) {
    P3_HIP(hipMemsetAsync(out, 0, sizeof(T), s));
    return PARS3_OK;
  }
  int64_t nb = cdiv(m, SCAN_TILE);
  dbuf<T> bsum, boff;
  P3_HIP(bsum.alloc(nb));
  P3_HIP(boff.alloc(nb + 1));
  k_scan_tile<T><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, out, bsum.p, m);
  P3_LAUNCHED();
  if (nb == 1) {
    k_scan_single_total<T><<<1, 64, 0, s>>>(out, bsum.p, m);
    P3_LAUNCHED();
  } else {
    P3_TRY(scan_impl<T>(bsum.p, boff.p, nb, s));
    k_scan_add<T><<<(unsigned)cdiv(m, 256), 256, 0, s>>>(out, boff.p, m);
    P3_LAUNCHED();
    P3_HIP(hipMemcpyAsync(out + m, boff.p + nb, sizeof(T), hipMemcpyDeviceToDevice, s));
  }
  // temporaries are freed by the destructors; make sure the stream is done
  // with them first
  P3_HIP(hipStreamSynchronize(s));
  return PARS3_OK;
}

pars3_status scan_i32(const int32_t *in, int32_t *out, int64_t m, hipStream_t s) { return scan_impl(in, out, m, s); }
pars3_status scan_i64(const int64_t *in, int64_t *out, int64_t m, hipStream_t s) { return scan_impl(in, out, m, s); }

// ------------------------------------------------------------------ radix sort
// LSD radix sort, 8-bit digits.  A block (4 waves) owns a chunk of 4096
// consecutive elements; each wave owns 1024 of them and walks them in order in
// groups of 64, ranking equal digits with ballots, so the scatter is stable.
static constexpr int RS_THREADS = 256;
static constexpr int RS_WAVE_ITEMS = 1024;
static constexpr int RS_CHUNK = RS_WAVE_ITEMS * (RS_THREADS / 64);

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t m, int shift,
                                                         uint32_t *__restrict__ hist, int64_t nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_CHUNK;
  for (int t = threadIdx.x; t < RS_CHUNK; t += RS_THREADS) {
    int64_t i = base + t;
    if (i < m) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                            const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
                                                            uint32_t *__restrict__ vout, int64_t m, int shift,
                                                            const uint32_t *__restrict__ offs, int64_t nb) {
  __shared__ uint32_t whist[RS_THREADS / 64][256];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = threadIdx.x; t < (RS_THREADS / 64) * 256; t += RS_THREADS) (&whist[0][0])[t] = 0;
  __syncthreads();
  const int64_t wbase = (int64_t)blockIdx.x * RS_CHUNK + (int64_t)wave * RS_WAVE_ITEMS;
  for (int g = 0; g < RS_WAVE_ITEMS; g += 64) {
    int64_t i = wbase + g + lane;
    if (i < m) atomicAdd(&whist[wave][(kin[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  // per-digit base of every wave: global offset of this block plus the counts
  // of the earlier waves of the block
  {
    const int d = threadIdx.x;  // 256 threads = 256 digits
    uint32_t run = offs[(int64_t)d * nb + blockIdx.x];
    for (int w = 0; w < RS_THREADS / 64; w++) {
      uint32_t c = whist[w][d];
      whist[w][d] = run;
      run += c;
    }
  }
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int g = 0; g < RS_WAVE_ITEMS; g += 64) {
    int64_t i = wbase + g + lane;
    bool valid = i < m;
    uint64_t key = valid ? kin[i] : 0ull;
    uint32_t val = valid ? vin[i] : 0u;
    uint32_t dig = (uint32_t)(key >> shift) & 255u;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      uint64_t bb = __ballot(valid && ((dig >> b) & 1u));
      same &= ((dig >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank = (uint32_t)__popcll(same & below);
    uint32_t cnt = (uint32_t)__popcll(same);
    uint32_t pos = 0;
    if (valid) pos = whist[wave][dig] + rank;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (valid && rank == cnt - 1) whist[wave][dig] += cnt;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      kout[pos] = key;
      vout[pos] = val;
    }
  }
}

pars3_status radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t m, int key_bits,
                              hipStream_t s) {
  if (m <= 1 || key_bits <= 0) return PARS3_OK;
  if (m > 0x7fffffffLL) return fail(PARS3_EINVAL, "radix sort: too many elements");
  int64_t nb = cdiv(m, RS_CHUNK);
  dbuf<uint32_t> hist, offs;
  P3_HIP(hist.alloc(256 * nb));
  P3_HIP(offs.alloc(256 * nb + 1));
  int passes = (key_bits + 7) / 8;
  uint64_t *ka = k0, *kb = k1;
  uint32_t *va = v0, *vb = v1;
  for (int p = 0; p < passes; p++) {
    int shift = 8 * p;
    k_rs_hist<<<(unsigned)nb, RS_THREADS, 0, s>>>(ka, m, shift, hist.p, nb);
    P3_LAUNCHED();
    P3_TRY(scan_i32((const int32_t *)hist.p, (int32_t *)offs.p, 256 * nb, s));
    k_rs_scatter<<<(unsigned)nb, RS_THREADS, 0, s>>>(ka, va, kb, vb, m, shift, offs.p, nb);
    P3_LAUNCHED();
    uint64_t *tk = ka;
    ka = kb;
    kb = tk;
    uint32_t *tv = va;
    va = vb;
    vb = tv;
  }
  if (ka != k0) {
    P3_HIP(hipMemcpyAsync(k0, ka, m * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    P3_HIP(hipMemcpyAsync(v0, va, m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
  P3_HIP(hipStreamSynchronize(s));
  return PARS3_OK;
}

// ------------------------------------------------------------------ fills
template <class T>
__global__ void k_fill(T *__restrict__ p, T v, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = v;
}
__global__ void k_iota(int32_t *__restrict__ p, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = (int32_t)i;
}

pars3_status fill_i32(int32_t *p, int32_t v, int64_t m, hipStream_t s) {
  if (m <= 0) return PARS3_OK;
  k_fill<int32_t><<<(unsigned)cdiv(m, 256), 256, 0, s>>>(p, v, m);
  P3_LAUNCHED();
  return PARS3_OK;
}
pars3_status fill_u64(uint64_t *p, uint64_t v, int64_t m, hipStream_t s) {
  if (m <= 0) return PARS3_OK;
  k_fill<uint64_t><<<(unsigned)cdiv(m, 256), 256, 0, s>>>(p, v, m);
  P3_LAUNCHED();
  return PARS3_OK;
}
pars3_status iota_i32(int32_t *p, int64_t m, hipStream_t s) {
  if (m <= 0) return PARS3_OK;
  k_iota<<<(unsigned)cdiv(m, 256), 256, 0, s>>>(p, m);
  P3_LAUNCHED();
  return PARS3_OK;
}

}  // namespace p3
