// Exhaustive autotuner over split and tile configurations.  Section 3.1.2
// leaves the outer bandwidth to the user and suggests reading it off the
// structure of the reordered matrix; on the GPU the choice also covers the
// inner band width and the tile height.  Each configuration of the grid is
// applied (re-split and layout rebuild; the reordering is kept), the product
// is timed with hipEvents on the caller's stream, and the fastest
// configuration is applied again at the end.  The table of timings is the
// training record of the learned selector.
#include <algorithm>
#include <chrono>
#include <atomic>
#include <vector>

#include "internal.h"

namespace p3 {

static constexpr int TT = 256;

__global__ void k_tune_fill(double *__restrict__ a, float *__restrict__ b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * TT + threadIdx.x;
  if (i >= m) return;
  // a fixed pattern in [-1, 1)
  const uint32_t h = (uint32_t)(i * 2654435761u) >> 8;
  const double v = (double)h * (2.0 / 16777216.0) - 1.0;
  if (a) a[i] = v;
  if (b) b[i] = (float)v;
}

}  // namespace p3

using p3::fail;

// t_out = -1: the paper's max(beta - 3, 0); -2: half the RCM bandwidth; never
// below w_in
static pars3_split_params resolve(pars3_split_params p, int32_t beta) {
  if (p.t_out == -1) p.t_out = std::max(beta - 3, 0);
  else if (p.t_out == -2) p.t_out = beta / 2;
  p.t_out = std::max(p.t_out, std::max(p.w_in, 0));
  return p;
}

static const int32_t kTiles[] = {64, 128, 256, 512, 1024};
static const int32_t kWin[] = {0, 1, 2, 4};

extern "C" pars3_status pars3_tune_grid_default(int32_t value_dtype, pars3_split_params *grid, int32_t cap,
                                                int32_t *count) {
  if (!count) return fail(PARS3_EINVAL, "tune grid: NULL count");
  if (value_dtype != PARS3_F64 && value_dtype != PARS3_F32 && value_dtype != PARS3_BF16)
    return fail(PARS3_EINVAL, "tune grid: bad value_dtype");
  // every tile configuration, then (FP64 and FP32 values) the full-CSR engine
  const int32_t tiles = (int32_t)(sizeof(kTiles) / sizeof(kTiles[0]) * sizeof(kWin) / sizeof(kWin[0]) * 2);
  const int32_t total = tiles + (value_dtype == PARS3_BF16 ? 0 : 1);
  *count = total;
  if (!grid) return PARS3_OK;
  if (cap < total) return fail(PARS3_EINVAL, "tune grid: capacity %d < %d", cap, total);
  int32_t q = 0;
  for (int32_t T : kTiles)
    for (int32_t w : kWin)
      for (int32_t half = 0; half < 2; half++) {
        pars3_split_params &p = grid[q++];
        pars3_split_params_default(&p);
        p.tile_rows = T;
        p.w_in = w;
        // t_out = -1: the paper's outer bandwidth 3; -2 here means half the
        // RCM bandwidth, resolved by pars3_autotune once beta is known
        p.t_out = half ? -2 : -1;
        p.value_dtype = value_dtype;
      }
  if (total > tiles) {
    pars3_split_params &p = grid[q++];
    pars3_split_params_default(&p);
    p.value_dtype = value_dtype;
    p.engine = PARS3_ENGINE_CSR;
  }
  return PARS3_OK;
}

extern "C" pars3_status pars3_autotune(pars3_matrix *A, const pars3_split_params *grid, int32_t ngrid, int32_t k,
                                       int32_t reps, pars3_tune_result *out, int32_t *best, void *stream) {
  using namespace p3;
  if (!A || !grid || ngrid < 1 || !out) return fail(PARS3_EINVAL, "autotune: NULL or empty argument");
  if (k != 1 && k != 2 && k != 4 && k != 8) return fail(PARS3_EINVAL, "autotune: k must be 1, 2, 4 or 8");
  if (reps < 1) return fail(PARS3_EINVAL, "autotune: reps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  // one split with the paper's boundaries gives beta (the reordering is
  // done once here and kept by every later re-split)
  {
    pars3_split_params p0 = grid[0];
    p0.w_in = 0;
    p0.t_out = -1;
    p0.engine = PARS3_ENGINE_TILES;
    P3_TRY(pars3_reorder(A, &p0, stream));
  }
  const int32_t beta = A->beta;
  const int64_t n = A->n;
  const int64_t m = std::max<int64_t>(n * k, 1);
  dbuf<double> x64, y64;
  dbuf<float> x32, y32;
  P3_HIP(x64.alloc(m));
  P3_HIP(y64.alloc(m));
  P3_HIP(x32.alloc(m));
  P3_HIP(y32.alloc(m));
  k_tune_fill<<<(unsigned)cdiv(m, TT), TT, 0, s>>>(x64.p, x32.p, m);
  P3_LAUNCHED();
  hipEvent_t e0, e1;
  P3_HIP(hipEventCreate(&e0));
  P3_HIP(hipEventCreate(&e1));
  pars3_status st = PARS3_OK;
  int32_t ib = -1;
  for (int32_t g = 0; g < ngrid && st == PARS3_OK; g++) {
    const pars3_split_params p = resolve(grid[g], beta);
    out[g].params = p;
    out[g].us = -1.0;
    st = pars3_reorder(A, &p, stream);
    if (st != PARS3_OK) break;
    const int vec = p.value_dtype == PARS3_F64 ? PARS3_F64 : PARS3_F32;
    const void *x = vec == PARS3_F64 ? (const void *)x64.p : (const void *)x32.p;
    void *y = vec == PARS3_F64 ? (void *)y64.p : (void *)y32.p;
    // warm-up (before the first configuration, products for at least 20 ms
    // of wall time: the GPU reaches its steady clock only after some
    // milliseconds of continuous work; the re-splits between configurations
    // keep it busy), then the median of three batches of reps products
    const auto w0 = std::chrono::steady_clock::now();
    for (int r = 0; st == PARS3_OK; r++) {
      st = spmv_rcm(A, 0.5, x, y, k, vec, s);
      if (st != PARS3_OK || r < 2) continue;
      if (g > 0) break;
      if ((r & 7) == 7) {
        if (hipStreamSynchronize(s) != hipSuccess) st = fail(PARS3_EHIP, "autotune: sync failed");
        if (std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count() >= 20.0) break;
      }
    }
    double t[3];
    for (int b = 0; b < 3 && st == PARS3_OK; b++) {
      if (hipEventRecord(e0, s) != hipSuccess) st = fail(PARS3_EHIP, "autotune: event record failed");
      for (int r = 0; r < reps && st == PARS3_OK; r++) st = spmv_rcm(A, 0.5, x, y, k, vec, s);
      if (st == PARS3_OK && hipEventRecord(e1, s) != hipSuccess) st = fail(PARS3_EHIP, "autotune: event record failed");
      float ms = 0.f;
      if (st == PARS3_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(PARS3_EHIP, "autotune: event timing failed");
      t[b] = 1e3 * (double)ms / reps;
    }
    if (st != PARS3_OK) break;
    std::sort(t, t + 3);
    out[g].params = A->params;
    out[g].us = t[1];
    if (ib < 0 || out[g].us < out[ib].us) ib = g;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PARS3_OK) {
    (void)hipGetLastError();
    return st;
  }
  if (best) *best = ib;
  // leave the handle with the fastest configuration
  pars3_split_params pb = out[ib].params;
  return pars3_reorder(A, &pb, stream);
}

extern "C" pars3_status pars3_select(pars3_matrix *A, pars3_mlp *m, const pars3_split_params *grid, int32_t ngrid,
                                     int32_t *choice, void *stream) {
  using namespace p3;
  if (!A || !m) return fail(PARS3_EINVAL, "select: NULL argument");
  if (!grid) {  // the grid stored with the network
    const std::vector<pars3_split_params> &g = mlp_grid(m);
    if (g.empty()) return fail(PARS3_ESTATE, "select: no grid given and none stored with the network");
    grid = g.data();
    ngrid = (int32_t)g.size();
  }
  if (ngrid < 1) return fail(PARS3_EINVAL, "select: empty grid");
  int32_t sz[4];
  P3_TRY(pars3_mlp_sizes(m, sz, nullptr));
  if ((sz[0] != 32 && sz[0] != 35) || sz[3] != ngrid)
    return fail(PARS3_EINVAL, "select: the network maps %d features to %d outputs; need 32 or 35 -> %d", sz[0],
                sz[3], ngrid);
  hipStream_t s = (hipStream_t)stream;
  // features of the reordered matrix (reorder with the paper's split first
  // when the handle has not been reordered)
  if (!A->perm_done) {
    pars3_split_params p0 = grid[0];
    p0.w_in = 0;
    p0.t_out = -1;
    p0.engine = PARS3_ENGINE_TILES;
    P3_TRY(pars3_reorder(A, &p0, stream));
  }
  // the 32 features, and for a 35-input network the 3 conflict features
  // over PARS3_SELECT_BLOCKS row blocks
  double f[35];
  P3_TRY(pars3_features(A, f, stream));
  if (sz[0] == 35) P3_TRY(pars3_conflict_features(A, PARS3_SELECT_BLOCKS, f + 32, stream));
  float ff[35];
  for (int k = 0; k < sz[0]; k++) ff[k] = (float)f[k];
  dbuf<float> xd;
  dbuf<int32_t> cd;
  P3_HIP(xd.alloc(sz[0]));
  P3_HIP(cd.alloc(1));
  P3_HIP(hipMemcpyAsync(xd.p, ff, sz[0] * sizeof(float), hipMemcpyHostToDevice, s));
  P3_TRY(pars3_mlp_select_rows(m, xd.p, 1, nullptr, cd.p, stream));
  int32_t c = -1;
  P3_HIP(hipMemcpyAsync(&c, cd.p, sizeof(c), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  if (c < 0 || c >= ngrid) return fail(PARS3_EHIP, "select: no configuration chosen");
  if (choice) *choice = c;
  if (!A->split_done) {
    pars3_split_params p0 = grid[0];
    p0.w_in = 0;
    p0.t_out = -1;
    p0.engine = PARS3_ENGINE_TILES;
    P3_TRY(pars3_reorder(A, &p0, stream));
  }
  const pars3_split_params p = resolve(grid[c], A->beta);
  return pars3_reorder(A, &p, stream);
}

// ------------------------------------------------------------ default selector
// The network that pars3_reorder(A, NULL, ...) consults.  The caller owns it;
// pars3_mlp_destroy of the network in use clears it.
namespace p3 {
static std::atomic<pars3_mlp *> g_selector{nullptr};

void forget_selector(const pars3_mlp *m) {
  pars3_mlp *cur = const_cast<pars3_mlp *>(m);
  g_selector.compare_exchange_strong(cur, nullptr);
}

bool has_selector() { return g_selector.load() != nullptr; }

pars3_status reorder_selected(pars3_matrix *A, void *stream) {
  pars3_mlp *m = g_selector.load();
  if (!m) return fail(PARS3_ESTATE, "reorder: no selector in use");
  return pars3_select(A, m, nullptr, 0, nullptr, stream);
}
}  // namespace p3

extern "C" pars3_status pars3_model_use(pars3_mlp *m) {
  if (m && (int32_t)p3::mlp_grid(m).size() < 1)
    return fail(PARS3_ESTATE, "model_use: the network has no configuration grid (pars3_mlp_set_grid)");
  p3::g_selector.store(m);
  return PARS3_OK;
}
