// Three-way split of the band and the layout the product kernel reads
// (Sections 1 and 3.1.2: diagonal/inner, middle and outer parts chosen by
// distance from the diagonal, the outer distance set by a user bandwidth).
//
// For a stored entry (i, j) of the reordered matrix, d = i - j:
//   inner  d <= w_in         -> diagonal-major band, no indices;
//   middle w_in < d <= t_out -> tile-pair blocks;
//   outer  d > t_out         -> tile-pair blocks of their own.
// Rows are cut into tiles of T rows.  Entry (i, j) of part p belongs to block
// (t, p, u) with t = i / T (row tile) and u = j / T (column tile, u <= t).
// Entries are sorted by (t, p, u, g, row) with g = (j - i) mod T the block
// diagonal: the blocks of a row tile are contiguous, and inside a block the
// entries of one diagonal are contiguous.  Along a diagonal rows and columns
// are all distinct, so the 64 lanes of a chunk mostly add into 64 different
// LDS rows on both the row side and the column side (lanes adding into one
// address are serialised).
// Each entry stores its value and the word ((i - t*T) << SH | (j - u*T)):
// 16 bits with SH = 8 for tiles of at most 256 rows, 32 bits with SH = 16
// for taller ones.  Per row
// tile: its block range; per column tile: the list of blocks whose column tile
// it is.  The product reads, per tile, its own blocks (row side) and the
// blocks of its column list (column side), cut into chunks of at most 64
// consecutive entries; the first CHUNKS_FIXED chunk descriptors of a tile sit
// at fixed positions, the rest in an overflow list.  All placement is a stable
// radix sort plus prefix sums, so the layout is deterministic.
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
  unsigned long long c0 = 0, c1 = 0, c2 = 0;
  for (int64_t e = (int64_t)blockIdx.x * TB + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * TB) {
    int32_t d = erow[e] - pcol[e];
    int8_t p = d <= w_in ? 0 : (d <= t_out ? 1 : 2);
    part[e] = p;
    c0 += p == 0;
    c1 += p == 1;
    c2 += p == 2;
  }
  agg_atomic_add<unsigned long long>(bc, 0, c0, true);
  agg_atomic_add<unsigned long long>(bc, 1, c1, true);
  agg_atomic_add<unsigned long long>(bc, 2, c2, true);
  __syncthreads();
  if (threadIdx.x < 3) atomicAdd(&cnt[threadIdx.x], bc[threadIdx.x]);
}

__device__ __forceinline__ void store_vals(int64_t at, double v, double *f64, float *f32, uint16_t *bf16) {
  if (f64) f64[at] = v;
  float f = (float)v;  // IEEE round to nearest even
  if (f32) f32[at] = f;
  if (bf16) {
    uint32_t u = __float_as_uint(f);
    uint16_t b;
    if ((u & 0x7fffffffu) > 0x7f800000u) b = (uint16_t)((u >> 16) | 0x0040u);
    else b = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    bf16[at] = b;
  }
}

// Inner band values go to their diagonal-major slot; block entries get a sort
// key (t, p, u, block diagonal, row offset) with the entry index as payload.
__global__ void k_inner_and_keys(const int32_t *__restrict__ erow, const int32_t *__restrict__ pcol,
                                 const double *__restrict__ pval, const int8_t *__restrict__ part, int64_t nnz,
                                 int32_t n, int32_t T, int lgT, int tbits, const int32_t *__restrict__ kpos,
                                 uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, double *if64, float *if32,
                                 uint16_t *ibf16) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int32_t i = erow[e], j = pcol[e];
  const int p = part[e];
  if (p == 0) {
    store_vals((int64_t)(i - j - 1) * n + i, pval[e], if64, if32, ibf16);
    return;
  }
  const uint64_t t = (uint64_t)(i >> lgT), u = (uint64_t)(j >> lgT);
  const uint64_t ri = (uint64_t)(i & (T - 1)), cj = (uint64_t)(j & (T - 1));
  uint64_t key = t;
  key = (key << 1) | (uint64_t)(p - 1);
  key = (key << tbits) | u;
  key = (key << lgT) | ((cj - ri) & (uint64_t)(T - 1));
  key = (key << lgT) | ri;
  const int32_t at = kpos[e];
  keys[at] = key;
  vals[at] = (uint32_t)e;
}
__global__ void k_block_flags(const uint64_t *__restrict__ keys, int64_t m, int lgT, int32_t *__restrict__ flag) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const uint64_t b = keys[q] >> (2 * lgT);
  flag[q] = (q == 0 || (keys[q - 1] >> (2 * lgT)) != b) ? 1 : 0;
}
// ---- entry order inside a block, for LDS adds without bank conflicts
// The product adds each entry's products into the LDS row sum of its row
// offset (row side) or column offset (column side).  gfx950 serves a
// wavefront's FP64 LDS add in four quarters of 16 lanes (16 x 8 bytes), and
// two lanes of one quarter whose offsets agree modulo 32 hit the same bank
// pair, for every LDS row stride the kernels use (1, 3, 5 and 9 words: all
// odd), so such a quarter takes two or more passes; lanes of different
// quarters never conflict.  Chunks start at multiples of 64 entries from the
// block start, so the quarters are the aligned runs of BO_RUN = 16 entries
// of a block.  The sort leaves a block in diagonal order, where runs along
// one diagonal have distinct row and column offsets; sparse diagonals mix
// into a run and collide.  Here each run of a block is refilled as a
// matching between row classes (offset mod 32) and column classes: entries
// are bucketed by (row class, column class); per run, rows propose to their
// most loaded free column class, columns accept the most loaded row class,
// augmenting paths complete the matching, and a class is allowed a second
// (third, ...) entry only when no matching covers the run.  Each (row,
// column) class pair gives its entries in diagonal order and a run keeps the
// order of the sort.  Mixing entries from all over the block spreads the x
// gathers of a run over more cache lines, so a block keeps the new order
// only if it costs less (bo_cost: passes against gather spread) than the
// sorted one.  One 64-thread workgroup per block segment; lanes 0-31 stand
// for the row classes, lanes 32-63 for the column classes.
static constexpr int BO_RUN = 16;
static constexpr int BO_NB = 32 * 32;

__device__ __forceinline__ int bo_bucket(uint64_t k, int lgT) {
  const uint32_t T1 = (1u << lgT) - 1u;
  const uint32_t ri = (uint32_t)k & T1, cj = ((uint32_t)(k >> lgT) + ri) & T1;
  return (int)(((ri & 31u) << 5) | (cj & 31u));
}
__device__ __forceinline__ uint32_t bo_or(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v |= (uint32_t)__shfl_xor((int)v, off, 64);
  return v;
}
__device__ __forceinline__ int bo_max(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}
// One run of BO_RUN entries (entry q of lane l & 31, or q < 0 for none; lanes
// with l & 31 >= BO_RUN pass q < 0): its LDS passes (row side + column side:
// the most loaded row class plus the most loaded column class) and the
// 16-row units of x its gathers touch on both sides.  Lanes 0-31 look at the
// row offsets (the row side's LDS slot, the column side's x row), lanes
// 32-63 at the column offsets.
struct bo_run {
  int passes, units;
};
// The cost that decides between the two orders of a block: BO_PASS_WEIGHT x
// passes + units.  The weight is a measured exchange rate: on the batched
// 8-right-hand-side product (256 matrices), weights of 10 and 20 took 0.447
// and 0.440 ms per launch (its 2D grids 0.100 and 0.083 ms, its 3D grids
// 0.107 and 0.110 ms); the single-matrix products did not move.
static constexpr int BO_PASS_WEIGHT = 20;
__device__ __forceinline__ int bo_cost(bo_run h) { return BO_PASS_WEIGHT * h.passes + h.units; }
// Lane src's value of v; src is the same on every lane (v_readlane).
__device__ __forceinline__ int bo_lane(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

__device__ __forceinline__ bo_run bo_run_eval(const uint64_t *__restrict__ keys, int32_t q, int lgT, int lane) {
  const uint32_t T1 = (1u << lgT) - 1u;
  int o = -1;
  if (q >= 0) {
    const uint64_t k = keys[q];
    const uint32_t ri = (uint32_t)k & T1, cj = ((uint32_t)(k >> lgT) + ri) & T1;
    o = (int)(lane < 32 ? ri : cj);
  }
  int mult = 0;
  bool first = o >= 0;
  for (int j = 0; j < BO_RUN; j++) {
    const int lo = bo_lane(o, j), hi = bo_lane(o, 32 + j);
    const int oj = lane < 32 ? lo : hi;
    mult += (o >= 0) & (oj >= 0) & ((oj & 31) == (o & 31));
    first &= !(j < (lane & 31) && oj >= 0 && (oj >> 4) == (o >> 4));
  }
  bo_run h;
  h.passes = bo_max(lane < 32 ? mult : 0) + bo_max(lane < 32 ? 0 : mult);
  h.units = (int)__popcll(__ballot(first));
  return h;
}

// A block is cut into ceil(m / BO_SEG) segments of equal size (rounded up to
// whole chunk halves, so that every segment starts at a run boundary), each
// regrouped on its own by one workgroup: a block of thousands of entries
// (1024-row tiles, dense rows) would otherwise serialise the launch behind
// one wavefront.  Segments of 512 entries cut the blocks of 256-row tiles of
// random geometric graphs (about 650 entries) in two and cost the batched
// 8-right-hand-side product 5%; at 2048 those stay whole.
static constexpr int32_t BO_SEG = 2048;
__global__ void k_bo_seg_count(const int32_t *__restrict__ bstart, int32_t nb, int32_t *__restrict__ cnt) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) cnt[b] = (bstart[b + 1] - bstart[b] + BO_SEG - 1) / BO_SEG;
}

__global__ __launch_bounds__(64) void k_bank_order(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                                                   const int32_t *__restrict__ bstart, const int32_t *__restrict__ segp,
                                                   int32_t nb, int lgT, uint64_t *__restrict__ keys_out,
                                                   uint32_t *__restrict__ vals_out, int32_t *__restrict__ lst,
                                                   int32_t *__restrict__ stats) {
  __shared__ int32_t head[BO_NB], tail[BO_NB];
  __shared__ int32_t s_grp[32];
  const int lane = threadIdx.x;
  const int cls = lane & 31;
  const bool isrow = lane < 32;
  // this workgroup's segment [s, e): its block by binary search over the
  // segment offsets, then its share of the block
  const int32_t g = blockIdx.x;
  int32_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (segp[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  const int32_t bs = bstart[lo], be = bstart[lo + 1], nseg = segp[lo + 1] - segp[lo];
  const int32_t size = ((be - bs + nseg - 1) / nseg + 31) & ~31;
  const int32_t s = min(be, bs + (g - segp[lo]) * size), e = min(be, s + size);
  int32_t *st = stats + 3 * (int64_t)g;  // runs, passes of the sorted order, passes kept
  // the sorted order's cost
  int32_t cost_orig = 0, pass_orig = 0, runs = 0;
  for (int32_t h0 = s; h0 < e; h0 += BO_RUN) {
    const bo_run hv = bo_run_eval(keys, cls < BO_RUN && h0 + cls < e ? h0 + cls : -1, lgT, lane);
    cost_orig += bo_cost(hv);
    pass_orig += hv.passes;
    runs++;
  }
  bool keep = runs <= 1 || pass_orig == 2 * runs;  // nothing to gain
  int32_t pass_new = 0;
  if (!keep) {
    // bucket sizes, their starts (exclusive scan, 16 buckets per lane), and
    // the stable bucket lists (entry positions in sorted order)
    for (int i = lane; i < BO_NB; i += 64) head[i] = 0;
    __syncthreads();
    for (int32_t q = s + lane; q < e; q += 64) atomicAdd(&head[bo_bucket(keys[q], lgT)], 1);
    __syncthreads();
    int32_t c16[16], tot = 0;
#pragma unroll
    for (int u = 0; u < 16; u++) {
      c16[u] = head[lane * 16 + u];
      tot += c16[u];
    }
    int32_t incl = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t v = __shfl_up(incl, d, 64);
      if (lane >= d) incl += v;
    }
    int32_t run = incl - tot;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; u++) {
      head[lane * 16 + u] = run;
      tail[lane * 16 + u] = run;
      run += c16[u];
    }
    __syncthreads();
    for (int32_t q0 = s; q0 < e; q0 += 64) {
      const int32_t q = q0 + lane;
      const int bk = q < e ? bo_bucket(keys[q], lgT) : -1;
      int rank = 0;
      for (int j = 0; j < 64; j++) rank += (j < lane) & (bo_lane(bk, j) == bk);
      const int32_t base = bk >= 0 ? tail[bk] : 0;
      __syncthreads();
      if (bk >= 0) {
        lst[s + base + rank] = q;
        atomicAdd(&tail[bk], 1);
      }
      __syncthreads();
    }
    // per lane: its class's nonempty partner classes and its entry count
    uint32_t adj = 0;
    int rem = 0;
    for (int o = 0; o < 32; o++) {
      const int bk = isrow ? (cls << 5 | o) : (o << 5 | cls);
      const int32_t c = tail[bk] - head[bk];
      rem += c;
      if (c) adj |= 1u << o;
    }
    int32_t cost_new = 0;
    for (int32_t out = s; out < e && !keep;) {
      const int need = min(BO_RUN, (int)(e - out));
      int cnt = 0;  // entries of this lane's class in the run
      int got = 0;
      // a class limit of 33 admits every remaining entry, so the loop ends by then
      for (int lim = 1; got < need && lim <= 40; lim++) {
        const bool ok = cnt < lim;
        const uint32_t cols_ok = (uint32_t)(__ballot(ok) >> 32);
        int mate = -1;
        // greedy: unmatched rows propose to their most loaded free column,
        // each column takes its most loaded proposer
        for (int round = 0; round < 32; round++) {
          const uint32_t mcols = (uint32_t)(__ballot(!isrow && mate >= 0) >> 32);
          const uint32_t av = (isrow && ok && mate < 0) ? (adj & cols_ok & ~mcols) : 0u;
          int prop = -1, best = -1;
          for (int c = 0; c < 32; c++) {
            const int rc = bo_lane(rem, 32 + c);
            if (((av >> c) & 1u) && rc > best) {
              best = rc;
              prop = c;
            }
          }
          if (!__ballot(prop >= 0)) break;
          int acc = -1, bestr = -1;
          for (int r = 0; r < 32; r++) {
            const int pr = bo_lane(prop, r), rr = bo_lane(rem, r);
            if (pr == cls && rr > bestr) {
              bestr = rr;
              acc = r;
            }
          }
          if (!isrow && acc >= 0) mate = acc;
          const int cm = __shfl(mate, 32 + max(prop, 0), 64);
          if (isrow && prop >= 0 && cm == cls) mate = prop;
        }
        // augmenting paths from the remaining free rows (BFS over column
        // classes; parents kept by the column lanes)
        uint32_t tried = 0;
        for (;;) {
          const uint32_t mrows = (uint32_t)__ballot(isrow && mate >= 0);
          if (got + __popc(mrows) >= need) break;
          const uint32_t mcols = (uint32_t)(__ballot(!isrow && mate >= 0) >> 32);
          const uint32_t cand =
              (uint32_t)__ballot(isrow && ok && mate < 0 && !((tried >> cls) & 1u) && (adj & cols_ok) != 0u);
          if (!cand) break;
          const int r0 = __ffs(cand) - 1;
          tried |= 1u << r0;
          uint32_t front = 1u << r0, seen = 0;
          int found = -1, par = -1;
          while (front) {
            uint32_t nb = (isrow && ((front >> cls) & 1u)) ? (adj & cols_ok) : 0u;
            nb = bo_or(nb) & ~seen;
            if (!nb) break;
            if (!isrow && ((nb >> cls) & 1u)) par = __ffs(adj & front) - 1;
            seen |= nb;
            const uint32_t freec = nb & ~mcols;
            if (freec) {
              found = __ffs(freec) - 1;
              break;
            }
            front = bo_or((!isrow && ((nb >> cls) & 1u)) ? (1u << mate) : 0u);
          }
          if (found < 0) continue;
          // flip the path back to r0 (at most 32 steps; every index is uniform)
          for (int c = found, step = 0; step < 33 && c >= 0 && c < 32; step++) {
            const int r = bo_lane(par, 32 + c);
            if (r < 0 || r >= 32) break;
            const int prev = bo_lane(mate, r);
            if (lane == r) mate = c;
            if (lane == 32 + c) mate = r;
            if (r == r0) break;
            c = prev;
          }
        }
        // take the most loaded matched pairs (at most need - got of them:
        // by the remaining entries of the row class plus those of its
        // column class, ties to the lower row class), so that heavy classes
        // are not left to pile up in the last runs
        const uint32_t mrows = (uint32_t)__ballot(isrow && mate >= 0);
        const int take = min(__popc(mrows), need - got);
        if (take == 0) continue;
        const int remc = __shfl(rem, 32 + (max(mate, 0) & 31), 64);
        const int key = (isrow && mate >= 0) ? rem + remc : -1;
        int slot = 0;
        for (int r = 0; r < 32; r++) {
          const int kr = bo_lane(key, r);
          slot += (kr > key) | ((kr == key) & (r < cls));
        }
        const bool use = isrow && mate >= 0 && slot < take;
        const int ru = __shfl(use ? mate : -1, max(mate, 0) & 31, 64);
        const bool col_used = !isrow && mate >= 0 && ru == cls;
        if (use) {
          const int bk = cls << 5 | mate;
          const int32_t at = head[bk];
          head[bk] = at + 1;
          s_grp[got + slot] = lst[s + at];
        }
        __syncthreads();
        if (use || col_used) {
          const int bk = isrow ? (cls << 5 | mate) : (mate << 5 | cls);
          if (head[bk] == tail[bk]) adj &= ~(1u << mate);
          cnt++;
          rem--;
        }
        got += take;
      }
      if (got < need) {  // not expected: keep the sorted order
        keep = true;
        break;
      }
      __syncthreads();
      const bo_run hv = bo_run_eval(keys, cls < need ? s_grp[cls] : -1, lgT, lane);
      cost_new += bo_cost(hv);
      pass_new += hv.passes;
      if (cost_new >= cost_orig) keep = true;  // cannot end cheaper any more
      if (lane < need) {
        const int32_t v = s_grp[lane];
        int rank = 0;
        for (int j = 0; j < need; j++) rank += s_grp[j] < v;
        keys_out[out + rank] = keys[v];
        vals_out[out + rank] = vals[v];
      }
      __syncthreads();
      out += need;
    }
  }
  if (keep) {
    for (int32_t q = s + lane; q < e; q += 64) {
      keys_out[q] = keys[q];
      vals_out[q] = vals[q];
    }
  }
  if (lane == 0) {
    st[0] = runs;
    st[1] = pass_orig;
    st[2] = keep ? pass_orig : pass_new;
  }
}
// Sums of the per-block statistics (one workgroup; int64 totals).
__global__ __launch_bounds__(TB) void k_sum3(const int32_t *__restrict__ a, int32_t nb, long long *__restrict__ out) {
  __shared__ long long red[3][TB];
  long long t[3] = {0, 0, 0};
  for (int32_t b = threadIdx.x; b < nb; b += TB)
    for (int k = 0; k < 3; k++) t[k] += a[3 * (int64_t)b + k];
  for (int k = 0; k < 3; k++) red[k][threadIdx.x] = t[k];
  __syncthreads();
  for (int w = TB / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 3; k++) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}
__global__ void k_block_starts(const int32_t *__restrict__ flag, const int32_t *__restrict__ bpos, int64_t m,
                               int32_t *__restrict__ bstart) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m && flag[q]) bstart[bpos[q]] = (int32_t)q;
}
__global__ void k_fill_blocks(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t m, int lgT,
                              int tbits, const int32_t *__restrict__ flag, const int32_t *__restrict__ bpos,
                              const double *__restrict__ pval, uint32_t *ent32, uint16_t *ent16, double *ef64,
                              float *ef32, uint16_t *ebf16, int32_t *__restrict__ pos_of,
                              int32_t *__restrict__ blk_start,
                              int32_t *__restrict__ blk_t, int32_t *__restrict__ blk_u,
                              int32_t *__restrict__ tcount, int32_t *__restrict__ ucount) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const uint64_t k = keys[q];
  const uint32_t e = vals[q];
  const uint32_t T1 = (1u << lgT) - 1u;
  const uint32_t ri = (uint32_t)(k & T1), cj = ((uint32_t)(k >> lgT) + ri) & T1;
  if (ent16) ent16[q] = (uint16_t)((ri << 8) | cj);
  else ent32[q] = (ri << 16) | cj;
  store_vals(q, pval[e], ef64, ef32, ebf16);
  pos_of[e] = (int32_t)q;
  if (flag[q]) {
    const uint64_t b = k >> (2 * lgT);
    const int32_t u = (int32_t)(b & ((1ull << tbits) - 1ull));
    const int32_t t = (int32_t)(b >> (tbits + 1));
    const int32_t id = bpos[q];
    blk_start[id] = (int32_t)q;
    blk_t[id] = t;
    blk_u[id] = u;
    atomicAdd(&tcount[t], 1);
    atomicAdd(&ucount[u], 1);
  }
}
__global__ void k_ulist_fill(const int32_t *__restrict__ blk_u, int32_t nb, const int32_t *__restrict__ uptr,
                             int32_t *__restrict__ fill, int32_t *__restrict__ tmp) {
  int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) tmp[uptr[blk_u[b]] + atomicAdd(&fill[blk_u[b]], 1)] = b;
}
// sort each list by its values (distinct): destination = rank in the list
__global__ void k_list_sort(const int32_t *__restrict__ ptr, int32_t nlists, const int32_t *__restrict__ in, int64_t m,
                            int32_t *__restrict__ out) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  int32_t lo = 0, hi = nlists - 1;  // the list that owns q
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  const int32_t v = in[q];
  int32_t rank = 0;
  for (int32_t r = ptr[lo]; r < ptr[lo + 1]; r++) rank += in[r] < v;
  out[ptr[lo] + rank] = v;
}
// Segment table of every tile: its own blocks (row side) and then the blocks
// of its column list (column side).
__global__ void k_seg_count(const int32_t *__restrict__ tblk_ptr, const int32_t *__restrict__ ublk_ptr, int32_t ntiles,
                            int32_t *__restrict__ cnt) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntiles) cnt[t] = (tblk_ptr[t + 1] - tblk_ptr[t]) + (ublk_ptr[t + 1] - ublk_ptr[t]);
}
__global__ void k_seg_fill(const int32_t *__restrict__ tblk_ptr, const int32_t *__restrict__ ublk_ptr,
                           const int32_t *__restrict__ ublk, const int32_t *__restrict__ blk_start,
                           const int32_t *__restrict__ blk_t, const int32_t *__restrict__ blk_u, int32_t ntiles,
                           const int32_t *__restrict__ tseg_ptr, int32_t *__restrict__ seg_start,
                           int32_t *__restrict__ seg_len, int32_t *__restrict__ seg_code) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int32_t q = tseg_ptr[t];
  for (int32_t b = tblk_ptr[t]; b < tblk_ptr[t + 1]; b++, q++) {
    seg_start[q] = blk_start[b];
    seg_len[q] = blk_start[b + 1] - blk_start[b];
    seg_code[q] = blk_u[b] << 1;
  }
  for (int32_t r = ublk_ptr[t]; r < ublk_ptr[t + 1]; r++, q++) {
    const int32_t b = ublk[r];
    seg_start[q] = blk_start[b];
    seg_len[q] = blk_start[b + 1] - blk_start[b];
    seg_code[q] = (blk_t[b] << 1) | 1;
  }
}
// Chunks: each segment of a tile cut into runs of at most 64 consecutive
// entries, one per wavefront step of the product.  Descriptor:
// x = first entry, y = other tile << 8 | column side << 7 | (length - 1).
__global__ void k_chunk_count(const int32_t *__restrict__ tseg_ptr, const int32_t *__restrict__ seg_len,
                              int32_t ntiles, int32_t *__restrict__ cnt) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int32_t c = 0;
  for (int32_t q = tseg_ptr[t]; q < tseg_ptr[t + 1]; q++) c += (seg_len[q] + 63) >> 6;
  cnt[t] = c;
}
__global__ void k_chunk_fill(const int32_t *__restrict__ tseg_ptr, const int32_t *__restrict__ seg_start,
                             const int32_t *__restrict__ seg_len, const int32_t *__restrict__ seg_code,
                             int32_t ntiles, const int32_t *__restrict__ tch_ptr, uint2 *__restrict__ chunk) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int32_t c = tch_ptr[t];
  for (int32_t q = tseg_ptr[t]; q < tseg_ptr[t + 1]; q++) {
    const uint32_t code = (uint32_t)seg_code[q];  // other tile << 1 | column side
    for (int32_t off = 0; off < seg_len[q]; off += 64, c++) {
      const int32_t len = min(64, seg_len[q] - off);
      chunk[c] = make_uint2((uint32_t)(seg_start[q] + off), (code << 7) | (uint32_t)(len - 1));
    }
  }
}
__global__ void k_overflow_count(const int32_t *__restrict__ tch_ptr, int32_t ntiles, int32_t *__restrict__ ocnt) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntiles) ocnt[t] = max(0, tch_ptr[t + 1] - tch_ptr[t] - CHUNKS_FIXED);
}
// One thread per fixed slot (t, s).  The fixed chunks of a tile are dealt to
// its 4 wavefronts round-robin (wavefront w takes chunks w, w + 4, ...), and
// the 8 chunks of one wavefront are stored next to each other, so a
// wavefront reads its descriptors with one 64-byte scalar load: slot
// s = 8 w + k holds chunk w + 4 k, or the empty marker past the tile's count.
// Slot 0 also moves the tile's overflow chunks.
__global__ void k_chunk_place(const int32_t *__restrict__ tch_ptr, const uint2 *__restrict__ chunk, int32_t ntiles,
                              const int32_t *__restrict__ ovf_ptr, uint2 *__restrict__ fix, uint2 *__restrict__ ovf) {
  constexpr int WAVES = 4, PER = CHUNKS_FIXED / WAVES;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)ntiles * CHUNKS_FIXED) return;
  const int32_t t = (int32_t)(g / CHUNKS_FIXED), sl = (int32_t)(g % CHUNKS_FIXED);
  const int32_t q = (sl % PER) * WAVES + sl / PER;
  const int32_t c0 = tch_ptr[t], cnt = tch_ptr[t + 1] - c0;
  fix[g] = q < cnt ? chunk[c0 + q] : make_uint2(0u, CHUNK_EMPTY);
  if (sl == 0)
    for (int32_t c = CHUNKS_FIXED; c < cnt; c++) ovf[ovf_ptr[t] + c - CHUNKS_FIXED] = chunk[c0 + c];
}
__global__ void k_pos_prefix(const int8_t *__restrict__ part, int64_t nnz, int32_t *__restrict__ flag) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) flag[e] = part[e] != 0;
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
  const int32_t w_in = p.w_in < 0 ? 0 : p.w_in;
  const int32_t t_out = p.t_out < 0 ? std::max(beta - 3, 0) : p.t_out;
  if (w_in > t_out) return fail(PARS3_EINVAL, "split: w_in (%d) > t_out (%d)", w_in, t_out);
  const int32_t T = p.tile_rows <= 0 ? 256 : p.tile_rows;
  if (T != 64 && T != 128 && T != 256 && T != 512 && T != 1024)
    return fail(PARS3_EINVAL, "split: tile_rows must be 64, 128, 256, 512 or 1024 (got %d)", T);
  if (w_in > 64) return fail(PARS3_EINVAL, "split: w_in must be <= 64 (got %d)", w_in);
  if (p.value_dtype < PARS3_F64 || p.value_dtype > PARS3_BF16) return fail(PARS3_EINVAL, "split: bad value dtype");
  const int lgT = bits_for((uint64_t)T) - 1;

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
  const int64_t m = (int64_t)(hc[1] + hc[2]);  // block entries

  // ---- value arrays of the stored precisions
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
  const int64_t nin = (int64_t)w_in * n;
  if (want64) {
    P3_HIP(L.in_f64.alloc(nin));
    P3_HIP(L.ent_f64.alloc(m));
    if (nin) P3_HIP(hipMemsetAsync(L.in_f64.p, 0, nin * sizeof(double), s));
  }
  if (want32) {
    P3_HIP(L.in_f32.alloc(nin));
    P3_HIP(L.ent_f32.alloc(m));
    if (nin) P3_HIP(hipMemsetAsync(L.in_f32.p, 0, nin * sizeof(float), s));
  }
  if (want16) {
    P3_HIP(L.in_bf16.alloc(nin));
    P3_HIP(L.ent_bf16.alloc(m));
    if (nin) P3_HIP(hipMemsetAsync(L.in_bf16.p, 0, nin * sizeof(uint16_t), s));
  }

  // ---- block entries: sort keys (t, p, u, block diagonal, row)
  const int32_t ntiles = (int32_t)cdiv(n, T);
  const int tbits = std::max(1, bits_for((uint64_t)std::max(ntiles - 1, 0)));
  const int key_bits = 2 * tbits + 1 + 2 * lgT;
  if (key_bits > 64) return fail(PARS3_EINVAL, "split: matrix too large for the block key (%d bits)", key_bits);
  if (ntiles > (1 << 23))
    return fail(PARS3_EINVAL, "split: %d tiles exceed the chunk descriptor's 2^23; use larger tile_rows", ntiles);
  dbuf<int32_t> kflag, kpos;
  dbuf<uint64_t> k0, k1;
  dbuf<uint32_t> v0, v1;
  P3_HIP(kflag.alloc(nnz));
  P3_HIP(kpos.alloc(nnz + 1));
  P3_HIP(k0.alloc(m));
  P3_HIP(k1.alloc(m));
  P3_HIP(v0.alloc(m));
  P3_HIP(v1.alloc(m));
  if (nnz > 0) {
    k_pos_prefix<<<nblk(nnz), TB, 0, s>>>(A->part.p, nnz, kflag.p);
    P3_LAUNCHED();
  }
  P3_TRY(scan_i32(kflag.p, kpos.p, nnz, s));
  if (nnz > 0) {
    k_inner_and_keys<<<nblk(nnz), TB, 0, s>>>(erow.p, A->pcol.p, A->pval.p, A->part.p, nnz, n, T, lgT, tbits, kpos.p,
                                              k0.p, v0.p, want64 ? L.in_f64.p : nullptr,
                                              want32 ? L.in_f32.p : nullptr, want16 ? L.in_bf16.p : nullptr);
    P3_LAUNCHED();
  }
  P3_TRY(radix_sort_pairs(k0.p, v0.p, k1.p, v1.p, m, key_bits, s));

  // ---- blocks
  dbuf<int32_t> bflag, bpos, tcount, ucount;
  P3_HIP(bflag.alloc(m));
  P3_HIP(bpos.alloc(m + 1));
  P3_HIP(tcount.alloc(ntiles));
  P3_HIP(ucount.alloc(ntiles));
  if (m > 0) {
    k_block_flags<<<nblk(m), TB, 0, s>>>(k0.p, m, lgT, bflag.p);
    P3_LAUNCHED();
  }
  P3_TRY(scan_i32(bflag.p, bpos.p, m, s));
  int32_t nb = 0;
  P3_HIP(hipMemcpyAsync(&nb, bpos.p + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  const int32_t m32 = (int32_t)m;
  const bool e16 = lgT <= ENT16_MAX_LGT;
  L.ent_rc.release();
  L.ent_rc16.release();
  if (e16) P3_HIP(L.ent_rc16.alloc(m));
  else P3_HIP(L.ent_rc.alloc(m));
  P3_HIP(L.pos_of.alloc(nnz));
  P3_HIP(L.blk_start.alloc(nb + 1));
  P3_HIP(L.blk_t.alloc(nb));
  P3_HIP(L.blk_u.alloc(nb));
  P3_HIP(L.tblk_ptr.alloc(ntiles + 1));
  P3_HIP(L.ublk_ptr.alloc(ntiles + 1));
  P3_HIP(L.ublk.alloc(nb));
  if (ntiles > 0) {
    P3_HIP(hipMemsetAsync(tcount.p, 0, ntiles * sizeof(int32_t), s));
    P3_HIP(hipMemsetAsync(ucount.p, 0, ntiles * sizeof(int32_t), s));
  }
  P3_HIP(hipMemcpyAsync(L.blk_start.p + nb, &m32, sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (nnz > 0) P3_TRY(fill_i32(L.pos_of.p, -1, nnz, s));
  if (m > 0) {
    // conflict-free runs inside each block: (k0, v0) -> (k1, v1)
    k_block_starts<<<nblk(m), TB, 0, s>>>(bflag.p, bpos.p, m, L.blk_start.p);
    P3_LAUNCHED();
    dbuf<int32_t> lst, bst, scnt, segp;
    dbuf<long long> tot;
    P3_HIP(scnt.alloc(nb));
    P3_HIP(segp.alloc(nb + 1));
    k_bo_seg_count<<<nblk(nb), TB, 0, s>>>(L.blk_start.p, nb, scnt.p);
    P3_LAUNCHED();
    P3_TRY(scan_i32(scnt.p, segp.p, nb, s));
    int32_t nseg = 0;
    P3_HIP(hipMemcpyAsync(&nseg, segp.p + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
    P3_HIP(lst.alloc(m));
    P3_HIP(bst.alloc(3 * (size_t)nseg));
    P3_HIP(tot.alloc(3));
    k_bank_order<<<(unsigned)nseg, 64, 0, s>>>(k0.p, v0.p, L.blk_start.p, segp.p, nb, lgT, k1.p, v1.p, lst.p,
                                               bst.p);
    P3_LAUNCHED();
    k_sum3<<<1, TB, 0, s>>>(bst.p, nseg, tot.p);
    P3_LAUNCHED();
    long long h3[3] = {0, 0, 0};
    P3_HIP(hipMemcpyAsync(h3, tot.p, sizeof(h3), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
    L.lds_runs = h3[0];
    L.lds_passes_sorted = h3[1];
    L.lds_passes = h3[2];
    std::swap(k0.p, k1.p);
    std::swap(v0.p, v1.p);
  } else {
    L.lds_runs = L.lds_passes_sorted = L.lds_passes = 0;
  }
  k1.release();
  v1.release();
  if (m > 0) {
    k_fill_blocks<<<nblk(m), TB, 0, s>>>(k0.p, v0.p, m, lgT, tbits, bflag.p, bpos.p, A->pval.p, L.ent_rc.p,
                                         L.ent_rc16.p, want64 ? L.ent_f64.p : nullptr,
                                         want32 ? L.ent_f32.p : nullptr, want16 ? L.ent_bf16.p : nullptr, L.pos_of.p,
                                         L.blk_start.p, L.blk_t.p, L.blk_u.p, tcount.p, ucount.p);
    P3_LAUNCHED();
  }
  P3_TRY(scan_i32(tcount.p, L.tblk_ptr.p, ntiles, s));
  P3_TRY(scan_i32(ucount.p, L.ublk_ptr.p, ntiles, s));
  if (nb > 0) {
    dbuf<int32_t> fill, tmp;
    P3_HIP(fill.alloc(ntiles));
    P3_HIP(tmp.alloc(nb));
    P3_HIP(hipMemsetAsync(fill.p, 0, ntiles * sizeof(int32_t), s));
    k_ulist_fill<<<nblk(nb), TB, 0, s>>>(L.blk_u.p, nb, L.ublk_ptr.p, fill.p, tmp.p);
    P3_LAUNCHED();
    k_list_sort<<<nblk(nb), TB, 0, s>>>(L.ublk_ptr.p, ntiles, tmp.p, nb, L.ublk.p);
    P3_LAUNCHED();
  }
  // per-tile segment tables (temporary), then the chunk lists the product reads
  {
    dbuf<int32_t> cnt, tseg_ptr, seg_start, seg_len, seg_code;
    P3_HIP(cnt.alloc(ntiles));
    P3_HIP(tseg_ptr.alloc(ntiles + 1));
    if (ntiles > 0) {
      k_seg_count<<<nblk(ntiles), TB, 0, s>>>(L.tblk_ptr.p, L.ublk_ptr.p, ntiles, cnt.p);
      P3_LAUNCHED();
    }
    P3_TRY(scan_i32(cnt.p, tseg_ptr.p, ntiles, s));
    int32_t nsegs = 0;
    P3_HIP(hipMemcpyAsync(&nsegs, tseg_ptr.p + ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
    P3_HIP(seg_start.alloc(nsegs));
    P3_HIP(seg_len.alloc(nsegs));
    P3_HIP(seg_code.alloc(nsegs));
    if (ntiles > 0 && nsegs > 0) {
      k_seg_fill<<<nblk(ntiles), TB, 0, s>>>(L.tblk_ptr.p, L.ublk_ptr.p, L.ublk.p, L.blk_start.p, L.blk_t.p, L.blk_u.p,
                                             ntiles, tseg_ptr.p, seg_start.p, seg_len.p, seg_code.p);
      P3_LAUNCHED();
      k_chunk_count<<<nblk(ntiles), TB, 0, s>>>(tseg_ptr.p, seg_len.p, ntiles, cnt.p);
      P3_LAUNCHED();
    } else if (ntiles > 0) {
      P3_TRY(fill_i32(cnt.p, 0, ntiles, s));
    }
    dbuf<int32_t> tch_ptr, ocnt;
    dbuf<uint2> chunk;
    P3_HIP(tch_ptr.alloc(ntiles + 1));
    P3_TRY(scan_i32(cnt.p, tch_ptr.p, ntiles, s));
    int32_t nch = 0;
    P3_HIP(hipMemcpyAsync(&nch, tch_ptr.p + ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
    P3_HIP(chunk.alloc(nch));
    if (ntiles > 0 && nch > 0) {
      k_chunk_fill<<<nblk(ntiles), TB, 0, s>>>(tseg_ptr.p, seg_start.p, seg_len.p, seg_code.p, ntiles, tch_ptr.p,
                                               chunk.p);
      P3_LAUNCHED();
    }
    // the first CHUNKS_FIXED chunks of every tile at fixed positions, the
    // rest in the overflow list
    P3_HIP(ocnt.alloc(ntiles));
    P3_HIP(L.ovf_ptr.alloc(ntiles + 1));
    P3_HIP(L.chunk_fix.alloc((size_t)ntiles * CHUNKS_FIXED));
    if (ntiles > 0) {
      k_overflow_count<<<nblk(ntiles), TB, 0, s>>>(tch_ptr.p, ntiles, ocnt.p);
      P3_LAUNCHED();
    }
    P3_TRY(scan_i32(ocnt.p, L.ovf_ptr.p, ntiles, s));
    int32_t nov = 0;
    P3_HIP(hipMemcpyAsync(&nov, L.ovf_ptr.p + ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P3_HIP(hipStreamSynchronize(s));
    P3_HIP(L.chunk_ovf.alloc(nov));
    if (ntiles > 0) {
      k_chunk_place<<<nblk((int64_t)ntiles * CHUNKS_FIXED), TB, 0, s>>>(tch_ptr.p, chunk.p, ntiles, L.ovf_ptr.p,
                                                                         L.chunk_fix.p, L.chunk_ovf.p);
      P3_LAUNCHED();
    }
    L.nchunks = nch;
    L.nchunks_ovf = nov;
  }
  // per-tile maxima of blocks (row side and column side), for the read-back
  std::vector<int32_t> ht(ntiles + 1), hu(ntiles + 1);
  if (ntiles) {
    P3_HIP(hipMemcpyAsync(ht.data(), L.tblk_ptr.p, (ntiles + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P3_HIP(hipMemcpyAsync(hu.data(), L.ublk_ptr.p, (ntiles + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  P3_HIP(hipStreamSynchronize(s));
  int32_t maxb = 0;
  for (int32_t t = 0; t < ntiles; t++) maxb = std::max(maxb, std::max(ht[t + 1] - ht[t], hu[t + 1] - hu[t]));

  L.T = T;
  L.lgT = lgT;
  L.w_in = w_in;
  L.t_out = t_out;
  L.ntiles = ntiles;
  L.nblocks = nb;
  L.max_blocks = maxb;
  L.nnz_blocked = m;
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
  return PARS3_OK;
}

}  // namespace p3
