// Skew-symmetric product y = shift*x + S*x, S = L - L^T, from the stored
// lower triangle only (eqs. (2)-(6), Section 3.1.2): every stored l_ij stands
// for the pair y_i += l_ij x_j and y_j -= l_ij x_i.  The same kernels serve
// the symmetric S = L + L^T of SSS storage (y_j += l_ij x_i) and its
// diagonal array D (y_i += d_i x_i, Section 1), selected per launch.
//
// One launch, one workgroup per tile of T rows, no global atomics and one
// plain store per output row.  The entries are stored once, grouped in
// tile-pair blocks (row tile t, column tile u).  The workgroup of tile t
// gathers into LDS (ds_add) every product that lands in its rows:
//   row side    : blocks (t, u) for all u      -> y_i += l_ij x_j, i in t;
//   column side : blocks (t', t) for all t'    -> y_j -= l_ij x_i, j in t;
// then writes y_i = shift*x_i + inner band (gathered per row in both
// directions from its diagonal-major store) + LDS sum.  The block (t', t)
// is thus read by two workgroups, t' and t.  In the banded reordered matrix
// t' - t stays within about beta/T tiles; tiles run in ascending order inside
// each XCD (see xcd_tile), so the second read of a block finds it in that
// XCD's L2 and the matrix crosses HBM about once: the transfer saving of
// storing one triangle (Section 3) is kept, while the exchange of conflicting
// products between owners of different rows (Section 3.1.2) becomes a read of
// shared data instead of a remote accumulation.
// Values are FP64, FP32 or BF16; vectors are FP64 for FP64 values and FP32
// otherwise; products are formed in the vector precision and summed in FP64
// in LDS.  k right-hand sides are stored row-major.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace p3 {

static constexpr int TB = 256;
static constexpr size_t LDS_DEFAULT = 64 * 1024;  // dynamic LDS available without an attribute
static constexpr int PRE = CHUNKS_FIXED / (TB / 64);  // chunks per wavefront whose loads are issued together
// LDS row stride of the FP64 row sums: K + 1 words for several right-hand
// sides, so that the K sums of rows with equal residues do not share banks
template <int K>
constexpr int KP = K == 1 ? 1 : K + 1;

// Device arrays seen as global-address-space pointers.  Loads through them
// are global loads (scalar loads where the address is wave-uniform) also when
// the pointer itself was read from memory, as in the batched tasks; through a
// generic pointer they would be flat loads, which the compiler waits for
// together with the LDS operations.
template <class T>
using gptr = const __attribute__((address_space(1))) T *;
template <class T>
using gmut = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> glb(const T *p) {
  return (gptr<T>)p;
}
template <class T>
__device__ __forceinline__ gmut<T> glbw(T *p) {
  return (gmut<T>)p;
}
// A chunk descriptor read as one 64-bit word (.x in the low half).
__device__ __forceinline__ uint2 load_desc(const uint2 *p, int64_t i) {
  const uint64_t v = glb((const uint64_t *)p)[i];
  return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

// Raw loads of stored values (normal, and nontemporal for a last use) and
// their conversion to the vector type; a BF16 value is the high half of an
// FP32 one.  The conversion is kept apart from the load so that a group of
// loads can all be issued before the first result is used.
template <class V>
struct vload {
  // register type of a raw value: BF16 bits are held zero-extended in a full
  // 32-bit register (two of them packed in one register would make the
  // compiler wait for the first load before packing)
  using R = typename std::conditional<sizeof(V) == 2, uint32_t, V>::type;
  static __device__ __forceinline__ R nt(gptr<V> p, int64_t i) { return (R)__builtin_nontemporal_load(p + i); }
  static __device__ __forceinline__ R ld(gptr<V> p, int64_t i) { return (R)p[i]; }
  template <class X>
  static __device__ __forceinline__ X cvt(R v) {
    if constexpr (sizeof(V) == 2) {
      // the empty statement keeps the shift here: without it the compiler
      // moves the shift up into the branch of the load, right after it, and
      // has to wait for that load there
      uint32_t u = v;
      asm volatile("" : "+v"(u));
      return (X)__uint_as_float(u << 16);
    } else {
      return (X)v;
    }
  }
};

// Entry words (row offset in its tile) << SH | (column offset in its tile):
// 16-bit words with SH = 8 for tiles of at most 256 rows, 32-bit words with
// SH = 16 for taller ones.  Loads return the word zero-extended in a full
// register, one load per register.  The compiler then keeps the same load
// and wait order for both widths, so no asm barrier is needed before the
// decode (one there cost 11 registers and slowed the solver epilogues).
template <class E>
struct eword {
  static constexpr int SH = sizeof(E) == 2 ? 8 : 16;
  static __device__ __forceinline__ uint32_t ld(gptr<E> p, int64_t i) { return (uint32_t)p[i]; }
  static __device__ __forceinline__ uint32_t nt(gptr<E> p, int64_t i) {
    return (uint32_t)__builtin_nontemporal_load(p + i);
  }
  static __device__ __forceinline__ void decode(uint32_t w, int32_t &ri, int32_t &cj) {
    ri = (int32_t)(w >> SH);
    cj = (int32_t)(w & ((1u << SH) - 1u));
  }
};

// The k values of one row of x (or y) as 16-byte vector accesses where the
// row is a whole number of them (rows of k >= 2 values are 16-byte aligned:
// the library requires 16-byte aligned vectors when k >= 2).
template <class X, int K>
struct rowvec {
  static constexpr int W = 16 / sizeof(X);  // values per 16 bytes
  static constexpr bool VEC = K >= W && K % W == 0;
  typedef X V4 __attribute__((ext_vector_type(W)));
  static __device__ __forceinline__ void load(gptr<X> p, int64_t row, X (&v)[K]) {
    if constexpr (VEC) {
      gptr<V4> q = (gptr<V4>)(p + row * K);
#pragma unroll
      for (int u = 0; u < K / W; u++) {
        const V4 t = q[u];
#pragma unroll
        for (int w = 0; w < W; w++) v[u * W + w] = t[w];
      }
    } else {
#pragma unroll
      for (int c = 0; c < K; c++) v[c] = p[row * K + c];
    }
  }
  static __device__ __forceinline__ void store(gmut<X> p, int64_t row, const X (&v)[K]) {
    if constexpr (VEC) {
      gmut<V4> q = (gmut<V4>)(p + row * K);
#pragma unroll
      for (int u = 0; u < K / W; u++) {
        V4 t;
#pragma unroll
        for (int w = 0; w < W; w++) t[w] = v[u * W + w];
        q[u] = t;
      }
    } else {
#pragma unroll
      for (int c = 0; c < K; c++) p[row * K + c] = v[c];
    }
  }
};

// Workgroups are dispatched round-robin over the 8 XCDs: block b runs on XCD
// b % 8.  Give every XCD a contiguous range of tiles, taken in ascending order.
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t ntiles) {
  const int32_t per = (ntiles + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// One group of chunks (one per q) in three phases: the entry loads, then the
// x gathers, then the products added into the LDS row sums; a descriptor
// with .y == CHUNK_EMPTY is skipped.  sym: the column side adds l_ij x_i
// (symmetric S) instead of subtracting it.  Every load of a phase is issued
// before any result is used.  Lanes past a chunk's end re-read its last entry
// (in bounds, the same cache line) and are masked only when their product is
// added; the only branches around loads test the wave-uniform descriptors.
// (A lane-divergent branch around a load whose result is used inside it
// makes the compiler wait for that load before the next one is issued.)
template <class V>
struct group_entries {
  uint32_t rc[PRE];
  typename vload<V>::R vv[PRE];
};
template <class X, int K>
struct group_gathers {
  int32_t slot[PRE];
  X coef[PRE], xv[PRE][K];
};

template <class V, class E>
__device__ __forceinline__ void group_load(const uint2 (&d)[PRE], int32_t lane, gptr<E> ent_rc, gptr<V> ent_v,
                                           group_entries<V> &g) {
#pragma unroll
  for (int q = 0; q < PRE; q++) {
    g.rc[q] = 0u;
    g.vv[q] = 0;
    if (d[q].y == CHUNK_EMPTY) continue;  // wave-uniform: no load at all
    const int32_t len = (int32_t)(d[q].y & 127u) + 1;
    const int64_t e = (int64_t)d[q].x + min(lane, len - 1);
    // the column side reads a block first and leaves it in L2; the row side
    // is its last use (nontemporal)
    if ((d[q].y >> 7) & 1u) {
      g.rc[q] = eword<E>::ld(ent_rc, e);
      g.vv[q] = vload<V>::ld(ent_v, e);
    } else {
      g.rc[q] = eword<E>::nt(ent_rc, e);
      g.vv[q] = vload<V>::nt(ent_v, e);
    }
  }
}

template <class V, class X, int K, class E>
__device__ __forceinline__ void group_gather(const uint2 (&d)[PRE], int32_t lane, int32_t lgT, bool sym,
                                             const group_entries<V> &g, gptr<X> x, group_gathers<X, K> &h) {
  int32_t xrow[PRE];
#pragma unroll
  for (int q = 0; q < PRE; q++) {
    h.slot[q] = -1;
    xrow[q] = 0;
    h.coef[q] = (X)0;
    if (d[q].y != CHUNK_EMPTY) {
      const int32_t len = (int32_t)(d[q].y & 127u) + 1;
      const bool col_side = (d[q].y >> 7) & 1u;
      const int32_t other = (int32_t)(d[q].y >> 8);
      int32_t ri, cj;
      eword<E>::decode(g.rc[q], ri, cj);
      const X val = vload<V>::template cvt<X>(g.vv[q]);
      h.slot[q] = lane < len ? (col_side ? cj : ri) : -1;
      xrow[q] = (other << lgT) + (col_side ? ri : cj);
      h.coef[q] = col_side && !sym ? -val : val;
    }
  }
#pragma unroll
  for (int q = 0; q < PRE; q++) {
    if (d[q].y == CHUNK_EMPTY) {
#pragma unroll
      for (int c = 0; c < K; c++) h.xv[q][c] = (X)0;
    } else {
      rowvec<X, K>::load(x, xrow[q], h.xv[q]);
    }
  }
}

template <class X, int K>
__device__ __forceinline__ void group_add(const group_gathers<X, K> &h, double *ys) {
#pragma unroll
  for (int q = 0; q < PRE; q++)
    if (h.slot[q] >= 0) {
#pragma unroll
      for (int c = 0; c < K; c++) atomicAdd(&ys[h.slot[q] * KP<K> + c], (double)(h.coef[q] * h.xv[q][c]));
    }
}

// The x gathers and LDS adds of a group, for 8 right-hand sides: in H parts
// of PRE / H chunks, since the x rows of all PRE chunks would hold 64
// registers (128 for FP64) and leave room for 5 wavefronts per SIMD or fewer
// instead of 8.  The group's entry loads still all go out together.
template <class V, class X, int K, class E>
__device__ __forceinline__ void gather_add_parts(const uint2 (&d)[PRE], int32_t lane, int32_t lgT, bool sym,
                                                 const group_entries<V> &g, gptr<X> x, double *ys) {
  constexpr int H = sizeof(X) == 8 ? 4 : 2;
  constexpr int QH = PRE / H;
  int32_t slot[PRE], xrow[PRE];
  X coef[PRE];
#pragma unroll
  for (int q = 0; q < PRE; q++) {
    slot[q] = -1;
    xrow[q] = 0;
    coef[q] = (X)0;
    if (d[q].y != CHUNK_EMPTY) {
      const int32_t len = (int32_t)(d[q].y & 127u) + 1;
      const bool col_side = (d[q].y >> 7) & 1u;
      const int32_t other = (int32_t)(d[q].y >> 8);
      int32_t ri, cj;
      eword<E>::decode(g.rc[q], ri, cj);
      const X val = vload<V>::template cvt<X>(g.vv[q]);
      slot[q] = lane < len ? (col_side ? cj : ri) : -1;
      xrow[q] = (other << lgT) + (col_side ? ri : cj);
      coef[q] = col_side && !sym ? -val : val;
    }
  }
#pragma unroll
  for (int h = 0; h < H; h++) {
    X xv[QH][K];
#pragma unroll
    for (int i = 0; i < QH; i++) {
      const int q = h * QH + i;
      if (d[q].y == CHUNK_EMPTY) {
#pragma unroll
        for (int c = 0; c < K; c++) xv[i][c] = (X)0;
      } else {
        rowvec<X, K>::load(x, xrow[q], xv[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < QH; i++) {
      const int q = h * QH + i;
      if (slot[q] >= 0) {
#pragma unroll
        for (int c = 0; c < K; c++) atomicAdd(&ys[slot[q] * KP<K> + c], (double)(coef[q] * xv[i][c]));
      }
    }
  }
}

template <class V, class X, int K, class E>
__device__ __forceinline__ void chunk_group(const uint2 (&d)[PRE], int32_t lane, int32_t lgT, bool sym,
                                            gptr<E> ent_rc, gptr<V> ent_v, gptr<X> x, double *ys) {
  group_entries<V> g;
  group_load<V, E>(d, lane, ent_rc, ent_v, g);
  if constexpr (K < 8) {
    group_gathers<X, K> h;
    group_gather<V, X, K, E>(d, lane, lgT, sym, g, x, h);
    group_add<X, K>(h, ys);
  } else {
    gather_add_parts<V, X, K, E>(d, lane, lgT, sym, g, x, ys);
  }
}

// What the solver epilogue reads besides the row sums: for the thread's first
// own row the vectors, and two of the iteration's coefficients.  In a
// single-matrix product they are requested when the tile starts, so their
// latency passes while the tile's gathers run instead of adding one more
// memory round trip after them (MRS to 1e-10 on a 2M-row stencil: 2.5%
// faster in FP64 and with FP32 inner solves, 8.5% with BF16 ones).  The
// batched product requests them at the end: there the early loads made the
// batched solve 2% slower.  (The five update coefficients are read at the end
// in both: held from the start they would take the scalar registers of one
// wavefront per SIMD.)
template <class X>
struct ep_pre {
  X sc = (X)1, zb = (X)0;
  bool upd = false;
  X z = (X)0, p1 = (X)0, p2 = (X)0, xs = (X)0;
};

template <class X, int K>
__device__ __forceinline__ void ep_load(const prod_task &a, int64_t row, ep_pre<X> &e) {
  if (a.scale) e.sc = (X)glb(a.scale)[0];
  if (a.z) {
    e.zb = (X)glb(a.beta)[0];
    if constexpr (K == 1) e.z = glb((const X *)a.z)[row];
  }
  if (K == 1 && a.vec) {
    // the rows are read whether or not the update is due (the buffers exist
    // for every solver task); only their use depends on the active flag
    e.upd = glb(a.active)[0] != 0;
    e.p1 = glb((const X *)a.p1)[row];
    e.p2 = glb((const X *)a.p2)[row];
    e.xs = glb((const X *)a.xs)[row];
  }
}

// Output phase of a tile (after its LDS row sums are complete): y = (shift
// + d_i) x + inner band + LDS sum (+ the solver epilogue), one store per row.
// PF: the epilogue's first-row vectors and coefficients were requested when
// the tile started (ep); otherwise they are read here.
template <class V, class X, int K, bool EP, bool GEN, bool PF>
__device__ __forceinline__ void tile_final(const prod_task &a, int32_t t, const X (&xown)[K], const ep_pre<X> &ep,
                                           const double *ys, double *s_red) {
  gptr<V> dia = glb((const V *)a.dia);
  gptr<X> x = glb((const X *)a.x);
  gmut<X> y = glbw((X *)a.y);
  gptr<X> z = glb((const X *)a.z);
  gptr<X> dg = GEN ? glb((const X *)a.dg) : nullptr;
  const int32_t n = a.n, w_in = a.w_in;
  const X shift = (X)a.shift;
  const bool sym = GEN && a.sym != 0;
  const int32_t r0 = t << a.lgT;
  const int32_t rows = min(1 << a.lgT, n - r0);
  // fused solver iteration: scale of S x, and the pending vector update
  X sc = ep.sc;
  bool upd = K == 1 && a.vec && ep.upd;
  if constexpr (EP && !PF) {
    sc = a.scale ? (X)glb(a.scale)[0] : (X)1;
    upd = K == 1 && a.vec && glb(a.active)[0];
  }
  double vd = 0.0, ve = 0.0, vg = 1.0, vc = 0.0, vn = 0.0;
  if (EP && upd) {
    gptr<double> vec = glb(a.vec);
    vd = vec[0];
    ve = vec[1];
    vg = vec[2];
    vc = vec[3];
    vn = vec[4];
  }
  double sq = 0.0;
  for (int32_t r = threadIdx.x, rr = 0; r < rows; r += TB, rr++) {
    const int64_t i = r0 + r;
    X acc[K];
#pragma unroll
    for (int c = 0; c < K; c++) acc[c] = (X)ys[r * KP<K> + c];
    // inner band in both directions, KB diagonals at a time: their loads are
    // all issued before the first is used (indices clamped into range; terms
    // outside the matrix, past w_in or on structural zeros are masked after)
    constexpr int KB = K <= 2 ? 4 : (K == 4 ? 2 : 1);
    for (int32_t k0 = 1; k0 <= w_in; k0 += KB) {
      typename vload<V>::R lv[KB], uv[KB];
      X xl[KB][K], xu[KB][K];
#pragma unroll
      for (int u = 0; u < KB; u++) {
        const int32_t k = min(k0 + u, w_in);
        const int64_t bse = (int64_t)(k - 1) * n;
        const int64_t il = i - k >= 0 ? i - k : 0, iu = i + k < n ? i + k : (int64_t)n - 1;
        lv[u] = vload<V>::nt(dia, bse + i);
        uv[u] = vload<V>::nt(dia, bse + iu);
        rowvec<X, K>::load(x, il, xl[u]);
        rowvec<X, K>::load(x, iu, xu[u]);
      }
#pragma unroll
      for (int u = 0; u < KB; u++) {
        const int32_t k = k0 + u;
        const X l = k <= w_in && i - k >= 0 ? vload<V>::template cvt<X>(lv[u]) : (X)0;  // S_i,i-k
        const X m = k <= w_in && i + k < n ? vload<V>::template cvt<X>(uv[u]) : (X)0;
        const X lu = sym ? m : -m;  // S_i,i+k
        if (l != (X)0) {
#pragma unroll
          for (int c = 0; c < K; c++) acc[c] += l * xl[u][c];
        }
        if (m != (X)0) {
#pragma unroll
          for (int c = 0; c < K; c++) acc[c] += lu * xu[u][c];
        }
      }
    }
    const X sh = dg ? shift + dg[i] : shift;
#pragma unroll
    for (int c = 0; c < K; c++) {
      const X xi = rr == 0 ? xown[c] : x[i * K + c];
      acc[c] = EP ? sh * xi + sc * acc[c] : sh * xi + acc[c];
    }
    if (EP && z) {
      const X zb = PF ? ep.zb : (X)glb(a.beta)[0];
      if constexpr (K == 1) {
        const X zi = PF && rr == 0 ? ep.z : z[i];
        acc[0] += zb * zi;
        if (upd) {
          gmut<X> p2 = glbw((X *)a.p2);
          gmut<X> xs = glbw((X *)a.xs);
          gptr<X> p1 = glb((const X *)a.p1);
          const X p1i = PF && rr == 0 ? ep.p1 : p1[i], p2i = PF && rr == 0 ? ep.p2 : p2[i];
          const X xsi = PF && rr == 0 ? ep.xs : xs[i];
          const double pn = ((double)zi * vn - vd * (double)p1i - ve * (double)p2i) / vg;
          p2[i] = (X)pn;
          xs[i] = (X)((double)xsi + vc * pn);
        }
      } else {
#pragma unroll
        for (int c = 0; c < K; c++) acc[c] += zb * z[i * K + c];
      }
    }
    rowvec<X, K>::store(y, i, acc);
#pragma unroll
    for (int c = 0; c < K; c++) sq += (double)acc[c] * (double)acc[c];
  }
  if (EP && a.partials) {
    // partial sum of squares of the tile's outputs, in a fixed order
#pragma unroll
    for (int d2 = 32; d2 >= 1; d2 >>= 1) sq += __shfl_xor(sq, d2, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int w = 0; w < TB / 64; w++) tot += s_red[w];
      a.partials[t] = tot;
    }
  }
}

// The tile's work list is a list of chunks, runs of at most 64 consecutive
// entries of one block.  A wavefront takes whole chunks, so a chunk's
// descriptor (first entry, length, other tile, side) is uniform over the
// wavefront and lives in scalar registers: each lane only loads its entry
// word, value and x element and adds one product into LDS.  The first group
// of descriptors sits at fixed positions per tile, so its loads depend on
// nothing.  Partial sums are kept in FP64 in LDS whatever the vector type
// (products are formed in the vector precision); LDS adds of FP64 measured
// faster than of FP32 here.  Called by every thread of the workgroup.  EP:
// the solver epilogue (y += beta z, per-tile sums of y^2) is compiled in.
// GEN: the task's kind (symmetric or skew) and diagonal array are honoured;
// without it the product is the skew one with the scalar shift only.  E:
// the type of the entry words (uint16_t for tiles of at most 256 rows).
template <class V, class X, int K, bool EP, bool GEN, class E, bool PF>
__device__ __forceinline__ void tile_body(const prod_task &a, int32_t t, double *ys, double *s_red) {
  gptr<V> ent_v = glb((const V *)a.ent_v);
  gptr<E> ent_rc = glb((const E *)a.ent_rc);
  gptr<X> x = glb((const X *)a.x);
  const int32_t n = a.n, lgT = a.lgT;
  const int32_t T = 1 << lgT;
  const int32_t r0 = t << lgT;
  const int32_t rows = min(T, n - r0);
  const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x >> 6);
  const int32_t lane = threadIdx.x & 63;
  // descriptors of the first group, the overflow range, the first group's
  // entries and x of the thread's first own row are requested before the
  // LDS row sums are cleared
  uint2 d[PRE];
#pragma unroll
  for (int q = 0; q < PRE; q++) d[q] = load_desc(a.chunk_fix, (int64_t)t * CHUNKS_FIXED + wave * PRE + q);
  const int32_t o0 = glb(a.ovf_ptr)[t], o1 = glb(a.ovf_ptr)[t + 1];
  group_entries<V> g;
  group_load<V, E>(d, lane, ent_rc, ent_v, g);
  // own x row, clamped into the matrix (a thread past the last row keeps a
  // value it never uses) so that no branch surrounds the load
  X xown[K];
  rowvec<X, K>::load(x, min((int64_t)r0 + threadIdx.x, (int64_t)n - 1), xown);
  ep_pre<X> ep;
  if constexpr (EP && PF) ep_load<X, K>(a, min((int64_t)r0 + threadIdx.x, (int64_t)n - 1), ep);
  for (int32_t s = threadIdx.x; s < rows * KP<K>; s += TB) ys[s] = 0.0;
  __syncthreads();
  if constexpr (K < 8) {
    group_gathers<X, K> h;
    group_gather<V, X, K, E>(d, lane, lgT, GEN && a.sym != 0, g, x, h);
    group_add<X, K>(h, ys);
  } else {
    gather_add_parts<V, X, K, E>(d, lane, lgT, GEN && a.sym != 0, g, x, ys);
  }
  for (int32_t cb = o0 + wave; cb < o1; cb += (TB / 64) * PRE) {
#pragma unroll
    for (int q = 0; q < PRE; q++) {
      const int32_t c = cb + q * (TB / 64);
      // past the end: a re-read of the last descriptor, marked empty (no
      // branch around the load, which would make the compiler wait for it)
      d[q] = load_desc(a.chunk_ovf, min(c, o1 - 1));
      if (c >= o1) d[q].y = CHUNK_EMPTY;
    }
    // all 8 descriptor loads go out before the first entry load (left to
    // itself the scheduler interleaves them and waits once per chunk)
    __builtin_amdgcn_sched_barrier(0);
    chunk_group<V, X, K, E>(d, lane, lgT, GEN && a.sym != 0, ent_rc, ent_v, x, ys);
  }
  __syncthreads();
  tile_final<V, X, K, EP, GEN, PF>(a, t, xown, ep, ys, s_red);
}

// One matrix: one workgroup per tile.  EP: with the solver epilogue (a
// finished solver's done flag skips the whole launch).  GEN: symmetric kind
// and diagonal array.  E: the entry word type of the layout's tile height.
template <class V, class X, int K, bool EP, bool GEN, class E>
__global__ __launch_bounds__(TB) void k_tile_product(const prod_task a) {
  __shared__ double s_red[TB / 64];
  extern __shared__ double ys[];
  // a finished solver skips its remaining products, except the one that
  // still carries its last vector update
  if (EP && a.done && glb(a.done)[0] && !(a.active && glb(a.active)[0])) return;
  const int32_t t = xcd_tile(blockIdx.x, a.ntiles);
  if (t >= a.ntiles) return;
  tile_body<V, X, K, EP, GEN, E, EP>(a, t, ys, s_red);
}


// Many matrices in one launch: the (matrix, tile) items are split into 8
// queues, one per XCD (workgroup b runs on XCD b % 8), each ordered by
// matrix and ascending tile.  Workgroup b takes item b / 8 of queue b % 8 (the
// grid covers the longest queue; workgroups past the end of a shorter one
// return at once), so each XCD walks its queue in order while the hardware
// dispatcher starts a new item as soon as any workgroup ends.  Items of a
// matrix whose solver has finished are skipped.  EW: the entry word size of
// every task (2 or 4 bytes), or 0 when the tasks mix tile heights on both
// sides of 256 rows and each item picks its type (a branch uniform over the
// workgroup).
template <class V, class X, int K, bool EP, bool GEN, int EW>
__global__ __launch_bounds__(TB) void k_batch_product(const prod_task *__restrict__ tasks,
                                                      const int2 *__restrict__ items,
                                                      const int32_t *__restrict__ qbeg) {
  __shared__ double s_red[TB / 64];
  extern __shared__ double ys[];
  const int q = blockIdx.x & 7;
  const int32_t it = qbeg[q] + (int32_t)(blockIdx.x >> 3);
  if (it >= qbeg[q + 1]) return;
  const int2 w = items[it];
  const prod_task &a = tasks[w.x];
  if (EP && a.done && glb(a.done)[0] && !(a.active && glb(a.active)[0])) return;
  if constexpr (EW == 2) {
    tile_body<V, X, K, EP, GEN, uint16_t, false>(a, w.y, ys, s_red);
  } else if constexpr (EW == 4) {
    tile_body<V, X, K, EP, GEN, uint32_t, false>(a, w.y, ys, s_red);
  } else {
    if (a.lgT <= ENT16_MAX_LGT) tile_body<V, X, K, EP, GEN, uint16_t, false>(a, w.y, ys, s_red);
    else tile_body<V, X, K, EP, GEN, uint32_t, false>(a, w.y, ys, s_red);
  }
}

template <class F>
static pars3_status raise_lds(F *kernel, size_t lds) {
  if (lds + sizeof(double) * (TB / 64) + 64 > LDS_DEFAULT)
    P3_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return PARS3_OK;
}

template <class V, class X, int K, bool EP, bool GEN, class E>
static pars3_status launch_e(pars3_matrix *A, const V *in_v, const V *ent_v, X shift, const X *x, X *y,
                             hipStream_t s, const epilogue<X> &ep) {
  const layout &L = A->lay;
  const int32_t n = (int32_t)A->n;
  if (n == 0) return PARS3_OK;
  const size_t lds = (size_t)L.T * KP<K> * sizeof(double);
  static bool raised = false;  // above the default dynamic LDS limit: ask for exactly what is needed
  if (!raised && lds + sizeof(double) * (TB / 64) > LDS_DEFAULT) {
    P3_TRY(raise_lds(k_tile_product<V, X, K, EP, GEN, E>, (size_t)1024 * KP<K> * sizeof(double)));
    raised = true;
  }
  prod_task a{};
  a.chunk_fix = L.chunk_fix.p;
  a.ovf_ptr = L.ovf_ptr.p;
  a.chunk_ovf = L.chunk_ovf.p;
  a.ent_rc = sizeof(E) == 2 ? (const void *)L.ent_rc16.p : (const void *)L.ent_rc.p;
  a.ent_v = ent_v;
  a.dia = in_v;
  a.w_in = L.w_in;
  a.ntiles = L.ntiles;
  a.lgT = L.lgT;
  a.n = n;
  a.sym = A->kind == PARS3_SYMMETRIC ? 1 : 0;
  a.dg = sizeof(X) == 8 ? (const void *)A->pdiag.p : (const void *)A->pdiag32.p;
  a.shift = (double)shift;
  a.x = x;
  a.y = y;
  a.z = ep.z;
  a.beta = ep.beta;
  a.partials = ep.partials;
  a.done = ep.done;
  a.scale = ep.scale;
  a.vec = ep.vec;
  a.active = ep.active;
  a.p1 = ep.p1;
  a.p2 = ep.p2;
  a.xs = ep.xs;
  P3_TRY(prof_mark(A, PROF_BAND, 0, s));
  const unsigned grid = (unsigned)(8 * cdiv(L.ntiles, 8));
  k_tile_product<V, X, K, EP, GEN, E><<<grid, TB, lds, s>>>(a);
  P3_LAUNCHED();
  P3_TRY(prof_mark(A, PROF_BAND, 1, s));
  return PARS3_OK;
}

template <class V, class X, int K, bool EP, bool GEN>
static pars3_status launch(pars3_matrix *A, const V *in_v, const V *ent_v, X shift, const X *x, X *y, hipStream_t s,
                           const epilogue<X> &ep) {
  if (A->lay.lgT <= ENT16_MAX_LGT) return launch_e<V, X, K, EP, GEN, uint16_t>(A, in_v, ent_v, shift, x, y, s, ep);
  return launch_e<V, X, K, EP, GEN, uint32_t>(A, in_v, ent_v, shift, x, y, s, ep);
}

template <class V, class X>
static pars3_status dispatch_k(pars3_matrix *A, const V *in_v, const V *ent_v, double shift, const void *x, void *y,
                               int k, hipStream_t s, const void *epv) {
  const X *xx = (const X *)x;
  X *yy = (X *)y;
  epilogue<X> ep{};
  if (epv) {
    // products with the solver epilogue are a kernel of their own
    ep = *(const epilogue<X> *)epv;
    if (k != 1) return fail(PARS3_EINVAL, "spmv: the solver epilogue takes one right-hand side");
    if (is_general(A)) return fail(PARS3_ESTATE, "spmv: the solver epilogue needs a skew matrix without diagonal");
    return launch<V, X, 1, true, false>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
  }
  if (is_general(A)) {
    switch (k) {
      case 1: return launch<V, X, 1, false, true>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
      case 2: return launch<V, X, 2, false, true>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
      case 4: return launch<V, X, 4, false, true>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
      case 8: return launch<V, X, 8, false, true>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
      default: return fail(PARS3_EINVAL, "spmv: k must be 1, 2, 4 or 8 (got %d)", k);
    }
  }
  switch (k) {
    case 1: return launch<V, X, 1, false, false>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
    case 2: return launch<V, X, 2, false, false>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
    case 4: return launch<V, X, 4, false, false>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
    case 8: return launch<V, X, 8, false, false>(A, in_v, ent_v, (X)shift, xx, yy, s, ep);
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

pars3_status spmv_ex(pars3_matrix *A, double shift, const void *x, void *y, int k, int vec_dtype, int value_dtype,
                     hipStream_t s, const void *ep) {
  const layout &L = A->lay;
  if (A->prof.on && A->prof.calls < PROF_MAX) A->prof.calls++;
  if (vec_dtype == PARS3_F64) {
    if (!A->has_f64) return fail(PARS3_ESTATE, "spmv: FP64 values are not stored (value_dtype/keep_fp64)");
    return dispatch_k<double, double>(A, L.in_f64.p, L.ent_f64.p, shift, x, y, k, s, ep);
  }
  if (vec_dtype == PARS3_F32) {
    const bool use32 = A->has_f32 && value_dtype != PARS3_BF16;
    const bool use16 = A->has_bf16 && value_dtype != PARS3_F32;
    if (use32) return dispatch_k<float, float>(A, L.in_f32.p, L.ent_f32.p, shift, x, y, k, s, ep);
    if (use16) return dispatch_k<uint16_t, float>(A, L.in_bf16.p, L.ent_bf16.p, shift, x, y, k, s, ep);
    return fail(PARS3_ESTATE, "spmv: no FP32 or BF16 values are stored for FP32 vectors");
  }
  return fail(PARS3_EINVAL, "spmv: vec_dtype must be PARS3_F64 or PARS3_F32");
}

pars3_status spmv_rcm(pars3_matrix *A, double shift, const void *x, void *y, int k, int vec_dtype, hipStream_t s) {
  // engine PARS3_ENGINE_CSR: one right-hand side in the CSR's own precision
  if (A->csr && k == 1 && vec_dtype == csr_vdtype(A->csr)) return csr_product(A->csr, shift, x, y, s);
  return spmv_ex(A, shift, x, y, k, vec_dtype, -1, s, nullptr);
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

// ------------------------------------------------------------ batched products
pars3_status make_task(const pars3_matrix *A, int vec_dtype, int value_dtype, prod_task *a, int *vkind) {
  const layout &L = A->lay;
  *a = prod_task{};
  a->chunk_fix = L.chunk_fix.p;
  a->ovf_ptr = L.ovf_ptr.p;
  a->chunk_ovf = L.chunk_ovf.p;
  a->ent_rc = L.lgT <= ENT16_MAX_LGT ? (const void *)L.ent_rc16.p : (const void *)L.ent_rc.p;
  a->w_in = L.w_in;
  a->ntiles = L.ntiles;
  a->lgT = L.lgT;
  a->n = (int32_t)A->n;
  a->sym = A->kind == PARS3_SYMMETRIC ? 1 : 0;
  a->dg = vec_dtype == PARS3_F64 ? (const void *)A->pdiag.p : (const void *)A->pdiag32.p;
  if (vec_dtype == PARS3_F64) {
    if (!A->has_f64) return fail(PARS3_ESTATE, "batch: a matrix has no FP64 values");
    a->ent_v = L.ent_f64.p;
    a->dia = L.in_f64.p;
    *vkind = PARS3_F64;
    return PARS3_OK;
  }
  const bool use32 = A->has_f32 && value_dtype != PARS3_BF16;
  const bool use16 = A->has_bf16 && value_dtype != PARS3_F32;
  if (use32) {
    a->ent_v = L.ent_f32.p;
    a->dia = L.in_f32.p;
    *vkind = PARS3_F32;
  } else if (use16) {
    a->ent_v = L.ent_bf16.p;
    a->dia = L.in_bf16.p;
    *vkind = PARS3_BF16;
  } else {
    return fail(PARS3_ESTATE, "batch: a matrix has no FP32 or BF16 values");
  }
  return PARS3_OK;
}

template <class V, class X, int K, bool EP, bool GEN, int EW>
static pars3_status launch_batch_e(const prod_task *tasks, const int2 *items, const int32_t *qbeg, int32_t grid,
                                   int32_t maxT, hipStream_t s) {
  const size_t lds = (size_t)maxT * KP<K> * sizeof(double);
  static bool raised = false;
  if (!raised && lds + sizeof(double) * (TB / 64) + 64 > LDS_DEFAULT) {
    P3_TRY(raise_lds(k_batch_product<V, X, K, EP, GEN, EW>, (size_t)1024 * KP<K> * sizeof(double)));
    raised = true;
  }
  k_batch_product<V, X, K, EP, GEN, EW><<<(unsigned)grid, TB, lds, s>>>(tasks, items, qbeg);
  P3_LAUNCHED();
  return PARS3_OK;
}

template <class V, class X, int K, bool EP, bool GEN>
static pars3_status launch_batch_k(const prod_task *tasks, const int2 *items, const int32_t *qbeg, int32_t grid,
                                   int32_t minT, int32_t maxT, hipStream_t s) {
  constexpr int32_t T16 = 1 << ENT16_MAX_LGT;
  if (maxT <= T16) return launch_batch_e<V, X, K, EP, GEN, 2>(tasks, items, qbeg, grid, maxT, s);
  if (minT > T16) return launch_batch_e<V, X, K, EP, GEN, 4>(tasks, items, qbeg, grid, maxT, s);
  return launch_batch_e<V, X, K, EP, GEN, 0>(tasks, items, qbeg, grid, maxT, s);
}

template <class V, class X, bool GEN>
static pars3_status launch_batch_g(int k, const prod_task *tasks, const int2 *items, const int32_t *qbeg,
                                   int32_t grid, int32_t minT, int32_t maxT, hipStream_t s) {
  switch (k) {
    case 1: return launch_batch_k<V, X, 1, false, GEN>(tasks, items, qbeg, grid, minT, maxT, s);
    case 2: return launch_batch_k<V, X, 2, false, GEN>(tasks, items, qbeg, grid, minT, maxT, s);
    case 4: return launch_batch_k<V, X, 4, false, GEN>(tasks, items, qbeg, grid, minT, maxT, s);
    case 8: return launch_batch_k<V, X, 8, false, GEN>(tasks, items, qbeg, grid, minT, maxT, s);
    default: return fail(PARS3_EINVAL, "batch: k must be 1, 2, 4 or 8 (got %d)", k);
  }
}

template <class V, class X>
static pars3_status launch_batch_v(int k, bool ep, bool gen, const prod_task *tasks, const int2 *items,
                                   const int32_t *qbeg, int32_t grid, int32_t minT, int32_t maxT, hipStream_t s) {
  if (ep) {
    if (k != 1) return fail(PARS3_EINVAL, "batch: the solver epilogue takes one right-hand side");
    if (gen) return fail(PARS3_ESTATE, "batch: the solver epilogue needs skew matrices without diagonal");
    return launch_batch_k<V, X, 1, true, false>(tasks, items, qbeg, grid, minT, maxT, s);
  }
  if (gen) return launch_batch_g<V, X, true>(k, tasks, items, qbeg, grid, minT, maxT, s);
  return launch_batch_g<V, X, false>(k, tasks, items, qbeg, grid, minT, maxT, s);
}

pars3_status launch_batch(int vkind, int k, bool ep, bool gen, const prod_task *tasks, const int2 *items,
                          const int32_t *qbeg, int32_t grid, int32_t minT, int32_t maxT, hipStream_t s) {
  if (vkind == PARS3_F64) return launch_batch_v<double, double>(k, ep, gen, tasks, items, qbeg, grid, minT, maxT, s);
  if (vkind == PARS3_F32) return launch_batch_v<float, float>(k, ep, gen, tasks, items, qbeg, grid, minT, maxT, s);
  return launch_batch_v<uint16_t, float>(k, ep, gen, tasks, items, qbeg, grid, minT, maxT, s);
}

}  // namespace p3
