// Reverse Cuthill-McKee on the GPU and the sign-fixing symmetric permutation
// (Sections 1 and 3.1.2: the matrix is reordered into a band before the
// split).
//
// The order is the one fixed by this tie-break: components in ascending
// (min degree, min index) of their nodes; in each component a George-Liu
// pseudo-peripheral start found from the (min degree, min index) node;
// Cuthill-McKee breadth-first order with neighbours taken in ascending
// (degree, index); the whole concatenated order reversed.
//
// Parallel formulation.  In a FIFO breadth-first search all nodes of level l
// leave the queue before any node of level l+1, and a node of level l+1 is
// queued by its earliest-queued neighbour in level l; children of one parent
// are queued in (degree, index) order.  Hence the order inside level l+1 is
// lexicographic in (min position of a level-l neighbour, degree, index).  Each
// level is therefore computed as: claim the parent (atomic min of positions),
// count the children of every frontier node, prefix-sum the counts, and let
// every frontier node write its children in its (degree, index)-sorted
// adjacency order.  All components advance together; a component's level l+1
// starts right after its level l.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace p3 {

static constexpr int TB = 256;
static inline unsigned nblk(int64_t m) { return (unsigned)std::max<int64_t>(1, cdiv(m, TB)); }

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ symmetrise
__global__ void k_count_upper(const int32_t *__restrict__ col, int64_t nnz, int32_t *__restrict__ ucnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&ucnt[col[e]], 1);
}
__global__ void k_degree(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ ucnt, int32_t n,
                         int32_t *__restrict__ deg) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) deg[v] = rowptr[v + 1] - rowptr[v] + ucnt[v];
}
// Row v of the adjacency: its stored lower columns, then (in arbitrary order)
// the rows that store v as a column.
__global__ void k_fill_adj(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t n,
                           const int32_t *__restrict__ aptr, int32_t *__restrict__ ufill, int32_t *__restrict__ adj) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t a = aptr[v];
  for (int32_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
    int32_t j = col[e];
    adj[a++] = j;
    int32_t slot = atomicAdd(&ufill[j], 1);
    adj[aptr[j] + (rowptr[j + 1] - rowptr[j]) + slot] = v;
  }
}
__device__ __forceinline__ int32_t row_of(const int32_t *__restrict__ ptr, int32_t n, int64_t e) {
  int32_t lo = 0, hi = n - 1;  // largest r with ptr[r] <= e
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
// Sort every adjacency row by (degree, index): each element's destination is
// the number of row elements with a smaller key (keys are distinct).
__global__ void k_sort_adj(const int32_t *__restrict__ aptr, const int32_t *__restrict__ adj, int32_t n, int64_t m,
                           const int32_t *__restrict__ deg, int32_t *__restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int32_t r = row_of(aptr, n, e);
  int32_t u = adj[e];
  uint64_t ku = ((uint64_t)(uint32_t)deg[u] << 32) | (uint32_t)u;
  int32_t rank = 0;
  for (int32_t t = aptr[r]; t < aptr[r + 1]; t++) {
    int32_t w = adj[t];
    uint64_t kw = ((uint64_t)(uint32_t)deg[w] << 32) | (uint32_t)w;
    rank += kw < ku;
  }
  out[aptr[r] + rank] = u;
}

// ------------------------------------------------------------ components
// Union-find with roots hooked larger-under-smaller by compare-and-swap; the
// final root of a component is its smallest node.
__device__ __forceinline__ int32_t uf_find(const int32_t *parent, int32_t x) {
  for (int guard = 0; guard < (1 << 26); guard++) {
    int32_t p = ld_relaxed(parent + x);
    if (p == x) return x;
    x = p;
  }
  return x;
}
__global__ void k_cc_hook(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t n,
                          int32_t *parent, int32_t *__restrict__ err) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
    int32_t j = col[e];
    bool done = false;
    for (int guard = 0; guard < (1 << 20) && !done; guard++) {
      int32_t a = uf_find(parent, i), b = uf_find(parent, j);
      if (a == b) {
        done = true;
        break;
      }
      if (a < b) {
        int32_t t = a;
        a = b;
        b = t;
      }
      if (atomicCAS(&parent[a], a, b) == a) done = true;
    }
    if (!done) atomicExch(err, 1);
  }
}
__global__ void k_cc_label(const int32_t *parent, int32_t n, int32_t *__restrict__ label) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) label[v] = uf_find(parent, v);
}
__global__ void k_comp_key(const int32_t *__restrict__ label, const int32_t *__restrict__ deg, int32_t n,
                           unsigned long long *__restrict__ ckey) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = v < n;
  const int64_t c = ok ? label[v] : 0;
  const unsigned long long key = ok ? (((unsigned long long)(uint32_t)deg[v] << 32) | (uint32_t)v) : ~0ull;
  agg_atomic_min<unsigned long long>(ckey, c, key, ok, ~0ull);
}
__global__ void k_is_root(const int32_t *__restrict__ label, int32_t n, int32_t *__restrict__ flag) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = label[v] == v;
}
__global__ void k_root_keys(const int32_t *__restrict__ label, const int32_t *__restrict__ rpos, int32_t n,
                            const unsigned long long *__restrict__ ckey, uint64_t *__restrict__ keys,
                            uint32_t *__restrict__ vals) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && label[v] == v) {
    keys[rpos[v]] = ckey[v];
    vals[rpos[v]] = (uint32_t)v;
  }
}
// rank of every root in component order; comp[v] = rank of v's component
__global__ void k_root_rank(const uint32_t *__restrict__ roots, int32_t C, int32_t *__restrict__ crank) {
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) crank[roots[c]] = c;
}
__global__ void k_comp_of(const int32_t *__restrict__ label, const int32_t *__restrict__ crank, int32_t n,
                          int32_t *__restrict__ comp, int32_t *__restrict__ csize) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = v < n;
  const int32_t c = ok ? crank[label[v]] : 0;
  if (ok) comp[v] = c;
  agg_atomic_add<int32_t>(csize, c, 1, ok);
}

// ------------------------------------------------------------ level BFS (levels only)
__global__ void k_bfs_seed(const int32_t *__restrict__ src, const int32_t *__restrict__ active, int32_t C,
                           int32_t *__restrict__ dist, int32_t *__restrict__ front, int32_t *__restrict__ fcount) {
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C && active[c]) {
    int32_t s = src[c];
    dist[s] = 0;
    front[atomicAdd(fcount, 1)] = s;
  }
}
__global__ void k_bfs_expand(const int32_t *__restrict__ front, int32_t f, const int32_t *__restrict__ aptr,
                             const int32_t *__restrict__ adj, int32_t *dist, int32_t level,
                             int32_t *__restrict__ next, int32_t *__restrict__ ncount) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f) return;
  int32_t v = front[t];
  for (int32_t e = aptr[v]; e < aptr[v + 1]; e++) {
    int32_t u = adj[e];
    if (ld_relaxed(dist + u) == -1 && atomicCAS(&dist[u], -1, level + 1) == -1) next[atomicAdd(ncount, 1)] = u;
  }
}
// eccentricity and (degree, index)-minimum of the last level, per component
__global__ void k_bfs_ecc(const int32_t *__restrict__ dist, const int32_t *__restrict__ comp, int32_t n,
                          int32_t *__restrict__ ecc) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = v < n && dist[v] >= 0;
  agg_atomic_max<int32_t>(ecc, ok ? comp[v] : 0, ok ? dist[v] : -1, ok, -1);
}
__global__ void k_bfs_cand(const int32_t *__restrict__ dist, const int32_t *__restrict__ comp,
                           const int32_t *__restrict__ deg, int32_t n, const int32_t *__restrict__ ecc,
                           unsigned long long *__restrict__ cand) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = v < n && dist[v] >= 0 && dist[v] == ecc[comp[v]];
  const unsigned long long key = ok ? (((unsigned long long)(uint32_t)deg[v] << 32) | (uint32_t)v) : ~0ull;
  agg_atomic_min<unsigned long long>(cand, ok ? comp[v] : 0, key, ok, ~0ull);
}
// George-Liu step per component (see rcm_gpu)
__global__ void k_gl_init(const unsigned long long *__restrict__ ckey_sorted, int32_t C, int32_t *__restrict__ s,
                          int32_t *__restrict__ active) {
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) {
    s[c] = (int32_t)(ckey_sorted[c] & 0xffffffffull);
    active[c] = 1;
  }
}
__global__ void k_gl_first(const int32_t *__restrict__ ecc, const unsigned long long *__restrict__ cand, int32_t C,
                           int32_t *__restrict__ ecc_s, unsigned long long *__restrict__ cand_s) {
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) {
    ecc_s[c] = ecc[c];
    cand_s[c] = cand[c];
  }
}
// before a round: a component whose candidate is its current start stops;
// the others search from their candidate u
__global__ void k_gl_pick(const int32_t *__restrict__ s, const unsigned long long *__restrict__ cand_s, int32_t C,
                          int32_t *__restrict__ active, int32_t *__restrict__ u, int32_t *__restrict__ nactive) {
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C || !active[c]) return;
  int32_t cu = (int32_t)(cand_s[c] & 0xffffffffull);
  if (cu == s[c]) {
    active[c] = 0;
  } else {
    u[c] = cu;
    atomicAdd(nactive, 1);
  }
}
// after a round: move to u if its eccentricity is larger, else stop
__global__ void k_gl_update(const int32_t *__restrict__ u, const int32_t *__restrict__ ecc,
                            const unsigned long long *__restrict__ cand, int32_t C, int32_t *__restrict__ active,
                            int32_t *__restrict__ s, int32_t *__restrict__ ecc_s,
                            unsigned long long *__restrict__ cand_s) {
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C || !active[c]) return;
  if (ecc[c] > ecc_s[c]) {
    s[c] = u[c];
    ecc_s[c] = ecc[c];
    cand_s[c] = cand[c];
  } else {
    active[c] = 0;
  }
}

// ------------------------------------------------------------ Cuthill-McKee levels
__global__ void k_cm_seed(const int32_t *__restrict__ s, const int32_t *__restrict__ cbase, int32_t C,
                          int32_t *__restrict__ pos, int32_t *__restrict__ order, int32_t *__restrict__ front) {
  int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) {
    int32_t v = s[c];
    pos[v] = cbase[c];
    order[cbase[c]] = v;
    front[c] = v;
  }
}
__global__ void k_cm_claim(const int32_t *__restrict__ front, int32_t f, const int32_t *__restrict__ aptr,
                           const int32_t *__restrict__ adj, const int32_t *__restrict__ pos, int32_t *parent) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f) return;
  int32_t v = front[t];
  int32_t pv = pos[v];
  for (int32_t e = aptr[v]; e < aptr[v + 1]; e++) {
    int32_t u = adj[e];
    if (pos[u] == -1) atomicMin(&parent[u], pv);
  }
}
__global__ void k_cm_count(const int32_t *__restrict__ front, int32_t f, const int32_t *__restrict__ aptr,
                           const int32_t *__restrict__ adj, const int32_t *__restrict__ pos,
                           const int32_t *__restrict__ parent, const int32_t *__restrict__ comp,
                           int32_t *__restrict__ cnt, int32_t *__restrict__ first_idx, int32_t *__restrict__ bend) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f) return;
  int32_t v = front[t];
  int32_t pv = pos[v];
  int32_t k = 0;
  for (int32_t e = aptr[v]; e < aptr[v + 1]; e++) {
    int32_t u = adj[e];
    k += (pos[u] == -1 && parent[u] == pv);
  }
  cnt[t] = k;
  int32_t c = comp[v];
  if (t == 0 || comp[front[t - 1]] != c) first_idx[c] = t;
  if (t == f - 1 || comp[front[t + 1]] != c) bend[c] = pv + 1;
}
__global__ void k_cm_emit(const int32_t *__restrict__ front, int32_t f, const int32_t *__restrict__ aptr,
                          const int32_t *__restrict__ adj, int32_t *pos, const int32_t *__restrict__ parent,
                          const int32_t *__restrict__ comp, const int32_t *__restrict__ coff,
                          const int32_t *__restrict__ first_idx, const int32_t *__restrict__ bend, int32_t n,
                          int32_t *__restrict__ order, int32_t *__restrict__ next, int32_t *__restrict__ err) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f) return;
  int32_t v = front[t];
  int32_t pv = pos[v];
  int32_t c = comp[v];
  int32_t p0 = bend[c] + coff[t] - coff[first_idx[c]];
  int32_t k = 0;
  for (int32_t e = aptr[v]; e < aptr[v + 1]; e++) {
    int32_t u = adj[e];
    if (parent[u] == pv && ld_relaxed(pos + u) == -1) {
      const int32_t at = p0 + k, nf = coff[t] + k;
      if (at < 0 || at >= n || nf >= n) {  // cannot happen for a consistent level; never write out of range
        atomicExch(err, 1);
        break;
      }
      pos[u] = at;
      order[at] = u;
      next[nf] = u;
      k++;
    }
  }
}
__global__ void k_reverse(const int32_t *__restrict__ order, const int32_t *__restrict__ pos, int32_t n,
                          int32_t *__restrict__ perm, int32_t *__restrict__ iperm) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    perm[k] = order[n - 1 - k];
    iperm[k] = n - 1 - pos[k];
  }
}
__global__ void k_count_negative(const int32_t *__restrict__ pos, int32_t n, int32_t *__restrict__ cnt) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && pos[v] < 0) atomicAdd(cnt, 1);
}

// ------------------------------------------------------------ host driver
template <class T>
static pars3_status d2h(T *host, const T *dev, size_t m, hipStream_t s) {
  P3_HIP(hipMemcpyAsync(host, dev, m * sizeof(T), hipMemcpyDeviceToHost, s));
  P3_HIP(hipStreamSynchronize(s));
  return PARS3_OK;
}

struct bfs_ws {
  dbuf<int32_t> dist, fa, fb, cnt;
};

// Multi-source BFS from src[c] for the active components; returns, per
// component, the eccentricity ecc[c] and the (degree, index)-minimum cand[c]
// of its last level.
static pars3_status level_bfs(int32_t n, int32_t C, const int32_t *aptr, const int32_t *adj, const int32_t *deg,
                              const int32_t *comp, const int32_t *src, const int32_t *active, int32_t *ecc,
                              unsigned long long *cand, bfs_ws &w, hipStream_t s) {
  P3_TRY(fill_i32(w.dist.p, -1, n, s));
  P3_HIP(hipMemsetAsync(w.cnt.p, 0, 2 * sizeof(int32_t), s));
  k_bfs_seed<<<nblk(C), TB, 0, s>>>(src, active, C, w.dist.p, w.fa.p, w.cnt.p);
  P3_LAUNCHED();
  int32_t f = 0;
  P3_TRY(d2h(&f, w.cnt.p, 1, s));
  int32_t *cur = w.fa.p, *nxt = w.fb.p;
  for (int32_t level = 0; f > 0; level++) {
    if (level > n) return fail(PARS3_EHIP, "bfs: level count exceeds n");
    P3_HIP(hipMemsetAsync(w.cnt.p + 1, 0, sizeof(int32_t), s));
    k_bfs_expand<<<nblk(f), TB, 0, s>>>(cur, f, aptr, adj, w.dist.p, level, nxt, w.cnt.p + 1);
    P3_LAUNCHED();
    P3_TRY(d2h(&f, w.cnt.p + 1, 1, s));
    std::swap(cur, nxt);
  }
  P3_TRY(fill_i32(ecc, -1, C, s));
  P3_TRY(fill_u64((uint64_t *)cand, ~0ull, C, s));
  k_bfs_ecc<<<nblk(n), TB, 0, s>>>(w.dist.p, comp, n, ecc);
  P3_LAUNCHED();
  k_bfs_cand<<<nblk(n), TB, 0, s>>>(w.dist.p, comp, deg, n, ecc, cand);
  P3_LAUNCHED();
  return PARS3_OK;
}

pars3_status identity_perm_gpu(pars3_matrix *A, hipStream_t s) {
  int32_t n = (int32_t)A->n;
  P3_HIP(A->perm.alloc(n));
  P3_HIP(A->iperm.alloc(n));
  P3_TRY(iota_i32(A->perm.p, n, s));
  P3_TRY(iota_i32(A->iperm.p, n, s));
  A->ncomp = 0;
  A->nlevels = 0;
  return PARS3_OK;
}

pars3_status rcm_gpu(pars3_matrix *A, hipStream_t s) {
  const int32_t n = (int32_t)A->n;
  const int64_t nnz = A->nnz;
  P3_HIP(A->perm.alloc(n));
  P3_HIP(A->iperm.alloc(n));
  if (n == 0) return PARS3_OK;
  const int64_t m = 2 * nnz;
  // ---- symmetrise: deg, aptr, adjacency sorted by (deg, index)
  dbuf<int32_t> ucnt, deg, aptr, adj0, adj, ufill;
  P3_HIP(ucnt.alloc(n));
  P3_HIP(deg.alloc(n));
  P3_HIP(aptr.alloc(n + 1));
  P3_HIP(adj0.alloc(m));
  P3_HIP(adj.alloc(m));
  P3_HIP(ufill.alloc(n));
  P3_HIP(hipMemsetAsync(ucnt.p, 0, n * sizeof(int32_t), s));
  P3_HIP(hipMemsetAsync(ufill.p, 0, n * sizeof(int32_t), s));
  k_count_upper<<<nblk(nnz), TB, 0, s>>>(A->col.p, nnz, ucnt.p);
  P3_LAUNCHED();
  k_degree<<<nblk(n), TB, 0, s>>>(A->rowptr.p, ucnt.p, n, deg.p);
  P3_LAUNCHED();
  P3_TRY(scan_i32(deg.p, aptr.p, n, s));
  k_fill_adj<<<nblk(n), TB, 0, s>>>(A->rowptr.p, A->col.p, n, aptr.p, ufill.p, adj0.p);
  P3_LAUNCHED();
  k_sort_adj<<<nblk(m), TB, 0, s>>>(aptr.p, adj0.p, n, m, deg.p, adj.p);
  P3_LAUNCHED();
  adj0.release();
  ufill.release();
  ucnt.release();

  // ---- components
  dbuf<int32_t> parent, label, err;
  P3_HIP(parent.alloc(n));
  P3_HIP(label.alloc(n));
  P3_HIP(err.alloc(1));
  P3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
  P3_TRY(iota_i32(parent.p, n, s));
  k_cc_hook<<<nblk(n), TB, 0, s>>>(A->rowptr.p, A->col.p, n, parent.p, err.p);
  P3_LAUNCHED();
  k_cc_label<<<nblk(n), TB, 0, s>>>(parent.p, n, label.p);
  P3_LAUNCHED();
  int32_t herr = 0;
  P3_TRY(d2h(&herr, err.p, 1, s));
  if (herr) return fail(PARS3_EHIP, "rcm: union-find did not converge");
  parent.release();
  dbuf<unsigned long long> ckey;
  P3_HIP(ckey.alloc(n));
  P3_TRY(fill_u64((uint64_t *)ckey.p, ~0ull, n, s));
  k_comp_key<<<nblk(n), TB, 0, s>>>(label.p, deg.p, n, ckey.p);
  P3_LAUNCHED();
  dbuf<int32_t> flag, rpos;
  P3_HIP(flag.alloc(n));
  P3_HIP(rpos.alloc(n + 1));
  k_is_root<<<nblk(n), TB, 0, s>>>(label.p, n, flag.p);
  P3_LAUNCHED();
  P3_TRY(scan_i32(flag.p, rpos.p, n, s));
  int32_t C = 0;
  P3_TRY(d2h(&C, rpos.p + n, 1, s));
  dbuf<uint64_t> rk0, rk1;
  dbuf<uint32_t> rv0, rv1;
  P3_HIP(rk0.alloc(C));
  P3_HIP(rk1.alloc(C));
  P3_HIP(rv0.alloc(C));
  P3_HIP(rv1.alloc(C));
  k_root_keys<<<nblk(n), TB, 0, s>>>(label.p, rpos.p, n, ckey.p, rk0.p, rv0.p);
  P3_LAUNCHED();
  // keys are deg << 32 | index, all 64 bits sorted
  P3_TRY(radix_sort_pairs(rk0.p, rv0.p, rk1.p, rv1.p, C, 64, s));
  dbuf<int32_t> crank, comp, csize, cbase;
  P3_HIP(crank.alloc(n));
  P3_HIP(comp.alloc(n));
  P3_HIP(csize.alloc(C));
  P3_HIP(cbase.alloc(C + 1));
  P3_HIP(hipMemsetAsync(csize.p, 0, C * sizeof(int32_t), s));
  k_root_rank<<<nblk(C), TB, 0, s>>>(rv0.p, C, crank.p);
  P3_LAUNCHED();
  k_comp_of<<<nblk(n), TB, 0, s>>>(label.p, crank.p, n, comp.p, csize.p);
  P3_LAUNCHED();
  P3_TRY(scan_i32(csize.p, cbase.p, C, s));
  label.release();
  crank.release();
  flag.release();
  rpos.release();
  ckey.release();

  // ---- George-Liu pseudo-peripheral search, all components together:
  // s = the (deg, index)-minimum node; levels from s; repeat: u = the
  // (deg, index)-minimum of the last level; if ecc(u) > ecc(s) move to u,
  // otherwise stop.
  dbuf<int32_t> gs, gu, gactive, gecc_s, ecc, nact;
  dbuf<unsigned long long> gcand_s, cand;
  P3_HIP(gs.alloc(C));
  P3_HIP(gu.alloc(C));
  P3_HIP(gactive.alloc(C));
  P3_HIP(gecc_s.alloc(C));
  P3_HIP(ecc.alloc(C));
  P3_HIP(nact.alloc(1));
  P3_HIP(gcand_s.alloc(C));
  P3_HIP(cand.alloc(C));
  bfs_ws w;
  P3_HIP(w.dist.alloc(n));
  P3_HIP(w.fa.alloc(n));
  P3_HIP(w.fb.alloc(n));
  P3_HIP(w.cnt.alloc(2));
  k_gl_init<<<nblk(C), TB, 0, s>>>((const unsigned long long *)rk0.p, C, gs.p, gactive.p);
  P3_LAUNCHED();
  P3_TRY(level_bfs(n, C, aptr.p, adj.p, deg.p, comp.p, gs.p, gactive.p, ecc.p, cand.p, w, s));
  k_gl_first<<<nblk(C), TB, 0, s>>>(ecc.p, cand.p, C, gecc_s.p, gcand_s.p);
  P3_LAUNCHED();
  for (int round = 0; round < n + 1; round++) {
    P3_HIP(hipMemsetAsync(nact.p, 0, sizeof(int32_t), s));
    k_gl_pick<<<nblk(C), TB, 0, s>>>(gs.p, gcand_s.p, C, gactive.p, gu.p, nact.p);
    P3_LAUNCHED();
    int32_t na = 0;
    P3_TRY(d2h(&na, nact.p, 1, s));
    if (na == 0) break;
    P3_TRY(level_bfs(n, C, aptr.p, adj.p, deg.p, comp.p, gu.p, gactive.p, ecc.p, cand.p, w, s));
    k_gl_update<<<nblk(C), TB, 0, s>>>(gu.p, ecc.p, cand.p, C, gactive.p, gs.p, gecc_s.p, gcand_s.p);
    P3_LAUNCHED();
  }
  w.dist.release();

  // ---- Cuthill-McKee levels with positions
  dbuf<int32_t> pos, par, order, cnt, coff, first_idx, bend;
  P3_HIP(pos.alloc(n));
  P3_HIP(par.alloc(n));
  P3_HIP(order.alloc(n));
  P3_HIP(cnt.alloc(n));
  P3_HIP(coff.alloc(n + 1));
  P3_HIP(first_idx.alloc(C));
  P3_HIP(bend.alloc(C));
  P3_TRY(fill_i32(pos.p, -1, n, s));
  P3_TRY(fill_i32(par.p, 0x7fffffff, n, s));
  P3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
  k_cm_seed<<<nblk(C), TB, 0, s>>>(gs.p, cbase.p, C, pos.p, order.p, w.fa.p);
  P3_LAUNCHED();
  int32_t f = C, levels = 0;
  int32_t *cur = w.fa.p, *nxt = w.fb.p;
  while (f > 0) {
    if (levels > n) return fail(PARS3_EHIP, "rcm: level count exceeds n");
    levels++;
    k_cm_claim<<<nblk(f), TB, 0, s>>>(cur, f, aptr.p, adj.p, pos.p, par.p);
    P3_LAUNCHED();
    k_cm_count<<<nblk(f), TB, 0, s>>>(cur, f, aptr.p, adj.p, pos.p, par.p, comp.p, cnt.p, first_idx.p, bend.p);
    P3_LAUNCHED();
    P3_TRY(scan_i32(cnt.p, coff.p, f, s));
    k_cm_emit<<<nblk(f), TB, 0, s>>>(cur, f, aptr.p, adj.p, pos.p, par.p, comp.p, coff.p, first_idx.p, bend.p, n,
                                     order.p, nxt, err.p);
    P3_LAUNCHED();
    int32_t fn = 0;
    P3_TRY(d2h(&fn, coff.p + f, 1, s));
    f = fn;
    std::swap(cur, nxt);
  }
  P3_TRY(d2h(&herr, err.p, 1, s));
  if (herr) return fail(PARS3_EHIP, "rcm: inconsistent level positions");
  // every node must have been placed
  P3_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t), s));
  k_count_negative<<<nblk(n), TB, 0, s>>>(pos.p, n, cnt.p);
  P3_LAUNCHED();
  int32_t missing = 0;
  P3_TRY(d2h(&missing, cnt.p, 1, s));
  if (missing) return fail(PARS3_EHIP, "rcm: %d nodes were not reached", missing);
  k_reverse<<<nblk(n), TB, 0, s>>>(order.p, pos.p, n, A->perm.p, A->iperm.p);
  P3_LAUNCHED();
  P3_HIP(hipStreamSynchronize(s));
  A->ncomp = C;
  A->nlevels = levels;
  return PARS3_OK;
}

// ------------------------------------------------------------ permutation
// Entry (i, j, l), i > j, lands at (p, q) = (iperm[i], iperm[j]); it is stored
// at (max, min) with value l if p > q and -l otherwise (S_ji = -S_ij, eq. (2));
// a symmetric S keeps l either way.
__global__ void k_perm_keys(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t n,
                            int64_t nnz, const int32_t *__restrict__ iperm, int bits, int sym,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int32_t i = row_of(rowptr, n, e);  // the last row whose pointer is <= e owns e
  int32_t p = iperm[i], q = iperm[col[e]];
  uint64_t hi = (uint64_t)(p > q ? p : q), lo = (uint64_t)(p > q ? q : p);
  keys[e] = (hi << bits) | lo;
  vals[e] = (uint32_t)e | (p > q || sym ? 0u : 0x80000000u);
}
__global__ void k_perm_fill(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t nnz, int bits,
                            const double *__restrict__ val, int32_t *__restrict__ pcol, double *__restrict__ pval,
                            int32_t *__restrict__ rcnt) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = t < nnz;
  int32_t row = 0;
  if (ok) {
    uint64_t k = keys[t];
    uint32_t pv = vals[t];
    row = (int32_t)(k >> bits);
    pcol[t] = (int32_t)(k & ((1ull << bits) - 1));
    double v = val[pv & 0x7fffffffu];
    pval[t] = (pv & 0x80000000u) ? -v : v;
  }
  agg_atomic_add<int32_t>(rcnt, row, 1, ok);
}

pars3_status permute_gpu(pars3_matrix *A, hipStream_t s) {
  const int32_t n = (int32_t)A->n;
  const int64_t nnz = A->nnz;
  P3_HIP(A->prow.alloc(n + 1));
  P3_HIP(A->pcol.alloc(nnz));
  P3_HIP(A->pval.alloc(nnz));
  if (nnz == 0) {
    P3_HIP(hipMemsetAsync(A->prow.p, 0, (n + 1) * sizeof(int32_t), s));
    P3_HIP(hipStreamSynchronize(s));
    return PARS3_OK;
  }
  int bits = std::max(1, bits_for((uint64_t)(n - 1)));
  dbuf<uint64_t> k0, k1;
  dbuf<uint32_t> v0, v1;
  dbuf<int32_t> rcnt;
  P3_HIP(k0.alloc(nnz));
  P3_HIP(k1.alloc(nnz));
  P3_HIP(v0.alloc(nnz));
  P3_HIP(v1.alloc(nnz));
  P3_HIP(rcnt.alloc(n));
  P3_HIP(hipMemsetAsync(rcnt.p, 0, n * sizeof(int32_t), s));
  k_perm_keys<<<nblk(nnz), TB, 0, s>>>(A->rowptr.p, A->col.p, n, nnz, A->iperm.p, bits,
                                       A->kind == PARS3_SYMMETRIC ? 1 : 0, k0.p, v0.p);
  P3_LAUNCHED();
  P3_TRY(radix_sort_pairs(k0.p, v0.p, k1.p, v1.p, nnz, 2 * bits, s));
  k_perm_fill<<<nblk(nnz), TB, 0, s>>>(k0.p, v0.p, nnz, bits, A->val.p, A->pcol.p, A->pval.p, rcnt.p);
  P3_LAUNCHED();
  P3_TRY(scan_i32(rcnt.p, A->prow.p, n, s));
  P3_HIP(hipStreamSynchronize(s));
  return PARS3_OK;
}

__global__ void k_perm_diag(const double *__restrict__ d, const int32_t *__restrict__ perm, int32_t n,
                            double *__restrict__ pd, float *__restrict__ pd32) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double v = d[perm[k]];
  pd[k] = v;
  pd32[k] = (float)v;
}

pars3_status permute_diagonal(pars3_matrix *A, hipStream_t s) {
  const int32_t n = (int32_t)A->n;
  P3_HIP(A->pdiag.alloc(n));
  P3_HIP(A->pdiag32.alloc(n));
  if (n > 0) {
    k_perm_diag<<<nblk(n), TB, 0, s>>>(A->diag.p, A->perm.p, n, A->pdiag.p, A->pdiag32.p);
    P3_LAUNCHED();
  }
  P3_HIP(hipStreamSynchronize(s));
  return PARS3_OK;
}

}  // namespace p3
