// rp_kernels.hip -- HIP kernels (gfx950) for reachability probabilities.
//
// Graph precomputation (Section 2.2 of Cormie-Bowins 2012), assembly of the
// reduced system (Section 2.3), the Jacobi sweep (Section 3.1 / 5.1), the
// BiCGStab building blocks (Section 3.2 / 5.2), FP64 iterative refinement and
// the adjoint gradient.
//
// Layout: the reduced rows of every instance are padded to a multiple of PAD
// rows and split into chunks; one 256-thread block works on one chunk, so a
// block's partial reduction (a max or a dot product) belongs to one instance.
// Per-instance finishing kernels reduce the chunk partials of an instance in
// a fixed order, which makes every scalar deterministic for a given layout.
// Sparse products use L lanes per row (L in 1..64), the lanes of a row read
// consecutive entries, so the col/val streams of a wavefront are coalesced.
#include <hipcub/hipcub.hpp>
#include "rp_internal.h"

#include <climits>

#include <math.h>

namespace rpk {

namespace {

__device__ __forceinline__ double mx(double a, double b) {
  // max that propagates NaN from either operand
  return (a > b || a != a) ? a : b;
}

__device__ __forceinline__ bool finite(double a) { return a == a && fabs(a) <= 1.7976931348623157e308; }

// Reduce NV doubles over the block (bit i of maxmask: max, else sum).  The
// result is valid in thread 0 only.  Fixed tree: deterministic.
template <int NV, int NT = BS>
__device__ __forceinline__ void block_reduce(double (&v)[NV], unsigned maxmask) {
  __shared__ double sh[NT / 64][NV];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; i++) {
    const bool ismax = (maxmask >> i) & 1u;
    double a = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      double b = __shfl_xor(a, o, 64);
      a = ismax ? mx(a, b) : a + b;
    }
    v[i] = a;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; i++) sh[w][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      const bool ismax = (maxmask >> i) & 1u;
      double a = sh[0][i];
      for (int j = 1; j < NT / 64; j++) a = ismax ? mx(a, sh[j][i]) : a + sh[j][i];
      v[i] = a;
    }
  }
}

// Reduce the chunk partials of instance k (NV values per chunk).
template <int NV>
__device__ __forceinline__ void reduce_instance(const Chunks& ch, int k, const double* partial,
                                                unsigned maxmask, double (&v)[NV]) {
#pragma unroll
  for (int i = 0; i < NV; i++) v[i] = 0.0;
  for (int c = ch.inst_c0[k] + threadIdx.x; c < ch.inst_c0[k + 1]; c += BS) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      const double p = partial[(size_t)c * NV + i];
      v[i] = ((maxmask >> i) & 1u) ? mx(v[i], p) : v[i] + p;
    }
  }
  block_reduce<NV>(v, maxmask);
}

__device__ __forceinline__ int find_inst(const int64_t* off, int K, int64_t v) {
  int lo = 0, hi = K - 1;  // largest k with off[k] <= v
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

template <typename T, int L>
__device__ __forceinline__ T row_sum(const MatView<T>& m, const T* __restrict__ x, int row, bool ok,
                                     int lane) {
  T acc = 0;
  if (ok) {
    const int k1 = m.rp[row + 1];
    for (int k = m.rp[row] + lane; k < k1; k += L) acc += m.val[k] * x[m.col[k]];
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
  return acc;
}

}  // namespace

// ============================================================================
// Precomputation
// ============================================================================

// Input check of the Markov chain (Section 2: entries in [0,1], rows sum to 1).
// One thread per row; the key (row << 8 | reason) of the first bad row wins.
// The precompute kernels give each row a group of PG lanes that walk its
// entries PG at a time (coalesced), with ballots for positions and ordered
// in-group shuffles wherever a sum must follow the entry order exactly.
constexpr int PG = 8;

// Ordered sum over the group's PG lanes of q (lane 0's term first), added to acc.
__device__ __forceinline__ double group_ordered_sum(double acc, double q) {
#pragma unroll
  for (int j = 0; j < PG; j++) acc += __shfl(q, j, PG);
  return acc;
}

// This group's PG bits of a wave ballot.
__device__ __forceinline__ unsigned group_bits(bool pred) {
  const unsigned long long m = __ballot(pred);
  return (unsigned)(m >> ((threadIdx.x & 63) & ~(PG - 1))) & ((1u << PG) - 1u);
}

__global__ __launch_bounds__(BS) void k_validate(int64_t n, int64_t nnz, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const int64_t* __restrict__ off, int32_t K, double tol,
                                                 int matrix, unsigned long long* bad) {
  const int64_t i = ((int64_t)blockIdx.x * BS + threadIdx.x) / PG;
  const int l = threadIdx.x % PG;
  if (i >= n) return;
  const int64_t k0 = rp[i], k1 = rp[i + 1];
  unsigned reason = 0;
  if (k1 < k0 || k0 < 0 || k1 > nnz) {
    reason = 1;
  } else {
    const int inst = find_inst(off, K, i);
    const int64_t lo = off[inst], hi = off[inst + 1];
    double sum = 0.0;
    bool diag = false;
    for (int64_t kb = k0; kb < k1; kb += PG) {
      const int64_t k = kb + l;
      unsigned r = 0;
      double q = 0.0;
      if (k < k1) {
        const int64_t c = col[k];
        const double v = val[k];
        if (c < 0 || c >= n) r = 2;
        else if (c < lo || c >= hi) r = 6;
        else if (k > k0 && c <= col[k - 1]) r = 3;
        else if (matrix ? !finite(v) : !(v >= 0.0 && v <= 1.0)) r = matrix ? 7 : 4;
        else q = v;
        if (r == 0 && c == i && v != 0.0) diag = true;
      }
      const unsigned fails = group_bits(r != 0);
      if (fails) {
        // the first failing entry of the row decides the reason
        reason = __shfl(r, __ffs(fails) - 1, PG);
        break;
      }
      sum = group_ordered_sum(sum, q);
    }
    if (!reason && matrix) {
      if (!group_bits(diag)) reason = 8;
    } else if (!reason) {
      const int64_t deg = k1 - k0;
      const double allow = tol * (deg > 1 ? (double)deg : 1.0);
      if (!(fabs(sum - 1.0) <= allow)) reason = 5;
    }
  }
  if (reason && l == 0) atomicMin(bad, ((unsigned long long)i << 8) | reason);
}

hipError_t launch_validate(hipStream_t st, int64_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                           const double* val, const int64_t* inst_off, int32_t K, double tol, int matrix,
                           unsigned long long* bad_key) {
  if (n > 0) k_validate<<<grid_for(n * PG), BS, 0, st>>>(n, nnz, rp, col, val, inst_off, K, tol, matrix, bad_key);
  return hipGetLastError();
}

// I - A of a general matrix A (diagonal stored): the solvers' system
// (I - P') x = b with P' = I - A has diagonal 1 - P'_ii = a_ii and
// off-diagonal part P'_ij = -a_ij, Jacobi's splitting of A (Section 3.1).
__global__ __launch_bounds__(BS) void k_identity_minus(int64_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col, const double* __restrict__ val,
                                                       double* __restrict__ out) {
  const int64_t i = ((int64_t)blockIdx.x * BS + threadIdx.x) / PG;
  const int l = threadIdx.x % PG;
  if (i >= n) return;
  for (int64_t k = rp[i] + l; k < rp[i + 1]; k += PG) out[k] = col[k] == i ? 1.0 - val[k] : -val[k];
}
hipError_t launch_identity_minus(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                                 double* out) {
  if (n > 0) k_identity_minus<<<grid_for(n * PG), BS, 0, st>>>(n, rp, col, val, out);
  return hipGetLastError();
}

// 1 / (|d_i| - sum_j |A_off(i,j)|) per reduced row (0 on padding rows, +inf
// where the row is not strictly dominant): its per-instance maximum is
// Varah's bound on ||A^{-1}||_inf.
__global__ __launch_bounds__(BS) void k_inv_gap(int64_t npad, const int32_t* __restrict__ row_state,
                                                const int32_t* __restrict__ arp, const double* __restrict__ aval,
                                                const double* __restrict__ d, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= npad) return;
  if (row_state[i] < 0) {
    out[i] = 0.0;
    return;
  }
  double off = 0.0;
  for (int32_t k = arp[i]; k < arp[i + 1]; k++) off += fabs(aval[k]);
  const double g = fabs(d[i]) - off;
  out[i] = g > 0.0 ? 1.0 / g : HUGE_VAL;
}
hipError_t launch_inv_gap(hipStream_t st, int64_t npad, const int32_t* row_state, const int32_t* arp,
                          const double* aval, const double* d, double* out) {
  if (npad > 0) k_inv_gap<<<grid_for(npad), BS, 0, st>>>(npad, row_state, arp, aval, d, out);
  return hipGetLastError();
}

__global__ void k_seed_goal(int64_t n, const uint8_t* __restrict__ goal, uint32_t* __restrict__ mark) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) mark[i] = goal[i] ? 1u : 0u;
}
__global__ void k_seed_complement(int64_t n, const uint32_t* __restrict__ src, uint32_t* __restrict__ mark) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) mark[i] = src[i] ? 0u : 1u;
}
hipError_t launch_seed_goal(hipStream_t st, int64_t n, const uint8_t* goal, uint32_t* mark) {
  if (n > 0) k_seed_goal<<<grid_for(n), BS, 0, st>>>(n, goal, mark);
  return hipGetLastError();
}
hipError_t launch_seed_complement(hipStream_t st, int64_t n, const uint32_t* src, uint32_t* mark) {
  if (n > 0) k_seed_complement<<<grid_for(n), BS, 0, st>>>(n, src, mark);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) p[i] = v;
}

// One pull step of the backward search of Section 2.2: an unmarked state
// whose row has an edge (P > 0) into a marked state becomes marked.  Marks set
// during the launch may already be seen by other threads of the same launch
// (monotone, so harmless); the host repeats launches until nothing changes.
// Steps are numbered from 1 and *changed holds the number of the last step
// that marked a state: a step whose predecessor marked nothing starts at the
// fixed point and returns at once; with the states taken grid-stride by at
// most kReachBlocks blocks, a step queued after convergence costs a few
// microseconds instead of a pass (or a launch of n * PG threads).
constexpr unsigned kReachBlocks = 4096;
__device__ __forceinline__ bool reach_settled(const int32_t* changed, int32_t step) {
  return step > 1 && *changed < step - 1;
}
__global__ __launch_bounds__(BS) void k_reach_step(int64_t n, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const double* __restrict__ val,
                                                   const uint8_t* __restrict__ blocked, uint32_t* mark,
                                                   int32_t* changed, int32_t step) {
  if (reach_settled(changed, step)) return;
  const int l = threadIdx.x % PG;
  const int64_t stride = (int64_t)gridDim.x * (BS / PG);
  for (int64_t v = ((int64_t)blockIdx.x * BS + threadIdx.x) / PG; v < n; v += stride) {
    if (mark[v] || (blocked && blocked[v])) continue;
    const int32_t k1 = rp[v + 1];
    for (int32_t kb = rp[v]; kb < k1; kb += PG) {
      const int32_t k = kb + l;
      const bool hit = k < k1 && val[k] > 0.0 && mark[col[k]];
      if (group_bits(hit)) {
        if (l == 0) {
          mark[v] = 1u;
          *changed = step;
        }
        break;
      }
    }
  }
}

// The whole backward search in one workgroup, for chains of at most
// kReachResident states: the marks live in LDS, pull steps repeat until a
// step marks nothing (at most n steps; a long path needs one step per state,
// which would otherwise be one launch each).
constexpr int kReachResident = 32768;
constexpr int kReachThreads = 1024;
__global__ __launch_bounds__(kReachThreads) void k_reach_resident(int32_t n, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const uint8_t* __restrict__ blocked, uint32_t* mark) {
  __shared__ uint8_t mk[kReachResident];
  __shared__ int32_t changed;
  for (int i = threadIdx.x; i < n; i += kReachThreads) mk[i] = mark[i] ? 1 : 0;
  const int l = threadIdx.x % PG;
  constexpr int RPB = kReachThreads / PG;
  while (true) {
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    for (int v = threadIdx.x / PG; v < n; v += RPB) {
      if (mk[v] || (blocked && blocked[v])) continue;
      const int32_t k1 = rp[v + 1];
      for (int32_t kb = rp[v]; kb < k1; kb += PG) {
        const int32_t k = kb + l;
        const bool hit = k < k1 && val[k] > 0.0 && mk[col[k]];
        if (group_bits(hit)) {
          if (l == 0) {
            mk[v] = 1;
            changed = 1;
          }
          break;
        }
      }
    }
    __syncthreads();
    if (!changed) break;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kReachThreads) mark[i] = mk[i];
}
hipError_t launch_reach_resident(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                                 const uint8_t* blocked, uint32_t* mark) {
  if (n <= 0) return hipSuccess;
  if (n > kReachResident) return hipErrorInvalidValue;
  k_reach_resident<<<1, kReachThreads, 0, st>>>((int32_t)n, rp, col, val, blocked, mark);
  return hipGetLastError();
}

hipError_t launch_reach_step(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col,
                             const double* val, const uint8_t* blocked, uint32_t* mark,
                             int32_t* changed, int32_t step) {
  if (n > 0)
    k_reach_step<<<std::min(grid_for(n * PG), kReachBlocks), BS, 0, st>>>(n, rp, col, val, blocked, mark, changed,
                                                                          step);
  return hipGetLastError();
}

// ---- deep searches: contraction of states with the same reachability ------
// A pull step marks one more level, so a long path (a birth-death chain of a
// million states) needs as many launches.  States that provably share their
// search result are merged first (union-find with atomic compare-and-swap
// links, the larger root always hung under the smaller, so no cycle forms):
//   * a mutual edge u -> v, v -> u (P > 0 both ways, neither blocked): each
//     reaches what the other reaches;
//   * a forced step: u (not blocked, not already marked) whose only successor
//     other than itself is v (not blocked): u reaches the target set exactly
//     when v does.
// The pull steps then run on the classes (one mark per class), whose
// longest chain is short for such chains; the final marks are the classes'.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  // path halving: every node on the way is pointed at its grandparent (an
  // ancestor: links only change roots, so a plain store cannot break a tree)
  while (true) {
    const int32_t p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    const int32_t g = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (g != p) __hip_atomic_store(&parent[x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = g;
  }
}
__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&parent[b], b, a) == b) return;
  }
}
__global__ void k_uf_init(int64_t n, int32_t* parent) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v < n) parent[v] = (int32_t)v;
}
// One thread per state u: its mutual edges (to higher states) and its forced
// step.  Columns are strictly ascending within a row, so the reverse edge is
// found by binary search in the successor's row.
__global__ __launch_bounds__(BS) void k_uf_union(int64_t n, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const uint8_t* __restrict__ blocked,
                                                 const uint32_t* __restrict__ mark, int32_t* parent) {
  const int64_t ul = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (ul >= n) return;
  const int32_t u = (int32_t)ul;
  if (blocked && blocked[u]) return;
  const int32_t k0 = rp[u], k1 = rp[u + 1];
  int32_t nsucc = 0, only = -1;
  for (int32_t k = k0; k < k1; k++) {
    if (!(val[k] > 0.0)) continue;
    const int32_t v = col[k];
    if (v == u) continue;
    nsucc++;
    only = v;
    if (v < u || (blocked && blocked[v])) continue;
    int32_t lo = rp[v], hi = rp[v + 1];
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (col[mid] < u) lo = mid + 1;
      else hi = mid;
    }
    if (lo < rp[v + 1] && col[lo] == u && val[lo] > 0.0) uf_union(parent, u, v);
  }
  if (nsucc == 1 && !mark[u] && !(blocked && blocked[only])) uf_union(parent, u, only);
}
// parent[v] <- root of v, and the class marks from the state marks.
__global__ void k_uf_flatten(int64_t n, int32_t* parent, const uint32_t* __restrict__ mark, uint32_t* cmark) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  const int32_t r = uf_find(parent, (int32_t)v);
  parent[v] = r;
  if (mark[v]) cmark[r] = 1u;
}
// Pull step on the classes (as k_reach_step, one mark per class root).
__global__ __launch_bounds__(BS) void k_reach_step_classes(int64_t n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const uint8_t* __restrict__ blocked,
                                                           const int32_t* __restrict__ root, uint32_t* cmark,
                                                           int32_t* changed, int32_t step) {
  if (reach_settled(changed, step)) return;
  const int l = threadIdx.x % PG;
  const int64_t stride = (int64_t)gridDim.x * (BS / PG);
  for (int64_t v = ((int64_t)blockIdx.x * BS + threadIdx.x) / PG; v < n; v += stride) {
    if (blocked && blocked[v]) continue;
    const int32_t r = root[v];
    if (cmark[r]) continue;
    const int32_t k1 = rp[v + 1];
    for (int32_t kb = rp[v]; kb < k1; kb += PG) {
      const int32_t k = kb + l;
      const bool hit = k < k1 && val[k] > 0.0 && cmark[root[col[k]]];
      if (group_bits(hit)) {
        if (l == 0) {
          cmark[r] = 1u;
          *changed = step;
        }
        break;
      }
    }
  }
}
// State marks from the class marks (blocked states keep theirs: never set).
__global__ void k_classes_expand(int64_t n, const uint8_t* __restrict__ blocked, const int32_t* __restrict__ root,
                                 const uint32_t* __restrict__ cmark, uint32_t* mark) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n || (blocked && blocked[v])) return;
  if (cmark[root[v]]) mark[v] = 1u;
}
hipError_t launch_reach_contract(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                                 const uint8_t* blocked, const uint32_t* mark, int32_t* parent, uint32_t* cmark) {
  if (n <= 0) return hipSuccess;
  k_uf_init<<<grid_for(n), BS, 0, st>>>(n, parent);
  k_uf_union<<<grid_for(n), BS, 0, st>>>(n, rp, col, val, blocked, mark, parent);
  k_fill_u32<<<grid_for(n), BS, 0, st>>>(cmark, n, 0u);
  k_uf_flatten<<<grid_for(n), BS, 0, st>>>(n, parent, mark, cmark);
  return hipGetLastError();
}
hipError_t launch_reach_step_classes(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col,
                                     const double* val, const uint8_t* blocked, const int32_t* root, uint32_t* cmark,
                                     int32_t* changed, int32_t step) {
  if (n > 0)
    k_reach_step_classes<<<std::min(grid_for(n * PG), kReachBlocks), BS, 0, st>>>(n, rp, col, val, blocked, root,
                                                                                  cmark, changed, step);
  return hipGetLastError();
}
hipError_t launch_classes_expand(hipStream_t st, int64_t n, const uint8_t* blocked, const int32_t* root,
                                 const uint32_t* cmark, uint32_t* mark) {
  if (n > 0) k_classes_expand<<<grid_for(n), BS, 0, st>>>(n, blocked, root, cmark, mark);
  return hipGetLastError();
}

__global__ void k_classes(int64_t n, const uint32_t* __restrict__ rg, const uint32_t* __restrict__ rs0,
                          const uint8_t* __restrict__ goal, int prob0_only, uint8_t* __restrict__ cls,
                          uint8_t* __restrict__ class_out, int32_t* __restrict__ flags) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  uint8_t c;
  if (!rg[v]) c = 0;
  else if (prob0_only) c = goal[v] ? 1 : 2;
  else c = rs0[v] ? 2 : 1;
  cls[v] = c;
  if (class_out) class_out[v] = c;
  if (flags) flags[v] = (c == 2) ? 1 : 0;
}

hipError_t launch_classes(hipStream_t st, int64_t n, const uint32_t* reach_goal,
                          const uint32_t* reach_s0, const uint8_t* goal, int prob0_only,
                          uint8_t* cls, uint8_t* class_out, int32_t* flags_sq) {
  if (n > 0)
    k_classes<<<grid_for(n), BS, 0, st>>>(n, reach_goal, reach_s0, goal, prob0_only, cls, class_out,
                                          flags_sq);
  return hipGetLastError();
}

// ---- exclusive scan of int32 (out has n+1 entries; out[n] = total) ----------
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = BS * SCAN_ITEMS;

__global__ void k_scan_block(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t n,
                             int32_t* __restrict__ bsum) {
  __shared__ int32_t wsum[BS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t tsum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    tsum += v[j];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t inc = tsum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int32_t woff = 0;
  for (int j = 0; j < w; j++) woff += wsum[j];
  int32_t run = woff + inc - tsum;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == BS - 1) bsum[blockIdx.x] = run;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ boff) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) out[i] += boff[i / SCAN_TILE];
}

__global__ void k_set_total(int32_t* dst, const int32_t* src) { *dst = *src; }

size_t scan_scratch_elems(int64_t n) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  size_t s = (size_t)nb + 1;
  if (nb > 1) s += (size_t)nb + 1 + scan_scratch_elems(nb);
  return s;
}

hipError_t launch_scan(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* scratch) {
  if (n <= 0) return hipMemsetAsync(out, 0, sizeof(int32_t), st);
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  int32_t* bsum = scratch;
  k_scan_block<<<(unsigned)nb, BS, 0, st>>>(in, out, n, bsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nb == 1) {
    k_set_total<<<1, 1, 0, st>>>(out + n, bsum);
    return hipGetLastError();
  }
  int32_t* bscan = scratch + nb + 1;
  e = launch_scan(st, bsum, bscan, nb, bscan + nb + 1);
  if (e != hipSuccess) return e;
  k_scan_add<<<grid_for(n), BS, 0, st>>>(out, n, bscan);
  k_set_total<<<1, 1, 0, st>>>(out + n, bscan + nb);
  return hipGetLastError();
}

__global__ void k_inst_counts(int32_t K, const int64_t* __restrict__ off, const int32_t* __restrict__ rank,
                              int32_t* __restrict__ counts) {
  const int k = blockIdx.x * BS + threadIdx.x;
  if (k < K) counts[k] = rank[off[k + 1]] - rank[off[k]];
}
hipError_t launch_inst_counts(hipStream_t st, int32_t K, const int64_t* inst_off, const int32_t* rank,
                              int32_t* counts) {
  k_inst_counts<<<grid_for(K), BS, 0, st>>>(K, inst_off, rank, counts);
  return hipGetLastError();
}

// Reduced numbering (Section 2.3): states of S_? keep their order; instance k
// starts at the padded offset roff[k].
__global__ void k_map(int64_t n, const uint8_t* __restrict__ cls, const int32_t* __restrict__ rank,
                      const int64_t* __restrict__ off, int32_t K, const int64_t* __restrict__ roff,
                      int32_t* __restrict__ map, int32_t* __restrict__ row_state) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  if (cls[v] == 2) {
    const int k = find_inst(off, K, v);
    const int64_t r = roff[k] + (int64_t)(rank[v] - rank[off[k]]);
    map[v] = (int32_t)r;
    row_state[r] = (int32_t)v;
  } else {
    map[v] = -1;
  }
}
hipError_t launch_map(hipStream_t st, int64_t n, const uint8_t* cls, const int32_t* rank,
                      const int64_t* inst_off, int32_t K, const int64_t* roff, int32_t* map,
                      int32_t* row_state, int32_t*) {
  if (n > 0) k_map<<<grid_for(n), BS, 0, st>>>(n, cls, rank, inst_off, K, roff, map, row_state);
  return hipGetLastError();
}

// Per reduced row: number of off-diagonal entries into S_?, d = 1 - P(s,s)
// and b = P(s, S_{=1}) summed in storage order (Section 2.3).  Padding rows
// get d = 1, b = 0 and no entries.
__global__ __launch_bounds__(BS) void k_row_count(int64_t npad, const int32_t* __restrict__ row_state,
                                                  const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, const uint8_t* __restrict__ cls,
                                                  int32_t* __restrict__ cnt, double* __restrict__ d64,
                                                  float* __restrict__ d32, double* __restrict__ b64, int any_sign) {
  const int64_t r = ((int64_t)blockIdx.x * BS + threadIdx.x) / PG;
  const int l = threadIdx.x % PG;
  if (r >= npad) return;
  const int32_t v = row_state[r];
  if (v < 0) {
    if (l == 0) { cnt[r] = 0; d64[r] = 1.0; d32[r] = 1.0f; b64[r] = 0.0; }
    return;
  }
  double pii = 0.0, bi = 0.0;
  int32_t c = 0;
  const int32_t k1 = rp[v + 1];
  for (int32_t kb = rp[v]; kb < k1; kb += PG) {
    const int32_t k = kb + l;
    bool toq = false;
    double diag = 0.0, q = 0.0;
    if (k < k1) {
      const int32_t t = col[k];
      const double p = val[k];
      if (t == v) {
        diag = p;
      } else if (any_sign ? p != 0.0 : p > 0.0) {
        const uint8_t ct = cls[t];
        toq = ct == 2;
        if (ct == 1) q = p;
      }
    }
    c += __popc(group_bits(toq));
    pii = group_ordered_sum(pii, diag);  // at most one non-zero term
    bi = group_ordered_sum(bi, q);       // in entry order, as a sequential sum
  }
  if (l == 0) {
    const double dd = 1.0 - pii;
    cnt[r] = c; d64[r] = dd; d32[r] = (float)dd; b64[r] = bi;
  }
}
hipError_t launch_row_count(hipStream_t st, int64_t npad, const int32_t* row_state, const int32_t* rp,
                            const int32_t* col, const double* val, const uint8_t* cls, int32_t* cnt,
                            double* d64, float* d32, double* b64, int any_sign) {
  if (npad > 0)
    k_row_count<<<grid_for(npad * PG), BS, 0, st>>>(npad, row_state, rp, col, val, cls, cnt, d64, d32, b64, any_sign);
  return hipGetLastError();
}

__global__ __launch_bounds__(BS) void k_fill_rows(int64_t npad, const int32_t* __restrict__ row_state,
                                                  const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, const uint8_t* __restrict__ cls,
                                                  const int32_t* __restrict__ map, const int32_t* __restrict__ arp,
                                                  int32_t* __restrict__ acol, double* __restrict__ av64,
                                                  float* __restrict__ av32, int any_sign) {
  const int64_t r = ((int64_t)blockIdx.x * BS + threadIdx.x) / PG;
  const int l = threadIdx.x % PG;
  if (r >= npad) return;
  const int32_t v = row_state[r];
  if (v < 0) return;
  int32_t pos = arp[r];
  const int32_t k1 = rp[v + 1];
  for (int32_t kb = rp[v]; kb < k1; kb += PG) {
    const int32_t k = kb + l;
    bool inc = false;
    int32_t t = 0;
    double p = 0.0;
    if (k < k1) {
      t = col[k];
      p = val[k];
      inc = t != v && (any_sign ? p != 0.0 : p > 0.0) && cls[t] == 2;
    }
    const unsigned gm = group_bits(inc);
    if (inc) {
      const int32_t q = pos + __popc(gm & ((1u << l) - 1u));
      acol[q] = map[t];
      av64[q] = p;
      av32[q] = (float)p;
    }
    pos += __popc(gm);
  }
}
hipError_t launch_fill_rows(hipStream_t st, int64_t npad, const int32_t* row_state, const int32_t* rp,
                            const int32_t* col, const double* val, const uint8_t* cls, const int32_t* map,
                            const int32_t* arp, int32_t* acol, double* av64, float* av32, int any_sign) {
  if (npad > 0)
    k_fill_rows<<<grid_for(npad * PG), BS, 0, st>>>(npad, row_state, rp, col, val, cls, map, arp, acol, av64, av32,
                                                    any_sign);
  return hipGetLastError();
}

// ---- transpose of A_off (for the adjoint system) -----------------------------
// The transposed matrix is the forward entries ordered by column: a stable
// radix sort of the entry indices by column (hipCUB) leaves the entries of
// each column in source-row order, so the transposed matrix, and every sum
// over it, is deterministic.  The rows and values are then gathered by entry
// index and the row pointers read off the sorted columns.  (It replaced a
// counting sort whose atomics were served in any order and whose transposed
// rows then had to be ranked: 3.70 -> 1.60 ms on 34.3 M entries.)
__global__ void k_iota(int64_t n, int32_t* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int32_t)i;
}
__global__ void k_tgather(int64_t z, const int32_t* __restrict__ perm, const int32_t* __restrict__ erow,
                          const double* __restrict__ av64, int32_t* __restrict__ tcol, double* __restrict__ tv64,
                          float* __restrict__ tv32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= z) return;
  const int32_t k = perm[i];
  const double v = av64[k];
  tcol[i] = erow[k];
  tv64[i] = v;
  tv32[i] = (float)v;
}
// trp[c] = first sorted position whose column is >= c (c = 0..npad), trp
// filled with -1 beforehand: thread i writes the columns between the sorted
// keys i-1 and i, at most kBoundRun of them; the columns of a longer run of
// empty columns (a hub whose column holds most entries, say) are left at -1
// and found by one binary search each (k_tbounds_rest), so no thread walks a
// long run alone.
constexpr int64_t kBoundRun = 64;
__global__ void k_tbounds(int64_t z, int64_t npad, const int32_t* __restrict__ key, int32_t* __restrict__ trp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > z) return;
  const int64_t prev = i == 0 ? -1 : (int64_t)key[i - 1];
  const int64_t cur = i == z ? npad : (int64_t)key[i];
  const int64_t last = cur - prev > kBoundRun ? prev + kBoundRun : cur;
  for (int64_t c = prev + 1; c <= last; c++) trp[c] = (int32_t)i;
}
__global__ void k_tbounds_rest(int64_t z, int64_t npad, const int32_t* __restrict__ key, int32_t* __restrict__ trp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > npad || trp[c] >= 0) return;
  int64_t lo = 0, hi = z;  // first position whose key is >= c
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if ((int64_t)key[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  trp[c] = (int32_t)lo;
}
static int column_bits(int64_t npad) {
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < npad) bits++;
  return bits;
}
hipError_t transpose_temp_bytes(int64_t npad, int64_t z, size_t* bytes) {
  size_t tb = 0;
  const hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const int32_t*)nullptr, (int32_t*)nullptr,
                                                          (const int32_t*)nullptr, (int32_t*)nullptr, (int)z, 0,
                                                          column_bits(npad));
  *bytes = std::max<size_t>(tb, 1);
  return e;
}
hipError_t launch_transpose(hipStream_t st, int64_t npad, int64_t z, const int32_t* arp, const int32_t* acol,
                            const double* av64, int32_t* trp, int32_t* tcol, double* tv64, float* tv32,
                            int32_t* erow, int32_t* idx, int32_t* key_out, int32_t* perm, void* temp,
                            size_t temp_bytes) {
  if (npad <= 0) return hipMemsetAsync(trp, 0, sizeof(int32_t), st);
  if (z > 0) {
    hipError_t e = launch_fill_erow(st, npad, arp, erow);
    if (e != hipSuccess) return e;
    k_iota<<<(unsigned)((z + 255) / 256), 256, 0, st>>>(z, idx);
    e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, acol, key_out, idx, perm, (int)z, 0, column_bits(npad),
                                           st);
    if (e != hipSuccess) return e;
    k_tgather<<<(unsigned)((z + 255) / 256), 256, 0, st>>>(z, perm, erow, av64, tcol, tv64, tv32);
  }
  k_fill_u32<<<grid_for(npad + 1), BS, 0, st>>>(reinterpret_cast<uint32_t*>(trp), npad + 1, 0xFFFFFFFFu);
  k_tbounds<<<(unsigned)((z + 1 + 255) / 256), 256, 0, st>>>(z, npad, key_out, trp);
  k_tbounds_rest<<<(unsigned)((npad + 1 + 255) / 256), 256, 0, st>>>(z, npad, key_out, trp);
  return hipGetLastError();
}

// ============================================================================
// Jacobi (Section 3.1): x'_i = (rhs_i + sum_{j != i} A_ij x_j) / d_i, double
// buffered, with the stopping measure reduced per instance in the same pass.
// ============================================================================

template <typename T, int L>
__global__ __launch_bounds__(BS) void k_jacobi(MatView<T> m, const T* __restrict__ rhs,
                                               const T* __restrict__ x, T* __restrict__ xn, Chunks ch,
                                               const int32_t* __restrict__ status,
                                               double* __restrict__ partial, int weighted) {
  const int c = blockIdx.x;
  if (status[ch.inst[c]] != ST_RUN) return;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = BS / L;
  double mloc = 0.0;
  for (int base = 0; base < nr; base += RPP) {
    const bool ok = base + g < nr;
    const int row = r0 + base + g;
    const T acc = row_sum<T, L>(m, x, row, ok, lane);
    if (ok && lane == 0) {
      const T nv = (rhs[row] + acc) / m.d[row];
      const double dl = fabs((double)nv - (double)x[row]);
      xn[row] = nv;
      mloc = mx(mloc, weighted ? (double)m.d[row] * dl : dl);
    }
  }
  double v[1] = {mloc};
  block_reduce<1>(v, 1u);
  if (threadIdx.x == 0) partial[c] = v[0];
}

template <typename T>
hipError_t launch_jacobi(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x, T* xn, Chunks ch,
                         const int32_t* status, double* partial, int weighted) {
  const unsigned g = (unsigned)ch.nchunk;
  switch (L) {
    case 1: k_jacobi<T, 1><<<g, BS, 0, st>>>(m, rhs, x, xn, ch, status, partial, weighted); break;
    case 2: k_jacobi<T, 2><<<g, BS, 0, st>>>(m, rhs, x, xn, ch, status, partial, weighted); break;
    case 4: k_jacobi<T, 4><<<g, BS, 0, st>>>(m, rhs, x, xn, ch, status, partial, weighted); break;
    case 8: k_jacobi<T, 8><<<g, BS, 0, st>>>(m, rhs, x, xn, ch, status, partial, weighted); break;
    case 16: k_jacobi<T, 16><<<g, BS, 0, st>>>(m, rhs, x, xn, ch, status, partial, weighted); break;
    case 32: k_jacobi<T, 32><<<g, BS, 0, st>>>(m, rhs, x, xn, ch, status, partial, weighted); break;
    case 64: k_jacobi<T, 64><<<g, BS, 0, st>>>(m, rhs, x, xn, ch, status, partial, weighted); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_jacobi<double>(hipStream_t, int, MatView<double>, const double*, const double*,
                                          double*, Chunks, const int32_t*, double*, int);
template hipError_t launch_jacobi<float>(hipStream_t, int, MatView<float>, const float*, const float*,
                                         float*, Chunks, const int32_t*, double*, int);

// In-place (asynchronous) Jacobi sweep: the iterate is overwritten row by
// row as the sweep goes, and every row sum reads whatever value each
// neighbour holds at that moment, the old one or one already updated in this
// sweep (the update the paper's Jacobi kernel performs on a single vector,
// Section 5.1; rows later in a block tend to see their block's new values,
// Gauss-Seidel fashion).  For a nonnegative A with spectral radius below one
// these asynchronous iterations converge to the same fixed point.  The
// change of a row is measured against the value it overwrites.  x is not
// __restrict__: it is read and written through the same pointer.
template <typename T, int L>
__global__ __launch_bounds__(BS) void k_jacobi_inplace(MatView<T> m, const T* __restrict__ rhs, T* x, Chunks ch,
                                                       const int32_t* __restrict__ status,
                                                       double* __restrict__ partial, int weighted) {
  const int c = blockIdx.x;
  if (status[ch.inst[c]] != ST_RUN) return;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = BS / L;
  double mloc = 0.0;
  for (int base = 0; base < nr; base += RPP) {
    const bool ok = base + g < nr;
    const int row = r0 + base + g;
    const T old = ok ? x[row] : (T)0;
    T acc = 0;
    if (ok) {
      const int k1 = m.rp[row + 1];
      for (int k = m.rp[row] + lane; k < k1; k += L) acc += m.val[k] * x[m.col[k]];
    }
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
    if (ok && lane == 0) {
      const T nv = (rhs[row] + acc) / m.d[row];
      x[row] = nv;
      const double dl = fabs((double)nv - (double)old);
      mloc = mx(mloc, weighted ? (double)m.d[row] * dl : dl);
    }
  }
  double v[1] = {mloc};
  block_reduce<1>(v, 1u);
  if (threadIdx.x == 0) partial[c] = v[0];
}

template <typename T>
hipError_t launch_jacobi_inplace(hipStream_t st, int L, MatView<T> m, const T* rhs, T* x, Chunks ch,
                                 const int32_t* status, double* partial, int weighted) {
  const unsigned g = (unsigned)ch.nchunk;
  switch (L) {
    case 1: k_jacobi_inplace<T, 1><<<g, BS, 0, st>>>(m, rhs, x, ch, status, partial, weighted); break;
    case 2: k_jacobi_inplace<T, 2><<<g, BS, 0, st>>>(m, rhs, x, ch, status, partial, weighted); break;
    case 4: k_jacobi_inplace<T, 4><<<g, BS, 0, st>>>(m, rhs, x, ch, status, partial, weighted); break;
    case 8: k_jacobi_inplace<T, 8><<<g, BS, 0, st>>>(m, rhs, x, ch, status, partial, weighted); break;
    case 16: k_jacobi_inplace<T, 16><<<g, BS, 0, st>>>(m, rhs, x, ch, status, partial, weighted); break;
    case 32: k_jacobi_inplace<T, 32><<<g, BS, 0, st>>>(m, rhs, x, ch, status, partial, weighted); break;
    case 64: k_jacobi_inplace<T, 64><<<g, BS, 0, st>>>(m, rhs, x, ch, status, partial, weighted); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_jacobi_inplace<double>(hipStream_t, int, MatView<double>, const double*, double*, Chunks,
                                                  const int32_t*, double*, int);
template hipError_t launch_jacobi_inplace<float>(hipStream_t, int, MatView<float>, const float*, float*, Chunks,
                                                 const int32_t*, double*, int);

// Row of every stored entry (erow[k] = i for rp[i] <= k < rp[i+1]), for the
// segmented-scan sweep.
__global__ void k_fill_erow(int64_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ erow) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; k++) erow[k] = (int32_t)i;
}
hipError_t launch_fill_erow(hipStream_t st, int64_t n, const int32_t* rp, int32_t* erow) {
  if (n <= 0) return hipSuccess;
  k_fill_erow<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, rp, erow);
  return hipGetLastError();
}

// Jacobi sweep whose row sums come from a backward segmented scan over the
// stored entries (the entry-parallel sparse product the paper cites for
// Jacobi on GPUs, Section 8): every thread forms one product a_ij x_j, and a
// suffix scan within each row's run of entries leaves the row's sum at its
// first entry, whose thread updates the row.  A block takes its chunk's
// entries BS at a time from the last window to the first; within a window
// each wavefront scans its 64 entries with shuffles, the waves' trailing
// runs are completed from the waves after them, and the run still open at
// the window's first entry carries into the window before it.  Rows without
// entries are updated on their own.  Sums are in scan order (a tree), not
// in column order.
template <typename T>
__global__ __launch_bounds__(BS) void k_jacobi_segscan(MatView<T> m, const int32_t* __restrict__ erow,
                                                       const T* __restrict__ rhs, const T* __restrict__ x,
                                                       T* __restrict__ xn, Chunks ch,
                                                       const int32_t* __restrict__ status,
                                                       double* __restrict__ partial, int weighted) {
  constexpr int NWV = BS / 64;
  __shared__ T wsum[NWV];
  __shared__ int wfirst[NWV], wlast[NWV];
  __shared__ T carry;
  __shared__ int crow;
  const int c = blockIdx.x;
  if (status[ch.inst[c]] != ST_RUN) return;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  const int e0 = m.rp[r0], e1 = m.rp[r0 + nr];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mloc = 0.0;
  auto update = [&](int row, T sum) {
    const T nv = (rhs[row] + sum) / m.d[row];
    const double dl = fabs((double)nv - (double)x[row]);
    xn[row] = nv;
    mloc = mx(mloc, weighted ? (double)m.d[row] * dl : dl);
  };
  for (int i = threadIdx.x; i < nr; i += BS)
    if (m.rp[r0 + i] == m.rp[r0 + i + 1]) update(r0 + i, (T)0);
  if (threadIdx.x == 0) {
    carry = (T)0;
    crow = -1;
  }
  const int npass = (e1 - e0 + BS - 1) / BS;
  for (int ps = npass - 1; ps >= 0; ps--) {
    const int e = e0 + ps * BS + (int)threadIdx.x;
    const bool ok = e < e1;
    const int r = ok ? erow[e] : -1;
    T p = ok ? m.val[e] * x[m.col[e]] : (T)0;
    // suffix sums over the lanes of the same row (a row's entries are
    // consecutive, so equal rows at distance d mean one run)
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const T q = __shfl_down(p, d, 64);
      const int rq = __shfl_down(r, d, 64);
      if (lane + d < 64 && rq == r) p += q;
    }
    __syncthreads();  // the previous window is done with the shared values
    if (lane == 0) {
      wsum[wave] = p;
      wfirst[wave] = r;
    }
    if (lane == 63) wlast[wave] = r;
    __syncthreads();
    // the wave's trailing run continues into the waves after it (and past
    // the window) while they hold nothing but that row
    const int rl = wlast[wave];
    T cin = (T)0;
    bool open = rl >= 0;
    for (int v = wave + 1; v < NWV && open; v++) {
      if (wfirst[v] != rl) {
        open = false;
        break;
      }
      cin += wsum[v];
      open = wlast[v] == rl;
    }
    if (open && crow == rl) cin += carry;
    if (r == rl) p += cin;
    if (ok && e == m.rp[r]) update(r, p);
    __syncthreads();  // every thread has read carry
    if (threadIdx.x == 0) {
      carry = p;
      crow = r;
    }
  }
  double v[1] = {mloc};
  block_reduce<1>(v, 1u);
  if (threadIdx.x == 0) partial[c] = v[0];
}

template <typename T>
hipError_t launch_jacobi_segscan(hipStream_t st, MatView<T> m, const int32_t* erow, const T* rhs, const T* x, T* xn,
                                 Chunks ch, const int32_t* status, double* partial, int weighted) {
  k_jacobi_segscan<T><<<(unsigned)ch.nchunk, BS, 0, st>>>(m, erow, rhs, x, xn, ch, status, partial, weighted);
  return hipGetLastError();
}
template hipError_t launch_jacobi_segscan<double>(hipStream_t, MatView<double>, const int32_t*, const double*,
                                                  const double*, double*, Chunks, const int32_t*, double*, int);
template hipError_t launch_jacobi_segscan<float>(hipStream_t, MatView<float>, const int32_t*, const float*,
                                                 const float*, float*, Chunks, const int32_t*, double*, int);

__global__ void k_fin_jacobi(Chunks ch, const double* __restrict__ partial, int32_t* status, int64_t* iters,
                             double* meas, const double* __restrict__ thr, int strict, int64_t max_iter,
                             int32_t* ndone) {
  const int k = blockIdx.x;
  if (status[k] != ST_RUN) return;
  double v[1];
  reduce_instance<1>(ch, k, partial, 1u, v);
  if (threadIdx.x == 0) {
    const double m = v[0];
    const int64_t it = iters[k] + 1;
    iters[k] = it;
    meas[k] = m;
    int32_t s = ST_RUN;
    if (!finite(m)) s = ST_NONFINITE;
    else if (strict ? (m < thr[k]) : (m <= thr[k])) s = ST_CONVERGED;
    else if (it >= max_iter) s = ST_MAXITER;
    if (s != ST_RUN) {
      status[k] = s;
      atomicAdd(ndone, 1);
    }
  }
}
hipError_t launch_fin_jacobi(hipStream_t st, Chunks ch, const double* partial, int32_t* status, int64_t* iters,
                             double* meas, const double* thr, int strict, int64_t max_iter, int32_t* ndone) {
  k_fin_jacobi<<<(unsigned)ch.K, BS, 0, st>>>(ch, partial, status, iters, meas, thr, strict, max_iter, ndone);
  return hipGetLastError();
}

// ============================================================================
// Jacobi with the instance's x staged in LDS.  Used when every instance's
// padded row block fits in one workgroup's LDS: each tile (a row range of one
// instance) copies x of its whole instance into LDS with coalesced loads, so
// the column gathers of the sweep read LDS instead of pulling a cache line
// from L2 per entry.  The stopping decision for the previous sweep is taken
// at the start of the next one by every block of the instance from the same
// per-tile partials (identical, deterministic result in every block), which
// removes the separate finishing launch per sweep.
// ============================================================================

constexpr int TNT = 1024;  // threads per tile block

// Decision on Jacobi sweep s-1 of an instance, taken by each wavefront on its
// own: the instance's per-tile maxima of that sweep are reduced across the
// lanes (pv holds pprev[t0 + lane] or 0 on entry; a max is exact, so every
// wavefront of every block of the instance reaches the same value) and
// compared with the threshold th.  Thread 0 of the instance's first tile
// records a stop.  Returns the wavefront-uniform status (ST_RUN: go on).
// Without a block-wide reduction the sweep needs no barrier for it, which
// measured ~3 us faster per sweep than a block reduction.
__device__ __forceinline__ int32_t jacobi_decide(const Tiles& tl, int c, int inst, int64_t s,
                                                 const double* __restrict__ pprev, double pv, double th,
                                                 int32_t* status, int64_t* iters, double* meas, int strict,
                                                 int64_t max_iter, int32_t* ndone) {
  const int lane = threadIdx.x & 63;
  const int t0 = tl.inst_t0[inst], t1 = tl.inst_t0[inst + 1];
  for (int t = t0 + 64 + lane; t < t1; t += 64) pv = mx(pv, pprev[t]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pv = mx(pv, __shfl_xor(pv, o, 64));
  int32_t st = ST_RUN;
  if (!finite(pv)) st = ST_NONFINITE;
  else if (strict ? (pv < th) : (pv <= th)) st = ST_CONVERGED;
  else if (s >= max_iter) st = ST_MAXITER;
  st = __builtin_amdgcn_readfirstlane(st);
  if (threadIdx.x == 0 && c == t0) {
    meas[inst] = pv;  // latest measure, also while running (stagnation watch)
    if (st != ST_RUN) {
      status[inst] = st;
      iters[inst] = s;
      atomicAdd(ndone, 1);
    }
  }
  return st;
}

// Copy x[w0, w0+nw) into LDS with 16-byte loads, several in flight per thread.
template <typename T, int NT>
__device__ __forceinline__ void stage_window(T* __restrict__ xs, const T* __restrict__ x, int w0, int nw) {
  constexpr int V = 16 / sizeof(T);
  const int nv = nw / V;  // w0 and nw are multiples of PAD, so x + w0 is 16-byte aligned
  const float4* __restrict__ src = reinterpret_cast<const float4*>(x + w0);
  float4* __restrict__ dst = reinterpret_cast<float4*>(xs);
  int i = threadIdx.x;
  for (; i + 3 * NT < nv; i += 4 * NT) {
    const float4 a = src[i], b = src[i + NT], c = src[i + 2 * NT], d = src[i + 3 * NT];
    dst[i] = a; dst[i + NT] = b; dst[i + 2 * NT] = c; dst[i + 3 * NT] = d;
  }
  for (; i < nv; i += NT) dst[i] = src[i];
  for (int k = nv * V + threadIdx.x; k < nw; k += NT) xs[k] = x[w0 + k];
}

// Rows are taken TU at a time per lane group and the first TJ entries of each
// lane are loaded before any is used, so a wavefront keeps TU*TJ independent
// col/val loads in flight; longer rows finish in a remainder loop.  (Loading
// the next batch before summing this one doubles the registers and halves
// the blocks per CU of the FP32 sweep; it measured slower.)
constexpr int TU = 2, TJ = 4;
constexpr int kNoEntry = INT_MIN;

// Tile handled by this block.  Workgroups are dispatched to the 8 XCDs in
// turn (block b runs on XCD b mod 8); numbering the tiles so that each XCD
// gets a contiguous range puts the tiles of one instance, which read the
// same x window and write the rows the others read next, under one L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  constexpr int X = 8;
  const int q = nblocks / X, r = nblocks % X, x = b % X, slot = b / X;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + slot;
}
// Tile of this block in a launch of one block per tile: the tile set's
// balanced order where it has one (the same per-XCD grouping, with the XCDs'
// shares of the work evened out and each XCD taking its largest tiles first).
__device__ __forceinline__ int tile_of(const Tiles& tl) {
  return tl.order ? tl.order[blockIdx.x] : xcd_tile(blockIdx.x, gridDim.x);
}

// x[w0 + c] for a tile whose window is of kind KIND (LDS window xs of nw
// rows starting at row w0, global vector xg).
template <int KIND, typename T>
__device__ __forceinline__ T xget(const T* __restrict__ xs, const T* __restrict__ xg, int c, int nw, int w0) {
  if (KIND == WIN_WHOLE) return xs[c];
  if (KIND == WIN_NONE) return xg[w0 + c];
  return ((unsigned)c < (unsigned)nw) ? xs[c] : xg[w0 + c];
}

// Column of entry k relative to the window start w0: the 16-bit copy where
// the window is the instance's whole block (it starts at the block's first
// row), the 32-bit index otherwise.
template <int KIND, typename T>
__device__ __forceinline__ int colrel(const MatView<T>& m, int k, int w0) {
  if (KIND == WIN_WHOLE) return (int)m.c16[k];
  return m.col[k] - w0;
}

template <typename T, int L>
struct RowBatch {
  int k0[TU], k1[TU];
  T bi[TU], di[TU];
  int cc[TU][TJ];
  T vv[TU][TJ];

  // rows base + u*RPP + g of the tile; rhs may be null (not needed)
  template <int KIND>
  __device__ __forceinline__ void load(const MatView<T>& m, const T* __restrict__ rhs, int r0, int nr, int base, int g,
                                       int lane, int w0) {
    constexpr int RPP = TNT / L;
#pragma unroll
    for (int u = 0; u < TU; u++) {
      const int i = base + u * RPP + g;
      if (i < nr) {
        k0[u] = m.rp[r0 + i];
        k1[u] = m.rp[r0 + i + 1];
        bi[u] = rhs ? rhs[r0 + i] : (T)0;
        di[u] = m.d[r0 + i];
      } else {
        k0[u] = 0; k1[u] = 0; bi[u] = 0; di[u] = 1;
      }
    }
#pragma unroll
    for (int u = 0; u < TU; u++)
#pragma unroll
      for (int j = 0; j < TJ; j++) {
        const int k = k0[u] + lane + j * L;
        if (k < k1[u]) { cc[u][j] = colrel<KIND>(m, k, w0); vv[u][j] = m.val[k]; }
        else { cc[u][j] = kNoEntry; vv[u][j] = 0; }
      }
  }

  // row sum of A_off times x for row u (valid in every lane of the group)
  template <int KIND>
  __device__ __forceinline__ T sum(const MatView<T>& m, const T* __restrict__ xs, const T* __restrict__ xg, int nw,
                                   int u, int lane, int w0) const {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < TJ; j++)
      if (cc[u][j] != kNoEntry) acc += vv[u][j] * xget<KIND>(xs, xg, cc[u][j], nw, w0);
    for (int k = k0[u] + lane + TJ * L; k < k1[u]; k += L) acc += m.val[k] * xget<KIND>(xs, xg, colrel<KIND>(m, k, w0), nw, w0);
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
    return acc;
  }
};

// Jacobi rows of one tile: xn = (rhs + A_off x) / d; returns the tile's max of
// the stopping measure (|dx|, or d |dx| when weighted).
template <typename T, int L, int KIND>
__device__ __forceinline__ double jacobi_rows(const MatView<T>& m, const T* __restrict__ rhs, const T* __restrict__ xs,
                                              const T* __restrict__ x, T* __restrict__ xn, int r0, int nr, int w0,
                                              int nw, int weighted) {
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = TNT / L;
  double mloc = 0.0;
  for (int base = 0; base < nr; base += RPP * TU) {
    RowBatch<T, L> rb;
    rb.template load<KIND>(m, rhs, r0, nr, base, g, lane, w0);
#pragma unroll
    for (int u = 0; u < TU; u++) {
      const T acc = rb.template sum<KIND>(m, xs, x, nw, u, lane, w0);
      const int i = base + u * RPP + g;
      if (i < nr && lane == 0) {
        const int row = r0 + i;
        const T nv = (rb.bi[u] + acc) / rb.di[u];
        const double dl = fabs((double)nv - (double)xget<KIND>(xs, x, row - w0, nw, w0));
        xn[row] = nv;
        mloc = mx(mloc, weighted ? (double)rb.di[u] * dl : dl);
      }
    }
  }
  return mloc;
}

// Start of a tiled sweep s: copy the x window into LDS and take the decision
// on sweep s-1.  The instance's per-tile maxima of sweep s-1 and its
// threshold are loaded before the window copy so that their latency overlaps
// it (the copy is wasted only on the sweep that stops).  Returns false when
// the instance stops (uniform over the block).
template <typename T>
__device__ __forceinline__ bool jacobi_begin(T* xs, const T* __restrict__ x, const Tiles& tl, int c, int inst, int kind,
                                             int w0, int nw, int64_t s, const double* __restrict__ pprev,
                                             int32_t* status, int64_t* iters, double* meas,
                                             const double* __restrict__ thr, int strict, int64_t max_iter,
                                             int32_t* ndone) {
  double pv = 0.0, th = 0.0;
  if (s > 0) {
    const int t = tl.inst_t0[inst] + (threadIdx.x & 63);
    if (t < tl.inst_t0[inst + 1]) pv = pprev[t];
    th = thr[inst];
  }
  if (kind != WIN_NONE) stage_window<T, TNT>(xs, x, w0, nw);
  if (s > 0 && jacobi_decide(tl, c, inst, s, pprev, pv, th, status, iters, meas, strict, max_iter, ndone) != ST_RUN)
    return false;
  if (kind != WIN_NONE) __syncthreads();
  return true;
}

template <typename T, int L>
__global__ __launch_bounds__(TNT) void k_jacobi_tile(MatView<T> m, const T* __restrict__ rhs, const T* __restrict__ x,
                                                     T* __restrict__ xn, Tiles tl, int64_t s_rel,
                                                     const double* __restrict__ pprev, double* __restrict__ pcur,
                                                     int32_t* status, int64_t* iters, double* meas,
                                                     const double* __restrict__ thr, int strict, int64_t max_iter,
                                                     int32_t* ndone, int weighted) {
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int c = tile_of(tl);
  const int inst = tl.inst[c];
  const int w0 = tl.w0[c], nw = tl.nw[c], kind = tl.kind[c];
  const int r0 = tl.row0[c], nr = tl.nrows[c];
  if (status[inst] != ST_RUN) return;
  const int64_t s = s_rel + (tl.sbase ? *tl.sbase : 0);
  if (!jacobi_begin<T>(xs, x, tl, c, inst, kind, w0, nw, s, pprev, status, iters, meas, thr, strict, max_iter, ndone))
    return;
  double mloc;
  if (kind == WIN_WHOLE) mloc = jacobi_rows<T, L, WIN_WHOLE>(m, rhs, xs, x, xn, r0, nr, w0, nw, weighted);
  else if (kind == WIN_BAND) mloc = jacobi_rows<T, L, WIN_BAND>(m, rhs, xs, x, xn, r0, nr, w0, nw, weighted);
  else mloc = jacobi_rows<T, L, WIN_NONE>(m, rhs, xs, x, xn, r0, nr, w0, nw, weighted);
  double v[1] = {mloc};
  block_reduce<1, TNT>(v, 1u);
  if (threadIdx.x == 0) pcur[c] = v[0];
}

template <typename T, int L>
static hipError_t launch_tile_L(hipStream_t st, MatView<T> m, const T* rhs, const T* x, T* xn, Tiles tl, int64_t s,
                                const double* pprev, double* pcur, int32_t* status, int64_t* iters, double* meas,
                                const double* thr, int strict, int64_t max_iter, int32_t* ndone, int weighted) {
  const size_t lds = (size_t)tl.maxw * sizeof(T);
  static size_t configured = 0;
  if (lds > configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_tile<T, L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    configured = lds;
  }
  k_jacobi_tile<T, L><<<(unsigned)tl.ntile, TNT, lds, st>>>(m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas,
                                                            thr, strict, max_iter, ndone, weighted);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi_tile(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x, T* xn, Tiles tl,
                              int64_t s, const double* pprev, double* pcur, int32_t* status, int64_t* iters,
                              double* meas, const double* thr, int strict, int64_t max_iter, int32_t* ndone,
                              int weighted) {
  switch (L) {
    case 1: return launch_tile_L<T, 1>(st, m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 2: return launch_tile_L<T, 2>(st, m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 4: return launch_tile_L<T, 4>(st, m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 8: return launch_tile_L<T, 8>(st, m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 16: return launch_tile_L<T, 16>(st, m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 32: return launch_tile_L<T, 32>(st, m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 64: return launch_tile_L<T, 64>(st, m, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_jacobi_tile<double>(hipStream_t, int, MatView<double>, const double*, const double*, double*,
                                               Tiles, int64_t, const double*, double*, int32_t*, int64_t*, double*,
                                               const double*, int, int64_t, int32_t*, int);
template hipError_t launch_jacobi_tile<float>(hipStream_t, int, MatView<float>, const float*, const float*, float*,
                                              Tiles, int64_t, const double*, double*, int32_t*, int64_t*, double*,
                                              const double*, int, int64_t, int32_t*, int);

// ---------------------------------------------------------------------------
// Resident Jacobi: one block holds a whole small instance -- both iterates in
// LDS -- and runs up to nsweeps sweeps in one launch, deciding after each one
// with the same rule as the tiled sweeps (stop on m < thr (strict) or
// m <= thr, on a non-finite m, or when the sweep count reaches max_iter).
// On exit the latest iterate goes to the buffer the sweep-count parity
// names (xb when odd), like the tiled sweeps leave it.  When the instance's
// rows fit one row batch the matrix rows stay in registers across sweeps.
template <typename T, int L>
__device__ __forceinline__ double resident_rows(const RowBatch<T, L>& rb, const MatView<T>& m, const T* __restrict__ cur,
                                                T* __restrict__ nxt, int base, int nr, int lane, int weighted) {
  constexpr int RPP = TNT / L;
  const int g = threadIdx.x / L;
  double mloc = 0.0;
#pragma unroll
  for (int u = 0; u < TU; u++) {
    const T acc = rb.template sum<WIN_WHOLE>(m, cur, nullptr, 0, u, lane, 0);
    const int i = base + u * RPP + g;
    if (i < nr && lane == 0) {
      const T nv = (rb.bi[u] + acc) / rb.di[u];
      const double dl = fabs((double)nv - (double)cur[i]);
      nxt[i] = nv;
      mloc = mx(mloc, weighted ? (double)rb.di[u] * dl : dl);
    }
  }
  return mloc;
}

template <typename T, int L>
__global__ __launch_bounds__(TNT) void k_jacobi_resident(MatView<T> m, const T* __restrict__ rhs, T* xa, T* xb,
                                                         Tiles tl, int64_t s0, int nsweeps, int32_t* status,
                                                         int64_t* iters, double* meas,
                                                         const double* __restrict__ thr, int strict,
                                                         int64_t max_iter, int32_t* ndone, int weighted) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ int32_t decision;
  const int c = blockIdx.x;
  const int inst = tl.inst[c];
  if (status[inst] != ST_RUN) return;
  const int r0 = tl.row0[c], nr = tl.nrows[c];  // the tile is the whole instance block (w0 = r0, nw = nr)
  T* X0 = reinterpret_cast<T*>(smem_raw);
  T* X1 = X0 + tl.maxw;
  stage_window<T, TNT>(X0, (s0 & 1) ? xb : xa, r0, nr);
  const int lane = threadIdx.x % L, g = threadIdx.x / L;
  constexpr int RPP = TNT / L;
  const bool one_batch = nr <= RPP * TU;
  RowBatch<T, L> rb;
  if (one_batch) rb.template load<WIN_WHOLE>(m, rhs, r0, nr, 0, g, lane, r0);
  __syncthreads();
  for (int it = 0; it < nsweeps; it++) {
    const T* cur = (it & 1) ? X1 : X0;
    T* nxt = (it & 1) ? X0 : X1;
    double mloc = 0.0;
    if (one_batch) {
      mloc = resident_rows<T, L>(rb, m, cur, nxt, 0, nr, lane, weighted);
    } else {
      for (int base = 0; base < nr; base += RPP * TU) {
        RowBatch<T, L> rbi;
        rbi.template load<WIN_WHOLE>(m, rhs, r0, nr, base, g, lane, r0);
        mloc = mx(mloc, resident_rows<T, L>(rbi, m, cur, nxt, base, nr, lane, weighted));
      }
    }
    double v[1] = {mloc};
    block_reduce<1, TNT>(v, 1u);
    const int64_t done = s0 + it + 1;  // sweeps completed
    if (threadIdx.x == 0) {
      const double mm = v[0];
      int32_t st = ST_RUN;
      if (!finite(mm)) st = ST_NONFINITE;
      else if (strict ? (mm < thr[inst]) : (mm <= thr[inst])) st = ST_CONVERGED;
      else if (done >= max_iter) st = ST_MAXITER;
      meas[inst] = mm;
      if (st != ST_RUN) {
        status[inst] = st;
        iters[inst] = done;
        atomicAdd(ndone, 1);
      }
      decision = st;
    }
    __syncthreads();
    if (decision != ST_RUN || it == nsweeps - 1) {
      T* dst = (done & 1) ? xb : xa;
      for (int i = threadIdx.x; i < nr; i += TNT) dst[r0 + i] = nxt[i];
      // a weighted measure is the residual of the previous iterate: keep it
      // in the other buffer, as the tiled sweeps do
      if (decision != ST_RUN && weighted) {
        T* dprev = (done & 1) ? xa : xb;
        for (int i = threadIdx.x; i < nr; i += TNT) dprev[r0 + i] = cur[i];
      }
      return;
    }
  }
}

template <typename T, int L>
static hipError_t resident_L(hipStream_t st, MatView<T> m, const T* rhs, T* xa, T* xb, Tiles tl, int64_t s0,
                             int nsweeps, int32_t* status, int64_t* iters, double* meas, const double* thr, int strict,
                             int64_t max_iter, int32_t* ndone, int weighted) {
  const size_t lds = 2 * (size_t)tl.maxw * sizeof(T);
  static size_t conf = 0;
  hipError_t e = set_lds(k_jacobi_resident<T, L>, lds, conf);
  if (e != hipSuccess) return e;
  k_jacobi_resident<T, L><<<(unsigned)tl.ntile, TNT, lds, st>>>(m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas,
                                                                thr, strict, max_iter, ndone, weighted);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi_resident(hipStream_t st, int L, MatView<T> m, const T* rhs, T* xa, T* xb, Tiles tl,
                                  int64_t s0, int nsweeps, int32_t* status, int64_t* iters, double* meas,
                                  const double* thr, int strict, int64_t max_iter, int32_t* ndone, int weighted) {
  if (tl.ntile <= 0 || nsweeps <= 0) return hipSuccess;
  switch (L) {
    case 1: return resident_L<T, 1>(st, m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 2: return resident_L<T, 2>(st, m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 4: return resident_L<T, 4>(st, m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 8: return resident_L<T, 8>(st, m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 16: return resident_L<T, 16>(st, m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    case 32: return resident_L<T, 32>(st, m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas, thr, strict, max_iter, ndone, weighted);
    default: return resident_L<T, 64>(st, m, rhs, xa, xb, tl, s0, nsweeps, status, iters, meas, thr, strict, max_iter, ndone, weighted);
  }
}
template hipError_t launch_jacobi_resident<double>(hipStream_t, int, MatView<double>, const double*, double*, double*,
                                                   Tiles, int64_t, int, int32_t*, int64_t*, double*, const double*,
                                                   int, int64_t, int32_t*, int);
template hipError_t launch_jacobi_resident<float>(hipStream_t, int, MatView<float>, const float*, float*, float*,
                                                  Tiles, int64_t, int, int32_t*, int64_t*, double*, const double*,
                                                  int, int64_t, int32_t*, int);

// ---------------------------------------------------------------------------
// Resident BiCGStab: one block holds a whole small instance and runs up to
// nsteps steps in one launch.  The vectors of the rows a lane group owns stay
// in registers (at most BR_SLOTS rows per group); p and s, which the products
// gather, live in LDS.  Every decision is the tiled one (bicg_decide and the
// two in-step breakdown tests) with the reductions done in the block; between
// launches the state goes through x, r, p, v, the partials pc/ps and the
// scalars in BicgState exactly as the tiled kernels leave them.
constexpr int BR_SLOTS = 2;

// Sum over the block of NV values (bit i of maxmask: max, else sum), result in
// every thread.
template <int NV>
__device__ __forceinline__ void block_allreduce(double (&v)[NV], unsigned maxmask) {
  __shared__ double bcast[NV];
  block_reduce<NV, TNT>(v, maxmask);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; i++) bcast[i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; i++) v[i] = bcast[i];
  __syncthreads();
}

// (M u)_row = d_row u_row - sum_j A(row, j) u_j with u in LDS (window = the
// instance block, columns from the 16-bit copy); valid in every lane of the group.
template <typename T, int L>
__device__ __forceinline__ T apply_row(const MatView<T>& m, const T* __restrict__ u, int row, int i, int lane) {
  T acc = 0;
  const int k1 = m.rp[row + 1];
  for (int k = m.rp[row] + lane; k < k1; k += L) acc += m.val[k] * u[m.c16[k]];
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
  return m.d[row] * u[i] - acc;
}

template <typename T, int L>
__global__ __launch_bounds__(TNT) void k_bicg_resident(MatView<T> m, const T* __restrict__ rhs, T* x, T* r, T* q,
                                                       T* p, T* v, Tiles tl, int64_t s0, int nsteps, int x_is_zero,
                                                       double* pc, double* ps, BicgState b) {
  extern __shared__ unsigned char smem_raw[];
  const int c = blockIdx.x;
  const int inst = tl.inst[c];
  if (b.status[inst] != ST_RUN) return;
  const int r0 = tl.row0[c], nr = tl.nrows[c];
  T* P = reinterpret_cast<T*>(smem_raw);
  T* S = P + tl.maxw;
  const int lane = threadIdx.x % L, g = threadIdx.x / L;
  constexpr int RPP = TNT / L;
  T xr[BR_SLOTS], rr[BR_SLOTS], qr[BR_SLOTS], pr[BR_SLOTS], vr[BR_SLOTS];
  double rnew, rmax, smax = 0.0, rho_prev = 0.0, alpha = 0.0, omega = 0.0;
  if (s0 == 0) {
    // start: r = rhs - M x (x = 0: r = rhs), q = r, p = v = 0
    if (!x_is_zero) {
      for (int i = threadIdx.x; i < nr; i += TNT) P[i] = x[r0 + i];
      __syncthreads();
    }
    double a[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < BR_SLOTS; u++) {
      const int i = u * RPP + g;
      xr[u] = rr[u] = qr[u] = pr[u] = vr[u] = 0;
      if (i < nr) {
        const int row = r0 + i;
        const T ri = x_is_zero ? rhs[row] : rhs[row] - apply_row<T, L>(m, P, row, i, lane);
        xr[u] = x_is_zero ? (T)0 : P[i];
        rr[u] = ri;
        qr[u] = ri;
        if (lane == 0) {
          q[row] = ri;
          a[0] += (double)ri * (double)ri;
          a[1] = mx(a[1], fabs((double)ri));
        }
      }
    }
    block_allreduce<2>(a, 2u);
    rnew = a[0];
    rmax = a[1];
  } else {
#pragma unroll
    for (int u = 0; u < BR_SLOTS; u++) {
      const int i = u * RPP + g;
      xr[u] = rr[u] = qr[u] = pr[u] = vr[u] = 0;
      if (i < nr) {
        const int row = r0 + i;
        xr[u] = x[row]; rr[u] = r[row]; qr[u] = q[row]; pr[u] = p[row]; vr[u] = v[row];
      }
    }
    rnew = pc[2 * c];
    rmax = pc[2 * c + 1];
    smax = ps[c];
    rho_prev = b.rho[((s0 - 1) & 1) * tl.K + inst];
    alpha = b.alpha[inst];
    omega = b.omega[inst];
  }
  int64_t j = s0;
  bool stopped = false;
  for (int it = 0;; it++, j++) {
    // decision on the state after j steps (as bicg_decide); after nsteps steps
    // the launch ends with it taken (a final one may stop the instance at
    // max_iter) and the next launch takes it again
    int32_t st = ST_RUN;
    double mm, beta = 0.0;
    if (j == 0) {
      mm = rmax;
      if (!finite(rnew) || !finite(rmax)) st = ST_NONFINITE;
      else if (rmax == 0.0) st = ST_CONVERGED;
      else if (b.measmode == MEAS_R && rmax <= b.thr[inst]) st = ST_CONVERGED;
    } else {
      mm = (b.measmode == MEAS_S) ? smax : rmax;
      if (!finite(rnew) || !finite(mm)) st = ST_NONFINITE;
      else if (mm <= b.thr[inst]) st = ST_CONVERGED;
      else if (j >= b.max_iter) st = ST_MAXITER;
      else if (rnew == 0.0 || omega == 0.0) st = ST_BREAKDOWN;
      else beta = (rnew / rho_prev) * (alpha / omega);
    }
    if (st == ST_RUN && it == nsteps) {
      if (threadIdx.x == 0) b.meas[inst] = mm;  // latest measure (stagnation watch)
      break;
    }
    if (st == ST_RUN) {
      const double rho = rnew;
      const T bt = (T)beta, w = (T)omega;
      // p = r + beta (p - omega v)
#pragma unroll
      for (int u = 0; u < BR_SLOTS; u++) {
        const int i = u * RPP + g;
        if (i < nr) {
          pr[u] = rr[u] + bt * (pr[u] - w * vr[u]);
          if (lane == 0) P[i] = pr[u];
        }
      }
      __syncthreads();
      // v = M p, q.v
      double a1[1] = {0.0};
#pragma unroll
      for (int u = 0; u < BR_SLOTS; u++) {
        const int i = u * RPP + g;
        if (i < nr) {
          vr[u] = apply_row<T, L>(m, P, r0 + i, i, lane);
          if (lane == 0) a1[0] += (double)qr[u] * (double)vr[u];
        }
      }
      block_allreduce<1>(a1, 0u);
      const double qv = a1[0];
      if (!finite(qv) || qv == 0.0) {
        st = finite(qv) ? ST_BREAKDOWN : ST_NONFINITE;
        mm = qv;
      } else {
        alpha = rho / qv;
        const T al = (T)alpha;
        // s = r - alpha v
        double a3[3] = {0.0, 0.0, 0.0};
        T sr[BR_SLOTS];
#pragma unroll
        for (int u = 0; u < BR_SLOTS; u++) {
          const int i = u * RPP + g;
          sr[u] = 0;
          if (i < nr) {
            sr[u] = rr[u] - al * vr[u];
            if (lane == 0) {
              S[i] = sr[u];
              a3[2] = mx(a3[2], fabs((double)sr[u]));
            }
          }
        }
        __syncthreads();
        // t = M s, (t.s, t.t)
        T tr[BR_SLOTS];
#pragma unroll
        for (int u = 0; u < BR_SLOTS; u++) {
          const int i = u * RPP + g;
          tr[u] = 0;
          if (i < nr) {
            tr[u] = apply_row<T, L>(m, S, r0 + i, i, lane);
            if (lane == 0) {
              a3[0] += (double)tr[u] * (double)sr[u];
              a3[1] += (double)tr[u] * (double)tr[u];
            }
          }
        }
        block_allreduce<3>(a3, 4u);
        smax = a3[2];
        if (!finite(a3[0]) || !finite(a3[1])) {
          st = ST_NONFINITE;
          mm = a3[0];
        } else {
          omega = (a3[1] == 0.0) ? 0.0 : a3[0] / a3[1];
          const T om = (T)omega;
          double a2[2] = {0.0, 0.0};
#pragma unroll
          for (int u = 0; u < BR_SLOTS; u++) {
            const int i = u * RPP + g;
            if (i < nr) {
              xr[u] = xr[u] + al * pr[u] + om * sr[u];
              rr[u] = sr[u] - om * tr[u];
              if (lane == 0) {
                a2[0] += (double)qr[u] * (double)rr[u];
                a2[1] = mx(a2[1], fabs((double)rr[u]));
              }
            }
          }
          block_allreduce<2>(a2, 2u);
          rnew = a2[0];
          rmax = a2[1];
          rho_prev = rho;
        }
      }
    }
    if (st != ST_RUN) {
      if (threadIdx.x == 0) {
        b.status[inst] = st;
        b.iters[inst] = j;
        b.meas[inst] = mm;
        atomicAdd(b.ndone, 1);
      }
      stopped = true;
      break;
    }
  }
  // state for the next launch (or the result)
#pragma unroll
  for (int u = 0; u < BR_SLOTS; u++) {
    const int i = u * RPP + g;
    if (i < nr && lane == 0) {
      const int row = r0 + i;
      x[row] = xr[u]; r[row] = rr[u]; p[row] = pr[u]; v[row] = vr[u];
    }
  }
  if (threadIdx.x == 0 && !stopped) {
    pc[2 * c] = rnew;
    pc[2 * c + 1] = rmax;
    ps[c] = smax;
    b.rho[((j - 1) & 1) * tl.K + inst] = rho_prev;
    b.alpha[inst] = alpha;
    b.omega[inst] = omega;
  }
}

template <typename T, int L>
static hipError_t bicg_resident_L(hipStream_t st, MatView<T> m, const T* rhs, T* x, T* r, T* q, T* p, T* v, Tiles tl,
                                  int64_t s0, int nsteps, int x_is_zero, double* pc, double* ps, BicgState b) {
  const size_t lds = 2 * (size_t)tl.maxw * sizeof(T);
  static size_t conf = 0;
  hipError_t e = set_lds(k_bicg_resident<T, L>, lds, conf);
  if (e != hipSuccess) return e;
  k_bicg_resident<T, L><<<(unsigned)tl.ntile, TNT, lds, st>>>(m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc,
                                                              ps, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bicg_resident(hipStream_t st, int L, MatView<T> m, const T* rhs, T* x, T* r, T* q, T* p, T* v,
                                Tiles tl, int64_t s0, int nsteps, int x_is_zero, double* pc, double* ps,
                                BicgState b) {
  if (tl.ntile <= 0 || nsteps <= 0) return hipSuccess;
  switch (L) {
    case 1: return bicg_resident_L<T, 1>(st, m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc, ps, b);
    case 2: return bicg_resident_L<T, 2>(st, m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc, ps, b);
    case 4: return bicg_resident_L<T, 4>(st, m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc, ps, b);
    case 8: return bicg_resident_L<T, 8>(st, m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc, ps, b);
    case 16: return bicg_resident_L<T, 16>(st, m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc, ps, b);
    case 32: return bicg_resident_L<T, 32>(st, m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc, ps, b);
    default: return bicg_resident_L<T, 64>(st, m, rhs, x, r, q, p, v, tl, s0, nsteps, x_is_zero, pc, ps, b);
  }
}
template hipError_t launch_bicg_resident<double>(hipStream_t, int, MatView<double>, const double*, double*, double*,
                                                 double*, double*, double*, Tiles, int64_t, int, int, double*, double*,
                                                 BicgState);
template hipError_t launch_bicg_resident<float>(hipStream_t, int, MatView<float>, const float*, float*, float*, float*,
                                                float*, float*, Tiles, int64_t, int, int, double*, double*, BicgState);

// Stopping decision after the last sweep of a batch of launches (s = sweeps
// completed), one block per instance; same rule as jacobi_decide.
__global__ void k_jacobi_check(Tiles tl, int64_t s_rel, const double* __restrict__ pprev, int32_t* status,
                               int64_t* iters, double* meas, const double* __restrict__ thr, int strict,
                               int64_t max_iter, int32_t* ndone) {
  const int k = blockIdx.x;
  if (status[k] != ST_RUN) return;
  const int64_t s = s_rel + (tl.sbase ? *tl.sbase : 0);
  const int t = tl.inst_t0[k] + (threadIdx.x & 63);
  const double pv = t < tl.inst_t0[k + 1] ? pprev[t] : 0.0;
  jacobi_decide(tl, tl.inst_t0[k], k, s, pprev, pv, thr[k], status, iters, meas, strict, max_iter, ndone);
}
hipError_t launch_jacobi_check(hipStream_t st, Tiles tl, int64_t s, const double* pprev, int32_t* status,
                               int64_t* iters, double* meas, const double* thr, int strict, int64_t max_iter,
                               int32_t* ndone) {
  k_jacobi_check<<<(unsigned)tl.K, BS, 0, st>>>(tl, s, pprev, status, iters, meas, thr, strict, max_iter, ndone);
  return hipGetLastError();
}

// ============================================================================
// BiCGStab on tiles (every instance block fits one workgroup's LDS).  One
// step is five launches: p-update, v = M p, s-update, t = M s, x/r-update.
// The scalar each launch needs (beta, alpha, omega) is reduced from the
// previous launch's per-tile partials by every block of the instance at the
// start of the launch (same order, same value everywhere), and the stopping
// test of step j is taken at the start of step j+1's p-update.  Scalars read
// and written by one launch (rho) are double-buffered by step parity.
// ============================================================================



__device__ __forceinline__ void bicg_stop(const Tiles& tl, int c, int inst, const BicgState& b, int32_t st,
                                          int64_t j, double m) {
  if (c == tl.inst_t0[inst]) {
    b.status[inst] = st;
    b.iters[inst] = j;
    b.meas[inst] = m;
    atomicAdd(b.ndone, 1);
  }
}

__device__ __forceinline__ double wave_uniform(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Reduce NV per-tile partials of instance inst inside each wavefront: lane l
// takes tiles t0 + l, t0 + l + 64, ... in order, then an xor butterfly, whose
// pairwise steps are commutative, leaves the same value in every lane; every
// wavefront of every block of the instance does the same operations, so the
// result is identical everywhere and deterministic, and no barrier is needed
// (a block-wide reduction here cost ~3 us per launch).  NT is unused.
template <int NV, int NT>
__device__ __forceinline__ void tile_reduce(const Tiles& tl, int inst, const double* __restrict__ part,
                                            unsigned maxmask, double (&v)[NV]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; i++) v[i] = 0.0;
  for (int t = tl.inst_t0[inst] + lane; t < tl.inst_t0[inst + 1]; t += 64) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      const double p = part[(size_t)t * NV + i];
      v[i] = ((maxmask >> i) & 1u) ? mx(v[i], p) : v[i] + p;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < NV; i++) {
      const double w = __shfl_xor(v[i], o, 64);
      v[i] = ((maxmask >> i) & 1u) ? mx(v[i], w) : v[i] + w;
    }
#pragma unroll
  for (int i = 0; i < NV; i++) v[i] = wave_uniform(v[i]);
}

// Stopping test of step j (j completed steps) and the beta of step j.
// pc: (q.r, max|r|) of step j-1 (or of the initial residual when j = 0);
// ps: max|s| of step j-1.  Returns false when the instance stops.
template <int NT>
__device__ __forceinline__ bool bicg_decide(const Tiles& tl, int c, int inst, int64_t j, const double* __restrict__ pc,
                                            const double* __restrict__ ps, const BicgState& b, double& beta) {
  double v[2];
  tile_reduce<2, NT>(tl, inst, pc, 2u, v);
  const double rnew = v[0], rmax = v[1];
  double smax = 0.0;
  if (j > 0) {
    double w[1];
    tile_reduce<1, NT>(tl, inst, ps, 1u, w);
    smax = w[0];
  }
  int32_t st = ST_RUN;
  double m;
  if (j == 0) {
    m = rmax;
    if (!finite(rnew) || !finite(rmax)) st = ST_NONFINITE;
    else if (rmax == 0.0) st = ST_CONVERGED;
    else if (b.measmode == MEAS_R && rmax <= b.thr[inst]) st = ST_CONVERGED;
    beta = 0.0;
  } else {
    m = (b.measmode == MEAS_S) ? smax : rmax;
    const double om = b.omega[inst];
    if (!finite(rnew) || !finite(m)) st = ST_NONFINITE;
    else if (m <= b.thr[inst]) st = ST_CONVERGED;
    else if (j >= b.max_iter) st = ST_MAXITER;
    else if (rnew == 0.0 || om == 0.0) st = ST_BREAKDOWN;
    else beta = (rnew / b.rho[((j - 1) & 1) * tl.K + inst]) * (b.alpha[inst] / om);
  }
  if (st != ST_RUN) {
    if (threadIdx.x == 0) bicg_stop(tl, c, inst, b, st, j, m);
    return false;
  }
  if (threadIdx.x == 0 && c == tl.inst_t0[inst]) {
    b.rho[(j & 1) * tl.K + inst] = rnew;
    b.meas[inst] = m;  // latest measure, also while running (stagnation watch)
  }
  return true;
}

// Rows of one tile for the BiCGStab start; KIND -1 means x = 0.
template <typename T, int L, int KIND>
__device__ __forceinline__ void bicg_init_rows(const MatView<T>& m, const T* __restrict__ rhs,
                                               const T* __restrict__ xs, const T* __restrict__ x, T* __restrict__ r,
                                               T* __restrict__ q, T* __restrict__ p, T* __restrict__ v, int r0, int nr,
                                               int w0, int nw, double* a) {
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = TNT / L;
  for (int base = 0; base < nr; base += RPP) {
    const bool ok = base + g < nr;
    const int row = r0 + base + g;
    T ri = 0;
    if (KIND >= 0) {
      T acc = 0;
      if (ok) {
        const int k1 = m.rp[row + 1];
        for (int k = m.rp[row] + lane; k < k1; k += L) acc += m.val[k] * xget<KIND>(xs, x, colrel<KIND>(m, k, w0), nw, w0);
      }
#pragma unroll
      for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
      if (ok && lane == 0) ri = rhs[row] - (m.d[row] * xget<KIND>(xs, x, row - w0, nw, w0) - acc);
    } else if (ok && lane == 0) {
      ri = rhs[row];
    }
    if (ok && lane == 0) {
      r[row] = ri; q[row] = ri; p[row] = 0; v[row] = 0;
      a[0] += (double)ri * (double)ri;
      a[1] = mx(a[1], fabs((double)ri));
    }
  }
}

// r = rhs - M x (or rhs when x = 0), q = r, p = v = 0; partials (q.r, max|r|)
template <typename T, int L>
__global__ __launch_bounds__(TNT) void k_bicg_init_tile(MatView<T> m, const T* __restrict__ rhs,
                                                        const T* __restrict__ x, int x_is_zero, T* __restrict__ r,
                                                        T* __restrict__ q, T* __restrict__ p, T* __restrict__ v,
                                                        Tiles tl, const int32_t* __restrict__ status,
                                                        double* __restrict__ pc) {
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int c = tile_of(tl);
  if (status[tl.inst[c]] != ST_RUN) return;
  const int r0 = tl.row0[c], nr = tl.nrows[c], w0 = tl.w0[c], nw = tl.nw[c], kind = tl.kind[c];
  if (!x_is_zero && kind != WIN_NONE) {
    stage_window<T, TNT>(xs, x, w0, nw);
    __syncthreads();
  }
  double a[2] = {0.0, 0.0};
  if (x_is_zero) bicg_init_rows<T, L, -1>(m, rhs, xs, x, r, q, p, v, r0, nr, w0, nw, a);
  else if (kind == WIN_WHOLE) bicg_init_rows<T, L, WIN_WHOLE>(m, rhs, xs, x, r, q, p, v, r0, nr, w0, nw, a);
  else if (kind == WIN_BAND) bicg_init_rows<T, L, WIN_BAND>(m, rhs, xs, x, r, q, p, v, r0, nr, w0, nw, a);
  else bicg_init_rows<T, L, WIN_NONE>(m, rhs, xs, x, r, q, p, v, r0, nr, w0, nw, a);
  block_reduce<2, TNT>(a, 2u);
  if (threadIdx.x == 0) { pc[2 * c] = a[0]; pc[2 * c + 1] = a[1]; }
}

// decision of step j, then p = r + beta (p - omega v)
template <typename T>
__global__ __launch_bounds__(TNT) void k_bicg_p_tile(const T* __restrict__ r, T* __restrict__ p, const T* __restrict__ v,
                                                     Tiles tl, int64_t j, const double* __restrict__ pc,
                                                     const double* __restrict__ ps, BicgState b) {
  const int c = tile_of(tl);
  const int inst = tl.inst[c];
  if (b.status[inst] != ST_RUN) return;
  double beta = 0.0;
  if (!bicg_decide<TNT>(tl, c, inst, j, pc, ps, b, beta)) return;
  const T bt = (T)beta, w = (T)(j > 0 ? b.omega[inst] : 0.0);
  const int r0 = tl.row0[c], nr = tl.nrows[c];
  for (int i = threadIdx.x; i < nr; i += TNT) {
    const int row = r0 + i;
    p[row] = r[row] + bt * (p[row] - w * v[row]);
  }
}

// y = M u = d u - A_off u with u staged in LDS; partials: mode 0 q.y, mode 1 (y.u, y.y)
// y = M u over one tile's rows; MODE 0 accumulates q.y, MODE 1 (y.u, y.y).
template <typename T, int L, int MODE, int KIND>
__device__ __forceinline__ void spmv_rows(const MatView<T>& m, const T* __restrict__ us, const T* __restrict__ u,
                                          T* __restrict__ y, const T* __restrict__ q, int r0, int nr, int w0, int nw,
                                          double* a) {
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = TNT / L;
  for (int base = 0; base < nr; base += RPP * TU) {
    RowBatch<T, L> rb;
    rb.template load<KIND>(m, nullptr, r0, nr, base, g, lane, w0);
#pragma unroll
    for (int uu = 0; uu < TU; uu++) {
      const T acc = rb.template sum<KIND>(m, us, u, nw, uu, lane, w0);
      const int i = base + uu * RPP + g;
      if (i < nr && lane == 0) {
        const int row = r0 + i;
        const T ui = xget<KIND>(us, u, row - w0, nw, w0);
        const T yi = rb.di[uu] * ui - acc;
        y[row] = yi;
        if (MODE == 0) {
          a[0] += (double)q[row] * (double)yi;
        } else {
          a[0] += (double)yi * (double)ui;
          a[1] += (double)yi * (double)yi;
        }
      }
    }
  }
}

template <typename T, int L, int MODE>
__global__ __launch_bounds__(TNT) void k_spmv_tile(MatView<T> m, const T* __restrict__ u, T* __restrict__ y,
                                                   const T* __restrict__ q, Tiles tl,
                                                   const int32_t* __restrict__ status, double* __restrict__ part) {
  extern __shared__ unsigned char smem_raw[];
  T* us = reinterpret_cast<T*>(smem_raw);
  const int c = tile_of(tl);
  if (status[tl.inst[c]] != ST_RUN) return;
  const int r0 = tl.row0[c], nr = tl.nrows[c], w0 = tl.w0[c], nw = tl.nw[c], kind = tl.kind[c];
  if (kind != WIN_NONE) {
    stage_window<T, TNT>(us, u, w0, nw);
    __syncthreads();
  }
  double a[2] = {0.0, 0.0};
  if (kind == WIN_WHOLE) spmv_rows<T, L, MODE, WIN_WHOLE>(m, us, u, y, q, r0, nr, w0, nw, a);
  else if (kind == WIN_BAND) spmv_rows<T, L, MODE, WIN_BAND>(m, us, u, y, q, r0, nr, w0, nw, a);
  else spmv_rows<T, L, MODE, WIN_NONE>(m, us, u, y, q, r0, nr, w0, nw, a);
  if (MODE == 0) {
    double b1[1] = {a[0]};
    block_reduce<1, TNT>(b1, 0u);
    if (threadIdx.x == 0) part[c] = b1[0];
  } else {
    block_reduce<2, TNT>(a, 0u);
    if (threadIdx.x == 0) { part[2 * c] = a[0]; part[2 * c + 1] = a[1]; }
  }
}

// alpha = rho / (q.v); s = r - alpha v; partial max|s|
template <typename T>
__global__ __launch_bounds__(TNT) void k_bicg_s_tile(const T* __restrict__ r, const T* __restrict__ v, T* __restrict__ s,
                                                     Tiles tl, int64_t j, const double* __restrict__ pa,
                                                     double* __restrict__ ps, BicgState b) {
  const int c = tile_of(tl);
  const int inst = tl.inst[c];
  if (b.status[inst] != ST_RUN) return;
  double qv[1];
  tile_reduce<1, TNT>(tl, inst, pa, 0u, qv);
  if (!finite(qv[0]) || qv[0] == 0.0) {
    if (threadIdx.x == 0) bicg_stop(tl, c, inst, b, finite(qv[0]) ? ST_BREAKDOWN : ST_NONFINITE, j, qv[0]);
    return;
  }
  const double alpha = b.rho[(j & 1) * tl.K + inst] / qv[0];
  if (threadIdx.x == 0 && c == tl.inst_t0[inst]) b.alpha[inst] = alpha;
  const T a = (T)alpha;
  const int r0 = tl.row0[c], nr = tl.nrows[c];
  double mloc = 0.0;
  for (int i = threadIdx.x; i < nr; i += TNT) {
    const int row = r0 + i;
    const T si = r[row] - a * v[row];
    s[row] = si;
    mloc = mx(mloc, fabs((double)si));
  }
  double b1[1] = {mloc};
  block_reduce<1, TNT>(b1, 1u);
  if (threadIdx.x == 0) ps[c] = b1[0];
}

// omega = (t.s)/(t.t); x += alpha p + omega s; r = s - omega t; partials (q.r, max|r|)
template <typename T>
__global__ __launch_bounds__(TNT) void k_bicg_xr_tile(T* __restrict__ x, const T* __restrict__ p, const T* __restrict__ s,
                                                      T* __restrict__ r, const T* __restrict__ t, const T* __restrict__ q,
                                                      Tiles tl, int64_t j, const double* __restrict__ pb,
                                                      double* __restrict__ pc, BicgState b) {
  const int c = tile_of(tl);
  const int inst = tl.inst[c];
  if (b.status[inst] != ST_RUN) return;
  double tv[2];
  tile_reduce<2, TNT>(tl, inst, pb, 0u, tv);
  if (!finite(tv[0]) || !finite(tv[1])) {
    if (threadIdx.x == 0) bicg_stop(tl, c, inst, b, ST_NONFINITE, j, tv[0]);
    return;
  }
  const double omega = (tv[1] == 0.0) ? 0.0 : tv[0] / tv[1];
  if (threadIdx.x == 0 && c == tl.inst_t0[inst]) b.omega[inst] = omega;
  const T a = (T)b.alpha[inst], w = (T)omega;
  const int r0 = tl.row0[c], nr = tl.nrows[c];
  double acc[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < nr; i += TNT) {
    const int row = r0 + i;
    const T si = s[row];
    x[row] = x[row] + a * p[row] + w * si;
    const T ri = si - w * t[row];
    r[row] = ri;
    acc[0] += (double)q[row] * (double)ri;
    acc[1] = mx(acc[1], fabs((double)ri));
  }
  block_reduce<2, TNT>(acc, 2u);
  if (threadIdx.x == 0) { pc[2 * c] = acc[0]; pc[2 * c + 1] = acc[1]; }
}

// stopping test after the last step of a batch (j completed steps)
__global__ void k_bicg_check(Tiles tl, int64_t j, const double* __restrict__ pc, const double* __restrict__ ps,
                             BicgState b) {
  const int k = blockIdx.x;
  if (b.status[k] != ST_RUN) return;
  double beta;
  bicg_decide<BS>(tl, tl.inst_t0[k], k, j, pc, ps, b, beta);
}

template <typename K>
static hipError_t set_lds(K kern, size_t lds, size_t& configured) {
  if (lds <= configured) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) configured = lds;
  return e;
}

template <typename T>
hipError_t launch_bicg_tile_init(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x, int x_is_zero, T* r,
                                 T* q, T* p, T* v, Tiles tl, const int32_t* status, double* pc) {
  const size_t lds = x_is_zero ? 0 : (size_t)tl.maxw * sizeof(T);
  const unsigned g = (unsigned)tl.ntile;
  static size_t conf[7] = {0, 0, 0, 0, 0, 0, 0};
  hipError_t e = hipSuccess;
#define RP_INIT_CASE(LL, IDX)                                                                          \
  case LL:                                                                                             \
    e = set_lds(k_bicg_init_tile<T, LL>, (size_t)tl.maxw * sizeof(T), conf[IDX]);                     \
    if (e != hipSuccess) return e;                                                                     \
    k_bicg_init_tile<T, LL><<<g, TNT, lds, st>>>(m, rhs, x, x_is_zero, r, q, p, v, tl, status, pc);     \
    break;
  switch (L) {
    RP_INIT_CASE(1, 0) RP_INIT_CASE(2, 1) RP_INIT_CASE(4, 2) RP_INIT_CASE(8, 3) RP_INIT_CASE(16, 4)
    RP_INIT_CASE(32, 5) RP_INIT_CASE(64, 6)
    default: return hipErrorInvalidValue;
  }
#undef RP_INIT_CASE
  return hipGetLastError();
}

// r = b - M x in FP64 with x staged in LDS; partial max|r| per tile
template <int L, int KIND>
__device__ __forceinline__ double residual_rows(const MatView<double>& m, const double* __restrict__ b,
                                                const double* __restrict__ xs, const double* __restrict__ x,
                                                double* __restrict__ r, int r0, int nr, int w0, int nw) {
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = TNT / L;
  double mloc = 0.0;
  for (int base = 0; base < nr; base += RPP) {
    const bool ok = base + g < nr;
    const int row = r0 + base + g;
    double acc = 0.0;
    if (ok) {
      const int k1 = m.rp[row + 1];
      for (int k = m.rp[row] + lane; k < k1; k += L) acc += m.val[k] * xget<KIND>(xs, x, colrel<KIND>(m, k, w0), nw, w0);
    }
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
    if (ok && lane == 0) {
      const double y = m.d[row] * xget<KIND>(xs, x, row - w0, nw, w0) - acc;
      const double ri = b[row] - y;
      r[row] = ri;
      mloc = mx(mloc, fabs(ri));
    }
  }
  return mloc;
}

template <int L>
__global__ __launch_bounds__(TNT) void k_residual_tile(MatView<double> m, const double* __restrict__ b,
                                                       const double* __restrict__ x, double* __restrict__ r, Tiles tl,
                                                       const int32_t* __restrict__ status,
                                                       double* __restrict__ part) {
  extern __shared__ unsigned char smem_raw[];
  double* xs = reinterpret_cast<double*>(smem_raw);
  const int c = tile_of(tl);
  if (status[tl.inst[c]] != ST_RUN) return;
  const int r0 = tl.row0[c], nr = tl.nrows[c], w0 = tl.w0[c], nw = tl.nw[c], kind = tl.kind[c];
  if (kind != WIN_NONE) {
    stage_window<double, TNT>(xs, x, w0, nw);
    __syncthreads();
  }
  double mloc;
  if (kind == WIN_WHOLE) mloc = residual_rows<L, WIN_WHOLE>(m, b, xs, x, r, r0, nr, w0, nw);
  else if (kind == WIN_BAND) mloc = residual_rows<L, WIN_BAND>(m, b, xs, x, r, r0, nr, w0, nw);
  else mloc = residual_rows<L, WIN_NONE>(m, b, xs, x, r, r0, nr, w0, nw);
  double v[1] = {mloc};
  block_reduce<1, TNT>(v, 1u);
  if (threadIdx.x == 0) part[c] = v[0];
}

template <int L>
static hipError_t residual_tile_L(hipStream_t st, MatView<double> m, const double* b, const double* x, double* r,
                                  Tiles tl, const int32_t* status, double* part) {
  const size_t lds = (size_t)tl.maxw * sizeof(double);
  static size_t conf = 0;
  hipError_t e = set_lds(k_residual_tile<L>, lds, conf);
  if (e != hipSuccess) return e;
  k_residual_tile<L><<<(unsigned)tl.ntile, TNT, lds, st>>>(m, b, x, r, tl, status, part);
  return hipGetLastError();
}
hipError_t launch_residual_tile(hipStream_t st, int L, MatView<double> m, const double* b, const double* x, double* r,
                                Tiles tl, const int32_t* status, double* part) {
  switch (L) {
    case 1: return residual_tile_L<1>(st, m, b, x, r, tl, status, part);
    case 2: return residual_tile_L<2>(st, m, b, x, r, tl, status, part);
    case 4: return residual_tile_L<4>(st, m, b, x, r, tl, status, part);
    case 8: return residual_tile_L<8>(st, m, b, x, r, tl, status, part);
    case 16: return residual_tile_L<16>(st, m, b, x, r, tl, status, part);
    case 32: return residual_tile_L<32>(st, m, b, x, r, tl, status, part);
    case 64: return residual_tile_L<64>(st, m, b, x, r, tl, status, part);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int L, int MODE>
static hipError_t spmv_tile_L(hipStream_t st, MatView<T> m, const T* u, T* y, const T* q, Tiles tl,
                              const int32_t* status, double* part) {
  const size_t lds = (size_t)tl.maxw * sizeof(T);
  static size_t conf = 0;
  hipError_t e = set_lds(k_spmv_tile<T, L, MODE>, lds, conf);
  if (e != hipSuccess) return e;
  k_spmv_tile<T, L, MODE><<<(unsigned)tl.ntile, TNT, lds, st>>>(m, u, y, q, tl, status, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv_tile(hipStream_t st, int L, int mode, MatView<T> m, const T* u, T* y, const T* q, Tiles tl,
                            const int32_t* status, double* part) {
#define RP_SPMV_CASE(LL)                                                                     \
  case LL:                                                                                   \
    return mode ? spmv_tile_L<T, LL, 1>(st, m, u, y, q, tl, status, part)                    \
                : spmv_tile_L<T, LL, 0>(st, m, u, y, q, tl, status, part);
  switch (L) {
    RP_SPMV_CASE(1) RP_SPMV_CASE(2) RP_SPMV_CASE(4) RP_SPMV_CASE(8) RP_SPMV_CASE(16) RP_SPMV_CASE(32) RP_SPMV_CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef RP_SPMV_CASE
}

template <typename T>
hipError_t launch_bicg_p_tile(hipStream_t st, const T* r, T* p, const T* v, Tiles tl, int64_t j, const double* pc,
                              const double* ps, BicgState b) {
  k_bicg_p_tile<T><<<(unsigned)tl.ntile, TNT, 0, st>>>(r, p, v, tl, j, pc, ps, b);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_bicg_s_tile(hipStream_t st, const T* r, const T* v, T* s, Tiles tl, int64_t j, const double* pa,
                              double* ps, BicgState b) {
  k_bicg_s_tile<T><<<(unsigned)tl.ntile, TNT, 0, st>>>(r, v, s, tl, j, pa, ps, b);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_bicg_xr_tile(hipStream_t st, T* x, const T* p, const T* s, T* r, const T* t, const T* q, Tiles tl,
                               int64_t j, const double* pb, double* pc, BicgState b) {
  k_bicg_xr_tile<T><<<(unsigned)tl.ntile, TNT, 0, st>>>(x, p, s, r, t, q, tl, j, pb, pc, b);
  return hipGetLastError();
}
hipError_t launch_bicg_check(hipStream_t st, Tiles tl, int64_t j, const double* pc, const double* ps, BicgState b) {
  k_bicg_check<<<(unsigned)tl.K, BS, 0, st>>>(tl, j, pc, ps, b);
  return hipGetLastError();
}

#define RP_BICG_TILE_INST(T)                                                                                         \
  template hipError_t launch_bicg_tile_init<T>(hipStream_t, int, MatView<T>, const T*, const T*, int, T*, T*, T*, T*, \
                                               Tiles, const int32_t*, double*);                                      \
  template hipError_t launch_spmv_tile<T>(hipStream_t, int, int, MatView<T>, const T*, T*, const T*, Tiles,           \
                                          const int32_t*, double*);                                                  \
  template hipError_t launch_bicg_p_tile<T>(hipStream_t, const T*, T*, const T*, Tiles, int64_t, const double*,       \
                                            const double*, BicgState);                                               \
  template hipError_t launch_bicg_s_tile<T>(hipStream_t, const T*, const T*, T*, Tiles, int64_t, const double*,       \
                                            double*, BicgState);                                                     \
  template hipError_t launch_bicg_xr_tile<T>(hipStream_t, T*, const T*, const T*, T*, const T*, const T*, Tiles,      \
                                             int64_t, const double*, double*, BicgState);
RP_BICG_TILE_INST(double)
RP_BICG_TILE_INST(float)
#undef RP_BICG_TILE_INST

// ============================================================================
// Sliced rows.  In the tile layout above a row is summed by a group of L
// lanes, so a wavefront issues a load slot per lane whether or not the row
// has an entry there.  Here a tile's rows are sorted by decreasing entry
// count within windows of a few hundred to a few thousand rows (ties in row
// order) and cut into slices of 64 rows, one row per lane;
// entry j of every lane of a slice sits in one contiguous 64-wide run, so each
// load instruction of a wavefront reads consecutive addresses and the slice
// width (its longest row) sets the padding.  A row is still summed by one
// lane in its CSR order, and the stopping measure and dot products use the
// same per-row formulas as the lane-group kernels.
// ============================================================================

constexpr int SKEYS = 256;  // sort keys: rows of SKEYS-1 or more entries share the last one

// Per tile (one block each): the order of its rows (row[s*64 + lane] for
// its slices, -1 past the last row) and the width of each slice.  Rows are
// sorted by decreasing length within consecutive windows of `window` rows (a
// multiple of SLICE), not across the whole tile: the rows of one cache line
// of x' (and of the right-hand side) then fall into slices that are swept at
// about the same time, so the line is completed in L2 before it is written
// back (sorting whole tiles of ~5,000 rows doubled the written bytes).
__global__ __launch_bounds__(TNT) void k_slice_order(const int32_t* __restrict__ rp, Tiles tl,
                                                     const int32_t* __restrict__ t_s0, int32_t window,
                                                     int32_t* __restrict__ row, int32_t* __restrict__ width) {
  __shared__ int32_t hist[SKEYS], start[SKEYS];
  const int c = blockIdx.x;
  const int r0 = tl.row0[c], nr = tl.nrows[c];
  const int s0 = t_s0[c], ns = t_s0[c + 1] - s0;
  int32_t* __restrict__ out = row + (size_t)s0 * SLICE;
  auto key = [&](int r) { return SKEYS - 1 - min(rp[r + 1] - rp[r], SKEYS - 1); };
  for (int p = nr + threadIdx.x; p < ns * SLICE; p += TNT) out[p] = -1;
  for (int q0 = 0; q0 < nr; q0 += window) {
    const int qn = min(window, nr - q0), rq = r0 + q0;
    for (int i = threadIdx.x; i < SKEYS; i += TNT) hist[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < qn; i += TNT) atomicAdd(&hist[key(rq + i)], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = q0;
      for (int k = 0; k < SKEYS; k++) {
        start[k] = acc;
        acc += hist[k];
      }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // One wavefront places the rows 64 at a time in row order (stable):
      // lanes with equal keys are ranked by lane, hist[k] counts the rows of
      // key k placed so far.
      const int lane = threadIdx.x;
      for (int k = lane; k < SKEYS; k += 64) hist[k] = 0;
      const unsigned long long below = (1ull << lane) - 1ull;
      for (int b = 0; b < qn; b += 64) {
        const int i = b + lane;
        const bool ok = i < qn;
        const int k = ok ? key(rq + i) : 0;
        unsigned long long same = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
          const unsigned long long set = __ballot((k >> bit) & 1);
          same &= ((k >> bit) & 1) ? set : ~set;
        }
        if (ok) {
          const int rank = __popcll(same & below), cnt = __popcll(same);
          const int base = hist[k];
          out[start[k] + base + rank] = rq + i;
          if (rank == cnt - 1) hist[k] = base + cnt;
        }
      }
    }
    __syncthreads();
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int s = wave; s < ns; s += TNT / 64) {
    const int r = out[s * SLICE + lane];
    int len = r >= 0 ? rp[r + 1] - rp[r] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
    if (lane == 0) width[s0 + s] = len;
  }
}
hipError_t launch_slice_order(hipStream_t st, const int32_t* rp, Tiles tl, const int32_t* t_s0, int32_t window,
                              int32_t* row, int32_t* width) {
  if (tl.ntile <= 0) return hipSuccess;
  if (window < SLICE || window % SLICE != 0) return hipErrorInvalidValue;
  k_slice_order<<<(unsigned)tl.ntile, TNT, 0, st>>>(rp, tl, t_s0, window, row, width);
  return hipGetLastError();
}

// One wavefront per slice: copy each lane's row into the slice (value 0 and
// column 0 past the row's end) and its diagonal entry (1 where no row).
template <typename T>
__global__ __launch_bounds__(BS) void k_slice_fill(MatView<T> m, Tiles tl, const int32_t* __restrict__ stile,
                                                   int32_t nslice, const int32_t* __restrict__ off,
                                                   const int32_t* __restrict__ width, const int32_t* __restrict__ row,
                                                   T* __restrict__ d, T* __restrict__ val, uint16_t* __restrict__ c16,
                                                   int32_t* __restrict__ c32) {
  const int s = blockIdx.x * (BS / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s >= nslice) return;
  const int t = stile[s];
  const int w0 = tl.w0[t];
  const bool whole = tl.kind[t] == WIN_WHOLE;
  const int r = row[(size_t)s * SLICE + lane];
  int k0 = 0, len = 0;
  T dr = (T)1;
  if (r >= 0) {
    k0 = m.rp[r];
    len = m.rp[r + 1] - k0;
    dr = m.d[r];
  }
  d[(size_t)s * SLICE + lane] = dr;
  const int W = width[s];
  const size_t o = (size_t)off[s] + lane;
  for (int j = 0; j < W; j++) {
    const size_t slot = o + (size_t)j * SLICE;
    T v = (T)0;
    int cr = 0;
    if (j < len) {
      v = m.val[k0 + j];
      cr = whole ? (int)m.c16[k0 + j] : m.col[k0 + j] - w0;
    }
    val[slot] = v;
    if (whole) c16[slot] = (uint16_t)cr;
    else c32[slot] = cr;
  }
}
template <typename T>
hipError_t launch_slice_fill(hipStream_t st, MatView<T> m, Tiles tl, const int32_t* stile, int32_t nslice,
                             const int32_t* off, const int32_t* width, const int32_t* row, T* d, T* val,
                             uint16_t* c16, int32_t* c32) {
  if (nslice <= 0) return hipSuccess;
  const unsigned g = (unsigned)((nslice + BS / 64 - 1) / (BS / 64));
  k_slice_fill<T><<<g, BS, 0, st>>>(m, tl, stile, nslice, off, width, row, d, val, c16, c32);
  return hipGetLastError();
}
template hipError_t launch_slice_fill<double>(hipStream_t, MatView<double>, Tiles, const int32_t*, int32_t,
                                              const int32_t*, const int32_t*, const int32_t*, double*, double*,
                                              uint16_t*, int32_t*);
template hipError_t launch_slice_fill<float>(hipStream_t, MatView<float>, Tiles, const int32_t*, int32_t,
                                             const int32_t*, const int32_t*, const int32_t*, float*, float*,
                                             uint16_t*, int32_t*);

// NS slices per wavefront at a time (independent sums), their entries loaded
// U per slice before any is used; the slice bounds are wavefront-uniform, so
// the guards are scalar branches and padding past a slice's width is never
// read.
// ---- column panels of the sliced rows ---------------------------------------
// Lane mask of the lanes below this one.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Exclusive prefix sum over the wavefront's lanes of a small count c (0..255)
// and the wavefront's total, one ballot per bit of c (four bits while every
// count is below 16).  Wave-uniform control flow.
__device__ __forceinline__ int lane_prefix(int c, int& total) {
  const int nb = __ballot(c >= 16) ? 8 : 4;
  int pre = 0;
  total = 0;
#pragma unroll
  for (int b = 0; b < 8; b++) {
    if (b < nb) {
      const unsigned long long m = __ballot((c >> b) & 1);
      pre += lanes_below(m) << b;
      total += __popcll(m) << b;
    }
  }
  return pre;
}

// One wavefront per paneled slice: per panel, each lane's count of entries
// (a count byte) and, per slice, the number of entries over all panels.
template <typename T>
__global__ __launch_bounds__(BS) void k_panel_count(MatView<T> m, Tiles tl, Sliced<T> sl,
                                                    const int32_t* __restrict__ pslice,
                                                    const int32_t* __restrict__ ptile, int32_t np,
                                                    uint8_t* __restrict__ cnt, int32_t* __restrict__ entries) {
  const int i = blockIdx.x * (BS / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= np) return;
  const int s = pslice[i], t = ptile[i];
  const int P = sl.npan[t];
  const int w0 = tl.w0[t];
  uint8_t* __restrict__ h = cnt + sl.hoff[t] + (size_t)(s - sl.t_s0[t]) * P * SLICE;
  const int r = sl.row[(size_t)s * SLICE + lane];
  int k = 0, k1 = 0;
  if (r >= 0) {
    k = m.rp[r];
    k1 = m.rp[r + 1];
  }
  int sum = k1 - k;
  for (int p = 0; p < P; p++) {
    const int end = w0 + (p + 1) * sl.pw;
    const int kp = k;
    while (k < k1 && m.col[k] < end) k++;
    h[p * SLICE + lane] = (uint8_t)(k - kp);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) entries[i] = sum;
}
template <typename T>
hipError_t launch_panel_count(hipStream_t st, MatView<T> m, Tiles tl, Sliced<T> sl, const int32_t* pslice,
                              const int32_t* ptile, int32_t npslice, uint8_t* cnt, int32_t* entries) {
  if (npslice <= 0) return hipSuccess;
  const unsigned g = (unsigned)((npslice + BS / 64 - 1) / (BS / 64));
  k_panel_count<T><<<g, BS, 0, st>>>(m, tl, sl, pslice, ptile, npslice, cnt, entries);
  return hipGetLastError();
}

// One wavefront per paneled slice: its entries, panel after panel, lane
// after lane within a panel (sl.pent laid out from the counts above).
template <typename T>
__global__ __launch_bounds__(BS) void k_panel_fill(MatView<T> m, Tiles tl, Sliced<T> sl,
                                                   const int32_t* __restrict__ pslice,
                                                   const int32_t* __restrict__ ptile, int32_t np, T* __restrict__ val,
                                                   uint16_t* __restrict__ c16) {
  const int i = blockIdx.x * (BS / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= np) return;
  const int s = pslice[i], t = ptile[i];
  const int P = sl.npan[t];
  const int w0 = tl.w0[t];
  const uint8_t* __restrict__ h = sl.cnt + sl.hoff[t] + (size_t)(s - sl.t_s0[t]) * P * SLICE;
  const int r = sl.row[(size_t)s * SLICE + lane];
  int k = r >= 0 ? m.rp[r] : 0;
  int e = sl.pent[s];
  for (int p = 0; p < P; p++) {
    const int start = w0 + p * sl.pw;
    const int c = h[p * SLICE + lane];
    int tot;
    const int pos = e + lane_prefix(c, tot);
    for (int j = 0; j < c; j++) {
      val[pos + j] = m.val[k + j];
      c16[pos + j] = (uint16_t)(m.col[k + j] - start);
    }
    k += c;
    e += tot;
  }
}
template <typename T>
hipError_t launch_panel_fill(hipStream_t st, MatView<T> m, Tiles tl, Sliced<T> sl, const int32_t* pslice,
                             const int32_t* ptile, int32_t npslice, T* val, uint16_t* c16) {
  if (npslice <= 0) return hipSuccess;
  const unsigned g = (unsigned)((npslice + BS / 64 - 1) / (BS / 64));
  k_panel_fill<T><<<g, BS, 0, st>>>(m, tl, sl, pslice, ptile, npslice, val, c16);
  return hipGetLastError();
}
#define RP_PANEL_INST(T)                                                                                             \
  template hipError_t launch_panel_count<T>(hipStream_t, MatView<T>, Tiles, Sliced<T>, const int32_t*,              \
                                            const int32_t*, int32_t, uint8_t*, int32_t*);                           \
  template hipError_t launch_panel_fill<T>(hipStream_t, MatView<T>, Tiles, Sliced<T>, const int32_t*,               \
                                           const int32_t*, int32_t, T*, uint16_t*);
RP_PANEL_INST(double)
RP_PANEL_INST(float)
#undef RP_PANEL_INST

// Row sums over all panels of a paneled tile: acc[q] for the slice
// sb + wave + 16 q (q < PanelShape<T>::MAXS).  Panel by panel the block
// stages the panel's piece of the iterate u into LDS; every wavefront then
// takes its slices QG at a time: the count bytes of the next group are
// loaded before the current group's entries are used, each lane finds its
// entries from a ballot prefix sum of the counts, and the first two entries
// of every lane of the group are loaded before any is used (further entries,
// rare with a few entries per row and panel, one at a time).  Each lane adds
// its row's entries in column order.
template <typename T, int MAXS = PanelShape<T>::MAXS>
__device__ __forceinline__ void panel_sums(const Sliced<T>& sl, T* __restrict__ us, const T* __restrict__ u, int c,
                                           int sb, int se, int w0, T (&acc)[MAXS]) {
  constexpr int NW = TNT / 64, QG = 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int P = sl.npan[c], ns = se - sb, rows = sl.pend[c] - w0;
  const uint8_t* __restrict__ hc = sl.cnt + sl.hoff[c];
  int base[MAXS];
#pragma unroll
  for (int q = 0; q < MAXS; q++) {
    const int sr = wave + NW * q;
    base[q] = sr < ns ? sl.pent[sb + sr] : 0;
    acc[q] = (T)0;
  }
  for (int p = 0; p < P; p++) {
    const int p0 = p * sl.pw, pn = min(sl.pw, rows - p0);
    if (p > 0) __syncthreads();  // every wavefront is done with the previous panel
    stage_window<T, TNT>(us, u, w0 + p0, pn);
    int cn[QG];
#pragma unroll
    for (int i = 0; i < QG; i++) {
      const int sr = wave + NW * i;
      cn[i] = sr < ns ? hc[((size_t)sr * P + p) * SLICE + lane] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int q0 = 0; q0 < MAXS; q0 += QG) {
      if (wave + NW * q0 >= ns) break;
      int nx[QG];
#pragma unroll
      for (int i = 0; i < QG; i++) {
        const int sr = wave + NW * (q0 + QG + i);
        nx[i] = (q0 + QG < MAXS && sr < ns) ? hc[((size_t)sr * P + p) * SLICE + lane] : 0;
      }
      int pos[QG];
#pragma unroll
      for (int i = 0; i < QG; i++) {
        int tot;
        pos[i] = base[q0 + i] + lane_prefix(cn[i], tot);
        base[q0 + i] += tot;
      }
      // unconditional loads (the arrays carry PANEL_SLACK spare entries past
      // the last one and a count is at most 255, so pos + j is always
      // inside): no branch on the lane mask between the loads, which lets
      // them all be in flight together; the select keeps the sum unchanged
      // where the entry is not the lane's own
      T v[QG][2];
      int cc[QG][2];
#pragma unroll
      for (int i = 0; i < QG; i++)
#pragma unroll
        for (int l = 0; l < 2; l++) {
          v[i][l] = sl.val[pos[i] + l];
          cc[i][l] = sl.c16[pos[i] + l];
        }
#pragma unroll
      for (int i = 0; i < QG; i++)
#pragma unroll
        for (int l = 0; l < 2; l++) {
          const T f = acc[q0 + i] + v[i][l] * us[cc[i][l]];  // one fused multiply-add, as elsewhere
          acc[q0 + i] = l < cn[i] ? f : acc[q0 + i];
        }
      int most = 0;
#pragma unroll
      for (int i = 0; i < QG; i++) most = max(most, cn[i]);
      for (int j = 2; __ballot(j < most); j++) {
        T vj[QG];
        int cj[QG];
#pragma unroll
        for (int i = 0; i < QG; i++) {
          vj[i] = sl.val[pos[i] + j];
          cj[i] = sl.c16[pos[i] + j];
        }
#pragma unroll
        for (int i = 0; i < QG; i++) {
          const T f = acc[q0 + i] + vj[i] * us[cj[i]];
          acc[q0 + i] = j < cn[i] ? f : acc[q0 + i];
        }
      }
#pragma unroll
      for (int i = 0; i < QG; i++) cn[i] = nx[i];
    }
  }
}

// Jacobi update of a paneled tile's rows (as jacobi_sliced_rows).
template <typename T>
__device__ __forceinline__ double jacobi_panel_rows(const Sliced<T>& sl, const T* __restrict__ rhs, T* __restrict__ xs,
                                                    const T* __restrict__ x, T* __restrict__ xn, int c, int sb, int se,
                                                    int w0, int weighted) {
  constexpr int NW = TNT / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int MAXS = PanelShape<T>::MAXS;
  T acc[MAXS];
  panel_sums<T>(sl, xs, x, c, sb, se, w0, acc);
  double mloc = 0.0;
#pragma unroll
  for (int q = 0; q < MAXS; q++) {
    const int s = sb + wave + NW * q;
    if (s >= se) break;
    const int row = sl.row[(size_t)s * SLICE + lane];
    if (row >= 0) {
      const T d = sl.d[(size_t)s * SLICE + lane];
      const T b = rhs ? rhs[row] : (T)0;
      const T nv = (b + acc[q]) / d;
      const double dl = fabs((double)nv - (double)x[row]);
      xn[row] = nv;
      mloc = mx(mloc, weighted ? (double)d * dl : dl);
    }
  }
  return mloc;
}

// Sparse product of a paneled tile's rows (as spmv_sliced_rows).
template <typename T, int MODE>
__device__ __forceinline__ void spmv_panel_rows(const Sliced<T>& sl, T* __restrict__ us, const T* __restrict__ u,
                                                T* __restrict__ y, const T* __restrict__ qv, int c, int sb, int se,
                                                int w0, double* a) {
  constexpr int NW = TNT / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int MAXS = PanelShape<T>::MAXS;
  T acc[MAXS];
  panel_sums<T>(sl, us, u, c, sb, se, w0, acc);
#pragma unroll
  for (int q = 0; q < MAXS; q++) {
    const int s = sb + wave + NW * q;
    if (s >= se) break;
    const int row = sl.row[(size_t)s * SLICE + lane];
    if (row >= 0) {
      const T ui = u[row];
      const T yi = sl.d[(size_t)s * SLICE + lane] * ui - acc[q];
      if (MODE == 2) {
        const T ri = qv[row] - yi;
        y[row] = ri;
        a[0] = mx(a[0], fabs((double)ri));
      } else if (MODE == 0) {
        y[row] = yi;
        a[0] += (double)qv[row] * (double)yi;
      } else {
        y[row] = yi;
        a[0] += (double)yi * (double)ui;
        a[1] += (double)yi * (double)yi;
      }
    }
  }
}

template <typename T, int U, int NS>
struct SliceGroup {
  int off[NS], W[NS], row[NS], Wm;
  T d[NS];
  T vv[NS][U];
  int cc[NS][U];

  __device__ __forceinline__ void setup(const Sliced<T>& sl, int s0, int se, int lane) {
    constexpr int NW = TNT / 64;
    Wm = 0;
#pragma unroll
    for (int q = 0; q < NS; q++) {
      const int s = s0 + q * NW;
      const bool ok = s < se;
      off[q] = ok ? sl.off[s] : 0;
      W[q] = ok ? sl.width[s] : 0;
      row[q] = ok ? sl.row[(size_t)s * SLICE + lane] : -1;
      d[q] = ok ? sl.d[(size_t)s * SLICE + lane] : (T)1;
      Wm = max(Wm, W[q]);
    }
  }
  template <int KIND, bool NT>
  __device__ __forceinline__ void chunk(const Sliced<T>& sl, int j, int lane) {
#pragma unroll
    for (int q = 0; q < NS; q++)
#pragma unroll
      for (int u = 0; u < U; u++) {
        vv[q][u] = 0;
        cc[q][u] = 0;
        if (j + u < W[q]) {
          const size_t k = (size_t)off[q] + (size_t)(j + u) * SLICE + lane;
          if (NT) {
            vv[q][u] = __builtin_nontemporal_load(sl.val + k);
            cc[q][u] = KIND == WIN_WHOLE ? (int)__builtin_nontemporal_load(sl.c16 + k)
                                         : __builtin_nontemporal_load(sl.c32 + k);
          } else {
            vv[q][u] = sl.val[k];
            cc[q][u] = KIND == WIN_WHOLE ? (int)sl.c16[k] : sl.c32[k];
          }
        }
      }
  }
};

template <typename T>
struct SliceShape;
template <>
struct SliceShape<double> {  // one 1024-thread block per CU: registers to spare
  static constexpr int U = 4, NS = 4;
};
template <>
struct SliceShape<float> {  // two blocks per CU: at most 64 VGPRs
  static constexpr int U = 8, NS = 1;
};

template <typename T, int KIND, bool NT>
__device__ __forceinline__ double jacobi_sliced_rows(const Sliced<T>& sl, const T* __restrict__ rhs,
                                                     const T* __restrict__ xs, const T* __restrict__ x,
                                                     T* __restrict__ xn, int sb, int se, int w0, int nw, int weighted) {
  constexpr int U = SliceShape<T>::U, NS = SliceShape<T>::NS, NW = TNT / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  double mloc = 0.0;
  for (int s0 = sb + wave; s0 < se; s0 += NW * NS) {
    SliceGroup<T, U, NS> g;
    g.setup(sl, s0, se, lane);
    T b[NS], acc[NS];
#pragma unroll
    for (int q = 0; q < NS; q++) {
      b[q] = (rhs && g.row[q] >= 0) ? rhs[g.row[q]] : (T)0;
      acc[q] = 0;
    }
    for (int j = 0; j < g.Wm; j += U) {
      g.template chunk<KIND, NT>(sl, j, lane);
#pragma unroll
      for (int q = 0; q < NS; q++)
#pragma unroll
        for (int u = 0; u < U; u++) acc[q] += g.vv[q][u] * xget<KIND>(xs, x, g.cc[q][u], nw, w0);
    }
#pragma unroll
    for (int q = 0; q < NS; q++) {
      const int row = g.row[q];
      if (row >= 0) {
        const T nv = (b[q] + acc[q]) / g.d[q];
        const double dl = fabs((double)nv - (double)xget<KIND>(xs, x, row - w0, nw, w0));
        xn[row] = nv;
        mloc = mx(mloc, weighted ? (double)g.d[q] * dl : dl);
      }
    }
  }
  return mloc;
}

template <typename T, bool NT, bool PANEL>
__global__ __launch_bounds__(TNT) void k_jacobi_sliced(Sliced<T> sl, const T* __restrict__ rhs,
                                                       const T* __restrict__ x, T* __restrict__ xn, Tiles tl, int64_t s_rel,
                                                       const double* __restrict__ pprev, double* __restrict__ pcur,
                                                       int32_t* status, int64_t* iters, double* meas,
                                                       const double* __restrict__ thr, int strict, int64_t max_iter,
                                                       int32_t* ndone, int weighted) {
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int c = tile_of(tl);
  const int inst = tl.inst[c];
  const int w0 = tl.w0[c], nw = tl.nw[c], kind = tl.kind[c];
  const int sb = sl.t_s0[c], se = sl.t_s0[c + 1];
  if (status[inst] != ST_RUN) return;
  const int64_t s = s_rel + (tl.sbase ? *tl.sbase : 0);
  if (!jacobi_begin<T>(xs, x, tl, c, inst, kind, w0, nw, s, pprev, status, iters, meas, thr, strict, max_iter, ndone))
    return;
  double mloc;
  if (PANEL && sl.npan[c] > 0) mloc = jacobi_panel_rows<T>(sl, rhs, xs, x, xn, c, sb, se, w0, weighted);
  else if (kind == WIN_WHOLE) mloc = jacobi_sliced_rows<T, WIN_WHOLE, NT>(sl, rhs, xs, x, xn, sb, se, w0, nw, weighted);
  else if (kind == WIN_BAND) mloc = jacobi_sliced_rows<T, WIN_BAND, NT>(sl, rhs, xs, x, xn, sb, se, w0, nw, weighted);
  else mloc = jacobi_sliced_rows<T, WIN_NONE, NT>(sl, rhs, xs, x, xn, sb, se, w0, nw, weighted);
  double v[1] = {mloc};
  block_reduce<1, TNT>(v, 1u);
  if (threadIdx.x == 0) pcur[c] = v[0];
}

template <typename T>
hipError_t launch_jacobi_sliced(hipStream_t st, Sliced<T> sl, const T* rhs, const T* x, T* xn, Tiles tl, int64_t s,
                                const double* pprev, double* pcur, int32_t* status, int64_t* iters, double* meas,
                                const double* thr, int strict, int64_t max_iter, int32_t* ndone, int weighted) {
  const size_t lds = (size_t)max(tl.maxw, sl.paneled ? sl.pw : 0) * sizeof(T);
  static size_t conf[4] = {0, 0, 0, 0};
  const int v = (sl.stream ? 1 : 0) + (sl.paneled ? 2 : 0);
  const auto kern = v == 0 ? k_jacobi_sliced<T, false, false> : v == 1 ? k_jacobi_sliced<T, true, false>
                  : v == 2 ? k_jacobi_sliced<T, false, true> : k_jacobi_sliced<T, true, true>;
  hipError_t e = set_lds(kern, lds, conf[v]);
  if (e != hipSuccess) return e;
  kern<<<(unsigned)tl.ntile, TNT, lds, st>>>(sl, rhs, x, xn, tl, s, pprev, pcur, status, iters, meas, thr, strict,
                                             max_iter, ndone, weighted);
  return hipGetLastError();
}
template hipError_t launch_jacobi_sliced<double>(hipStream_t, Sliced<double>, const double*, const double*, double*,
                                                 Tiles, int64_t, const double*, double*, int32_t*, int64_t*, double*,
                                                 const double*, int, int64_t, int32_t*, int);
template hipError_t launch_jacobi_sliced<float>(hipStream_t, Sliced<float>, const float*, const float*, float*, Tiles,
                                                int64_t, const double*, double*, int32_t*, int64_t*, double*,
                                                const double*, int, int64_t, int32_t*, int);

// Resident sweeps on sliced rows (the tail of a tiled solve on sliced rows,
// every tile of the instance with a whole-block window): as
// k_jacobi_resident -- both iterates of the instance in LDS, many sweeps per
// launch, the decision after each -- but the wavefronts take the instance's
// slices [s_lo, s_hi) as the sliced sweep does, so every row sum is the
// sliced sweep's bit for bit, and U x NS entries of different slices are in
// flight where one lane per row would wait on a long row's entries one
// after another.
template <typename T>
__device__ __forceinline__ double resident_sliced_rows(const Sliced<T>& sl, const T* __restrict__ rhs,
                                                       const T* cur, T* nxt, int sb, int se, int r0,
                                                       int weighted) {
  constexpr int U = SliceShape<T>::U, NS = SliceShape<T>::NS, NW = TNT / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  double mloc = 0.0;
  for (int s0 = sb + wave; s0 < se; s0 += NW * NS) {
    SliceGroup<T, U, NS> g;
    g.setup(sl, s0, se, lane);
    T b[NS], acc[NS];
#pragma unroll
    for (int q = 0; q < NS; q++) {
      b[q] = (rhs && g.row[q] >= 0) ? rhs[g.row[q]] : (T)0;
      acc[q] = 0;
    }
    for (int j = 0; j < g.Wm; j += U) {
      g.template chunk<WIN_WHOLE, false>(sl, j, lane);
#pragma unroll
      for (int q = 0; q < NS; q++)
#pragma unroll
        for (int u = 0; u < U; u++) acc[q] += g.vv[q][u] * cur[g.cc[q][u]];
    }
#pragma unroll
    for (int q = 0; q < NS; q++) {
      const int row = g.row[q];
      if (row >= 0) {
        const T nv = (b[q] + acc[q]) / g.d[q];
        const double dl = fabs((double)nv - (double)cur[row - r0]);
        nxt[row - r0] = nv;
        mloc = mx(mloc, weighted ? (double)g.d[q] * dl : dl);
      }
    }
  }
  return mloc;
}

template <typename T>
__global__ __launch_bounds__(TNT) void k_jacobi_resident_sliced(Sliced<T> sl, const T* __restrict__ rhs, T* xa, T* xb,
                                                                Tiles tl, const int32_t* __restrict__ s_lo,
                                                                const int32_t* __restrict__ s_hi, int64_t s0,
                                                                int nsweeps, int32_t* status, int64_t* iters,
                                                                double* meas, const double* __restrict__ thr,
                                                                int strict, int64_t max_iter, int32_t* ndone,
                                                                int weighted) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ int32_t decision;
  const int c = blockIdx.x;
  const int inst = tl.inst[c];
  if (status[inst] != ST_RUN) return;
  const int r0 = tl.row0[c], nr = tl.nrows[c];  // the instance block
  const int sb = s_lo[c], se = s_hi[c];
  T* X0 = reinterpret_cast<T*>(smem_raw);
  T* X1 = X0 + tl.maxw;
  stage_window<T, TNT>(X0, (s0 & 1) ? xb : xa, r0, nr);
  __syncthreads();
  for (int it = 0; it < nsweeps; it++) {
    const T* cur = (it & 1) ? X1 : X0;
    T* nxt = (it & 1) ? X0 : X1;
    double v[1] = {resident_sliced_rows<T>(sl, rhs, cur, nxt, sb, se, r0, weighted)};
    block_reduce<1, TNT>(v, 1u);
    const int64_t done = s0 + it + 1;  // sweeps completed
    if (threadIdx.x == 0) {
      const double mm = v[0];
      int32_t st = ST_RUN;
      if (!finite(mm)) st = ST_NONFINITE;
      else if (strict ? (mm < thr[inst]) : (mm <= thr[inst])) st = ST_CONVERGED;
      else if (done >= max_iter) st = ST_MAXITER;
      meas[inst] = mm;
      if (st != ST_RUN) {
        status[inst] = st;
        iters[inst] = done;
        atomicAdd(ndone, 1);
      }
      decision = st;
    }
    __syncthreads();
    if (decision != ST_RUN || it == nsweeps - 1) {
      T* dst = (done & 1) ? xb : xa;
      for (int i = threadIdx.x; i < nr; i += TNT) dst[r0 + i] = nxt[i];
      // a weighted measure is the residual of the previous iterate: keep it
      // in the other buffer, as the tiled sweeps do
      if (decision != ST_RUN && weighted) {
        T* dprev = (done & 1) ? xa : xb;
        for (int i = threadIdx.x; i < nr; i += TNT) dprev[r0 + i] = cur[i];
      }
      return;
    }
  }
}

template <typename T>
hipError_t launch_jacobi_resident_sliced(hipStream_t st, Sliced<T> sl, const T* rhs, T* xa, T* xb, Tiles tl,
                                         const int32_t* s_lo, const int32_t* s_hi, int64_t s0, int nsweeps,
                                         int32_t* status, int64_t* iters, double* meas, const double* thr,
                                         int strict, int64_t max_iter, int32_t* ndone, int weighted) {
  if (tl.ntile <= 0 || nsweeps <= 0) return hipSuccess;
  const size_t lds = 2 * (size_t)tl.maxw * sizeof(T);
  static size_t conf = 0;
  hipError_t e = set_lds(k_jacobi_resident_sliced<T>, lds, conf);
  if (e != hipSuccess) return e;
  k_jacobi_resident_sliced<T><<<(unsigned)tl.ntile, TNT, lds, st>>>(sl, rhs, xa, xb, tl, s_lo, s_hi, s0, nsweeps,
                                                                    status, iters, meas, thr, strict, max_iter,
                                                                    ndone, weighted);
  return hipGetLastError();
}
template hipError_t launch_jacobi_resident_sliced<double>(hipStream_t, Sliced<double>, const double*, double*,
                                                          double*, Tiles, const int32_t*, const int32_t*, int64_t,
                                                          int, int32_t*, int64_t*, double*, const double*, int,
                                                          int64_t, int32_t*, int);
template hipError_t launch_jacobi_resident_sliced<float>(hipStream_t, Sliced<float>, const float*, float*, float*,
                                                         Tiles, const int32_t*, const int32_t*, int64_t, int,
                                                         int32_t*, int64_t*, double*, const double*, int, int64_t,
                                                         int32_t*, int);

// y = d u - A_off u on sliced rows, with the dot products of the lane-group
// kernel (MODE 0: q.y; MODE 1: y.u and y.y), or (MODE 2) the FP64 residual
// y <- qv - y of the refinement with its max |.| (qv is then b).
template <typename T, int MODE, int KIND, bool NT>
__device__ __forceinline__ void spmv_sliced_rows(const Sliced<T>& sl, const T* __restrict__ us,
                                                 const T* __restrict__ u, T* __restrict__ y, const T* __restrict__ qv,
                                                 int sb, int se, int w0, int nw, double* a) {
  constexpr int U = SliceShape<T>::U, NS = SliceShape<T>::NS, NW = TNT / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int s0 = sb + wave; s0 < se; s0 += NW * NS) {
    SliceGroup<T, U, NS> g;
    g.setup(sl, s0, se, lane);
    T acc[NS];
#pragma unroll
    for (int q = 0; q < NS; q++) acc[q] = 0;
    for (int j = 0; j < g.Wm; j += U) {
      g.template chunk<KIND, NT>(sl, j, lane);
#pragma unroll
      for (int q = 0; q < NS; q++)
#pragma unroll
        for (int k = 0; k < U; k++) acc[q] += g.vv[q][k] * xget<KIND>(us, u, g.cc[q][k], nw, w0);
    }
#pragma unroll
    for (int q = 0; q < NS; q++) {
      const int row = g.row[q];
      if (row >= 0) {
        const T ui = xget<KIND>(us, u, row - w0, nw, w0);
        const T yi = g.d[q] * ui - acc[q];
        if (MODE == 2) {
          const T ri = qv[row] - yi;
          y[row] = ri;
          a[0] = mx(a[0], fabs((double)ri));
        } else if (MODE == 0) {
          y[row] = yi;
          a[0] += (double)qv[row] * (double)yi;
        } else {
          y[row] = yi;
          a[0] += (double)yi * (double)ui;
          a[1] += (double)yi * (double)yi;
        }
      }
    }
  }
}

template <typename T, int MODE, bool NT, bool PANEL>
__global__ __launch_bounds__(TNT) void k_spmv_sliced(Sliced<T> sl, const T* __restrict__ u, T* __restrict__ y,
                                                     const T* __restrict__ qv, Tiles tl,
                                                     const int32_t* __restrict__ status, double* __restrict__ part) {
  extern __shared__ unsigned char smem_raw[];
  T* us = reinterpret_cast<T*>(smem_raw);
  const int c = tile_of(tl);
  if (status[tl.inst[c]] != ST_RUN) return;
  const int w0 = tl.w0[c], nw = tl.nw[c], kind = tl.kind[c];
  const int sb = sl.t_s0[c], se = sl.t_s0[c + 1];
  if (kind != WIN_NONE) {
    stage_window<T, TNT>(us, u, w0, nw);
    __syncthreads();
  }
  double a[2] = {0.0, 0.0};
  if (PANEL && sl.npan[c] > 0) spmv_panel_rows<T, MODE>(sl, us, u, y, qv, c, sb, se, w0, a);
  else if (kind == WIN_WHOLE) spmv_sliced_rows<T, MODE, WIN_WHOLE, NT>(sl, us, u, y, qv, sb, se, w0, nw, a);
  else if (kind == WIN_BAND) spmv_sliced_rows<T, MODE, WIN_BAND, NT>(sl, us, u, y, qv, sb, se, w0, nw, a);
  else spmv_sliced_rows<T, MODE, WIN_NONE, NT>(sl, us, u, y, qv, sb, se, w0, nw, a);
  if (MODE != 1) {
    double b1[1] = {a[0]};
    block_reduce<1, TNT>(b1, MODE == 2 ? 1u : 0u);
    if (threadIdx.x == 0) part[c] = b1[0];
  } else {
    block_reduce<2, TNT>(a, 0u);
    if (threadIdx.x == 0) {
      part[2 * c] = a[0];
      part[2 * c + 1] = a[1];
    }
  }
}

template <typename T, int MODE>
static hipError_t spmv_sliced_M(hipStream_t st, Sliced<T> sl, const T* u, T* y, const T* qv, Tiles tl,
                                const int32_t* status, double* part) {
  const size_t lds = (size_t)max(tl.maxw, sl.paneled ? sl.pw : 0) * sizeof(T);
  static size_t conf[4] = {0, 0, 0, 0};
  const int v = (sl.stream ? 1 : 0) + (sl.paneled ? 2 : 0);
  const auto kern = v == 0 ? k_spmv_sliced<T, MODE, false, false> : v == 1 ? k_spmv_sliced<T, MODE, true, false>
                  : v == 2 ? k_spmv_sliced<T, MODE, false, true> : k_spmv_sliced<T, MODE, true, true>;
  hipError_t e = set_lds(kern, lds, conf[v]);
  if (e != hipSuccess) return e;
  kern<<<(unsigned)tl.ntile, TNT, lds, st>>>(sl, u, y, qv, tl, status, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_spmv_sliced(hipStream_t st, int mode, Sliced<T> sl, const T* u, T* y, const T* qv, Tiles tl,
                              const int32_t* status, double* part) {
  if (mode == 2) return spmv_sliced_M<T, 2>(st, sl, u, y, qv, tl, status, part);
  return mode ? spmv_sliced_M<T, 1>(st, sl, u, y, qv, tl, status, part)
              : spmv_sliced_M<T, 0>(st, sl, u, y, qv, tl, status, part);
}
template hipError_t launch_spmv_sliced<double>(hipStream_t, int, Sliced<double>, const double*, double*,
                                               const double*, Tiles, const int32_t*, double*);
template hipError_t launch_spmv_sliced<float>(hipStream_t, int, Sliced<float>, const float*, float*, const float*,
                                              Tiles, const int32_t*, double*);

// ============================================================================
// BiCGStab (Section 3.2), one instance-batched step per kernel; all scalars
// (rho = q.r, alpha, omega, beta) are FP64 device arrays, one per instance.
// ============================================================================

// r = rhs - M x (x = 0: r = rhs), q = r, p = v = 0; partials q.r and max|r|.
template <typename T, int L>
__global__ __launch_bounds__(BS) void k_bicg_init(MatView<T> m, const T* __restrict__ rhs,
                                                  const T* __restrict__ x, int x_is_zero, T* __restrict__ r,
                                                  T* __restrict__ q, T* __restrict__ p, T* __restrict__ v,
                                                  Chunks ch, const int32_t* __restrict__ status,
                                                  double* __restrict__ partial) {
  const int c = blockIdx.x;
  if (status[ch.inst[c]] != ST_RUN) return;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = BS / L;
  double a[2] = {0.0, 0.0};
  for (int base = 0; base < nr; base += RPP) {
    const bool ok = base + g < nr;
    const int row = r0 + base + g;
    T acc = 0;
    if (!x_is_zero) acc = row_sum<T, L>(m, x, row, ok, lane);
    if (ok && lane == 0) {
      const T ri = x_is_zero ? rhs[row] : rhs[row] - (m.d[row] * x[row] - acc);
      r[row] = ri; q[row] = ri; p[row] = 0; v[row] = 0;
      a[0] += (double)ri * (double)ri;
      a[1] = mx(a[1], fabs((double)ri));
    }
  }
  block_reduce<2>(a, 2u);
  if (threadIdx.x == 0) { partial[2 * c] = a[0]; partial[2 * c + 1] = a[1]; }
}

template <typename T>
hipError_t launch_bicg_init(hipStream_t st, int L, MatView<T> m, const T* rhs, const T* x, int x_is_zero, T* r,
                            T* q, T* p, T* v, Chunks ch, const int32_t* status, double* partial2) {
  const unsigned g = (unsigned)ch.nchunk;
  switch (L) {
    case 1: k_bicg_init<T, 1><<<g, BS, 0, st>>>(m, rhs, x, x_is_zero, r, q, p, v, ch, status, partial2); break;
    case 2: k_bicg_init<T, 2><<<g, BS, 0, st>>>(m, rhs, x, x_is_zero, r, q, p, v, ch, status, partial2); break;
    case 4: k_bicg_init<T, 4><<<g, BS, 0, st>>>(m, rhs, x, x_is_zero, r, q, p, v, ch, status, partial2); break;
    case 8: k_bicg_init<T, 8><<<g, BS, 0, st>>>(m, rhs, x, x_is_zero, r, q, p, v, ch, status, partial2); break;
    case 16: k_bicg_init<T, 16><<<g, BS, 0, st>>>(m, rhs, x, x_is_zero, r, q, p, v, ch, status, partial2); break;
    case 32: k_bicg_init<T, 32><<<g, BS, 0, st>>>(m, rhs, x, x_is_zero, r, q, p, v, ch, status, partial2); break;
    case 64: k_bicg_init<T, 64><<<g, BS, 0, st>>>(m, rhs, x, x_is_zero, r, q, p, v, ch, status, partial2); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_bicg_init<double>(hipStream_t, int, MatView<double>, const double*, const double*, int,
                                             double*, double*, double*, double*, Chunks, const int32_t*, double*);
template hipError_t launch_bicg_init<float>(hipStream_t, int, MatView<float>, const float*, const float*, int,
                                            float*, float*, float*, float*, Chunks, const int32_t*, double*);

__global__ void k_fin_bicg_init(Chunks ch, const double* __restrict__ partial, int32_t* status, double* rho,
                                double* alpha, double* omega, double* beta, double* meas,
                                const double* __restrict__ thr, int measmode, int32_t* ndone) {
  const int k = blockIdx.x;
  if (status[k] != ST_RUN) return;
  double v[2];
  reduce_instance<2>(ch, k, partial, 2u, v);
  if (threadIdx.x == 0) {
    rho[k] = v[0]; alpha[k] = 1.0; omega[k] = 1.0; beta[k] = 0.0; meas[k] = v[1];
    int32_t s = ST_RUN;
    if (!finite(v[0]) || !finite(v[1])) s = ST_NONFINITE;
    else if (v[1] == 0.0) s = ST_CONVERGED;  // r = 0: x is exact
    else if (measmode == MEAS_R && v[1] <= thr[k]) s = ST_CONVERGED;
    if (s != ST_RUN) { status[k] = s; atomicAdd(ndone, 1); }
  }
}
hipError_t launch_fin_bicg_init(hipStream_t st, Chunks ch, const double* partial2, int32_t* status, double* rho,
                                double* alpha, double* omega, double* beta, double* meas, const double* thr,
                                int measmode, int32_t* ndone) {
  k_fin_bicg_init<<<(unsigned)ch.K, BS, 0, st>>>(ch, partial2, status, rho, alpha, omega, beta, meas, thr,
                                                 measmode, ndone);
  return hipGetLastError();
}

// p = r + beta (p - omega v)
template <typename T>
__global__ __launch_bounds__(BS) void k_bicg_p(const T* __restrict__ r, T* __restrict__ p, const T* __restrict__ v,
                                               const double* __restrict__ beta, const double* __restrict__ omega,
                                               Chunks ch, const int32_t* __restrict__ status) {
  const int c = blockIdx.x;
  const int k = ch.inst[c];
  if (status[k] != ST_RUN) return;
  const T b = (T)beta[k], w = (T)omega[k];
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  for (int i = threadIdx.x; i < nr; i += BS) {
    const int row = r0 + i;
    p[row] = r[row] + b * (p[row] - w * v[row]);
  }
}
template <typename T>
hipError_t launch_bicg_p(hipStream_t st, const T* r, T* p, const T* v, const double* beta, const double* omega,
                         Chunks ch, const int32_t* status) {
  k_bicg_p<T><<<(unsigned)ch.nchunk, BS, 0, st>>>(r, p, v, beta, omega, ch, status);
  return hipGetLastError();
}
template hipError_t launch_bicg_p<double>(hipStream_t, const double*, double*, const double*, const double*,
                                          const double*, Chunks, const int32_t*);
template hipError_t launch_bicg_p<float>(hipStream_t, const float*, float*, const float*, const double*,
                                         const double*, Chunks, const int32_t*);

// y = M u = d u - A_off u with partial dot products accumulated in FP64:
// mode 0: q.y ; mode 1: y.u and y.y
template <typename T, int L, int MODE>
__global__ __launch_bounds__(BS) void k_spmv_dot(MatView<T> m, const T* __restrict__ u, T* __restrict__ y,
                                                 const T* __restrict__ q, Chunks ch,
                                                 const int32_t* __restrict__ status, double* __restrict__ partial) {
  const int c = blockIdx.x;
  if (status[ch.inst[c]] != ST_RUN) return;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = BS / L;
  double a[2] = {0.0, 0.0};
  for (int base = 0; base < nr; base += RPP) {
    const bool ok = base + g < nr;
    const int row = r0 + base + g;
    const T acc = row_sum<T, L>(m, u, row, ok, lane);
    if (ok && lane == 0) {
      const T ui = u[row];
      const T yi = m.d[row] * ui - acc;
      y[row] = yi;
      if (MODE == 0) {
        a[0] += (double)q[row] * (double)yi;
      } else {
        a[0] += (double)yi * (double)ui;
        a[1] += (double)yi * (double)yi;
      }
    }
  }
  if (MODE == 0) {
    double b1[1] = {a[0]};
    block_reduce<1>(b1, 0u);
    if (threadIdx.x == 0) partial[c] = b1[0];
  } else {
    block_reduce<2>(a, 0u);
    if (threadIdx.x == 0) { partial[2 * c] = a[0]; partial[2 * c + 1] = a[1]; }
  }
}

template <typename T, int MODE>
static hipError_t launch_spmv_mode(hipStream_t st, int L, MatView<T> m, const T* u, T* y, const T* q, Chunks ch,
                                   const int32_t* status, double* partial) {
  const unsigned g = (unsigned)ch.nchunk;
  switch (L) {
    case 1: k_spmv_dot<T, 1, MODE><<<g, BS, 0, st>>>(m, u, y, q, ch, status, partial); break;
    case 2: k_spmv_dot<T, 2, MODE><<<g, BS, 0, st>>>(m, u, y, q, ch, status, partial); break;
    case 4: k_spmv_dot<T, 4, MODE><<<g, BS, 0, st>>>(m, u, y, q, ch, status, partial); break;
    case 8: k_spmv_dot<T, 8, MODE><<<g, BS, 0, st>>>(m, u, y, q, ch, status, partial); break;
    case 16: k_spmv_dot<T, 16, MODE><<<g, BS, 0, st>>>(m, u, y, q, ch, status, partial); break;
    case 32: k_spmv_dot<T, 32, MODE><<<g, BS, 0, st>>>(m, u, y, q, ch, status, partial); break;
    case 64: k_spmv_dot<T, 64, MODE><<<g, BS, 0, st>>>(m, u, y, q, ch, status, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <typename T>
hipError_t launch_spmv_dot(hipStream_t st, int L, int mode, MatView<T> m, const T* u, T* y, const T* q, Chunks ch,
                           const int32_t* status, double* partial) {
  return mode == 0 ? launch_spmv_mode<T, 0>(st, L, m, u, y, q, ch, status, partial)
                   : launch_spmv_mode<T, 1>(st, L, m, u, y, q, ch, status, partial);
}
template hipError_t launch_spmv_dot<double>(hipStream_t, int, int, MatView<double>, const double*, double*,
                                            const double*, Chunks, const int32_t*, double*);
template hipError_t launch_spmv_dot<float>(hipStream_t, int, int, MatView<float>, const float*, float*,
                                           const float*, Chunks, const int32_t*, double*);

// alpha = rho / (q.v)
__global__ void k_fin_alpha(Chunks ch, const double* __restrict__ partial, int32_t* status,
                            const double* __restrict__ rho, double* alpha, int32_t* ndone) {
  const int k = blockIdx.x;
  if (status[k] != ST_RUN) return;
  double v[1];
  reduce_instance<1>(ch, k, partial, 0u, v);
  if (threadIdx.x == 0) {
    const double qv = v[0];
    int32_t s = ST_RUN;
    if (!finite(qv)) s = ST_NONFINITE;
    else if (qv == 0.0) s = ST_BREAKDOWN;
    else alpha[k] = rho[k] / qv;
    if (s != ST_RUN) { status[k] = s; atomicAdd(ndone, 1); }
  }
}
hipError_t launch_fin_alpha(hipStream_t st, Chunks ch, const double* partial, int32_t* status, const double* rho,
                            double* alpha, int32_t* ndone) {
  k_fin_alpha<<<(unsigned)ch.K, BS, 0, st>>>(ch, partial, status, rho, alpha, ndone);
  return hipGetLastError();
}

// s = r - alpha v, partial max|s|
template <typename T>
__global__ __launch_bounds__(BS) void k_bicg_s(const T* __restrict__ r, const T* __restrict__ v, T* __restrict__ s,
                                               const double* __restrict__ alpha, Chunks ch,
                                               const int32_t* __restrict__ status, double* __restrict__ partial) {
  const int c = blockIdx.x;
  const int k = ch.inst[c];
  if (status[k] != ST_RUN) return;
  const T a = (T)alpha[k];
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  double m = 0.0;
  for (int i = threadIdx.x; i < nr; i += BS) {
    const int row = r0 + i;
    const T si = r[row] - a * v[row];
    s[row] = si;
    m = mx(m, fabs((double)si));
  }
  double b1[1] = {m};
  block_reduce<1>(b1, 1u);
  if (threadIdx.x == 0) partial[c] = b1[0];
}
template <typename T>
hipError_t launch_bicg_s(hipStream_t st, const T* r, const T* v, T* s, const double* alpha, Chunks ch,
                         const int32_t* status, double* partial) {
  k_bicg_s<T><<<(unsigned)ch.nchunk, BS, 0, st>>>(r, v, s, alpha, ch, status, partial);
  return hipGetLastError();
}
template hipError_t launch_bicg_s<double>(hipStream_t, const double*, const double*, double*, const double*,
                                          Chunks, const int32_t*, double*);
template hipError_t launch_bicg_s<float>(hipStream_t, const float*, const float*, float*, const double*, Chunks,
                                         const int32_t*, double*);

// omega = (t.s) / (t.t), zero when t = 0
__global__ void k_fin_omega(Chunks ch, const double* __restrict__ partial, int32_t* status, double* omega,
                            int32_t* ndone) {
  const int k = blockIdx.x;
  if (status[k] != ST_RUN) return;
  double v[2];
  reduce_instance<2>(ch, k, partial, 0u, v);
  if (threadIdx.x == 0) {
    const double ts = v[0], tt = v[1];
    if (!finite(ts) || !finite(tt)) {
      status[k] = ST_NONFINITE;
      atomicAdd(ndone, 1);
    } else {
      omega[k] = (tt == 0.0) ? 0.0 : ts / tt;
    }
  }
}
hipError_t launch_fin_omega(hipStream_t st, Chunks ch, const double* partial2, int32_t* status, double* omega,
                            int32_t* ndone) {
  k_fin_omega<<<(unsigned)ch.K, BS, 0, st>>>(ch, partial2, status, omega, ndone);
  return hipGetLastError();
}

// x += alpha p + omega s ; r = s - omega t ; partials q.r and max|r|
template <typename T>
__global__ __launch_bounds__(BS) void k_bicg_xr(T* __restrict__ x, const T* __restrict__ p, const T* __restrict__ s,
                                                T* __restrict__ r, const T* __restrict__ t, const T* __restrict__ q,
                                                const double* __restrict__ alpha, const double* __restrict__ omega,
                                                Chunks ch, const int32_t* __restrict__ status,
                                                double* __restrict__ partial) {
  const int c = blockIdx.x;
  const int k = ch.inst[c];
  if (status[k] != ST_RUN) return;
  const T a = (T)alpha[k], w = (T)omega[k];
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  double acc[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < nr; i += BS) {
    const int row = r0 + i;
    const T si = s[row];
    x[row] = x[row] + a * p[row] + w * si;
    const T ri = si - w * t[row];
    r[row] = ri;
    acc[0] += (double)q[row] * (double)ri;
    acc[1] = mx(acc[1], fabs((double)ri));
  }
  block_reduce<2>(acc, 2u);
  if (threadIdx.x == 0) { partial[2 * c] = acc[0]; partial[2 * c + 1] = acc[1]; }
}
template <typename T>
hipError_t launch_bicg_xr(hipStream_t st, T* x, const T* p, const T* s, T* r, const T* t, const T* q,
                          const double* alpha, const double* omega, Chunks ch, const int32_t* status,
                          double* partial2) {
  k_bicg_xr<T><<<(unsigned)ch.nchunk, BS, 0, st>>>(x, p, s, r, t, q, alpha, omega, ch, status, partial2);
  return hipGetLastError();
}
template hipError_t launch_bicg_xr<double>(hipStream_t, double*, const double*, const double*, double*,
                                           const double*, const double*, const double*, const double*, Chunks,
                                           const int32_t*, double*);
template hipError_t launch_bicg_xr<float>(hipStream_t, float*, const float*, const float*, float*, const float*,
                                          const float*, const double*, const double*, Chunks, const int32_t*,
                                          double*);

// rho_new = q.r ; beta = (rho_new / rho)(alpha / omega) ; stopping test.
__global__ void k_fin_rho(Chunks ch, const double* __restrict__ pxr, const double* __restrict__ ps, int32_t* status,
                          double* rho, const double* __restrict__ alpha, const double* __restrict__ omega,
                          double* beta, int64_t* iters, double* meas, const double* __restrict__ thr, int measmode,
                          int64_t max_iter, int32_t* ndone) {
  const int k = blockIdx.x;
  if (status[k] != ST_RUN) return;
  double v[2];
  reduce_instance<2>(ch, k, pxr, 2u, v);
  __syncthreads();
  double w[1];
  reduce_instance<1>(ch, k, ps, 1u, w);
  if (threadIdx.x == 0) {
    const double rnew = v[0], rmax = v[1], smax = w[0];
    const int64_t it = iters[k] + 1;
    iters[k] = it;
    const double m = (measmode == MEAS_S) ? smax : rmax;
    meas[k] = m;
    int32_t s = ST_RUN;
    if (!finite(rnew) || !finite(m)) s = ST_NONFINITE;
    else if (m <= thr[k]) s = ST_CONVERGED;
    else if (it >= max_iter) s = ST_MAXITER;
    else if (rnew == 0.0 || omega[k] == 0.0) s = ST_BREAKDOWN;
    else {
      beta[k] = (rnew / rho[k]) * (alpha[k] / omega[k]);
      rho[k] = rnew;
    }
    if (s != ST_RUN) { status[k] = s; atomicAdd(ndone, 1); }
  }
}
hipError_t launch_fin_rho(hipStream_t st, Chunks ch, const double* partial_xr, const double* partial_s,
                          int32_t* status, double* rho, const double* alpha, const double* omega, double* beta,
                          int64_t* iters, double* meas, const double* thr, int measmode, int64_t max_iter,
                          int32_t* ndone) {
  k_fin_rho<<<(unsigned)ch.K, BS, 0, st>>>(ch, partial_xr, partial_s, status, rho, alpha, omega, beta, iters, meas,
                                           thr, measmode, max_iter, ndone);
  return hipGetLastError();
}

// ============================================================================
// FP64 iterative refinement
// ============================================================================

// r = b - M x in FP64, partial max|r|
template <int L>
__global__ __launch_bounds__(BS) void k_residual64(MatView<double> m, const double* __restrict__ b,
                                                   const double* __restrict__ x, double* __restrict__ r, Chunks ch,
                                                   const int32_t* __restrict__ status, double* __restrict__ partial) {
  const int c = blockIdx.x;
  if (status[ch.inst[c]] != ST_RUN) return;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  constexpr int RPP = BS / L;
  double mloc = 0.0;
  for (int base = 0; base < nr; base += RPP) {
    const bool ok = base + g < nr;
    const int row = r0 + base + g;
    const double acc = row_sum<double, L>(m, x, row, ok, lane);
    if (ok && lane == 0) {
      const double y = m.d[row] * x[row] - acc;
      const double ri = b[row] - y;
      r[row] = ri;
      mloc = mx(mloc, fabs(ri));
    }
  }
  double v[1] = {mloc};
  block_reduce<1>(v, 1u);
  if (threadIdx.x == 0) partial[c] = v[0];
}
hipError_t launch_residual64(hipStream_t st, int L, MatView<double> m, const double* b, const double* x,
                             double* r, Chunks ch, const int32_t* status, double* partial) {
  const unsigned g = (unsigned)ch.nchunk;
  switch (L) {
    case 1: k_residual64<1><<<g, BS, 0, st>>>(m, b, x, r, ch, status, partial); break;
    case 2: k_residual64<2><<<g, BS, 0, st>>>(m, b, x, r, ch, status, partial); break;
    case 4: k_residual64<4><<<g, BS, 0, st>>>(m, b, x, r, ch, status, partial); break;
    case 8: k_residual64<8><<<g, BS, 0, st>>>(m, b, x, r, ch, status, partial); break;
    case 16: k_residual64<16><<<g, BS, 0, st>>>(m, b, x, r, ch, status, partial); break;
    case 32: k_residual64<32><<<g, BS, 0, st>>>(m, b, x, r, ch, status, partial); break;
    case 64: k_residual64<64><<<g, BS, 0, st>>>(m, b, x, r, ch, status, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Outer test: converged when (certified) tb*||r|| <= tol or ||r|| <= tol.
// Otherwise prepares the scale of the next correction and the threshold of
// the inner solve (relative to the scaled right-hand side).
// A refinement that has not halved the best residual for kStall steps in a
// row has reached the rounding floor of the FP64 residual: it stops there
// (reported as not converged) instead of running to max_refine.
constexpr int kStall = 3;

__global__ void k_fin_outer(Chunks ch, const double* __restrict__ partial, int32_t* status, int64_t* outer_it,
                            double* rn, double* scale, const double* __restrict__ tb, double tol, int certified,
                            int32_t max_refine, double* thr_in, double inner_tol, double floor_rel, double margin,
                            double* rbest, int32_t* stall, const int64_t* __restrict__ tot_it, int64_t max_iter,
                            int32_t* ndone) {
  const int k = blockIdx.x;
  if (status[k] != ST_RUN) return;
  double v[1];
  reduce_instance<1>(ch, k, partial, 1u, v);
  if (threadIdx.x == 0) {
    const double r = v[0];
    const int64_t it = outer_it[k] + 1;
    outer_it[k] = it;
    rn[k] = r;
    const double t = (tb && tb[k] > 0.0) ? tb[k] : 1.0;
    const bool conv = certified ? (t * r <= tol) : (r <= tol);
    if (it == 1 || r < 0.5 * rbest[k]) {
      rbest[k] = r;
      stall[k] = 0;
    } else {
      stall[k] += 1;
    }
    int32_t s = ST_RUN;
    if (!finite(r)) s = ST_NONFINITE;
    else if (conv) s = ST_CONVERGED;
    else if (it > max_refine || stall[k] >= kStall || tot_it[k] >= max_iter) s = ST_MAXITER;
    else {
      scale[k] = r;
      const double target = certified ? tol / t : tol;
      double th = fmin(inner_tol, margin * target / r);
      th = fmax(th, floor_rel * t);
      thr_in[k] = th;
    }
    if (s != ST_RUN) { status[k] = s; atomicAdd(ndone, 1); }
  }
}
hipError_t launch_fin_outer(hipStream_t st, Chunks ch, const double* partial, int32_t* status, int64_t* outer_it,
                            double* rn, double* scale, const double* tb, double tol, int certified,
                            int32_t max_refine, double* thr_in, double inner_tol, double floor_rel, double margin,
                            double* rbest, int32_t* stall, const int64_t* tot_it, int64_t max_iter,
                            int32_t* ndone) {
  k_fin_outer<<<(unsigned)ch.K, BS, 0, st>>>(ch, partial, status, outer_it, rn, scale, tb, tol, certified,
                                             max_refine, thr_in, inner_tol, floor_rel, margin, rbest, stall, tot_it,
                                             max_iter, ndone);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(BS) void k_scale_rhs(const double* __restrict__ r64, const double* __restrict__ scale,
                                                  T* __restrict__ rhs, Chunks ch, const int32_t* __restrict__ status) {
  const int c = blockIdx.x;
  const int k = ch.inst[c];
  if (status[k] != ST_RUN) return;
  const double inv = 1.0 / scale[k];
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  for (int i = threadIdx.x; i < nr; i += BS) rhs[r0 + i] = (T)(r64[r0 + i] * inv);
}
template <typename T>
hipError_t launch_scale_rhs(hipStream_t st, const double* r64, const double* scale, T* rhs, Chunks ch,
                            const int32_t* status) {
  k_scale_rhs<T><<<(unsigned)ch.nchunk, BS, 0, st>>>(r64, scale, rhs, ch, status);
  return hipGetLastError();
}
template hipError_t launch_scale_rhs<double>(hipStream_t, const double*, const double*, double*, Chunks,
                                             const int32_t*);
template hipError_t launch_scale_rhs<float>(hipStream_t, const double*, const double*, float*, Chunks,
                                            const int32_t*);

// x64 += scale * correction.  The correction sits in xa or xb by the parity
// of the Jacobi count par[k] (iterate x_m after m sweeps); with prev set the
// iterate before it, x_{m-1}, is taken (its residual is what a weighted
// Jacobi stopping measure evaluated).
template <typename T>
__global__ __launch_bounds__(BS) void k_correct(double* __restrict__ x64, const T* __restrict__ xa,
                                                const T* __restrict__ xb, const int64_t* __restrict__ par,
                                                int prev, const int32_t* __restrict__ status_in,
                                                const double* __restrict__ scale, Chunks ch,
                                                const int32_t* __restrict__ status_out) {
  const int c = blockIdx.x;
  const int k = ch.inst[c];
  if (status_out[k] != ST_RUN || status_in[k] == ST_NONFINITE) return;
  const int64_t m = par ? par[k] - (prev && par[k] > 0 ? 1 : 0) : 0;
  const T* src = (m & 1) ? xb : xa;
  const double sc = scale[k];
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  for (int i = threadIdx.x; i < nr; i += BS) x64[r0 + i] += sc * (double)src[r0 + i];
}
template <typename T>
hipError_t launch_correct(hipStream_t st, double* x64, const T* xa, const T* xb, const int64_t* parity_iters,
                          int prev, const int32_t* status_in, const double* scale, Chunks ch,
                          const int32_t* status_out) {
  k_correct<T><<<(unsigned)ch.nchunk, BS, 0, st>>>(x64, xa, xb, parity_iters, prev, status_in, scale, ch,
                                                   status_out);
  return hipGetLastError();
}
template hipError_t launch_correct<double>(hipStream_t, double*, const double*, const double*, const int64_t*, int,
                                           const int32_t*, const double*, Chunks, const int32_t*);
template hipError_t launch_correct<float>(hipStream_t, double*, const float*, const float*, const int64_t*, int,
                                          const int32_t*, const double*, Chunks, const int32_t*);

__global__ void k_inner_init(int32_t K, const int32_t* __restrict__ status_out, const int64_t* __restrict__ nq,
                             int32_t* status_in, int64_t* iters_in, int32_t* ndone) {
  __shared__ int32_t cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int32_t local = 0;
  for (int k = threadIdx.x; k < K; k += BS) {
    const bool skip = (status_out && status_out[k] != ST_RUN) || nq[k] == 0;
    status_in[k] = skip ? ST_SKIP : ST_RUN;
    iters_in[k] = 0;
    local += skip ? 1 : 0;
  }
  atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) *ndone = cnt;
}
hipError_t launch_inner_init(hipStream_t st, int32_t K, const int32_t* status_out, const int64_t* nq,
                             int32_t* status_in, int64_t* iters_in, int32_t* ndone) {
  k_inner_init<<<1, BS, 0, st>>>(K, status_out, nq, status_in, iters_in, ndone);
  return hipGetLastError();
}

// Stagnation watch of the paper's stopping rule, run after each batch of
// iterations (launched = iterations completed by every running instance):
// an instance whose latest stopping measure meas[k] has not fallen below
// half of its best value for more than max(min_window, it_best) iterations
// -- the measure sits at the rounding floor of the arithmetic, above the
// tolerance -- stops as ST_STALLED.  best / best_it start at +inf / 0.
__global__ void k_stall(int32_t K, int64_t launched, int32_t* status, int64_t* iters, const double* __restrict__ meas,
                        double* best, int64_t* best_it, int64_t min_window, int32_t* ndone) {
  for (int k = blockIdx.x * BS + threadIdx.x; k < K; k += gridDim.x * BS) {
    if (status[k] != ST_RUN) continue;
    const double m = meas[k];
    const int64_t bi = best_it[k];
    if (m < 0.5 * best[k]) {
      best[k] = m;
      best_it[k] = launched;
    } else if (launched - bi > (min_window > bi ? min_window : bi)) {
      status[k] = ST_STALLED;
      iters[k] = launched;
      atomicAdd(ndone, 1);
    }
  }
}
hipError_t launch_stall(hipStream_t st, int32_t K, int64_t launched, int32_t* status, int64_t* iters,
                        const double* meas, double* best, int64_t* best_it, int64_t min_window, int32_t* ndone) {
  k_stall<<<(unsigned)((K + BS - 1) / BS), BS, 0, st>>>(K, launched, status, iters, meas, best, best_it, min_window,
                                                        ndone);
  return hipGetLastError();
}

// After an inner solve: add its iterations to the instance's total and keep
// its last stopping measure (instances refined in this outer step only).
__global__ void k_accum_inner(int32_t K, const int32_t* __restrict__ status_out, const int64_t* __restrict__ iters_in,
                              const double* __restrict__ meas_in, int64_t* tot_it, double* last_meas) {
  for (int k = blockIdx.x * BS + threadIdx.x; k < K; k += gridDim.x * BS) {
    if (status_out[k] != ST_RUN) continue;
    tot_it[k] += iters_in[k];
    last_meas[k] = meas_in[k];
  }
}
hipError_t launch_accum_inner(hipStream_t st, int32_t K, const int32_t* status_out, const int64_t* iters_in,
                              const double* meas_in, int64_t* tot_it, double* last_meas) {
  k_accum_inner<<<(unsigned)((K + BS - 1) / BS), BS, 0, st>>>(K, status_out, iters_in, meas_in, tot_it, last_meas);
  return hipGetLastError();
}

template <typename T>
__global__ void k_gather_full(int64_t npad, const int32_t* __restrict__ row_state, const double* __restrict__ full,
                              T* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (r >= npad) return;
  const int32_t v = row_state[r];
  out[r] = v >= 0 ? (T)full[v] : (T)0;
}
template <typename T>
hipError_t launch_gather_full(hipStream_t st, int64_t npad, const int32_t* row_state, const double* full, T* out) {
  if (npad > 0) k_gather_full<T><<<grid_for(npad), BS, 0, st>>>(npad, row_state, full, out);
  return hipGetLastError();
}
template hipError_t launch_gather_full<double>(hipStream_t, int64_t, const int32_t*, const double*, double*);
template hipError_t launch_gather_full<float>(hipStream_t, int64_t, const int32_t*, const double*, float*);

// Full state vector: 0 on S_{=0}, s1_value on S_{=1}, the reduced solution on S_?.
__global__ void k_scatter_full(int64_t n, const uint8_t* __restrict__ cls, const int32_t* __restrict__ map,
                               const int64_t* __restrict__ off, int32_t K, const double* __restrict__ xa,
                               const double* __restrict__ xb, const int64_t* __restrict__ par, double s1,
                               double* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  const uint8_t c = cls[v];
  double val;
  if (c == 0) val = 0.0;
  else if (c == 1) val = s1;
  else {
    const double* src = xa;
    if (par) {
      const int k = find_inst(off, K, v);
      if (par[k] & 1) src = xb;
    }
    val = src[map[v]];
  }
  out[v] = val;
}
hipError_t launch_scatter_full(hipStream_t st, int64_t n, const uint8_t* cls, const int32_t* map,
                               const int64_t* inst_off, int32_t K, const double* xa, const double* xb,
                               const int64_t* parity_iters, double s1_value, double* out) {
  if (n > 0)
    k_scatter_full<<<grid_for(n), BS, 0, st>>>(n, cls, map, inst_off, K, xa, xb, parity_iters, s1_value, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(BS) void k_copy_sel(Chunks ch, const double* __restrict__ xa,
                                                 const double* __restrict__ xb, const int64_t* __restrict__ par,
                                                 double* __restrict__ out) {
  const int c = blockIdx.x;
  const int k = ch.inst[c];
  const double* src = (par && (par[k] & 1)) ? xb : xa;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  for (int i = threadIdx.x; i < nr; i += BS) out[r0 + i] = src[r0 + i];
}
hipError_t launch_copy_sel(hipStream_t st, Chunks ch, const double* xa, const double* xb,
                           const int64_t* parity_iters, double* out) {
  k_copy_sel<<<(unsigned)ch.nchunk, BS, 0, st>>>(ch, xa, xb, parity_iters, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(BS) void k_absmax(const double* __restrict__ x, Chunks ch, double* __restrict__ partial) {
  const int c = blockIdx.x;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  double m = 0.0;
  for (int i = threadIdx.x; i < nr; i += BS) m = mx(m, fabs(x[r0 + i]));
  double v[1] = {m};
  block_reduce<1>(v, 1u);
  if (threadIdx.x == 0) partial[c] = v[0];
}
hipError_t launch_absmax(hipStream_t st, const double* x, Chunks ch, double* partial) {
  k_absmax<<<(unsigned)ch.nchunk, BS, 0, st>>>(x, ch, partial);
  return hipGetLastError();
}
__global__ void k_fin_absmax(Chunks ch, const double* __restrict__ partial, double* out) {
  const int k = blockIdx.x;
  double v[1];
  reduce_instance<1>(ch, k, partial, 1u, v);
  if (threadIdx.x == 0) out[k] = v[0];
}
hipError_t launch_fin_absmax(hipStream_t st, Chunks ch, const double* partial, double* out) {
  k_fin_absmax<<<(unsigned)ch.K, BS, 0, st>>>(ch, partial, out);
  return hipGetLastError();
}

// dL/dP(s,s') = lambda_s * x_{s'} on every stored entry of a row in S_?.
__global__ __launch_bounds__(BS) void k_gradient(int64_t n, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, const uint8_t* __restrict__ cls,
                                                 const int32_t* __restrict__ map, const double* __restrict__ lam,
                                                 const double* __restrict__ xfull, double* __restrict__ g) {
  const int64_t v = ((int64_t)blockIdx.x * BS + threadIdx.x) / PG;
  const int l = threadIdx.x % PG;
  if (v >= n) return;
  const int32_t k0 = rp[v], k1 = rp[v + 1];
  if (cls[v] != 2) {
    for (int32_t k = k0 + l; k < k1; k += PG) g[k] = 0.0;
    return;
  }
  const double lv = lam[map[v]];
  for (int32_t k = k0 + l; k < k1; k += PG) g[k] = lv * xfull[col[k]];
}
hipError_t launch_gradient(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const uint8_t* cls,
                           const int32_t* map, const double* lam, const double* xfull, double* g) {
  if (n > 0) k_gradient<<<grid_for(n * PG), BS, 0, st>>>(n, rp, col, cls, map, lam, xfull, g);
  return hipGetLastError();
}

__global__ void k_gather_at(const int32_t* __restrict__ src, const int64_t* __restrict__ idx, int32_t count,
                            int32_t* __restrict__ out) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < count) out[i] = src[idx[i]];
}
hipError_t launch_gather_at(hipStream_t st, const int32_t* src, const int64_t* idx, int32_t count, int32_t* out) {
  if (count > 0) k_gather_at<<<grid_for(count), BS, 0, st>>>(src, idx, count, out);
  return hipGetLastError();
}

// 16-bit columns relative to the first row of the instance block, for blocks
// of at most 65,536 rows (0 elsewhere: never read there).
__global__ __launch_bounds__(BS) void k_col16(Chunks ch, const int64_t* __restrict__ roff,
                                              const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                              uint16_t* __restrict__ c16) {
  const int c = blockIdx.x;
  const int k = ch.inst[c];
  const int64_t lo = roff[k];
  const bool fits = roff[k + 1] - lo <= 65536;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  const int e0 = rp[r0], e1 = rp[r0 + nr];
  for (int e = e0 + threadIdx.x; e < e1; e += BS) c16[e] = fits ? (uint16_t)(col[e] - lo) : (uint16_t)0;
}
hipError_t launch_col16(hipStream_t st, Chunks ch, const int64_t* roff, const int32_t* rp, const int32_t* col,
                        uint16_t* c16) {
  if (ch.nchunk > 0) k_col16<<<(unsigned)ch.nchunk, BS, 0, st>>>(ch, roff, rp, col, c16);
  return hipGetLastError();
}

// Per-instance histogram of log2(|col - row| + 1) over the off-diagonal
// entries (32 bins), to size the LDS window of tiles of large instances.
__global__ __launch_bounds__(BS) void k_band_hist(Chunks ch, const int32_t* __restrict__ arp,
                                                  const int32_t* __restrict__ acol, int32_t* hist) {
  __shared__ int32_t h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const int c = blockIdx.x;
  const int r0 = ch.row0[c], nr = ch.nrows[c];
  for (int i = threadIdx.x; i < nr; i += BS) {
    const int row = r0 + i;
    for (int k = arp[row]; k < arp[row + 1]; k++) {
      const unsigned d = (unsigned)abs(acol[k] - row) + 1u;
      atomicAdd(&h[31 - __clz(d)], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&hist[ch.inst[c] * 32 + threadIdx.x], h[threadIdx.x]);
}
hipError_t launch_band_hist(hipStream_t st, Chunks ch, const int32_t* arp, const int32_t* acol, int32_t* hist) {
  if (ch.nchunk > 0) k_band_hist<<<(unsigned)ch.nchunk, BS, 0, st>>>(ch, arp, acol, hist);
  return hipGetLastError();
}

// Copy one device int32 to host-mapped memory, then publish the sequence
// number (system-scope release, so the host sees the value first).
__global__ void k_publish_next(const int32_t* __restrict__ src, int32_t* dst, int32_t* seq) {
  if (threadIdx.x == 0) {
    const int32_t q = *seq + 1;
    *seq = q;
    dst[0] = *src;
    __threadfence_system();
    __hip_atomic_store(&dst[1], q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}
hipError_t launch_publish_next(hipStream_t st, const int32_t* src, int32_t* dst, int32_t* seq) {
  k_publish_next<<<1, 64, 0, st>>>(src, dst, seq);
  return hipGetLastError();
}
__global__ void k_advance(int64_t* base, int64_t n) {
  if (threadIdx.x == 0) *base += n;
}
hipError_t launch_advance(hipStream_t st, int64_t* base, int64_t n) {
  k_advance<<<1, 64, 0, st>>>(base, n);
  return hipGetLastError();
}
__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0) *p = v;
}
hipError_t launch_set_i64(hipStream_t st, int64_t* p, int64_t v) {
  k_set_i64<<<1, 64, 0, st>>>(p, v);
  return hipGetLastError();
}
__global__ void k_set_i32(int32_t* p, int32_t v) {
  if (threadIdx.x == 0) *p = v;
}
hipError_t launch_set_i32(hipStream_t st, int32_t* p, int32_t v) {
  k_set_i32<<<1, 64, 0, st>>>(p, v);
  return hipGetLastError();
}

__global__ void k_publish(const int32_t* __restrict__ src, int32_t* dst, int32_t seq) {
  if (threadIdx.x == 0) {
    dst[0] = *src;
    __threadfence_system();
    __hip_atomic_store(&dst[1], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}
hipError_t launch_publish(hipStream_t st, const int32_t* src, int32_t* dst, int32_t seq) {
  k_publish<<<1, 64, 0, st>>>(src, dst, seq);
  return hipGetLastError();
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, int64_t n, uint32_t v) {
  if (n > 0) k_fill_u32<<<grid_for(n), BS, 0, st>>>(p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(hipStream_t st, double* p, int64_t n, double v) {
  if (n > 0) k_fill_f64<<<grid_for(n), BS, 0, st>>>(p, n, v);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Strongly connected components of S_? (the decomposition Section 8 proposes:
// components solved in reverse topological order, the one-state ones by
// substitution).  Graph: reduced row v -> column w for every stored entry
// with A(v,w) > 0 (self-loops sit in d).  Coloring algorithm: sink states
// are trimmed as one-state components, then every unassigned state takes the
// largest index among the unassigned states that reach it (forward max
// propagation); a state whose color is its own index roots the component of
// all states of that color that reach it (backward search inside the color);
// those are assigned and the rest go round again.  Passes alternate between
// ascending and descending state order: values written earlier in a pass are
// often seen later in the same pass, so a chain of dependencies in either
// direction settles in few passes.  Every update is monotone (-1 -> id,
// color up, mark 0 -> 1), so a value read stale only delays it, and a pass
// that changes nothing has read only values written before it: the host
// stops at such a pass.

__device__ __forceinline__ int64_t pass_index(int64_t i, int64_t n, int dir) { return dir ? n - 1 - i : i; }

__global__ void k_scc_trim(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const double* __restrict__ val, int32_t* comp, int dir, int32_t* changed) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const int64_t v = pass_index(i, n, dir);
  if (comp[v] >= 0) return;
  for (int e = rp[v]; e < rp[v + 1]; e++) {
    const int w = col[e];
    if (val[e] > 0.0 && w != v && __atomic_load_n(&comp[w], __ATOMIC_RELAXED) < 0) return;
  }
  __atomic_store_n(&comp[v], (int32_t)v, __ATOMIC_RELAXED);
  *changed = 1;
}

__global__ void k_scc_color_init(int64_t n, const int32_t* __restrict__ comp, int32_t* __restrict__ color,
                                 int32_t* __restrict__ mark) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  color[v] = comp[v] < 0 ? (int32_t)v : -1;
  mark[v] = 0;
}

__global__ void k_scc_color(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const double* __restrict__ val, const int32_t* __restrict__ comp, int32_t* color,
                            int dir, int32_t* changed) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const int64_t u = pass_index(i, n, dir);
  if (comp[u] >= 0) return;
  const int32_t cu = __atomic_load_n(&color[u], __ATOMIC_RELAXED);
  int ch = 0;
  for (int e = rp[u]; e < rp[u + 1]; e++) {
    const int w = col[e];
    if (val[e] > 0.0 && comp[w] < 0 && atomicMax(&color[w], cu) < cu) ch = 1;
  }
  if (ch) *changed = 1;
}

__global__ void k_scc_root(int64_t n, const int32_t* __restrict__ comp, const int32_t* __restrict__ color,
                           int32_t* __restrict__ mark) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  if (comp[v] < 0 && color[v] == (int32_t)v) mark[v] = 1;
}

__global__ void k_scc_mark(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const double* __restrict__ val, const int32_t* __restrict__ comp,
                           const int32_t* __restrict__ color, int32_t* mark, int dir, int32_t* changed) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const int64_t v = pass_index(i, n, dir);
  if (comp[v] >= 0 || __atomic_load_n(&mark[v], __ATOMIC_RELAXED)) return;
  const int32_t cv = color[v];
  for (int e = rp[v]; e < rp[v + 1]; e++) {
    const int w = col[e];
    if (val[e] > 0.0 && comp[w] < 0 && color[w] == cv && __atomic_load_n(&mark[w], __ATOMIC_RELAXED)) {
      __atomic_store_n(&mark[v], 1, __ATOMIC_RELAXED);
      *changed = 1;
      return;
    }
  }
}

// marked states join their root's component; counts the states left
__global__ void k_scc_assign(int64_t n, int32_t* __restrict__ comp, const int32_t* __restrict__ color,
                             const int32_t* __restrict__ mark, int32_t* __restrict__ left) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  if (comp[v] >= 0) return;
  if (mark[v]) comp[v] = color[v];
  else atomicAdd(left, 1);
}

// smallest row and size of every component (indexed by its id); over the
// rows of states (not padding): cnt[0] components, cnt[1] components of
// more than one state, cnt[2] the largest size
__global__ void k_scc_stats(int64_t n, const int32_t* __restrict__ comp, const int32_t* __restrict__ row_state,
                            int32_t* __restrict__ minrow, int32_t* __restrict__ size, int32_t* __restrict__ cnt) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  const int c = comp[v];
  atomicMin(&minrow[c], (int32_t)v);
  const int before = atomicAdd(&size[c], 1);
  if (row_state[v] < 0) return;
  if (before == 0) atomicAdd(&cnt[0], 1);
  if (before == 1) atomicAdd(&cnt[1], 1);
  atomicMax(&cnt[2], before + 1);
}

// level of a component: 0 when no edge leaves it, else 1 + the largest level
// an edge leads to (longest path to a sink of the condensation)
__global__ void k_scc_level(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const double* __restrict__ val, const int32_t* __restrict__ comp, int32_t* lvl, int dir,
                            int32_t* changed) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const int64_t v = pass_index(i, n, dir);
  const int cv = comp[v];
  int best = 0;
  for (int e = rp[v]; e < rp[v + 1]; e++) {
    const int cw = comp[col[e]];
    if (val[e] > 0.0 && cw != cv) best = max(best, __atomic_load_n(&lvl[cw], __ATOMIC_RELAXED) + 1);
  }
  if (best > 0 && atomicMax(&lvl[cv], best) < best) *changed = 1;
}

// per row: sort key 2 level + (1 if its component has more than one state),
// so that inside a level the one-state components come first; the largest
// level and the rows in larger components
__global__ void k_scc_rowlevel(int64_t n, const int32_t* __restrict__ comp, const int32_t* __restrict__ lvl,
                               const int32_t* __restrict__ size, int32_t* __restrict__ key,
                               int32_t* __restrict__ rowid, int32_t* __restrict__ maxlvl,
                               int32_t* __restrict__ cyclic_rows) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  const int c = comp[v];
  const int cyc = size[c] > 1 ? 1 : 0;
  key[v] = 2 * lvl[c] + cyc;
  rowid[v] = (int32_t)v;
  atomicMax(maxlvl, lvl[c]);
  if (cyc) atomicAdd(cyclic_rows, 1);
}

// rows per sort key
__global__ void k_scc_levelcount(int64_t n, const int32_t* __restrict__ key, int32_t* __restrict__ count) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (v >= n) return;
  atomicAdd(&count[key[v]], 1);
}

// labels and levels per state of the chain: smallest state index of the
// component (rows keep the states' order inside an instance), -1 outside S_?
__global__ void k_scc_out(int64_t nfull, const int32_t* __restrict__ map, const int32_t* __restrict__ comp,
                          const int32_t* __restrict__ minrow, const int32_t* __restrict__ lvl,
                          const int32_t* __restrict__ row_state, int32_t* __restrict__ label,
                          int32_t* __restrict__ level) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= nfull) return;
  const int r = map[i];
  const int c = r >= 0 ? comp[r] : -1;
  if (label) label[i] = r >= 0 ? row_state[minrow[c]] : -1;
  if (level) level[i] = r >= 0 ? lvl[c] : -1;
}

// Rows rows[0..nr) of one level, one thread each, x updated in place:
// x_v = (b_v + sum_w A(v,w) x_w) / d_v.  For a level of one-state components
// this is back substitution (every w lies in a lower, solved level); inside a
// larger component it is an in-place Jacobi sweep.  The largest change goes
// to *dmax as the bits of a nonnegative double (ordered like the values).
__global__ void k_scc_rows(const int32_t* __restrict__ rows, int32_t nr, MatView<double> m,
                           const double* __restrict__ b, double* x, unsigned long long* dmax) {
  const int i = blockIdx.x * BS + threadIdx.x;
  double dl = 0.0;
  if (i < nr) {
    const int v = rows[i];
    double acc = 0.0;
    for (int e = m.rp[v]; e < m.rp[v + 1]; e++) acc += m.val[e] * x[m.col[e]];
    const double nv = (b[v] + acc) / m.d[v];
    dl = fabs(nv - x[v]);
    x[v] = nv;
  }
  for (int o = 32; o > 0; o >>= 1) dl = fmax(dl, __shfl_xor(dl, o, 64));
  if ((threadIdx.x & 63) == 0 && dl > 0.0) atomicMax(dmax, (unsigned long long)__double_as_longlong(dl));
}

hipError_t launch_scc_trim(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                           int32_t* comp, int dir, int32_t* changed) {
  if (n > 0) k_scc_trim<<<grid_for(n), BS, 0, st>>>(n, rp, col, val, comp, dir, changed);
  return hipGetLastError();
}
hipError_t launch_scc_color_init(hipStream_t st, int64_t n, const int32_t* comp, int32_t* color, int32_t* mark) {
  if (n > 0) k_scc_color_init<<<grid_for(n), BS, 0, st>>>(n, comp, color, mark);
  return hipGetLastError();
}
hipError_t launch_scc_color(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                            const int32_t* comp, int32_t* color, int dir, int32_t* changed) {
  if (n > 0) k_scc_color<<<grid_for(n), BS, 0, st>>>(n, rp, col, val, comp, color, dir, changed);
  return hipGetLastError();
}
hipError_t launch_scc_root(hipStream_t st, int64_t n, const int32_t* comp, const int32_t* color, int32_t* mark) {
  if (n > 0) k_scc_root<<<grid_for(n), BS, 0, st>>>(n, comp, color, mark);
  return hipGetLastError();
}
hipError_t launch_scc_mark(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                           const int32_t* comp, const int32_t* color, int32_t* mark, int dir, int32_t* changed) {
  if (n > 0) k_scc_mark<<<grid_for(n), BS, 0, st>>>(n, rp, col, val, comp, color, mark, dir, changed);
  return hipGetLastError();
}
hipError_t launch_scc_assign(hipStream_t st, int64_t n, int32_t* comp, const int32_t* color, const int32_t* mark,
                             int32_t* left) {
  if (n > 0) k_scc_assign<<<grid_for(n), BS, 0, st>>>(n, comp, color, mark, left);
  return hipGetLastError();
}
hipError_t launch_scc_stats(hipStream_t st, int64_t n, const int32_t* comp, const int32_t* row_state,
                            int32_t* minrow, int32_t* size, int32_t* cnt) {
  if (n > 0) k_scc_stats<<<grid_for(n), BS, 0, st>>>(n, comp, row_state, minrow, size, cnt);
  return hipGetLastError();
}
hipError_t launch_scc_level(hipStream_t st, int64_t n, const int32_t* rp, const int32_t* col, const double* val,
                            const int32_t* comp, int32_t* lvl, int dir, int32_t* changed) {
  if (n > 0) k_scc_level<<<grid_for(n), BS, 0, st>>>(n, rp, col, val, comp, lvl, dir, changed);
  return hipGetLastError();
}
hipError_t launch_scc_rowlevel(hipStream_t st, int64_t n, const int32_t* comp, const int32_t* lvl,
                               const int32_t* size, int32_t* key, int32_t* rowid, int32_t* maxlvl,
                               int32_t* cyclic_rows) {
  if (n > 0) k_scc_rowlevel<<<grid_for(n), BS, 0, st>>>(n, comp, lvl, size, key, rowid, maxlvl, cyclic_rows);
  return hipGetLastError();
}
hipError_t launch_scc_levelcount(hipStream_t st, int64_t n, const int32_t* key, int32_t* count) {
  if (n > 0) k_scc_levelcount<<<grid_for(n), BS, 0, st>>>(n, key, count);
  return hipGetLastError();
}
hipError_t launch_scc_out(hipStream_t st, int64_t nfull, const int32_t* map, const int32_t* comp,
                          const int32_t* minrow, const int32_t* lvl, const int32_t* row_state, int32_t* label,
                          int32_t* level) {
  if (nfull > 0) k_scc_out<<<grid_for(nfull), BS, 0, st>>>(nfull, map, comp, minrow, lvl, row_state, label, level);
  return hipGetLastError();
}
hipError_t launch_scc_rows(hipStream_t st, const int32_t* rows, int32_t nr, MatView<double> m, const double* b,
                           double* x, unsigned long long* dmax) {
  if (nr > 0) k_scc_rows<<<(unsigned)((nr + BS - 1) / BS), BS, 0, st>>>(rows, nr, m, b, x, dmax);
  return hipGetLastError();
}

// Stable sort of (key, val) pairs by key, keys in [0, 2^end_bit): the result
// goes to key_out / val_out.  temp == nullptr: *temp_bytes receives the
// workspace size.  (hipCUB's device radix sort.)
hipError_t launch_sort_by_key(hipStream_t st, int32_t* key, int32_t* val, int32_t* key_out, int32_t* val_out,
                              int64_t n, int end_bit, void* temp, size_t* temp_bytes) {
  return hipcub::DeviceRadixSort::SortPairs(temp, *temp_bytes, key, key_out, val, val_out, (int)n, 0, end_bit, st);
}

}  // namespace rpk
