// Setup kernels of Algorithm 1: input checks, classic strength of connection
// (Section 2.1.1), the undirected strong graph, MIS(2) rounds (Algorithm 2),
// nearest-root aggregation, aggregate segments and the interpolation of
// Algorithm 3.  One thread per row / node: these run once per level and their
// rows are short, so the simple mapping keeps the integer decisions exact.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "amg_internal.hpp"
#include "device_utils.hpp"

namespace amg {

namespace {
constexpr int kT = 256;
inline int grid_for(long n) { return (int)((n + kT - 1) / kT); }

constexpr uint64_t kLow62 = (1ull << 62) - 1;
// tuple state field (top two bits) = s + 1: 0 non-MIS, 1 undecided, 2 MIS
__device__ __forceinline__ int tstate(uint64_t t) { return (int)(t >> 62); }

__global__ void k_check_matrix(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ val, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int s = rp[i], e = rp[i + 1];
  int bits = 0;
  if (e < s) { atomic_or_flag(err, kErrBadColumn); return; }
  bool have_diag = false;
  int prev = -1;
  for (int k = s; k < e; ++k) {
    int j = ci[k];
    double a = val[k];
    if (j < 0 || j >= n || j <= prev) bits |= kErrBadColumn;
    if (!isfinite(a)) bits |= kErrNonFinite;
    if (j == i) { have_diag = true; if (a == 0.0) bits |= kErrZeroDiag; }
    prev = j;
  }
  if (!have_diag) bits |= kErrZeroDiag;
  if (bits) atomic_or_flag(err, bits);
}

__global__ void k_check_rowptr(int n, const int* __restrict__ rp, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && rp[i] > rp[i + 1]) atomic_or_flag(err, kErrBadColumn);
}

__global__ void k_check_index(int n, const int* __restrict__ idx, int limit, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (idx[i] < 0 || idx[i] >= limit)) atomic_or_flag(err, kErrBadColumn);
}

// C_ij = [-s_i a_ij > alpha * max_{-s_i a_ij > 0} (-s_i a_ij)], s_i = sign(a_ii).
// G lanes per row; the maximum is exact, so the lane split changes nothing.
template <int G>
__global__ void __launch_bounds__(256) k_strength(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const double* __restrict__ val, double alpha,
                                                  uint8_t* __restrict__ strong, double* __restrict__ diag) {
  RowGroup<G> rg;
  for (long i0 = rg.gid; i0 < n; i0 += rg.ngroups) {
    const int i = (int)i0;
    const int s = rp[i], e = rp[i + 1];
    int kd = -1;   // the last diagonal entry of the row counts
    double d = 0.0;
    for (int k = s + rg.lane; k < e; k += G)
      if (ci[k] == i) { kd = k; d = val[k]; }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      const int ok = __shfl_xor(kd, off, G);
      const double od = __shfl_xor(d, off, G);
      if (ok > kd) { kd = ok; d = od; }
    }
    const double sg = d > 0.0 ? 1.0 : -1.0;
    double m = 0.0;
    for (int k = s + rg.lane; k < e; k += G) {
      const double t = -sg * val[k];
      if (t > m) m = t;            // the running max only ever holds positive values
    }
    m = RowGroup<G>::max(m);
    const double thr = __dmul_rn(alpha, m);
    for (int k = s + rg.lane; k < e; k += G) strong[k] = (-sg * val[k] > thr) ? 1 : 0;
    if (rg.lane == 0) diag[i] = d;
  }
}

__device__ __forceinline__ int find_in_row(const int* __restrict__ ci, int lo, int hi, int key) {
  // binary search in ci[lo, hi) (sorted); returns the position or -1
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int c = ci[mid];
    if (c == key) return mid;
    if (c < key) lo = mid + 1; else hi = mid;
  }
  return -1;
}

// G = C union C^T over A's (structurally symmetric) pattern; influence counts
// cnt_i = #{j : C_ji = 1}.
template <int G>
__global__ void __launch_bounds__(256) k_graph_count(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const uint8_t* __restrict__ strong,
                                                     uint8_t* __restrict__ gmask, int* __restrict__ gdeg,
                                                     int* __restrict__ cnt, int* err) {
  RowGroup<G> rg;
  bool nonsym = false;
  for (long i0 = rg.gid; i0 < n; i0 += rg.ngroups) {
    const int i = (int)i0;
    const int s = rp[i], e = rp[i + 1];
    int gd = 0, c = 0;
    for (int k = s + rg.lane; k < e; k += G) {
      const int j = ci[k];
      if (j == i) { gmask[k] = 0; continue; }
      const int t = find_in_row(ci, rp[j], rp[j + 1], i);
      if (t < 0) nonsym = true;
      const bool cji = t >= 0 && strong[t];
      const bool g = strong[k] || cji;
      gmask[k] = g ? 1 : 0;
      gd += g;
      c += cji;
    }
    gd = RowGroup<G>::sum(gd);
    c = RowGroup<G>::sum(c);
    if (rg.lane == 0) {
      gdeg[i] = gd;
      cnt[i] = c;
    }
  }
  if (nonsym) atomic_or_flag(err, kErrNonSymPattern);
}

// Columns of G in the order of A's row (a group ballot places each kept entry).
template <int G>
__global__ void __launch_bounds__(256) k_graph_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const uint8_t* __restrict__ gmask,
                                                    const int* __restrict__ gptr, int* __restrict__ gcol) {
  RowGroup<G> rg;
  const uint64_t below = (1ull << rg.lane) - 1;
  for (long i0 = rg.gid; i0 < n; i0 += rg.ngroups) {
    const int i = (int)i0;
    const int s = rp[i], e = rp[i + 1];
    int o = gptr[i];
    for (int base = s; base < e; base += G) {
      const int k = base + rg.lane;
      const bool keep = k < e && gmask[k];
      const uint64_t bits = RowGroup<G>::group_bits(__ballot(keep));
      if (keep) gcol[o + __popcll(bits & below)] = ci[k];
      o += __popcll(bits);
    }
  }
}

// Tuple T_i = (s_i, v_i, i) packed so that integer order is lexicographic
// order: bits 63..62 = s_i + 1, bits 61..32 = influence count, bits 31..0 =
// node hash (a bijection of i, so the hash both breaks ties and names i).
// With lbase (batched systems) the hash takes the index local to the row's
// system, i - lbase[i], so each system draws the priorities it would alone.
__global__ void k_mis_init(int n, const int* __restrict__ cnt, uint32_t seed,
                           uint64_t* __restrict__ T, uint64_t* __restrict__ M1, int* mc, int* err,
                           const int* __restrict__ lbase) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * kMisSlots)   // round 0 starts pending (if there are nodes)
    __hip_atomic_store(&mc[mis_word(i / kMisSlots, i % kMisSlots)], i == 0 && n > 0 ? 1 : 0, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  if (i == 0) __hip_atomic_store(&mc[kMisRoundsWord], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (i >= n) return;
  int c = cnt[i];
  if (c >= (1 << 21)) atomic_or_flag(err, kErrCountOverflow);
  const uint32_t li = (uint32_t)(lbase ? i - lbase[i] : i);
  T[i] = (1ull << 62) | ((uint64_t)(c & ((1 << 30) - 1)) << 32) | (uint64_t)node_hash(li, seed);
  M1[i] = 0;
}

template <int G>
__device__ __forceinline__ uint64_t group_max_u64(uint64_t v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(v, off, G);
    v = o > v ? o : v;
  }
  return v;
}

// Whether the previous round left a node undecided (round 0: whether there
// are nodes), for the whole block: the first wave reads the 64 counters of
// the round's parity with atomic loads (they were formed by atomics of
// other XCDs).
__device__ __forceinline__ bool mis_pending(const int* mc, int round, int* s_flag) {
  if (threadIdx.x < kMisSlots) {
    const int v = __hip_atomic_load(&mc[mis_word(round & 1, threadIdx.x)], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t any = __ballot(v != 0);
    if (threadIdx.x == 0) *s_flag = any != 0;
  }
  __syncthreads();
  return *s_flag != 0;
}

// Node groups of one MIS(2) sweep: grid of at most kMisBlocks blocks (a
// multiple of 8), each taking a contiguous run of node groups, so per-block
// flags stay few and no flag is written by more than one block.
constexpr int kMisBlocks = 2048;

// First max sweep of a round: M1_i = max(T_i, max_{j in N_i} T_j), G lanes per
// node.  A node whose M1 already holds an MIS tuple keeps it: two MIS(2) nodes
// never share a closed neighbourhood, so that maximum cannot change again.
// With a node list (late rounds), the sweep visits list[0 .. *count) instead
// of 0 .. n.
template <int G>
__global__ void __launch_bounds__(256) k_mis_sweep1(int n, const int* __restrict__ gptr,
                                                    const int* __restrict__ gcol,
                                                    const uint64_t* __restrict__ T,
                                                    uint64_t* __restrict__ M1, int* mc, int round,
                                                    const int* __restrict__ list, const int* __restrict__ count) {
  __shared__ int s_flag;
  // the counters of this round's second sweep start from zero (they last held
  // the previous round's counts, read by that round's sweeps only)
  if (blockIdx.x == 0 && threadIdx.x < kMisSlots)
    __hip_atomic_store(&mc[mis_word((round + 1) & 1, threadIdx.x)], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!mis_pending(mc, round, &s_flag)) return;   // nothing undecided
  constexpr int NPB = 256 / G;                // nodes per block step
  const int lane = threadIdx.x & (G - 1);
  const int m = list ? *count : n;
  const int groups = (m + NPB - 1) / NPB;
  const int per = (groups + gridDim.x - 1) / gridDim.x;
  const int g0 = xcd_block_index() * per, g1 = min(groups, g0 + per);
  for (int g = g0; g < g1; ++g) {
    const int q = g * NPB + threadIdx.x / G;
    const int i = q < m ? (list ? list[q] : q) : n;
    uint64_t t = 0;
    bool work = false;
    if (i < n) {
      const uint64_t prev = M1[i];
      work = tstate(prev) != 2;
      if (work) {
        if (lane == 0) t = T[i];
        for (int k = gptr[i] + lane; k < gptr[i + 1]; k += G) {
          uint64_t u = T[gcol[k]];
          t = u > t ? u : t;
        }
      }
    }
    t = group_max_u64<G>(t);
    if (work && lane == 0) M1[i] = t;
  }
}

// Second sweep plus the state update (undecided nodes only): a node whose
// distance-2 max is its own tuple joins the MIS; one that sees an MIS tuple
// leaves.  Each block records whether it left a node undecided.
template <int G>
__global__ void __launch_bounds__(256) k_mis_sweep2(int n, const int* __restrict__ gptr,
                                                    const int* __restrict__ gcol, uint64_t* __restrict__ T,
                                                    const uint64_t* __restrict__ M1, int* mc, int round,
                                                    const int* __restrict__ list, const int* __restrict__ count) {
  __shared__ int s_flag;
  if (!mis_pending(mc, round, &s_flag)) return;
  constexpr int NPB = 256 / G;
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  const int lane = threadIdx.x & (G - 1);
  const int m = list ? *count : n;
  const int groups = (m + NPB - 1) / NPB;
  const int per = (groups + gridDim.x - 1) / gridDim.x;
  const int g0 = xcd_block_index() * per, g1 = min(groups, g0 + per);
  int undecided = 0;
  for (int g = g0; g < g1; ++g) {
    const int q = g * NPB + threadIdx.x / G;
    const int i = q < m ? (list ? list[q] : q) : n;
    uint64_t own = 0, t = 0;
    if (i < n) {
      own = T[i];
      if (tstate(own) == 1) {
        if (lane == 0) t = M1[i];
        for (int k = gptr[i] + lane; k < gptr[i + 1]; k += G) {
          uint64_t u = M1[gcol[k]];
          t = u > t ? u : t;
        }
      }
    }
    t = group_max_u64<G>(t);
    if (i < n && lane == 0 && tstate(own) == 1) {
      if (t == own) {
        T[i] = (own & kLow62) | (2ull << 62);
      } else if (tstate(t) == 2) {
        T[i] = own & kLow62;
      } else {
        undecided = 1;
      }
    }
  }
  if (undecided) s_any = 1;   // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) {
    // spread over 64 counters in separate lines, so the blocks' atomics do
    // not queue on one address
    if (s_any)
      __hip_atomic_fetch_add(&mc[mis_word((round + 1) & 1, blockIdx.x % kMisSlots)], 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    if (blockIdx.x == 0) __hip_atomic_fetch_add(&mc[kMisRoundsWord], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// MIS(k), k > 2 (Section 2.1.2, aggressive coarsening): the sweeps between
// the first and the last of a round, out_i = max(in_i, max_{j in N_i} in_j),
// so after sweep d every node holds the largest tuple within distance d.
template <int G>
__global__ void __launch_bounds__(256) k_misk_sweep(int n, const int* __restrict__ gptr,
                                                    const int* __restrict__ gcol,
                                                    const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                    int* mc, int round) {
  __shared__ int s_flag;
  if (!mis_pending(mc, round, &s_flag)) return;
  constexpr int NPB = 256 / G;
  const int lane = threadIdx.x & (G - 1);
  const int groups = (n + NPB - 1) / NPB;
  const int per = (groups + gridDim.x - 1) / gridDim.x;
  const int g0 = xcd_block_index() * per, g1 = min(groups, g0 + per);
  for (int g = g0; g < g1; ++g) {
    const int i = g * NPB + threadIdx.x / G;
    uint64_t t = 0;
    if (i < n) {
      if (lane == 0) t = in[i];
      for (int k = gptr[i] + lane; k < gptr[i + 1]; k += G) {
        const uint64_t u = in[gcol[k]];
        t = u > t ? u : t;
      }
    }
    t = group_max_u64<G>(t);
    if (i < n && lane == 0) out[i] = t;
  }
}

// Late-round node list: the closed neighbourhoods of the undecided nodes.
// Only those nodes' first-sweep maxima are still read by an undecided node,
// and they include every node the second sweep can still change (the sweep
// skips the decided ones).  The flag array starts zeroed.
__global__ void k_mis_mark(int n, const int* __restrict__ gptr, const int* __restrict__ gcol,
                           const uint64_t* __restrict__ T, int* __restrict__ near) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || tstate(T[i]) != 1) return;
  near[i] = 1;
  for (int k = gptr[i]; k < gptr[i + 1]; ++k) near[gcol[k]] = 1;   // every writer stores 1
}
__global__ void k_compact(int n, const int* __restrict__ flag, const int* __restrict__ pos, int* __restrict__ list) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) list[pos[i]] = i;
}

__global__ void k_root_flags(int n, const uint64_t* __restrict__ T, int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = tstate(T[i]) == 2 ? 1 : 0;
}

// Largest tuple over a group's lanes, the first entry of the row among equal
// ones (the order a sequential scan of the row would keep).
template <int G>
__device__ __forceinline__ void group_argmax(uint64_t& best, int& bk, int& bj) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    const uint64_t ob = __shfl_xor(best, off, G);
    const int ok = __shfl_xor(bk, off, G);
    const int oj = __shfl_xor(bj, off, G);
    if (ob > best || (ob == best && ok < bk)) { best = ob; bk = ok; bj = oj; }
  }
}

// Round 1: roots take themselves; nodes next to roots take the adjacent root
// with the largest tuple.  G lanes per node.
template <int G>
__global__ void __launch_bounds__(256) k_agg_round1(int n, const int* __restrict__ gptr,
                                                    const int* __restrict__ gcol, const uint64_t* __restrict__ T,
                                                    int* __restrict__ choice) {
  RowGroup<G> rg;
  for (long i0 = rg.gid; i0 < n; i0 += rg.ngroups) {
    const int i = (int)i0;
    const uint64_t own = T[i];
    if (tstate(own) == 2) {
      if (rg.lane == 0) choice[i] = i;
      continue;
    }
    uint64_t best = 0;
    int bk = INT_MAX, bj = -1;
    const int e = gptr[i + 1];
    for (int k = gptr[i] + rg.lane; k < e; k += G) {
      const int j = gcol[k];
      const uint64_t u = T[j];
      if (tstate(u) == 2 && u > best) { best = u; bk = k; bj = j; }
    }
    group_argmax<G>(best, bk, bj);
    if (rg.lane == 0) choice[i] = bj;
  }
}

// Round 2: the remaining nodes (distance 2 from every root) take, among the
// roots chosen by their round-1 neighbours, the one with the largest tuple.
template <int G>
__global__ void __launch_bounds__(256) k_agg_round2(int n, const int* __restrict__ gptr,
                                                    const int* __restrict__ gcol, const uint64_t* __restrict__ T,
                                                    const int* __restrict__ choice,
                                                    const int* __restrict__ root_id, int* __restrict__ agg,
                                                    int* err) {
  RowGroup<G> rg;
  for (long i0 = rg.gid; i0 < n; i0 += rg.ngroups) {
    const int i = (int)i0;
    int c = choice[i];
    if (c < 0) {
      uint64_t best = 0;
      int bk = INT_MAX;
      const int e = gptr[i + 1];
      for (int k = gptr[i] + rg.lane; k < e; k += G) {
        const int cj = choice[gcol[k]];
        if (cj >= 0) {
          const uint64_t u = T[cj];
          if (u > best) { best = u; bk = k; c = cj; }
        }
      }
      group_argmax<G>(best, bk, c);
    }
    if (rg.lane != 0) continue;
    if (c < 0) {
      atomic_or_flag(err, kErrUnassigned);
      agg[i] = 0;
      continue;
    }
    agg[i] = root_id[c];
  }
}

// MIS(k) aggregation, rounds 2..k: a node still without a root takes, among
// the roots its neighbours chose in the previous round, the one with the
// largest tuple (a neighbour assigned at all was assigned in that round, one
// step nearer its root); the others keep their choice.  Double buffered.
template <int G>
__global__ void __launch_bounds__(256) k_agg_round_next(int n, const int* __restrict__ gptr,
                                                        const int* __restrict__ gcol,
                                                        const uint64_t* __restrict__ T,
                                                        const int* __restrict__ cin, int* __restrict__ cout) {
  RowGroup<G> rg;
  for (long i0 = rg.gid; i0 < n; i0 += rg.ngroups) {
    const int i = (int)i0;
    int c = cin[i];
    if (c < 0) {
      uint64_t best = 0;
      int bk = INT_MAX;
      const int e = gptr[i + 1];
      for (int k = gptr[i] + rg.lane; k < e; k += G) {
        const int cj = cin[gcol[k]];
        if (cj >= 0) {
          const uint64_t u = T[cj];
          if (u > best) { best = u; bk = k; c = cj; }
        }
      }
      group_argmax<G>(best, bk, c);
    }
    if (rg.lane == 0) cout[i] = c;
  }
}

// Coarse index of every node's root (an unassigned node is an error).
__global__ void k_agg_map(int n, const int* __restrict__ choice, const int* __restrict__ root_id,
                          int* __restrict__ agg, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = choice[i];
  if (c < 0) {
    atomic_or_flag(err, kErrUnassigned);
    agg[i] = 0;
    return;
  }
  agg[i] = root_id[c];
}

__global__ void k_agg_count(int n, const int* __restrict__ agg, int* counts) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && agg[i] >= 0) atomicAdd(&counts[agg[i]], 1);   // -1: row of a system not coarsened
}

__global__ void k_agg_scatter(int n, const int* __restrict__ agg, const int* __restrict__ agg_ptr,
                              int* fill, int* __restrict__ agg_rows) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int I = agg[i];
  if (I < 0) return;
  int pos = atomicAdd(&fill[I], 1);
  agg_rows[agg_ptr[I] + pos] = i;
}

__device__ void sift_down(int* a, int start, int end) {
  int root = start;
  while (2 * root + 1 <= end) {
    int child = 2 * root + 1;
    if (child + 1 <= end && a[child] < a[child + 1]) ++child;
    if (a[root] < a[child]) {
      int t = a[root]; a[root] = a[child]; a[child] = t;
      root = child;
    } else {
      return;
    }
  }
}

// Each aggregate's member list sorted ascending (atomics left it in arrival
// order).  A group of 32 lanes takes one aggregate: with at most 32 members
// every member finds its rank by counting the smaller ones (members are
// distinct), so the sort costs one load, one pass over LDS and one store per
// member; longer lists fall back to a heap sort by the group's first lane.
constexpr int kSortGroup = 32;
__global__ void __launch_bounds__(256) k_agg_sort(int nc, const int* __restrict__ agg_ptr,
                                                  int* __restrict__ agg_rows) {
  constexpr int NG = 256 / kSortGroup;
  __shared__ int sv[NG][kSortGroup];
  const int grp = threadIdx.x / kSortGroup, lane = threadIdx.x % kSortGroup;
  const int chunks = (nc + NG - 1) / NG;
  for (int c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int I = c * NG + grp;
    int m = 0, x = 0;
    int* a = nullptr;
    if (I < nc) {
      a = agg_rows + agg_ptr[I];
      m = agg_ptr[I + 1] - agg_ptr[I];
      if (m <= kSortGroup && lane < m) x = a[lane];
    }
    if (m <= kSortGroup && lane < m) sv[grp][lane] = x;
    __syncthreads();
    if (m <= kSortGroup) {
      if (lane < m) {
        int rank = 0;
        for (int q = 0; q < m; ++q) rank += sv[grp][q] < x;
        a[rank] = x;
      }
    } else if (lane == 0) {
      for (int start = (m - 2) / 2; start >= 0; --start) sift_down(a, start, m - 1);
      for (int end = m - 1; end > 0; --end) {
        int t = a[0]; a[0] = a[end]; a[end] = t;
        sift_down(a, 0, end - 1);
      }
    }
    __syncthreads();
  }
}

// Algorithm 3: B_{k+1}(I) = ||R_k(I,:)||_2 with R_k(I,i) = B_k(i), summed in
// ascending i; then P_k(i, I) = B_k(i) / B_{k+1}(I).
__global__ void k_interp_coarse(int nc, const int* __restrict__ agg_ptr, const int* __restrict__ agg_rows,
                                const double* __restrict__ B, double* __restrict__ Bc) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  double s = 0.0;
  for (int k = agg_ptr[I]; k < agg_ptr[I + 1]; ++k) {
    double b = B[agg_rows[k]];
    s = __dadd_rn(s, __dmul_rn(b, b));
  }
  Bc[I] = sqrt(s);
}

__global__ void k_interp_fine(int n, const int* __restrict__ agg, const double* __restrict__ B,
                              const double* __restrict__ Bc, double* __restrict__ pval) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pval[i] = agg[i] >= 0 ? B[i] / Bc[agg[i]] : 0.0;
}

__global__ void k_node_hash(int n, uint32_t stream, uint32_t* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = node_hash((uint32_t)i, stream);
}

__global__ void k_jacobi_weights(int n, double omega, const double* __restrict__ diag,
                                 double* __restrict__ wdinv, float* __restrict__ wdinv32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double w = omega / diag[i];
  wdinv[i] = w;
  if (wdinv32) wdinv32[i] = (float)w;
}

__global__ void k_to_float(size_t n, const double* __restrict__ in, float* __restrict__ out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = (float)in[i];
}

__global__ void k_state_from_tuple(int n, const uint64_t* __restrict__ T, int8_t* __restrict__ st) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) st[i] = (int8_t)(tstate(T[i]) - 1);
}

// Sliced ELL: slice width = longest row of its 64 rows (one wave per slice).
// Per slice of H slots, H x its longest row (the slice's element count); slot
// i holds row perm[i] (perm null: row i).
template <int H>
__global__ void k_sell_widths(int n, int nsl, const int* __restrict__ rp, const int* __restrict__ perm,
                              int* __restrict__ widths) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = perm && slot < nsl * H ? perm[slot] : slot;
  int len = row < n ? rp[row + 1] - rp[row] : 0;
#pragma unroll
  for (int off = H / 2; off > 0; off >>= 1) {
    const int o = __shfl_xor(len, off, kWave);
    len = o > len ? o : len;
  }
  if ((threadIdx.x & (H - 1)) == 0 && slot / H < nsl) widths[slot / H] = len * H;
}

// Sliced diagonals, one wave per 64-row slice: the distinct offsets col - row
// of the slice's rows in ascending order, found by merging (each lane walks
// its row's sorted columns; the wave minimum of the lanes' next offsets is
// the next diagonal, and the lanes holding it step past it).  COUNT: their
// number per slice into cnt, *over raised when a slice has more than cap.
// FILL: the offsets and values at the positions of dg_ptr (zero where a row
// has no entry on a diagonal); the same pass refreshes the values when A's
// values change on the same pattern.
template <bool FILL>
__global__ void __launch_bounds__(256) k_sdia_build(int n, int nslices, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const double* __restrict__ val,
                                                    int cap, int* __restrict__ cnt, const int* __restrict__ dg_ptr,
                                                    int* __restrict__ dg_off, double* __restrict__ dg_val,
                                                    float* __restrict__ dg_val32, int* __restrict__ over) {
  const int sl = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  if (sl >= nslices) return;   // the whole wave
  const int lane = threadIdx.x & (kWave - 1);
  const int row = sl * kWave + lane;
  int e = row < n ? rp[row] : 0;
  const int end = row < n ? rp[row + 1] : 0;
  const int base = FILL ? dg_ptr[sl] : 0;
  int q = 0;
  while (true) {
    const int mine = e < end ? ci[e] - row : INT_MAX;
    int d = mine;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      const int o = __shfl_xor(d, off, kWave);
      d = o < d ? o : d;
    }
    if (d == INT_MAX) break;
    if (!FILL && q == cap) {
      if (lane == 0) atomicOr(over, 1);
      break;
    }
    if (FILL) {
      if (lane == 0) dg_off[base + q] = d;
      const double v = mine == d ? val[e] : 0.0;
      const size_t idx = (size_t)(base + q) * kWave + lane;
      dg_val[idx] = v;
      if (dg_val32) dg_val32[idx] = (float)v;
    }
    if (mine == d) ++e;
    ++q;
  }
  if (!FILL && lane == 0) cnt[sl] = q;
}

// The row order of the copies in shorter slices: within each window of 256
// rows, rows by decreasing length (ties by index), a bitonic sort of
// (length, index) keys in LDS.  perm has a whole number of windows; its slots
// past n get indices >= n (padding).
constexpr int kOrderWindow = 64;
__global__ void __launch_bounds__(256) k_window_order(int n, const int* __restrict__ rp, int* __restrict__ perm) {
  __shared__ uint32_t key[256];
  const int t = threadIdx.x;
  const int w0 = blockIdx.x * 256;
  const int row = w0 + t;
  const int len = row < n ? rp[row + 1] - rp[row] : 0;
  // longer rows first; rows past n (length key 0xFFFF) last
  const uint32_t lk = row < n ? 0xFFFEu - (uint32_t)min(len, 0xFFFE) : 0xFFFFu;
  key[t] = (lk << 16) | (uint32_t)t;   // t: the index in the block; windows sort within themselves
  for (int k = 2; k <= kOrderWindow; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      const int p = t ^ j;
      if (p > t) {
        const uint32_t a = key[t], b = key[p];
        const bool up = k == kOrderWindow || (t & k) == 0;   // every window ends ascending
        if ((a > b) == up) {
          key[t] = b;
          key[p] = a;
        }
      }
    }
  }
  __syncthreads();
  perm[w0 + t] = w0 + (int)(key[t] & 0xFFFFu);
}

// Fill the slices: entry k of the row in slot s*H+l at sl_ptr[s] + H k + l;
// padding (short rows and the slots past n) has value 0 and a valid column
// (the row itself, or n - 1 past the end).  sl_dcol (may be null)
// holds col - row in 16 bits; an offset that does not fit raises *wide (the
// 16-bit copy is then unusable).
template <int H>
__global__ void k_sell_fill(int n, int nslices, const int* __restrict__ rp, const int* __restrict__ ci,
                            const double* __restrict__ val, const int* __restrict__ sl_ptr,
                            const int* __restrict__ perm, int* __restrict__ sl_col, int16_t* __restrict__ sl_dcol,
                            int* __restrict__ wide, double* __restrict__ sl_val, float* __restrict__ sl_val32) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = slot / H, l = slot & (H - 1);
  if (sl >= nslices) return;
  const int row = perm ? perm[slot] : slot;
  const int base = sl_ptr[sl];
  const int w = (sl_ptr[sl + 1] - base) / H;
  const int s0 = row < n ? rp[row] : 0;
  const int len = row < n ? rp[row + 1] - s0 : 0;
  bool fits = true;
  for (int k = 0; k < w; ++k) {
    const int idx = base + k * H + l;
    int c = row < n ? row : n - 1;
    double v = 0.0;
    if (k < len) { c = ci[s0 + k]; v = val[s0 + k]; }
    sl_col[idx] = c;
    const int d = c - row;
    fits = fits && d >= -32768 && d <= 32767;
    if (sl_dcol) sl_dcol[idx] = (int16_t)d;
    sl_val[idx] = v;
    if (sl_val32) sl_val32[idx] = (float)v;
  }
  if (!fits && wide) atomicOr(wide, 1);
}

__global__ void k_gather_double(int m, const int* __restrict__ idx, const double* __restrict__ src,
                                double* __restrict__ dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) dst[k] = src[idx[k]];
}

__global__ void k_fill_double(size_t n, double* p, double v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_int(size_t n, int* p, int v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}
// Values the host waits for, written straight into its pinned mirror: one
// launch replaces a copy per value.  Wave w reads item w (its count values
// spread over the lanes); slot 63 receives the error word.
__global__ void __launch_bounds__(512) k_mailbox(Mailbox m, const int* __restrict__ err, int* host) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (w < m.n) {
    int v = 0;
    for (int c = lane; c < m.count[w]; c += kWave)
      v += __hip_atomic_load(m.src[w] + (size_t)c * m.stride[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (lane == 0) host[m.slot[w]] = v;
  }
  if (threadIdx.x == 0) host[63] = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
}  // namespace

void launch_check_rowptr(int n, const int* rp, int* err, hipStream_t s) {
  k_check_rowptr<<<grid_for(n), kT, 0, s>>>(n, rp, err);
}
void launch_check_index(int n, const int* idx, int limit, int* err, hipStream_t s) {
  k_check_index<<<grid_for(n), kT, 0, s>>>(n, idx, limit, err);
}
void launch_check_matrix(int n, const int* rp, const int* ci, const double* val, int* err, hipStream_t s) {
  k_check_matrix<<<grid_for(n), kT, 0, s>>>(n, rp, ci, val, err);
}
void launch_mailbox(const Mailbox& m, const int* err, int* host, hipStream_t s) {
  k_mailbox<<<1, 512, 0, s>>>(m, err, host);
}

int group_lanes(int n, long entries) {
  int g = 1;
  while (g < 32 && 4L * g * n < entries) g <<= 1;
  while (g < 32 && (long)g * n < (1L << 19)) g <<= 1;
  return g;
}


void launch_strength(int n, int nnz, const int* rp, const int* ci, const double* val, double alpha,
                     uint8_t* strong, double* diag, hipStream_t s) {
  if (n <= 0) return;
  const int G = group_lanes(n, nnz);
  with_lanes(G, [&](auto g) {
    k_strength<decltype(g)::value><<<group_grid(n, G), kT, 0, s>>>(n, rp, ci, val, alpha, strong, diag);
  });
}
void launch_graph_count(int n, int nnz, const int* rp, const int* ci, const uint8_t* strong, uint8_t* gmask,
                        int* gdeg, int* cnt, int* err, hipStream_t s) {
  if (n <= 0) return;
  const int G = group_lanes(n, nnz);
  with_lanes(G, [&](auto g) {
    k_graph_count<decltype(g)::value><<<group_grid(n, G), kT, 0, s>>>(n, rp, ci, strong, gmask, gdeg, cnt, err);
  });
}
void launch_graph_fill(int n, int nnz, const int* rp, const int* ci, const uint8_t* gmask, const int* gptr,
                       int* gcol, hipStream_t s) {
  if (n <= 0) return;
  const int G = group_lanes(n, nnz);
  with_lanes(G, [&](auto g) {
    k_graph_fill<decltype(g)::value><<<group_grid(n, G), kT, 0, s>>>(n, rp, ci, gmask, gptr, gcol);
  });
}
void launch_mis_init(int n, const int* cnt, uint32_t seed, uint64_t* T, uint64_t* M1, int* mc, int* err,
                     hipStream_t s, const int* lbase) {
  k_mis_init<<<grid_for(n > 2 * kMisSlots ? n : 2 * kMisSlots), kT, 0, s>>>(n, cnt, seed, T, M1, mc, err, lbase);
}
template <int G>
static void mis_round_g(int n, const int* gptr, const int* gcol, uint64_t* T, uint64_t* M1, int* mc, int round,
                        const MisLists* ml, hipStream_t s) {
  long g = ((long)n * G + kT - 1) / kT;
  if (g < 1) g = 1;
  if (g > kMisBlocks) g = kMisBlocks;
  if (ml) {   // the lists hold a few percent of the nodes
    long gl = g / 8;
    g = gl < 8 ? 8 : gl;
  }
  k_mis_sweep1<G><<<(int)g, kT, 0, s>>>(n, gptr, gcol, T, M1, mc, round, ml ? ml->near : nullptr,
                                        ml ? ml->count : nullptr);
  k_mis_sweep2<G><<<(int)g, kT, 0, s>>>(n, gptr, gcol, T, M1, mc, round, ml ? ml->near : nullptr,
                                        ml ? ml->count : nullptr);
}

void launch_mis_round(int n, const int* gptr, const int* gcol, uint64_t* T, uint64_t* M1, int* mc,
                      int round, int lanes, hipStream_t s, const MisLists* ml) {
  switch (lanes) {
    case 1: mis_round_g<1>(n, gptr, gcol, T, M1, mc, round, ml, s); break;
    case 2: mis_round_g<2>(n, gptr, gcol, T, M1, mc, round, ml, s); break;
    case 4: mis_round_g<4>(n, gptr, gcol, T, M1, mc, round, ml, s); break;
    case 8: mis_round_g<8>(n, gptr, gcol, T, M1, mc, round, ml, s); break;
    case 16: mis_round_g<16>(n, gptr, gcol, T, M1, mc, round, ml, s); break;
    default: mis_round_g<32>(n, gptr, gcol, T, M1, mc, round, ml, s); break;
  }
}

// One MIS(k) round for k > 2: the first sweep (distance-1 maxima into M1,
// settled ones kept), k - 2 plain sweeps alternating between Ma and Mb, and
// the last sweep with the state update.
template <int G>
static void misk_round_g(int n, const int* gptr, const int* gcol, uint64_t* T, uint64_t* M1, uint64_t* Ma,
                         uint64_t* Mb, int* mc, int round, int k, hipStream_t s) {
  long g = ((long)n * G + kT - 1) / kT;
  if (g < 1) g = 1;
  if (g > kMisBlocks) g = kMisBlocks;
  k_mis_sweep1<G><<<(int)g, kT, 0, s>>>(n, gptr, gcol, T, M1, mc, round, nullptr, nullptr);
  const uint64_t* in = M1;
  for (int d = 2; d < k; ++d) {
    uint64_t* out = (d & 1) ? Mb : Ma;
    k_misk_sweep<G><<<(int)g, kT, 0, s>>>(n, gptr, gcol, in, out, mc, round);
    in = out;
  }
  k_mis_sweep2<G><<<(int)g, kT, 0, s>>>(n, gptr, gcol, T, in, mc, round, nullptr, nullptr);
}

void launch_misk_round(int n, const int* gptr, const int* gcol, uint64_t* T, uint64_t* M1, uint64_t* Ma,
                       uint64_t* Mb, int* mc, int round, int k, int lanes, hipStream_t s) {
  switch (lanes) {
    case 1: misk_round_g<1>(n, gptr, gcol, T, M1, Ma, Mb, mc, round, k, s); break;
    case 2: misk_round_g<2>(n, gptr, gcol, T, M1, Ma, Mb, mc, round, k, s); break;
    case 4: misk_round_g<4>(n, gptr, gcol, T, M1, Ma, Mb, mc, round, k, s); break;
    case 8: misk_round_g<8>(n, gptr, gcol, T, M1, Ma, Mb, mc, round, k, s); break;
    case 16: misk_round_g<16>(n, gptr, gcol, T, M1, Ma, Mb, mc, round, k, s); break;
    default: misk_round_g<32>(n, gptr, gcol, T, M1, Ma, Mb, mc, round, k, s); break;
  }
}

void launch_mis_lists(int n, const int* gptr, const int* gcol, const uint64_t* T, const MisLists& ml,
                      ScanCtx& sc, hipStream_t s) {
  launch_fill_int((size_t)n, ml.fnear, 0, s);
  k_mis_mark<<<grid_for(n), kT, 0, s>>>(n, gptr, gcol, T, ml.fnear);
  scan_to_ptr(ml.fnear, ml.pnear, n, sc, s);
  k_compact<<<grid_for(n), kT, 0, s>>>(n, ml.fnear, ml.pnear, ml.near);
}
void launch_root_flags(int n, const uint64_t* T, int* flags, hipStream_t s) {
  k_root_flags<<<grid_for(n), kT, 0, s>>>(n, T, flags);
}
void launch_aggregate(int n, int nnzg, const int* gptr, const int* gcol, const uint64_t* T, const int* root_id,
                      int* choice, int* agg, int* err, hipStream_t s) {
  if (n <= 0) return;
  const int G = group_lanes(n, nnzg);
  with_lanes(G, [&](auto g) {
    constexpr int L = decltype(g)::value;
    k_agg_round1<L><<<group_grid(n, G), kT, 0, s>>>(n, gptr, gcol, T, choice);
    k_agg_round2<L><<<group_grid(n, G), kT, 0, s>>>(n, gptr, gcol, T, choice, root_id, agg, err);
  });
}
void launch_aggregate_k(int n, int nnzg, const int* gptr, const int* gcol, const uint64_t* T, const int* root_id,
                        int k, int* choice, int* choice2, int* agg, int* err, hipStream_t s) {
  if (n <= 0) return;
  const int G = group_lanes(n, nnzg);
  with_lanes(G, [&](auto g) {
    constexpr int L = decltype(g)::value;
    k_agg_round1<L><<<group_grid(n, G), kT, 0, s>>>(n, gptr, gcol, T, choice);
    int* in = choice;
    int* out = choice2;
    for (int r = 2; r <= k; ++r) {
      k_agg_round_next<L><<<group_grid(n, G), kT, 0, s>>>(n, gptr, gcol, T, in, out);
      int* t = in;
      in = out;
      out = t;
    }
    k_agg_map<<<grid_for(n), kT, 0, s>>>(n, in, root_id, agg, err);
  });
}
void launch_agg_count(int n, const int* agg, int* counts, hipStream_t s) {
  k_agg_count<<<grid_for(n), kT, 0, s>>>(n, agg, counts);
}
void launch_agg_scatter(int n, const int* agg, const int* agg_ptr, int* fill, int* agg_rows, hipStream_t s) {
  k_agg_scatter<<<grid_for(n), kT, 0, s>>>(n, agg, agg_ptr, fill, agg_rows);
}
void launch_agg_sort(int nc, const int* agg_ptr, int* agg_rows, hipStream_t s) {
  if (nc <= 0) return;
  long g = (nc + 7) / 8;
  if (g > 8192) g = 8192;
  k_agg_sort<<<(int)g, 256, 0, s>>>(nc, agg_ptr, agg_rows);
}
void launch_interp(int n, int nc, const int* agg, const int* agg_ptr, const int* agg_rows,
                   const double* B, double* Bc, double* pval, hipStream_t s) {
  k_interp_coarse<<<grid_for(nc), kT, 0, s>>>(nc, agg_ptr, agg_rows, B, Bc);
  k_interp_fine<<<grid_for(n), kT, 0, s>>>(n, agg, B, Bc, pval);
}
void launch_node_hash(int n, uint32_t stream, uint32_t* out, hipStream_t s) {
  if (n > 0) k_node_hash<<<grid_for(n), kT, 0, s>>>(n, stream, out);
}
void launch_jacobi_weights(int n, double omega, const double* diag, double* wdinv, float* wdinv32,
                           hipStream_t s) {
  k_jacobi_weights<<<grid_for(n), kT, 0, s>>>(n, omega, diag, wdinv, wdinv32);
}
void launch_to_float(size_t n, const double* in, float* out, hipStream_t s) {
  if (n == 0) return;
  long g = (long)((n + kT - 1) / kT);
  k_to_float<<<(int)(g < 8192 ? g : 8192), kT, 0, s>>>(n, in, out);
}
void launch_state_from_tuple(int n, const uint64_t* T, int8_t* state, hipStream_t s) {
  k_state_from_tuple<<<grid_for(n), kT, 0, s>>>(n, T, state);
}
void launch_fill_int(size_t n, int* p, int v, hipStream_t s) {
  if (n == 0) return;
  long g = (long)((n + kT - 1) / kT);
  k_fill_int<<<(int)(g < 8192 ? g : 8192), kT, 0, s>>>(n, p, v);
}

void launch_sell_widths(int n, const int* rp, int* widths, hipStream_t s, int slice_h, const int* perm) {
  const int nsl = (n + slice_h - 1) / slice_h;
  const int g = (int)(((long)nsl * slice_h + kT - 1) / kT);
  if (slice_h == 32) k_sell_widths<32><<<g, kT, 0, s>>>(n, nsl, rp, perm, widths);
  else if (slice_h == 16) k_sell_widths<16><<<g, kT, 0, s>>>(n, nsl, rp, perm, widths);
  else k_sell_widths<64><<<g, kT, 0, s>>>(n, nsl, rp, perm, widths);
}
void launch_sell_fill(int n, int nslices, const int* rp, const int* ci, const double* val, const int* sl_ptr,
                      int* sl_col, int16_t* sl_dcol, int* wide, double* sl_val, float* sl_val32, hipStream_t s,
                      int slice_h, const int* perm) {
  const int g = (int)(((long)nslices * slice_h + kT - 1) / kT);
  if (slice_h == 32)
    k_sell_fill<32><<<g, kT, 0, s>>>(n, nslices, rp, ci, val, sl_ptr, perm, sl_col, sl_dcol, wide, sl_val,
                                     sl_val32);
  else if (slice_h == 16)
    k_sell_fill<16><<<g, kT, 0, s>>>(n, nslices, rp, ci, val, sl_ptr, perm, sl_col, sl_dcol, wide, sl_val,
                                     sl_val32);
  else
    k_sell_fill<64><<<g, kT, 0, s>>>(n, nslices, rp, ci, val, sl_ptr, perm, sl_col, sl_dcol, wide, sl_val,
                                     sl_val32);
}
void launch_sdia_count(int n, const int* rp, const int* ci, int cap, int* cnt, int* over, hipStream_t s) {
  const int nsl = (n + kWave - 1) / kWave;
  const int g = (int)(((long)nsl * kWave + 255) / 256);
  if (nsl > 0)
    k_sdia_build<false><<<g, 256, 0, s>>>(n, nsl, rp, ci, nullptr, cap, cnt, nullptr, nullptr, nullptr, nullptr,
                                          over);
}
void launch_sdia_fill(int n, const int* rp, const int* ci, const double* val, const int* dg_ptr, int* dg_off,
                      double* dg_val, float* dg_val32, hipStream_t s) {
  const int nsl = (n + kWave - 1) / kWave;
  const int g = (int)(((long)nsl * kWave + 255) / 256);
  if (nsl > 0)
    k_sdia_build<true><<<g, 256, 0, s>>>(n, nsl, rp, ci, val, 0, nullptr, dg_ptr, dg_off, dg_val, dg_val32,
                                         nullptr);
}
// the CSR columns as 16-bit offsets, one thread per row
__global__ void k_ci16(int n, const int* __restrict__ rp, const int* __restrict__ ci, int16_t* __restrict__ ci16) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    for (int k = rp[i]; k < rp[i + 1]; ++k) ci16[k] = (int16_t)(ci[k] - i);
}
void launch_ci16(int n, const int* rp, const int* ci, int16_t* ci16, hipStream_t s) {
  if (n > 0) k_ci16<<<grid_for(n), kT, 0, s>>>(n, rp, ci, ci16);
}
void launch_window_order(int n, const int* rp, int* perm, hipStream_t s) {
  if (n > 0) k_window_order<<<(n + 255) / 256, 256, 0, s>>>(n, rp, perm);
}
void launch_gather_double(int m, const int* idx, const double* src, double* dst, hipStream_t s) {
  if (m > 0) k_gather_double<<<grid_for(m), kT, 0, s>>>(m, idx, src, dst);
}
void launch_fill_double(size_t n, double* p, double v, hipStream_t s) {
  if (n == 0) return;
  long g = (long)((n + kT - 1) / kT);
  k_fill_double<<<(int)(g < 8192 ? g : 8192), kT, 0, s>>>(n, p, v);
}

}  // namespace amg
