// Galerkin product by aggregate index (Section 3.1, eq. galerkin):
//   (A_{k+1})_IJ = sum_{i in G_I} sum_{j in G_J} P_iI A_ij P_jJ.
// Instead of a global sort of all (I, J) tuples, each coarse row I is built
// from its own aggregate segment G_I, in four steps:
//   1. term offsets: the entries of the fine rows, taken in segment order
//      (aggregate by aggregate, members ascending, entries in column order),
//      are numbered by a scan of the row lengths;
//   2. the terms: every entry (i, j) of a member row is the term
//      (J = agg(j), (P_iI a_ij) P_jJ) with its number in segment order; the
//      first reduce pass forms the terms of its rows itself, from A, and
//      writes those of wider rows to their numbered places;
//   3. reduce: one wave per coarse row holds the row's terms in registers,
//      finds the distinct J with an LDS hash, places every term after the
//      earlier terms of the same J (ballot peeling within a chunk of 64), and
//      sums each J's terms in segment order; the sorted (J, sum) pairs
//      overwrite the head of the row's term range;
//   4. a scan of the distinct counts makes the row pointers and a copy
//      compacts the rows.
// Each coarse entry is the sum of its terms in segment order, so the result
// does not depend on timing.  Rows with more terms than a wave holds go to a
// wider wave, and the rare rows beyond that to a block-per-row extraction.
#include <climits>

#include "amg_internal.hpp"
#include "device_utils.hpp"

namespace amg {

namespace {
constexpr int kBig = 256;        // threads per block on the extraction path
constexpr int kSmallC = 2;       // terms per lane of the first reduce pass
constexpr int kWideC = 8;        // terms per lane of the second
constexpr int kMaxWaveTerms = kWave * kWideC;

// Step 1: number of terms of the k-th fine row in segment order (0 beyond the
// rows that belong to an aggregate).
__global__ void k_gal_lens(int n, const int* __restrict__ rp, const int* __restrict__ agg_ptr, int nc,
                           const int* __restrict__ agg_rows, int* __restrict__ lens) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int len = 0;
  if (k < agg_ptr[nc]) {
    const int i = agg_rows[k];
    len = rp[i + 1] - rp[i];
  }
  lens[k] = len;
}

// The fine side of a direct reduce: A's rows, the aggregates and P.
struct GalFine {
  const int* rp;
  const int* ci;
  const double* val;
  const int* agg;
  const double* pval;
  const int* agg_rows;
};

// Step 3 for rows of at most 64*C terms, one wave per row (HS hash slots).
// Rows with more terms are appended to out_list.  DIRECT: the wave forms its
// row's terms itself from A (term t of the row: the member k whose term range
// holds t, found by binary search over the members' offsets staged in LDS,
// then its entry), instead of reading them from an expand pass; a row with
// more terms writes its terms to its range for the wider passes.  The terms,
// their order and their sums are those of the expand pass.
template <int C, bool LISTED, bool DIRECT = false>
__global__ void __launch_bounds__(kWave) k_gal_reduce(int nc, const int* __restrict__ agg_ptr,
                                                      const int* __restrict__ toff, int* __restrict__ tkey,
                                                      double* __restrict__ tval, int* __restrict__ ucount,
                                                      const int* __restrict__ in_list,
                                                      const int* __restrict__ in_count, int* __restrict__ out_list,
                                                      int* __restrict__ out_count, GalFine fine) {
  constexpr int CAP = kWave * C;
  constexpr int HS = CAP;   // U <= CAP, so linear probing always ends
  constexpr int HB = C == 1 ? 6 : C == 2 ? 7 : C == 4 ? 8 : C == 8 ? 9 : 10;
  static_assert((1 << HB) == HS, "C must be a power of two up to 16");
  __shared__ int hkey[HS], hcnt[HS], hrun[HS], hrank[HS];
  __shared__ int ukey[CAP], skey[CAP], sbase[CAP + 1];
  __shared__ double sv[CAP];
  __shared__ int moff[DIRECT ? CAP + 1 : 1];
  const int lane = threadIdx.x;
  const uint64_t below = (1ull << lane) - 1;
  const int count = LISTED ? *in_count : nc;
  for (int idx = xcd_block_index(); idx < count; idx += gridDim.x) {
    const int I = LISTED ? in_list[idx] : idx;
    const int m0 = agg_ptr[I], m1 = agg_ptr[I + 1];
    const int t0 = toff[m0];
    const int T = toff[m1] - t0;
    // term t (0 <= t < T, segment order) of a direct row: (J, (P_i a_ij) P_j)
    auto term = [&](int t, int& Jt, double& Vt) {
      int lo = 0, hi = m1 - m0 - 1;   // the last member whose range starts at or before t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (moff[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
      const int i = fine.agg_rows[m0 + lo];
      const int x = fine.rp[i] + (t - moff[lo]);
      const int j = fine.ci[x];
      Jt = fine.agg[j];
      Vt = __dmul_rn(__dmul_rn(fine.pval[i], fine.val[x]), fine.pval[j]);
    };
    if (DIRECT) {   // the members' term offsets, relative to the row
      if (T > CAP) {
        // a wide row: its members may exceed the LDS stage; expand by member
        for (int k = m0; k < m1; ++k) {
          const int i = fine.agg_rows[k];
          const int s0 = fine.rp[i], o = toff[k] - s0;
          const double pi = fine.pval[i];
          for (int x = s0 + lane; x < fine.rp[i + 1]; x += kWave) {
            const int j = fine.ci[x];
            tkey[o + x] = fine.agg[j];
            tval[o + x] = __dmul_rn(__dmul_rn(pi, fine.val[x]), fine.pval[j]);
          }
        }
      } else {
        for (int q = lane; q < m1 - m0; q += kWave) moff[q] = toff[m0 + q] - t0;
      }
      __syncthreads();
    }
    if (T > CAP) {
      if (lane == 0) out_list[atomicAdd(out_count, 1)] = I;
      continue;
    }
    for (int q = lane; q < HS; q += kWave) { hkey[q] = -1; hcnt[q] = 0; hrun[q] = 0; }
    int J[C], Q[C];
    double V[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = c * kWave + lane;
      J[c] = -1; Q[c] = 0; V[c] = 0.0;
      if (t < T) {
        if (DIRECT) term(t, J[c], V[c]);
        else { J[c] = tkey[t0 + t]; V[c] = tval[t0 + t]; }
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (c * kWave + lane < T) {
        int q = (int)(((uint32_t)J[c] * 0x9E3779B1u) >> (32 - HB));
        while (true) {
          const int prev = atomicCAS(&hkey[q], -1, J[c]);
          if (prev == -1 || prev == J[c]) break;
          q = q + 1 == HS ? 0 : q + 1;
        }
        atomicAdd(&hcnt[q], 1);
        Q[c] = q;
      }
    }
    __syncthreads();
    // the occupied slots, in slot order
    int U = 0;
    for (int base = 0; base < HS; base += kWave) {
      const int q = base + lane;
      const bool occ = hkey[q] != -1;
      const uint64_t bits = __ballot(occ);
      if (occ) ukey[U + __popcll(bits & below)] = q;
      U += __popcll(bits);
    }
    __syncthreads();
    // rank of every distinct J (they are distinct, so ranks are a permutation)
    for (int u = lane; u < U; u += kWave) {
      const int q = ukey[u], key = hkey[q];
      int r = 0;
      for (int v = 0; v < U; ++v) r += hkey[ukey[v]] < key;
      hrank[q] = r;
      skey[r] = key;
      sbase[r] = hcnt[q];
    }
    __syncthreads();
    // exclusive scan of the per-J term counts, in rank order
    int run = 0;
    for (int base = 0; base < U; base += kWave) {
      const int r = base + lane;
      const int v = r < U ? sbase[r] : 0;
      int incl = v;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += t;
      }
      __syncthreads();
      if (r < U) sbase[r] = run + incl - v;
      run += __shfl(incl, kWave - 1, kWave);
      __syncthreads();
    }
    if (lane == 0) sbase[U] = run;
    // place the terms: within a J, in segment order
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (c * kWave >= T) break;
      const bool act = c * kWave + lane < T;
      const int q = Q[c];
      uint64_t rem = __ballot(act);
      int before = 0, lead_add = 0;
      while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int ql = __shfl(q, leader, kWave);
        const uint64_t m = __ballot(act && q == ql);
        if (act && q == ql) before = __popcll(m & below);
        if (lane == leader) lead_add = __popcll(m);
        rem &= ~m;
      }
      if (act) sv[sbase[hrank[q]] + hrun[q] + before] = V[c];
      __syncthreads();
      if (lead_add) hrun[q] += lead_add;
      __syncthreads();
    }
    // sums in segment order; sorted pairs over the head of the term range
    for (int r = lane; r < U; r += kWave) {
      double s = 0.0;
      for (int x = sbase[r]; x < sbase[r + 1]; ++x) s = __dadd_rn(s, sv[x]);
      tkey[t0 + r] = skey[r];
      tval[t0 + r] = s;
    }
    if (lane == 0) ucount[I] = U;
    __syncthreads();
  }
}

__device__ __forceinline__ int block_min_int(int v, int* red) {
  for (int off = kWave / 2; off > 0; off >>= 1) {
    int o = __shfl_xor(v, off, kWave);
    v = o < v ? o : v;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  int r = red[0];
  for (int w = 1; w < kBig / kWave; ++w) r = red[w] < r ? red[w] : r;
  __syncthreads();
  return r;
}

// Rows beyond the widest wave: repeatedly take the smallest J above the last
// one over the row's terms, then sum its terms (fixed thread assignment and
// reduction order).  The count pass runs before the row pointers exist, the
// fill pass writes the final row directly.
template <bool FILL>
__global__ void __launch_bounds__(kBig) k_gal_big(const int* __restrict__ agg_ptr, const int* __restrict__ toff,
                                                  const int* __restrict__ tkey, const double* __restrict__ tval,
                                                  int* __restrict__ ucount, const int* __restrict__ ovf_list,
                                                  const int* __restrict__ ovf_count, const int* __restrict__ rp_c,
                                                  int* __restrict__ ci_c, double* __restrict__ val_c) {
  __shared__ int ired[kBig / kWave];
  __shared__ double dred[kBig / kWave];
  const int count = *ovf_count;
  for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int I = ovf_list[idx];
    const int t0 = toff[agg_ptr[I]], t1 = toff[agg_ptr[I + 1]];
    const int out0 = FILL ? rp_c[I] : 0;
    int last = -1, U = 0;
    while (true) {
      int mn = INT_MAX;
      for (int t = t0 + threadIdx.x; t < t1; t += kBig) {
        const int key = tkey[t];
        if (key > last && key < mn) mn = key;
      }
      mn = block_min_int(mn, ired);
      if (mn == INT_MAX) break;
      if (FILL) {
        double s = 0.0;
        for (int t = t0 + threadIdx.x; t < t1; t += kBig)
          if (tkey[t] == mn) s = __dadd_rn(s, tval[t]);
        double v[1] = {s};
        block_sum<1>(v, dred);
        if (threadIdx.x == 0) {
          ci_c[out0 + U] = mn;
          val_c[out0 + U] = v[0];
        }
      }
      ++U;
      last = mn;
    }
    if (!FILL && threadIdx.x == 0) ucount[I] = U;
    __syncthreads();
  }
}

// Step 4: rows reduced in place move to their final position (rows beyond
// the widest wave were written by the extraction path).
template <int G>
__global__ void __launch_bounds__(256) k_gal_compact(int nc, const int* __restrict__ agg_ptr,
                                                     const int* __restrict__ toff, const int* __restrict__ tkey,
                                                     const double* __restrict__ tval, const int* __restrict__ rp_c,
                                                     int* __restrict__ ci_c, double* __restrict__ val_c) {
  RowGroup<G> rg;
  for (long I0 = rg.gid; I0 < nc; I0 += rg.ngroups) {
    const int I = (int)I0;
    const int t0 = toff[agg_ptr[I]];
    if (toff[agg_ptr[I + 1]] - t0 > kMaxWaveTerms) continue;
    const int o = rp_c[I], U = rp_c[I + 1] - o;
    for (int u = rg.lane; u < U; u += G) {
      ci_c[o + u] = tkey[t0 + u];
      val_c[o + u] = tval[t0 + u];
    }
  }
}
}  // namespace

// Steps 1-3: on return ucount[I] holds the number of distinct J of every row.
void launch_galerkin_stage(const GalerkinScratch& g, int n, int nc, int nnz, const int* rp, const int* ci,
                           const double* val, const int* agg, const double* pval, const int* agg_ptr,
                           const int* agg_rows, ScanCtx& sc, hipStream_t s) {
  if (nc <= 0) return;
  k_gal_lens<<<(n + 255) / 256 > 0 ? (n + 255) / 256 : 1, 256, 0, s>>>(n, rp, agg_ptr, nc, agg_rows, g.lens);
  scan_to_ptr(g.lens, g.toff, n, sc, s);
  const GalFine fine{rp, ci, val, agg, pval, agg_rows};
  int* list1 = g.list;
  int* list2 = g.list + nc;
  launch_fill_int(2, g.ctl, 0, s);
  // the small-row reduce forms its rows' terms from A and writes the terms of
  // wider rows for the passes below (before: a separate expand pass over A,
  // 0.53 ms on C3's level 0, and 0.41 ms of reduce)
  (void)nnz;
  k_gal_reduce<kSmallC, false, true><<<nc, kWave, 0, s>>>(nc, agg_ptr, g.toff, g.tkey, g.tval, g.ucount, nullptr,
                                                          nullptr, list1, g.ctl, fine);
  k_gal_reduce<kWideC, true><<<2048, kWave, 0, s>>>(nc, agg_ptr, g.toff, g.tkey, g.tval, g.ucount, list1, g.ctl,
                                                    list2, g.ctl + 1, fine);
  k_gal_big<false><<<256, kBig, 0, s>>>(agg_ptr, g.toff, g.tkey, g.tval, g.ucount, list2, g.ctl + 1, nullptr,
                                        nullptr, nullptr);
}

// Step 4 once the row pointers rp_c exist.
void launch_galerkin_finish(const GalerkinScratch& g, int nc, const int* agg_ptr, const int* rp_c, int* ci_c,
                            double* val_c, hipStream_t s) {
  if (nc <= 0) return;
  const int G = group_lanes(nc, (long)nc * 16);
  with_lanes(G, [&](auto gl) {
    k_gal_compact<decltype(gl)::value><<<group_grid(nc, G), 256, 0, s>>>(nc, agg_ptr, g.toff, g.tkey, g.tval, rp_c,
                                                                         ci_c, val_c);
  });
  k_gal_big<true><<<256, kBig, 0, s>>>(agg_ptr, g.toff, g.tkey, g.tval, nullptr, g.list + nc, g.ctl + 1, rp_c,
                                       ci_c, val_c);
}

}  // namespace amg
