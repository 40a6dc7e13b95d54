// Galerkin product by aggregate index (Section 3.1, eq. galerkin):
//   (A_{k+1})_IJ = sum_{i in G_I} sum_{j in G_J} P_iI A_ij P_jJ.
// Instead of a global sort of all (I, J) tuples, each coarse row I is built
// from its own aggregate segment G_I: the terms (J, (P_iI a_ij) P_jJ) of the
// segment's fine rows are staged in LDS, unique J are found with an LDS hash
// (first occurrence wins, so the result does not depend on timing), and each
// coarse entry is the sum of its terms in segment order.  A count pass sizes
// the rows, a scan makes the row pointers, a fill pass writes sorted columns.
// Rows whose segment holds more than 256 terms are staged by a whole block
// (up to 1536 terms); larger ones go to a block-per-row path that extracts
// the distinct J in ascending order without staging.
#include <climits>

#include "amg_internal.hpp"
#include "device_utils.hpp"

namespace amg {

namespace {
constexpr int kBig = 256;       // threads per block on the large-row path

// One coarse row per group of NT threads (NT = 64: a wave; NT = 256: a block).
// Terms are staged in LDS up to CAP; rows with more terms go to the next
// overflow list in the count pass and are skipped in the fill pass.
template <int NT, int CAP, int HB, bool FILL, bool LISTED>
__global__ void __launch_bounds__(NT) k_galerkin_stage(
    int nc, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
    const int* __restrict__ agg, const double* __restrict__ pval, const int* __restrict__ agg_ptr,
    const int* __restrict__ agg_rows, int* __restrict__ row_count, const int* __restrict__ in_list,
    const int* __restrict__ in_count, int* __restrict__ out_list, int* __restrict__ out_count,
    const int* __restrict__ rp_c, int* __restrict__ ci_c, double* __restrict__ val_c) {
  constexpr int HS = 1 << HB;
  __shared__ int keys[CAP];
  __shared__ double vals[FILL ? CAP : 1];
  __shared__ int hkey[HS];
  __shared__ int hfirst[HS];
  __shared__ int ukeys[CAP];
  __shared__ int tmp[NT / kWave + 1];
  __shared__ int s_cnt;
  __shared__ int m_start[NT], m_off[NT + 1];   // staging: member rows of one step
  __shared__ double m_pi[FILL ? NT : 1];
  const int tid = threadIdx.x;
  const int count = LISTED ? *in_count : nc;
  for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int I = LISTED ? in_list[idx] : idx;
    const int sb = agg_ptr[I], se = agg_ptr[I + 1];
    int T = 0;
    for (int base = sb; base < se; base += NT) {
      const int k = base + tid;
      int len = 0;
      if (k < se) { const int i = agg_rows[k]; len = rp[i + 1] - rp[i]; }
      int tot;
      (void)block_exclusive_scan(len, tmp, &tot);
      T += tot;
    }
    if (T > CAP) {
      if (!FILL && tid == 0) out_list[atomicAdd(out_count, 1)] = I;
      continue;
    }
    for (int q = tid; q < HS; q += NT) { hkey[q] = -1; hfirst[q] = INT_MAX; }
    if (tid == 0) s_cnt = 0;
    // stage the terms in segment order (row by row, entries in column order);
    // lanes take terms, not rows, so the gathers of a step are independent
    int off = 0;
    for (int base = sb; base < se; base += NT) {
      const int k = base + tid;
      int i = -1, len = 0, start = 0;
      if (k < se) { i = agg_rows[k]; start = rp[i]; len = rp[i + 1] - start; }
      int tot;
      const int pos = block_exclusive_scan(len, tmp, &tot);
      m_start[tid] = start;
      m_off[tid] = pos;
      if (FILL) m_pi[tid] = i >= 0 ? pval[i] : 0.0;
      if (tid == 0) m_off[NT] = tot;
      __syncthreads();
      for (int t = tid; t < tot; t += NT) {
        int lo = 0, hi = NT;   // member m with m_off[m] <= t < m_off[m + 1]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (m_off[mid] <= t) lo = mid; else hi = mid;
        }
        const int e = m_start[lo] + (t - m_off[lo]);
        const int j = ci[e];
        keys[off + t] = agg[j];
        if (FILL) vals[off + t] = __dmul_rn(__dmul_rn(m_pi[lo], val[e]), pval[j]);
      }
      off += tot;
      __syncthreads();
    }
    for (int t = tid; t < T; t += NT) {
      const int J = keys[t];
      int q = (int)(((uint32_t)J * 0x9E3779B1u) >> (32 - HB));
      while (true) {
        const int prev = atomicCAS(&hkey[q], -1, J);
        if (prev == -1 || prev == J) { atomicMin(&hfirst[q], t); break; }
        q = (q + 1) & (HS - 1);
      }
    }
    __syncthreads();
    for (int t = tid; t < T; t += NT) {
      const int J = keys[t];
      int q = (int)(((uint32_t)J * 0x9E3779B1u) >> (32 - HB));
      while (hkey[q] != J) q = (q + 1) & (HS - 1);
      if (hfirst[q] == t) ukeys[atomicAdd(&s_cnt, 1)] = J;
    }
    __syncthreads();
    const int U = s_cnt;
    if (!FILL) {
      if (tid == 0) row_count[I] = U;
    } else {
      const int out0 = rp_c[I];
      for (int u = tid; u < U; u += NT) {
        const int J = ukeys[u];
        int rank = 0;
        for (int v = 0; v < U; ++v) rank += ukeys[v] < J;
        double sum = 0.0;
        for (int t = 0; t < T; ++t)
          if (keys[t] == J) sum = __dadd_rn(sum, vals[t]);
        ci_c[out0 + rank] = J;
        val_c[out0 + rank] = sum;
      }
    }
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

// Large coarse rows: repeatedly take the smallest J above the last one over
// all terms of the segment, then sum its terms (fixed thread assignment and
// reduction order).  Grid-strides over the overflow list.
template <bool FILL>
__global__ void __launch_bounds__(kBig) k_galerkin_big(
    const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
    const int* __restrict__ agg, const double* __restrict__ pval, const int* __restrict__ agg_ptr,
    const int* __restrict__ agg_rows, int* __restrict__ row_count, const int* __restrict__ ovf_list,
    const int* __restrict__ ovf_count, const int* __restrict__ rp_c, int* __restrict__ ci_c,
    double* __restrict__ val_c) {
  __shared__ int ired[kBig / kWave];
  __shared__ double dred[kBig / kWave];
  const int count = *ovf_count;
  for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int I = ovf_list[idx];
    const int sb = agg_ptr[I], se = agg_ptr[I + 1];
    const int out0 = FILL ? rp_c[I] : 0;
    int last = -1, U = 0;
    while (true) {
      int mn = INT_MAX;
      for (int k = sb + threadIdx.x; k < se; k += kBig) {
        int i = agg_rows[k];
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
          int J = agg[ci[e]];
          if (J > last && J < mn) mn = J;
        }
      }
      mn = block_min_int(mn, ired);
      if (mn == INT_MAX) break;
      if (FILL) {
        double s = 0.0;
        for (int k = sb + threadIdx.x; k < se; k += kBig) {
          int i = agg_rows[k];
          double pi = pval[i];
          for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (agg[j] == mn) s = __dadd_rn(s, __dmul_rn(__dmul_rn(pi, val[e]), pval[j]));
          }
        }
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
    if (!FILL && threadIdx.x == 0) row_count[I] = U;
    __syncthreads();
  }
}
}  // namespace

// Count pass: waves take rows of up to 256 terms; blocks take the rows
// listed as larger (up to 1536 terms); the rest go to the extraction path.
void launch_galerkin_count(int nc, const int* rp, const int* ci, const int* agg, const int* agg_ptr,
                           const int* agg_rows, int* row_count, int* ovf_list, int* ctl_ovf, hipStream_t s) {
  if (nc <= 0) return;
  int* list1 = ovf_list;
  int* list2 = ovf_list + nc;
  launch_fill_int(2, ctl_ovf, 0, s);
  k_galerkin_stage<kWave, 256, 9, false, false><<<nc, kWave, 0, s>>>(
      nc, rp, ci, nullptr, agg, nullptr, agg_ptr, agg_rows, row_count, nullptr, nullptr, list1, ctl_ovf, nullptr,
      nullptr, nullptr);
  k_galerkin_stage<256, 1536, 12, false, true><<<1024, 256, 0, s>>>(
      nc, rp, ci, nullptr, agg, nullptr, agg_ptr, agg_rows, row_count, list1, ctl_ovf, list2, ctl_ovf + 1,
      nullptr, nullptr, nullptr);
  k_galerkin_big<false><<<256, kBig, 0, s>>>(rp, ci, nullptr, agg, nullptr, agg_ptr, agg_rows, row_count, list2,
                                             ctl_ovf + 1, nullptr, nullptr, nullptr);
}

void launch_galerkin_fill(int nc, const int* rp, const int* ci, const double* val, const int* agg,
                          const double* pval, const int* agg_ptr, const int* agg_rows, const int* rp_c,
                          int* ci_c, double* val_c, const int* ovf_list, const int* ctl_ovf, hipStream_t s) {
  if (nc <= 0) return;
  const int* list1 = ovf_list;
  const int* list2 = ovf_list + nc;
  k_galerkin_stage<kWave, 256, 9, true, false><<<nc, kWave, 0, s>>>(
      nc, rp, ci, val, agg, pval, agg_ptr, agg_rows, nullptr, nullptr, nullptr, nullptr, nullptr, rp_c, ci_c,
      val_c);
  k_galerkin_stage<256, 1536, 12, true, true><<<1024, 256, 0, s>>>(
      nc, rp, ci, val, agg, pval, agg_ptr, agg_rows, nullptr, list1, ctl_ovf, nullptr, nullptr, rp_c, ci_c, val_c);
  k_galerkin_big<true><<<256, kBig, 0, s>>>(rp, ci, val, agg, pval, agg_ptr, agg_rows, nullptr, list2,
                                            ctl_ovf + 1, rp_c, ci_c, val_c);
}

}  // namespace amg
