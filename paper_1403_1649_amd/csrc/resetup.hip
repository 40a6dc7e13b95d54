// Numeric re-setup on a fixed pattern (Section 3.1: when only the values of
// A_0 change, the indices of the Galerkin product's sort and segmented
// reduction are kept and replayed).  The aggregation and P_k of every level
// stay; A_{k+1} = P_k^T A_k P_k is formed again from stored term lists:
//   * per level, the terms of every coarse entry c = (I, J) in segment order
//     (members of aggregate I ascending, entries of a member row in column
//     order), as fine entry f and fine row i, found once by a walk over the
//     aggregate segments and a binary search of J in coarse row I;
//   * the replay sums (P_i a_f) P_j over a coarse entry's terms in that
//     order, the same products and the same order as the first setup's
//     reduce, so the values agree with a full setup on the same aggregation
//     bit for bit on every coarse row the wave reduce handled.
#include "kernels_common.hpp"

namespace amg {

namespace {
constexpr int kT = 256;

inline int grid1(long n) {
  long g = (n + kT - 1) / kT;
  if (g < 1) g = 1;
  return (int)(g < 65536 ? g : 65536);
}

// One thread per coarse row I walks its terms in segment order.  COUNT: the
// number of terms of every coarse entry; FILL: each term (f, i) at
// tptr[c] + (terms of c placed so far), with cur[] zero on entry.
template <bool FILL>
__global__ void __launch_bounds__(kT) k_rs_terms(int nc, const int* __restrict__ agg_ptr,
                                                 const int* __restrict__ agg_rows, const int* __restrict__ rp,
                                                 const int* __restrict__ ci, const int* __restrict__ agg,
                                                 const int* __restrict__ rp_c, const int* __restrict__ ci_c,
                                                 int* __restrict__ cur, const int* __restrict__ tptr,
                                                 int* __restrict__ tf, int* __restrict__ ti, int* err) {
  for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
    const int c0 = rp_c[I], c1 = rp_c[I + 1];
    for (int m = agg_ptr[I]; m < agg_ptr[I + 1]; ++m) {
      const int i = agg_rows[m];
      for (int f = rp[i]; f < rp[i + 1]; ++f) {
        const int J = agg[ci[f]];
        int lo = c0, hi = c1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (ci_c[mid] < J) lo = mid + 1;
          else hi = mid;
        }
        if (lo >= c1 || ci_c[lo] != J) {   // the coarse pattern lacks (I, J): not the setup's product
          atomic_or_flag(err, kErrBadColumn);
          continue;
        }
        if (FILL) {
          const int t = tptr[lo] + cur[lo]++;
          tf[t] = f;
          ti[t] = i;
        } else {
          cur[lo] += 1;
        }
      }
    }
  }
}

// A_{k+1} values: one thread per coarse entry, its terms summed in order.
// Products and sums stay separately rounded (no fused multiply-add), as in the
// setup, where the terms are stored before they are summed: the operators are
// written here, under the pragma (the rounding intrinsics are inline functions
// whose operations the compiler may still fuse).
__global__ void __launch_bounds__(kT) k_rs_values(int nnz_c, const int* __restrict__ tptr,
                                                  const int* __restrict__ tf, const int* __restrict__ ti,
                                                  const int* __restrict__ ci, const double* __restrict__ val,
                                                  const double* __restrict__ pval, double* __restrict__ val_c) {
#pragma clang fp contract(off)
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nnz_c; c += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int t = tptr[c]; t < tptr[c + 1]; ++t) {
      const int f = tf[t];
      const double term = (pval[ti[t]] * val[f]) * pval[ci[f]];
      s = s + term;
    }
    val_c[c] = s;
  }
}

// a_ii of every row (columns are strictly increasing, one diagonal entry)
__global__ void __launch_bounds__(kT) k_rs_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const double* __restrict__ val, double* __restrict__ diag) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) d = val[k];
    diag[i] = d;
  }
}

// New values of a sliced-ELL copy (the slice layout and the columns stay):
// element (slot s*H + l, k) at sl_ptr[s] + H k + l, zero padding; slot i
// holds row perm[i] (perm null: row i).
template <int H>
__global__ void __launch_bounds__(kT) k_rs_sell_values(int n, int nslices, const int* __restrict__ rp,
                                                       const double* __restrict__ val,
                                                       const int* __restrict__ sl_ptr, const int* __restrict__ perm,
                                                       double* __restrict__ sl_val, float* __restrict__ sl_val32) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = slot / H, l = slot & (H - 1);
  if (sl >= nslices) return;
  const int row = perm ? perm[slot] : slot;
  const int base = sl_ptr[sl];
  const int w = (sl_ptr[sl + 1] - base) / H;
  const int s0 = row < n ? rp[row] : 0;
  const int len = row < n ? rp[row + 1] - s0 : 0;
  for (int k = 0; k < w; ++k) {
    const int idx = base + k * H + l;
    const double v = k < len ? val[s0 + k] : 0.0;
    sl_val[idx] = v;
    if (sl_val32) sl_val32[idx] = (float)v;
  }
}
struct Coef16 {
  double v[16];
};
__global__ void k_set16(double* __restrict__ dst, Coef16 c) {
  if (threadIdx.x < 16) dst[threadIdx.x] = c.v[threadIdx.x];
}
}  // namespace

// 16 doubles from the host into device memory, passed as kernel arguments (the
// host array may go away as soon as this returns).
void launch_set16(double* dst, const double* host16, hipStream_t s) {
  Coef16 c;
  for (int q = 0; q < 16; ++q) c.v[q] = host16[q];
  k_set16<<<1, 64, 0, s>>>(dst, c);
}

void launch_rs_count(const Level& lv, const Level& lc, int* cnt, int* err, hipStream_t s) {
  k_rs_terms<false><<<grid1(lv.nc), kT, 0, s>>>(lv.nc, lv.agg_ptr, lv.agg_rows, lv.rp, lv.ci, lv.agg, lc.rp, lc.ci,
                                                cnt, nullptr, nullptr, nullptr, err);
}

void launch_rs_fill(const Level& lv, const Level& lc, int* cur, int* tf, int* ti, int* err, hipStream_t s) {
  k_rs_terms<true><<<grid1(lv.nc), kT, 0, s>>>(lv.nc, lv.agg_ptr, lv.agg_rows, lv.rp, lv.ci, lv.agg, lc.rp, lc.ci,
                                               cur, lv.rs_tptr, tf, ti, err);
}

void launch_rs_values(const Level& lv, Level& lc, hipStream_t s) {
  if (lc.nnz > 0)
    k_rs_values<<<grid1(lc.nnz), kT, 0, s>>>(lc.nnz, lv.rs_tptr, lv.rs_f, lv.rs_i, lv.ci, lv.val, lv.pval, lc.val);
}

void launch_rs_diag(const Level& lv, hipStream_t s) {
  k_rs_diag<<<grid1(lv.n), kT, 0, s>>>(lv.n, lv.rp, lv.ci, lv.val, lv.diag);
}

void launch_rs_sell_values(const Level& lv, hipStream_t s) {
  if (lv.nslices > 0 && lv.sl_val)
    k_rs_sell_values<64><<<(lv.nslices * kWave + kT - 1) / kT, kT, 0, s>>>(lv.n, lv.nslices, lv.rp, lv.val,
                                                                           lv.sl_ptr, nullptr, lv.sl_val,
                                                                           lv.sl_val32);
  if (lv.dia.val)   // the sliced diagonals, when the level keeps them
    launch_sdia_fill(lv.n, lv.rp, lv.ci, lv.val, lv.dia.ptr, lv.dia.off, lv.dia.val, lv.dia.val32, s);
  const Level::ShortSell& q = lv.sh;   // the copy in shorter slices, when the level keeps one
  if (q.nslices > 0 && q.val) {
    const int g = (int)(((long)q.nslices * q.h + kT - 1) / kT);
    if (q.h == 32)
      k_rs_sell_values<32><<<g, kT, 0, s>>>(lv.n, q.nslices, lv.rp, lv.val, q.ptr, q.perm, q.val, q.val32);
    else
      k_rs_sell_values<16><<<g, kT, 0, s>>>(lv.n, q.nslices, lv.rp, lv.val, q.ptr, q.perm, q.val, q.val32);
  }
}

}  // namespace amg
