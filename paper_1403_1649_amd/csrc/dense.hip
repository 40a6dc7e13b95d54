// Coarsest-level exact solve (Algorithms 4/5, "exact solution of coarse
// grid"; Section 3 keeps that level near 600 unknowns).  The dense A_L is
// inverted once in setup by Gauss-Jordan elimination with partial pivoting,
// so each coarse solve in the cycle is one dense mat-vec (a GEMV over at most
// dense_max^2 entries) instead of two sequential triangular solves.
//
// The elimination runs as one kernel of at most 128 blocks: each block owns a
// band of columns (in LDS when the bands fit, else in the row-major work
// matrix in global memory); per pivot step the owner of
// column k picks the pivot and publishes column k, one grid barrier, then
// every block updates its band.  A single block needs no grid barrier.  The
// barrier needs all blocks resident at once, so the kernel is launched as a
// cooperative launch, which the runtime refuses (an error, not a hang) when
// the grid cannot be resident together; the grid never exceeds 128 one-CU
// workgroups of the 256 CUs.
#include <algorithm>
#include <cmath>
#include <vector>

#include "amg_internal.hpp"
#include "device_utils.hpp"

namespace amg {

namespace {
constexpr int kGJThreads = 1024;

__global__ void k_dense_zero(size_t nn, double* W) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t st = (size_t)gridDim.x * blockDim.x;
  for (; i < nn; i += st) W[i] = 0.0;
}

__global__ void k_dense_scatter(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ val, double* __restrict__ W) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) W[(size_t)i * n + ci[k]] = val[k];
}

__device__ __forceinline__ void grid_barrier(int* sync, int nblocks) {
  if (nblocks == 1) {
    __syncthreads();
    return;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int gen = __hip_atomic_load(&sync[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const int arrived = __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&sync[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&sync[1], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(&sync[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen)
        __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  __threadfence();
}

// In-place Gauss-Jordan inversion of the n x n row-major W.  piv[k] records
// the row exchanged with row k at step k; colbuf holds 2 x n doubles.
__global__ void __launch_bounds__(kGJThreads) k_gauss_jordan(int n, int band, double* __restrict__ W,
                                                             int* __restrict__ piv,
                                                             double* __restrict__ colbuf, int* sync,
                                                             int* err) {
  __shared__ double s_rowk[1024];
  __shared__ double s_val[kGJThreads / kWave];
  __shared__ int s_idx[kGJThreads / kWave];
  const int nb = gridDim.x;
  const int c0 = blockIdx.x * band;
  const int c1 = min(n, c0 + band);
  const int w = c1 - c0;
  for (int k = 0; k < n; ++k) {
    double* cb = colbuf + (size_t)(k & 1) * n;
    const int owner = k / band;
    if ((int)blockIdx.x == owner) {
      // pivot: the largest |W[i][k]| over rows i >= k (smallest index on ties)
      double best = -1.0;
      int bi = k;
      for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double a = fabs(W[(size_t)i * n + k]);
        if (a > best) { best = a; bi = i; }
      }
      for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bi, off, kWave);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if ((threadIdx.x & (kWave - 1)) == 0) {
        s_val[threadIdx.x / kWave] = best;
        s_idx[threadIdx.x / kWave] = bi;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x / kWave); ++q)
          if (s_val[q] > best || (s_val[q] == best && s_idx[q] < bi)) { best = s_val[q]; bi = s_idx[q]; }
        piv[k] = bi;
        if (!(best > 0.0)) atomic_or_flag(err, kErrSingular);
      }
      for (int i = threadIdx.x; i < n; i += blockDim.x) cb[i] = W[(size_t)i * n + k];
    }
    grid_barrier(sync, nb);
    const int p = __hip_atomic_load(&piv[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // column k after the exchange of rows k and p
    const double ck = cb[p];
    // exchange rows k and p inside this band, keep the (exchanged) row k
    for (int j = threadIdx.x; j < w; j += blockDim.x) {
      const int col = c0 + j;
      double a = W[(size_t)k * n + col];
      if (p != k) {
        const double b = W[(size_t)p * n + col];
        W[(size_t)p * n + col] = a;
        a = b;
      }
      s_rowk[j] = a;
    }
    __syncthreads();
    const double inv = 1.0 / ck;
    for (int e = threadIdx.x; e < n * w; e += blockDim.x) {
      const int i = e / w;
      const int j = e - i * w;
      const int col = c0 + j;
      const double ci = (i == k) ? ck : (i == p ? cb[k] : cb[i]);
      double* dst = W + (size_t)i * n + col;
      if (col == k) {
        *dst = (i == k) ? inv : -ci * inv;
      } else if (i == k) {
        *dst = s_rowk[j] * inv;
      } else {
        *dst -= ci * (s_rowk[j] * inv);
      }
    }
    __syncthreads();
  }
}

// One Gauss-Jordan step k applied to a block's LDS band (column-major,
// S[j*n + i] = W[i][c0 + j]): rows k and p exchanged, then the update with
// the pre-exchange pivot column `col` (LDS) and the staged pivot row.
__device__ __forceinline__ void gj_apply(double* S, int n, int c0, int w, int k, int p, const double* col,
                                         double* s_rowk) {
  const int tid = threadIdx.x;
  const double ck = col[p];
  for (int j = tid; j < w; j += blockDim.x) {
    double a = S[(size_t)j * n + k];
    if (p != k) {
      const double b = S[(size_t)j * n + p];
      S[(size_t)j * n + p] = a;
      a = b;
    }
    s_rowk[j] = a;
  }
  __syncthreads();
  const double inv = 1.0 / ck;
  for (int e = tid; e < w * n; e += blockDim.x) {
    const int j = e / n, i = e - j * n;
    const int colj = c0 + j;
    const double ci = (i == k) ? ck : (i == p ? col[k] : col[i]);
    double* dst = S + (size_t)j * n + i;
    if (colj == k) {
      *dst = (i == k) ? inv : -ci * inv;
    } else if (i == k) {
      *dst = s_rowk[j] * inv;
    } else {
      *dst -= ci * (s_rowk[j] * inv);
    }
  }
  __syncthreads();
}

// Gauss-Jordan with each block's band of columns resident in LDS.  The owner
// of a band runs that band's pivot steps on its own (no grid barrier: its
// columns already hold every earlier step), publishes the pivot rows and the
// pre-exchange pivot columns, and after one grid barrier the other blocks
// replay those steps on their bands.  Grid barriers: one per band.
__global__ void __launch_bounds__(kGJThreads) k_gauss_jordan_lds(int n, int band, double* __restrict__ W,
                                                                 int* __restrict__ piv,
                                                                 double* __restrict__ colbuf, int* sync,
                                                                 int* err) {
  extern __shared__ double S[];
  double* s_col = S + (size_t)band * n;
  double* s_rowk = s_col + n;
  __shared__ double s_val[kGJThreads / kWave];
  __shared__ int s_idx[kGJThreads / kWave];
  __shared__ int s_p;
  const int nb = gridDim.x;
  const int c0 = blockIdx.x * band;
  const int w = min(n, c0 + band) - c0;
  const int tid = threadIdx.x;
  for (int e = tid; e < w * n; e += blockDim.x) {
    const int i = e / w, j = e - i * w;
    S[j * n + i] = W[(size_t)i * n + c0 + j];
  }
  __syncthreads();
  for (int pb = 0; pb < nb; ++pb) {
    const int pc0 = pb * band, pc1 = min(n, pc0 + band);
    if ((int)blockIdx.x == pb) {
      for (int k = pc0; k < pc1; ++k) {
        const double* col = S + (size_t)(k - c0) * n;
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < n; i += blockDim.x) {
          const double a = fabs(col[i]);
          if (a > best) { best = a; bi = i; }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, kWave);
          const int oi = __shfl_xor(bi, off, kWave);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if ((tid & (kWave - 1)) == 0) {
          s_val[tid / kWave] = best;
          s_idx[tid / kWave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
          for (int q = 1; q < (int)(blockDim.x / kWave); ++q)
            if (s_val[q] > best || (s_val[q] == best && s_idx[q] < bi)) { best = s_val[q]; bi = s_idx[q]; }
          piv[k] = bi;
          s_p = bi;
          if (!(best > 0.0)) atomic_or_flag(err, kErrSingular);
        }
        for (int i = tid; i < n; i += blockDim.x) {
          s_col[i] = col[i];
          if (nb > 1) colbuf[(size_t)k * n + i] = col[i];
        }
        __syncthreads();
        gj_apply(S, n, c0, w, k, s_p, s_col, s_rowk);
      }
    }
    if (nb > 1) {
      grid_barrier(sync, nb);
      if ((int)blockIdx.x != pb) {
        for (int k = pc0; k < pc1; ++k) {
          const int p = __hip_atomic_load(&piv[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          for (int i = tid; i < n; i += blockDim.x) s_col[i] = colbuf[(size_t)k * n + i];
          __syncthreads();
          gj_apply(S, n, c0, w, k, p, s_col, s_rowk);
        }
      }
    }
  }
  for (int e = tid; e < w * n; e += blockDim.x) {
    const int i = e / w, j = e - i * w;
    W[(size_t)i * n + c0 + j] = S[j * n + i];
  }
}

// Undo the row exchanges as column exchanges (last step first) and emit the
// float64 and float32 inverses.
__global__ void k_gj_unpermute(int n, const double* __restrict__ W, const int* __restrict__ piv,
                               double* __restrict__ inv, float* __restrict__ inv32, int* perm_tmp) {
  extern __shared__ int s_perm[];
  if (threadIdx.x == 0) {
    for (int j = 0; j < n; ++j) s_perm[j] = j;
    for (int k = n - 1; k >= 0; --k) {
      const int p = piv[k];
      const int t = s_perm[k];
      s_perm[k] = s_perm[p];
      s_perm[p] = t;
    }
  }
  __syncthreads();
  (void)perm_tmp;
  const size_t nn = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n);
    const int j = (int)(e - (size_t)i * n);
    const double v = W[(size_t)i * n + s_perm[j]];
    inv[e] = v;
    if (inv32) inv32[e] = (float)v;
  }
}
// Batched systems: one workgroup inverts one terminal system.  Its bands of
// columns pass through LDS one after another (left-looking): a band first
// replays the pivot steps already taken (pivot rows in piv, pre-exchange pivot
// columns in cb), then takes its own steps and publishes them; a second pass
// replays the later steps on the earlier bands.  Each element sees the same
// sequence of updates as in k_gauss_jordan_lds, so the inverse is the same.
__global__ void __launch_bounds__(kGJThreads) k_gj_batched(const TermInfo* __restrict__ ti, double* __restrict__ work,
                                                           double* __restrict__ cbuf, int* __restrict__ pivbuf,
                                                           int lds_doubles, int* err) {
  extern __shared__ double S[];
  __shared__ double s_val[kGJThreads / kWave];
  __shared__ int s_idx[kGJThreads / kWave];
  __shared__ int s_p;
  const TermInfo t = ti[blockIdx.x];
  const int n = t.n;
  double* W = work + t.off;
  double* cb = cbuf + t.off;
  int* piv = pivbuf + t.row0;
  const int band = min(n, (lds_doubles - n) / (n + 1));
  double* s_col = S + (size_t)band * n;
  double* s_rowk = s_col + n;
  const int nb = (n + band - 1) / band;
  const int tid = threadIdx.x;
  auto load = [&](int c0, int w) {
    for (int e = tid; e < w * n; e += blockDim.x) {
      const int i = e / w, j = e - i * w;
      S[j * n + i] = W[(size_t)i * n + c0 + j];
    }
    __syncthreads();
  };
  auto store = [&](int c0, int w) {
    for (int e = tid; e < w * n; e += blockDim.x) {
      const int i = e / w, j = e - i * w;
      W[(size_t)i * n + c0 + j] = S[j * n + i];
    }
    __threadfence_block();
    __syncthreads();
  };
  auto replay = [&](int c0, int w, int k) {
    const int p = piv[k];
    for (int i = tid; i < n; i += blockDim.x) s_col[i] = cb[(size_t)k * n + i];
    __syncthreads();
    gj_apply(S, n, c0, w, k, p, s_col, s_rowk);
  };
  for (int pb = 0; pb < nb; ++pb) {
    const int c0 = pb * band, w = min(n, c0 + band) - c0;
    load(c0, w);
    for (int k = 0; k < c0; ++k) replay(c0, w, k);
    for (int k = c0; k < c0 + w; ++k) {
      const double* col = S + (size_t)(k - c0) * n;
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < n; i += blockDim.x) {
        const double a = fabs(col[i]);
        if (a > best) { best = a; bi = i; }
      }
      for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bi, off, kWave);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if ((tid & (kWave - 1)) == 0) {
        s_val[tid / kWave] = best;
        s_idx[tid / kWave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        for (int q = 1; q < (int)(blockDim.x / kWave); ++q)
          if (s_val[q] > best || (s_val[q] == best && s_idx[q] < bi)) { best = s_val[q]; bi = s_idx[q]; }
        piv[k] = bi;
        s_p = bi;
        if (!(best > 0.0)) atomic_or_flag(err, kErrSingular);
      }
      for (int i = tid; i < n; i += blockDim.x) {
        s_col[i] = col[i];
        cb[(size_t)k * n + i] = col[i];
      }
      __threadfence_block();
      __syncthreads();
      gj_apply(S, n, c0, w, k, s_p, s_col, s_rowk);
    }
    store(c0, w);
  }
  for (int pb = 0; pb + 1 < nb; ++pb) {
    const int c0 = pb * band, w = min(n, c0 + band) - c0;
    load(c0, w);
    for (int k = c0 + w; k < n; ++k) replay(c0, w, k);
    store(c0, w);
  }
}

// Undo the row exchanges of each system as column exchanges (last step
// first); one workgroup per system.
__global__ void k_gj_unpermute_batched(const TermInfo* __restrict__ ti, const double* __restrict__ work,
                                       const int* __restrict__ pivbuf, double* __restrict__ inv,
                                       float* __restrict__ inv32) {
  extern __shared__ int s_perm[];
  const TermInfo t = ti[blockIdx.x];
  const int n = t.n;
  const int* piv = pivbuf + t.row0;
  if (threadIdx.x == 0) {
    for (int j = 0; j < n; ++j) s_perm[j] = j;
    for (int k = n - 1; k >= 0; --k) {
      const int p = piv[k];
      const int q = s_perm[k];
      s_perm[k] = s_perm[p];
      s_perm[p] = q;
    }
  }
  __syncthreads();
  const double* W = work + t.off;
  const size_t nn = (size_t)n * n;
  for (size_t e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = (int)(e / n);
    const int j = (int)(e - (size_t)i * n);
    const double v = W[(size_t)i * n + s_perm[j]];
    inv[t.off + e] = v;
    if (inv32) inv32[t.off + e] = (float)v;
  }
}

// dense copy of each terminal system's diagonal block (columns shifted to the
// system's first row)
__global__ void k_dense_scatter_batched(const TermInfo* __restrict__ ti, const int* __restrict__ rp,
                                        const int* __restrict__ ci, const double* __restrict__ val,
                                        double* __restrict__ work) {
  const TermInfo t = ti[blockIdx.x];
  double* W = work + t.off;
  for (int r = threadIdx.x; r < t.n; r += blockDim.x) {
    const int row = t.row0 + r;
    for (int k = rp[row]; k < rp[row + 1]; ++k) W[(size_t)r * t.n + (ci[k] - t.row0)] = val[k];
  }
}
// ---------------------------------------------------------------- SPD, blocked
// A symmetric positive definite matrix needs no pivoting in Gauss-Jordan
// elimination: every pivot is a diagonal entry of a Schur complement, hence
// positive.  Panels of b columns: the panel's b steps run in one workgroup
// with the panel held in registers (no pivot search, so one step is two
// barriers and one broadcast of the pivot row); every other column then receives the panel's combined
// elementary transformation M = I + (Y - E) E^T at once, where Y is the panel
// after its steps and E the unit columns of the panel's pivot rows:
// A_J <- A_J + (Y - E) T with T = the panel's pivot rows of A_J before the
// update.  That rank-b update is a tiled product over all columns of all
// systems; no grid barrier is needed because panel and update are separate
// launches.  A non-positive or non-finite pivot raises kErrNotSPD and the
// caller falls back to the pivoting kernels.
constexpr int kPanelThreads = 1024;
constexpr int kUpdTile = 64;

// The panel: thread t owns rows t, t + 1024, ... (R of them) and keeps their
// B panel entries in registers (B * R = 32); per step only the pivot row goes
// through LDS.  In-place Gauss-Jordan step k restricted to the panel:
// pivot row scaled by 1/p, other rows minus their column-k entry times the
// scaled pivot row, column k replaced by -a_ik/p (and 1/p at the pivot).
template <int B, int R>
__global__ void __launch_bounds__(kPanelThreads) k_gjb_panel_reg(const TermInfo* __restrict__ ti,
                                                                 double* __restrict__ work,
                                                                 double* __restrict__ ybuf,
                                                                 double* __restrict__ tbuf, int K, int* err) {
  __shared__ double s_row[B];
  const TermInfo t = ti[blockIdx.x];
  const int n = t.n, c0 = K * B;
  if (c0 >= n) return;
  const int w = min(B, n - c0);
  double* W = work + t.off;
  double* Y = ybuf + (size_t)t.row0 * B;
  double* T = tbuf + (size_t)t.row0 * B;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int e = tid; e < w * n; e += nt) {
    const int j = e / n, J = e - j * n;
    T[(size_t)j * n + J] = W[(size_t)(c0 + j) * n + J];
  }
  double P[R][B];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + r * nt;
#pragma unroll
    for (int q = 0; q < B; ++q) P[r][q] = (i < n && q < w) ? W[(size_t)i * n + c0 + q] : 0.0;
  }
  // the step loop stays rolled (one copy of the unrolled column loop), so the
  // pivot column entry is selected with compares instead of a runtime index
#pragma unroll 1
  for (int j = 0; j < w; ++j) {
    const int k = c0 + j;
    if (tid == k % nt) {
      const int rk = k / nt;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r == rk) {
#pragma unroll
          for (int q = 0; q < B; ++q) s_row[q] = P[r][q];
        }
    }
    __syncthreads();
    const double p = s_row[j];
    if (tid == 0 && !(p > 0.0 && p < INFINITY)) atomic_or_flag(err, kErrNotSPD);
    const double inv = 1.0 / p;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + r * nt;
      double c = 0.0;
#pragma unroll
      for (int q = 0; q < B; ++q) c = (q == j) ? P[r][q] : c;
#pragma unroll
      for (int q = 0; q < B; ++q) {
        if (q == j) {
          P[r][q] = (i == k) ? inv : -c * inv;
        } else {
          const double rk = s_row[q] * inv;
          P[r][q] = (i == k) ? rk : P[r][q] - c * rk;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + r * nt;
    if (i >= n) continue;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (q < w) {
        W[(size_t)i * n + c0 + q] = P[r][q];
        Y[(size_t)i * B + q] = P[r][q];
      }
    }
  }
}

// The panel in two launches, so that one workgroup per system only does the
// b steps on the b x b pivot block.  A step is linear in every non-pivot row:
// row <- row * E_j, where E_j depends only on the pivot row of step j.  So the
// pivot block's workgroup also runs the steps on b virtual rows that start as
// the unit rows, which end as X = E_0 E_1 ... E_{b-1}; every other row of the
// panel is then row * X, a (n - b) x b x b product done by many workgroups.
// k_gjb_pivot: one workgroup per system, the 64 x 32 block (32 pivot rows,
// then the 32 virtual rows) in LDS and every element updated in parallel at
// each step (two per thread), with the arithmetic of the register panel:
// pivot row s / p, column j -c / p (1 / p at the pivot), others a - c (s / p).
__global__ void __launch_bounds__(1024) k_gjb_pivot(const TermInfo* __restrict__ ti, double* __restrict__ work,
                                                    double* __restrict__ ybuf, double* __restrict__ xbuf, int K,
                                                    int* err) {
  constexpr int B = 32, ROWS = 2 * B;
  __shared__ double M[ROWS][B + 1];
  const TermInfo t = ti[blockIdx.x];
  const int n = t.n, c0 = K * B;
  if (c0 >= n) return;
  const int w = min(B, n - c0);
  double* W = work + t.off;
  double* Y = ybuf + (size_t)t.row0 * B;
  const int tid = threadIdx.x;
  for (int e = tid; e < ROWS * B; e += 1024) {
    const int i = e / B, q = e % B;
    M[i][q] = i < B ? ((i < w && q < w) ? W[(size_t)(c0 + i) * n + c0 + q] : 0.0) : (q == i - B ? 1.0 : 0.0);
  }
  __syncthreads();
#pragma unroll 1
  for (int j = 0; j < w; ++j) {
    const double p = M[j][j];
    if (tid == 0 && !(p > 0.0 && p < INFINITY)) atomic_or_flag(err, kErrNotSPD);
    const double inv = 1.0 / p;
    double nv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + h * 1024, i = e / B, q = e % B;
      const double c = M[i][j];
      if (q == j) {
        nv[h] = (i == j) ? inv : -c * inv;
      } else {
        const double rk = M[j][q] * inv;
        nv[h] = (i == j) ? rk : M[i][q] - c * rk;
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + h * 1024;
      M[e / B][e % B] = nv[h];
    }
    __syncthreads();
  }
  double* X = xbuf + (size_t)blockIdx.x * B * B;
  for (int e = tid; e < ROWS * B; e += 1024) {
    const int i = e / B, q = e % B;
    if (i < B) {
      if (i < w && q < w) {
        W[(size_t)(c0 + i) * n + c0 + q] = M[i][q];
        Y[(size_t)(c0 + i) * B + q] = M[i][q];
      }
    } else {
      X[(i - B) * B + q] = M[i][q];
    }
  }
}

// k_gjb_apply: the non-pivot rows of every system's 32-column panel times X
// on the FP64 matrix cores (each wave 16 rows x 32 columns: 2 MFMA tiles, 8
// k-steps).  Work items are (system, block of 256 rows) pairs from the host's
// table.
__global__ void __launch_bounds__(256) k_gjb_apply(const TermInfo* __restrict__ ti, const int* __restrict__ items,
                                                   double* __restrict__ work, double* __restrict__ ybuf,
                                                   const double* __restrict__ xbuf, int K) {
  constexpr int B = 32;
  __shared__ double sX[B][B + 1];
  const int sys = items[2 * blockIdx.x], rb = items[2 * blockIdx.x + 1];
  const TermInfo t = ti[sys];
  const int n = t.n, c0 = K * B;
  if (c0 >= n) return;
  const int w = min(B, n - c0);
  double* W = work + t.off;
  double* Y = ybuf + (size_t)t.row0 * B;
  const double* X = xbuf + (size_t)sys * B * B;
  for (int e = threadIdx.x; e < B * B; e += 256) sX[e / B][e % B] = X[e];
  __syncthreads();
  const int wv = threadIdx.x / kWave, l = threadIdx.x & (kWave - 1);
  for (int R0 = rb * 256 + wv * 16; R0 < min(n, (rb + 1) * 256); R0 += 64) {
    const int ar = R0 + (l & 15);
    const bool arow = ar < n && !(ar >= c0 && ar < c0 + w);
    f64x4 acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
    for (int kk = 0; kk < B; kk += 4) {
      const int kc = kk + (l >> 4);
      const double av = (arow && kc < w) ? W[(size_t)ar * n + c0 + kc] : 0.0;
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) acc[sc] = mfma_f64_16x16x4(av, sX[kc][16 * sc + (l & 15)], acc[sc]);
    }
#pragma unroll
    for (int sc = 0; sc < 2; ++sc)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = R0 + mfma_row(l, i), col = 16 * sc + mfma_col(l);
        if (row < n && !(row >= c0 && row < c0 + w) && col < w) {
          W[(size_t)row * n + c0 + col] = acc[sc][i];
          Y[(size_t)row * B + col] = acc[sc][i];
        }
      }
  }
}

// A_J += (Y - E) T for every column J outside the panel: 64 x 64 output tiles
// on the FP64 matrix cores (each wave a 32 x 32 quadrant = 2 x 2 MFMA tiles,
// k in steps of 4 over the panel width, zero-padded); the panel's pivot rows
// get Y T directly.
// mode 0: every row of the tile, T from tbuf (copied before the panel wrote
// its pivot rows); mode 1: the rows outside the pivot block only, T read from
// the pivot rows of A themselves (no launch writes them until mode 2); mode 2:
// the pivot rows only (tiles (system, column tile), rows from c0), each
// workgroup reading its columns of the pivot rows before writing them.
__global__ void __launch_bounds__(256) k_gjb_update(const TermInfo* __restrict__ ti, const int* __restrict__ tiles,
                                                    double* __restrict__ work, const double* __restrict__ ybuf,
                                                    const double* __restrict__ tbuf, int K, int b, int mode) {
  __shared__ double sY[kUpdTile][33];
  __shared__ double sT[32][kUpdTile + 1];
  const TermInfo t = ti[tiles[2 * blockIdx.x]];
  const int n = t.n, c0 = K * b;
  if (c0 >= n) return;
  const int w = min(b, n - c0);
  const int nt = (n + kUpdTile - 1) / kUpdTile;
  const int tile = tiles[2 * blockIdx.x + 1];
  const int r0 = mode == 2 ? c0 : (tile / nt) * kUpdTile, q0 = (tile % nt) * kUpdTile;
  if (q0 >= c0 && q0 + kUpdTile <= c0 + w) return;   // tile entirely inside the panel
  if (mode == 1 && r0 >= c0 && r0 + kUpdTile <= c0 + w) return;   // pivot rows only: mode 2
  double* W = work + t.off;
  const double* Y = ybuf + (size_t)t.row0 * b;
  const double* T = mode == 0 ? tbuf + (size_t)t.row0 * b : W + (size_t)c0 * n;
  const int tid = threadIdx.x;
  const int kw = (w + 3) & ~3;   // panel width padded to the MFMA k step
  for (int e = tid; e < kUpdTile * kw; e += 256) {
    const int i = e / kw, j = e - i * kw;
    sY[i][j] = (r0 + i < n && j < w) ? Y[(size_t)(r0 + i) * b + j] : 0.0;
  }
  for (int e = tid; e < kw * kUpdTile; e += 256) {
    const int j = e / kUpdTile, c = e - j * kUpdTile;
    sT[j][c] = (q0 + c < n && j < w) ? T[(size_t)j * n + q0 + c] : 0.0;
  }
  __syncthreads();
  const int wv = tid / kWave, l = tid & (kWave - 1);
  const int qr = (wv >> 1) * 32, qc = (wv & 1) * 32;   // this wave's quadrant
  f64x4 acc[2][2];
#pragma unroll
  for (int sr = 0; sr < 2; ++sr)
#pragma unroll
    for (int sc = 0; sc < 2; ++sc)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + qr + 16 * sr + mfma_row(l, i), col = q0 + qc + 16 * sc + mfma_col(l);
        const bool pivot_row = row >= c0 && row < c0 + w;
        acc[sr][sc][i] = (row < n && col < n && !pivot_row) ? W[(size_t)row * n + col] : 0.0;
      }
  for (int kk = 0; kk < kw; kk += 4) {
    double av[2], bv[2];
#pragma unroll
    for (int sr = 0; sr < 2; ++sr) av[sr] = sY[qr + 16 * sr + (l & 15)][kk + (l >> 4)];
#pragma unroll
    for (int sc = 0; sc < 2; ++sc) bv[sc] = sT[kk + (l >> 4)][qc + 16 * sc + (l & 15)];
#pragma unroll
    for (int sr = 0; sr < 2; ++sr)
#pragma unroll
      for (int sc = 0; sc < 2; ++sc) acc[sr][sc] = mfma_f64_16x16x4(av[sr], bv[sc], acc[sr][sc]);
  }
#pragma unroll
  for (int sr = 0; sr < 2; ++sr)
#pragma unroll
    for (int sc = 0; sc < 2; ++sc)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + qr + 16 * sr + mfma_row(l, i), col = q0 + qc + 16 * sc + mfma_col(l);
        const bool pivot_row = row >= c0 && row < c0 + w;
        const bool mine = mode == 0 || (mode == 1) != pivot_row;
        if (mine && row < n && col < n && (col < c0 || col >= c0 + w)) W[(size_t)row * n + col] = acc[sr][sc][i];
      }
}

__global__ void k_dense_to_float(size_t nn, const double* __restrict__ in, float* __restrict__ out) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x)
    out[e] = (float)in[e];
}

}  // namespace

void launch_dense_inverse(int n, const int* rp, const int* ci, const double* val, double* work, double* inv,
                          float* inv32, int* sync, int* err, hipStream_t s) {
  const size_t nn = (size_t)n * n;
  k_dense_zero<<<(int)std::min<size_t>((nn + 255) / 256, 4096), 256, 0, s>>>(nn, work);
  k_dense_scatter<<<(n + 255) / 256, 256, 0, s>>>(n, rp, ci, val, work);
  int* piv = sync + 4;
  double* colbuf = work + nn;   // 2n doubles (global path) or n*n (LDS path)
  launch_fill_int(4, sync, 0, s);
  // LDS-resident bands when at most 128 blocks hold the matrix, else bands in
  // global memory (at most 64 blocks, band <= 1024 for the LDS pivot row)
  int dev = 0, lds_max = 0;
  AMG_HIP(hipGetDevice(&dev));
  AMG_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const long budget = (long)lds_max - 4096;   // static LDS of the kernel
  long band = budget / 8 / (n + 1) - 1;
  if (band >= 1) {
    long nb = (n + band - 1) / band;
    band = (n + nb - 1) / nb;
    nb = (n + band - 1) / band;
    if (nb <= 128) {
      const size_t bytes = ((size_t)band * n + n + band) * sizeof(double);
      AMG_HIP(hipFuncSetAttribute((const void*)k_gauss_jordan_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes));
      int bandi = (int)band;
      void* args[] = {&n, &bandi, &work, &piv, &colbuf, &sync, &err};
      AMG_HIP(hipLaunchCooperativeKernel((const void*)k_gauss_jordan_lds, dim3((unsigned)nb), dim3(kGJThreads), args,
                                         (unsigned)bytes, s));
      const int g = (int)std::min<size_t>((nn + 255) / 256, 1024);
      k_gj_unpermute<<<g, 256, n * sizeof(int), s>>>(n, work, piv, inv, inv32, nullptr);
      return;
    }
  }
  int nbg = (int)std::min<long>(64, std::max<long>(1, (long)nn / 16384));
  int bandg = (n + nbg - 1) / nbg;
  if (bandg > 1024) bandg = 1024;
  nbg = (n + bandg - 1) / bandg;
  {
    void* args[] = {&n, &bandg, &work, &piv, &colbuf, &sync, &err};
    AMG_HIP(hipLaunchCooperativeKernel((const void*)k_gauss_jordan, dim3((unsigned)nbg), dim3(kGJThreads), args, 0u, s));
  }
  const int g = (int)std::min<size_t>((nn + 255) / 256, 1024);
  k_gj_unpermute<<<g, 256, n * sizeof(int), s>>>(n, work, piv, inv, inv32, nullptr);
}

}  // namespace amg

namespace amg {

void launch_dense_inverse_batched(const Level& lv, int nterm, const TermInfo* d_term, const TermInfo* h_term,
                                  double* work, int* piv, double* inv, float* inv32, int* err, hipStream_t s) {
  if (nterm == 0) return;
  size_t total = 0;
  int nmax = 0;
  for (int t = 0; t < nterm; ++t) {
    total += (size_t)h_term[t].n * h_term[t].n;
    nmax = std::max(nmax, h_term[t].n);
  }
  double* cbuf = work + total;   // pre-exchange pivot columns, n x n per system
  launch_fill_double(total, work, 0.0, s);
  k_dense_scatter_batched<<<nterm, 256, 0, s>>>(d_term, lv.rp, lv.ci, lv.val, work);
  int dev = 0, lds_max = 0;
  AMG_HIP(hipGetDevice(&dev));
  AMG_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const long budget = (long)lds_max - 4096;   // static LDS of the kernel
  const long need = (long)nmax * nmax + 2L * nmax;
  const long lds_d = std::min(need, budget / 8);
  if ((lds_d - nmax) / (nmax + 1) < 1) throw Error(AMG_ECOARSEN, "coarsest system too large for the LDS band");
  const size_t bytes = (size_t)lds_d * sizeof(double);
  AMG_HIP(hipFuncSetAttribute((const void*)k_gj_batched, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  k_gj_batched<<<nterm, kGJThreads, bytes, s>>>(d_term, work, cbuf, piv, (int)lds_d, err);
  k_gj_unpermute_batched<<<nterm, 256, nmax * sizeof(int), s>>>(d_term, work, piv, inv, inv32);
}

}  // namespace amg

namespace amg {

// Inverses of symmetric positive definite diagonal blocks (one per TermInfo)
// in place in inv (row-major n x n at each TermInfo's offset), blocked
// Gauss-Jordan without pivoting; inv32 (optional) receives the float copy.
// Raises kErrNotSPD on a non-positive pivot; the caller then redoes the
// inversion with pivoting.  Scratch from tmp.
void launch_dense_inverse_spd(int nterm, const TermInfo* d_term, const TermInfo* h_term, int nrows, const int* rp,
                              const int* ci, const double* val, double* inv, float* inv32, Arena& tmp, int* err,
                              hipStream_t s) {
  if (nterm == 0) return;
  size_t total = 0;
  int nmax = 0;
  std::vector<int> tiles;
  for (int t = 0; t < nterm; ++t) {
    const int n = h_term[t].n;
    total += (size_t)n * n;
    nmax = std::max(nmax, n);
    const int nt = (n + kUpdTile - 1) / kUpdTile;
    for (int q = 0; q < nt * nt; ++q) {
      tiles.push_back(t);
      tiles.push_back(q);
    }
  }
  // panel width b and rows per thread R with b * R = 32 register doubles; a
  // workgroup of just enough waves for the largest system
  int b = 32, R = 1;
  while (R * kPanelThreads < nmax) {
    b /= 2;
    R *= 2;
  }
  const int pth = R > 1 ? kPanelThreads : std::max(kWave, (nmax + kWave - 1) / kWave * kWave);
  if (b < 4) throw Error(AMG_ECOARSEN, "coarsest system too large for the register panel");
  launch_fill_double(total, inv, 0.0, s);
  k_dense_scatter_batched<<<nterm, 256, 0, s>>>(d_term, rp, ci, val, inv);
  double* ybuf = tmp.alloc_n<double>((size_t)nrows * b);
  double* tbuf = tmp.alloc_n<double>((size_t)nrows * b);
  int* d_tiles = tmp.alloc_n<int>(tiles.size());
  AMG_HIP(hipMemcpyAsync(d_tiles, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, s));
  const int npanels = (nmax + b - 1) / b;
  const int ntiles = (int)(tiles.size() / 2);
  // panels of 32 columns: pivot block + product; narrower panels (systems of
  // more than 1024 rows) keep the one-workgroup register panel
  int* d_items = nullptr;
  int* d_ptiles = nullptr;
  double* xbuf = nullptr;
  int nitems = 0, nptiles = 0;
  if (b == 32) {
    std::vector<int> items, ptiles;
    for (int t = 0; t < nterm; ++t) {
      for (int rb = 0; rb * 256 < h_term[t].n; ++rb) {
        items.push_back(t);
        items.push_back(rb);
      }
      for (int q = 0; q * kUpdTile < h_term[t].n; ++q) {   // mode-2 tiles: one per column tile
        ptiles.push_back(t);
        ptiles.push_back(q);
      }
    }
    nitems = (int)(items.size() / 2);
    nptiles = (int)(ptiles.size() / 2);
    d_items = tmp.alloc_n<int>(items.size());
    d_ptiles = tmp.alloc_n<int>(ptiles.size());
    xbuf = tmp.alloc_n<double>((size_t)nterm * 32 * 32);
    AMG_HIP(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(d_ptiles, ptiles.data(), ptiles.size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  for (int K = 0; K < npanels; ++K) {
    switch (b) {
      case 32:
        k_gjb_pivot<<<nterm, 1024, 0, s>>>(d_term, inv, ybuf, xbuf, K, err);
        k_gjb_apply<<<nitems, 256, 0, s>>>(d_term, d_items, inv, ybuf, xbuf, K);
        k_gjb_update<<<ntiles, 256, 0, s>>>(d_term, d_tiles, inv, ybuf, nullptr, K, b, 1);
        k_gjb_update<<<nptiles, 256, 0, s>>>(d_term, d_ptiles, inv, ybuf, nullptr, K, b, 2);
        continue;
      case 16: k_gjb_panel_reg<16, 2><<<nterm, pth, 0, s>>>(d_term, inv, ybuf, tbuf, K, err); break;
      case 8: k_gjb_panel_reg<8, 4><<<nterm, pth, 0, s>>>(d_term, inv, ybuf, tbuf, K, err); break;
      default: k_gjb_panel_reg<4, 8><<<nterm, pth, 0, s>>>(d_term, inv, ybuf, tbuf, K, err); break;
    }
    k_gjb_update<<<ntiles, 256, 0, s>>>(d_term, d_tiles, inv, ybuf, tbuf, K, b, 0);
  }
  if (inv32) k_dense_to_float<<<(int)std::min<size_t>((total + 255) / 256, 4096), 256, 0, s>>>(total, inv, inv32);
  AMG_HIP(hipStreamSynchronize(s));   // the host tile table is read before it goes away
}

}  // namespace amg
