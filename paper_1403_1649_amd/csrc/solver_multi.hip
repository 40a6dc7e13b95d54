// Several right-hand sides with one hierarchy: the cycle of Algorithms 4/5 and
// the outer flexible CG applied to a row-major block X[n][R] (R <= 64).
// Each matrix row is handled by W = pow2(R) lanes, lane c owning column c:
// the row's values and columns are loaded once (a broadcast within the lane
// group) and the gathered X rows are contiguous, so A is streamed once for
// all R columns.  Per level, an autotuner may instead split the columns into
// tiles of W/2 or W/4 (one pass over A each), where the narrower gathered
// working set stays in the caches.  Every scalar of the K-cycle and of the outer iteration is
// per column, and so is the K-cycle branch: the second inner step runs when
// any column needs it, and only the columns that need it use its result, so
// each column follows exactly the arithmetic of a single-column solve.
// Converged columns stop updating; kernels stop when no column is running.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <vector>

#include "kernels_common.hpp"

namespace amg {

namespace {

constexpr int kMaxRhs = 64;
constexpr int kMultiBlocks = 2048;   // reducing block kernels: blocks (and partials per total)

// per-column scalar slots: slot s of column c at sc[s * R + c]
enum : int {
  mBB = 0, mRtol2, mAlpha, mBeta, mPQ, mRR, mTrue, mK0,   // K-level k: mK0 + 16 k + KSlot
  mSlots = mK0 + 16 * 24,
};
// per-column int flags: word w of column c at fl[w * R + c]
enum : int {
  fRun = 0, fIters, fK0,   // K-level k: fK0 + 2 k (+0 step-2, +1 use-d)
  fWords = fK0 + 2 * 24,
};
// single words (any column): any running, any step 2 on level k
enum : int { aRun = 0, aK0 = 1, aWords = 1 + 24 };

struct MCtx {
  int R;
  double* sc;
  int* fl;
  int* any;
  double* part;
  int* err;
  double* tot;        // totals of a reduction, NV * R
  unsigned* ticket;   // arrival counter of the finalize blocks (zero between kernels)
};

struct ActAny {
  const int* p;
  __device__ __forceinline__ bool on() const { return p == nullptr || *p != 0; }
};

// per-block partials of columns c0 .. c0 + W - 1
template <int NV, int W>
__device__ __forceinline__ void write_partials_m(double (&acc)[NV], int R, int c0, double* part) {
  __shared__ double red[NV][kBlock / kWave][W];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = W; off < kWave; off <<= 1) acc[k] += __shfl_xor(acc[k], off, kWave);
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane < W) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid][lane] = acc[k];
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < W && c0 + c < R) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < kBlock / kWave; ++w) s += red[k][w][c];
      part[((size_t)k * R + c0 + c) * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Per-column totals, then the op's per-column and all-column finalizers.
// One block per (value, column) total: its threads add the partials of blocks
// t, t + 256, ... in order and a fixed block reduction combines them, so the
// totals do not depend on timing; the last block to arrive (a ticket counter,
// after a release fence of the one value each block wrote) runs the
// finalizers on all totals.
constexpr int kFinMBlock = 256;
template <class Op>
__global__ void __launch_bounds__(kFinMBlock) k_finalize_m(Op op, const double* __restrict__ part, int nb, int R,
                                                           double* tot, unsigned* ticket) {
  if (!op.active()) return;
  constexpr int NV = Op::NV;
  __shared__ double red[kFinMBlock / kWave];
  __shared__ int s_last;
  const int q = blockIdx.x;
  const double* p = part + (size_t)q * nb;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += kFinMBlock) v[0] += p[b];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) {
    tot[q] = v[0];
    __threadfence();
    s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const int c = threadIdx.x;
  if (c < R) {
    double t[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] = __hip_atomic_load(&tot[k * R + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    op.finalize(c, t);
  }
  __syncthreads();
  if (c == 0) {
    op.finalize_all();
    *ticket = 0u;
  }
}

__device__ __forceinline__ int xcd_block() {
  const int g = gridDim.x, b = blockIdx.x;
  if (g < 8 || (g & 7)) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

// rows of A times columns c0 .. c0 + W - 1 of the block, W lanes per row
template <typename T, int W, class Op>
__global__ void __launch_bounds__(kBlock) k_rows_m(int n, int R, int c0, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const T* __restrict__ av,
                                                   Op op, double* part) {
  if (!op.active()) {
    if (blockIdx.x == 0 && threadIdx.x == 0) op.idle();
    return;
  }
  constexpr int NV = Op::NV > 0 ? Op::NV : 1;
  constexpr int RPB = kBlock / W;
  const int c = c0 + (threadIdx.x & (W - 1));
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  // The blocks of one XCD (block ids congruent mod 8) own a contiguous eighth
  // of the row groups and sweep it side by side, group j, j + blocks, ...:
  // the rows they gather at any time lie in one window of the XCD's L2.
  const int groups = (n + RPB - 1) / RPB;
  const int nx = (gridDim.x >= 8 && !(gridDim.x & 7)) ? 8 : 1;
  const int bpx = gridDim.x / nx;
  const int gpx = (groups + nx - 1) / nx;
  const int gbeg = (blockIdx.x % nx) * gpx, gend = min(groups, gbeg + gpx);
  for (int g = gbeg + blockIdx.x / nx; g < gend; g += bpx) {
    const int row = g * RPB + threadIdx.x / W;
    if (row < n && c < R) {
      T sum = T(0);
      const int e = rp[row + 1];
      // eight entries at a time: their columns and values, then the eight
      // gathered block rows, then the products in entry order, so the
      // gathers of a chunk are in flight together
      for (int k0 = rp[row]; k0 < e; k0 += 8) {
        int cj[8];
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          cj[q] = k0 + q < e ? ci[k0 + q] : 0;
          v[q] = k0 + q < e ? av[k0 + q] : T(0);
        }
        T xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) xv[q] = k0 + q < e ? op.x(cj[q], c) : T(0);
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (k0 + q < e) sum += v[q] * xv[q];
      }
      op.row(row, c, sum, acc);
    }
  }
  if constexpr (Op::NV > 0) write_partials_m<Op::NV, W>(acc, R, c0, part);
}

template <int W, class Op>
__global__ void __launch_bounds__(kBlock) k_elem_m(int n, int R, Op op, double* part) {
  if (!op.active()) {
    if (blockIdx.x == 0 && threadIdx.x == 0) op.idle();
    return;
  }
  constexpr int NV = Op::NV > 0 ? Op::NV : 1;
  constexpr int RPB = kBlock / W;
  const int c = threadIdx.x & (W - 1);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const int groups = (n + RPB - 1) / RPB;
  const int per = (groups + gridDim.x - 1) / gridDim.x;
  const int g0 = xcd_block() * per, g1 = min(groups, g0 + per);
  for (int g = g0; g < g1; ++g) {
    const int i = g * RPB + threadIdx.x / W;
    if (i < n && c < R) op.elem(i, c, acc);
  }
  if constexpr (Op::NV > 0) write_partials_m<Op::NV, W>(acc, R, 0, part);
}

inline int grid_m(int n, int W, bool reduce) {
  long rpb = kBlock / W;
  long g = (n + rpb - 1) / rpb;
  const long cap = reduce ? kMultiBlocks : kMaxPartialBlocks;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  if (g > 8) g &= ~7L;
  return (int)g;
}

// The columns in tiles of W (one pass over the rows per tile, so a tile's
// gathered block rows are a narrower working set in the caches), then the
// totals of all columns.
template <typename T, int W, class Op>
void rows_m_w(int n, const MCtx& m, const int* rp, const int* ci, const T* av, const Op& op, hipStream_t s) {
  const int g = grid_m(n, W, Op::NV > 0);
  for (int c0 = 0; c0 < m.R; c0 += W) k_rows_m<T, W, Op><<<g, kBlock, 0, s>>>(n, m.R, c0, rp, ci, av, op, m.part);
  if constexpr (Op::NV > 0) k_finalize_m<Op><<<Op::NV * m.R, kFinMBlock, 0, s>>>(op, m.part, g, m.R, m.tot, m.ticket);
}

template <int W, class Op>
void elem_m_w(int n, const MCtx& m, const Op& op, hipStream_t s) {
  const int g = grid_m(n, W, Op::NV > 0);
  k_elem_m<W, Op><<<g, kBlock, 0, s>>>(n, m.R, op, m.part);
  if constexpr (Op::NV > 0) k_finalize_m<Op><<<Op::NV * m.R, kFinMBlock, 0, s>>>(op, m.part, g, m.R, m.tot, m.ticket);
}

inline int width_of(int R) {
  int w = 1;
  while (w < R) w <<= 1;
  return w;
}

// tile: columns per pass (a power of two; 0 = all columns in one pass)
template <typename T, class Op>
void rows_m(int n, const MCtx& m, int tile, const int* rp, const int* ci, const T* av, const Op& op, hipStream_t s) {
  switch (tile > 0 ? std::min(tile, width_of(m.R)) : width_of(m.R)) {
    case 1: rows_m_w<T, 1>(n, m, rp, ci, av, op, s); break;
    case 2: rows_m_w<T, 2>(n, m, rp, ci, av, op, s); break;
    case 4: rows_m_w<T, 4>(n, m, rp, ci, av, op, s); break;
    case 8: rows_m_w<T, 8>(n, m, rp, ci, av, op, s); break;
    case 16: rows_m_w<T, 16>(n, m, rp, ci, av, op, s); break;
    case 32: rows_m_w<T, 32>(n, m, rp, ci, av, op, s); break;
    default: rows_m_w<T, 64>(n, m, rp, ci, av, op, s); break;
  }
}

template <class Op>
void elem_m(int n, const MCtx& m, const Op& op, hipStream_t s) {
  switch (width_of(m.R)) {
    case 1: elem_m_w<1>(n, m, op, s); break;
    case 2: elem_m_w<2>(n, m, op, s); break;
    case 4: elem_m_w<4>(n, m, op, s); break;
    case 8: elem_m_w<8>(n, m, op, s); break;
    case 16: elem_m_w<16>(n, m, op, s); break;
    case 32: elem_m_w<32>(n, m, op, s); break;
    default: elem_m_w<64>(n, m, op, s); break;
  }
}

// ------------------------------------------------------------------ ops
#define M_COMMON                                                  \
  __device__ bool active() const { return a.on(); }              \
  __device__ void idle() const {}                                \
  __device__ void finalize_all() const {}

template <typename T>
struct MPresmoothResid {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const T* b;
  const T* wd;
  T* xt;
  T* r;
  M_COMMON
  __device__ T x(int j, int c) const { return wd[j] * b[(size_t)j * R + c]; }
  __device__ void row(int i, int c, T ax, double*) const {
    const size_t q = (size_t)i * R + c;
    const T bi = b[q];
    xt[q] = wd[i] * bi;
    r[q] = bi - ax;
  }
  __device__ void finalize(int, const double*) const {}
};

template <typename T>
struct MResidSmooth {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const T* b;
  const T* xt;
  const T* wd;
  T* xo;
  M_COMMON
  __device__ T x(int j, int c) const { return xt[(size_t)j * R + c]; }
  __device__ void row(int i, int c, T ax, double*) const {
    const size_t q = (size_t)i * R + c;
    xo[q] = xt[q] + wd[i] * (b[q] - ax);
  }
  __device__ void finalize(int, const double*) const {}
};

template <typename T, bool DOT>
struct MRestrict {   // rows of R = P^T (aggregates) times the block
  static constexpr int NV = DOT ? 1 : 0;
  ActAny a;
  int R;
  const T* r;
  T* rcv;
  double* K;   // per-column K slots of this level (slot * R + c)
  M_COMMON
  __device__ T x(int j, int c) const { return r[(size_t)j * R + c]; }
  __device__ void row(int I, int c, T s, double* acc) const {
    rcv[(size_t)I * R + c] = s;
    if (DOT) acc[0] += (double)s * (double)s;
  }
  __device__ void finalize(int c, const double* v) const {
    if (DOT) K[kKRcRc * R + c] = v[0];
  }
};

template <typename T>
struct MProlong {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const int* agg;
  const T* pval;
  const T* cc;
  T* xt;
  M_COMMON
  __device__ void elem(int i, int c, double*) const {
    xt[(size_t)i * R + c] += pval[i] * cc[(size_t)agg[i] * R + c];
  }
  __device__ void finalize(int, const double*) const {}
};

template <typename T>
struct MKDots1 {
  static constexpr int NV = 2;
  ActAny a;
  int R;
  const T* cc;
  const T* rcv;
  T* v;
  double* K;
  int gmres;
  M_COMMON
  __device__ T x(int j, int c) const { return cc[(size_t)j * R + c]; }
  __device__ void row(int i, int c, T ax, double* acc) const {
    const size_t q = (size_t)i * R + c;
    v[q] = ax;
    const double l = gmres ? (double)ax : (double)cc[q];
    acc[0] += l * (double)ax;
    acc[1] += l * (double)rcv[q];
  }
  __device__ void finalize(int c, const double* s) const {
    K[kKRho1 * R + c] = s[0];
    K[kKAlpha1 * R + c] = s[1];
  }
};

template <typename T>
struct MRtilde {
  static constexpr int NV = 1;
  ActAny a;
  int R;
  const T* rcv;
  const T* v;
  T* rt;
  double* K;
  int* F;       // per-column: F[c] step 2, F[R + c] use d
  int* any2;    // any column needs step 2
  double t;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const { *any2 = 0; }
  __device__ void elem(int i, int c, double* acc) const {
    const size_t q = (size_t)i * R + c;
    const T ar = (T)(K[kKAlpha1 * R + c] / K[kKRho1 * R + c]);
    const T u = rcv[q] - ar * v[q];
    rt[q] = u;
    acc[0] += (double)u * (double)u;
  }
  __device__ void finalize(int c, const double* s) const {
    const double rho1 = K[kKRho1 * R + c];
    K[kKRtRt * R + c] = s[0];
    F[R + c] = 0;
    if (rho1 > 0.0) {
      K[kKCoefC * R + c] = K[kKAlpha1 * R + c] / rho1;
      F[c] = (sqrt(s[0]) <= t * sqrt(K[kKRcRc * R + c])) ? 0 : 1;
    } else {
      K[kKCoefC * R + c] = 0.0;
      F[c] = 0;
    }
  }
  __device__ void finalize_all() const {
    int any = 0;
    for (int c = 0; c < R; ++c) any |= F[c];
    *any2 = any;
  }
};

template <typename T>
struct MKDots2 {
  static constexpr int NV = 3;
  ActAny a;
  int R;
  const T* d;
  const T* v;
  const T* rt;
  T* w;
  double* K;
  int* F;
  int gmres;
  M_COMMON
  __device__ T x(int j, int c) const { return d[(size_t)j * R + c]; }
  __device__ void row(int i, int c, T ax, double* acc) const {
    const size_t q = (size_t)i * R + c;
    w[q] = ax;
    const double l = gmres ? (double)ax : (double)d[q];
    acc[0] += l * (double)v[q];
    acc[1] += l * (double)ax;
    acc[2] += l * (double)rt[q];
  }
  __device__ void finalize(int c, const double* s) const {
    if (!F[c]) return;
    const double gamma = s[0], beta = s[1], alpha2 = s[2];
    const double rho1 = K[kKRho1 * R + c], alpha1 = K[kKAlpha1 * R + c];
    const double rho2 = beta - gamma * gamma / rho1;
    if (rho2 > 0.0) {
      K[kKCoefC * R + c] = alpha1 / rho1 - gamma * alpha2 / (rho1 * rho2);
      K[kKCoefD * R + c] = alpha2 / rho2;
      F[R + c] = 1;
    }
  }
};

template <typename T>
struct MProlongK {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const int* agg;
  const T* pval;
  const T* cc;
  const T* d;
  T* xt;
  const double* K;
  const int* F;
  M_COMMON
  __device__ void elem(int i, int c, double*) const {
    const size_t I = (size_t)agg[i] * R + c;
    T xc = (T)K[kKCoefC * R + c] * cc[I];
    if (F[R + c]) xc += (T)K[kKCoefD * R + c] * d[I];
    xt[(size_t)i * R + c] += pval[i] * xc;
  }
  __device__ void finalize(int, const double*) const {}
};

// coarsest level: X_L = A_L^-1 B_L on the FP64 matrix cores, one block per
// 16 x 16 tile of X (rows x right-hand sides); the block's four waves split
// the inner dimension (in steps of 4 over the inverse's columns, zero-padded)
// into four contiguous parts and their accumulators are added in wave order
// through LDS.  Operands of the FP32 cycle are widened.
constexpr int kGemmSplit = kBlock / kWave;
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gemm_coarse(int n, int R, const double* __restrict__ Ainv,
                                                        const T* __restrict__ B, T* __restrict__ X, ActAny a) {
  if (!a.on()) return;
  __shared__ double part[kGemmSplit][4][kWave];
  const int tiles_c = (R + 15) / 16;
  const int tile = blockIdx.x;
  const int w = threadIdx.x / kWave;
  const int l = threadIdx.x & (kWave - 1);
  const int R0 = (tile / tiles_c) * 16, C0 = (tile % tiles_c) * 16;
  const int ar = R0 + (l & 15), bc = C0 + (l & 15);
  const int ksteps = (n + 3) / 4;
  const int per = (ksteps + kGemmSplit - 1) / kGemmSplit;
  const int k0 = w * per * 4, k1 = min(n, (w + 1) * per * 4);
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k = k0; k < k1; k += 4) {
    const int kk = k + (l >> 4);
    const double av = (ar < n && kk < k1) ? Ainv[(size_t)ar * n + kk] : 0.0;
    const double bv = (bc < R && kk < k1) ? (double)B[(size_t)kk * R + bc] : 0.0;
    acc = mfma_f64_16x16x4(av, bv, acc);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) part[w][i][l] = acc[i];
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = part[0][i][l];
    for (int q = 1; q < kGemmSplit; ++q) v += part[q][i][l];
    const int row = R0 + mfma_row(l, i), col = C0 + mfma_col(l);
    if (row < n && col < R) X[(size_t)row * R + col] = (T)v;
  }
}

// outer flexible CG, per column
struct MFcgInit {
  static constexpr int NV = 1;
  ActAny a;
  int R;
  const double* b;
  double* r;
  double* xv;
  double* sc;
  int* fl;
  int* any;
  int* err;
  double rtol;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, int c, double* acc) const {
    const size_t q = (size_t)i * R + c;
    const double t = b[q];
    r[q] = t;
    xv[q] = 0.0;
    acc[0] += t * t;
  }
  __device__ void finalize(int c, const double* s) const {
    sc[mBB * R + c] = s[0];
    sc[mRtol2 * R + c] = rtol * rtol * s[0];
    fl[fIters * R + c] = 0;
    fl[fRun * R + c] = s[0] > 0.0 ? 1 : 0;
    if (!__builtin_isfinite(s[0])) {
      *err |= kErrNonFinite;
      fl[fRun * R + c] = 0;
    }
  }
  __device__ void finalize_all() const {
    int x = 0;
    for (int c = 0; c < R; ++c) x |= fl[fRun * R + c];
    any[aRun] = x;
  }
};

struct MFcgSpmv {
  static constexpr int NV = 2;
  ActAny a;
  int R;
  const double* p;
  const double* r;
  double* q;
  double* sc;
  int* fl;
  int* any;
  int* err;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ double x(int j, int c) const { return p[(size_t)j * R + c]; }
  __device__ void row(int i, int c, double ax, double* acc) const {
    const size_t k = (size_t)i * R + c;
    q[k] = ax;
    acc[0] += p[k] * ax;
    acc[1] += p[k] * r[k];
  }
  __device__ void finalize(int c, const double* s) const {
    if (!fl[fRun * R + c]) return;
    sc[mPQ * R + c] = s[0];
    sc[mAlpha * R + c] = s[1] / s[0];
    fl[fIters * R + c] += 1;
    if (!(s[0] > 0.0)) {
      *err |= __builtin_isfinite(s[0]) ? kErrBreakdown : kErrNonFinite;
      fl[fRun * R + c] = 0;
    }
  }
  __device__ void finalize_all() const {
    int x = 0;
    for (int c = 0; c < R; ++c) x |= fl[fRun * R + c];
    any[aRun] = x;
  }
};

struct MFcgUpdate {
  static constexpr int NV = 1;
  ActAny a;
  int R;
  const double* p;
  const double* q;
  double* xv;
  double* r;
  double* sc;
  int* fl;
  int* any;
  int* err;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, int c, double* acc) const {
    if (!fl[fRun * R + c]) return;
    const size_t k = (size_t)i * R + c;
    const double al = sc[mAlpha * R + c];
    xv[k] += al * p[k];
    const double t = r[k] - al * q[k];
    r[k] = t;
    acc[0] += t * t;
  }
  __device__ void finalize(int c, const double* s) const {
    if (!fl[fRun * R + c]) return;
    sc[mRR * R + c] = s[0];
    if (!__builtin_isfinite(s[0])) {
      *err |= kErrNonFinite;
      fl[fRun * R + c] = 0;
    } else if (s[0] <= sc[mRtol2 * R + c]) {
      fl[fRun * R + c] = 0;
    }
  }
  __device__ void finalize_all() const {
    int x = 0;
    for (int c = 0; c < R; ++c) x |= fl[fRun * R + c];
    any[aRun] = x;
  }
};

template <typename T>
struct MDotZQ {
  static constexpr int NV = 1;
  ActAny a;
  int R;
  const T* z;
  const double* q;
  double* sc;
  M_COMMON
  __device__ void elem(int i, int c, double* acc) const {
    const size_t k = (size_t)i * R + c;
    acc[0] += (double)z[k] * q[k];
  }
  __device__ void finalize(int c, const double* s) const { sc[mBeta * R + c] = -s[0] / sc[mPQ * R + c]; }
};

template <typename T>
struct MPUpdate {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const T* z;
  double* p;
  const double* sc;
  const int* fl;
  int first;
  M_COMMON
  __device__ void elem(int i, int c, double*) const {
    if (!fl[fRun * R + c]) return;
    const size_t k = (size_t)i * R + c;
    p[k] = first ? (double)z[k] : (double)z[k] + sc[mBeta * R + c] * p[k];
  }
  __device__ void finalize(int, const double*) const {}
};

struct MToFloat {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const double* in;
  float* out;
  M_COMMON
  __device__ void elem(int i, int c, double*) const {
    const size_t k = (size_t)i * R + c;
    out[k] = (float)in[k];
  }
  __device__ void finalize(int, const double*) const {}
};

struct MTrueResid {
  static constexpr int NV = 1;
  ActAny a;
  int R;
  const double* b;
  const double* xv;
  double* r;
  double* sc;
  M_COMMON
  __device__ double x(int j, int c) const { return xv[(size_t)j * R + c]; }
  __device__ void row(int i, int c, double ax, double* acc) const {
    const size_t k = (size_t)i * R + c;
    const double t = b[k] - ax;
    r[k] = t;
    acc[0] += t * t;
  }
  __device__ void finalize(int c, const double* s) const { sc[mTrue * R + c] = s[0]; }
};

// Y = A X: the kernel the block autotuner times
template <typename T>
struct MSpmvT {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const T* xin;
  T* y;
  M_COMMON
  __device__ T x(int j, int c) const { return xin[(size_t)j * R + c]; }
  __device__ void row(int i, int c, T ax, double*) const { y[(size_t)i * R + c] = ax; }
  __device__ void finalize(int, const double*) const {}
};

// restart the columns whose recurrence converged but whose true residual did
// not: r = b - A x for them, running again
struct MRestartMask {
  static constexpr int NV = 0;
  ActAny a;
  int R;
  const double* rtrue;
  double* r;
  const int* again;   // host-chosen columns
  int* fl;
  int* any;
  M_COMMON
  __device__ void elem(int i, int c, double*) const {
    if (!again[c]) return;
    const size_t k = (size_t)i * R + c;
    r[k] = rtrue[k];
    if (i == 0) {
      fl[fRun * R + c] = 1;
      any[aRun] = 1;
    }
  }
  __device__ void finalize(int, const double*) const {}
};

#undef M_COMMON

// ------------------------------------------------------------ typed views
template <typename T> const T* vals_t(const Level& l);
template <> const double* vals_t<double>(const Level& l) { return l.val; }
template <> const float* vals_t<float>(const Level& l) { return l.val32; }
template <typename T> const T* wdinv_t(const Level& l);
template <> const double* wdinv_t<double>(const Level& l) { return l.wdinv; }
template <> const float* wdinv_t<float>(const Level& l) { return l.wdinv32; }
template <typename T> const T* pvals_t(const Level& l);
template <> const double* pvals_t<double>(const Level& l) { return l.pval; }
template <> const float* pvals_t<float>(const Level& l) { return l.pval32; }
template <typename T> const T* rvals_t(const Level& l);
template <> const double* rvals_t<double>(const Level& l) { return l.rval; }
template <> const float* rvals_t<float>(const Level& l) { return l.rval32; }

// per-level work blocks [n][R] (or [n_{k+1}][R])
struct MLevel {
  void *r, *xt, *rc, *c, *v, *rt, *d, *w;
};

struct MWork {
  int R = 0;
  Arena arena;
  std::vector<MLevel> lv;
  std::vector<int> tile;    // per level: columns per pass of the cycle's block kernels (0 = all)
  int tile0 = 0;            // ... of the FP64 level-0 products of the outer iteration
  double tune_ms = 0.0;     // host time of choosing them
  double *r = nullptr, *p = nullptr, *q = nullptr, *xv = nullptr, *rtrue = nullptr;
  void* z = nullptr;
  void* bz = nullptr;
  MCtx m{};
  int* again = nullptr;
};

template <typename T>
void coarse_m(Hierarchy& h, const MCtx& m, const T* b, T* x, const int* act) {
  const int n = h.levels.back().n;
  const int tiles = ((n + 15) / 16) * ((m.R + 15) / 16);
  k_gemm_coarse<T><<<tiles, kBlock, 0, h.stream>>>(n, m.R, h.cinv, b, x, ActAny{act});
}

template <typename T>
void cycle_m(Hierarchy& h, MWork& W, int k, const T* b, T* xo, const int* act) {
  const MCtx& m = W.m;
  hipStream_t s = h.stream;
  if (h.L() == 0) {
    coarse_m<T>(h, m, b, xo, act);
    return;
  }
  Level& lv = h.levels[k];
  MLevel& ml = W.lv[k];
  const int R = m.R, L = h.L();
  T* xt = static_cast<T*>(ml.xt);
  T* r = static_cast<T*>(ml.r);
  T* rcv = static_cast<T*>(ml.rc);
  T* c = static_cast<T*>(ml.c);
  const T* wd = wdinv_t<T>(lv);
  const T* pv = pvals_t<T>(lv);
  const ActAny A{act};
  const int tk = W.tile[k];                                  // columns per pass on level k's rows
  const int tc = k + 1 < L ? W.tile[k + 1] : 0;              // ... and on level k+1's
  rows_m<T>(lv.n, m, tk, lv.rp, lv.ci, vals_t<T>(lv), MPresmoothResid<T>{A, R, b, wd, xt, r}, s);
  const bool kcyc = k < h.opt.kcycle_levels && k + 1 < L;
  if (!kcyc) {
    rows_m<T>(lv.nc, m, tk, lv.agg_ptr, lv.agg_rows, rvals_t<T>(lv), MRestrict<T, false>{A, R, r, rcv, nullptr}, s);
    if (k + 1 == L) coarse_m<T>(h, m, rcv, c, act);
    else cycle_m<T>(h, W, k + 1, rcv, c, act);
    elem_m(lv.n, m, MProlong<T>{A, R, lv.agg, pv, c, xt}, s);
  } else {
    Level& lc = h.levels[k + 1];
    double* K = m.sc + (size_t)(mK0 + 16 * k) * R;
    int* F = m.fl + (size_t)(fK0 + 2 * k) * R;
    int* any2 = m.any + aK0 + k;
    T* v = static_cast<T*>(ml.v);
    T* rt = static_cast<T*>(ml.rt);
    T* d = static_cast<T*>(ml.d);
    T* w = static_cast<T*>(ml.w);
    const int gm = h.opt.krylov == AMG_KRYLOV_FGMRES ? 1 : 0;
    rows_m<T>(lv.nc, m, tk, lv.agg_ptr, lv.agg_rows, rvals_t<T>(lv), MRestrict<T, true>{A, R, r, rcv, K}, s);
    cycle_m<T>(h, W, k + 1, rcv, c, act);
    rows_m<T>(lc.n, m, tc, lc.rp, lc.ci, vals_t<T>(lc), MKDots1<T>{A, R, c, rcv, v, K, gm}, s);
    elem_m(lc.n, m, MRtilde<T>{A, R, rcv, v, rt, K, F, any2, h.opt.kcycle_t}, s);
    cycle_m<T>(h, W, k + 1, rt, d, any2);
    rows_m<T>(lc.n, m, tc, lc.rp, lc.ci, vals_t<T>(lc), MKDots2<T>{ActAny{any2}, R, d, v, rt, w, K, F, gm}, s);
    elem_m(lv.n, m, MProlongK<T>{A, R, lv.agg, pv, c, d, xt, K, F}, s);
  }
  rows_m<T>(lv.n, m, tk, lv.rp, lv.ci, vals_t<T>(lv), MResidSmooth<T>{A, R, b, xt, wd, xo}, s);
}

template <typename T>
void precondition_m(Hierarchy& h, MWork& W, const int* act) {
  const int n = h.levels[0].n;
  if constexpr (sizeof(T) == sizeof(float)) {
    elem_m(n, W.m, MToFloat{ActAny{act}, W.m.R, W.r, static_cast<float*>(W.bz)}, h.stream);
    cycle_m<float>(h, W, 0, static_cast<const float*>(W.bz), static_cast<float*>(W.z), act);
  } else {
    cycle_m<double>(h, W, 0, W.r, static_cast<double*>(W.z), act);
  }
}

template <typename T>
void iteration_m(Hierarchy& h, MWork& W) {
  const MCtx& m = W.m;
  const Level& l0 = h.levels[0];
  const int n = l0.n, R = m.R;
  const int* run = m.any + aRun;
  const ActAny A{run};
  hipStream_t s = h.stream;
  rows_m<double>(n, m, W.tile0, l0.rp, l0.ci, l0.val, MFcgSpmv{A, R, W.p, W.r, W.q, m.sc, m.fl, m.any, m.err}, s);
  elem_m(n, m, MFcgUpdate{A, R, W.p, W.q, W.xv, W.r, m.sc, m.fl, m.any, m.err}, s);
  precondition_m<T>(h, W, run);
  elem_m(n, m, MDotZQ<T>{A, R, static_cast<const T*>(W.z), W.q, m.sc}, s);
  elem_m(n, m, MPUpdate<T>{A, R, static_cast<const T*>(W.z), W.p, m.sc, m.fl, 0}, s);
}

template <typename T>
void restart_m(Hierarchy& h, MWork& W) {
  const int* run = W.m.any + aRun;
  precondition_m<T>(h, W, run);
  elem_m(h.levels[0].n, W.m, MPUpdate<T>{ActAny{run}, W.m.R, static_cast<const T*>(W.z), W.p, W.m.sc, W.m.fl, 1},
         h.stream);
}

void alloc_work(Hierarchy& h, MWork& W, int R) {
  const size_t es = h.mixed() ? sizeof(float) : sizeof(double);
  W.R = R;
  const int L = h.L();
  W.lv.assign(std::max(L, 1), MLevel{});
  W.tile.assign(std::max(L, 1), 0);
  for (int k = 0; k < L; ++k) {
    const Level& lv = h.levels[k];
    MLevel& ml = W.lv[k];
    const size_t n = (size_t)lv.n * R, nc = (size_t)lv.nc * R;
    ml.r = W.arena.alloc(n * es);
    ml.xt = W.arena.alloc(n * es);
    ml.rc = W.arena.alloc(nc * es);
    ml.c = W.arena.alloc(nc * es);
    if (k < h.opt.kcycle_levels) {
      ml.v = W.arena.alloc(nc * es);
      ml.rt = W.arena.alloc(nc * es);
      ml.d = W.arena.alloc(nc * es);
      ml.w = W.arena.alloc(nc * es);
    }
  }
  const size_t n0 = (size_t)h.levels[0].n * R;
  W.r = W.arena.alloc_n<double>(n0);
  W.p = W.arena.alloc_n<double>(n0);
  W.q = W.arena.alloc_n<double>(n0);
  W.xv = W.arena.alloc_n<double>(n0);
  W.z = W.arena.alloc(n0 * es);
  if (h.mixed()) W.bz = W.arena.alloc(n0 * es);
  W.m.R = R;
  W.m.sc = W.arena.alloc_n<double>((size_t)mSlots * R);
  W.m.fl = W.arena.alloc_n<int>((size_t)fWords * R);
  W.m.any = W.arena.alloc_n<int>(aWords);
  W.m.part = W.arena.alloc_n<double>((size_t)3 * R * kMultiBlocks);
  W.m.tot = W.arena.alloc_n<double>((size_t)3 * R);
  W.m.ticket = W.arena.alloc_n<unsigned>(64);
  launch_fill_int(64, reinterpret_cast<int*>(W.m.ticket), 0, h.stream);
  W.m.err = h.d_err;
  W.again = W.arena.alloc_n<int>(kMaxRhs);
  launch_fill_int((size_t)fWords * R, W.m.fl, 0, h.stream);
  launch_fill_int(aWords, W.m.any, 0, h.stream);
}

// Columns per pass of the block row kernels, per level and arithmetic type:
// the pre-smoothing-sized product Y = A_k X timed with all W = pow2(R)
// columns in one pass and in tiles of W/2 and W/4 (at least 8 columns), the
// fastest kept (ties to the wider tile).  Small levels, latency-bound, take
// all columns.  Cached like the single-vector choices, keyed by the column
// count as well; AMG_TUNE_FORCE_TILE = 8, 16, ... pins the tile (for tests).
constexpr int kTileTuneRows = 65536;

template <typename T>
int tune_tile(Hierarchy& h, const Level& lv, const MWork& W, T* x, T* y) {
  const int R = W.R, wf = width_of(R);
  if (const char* f = std::getenv("AMG_TUNE_FORCE_TILE")) {
    const int t = std::atoi(f);
    return (t > 0 && (t & (t - 1)) == 0) ? std::min(t, wf) : 0;
  }
  if (lv.n <= kTileTuneRows || wf < 16) return 0;
  TuneKey key;
  key.n = lv.n;
  key.nnz = lv.nnz;
  key.bytes = (int)sizeof(T);
  key.nrhs = R;
  key.rowstat = lv.sl_total;
  Level::Tune t;
  if (tune_cache_get(key, &t)) return t.tile;
  hipStream_t s = h.stream;
  AMG_HIP(hipMemsetAsync(x, 0, (size_t)lv.n * R * sizeof(T), s));
  const T* av = vals_t<T>(lv);
  const MSpmvT<T> op{ActAny{nullptr}, R, x, y};
  hipEvent_t e0 = h.ev[2], e1 = h.ev[3];
  float best_us = 1e30f;
  int best = wf;
  for (int tw = wf; tw >= 8 && tw * 4 >= wf; tw >>= 1) {
    rows_m<T>(lv.n, W.m, tw, lv.rp, lv.ci, av, op, s);
    float us = 1e30f;
    for (int trial = 0; trial < 2; ++trial) {
      AMG_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 4; ++r) rows_m<T>(lv.n, W.m, tw, lv.rp, lv.ci, av, op, s);
      AMG_HIP(hipEventRecord(e1, s));
      AMG_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
      us = std::min(us, ms * 1000.f / 4);
    }
    if (std::getenv("AMG_DEBUG"))
      std::fprintf(stderr, "amg: block tile n=%d R=%d bytes=%d tile=%d: %.2f us\n", lv.n, R, (int)sizeof(T), tw, us);
    if (us < best_us * 0.98f) {
      best_us = us;
      best = tw;
    }
  }
  t = Level::Tune{};
  t.tile = best == wf ? 0 : best;
  t.us = best_us;
  tune_cache_put(key, t);
  return t.tile;
}

void tune_tiles(Hierarchy& h, MWork& W) {
  const auto t0 = std::chrono::steady_clock::now();
  const int L = h.L();
  for (int k = 0; k < L; ++k) {
    const Level& lv = h.levels[k];
    const MLevel& ml = W.lv[k];
    W.tile[k] = h.mixed() ? tune_tile<float>(h, lv, W, static_cast<float*>(ml.xt), static_cast<float*>(ml.r))
                          : tune_tile<double>(h, lv, W, static_cast<double*>(ml.xt), static_cast<double*>(ml.r));
  }
  if (L > 0) W.tile0 = h.mixed() ? tune_tile<double>(h, h.levels[0], W, W.p, W.q) : W.tile[0];
  AMG_HIP(hipStreamSynchronize(h.stream));
  W.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (std::getenv("AMG_DEBUG")) {
    for (int k = 0; k < L; ++k) std::fprintf(stderr, "amg: block tile level %d R=%d: %d\n", k, W.R, W.tile[k]);
    std::fprintf(stderr, "amg: block tile level 0 fp64 R=%d: %d (%.1f ms)\n", W.R, W.tile0, W.tune_ms);
  }
}

// The block workspace of one column count and the block iteration and
// (re)start captured into HIP graphs: every kernel of an iteration reads its
// device flags, so one graph serves all branches, and the workspace stays with
// the hierarchy, so the graphs stay valid for later solves with as many columns.
struct MultiState {
  MWork W;
  hipGraphExec_t g_iter = nullptr;
  hipGraphExec_t g_restart = nullptr;
  MultiState() = default;
  MultiState(const MultiState&) = delete;
  MultiState& operator=(const MultiState&) = delete;
  ~MultiState() {
    if (g_iter) (void)hipGraphExecDestroy(g_iter);
    if (g_restart) (void)hipGraphExecDestroy(g_restart);
  }
};

void capture_multi(Hierarchy& h, MultiState& st) {
  hipStream_t user = h.stream;
  hipStream_t cs = nullptr;
  AMG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  auto finish = [&](hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    AMG_HIP(hipStreamEndCapture(cs, &g));
    AMG_HIP(hipGraphInstantiate(out, g, nullptr, nullptr, 0));
    AMG_HIP(hipGraphDestroy(g));
  };
  try {
    h.stream = cs;
    h.capturing = true;
    AMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    if (h.mixed()) iteration_m<float>(h, st.W);
    else iteration_m<double>(h, st.W);
    finish(&st.g_iter);
    AMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    if (h.mixed()) restart_m<float>(h, st.W);
    else restart_m<double>(h, st.W);
    finish(&st.g_restart);
  } catch (...) {
    h.stream = user;
    h.capturing = false;
    (void)hipStreamDestroy(cs);
    throw;
  }
  h.stream = user;
  h.capturing = false;
  AMG_HIP(hipStreamDestroy(cs));
}

// The workspace (and graphs) for R columns: the one kept from an earlier call
// with as many columns, or a new one.
MultiState& multi_state(Hierarchy& h, int R) {
  MultiState* st = static_cast<MultiState*>(h.multi.get());
  if (st && st->W.R == R) return *st;
  AMG_HIP(hipStreamSynchronize(h.stream));   // the old workspace is idle before it goes
  h.multi.reset();
  auto ns = std::make_shared<MultiState>();
  alloc_work(h, ns->W, R);
  if (!(h.opt.flags & AMG_FLAG_NO_TUNE)) tune_tiles(h, ns->W);
  if (!(h.opt.flags & AMG_FLAG_NO_GRAPH)) capture_multi(h, *ns);
  h.multi = ns;
  return *ns;
}

void enqueue_iteration_m(Hierarchy& h, MultiState& st) {
  if (st.g_iter) AMG_HIP(hipGraphLaunch(st.g_iter, h.stream));
  else if (h.mixed()) iteration_m<float>(h, st.W);
  else iteration_m<double>(h, st.W);
}

void enqueue_restart_m(Hierarchy& h, MultiState& st) {
  if (st.g_restart) AMG_HIP(hipGraphLaunch(st.g_restart, h.stream));
  else if (h.mixed()) restart_m<float>(h, st.W);
  else restart_m<double>(h, st.W);
}

}  // namespace

// The column tiles of the block solve with R columns (its workspace must be
// the hierarchy's current one): tiles[k], k < L, for the cycle's kernels on
// level k's rows, tiles[L] for the FP64 level-0 products of the outer
// iteration; a tile of W = pow2(R) is one pass over all columns.
int multi_tiles(const Hierarchy& h, int R, int* tiles, int cap, double* tune_ms) {
  const MultiState* st = static_cast<const MultiState*>(h.multi.get());
  const int L = h.L();
  if (!st || st->W.R != R || cap < L + 1) return AMG_EINVAL;
  const int wf = width_of(R);
  for (int k = 0; k < L; ++k) tiles[k] = st->W.tile[k] > 0 ? st->W.tile[k] : wf;
  tiles[L] = st->W.tile0 > 0 ? st->W.tile0 : wf;
  if (tune_ms) *tune_ms = st->W.tune_ms;
  return AMG_OK;
}

// Solve A X = B for R columns from X_0 = 0.  iters / relres: host arrays[R].
int solve_multi_impl(Hierarchy& h, int R, const double* B, double rtol, double* X, int* iters, double* relres) {
  if (R < 1 || R > kMaxRhs) throw Error(AMG_EINVAL, "nrhs must be in [1, 64]");
  hipStream_t s = h.stream;
  struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
  MultiState& st = multi_state(h, R);
  MWork& W = st.W;
  launch_fill_int((size_t)fWords * R, W.m.fl, 0, s);
  launch_fill_int(aWords, W.m.any, 0, s);
  const Level& l0 = h.levels[0];
  const int n = l0.n;
  std::vector<int> hfl((size_t)fWords * R);
  std::vector<double> hsc((size_t)mK0 * R);
  std::vector<int> again(R);
  elem_m(n, W.m, MFcgInit{ActAny{nullptr}, R, B, W.r, W.xv, W.m.sc, W.m.fl, W.m.any, W.m.err, rtol}, s);
  enqueue_restart_m(h, st);
  const int max_iter = h.opt.max_iter;
  int enqueued = 0;
  int status = AMG_OK;
  int* hp = static_cast<int*>(h.h_pinned);
  while (true) {
    const int batch = std::min(4, max_iter - enqueued);
    for (int i = 0; i < batch; ++i) enqueue_iteration_m(h, st);
    enqueued += batch;
    AMG_HIP(hipGetLastError());
    AMG_HIP(hipMemcpyAsync(hp, W.m.any + aRun, sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hp + 1, h.d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    if (hp[1]) {
      if (hp[1] & kErrNonFinite) throw Error(AMG_ENANINF, "non-finite value in the iteration");
      if (hp[1] & kErrBreakdown) throw Error(AMG_EBREAKDOWN, "Krylov breakdown");
      throw Error(AMG_EHIP, "device error bits " + std::to_string(hp[1]));
    }
    if (hp[0] && enqueued < max_iter) continue;
    rows_m<double>(n, W.m, W.tile0, l0.rp, l0.ci, l0.val, MTrueResid{ActAny{nullptr}, R, B, W.xv, W.q, W.m.sc}, s);
    AMG_HIP(hipMemcpyAsync(hfl.data(), W.m.fl, hfl.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hsc.data(), W.m.sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    bool any_again = false;
    for (int c = 0; c < R; ++c) {
      const double bb = hsc[mBB * R + c];
      const double rel = bb > 0.0 ? std::sqrt(hsc[mTrue * R + c] / bb) : 0.0;
      if (!std::isfinite(rel)) throw Error(AMG_ENANINF, "non-finite residual");
      iters[c] = hfl[fIters * R + c];
      relres[c] = rel;
      again[c] = (rel > rtol && bb > 0.0 && iters[c] < max_iter && enqueued < max_iter) ? 1 : 0;
      any_again |= again[c] != 0;
      if (rel > rtol && bb > 0.0 && !again[c]) status = AMG_ENOTCONV;
    }
    if (!any_again) break;
    AMG_HIP(hipMemcpyAsync(W.again, again.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
    elem_m(n, W.m, MRestartMask{ActAny{nullptr}, R, W.q, W.r, W.again, W.m.fl, W.m.any}, s);
    enqueue_restart_m(h, st);
  }
  AMG_HIP(hipMemcpyAsync(X, W.xv, (size_t)n * R * sizeof(double), hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipStreamSynchronize(s));
  return status;
}

}  // namespace amg
