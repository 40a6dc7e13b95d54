// Many independent systems in one launch sequence.  The systems sit on the
// block diagonal of one matrix; every level of the hierarchy is again block
// diagonal, system s owning a contiguous row range (empty once it has passed
// its coarsest level).  Setup (Algorithm 1) runs each kernel once over all
// systems; the solve runs the cycle of Algorithms 4/5 and the outer flexible
// CG over all rows at once with every scalar kept per system, so each system
// follows the arithmetic of a solve on its own.
//
// Reductions are segmented by a block table: each block covers rows of one
// system only, writes one partial per reduction, and a one-block finalize
// sums each system's blocks in order (deterministic, no atomics).  The table
// also gives every block its system, so per-system scalars are read once per
// block and blocks of systems that are masked off (converged, or not taking
// the second inner K-cycle step) skip their rows.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels_common.hpp"

namespace amg {

namespace {

constexpr int kBatchBlocks = 8192;   // target number of blocks per level

// per-system scalar slots: slot q of system s at sc[q * nsys + s]
enum : int {
  bBB = 0, bRtol2, bAlpha, bBeta, bPQ, bRR, bTrue, bArnNorm, bArn,   // Arnoldi H: bArn + 8 i + j, norms bArn + 48 + j
  bK0 = bArn + 64,                                                  // K-level k: bK0 + 16 k + KSlot
  bSlots = bK0 + 16 * 24,
};
// per-system int flags: word w of system s at fl[w * nsys + s]
enum : int { fRun = 0, fIters, fK0, fWords = fK0 + 2 * 24 };   // K-level k: fK0 + 2k (+0 step 2, +1 use d)
// words over all systems
enum : int { aRun = 0, aK0 = 1, aWords = 1 + 24 };

constexpr int kBNV = 3;   // largest number of fused reductions

// ---------------------------------------------------------------- skeletons
struct Mask {
  const int* any;    // kernel-wide enable (nullable)
  const int* sys;    // per-system enable (nullable)
  __device__ __forceinline__ bool active() const { return any == nullptr || *any != 0; }
  __device__ __forceinline__ bool on(int s) const { return sys == nullptr || sys[s] != 0; }
};

__device__ __forceinline__ int logical_block() {
  const int g = gridDim.x, b = blockIdx.x;
  if (g < 8 || (g & 7)) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

template <int NV>
__device__ __forceinline__ void write_part(double (&acc)[NV], double* part, int nb, int lb) {
  __shared__ double red[NV * (kBlock / kWave)];
  block_sum<NV>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(size_t)k * nb + lb] = acc[k];
  }
}

// Op: NV, Mask m, T x(int j), row(int i, int s, T ax, double* acc),
//     finalize(int s, const double* v), skip(int s), finalize_all()
template <typename T, int LPR, class Op>
__global__ void __launch_bounds__(kBlock) k_brows(const int* __restrict__ blk, int nb, const int* __restrict__ rp,
                                                  const int* __restrict__ ci, const T* __restrict__ av, Op op,
                                                  double* part) {
  if (!op.m.active()) return;
  constexpr int NV = Op::NV > 0 ? Op::NV : 1;
  constexpr int RPB = kBlock / LPR;
  const int lb = logical_block();
  const int sys = blk[3 * lb], r0 = blk[3 * lb + 1], r1 = blk[3 * lb + 2];
  const int lane = threadIdx.x & (LPR - 1);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (sys >= 0 && op.m.on(sys)) {
    for (int base = r0; base < r1; base += RPB) {
      const int row = base + threadIdx.x / LPR;
      T sum = T(0);
      if (row < r1) {
        const int s = rp[row], e = rp[row + 1];
        for (int k = s + lane; k < e; k += LPR) sum += av[k] * op.x(ci[k]);
      }
      sum = group_sum<LPR>(sum);
      if (row < r1 && lane == 0) op.row(row, sys, sum, acc);
    }
  }
  if constexpr (Op::NV > 0) write_part<Op::NV>(acc, part, nb, lb);
}

template <class Op>
__global__ void __launch_bounds__(kBlock) k_belem(const int* __restrict__ blk, int nb, Op op, double* part) {
  if (!op.m.active()) return;
  constexpr int NV = Op::NV > 0 ? Op::NV : 1;
  const int lb = logical_block();
  const int sys = blk[3 * lb], r0 = blk[3 * lb + 1], r1 = blk[3 * lb + 2];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (sys >= 0 && op.m.on(sys)) {
    for (int i = r0 + threadIdx.x; i < r1; i += kBlock) op.elem(i, sys, acc);
  }
  if constexpr (Op::NV > 0) write_part<Op::NV>(acc, part, nb, lb);
}

// per-system totals: one wave per system (lanes stride over its blocks, then
// a fixed shuffle tree), so the sum order is fixed; masked-off systems get
// skip()
constexpr int kFinThreads = 1024;

template <class Op>
__global__ void __launch_bounds__(kFinThreads) k_bfinal(Op op, const double* __restrict__ part, int nb,
                                                        const int* __restrict__ blk_sys, int nsys) {
  if (!op.m.active()) return;
  constexpr int NV = Op::NV;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  for (int s = wv; s < nsys; s += kFinThreads / kWave) {
    if (!op.m.on(s)) {
      if (lane == 0) op.skip(s);
      continue;
    }
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = 0.0;
      for (int b = blk_sys[s] + lane; b < blk_sys[s + 1]; b += kWave) t += part[(size_t)k * nb + b];
      v[k] = wave_sum(t);
    }
    if (lane == 0) op.finalize(s, v);
  }
  __syncthreads();
  if (threadIdx.x == 0) op.finalize_all();
}

struct BCtx {
  int nsys;
  double* part;
};

// rows of a CSR matrix (rp, ci, av) whose rows are those of the level `tab`
// (A_k itself, or R_k = P_k^T over the rows of level k+1)
template <typename T, class Op>
void brows_on(const Level& tab, int lpr, const int* rp, const int* ci, const T* av, const BCtx& c, const Op& op,
              hipStream_t s) {
  if (tab.nblk == 0) return;
  const int g = tab.nblk;
  switch (lpr) {
    case 2: k_brows<T, 2, Op><<<g, kBlock, 0, s>>>(tab.blk, g, rp, ci, av, op, c.part); break;
    case 4: k_brows<T, 4, Op><<<g, kBlock, 0, s>>>(tab.blk, g, rp, ci, av, op, c.part); break;
    case 8: k_brows<T, 8, Op><<<g, kBlock, 0, s>>>(tab.blk, g, rp, ci, av, op, c.part); break;
    case 16: k_brows<T, 16, Op><<<g, kBlock, 0, s>>>(tab.blk, g, rp, ci, av, op, c.part); break;
    case 32: k_brows<T, 32, Op><<<g, kBlock, 0, s>>>(tab.blk, g, rp, ci, av, op, c.part); break;
    default: k_brows<T, 64, Op><<<g, kBlock, 0, s>>>(tab.blk, g, rp, ci, av, op, c.part); break;
  }
  if constexpr (Op::NV > 0) k_bfinal<Op><<<1, kFinThreads, 0, s>>>(op, c.part, g, tab.blk_sys, c.nsys);
}

template <typename T, class Op>
void brows(const Level& lv, int lpr, const BCtx& c, const T* av, const Op& op, hipStream_t s) {
  brows_on<T>(lv, lpr, lv.rp, lv.ci, av, c, op, s);
}

// Sliced ELL of a batch level: slices of 64 rows aligned to each system's
// first row (the last slice of a system may be short), column-major inside a
// slice.  Blocks of the row table start at system offsets in multiples of
// 256 rows, so each block covers whole slices; wave q of a block takes the
// block's slices q, q + 4, ...
template <typename T, class Op>
__global__ void __launch_bounds__(kBlock) k_bsell(const int* __restrict__ blk, int nb, const int* __restrict__ sys_off,
                                                  const int* __restrict__ sl_base, const int* __restrict__ sl_ptr,
                                                  const int* __restrict__ sl_col, const T* __restrict__ sl_val, Op op,
                                                  double* part) {
  if (!op.m.active()) return;
  constexpr int NV = Op::NV > 0 ? Op::NV : 1;
  const int lb = logical_block();
  const int sys = blk[3 * lb], r0 = blk[3 * lb + 1], r1 = blk[3 * lb + 2];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (sys >= 0 && op.m.on(sys)) {
    const int so = sys_off[sys], sb = sl_base[sys];
    for (int r = r0 + wv * kWave; r < r1; r += kBlock) {
      const int sl = sb + (r - so) / kWave;
      const int row = r + lane;
      const int base = sl_ptr[sl];
      const int w = (sl_ptr[sl + 1] - base) / kWave;
      const int* cp = sl_col + base + lane;
      const T* vp = sl_val + base + lane;
      T sum = T(0);
      for (int k0 = 0; k0 < w; k0 += 8) {
        int cc[8];
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool in = k0 + q < w;
          cc[q] = in ? cp[(k0 + q) * kWave] : 0;
          v[q] = in ? vp[(k0 + q) * kWave] : T(0);
        }
        T xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) xv[q] = k0 + q < w ? op.x(cc[q]) : T(0);
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (k0 + q < w) sum += v[q] * xv[q];
      }
      if (row < r1) op.row(row, sys, sum, acc);
    }
  }
  if constexpr (Op::NV > 0) write_part<Op::NV>(acc, part, nb, lb);
}

template <typename T> const T* bsv(const Level& l);
template <> const double* bsv<double>(const Level& l) { return l.sl_val; }
template <> const float* bsv<float>(const Level& l) { return l.sl_val32; }
template <typename T> const T* bav(const Level& l);
template <> const double* bav<double>(const Level& l) { return l.val; }
template <> const float* bav<float>(const Level& l) { return l.val32; }

// A_k applied by a row operation, in the level's format
template <typename T, class Op>
void blevel(const Level& lv, const BCtx& c, const Op& op, hipStream_t s) {
  if (!lv.bsell) {
    brows_on<T>(lv, lv.lpr, lv.rp, lv.ci, bav<T>(lv), c, op, s);
    return;
  }
  if (lv.nblk == 0) return;
  const int g = lv.nblk;
  k_bsell<T, Op><<<g, kBlock, 0, s>>>(lv.blk, g, lv.d_sys_off, lv.sl_base, lv.sl_ptr, lv.sl_col, bsv<T>(lv), op,
                                      c.part);
  if constexpr (Op::NV > 0) k_bfinal<Op><<<1, kFinThreads, 0, s>>>(op, c.part, g, lv.blk_sys, c.nsys);
}

template <class Op>
void belem(const Level& lv, const BCtx& c, const Op& op, hipStream_t s) {
  if (lv.nblk == 0) return;
  const int g = lv.nblk;
  k_belem<Op><<<g, kBlock, 0, s>>>(lv.blk, g, op, c.part);
  if constexpr (Op::NV > 0) k_bfinal<Op><<<1, kFinThreads, 0, s>>>(op, c.part, g, lv.blk_sys, c.nsys);
}

#define B_NOFIN                                                   \
  __device__ void finalize(int, const double*) const {}          \
  __device__ void skip(int) const {}                             \
  __device__ void finalize_all() const {}

// ---------------------------------------------------------------- setup ops
struct BLocalBase {
  static constexpr int NV = 0;
  Mask m;
  const int* sys_off;
  int* lbase;
  __device__ void elem(int i, int s, double*) const { lbase[i] = sys_off[s]; }
  B_NOFIN
};

// every entry of a system's rows must stay inside the system
struct BCheckBlocks {
  static constexpr int NV = 0;
  Mask m;
  const int* sys_off;
  const int* rp;
  const int* ci;
  int* err;
  __device__ void elem(int i, int s, double*) const {
    const int lo = sys_off[s], hi = sys_off[s + 1];
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int c = ci[k];
      if (c < lo || c >= hi) atomic_or_flag(err, kErrCrossSystem);
    }
  }
  B_NOFIN
};

// coarse ids: roots of coarsened systems renumbered without the roots of the
// systems that stop here (their rows get -1)
struct BRemapAgg {
  static constexpr int NV = 0;
  Mask m;
  const int* cont;
  const int* shift;
  int* agg;
  __device__ void elem(int i, int s, double*) const { agg[i] = cont[s] ? agg[i] - shift[s] : -1; }
  B_NOFIN
};

struct BJacobi {
  static constexpr int NV = 0;
  Mask m;
  const double* omega;
  const double* diag;
  double* wdinv;
  float* wdinv32;
  __device__ void elem(int i, int s, double*) const {
    const double om = omega[s];
    const double w = om != 0.0 ? om / diag[i] : 0.0;
    wdinv[i] = w;
    if (wdinv32) wdinv32[i] = (float)w;
  }
  B_NOFIN
};

// Arnoldi on D^-1 A per system (Section 2.2.1): start vector from the hash of
// the local row index, normalised per system
struct BArnStart {
  static constexpr int NV = 1;
  Mask m;
  const int* sys_off;
  double* q;
  double* sc;
  int nsys;
  uint32_t stream;
  __device__ void elem(int i, int s, double* acc) const {
    const double u = unit_uniform((uint32_t)(i - sys_off[s]), stream);
    q[i] = u;
    acc[0] += u * u;
  }
  __device__ void finalize(int s, const double* v) const { sc[bArnNorm * nsys + s] = sqrt(v[0]); }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

struct BDivide {
  static constexpr int NV = 0;
  Mask m;
  const double* in;
  double* out;
  const double* den;   // per system
  __device__ void elem(int i, int s, double*) const { out[i] = in[i] / den[s]; }
  B_NOFIN
};

struct BArnSpmv {
  static constexpr int NV = 2;
  Mask m;
  const double* q;
  const double* q0;
  const double* diag;
  double* w;
  double* sc;
  int nsys, j;
  __device__ double x(int c) const { return q[c]; }
  __device__ void row(int i, int, double ax, double* acc) const {
    const double t = (1.0 / diag[i]) * ax;
    w[i] = t;
    acc[0] += t * t;
    acc[1] += q0[i] * t;
  }
  __device__ void finalize(int s, const double* v) const {
    sc[(bArn + 48 + j) * nsys + s] = sqrt(v[0]);
    sc[(bArn + j) * nsys + s] = v[1];
  }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

// modified Gram-Schmidt: w -= H[i][j] q_i, then q_{i+1}'w (or ||w|| last)
struct BArnAxpyDot {
  static constexpr int NV = 1;
  Mask m;
  const double* qi;
  const double* qn;
  double* w;
  const double* h;     // per system
  double* out;         // per system
  __device__ void elem(int i, int s, double* acc) const {
    const double t = w[i] - h[s] * qi[i];
    w[i] = t;
    acc[0] += (qn ? qn[i] : t) * t;
  }
  __device__ void finalize(int s, const double* v) const { out[s] = qn ? v[0] : sqrt(v[0]); }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

// ---------------------------------------------------------------- cycle ops
template <typename T>
struct BPresmoothResid {
  static constexpr int NV = 0;
  Mask m;
  const T* b;
  const T* wd;
  T* xt;
  T* r;
  __device__ T x(int j) const { return wd[j] * b[j]; }
  __device__ void row(int i, int, T ax, double*) const {
    const T bi = b[i];
    xt[i] = wd[i] * bi;
    r[i] = bi - ax;
  }
  B_NOFIN
};

template <typename T>
struct BResidSmooth {
  static constexpr int NV = 0;
  Mask m;
  const T* b;
  const T* xt;
  const T* wd;
  T* xo;
  __device__ T x(int j) const { return xt[j]; }
  __device__ void row(int i, int, T ax, double*) const { xo[i] = xt[i] + wd[i] * (b[i] - ax); }
  B_NOFIN
};

template <typename T, bool DOT>
struct BRestrict {   // rows of R = P^T (aggregates, the rows of the next level)
  static constexpr int NV = DOT ? 1 : 0;
  Mask m;
  const T* r;
  T* rcv;
  double* K;   // K slots of this level: slot q of system s at K[q * nsys + s]
  int nsys;
  __device__ T x(int j) const { return r[j]; }
  __device__ void row(int I, int, T s, double* acc) const {
    rcv[I] = s;
    if (DOT) acc[0] += (double)s * (double)s;
  }
  __device__ void finalize(int s, const double* v) const {
    if (DOT) K[kKRcRc * nsys + s] = v[0];
  }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

template <typename T>
struct BProlong {
  static constexpr int NV = 0;
  Mask m;
  const int* agg;
  const T* pval;
  const T* cc;
  T* xt;
  __device__ void elem(int i, int, double*) const {
    const int a = agg[i];
    if (a >= 0) xt[i] += pval[i] * cc[a];
  }
  B_NOFIN
};

template <typename T>
struct BKDots1 {
  static constexpr int NV = 2;
  Mask m;
  const T* cc;
  const T* rcv;
  T* v;
  double* K;
  int nsys;
  __device__ T x(int j) const { return cc[j]; }
  __device__ void row(int i, int, T ax, double* acc) const {
    v[i] = ax;
    acc[0] += (double)cc[i] * (double)ax;
    acc[1] += (double)cc[i] * (double)rcv[i];
  }
  __device__ void finalize(int s, const double* v2) const {
    K[kKRho1 * nsys + s] = v2[0];
    K[kKAlpha1 * nsys + s] = v2[1];
  }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

// r~ = r_c - (alpha1/rho1) v and the per-system branch of Algorithm 5; a
// system whose next level is its coarsest takes the V-cycle step (coefficient
// 1, no second step), as it would alone
template <typename T>
struct BRtilde {
  static constexpr int NV = 1;
  Mask m;
  const T* rcv;
  const T* v;
  T* rt;
  double* K;
  int* F;        // F[s]: second step; F[nsys + s]: use d
  int* any2;
  const int* kv;
  double t;
  int nsys;
  __device__ void elem(int i, int s, double* acc) const {
    const T ar = (T)(K[kKAlpha1 * nsys + s] / K[kKRho1 * nsys + s]);
    const T u = rcv[i] - ar * v[i];
    rt[i] = u;
    acc[0] += (double)u * (double)u;
  }
  __device__ void finalize(int s, const double* v2) const {
    F[nsys + s] = 0;
    if (!kv[s]) {
      K[kKCoefC * nsys + s] = 1.0;
      F[s] = 0;
      return;
    }
    const double rho1 = K[kKRho1 * nsys + s];
    K[kKRtRt * nsys + s] = v2[0];
    if (rho1 > 0.0) {
      K[kKCoefC * nsys + s] = K[kKAlpha1 * nsys + s] / rho1;
      F[s] = (sqrt(v2[0]) <= t * sqrt(K[kKRcRc * nsys + s])) ? 0 : 1;
    } else {
      K[kKCoefC * nsys + s] = 0.0;
      F[s] = 0;
    }
  }
  __device__ void skip(int s) const {
    F[s] = 0;
    F[nsys + s] = 0;
  }
  __device__ void finalize_all() const {
    int a = 0;
    for (int s = 0; s < nsys; ++s) a |= F[s];
    *any2 = a;
  }
};

template <typename T>
struct BKDots2 {
  static constexpr int NV = 3;
  Mask m;
  const T* d;
  const T* v;
  const T* rt;
  T* w;
  double* K;
  int* F;
  int nsys;
  __device__ T x(int j) const { return d[j]; }
  __device__ void row(int i, int, T ax, double* acc) const {
    w[i] = ax;
    acc[0] += (double)d[i] * (double)v[i];
    acc[1] += (double)d[i] * (double)ax;
    acc[2] += (double)d[i] * (double)rt[i];
  }
  __device__ void finalize(int s, const double* v2) const {
    const double gamma = v2[0], beta = v2[1], alpha2 = v2[2];
    const double rho1 = K[kKRho1 * nsys + s], alpha1 = K[kKAlpha1 * nsys + s];
    const double rho2 = beta - gamma * gamma / rho1;
    if (rho2 > 0.0) {
      K[kKCoefC * nsys + s] = alpha1 / rho1 - gamma * alpha2 / (rho1 * rho2);
      K[kKCoefD * nsys + s] = alpha2 / rho2;
      F[nsys + s] = 1;
    }
  }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

template <typename T>
struct BProlongK {
  static constexpr int NV = 0;
  Mask m;
  const int* agg;
  const T* pval;
  const T* cc;
  const T* d;
  T* xt;
  const double* K;
  const int* F;
  int nsys;
  __device__ void elem(int i, int s, double*) const {
    const int a = agg[i];
    if (a < 0) return;
    T xc = (T)K[kKCoefC * nsys + s] * cc[a];
    if (F[nsys + s]) xc += (T)K[kKCoefD * nsys + s] * d[a];
    xt[i] += pval[i] * xc;
  }
  B_NOFIN
};

// coarsest level of each terminal system: x = A_s^-1 b on its rows, one wave
// per row, the inverse row read contiguously
template <typename T>
__global__ void __launch_bounds__(kBlock) k_term_gemv(const int* __restrict__ tblk, const TermInfo* __restrict__ ti,
                                                      const T* __restrict__ inv, const T* __restrict__ b,
                                                      T* __restrict__ x, Mask m) {
  if (!m.active()) return;
  const int t = tblk[2 * blockIdx.x];
  const TermInfo e = ti[t];
  if (!m.on(e.sys)) return;
  const int r = tblk[2 * blockIdx.x + 1] + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (r >= e.n) return;
  const T* Ar = inv + e.off + (size_t)r * e.n;
  const T* bs = b + e.row0;
  T s = T(0);
  for (int j = lane; j < e.n; j += kWave) s += Ar[j] * bs[j];
  s = wave_sum(s);
  if (lane == 0) x[e.row0 + r] = s;
}

// ---------------------------------------------------------------- outer ops
struct BFcgInit {
  static constexpr int NV = 1;
  Mask m;
  const double* b;
  double* r;
  double* xv;
  double* sc;
  int* fl;
  int* any;
  int* err;
  double rtol;
  int nsys;
  __device__ void elem(int i, int, double* acc) const {
    const double t = b[i];
    r[i] = t;
    xv[i] = 0.0;
    acc[0] += t * t;
  }
  __device__ void finalize(int s, const double* v) const {
    sc[bBB * nsys + s] = v[0];
    sc[bRtol2 * nsys + s] = rtol * rtol * v[0];
    fl[fIters * nsys + s] = 0;
    fl[fRun * nsys + s] = v[0] > 0.0 ? 1 : 0;
    if (!__builtin_isfinite(v[0])) {
      atomic_or_flag(err, kErrNonFinite);
      fl[fRun * nsys + s] = 0;
    }
  }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {
    int a = 0;
    for (int s = 0; s < nsys; ++s) a |= fl[fRun * nsys + s];
    any[aRun] = a;
  }
};

struct BFcgSpmv {
  static constexpr int NV = 2;
  Mask m;
  const double* p;
  const double* r;
  double* q;
  double* sc;
  int* fl;
  int* err;
  int nsys;
  __device__ double x(int j) const { return p[j]; }
  __device__ void row(int i, int, double ax, double* acc) const {
    q[i] = ax;
    acc[0] += p[i] * ax;
    acc[1] += p[i] * r[i];
  }
  __device__ void finalize(int s, const double* v) const {
    sc[bPQ * nsys + s] = v[0];
    sc[bAlpha * nsys + s] = v[1] / v[0];
    fl[fIters * nsys + s] += 1;
    if (!(v[0] > 0.0)) {
      atomic_or_flag(err, __builtin_isfinite(v[0]) ? kErrBreakdown : kErrNonFinite);
      fl[fRun * nsys + s] = 0;
    }
  }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

struct BFcgUpdate {
  static constexpr int NV = 1;
  Mask m;
  const double* p;
  const double* q;
  double* xv;
  double* r;
  float* r32;    // float copy of r for the mixed cycle (nullable)
  double* sc;
  int* fl;
  int* any;
  int* err;
  int nsys;
  __device__ void elem(int i, int s, double* acc) const {
    const double al = sc[bAlpha * nsys + s];
    xv[i] += al * p[i];
    const double t = r[i] - al * q[i];
    r[i] = t;
    if (r32) r32[i] = (float)t;
    acc[0] += t * t;
  }
  __device__ void finalize(int s, const double* v) const {
    sc[bRR * nsys + s] = v[0];
    if (!__builtin_isfinite(v[0])) {
      atomic_or_flag(err, kErrNonFinite);
      fl[fRun * nsys + s] = 0;
    } else if (v[0] <= sc[bRtol2 * nsys + s]) {
      fl[fRun * nsys + s] = 0;
    }
  }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {
    int a = 0;
    for (int s = 0; s < nsys; ++s) a |= fl[fRun * nsys + s];
    any[aRun] = a;
  }
};

struct BToFloat {
  static constexpr int NV = 0;
  Mask m;
  const double* in;
  float* out;
  __device__ void elem(int i, int, double*) const { out[i] = (float)in[i]; }
  B_NOFIN
};

template <typename T>
struct BDotZQ {
  static constexpr int NV = 1;
  Mask m;
  const T* z;
  const double* q;
  double* sc;
  int nsys;
  __device__ void elem(int i, int, double* acc) const { acc[0] += (double)z[i] * q[i]; }
  __device__ void finalize(int s, const double* v) const { sc[bBeta * nsys + s] = -v[0] / sc[bPQ * nsys + s]; }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

template <typename T>
struct BPUpdate {
  static constexpr int NV = 0;
  Mask m;
  const T* z;
  double* p;
  const double* sc;
  int nsys, first;
  __device__ void elem(int i, int s, double*) const {
    p[i] = first ? (double)z[i] : (double)z[i] + sc[bBeta * nsys + s] * p[i];
  }
  B_NOFIN
};

struct BTrueResid {
  static constexpr int NV = 1;
  Mask m;
  const double* b;
  const double* xv;
  double* r;
  double* sc;
  int nsys;
  __device__ double x(int j) const { return xv[j]; }
  __device__ void row(int i, int, double ax, double* acc) const {
    const double t = b[i] - ax;
    r[i] = t;
    acc[0] += t * t;
  }
  __device__ void finalize(int s, const double* v) const { sc[bTrue * nsys + s] = v[0]; }
  __device__ void skip(int) const {}
  __device__ void finalize_all() const {}
};

struct BCopy {
  static constexpr int NV = 0;
  Mask m;
  const double* in;
  double* out;
  __device__ void elem(int i, int, double*) const { out[i] = in[i]; }
  B_NOFIN
};

#undef B_NOFIN

__global__ void k_gather(int m, const int* __restrict__ src, const int* __restrict__ idx, int* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = src[idx[i]];
}

// ------------------------------------------------------------ typed views
template <typename T> const T* bvals(const Level& l);
template <> const double* bvals<double>(const Level& l) { return l.val; }
template <> const float* bvals<float>(const Level& l) { return l.val32; }
template <typename T> const T* bwd(const Level& l);
template <> const double* bwd<double>(const Level& l) { return l.wdinv; }
template <> const float* bwd<float>(const Level& l) { return l.wdinv32; }
template <typename T> const T* bpv(const Level& l);
template <> const double* bpv<double>(const Level& l) { return l.pval; }
template <> const float* bpv<float>(const Level& l) { return l.pval32; }
template <typename T> const T* brv(const Level& l);
template <> const double* brv<double>(const Level& l) { return l.rval; }
template <> const float* brv<float>(const Level& l) { return l.rval32; }
template <typename T> const T* btinv(const Level& l);
template <> const double* btinv<double>(const Level& l) { return l.tinv; }
template <> const float* btinv<float>(const Level& l) { return l.tinv32; }

BCtx bctx(const Hierarchy& h) { return BCtx{h.nsys, h.b_part}; }

// ------------------------------------------------------------------ cycle
template <typename T>
void term_solve(Hierarchy& h, const Level& lv, const T* b, T* x, Mask m) {
  if (lv.ntblk == 0) return;
  k_term_gemv<T><<<lv.ntblk, kBlock, 0, h.stream>>>(lv.tblk, lv.d_term, btinv<T>(lv), b, x, m);
}

template <typename T>
void cycle_b(Hierarchy& h, int k, const T* b, T* xo, Mask m) {
  hipStream_t s = h.stream;
  const BCtx c = bctx(h);
  const int L = h.L();
  Level& lv = h.levels[k];
  if (k == L) {   // every system present here ends here
    term_solve<T>(h, lv, b, xo, m);
    return;
  }
  const int nsys = h.nsys;
  T* xt = static_cast<T*>(lv.xt);
  T* r = static_cast<T*>(lv.r);
  T* rcv = static_cast<T*>(lv.rc);
  T* cc = static_cast<T*>(lv.c);
  const T* wd = bwd<T>(lv);
  const T* pv = bpv<T>(lv);
  Level& lc = h.levels[k + 1];
  blevel<T>(lv, c, BPresmoothResid<T>{m, b, wd, xt, r}, s);
  const T* rv = brv<T>(lv);
  if (!lv.kcyc) {
    brows_on<T>(lc, lv.rlpr, lv.agg_ptr, lv.agg_rows, rv, c, BRestrict<T, false>{m, r, rcv, nullptr, nsys}, s);
    cycle_b<T>(h, k + 1, rcv, cc, m);
    belem(lv, c, BProlong<T>{m, lv.agg, pv, cc, xt}, s);
  } else {
    double* K = h.b_sc + (size_t)(bK0 + 16 * k) * nsys;
    int* F = h.b_fl + (size_t)(fK0 + 2 * k) * nsys;
    int* any2 = h.b_any + aK0 + k;
    T* v = static_cast<T*>(lv.v);
    T* rt = static_cast<T*>(lv.rt);
    T* d = static_cast<T*>(lv.d);
    T* w = static_cast<T*>(lv.w);
    brows_on<T>(lc, lv.rlpr, lv.agg_ptr, lv.agg_rows, rv, c, BRestrict<T, true>{m, r, rcv, K, nsys}, s);
    cycle_b<T>(h, k + 1, rcv, cc, m);
    blevel<T>(lc, c, BKDots1<T>{m, cc, rcv, v, K, nsys}, s);
    belem(lc, c, BRtilde<T>{m, rcv, v, rt, K, F, any2, lv.kv, h.opt.kcycle_t, nsys}, s);
    const Mask m2{any2, F};
    cycle_b<T>(h, k + 1, rt, d, m2);
    blevel<T>(lc, c, BKDots2<T>{m2, d, v, rt, w, K, F, nsys}, s);
    belem(lv, c, BProlongK<T>{m, lv.agg, pv, cc, d, xt, K, F, nsys}, s);
  }
  blevel<T>(lv, c, BResidSmooth<T>{m, b, xt, wd, xo}, s);
  term_solve<T>(h, lv, b, xo, m);   // systems whose coarsest level is this one
}

template <typename T>
void precondition_b(Hierarchy& h, Mask m, bool r32_ready) {
  const Level& l0 = h.levels[0];
  if constexpr (sizeof(T) == sizeof(float)) {
    if (!r32_ready) belem(l0, bctx(h), BToFloat{m, h.r, static_cast<float*>(h.bz)}, h.stream);
    cycle_b<float>(h, 0, static_cast<const float*>(h.bz), static_cast<float*>(h.z), m);
  } else {
    (void)r32_ready;
    cycle_b<double>(h, 0, h.r, static_cast<double*>(h.z), m);
  }
}

template <typename T>
void iteration_b(Hierarchy& h) {
  const Level& l0 = h.levels[0];
  const BCtx c = bctx(h);
  const int nsys = h.nsys;
  const Mask m{h.b_any + aRun, h.b_fl + fRun * nsys};
  hipStream_t s = h.stream;
  float* r32 = sizeof(T) == sizeof(float) ? static_cast<float*>(h.bz) : nullptr;
  blevel<double>(l0, c, BFcgSpmv{m, h.p, h.r, h.q, h.b_sc, h.b_fl, h.d_err, nsys}, s);
  belem(l0, c, BFcgUpdate{m, h.p, h.q, h.xint, h.r, r32, h.b_sc, h.b_fl, h.b_any, h.d_err, nsys}, s);
  precondition_b<T>(h, m, r32 != nullptr);
  belem(l0, c, BDotZQ<T>{m, static_cast<const T*>(h.z), h.q, h.b_sc, nsys}, s);
  belem(l0, c, BPUpdate<T>{m, static_cast<const T*>(h.z), h.p, h.b_sc, nsys, 0}, s);
}

template <typename T>
void restart_b(Hierarchy& h) {
  const int nsys = h.nsys;
  const Mask m{h.b_any + aRun, h.b_fl + fRun * nsys};
  precondition_b<T>(h, m, false);
  belem(h.levels[0], bctx(h), BPUpdate<T>{m, static_cast<const T*>(h.z), h.p, h.b_sc, nsys, 1}, h.stream);
}

}  // namespace

// ---------------------------------------------------------------- setup API
int batch_max_blocks(int nsys);
// Block table of a level from its host system offsets: blocks of at most rb
// rows inside one system, rb a multiple of 256 chosen so that about 8192
// blocks cover the level (enough waves in flight to hide the row kernels'
// dependent loads).
void batch_blocks(Hierarchy& h, Level& lv) {
  const int nsys = h.nsys;
  const long n = lv.n;
  int rb = (int)(((n + kBatchBlocks - 1) / kBatchBlocks + 255) / 256 * 256);
  if (rb < 256) rb = 256;
  std::vector<int> tab;
  std::vector<int> bs(nsys + 1);
  int nb = 0;
  for (int s = 0; s < nsys; ++s) {
    bs[s] = nb;
    for (int r = lv.sys_off[s]; r < lv.sys_off[s + 1]; r += rb) {
      tab.push_back(s);
      tab.push_back(r);
      tab.push_back(std::min(r + rb, lv.sys_off[s + 1]));
      ++nb;
    }
  }
  bs[nsys] = nb;
  if (nb + 7 > batch_max_blocks(nsys)) throw Error(AMG_EHIP, "block table larger than its bound");
  while (nb > 8 && (nb & 7)) {
    tab.push_back(-1);
    tab.push_back(0);
    tab.push_back(0);
    ++nb;
  }
  lv.nblk = nb;
  lv.blk = h.arena.alloc_n<int>(std::max<size_t>(tab.size(), 3));
  lv.blk_sys = h.arena.alloc_n<int>(nsys + 1);
  lv.d_sys_off = h.arena.alloc_n<int>(nsys + 1);
  if (!tab.empty())
    AMG_HIP(hipMemcpyAsync(lv.blk, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, h.stream));
  AMG_HIP(hipMemcpyAsync(lv.blk_sys, bs.data(), bs.size() * sizeof(int), hipMemcpyHostToDevice, h.stream));
  AMG_HIP(hipMemcpyAsync(lv.d_sys_off, lv.sys_off.data(), (nsys + 1) * sizeof(int), hipMemcpyHostToDevice,
                         h.stream));
  // pageable sources: the copies above finish before the host vectors go away
  AMG_HIP(hipStreamSynchronize(h.stream));
}

void batch_local_base(const Level& lv, int* lbase, hipStream_t s) {
  BCtx c{0, nullptr};
  belem(lv, c, BLocalBase{Mask{nullptr, nullptr}, lv.d_sys_off, lbase}, s);
}

namespace {
__global__ void k_bsell_widths(int nsl, const int* __restrict__ srow, const int* __restrict__ rp,
                               int* __restrict__ widths) {
  const int sl = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  int len = 0;
  if (sl < nsl) {
    const int row = srow[2 * sl] + lane;
    if (row < srow[2 * sl + 1]) len = rp[row + 1] - rp[row];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const int o = __shfl_xor(len, off, kWave);
    len = o > len ? o : len;
  }
  if (sl < nsl && lane == 0) widths[sl] = len * kWave;
}

// entry k of slice row l at sl_ptr[sl] + 64 k + l; padding has value 0 and a
// column inside the slice's system (the row itself, or the slice's first row)
__global__ void k_bsell_fill(int nsl, const int* __restrict__ srow, const int* __restrict__ rp,
                             const int* __restrict__ ci, const double* __restrict__ val,
                             const int* __restrict__ sl_ptr, int* __restrict__ sl_col, double* __restrict__ sl_val,
                             float* __restrict__ sl_val32) {
  const int sl = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (sl >= nsl) return;
  const int row = srow[2 * sl] + lane;
  const bool valid = row < srow[2 * sl + 1];
  const int s0 = valid ? rp[row] : 0;
  const int len = valid ? rp[row + 1] - s0 : 0;
  const int base = sl_ptr[sl];
  const int w = (sl_ptr[sl + 1] - base) / kWave;
  for (int k = 0; k < w; ++k) {
    const int idx = base + k * kWave + lane;
    int c = valid ? row : srow[2 * sl];
    double v = 0.0;
    if (k < len) {
      c = ci[s0 + k];
      v = val[s0 + k];
    }
    sl_col[idx] = c;
    sl_val[idx] = v;
    if (sl_val32) sl_val32[idx] = (float)v;
  }
}
}  // namespace

// Sliced-ELL copy of a batch level (used when its rows are short: at most 12
// entries on average).
void batch_build_sell(Hierarchy& h, Arena& tmp, Level& lv) {
  const int nsys = h.nsys;
  lv.bsell = lv.nnz <= 12L * lv.n ? 1 : 0;
  if (!lv.bsell) return;
  std::vector<int> srow, base(nsys + 1);
  int nsl = 0;
  for (int q = 0; q < nsys; ++q) {
    base[q] = nsl;
    for (int r = lv.sys_off[q]; r < lv.sys_off[q + 1]; r += kWave) {
      srow.push_back(r);
      srow.push_back(std::min(r + kWave, lv.sys_off[q + 1]));
      ++nsl;
    }
  }
  base[nsys] = nsl;
  hipStream_t s = h.stream;
  int* d_srow = tmp.alloc_n<int>(std::max<size_t>(srow.size(), 2));
  int* widths = tmp.alloc_n<int>(std::max(nsl, 1));
  lv.sl_base = h.arena.alloc_n<int>(nsys + 1);
  lv.sl_ptr = h.arena.alloc_n<int>(nsl + 1);
  lv.nslices = nsl;
  AMG_HIP(hipMemcpyAsync(d_srow, srow.data(), srow.size() * sizeof(int), hipMemcpyHostToDevice, s));
  AMG_HIP(hipMemcpyAsync(lv.sl_base, base.data(), base.size() * sizeof(int), hipMemcpyHostToDevice, s));
  const int g = (nsl + kBlock / kWave - 1) / (kBlock / kWave);
  k_bsell_widths<<<g, kBlock, 0, s>>>(nsl, d_srow, lv.rp, widths);
  scan_to_ptr(widths, lv.sl_ptr, nsl, h.scan, s);
  int total = 0;
  AMG_HIP(hipMemcpyAsync(&total, lv.sl_ptr + nsl, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  lv.sl_col = h.arena.alloc_n<int>(std::max(total, 1));
  lv.sl_val = h.arena.alloc_n<double>(std::max(total, 1));
  if (h.mixed()) lv.sl_val32 = h.arena.alloc_n<float>(std::max(total, 1));
  k_bsell_fill<<<g, kBlock, 0, s>>>(nsl, d_srow, lv.rp, lv.ci, lv.val, lv.sl_ptr, lv.sl_col, lv.sl_val, lv.sl_val32);
  AMG_HIP(hipStreamSynchronize(s));   // the host slice table is read before it goes away
}

void batch_check_blocks(const Level& lv, int* err, hipStream_t s) {
  BCtx c{0, nullptr};
  belem(lv, c, BCheckBlocks{Mask{nullptr, nullptr}, lv.d_sys_off, lv.rp, lv.ci, err}, s);
}

void batch_gather(int m, const int* src, const int* idx, int* dst, hipStream_t s) {
  if (m > 0) k_gather<<<(m + 255) / 256, 256, 0, s>>>(m, src, idx, dst);
}

void batch_remap_agg(const Level& lv, const int* cont, const int* shift, int* agg, hipStream_t s) {
  BCtx c{0, nullptr};
  belem(lv, c, BRemapAgg{Mask{nullptr, nullptr}, cont, shift, agg}, s);
}

void batch_jacobi_weights(const Level& lv, const double* omega_sys, double* wdinv, float* wdinv32,
                          hipStream_t s) {
  BCtx c{0, nullptr};
  belem(lv, c, BJacobi{Mask{nullptr, nullptr}, omega_sys, lv.diag, wdinv, wdinv32}, s);
}

// Per-system Arnoldi (m steps, modified Gram-Schmidt) on the systems enabled
// by mask; H_out receives, per system, H[i][j] at [s*64 + 8i + j] and the
// norms ||D^-1 A q_j|| at [s*64 + 48 + j].
void batch_arnoldi(Hierarchy& h, Level& lv, int m, uint32_t stream, const int* mask, double* Q, double* w,
                   double* H_out) {
  hipStream_t s = h.stream;
  const int n = lv.n, nsys = h.nsys;
  const BCtx c = bctx(h);
  const Mask mk{nullptr, mask};
  double* sc = h.b_sc;
  belem(lv, c, BArnStart{mk, lv.d_sys_off, Q, sc, nsys, stream}, s);
  belem(lv, c, BDivide{mk, Q, Q, sc + (size_t)bArnNorm * nsys}, s);
  for (int j = 0; j < m; ++j) {
    const double* qj = Q + (size_t)j * n;
    blevel<double>(lv, c, BArnSpmv{mk, qj, Q, lv.diag, w, sc, nsys, j}, s);
    for (int i = 0; i <= j; ++i) {
      const double* qi = Q + (size_t)i * n;
      const double* qn = i < j ? Q + (size_t)(i + 1) * n : nullptr;
      belem(lv, c,
            BArnAxpyDot{mk, qi, qn, w, sc + (size_t)(bArn + i * 8 + j) * nsys,
                        sc + (size_t)(bArn + (i + 1) * 8 + j) * nsys},
            s);
    }
    belem(lv, c, BDivide{mk, w, Q + (size_t)(j + 1) * n, sc + (size_t)(bArn + (j + 1) * 8 + j) * nsys}, s);
  }
  std::vector<double> hs((size_t)64 * nsys);
  AMG_HIP(hipMemcpyAsync(hs.data(), sc + (size_t)bArn * nsys, hs.size() * sizeof(double), hipMemcpyDeviceToHost,
                         s));
  AMG_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < 64; ++q)
    for (int t = 0; t < nsys; ++t) H_out[(size_t)t * 64 + q] = hs[(size_t)q * nsys + t];
}

// Per-system control block and block partials (setup and solve).  A level
// of n rows has at most n / rb + nsys <= 2048 + nsys blocks before padding.
int batch_max_blocks(int nsys) { return kBatchBlocks + nsys + 8; }

void batch_control(Hierarchy& h) {
  const int nsys = h.nsys;
  const int maxblk = batch_max_blocks(nsys);
  h.b_sc = h.arena.alloc_n<double>((size_t)bSlots * nsys);
  h.b_fl = h.arena.alloc_n<int>((size_t)fWords * nsys);
  h.b_any = h.arena.alloc_n<int>(aWords);
  h.b_part = h.arena.alloc_n<double>((size_t)kBNV * maxblk);
  h.b_again = h.arena.alloc_n<int>(nsys);
  launch_fill_int((size_t)fWords * nsys, h.b_fl, 0, h.stream);
  launch_fill_int(aWords, h.b_any, 0, h.stream);
  launch_fill_double((size_t)bSlots * nsys, h.b_sc, 0.0, h.stream);
}

// One outer iteration and the (re)start sequence captured as HIP graphs on a
// capture stream (the kernels read every branch decision from device flags,
// so one recording serves every replay).
void build_batch_graphs(Hierarchy& h) {
  hipStream_t user = h.stream;
  hipStream_t cs = nullptr;
  AMG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const bool mixed = h.mixed();
  auto finish = [&](hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    AMG_HIP(hipStreamEndCapture(cs, &g));
    AMG_HIP(hipGraphInstantiate(out, g, nullptr, nullptr, 0));
    AMG_HIP(hipGraphDestroy(g));
  };
  try {
    h.stream = cs;
    AMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    if (mixed) iteration_b<float>(h);
    else iteration_b<double>(h);
    hipGraphExec_t it = nullptr;
    finish(&it);
    h.g_iter.push_back(it);
    AMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    if (mixed) restart_b<float>(h);
    else restart_b<double>(h);
    finish(&h.g_restart);
  } catch (...) {
    h.stream = user;
    (void)hipStreamDestroy(cs);
    throw;
  }
  h.stream = user;
  AMG_HIP(hipStreamDestroy(cs));
}

namespace {
void launch_iteration_b(Hierarchy& h) {
  if (!h.g_iter.empty()) AMG_HIP(hipGraphLaunch(h.g_iter[0], h.stream));
  else if (h.mixed()) iteration_b<float>(h);
  else iteration_b<double>(h);
}
void launch_restart_b(Hierarchy& h) {
  if (h.g_restart) AMG_HIP(hipGraphLaunch(h.g_restart, h.stream));
  else if (h.mixed()) restart_b<float>(h);
  else restart_b<double>(h);
}
}  // namespace

// ---------------------------------------------------------------- solve
// Outer flexible CG per system from x_0 = 0; iters / relres: host [nsys].
int solve_batch_impl(Hierarchy& h, const double* b, double rtol, double* x, int* iters, double* relres) {
  hipStream_t s = h.stream;
  struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
  const int nsys = h.nsys;
  const Level& l0 = h.levels[0];
  const BCtx c = bctx(h);
  const bool mixed = h.mixed();
  const Mask all{nullptr, nullptr};
  std::vector<int> hfl((size_t)2 * nsys);
  std::vector<double> hsc((size_t)bArn * nsys);
  std::vector<int> again(nsys);
  belem(l0, c, BFcgInit{all, b, h.r, h.xint, h.b_sc, h.b_fl, h.b_any, h.d_err, rtol, nsys}, s);
  launch_restart_b(h);
  const int max_iter = h.opt.max_iter;
  int enqueued = 0;
  int status = AMG_OK;
  int* hp = static_cast<int*>(h.h_pinned);
  while (true) {
    const int batch = std::min(4, max_iter - enqueued);
    for (int i = 0; i < batch; ++i) launch_iteration_b(h);
    enqueued += batch;
    AMG_HIP(hipGetLastError());
    AMG_HIP(hipMemcpyAsync(hp, h.b_any + aRun, sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hp + 1, h.d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    if (hp[1]) {
      if (hp[1] & kErrNonFinite) throw Error(AMG_ENANINF, "non-finite value in the iteration");
      if (hp[1] & kErrBreakdown) throw Error(AMG_EBREAKDOWN, "Krylov breakdown");
      throw Error(AMG_EHIP, "device error bits " + std::to_string(hp[1]));
    }
    if (hp[0] && enqueued < max_iter) continue;
    blevel<double>(l0, c, BTrueResid{all, b, h.xint, h.q, h.b_sc, nsys}, s);
    AMG_HIP(hipMemcpyAsync(hfl.data(), h.b_fl, hfl.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hsc.data(), h.b_sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    bool any_again = false;
    for (int q = 0; q < nsys; ++q) {
      const double bb = hsc[bBB * nsys + q];
      const double rel = bb > 0.0 ? std::sqrt(hsc[bTrue * nsys + q] / bb) : 0.0;
      if (!std::isfinite(rel)) throw Error(AMG_ENANINF, "non-finite residual");
      iters[q] = hfl[fIters * nsys + q];
      relres[q] = rel;
      again[q] = (rel > rtol && bb > 0.0 && iters[q] < max_iter && enqueued < max_iter) ? 1 : 0;
      any_again |= again[q] != 0;
      if (rel > rtol && bb > 0.0 && !again[q]) status = AMG_ENOTCONV;
    }
    if (!any_again) break;
    // restart the systems whose recurrence converged but whose true residual
    // did not: r = b - A x, running again
    AMG_HIP(hipMemcpyAsync(h.b_again, again.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(h.b_fl + fRun * nsys, h.b_again, nsys * sizeof(int), hipMemcpyDeviceToDevice, s));
    launch_fill_int(1, h.b_any + aRun, 1, s);
    belem(l0, c, BCopy{Mask{nullptr, h.b_again}, h.q, h.r}, s);
    AMG_HIP(hipStreamSynchronize(s));   // the pageable `again` is read before it changes
    launch_restart_b(h);
  }
  AMG_HIP(hipMemcpyAsync(x, h.xint, (size_t)l0.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipStreamSynchronize(s));
  return status;
}

}  // namespace amg
