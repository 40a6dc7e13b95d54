// Solve phase: damped Jacobi (eq. damped_jacobi), the V-cycle (Algorithm 4)
// and K-cycle (Algorithm 5) preconditioners, flexible CG outside, and the
// Arnoldi estimate of rho(D^-1 A) used by setup (Section 2.2.1).
//
// All scalars of the K-cycle and of the outer iteration live in device
// memory; the branch "skip the second inner step when ||r~|| <= t ||r||" and
// the convergence test are device flags read by every kernel of the guarded
// region, so a whole outer iteration is enqueued without host round-trips.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "kernels_common.hpp"

namespace amg {

namespace {

struct Act {
  const int* p;
  __device__ __forceinline__ bool on() const { return p == nullptr || *p != 0; }
};

// ------------------------------------------------------------------ row ops
template <typename T>
struct OpSpmv {
  static constexpr int NV = 0;
  Act a;
  const T* xv;
  T* y;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return xv[j]; }
  __device__ void row(int i, T ax, double*) const { y[i] = ax; }
  __device__ void finalize(const double*) const {}
};

// pre-smoothing from a zero guess and the residual: x = w.*b, r = b - A x
template <typename T>
struct OpPresmoothResid {
  static constexpr int NV = 0;
  Act a;
  const T* b;
  const T* wd;
  T* xt;
  T* r;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return wd[j] * b[j]; }
  __device__ void row(int i, T ax, double*) const {
    const T bi = b[i];
    xt[i] = wd[i] * bi;
    r[i] = bi - ax;
  }
  __device__ void finalize(const double*) const {}
};

// On small levels (at most kFuseCorrectionRows rows, where a launch costs more
// than the work) the coarse-grid correction is applied where the
// post-smoothing reads the iterate, x_j + P_j (correction of aggregate agg_j),
// so it needs no pass of its own; larger levels run the prolongation as its
// own pass, which is cheaper than three extra gathers per nonzero.  V-cycle: the correction is c; K-cycle: coef_c c (+ coef_d d when
// the second inner step was kept).
constexpr int kFuseCorrectionRows = 65536;

template <typename T>
struct CorrV {
  const int* agg;
  const T* pval;
  const T* c;
  __device__ T at(const T* xt, int j) const { return xt[j] + pval[j] * c[agg[j]]; }
};

template <typename T>
struct CorrNone {   // correction already applied by a prolongation pass
  __device__ T at(const T* xt, int j) const { return xt[j]; }
};

template <typename T>
struct CorrK {
  const int* agg;
  const T* pval;
  const T* c;
  const T* d;
  const double* K;
  const int* F;
  __device__ T at(const T* xt, int j) const {
    const int I = agg[j];
    T xc = (T)K[kKCoefC] * c[I];
    if (F[1]) xc += (T)K[kKCoefD] * d[I];
    return xt[j] + pval[j] * xc;
  }
};

// new residual and post-smoothing on the corrected iterate x = xt + P e:
// r = b - A x, x_out = x + w.*r
template <typename T, class Corr>
struct OpResidSmooth {
  static constexpr int NV = 0;
  Act a;
  const T* b;
  const T* xt;
  const T* wd;
  T* xo;
  Corr corr;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return corr.at(xt, j); }
  __device__ void row(int i, T ax, double*) const { xo[i] = corr.at(xt, i) + wd[i] * (b[i] - ax); }
  __device__ void finalize(const double*) const {}
};

// the same at level 0 of the outer iteration, with z'q for the FCG beta
template <typename T, class Corr>
struct OpResidSmoothDot {
  static constexpr int NV = 1;
  Act a;
  const T* b;
  const T* xt;
  const T* wd;
  T* xo;
  Corr corr;
  const double* q;
  double* sc;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return corr.at(xt, j); }
  __device__ void row(int i, T ax, double* acc) const {
    const T z = corr.at(xt, i) + wd[i] * (b[i] - ax);
    xo[i] = z;
    acc[0] += (double)z * q[i];
  }
  __device__ void finalize(const double* s) const { sc[kScBeta] = -s[0] / sc[kScPQ]; }
};

// ---- Chebyshev smoothing (the polynomial smoother of Section 5): the
// three-term Chebyshev recurrence on M = D^-1 A over [a, b].  First step from
// an iterate x0: r = D^-1 (b - A x0), d = r / theta, x = x0 + d; each later
// step j: r -= D^-1 A d, d = c1_j d + c2_j r, x += d.  Device coefficients
// K[0] = 1 / theta, K[2j - 1] = c1_j, K[2j] = c2_j (j >= 1 counts the later
// steps); dv = 1 / a_ii.

// pre-smoothing from x0 = 0, first and second step in one pass: the gathered
// d_j = (dv_j b_j) / theta, and at row i the second step's update
template <typename T>
struct OpChebPre2 {
  static constexpr int NV = 0;
  Act a;
  const T* b;
  const T* dv;
  const double* K;
  T* r;
  T* dout;
  T* xo;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return (T)K[0] * (dv[j] * b[j]); }
  __device__ void row(int i, T ad, double*) const {
    const T r0 = dv[i] * b[i];
    const T d0 = (T)K[0] * r0;
    const T rr = r0 - dv[i] * ad;
    const T dn = (T)K[1] * d0 + (T)K[2] * rr;
    r[i] = rr;
    dout[i] = dn;
    xo[i] = d0 + dn;
  }
  __device__ void finalize(const double*) const {}
};

// pre-smoothing of degree one from x0 = 0 with the residual: x = d, r = b - A x
template <typename T>
struct OpChebPre1Resid {
  static constexpr int NV = 0;
  Act a;
  const T* b;
  const T* dv;
  const double* K;
  T* xt;
  T* r;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return (T)K[0] * (dv[j] * b[j]); }
  __device__ void row(int i, T ax, double*) const {
    xt[i] = (T)K[0] * (dv[i] * b[i]);
    r[i] = b[i] - ax;
  }
  __device__ void finalize(const double*) const {}
};

// a later step j (din gathered, dout written: two buffers)
template <typename T>
struct OpChebStep {
  static constexpr int NV = 0;
  Act a;
  const T* dv;
  const T* din;
  T* dout;
  T* r;
  T* xo;
  const double* K;
  int j;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int c) const { return din[c]; }
  __device__ void row(int i, T ad, double*) const {
    const T rr = r[i] - dv[i] * ad;
    const T dn = (T)K[2 * j - 1] * din[i] + (T)K[2 * j] * rr;
    r[i] = rr;
    dout[i] = dn;
    xo[i] += dn;
  }
  __device__ void finalize(const double*) const {}
};

// first post-smoothing step on the corrected iterate x0 = xt + P e
template <typename T, class Corr>
struct OpChebPost1 {
  static constexpr int NV = 0;
  Act a;
  const T* b;
  const T* xt;
  const T* dv;
  const double* K;
  T* r;
  T* dout;
  T* xo;
  Corr corr;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return corr.at(xt, j); }
  __device__ void row(int i, T ax, double*) const {
    const T rr = dv[i] * (b[i] - ax);
    const T d = (T)K[0] * rr;
    r[i] = rr;
    dout[i] = d;
    xo[i] = corr.at(xt, i) + d;
  }
  __device__ void finalize(const double*) const {}
};

// residual of a given iterate: r = b - A x
template <typename T>
struct OpResid {
  static constexpr int NV = 0;
  Act a;
  const T* b;
  const T* xv;
  T* r;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return xv[j]; }
  __device__ void row(int i, T ax, double*) const { r[i] = b[i] - ax; }
  __device__ void finalize(const double*) const {}
};

// ---- multi-colour symmetric Gauss-Seidel (Section 2.2.1): the rows of one
// colour share no entry of A, so x_i += (b_i - (A x)_i) / a_ii for all of them
// at once, in place (no row of the colour reads another's x_i).  LPR lanes
// per listed row.
template <typename T, int LPR>
__global__ void __launch_bounds__(256) k_sgs_color(int m, const int* __restrict__ rows, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const T* __restrict__ av,
                                                   const T* __restrict__ b, const T* __restrict__ dv, T* x, Act a) {
  if (!a.on()) return;
  constexpr int RPB = 256 / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  for (int q0 = blockIdx.x * RPB; q0 < m; q0 += gridDim.x * RPB) {
    const int q = q0 + threadIdx.x / LPR;
    T sum = T(0);
    int i = -1;
    if (q < m) {
      i = rows[q];
      for (int k = rp[i] + lane; k < rp[i + 1]; k += LPR) sum += av[k] * x[ci[k]];
    }
    sum = group_sum<LPR>(sum);
    if (q < m && lane == 0) x[i] += (b[i] - sum) * dv[i];
  }
}

// x = value (guarded)
template <typename T>
struct OpFillAct {
  static constexpr int NV = 0;
  Act a;
  T* p;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { p[i] = T(0); }
  __device__ void finalize(const double*) const {}
};

// xo = the corrected iterate xt + P e
template <typename T, class Corr>
struct OpApplyCorr {
  static constexpr int NV = 0;
  Act a;
  const T* xt;
  T* xo;
  Corr corr;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { xo[i] = corr.at(xt, i); }
  __device__ void finalize(const double*) const {}
};

// first inner step: v = A c, rho1 and alpha1 (CG: c'v, c'r; GMRES: v'v, v'r),
// and the test of the second step in the same reduction: with a = alpha1 /
// rho1, ||r~||^2 = ||r_c - a v||^2 = r_c'r_c - 2 a v'r_c + a^2 v'v, so the
// flag is decided here and r~ itself is formed only when the step runs
template <typename T>
struct OpKDots1 {
  static constexpr int NV = 5;
  Act a;
  const T* c;
  const T* rcv;
  T* v;
  double* K;
  int* F;
  int gmres;
  double t;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const { F[0] = 0; }
  __device__ T x(int j) const { return c[j]; }
  __device__ void row(int i, T ax, double* acc) const {
    v[i] = ax;
    const double av = (double)ax, rr = (double)rcv[i];
    const double l = gmres ? av : (double)c[i];
    acc[0] += l * av;
    acc[1] += l * rr;
    acc[2] += rr * rr;
    acc[3] += av * av;
    acc[4] += av * rr;
  }
  __device__ void finalize(const double* s) const {
    const double rho1 = s[0], alpha1 = s[1];
    K[kKRho1] = rho1;
    K[kKAlpha1] = alpha1;
    K[kKRcRc] = s[2];
    F[1] = 0;
    if (rho1 > 0.0) {
      const double ar = alpha1 / rho1;
      double rt2 = s[2] - 2.0 * ar * s[4] + ar * ar * s[3];
      rt2 = rt2 > 0.0 ? rt2 : 0.0;
      K[kKRtRt] = rt2;
      K[kKCoefC] = ar;
      F[0] = (sqrt(rt2) <= t * sqrt(s[2])) ? 0 : 1;
    } else {
      K[kKRtRt] = s[2];
      K[kKCoefC] = 0.0;
      F[0] = 0;
    }
  }
};

// second inner step: w = A d; gamma, beta, alpha2; then the combination
// coefficients of x_{k+1} = coef_c c + coef_d d
template <typename T>
struct OpKDots2 {
  static constexpr int NV = 3;
  Act a;
  const T* d;
  const T* v;
  const T* rt;
  T* w;
  double* K;
  int* F;
  int gmres;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return d[j]; }
  __device__ void row(int i, T ax, double* acc) const {
    w[i] = ax;
    const double l = gmres ? (double)ax : (double)d[i];
    acc[0] += l * (double)v[i];
    acc[1] += l * (double)ax;
    acc[2] += l * (double)rt[i];
  }
  __device__ void finalize(const double* s) const {
    const double gamma = s[0], beta = s[1], alpha2 = s[2];
    const double rho1 = K[kKRho1], alpha1 = K[kKAlpha1];
    K[kKGamma] = gamma;
    K[kKBeta] = beta;
    K[kKAlpha2] = alpha2;
    const double rho2 = beta - gamma * gamma / rho1;
    if (rho2 > 0.0) {
      K[kKCoefC] = alpha1 / rho1 - gamma * alpha2 / (rho1 * rho2);
      K[kKCoefD] = alpha2 / rho2;
      F[1] = 1;
    }
  }
};

// outer FCG: q = A p with p'q and p'r; alpha = p'r / p'q
struct OpFcgSpmv {
  static constexpr int NV = 2;
  Act a;
  const double* p;
  const double* r;
  double* q;
  double* sc;
  int* ctl;
  int* err;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ double x(int j) const { return p[j]; }
  __device__ void row(int i, double ax, double* acc) const {
    q[i] = ax;
    acc[0] += p[i] * ax;
    acc[1] += p[i] * r[i];
  }
  __device__ void finalize(const double* s) const {
    sc[kScPQ] = s[0];
    sc[kScAlpha] = s[1] / s[0];
    ctl[kCtlIters] += 1;
    if (!(s[0] > 0.0)) {
      *err |= __builtin_isfinite(s[0]) ? kErrBreakdown : kErrNonFinite;
      ctl[kCtlRunning] = 0;
    }
  }
};

// b - A x and its squared norm (true residual)
struct OpTrueResid {
  static constexpr int NV = 1;
  Act a;
  const double* b;
  const double* xv;
  double* r;
  double* sc;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ double x(int j) const { return xv[j]; }
  __device__ void row(int i, double ax, double* acc) const {
    const double t = b[i] - ax;
    r[i] = t;
    acc[0] += t * t;
  }
  __device__ void finalize(const double* s) const { sc[kScTrue] = s[0]; }
};

// Arnoldi step j (classical Gram-Schmidt): w = D^-1 A q_j with ||w||^2 and
// the projections q_k'w, k <= j, in the same pass (the basis q_k at Q + k n)
struct OpArnSpmv {
  static constexpr int NV = 1 + kArnMax;
  const double* q;
  const double* Q;
  const double* diag;
  double* w;
  double* sc;
  int j;
  int n;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ double x(int c) const { return q[c]; }
  __device__ void row(int i, double ax, double* acc) const {
    const double t = (1.0 / diag[i]) * ax;
    w[i] = t;
    acc[0] += t * t;
#pragma unroll
    for (int k = 0; k < kArnMax; ++k)
      if (k <= j) acc[1 + k] += Q[(size_t)k * n + i] * t;
  }
  __device__ void finalize(const double* s) const {
    sc[kScArn + 48 + j] = sqrt(s[0]);
    for (int k = 0; k <= j; ++k) sc[kScArn + k * 8 + j] = s[1 + k];
  }
};

// ------------------------------------------------------------ element ops
struct OpFcgInit {
  static constexpr int NV = 1;
  const double* b;
  double* r;
  double* xv;
  double* sc;
  int* ctl;
  int* err;
  double rtol;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double* acc) const {
    const double t = b[i];
    r[i] = t;
    xv[i] = 0.0;
    acc[0] += t * t;
  }
  __device__ void finalize(const double* s) const {
    sc[kScBB] = s[0];
    sc[kScRtol2] = rtol * rtol * s[0];
    ctl[kCtlIters] = 0;
    ctl[kCtlRunning] = s[0] > 0.0 ? 1 : 0;
    if (!__builtin_isfinite(s[0])) {
      *err |= kErrNonFinite;
      ctl[kCtlRunning] = 0;
    }
  }
};

struct OpFcgUpdate {
  static constexpr int NV = 1;
  Act a;
  const double* p;
  const double* q;
  double* xv;
  double* r;
  double* sc;
  int* ctl;
  int* err;
  float* r32;   // mixed precision: the cycle's FP32 right-hand side
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double* acc) const {
    const double al = sc[kScAlpha];
    // x is touched again only by the next update: stream it past the caches
    __builtin_nontemporal_store(__builtin_nontemporal_load(xv + i) + al * p[i], xv + i);
    const double t = r[i] - al * q[i];
    r[i] = t;
    if (r32) r32[i] = (float)t;
    acc[0] += t * t;
  }
  __device__ void finalize(const double* s) const {
    sc[kScRR] = s[0];
    if (!__builtin_isfinite(s[0])) {
      *err |= kErrNonFinite;
      ctl[kCtlRunning] = 0;
    } else if (s[0] <= sc[kScRtol2]) {
      ctl[kCtlRunning] = 0;
    }
  }
};

template <typename T>
struct OpDotZQ {
  static constexpr int NV = 1;
  Act a;
  const T* z;
  const double* q;
  double* sc;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double* acc) const { acc[0] += (double)z[i] * q[i]; }
  __device__ void finalize(const double* s) const { sc[kScBeta] = -s[0] / sc[kScPQ]; }
};

template <typename T>
struct OpPUpdate {
  static constexpr int NV = 0;
  Act a;
  const T* z;
  double* p;
  const double* sc;
  int first;  // p = z
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const {
    p[i] = first ? (double)z[i] : (double)z[i] + sc[kScBeta] * p[i];
  }
  __device__ void finalize(const double*) const {}
};

struct OpToFloat {
  static constexpr int NV = 0;
  Act a;
  const double* in;
  float* out;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { out[i] = (float)in[i]; }
  __device__ void finalize(const double*) const {}
};

struct OpCopy {
  static constexpr int NV = 0;
  const double* in;
  double* out;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { out[i] = in[i]; }
  __device__ void finalize(const double*) const {}
};

// restriction r_c = P^T r by aggregate segments (ascending fine index); the
// K-cycle takes ||r_c||^2 with the first inner step's dots (OpKDots1).
// xtc non-null: also the coarse level's first smoothing step from zero,
// xtc = wdc .* r_c, so its pre-smoothing gathers one array instead of two.
template <typename T>
struct OpRestrict {   // rows of R = P^T (aggregates)
  static constexpr int NV = 0;
  Act a;
  const T* r;
  T* rcv;
  const T* wdc = nullptr;
  T* xtc = nullptr;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ T x(int j) const { return r[j]; }
  __device__ void row(int I, T s, double*) const {
    rcv[I] = s;
    if (xtc) xtc[I] = wdc[I] * s;
  }
  __device__ void finalize(const double*) const {}
};

// prolongation x += P c
template <typename T>
struct OpProlong {
  static constexpr int NV = 0;
  Act a;
  const int* agg;
  const T* pval;
  const T* c;
  T* xt;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { xt[i] += pval[i] * c[agg[i]]; }
  __device__ void finalize(const double*) const {}
};

// prolongation of the K-cycle combination x += P (coef_c c + coef_d d)
template <typename T>
struct OpProlongK {
  static constexpr int NV = 0;
  Act a;
  const int* agg;
  const T* pval;
  const T* c;
  const T* d;
  T* xt;
  const double* K;
  const int* F;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const {
    const int I = agg[i];
    const T cc = (T)K[kKCoefC];
    T xc = cc * c[I];
    if (F[1]) xc += (T)K[kKCoefD] * d[I];
    xt[i] += pval[i] * xc;
  }
  __device__ void finalize(const double*) const {}
};

// r~ = r_c - (alpha1/rho1) v, the right-hand side of the second inner step
// (only when that step runs); xt non-null: also xt = wd .* r~, as OpRestrict
template <typename T>
struct OpRtilde {
  static constexpr int NV = 0;
  Act a;
  const T* rcv;
  const T* v;
  T* rt;
  const double* K;
  const T* wd = nullptr;
  T* xt = nullptr;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const {
    const T ar = (T)(K[kKAlpha1] / K[kKRho1]);
    const T v2 = rcv[i] - ar * v[i];
    rt[i] = v2;
    if (xt) xt[i] = wd[i] * v2;
  }
  __device__ void finalize(const double*) const {}
};

struct OpHashVector {
  static constexpr int NV = 0;
  double* q;
  uint32_t stream;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { q[i] = unit_uniform((uint32_t)i, stream); }
  __device__ void finalize(const double*) const {}
};

struct OpArnStart {
  static constexpr int NV = 1;
  double* q;
  double* sc;
  uint32_t stream;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double* acc) const {
    const double u = unit_uniform((uint32_t)i, stream);
    q[i] = u;
    acc[0] += u * u;
  }
  __device__ void finalize(const double* s) const { sc[kScArn + 56] = sqrt(s[0]); }
};

struct OpDivide {
  static constexpr int NV = 0;
  const double* in;
  double* out;
  const double* den;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { out[i] = in[i] / *den; }
  __device__ void finalize(const double*) const {}
};

// the projections off w in one pass, w -= sum_k h_kj q_k (k = 0..j in
// order), and h_{j+1,j} = ||w||
struct OpArnUpdate {
  static constexpr int NV = 1;
  const double* Q;
  double* w;
  const double* sc;
  double* out;
  int j;
  int n;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double* acc) const {
    double t = w[i];
#pragma unroll
    for (int k = 0; k < kArnMax; ++k)
      if (k <= j) t -= sc[kScArn + k * 8 + j] * Q[(size_t)k * n + i];
    w[i] = t;
    acc[0] += t * t;
  }
  __device__ void finalize(const double* s) const { *out = sqrt(s[0]); }
};

struct OpSetCtl {
  static constexpr int NV = 0;
  int* ctl;
  int word, value;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const {
    if (i == 0) ctl[word] = value;
  }
  __device__ void finalize(const double*) const {}
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gemv(int n, const T* __restrict__ A, const T* __restrict__ xv,
                                                 T* __restrict__ y, Act a) {
  if (!a.on()) return;
  const int row = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  T s = T(0);
  const T* Ar = A + (size_t)row * n;
  for (int j = lane; j < n; j += kWave) s += Ar[j] * xv[j];
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// ------------------------------------------------------------ typed views
// Small V-cycle levels: pre-smoothing, residual and restriction in one pass
// by aggregate, one block per aggregate: LPR lanes per member row (the row
// kernels' lane split), 256/LPR members at a time, the restricted value summed
// over the members in segment order through LDS, so the fine residual is
// never stored.  x = w.*b on the members, r_c(I) = sum_i R(I,i) (b_i - (A x)_i).
template <typename T, int LPR>
__global__ void __launch_bounds__(256) k_presmooth_restrict(int nc, const int* __restrict__ agg_ptr,
                                                            const int* __restrict__ agg_rows,
                                                            const T* __restrict__ rv, const int* __restrict__ rp,
                                                            const int* __restrict__ ci, const T* __restrict__ av,
                                                            const T* __restrict__ b, const T* __restrict__ wd,
                                                            T* __restrict__ xt, T* __restrict__ rcv, Act a) {
  if (!a.on()) return;
  constexpr int MPB = 256 / LPR;   // members per pass
  __shared__ T part[MPB];
  const int slot = threadIdx.x / LPR, lane = threadIdx.x & (LPR - 1);
  for (int I = xcd_block_index(); I < nc; I += gridDim.x) {
    const int s = agg_ptr[I], e = agg_ptr[I + 1];
    T acc = T(0);
    for (int base = s; base < e; base += MPB) {
      const int k = base + slot;
      T sum = T(0);
      int i = -1;
      if (k < e) {
        i = agg_rows[k];
        const int r0 = rp[i], r1 = rp[i + 1];
        for (int x = r0 + lane; x < r1; x += LPR) {
          const int j = ci[x];
          sum += av[x] * (wd[j] * b[j]);
        }
      }
      sum = group_sum<LPR>(sum);
      if (lane == 0 && k < e) {
        const T bi = b[i];
        xt[i] = wd[i] * bi;
        part[slot] = rv[k] * (bi - sum);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const int m = min(MPB, e - base);
        for (int q = 0; q < m; ++q) acc += part[q];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) rcv[I] = acc;
  }
}

template <typename T> const T* vals(const Level& l);
template <> const double* vals<double>(const Level& l) { return l.val; }
template <> const float* vals<float>(const Level& l) { return l.val32; }
template <typename T> const T* wdinv(const Level& l);
template <> const double* wdinv<double>(const Level& l) { return l.wdinv; }
template <> const float* wdinv<float>(const Level& l) { return l.wdinv32; }
template <typename T> const T* rvals(const Level& l);
template <> const double* rvals<double>(const Level& l) { return l.rval; }
template <> const float* rvals<float>(const Level& l) { return l.rval32; }
template <typename T> const T* pvals(const Level& l);
template <> const double* pvals<double>(const Level& l) { return l.pval; }
template <> const float* pvals<float>(const Level& l) { return l.pval32; }
template <typename T> const T* cinv(const Hierarchy& h);
template <> const double* cinv<double>(const Hierarchy& h) { return h.cinv; }
template <> const float* cinv<float>(const Hierarchy& h) { return h.cinv32; }

inline RedCtx red(Hierarchy& h) { return RedCtx{h.d_part, h.d_ticket}; }

template <typename T> const Level::Tune& tune_of(const Level& l);
template <> const Level::Tune& tune_of<double>(const Level& l) { return l.t64; }
template <> const Level::Tune& tune_of<float>(const Level& l) { return l.t32; }
template <typename T> const T* sell_vals(const Level& l);
template <> const double* sell_vals<double>(const Level& l) { return l.sl_val; }
template <> const float* sell_vals<float>(const Level& l) { return l.sl_val32; }
template <typename T> const T* short_vals(const Level& l);
template <> const double* short_vals<double>(const Level& l) { return l.sh.val; }
template <> const float* short_vals<float>(const Level& l) { return l.sh.val32; }
template <typename T> const T* dia_vals(const Level& l);
template <> const double* dia_vals<double>(const Level& l) { return l.dia.val; }
template <> const float* dia_vals<float>(const Level& l) { return l.dia.val32; }

// A row operation on A_k with the level's tuned kernel (CSR, sliced ELL in
// 64-row slices or in the level's shorter slices, or sliced diagonals).
template <typename T, class Op>
void launch_level(const Level& lv, const Op& op, RedCtx rc, hipStream_t s) {
  const Level::Tune& t = tune_of<T>(lv);
  if (t.fmt == 4 && lv.ci16)
    launch_rows16<T>(lv.n, t.lpr, lv.rp, lv.ci16, vals<T>(lv), op, rc, s);
  else if (t.fmt == 3 && dia_vals<T>(lv))
    launch_sdia<T>(lv.n, lv.dia.nslices, lv.dia.ptr, lv.dia.off, dia_vals<T>(lv), op, rc, s, t.pz);
  else if (t.fmt >= 1 && t.sh > 0 && t.sh == lv.sh.h && short_vals<T>(lv))
    launch_sell<T>(lv.n, lv.sh.nslices, lv.sh.ptr, lv.sh.col, short_vals<T>(lv), op, rc, s,
                   t.fmt == 2 ? lv.sh.dcol : nullptr, 0, lv.sh.h, lv.sh.perm);
  else if (t.fmt >= 1 && lv.sl_ptr)
    launch_sell<T>(lv.n, lv.nslices, lv.sl_ptr, lv.sl_col, sell_vals<T>(lv), op, rc, s,
                   t.fmt == 2 ? lv.sl_dcol : nullptr, t.pz);
  else launch_rows<T>(lv.n, t.lpr, lv.rp, lv.ci, vals<T>(lv), op, rc, s);
}

// The probed kernel: while the outer iteration is being captured, close the
// current graph segment and keep the launch for the host to issue between
// segments; otherwise launch it (between HIP events when a probe is set).
void probe_point(Hierarchy& h, bool selected, std::function<void(hipStream_t)> fn) {
  if (selected && h.split_at_probe) {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    AMG_HIP(hipStreamEndCapture(h.cap_stream, &g));
    AMG_HIP(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
    AMG_HIP(hipGraphDestroy(g));
    h.g_iter.push_back(e);
    h.probe_fn = std::move(fn);
    AMG_HIP(hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeRelaxed));
    return;
  }
  const bool timed = selected && h.pev[0] && !h.capturing;
  if (timed) AMG_HIP(hipEventRecord(h.pev[0], h.stream));
  fn(h.stream);
  if (timed) AMG_HIP(hipEventRecord(h.pev[1], h.stream));
}

// ------------------------------------------------------------ V-cycle tail, one launch
// The V-cycle levels below the K-cycle that take the fused small-level path,
// with the coarse solve, run as one persistent launch instead of one kernel
// per step: the steps are phases (pre-smoothing + restriction per level down,
// the coarse product, residual + post-smoothing + prolongation per level up),
// each cut into work items.  Blocks take items in one global order from a
// ticket counter and an item waits until every item of the previous phase is
// done (a per-phase counter).  A block only ever waits for items with smaller
// tickets, which blocks already running hold, so the launch cannot deadlock
// whatever the number of blocks resident.  Each item computes what the
// per-step kernels compute, in the same order (same lanes per row, same
// sums), so the results are the same bit for bit.  Data written by other
// blocks of the launch are read with device-coherent loads after an acquire
// fence; items publish with a release fence before their counter increment.
// The last block to leave clears the counters for the next launch.
// Opt-in (AMG_FLAG_PERSISTENT_TAIL): on C3 one such launch (levels 2-4, 1,024
// or 256 blocks, 4 or 16 aggregates / row groups per item) took 340-480 us
// against 47 us for the five per-step kernels it replaces; the item
// counters' device-scope atomics and the release fence per item cost more
// than the launch gaps saved.
constexpr int kTailMax = 8;            // levels in one tail launch
constexpr int kTailAggPerItem = 16;    // aggregates per pre-smoothing item
constexpr int kTailGroupsPerItem = 16; // row groups per post-smoothing item
constexpr int kTailGrid = 256;
constexpr long kTailSpin = 1L << 22;   // bound of a wait (an error, not a hang, if ever reached)

template <typename T>
struct TailLevel {
  int n, nc, lpr;
  const int* rp;
  const int* ci;
  const T* av;
  const int* agg_ptr;
  const int* agg_rows;
  const T* rv;
  const int* agg;
  const T* pv;
  const T* wd;
  const T* b;   // right-hand side (written in this launch except on the first level)
  T* xt;        // pre-smoothed iterate
  T* rc;        // restricted residual = right-hand side of the next level
  T* c;         // correction = iterate of the next level
  T* xo;        // smoothed output
};

template <typename T>
struct TailArgs {
  int nlev, nphase, ncoarse;
  const T* cinv;
  unsigned* ctl;   // [0] ticket, [1] blocks that left, [2 + p] items done in phase p
  int* err;
  int start[2 * kTailMax + 2];   // first item of each phase; start[nphase] = all items
  TailLevel<T> lv[kTailMax];
};

// a value written by another block of this launch: a vector load (the
// addresses differ across lanes) after the acquire fence of the wait
template <typename T>
__device__ __forceinline__ T tail_ld(const T* p) {
  return *p;
}
template <typename T>
__device__ __forceinline__ T tail_ldb(const T* p, bool first) {
  return first ? *p : tail_ld(p);
}

// aggregates [I0, I1) of a level: the arithmetic of k_presmooth_restrict
template <typename T, int LPR>
__device__ void tail_presmooth(const TailLevel<T>& L, bool first, int I0, int I1, T* part) {
  constexpr int MPB = 256 / LPR;
  const int slot = threadIdx.x / LPR, lane = threadIdx.x & (LPR - 1);
  for (int I = I0; I < I1; ++I) {
    const int s = L.agg_ptr[I], e = L.agg_ptr[I + 1];
    T acc = T(0);
    for (int base = s; base < e; base += MPB) {
      const int k = base + slot;
      T sum = T(0);
      int i = -1;
      if (k < e) {
        i = L.agg_rows[k];
        const int r0 = L.rp[i], r1 = L.rp[i + 1];
        for (int x = r0 + lane; x < r1; x += LPR) {
          const int j = L.ci[x];
          sum += L.av[x] * (L.wd[j] * tail_ldb(L.b + j, first));
        }
      }
      sum = group_sum<LPR>(sum);
      if (lane == 0 && k < e) {
        const T bi = tail_ldb(L.b + i, first);
        L.xt[i] = L.wd[i] * bi;
        part[slot] = L.rv[k] * (bi - sum);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const int m = min(MPB, e - base);
        for (int q = 0; q < m; ++q) acc += part[q];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) L.rc[I] = acc;
  }
}

// row groups [g0, g1) of a level: the arithmetic of k_rows with
// OpResidSmooth<T, CorrV<T>> (x_j = xt_j + P_j c_agg(j))
template <typename T, int LPR>
__device__ void tail_postsmooth(const TailLevel<T>& L, bool first, int g0, int g1) {
  constexpr int RPB = 256 / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  auto corr = [&](int j) { return tail_ld(L.xt + j) + L.pv[j] * tail_ld(L.c + L.agg[j]); };
  for (int g = g0; g < g1; ++g) {
    const int row = g * RPB + threadIdx.x / LPR;
    T sum = T(0);
    if (row < L.n) {
      const int s = L.rp[row], e = L.rp[row + 1];
      for (int k0 = s + lane; k0 < e; k0 += 4 * LPR) {
        int c[4];
        T v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = k0 + q * LPR;
          c[q] = k < e ? L.ci[k] : 0;
          v[q] = k < e ? L.av[k] : T(0);
        }
        T xv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) xv[q] = k0 + q * LPR < e ? corr(c[q]) : T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k0 + q * LPR < e) sum += v[q] * xv[q];
      }
    }
    sum = group_sum<LPR>(sum);
    if (row < L.n && lane == 0) L.xo[row] = corr(row) + L.wd[row] * (tail_ldb(L.b + row, first) - sum);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_vtail(TailArgs<T> a, Act act) {
  if (!act.on()) return;
  __shared__ int s_item;
  __shared__ T part[32];
  const int total = a.start[a.nphase];
  int ready = 0;   // leading phases known to be complete
  while (true) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.ctl[0], 1u);
    __syncthreads();
    const int t = s_item;
    __syncthreads();
    if (t >= total) break;
    int p = 0;
    while (t >= a.start[p + 1]) ++p;
    if (p > ready) {   // phases complete in order: wait for phase p - 1
      __shared__ int s_ok;
      if (threadIdx.x == 0) {
        const unsigned need = (unsigned)(a.start[p] - a.start[p - 1]);
        long spins = 0;
        while (__hip_atomic_load(&a.ctl[2 + p - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need &&
               ++spins < kTailSpin)
          __builtin_amdgcn_s_sleep(8);
        s_ok = spins < kTailSpin;
        if (!s_ok) atomic_or_flag(a.err, kErrTimeout);
      }
      __syncthreads();
      if (!s_ok) break;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      ready = p;
    }
    const int it = t - a.start[p];
    if (p < a.nlev) {                       // pre-smoothing + restriction, down
      const TailLevel<T>& L = a.lv[p];
      const int I0 = it * kTailAggPerItem, I1 = min(L.nc, I0 + kTailAggPerItem);
      if (L.lpr == 8) tail_presmooth<T, 8>(L, p == 0, I0, I1, part);
      else if (L.lpr == 16) tail_presmooth<T, 16>(L, p == 0, I0, I1, part);
      else tail_presmooth<T, 32>(L, p == 0, I0, I1, part);
    } else if (p == a.nlev) {               // coarse product, one wave per row
      const TailLevel<T>& L = a.lv[a.nlev - 1];
      const int n = a.ncoarse;
      const int row = it * (kBlock / kWave) + threadIdx.x / kWave;
      const int lane = threadIdx.x & (kWave - 1);
      T s = T(0);
      if (row < n) {
        const T* Ar = a.cinv + (size_t)row * n;
        for (int j = lane; j < n; j += kWave) s += Ar[j] * tail_ld(L.rc + j);
      }
      s = wave_sum(s);
      if (row < n && lane == 0) L.c[row] = s;
    } else {                                // residual + post-smoothing + prolongation, up
      const int q = a.nlev - 1 - (p - a.nlev - 1);
      const TailLevel<T>& L = a.lv[q];
      const int rpb = 256 / L.lpr;
      const int groups = (L.n + rpb - 1) / rpb;
      const int g0 = it * kTailGroupsPerItem, g1 = min(groups, g0 + kTailGroupsPerItem);
      if (L.lpr == 8) tail_postsmooth<T, 8>(L, q == 0, g0, g1);
      else if (L.lpr == 16) tail_postsmooth<T, 16>(L, q == 0, g0, g1);
      else tail_postsmooth<T, 32>(L, q == 0, g0, g1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();   // the item's writes before its count
      atomicAdd(&a.ctl[2 + p], 1u);
    }
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(&a.ctl[1], 1u) == gridDim.x - 1) {   // every other block has left
      a.ctl[0] = 0u;
      a.ctl[1] = 0u;
      for (int q = 0; q < a.nphase; ++q) a.ctl[2 + q] = 0u;
    }
  }
}

// The first level of the tail (h.L() when there is none): from there down
// every level is a V-cycle level on the fused small-level path with 8, 16 or
// 32 lanes per row and the Jacobi (plain or learned) smoother.
template <typename T>
int tail_first(const Hierarchy& h) {
  const int L = h.L();
  if (L == 0 || h.nsys > 0 || !(h.opt.flags & AMG_FLAG_PERSISTENT_TAIL) || h.opt.smoother == AMG_SMOOTHER_CHEBYSHEV ||
      h.opt.smoother == AMG_SMOOTHER_MCSGS || !h.d_tail)
    return L;
  int k0 = L;
  while (k0 - 1 >= 1 && k0 - 1 >= h.opt.kcycle_levels) {
    const Level& lv = h.levels[k0 - 1];
    const int lpr = tune_of<T>(lv).lpr;
    if (lv.n > kFuseCorrectionRows || (lpr != 8 && lpr != 16 && lpr != 32)) break;
    --k0;
  }
  if (L - k0 > kTailMax) k0 = L - kTailMax;
  return k0;
}

// cycle(k0) below the K-cycle as one launch; false when level k0 does not
// start the tail
template <typename T>
bool vtail(Hierarchy& h, int k0, const T* b, T* xo, const int* act) {
  const int L = h.L();
  if (k0 >= L || tail_first<T>(h) != k0) return false;
  TailArgs<T> a{};
  a.nlev = L - k0;
  a.ncoarse = h.levels[L].n;
  a.cinv = cinv<T>(h);
  a.ctl = h.d_tail;
  a.err = h.d_err;
  int items = 0, p = 0;
  auto phase = [&](int n_items) { a.start[p++] = items; items += n_items; };
  for (int q = 0; q < a.nlev; ++q) {
    const Level& lv = h.levels[k0 + q];
    TailLevel<T>& t = a.lv[q];
    t.n = lv.n;
    t.nc = lv.nc;
    t.lpr = tune_of<T>(lv).lpr;
    t.rp = lv.rp;
    t.ci = lv.ci;
    t.av = vals<T>(lv);
    t.agg_ptr = lv.agg_ptr;
    t.agg_rows = lv.agg_rows;
    t.rv = rvals<T>(lv);
    t.agg = lv.agg;
    t.pv = pvals<T>(lv);
    t.wd = wdinv<T>(lv);
    t.b = q == 0 ? b : static_cast<const T*>(h.levels[k0 + q - 1].rc);
    t.xt = static_cast<T*>(lv.xt);
    t.rc = static_cast<T*>(lv.rc);
    t.c = static_cast<T*>(lv.c);
    t.xo = q == 0 ? xo : static_cast<T*>(h.levels[k0 + q - 1].c);
    phase((lv.nc + kTailAggPerItem - 1) / kTailAggPerItem);
  }
  phase((a.ncoarse + kBlock / kWave - 1) / (kBlock / kWave));
  for (int q = a.nlev - 1; q >= 0; --q) {
    const int rpb = 256 / a.lv[q].lpr;
    const int groups = (a.lv[q].n + rpb - 1) / rpb;
    phase((groups + kTailGroupsPerItem - 1) / kTailGroupsPerItem);
  }
  a.nphase = p;
  a.start[p] = items;
  const int grid = std::min(kTailGrid, items);
  k_vtail<T><<<grid, 256, 0, h.stream>>>(a, Act{act});
  return true;
}

template <typename T>
void coarse_solve(Hierarchy& h, const T* b, T* x, const int* act) {
  const int n = h.levels.back().n;
  const int rpb = kBlock / kWave;
  k_gemv<T><<<(n + rpb - 1) / rpb, kBlock, 0, h.stream>>>(n, cinv<T>(h), b, x, Act{act});
}

// Residual + post-smoothing of level k on the corrected iterate (and z'q at
// the top of the outer iteration when fuse_q is given).
// Chebyshev vectors of a level in the cycle precision: r, two d buffers
template <typename T>
struct ChebVecs {
  T* r;
  T* d0;
  T* d1;
};
template <typename T>
ChebVecs<T> cheb_vecs(const Level& lv) {
  return ChebVecs<T>{static_cast<T*>(lv.cr), static_cast<T*>(lv.cd0), static_cast<T*>(lv.cd1)};
}

// Pre-smoothing by Chebyshev from x = 0 (degree m = cheb_degree), then the
// residual r_out = b - A x.
template <typename T>
void cheb_pre(Hierarchy& h, const Level& lv, int k, Act A, const T* b, T* xt, T* r_out) {
  const Level* lp = &lv;
  RedCtx rc = red(h);
  const T* dv = wdinv<T>(lv);
  const int m = h.opt.cheb_degree;
  const bool sel = k == 0 && h.opt.probe == AMG_PROBE_L0_PRESMOOTH;
  if (m == 1) {
    const OpChebPre1Resid<T> op{A, b, dv, lv.cheb, xt, r_out};
    probe_point(h, sel, [=](hipStream_t st) { launch_level<T>(*lp, op, rc, st); });
    return;
  }
  ChebVecs<T> cv = cheb_vecs<T>(lv);
  {
    const OpChebPre2<T> op{A, b, dv, lv.cheb, cv.r, cv.d0, xt};
    probe_point(h, sel, [=](hipStream_t st) { launch_level<T>(*lp, op, rc, st); });
  }
  T* din = cv.d0;
  T* dout = cv.d1;
  for (int j = 2; j < m; ++j) {
    launch_level<T>(lv, OpChebStep<T>{A, dv, din, dout, cv.r, xt, lv.cheb, j}, rc, h.stream);
    std::swap(din, dout);
  }
  launch_level<T>(lv, OpResid<T>{A, b, xt, r_out}, rc, h.stream);
}

// Post-smoothing by Chebyshev on the corrected iterate, into xo.
template <typename T, class Corr>
void cheb_post(Hierarchy& h, const Level& lv, int k, Act A, const T* b, const T* xt, T* xo, Corr corr) {
  const Level* lp = &lv;
  RedCtx rc = red(h);
  const T* dv = wdinv<T>(lv);
  ChebVecs<T> cv = cheb_vecs<T>(lv);
  {
    const OpChebPost1<T, Corr> op{A, b, xt, dv, lv.cheb, cv.r, cv.d0, xo, corr};
    probe_point(h, k == 0 && h.opt.probe == AMG_PROBE_L0_POSTSMOOTH,
                [=](hipStream_t st) { launch_level<T>(*lp, op, rc, st); });
  }
  T* din = cv.d0;
  T* dout = cv.d1;
  for (int j = 1; j < h.opt.cheb_degree; ++j) {
    launch_level<T>(lv, OpChebStep<T>{A, dv, din, dout, cv.r, xo, lv.cheb, j}, rc, h.stream);
    std::swap(din, dout);
  }
}

// One symmetric Gauss-Seidel step on x in place: the colours forward, then
// backward.
template <typename T>
void sgs_sweeps(Hierarchy& h, const Level& lv, Act A, const T* b, T* x) {
  const int nc = (int)lv.coff.size() - 1;
  const int lpr = lv.lpr < 2 ? 2 : lv.lpr > 32 ? 32 : lv.lpr;
  for (int pass = 0; pass < 2 * nc; ++pass) {
    const int c = pass < nc ? pass : 2 * nc - 1 - pass;
    const int m = lv.coff[c + 1] - lv.coff[c];
    if (m <= 0) continue;
    const int* rows = lv.crow + lv.coff[c];
    long g = ((long)m * lpr + 255) / 256;
    if (g > 4096) g = 4096;
    with_lanes(lpr, [&](auto gl) {
      k_sgs_color<T, decltype(gl)::value><<<(int)g, 256, 0, h.stream>>>(m, rows, lv.rp, lv.ci, vals<T>(lv), b,
                                                                          wdinv<T>(lv), x, A);
    });
  }
}

template <typename T, class Corr>
void post_smooth(Hierarchy& h, const Level& lv, int k, Act A, const T* b, const T* xt, const T* wd, T* xo, Corr corr,
                 const double* fuse_q, RedCtx rc) {
  const Level* lp = &lv;
  const bool sel = k == 0 && h.opt.probe == AMG_PROBE_L0_POSTSMOOTH;
  if (h.opt.smoother == AMG_SMOOTHER_MCSGS) {
    launch_elem(lv.n, OpApplyCorr<T, Corr>{A, xt, xo, corr}, rc, h.stream);
    sgs_sweeps<T>(h, lv, A, b, xo);
    if (fuse_q) launch_elem(lv.n, OpDotZQ<T>{A, xo, fuse_q, h.d_sc}, rc, h.stream);
    return;
  }
  if (h.opt.smoother == AMG_SMOOTHER_CHEBYSHEV) {
    cheb_post<T>(h, lv, k, A, b, xt, xo, corr);
    if (fuse_q) launch_elem(lv.n, OpDotZQ<T>{A, xo, fuse_q, h.d_sc}, rc, h.stream);
    return;
  }
  if (fuse_q) {
    const OpResidSmoothDot<T, Corr> op{A, b, xt, wd, xo, corr, fuse_q, h.d_sc};
    probe_point(h, sel, [=](hipStream_t st) { launch_level<T>(*lp, op, rc, st); });
  } else {
    const OpResidSmooth<T, Corr> op{A, b, xt, wd, xo, corr};
    probe_point(h, sel, [=](hipStream_t st) { launch_level<T>(*lp, op, rc, st); });
  }
}

// Whether cycle(k) pre-smooths with the row kernel of its level from a zero
// guess (damped Jacobi, a level that is not the coarsest and does not take the
// fused pre-smoothing + restriction of small V-cycle levels): then whoever
// writes its right-hand side can also write the first step x = wd .* b.
bool plain_presmooth(const Hierarchy& h, int k) {
  const int L = h.L();
  if (k <= 0 || k >= L || h.opt.smoother == AMG_SMOOTHER_CHEBYSHEV || h.opt.smoother == AMG_SMOOTHER_MCSGS)
    return false;
  const bool kcyc = k < h.opt.kcycle_levels && k + 1 < L;
  return kcyc || h.levels[k].n > kFuseCorrectionRows;
}

// cycle(k): x_out = M_k b with a zero initial guess (Algorithm 5 on the top
// kcycle_levels levels, Algorithm 4 below); `act` guards every kernel.
// x0: the level's xt already holds wd .* b (written with b by the kernel
// that formed it), so the pre-smoothing takes the residual of that iterate.
template <typename T>
void cycle(Hierarchy& h, int k, const T* b, T* xo, const int* act, const double* fuse_q = nullptr,
           bool x0 = false) {
  if (h.L() == 0) {
    coarse_solve<T>(h, b, xo, act);
    return;
  }
  if (!fuse_q && vtail<T>(h, k, b, xo, act)) return;
  Level& lv = h.levels[k];
  hipStream_t s = h.stream;
  RedCtx rc = red(h);
  T* xt = static_cast<T*>(lv.xt);
  T* r = static_cast<T*>(lv.r);
  T* rcv = static_cast<T*>(lv.rc);
  T* c = static_cast<T*>(lv.c);
  const T* wd = wdinv<T>(lv);
  const T* pv = pvals<T>(lv);
  const int L = h.L();
  const Act A{act};

  const bool kcyc = k < h.opt.kcycle_levels && k + 1 < L;
  const bool cheb = h.opt.smoother == AMG_SMOOTHER_CHEBYSHEV;
  const bool sgs = h.opt.smoother == AMG_SMOOTHER_MCSGS;
  if (cheb || sgs) {
    if (cheb) {
      cheb_pre<T>(h, lv, k, A, b, xt, r);
    } else {   // from x = 0, then the residual
      launch_elem(lv.n, OpFillAct<T>{A, xt}, rc, s);
      sgs_sweeps<T>(h, lv, A, b, xt);
      launch_level<T>(lv, OpResid<T>{A, b, xt, r}, rc, s);
    }
  } else if (!kcyc && k > 0 && lv.n <= kFuseCorrectionRows) {
    const int lpr = tune_of<T>(lv).lpr;
    const int grid = lv.nc < 1 ? 1 : lv.nc < 65536 ? lv.nc : 65536;
    with_lanes(lpr, [&](auto g) {
      k_presmooth_restrict<T, decltype(g)::value><<<grid, 256, 0, s>>>(
          lv.nc, lv.agg_ptr, lv.agg_rows, rvals<T>(lv), lv.rp, lv.ci, vals<T>(lv), b, wd, xt, rcv, A);
    });
  } else {
    const Level* lp = &lv;
    if (x0) {
      launch_level<T>(lv, OpResid<T>{A, b, xt, r}, rc, s);
    } else {
      const OpPresmoothResid<T> op{A, b, wd, xt, r};
      probe_point(h, k == 0 && h.opt.probe == AMG_PROBE_L0_PRESMOOTH,
                  [=](hipStream_t st) { launch_level<T>(*lp, op, rc, st); });
    }
  }
  // the next level's first smoothing step goes out with its right-hand side
  const bool nx0 = k + 1 < L && plain_presmooth(h, k + 1);
  const T* wdn = nx0 ? wdinv<T>(h.levels[k + 1]) : nullptr;
  T* xtn = nx0 ? static_cast<T*>(h.levels[k + 1].xt) : nullptr;
  if (!kcyc && !(!cheb && !sgs && k > 0 && lv.n <= kFuseCorrectionRows))
    launch_rows<T>(lv.nc, lv.rlpr, lv.agg_ptr, lv.agg_rows, rvals<T>(lv), OpRestrict<T>{A, r, rcv, wdn, xtn}, rc,
                   s);
  if (!kcyc) {
    if (k + 1 == L) coarse_solve<T>(h, rcv, c, act);
    else cycle<T>(h, k + 1, rcv, c, act, nullptr, nx0);
    if (lv.n <= kFuseCorrectionRows) {
      post_smooth<T>(h, lv, k, A, b, xt, wd, xo, CorrV<T>{lv.agg, pv, c}, fuse_q, rc);
    } else {
      launch_elem(lv.n, OpProlong<T>{A, lv.agg, pv, c, xt}, rc, s);
      post_smooth<T>(h, lv, k, A, b, xt, wd, xo, CorrNone<T>{}, fuse_q, rc);
    }
  } else {
    Level& lc = h.levels[k + 1];
    double* K = h.d_sc + kScK + 16 * k;
    int* F = h.d_ctl + kCtlKFlags + 4 * k;
    T* v = static_cast<T*>(lv.v);
    T* rt = static_cast<T*>(lv.rt);
    T* d = static_cast<T*>(lv.d);
    T* w = static_cast<T*>(lv.w);
    const int gm = h.opt.krylov == AMG_KRYLOV_FGMRES ? 1 : 0;
    launch_rows<T>(lv.nc, lv.rlpr, lv.agg_ptr, lv.agg_rows, rvals<T>(lv), OpRestrict<T>{A, r, rcv, wdn, xtn}, rc,
                   s);
    cycle<T>(h, k + 1, rcv, c, act, nullptr, nx0);                     // first inner iteration
    launch_level<T>(lc, OpKDots1<T>{A, c, rcv, v, K, F, gm, h.opt.kcycle_t}, rc, s);
    launch_elem(lc.n, OpRtilde<T>{Act{F}, rcv, v, rt, K, wdn, xtn}, rc, s);
    cycle<T>(h, k + 1, rt, d, F, nullptr, nx0);                        // second inner iteration
    launch_level<T>(lc, OpKDots2<T>{Act{F}, d, v, rt, w, K, F, gm}, rc, s);
    if (lv.n <= kFuseCorrectionRows) {
      post_smooth<T>(h, lv, k, A, b, xt, wd, xo, CorrK<T>{lv.agg, pv, c, d, K, F}, fuse_q, rc);
    } else {
      launch_elem(lv.n, OpProlongK<T>{A, lv.agg, pv, c, d, xt, K, F}, rc, s);
      post_smooth<T>(h, lv, k, A, b, xt, wd, xo, CorrNone<T>{}, fuse_q, rc);
    }
  }
}

void set_ctl(Hierarchy& h, int word, int value) {
  launch_elem(1, OpSetCtl{h.d_ctl, word, value}, red(h), h.stream);
}

// z = M r.  fuse_q: compute z'q (the FCG beta) inside the cycle's last
// kernel; r32_ready: the FP32 copy of r is already written (mixed mode).
// Returns whether z'q was computed.
template <typename T>
bool precondition(Hierarchy& h, const int* act, const double* fuse_q = nullptr, bool r32_ready = false) {
  hipStream_t s = h.stream;
  if constexpr (sizeof(T) == sizeof(float)) {
    if (!r32_ready) launch_elem(h.levels[0].n, OpToFloat{Act{act}, h.r, static_cast<float*>(h.bz)}, red(h), s);
    cycle<float>(h, 0, static_cast<const float*>(h.bz), static_cast<float*>(h.z), act, fuse_q);
  } else {
    cycle<double>(h, 0, h.r, static_cast<double*>(h.z), act, fuse_q);
  }
  return fuse_q != nullptr && h.L() > 0;
}

template <typename T>
void fcg_iteration(Hierarchy& h, const int* run) {
  Level& l0 = h.levels[0];
  hipStream_t s = h.stream;
  RedCtx rc = red(h);
  const int n = l0.n;
  {
    const Level* lp = &l0;
    const OpFcgSpmv op{Act{run}, h.p, h.r, h.q, h.d_sc, h.d_ctl, h.d_err};
    probe_point(h, h.opt.probe == AMG_PROBE_OUTER_SPMV,
                [=](hipStream_t st) { launch_level<double>(*lp, op, rc, st); });
  }
  float* r32 = sizeof(T) == sizeof(float) ? static_cast<float*>(h.bz) : nullptr;
  launch_elem(n, OpFcgUpdate{Act{run}, h.p, h.q, h.xint, h.r, h.d_sc, h.d_ctl, h.d_err, r32}, rc, s);
  if (!precondition<T>(h, run, h.q, r32 != nullptr))
    launch_elem(n, OpDotZQ<T>{Act{run}, static_cast<const T*>(h.z), h.q, h.d_sc}, rc, s);
  launch_elem(n, OpPUpdate<T>{Act{run}, static_cast<const T*>(h.z), h.p, h.d_sc, 0}, rc, s);
}

template <typename T>
void fcg_restart(Hierarchy& h, const int* run) {
  const int n = h.levels[0].n;
  precondition<T>(h, run);
  launch_elem(n, OpPUpdate<T>{Act{run}, static_cast<const T*>(h.z), h.p, h.d_sc, 1}, red(h), h.stream);
}

void check_err(Hierarchy& h, int bits) {
  if (!bits) return;
  if (bits & kErrNonFinite) throw Error(AMG_ENANINF, "non-finite value in the iteration");
  if (bits & kErrBreakdown) throw Error(AMG_EBREAKDOWN, "Krylov breakdown: p^T A p <= 0");
  if (bits & kErrTimeout) throw Error(AMG_EHIP, "a wait of the one-launch V-cycle tail ran out");
  throw Error(AMG_EHIP, "device error bits " + std::to_string(bits));
}

void enqueue_iterations(Hierarchy& h, int count, bool mixed) {
  const int* run = h.d_ctl + kCtlRunning;
  for (int i = 0; i < count; ++i) {
    if (h.g_iter.empty()) {
      if (mixed) fcg_iteration<float>(h, run);
      else fcg_iteration<double>(h, run);
      continue;
    }
    AMG_HIP(hipGraphLaunch(h.g_iter[0], h.stream));
    if (h.g_iter.size() > 1) {
      AMG_HIP(hipEventRecord(h.pev[0], h.stream));
      h.probe_fn(h.stream);
      AMG_HIP(hipEventRecord(h.pev[1], h.stream));
      AMG_HIP(hipGraphLaunch(h.g_iter[1], h.stream));
    }
  }
}

void enqueue_restart(Hierarchy& h, bool mixed) {
  const int* run = h.d_ctl + kCtlRunning;
  if (h.g_restart) AMG_HIP(hipGraphLaunch(h.g_restart, h.stream));
  else if (mixed) fcg_restart<float>(h, run);
  else fcg_restart<double>(h, run);
}

// Outer flexible CG.  Iterations are enqueued in batches between host checks
// of the device convergence flag; the batch length follows the residual
// reduction observed so far (iterations after convergence are no-ops).
int fcg(Hierarchy& h, const double* b, double rtol, double* x, int* iters, double* relres) {
  Level& l0 = h.levels[0];
  hipStream_t s = h.stream;
  RedCtx rc = red(h);
  const int n = l0.n;
  const bool mixed = h.mixed();
  int* hp = static_cast<int*>(h.h_pinned);
  double* hd = reinterpret_cast<double*>(hp + 16);

  launch_elem(n, OpFcgInit{b, h.r, h.xint, h.d_sc, h.d_ctl, h.d_err, rtol}, rc, s);
  enqueue_restart(h, mixed);
  const int max_iter = h.opt.max_iter;
  const int cap = h.opt.check_every > 0 ? h.opt.check_every : 1;
  int enqueued = 0, batch = 1, it_prev = 0;
  double rel_prev = 1.0;
  int status = AMG_OK;
  while (true) {
    if (enqueued + batch > max_iter) batch = max_iter - enqueued;
    enqueue_iterations(h, batch, mixed);
    enqueued += batch;
    AMG_HIP(hipGetLastError());
    AMG_HIP(hipMemcpyAsync(hp, h.d_ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hp + 2, h.d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hd, h.d_sc, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    check_err(h, hp[2]);
    const int running = hp[kCtlRunning];
    const int done = hp[kCtlIters];
    if (running && h.pev[0]) {
      // the batch's last iteration ran every kernel: sample the probed one
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, h.pev[0], h.pev[1]) == hipSuccess) {
        h.probe_ms += ms;
        h.probe_samples += 1;
      }
    }
    if (running && enqueued < max_iter) {
      const double rel = std::sqrt(hd[kScRR] / hd[kScBB]);
      batch = 1;
      if (done > it_prev && rel < rel_prev && rel > 0.0) {
        const double f = std::pow(rel / rel_prev, 1.0 / (done - it_prev));
        if (f < 1.0) {
          const double need = std::ceil(std::log(rtol / rel) / std::log(f));
          batch = need < 1.0 ? 1 : (need > cap ? cap : (int)need);
        }
      }
      rel_prev = rel;
      it_prev = done;
      continue;
    }
    // recompute the true residual in FP64
    launch_level<double>(l0, OpTrueResid{Act{nullptr}, b, h.xint, h.q, h.d_sc}, rc, s);
    AMG_HIP(hipMemcpyAsync(hd, h.d_sc, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    const double bb = hd[kScBB];
    const double rel = bb > 0.0 ? std::sqrt(hd[kScTrue] / bb) : 0.0;
    *iters = done;
    *relres = rel;
    if (!std::isfinite(rel)) throw Error(AMG_ENANINF, "non-finite residual");
    if (rel <= rtol || bb == 0.0) break;
    if (done >= max_iter || enqueued >= max_iter) {
      status = AMG_ENOTCONV;
      break;
    }
    // the recurrence residual met the tolerance but the true one did not:
    // restart from the true residual
    launch_elem(n, OpCopy{h.q, h.r}, rc, s);
    set_ctl(h, kCtlRunning, 1);
    enqueue_restart(h, mixed);
    batch = 1;
  }
  AMG_HIP(hipMemcpyAsync(x, h.xint, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return status;
}
// ------------------------------------------------------------ flexible GMRES
// Right-preconditioned FGMRES(m) (flexible: the preconditioned vectors z_j
// are kept and x = x_0 + Z y).  Hessenberg entries come from device dots,
// the Givens rotations, the residual estimate |g_{j+1}| and the triangular
// solve run in one-thread kernels, so a restart cycle is enqueued without
// host round-trips.  Device block `gm`: H[(m+1) x m] (row stride m), cs[m],
// sn[m], g[m+1], y[m], then [bnorm, jdone].
struct GmView {
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* y;
  double* misc;   // misc[0] = ||b||, misc[1] = inner steps of this cycle
  int m;
};

inline GmView gm_view(double* base, int m) {
  GmView v;
  v.m = m;
  v.H = base;
  v.cs = v.H + (size_t)(m + 1) * m;
  v.sn = v.cs + m;
  v.g = v.sn + m;
  v.y = v.g + m + 1;
  v.misc = v.y + m;
  return v;
}

// r = b - A x with ||r||^2: starts a cycle (g = [beta, 0, ...]); on the first
// cycle also records ||b|| (x = 0 there)
struct OpGmInit {
  static constexpr int NV = 1;
  Act a;
  const double* b;
  const double* xv;
  double* r;
  GmView gv;
  int first;
  double rtol;
  int* ctl;
  int* err;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ double x(int j) const { return xv[j]; }
  __device__ void row(int i, double ax, double* acc) const {
    const double t = b[i] - ax;
    r[i] = t;
    acc[0] += t * t;
  }
  __device__ void finalize(const double* s) const {
    const double beta = sqrt(s[0]);
    if (first) gv.misc[0] = beta;
    gv.misc[1] = 0.0;
    gv.g[0] = beta;
    for (int j = 1; j <= gv.m; ++j) gv.g[j] = 0.0;
    if (!__builtin_isfinite(beta)) {
      *err |= kErrNonFinite;
      ctl[kCtlRunning] = 0;
    } else {
      ctl[kCtlRunning] = beta > rtol * gv.misc[0] ? 1 : 0;
    }
  }
};

// w = A z_j (z in the cycle precision) with v_0' w -> H[0][j]
template <typename T>
struct OpGmSpmv {
  static constexpr int NV = 1;
  Act a;
  const T* z;
  const double* v0;
  double* w;
  double* hout;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ double x(int j) const { return (double)z[j]; }
  __device__ void row(int i, double ax, double* acc) const {
    w[i] = ax;
    acc[0] += v0[i] * ax;
  }
  __device__ void finalize(const double* s) const { *hout = s[0]; }
};

struct OpGmAxpyDot {
  static constexpr int NV = 1;
  Act a;
  const double* vi;
  const double* vn;   // nullptr: the norm of w
  double* w;
  const double* hcoef;
  double* out;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double* acc) const {
    const double t = w[i] - (*hcoef) * vi[i];
    w[i] = t;
    acc[0] += (vn ? vn[i] : t) * t;
  }
  __device__ void finalize(const double* s) const { *out = vn ? s[0] : sqrt(s[0]); }
};

struct OpGmScale {
  static constexpr int NV = 0;
  Act a;
  const double* in;
  double* out;
  const double* den;
  __device__ bool active() const { return a.on(); }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { out[i] = in[i] / *den; }
  __device__ void finalize(const double*) const {}
};

// Givens update of column j and the convergence test
__global__ void k_gm_givens(GmView gv, int j, double rtol, int* ctl, int* err) {
  if (!ctl[kCtlRunning]) return;
  const int m = gv.m;
  double* Hc = gv.H;   // H[i][j] at Hc[i * m + j]
  for (int i = 0; i < j; ++i) {
    const double t = gv.cs[i] * Hc[i * m + j] + gv.sn[i] * Hc[(i + 1) * m + j];
    Hc[(i + 1) * m + j] = -gv.sn[i] * Hc[i * m + j] + gv.cs[i] * Hc[(i + 1) * m + j];
    Hc[i * m + j] = t;
  }
  const double hjj = Hc[j * m + j], hj1 = Hc[(j + 1) * m + j];
  const double den = hypot(hjj, hj1);
  ctl[kCtlIters] += 1;
  gv.misc[1] = j + 1;
  if (!(den > 0.0) || !__builtin_isfinite(den)) {
    if (!__builtin_isfinite(den)) *err |= kErrNonFinite;
    ctl[kCtlRunning] = 0;
    gv.misc[1] = j;   // nothing usable from this column
    return;
  }
  gv.cs[j] = hjj / den;
  gv.sn[j] = hj1 / den;
  Hc[j * m + j] = den;
  Hc[(j + 1) * m + j] = 0.0;
  gv.g[j + 1] = -gv.sn[j] * gv.g[j];
  gv.g[j] = gv.cs[j] * gv.g[j];
  if (fabs(gv.g[j + 1]) <= rtol * gv.misc[0] || hj1 == 0.0) ctl[kCtlRunning] = 0;
}

// y = R^-1 g over the inner steps of the cycle (back substitution)
__global__ void k_gm_trisolve(GmView gv) {
  const int k = (int)gv.misc[1];
  const int m = gv.m;
  for (int i = k - 1; i >= 0; --i) {
    double t = gv.g[i];
    for (int q = i + 1; q < k; ++q) t -= gv.H[i * m + q] * gv.y[q];
    gv.y[i] = t / gv.H[i * m + i];
  }
}

// x += Z y
template <typename T>
struct OpGmUpdate {
  static constexpr int NV = 0;
  const T* Z;
  size_t ld;
  GmView gv;
  double* xv;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const {
    const int k = (int)gv.misc[1];
    double t = xv[i];
    for (int j = 0; j < k; ++j) t += gv.y[j] * (double)Z[(size_t)j * ld + i];
    xv[i] = t;
  }
  __device__ void finalize(const double*) const {}
};

template <typename T>
int fgmres(Hierarchy& h, const double* b, double rtol, double* x, int* iters, double* relres) {
  Level& l0 = h.levels[0];
  hipStream_t s = h.stream;
  RedCtx rc = red(h);
  const int n = l0.n;
  const int m = std::max(1, std::min(h.opt.gmres_restart, 64));
  Arena ws;
  struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
  double* V = ws.alloc_n<double>((size_t)(m + 1) * n);
  T* Z = ws.alloc_n<T>((size_t)m * n);
  float* v32 = sizeof(T) == sizeof(float) ? ws.alloc_n<float>(n) : nullptr;
  double* w = ws.alloc_n<double>(n);
  double* gmem = ws.alloc_n<double>((size_t)(m + 1) * m + 4 * m + 4);
  GmView gv = gm_view(gmem, m);
  const int* run = h.d_ctl + kCtlRunning;
  const Act A{run};
  double* xv = h.xint;
  int* hp = static_cast<int*>(h.h_pinned);
  double* hd = reinterpret_cast<double*>(hp + 16);
  launch_fill_double(n, xv, 0.0, s);
  set_ctl(h, kCtlIters, 0);
  int status = AMG_OK;
  bool first = true;
  int done_before = 0;
  while (true) {
    const int steps = std::min(m, h.opt.max_iter - done_before);
    launch_level<double>(l0, OpGmInit{Act{nullptr}, b, xv, w, gv, first ? 1 : 0, rtol, h.d_ctl, h.d_err}, rc, s);
    first = false;
    launch_elem(n, OpGmScale{A, w, V, gv.g}, rc, s);
    for (int j = 0; j < steps; ++j) {
      double* vj = V + (size_t)j * n;
      T* zj = Z + (size_t)j * n;
      if constexpr (sizeof(T) == sizeof(float)) {
        launch_elem(n, OpToFloat{A, vj, v32}, rc, s);
        cycle<float>(h, 0, v32, reinterpret_cast<float*>(zj), run);
      } else {
        cycle<double>(h, 0, vj, reinterpret_cast<double*>(zj), run);
      }
      launch_level<double>(l0, OpGmSpmv<T>{A, zj, V, w, gv.H + j}, rc, s);
      for (int i = 0; i <= j; ++i) {
        const double* vi = V + (size_t)i * n;
        const double* vn = i < j ? V + (size_t)(i + 1) * n : nullptr;
        launch_elem(n, OpGmAxpyDot{A, vi, vn, w, gv.H + (size_t)i * m + j, gv.H + (size_t)(i + 1) * m + j}, rc, s);
      }
      launch_elem(n, OpGmScale{A, w, V + (size_t)(j + 1) * n, gv.H + (size_t)(j + 1) * m + j}, rc, s);
      k_gm_givens<<<1, 1, 0, s>>>(gv, j, rtol, h.d_ctl, h.d_err);
    }
    k_gm_trisolve<<<1, 1, 0, s>>>(gv);
    launch_elem(n, OpGmUpdate<T>{Z, (size_t)n, gv, xv}, rc, s);
    AMG_HIP(hipGetLastError());
    AMG_HIP(hipMemcpyAsync(hp, h.d_ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hp + 2, h.d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(hd, gv.misc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    check_err(h, hp[2]);
    const int done = hp[kCtlIters];
    done_before = done;
    const double bnorm = hd[0];
    // true residual
    launch_level<double>(l0, OpTrueResid{Act{nullptr}, b, xv, h.q, h.d_sc}, rc, s);
    AMG_HIP(hipMemcpyAsync(hd, h.d_sc + kScTrue, sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    const double rel = bnorm > 0.0 ? std::sqrt(hd[0]) / bnorm : 0.0;
    if (!std::isfinite(rel)) throw Error(AMG_ENANINF, "non-finite residual");
    *iters = done;
    *relres = rel;
    if (rel <= rtol || bnorm == 0.0) break;
    if (done >= h.opt.max_iter) {
      status = AMG_ENOTCONV;
      break;
    }
  }
  AMG_HIP(hipMemcpyAsync(x, xv, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return status;
}

// ------------------------------------------------------------ autotuner
std::mutex g_tune_mu;
std::map<TuneKey, Level::Tune>& tune_cache() {
  static auto& c = *new std::map<TuneKey, Level::Tune>();   // never destroyed (no exit-time destructor)
  static bool loaded = false;
  if (!loaded) {
    loaded = true;
    if (const char* path = std::getenv("AMG_TUNE_CACHE")) {
      if (FILE* f = std::fopen(path, "r")) {
        TuneKey k{};
        Level::Tune t{};
        while (std::fscanf(f,
                           " {\"n\": %d, \"nnz\": %d, \"bytes\": %d, \"nrhs\": %d, \"rowstat\": %ld, \"fmt\": %d, "
                           "\"lpr\": %d, \"pz\": %d, \"sh\": %d, \"tile\": %d, \"us\": %f}",
                           &k.n, &k.nnz, &k.bytes, &k.nrhs, &k.rowstat, &t.fmt, &t.lpr, &t.pz, &t.sh, &t.tile,
                           &t.us) == 11)
          c[k] = t;
        std::fclose(f);
      }
    }
  }
  return c;
}

}  // namespace

bool TuneKey::operator<(const TuneKey& o) const {
  return std::tie(n, nnz, bytes, nrhs, rowstat) < std::tie(o.n, o.nnz, o.bytes, o.nrhs, o.rowstat);
}

bool tune_cache_get(const TuneKey& k, Level::Tune* t) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto& c = tune_cache();
  auto it = c.find(k);
  if (it == c.end()) return false;
  *t = it->second;
  return true;
}

void tune_cache_put(const TuneKey& k, const Level::Tune& t) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_cache()[k] = t;
  if (const char* path = std::getenv("AMG_TUNE_CACHE")) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f,
                   "{\"n\": %d, \"nnz\": %d, \"bytes\": %d, \"nrhs\": %d, \"rowstat\": %ld, \"fmt\": %d, "
                   "\"lpr\": %d, \"pz\": %d, \"sh\": %d, \"tile\": %d, \"us\": %.3f}\n",
                   k.n, k.nnz, k.bytes, k.nrhs, k.rowstat, t.fmt, t.lpr, t.pz, t.sh, t.tile, t.us);
      std::fclose(f);
    }
  }
}

namespace {

// The largest column offset col - row of a level (rows are sorted, so the
// last entry of each row), read back to the host.
__global__ void k_max_offset(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int e = rp[i + 1];
    if (e > rp[i]) atomicMax(out, ci[e - 1] - i);
  }
}

int max_column_offset(Hierarchy& h, const Level& lv) {
  int* d = h.d_ctl + kCtlAggFill;   // scratch word, free outside the Galerkin product
  launch_fill_int(1, d, 0, h.stream);
  const long g = ((long)lv.n + 255) / 256;
  k_max_offset<<<(int)(g < 4096 ? g : 4096), 256, 0, h.stream>>>(lv.n, lv.rp, lv.ci, d);
  int v = 0;
  AMG_HIP(hipMemcpyAsync(&v, d, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  AMG_HIP(hipStreamSynchronize(h.stream));
  return v;
}

template <typename T>
struct OpFillT {
  static constexpr int NV = 0;
  T* p;
  T v;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { p[i] = v; }
  __device__ void finalize(const double*) const {}
};

// Schedules (block_steps) of the 64-row slice kernels worth timing on a
// level of nslices slices whose largest column offset is off rows:
// contiguous (0), the XCD sweep (-1) and plane-ordered (the plane in 4-slice
// steps, when it is a whole number of steps that tiles the slices, as on
// lexicographic grids).  AMG_TUNE_SCHEDULE = contiguous, sweep or plane
// keeps that one where it applies (tests).
std::vector<int> schedules(int nslices, int off) {
  std::vector<int> v{0, -1};
  const int steps = (nslices + 3) / 4;
  if (off > 0 && off % 256 == 0) {
    const int p = off / 256;
    if (nslices % 4 == 0 && steps % p == 0 && steps / p >= 2) v.push_back(p);
  }
  if (const char* f = std::getenv("AMG_TUNE_SCHEDULE")) {
    const std::string w(f);
    std::vector<int> k;
    for (int c : v)
      if ((w == "contiguous" && c == 0) || (w == "sweep" && c == -1) || (w == "plane" && c > 0))
        k.push_back(c);
    if (!k.empty()) return k;
  }
  return v;
}

// Time the pre-smoothing kernel for CSR with 2..32 lanes per row (with 32-
// and 16-bit columns) and for sliced ELL with 32- and 16-bit columns (in the
// schedules above); keep the fastest (AMG_TUNE_FORCE = csr, csr16, sell,
// sell16 or sdia pins the format where the level has it, for tests).  Results are cached per level shape (n, nnz,
// sliced-ELL size) and value size for the process and, when AMG_TUNE_CACHE
// names a file, across processes (one JSON object per line).
template <typename T>
Level::Tune tune_one(Hierarchy& h, Level& lv, T* x, T* y) {
  if (lv.n <= kFuseCorrectionRows) {
    // small levels are latency-bound and their kernels gather more than a
    // plain SpMV (the fused correction), so a timed SpMV is a poor and noisy
    // proxy there: take 8..32 lanes, about two entries per lane (against one:
    // C3 solve 34.2 -> 33.2 ms, C2 8.84 -> 8.74 ms; against 16 lanes on every
    // small level: 33.1 and 8.86 ms)
    Level::Tune t;
    t.fmt = 0;
    t.lpr = 8;
    while (t.lpr < 32 && 2L * t.lpr * lv.n < lv.nnz) t.lpr <<= 1;
    return t;
  }
  TuneKey key;
  key.n = lv.n;
  key.nnz = lv.nnz;
  key.bytes = (int)sizeof(T);
  key.nrhs = 1;
  key.rowstat = lv.sl_total;
  const char* force = std::getenv("AMG_TUNE_FORCE");
  if (!force && !std::getenv("AMG_TUNE_SLICE") && !std::getenv("AMG_TUNE_SCHEDULE")) {
    Level::Tune t;
    if (tune_cache_get(key, &t)) return t;
  }
  hipStream_t s = h.stream;
  RedCtx rc = red(h);
  launch_elem(lv.n, OpFillT<T>{x, T(1)}, rc, s);
  Level::Tune best;
  best.us = 1e30f;
  hipEvent_t e0 = h.ev[2], e1 = h.ev[3];
  const int reps = 8;
  constexpr float kPreferFewerBytes = 1.05f;
  auto time_it = [&](auto&& launch) {   // the better of two timed runs
    launch();
    float best_us = 1e30f;
    for (int trial = 0; trial < 2; ++trial) {
      AMG_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) launch();
      AMG_HIP(hipEventRecord(e1, s));
      AMG_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
      best_us = std::min(best_us, ms * 1000.f / reps);
    }
    return best_us;
  };
  // the pre-smoothing kernel (two gathered arrays per entry), the commonest
  // row kernel of a cycle
  const OpPresmoothResid<T> op{Act{nullptr}, x, x, y, y};
  for (int lpr = 2; lpr <= 32; lpr <<= 1) {
    const float us = time_it([&] { launch_rows<T>(lv.n, lpr, lv.rp, lv.ci, vals<T>(lv), op, rc, s); });
    if (us < best.us) { best.us = us; best.fmt = 0; best.lpr = lpr; }
  }
  if (lv.ci16) {   // 16-bit column offsets: 2 bytes less per entry, taken within kPreferFewerBytes of CSR
    // the same rows and lanes as CSR with fewer bytes: timed with CSR's best lanes only
    const int lpr = best.lpr;
    const float us = time_it([&] { launch_rows16<T>(lv.n, lpr, lv.rp, lv.ci16, vals<T>(lv), op, rc, s); });
    if (std::getenv("AMG_DEBUG"))
      std::fprintf(stderr, "amg: level n=%d CSR 16-bit offsets lanes=%d: %.2f us (best so far %.2f)\n", lv.n, lpr,
                   us, best.us);
    if (us <= kPreferFewerBytes * best.us) { best.us = std::min(us, best.us); best.fmt = 4; }
  }
  const int off = (lv.sl_ptr && sell_vals<T>(lv)) || dia_vals<T>(lv) ? max_column_offset(h, lv) : 0;
  if (lv.sl_ptr && sell_vals<T>(lv)) {
    for (int p : schedules(lv.nslices, off)) {
      const float us = time_it([&] {
        launch_sell<T>(lv.n, lv.nslices, lv.sl_ptr, lv.sl_col, sell_vals<T>(lv), op, rc, s, nullptr, p);
      });
      if (us < best.us) { best.us = us; best.fmt = 1; best.lpr = lv.lpr; best.pz = p; }
      if (lv.sl_dcol) {
        // 16-bit offsets move 2 bytes less per entry.  Back-to-back timed
        // launches find part of a level's data in the Infinity Cache, which
        // in the cycle (other levels' kernels in between) it is not, so they
        // understate that saving: the 16-bit form is kept unless the 32-bit
        // one is more than kPreferFewerBytes faster (C3 mixed, level 0 in FP32: 32-bit
        // columns timed faster, 16-bit offsets solved 1.3 ms faster).
        const float u16 = time_it([&] {
          launch_sell<T>(lv.n, lv.nslices, lv.sl_ptr, lv.sl_col, sell_vals<T>(lv), op, rc, s, lv.sl_dcol, p);
        });
        const bool over32 = best.fmt == 1 && best.pz == p && u16 <= kPreferFewerBytes * best.us;
        if (u16 < best.us || over32) { best.us = u16; best.fmt = 2; best.lpr = lv.lpr; best.pz = p; }
      }
    }
  }
  if (lv.sh.ptr && short_vals<T>(lv)) {   // the copy in shorter slices, 32- and 16-bit columns
    for (int f = 1; f <= 2; ++f) {
      if (f == 2 && !lv.sh.dcol) break;
      const float us = time_it([&] {
        launch_sell<T>(lv.n, lv.sh.nslices, lv.sh.ptr, lv.sh.col, short_vals<T>(lv), op, rc, s,
                       f == 2 ? lv.sh.dcol : nullptr, 0, lv.sh.h, lv.sh.perm);
      });
      if (std::getenv("AMG_DEBUG"))
        std::fprintf(stderr, "amg: level n=%d %d-row slices fmt=%d: %.2f us (best so far %.2f)\n", lv.n, lv.sh.h, f,
                     us, best.us);
      if (us < best.us) { best.us = us; best.fmt = f; best.lpr = lv.lpr; best.pz = 0; best.sh = lv.sh.h; }
    }
  }
  if (dia_vals<T>(lv)) {   // sliced diagonals, in the same schedules
    for (int p : schedules(lv.dia.nslices, off)) {
      const float us = time_it([&] {
        launch_sdia<T>(lv.n, lv.dia.nslices, lv.dia.ptr, lv.dia.off, dia_vals<T>(lv), op, rc, s, p);
      });
      if (std::getenv("AMG_DEBUG"))
        std::fprintf(stderr, "amg: level n=%d sliced diagonals pz=%d: %.2f us (best so far %.2f)\n", lv.n, p, us,
                     best.us);
      // fewer bytes than any sliced ELL: preferred within kPreferFewerBytes, as the 16-bit offsets are
      const bool over_sell = (best.fmt == 1 || best.fmt == 2) && best.sh == 0 && us <= kPreferFewerBytes * best.us;
      if (us < best.us || over_sell) { best.us = us; best.fmt = 3; best.lpr = lv.lpr; best.pz = p; best.sh = 0; }
    }
  }
  if (force) {   // "csr", "csr16", "sell", "sell16" or "sdia", the sliced ELL optionally ":32" or ":16" (slice height)
    std::string w(force);
    int fh = 0;
    const size_t colon = w.find(':');
    if (colon != std::string::npos) {
      fh = std::atoi(w.c_str() + colon + 1);
      w = w.substr(0, colon);
    }
    const bool short_ok = fh > 0 && lv.sh.h == fh && short_vals<T>(lv) != nullptr;
    if (w == "csr") {
      best.fmt = 0;
      best.sh = 0;
    } else if (w == "csr16") {
      if (lv.ci16) {
        best.fmt = 4;
        best.sh = 0;
        if (best.lpr < 2) best.lpr = 4;
      }
    } else if (w == "sdia") {
      if (dia_vals<T>(lv)) {
        best.fmt = 3;
        best.sh = 0;
      }
    } else if (w == "sell" && lv.sl_ptr) {
      best.fmt = 1;
      best.sh = short_ok ? fh : 0;
    } else if (w == "sell16" && lv.sl_dcol) {
      best.fmt = 2;
      best.sh = short_ok && lv.sh.dcol ? fh : 0;
    }
    if (best.sh) best.pz = 0;
    else if (best.fmt != 0 && std::getenv("AMG_TUNE_SCHEDULE"))
      best.pz = schedules(best.fmt == 3 ? lv.dia.nslices : lv.nslices, off).front();
    return best;   // not cached
  }
  if (!std::getenv("AMG_TUNE_SLICE") && !std::getenv("AMG_TUNE_SCHEDULE")) tune_cache_put(key, best);
  return best;
}

}  // namespace

void autotune_levels(Hierarchy& h) {
  const bool debug = std::getenv("AMG_DEBUG") != nullptr;
  const char* force_h = std::getenv("AMG_TUNE_SLICE");   // 32 or 16: build that slice height (tests)
  const bool pinned = force_h || std::getenv("AMG_TUNE_FORCE") || std::getenv("AMG_TUNE_SCHEDULE");
  for (int k = 0; k < h.L(); ++k) {
    Level& lv = h.levels[k];
    // candidate copies in shorter slices (rows that vary in length) and in
    // sliced diagonals (structured levels); not built when the cached
    // decisions of this level shape use neither
    bool need_sh = lv.n > kFuseCorrectionRows && lv.sl_ptr;
    bool need_dia = need_sh;
    bool need_c16 = need_sh && lv.sl_dcol;   // the offsets fit in 16 bits
    if (need_sh && !pinned) {
      TuneKey key;
      key.n = lv.n;
      key.nnz = lv.nnz;
      key.rowstat = lv.sl_total;
      Level::Tune c32, c64;
      key.bytes = 4;
      const bool h32 = !h.mixed() || tune_cache_get(key, &c32);
      key.bytes = 8;
      const bool use64 = !h.mixed() || k == 0;
      const bool h64 = !use64 || tune_cache_get(key, &c64);
      if (h32 && h64) {
        need_sh = (h.mixed() && c32.sh > 0) || (use64 && c64.sh > 0);
        need_dia = (h.mixed() && c32.fmt == 3) || (use64 && c64.fmt == 3);
        need_c16 = need_c16 && ((h.mixed() && c32.fmt == 4) || (use64 && c64.fmt == 4));
      }
    }
    if (need_sh) build_short_sell(h, lv, force_h ? std::atoi(force_h) : 0);
    if (need_dia) build_sdia(h, lv);
    if (need_c16 && !lv.ci16) {
      auto mem = std::make_shared<Arena>();
      lv.ci16 = mem->alloc_n<int16_t>((size_t)std::max(lv.nnz, 1));
      launch_ci16(lv.n, lv.rp, lv.ci, lv.ci16, h.stream);
      lv.ci16_mem = mem;
    }
    if (h.mixed()) {
      lv.t32 = tune_one<float>(h, lv, static_cast<float*>(lv.xt), static_cast<float*>(lv.r));
      if (k == 0) lv.t64 = tune_one<double>(h, lv, h.p, h.q);
    } else {
      lv.t64 = tune_one<double>(h, lv, static_cast<double*>(lv.xt), static_cast<double*>(lv.r));
    }
    if (lv.sh.ptr && lv.t64.sh != lv.sh.h && lv.t32.sh != lv.sh.h) {   // not chosen: release it
      lv.sh = Level::ShortSell{};
      lv.sh_mem.reset();
    }
    if (lv.dia.ptr && lv.t64.fmt != 3 && lv.t32.fmt != 3) {
      lv.dia = Level::Sdia{};
      lv.dia_mem.reset();
    }
    if (lv.ci16 && lv.t64.fmt != 4 && lv.t32.fmt != 4) {
      lv.ci16 = nullptr;
      lv.ci16_mem.reset();
    }
    if (debug)
      std::fprintf(stderr,
                   "amg: tune level %d n=%d fp64 fmt=%d lpr=%d pz=%d sh=%d %.2f us | fp32 fmt=%d lpr=%d pz=%d sh=%d "
                   "%.2f us\n",
                   k, lv.n, lv.t64.fmt, lv.t64.lpr, lv.t64.pz, lv.t64.sh, lv.t64.us, lv.t32.fmt, lv.t32.lpr,
                   lv.t32.pz, lv.t32.sh, lv.t32.us);
  }
}

int solve_fcg_impl(Hierarchy& h, const double* b, double rtol, double* x, int* iters, double* relres) {
  if (h.opt.krylov == AMG_KRYLOV_FGMRES) {
    if (h.mixed()) return fgmres<float>(h, b, rtol, x, iters, relres);
    return fgmres<double>(h, b, rtol, x, iters, relres);
  }
  return fcg(h, b, rtol, x, iters, relres);
}

// Capture one outer iteration and the (re)start sequence into HIP graphs on
// a private stream; the solve replays them on the caller's stream.  Every
// captured kernel reads its device flag, so one graph serves all branches.
void build_solve_graphs(Hierarchy& h) {
  hipStream_t user = h.stream;
  hipStream_t cs = nullptr;
  AMG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const int* run = h.d_ctl + kCtlRunning;
  const bool mixed = h.mixed();
  auto finish = [&](hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    AMG_HIP(hipStreamEndCapture(cs, &g));
    AMG_HIP(hipGraphInstantiate(out, g, nullptr, nullptr, 0));
    AMG_HIP(hipGraphDestroy(g));
  };
  try {
    h.stream = cs;
    h.cap_stream = cs;
    h.capturing = true;
    // outer iteration, split at the probed kernel when a probe is selected
    h.split_at_probe = h.opt.probe != AMG_PROBE_NONE && h.pev[0];
    AMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    if (mixed) fcg_iteration<float>(h, run);
    else fcg_iteration<double>(h, run);
    hipGraphExec_t last = nullptr;
    finish(&last);
    h.g_iter.push_back(last);
    h.split_at_probe = false;
    // (re)start sequence
    AMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    if (mixed) fcg_restart<float>(h, run);
    else fcg_restart<double>(h, run);
    finish(&h.g_restart);
  } catch (...) {
    h.stream = user;
    h.capturing = false;
    h.split_at_probe = false;
    (void)hipStreamDestroy(cs);
    throw;
  }
  h.stream = user;
  h.capturing = false;
  h.cap_stream = nullptr;
  AMG_HIP(hipStreamDestroy(cs));
}

// Arnoldi on D^-1 A_k (modified Gram-Schmidt) from the seeded start vector,
// enqueued on stream s with scalar slots sc (kScArn .. kScArn + 64) and
// reduction context rc; the (m+1) x m Hessenberg matrix (row stride 8) and
// the norms ||D^-1 A q_j|| (at 48 + j) are copied to host_out (pinned, 56
// doubles) without waiting.
void arnoldi_enqueue(Hierarchy& h, const Level& lv, int m, uint32_t stream, double* Q, double* w, double* sc,
                     RedCtx rc, double* host_out, hipStream_t s) {
  (void)h;
  const int n = lv.n;
  launch_elem(n, OpArnStart{Q, sc, stream}, rc, s);
  launch_elem(n, OpDivide{Q, Q, sc + kScArn + 56}, rc, s);
  for (int j = 0; j < m; ++j) {
    const double* qj = Q + (size_t)j * n;
    const OpArnSpmv op{qj, Q, lv.diag, w, sc, j, n};
    if (lv.nslices > 0 && lv.nnz <= 12L * n)   // short, even rows: sliced ELL
      launch_sell<double>(n, lv.nslices, lv.sl_ptr, lv.sl_col, lv.sl_val, op, rc, s, lv.sl_dcol);
    else
      launch_rows<double>(n, lv.lpr, lv.rp, lv.ci, lv.val, op, rc, s);
    launch_elem(n, OpArnUpdate{Q, w, sc, sc + kScArn + (j + 1) * 8 + j, j, n}, rc, s);
    launch_elem(n, OpDivide{w, Q + (size_t)(j + 1) * n, sc + kScArn + (j + 1) * 8 + j}, rc, s);
  }
  AMG_HIP(hipMemcpyAsync(host_out, sc + kScArn, 56 * sizeof(double), hipMemcpyDeviceToHost, s));
}

// The same on the hierarchy's stream, waiting for the result.
void arnoldi(Hierarchy& h, Level& lv, int m, uint32_t stream, double* Q, double* w, double* H_out,
             double* wnorm_out) {
  double* hd = static_cast<double*>(h.h_pinned) + kPinnedArn;
  arnoldi_enqueue(h, lv, m, stream, Q, w, h.d_sc, red(h), hd, h.stream);
  AMG_HIP(hipStreamSynchronize(h.stream));
  for (int i = 0; i < 48; ++i) H_out[i] = hd[i];
  for (int j = 0; j < 8; ++j) wnorm_out[j] = hd[48 + j];
}

int pick_lanes_per_row(int n, int nnz) { return pick_lpr(n, nnz); }

// q_i = unit_uniform(i, stream), the seeded hash vector in [-1, 1)
void launch_hash_vector(int n, uint32_t stream, double* q, hipStream_t s) {
  launch_elem(n, OpHashVector{q, stream}, RedCtx{nullptr, nullptr}, s);
}

void spmv_sell_level(Hierarchy& h, const Level& lv, const double* x, double* y, bool offsets16) {
  launch_sell<double>(lv.n, lv.nslices, lv.sl_ptr, lv.sl_col, lv.sl_val, OpSpmv<double>{Act{nullptr}, x, y},
                      red(h), h.stream, offsets16 ? lv.sl_dcol : nullptr);
}

// Column s of a row-major [n][S] block to a vector and back, and the
// coarse-corrected error e - P y.
struct OpColGet {
  static constexpr int NV = 0;
  const double* E;
  int S, s;
  double* v;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { v[i] = E[(size_t)i * S + s]; }
  __device__ void finalize(const double*) const {}
};
struct OpCoarseCorrect {
  static constexpr int NV = 0;
  const double* e;
  const int* agg;
  const double* pv;
  const double* y;
  double* out;
  int S, s;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const {
    const int a = agg[i];
    out[(size_t)i * S + s] = a >= 0 ? e[i] - pv[i] * y[a] : e[i];
  }
  __device__ void finalize(const double*) const {}
};
struct OpAddTo {
  static constexpr int NV = 0;
  const double* z;
  double* y;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double*) const { y[i] += z[i]; }
  __device__ void finalize(const double*) const {}
};

// The two-grid error after the coarse correction of level k (the error the
// smoother of level k must damp in a cycle, Algorithm 4):
//   out_s = (I - P_k B P_k^T A_k) e_s,  B ~ A_{k+1}^-1,
// B the exact coarse inverse when level k+1 is the coarsest, else `cycles`
// steps of y <- y + M_{k+1}(r_c - A_{k+1} y) from y = 0 with the hierarchy's
// own cycle M_{k+1} from level k+1.  E, out: device [n_k][S] row-major.
// FP64 hierarchies (the cycle from level k+1 runs on the FP64 operators).
void coarse_corrected_errors(Hierarchy& h, int k, const double* E, int S, int cycles, double* out) {
  const int L = h.L();
  if (k < 0 || k >= L) throw Error(AMG_EINVAL, "coarse_corrected_errors: level has no coarse level");
  if (h.mixed()) throw Error(AMG_EUNSUPPORTED, "coarse_corrected_errors: mixed-precision hierarchy");
  const Level& lv = h.levels[k];
  const Level& lc = h.levels[k + 1];
  const int n = lv.n, nc = lc.n;
  hipStream_t s = h.stream;
  RedCtx rc = red(h);
  Arena tmp;
  double* e = tmp.alloc_n<double>(n);
  double* r = tmp.alloc_n<double>(n);
  double* bc = tmp.alloc_n<double>(nc);
  double* y = tmp.alloc_n<double>(nc);
  double* res = tmp.alloc_n<double>(nc);
  double* z = tmp.alloc_n<double>(nc);
  const int steps = k + 1 == L ? 1 : std::max(cycles, 1);
  for (int q = 0; q < S; ++q) {
    launch_elem(n, OpColGet{E, S, q, e}, rc, s);
    launch_level<double>(lv, OpSpmv<double>{Act{nullptr}, e, r}, rc, s);
    launch_rows<double>(lv.nc, lv.rlpr, lv.agg_ptr, lv.agg_rows, rvals<double>(lv),
                        OpRestrict<double>{Act{nullptr}, r, bc}, rc, s);
    launch_fill_double(nc, y, 0.0, s);
    for (int it = 0; it < steps; ++it) {
      launch_level<double>(lc, OpResid<double>{Act{nullptr}, bc, y, res}, rc, s);
      if (k + 1 == L) coarse_solve<double>(h, res, z, nullptr);
      else cycle<double>(h, k + 1, res, z, nullptr);
      launch_elem(nc, OpAddTo{z, y}, rc, s);
    }
    launch_elem(n, OpCoarseCorrect{e, lv.agg, lv.pval, y, out, S, q}, rc, s);
  }
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
}

// y = A_k x with level k's tuned FP64 kernel
void level_spmv(const Hierarchy& h, int k, const double* x, double* y, hipStream_t s) {
  launch_level<double>(h.levels[k], OpSpmv<double>{Act{nullptr}, x, y}, RedCtx{nullptr, nullptr}, s);
}

// y = A x for a caller's matrix (float64)
void spmv_f64(int n, int nnz, const int* rp, const int* ci, const double* val, const double* x, double* y,
              int lpr, hipStream_t s) {
  if (lpr <= 0) lpr = pick_lpr(n, nnz);
  RedCtx rc{nullptr, nullptr};
  launch_rows<double>(n, lpr, rp, ci, val, OpSpmv<double>{Act{nullptr}, x, y}, rc, s);
}

}  // namespace amg
