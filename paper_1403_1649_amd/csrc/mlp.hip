// Learned per-row Jacobi weights: omega_i = sigmoid(y_i) * 2|a_ii| /
// (|a_ii| + sum_{j != i} |a_ij|), y = MLP(features of row i), 9 -> 32 -> 32 -> 1
// with ReLU.  Operands are bfloat16 (round to nearest even), products and sums
// in FP32, biases FP32; hidden activations are rounded to bfloat16 before the
// next layer.  The bound makes 2 D Omega^-1 - A strictly diagonally dominant
// with a positive diagonal, so the smoother converges for SPD A.
//
// Training loss on a level (S samples with no coarse-space component,
// e = v - P P^T v):  L = (1/S) sum_s ||(I - W A) e||_A^2 / ||e||_A^2.
// Weight layout (1409 FP32 masters): W1[32][9], b1[32], W2[32][32], b2[32],
// W3[32], b3.
#include <cmath>

#include "kernels_common.hpp"

namespace amg {

namespace {
constexpr int kIn = 9, kH = 32;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kNP = oB3 + 1;   // 1409

__device__ __forceinline__ float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// log|a_ii| summed over the level (for the level mean)
struct OpLogDiagSum {
  static constexpr int NV = 1;
  const double* diag;
  double* out;
  __device__ bool active() const { return true; }
  __device__ void idle() const {}
  __device__ void elem(int i, double* acc) const { acc[0] += log(fabs(diag[i])); }
  __device__ void finalize(const double* s) const { *out = s[0]; }
};

__global__ void __launch_bounds__(256) k_features(int n, int level, const int* __restrict__ rp,
                                                  const int* __restrict__ ci, const double* __restrict__ val,
                                                  const double* __restrict__ logsum, float* __restrict__ F,
                                                  double* __restrict__ beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double mean = *logsum / n;
  double d = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k)
    if (ci[k] == i) d = val[k];
  const double ad = fabs(d);
  double top[6] = {0, 0, 0, 0, 0, 0};
  double rs = 0.0, offabs = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    rs += val[k];
    if (ci[k] == i) continue;
    const double a = fabs(val[k]);
    offabs += a;
    double t = a / ad;
    for (int q = 0; q < 6; ++q) {   // keep the six largest, descending
      if (t > top[q]) { const double u = top[q]; top[q] = t; t = u; }
    }
  }
  float* f = F + (size_t)i * kIn;
  f[0] = bf16r((float)(log(ad) - mean));
  for (int q = 0; q < 6; ++q) f[1 + q] = bf16r((float)top[q]);
  f[7] = bf16r((float)(rs / d));
  f[8] = bf16r((float)level);
  if (beta) beta[i] = 2.0 * ad / (ad + offabs);
}

// forward pass of one row with the weights in LDS (already bf16-rounded)
struct Fwd {
  float z1[kH], h1[kH], z2[kH], h2[kH], y;
};

__device__ __forceinline__ void mlp_forward(const float* __restrict__ w, const float* __restrict__ x, Fwd& o) {
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float s = w[oB1 + j];
#pragma unroll
    for (int q = 0; q < kIn; ++q) s = fmaf(w[oW1 + j * kIn + q], x[q], s);
    o.z1[j] = s;
    o.h1[j] = bf16r(fmaxf(s, 0.f));
  }
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float s = w[oB2 + j];
#pragma unroll
    for (int q = 0; q < kH; ++q) s = fmaf(w[oW2 + j * kH + q], o.h1[q], s);
    o.z2[j] = s;
    o.h2[j] = bf16r(fmaxf(s, 0.f));
  }
  float y = w[oB3];
#pragma unroll
  for (int q = 0; q < kH; ++q) y = fmaf(w[oW3 + q], o.h2[q], y);
  o.y = y;
}

__device__ __forceinline__ void load_weights(const float* __restrict__ wmaster, float* s_w) {
  for (int q = threadIdx.x; q < kNP; q += blockDim.x) {
    const bool bias = (q >= oB1 && q < oW2) || (q >= oB2 && q < oW3) || q == oB3;
    s_w[q] = bias ? wmaster[q] : bf16r(wmaster[q]);
  }
  __syncthreads();
}

// omega_i and omega_i / a_ii for a level
__global__ void __launch_bounds__(256) k_mlp_omega(int n, const float* __restrict__ F, const double* __restrict__ beta,
                                                   const double* __restrict__ diag, const float* __restrict__ wm,
                                                   double* __restrict__ omega, double* __restrict__ wdinv,
                                                   float* __restrict__ wdinv32, double* __restrict__ sig_out) {
  __shared__ float s_w[kNP];
  load_weights(wm, s_w);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[kIn];
#pragma unroll
  for (int q = 0; q < kIn; ++q) x[q] = F[(size_t)i * kIn + q];
  Fwd o;
  mlp_forward(s_w, x, o);
  const double sg = 1.0 / (1.0 + exp(-(double)o.y));
  const double om = sg * beta[i];
  if (omega) omega[i] = om;
  if (sig_out) sig_out[i] = sg;
  if (wdinv) {
    const double wd = om / diag[i];
    wdinv[i] = wd;
    if (wdinv32) wdinv32[i] = (float)wd;
  }
}

// ---------------------------------------------------------------- loss pipeline
// v_s[i] = unit_uniform(i, seed + s) (or the caller's extra samples), then
// restricted per aggregate: c[I][s] = sum_{i in G_I} pval_i v_s[i]
__global__ void k_err_raw(int n, int S, int S_rand, uint32_t seed, const double* __restrict__ extra, double* __restrict__ V) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * S) return;
  const int i = (int)(t / S), s = (int)(t - (long)i * S);
  V[t] = s < S_rand ? unit_uniform((uint32_t)i, seed + (uint32_t)s) : extra[(size_t)i * (S - S_rand) + (s - S_rand)];
}

__global__ void k_err_restrict(int nc, int S, const int* __restrict__ agg_ptr, const int* __restrict__ agg_rows,
                               const double* __restrict__ pval, const double* __restrict__ V, double* __restrict__ C) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nc * S) return;
  const int I = (int)(t / S), s = (int)(t - (long)I * S);
  double acc = 0.0;
  for (int k = agg_ptr[I]; k < agg_ptr[I + 1]; ++k) {
    const int i = agg_rows[k];
    acc += pval[i] * V[(size_t)i * S + s];
  }
  C[t] = acc;
}

// e_s -= P (P^T e_s) for the first S_proj samples (the others stay as given)
__global__ void k_err_project(int n, int S, int S_proj, const int* __restrict__ agg, const double* __restrict__ pval,
                              const double* __restrict__ C, double* __restrict__ E) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * S) return;
  const int i = (int)(t / S), s = (int)(t - (long)i * S);
  if (s < S_proj) E[t] -= pval[i] * C[(size_t)agg[i] * S + s];
}

// Y = A X for a [n][S] block (thread per entry)
__global__ void k_spmm_simple(int n, int S, const int* __restrict__ rp, const int* __restrict__ ci,
                              const double* __restrict__ val, const double* __restrict__ X, double* __restrict__ Y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * S) return;
  const int i = (int)(t / S), s = (int)(t - (long)i * S);
  double acc = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) acc += val[k] * X[(size_t)ci[k] * S + s];
  Y[t] = acc;
}

// per-sample dot products d[s] = sum_i X[i][s] Y[i][s] (two passes, block order)
__global__ void __launch_bounds__(256) k_coldot_part(int n, int S, const double* __restrict__ X,
                                                     const double* __restrict__ Y, double* __restrict__ part) {
  __shared__ double red[256];
  for (int s = 0; s < S; ++s) {
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
      acc += X[(size_t)i * S + s] * Y[(size_t)i * S + s];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)s * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ void k_coldot_final(int S, int nb, const double* __restrict__ part, double* __restrict__ out) {
  const int s = threadIdx.x;
  if (s >= S) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += part[(size_t)s * nb + b];
  out[s] = acc;
}

// E2 = E - (omega / a) .* AE
__global__ void k_smooth_err(int n, int S, const double* __restrict__ omega, const double* __restrict__ diag,
                             const double* __restrict__ E, const double* __restrict__ AE, double* __restrict__ E2) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * S) return;
  const int i = (int)(t / S);
  E2[t] = E[t] - omega[i] / diag[i] * AE[t];
}

// dL/dy_i = (-2/S) sum_s AE2[i][s] AE[i][s] / (ee_s a_ii) * beta_i sigma_i (1 - sigma_i)
__global__ void k_dy(int n, int S, const double* __restrict__ AE, const double* __restrict__ AE2,
                     const double* __restrict__ ee, const double* __restrict__ diag, const double* __restrict__ beta,
                     const double* __restrict__ sig, float* __restrict__ dy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int s = 0; s < S; ++s) acc += AE2[(size_t)i * S + s] * AE[(size_t)i * S + s] / ee[s];
  const double dom = -2.0 / S * acc / diag[i];
  dy[i] = (float)(dom * beta[i] * sig[i] * (1.0 - sig[i]));
}

// Backward pass: tiles of 64 rows per wave; the per-row vectors go to LDS and
// the 1409 weight-gradient entries are accumulated by the wave's 64 lanes in
// a fixed row order; one partial vector per block.
constexpr int kTile = 64;
__global__ void __launch_bounds__(kTile) k_mlp_backward(int n, const float* __restrict__ F, const float* __restrict__ dy,
                                                        const float* __restrict__ wm, float* __restrict__ part) {
  __shared__ float s_w[kNP];
  __shared__ float s_x[kTile][kIn];
  __shared__ float s_h1[kTile][kH];
  __shared__ float s_h2[kTile][kH];
  __shared__ float s_dz1[kTile][kH];
  __shared__ float s_dz2[kTile][kH];
  __shared__ float s_dy[kTile];
  load_weights(wm, s_w);
  constexpr int kPer = (kNP + kTile - 1) / kTile;   // 23 entries per lane
  float acc[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) acc[q] = 0.f;
  const int lane = threadIdx.x;
  const int tiles = (n + kTile - 1) / kTile;
  for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int i = t * kTile + lane;
    if (i < n) {
      float x[kIn];
#pragma unroll
      for (int q = 0; q < kIn; ++q) x[q] = F[(size_t)i * kIn + q];
      Fwd o;
      mlp_forward(s_w, x, o);
      const float g = dy[i];
      float dz2[kH];
#pragma unroll
      for (int j = 0; j < kH; ++j) dz2[j] = o.z2[j] > 0.f ? g * s_w[oW3 + j] : 0.f;
#pragma unroll
      for (int m = 0; m < kH; ++m) {
        float dh = 0.f;
#pragma unroll
        for (int j = 0; j < kH; ++j) dh = fmaf(dz2[j], s_w[oW2 + j * kH + m], dh);
        s_dz1[lane][m] = o.z1[m] > 0.f ? dh : 0.f;
      }
#pragma unroll
      for (int q = 0; q < kIn; ++q) s_x[lane][q] = x[q];
#pragma unroll
      for (int j = 0; j < kH; ++j) {
        s_h1[lane][j] = o.h1[j];
        s_h2[lane][j] = o.h2[j];
        s_dz2[lane][j] = dz2[j];
      }
      s_dy[lane] = g;
    } else {
#pragma unroll
      for (int q = 0; q < kIn; ++q) s_x[lane][q] = 0.f;
#pragma unroll
      for (int j = 0; j < kH; ++j) { s_h1[lane][j] = 0.f; s_h2[lane][j] = 0.f; s_dz1[lane][j] = 0.f; s_dz2[lane][j] = 0.f; }
      s_dy[lane] = 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int p = lane + q * kTile;
      if (p >= kNP) break;
      float a = acc[q];
      if (p < oB1) {                       // W1[m][c] += dz1[m] x[c]
        const int m = p / kIn, c = p - m * kIn;
        for (int r = 0; r < kTile; ++r) a = fmaf(s_dz1[r][m], s_x[r][c], a);
      } else if (p < oW2) {                // b1
        const int m = p - oB1;
        for (int r = 0; r < kTile; ++r) a += s_dz1[r][m];
      } else if (p < oB2) {                // W2[j][m] += dz2[j] h1[m]
        const int j = (p - oW2) / kH, m = (p - oW2) - j * kH;
        for (int r = 0; r < kTile; ++r) a = fmaf(s_dz2[r][j], s_h1[r][m], a);
      } else if (p < oW3) {                // b2
        const int j = p - oB2;
        for (int r = 0; r < kTile; ++r) a += s_dz2[r][j];
      } else if (p < oB3) {                // W3[j] += dy h2[j]
        const int j = p - oW3;
        for (int r = 0; r < kTile; ++r) a = fmaf(s_dy[r], s_h2[r][j], a);
      } else {                             // b3
        for (int r = 0; r < kTile; ++r) a += s_dy[r];
      }
      acc[q] = a;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int p = lane + q * kTile;
    if (p < kNP) part[(size_t)blockIdx.x * kNP + p] = acc[q];
  }
}

__global__ void k_grad_final(int nb, const float* __restrict__ part, float* __restrict__ grad, int accumulate) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNP) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * kNP + p];
  grad[p] = accumulate ? grad[p] + (float)s : (float)s;
}

__global__ void k_adam(int n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline int nblk(long n, int t = 256) { return (int)((n + t - 1) / t); }
}  // namespace

int mlp_num_params() { return kNP; }

// level mean of log|a_ii| and the features of every row (float [n][9]);
// beta (optional) receives the omega bound 2|a_ii| / (|a_ii| + sum |a_ij|)
void mlp_features(Hierarchy& h, const Level& lv, int level, float* F, double* beta) {
  hipStream_t s = h.stream;
  double* slot = h.d_sc + kScArn + 60;
  launch_elem(lv.n, OpLogDiagSum{lv.diag, slot}, RedCtx{h.d_part, h.d_ticket}, s);
  k_features<<<nblk(lv.n), 256, 0, s>>>(lv.n, level, lv.rp, lv.ci, lv.val, slot, F, beta);
}

void mlp_omega(Hierarchy& h, const Level& lv, const float* F, const double* beta, const float* wdev, double* omega,
               double* wdinv, float* wdinv32, double* sig) {
  k_mlp_omega<<<nblk(lv.n), 256, 0, h.stream>>>(lv.n, F, beta, lv.diag, wdev, omega, wdinv, wdinv32, sig);
}

// Smoothing loss of a level and (optionally) its gradient.  Work arrays from
// `tmp`.  Returns the loss (synchronises); grad (device, kNP) when non-null.
double mlp_loss_grad(Hierarchy& h, Arena& tmp, const Level& lv, int level, const float* wdev, int S_rand,
                     uint32_t seed, const double* extra, int S_extra, const double* omega_fixed, float* grad,
                     int accumulate, bool raw_extra) {
  hipStream_t s = h.stream;
  const int n = lv.n, S = S_rand + S_extra;
  if (S < 1 || S > 64) throw Error(AMG_EINVAL, "1 to 64 error samples");
  const size_t nS = (size_t)n * S;
  double* E = tmp.alloc_n<double>(nS);
  double* C = tmp.alloc_n<double>((size_t)lv.nc * S);
  double* AE = tmp.alloc_n<double>(nS);
  double* E2 = tmp.alloc_n<double>(nS);
  double* AE2 = tmp.alloc_n<double>(nS);
  double* ee = tmp.alloc_n<double>(64);
  double* num = tmp.alloc_n<double>(64);
  const int nbd = 256;
  double* dpart = tmp.alloc_n<double>((size_t)64 * nbd);
  k_err_raw<<<nblk((long)nS), 256, 0, s>>>(n, S, S_rand, seed, extra, E);
  k_err_restrict<<<nblk((long)lv.nc * S), 256, 0, s>>>(lv.nc, S, lv.agg_ptr, lv.agg_rows, lv.pval, E, C);
  k_err_project<<<nblk((long)nS), 256, 0, s>>>(n, S, raw_extra ? S_rand : S, lv.agg, lv.pval, C, E);
  k_spmm_simple<<<nblk((long)nS), 256, 0, s>>>(n, S, lv.rp, lv.ci, lv.val, E, AE);
  k_coldot_part<<<nbd, 256, 0, s>>>(n, S, E, AE, dpart);
  k_coldot_final<<<1, 64, 0, s>>>(S, nbd, dpart, ee);
  float* F = tmp.alloc_n<float>((size_t)n * kIn);
  double* beta = tmp.alloc_n<double>(n);
  double* om = tmp.alloc_n<double>(n);
  double* sig = tmp.alloc_n<double>(n);
  mlp_features(h, lv, level, F, beta);
  const double* omega = omega_fixed;
  if (!omega) {
    mlp_omega(h, lv, F, beta, wdev, om, nullptr, nullptr, sig);
    omega = om;
  }
  k_smooth_err<<<nblk((long)nS), 256, 0, s>>>(n, S, omega, lv.diag, E, AE, E2);
  k_spmm_simple<<<nblk((long)nS), 256, 0, s>>>(n, S, lv.rp, lv.ci, lv.val, E2, AE2);
  k_coldot_part<<<nbd, 256, 0, s>>>(n, S, E2, AE2, dpart);
  k_coldot_final<<<1, 64, 0, s>>>(S, nbd, dpart, num);
  if (grad && !omega_fixed) {
    float* dy = tmp.alloc_n<float>(n);
    k_dy<<<nblk(n), 256, 0, s>>>(n, S, AE, AE2, ee, lv.diag, beta, sig, dy);
    const int tiles = (n + kTile - 1) / kTile;
    const int nb = tiles < 1024 ? tiles : 1024;
    float* part = tmp.alloc_n<float>((size_t)nb * kNP);
    k_mlp_backward<<<nb, kTile, 0, s>>>(n, F, dy, wdev, part);
    k_grad_final<<<nblk(kNP), 256, 0, s>>>(nb, part, grad, accumulate);
  }
  std::vector<double> he(64), hn(64);
  AMG_HIP(hipMemcpyAsync(he.data(), ee, S * sizeof(double), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipMemcpyAsync(hn.data(), num, S * sizeof(double), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  AMG_HIP(hipGetLastError());
  double L = 0.0;
  for (int q = 0; q < S; ++q) L += hn[q] / he[q];
  return L / S;
}

void mlp_adam(float* w, float* m, float* v, const float* g, int n, int step, float lr, float b1, float b2, float eps,
              hipStream_t s) {
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  k_adam<<<nblk(n), 256, 0, s>>>(n, w, m, v, g, lr, b1, b2, eps, c1, c2);
}

}  // namespace amg
