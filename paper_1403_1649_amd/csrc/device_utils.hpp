// Device-side primitives shared by the HIP kernels (wave64 CDNA4).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <stdint.h>

namespace amg {

constexpr int kWave = 64;

// MurmurHash3 32-bit finaliser: a bijection of uint32 (every step invertible).
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Seeded counter hash of a node index: fmix32(i + stream * 0x9E3779B9 mod 2^32).
__device__ __forceinline__ uint32_t node_hash(uint32_t i, uint32_t stream) {
  return fmix32(i + stream * 0x9E3779B9u);
}

// Exact float64 in [-1, 1): hash * 2^-31 - 1.
__device__ __forceinline__ double unit_uniform(uint32_t i, uint32_t stream) {
  return (double)node_hash(i, stream) * 4.656612873077392578125e-10 - 1.0;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over a sub-group of G consecutive lanes (G a power of two <= 64);
// the result is valid in every lane of the group.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Block-wide sum of NV values (fixed combination order: lanes, then waves).
// `red` must hold NV * (blockDim.x / 64) doubles of LDS.  Result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * nw + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[k * nw + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Exclusive scan of one int per thread over the block; returns the exclusive
// prefix, *total receives the block sum (valid in all threads).
// `tmp` must hold blockDim.x/64 + 1 ints of LDS.
__device__ __forceinline__ int block_exclusive_scan(int v, int* tmp, int* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  int incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) tmp[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < nw; ++w) {
      int t = tmp[w];
      tmp[w] = run;
      run += t;
    }
    tmp[nw] = run;
  }
  __syncthreads();
  int res = incl - v + tmp[wid];
  *total = tmp[nw];
  __syncthreads();
  return res;
}

// FP64 matrix-core step D = A B + C on a 16 x 16 tile with k = 4
// (v_mfma_f64_16x16x4f64).  Operands per lane l of the wave: a = A[l % 16][l / 16],
// b = B[l / 16][l % 16]; the accumulator holds D[l / 16 + 4 i][l % 16] in
// element i (rows interleaved by four; checked on the device).
typedef double f64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f64x4 mfma_f64_16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int mfma_row(int lane, int i) { return (lane >> 4) + 4 * i; }
__device__ __forceinline__ int mfma_col(int lane) { return lane & 15; }

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// This bijection of [0, gridDim.x) gives every XCD a contiguous run of
// logical blocks, so rows that gather from overlapping neighbourhoods share
// an L2 (XCD x holds the blocks b = 8 s + x).
__device__ __forceinline__ int xcd_block_index() {
  const int g = gridDim.x, b = blockIdx.x;
  if (g < 8) return b;
  const int x = b & 7, f = g >> 3, r = g & 7;
  return x * f + (x < r ? x : r) + (b >> 3);
}

// Rows by groups of G lanes (G divides the wave): group id and lane of this
// thread, and the group-wide reductions the row kernels use.
template <int G>
struct RowGroup {
  long gid, ngroups;
  int lane;
  __device__ RowGroup()
      : gid(((long)xcd_block_index() * blockDim.x + threadIdx.x) / G),
        ngroups((long)gridDim.x * blockDim.x / G),
        lane(threadIdx.x & (G - 1)) {}
  __device__ static int sum(int v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
  }
  __device__ static double max(double v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off, G);
      v = o > v ? o : v;
    }
    return v;
  }
  // bits of this group's lanes in a wave ballot
  __device__ static uint64_t group_bits(uint64_t ballot) {
    if (G == 64) return ballot;
    const int shift = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    return (ballot >> shift) & ((1ull << G) - 1);
  }
};


// Grid for n rows at G lanes each (256-thread blocks, grid-stride beyond).
inline int group_grid(int n, int G) {
  long b = ((long)n * G + 255) / 256;
  if (b < 1) b = 1;
  return (int)(b < 65536 ? b : 65536);
}
// Calls f(std::integral_constant<int, G>) for G = the lanes per row.
template <typename F>
void with_lanes(int G, F&& f) {
  switch (G) {
    case 1: f(std::integral_constant<int, 1>()); break;
    case 2: f(std::integral_constant<int, 2>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 8: f(std::integral_constant<int, 8>()); break;
    case 16: f(std::integral_constant<int, 16>()); break;
    default: f(std::integral_constant<int, 32>()); break;
  }
}

// Device-scope atomic helpers.
__device__ __forceinline__ void atomic_or_flag(int* p, int bits) {
  __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


}  // namespace amg
