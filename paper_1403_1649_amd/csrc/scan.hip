// Device-wide scan of int32 counts into CSR-style pointers:
// ptr[0] = 0, ptr[i+1] = counts[0] + ... + counts[i].
// Three passes: per-block local scans, one block scanning the block sums,
// then a uniform add.  Used for coarse numbering and row pointers in setup.
#include "amg_internal.hpp"
#include "device_utils.hpp"

namespace amg {

namespace {
constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;

__global__ void __launch_bounds__(kThreads) k_scan_local(const int* __restrict__ counts,
                                                         int* __restrict__ ptr, int n,
                                                         int* __restrict__ bsum) {
  __shared__ int tile[kTile];
  __shared__ int tmp[kThreads / kWave + 1];
  const int base = blockIdx.x * kTile;
  // coalesced load of the tile into LDS
  for (int k = threadIdx.x; k < kTile; k += kThreads) {
    int idx = base + k;
    tile[k] = idx < n ? counts[idx] : 0;
  }
  __syncthreads();
  int v[kItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    v[k] = tile[threadIdx.x * kItems + k];
    s += v[k];
  }
  int total;
  int run = block_exclusive_scan(s, tmp, &total);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    run += v[k];
    tile[threadIdx.x * kItems + k] = run;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kTile; k += kThreads) {
    int idx = base + k;
    if (idx < n) ptr[idx + 1] = tile[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) k_scan_top(int* bsum, int nb) {
  __shared__ int tmp[1024 / kWave + 1];
  int carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    int idx = base + threadIdx.x;
    int v = idx < nb ? bsum[idx] : 0;
    int total;
    int ex = block_exclusive_scan(v, tmp, &total);
    if (idx < nb) bsum[idx] = ex + carry;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void __launch_bounds__(kThreads) k_scan_add(int* __restrict__ ptr, int n,
                                                       const int* __restrict__ bsum) {
  const int b = blockIdx.x;
  const int add = bsum[b];
  const int base = b * kTile;
  for (int k = threadIdx.x; k < kTile; k += kThreads) {
    int idx = base + k;
    if (idx < n) ptr[idx + 1] += add;
  }
  if (b == 0 && threadIdx.x == 0) ptr[0] = 0;
}
}  // namespace

int scan_blocks_needed(int n) { return (n + kTile - 1) / kTile; }

void scan_to_ptr(const int* counts, int* ptr, int n, int* block_sums, hipStream_t s) {
  if (n <= 0) {
    launch_fill_int(1, ptr, 0, s);
    return;
  }
  const int nb = scan_blocks_needed(n);
  k_scan_local<<<nb, kThreads, 0, s>>>(counts, ptr, n, block_sums);
  k_scan_top<<<1, 1024, 0, s>>>(block_sums, nb);
  k_scan_add<<<nb, kThreads, 0, s>>>(ptr, n, block_sums);
}

}  // namespace amg
