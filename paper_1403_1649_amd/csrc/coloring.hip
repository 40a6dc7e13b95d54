// Multi-colour ordering for the symmetric Gauss-Seidel smoother (Section
// 2.2.1): rows of one colour share no entry of A, so a Gauss-Seidel sweep
// updates a whole colour at once.  The colouring is first-fit in decreasing
// node-hash priority h_i = fmix32(i + stream * 0x9E3779B9), built in
// synchronous rounds (Jones-Plassmann): an uncoloured row whose priority
// beats every uncoloured neighbour takes the smallest colour its coloured
// neighbours leave free.  Every neighbour of higher priority is coloured by
// then, so the result is the sequential first-fit colouring, bit for bit.
#include "kernels_common.hpp"

namespace amg {

namespace {
constexpr int kT = 256;

inline int grid1(long n) {
  long g = (n + kT - 1) / kT;
  if (g < 1) g = 1;
  return (int)(g < 65536 ? g : 65536);
}

// One round: cin -> cout.  left[round & 1] counts the rows still uncoloured
// after the round (one atomic per wave); the round also clears the other
// counter for the next round.  Colours are limited to 64 (bit mask).
__global__ void __launch_bounds__(kT) k_color_round(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                    uint32_t stream, const int* __restrict__ cin,
                                                    int* __restrict__ cout, int* left, int round, int* err) {
  if (blockIdx.x == 0 && threadIdx.x == 0) left[(round + 1) & 1] = 0;
  int undecided = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int c = cin[i];
    if (c < 0) {
      const uint32_t p = node_hash((uint32_t)i, stream);
      uint64_t used = 0;
      bool wait = false;
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int j = ci[k];
        if (j == i) continue;
        const int cj = cin[j];
        if (cj < 0) wait = wait || node_hash((uint32_t)j, stream) > p;
        else used |= 1ull << cj;
      }
      if (!wait) {
        if (~used == 0ull) {
          atomic_or_flag(err, kErrColors);
          c = 63;
        } else {
          c = __ffsll((unsigned long long)~used) - 1;
        }
      } else {
        undecided = 1;
      }
    }
    cout[i] = c;
  }
  const uint64_t b = __ballot(undecided);
  if ((threadIdx.x & (kWave - 1)) == 0 && b)
    __hip_atomic_fetch_add(&left[round & 1], __popcll(b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kT) k_color_count(int n, const int* __restrict__ col, int* cnt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicAdd(&cnt[col[i]], 1);
}

// rows of colour c at crow[coff[c] .. coff[c+1]) (order within a colour is
// immaterial: its rows are updated independently)
__global__ void __launch_bounds__(kT) k_color_scatter(int n, const int* __restrict__ col,
                                                      const int* __restrict__ coff, int* fill,
                                                      int* __restrict__ crow) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c = col[i];
    crow[coff[c] + atomicAdd(&fill[c], 1)] = i;
  }
}
}  // namespace

void launch_color_round(int n, const int* rp, const int* ci, uint32_t stream, const int* cin, int* cout, int* left,
                        int round, int* err, hipStream_t s) {
  k_color_round<<<grid1(n), kT, 0, s>>>(n, rp, ci, stream, cin, cout, left, round, err);
}

void launch_color_lists(int n, const int* col, int* cnt, const int* coff, int* crow, hipStream_t s) {
  k_color_scatter<<<grid1(n), kT, 0, s>>>(n, col, coff, cnt, crow);
}

void launch_color_count(int n, const int* col, int* cnt, hipStream_t s) {
  k_color_count<<<grid1(n), kT, 0, s>>>(n, col, cnt);
}

}  // namespace amg
