// Device-wide scan of int32 counts into CSR-style pointers:
// ptr[0] = 0, ptr[i+1] = counts[0] + ... + counts[i].
// One pass with decoupled look-back: every block takes its tile in the order
// the blocks start (a ticket; the last one resets the counter for the next
// call), scans it, publishes its tile sum, then reads the published words of
// earlier tiles, 64 at a time (one per lane of the first wave), back to the
// nearest one that carries an inclusive prefix, and publishes its own.  A
// status word packs a call epoch, a 2-bit state and the 32-bit value, so one
// 64-bit atomic store publishes it and words left by earlier calls never
// match.  Used for coarse numbering and row pointers in setup.
#include "amg_internal.hpp"
#include "device_utils.hpp"

namespace amg {

namespace {
constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;

__device__ __forceinline__ uint64_t scan_word(uint32_t epoch, uint32_t state, int v) {
  return ((uint64_t)epoch << 34) | ((uint64_t)state << 32) | (uint32_t)v;
}

__global__ void __launch_bounds__(kThreads) k_scan(const int* __restrict__ counts, int* __restrict__ ptr, int n,
                                                   uint64_t* status, unsigned long long* ticket,
                                                   uint32_t epoch) {
  __shared__ int tile[kTile];
  __shared__ int tmp[kThreads / kWave + 1];
  __shared__ int s_tile, s_prefix;
  if (threadIdx.x == 0) {
    const int t = (int)atomicAdd(ticket, 1ull);
    if (t == (int)gridDim.x - 1) atomicExch(ticket, 0ull);   // every ticket is taken
    s_tile = t;
  }
  __syncthreads();
  const int t = s_tile;
  const int base = t * kTile;
  for (int k = threadIdx.x; k < kTile; k += kThreads) {
    const int idx = base + k;
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
  if (threadIdx.x < kWave) {
    // the first wave publishes, then looks back 64 tiles at a time: lane l
    // reads tile p - l; the window counts once every tile up to the nearest
    // inclusive prefix has published
    const int lane = threadIdx.x;
    int prefix = 0;
    if (t == 0) {
      if (lane == 0)
        __hip_atomic_store(&status[0], scan_word(epoch, 2, total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(&status[t], scan_word(epoch, 1, total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int p = t - 1;;) {
        const int q = p - lane;
        uint32_t st = 2;
        int v = 0;
        if (q >= 0) {
          const uint64_t w = __hip_atomic_load(&status[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          st = (uint32_t)(w >> 34) == epoch ? (uint32_t)(w >> 32) & 3u : 0u;
          v = (int)(uint32_t)w;
        }
        const uint64_t inc = __ballot(st == 2), none = __ballot(st == 0);
        const int first = inc ? __ffsll((unsigned long long)inc) - 1 : kWave;   // nearest inclusive
        const uint64_t upto = first == kWave ? ~0ull : ((2ull << first) - 1);
        if (none & upto) {   // a tile before it has not published yet
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        int x = lane <= first ? v : 0;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
        prefix += x;
        if (first < kWave) break;
        p -= kWave;
      }
      if (lane == 0)
        __hip_atomic_store(&status[t], scan_word(epoch, 2, prefix + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) s_prefix = prefix;
  }
  __syncthreads();
  const int prefix = s_prefix;
  for (int k = threadIdx.x; k < kTile; k += kThreads) {
    const int idx = base + k;
    if (idx < n) ptr[idx + 1] = tile[k] + prefix;
  }
  if (t == 0 && threadIdx.x == 0) ptr[0] = 0;
}
}  // namespace

int scan_blocks_needed(int n) { return (n + kTile - 1) / kTile; }

void init_scan(ScanCtx& sc, Arena& arena, int nmax, hipStream_t s) {
  const int nb = scan_blocks_needed(nmax > 0 ? nmax : 1);
  sc.status = arena.alloc_n<uint64_t>((size_t)nb + 1);
  sc.ticket = reinterpret_cast<unsigned long long*>(sc.status + nb);
  sc.max_blocks = nb;
  sc.epoch = 1;   // zeroed words carry epoch 0 and never match
  launch_fill_int(2 * ((size_t)nb + 1), reinterpret_cast<int*>(sc.status), 0, s);
}

void scan_to_ptr(const int* counts, int* ptr, int n, ScanCtx& sc, hipStream_t s) {
  if (n <= 0) {
    launch_fill_int(1, ptr, 0, s);
    return;
  }
  const int nb = scan_blocks_needed(n);
  if (nb > sc.max_blocks) throw Error(AMG_EINVAL, "scan longer than its scratch");
  k_scan<<<nb, kThreads, 0, s>>>(counts, ptr, n, sc.status, sc.ticket, sc.epoch);
  sc.epoch = sc.epoch + 1 < (1u << 30) ? sc.epoch + 1 : 1u;
}

}  // namespace amg
