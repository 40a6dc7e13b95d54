// Generic launch skeletons of the solve phase: a CSR row kernel (L lanes per
// row, wave64 sub-groups) and an elementwise kernel, both with an optional
// fused reduction.  Reductions are deterministic: each block reduces in a
// fixed order and writes one partial per block; the partials are then summed
// in block order (by a one-block finalize kernel, or for grids of at most
// kTailBlocks blocks by the last block of the kernel itself) and handed to
// the operation's finalizer, which writes device scalars and flags.  Every operation carries an `active` flag read at
// kernel entry, so branches of the K-cycle and the outer iteration are
// decided on the device.
#pragma once
#include <atomic>

#include "amg_internal.hpp"
#include "device_utils.hpp"

namespace amg {

constexpr int kBlock = 256;

// Grids of at most kTailBlocks blocks finish their reduction in the kernel:
// the last block to arrive (a ticket counter) sums the partials in block
// order, exactly as k_finalize does, and runs the finalizer; larger grids use
// the separate finalize kernel.  The limit is set by the release fence each
// block needs before taking its ticket: at device scope it writes back the
// XCD's L2, which grows expensive when many blocks of a large kernel do it.
constexpr int kTailBlocks = 64;


template <int NV, class Op>
__device__ __forceinline__ void write_partials(double (&acc)[NV], RedCtx rc, const Op& op, bool tail) {
  static_assert(NV <= kMaxReduce, "the partials buffer holds kMaxReduce values per block");
  __shared__ double red[NV * (kBlock / kWave)];
  __shared__ int s_last;
  block_sum<NV>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) rc.part[k * gridDim.x + blockIdx.x] = acc[k];
  }
  if (!tail) return;
  if (threadIdx.x == 0) {
    __threadfence();   // the partial is visible before the ticket is taken
    s_last = atomicAdd(rc.ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const int nb = gridDim.x;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) t += rc.part[k * nb + b];
    v[k] = t;
  }
  block_sum<NV>(v, red);
  if (threadIdx.x == 0) {
    op.finalize(v);
    *rc.ticket = 0u;
  }
}

// The one-block finalize reads the partials with 1024 threads (2048 blocks x
// up to 3 values: a few loads per thread): on the 128^3 Poisson solve, 15
// finalizes per iteration, 9.51 -> 9.25 ms against 256 threads.
constexpr int kFinBlock = 1024;
template <class Op>
__global__ void __launch_bounds__(kFinBlock) k_finalize(Op op, const double* __restrict__ part, int nb) {
  if (!op.active()) return;
  constexpr int NV = Op::NV;
  __shared__ double red[NV * (kFinBlock / kWave)];
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kFinBlock) s += part[k * nb + b];
    v[k] = s;
  }
  block_sum<NV>(v, red);
  if (threadIdx.x == 0) op.finalize(v);
}

// y-side of a sparse row operation: Op provides
//   static constexpr int NV;           number of fused reductions
//   bool active() const;               kernel-wide enable
//   void idle() const;                 run by thread 0 of block 0 when inactive
//   T x(int j) const;                  the gathered operand
//   void row(int i, T ax, double* acc) the epilogue of row i
//   void finalize(const double* v)     totals of the reductions

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// The logical block index gives every XCD a contiguous run of blocks, and
// each logical block a contiguous chunk of the work, so the neighbouring rows
// whose x entries overlap share one L2.
__device__ __forceinline__ int xcd_logical_block() {
  const int g = gridDim.x, b = blockIdx.x;
  if (g < 8 || (g & 7)) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

// Schedules of the slice kernels, whose unit of work is a step of 4 slices
// (one per wave of a block).  sched:
//    0   contiguous: each logical block a run of ceil(steps / grid) steps;
//   > 0  plane-ordered over planes of sched steps (a grid plane of rows, the
//        largest column offset of the level; steps a multiple of it): logical
//        step u of that run executes step (u % planes) * sched + u / planes,
//        so a block walks the same rows plane after plane and finds what it
//        gathers from the next plane in the cache;
//   -1   XCD sweep: each XCD a contiguous eighth of the steps, which its B
//        blocks take together (its block j: steps j, j + B, j + 2B, ... of
//        that eighth), so what the XCD reads at a time is one run of
//        adjacent rows and their neighbours (grids that are not a multiple
//        of 8: block j takes steps j, j + grid, ...).
struct Steps {
  int u, end, inc, planes, pstep;
  __device__ int step() const { return pstep > 0 ? (u % planes) * pstep + u / planes : u; }
};

__device__ __forceinline__ Steps block_steps(int steps, int sched) {
  Steps r;
  r.inc = 1;
  r.pstep = sched > 0 ? sched : 0;
  r.planes = sched > 0 ? steps / sched : 1;
  const int g = gridDim.x;
  if (sched == -1) {
    if (g >= 8 && !(g & 7)) {
      const int per8 = (steps + 7) / 8, x = blockIdx.x & 7;
      r.u = x * per8 + (blockIdx.x >> 3);
      r.end = min(steps, (x + 1) * per8);
      r.inc = g >> 3;
    } else {
      r.u = blockIdx.x;
      r.end = steps;
      r.inc = g;
    }
    return r;
  }
  const int per = (steps + g - 1) / g;
  r.u = xcd_logical_block() * per;
  r.end = min(steps, r.u + per);
  return r;
}

// D16: the columns come as 16-bit offsets col - row (Level::ci16).
template <typename T, int LPR, class Op, bool D16 = false>
__global__ void __launch_bounds__(kBlock) k_rows(int n, const int* __restrict__ rp,
                                                 const void* __restrict__ cols,
                                                 const T* __restrict__ av, Op op, RedCtx rc) {
  if (!op.active()) {
    if (blockIdx.x == 0 && threadIdx.x == 0) op.idle();
    return;
  }
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  double acc[Op::NV > 0 ? Op::NV : 1];
#pragma unroll
  for (int k = 0; k < (Op::NV > 0 ? Op::NV : 1); ++k) acc[k] = 0.0;
  const int groups = (n + RPB - 1) / RPB;
  const int per = (groups + gridDim.x - 1) / gridDim.x;
  const int g0 = xcd_logical_block() * per;
  const int g1 = min(groups, g0 + per);
  for (int g = g0; g < g1; ++g) {
    const int row = g * RPB + threadIdx.x / LPR;
    T sum = T(0);
    if (row < n) {
      const int s = rp[row], e = rp[row + 1];
      // a lane's entries four at a time: the column and value loads, then the
      // gathers, then the products in entry order (the same sum as one entry
      // at a time), so four gathers are in flight instead of one
      for (int k0 = s + lane; k0 < e; k0 += 4 * LPR) {
        int c[4];
        T v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = k0 + q * LPR;
          if constexpr (D16) c[q] = k < e ? row + (int)static_cast<const int16_t*>(cols)[k] : 0;
          else c[q] = k < e ? static_cast<const int*>(cols)[k] : 0;
          v[q] = k < e ? av[k] : T(0);
        }
        T xv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) xv[q] = k0 + q * LPR < e ? op.x(c[q]) : T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k0 + q * LPR < e) sum += v[q] * xv[q];
      }
    }
    sum = group_sum<LPR>(sum);
    if (row < n && lane == 0) op.row(row, sum, acc);
  }
  if constexpr (Op::NV > 0) write_partials<Op::NV>(acc, rc, op, rc.ticket != nullptr);
}

// Sliced ELL with slices of H rows (H = 64, 32 or 16): slice s holds the rows
// of slots s*H .. s*H + H - 1 column-major, element (slot s*H + l, k) at
// sl_ptr[s] + H k + l, padded with zero values that point at the row itself.
// Slot i holds row perm[i] (perm null: row i); the copies in shorter slices
// order the rows of each 256-row window by decreasing length, so a slice's
// rows are of nearly equal length and the padding small.  One wave per slice
// and G = 64/H lanes per row: lane j*H + l takes entries j, j + G, ... of the
// row in slot l, so every value and column load of a wave is one contiguous
// run of 64 elements; the G partial sums are added by lane exchange (lane xor
// H, 2H, ...).
// D16: the columns come as 16-bit offsets col - row (128 bytes per wave and
// entry instead of 256), for levels whose couplings all lie within 32767
// rows, as on the lexicographically ordered grids.
// pstep: the schedule of the block steps (block_steps).
template <typename T, class Op, bool D16, int H = kWave>
__global__ void __launch_bounds__(kBlock) k_sell(int n, int nslices, const int* __restrict__ sl_ptr,
                                                 const void* __restrict__ sl_cols, const T* __restrict__ sl_val,
                                                 const int* __restrict__ perm, Op op, RedCtx rc, int pstep) {
  static_assert(H == 64 || H == 32 || H == 16, "slice height");
  constexpr int G = kWave / H;   // lanes per row
  if (!op.active()) {
    if (blockIdx.x == 0 && threadIdx.x == 0) op.idle();
    return;
  }
  double acc[Op::NV > 0 ? Op::NV : 1];
#pragma unroll
  for (int k = 0; k < (Op::NV > 0 ? Op::NV : 1); ++k) acc[k] = 0.0;
  constexpr int SPB = kBlock / kWave;   // slices per block step
  const int lane = threadIdx.x & (kWave - 1);
  const int j = lane / H;               // this lane's entries: j, j + G, j + 2G, ...
  const int wv = threadIdx.x / kWave;
  const int steps = (nslices + SPB - 1) / SPB;
  for (Steps st = block_steps(steps, pstep); st.u < st.end; st.u += st.inc) {
    const int sl = st.step() * SPB + wv;
    if (sl >= nslices) continue;
    const int slot = sl * H + (lane & (H - 1));
    const int row = perm ? perm[slot] : slot;
    const int base = __builtin_amdgcn_readfirstlane(sl_ptr[sl]);   // wave-uniform
    const int w = (__builtin_amdgcn_readfirstlane(sl_ptr[sl + 1]) - base) / H;
    T sum = T(0);
    const int* cp = static_cast<const int*>(sl_cols) + base + lane;
    const int16_t* dp = static_cast<const int16_t*>(sl_cols) + base + lane;
    const T* vp = sl_val + base + lane;
    // chunks of 8 entries per lane: all column and value loads of a chunk,
    // then all gathers, then the FMAs in entry order, so a chunk costs one
    // round trip.  Entry k0 + G q + j of the row sits at H k0 + 64 q + lane.
    for (int k0 = 0; k0 < w; k0 += 8 * G) {
      int c[8];
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const bool in = k0 + G * q + j < w;
        const int off = H * k0 + kWave * q;
        if constexpr (D16) c[q] = in ? row + (int)dp[off] : 0;
        else c[q] = in ? cp[off] : 0;
        // the values stream through once per pass: non-temporal loads keep
        // them from displacing what the next kernels reuse from the caches
        // (the coarse levels' data in the Infinity Cache); 128^3 Poisson
        // solve 9.20 -> 8.92 ms
        v[q] = in ? __builtin_nontemporal_load(vp + off) : T(0);
      }
      T xv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) xv[q] = k0 + G * q + j < w ? op.x(c[q]) : T(0);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + G * q + j < w) sum += v[q] * xv[q];
    }
    if constexpr (G > 1) {
#pragma unroll
      for (int o = H; o < kWave; o <<= 1) sum += __shfl_xor(sum, o, kWave);
    }
    if (row < n && j == 0) op.row(row, sum, acc);
  }
  if constexpr (Op::NV > 0) write_partials<Op::NV>(acc, rc, op, rc.ticket != nullptr);
}

// Sliced diagonals: slices of 64 rows (one wave), each with its own short
// list of diagonal offsets d (col = row + d, ascending): slice s holds
// offsets dg_off[dg_ptr[s] .. dg_ptr[s+1]) and, for the q-th of them, the
// value of row s*64 + l at (dg_ptr[s] + q) * 64 + l (zero where the row has no
// entry on that diagonal).  No column is stored: the offset is one scalar per
// wave and diagonal, so a level from a structured grid moves 8 bytes per entry
// (4 in FP32) plus the vectors.  pstep: the schedule (block_steps).
template <typename T, class Op>
__global__ void __launch_bounds__(kBlock) k_sdia(int n, int nslices, const int* __restrict__ dg_ptr,
                                                 const int* __restrict__ dg_off, const T* __restrict__ dg_val,
                                                 Op op, RedCtx rc, int pstep) {
  if (!op.active()) {
    if (blockIdx.x == 0 && threadIdx.x == 0) op.idle();
    return;
  }
  double acc[Op::NV > 0 ? Op::NV : 1];
#pragma unroll
  for (int k = 0; k < (Op::NV > 0 ? Op::NV : 1); ++k) acc[k] = 0.0;
  constexpr int SPB = kBlock / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int steps = (nslices + SPB - 1) / SPB;
  for (Steps st = block_steps(steps, pstep); st.u < st.end; st.u += st.inc) {
    const int sl = st.step() * SPB + wv;
    if (sl >= nslices) continue;
    const int row = sl * kWave + lane;
    // wave-uniform: the offsets come by scalar loads and the entry loop needs
    // no lane masks (so no wait between the loads of a chunk)
    const int base = __builtin_amdgcn_readfirstlane(dg_ptr[sl]);
    const int w = __builtin_amdgcn_readfirstlane(dg_ptr[sl + 1]) - base;
    const T* vp = dg_val + (size_t)base * kWave + lane;
    T sum = T(0);
    for (int k0 = 0; k0 < w; k0 += 8) {
      int c[8];
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        // the chunk's offsets unconditionally (scalar loads; slots past the
        // slice repeat its last offset); padding may point past either end
        // of the rows: clamp (its value is zero)
        const int col = row + dg_off[base + min(k0 + q, w - 1)];
        c[q] = col < 0 ? 0 : (col >= n ? n - 1 : col);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = k0 + q < w ? __builtin_nontemporal_load(vp + (size_t)(k0 + q) * kWave) : T(0);
      T xv[8];   // padding slots gather their slice's last column again (a cache hit)
#pragma unroll
      for (int q = 0; q < 8; ++q) xv[q] = op.x(c[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q < w) sum += v[q] * xv[q];
    }
    if (row < n) op.row(row, sum, acc);
  }
  if constexpr (Op::NV > 0) write_partials<Op::NV>(acc, rc, op, rc.ticket != nullptr);
}

// Elementwise operation over [0, n): Op provides NV, active(), idle(),
// elem(int i, double* acc), finalize(const double*).
template <class Op>
__global__ void __launch_bounds__(kBlock) k_elem(int n, Op op, RedCtx rc) {
  if (!op.active()) {
    if (blockIdx.x == 0 && threadIdx.x == 0) op.idle();
    return;
  }
  double acc[Op::NV > 0 ? Op::NV : 1];
#pragma unroll
  for (int k = 0; k < (Op::NV > 0 ? Op::NV : 1); ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) op.elem(i, acc);
  if constexpr (Op::NV > 0) write_partials<Op::NV>(acc, rc, op, rc.ticket != nullptr);
}

// Grid of the row kernels: one block per 256-row (or RPB-row) group up to a
// cap of 2048 resident blocks (8 per CU); a multiple of 8 above 8 blocks so
// that the XCD-aware mapping is a bijection.
inline int rows_grid(int n, int lpr, bool reduce) {
  (void)reduce;
  long rpb = kBlock / lpr;
  long g = (n + rpb - 1) / rpb;
  const long cap = kMaxPartialBlocks;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  if (g > 8) g &= ~7L;
  return (int)g;
}

inline int elem_grid(int n, bool reduce) {
  long g = ((long)n + kBlock - 1) / kBlock;
  long cap = reduce ? kMaxPartialBlocks : 65536;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

// Blocks of kernel k that the device holds at once, at most
// kMaxPartialBlocks: a slice kernel gives each block a fixed share of the
// steps, so a grid larger than what is resident would run its last blocks
// in a second, mostly empty round (kernels whose registers allow fewer than
// 8 blocks of 256 threads per CU).  Per kernel instance, taken once (host
// threads that race on the first launch compute the same value).
template <class K>
int resident_blocks(K k) {
  static std::atomic<int> cached{0};
  int g = cached.load(std::memory_order_relaxed);
  if (g == 0) {
    int per = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kBlock, 0) != hipSuccess || per < 1) per = 8;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    const long r = (long)per * cus;
    g = (int)(r < kMaxPartialBlocks ? r : kMaxPartialBlocks);
    cached.store(g, std::memory_order_relaxed);
  }
  return g;
}

template <typename T, int LPR, class Op, bool D16 = false>
void launch_rows_l(int n, const int* rp, const void* ci, const T* av, const Op& op, RedCtx rc, hipStream_t s) {
  int g = rows_grid(n, LPR, Op::NV > 0);
  const int cap = resident_blocks(k_rows<T, LPR, Op, D16>);
  if (g > cap) g = cap > 8 ? cap & ~7 : cap;
  const bool tail = Op::NV > 0 && g <= kTailBlocks && rc.ticket != nullptr;
  const RedCtx r2{rc.part, tail ? rc.ticket : nullptr};
  k_rows<T, LPR, Op, D16><<<g, kBlock, 0, s>>>(n, rp, ci, av, op, r2);
  if constexpr (Op::NV > 0)
    if (!tail) k_finalize<Op><<<1, kFinBlock, 0, s>>>(op, rc.part, g);
}

template <typename T, class Op>
void launch_rows(int n, int lpr, const int* rp, const int* ci, const T* av, const Op& op, RedCtx rc,
                 hipStream_t s) {
  switch (lpr) {
    case 1: launch_rows_l<T, 1>(n, rp, ci, av, op, rc, s); break;
    case 2: launch_rows_l<T, 2>(n, rp, ci, av, op, rc, s); break;
    case 4: launch_rows_l<T, 4>(n, rp, ci, av, op, rc, s); break;
    case 8: launch_rows_l<T, 8>(n, rp, ci, av, op, rc, s); break;
    case 16: launch_rows_l<T, 16>(n, rp, ci, av, op, rc, s); break;
    case 32: launch_rows_l<T, 32>(n, rp, ci, av, op, rc, s); break;
    default: launch_rows_l<T, 64>(n, rp, ci, av, op, rc, s); break;
  }
}

// The same with the columns as 16-bit offsets (2 to 32 lanes per row).
template <typename T, class Op>
void launch_rows16(int n, int lpr, const int* rp, const int16_t* ci16, const T* av, const Op& op, RedCtx rc,
                   hipStream_t s) {
  switch (lpr) {
    case 2: launch_rows_l<T, 2, Op, true>(n, rp, ci16, av, op, rc, s); break;
    case 4: launch_rows_l<T, 4, Op, true>(n, rp, ci16, av, op, rc, s); break;
    case 8: launch_rows_l<T, 8, Op, true>(n, rp, ci16, av, op, rc, s); break;
    case 16: launch_rows_l<T, 16, Op, true>(n, rp, ci16, av, op, rc, s); break;
    default: launch_rows_l<T, 32, Op, true>(n, rp, ci16, av, op, rc, s); break;
  }
}


// Grid of a slice kernel over `steps` steps: one block per step up to the
// resident cap, a multiple of 8 above 8 blocks (the XCD mapping).
inline int step_grid(int steps, int resident) {
  long g = steps;
  if (g < 1) g = 1;
  if (g > resident) g = resident;
  if (g > 8) g &= ~7L;
  return (int)g;
}

// sl_dcol non-null: the kernel reads the 16-bit column offsets instead of sl_col.


template <typename T, class Op, bool D16, int H>
void launch_sell_h(int n, int nslices, const int* sl_ptr, const void* cols, const T* sl_val, const int* perm,
                   const Op& op, RedCtx rc, hipStream_t s, int pstep) {
  const int g = step_grid((nslices + kBlock / kWave - 1) / (kBlock / kWave), resident_blocks(k_sell<T, Op, D16, H>));
  const bool tail = Op::NV > 0 && g <= kTailBlocks && rc.ticket != nullptr;
  const RedCtx r2{rc.part, tail ? rc.ticket : nullptr};
  k_sell<T, Op, D16, H><<<g, kBlock, 0, s>>>(n, nslices, sl_ptr, cols, sl_val, perm, op, r2, pstep);
  if constexpr (Op::NV > 0)
    if (!tail) k_finalize<Op><<<1, kFinBlock, 0, s>>>(op, rc.part, g);
}

// slice_h: the slice height of the copy (64, 32 or 16 rows); perm: its row
// order (null: rows in order)
template <typename T, class Op>
void launch_sell(int n, int nslices, const int* sl_ptr, const int* sl_col, const T* sl_val, const Op& op,
                 RedCtx rc, hipStream_t s, const int16_t* sl_dcol = nullptr, int pstep = 0, int slice_h = kWave,
                 const int* perm = nullptr) {
  if (slice_h != kWave) pstep = 0;
  const void* cols = sl_dcol ? static_cast<const void*>(sl_dcol) : static_cast<const void*>(sl_col);
  if (sl_dcol) {
    if (slice_h == 32) launch_sell_h<T, Op, true, 32>(n, nslices, sl_ptr, cols, sl_val, perm, op, rc, s, pstep);
    else if (slice_h == 16) launch_sell_h<T, Op, true, 16>(n, nslices, sl_ptr, cols, sl_val, perm, op, rc, s, pstep);
    else launch_sell_h<T, Op, true, 64>(n, nslices, sl_ptr, cols, sl_val, perm, op, rc, s, pstep);
  } else {
    if (slice_h == 32) launch_sell_h<T, Op, false, 32>(n, nslices, sl_ptr, cols, sl_val, perm, op, rc, s, pstep);
    else if (slice_h == 16) launch_sell_h<T, Op, false, 16>(n, nslices, sl_ptr, cols, sl_val, perm, op, rc, s, pstep);
    else launch_sell_h<T, Op, false, 64>(n, nslices, sl_ptr, cols, sl_val, perm, op, rc, s, pstep);
  }
}

template <typename T, class Op>
void launch_sdia(int n, int nslices, const int* dg_ptr, const int* dg_off, const T* dg_val, const Op& op,
                 RedCtx rc, hipStream_t s, int pstep = 0) {
  const int g = step_grid((nslices + kBlock / kWave - 1) / (kBlock / kWave), resident_blocks(k_sdia<T, Op>));
  const bool tail = Op::NV > 0 && g <= kTailBlocks && rc.ticket != nullptr;
  const RedCtx r2{rc.part, tail ? rc.ticket : nullptr};
  k_sdia<T, Op><<<g, kBlock, 0, s>>>(n, nslices, dg_ptr, dg_off, dg_val, op, r2, pstep);
  if constexpr (Op::NV > 0)
    if (!tail) k_finalize<Op><<<1, kFinBlock, 0, s>>>(op, rc.part, (int)g);
}

template <class Op>
void launch_elem(int n, const Op& op, RedCtx rc, hipStream_t s) {
  const int g = elem_grid(n, Op::NV > 0);
  const bool tail = Op::NV > 0 && g <= kTailBlocks && rc.ticket != nullptr;
  k_elem<Op><<<g, kBlock, 0, s>>>(n, op, RedCtx{rc.part, tail ? rc.ticket : nullptr});
  if constexpr (Op::NV > 0)
    if (!tail) k_finalize<Op><<<1, kFinBlock, 0, s>>>(op, rc.part, g);
}

inline int pick_lpr(int n, int nnz) {
  double avg = n > 0 ? (double)nnz / n : 1.0;
  int l = 1;
  while (l < avg && l < 64) l <<= 1;
  return l < 2 ? 2 : l;
}

}  // namespace amg
