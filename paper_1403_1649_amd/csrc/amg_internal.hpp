// Internal host-side declarations of the aggregation-AMG library: status
// handling, the device arena, the level / hierarchy records and the kernel
// launchers implemented in the .hip translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/amg.h"

namespace amg {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define AMG_HIP(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::amg::Error(AMG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device error bits raised by kernels (atomic OR into one int per hierarchy).
enum : int {
  kErrZeroDiag = 1,
  kErrNonSymPattern = 2,
  kErrNonFinite = 4,
  kErrCountOverflow = 8,
  kErrUnassigned = 16,
  kErrSingular = 32,
  kErrBreakdown = 64,
  kErrBadColumn = 128,
  kErrCrossSystem = 256,
  kErrNotSPD = 512,
  kErrColors = 1024,
  kErrTimeout = 2048,   // a bounded wait of a persistent launch ran out
};

// ---------------------------------------------------------------- memory
// Device memory for one hierarchy: large chunks, bump-allocated with 256-byte
// alignment, returned to a process-wide cache on destruction so that repeated
// setups do not pay hipMalloc again.
class Arena {
 public:
  Arena() = default;
  ~Arena();
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  void reserve(size_t bytes);
  void* alloc(size_t bytes);
  template <typename T>
  T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
  size_t used() const { return used_; }

 private:
  struct Chunk { char* base; size_t size; size_t off; };
  std::vector<Chunk> chunks_;
  size_t used_ = 0;
};

// Scratch of the single-pass device scan: one status word per tile, then the
// 64-bit ticket counter (zero between calls); the call epoch.
struct ScanCtx {
  uint64_t* status = nullptr;
  unsigned long long* ticket = nullptr;
  int max_blocks = 0;
  uint32_t epoch = 1;
};

// ---------------------------------------------------------------- records
struct TermInfo;

struct Level {
  // A_k (float64, device); val32 is the float32 copy used by the mixed cycle
  int n = 0, nnz = 0;
  int* rp = nullptr;
  int* ci = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
  double* diag = nullptr;      // a_ii
  double* B = nullptr;         // near null space vector B_k
  int lpr = 8;                 // lanes per row picked from the average row length
  // sliced ELL copy for the solve (slices of 64 rows, column-major per slice)
  int nslices = 0;
  int* sl_ptr = nullptr;       // element offset of each slice (nslices + 1)
  int* sl_col = nullptr;
  // the same columns as 16-bit offsets col - row, when every offset of the
  // level fits (null otherwise); sl_wide is the device flag the fill raises
  // when one does not
  int16_t* sl_dcol = nullptr;
  int* sl_wide = nullptr;
  double* sl_val = nullptr;
  float* sl_val32 = nullptr;
  long sl_total = 0;           // stored sliced-ELL elements (64 x the longest row, summed over slices)
  // a second sliced-ELL copy in shorter slices (h = 32 or 16 rows, 64/h lanes
  // per row) over rows ordered by length within 256-row windows, built for
  // the autotuner on levels whose rows vary in length and kept while it is
  // the chosen kernel; its memory is held by sh_mem
  struct ShortSell {
    int h = 0, nslices = 0;
    long total = 0;
    int* perm = nullptr;       // slot -> row: each 256-row window by decreasing row length
    int* ptr = nullptr;
    int* col = nullptr;
    int16_t* dcol = nullptr;
    double* val = nullptr;
    float* val32 = nullptr;
  } sh;
  std::shared_ptr<Arena> sh_mem;
  // sliced diagonals (levels from structured grids): per 64-row slice its
  // diagonal offsets and their values, no columns; built for the autotuner
  // where every slice has few diagonals, kept while it is the chosen kernel
  struct Sdia {
    int nslices = 0;
    long total = 0;              // diagonals over all slices
    int* ptr = nullptr;          // first diagonal of each slice (nslices + 1)
    int* off = nullptr;          // offsets col - row
    double* val = nullptr;       // [total][64]
    float* val32 = nullptr;
  } dia;
  std::shared_ptr<Arena> dia_mem;
  // the CSR columns as 16-bit offsets col - row (2 bytes per entry instead of
  // 4), for the row kernels on levels whose offsets all fit (those with the
  // 16-bit sliced ELL); built for the autotuner, kept while it is chosen
  int16_t* ci16 = nullptr;
  std::shared_ptr<Arena> ci16_mem;
  // kernel choice per arithmetic type (autotuned): fmt 0 = CSR with lpr lanes
  // per row, fmt 1 = sliced ELL, fmt 2 = sliced ELL with 16-bit column offsets,
  // fmt 3 = sliced diagonals, fmt 4 = CSR with 16-bit column offsets
  // pz: schedule of the slice kernels (0 contiguous, -1 XCD sweep, > 0
  // plane-ordered over that many steps)
  // tile: columns per pass of the block kernels (several right-hand sides)
  // sh: slice height of the sliced-ELL copy used (0 = the 64-row copy)
  struct Tune { int fmt = 0; int lpr = 8; float us = 0.f; int pz = 0; int tile = 0; int sh = 0; } t64, t32;
  // setup products (absent on the coarsest level)
  uint8_t* strong = nullptr;   // strength mask C over A_k's pattern
  uint64_t* tuple = nullptr;   // final MIS(2) tuples (state in the top two bits)
  int mis_rounds = 0;
  int nc = 0;                  // n_{k+1}
  int* agg = nullptr;          // aggregate index per fine node
  int* agg_ptr = nullptr;      // aggregate segments: rows of aggregate I are
  int* agg_rows = nullptr;     //   agg_rows[agg_ptr[I] .. agg_ptr[I+1]) ascending
  double* pval = nullptr;      // the single nonzero of row i of P_k
  float* pval32 = nullptr;
  // R_k = P_k^T in CSR: row I = aggregate I, columns agg_rows[agg_ptr[I] ..],
  // values rval[k] = pval[agg_rows[k]] (nr = rows that belong to an aggregate)
  double* rval = nullptr;
  float* rval32 = nullptr;
  int nr = 0;
  int rlpr = 8;                // lanes per aggregate of the restriction kernel
  double omega = 0.0, rho = 0.0;
  double* wdinv = nullptr;     // omega / a_ii (or omega_i / a_ii with learned weights)
  int learned = 0;             // learned weights in use on this level
  double loss_plain = 0.0, loss_learned = 0.0;
  float* wdinv32 = nullptr;
  // solve scratch (typed by the cycle precision; size n or n_{k+1})
  void* r = nullptr;           // fine residual
  void* xt = nullptr;          // fine iterate inside the cycle
  void* rc = nullptr;          // restricted residual
  void* c = nullptr;           // first inner correction (or the V-cycle correction)
  void* v = nullptr;           // A_{k+1} c
  void* rt = nullptr;          // r~
  void* d = nullptr;           // second inner correction
  void* w = nullptr;           // A_{k+1} d
  // batched systems (block-diagonal A_0): system s owns rows
  // [sys_off[s], sys_off[s+1]) of this level, an empty range once a finer
  // level was its coarsest
  std::vector<int> sys_off;    // host copy
  int* d_sys_off = nullptr;
  int* blk = nullptr;          // block table: (system, row0, row1) per block; system -1 pads
  int nblk = 0;                // table entries (a multiple of 8 above 8)
  int* blk_sys = nullptr;      // blocks of system s: [blk_sys[s], blk_sys[s+1])
  int* sl_base = nullptr;      // sliced ELL of a batch: first slice of each system
  int bsell = 0;               // batch level uses its sliced-ELL copy
  int* kv = nullptr;           // per system: the K-cycle applies on this level
  int kcyc = 0;                // some system takes the K-cycle on this level
  std::vector<int> term;       // systems whose coarsest level this is
  TermInfo* d_term = nullptr;
  int* tblk = nullptr;         // coarse GEMV blocks: (terminal index, first local row)
  int ntblk = 0;
  double* tinv = nullptr;      // row-major dense inverses of the terminal systems
  float* tinv32 = nullptr;
  std::vector<double> sys_omega, sys_rho;
  // Chebyshev smoother: device coefficients [1/theta, (c1, c2) per later
  // step] and its vectors (cycle precision, size n): residual, two directions
  double* cheb = nullptr;
  double cheb_host[16] = {};
  void* cr = nullptr;
  void* cd0 = nullptr;
  void* cd1 = nullptr;
  // multi-colour Gauss-Seidel smoother: colour of every row and the rows of
  // colour c at crow[coff[c] .. coff[c+1]) (coff on the host)
  int* colors = nullptr;
  int* crow = nullptr;
  std::vector<int> coff;
  // numeric re-setup (built by the first amg_resetup): the terms of every
  // entry c of A_{k+1} in segment order at rs_tptr[c] .. rs_tptr[c+1]: fine
  // entry rs_f[t] of fine row rs_i[t]
  int* rs_tptr = nullptr;
  int* rs_f = nullptr;
  int* rs_i = nullptr;
};

// A system whose coarsest level is a given level: its rows there and the
// offset of its dense inverse (n x n, row-major) in the level's inverse block.
struct TermInfo {
  int sys, row0, n, pad;
  long long off;
};

struct Hierarchy {
  amg_options opt{};
  std::vector<Level> levels;
  Arena arena;
  hipStream_t stream = nullptr;
  int dim_hint = 3;
  // coarsest level: explicit inverse (row-major n_L x n_L)
  double* cinv = nullptr;
  float* cinv32 = nullptr;
  // device control block
  int* d_err = nullptr;        // error bits
  int* d_ctl = nullptr;        // integer control words (flags, counters)
  double* d_sc = nullptr;      // scalar slots (dots, coefficients)
  double* d_part = nullptr;    // per-block partial sums of reductions
  unsigned* d_ticket = nullptr;// last-block tickets
  unsigned* d_tail = nullptr;  // counters of the one-launch V-cycle tail (zero between launches)
  ScanCtx scan;                // look-back words of device scans
  int* d_mis = nullptr;        // MIS(2) round counters (kMisWords ints)
  // pinned host mirror for read-backs
  void* h_pinned = nullptr;
  // outer solve vectors (float64, size n_0)
  double *r = nullptr, *p = nullptr, *q = nullptr;
  void* z = nullptr;           // preconditioned residual (cycle precision)
  void* bz = nullptr;          // cycle right-hand side in cycle precision (mixed mode)
  double* xint = nullptr;      // iterate of the outer solve (copied to the caller's x at exit)
  float* mlp_w = nullptr;      // device copy of the learned-weight parameters
  // captured launch sequences of one outer iteration (one segment, or two
  // around the probed kernel, which is then launched from the host between
  // them) and of the (re)start
  std::vector<hipGraphExec_t> g_iter;
  hipGraphExec_t g_restart = nullptr;
  std::function<void(hipStream_t)> probe_fn;
  hipStream_t cap_stream = nullptr;
  bool capturing = false;      // inside any stream capture
  bool split_at_probe = false; // capturing the outer iteration with a probe
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t pev[2] = {nullptr, nullptr};   // around the probed kernel
  double probe_ms = 0.0;
  int probe_samples = 0;
  float setup_ms = 0.f, solve_ms = 0.f, resetup_ms = 0.f;
  double tune_ms = 0.0, capture_ms = 0.0;   // host time of the autotuner and of the graph capture in setup
  // learned weights judged by probe solves: kept?, iterations and true
  // relative residuals with the plain weights and with the learned ones
  int judge_kept = -1, judge_it_plain = 0, judge_it_learned = 0;
  double judge_rel_plain = 0.0, judge_rel_learned = 0.0;
  // batched systems: count (0 = one system), per-system control of the solve
  // and the results of the last solve
  int nsys = 0;
  double* b_sc = nullptr;      // per-system scalar slots [slot][nsys]
  int* b_fl = nullptr;         // per-system flags [word][nsys]
  int* b_any = nullptr;        // flags over all systems
  double* b_part = nullptr;    // block partials (3 per block of the largest table)
  int* b_again = nullptr;      // systems restarted from their true residual
  std::vector<int> b_iters;
  std::vector<double> b_relres;
  // several right-hand sides: the block workspace and the captured block
  // iteration of the last amg_solve_multi, kept for the next call with the
  // same number of columns (solver_multi.hip)
  std::shared_ptr<void> multi;
  bool mixed() const { return opt.precision == AMG_PREC_MIXED; }
  int L() const { return (int)levels.size() - 1; }
  ~Hierarchy();
};

// Slots of the device control block.
enum CtlWord : int {
  kCtlRunning = 0,     // outer iteration active
  kCtlIters = 1,       // outer iterations performed
  kCtlOne = 5,         // constant 1 (an always-active flag)
  kCtlAggFill = 6,     // scratch counters of the Galerkin tiers (two words)
  kCtlKFlags = 16,     // per level k: [16 + 4k] step-2 flag, [17 + 4k] use-d flag
  kCtlWords = 128,
};
enum ScSlot : int {
  kScBB = 0, kScRtol2 = 1, kScAlpha = 2, kScBeta = 3, kScPQ = 4, kScRR = 5,
  kScTrue = 6, kScArn = 8,     // Arnoldi: [8 .. 8+64)
  kScK = 80,                   // per level k: 16 slots from 80 + 16k
  kScWords = 80 + 16 * 24,
};
enum KSlot : int {
  kKRho1 = 0, kKAlpha1 = 1, kKRcRc = 2, kKRtRt = 3, kKGamma = 4, kKBeta = 5,
  kKAlpha2 = 6, kKCoefC = 7, kKCoefD = 8,
};
constexpr int kMaxPartialBlocks = 2048;
constexpr int kMaxReduce = 8;        // values one reduction may carry (partials: kMaxReduce x blocks)
constexpr int kArnMax = 5;           // Arnoldi steps at most (amg_options.arnoldi_m)
static_assert(1 + kArnMax <= kMaxReduce, "an Arnoldi step's norm and projections in one reduction");
// pinned host mirror: ints 0..63 for control read-backs, then (in doubles
// from kPinnedArn) the Arnoldi results
constexpr int kPinnedArn = 64;
constexpr size_t kPinnedBytes = (kPinnedArn + 64) * sizeof(double);
constexpr int kBlockRowsGemv = 4;   // rows per 256-thread block of a dense GEMV (one wave per row)

// ---------------------------------------------------------------- launchers
// scan.hip
void init_scan(ScanCtx& sc, Arena& arena, int nmax, hipStream_t s);
void scan_to_ptr(const int* counts, int* ptr, int n, ScanCtx& sc, hipStream_t s);
int scan_blocks_needed(int n);

// setup_kernels.hip
void launch_check_rowptr(int n, const int* rp, int* err, hipStream_t s);
void launch_check_index(int n, const int* idx, int limit, int* err, hipStream_t s);
void launch_check_matrix(int n, const int* rp, const int* ci, const double* val, int* err, hipStream_t s);
// Up to 8 device ints copied to host pinned slots (0..62) by one launch,
// together with the error word (slot 63).
struct Mailbox {
  const int* src[8];
  int slot[8];
  int count[8];    // the slot receives the sum of count ints at this stride
  int stride[8];
  int n;
};
void launch_mailbox(const Mailbox& m, const int* err, int* host, hipStream_t s);
// Lanes per row of the row-group setup kernels: about four entries per lane,
// more on small levels so that a launch still covers the chip.
int group_lanes(int n, long entries);
void launch_strength(int n, int nnz, const int* rp, const int* ci, const double* val, double alpha,
                     uint8_t* strong, double* diag, hipStream_t s);
void launch_graph_count(int n, int nnz, const int* rp, const int* ci, const uint8_t* strong,
                        uint8_t* gmask, int* gdeg, int* cnt, int* err, hipStream_t s);
void launch_graph_fill(int n, int nnz, const int* rp, const int* ci, const uint8_t* gmask,
                       const int* gptr, int* gcol, hipStream_t s);
void launch_mis_init(int n, const int* cnt, uint32_t seed, uint64_t* T, uint64_t* M1, int* mc, int* err,
                     hipStream_t s, const int* lbase = nullptr);
// MIS(2) round counters (int array of kMisWords, touched only by atomics):
// per round parity, 64 counters of blocks that left a node undecided, each
// in a 128-byte line of its own; then the number of rounds that found one.
constexpr int kMisSlots = 64;
__host__ __device__ constexpr int mis_word(int parity, int slot) { return (parity * kMisSlots + slot) * 32; }
constexpr int kMisRoundsWord = 2 * kMisSlots * 32;
constexpr int kMisWords = kMisRoundsWord + 32;
// one MIS(2) round (two sweeps; the second counts the blocks that left a node
// undecided, for the next round's early exit)
// late-round node list of MIS(2) (setup_kernels.hip): flags fnear[n], their
// scan pnear[n+1] (pnear[n] = the list's length, read by the sweeps) and the
// list near[n]
struct MisLists {
  int *fnear, *pnear, *near, *count;
};
void launch_mis_lists(int n, const int* gptr, const int* gcol, const uint64_t* T, const MisLists& ml,
                      ScanCtx& sc, hipStream_t s);
void launch_mis_round(int n, const int* gptr, const int* gcol, uint64_t* T, uint64_t* M1, int* mc, int round,
                      int lanes, hipStream_t s,
                      const MisLists* ml = nullptr);
// MIS(k), k > 2: one round of k sweeps (M1 as in MIS(2); Ma, Mb scratch), and
// the k-round nearest-root aggregation (choice, choice2 scratch)
void launch_misk_round(int n, const int* gptr, const int* gcol, uint64_t* T, uint64_t* M1, uint64_t* Ma,
                       uint64_t* Mb, int* mc, int round, int k, int lanes, hipStream_t s);
void launch_aggregate_k(int n, int nnzg, const int* gptr, const int* gcol, const uint64_t* T, const int* root_id,
                        int k, int* choice, int* choice2, int* agg, int* err, hipStream_t s);
void launch_root_flags(int n, const uint64_t* T, int* flags, hipStream_t s);
void launch_aggregate(int n, int nnzg, const int* gptr, const int* gcol, const uint64_t* T, const int* root_id,
                      int* choice, int* agg, int* err, hipStream_t s);
void launch_agg_count(int n, const int* agg, int* counts, hipStream_t s);
void launch_agg_scatter(int n, const int* agg, const int* agg_ptr, int* fill, int* agg_rows, hipStream_t s);
void launch_agg_sort(int nc, const int* agg_ptr, int* agg_rows, hipStream_t s);
void launch_interp(int n, int nc, const int* agg, const int* agg_ptr, const int* agg_rows,
                   const double* B, double* Bc, double* pval, hipStream_t s);
void launch_node_hash(int n, uint32_t stream, uint32_t* out, hipStream_t s);
void launch_jacobi_weights(int n, double omega, const double* diag, double* wdinv, float* wdinv32, hipStream_t s);
void launch_to_float(size_t n, const double* in, float* out, hipStream_t s);
void launch_state_from_tuple(int n, const uint64_t* T, int8_t* state, hipStream_t s);
void launch_fill_int(size_t n, int* p, int v, hipStream_t s);
void launch_fill_double(size_t n, double* p, double v, hipStream_t s);
void launch_gather_double(int m, const int* idx, const double* src, double* dst, hipStream_t s);
// sliced ELL in slices of slice_h = 64, 32 or 16 rows
// (perm: slot -> row, null for rows in order)
void launch_sell_widths(int n, const int* rp, int* widths, hipStream_t s, int slice_h = 64,
                        const int* perm = nullptr);
void launch_sell_fill(int n, int nslices, const int* rp, const int* ci, const double* val, const int* sl_ptr,
                      int* sl_col, int16_t* sl_dcol, int* wide, double* sl_val, float* sl_val32, hipStream_t s,
                      int slice_h = 64, const int* perm = nullptr);
// rows of each 256-row window by decreasing length; perm: ceil(n/256)*256 slots
void launch_window_order(int n, const int* rp, int* perm, hipStream_t s);
// sliced diagonals: per 64-row slice the number of distinct offsets (*over
// raised above cap), then offsets and values at dg_ptr
// ci16[k] = ci[k] - row for the entries of each row (offsets known to fit)
void launch_ci16(int n, const int* rp, const int* ci, int16_t* ci16, hipStream_t s);
void launch_sdia_count(int n, const int* rp, const int* ci, int cap, int* cnt, int* over, hipStream_t s);
void launch_sdia_fill(int n, const int* rp, const int* ci, const double* val, const int* dg_ptr, int* dg_off,
                      double* dg_val, float* dg_val32, hipStream_t s);

// galerkin.hip: scratch of one Galerkin product (n fine rows, nnz entries,
// nc coarse rows): lens[n], inv[n], toff[n+1], tkey[nnz], tval[nnz],
// ucount[nc], list[2 nc], ctl: two counters.
struct GalerkinScratch {
  int* lens;
  int* toff;
  int* tkey;
  double* tval;
  int* ucount;
  int* list;
  int* ctl;
};
void launch_galerkin_stage(const GalerkinScratch& g, int n, int nc, int nnz, const int* rp, const int* ci,
                           const double* val, const int* agg, const double* pval, const int* agg_ptr,
                           const int* agg_rows, ScanCtx& sc, hipStream_t s);
void launch_galerkin_finish(const GalerkinScratch& g, int nc, const int* agg_ptr, const int* rp_c, int* ci_c,
                            double* val_c, hipStream_t s);

// dense.hip
void launch_dense_inverse(int n, const int* rp, const int* ci, const double* val, double* work,
                          double* inv, float* inv32, int* sync, int* err, hipStream_t s);

// arnoldi / reductions (solve_kernels.hip)
// Reduction context of the solve-phase kernels: per-block partials and the
// arrival counter of the in-kernel finalize (zero between kernels).
struct RedCtx {
  double* part;       // kMaxPartialBlocks * kMaxReduce doubles
  unsigned* ticket;
};
void arnoldi_enqueue(Hierarchy& h, const Level& lv, int m, uint32_t stream, double* Q, double* w, double* sc,
                     RedCtx rc, double* host_out, hipStream_t s);
void arnoldi(Hierarchy& h, Level& lv, int m, uint32_t stream, double* Q, double* w, double* H_out,
             double* wnorm_out);

// cycle and outer solvers (solver.hip)
int solve_fcg_impl(Hierarchy& h, const double* b, double rtol, double* x, int* iters, double* relres);
void build_solve_graphs(Hierarchy& h);
void autotune_levels(Hierarchy& h);
// Autotuner cache, per process and (AMG_TUNE_CACHE) across processes: one
// decision per level shape, value size and column count.  rowstat: the
// level's sliced-ELL element count, which measures how uneven its rows are.
struct TuneKey {
  int n = 0, nnz = 0, bytes = 0, nrhs = 1;
  long rowstat = 0;
  bool operator<(const TuneKey& o) const;
};
bool tune_cache_get(const TuneKey& k, Level::Tune* t);
void tune_cache_put(const TuneKey& k, const Level::Tune& t);
int mlp_num_params();
void mlp_features(Hierarchy& h, const Level& lv, int level, float* F, double* beta);
void mlp_omega(Hierarchy& h, const Level& lv, const float* F, const double* beta, const float* wdev, double* omega,
               double* wdinv, float* wdinv32, double* sig);
double mlp_loss_grad(Hierarchy& h, Arena& tmp, const Level& lv, int level, const float* wdev, int S_rand,
                     uint32_t seed, const double* extra, int S_extra, const double* omega_fixed, float* grad,
                     int accumulate, bool raw_extra = false);
void mlp_adam(float* w, float* m, float* v, const float* g, int n, int step, float lr, float b1, float b2, float eps,
              hipStream_t s);
int solve_multi_impl(Hierarchy& h, int R, const double* B, double rtol, double* X, int* iters, double* relres);
int multi_tiles(const Hierarchy& h, int R, int* tiles, int cap, double* tune_ms);
// batch.hip: independent systems on the block diagonal
void batch_blocks(Hierarchy& h, Level& lv);
void batch_local_base(const Level& lv, int* lbase, hipStream_t s);
void batch_check_blocks(const Level& lv, int* err, hipStream_t s);
void batch_build_sell(Hierarchy& h, Arena& tmp, Level& lv);
void batch_gather(int m, const int* src, const int* idx, int* dst, hipStream_t s);
void batch_remap_agg(const Level& lv, const int* cont, const int* shift, int* agg, hipStream_t s);
void batch_arnoldi(Hierarchy& h, Level& lv, int m, uint32_t stream, const int* mask, double* Q, double* w,
                   double* H_out /* host [nsys][64] */);
void batch_jacobi_weights(const Level& lv, const double* omega_sys, double* wdinv, float* wdinv32,
                          hipStream_t s);
void batch_control(Hierarchy& h);
void build_batch_graphs(Hierarchy& h);
int solve_batch_impl(Hierarchy& h, const double* b, double rtol, double* x, int* iters, double* relres);
// dense.hip: inverses of the terminal systems of a level, one workgroup each
void launch_dense_inverse_batched(const Level& lv, int nterm, const TermInfo* d_term, const TermInfo* h_term,
                                  double* work, int* piv, double* inv, float* inv32, int* err, hipStream_t s);
void launch_dense_inverse_spd(int nterm, const TermInfo* d_term, const TermInfo* h_term, int nrows, const int* rp,
                              const int* ci, const double* val, double* inv, float* inv32, Arena& tmp, int* err,
                              hipStream_t s);
void build_batch_hierarchy(Hierarchy& h, const amg_csr& A, const int* sys_off);
void spmv_sell_level(Hierarchy& h, const Level& lv, const double* x, double* y, bool offsets16);
void level_spmv(const Hierarchy& h, int k, const double* x, double* y, hipStream_t s);
void coarse_corrected_errors(Hierarchy& h, int k, const double* E, int S, int cycles, double* out);
void launch_hash_vector(int n, uint32_t stream, double* q, hipStream_t s);
void spmv_sell_f64(Hierarchy& h, const amg_csr& A, const double* x, double* y, bool offsets16);
void spmv_f64(int n, int nnz, const int* rp, const int* ci, const double* val, const double* x, double* y,
              int lpr, hipStream_t s);
int pick_lanes_per_row(int n, int nnz);

// noalloc.hip: the Galerkin product with its scratch in a static device array;
// returns AMG_EINVAL (nnz_c set, col_c / val_c untouched) when cap < nnz_c.
int galerkin_noalloc(const amg_csr& A, const int* agg, const double* pval, int nc, int* row_ptr_c, int* col_c,
                     double* val_c, int cap, int* nnz_c, hipStream_t s);

// resetup.hip: numeric re-setup on a fixed pattern
void launch_rs_count(const Level& lv, const Level& lc, int* cnt, int* err, hipStream_t s);
void launch_rs_fill(const Level& lv, const Level& lc, int* cur, int* tf, int* ti, int* err, hipStream_t s);
void launch_rs_values(const Level& lv, Level& lc, hipStream_t s);
void launch_rs_diag(const Level& lv, hipStream_t s);
void launch_rs_sell_values(const Level& lv, hipStream_t s);
// the short-slice copy of a level, when it pays (slice_h = 0) or in slices of
// slice_h = 32 or 16 rows (hierarchy.cpp)
void build_short_sell(Hierarchy& h, Level& lv, int slice_h);
// the sliced-diagonal copy of a level, when its slices have few diagonals
void build_sdia(Hierarchy& h, Level& lv);
void launch_set16(double* dst, const double* host16, hipStream_t s);
// coloring.hip: first-fit colouring by node-hash priority in synchronous rounds
void launch_color_round(int n, const int* rp, const int* ci, uint32_t stream, const int* cin, int* cout, int* left,
                        int round, int* err, hipStream_t s);
void launch_color_count(int n, const int* col, int* cnt, hipStream_t s);
void launch_color_lists(int n, const int* col, int* cnt, const int* coff, int* crow, hipStream_t s);

// host runtime (hierarchy.cpp)
double hessenberg_spectral_radius(const double* H, int m);
void init_control(Hierarchy& h);
void build_hierarchy(Hierarchy& h, const amg_csr& A);
void resetup_hierarchy(Hierarchy& h, const double* val);
size_t release_cached_chunks();
void galerkin_standalone(Hierarchy& h, const amg_csr& A, const int* agg, const double* pval, int nc,
                         int* nnz_c, int** rp_c, int** ci_c, double** val_c);

}  // namespace amg
