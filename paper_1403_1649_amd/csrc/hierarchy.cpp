// Host runtime of setup (Algorithm 1): device arena, the level loop that
// drives the setup kernels, the Arnoldi spectral estimate with a small
// complex-shift QR eigenvalue solve on the host, and the dense coarsest-level
// inverse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "amg_internal.hpp"

namespace amg {

// ---------------------------------------------------------------- arena
namespace {
std::mutex g_cache_mu;
// Never destroyed: no destructor of the library runs at process exit, when the
// HIP runtime may already be shut down.
std::multimap<size_t, void*>& chunk_cache() {
  static auto* c = new std::multimap<size_t, void*>();
  return *c;
}
constexpr size_t kMinChunk = size_t(64) << 20;
constexpr size_t kAlign = 256;

void* take_chunk(size_t want, size_t* got) {
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto& c = chunk_cache();
    auto it = c.lower_bound(want);
    if (it != c.end() && it->first <= 4 * want + kMinChunk) {
      *got = it->first;
      void* p = it->second;
      c.erase(it);
      return p;
    }
  }
  size_t sz = std::max(want, kMinChunk);
  void* p = nullptr;
  if (hipMalloc(&p, sz) != hipSuccess) {
    (void)hipGetLastError();
    // release cached chunks and retry once
    std::lock_guard<std::mutex> g(g_cache_mu);
    for (auto& kv : chunk_cache()) (void)hipFree(kv.second);
    chunk_cache().clear();
    if (hipMalloc(&p, sz) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(AMG_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
    }
  }
  *got = sz;
  return p;
}

void give_chunk(void* p, size_t sz) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  chunk_cache().emplace(sz, p);
}
}  // namespace

size_t release_cached_chunks() {
  std::lock_guard<std::mutex> g(g_cache_mu);
  size_t bytes = 0;
  for (auto& kv : chunk_cache()) {
    bytes += kv.first;
    (void)hipFree(kv.second);
  }
  chunk_cache().clear();
  return bytes;
}

Arena::~Arena() {
  for (auto& c : chunks_) give_chunk(c.base, c.size);
}

void Arena::reserve(size_t bytes) {
  size_t got = 0;
  char* p = static_cast<char*>(take_chunk(bytes, &got));
  chunks_.push_back(Chunk{p, got, 0});
}

void* Arena::alloc(size_t bytes) {
  bytes = (bytes + kAlign - 1) / kAlign * kAlign;
  if (bytes == 0) bytes = kAlign;
  for (auto& c : chunks_) {
    if (c.off + bytes <= c.size) {
      void* p = c.base + c.off;
      c.off += bytes;
      used_ += bytes;
      return p;
    }
  }
  reserve(bytes);
  Chunk& c = chunks_.back();
  void* p = c.base + c.off;
  c.off += bytes;
  used_ += bytes;
  return p;
}

Hierarchy::~Hierarchy() {
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto& g : g_iter) (void)hipGraphExecDestroy(g);
  if (g_restart) (void)hipGraphExecDestroy(g_restart);
  if (h_pinned) (void)hipHostFree(h_pinned);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : pev)
    if (e) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------- eigenvalues
// Largest eigenvalue modulus of a real upper Hessenberg matrix (m <= 8) by the
// shifted QR algorithm in complex arithmetic: Givens rotations reduce
// H - mu I to triangular form, the product RQ + mu I is the next iterate,
// Wilkinson shifts from the trailing 2x2 block, deflation on a negligible
// subdiagonal entry.
double hessenberg_spectral_radius(const double* Hin, int m) {
  using cd = std::complex<double>;
  if (m <= 0) return 0.0;
  cd H[8][8];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) H[i][j] = cd(Hin[i * m + j], 0.0);
  double rho = 0.0;
  int hi = m - 1;
  int iter = 0;
  while (hi >= 0) {
    if (hi == 0) {
      rho = std::max(rho, std::abs(H[0][0]));
      break;
    }
    int l = hi;
    while (l > 0) {
      const double scale = std::abs(H[l][l]) + std::abs(H[l - 1][l - 1]);
      if (std::abs(H[l][l - 1]) <= 1e-15 * (scale > 0.0 ? scale : 1.0)) break;
      --l;
    }
    if (l == hi) {
      rho = std::max(rho, std::abs(H[hi][hi]));
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 200) {
      for (int i = l; i <= hi; ++i) rho = std::max(rho, std::abs(H[i][i]));
      break;
    }
    // Wilkinson shift: eigenvalue of the trailing 2x2 closer to H[hi][hi]
    const cd a = H[hi - 1][hi - 1], b = H[hi - 1][hi], c = H[hi][hi - 1], d = H[hi][hi];
    const cd tr = a + d, det = a * d - b * c;
    const cd disc = std::sqrt(tr * tr * 0.25 - det);
    const cd mu1 = tr * 0.5 + disc, mu2 = tr * 0.5 - disc;
    cd mu = std::abs(mu1 - d) < std::abs(mu2 - d) ? mu1 : mu2;
    if (iter % 11 == 10) mu = d + cd(std::abs(c), 0.0);   // exceptional shift
    for (int i = l; i <= hi; ++i) H[i][i] -= mu;
    cd cs[8], sn[8];
    for (int k = l; k < hi; ++k) {
      const cd x = H[k][k], y = H[k + 1][k];
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      if (r == 0.0) { cs[k] = 1.0; sn[k] = 0.0; continue; }
      cs[k] = x / r;
      sn[k] = y / r;
      for (int j = k; j <= hi; ++j) {
        const cd u = H[k][j], v = H[k + 1][j];
        H[k][j] = std::conj(cs[k]) * u + std::conj(sn[k]) * v;
        H[k + 1][j] = -sn[k] * u + cs[k] * v;
      }
    }
    for (int k = l; k < hi; ++k) {
      const int top = std::min(k + 2, hi);
      for (int i = l; i <= top; ++i) {
        const cd u = H[i][k], v = H[i][k + 1];
        H[i][k] = u * cs[k] + v * sn[k];
        H[i][k + 1] = -u * std::conj(sn[k]) + v * std::conj(cs[k]);
      }
    }
    for (int i = l; i <= hi; ++i) H[i][i] += mu;
  }
  return rho;
}

// ---------------------------------------------------------------- setup
namespace {

struct Sync {
  Hierarchy& h;
  Mailbox m{};
  int* hp() { return static_cast<int*>(h.h_pinned); }
  // ask for one device int in pinned slot `slot` at the next wait
  void fetch(const int* dptr, int slot, int count = 1, int stride = 1) {
    if (m.n == 8) throw Error(AMG_EINVAL, "more than 8 pending read-backs");
    m.src[m.n] = dptr;
    m.slot[m.n] = slot;
    m.count[m.n] = count;
    m.stride[m.n] = stride;
    ++m.n;
  }
  void wait_and_check() {
    AMG_HIP(hipGetLastError());   // a failed launch surfaces here
    launch_mailbox(m, h.d_err, hp(), h.stream);
    m.n = 0;
    AMG_HIP(hipStreamSynchronize(h.stream));
    AMG_HIP(hipGetLastError());
    const int e = hp()[63];
    if (!e) return;
    if (e & kErrNonFinite) throw Error(AMG_ENANINF, "non-finite matrix entry");
    if (e & kErrZeroDiag) throw Error(AMG_EINVAL, "zero or missing diagonal entry");
    if (e & kErrBadColumn) throw Error(AMG_EINVAL, "column index out of range or not strictly increasing");
    if (e & kErrNonSymPattern) throw Error(AMG_EINVAL, "sparsity pattern is not structurally symmetric");
    if (e & kErrCountOverflow) throw Error(AMG_EINVAL, "strong influence count exceeds 2^21");
    if (e & kErrUnassigned) throw Error(AMG_ECOARSEN, "node farther than k from every MIS(k) node");
    if (e & kErrSingular) throw Error(AMG_EBREAKDOWN, "coarsest matrix is singular");
    if (e & kErrCrossSystem) throw Error(AMG_EINVAL, "a matrix entry couples two systems of the batch");
    if (e & kErrColors) throw Error(AMG_EUNSUPPORTED, "the multi-colour ordering needs more than 64 colours");
    if (e & kErrTimeout) throw Error(AMG_EHIP, "a wait of the one-launch V-cycle tail ran out");
    throw Error(AMG_EHIP, "device error bits " + std::to_string(e));
  }
  // true (and the bit cleared) when the SPD elimination met a non-positive pivot
  bool take_not_spd() {
    Mailbox none{};
    launch_mailbox(none, h.d_err, hp(), h.stream);
    AMG_HIP(hipStreamSynchronize(h.stream));
    const int e = hp()[63];
    if (!(e & kErrNotSPD)) return false;
    launch_fill_int(1, h.d_err, e & ~kErrNotSPD, h.stream);
    return true;
  }
};

void alloc_solve_vectors(Hierarchy& h) {
  const size_t es = h.mixed() ? sizeof(float) : sizeof(double);
  const int L = h.L();
  for (int k = 0; k < L; ++k) {
    Level& lv = h.levels[k];
    const size_t n = lv.n, nc = lv.nc;
    lv.r = h.arena.alloc(n * es);
    lv.xt = h.arena.alloc(n * es);
    lv.rc = h.arena.alloc(nc * es);
    lv.c = h.arena.alloc(nc * es);
    if (h.opt.smoother == AMG_SMOOTHER_CHEBYSHEV) {
      lv.cr = h.arena.alloc(n * es);
      lv.cd0 = h.arena.alloc(n * es);
      lv.cd1 = h.arena.alloc(n * es);
    }
    if (k < h.opt.kcycle_levels) {
      lv.v = h.arena.alloc(nc * es);
      lv.rt = h.arena.alloc(nc * es);
      lv.d = h.arena.alloc(nc * es);
      lv.w = h.arena.alloc(nc * es);
    }
  }
  const size_t n0 = h.levels[0].n;
  h.r = h.arena.alloc_n<double>(n0);
  h.p = h.arena.alloc_n<double>(n0);
  h.q = h.arena.alloc_n<double>(n0);
  h.z = h.arena.alloc(n0 * es);
  h.xint = h.arena.alloc_n<double>(n0);
  if (h.mixed()) h.bz = h.arena.alloc(n0 * es);
}

// Sliced-ELL copy of A_k for the solve kernels.
// First half: slice widths and their scan; the total goes to pinned slot
// `slot` at the next wait of `sy`.
void sell_begin(Hierarchy& h, Arena& tmp, Level& lv, Sync& sy, int slot) {
  const int nsl = (lv.n + 63) / 64;
  int* widths = tmp.alloc_n<int>(nsl);
  launch_sell_widths(lv.n, lv.rp, widths, h.stream);
  lv.nslices = nsl;
  lv.sl_ptr = h.arena.alloc_n<int>(nsl + 1);
  scan_to_ptr(widths, lv.sl_ptr, nsl, h.scan, h.stream);
  sy.fetch(lv.sl_ptr + nsl, slot);
}
// Second half; the 16-bit offsets stay usable only if the flag read back in
// pinned slot `slot` at the next wait of `sy` is clear (sell_take_wide).
void sell_finish(Hierarchy& h, Level& lv, size_t total, Sync& sy, int slot) {
  lv.sl_total = (long)total;
  lv.sl_col = h.arena.alloc_n<int>(total);
  lv.sl_dcol = h.arena.alloc_n<int16_t>(total);
  lv.sl_wide = h.arena.alloc_n<int>(1);
  lv.sl_val = h.arena.alloc_n<double>(total);
  if (h.mixed()) lv.sl_val32 = h.arena.alloc_n<float>(total);
  launch_fill_int(1, lv.sl_wide, 0, h.stream);
  launch_sell_fill(lv.n, lv.nslices, lv.rp, lv.ci, lv.val, lv.sl_ptr, lv.sl_col, lv.sl_dcol, lv.sl_wide, lv.sl_val,
                   lv.sl_val32, h.stream);
  sy.fetch(lv.sl_wide, slot);
}
void sell_take_wide(Level& lv, Sync& sy, int slot) {
  if (sy.hp()[slot]) lv.sl_dcol = nullptr;
}
void build_sell(Hierarchy& h, Arena& tmp, Level& lv, bool offsets16 = false) {
  Sync sy{h};
  sell_begin(h, tmp, lv, sy, 0);
  sy.wait_and_check();
  sell_finish(h, lv, (size_t)sy.hp()[0], sy, 0);
  if (!offsets16) {   // not checked, so not used
    lv.sl_dcol = nullptr;
    return;
  }
  sy.wait_and_check();
  sell_take_wide(lv, sy, 0);
}

}  // namespace

void spmv_sell_f64(Hierarchy& h, const amg_csr& A, const double* x, double* y, bool offsets16) {
  Arena tmp;
  struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{h.stream};
  Level lv;
  lv.n = A.n;
  lv.nnz = A.nnz;
  lv.rp = const_cast<int*>(A.row_ptr);
  lv.ci = const_cast<int*>(A.col_idx);
  lv.val = const_cast<double*>(A.val);
  build_sell(h, tmp, lv, offsets16);
  if (offsets16 && !lv.sl_dcol) throw Error(AMG_EINVAL, "a column offset col - row does not fit in 16 bits");
  spmv_sell_level(h, lv, x, y, offsets16);
  Sync sy{h};
  sy.wait_and_check();
}

// The short-slice copy of a level whose rows vary in length: the rows of
// every 256-row window ordered by decreasing length, then slices of 16 rows
// (4 lanes per row) where rows average at least 12 entries, else of 32; built
// when it stores at least kShortSellGain fewer elements than the 64-row copy
// in row order.  slice_h = 32 or 16 builds that height regardless (tests).
// Its memory is an arena of its own, released when the level drops the copy.
constexpr double kShortSellGain = 0.08;

void build_short_sell(Hierarchy& h, Level& lv, int slice_h) {
  lv.sh = Level::ShortSell{};
  lv.sh_mem.reset();
  if (lv.n <= 0 || !lv.sl_ptr) return;
  const bool forced = slice_h == 32 || slice_h == 16;
  const int H = forced ? slice_h : (lv.nnz >= 12L * lv.n ? 16 : 32);
  auto mem = std::make_shared<Arena>();
  const int nwin = (lv.n + 255) / 256;
  const int nsl = (lv.n + H - 1) / H;
  int* perm = mem->alloc_n<int>((size_t)nwin * 256);
  int* widths = mem->alloc_n<int>(nsl);
  int* ptr = mem->alloc_n<int>(nsl + 1);
  launch_window_order(lv.n, lv.rp, perm, h.stream);
  launch_sell_widths(lv.n, lv.rp, widths, h.stream, H, perm);
  scan_to_ptr(widths, ptr, nsl, h.scan, h.stream);
  Sync sy{h};
  sy.fetch(ptr + nsl, 0);
  sy.wait_and_check();
  const long total = sy.hp()[0];
  if (std::getenv("AMG_DEBUG"))
    std::fprintf(stderr, "amg: sliced ELL elements n=%d nnz=%d: 64 rows in order %ld, %d rows by length %ld\n", lv.n,
                 lv.nnz, lv.sl_total, H, total);
  if (!forced && (double)total > (1.0 - kShortSellGain) * (double)lv.sl_total) return;
  Level::ShortSell sh;
  sh.h = H;
  sh.nslices = nsl;
  sh.total = total;
  sh.perm = perm;
  sh.ptr = ptr;
  const size_t t = (size_t)std::max(total, 1L);
  sh.col = mem->alloc_n<int>(t);
  sh.dcol = lv.sl_dcol ? mem->alloc_n<int16_t>(t) : nullptr;   // the offsets fit: they do in the 64-row copy
  sh.val = mem->alloc_n<double>(t);
  sh.val32 = h.mixed() ? mem->alloc_n<float>(t) : nullptr;
  launch_sell_fill(lv.n, sh.nslices, lv.rp, lv.ci, lv.val, sh.ptr, sh.col, sh.dcol, nullptr, sh.val, sh.val32,
                   h.stream, sh.h, sh.perm);
  lv.sh = sh;
  lv.sh_mem = mem;
}

// The sliced-diagonal copy of a level: built when no 64-row slice has more
// than kSdiaCap distinct offsets col - row and the stored values (diagonals x
// 64) exceed the level's entries by at most kSdiaPad; its memory is an arena
// of its own, released when the level drops the copy.
constexpr int kSdiaCap = 32;
constexpr double kSdiaPad = 0.10;
constexpr int kSdiaRows = 64;   // rows per slice (one wave)

void build_sdia(Hierarchy& h, Level& lv) {
  lv.dia = Level::Sdia{};
  lv.dia_mem.reset();
  if (lv.n <= 0 || lv.nnz <= 0) return;
  auto mem = std::make_shared<Arena>();
  const int nsl = (lv.n + kSdiaRows - 1) / kSdiaRows;
  int* cnt = mem->alloc_n<int>(nsl);
  int* ptr = mem->alloc_n<int>(nsl + 1);
  int* over = mem->alloc_n<int>(1);
  launch_fill_int(1, over, 0, h.stream);
  launch_sdia_count(lv.n, lv.rp, lv.ci, kSdiaCap, cnt, over, h.stream);
  scan_to_ptr(cnt, ptr, nsl, h.scan, h.stream);
  Sync sy{h};
  sy.fetch(ptr + nsl, 0);
  sy.fetch(over, 1);
  sy.wait_and_check();
  const long total = sy.hp()[0];
  const bool over_cap = sy.hp()[1] != 0;
  if (std::getenv("AMG_DEBUG"))
    std::fprintf(stderr, "amg: sliced diagonals n=%d nnz=%d: %ld values%s\n", lv.n, lv.nnz, total * kSdiaRows,
                 over_cap ? " (a slice over the cap)" : "");
  if (over_cap || (double)total * kSdiaRows > (1.0 + kSdiaPad) * (double)lv.nnz) return;
  Level::Sdia d;
  d.nslices = nsl;
  d.total = total;
  d.ptr = ptr;
  d.off = mem->alloc_n<int>((size_t)std::max(total, 1L));
  d.val = mem->alloc_n<double>((size_t)std::max(total, 1L) * kSdiaRows);
  d.val32 = h.mixed() ? mem->alloc_n<float>((size_t)std::max(total, 1L) * kSdiaRows) : nullptr;
  launch_sdia_fill(lv.n, lv.rp, lv.ci, lv.val, d.ptr, d.off, d.val, d.val32, h.stream);
  lv.dia = d;
  lv.dia_mem = mem;
}

namespace {

void make_float_copies(Hierarchy& h) {
  for (int k = 0; k < (int)h.levels.size(); ++k) {
    Level& lv = h.levels[k];
    lv.val32 = h.arena.alloc_n<float>(lv.nnz);
    launch_to_float(lv.nnz, lv.val, lv.val32, h.stream);
    if (k < h.L()) {
      lv.pval32 = h.arena.alloc_n<float>(lv.n);
      launch_to_float(lv.n, lv.pval, lv.pval32, h.stream);
      lv.rval32 = h.arena.alloc_n<float>(std::max(lv.nr, 1));
      launch_to_float(lv.nr, lv.rval, lv.rval32, h.stream);
    }
  }
}
}  // namespace

// Aggregate segments: members of aggregate I at agg_rows[agg_ptr[I]..agg_ptr[I+1]),
// ascending.  Scratch from `tmp`.
static void build_segments(Hierarchy& h, Arena& tmp, int n, int nc, const int* agg, int* agg_ptr,
                           int* agg_rows) {
  hipStream_t s = h.stream;
  int* counts = tmp.alloc_n<int>(nc);
  launch_fill_int(nc, counts, 0, s);
  launch_agg_count(n, agg, counts, s);
  scan_to_ptr(counts, agg_ptr, nc, h.scan, s);
  launch_fill_int(nc, counts, 0, s);
  launch_agg_scatter(n, agg, agg_ptr, counts, agg_rows, s);
  launch_agg_sort(nc, agg_ptr, agg_rows, s);
}

// Galerkin product A_c = P^T A P for given segments (count, scan, fill).
static void galerkin_product(Hierarchy& h, Arena& tmp, Arena& out, const Level& lv, int nc,
                             const int* agg, const double* pval, const int* agg_ptr, const int* agg_rows,
                             int** rp_c, int** ci_c, double** val_c, int* nnz_c) {
  hipStream_t s = h.stream;
  Sync sy{h};
  const int n = lv.n, nnz = lv.nnz;
  GalerkinScratch g;
  g.lens = tmp.alloc_n<int>(n > 0 ? n : 1);
  g.toff = tmp.alloc_n<int>((size_t)n + 1);
  g.tkey = tmp.alloc_n<int>(nnz > 0 ? nnz : 1);
  g.tval = tmp.alloc_n<double>(nnz > 0 ? nnz : 1);
  g.ucount = tmp.alloc_n<int>(nc > 0 ? nc : 1);
  g.list = tmp.alloc_n<int>(2 * (size_t)(nc > 0 ? nc : 1));
  g.ctl = h.d_ctl + kCtlAggFill;
  launch_galerkin_stage(g, n, nc, nnz, lv.rp, lv.ci, lv.val, agg, pval, agg_ptr, agg_rows, h.scan, s);
  *rp_c = out.alloc_n<int>((size_t)nc + 1);
  scan_to_ptr(g.ucount, *rp_c, nc, h.scan, s);
  sy.fetch(*rp_c + nc, 0);
  sy.wait_and_check();
  *nnz_c = sy.hp()[0];
  *ci_c = out.alloc_n<int>(*nnz_c > 0 ? *nnz_c : 1);
  *val_c = out.alloc_n<double>(*nnz_c > 0 ? *nnz_c : 1);
  launch_galerkin_finish(g, nc, agg_ptr, *rp_c, *ci_c, *val_c, s);
}

void galerkin_standalone(Hierarchy& h, const amg_csr& A, const int* agg, const double* pval, int nc,
                         int* nnz_c, int** rp_c, int** ci_c, double** val_c) {
  Arena& tmp = h.arena;
  Level lv;
  lv.n = A.n;
  lv.nnz = A.nnz;
  lv.rp = const_cast<int*>(A.row_ptr);
  lv.ci = const_cast<int*>(A.col_idx);
  lv.val = const_cast<double*>(A.val);
  Sync sy0{h};
  AMG_HIP(hipMemcpyAsync(sy0.hp(), A.row_ptr, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  AMG_HIP(hipMemcpyAsync(sy0.hp() + 1, A.row_ptr + A.n, sizeof(int), hipMemcpyDeviceToHost, h.stream));
  sy0.wait_and_check();
  if (sy0.hp()[0] != 0 || sy0.hp()[1] != A.nnz) throw Error(AMG_EINVAL, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  launch_check_rowptr(A.n, A.row_ptr, h.d_err, h.stream);
  sy0.wait_and_check();
  launch_check_matrix(A.n, A.row_ptr, A.col_idx, A.val, h.d_err, h.stream);
  launch_check_index(A.n, agg, nc, h.d_err, h.stream);
  sy0.wait_and_check();
  int* agg_ptr = tmp.alloc_n<int>(nc + 1);
  int* agg_rows = tmp.alloc_n<int>(A.n);
  build_segments(h, tmp, A.n, nc, agg, agg_ptr, agg_rows);
  galerkin_product(h, tmp, tmp, lv, nc, agg, pval, agg_ptr, agg_rows, rp_c, ci_c, val_c, nnz_c);
  Sync sy{h};
  sy.wait_and_check();
}

void init_control(Hierarchy& h) {
  h.d_err = h.arena.alloc_n<int>(64);
  h.d_ctl = h.arena.alloc_n<int>(kCtlWords);
  h.d_sc = h.arena.alloc_n<double>(kScWords);
  h.d_part = h.arena.alloc_n<double>((size_t)kMaxPartialBlocks * kMaxReduce);
  h.d_ticket = h.arena.alloc_n<unsigned>(64);
  h.d_tail = h.arena.alloc_n<unsigned>(64);
  h.d_mis = h.arena.alloc_n<int>(kMisWords);
  launch_fill_int(64, h.d_err, 0, h.stream);
  launch_fill_int(kCtlWords, h.d_ctl, 0, h.stream);
  launch_fill_double(kScWords, h.d_sc, 0.0, h.stream);   // arena memory is recycled, not cleared
  launch_fill_int(64, reinterpret_cast<int*>(h.d_ticket), 0, h.stream);
  launch_fill_int(64, reinterpret_cast<int*>(h.d_tail), 0, h.stream);
  launch_fill_int(1, h.d_ctl + kCtlOne, 1, h.stream);
  if (!h.h_pinned) AMG_HIP(hipHostMalloc(&h.h_pinned, kPinnedBytes, hipHostMallocDefault));
}

// omega_k = jacobi_scale / rho from the Arnoldi Hessenberg H (row stride 8,
// m columns; wn = ||D^-1 A q_j||), then the weights omega_k / a_ii.
// Levels above this size sweep node lists after the first MIS(2) read-back
// (C2 level 0, 16 rounds: after 8 rounds 0.2 % of the nodes are undecided).
constexpr int kMisListRows = 65536;

static void set_jacobi_weight(Hierarchy& h, Level& lv, int m, const double* Hh, const double* wn) {
  int size = m;
  for (int j = 0; j < m; ++j) {
    if (Hh[(j + 1) * 8 + j] <= 1e-14 * wn[j]) { size = j + 1; break; }
  }
  // upper Hessenberg: the slots below the subdiagonal are never written
  double Hs[64];
  for (int i = 0; i < size; ++i)
    for (int j = 0; j < size; ++j) Hs[i * size + j] = i <= j + 1 ? Hh[i * 8 + j] : 0.0;
  lv.rho = hessenberg_spectral_radius(Hs, size);
  if (!(lv.rho > 0.0) || !std::isfinite(lv.rho)) throw Error(AMG_EBREAKDOWN, "spectral radius estimate not positive");
  lv.omega = h.opt.jacobi_scale / lv.rho;
  if (h.opt.smoother == AMG_SMOOTHER_CHEBYSHEV) {
    // the polynomial acts on D^-1 A: the scaling is 1 / a_ii; the interval
    // [b / ratio, b] around the estimate, b = upper * rho, gives the
    // recurrence coefficients (centre theta, half-width delta)
    const double bb = h.opt.cheb_upper * lv.rho, aa = bb / h.opt.cheb_ratio;
    const double theta = 0.5 * (bb + aa), delta = 0.5 * (bb - aa), sigma = theta / delta;
    double* c = lv.cheb_host;
    c[0] = 1.0 / theta;
    double rho_prev = 1.0 / sigma;
    for (int j = 1; j < h.opt.cheb_degree; ++j) {
      const double rj = 1.0 / (2.0 * sigma - rho_prev);
      c[2 * j - 1] = rj * rho_prev;
      c[2 * j] = 2.0 * rj / delta;
      rho_prev = rj;
    }
    if (!lv.cheb) lv.cheb = h.arena.alloc_n<double>(16);
    launch_set16(lv.cheb, c, h.stream);
    launch_jacobi_weights(lv.n, 1.0, lv.diag, lv.wdinv, lv.wdinv32, h.stream);
    return;
  }
  if (h.opt.smoother == AMG_SMOOTHER_MCSGS) {   // Gauss-Seidel divides by a_ii
    launch_jacobi_weights(lv.n, 1.0, lv.diag, lv.wdinv, lv.wdinv32, h.stream);
    return;
  }
  launch_jacobi_weights(lv.n, lv.omega, lv.diag, lv.wdinv, lv.wdinv32, h.stream);
}

// Dense inverse of the coarsest level (allocated on the first call): flexible
// CG assumes a symmetric positive definite operator, so blocked elimination
// without pivoting, unless a pivot says otherwise; partial pivoting for
// FGMRES or a non-positive pivot.
static void coarse_inverse(Hierarchy& h, Arena& tmp, Sync& sy) {
  hipStream_t s = h.stream;
  const amg_options& o = h.opt;
  Level& cl = h.levels.back();
  if (cl.n > o.dense_max)
    throw Error(AMG_ECOARSEN, "coarsest level has " + std::to_string(cl.n) + " unknowns");
  const size_t nn = (size_t)cl.n * cl.n;
  double* work = tmp.alloc_n<double>(2 * nn + 2 * (size_t)cl.n);
  int* gj_sync = tmp.alloc_n<int>(4 + cl.n);
  if (!h.cinv) {
    h.cinv = h.arena.alloc_n<double>(nn);
    if (h.mixed()) h.cinv32 = h.arena.alloc_n<float>(nn);
  }
  bool inverted = false;
  if (o.krylov == AMG_KRYLOV_FCG) {
    const TermInfo t{0, 0, cl.n, 0, 0};
    TermInfo* dt = tmp.alloc_n<TermInfo>(1);
    AMG_HIP(hipMemcpyAsync(dt, &t, sizeof(TermInfo), hipMemcpyHostToDevice, s));
    launch_dense_inverse_spd(1, dt, &t, cl.n, cl.rp, cl.ci, cl.val, h.cinv, h.cinv32, tmp, h.d_err, s);
    inverted = !sy.take_not_spd();
  }
  if (!inverted) launch_dense_inverse(cl.n, cl.rp, cl.ci, cl.val, work, h.cinv, h.cinv32, gj_sync, h.d_err, s);
}

// Multi-colour ordering of level k (symmetric Gauss-Seidel smoother): rounds
// of first-fit colouring by node-hash priority (stream seed + 2) until every
// row has a colour, then the rows of each colour listed together.
static void color_level(Hierarchy& h, Arena& tmp, Level& lv, Sync& sy) {
  hipStream_t s = h.stream;
  const int n = lv.n;
  int* in = tmp.alloc_n<int>(n);
  int* out = tmp.alloc_n<int>(n);
  int* left = tmp.alloc_n<int>(2);
  launch_fill_int(n, in, -1, s);
  launch_fill_int(2, left, 0, s);
  int round = 0;
  while (true) {
    for (int b = 0; b < 4; ++b, ++round) {
      launch_color_round(n, lv.rp, lv.ci, h.opt.seed + 2, in, out, left, round, h.d_err, s);
      std::swap(in, out);
    }
    sy.fetch(left + ((round - 1) & 1), 0);
    sy.wait_and_check();
    if (sy.hp()[0] == 0) break;
    if (round > 100000) throw Error(AMG_ECOARSEN, "colouring rounds did not terminate");
  }
  lv.colors = h.arena.alloc_n<int>(n);
  AMG_HIP(hipMemcpyAsync(lv.colors, in, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s));
  int* cnt = tmp.alloc_n<int>(64);
  launch_fill_int(64, cnt, 0, s);
  launch_color_count(n, lv.colors, cnt, s);
  int hc[64];
  AMG_HIP(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  int nc = 0;
  for (int c = 0; c < 64; ++c)
    if (hc[c] > 0) nc = c + 1;
  lv.coff.assign(nc + 1, 0);
  for (int c = 0; c < nc; ++c) lv.coff[c + 1] = lv.coff[c] + hc[c];
  int* dcoff = tmp.alloc_n<int>(nc + 1);
  AMG_HIP(hipMemcpyAsync(dcoff, lv.coff.data(), (nc + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  lv.crow = h.arena.alloc_n<int>(n);
  launch_fill_int(64, cnt, 0, s);
  launch_color_lists(n, lv.colors, cnt, dcoff, lv.crow, s);
  AMG_HIP(hipStreamSynchronize(s));   // the host offsets array is read by the copy above
}

// The learned weights face the method's own judge (iteration count, then the
// final residual): a probe solve of A x = A u (u hashed from seed + 3) to a
// loose tolerance with the learned weights and with the plain omega_k / a_ii
// on every level; the learned ones stay only when they need fewer
// iterations, or as many and end with a smaller true residual.
constexpr double kJudgeRtol = 1e-4;
static void judge_learned(Hierarchy& h, Arena& tmp) {
  const int L = h.L();
  bool any = false;
  for (int k = 0; k < L; ++k) any = any || h.levels[k].learned;
  if (!any) return;
  hipStream_t s = h.stream;
  const int n = h.levels[0].n;
  double* u = tmp.alloc_n<double>(n);
  double* b = tmp.alloc_n<double>(n);
  double* x = tmp.alloc_n<double>(n);
  launch_hash_vector(n, h.opt.seed + 3, u, s);
  level_spmv(h, 0, u, b, s);
  std::vector<double*> keep64(L, nullptr);
  std::vector<float*> keep32(L, nullptr);
  for (int k = 0; k < L; ++k) {
    Level& lv = h.levels[k];
    if (!lv.learned) continue;
    keep64[k] = tmp.alloc_n<double>(lv.n);
    AMG_HIP(hipMemcpyAsync(keep64[k], lv.wdinv, (size_t)lv.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (lv.wdinv32) {
      keep32[k] = tmp.alloc_n<float>(lv.n);
      AMG_HIP(hipMemcpyAsync(keep32[k], lv.wdinv32, (size_t)lv.n * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
  }
  auto probe = [&](int* it, double* rel) {
    const int mi = h.opt.max_iter;
    h.opt.max_iter = 500;
    try {
      (void)solve_fcg_impl(h, b, kJudgeRtol, x, it, rel);
    } catch (...) {
      h.opt.max_iter = mi;
      throw;
    }
    h.opt.max_iter = mi;
  };
  probe(&h.judge_it_learned, &h.judge_rel_learned);
  for (int k = 0; k < L; ++k) {
    Level& lv = h.levels[k];
    if (lv.learned) launch_jacobi_weights(lv.n, lv.omega, lv.diag, lv.wdinv, lv.wdinv32, s);
  }
  probe(&h.judge_it_plain, &h.judge_rel_plain);
  const bool keep = h.judge_it_learned < h.judge_it_plain ||
                    (h.judge_it_learned == h.judge_it_plain && h.judge_rel_learned < h.judge_rel_plain);
  h.judge_kept = keep ? 1 : 0;
  for (int k = 0; k < L; ++k) {
    Level& lv = h.levels[k];
    if (!lv.learned) continue;
    if (!keep) {
      lv.learned = 0;
      continue;
    }
    AMG_HIP(hipMemcpyAsync(lv.wdinv, keep64[k], (size_t)lv.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (keep32[k])
      AMG_HIP(hipMemcpyAsync(lv.wdinv32, keep32[k], (size_t)lv.n * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  AMG_HIP(hipStreamSynchronize(s));
}

void build_hierarchy(Hierarchy& h, const amg_csr& A) {
  hipStream_t s = h.stream;
  const amg_options& o = h.opt;
  Sync sy{h};
  Arena tmp;
  // on any exit, drain the stream before the scratch chunks go back to the cache
  struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
  // scan scratch sized for the largest level
  init_scan(h.scan, h.arena, std::max(A.n, A.nnz), s);

  Level l0;
  l0.n = A.n;
  l0.nnz = A.nnz;
  if (o.flags & AMG_FLAG_BORROW_A) {   // the caller keeps A alive and unchanged; nothing writes level 0
    l0.rp = const_cast<int*>(A.row_ptr);
    l0.ci = const_cast<int*>(A.col_idx);
    l0.val = const_cast<double*>(A.val);
  } else {
    l0.rp = h.arena.alloc_n<int>(A.n + 1);
    l0.ci = h.arena.alloc_n<int>(A.nnz);
    l0.val = h.arena.alloc_n<double>(A.nnz);
    AMG_HIP(hipMemcpyAsync(l0.rp, A.row_ptr, (A.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(l0.ci, A.col_idx, (size_t)A.nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(l0.val, A.val, (size_t)A.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  // the row pointers must be consistent before any kernel walks the rows
  sy.fetch(l0.rp, 0);
  sy.fetch(l0.rp + A.n, 1);
  sy.wait_and_check();
  if (sy.hp()[0] != 0 || sy.hp()[1] != A.nnz) throw Error(AMG_EINVAL, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  launch_check_rowptr(l0.n, l0.rp, h.d_err, s);   // monotone: every row lies inside [0, nnz)
  sy.wait_and_check();
  launch_check_matrix(l0.n, l0.rp, l0.ci, l0.val, h.d_err, s);
  l0.B = h.arena.alloc_n<double>(A.n);
  launch_fill_double(A.n, l0.B, 1.0, s);   // B_0 = 1, the constant near null space vector
  h.levels.push_back(l0);
  sy.wait_and_check();

  const bool debug = std::getenv("AMG_DEBUG") != nullptr;
  if (o.smoother == AMG_SMOOTHER_LEARNED) {
    if (!o.mlp_weights) throw Error(AMG_EINVAL, "learned smoother without weights");
    const int np = mlp_num_params();
    for (int q = 0; q < np; ++q)
      if (!std::isfinite(o.mlp_weights[q])) throw Error(AMG_EINVAL, "non-finite MLP weight");
    h.mlp_w = h.arena.alloc_n<float>(np);
    AMG_HIP(hipMemcpyAsync(h.mlp_w, o.mlp_weights, np * sizeof(float), hipMemcpyHostToDevice, s));
    sy.wait_and_check();
    h.opt.mlp_weights = nullptr;   // the host pointer is not kept
  }
  // The Arnoldi of a level runs behind the next level's first kernels: its
  // Hessenberg matrix is read at the next sync, not waited for on its own.
  int arn_level = -1, arn_m = 0;
  double* arn_host = static_cast<double*>(h.h_pinned) + kPinnedArn;
  auto take_arnoldi = [&]() {
    if (arn_level < 0) return;
    double Hh[48], wn[8];
    for (int i = 0; i < 48; ++i) Hh[i] = arn_host[i];
    for (int j = 0; j < 8; ++j) wn[j] = arn_host[48 + j];
    Level& la = h.levels[arn_level];
    set_jacobi_weight(h, la, arn_m, Hh, wn);
    if (debug) std::fprintf(stderr, "amg: level %d rho=%.6f omega=%.6f\n", arn_level, la.rho, la.omega);
    arn_level = -1;
  };
  while (true) {
    const int k = (int)h.levels.size() - 1;
    Level& lv = h.levels[k];
    lv.diag = h.arena.alloc_n<double>(lv.n);
    lv.lpr = pick_lanes_per_row(lv.n, lv.nnz);
    lv.t64.lpr = lv.t32.lpr = lv.lpr;
    if (lv.n <= o.coarse_max || k + 1 >= o.max_levels) break;
    const int n = lv.n, nnz = lv.nnz;

    // the sliced-ELL copy serves the solve and, on stencil-like levels, the
    // Arnoldi mat-vecs; its size is read back with the first MIS(2) count
    sell_begin(h, tmp, lv, sy, 2);

    // strength (Section 2.1.1) and the strong graph G = C u C^T
    lv.strong = h.arena.alloc_n<uint8_t>(nnz);
    launch_strength(n, nnz, lv.rp, lv.ci, lv.val, o.strength_alpha, lv.strong, lv.diag, s);
    uint8_t* gmask = tmp.alloc_n<uint8_t>(nnz);
    int* gdeg = tmp.alloc_n<int>(n);
    int* cnt = tmp.alloc_n<int>(n);
    launch_graph_count(n, nnz, lv.rp, lv.ci, lv.strong, gmask, gdeg, cnt, h.d_err, s);
    int* gptr = tmp.alloc_n<int>(n + 1);
    scan_to_ptr(gdeg, gptr, n, h.scan, s);
    sy.fetch(gptr + n, 3);
    // the pattern is structurally symmetric with a full diagonal (checked),
    // so G has at most nnz - n entries: no read-back before the fill
    int* gcol = tmp.alloc_n<int>(nnz > 0 ? nnz : 1);
    launch_graph_fill(n, nnz, lv.rp, lv.ci, gmask, gptr, gcol, s);

    // MIS(2) rounds (Algorithm 2); MIS(k) with k sweeps per round (Section 2.1.2)
    const int mk = o.mis_k;
    lv.tuple = h.arena.alloc_n<uint64_t>(n);
    uint64_t* M1 = tmp.alloc_n<uint64_t>(n);
    uint64_t* Ma = mk > 2 ? tmp.alloc_n<uint64_t>(n) : nullptr;
    uint64_t* Mb = mk > 3 ? tmp.alloc_n<uint64_t>(n) : nullptr;
    launch_mis_init(n, cnt, o.seed, lv.tuple, M1, h.d_mis, h.d_err, s);
    int round = 0;
    int batch = 8;   // rounds between read-backs: a round after the last exits at entry
    int nnzg = -1;
    bool arn_due = false;   // the previous level's Hessenberg matrix has arrived
    const int glanes = group_lanes(n, (long)nnz - n);
    MisLists ml{};
    bool lists = false;   // late rounds sweep only the nodes that can still change
    while (true) {
      for (int b = 0; b < batch; ++b, ++round) {
        if (mk == 2) launch_mis_round(n, gptr, gcol, lv.tuple, M1, h.d_mis, round, glanes, s, lists ? &ml : nullptr);
        else launch_misk_round(n, gptr, gcol, lv.tuple, M1, Ma, Mb, h.d_mis, round, mk, glanes, s);
      }
      if (arn_due) {   // its eigenvalues on the host while the rounds run
        take_arnoldi();
        arn_due = false;
      }
      sy.fetch(h.d_mis + mis_word(round & 1, 0), 0, kMisSlots, mis_word(0, 1));
      sy.fetch(h.d_mis + kMisRoundsWord, 1);
      sy.wait_and_check();
      if (nnzg < 0) {   // the level's first read-back also brings the sizes of G and of the sliced ELL
        nnzg = sy.hp()[3];
        sell_finish(h, lv, (size_t)sy.hp()[2], sy, 4);
        arn_due = true;
      }
      if (sy.hp()[0] == 0) break;
      if (round > 4096) throw Error(AMG_ECOARSEN, "MIS(2) rounds did not terminate");
      batch = 4;
      if (!lists && mk == 2 && n > kMisListRows) {
        ml.fnear = tmp.alloc_n<int>(n);
        ml.pnear = tmp.alloc_n<int>((size_t)n + 1);
        ml.near = tmp.alloc_n<int>(n);
        ml.count = ml.pnear + n;
        launch_mis_lists(n, gptr, gcol, lv.tuple, ml, h.scan, s);
        lists = true;
      }
    }
    lv.mis_rounds = sy.hp()[1];
    if (debug) std::fprintf(stderr, "amg: level %d n=%d nnz=%d nnz(G)=%d mis_rounds=%d\n", k, n, nnz, nnzg,
                            lv.mis_rounds);

    // aggregates: coarse ids of the roots, nearest-root assignment
    int* flags = tmp.alloc_n<int>(n);
    int* root_id = tmp.alloc_n<int>(n + 1);
    launch_root_flags(n, lv.tuple, flags, s);
    scan_to_ptr(flags, root_id, n, h.scan, s);
    sy.fetch(root_id + n, 0);
    if (arn_due) take_arnoldi();
    sy.wait_and_check();
    if (lv.sl_wide) sell_take_wide(lv, sy, 4);   // fetched with the first MIS(2) count or here
    const int nc = sy.hp()[0];
    if (nc <= 0 || nc > 0.9 * n) {
      lv.strong = nullptr;   // stalled: this level is the coarsest
      lv.tuple = nullptr;
      break;
    }
    int* choice = tmp.alloc_n<int>(n);
    lv.agg = h.arena.alloc_n<int>(n);
    if (mk == 2) {
      launch_aggregate(n, nnzg, gptr, gcol, lv.tuple, root_id, choice, lv.agg, h.d_err, s);
    } else {
      int* choice2 = tmp.alloc_n<int>(n);
      launch_aggregate_k(n, nnzg, gptr, gcol, lv.tuple, root_id, mk, choice, choice2, lv.agg, h.d_err, s);
    }
    lv.nc = nc;
    lv.agg_ptr = h.arena.alloc_n<int>(nc + 1);
    lv.agg_rows = h.arena.alloc_n<int>(n);
    build_segments(h, tmp, n, nc, lv.agg, lv.agg_ptr, lv.agg_rows);

    // interpolation (Algorithm 3)
    Level lc;
    lc.n = nc;
    lc.B = h.arena.alloc_n<double>(nc);
    lv.pval = h.arena.alloc_n<double>(n);
    launch_interp(n, nc, lv.agg, lv.agg_ptr, lv.agg_rows, lv.B, lc.B, lv.pval, s);
    lv.nr = n;
    lv.rval = h.arena.alloc_n<double>(n);
    launch_gather_double(n, lv.agg_rows, lv.pval, lv.rval, s);
    lv.rlpr = pick_lanes_per_row(nc, n);

    // Galerkin product (Section 3.1)
    galerkin_product(h, tmp, h.arena, lv, nc, lv.agg, lv.pval, lv.agg_ptr, lv.agg_rows, &lc.rp, &lc.ci,
                     &lc.val, &lc.nnz);

    // damped Jacobi weight (Section 2.2.1)
    const int m = std::min(o.arnoldi_m, n);
    double* Q = tmp.alloc_n<double>((size_t)(m + 1) * n);
    double* w = tmp.alloc_n<double>(n);
    lv.wdinv = h.arena.alloc_n<double>(n);
    if (h.mixed()) lv.wdinv32 = h.arena.alloc_n<float>(n);
    if (debug) std::fprintf(stderr, "amg: level %d nc=%d nnz_c=%d\n", k, nc, lc.nnz);
    if (o.smoother != AMG_SMOOTHER_LEARNED) {
      arnoldi_enqueue(h, lv, m, o.seed + 1, Q, w, h.d_sc, RedCtx{h.d_part, h.d_ticket}, arn_host, s);
      arn_level = k;
      arn_m = m;
    } else {
      double Hh[48], wn[8];
      arnoldi(h, lv, m, o.seed + 1, Q, w, Hh, wn);
      set_jacobi_weight(h, lv, m, Hh, wn);
      if (debug) std::fprintf(stderr, "amg: level %d rho=%.6f omega=%.6f\n", k, lv.rho, lv.omega);
      // learned per-row weights on every level whose smoothing loss on
      // validation samples is finite (the losses, with omega_k and with the
      // network, are kept for the caller); the probe-solve judge after the
      // setup then keeps them or returns to omega_k (a smaller one-step loss
      // did not predict fewer iterations: larger weights with a larger loss
      // gave fewer)
      const bool always = (o.flags & AMG_FLAG_LEARNED_ALWAYS) != 0;
      Arena vt;
      bool keep = always;
      if (!always) {
        double* omv = vt.alloc_n<double>(n);
        launch_fill_double(n, omv, lv.omega, s);
        lv.loss_plain = mlp_loss_grad(h, vt, lv, k, h.mlp_w, 4, 0x5eed0000u + k, nullptr, 0, omv, nullptr, 0);
        lv.loss_learned = mlp_loss_grad(h, vt, lv, k, h.mlp_w, 4, 0x5eed0000u + k, nullptr, 0, nullptr, nullptr, 0);
        keep = std::isfinite(lv.loss_learned);
      }
      if (keep) {
        float* F = vt.alloc_n<float>((size_t)n * 9);
        double* beta = vt.alloc_n<double>(n);
        mlp_features(h, lv, k, F, beta);
        mlp_omega(h, lv, F, beta, h.mlp_w, nullptr, lv.wdinv, lv.wdinv32, nullptr);
        lv.learned = 1;
      }
      sy.wait_and_check();
    }
    h.levels.push_back(lc);
  }

  coarse_inverse(h, tmp, sy);
  if (o.smoother == AMG_SMOOTHER_MCSGS)
    for (int k = 0; k < h.L(); ++k) color_level(h, tmp, h.levels[k], sy);
  if (h.mixed()) make_float_copies(h);
  alloc_solve_vectors(h);
  for (int k = 0; k < h.L(); ++k)
    if (h.levels[k].nslices == 0) build_sell(h, tmp, h.levels[k]);
  sy.wait_and_check();
  take_arnoldi();
  using clk = std::chrono::steady_clock;
  const auto t_tune = clk::now();
  if (!(o.flags & AMG_FLAG_NO_TUNE)) autotune_levels(h);
  if (o.smoother == AMG_SMOOTHER_LEARNED && !(o.flags & AMG_FLAG_LEARNED_ALWAYS)) judge_learned(h, tmp);
  const auto t_graph = clk::now();
  h.tune_ms = std::chrono::duration<double, std::milli>(t_graph - t_tune).count();
  if (o.probe != AMG_PROBE_NONE) {
    AMG_HIP(hipEventCreate(&h.pev[0]));
    AMG_HIP(hipEventCreate(&h.pev[1]));
  }
  if (!(o.flags & AMG_FLAG_NO_GRAPH) && o.krylov == AMG_KRYLOV_FCG) build_solve_graphs(h);
  h.capture_ms = std::chrono::duration<double, std::milli>(clk::now() - t_graph).count();
}


// Numeric re-setup on the fixed pattern (Section 3.1, index reuse): new
// values of A_0; every level keeps its strength, MIS(2), aggregates and P_k;
// A_{k+1} is replayed from the stored term lists (built by the first call),
// then the diagonals, the sliced-ELL values and FP32 copies, each level's
// Jacobi weight (Arnoldi) and the coarse inverse are formed again.  The
// autotuned kernels and the captured solve graphs stay; with a borrowed A_0
// given at a new address the graphs are captured again.
void resetup_hierarchy(Hierarchy& h, const double* val) {
  hipStream_t s = h.stream;
  const amg_options& o = h.opt;
  Sync sy{h};
  Arena tmp;
  struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
  Level& l0 = h.levels[0];
  bool repoint = false;
  if (o.flags & AMG_FLAG_BORROW_A) {
    if (val != l0.val) {
      l0.val = const_cast<double*>(val);
      repoint = true;
    }
  } else if (val != l0.val) {
    AMG_HIP(hipMemcpyAsync(l0.val, val, (size_t)l0.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  launch_check_matrix(l0.n, l0.rp, l0.ci, l0.val, h.d_err, s);
  sy.wait_and_check();
  const int L = h.L();
  for (int k = 0; k < L; ++k) {   // term lists in segment order, once per hierarchy
    Level& lv = h.levels[k];
    Level& lc = h.levels[k + 1];
    if (lv.rs_tptr) continue;
    int* cnt = tmp.alloc_n<int>(lc.nnz > 0 ? lc.nnz : 1);
    launch_fill_int(lc.nnz, cnt, 0, s);
    launch_rs_count(lv, lc, cnt, h.d_err, s);
    lv.rs_tptr = h.arena.alloc_n<int>((size_t)lc.nnz + 1);
    scan_to_ptr(cnt, lv.rs_tptr, lc.nnz, h.scan, s);
    lv.rs_f = h.arena.alloc_n<int>(lv.nnz);
    lv.rs_i = h.arena.alloc_n<int>(lv.nnz);
    launch_fill_int(lc.nnz, cnt, 0, s);
    launch_rs_fill(lv, lc, cnt, lv.rs_f, lv.rs_i, h.d_err, s);
  }
  for (int k = 0; k < L; ++k) launch_rs_values(h.levels[k], h.levels[k + 1], s);
  for (int k = 0; k <= L; ++k) {
    Level& lv = h.levels[k];
    launch_rs_diag(lv, s);
    launch_rs_sell_values(lv, s);
    if (h.mixed()) launch_to_float(lv.nnz, lv.val, lv.val32, s);
  }
  sy.wait_and_check();
  for (int k = 0; k < L; ++k) {
    Level& lv = h.levels[k];
    const int m = std::min(o.arnoldi_m, lv.n);
    Arena at;
    double* Q = at.alloc_n<double>((size_t)(m + 1) * lv.n);
    double* w = at.alloc_n<double>(lv.n);
    double Hh[48], wn[8];
    arnoldi(h, lv, m, o.seed + 1, Q, w, Hh, wn);
    set_jacobi_weight(h, lv, m, Hh, wn);
  }
  coarse_inverse(h, tmp, sy);
  sy.wait_and_check();
  if (repoint) h.multi.reset();   // the kept block workspace's graphs read level 0's old values
  if (repoint && !h.g_iter.empty()) {
    for (auto& g : h.g_iter) (void)hipGraphExecDestroy(g);
    h.g_iter.clear();
    if (h.g_restart) (void)hipGraphExecDestroy(h.g_restart);
    h.g_restart = nullptr;
    build_solve_graphs(h);
  }
}


// ---------------------------------------------------------------- batches
// Algorithm 1 for independent systems on the block diagonal, each coarsened
// as if alone: the node hash takes the row index local to the system, each
// system stops by the rule of Algorithm 1 applied to its own size and
// coarsening ratio, and its Jacobi weight comes from its own Arnoldi
// estimate.  A system that stops on level k keeps its rows there (with a zero
// smoother weight and no aggregate) and is solved by its dense inverse.
void build_batch_hierarchy(Hierarchy& h, const amg_csr& A, const int* sys_off) {
  hipStream_t s = h.stream;
  const amg_options& o = h.opt;
  const int nsys = h.nsys;
  Sync sy{h};
  Arena tmp;
  struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
  init_scan(h.scan, h.arena, std::max(A.n, A.nnz), s);
  batch_control(h);   // per-system scalars and block partials, used from the first Arnoldi on

  Level l0;
  l0.n = A.n;
  l0.nnz = A.nnz;
  l0.rp = h.arena.alloc_n<int>(A.n + 1);
  l0.ci = h.arena.alloc_n<int>(A.nnz);
  l0.val = h.arena.alloc_n<double>(A.nnz);
  AMG_HIP(hipMemcpyAsync(l0.rp, A.row_ptr, (A.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipMemcpyAsync(l0.ci, A.col_idx, (size_t)A.nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipMemcpyAsync(l0.val, A.val, (size_t)A.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  sy.fetch(l0.rp, 0);
  sy.fetch(l0.rp + A.n, 1);
  sy.wait_and_check();
  if (sy.hp()[0] != 0 || sy.hp()[1] != A.nnz) throw Error(AMG_EINVAL, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  launch_check_rowptr(l0.n, l0.rp, h.d_err, s);
  sy.wait_and_check();
  launch_check_matrix(l0.n, l0.rp, l0.ci, l0.val, h.d_err, s);
  l0.sys_off.assign(sys_off, sys_off + nsys + 1);
  batch_blocks(h, l0);
  batch_check_blocks(l0, h.d_err, s);
  l0.B = h.arena.alloc_n<double>(A.n);
  launch_fill_double(A.n, l0.B, 1.0, s);
  h.levels.push_back(l0);
  sy.wait_and_check();

  const bool debug = std::getenv("AMG_DEBUG") != nullptr;
  std::vector<int> term_level(nsys, -1);
  std::vector<int> hroot(nsys + 1), cont(nsys), shift(nsys);
  std::vector<double> Hs((size_t)64 * nsys), omega(nsys);
  int* d_sysint = tmp.alloc_n<int>(2 * (size_t)nsys + 1);
  double* d_omega = tmp.alloc_n<double>(nsys);
  while (true) {
    const int k = (int)h.levels.size() - 1;
    Level& lv = h.levels[k];
    const int n = lv.n, nnz = lv.nnz;
    lv.diag = h.arena.alloc_n<double>(n);
    lv.lpr = pick_lanes_per_row(n, nnz);
    batch_build_sell(h, tmp, lv);
    std::vector<int> present(nsys), size_term(nsys);
    bool any_cont = false;
    for (int q = 0; q < nsys; ++q) {
      const int ns = lv.sys_off[q + 1] - lv.sys_off[q];
      present[q] = ns > 0;
      size_term[q] = present[q] && (ns <= o.coarse_max || k + 1 >= o.max_levels);
      any_cont |= present[q] && !size_term[q];
    }
    if (!any_cont) break;

    // strength, strong graph, MIS(2) with per-system priorities
    lv.strong = h.arena.alloc_n<uint8_t>(nnz);
    launch_strength(n, nnz, lv.rp, lv.ci, lv.val, o.strength_alpha, lv.strong, lv.diag, s);
    uint8_t* gmask = tmp.alloc_n<uint8_t>(nnz);
    int* gdeg = tmp.alloc_n<int>(n);
    int* cnt = tmp.alloc_n<int>(n);
    launch_graph_count(n, nnz, lv.rp, lv.ci, lv.strong, gmask, gdeg, cnt, h.d_err, s);
    int* gptr = tmp.alloc_n<int>(n + 1);
    scan_to_ptr(gdeg, gptr, n, h.scan, s);
    sy.fetch(gptr + n, 0);
    sy.wait_and_check();
    const int nnzg = sy.hp()[0];
    int* gcol = tmp.alloc_n<int>(nnzg > 0 ? nnzg : 1);
    launch_graph_fill(n, nnz, lv.rp, lv.ci, gmask, gptr, gcol, s);
    int* lbase = tmp.alloc_n<int>(n);
    batch_local_base(lv, lbase, s);
    lv.tuple = h.arena.alloc_n<uint64_t>(n);
    uint64_t* M1 = tmp.alloc_n<uint64_t>(n);
    launch_mis_init(n, cnt, o.seed, lv.tuple, M1, h.d_mis, h.d_err, s, lbase);
    int round = 0;
    int batch = 8;
    const int glanes = group_lanes(n, nnzg);
    while (true) {
      for (int b = 0; b < batch; ++b, ++round)
        launch_mis_round(n, gptr, gcol, lv.tuple, M1, h.d_mis, round, glanes, s);
      sy.fetch(h.d_mis + mis_word(round & 1, 0), 0, kMisSlots, mis_word(0, 1));
      sy.fetch(h.d_mis + kMisRoundsWord, 1);
      sy.wait_and_check();
      if (sy.hp()[0] == 0) break;
      if (round > 4096) throw Error(AMG_ECOARSEN, "MIS(2) rounds did not terminate");
      batch = 4;
    }
    lv.mis_rounds = sy.hp()[1];

    // roots per system; a system whose coarsening stalls stops here
    int* flags = tmp.alloc_n<int>(n);
    int* root_id = tmp.alloc_n<int>(n + 1);
    launch_root_flags(n, lv.tuple, flags, s);
    scan_to_ptr(flags, root_id, n, h.scan, s);
    batch_gather(nsys + 1, root_id, lv.d_sys_off, d_sysint, s);
    AMG_HIP(hipMemcpyAsync(hroot.data(), d_sysint, (nsys + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    sy.wait_and_check();
    std::vector<int> next_off(nsys + 1, 0);
    int nc = 0;
    bool any_c = false;
    for (int q = 0; q < nsys; ++q) {
      const int ns = lv.sys_off[q + 1] - lv.sys_off[q];
      const int ncs = hroot[q + 1] - hroot[q];
      const bool stop = present[q] && (size_term[q] || ncs <= 0 || ncs > 0.9 * ns);
      cont[q] = present[q] && !stop ? 1 : 0;
      if (stop) {
        lv.term.push_back(q);
        term_level[q] = k;
      }
      next_off[q] = nc;
      shift[q] = hroot[q] - nc;
      if (cont[q]) nc += ncs;
      any_c |= cont[q] != 0;
    }
    next_off[nsys] = nc;
    if (!any_c) {   // every remaining system stops here: this is the coarsest level
      lv.term.clear();
      for (int q = 0; q < nsys; ++q)
        if (term_level[q] == k) term_level[q] = -1;
      lv.strong = nullptr;
      lv.tuple = nullptr;
      break;
    }
    AMG_HIP(hipMemcpyAsync(d_sysint, cont.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(d_sysint + nsys, shift.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
    int* choice = tmp.alloc_n<int>(n);
    lv.agg = h.arena.alloc_n<int>(n);
    launch_aggregate(n, nnzg, gptr, gcol, lv.tuple, root_id, choice, lv.agg, h.d_err, s);
    batch_remap_agg(lv, d_sysint, d_sysint + nsys, lv.agg, s);
    lv.nc = nc;
    lv.agg_ptr = h.arena.alloc_n<int>(nc + 1);
    lv.agg_rows = h.arena.alloc_n<int>(n);
    build_segments(h, tmp, n, nc, lv.agg, lv.agg_ptr, lv.agg_rows);

    Level lc;
    lc.n = nc;
    lc.B = h.arena.alloc_n<double>(nc);
    lv.pval = h.arena.alloc_n<double>(n);
    launch_interp(n, nc, lv.agg, lv.agg_ptr, lv.agg_rows, lv.B, lc.B, lv.pval, s);
    lv.nr = 0;
    for (int q = 0; q < nsys; ++q)
      if (cont[q]) lv.nr += lv.sys_off[q + 1] - lv.sys_off[q];
    lv.rval = h.arena.alloc_n<double>(std::max(lv.nr, 1));
    launch_gather_double(lv.nr, lv.agg_rows, lv.pval, lv.rval, s);
    lv.rlpr = pick_lanes_per_row(nc, lv.nr);
    galerkin_product(h, tmp, h.arena, lv, nc, lv.agg, lv.pval, lv.agg_ptr, lv.agg_rows, &lc.rp, &lc.ci,
                     &lc.val, &lc.nnz);

    // per-system damped Jacobi weight
    int m = 0;
    for (int q = 0; q < nsys; ++q)
      if (cont[q]) m = std::max(m, std::min(o.arnoldi_m, lv.sys_off[q + 1] - lv.sys_off[q]));
    double* Q = tmp.alloc_n<double>((size_t)(m + 1) * n);
    double* w = tmp.alloc_n<double>(n);
    AMG_HIP(hipMemcpyAsync(d_sysint, cont.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
    batch_arnoldi(h, lv, m, o.seed + 1, d_sysint, Q, w, Hs.data());
    lv.sys_omega.assign(nsys, 0.0);
    lv.sys_rho.assign(nsys, 0.0);
    for (int q = 0; q < nsys; ++q) {
      omega[q] = 0.0;
      if (!cont[q]) continue;
      const double* Hq = Hs.data() + (size_t)q * 64;
      const int mq = std::min(o.arnoldi_m, lv.sys_off[q + 1] - lv.sys_off[q]);
      int size = mq;
      for (int j = 0; j < mq; ++j) {
        if (Hq[(j + 1) * 8 + j] <= 1e-14 * Hq[48 + j]) { size = j + 1; break; }
      }
      double Hsq[64];
      for (int i = 0; i < size; ++i)
        for (int j = 0; j < size; ++j) Hsq[i * size + j] = i <= j + 1 ? Hq[i * 8 + j] : 0.0;
      const double rho = hessenberg_spectral_radius(Hsq, size);
      if (!(rho > 0.0) || !std::isfinite(rho))
        throw Error(AMG_EBREAKDOWN, "spectral radius estimate not positive (system " + std::to_string(q) + ")");
      lv.sys_rho[q] = rho;
      omega[q] = lv.sys_omega[q] = o.jacobi_scale / rho;
    }
    AMG_HIP(hipMemcpyAsync(d_omega, omega.data(), nsys * sizeof(double), hipMemcpyHostToDevice, s));
    lv.wdinv = h.arena.alloc_n<double>(n);
    if (h.mixed()) lv.wdinv32 = h.arena.alloc_n<float>(n);
    batch_jacobi_weights(lv, d_omega, lv.wdinv, lv.wdinv32, s);
    sy.wait_and_check();   // pageable host sources above stay valid until here
    if (debug)
      std::fprintf(stderr, "amg batch: level %d n=%d nnz=%d mis_rounds=%d nc=%d stop=%zu\n", k, n, nnz,
                   lv.mis_rounds, nc, lv.term.size());
    lc.sys_off = next_off;
    h.levels.push_back(lc);
    batch_blocks(h, h.levels.back());
  }

  // the coarsest level: every system present there stops
  const int L = (int)h.levels.size() - 1;
  {
    Level& cl = h.levels[L];
    for (int q = 0; q < nsys; ++q)
      if (cl.sys_off[q + 1] > cl.sys_off[q]) {
        cl.term.push_back(q);
        term_level[q] = L;
      }
  }
  // dense inverses of the systems stopping on each level
  for (int k = 0; k <= L; ++k) {
    Level& lv = h.levels[k];
    if (lv.term.empty()) continue;
    std::vector<TermInfo> ti;
    std::vector<int> tb;
    long long off = 0;
    for (size_t t = 0; t < lv.term.size(); ++t) {
      const int q = lv.term[t];
      const int ns = lv.sys_off[q + 1] - lv.sys_off[q];
      if (ns > o.dense_max)
        throw Error(AMG_ECOARSEN, "system " + std::to_string(q) + " stops with " + std::to_string(ns) + " unknowns");
      ti.push_back(TermInfo{q, lv.sys_off[q], ns, 0, off});
      off += (long long)ns * ns;
      for (int r = 0; r < ns; r += kBlockRowsGemv) {
        tb.push_back((int)t);
        tb.push_back(r);
      }
    }
    const int nt = (int)ti.size();
    lv.d_term = h.arena.alloc_n<TermInfo>(nt);
    lv.tblk = h.arena.alloc_n<int>(tb.size());
    lv.ntblk = (int)(tb.size() / 2);
    lv.tinv = h.arena.alloc_n<double>((size_t)off);
    if (h.mixed()) lv.tinv32 = h.arena.alloc_n<float>((size_t)off);
    AMG_HIP(hipMemcpyAsync(lv.d_term, ti.data(), nt * sizeof(TermInfo), hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(lv.tblk, tb.data(), tb.size() * sizeof(int), hipMemcpyHostToDevice, s));
    Arena work;
    launch_dense_inverse_spd(nt, lv.d_term, ti.data(), lv.n, lv.rp, lv.ci, lv.val, lv.tinv, lv.tinv32, work,
                             h.d_err, s);
    if (sy.take_not_spd()) {   // some system is not SPD: eliminate all of them with pivoting
      double* wk = work.alloc_n<double>(2 * (size_t)off);
      int* piv = work.alloc_n<int>(lv.n);
      launch_dense_inverse_batched(lv, nt, lv.d_term, ti.data(), wk, piv, lv.tinv, lv.tinv32, h.d_err, s);
    }
    sy.wait_and_check();
  }
  // K-cycle levels: a system takes the K-cycle on level k when its next level
  // is not its coarsest (as the single-system cycle does)
  for (int k = 0; k < L && k < o.kcycle_levels; ++k) {
    Level& lv = h.levels[k];
    const Level& lc = h.levels[k + 1];
    std::vector<int> kv(nsys, 0);
    for (int q = 0; q < nsys; ++q) {
      kv[q] = (lc.sys_off[q + 1] > lc.sys_off[q] && term_level[q] > k + 1) ? 1 : 0;
      lv.kcyc |= kv[q];
    }
    lv.kv = h.arena.alloc_n<int>(nsys);
    AMG_HIP(hipMemcpyAsync(lv.kv, kv.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
    sy.wait_and_check();
  }
  if (h.mixed()) make_float_copies(h);
  alloc_solve_vectors(h);
  sy.wait_and_check();
  if (!(o.flags & AMG_FLAG_NO_GRAPH)) build_batch_graphs(h);
}

}  // namespace amg
