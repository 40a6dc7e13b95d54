// extern "C" entry points declared in include/amg.h.  Argument checks on the
// host, then the internal runtime; no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "amg_internal.hpp"

struct amg_hierarchy {
  amg::Hierarchy h;
};

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const std::string& msg) {
  g_last_error = msg;
  if (std::getenv("AMG_VERBOSE")) std::fprintf(stderr, "amg: %s\n", msg.c_str());
  return code;
}

int32_t run_guarded(const char* where, void (*fn)(void*), void* ctx) {
  try {
    fn(ctx);
    return AMG_OK;
  } catch (const amg::Error& e) {
    return fail(e.code, std::string(where) + ": " + e.what());
  } catch (const std::bad_alloc&) {
    return fail(AMG_ENOMEM, std::string(where) + ": host allocation failed");
  } catch (const std::exception& e) {
    return fail(AMG_EHIP, std::string(where) + ": " + e.what());
  }
}

template <class F>
int32_t guarded(const char* where, F&& f) {
  return run_guarded(where, [](void* c) { (*static_cast<F*>(c))(); }, &f);
}

bool csr_args_ok(const amg_csr* A) {
  return A && A->n > 0 && A->nnz >= A->n && A->row_ptr && A->col_idx && A->val;
}

}  // namespace

extern "C" {

void amg_default_options(amg_options* opt, int32_t dim) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->strength_alpha = dim == 2 ? 0.25 : 0.5;
  opt->coarse_max = 600;
  opt->max_levels = 20;
  opt->kcycle_levels = 2;
  opt->kcycle_t = 0.25;
  opt->jacobi_scale = 4.0 / 3.0;
  opt->arnoldi_m = 5;
  opt->seed = 0;
  opt->krylov = AMG_KRYLOV_FCG;
  opt->gmres_restart = 30;
  opt->precision = AMG_PREC_FP64;
  opt->smoother = AMG_SMOOTHER_JACOBI;
  opt->max_iter = 200;
  opt->dense_max = 4096;
  opt->probe = AMG_PROBE_NONE;
  opt->check_every = 16;
  opt->flags = 0;
  opt->mlp_weights = nullptr;
  opt->mis_k = 2;
  opt->cheb_degree = 2;
  opt->cheb_ratio = 4.0;
  opt->cheb_upper = 1.1;
}

const char* amg_status_string(int32_t status) {
  switch (status) {
    case AMG_OK: return "AMG_OK";
    case AMG_EINVAL: return "AMG_EINVAL: invalid argument or matrix";
    case AMG_ENOMEM: return "AMG_ENOMEM: allocation failed";
    case AMG_EHIP: return "AMG_EHIP: HIP runtime error";
    case AMG_ENOTCONV: return "AMG_ENOTCONV: iteration limit reached";
    case AMG_EBREAKDOWN: return "AMG_EBREAKDOWN: breakdown";
    case AMG_ECOARSEN: return "AMG_ECOARSEN: coarsening failed";
    case AMG_ENANINF: return "AMG_ENANINF: non-finite value";
    case AMG_EUNSUPPORTED: return "AMG_EUNSUPPORTED: unsupported option";
    default: return "AMG: unknown status";
  }
}

const char* amg_last_error(void) { return g_last_error.c_str(); }

int32_t amg_setup(const amg_csr* A, const amg_options* opt, hipStream_t s, amg_hierarchy** out) {
  if (!out) return fail(AMG_EINVAL, "amg_setup: out is NULL");
  *out = nullptr;
  if (!csr_args_ok(A)) return fail(AMG_EINVAL, "amg_setup: bad matrix descriptor");
  amg_options o;
  if (opt) o = *opt; else amg_default_options(&o, 3);
  if (!(o.strength_alpha >= 0.0) || o.coarse_max < 1 || o.max_levels < 1 || o.kcycle_levels < 0 ||
      o.kcycle_levels > 24 || !(o.kcycle_t >= 0.0) || !(o.jacobi_scale > 0.0) || o.arnoldi_m < 1 ||
      o.arnoldi_m > 5 || o.max_iter < 0 || o.dense_max < 1 || o.dense_max > 8192)
    return fail(AMG_EINVAL, "amg_setup: option out of range");
  if (o.krylov != AMG_KRYLOV_FCG && o.krylov != AMG_KRYLOV_FGMRES) return fail(AMG_EINVAL, "amg_setup: krylov");
  if (o.gmres_restart < 1 || o.gmres_restart > 64) return fail(AMG_EINVAL, "amg_setup: gmres_restart in [1, 64]");
  if (o.precision != AMG_PREC_FP64 && o.precision != AMG_PREC_MIXED)
    return fail(AMG_EINVAL, "amg_setup: unknown precision");
  if (o.smoother != AMG_SMOOTHER_JACOBI && o.smoother != AMG_SMOOTHER_LEARNED &&
      o.smoother != AMG_SMOOTHER_CHEBYSHEV && o.smoother != AMG_SMOOTHER_MCSGS)
    return fail(AMG_EINVAL, "amg_setup: smoother");
  if (o.smoother == AMG_SMOOTHER_CHEBYSHEV &&
      (o.cheb_degree < 1 || o.cheb_degree > 8 || !(o.cheb_ratio > 1.0) || !(o.cheb_upper > 0.0) ||
       !std::isfinite(o.cheb_ratio) || !std::isfinite(o.cheb_upper)))
    return fail(AMG_EINVAL, "amg_setup: Chebyshev degree in [1, 8], ratio > 1, upper > 0");
  if (o.smoother == AMG_SMOOTHER_LEARNED && !o.mlp_weights)
    return fail(AMG_EINVAL, "amg_setup: the learned smoother needs mlp_weights");
  if (o.probe < AMG_PROBE_NONE || o.probe > AMG_PROBE_OUTER_SPMV) return fail(AMG_EINVAL, "amg_setup: probe");
  if (o.mis_k < 2 || o.mis_k > 8) return fail(AMG_EINVAL, "amg_setup: mis_k in [2, 8]");
  auto* H = new (std::nothrow) amg_hierarchy();
  if (!H) return fail(AMG_ENOMEM, "amg_setup: host allocation");
  int32_t st = guarded("amg_setup", [&] {
    amg::Hierarchy& h = H->h;
    h.opt = o;
    h.stream = s;
    for (auto& e : h.ev) AMG_HIP(hipEventCreate(&e));
    AMG_HIP(hipEventRecord(h.ev[0], s));
    amg::init_control(h);
    amg::build_hierarchy(h, *A);
    AMG_HIP(hipEventRecord(h.ev[1], s));
    AMG_HIP(hipEventSynchronize(h.ev[1]));
    AMG_HIP(hipEventElapsedTime(&h.setup_ms, h.ev[0], h.ev[1]));
  });
  if (st != AMG_OK) {
    delete H;
    return st;
  }
  *out = H;
  return AMG_OK;
}

int32_t amg_setup_batched(const amg_csr* A, int32_t nsys, const int32_t* sys_off, const amg_options* opt,
                          hipStream_t s, amg_hierarchy** out) {
  if (!out) return fail(AMG_EINVAL, "amg_setup_batched: out is NULL");
  *out = nullptr;
  if (!csr_args_ok(A)) return fail(AMG_EINVAL, "amg_setup_batched: bad matrix descriptor");
  if (nsys < 1 || nsys > A->n || !sys_off) return fail(AMG_EINVAL, "amg_setup_batched: nsys or sys_off");
  if (sys_off[0] != 0 || sys_off[nsys] != A->n)
    return fail(AMG_EINVAL, "amg_setup_batched: sys_off must run from 0 to n");
  for (int32_t q = 0; q < nsys; ++q)
    if (sys_off[q + 1] <= sys_off[q]) return fail(AMG_EINVAL, "amg_setup_batched: empty or decreasing system");
  amg_options o;
  if (opt) o = *opt; else amg_default_options(&o, 2);
  if (!(o.strength_alpha >= 0.0) || o.coarse_max < 1 || o.max_levels < 1 || o.kcycle_levels < 0 ||
      o.kcycle_levels > 24 || !(o.kcycle_t >= 0.0) || !(o.jacobi_scale > 0.0) || o.arnoldi_m < 1 ||
      o.arnoldi_m > 5 || o.max_iter < 0 || o.dense_max < 1 || o.dense_max > 8192)
    return fail(AMG_EINVAL, "amg_setup_batched: option out of range");
  if (o.precision != AMG_PREC_FP64 && o.precision != AMG_PREC_MIXED)
    return fail(AMG_EINVAL, "amg_setup_batched: unknown precision");
  if (o.krylov != AMG_KRYLOV_FCG) return fail(AMG_EUNSUPPORTED, "amg_setup_batched: batches use flexible CG");
  if (o.smoother != AMG_SMOOTHER_JACOBI)
    return fail(AMG_EUNSUPPORTED, "amg_setup_batched: batches use the damped Jacobi smoother");
  if (o.probe != AMG_PROBE_NONE) return fail(AMG_EUNSUPPORTED, "amg_setup_batched: no kernel probe in batches");
  if (o.mis_k != 2) return fail(AMG_EUNSUPPORTED, "amg_setup_batched: batches use MIS(2)");
  auto* H = new (std::nothrow) amg_hierarchy();
  if (!H) return fail(AMG_ENOMEM, "amg_setup_batched: host allocation");
  int32_t st = guarded("amg_setup_batched", [&] {
    amg::Hierarchy& h = H->h;
    h.opt = o;
    h.stream = s;
    h.nsys = nsys;
    for (auto& e : h.ev) AMG_HIP(hipEventCreate(&e));
    AMG_HIP(hipEventRecord(h.ev[0], s));
    amg::init_control(h);
    amg::build_batch_hierarchy(h, *A, sys_off);
    AMG_HIP(hipEventRecord(h.ev[1], s));
    AMG_HIP(hipEventSynchronize(h.ev[1]));
    AMG_HIP(hipEventElapsedTime(&h.setup_ms, h.ev[0], h.ev[1]));
  });
  if (st != AMG_OK) {
    delete H;
    return st;
  }
  *out = H;
  return AMG_OK;
}

int32_t amg_level_format(const amg_hierarchy* H, int32_t k, int32_t precision, int32_t* format,
                         int32_t* lanes_per_row, float* us) {
  if (!H || k < 0 || k + 1 >= (int32_t)H->h.levels.size() || !format || !lanes_per_row)
    return fail(AMG_EINVAL, "amg_level_format: bad argument");
  if (precision != AMG_PREC_FP64 && precision != AMG_PREC_MIXED) return fail(AMG_EINVAL, "amg_level_format: precision");
  const amg::Level& lv = H->h.levels[k];
  const amg::Level::Tune& t = precision == AMG_PREC_FP64 ? lv.t64 : lv.t32;
  *format = t.fmt;
  *lanes_per_row = t.fmt == 0 || t.fmt == 4 ? t.lpr : t.fmt == 3 ? 1 : 64 / (t.sh > 0 ? t.sh : 64);   // sliced: 64 / slice height
  if (us) *us = t.us;
  return AMG_OK;
}

int32_t amg_level_spmv(const amg_hierarchy* H, int32_t k, const double* x, double* y, hipStream_t s) {
  if (!H || k < 0 || k >= (int32_t)H->h.levels.size() || !x || !y) return fail(AMG_EINVAL, "amg_level_spmv: bad argument");
  return guarded("amg_level_spmv", [&] {
    amg::level_spmv(H->h, k, x, y, s);
    AMG_HIP(hipGetLastError());
  });
}

int32_t amg_batch_results(const amg_hierarchy* H, int32_t* iters, double* relres) {
  if (!H || H->h.nsys == 0) return fail(AMG_EINVAL, "amg_batch_results: not a batched hierarchy");
  if (H->h.b_iters.empty()) return fail(AMG_EINVAL, "amg_batch_results: no solve yet");
  for (int q = 0; q < H->h.nsys; ++q) {
    if (iters) iters[q] = H->h.b_iters[q];
    if (relres) relres[q] = H->h.b_relres[q];
  }
  return AMG_OK;
}

int32_t amg_batch_level(const amg_hierarchy* H, int32_t k, int32_t* sys_off, double* omega) {
  if (!H || H->h.nsys == 0) return fail(AMG_EINVAL, "amg_batch_level: not a batched hierarchy");
  if (k < 0 || k >= (int32_t)H->h.levels.size()) return fail(AMG_EINVAL, "amg_batch_level: level");
  const amg::Level& lv = H->h.levels[k];
  for (int q = 0; q <= H->h.nsys; ++q)
    if (sys_off) sys_off[q] = lv.sys_off[q];
  for (int q = 0; q < H->h.nsys; ++q)
    if (omega) omega[q] = lv.sys_omega.empty() ? 0.0 : lv.sys_omega[q];
  return AMG_OK;
}

int32_t amg_resetup(amg_hierarchy* H, const double* val, hipStream_t s) {
  if (!H || !val) return fail(AMG_EINVAL, "amg_resetup: NULL argument");
  amg::Hierarchy& h = H->h;
  if (h.nsys > 0) return fail(AMG_EUNSUPPORTED, "amg_resetup: batched hierarchy");
  if (h.opt.smoother == AMG_SMOOTHER_LEARNED) return fail(AMG_EUNSUPPORTED, "amg_resetup: learned smoother");
  return guarded("amg_resetup", [&] {
    h.stream = s;
    AMG_HIP(hipEventRecord(h.ev[0], s));
    amg::resetup_hierarchy(h, val);
    AMG_HIP(hipEventRecord(h.ev[1], s));
    AMG_HIP(hipEventSynchronize(h.ev[1]));
    AMG_HIP(hipEventElapsedTime(&h.resetup_ms, h.ev[0], h.ev[1]));
  });
}

int32_t amg_solve(amg_hierarchy* H, const double* b, double rtol, double* x, int32_t* iters, double* relres,
                  hipStream_t s) {
  if (!H || !b || !x || !iters || !relres) return fail(AMG_EINVAL, "amg_solve: NULL argument");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(AMG_EINVAL, "amg_solve: rtol must be positive");
  int32_t status = AMG_OK;
  int32_t st = guarded("amg_solve", [&] {
    amg::Hierarchy& h = H->h;
    h.stream = s;
    AMG_HIP(hipEventRecord(h.ev[2], s));
    int it = 0;
    double rel = 0.0;
    if (h.nsys > 0) {
      h.b_iters.assign(h.nsys, 0);
      h.b_relres.assign(h.nsys, 0.0);
      status = amg::solve_batch_impl(h, b, rtol, x, h.b_iters.data(), h.b_relres.data());
      for (int q = 0; q < h.nsys; ++q) {
        it = std::max(it, h.b_iters[q]);
        rel = std::max(rel, h.b_relres[q]);
      }
    } else {
      status = amg::solve_fcg_impl(h, b, rtol, x, &it, &rel);
    }
    AMG_HIP(hipEventRecord(h.ev[3], s));
    AMG_HIP(hipEventSynchronize(h.ev[3]));
    AMG_HIP(hipEventElapsedTime(&h.solve_ms, h.ev[2], h.ev[3]));
    *iters = it;
    *relres = rel;
  });
  if (st != AMG_OK) return st;
  if (status != AMG_OK) return fail(status, "amg_solve: iteration limit reached");
  return AMG_OK;
}

int32_t amg_solve_multi(amg_hierarchy* H, int32_t nrhs, const double* B, double rtol, double* X, int32_t* iters,
                        double* relres, hipStream_t s) {
  if (!H || !B || !X || !iters || !relres) return fail(AMG_EINVAL, "amg_solve_multi: NULL argument");
  if (nrhs < 1 || nrhs > 64) return fail(AMG_EINVAL, "amg_solve_multi: nrhs must be in [1, 64]");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(AMG_EINVAL, "amg_solve_multi: rtol must be positive");
  if (H->h.nsys > 0) return fail(AMG_EUNSUPPORTED, "amg_solve_multi: batched hierarchy");
  if (H->h.opt.smoother == AMG_SMOOTHER_CHEBYSHEV || H->h.opt.smoother == AMG_SMOOTHER_MCSGS)
    return fail(AMG_EUNSUPPORTED, "amg_solve_multi: the block cycle smooths by Jacobi only");
  int32_t status = AMG_OK;
  int32_t st = guarded("amg_solve_multi", [&] {
    amg::Hierarchy& h = H->h;
    h.stream = s;
    AMG_HIP(hipEventRecord(h.ev[2], s));
    status = amg::solve_multi_impl(h, nrhs, B, rtol, X, iters, relres);
    AMG_HIP(hipEventRecord(h.ev[3], s));
    AMG_HIP(hipEventSynchronize(h.ev[3]));
    AMG_HIP(hipEventElapsedTime(&h.solve_ms, h.ev[2], h.ev[3]));
  });
  if (st != AMG_OK) return st;
  if (status != AMG_OK) return fail(status, "amg_solve_multi: a column reached the iteration limit");
  return AMG_OK;
}

void amg_destroy(amg_hierarchy* H) { delete H; }

size_t amg_release_cached_memory(void) {
  try {
    return amg::release_cached_chunks();
  } catch (...) {
    return 0;
  }
}

int32_t amg_num_levels(const amg_hierarchy* H) { return H ? (int32_t)H->h.levels.size() : 0; }

int32_t amg_level_info(const amg_hierarchy* H, int32_t k, int32_t* n, int32_t* nnz, double* omega,
                       int32_t* n_coarse, int32_t* mis_rounds) {
  if (!H || k < 0 || k >= (int32_t)H->h.levels.size()) return fail(AMG_EINVAL, "amg_level_info: level");
  const amg::Level& lv = H->h.levels[k];
  const bool coarsest = k == (int32_t)H->h.levels.size() - 1;
  if (n) *n = lv.n;
  if (nnz) *nnz = lv.nnz;
  if (omega) *omega = coarsest ? 0.0 : lv.omega;
  if (n_coarse) *n_coarse = coarsest ? 0 : lv.nc;
  if (mis_rounds) *mis_rounds = coarsest ? 0 : lv.mis_rounds;
  return AMG_OK;
}

int32_t amg_export_level(const amg_hierarchy* H, int32_t k, int32_t* row_ptr, int32_t* col_idx, double* val,
                         uint8_t* strong, int8_t* state, int32_t* agg, double* pval, double* B) {
  if (!H || k < 0 || k >= (int32_t)H->h.levels.size()) return fail(AMG_EINVAL, "amg_export_level: level");
  const amg::Hierarchy& h = H->h;
  const amg::Level& lv = h.levels[k];
  const bool coarsest = k == (int32_t)h.levels.size() - 1;
  if (coarsest && (strong || state || agg || pval))
    return fail(AMG_EINVAL, "amg_export_level: the coarsest level has no aggregation");
  return guarded("amg_export_level", [&] {
    hipStream_t s = h.stream;
    if (row_ptr) AMG_HIP(hipMemcpyAsync(row_ptr, lv.rp, (lv.n + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    if (col_idx) AMG_HIP(hipMemcpyAsync(col_idx, lv.ci, (size_t)lv.nnz * sizeof(int), hipMemcpyDeviceToHost, s));
    if (val) AMG_HIP(hipMemcpyAsync(val, lv.val, (size_t)lv.nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    if (strong) AMG_HIP(hipMemcpyAsync(strong, lv.strong, (size_t)lv.nnz, hipMemcpyDeviceToHost, s));
    if (agg) AMG_HIP(hipMemcpyAsync(agg, lv.agg, (size_t)lv.n * sizeof(int), hipMemcpyDeviceToHost, s));
    if (pval) AMG_HIP(hipMemcpyAsync(pval, lv.pval, (size_t)lv.n * sizeof(double), hipMemcpyDeviceToHost, s));
    if (B) AMG_HIP(hipMemcpyAsync(B, lv.B, (size_t)lv.n * sizeof(double), hipMemcpyDeviceToHost, s));
    if (state) {
      int8_t* dst = nullptr;
      AMG_HIP(hipMallocAsync((void**)&dst, lv.n, s));
      amg::launch_state_from_tuple(lv.n, lv.tuple, dst, s);
      AMG_HIP(hipMemcpyAsync(state, dst, lv.n, hipMemcpyDeviceToHost, s));
      AMG_HIP(hipFreeAsync(dst, s));
    }
    AMG_HIP(hipStreamSynchronize(s));
  });
}

int32_t amg_spmv(const amg_csr* A, const double* x, double* y, int32_t lanes_per_row, hipStream_t s) {
  if (!csr_args_ok(A) || !x || !y) return fail(AMG_EINVAL, "amg_spmv: bad argument");
  if (lanes_per_row == -1 || lanes_per_row == -2) {
    return guarded("amg_spmv", [&] {
      amg::Hierarchy h;
      h.stream = s;
      amg::init_control(h);
      amg::init_scan(h.scan, h.arena, A->n, s);
      amg::spmv_sell_f64(h, *A, x, y, lanes_per_row == -2);
    });
  }
  if (lanes_per_row < 0 || lanes_per_row > 64 || (lanes_per_row & (lanes_per_row - 1)))
    return fail(AMG_EINVAL, "amg_spmv: lanes_per_row must be -2, -1, 0 or a power of two <= 64");
  return guarded("amg_spmv", [&] {
    amg::spmv_f64(A->n, A->nnz, A->row_ptr, A->col_idx, A->val, x, y, lanes_per_row, s);
    AMG_HIP(hipGetLastError());
  });
}

int32_t amg_node_hash(int32_t n, uint32_t stream, uint32_t* out, hipStream_t s) {
  if (n < 0 || (n > 0 && !out)) return fail(AMG_EINVAL, "amg_node_hash: bad argument");
  return guarded("amg_node_hash", [&] {
    amg::launch_node_hash(n, stream, out, s);
    AMG_HIP(hipGetLastError());
  });
}

int32_t amg_galerkin(const amg_csr* A, const int32_t* agg, const double* pval, int32_t nc, int32_t* nnz_c,
                     int32_t* row_ptr_c, int32_t* col_c, double* val_c, int32_t cap, hipStream_t s) {
  if (!csr_args_ok(A) || !agg || !pval || nc < 1 || nc > A->n || !nnz_c)
    return fail(AMG_EINVAL, "amg_galerkin: bad argument");
  int32_t too_small = 0;
  int32_t st = guarded("amg_galerkin", [&] {
    amg::Hierarchy h;
    h.stream = s;
    h.opt.dense_max = 1;
    amg::init_control(h);
    amg::init_scan(h.scan, h.arena, A->nnz > A->n ? A->nnz : A->n, s);
    int *rp = nullptr, *ci = nullptr;
    double* v = nullptr;
    int nz = 0;
    amg::galerkin_standalone(h, *A, agg, pval, nc, &nz, &rp, &ci, &v);
    *nnz_c = nz;
    if (cap < nz || !row_ptr_c || !col_c || !val_c) {
      too_small = 1;
      return;
    }
    AMG_HIP(hipMemcpyAsync(row_ptr_c, rp, (nc + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(col_c, ci, (size_t)nz * sizeof(int), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(val_c, v, (size_t)nz * sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
  });
  if (st != AMG_OK) return st;
  if (too_small) return fail(AMG_EINVAL, "amg_galerkin: output capacity too small");
  return AMG_OK;
}

int32_t amg_galerkin_noalloc(const amg_csr* A, const int32_t* agg, const double* pval, int32_t nc,
                             int32_t* row_ptr_c, int32_t* col_c, double* val_c, int32_t cap, int32_t* nnz_c,
                             hipStream_t s) {
  if (!csr_args_ok(A) || !agg || !pval || nc < 1 || nc > A->n || !nnz_c || !row_ptr_c || cap < 0 ||
      (cap > 0 && (!col_c || !val_c)))
    return fail(AMG_EINVAL, "amg_galerkin_noalloc: bad argument");
  int32_t code = AMG_OK;
  int32_t st = guarded("amg_galerkin_noalloc", [&] {
    code = amg::galerkin_noalloc(*A, agg, pval, nc, row_ptr_c, col_c, val_c, cap, nnz_c, s);
  });
  if (st != AMG_OK) return st;
  if (code != AMG_OK) return fail(code, "amg_galerkin_noalloc: output capacity too small");
  return AMG_OK;
}

int32_t amg_hessenberg_radius(const double* H, int32_t m, double* rho) {
  if (!H || !rho || m < 1 || m > 8) return fail(AMG_EINVAL, "amg_hessenberg_radius: bad argument");
  *rho = amg::hessenberg_spectral_radius(H, m);
  return AMG_OK;
}

int32_t amg_timings(const amg_hierarchy* H, double* setup_ms, double* solve_ms) {
  if (!H) return fail(AMG_EINVAL, "amg_timings: NULL hierarchy");
  if (setup_ms) *setup_ms = H->h.setup_ms;
  if (solve_ms) *solve_ms = H->h.solve_ms;
  return AMG_OK;
}

int32_t amg_resetup_time(const amg_hierarchy* H, double* ms) {
  if (!H || !ms) return fail(AMG_EINVAL, "amg_resetup_time: NULL argument");
  *ms = H->h.resetup_ms;
  return AMG_OK;
}

int32_t amg_setup_phases(const amg_hierarchy* H, double* tune_ms, double* capture_ms) {
  if (!H) return fail(AMG_EINVAL, "amg_setup_phases: NULL hierarchy");
  if (tune_ms) *tune_ms = H->h.tune_ms;
  if (capture_ms) *capture_ms = H->h.capture_ms;
  return AMG_OK;
}

int32_t amg_multi_tiles(const amg_hierarchy* H, int32_t nrhs, int32_t* tiles, int32_t cap, double* tune_ms) {
  if (!H || !tiles) return fail(AMG_EINVAL, "amg_multi_tiles: NULL argument");
  const int rc = amg::multi_tiles(H->h, nrhs, tiles, cap, tune_ms);
  if (rc != AMG_OK) return fail(rc, "amg_multi_tiles: no block solve with this column count, or cap too small");
  return AMG_OK;
}

int32_t amg_mlp_num_params(void) { return amg::mlp_num_params(); }

static bool level_ok(const amg_hierarchy* H, int32_t k) {
  return H && k >= 0 && k + 1 < (int32_t)H->h.levels.size();
}

int32_t amg_mlp_features(const amg_hierarchy* H, int32_t k, float* feats, hipStream_t s) {
  if (!level_ok(H, k) || !feats) return fail(AMG_EINVAL, "amg_mlp_features: bad argument");
  if (H->h.nsys > 0) return fail(AMG_EUNSUPPORTED, "amg_mlp_features: batched hierarchy");
  return guarded("amg_mlp_features", [&] {
    amg::Hierarchy& h = const_cast<amg::Hierarchy&>(H->h);
    hipStream_t keep = h.stream;
    h.stream = s;
    amg::mlp_features(h, h.levels[k], k, feats, nullptr);
    h.stream = keep;
    AMG_HIP(hipGetLastError());
  });
}

int32_t amg_mlp_omega(const amg_hierarchy* H, int32_t k, const float* w, double* omega, hipStream_t s) {
  if (!level_ok(H, k) || !w || !omega) return fail(AMG_EINVAL, "amg_mlp_omega: bad argument");
  if (H->h.nsys > 0) return fail(AMG_EUNSUPPORTED, "amg_mlp_omega: batched hierarchy");
  return guarded("amg_mlp_omega", [&] {
    amg::Hierarchy& h = const_cast<amg::Hierarchy&>(H->h);
    hipStream_t keep = h.stream;
    h.stream = s;
    amg::Arena tmp;
    struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
    const amg::Level& lv = h.levels[k];
    float* F = tmp.alloc_n<float>((size_t)lv.n * 9);
    double* beta = tmp.alloc_n<double>(lv.n);
    amg::mlp_features(h, lv, k, F, beta);
    amg::mlp_omega(h, lv, F, beta, w, omega, nullptr, nullptr, nullptr);
    h.stream = keep;
    AMG_HIP(hipGetLastError());
  });
}

int32_t amg_mlp_loss_grad(const amg_hierarchy* H, int32_t k, const float* w, int32_t nsamples, uint32_t seed,
                          const double* extra, int32_t n_extra, double* loss, float* grad, int32_t flags,
                          hipStream_t s) {
  if (!level_ok(H, k) || !w || !loss || nsamples < 0 || n_extra < 0 || (n_extra > 0 && !extra) ||
      nsamples + n_extra < 1 || nsamples + n_extra > 64)
    return fail(AMG_EINVAL, "amg_mlp_loss_grad: bad argument");
  if (H->h.nsys > 0) return fail(AMG_EUNSUPPORTED, "amg_mlp_loss_grad: batched hierarchy");
  return guarded("amg_mlp_loss_grad", [&] {
    amg::Hierarchy& h = const_cast<amg::Hierarchy&>(H->h);
    hipStream_t keep = h.stream;
    h.stream = s;
    amg::Arena tmp;
    struct Drain { hipStream_t s; ~Drain() { (void)hipStreamSynchronize(s); } } drain{s};
    *loss = amg::mlp_loss_grad(h, tmp, h.levels[k], k, w, nsamples, seed, extra, n_extra, nullptr, grad,
                               flags & AMG_MLP_ACCUMULATE, (flags & AMG_MLP_RAW_EXTRA) != 0);
    h.stream = keep;
  });
}

int32_t amg_mlp_coarse_corrected(const amg_hierarchy* H, int32_t k, const double* E, int32_t nsamples,
                                 int32_t cycles, double* out, hipStream_t s) {
  if (!level_ok(H, k) || !E || !out || nsamples < 1 || cycles < 1)
    return fail(AMG_EINVAL, "amg_mlp_coarse_corrected: bad argument");
  if (H->h.nsys > 0) return fail(AMG_EUNSUPPORTED, "amg_mlp_coarse_corrected: batched hierarchy");
  return guarded("amg_mlp_coarse_corrected", [&] {
    amg::Hierarchy& h = const_cast<amg::Hierarchy&>(H->h);
    hipStream_t keep = h.stream;
    h.stream = s;
    struct Restore { amg::Hierarchy& h; hipStream_t s; ~Restore() { h.stream = s; } } restore{h, keep};
    amg::coarse_corrected_errors(h, k, E, nsamples, cycles, out);
  });
}

int32_t amg_mlp_adam(float* w, float* m, float* v, const float* g, int32_t n, int32_t step, float lr, float b1,
                     float b2, float eps, hipStream_t s) {
  if (!w || !m || !v || !g || n < 1 || step < 1) return fail(AMG_EINVAL, "amg_mlp_adam: bad argument");
  return guarded("amg_mlp_adam", [&] {
    amg::mlp_adam(w, m, v, g, n, step, lr, b1, b2, eps, s);
    AMG_HIP(hipGetLastError());
  });
}

int32_t amg_level_smoother(const amg_hierarchy* H, int32_t k, int32_t* learned, double* loss_plain,
                           double* loss_learned) {
  if (!H || k < 0 || k >= (int32_t)H->h.levels.size()) return fail(AMG_EINVAL, "amg_level_smoother: level");
  const amg::Level& lv = H->h.levels[k];
  if (learned) *learned = lv.learned;
  if (loss_plain) *loss_plain = lv.loss_plain;
  if (loss_learned) *loss_learned = lv.loss_learned;
  return AMG_OK;
}

int32_t amg_learned_judge(const amg_hierarchy* H, int32_t* kept, int32_t* iters_plain, double* relres_plain,
                          int32_t* iters_learned, double* relres_learned) {
  if (!H) return fail(AMG_EINVAL, "amg_learned_judge: NULL hierarchy");
  const amg::Hierarchy& h = H->h;
  if (kept) *kept = h.judge_kept;
  if (iters_plain) *iters_plain = h.judge_it_plain;
  if (relres_plain) *relres_plain = h.judge_rel_plain;
  if (iters_learned) *iters_learned = h.judge_it_learned;
  if (relres_learned) *relres_learned = h.judge_rel_learned;
  return AMG_OK;
}

int32_t amg_level_colors(const amg_hierarchy* H, int32_t k, int32_t* colors, int32_t* ncolors) {
  if (!H || k < 0 || k >= (int32_t)H->h.levels.size() - 1) return fail(AMG_EINVAL, "amg_level_colors: level");
  const amg::Level& lv = H->h.levels[k];
  if (!lv.colors) return fail(AMG_EINVAL, "amg_level_colors: no colour ordering on this hierarchy");
  return guarded("amg_level_colors", [&] {
    if (ncolors) *ncolors = (int32_t)lv.coff.size() - 1;
    if (colors) {
      AMG_HIP(hipStreamSynchronize(H->h.stream));
      AMG_HIP(hipMemcpy(colors, lv.colors, (size_t)lv.n * sizeof(int), hipMemcpyDeviceToHost));
    }
  });
}

int32_t amg_export_jacobi(const amg_hierarchy* H, int32_t k, double* wdinv) {
  if (!level_ok(H, k) || !wdinv) return fail(AMG_EINVAL, "amg_export_jacobi: bad argument");
  return guarded("amg_export_jacobi", [&] {
    const amg::Level& lv = H->h.levels[k];
    AMG_HIP(hipMemcpyAsync(wdinv, lv.wdinv, (size_t)lv.n * sizeof(double), hipMemcpyDeviceToHost, H->h.stream));
    AMG_HIP(hipStreamSynchronize(H->h.stream));
  });
}

int32_t amg_probe_timing(const amg_hierarchy* H, double* avg_ms, int32_t* samples) {
  if (!H || !avg_ms || !samples) return fail(AMG_EINVAL, "amg_probe_timing: NULL argument");
  *samples = H->h.probe_samples;
  *avg_ms = H->h.probe_samples ? H->h.probe_ms / H->h.probe_samples : 0.0;
  return AMG_OK;
}

}  // extern "C"
