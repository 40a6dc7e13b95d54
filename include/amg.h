/*
 * amg.h — C ABI of the MI355X aggregation algebraic multigrid library.
 *
 * Method: Gandham, Esler & Zhang, "A GPU Accelerated Aggregation Algebraic
 * Multigrid Method" (arXiv 1403.1649).  The library solves A x = b
 * (Section 2, eq. axb) with an outer flexible Krylov method preconditioned by
 * one K-/V-cycle (Section 2.2, Algorithms 4 and 5) over a hierarchy built by
 * Algorithm 1 (strength, MIS(2) aggregation, one-nonzero-per-row
 * interpolation, Galerkin product by aggregate index).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the argument is marked (host).
 *  - Matrices are square, 0-based CSR: int32 row_ptr[n+1], int32
 *    col_idx[nnz] strictly increasing within each row, float64 val[nnz]; every
 *    row stores a nonzero diagonal; the pattern must be structurally
 *    symmetric (values may be nonsymmetric).
 *  - Work is ordered on the caller's stream.  Calls that return host results
 *    (sizes, iteration counts, residuals) synchronise that stream before they
 *    return; the others only enqueue.
 *  - The caller owns every buffer it passes; the library owns the hierarchy
 *    and all device memory inside it.  One hierarchy serves one stream at a
 *    time; distinct hierarchies are independent.
 *  - No call throws; each returns an amg_status.  On error, outputs are
 *    unspecified unless stated otherwise.
 */
#ifndef AMG_H
#define AMG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMG_OK = 0,
  AMG_EINVAL = 1,       /* bad argument: shape, CSR structure, zero diagonal, nonsymmetric pattern */
  AMG_ENOMEM = 2,       /* device or pinned-host allocation failed */
  AMG_EHIP = 3,         /* a HIP runtime call failed */
  AMG_ENOTCONV = 4,     /* max_iter reached; x holds the last iterate, relres is set */
  AMG_EBREAKDOWN = 5,   /* Krylov breakdown (p^T A p <= 0) or a non-positive spectral estimate */
  AMG_ECOARSEN = 6,     /* coarsening stalled above the dense-solve limit, or an unsupported aggregate */
  AMG_ENANINF = 7,      /* non-finite value in the matrix, the right-hand side or the iteration */
  AMG_EUNSUPPORTED = 8  /* option combination the library does not provide */
} amg_status;

typedef enum { AMG_KRYLOV_FCG = 0, AMG_KRYLOV_FGMRES = 1 } amg_krylov;
typedef enum { AMG_PREC_FP64 = 0, AMG_PREC_MIXED = 1 } amg_precision;
/* Smoothers: damped Jacobi (eq. damped_jacobi), learned per-row Jacobi weights
 * (an extension), the Chebyshev polynomial smoother (Section 5) of degree
 * cheb_degree on D^-1 A over [b / cheb_ratio, b], b = cheb_upper * the Arnoldi
 * estimate of rho(D^-1 A), and multi-colour symmetric Gauss-Seidel (Section
 * 2.2.1): rows coloured first-fit in decreasing node-hash priority (stream
 * seed + 2; at most 64 colours), one sweep over the colours forward and one
 * backward per smoothing step. */
typedef enum { AMG_SMOOTHER_JACOBI = 0, AMG_SMOOTHER_LEARNED = 1, AMG_SMOOTHER_CHEBYSHEV = 2,
               AMG_SMOOTHER_MCSGS = 3 } amg_smoother;
/* Kernels that amg_probe_timing can report: the level-0 pre-smoothing plus
 * residual kernel (x = omega D^-1 b, r = b - A x), the level-0 residual plus
 * post-smoothing kernel, and the outer Krylov mat-vec q = A p. */
typedef enum { AMG_PROBE_NONE = 0, AMG_PROBE_L0_PRESMOOTH = 1, AMG_PROBE_L0_POSTSMOOTH = 2,
               AMG_PROBE_OUTER_SPMV = 3 } amg_probe;

/* Options (Sections 2.1.1, 2.2, 2.2.1, 3). */
typedef struct {
  double strength_alpha;  /* alpha of the classic strength test; 0.25 (2-D), 0.5 (3-D) */
  int32_t coarse_max;     /* coarsen while a level has more unknowns than this (600) */
  int32_t max_levels;     /* hard limit on the number of levels (20) */
  int32_t kcycle_levels;  /* levels 0..kcycle_levels-1 use K-cycles, the rest V-cycles (2) */
  double kcycle_t;        /* second inner Krylov step skipped when ||r~|| <= t ||r|| (0.25) */
  double jacobi_scale;    /* omega = jacobi_scale / rho(D^-1 A) (4/3) */
  int32_t arnoldi_m;      /* Arnoldi steps for rho(D^-1 A), at most 5 (5) */
  uint32_t seed;          /* node-hash seed of the MIS(2) priorities; Arnoldi uses seed+1 */
  int32_t krylov;         /* amg_krylov: outer method and K-cycle variant (FCG) */
  int32_t gmres_restart;  /* FGMRES restart length (30) */
  int32_t precision;      /* amg_precision (FP64) */
  int32_t smoother;       /* amg_smoother (JACOBI) */
  int32_t max_iter;       /* outer iteration limit (200) */
  int32_t dense_max;      /* largest coarsest level accepted after a stall (4096) */
  int32_t probe;          /* amg_probe: level-0 kernel timed with HIP events during solves (0) */
  int32_t check_every;    /* largest number of outer iterations enqueued between host
                             convergence checks; the batch adapts to the observed rate (16) */
  uint32_t flags;         /* AMG_FLAG_* bits (0) */
  const float* mlp_weights; /* (host) AMG_SMOOTHER_LEARNED: the 1409 FP32 weights of
                               amg_mlp_num_params(), copied during setup (NULL) */
  int32_t mis_k;          /* roots form an MIS(k) (Section 2.1.2): 2 as Algorithm 2, up to
                             8 for aggressive coarsening (k sweeps per round, nodes join the
                             nearest root within distance k) (2) */
  int32_t cheb_degree;    /* AMG_SMOOTHER_CHEBYSHEV: mat-vecs per smoothing step, 1..8 (2) */
  double cheb_ratio;      /* AMG_SMOOTHER_CHEBYSHEV: damped interval [b / ratio, b] (4) */
  double cheb_upper;      /* AMG_SMOOTHER_CHEBYSHEV: b = cheb_upper * rho(D^-1 A) estimate (1.1) */
} amg_options;

/* amg_options.flags: launch every kernel from the host instead of replaying
 * the captured HIP graph of an outer iteration (for debugging and timing). */
#define AMG_FLAG_NO_GRAPH 1u
/* amg_options.flags: skip the per-level kernel autotuner (CSR kernels with
 * lanes per row from the average row length). */
#define AMG_FLAG_NO_TUNE 2u
/* amg_options.flags: with AMG_SMOOTHER_LEARNED, keep the learned weights on
 * every level without the setup-time comparison against plain omega_k (for
 * weights already validated by the caller on actual solves). */
#define AMG_FLAG_LEARNED_ALWAYS 8u
/* amg_options.flags: amg_setup borrows A instead of copying it: level 0 of the
 * hierarchy reads the caller's row_ptr, col_idx and val, which must stay
 * allocated and unchanged until amg_destroy (or until amg_resetup hands over
 * new values).  The library never writes them. */
#define AMG_FLAG_BORROW_A 16u
/* amg_options.flags: run the V-cycle levels below the K-cycle (the small
 * levels of Algorithm 4 with Jacobi smoothing, and the coarse solve) as one
 * persistent launch per V-cycle instead of one kernel per step.  The results
 * are the same bit for bit; the launch is slower on MI355X (its cross-block
 * waits cost more than the launches they replace), so it is off by default. */
#define AMG_FLAG_PERSISTENT_TAIL 32u

/* A matrix handed to the library: device arrays, see the conventions above. */
typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
} amg_csr;

typedef struct amg_hierarchy amg_hierarchy;

/* Fill *opt with the defaults listed above; dim selects alpha (2 -> 0.25,
 * otherwise 0.5; Section 2.1.1). */
void amg_default_options(amg_options* opt, int32_t dim);

/* Human-readable name of a status code (static storage). */
const char* amg_status_string(int32_t status);

/* (host) message of the last failed call on this thread (empty if none).
 * Valid until the next failing call on the same thread. */
const char* amg_last_error(void);

/* Algorithm 1: build the hierarchy A_k, P_k (one nonzero per row, eq.
 * null_space), B_k and A_{k+1} = P_k^T A_k P_k (Section 3.1, eq. galerkin)
 * until a level has at most coarse_max unknowns; per level the damped Jacobi
 * weight of eq. damped_jacobi from an Arnoldi estimate of rho(D^-1 A), and a
 * dense factorisation of the coarsest level (Section 3).
 * A: device CSR, copied (the caller may free it after the call returns)
 * unless opt->flags holds AMG_FLAG_BORROW_A.
 * opt: (host) options, NULL for amg_default_options(dim=3); kcycle_levels
 * at most 24.
 * out: (host) receives the new hierarchy; free it with amg_destroy.
 * Errors: EINVAL (structure, zero diagonal, nonsymmetric pattern), ENANINF,
 * ECOARSEN, ENOMEM, EHIP; *out is NULL on error.  Synchronises s. */
int32_t amg_setup(const amg_csr* A, const amg_options* opt, hipStream_t s, amg_hierarchy** out);

/* Numeric re-setup on a fixed pattern (Section 3.1: when only the values of
 * A_0 change, as across the steps of a Newton iteration, the indices of the
 * Galerkin product are stored and reused).  val: device float64[nnz], the new
 * values of A_0 on the pattern given to amg_setup (same row_ptr, col_idx).
 * Every level keeps its strength mask, MIS(2) state, aggregates and P_k;
 * A_{k+1} = P_k^T A_k P_k is formed again from term lists that the first call
 * stores (8 bytes per stored entry of each non-coarsest level, kept until
 * amg_destroy), then every level's damped Jacobi weight (eq. damped_jacobi,
 * Arnoldi estimate) and the coarsest inverse; the autotuned kernels stay.
 * Without AMG_FLAG_BORROW_A the values are copied (the caller may free val
 * after the call); with it, level 0 reads val from then on, which must stay
 * allocated and unchanged until amg_destroy or the next amg_resetup.
 * Errors: EINVAL (zero diagonal), ENANINF, EBREAKDOWN (spectral estimate),
 * EUNSUPPORTED (batched hierarchy, learned smoother), ENOMEM, EHIP; after an
 * error the hierarchy is only fit for amg_destroy.  Synchronises s. */
int32_t amg_resetup(amg_hierarchy* h, const double* val, hipStream_t s);

/* (host) duration in ms of the last amg_resetup, from HIP events on its stream. */
int32_t amg_resetup_time(const amg_hierarchy* h, double* ms);

/* Outer Krylov solve of A x = b to ||b - A x|| <= rtol ||b|| from x_0 = 0,
 * preconditioned by one cycle (Algorithms 4 and 5 with the K-cycle on the
 * top kcycle_levels levels; Section 2.2).
 * b, x: device float64[n]; x is overwritten.  iters, relres: (host) outputs
 * (outer iterations; true relative residual recomputed in FP64 at exit).
 * Errors: ENOTCONV (x = last iterate), EBREAKDOWN, ENANINF, EHIP.
 * Synchronises s. */
int32_t amg_solve(amg_hierarchy* h, const double* b, double rtol, double* x,
                  int32_t* iters, double* relres, hipStream_t s);

/* The same solve for nrhs right-hand sides at once, each column as if solved
 * alone: B, X: device float64 row-major [n][nrhs] (1 <= nrhs <= 64); the
 * cycle is applied to the whole block (A streamed once for all columns) with
 * per-column K-cycle scalars and branches and a per-column outer iteration
 * that stops updating a column once it has converged.
 * iters, relres: (host) arrays of nrhs.  Errors as amg_solve (ENOTCONV when
 * any column did not converge).  Synchronises s. */
int32_t amg_solve_multi(amg_hierarchy* h, int32_t nrhs, const double* B, double rtol, double* X,
                        int32_t* iters, double* relres, hipStream_t s);

/* Column tiles the autotuner chose for the block solve with nrhs columns
 * (the one amg_solve_multi last ran on h; its workspace is kept for the next
 * solve with as many columns).  The block kernels take a row's entries once
 * per tile of columns: W = pow2(nrhs) is one pass, W/2 or W/4 two or four
 * passes over A with a narrower gathered working set (Section 3: the sparse
 * products of the cycle, here for a block of vectors).
 * tiles: (host) int32[cap] with cap >= amg_num_levels(h); tiles[k] for the
 * cycle's kernels on level k's rows (k < amg_num_levels(h) - 1), and
 * tiles[amg_num_levels(h) - 1] for the FP64 level-0 products of the outer
 * iteration.  tune_ms (host, may be NULL): host time of the choice (near 0
 * when it came from the cache).  EINVAL when the last block solve had
 * another column count, or none ran, or cap is too small. */
int32_t amg_multi_tiles(const amg_hierarchy* h, int32_t nrhs, int32_t* tiles, int32_t cap, double* tune_ms);

/* Independent systems in one hierarchy, each set up and solved as if alone
 * (Algorithm 1 and the solve of Algorithms 4/5 applied per system).  A is
 * their block-diagonal matrix: system q owns rows and columns
 * [sys_off[q], sys_off[q+1]) and no entry may couple two systems.  Each
 * setup kernel runs once over all systems: the node hash of the MIS(2)
 * priorities takes the row index local to its system; a system stops
 * coarsening by the rule of Algorithm 1 applied to its own size and
 * coarsening ratio and is solved there by its own dense inverse; its damped
 * Jacobi weight (eq. damped_jacobi) comes from its own Arnoldi estimate.
 * nsys: 1 <= nsys <= n.  sys_off: (host) int32[nsys+1] with sys_off[0] = 0,
 * sys_off[nsys] = n and every system nonempty.  A: device CSR (copied).
 * opt: (host) options, NULL for amg_default_options(dim=2); the batch uses
 * flexible CG and the Jacobi smoother without probe (EUNSUPPORTED otherwise);
 * of the flags only AMG_FLAG_NO_GRAPH applies.
 * amg_solve on such a hierarchy runs one outer flexible CG per system with
 * per-system scalars and stopping test (||b_q - A_q x_q|| <= rtol ||b_q||); it
 * returns the largest iteration count and relative residual over the systems
 * and ENOTCONV when any system did not converge; amg_batch_results gives the
 * per-system values.  amg_solve_multi and the amg_mlp_* calls return
 * EUNSUPPORTED on a batched hierarchy.
 * Errors: as amg_setup, and EINVAL when an entry couples two systems.
 * Synchronises s. */
int32_t amg_setup_batched(const amg_csr* A, int32_t nsys, const int32_t* sys_off, const amg_options* opt,
                          hipStream_t s, amg_hierarchy** out);

/* SpMV format the autotuner chose for level k in the given arithmetic
 * (amg_precision: FP64 for the float64 kernels, MIXED for the float32 cycle):
 * format (host) 0 = CSR with *lanes_per_row lanes per row, 1 = sliced ELL,
 * 2 = sliced ELL with 16-bit column offsets col - row, 3 = sliced diagonals
 * (per 64-row slice a list of offsets col - row and their values, no column
 * indices; built for levels whose slices have few diagonals, as on
 * structured grids; *lanes_per_row = 1), 4 = CSR with its columns as 16-bit
 * offsets col - row (levels whose offsets all fit; *lanes_per_row lanes per
 * row); for the sliced ELL,
 * *lanes_per_row = 64 / slice height (1: 64-row slices; 2 or 4: the level's
 * copy in 32- or 16-row slices, built where rows vary in length);
 * us (host, may be NULL) = its timed duration (0 if the level was not timed).
 * EINVAL if k is not a level that runs a cycle. */
int32_t amg_level_format(const amg_hierarchy* h, int32_t k, int32_t precision, int32_t* format,
                         int32_t* lanes_per_row, float* us);

/* y = A_k x on level k of a hierarchy, float64, with the kernel the
 * autotuner chose for that level in FP64 (amg_level_format; CSR on levels it
 * did not time): the sparse mat-vec of Section 3 as the solve runs it.
 * x[n_k] and y[n_k] are device vectors owned by the caller (n_k from
 * amg_level_info; not checked).  Enqueue only, on s.  EINVAL for a NULL
 * hierarchy or vector or a level outside [0, amg_num_levels). */
int32_t amg_level_spmv(const amg_hierarchy* h, int32_t k, const double* x, double* y, hipStream_t s);

/* Per-system outer iterations and true relative residuals of the last
 * amg_solve on a batched hierarchy.  iters: (host) int32[nsys] or NULL;
 * relres: (host) float64[nsys] or NULL.  EINVAL if the hierarchy is not
 * batched or has not been solved with. */
int32_t amg_batch_results(const amg_hierarchy* h, int32_t* iters, double* relres);

/* Level k of a batched hierarchy: sys_off (host int32[nsys+1] or NULL)
 * receives the row range of every system on that level (an empty range once
 * a finer level was the system's coarsest); omega (host float64[nsys] or NULL)
 * the system's damped Jacobi weight on that level (0 where the system does
 * not coarsen from level k).  EINVAL if not batched or k is out of range. */
int32_t amg_batch_level(const amg_hierarchy* h, int32_t k, int32_t* sys_off, double* omega);

/* ---- Learned per-row Jacobi weights (an extension beyond the paper, which
 * fixes one omega per level by eq. damped_jacobi).  omega_i = sigmoid(y_i) *
 * 2|a_ii| / (|a_ii| + sum_{j!=i} |a_ij|), y = MLP 9->32->32->1 (ReLU) of the row
 * features [log|a_ii| - level mean, six largest |a_ij|/|a_ii| descending,
 * row sum / a_ii, level]; bfloat16 weights and inputs, FP32 accumulation.
 * The bound keeps the smoother convergent for SPD A.  With
 * opt.smoother = AMG_SMOOTHER_LEARNED, setup uses the learned weights on a
 * level only when they lower the smoothing loss below the plain omega_k on
 * four validation samples, and then keeps them only when a probe solve with
 * them needs fewer iterations than with plain damped Jacobi (amg_learned_judge);
 * it falls back to plain damped Jacobi otherwise. */

/* Two-grid errors for training the learned weights of level k (the errors a
 * smoother of level k must damp in a cycle, Algorithm 4: after the coarse
 * correction): out_s = (I - P_k B P_k^T A_k) e_s for the nsamples columns of
 * E, with B = A_{k+1}^-1 exactly when level k+1 is the coarsest, else
 * `cycles` steps of y <- y + M_{k+1}(r_c - A_{k+1} y) from y = 0, M_{k+1} the
 * hierarchy's own cycle from level k+1.  E, out: device float64 [n_k][nsamples]
 * row-major (may not alias).  k < amg_num_levels(h) - 1, nsamples >= 1,
 * cycles >= 1.  EUNSUPPORTED on mixed-precision or batched hierarchies.
 * Synchronises s. */
int32_t amg_mlp_coarse_corrected(const amg_hierarchy* h, int32_t k, const double* E, int32_t nsamples,
                                 int32_t cycles, double* out, hipStream_t s);

/* Number of MLP parameters (1409): W1[32][9], b1[32], W2[32][32], b2[32], W3[32], b3. */
int32_t amg_mlp_num_params(void);

/* feats: device float [n_k][9], the bfloat16-rounded features of level k. */
int32_t amg_mlp_features(const amg_hierarchy* h, int32_t k, float* feats, hipStream_t s);

/* omega: device float64 [n_k], the learned weights of level k for the device
 * parameter vector w (FP32 masters, rounded to bfloat16 inside). */
int32_t amg_mlp_omega(const amg_hierarchy* h, int32_t k, const float* w, double* omega, hipStream_t s);

/* Smoothing loss of level k, L = (1/S) sum_s ||(I - W A) e_s||_A^2 / ||e_s||_A^2,
 * W = diag(omega_i / a_ii), over S = nsamples + n_extra error samples with the
 * coarse-space component removed (e = v - P P^T v): v = unit_uniform(i,
 * seed + s) for the first nsamples and the caller's device [n_k][n_extra]
 * row-major block `extra` for the rest.  loss: (host).  grad (device float
 * [1409], may be NULL): dL/dw.  flags: bit 0 (AMG_MLP_ACCUMULATE) adds to
 * grad instead of overwriting it; bit 1 (AMG_MLP_RAW_EXTRA) uses the extra
 * samples as given, without removing their coarse-space component (for
 * errors that the solver itself left, which the coarse correction has
 * already acted on).  1 <= S <= 64.  Synchronises s. */
#define AMG_MLP_ACCUMULATE 1
#define AMG_MLP_RAW_EXTRA 2
int32_t amg_mlp_loss_grad(const amg_hierarchy* h, int32_t k, const float* w, int32_t nsamples, uint32_t seed,
                          const double* extra, int32_t n_extra, double* loss, float* grad, int32_t flags,
                          hipStream_t s);

/* Adam step on device arrays of n floats: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, w -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
int32_t amg_mlp_adam(float* w, float* m, float* v, const float* g, int32_t n, int32_t step, float lr, float b1,
                     float b2, float eps, hipStream_t s);

/* (host) smoother used on level k: *learned = 1 when the learned weights
 * passed validation there, with the validation losses of plain omega_k and of
 * the learned weights (0 when not evaluated). */
int32_t amg_level_smoother(const amg_hierarchy* h, int32_t k, int32_t* learned, double* loss_plain,
                           double* loss_learned);

/* (host) the multi-colour ordering of level k (AMG_SMOOTHER_MCSGS): colors
 * int32[n_k] (may be NULL) and *ncolors (may be NULL).  EINVAL when the
 * hierarchy does not smooth by colours or k has no smoother. */
int32_t amg_level_colors(const amg_hierarchy* h, int32_t k, int32_t* colors, int32_t* ncolors);

/* (host) the setup's judgement of the learned weights (AMG_SMOOTHER_LEARNED
 * without AMG_FLAG_LEARNED_ALWAYS, when some level passed the loss check): a
 * probe solve of A x = A u (u hashed from seed + 3) to relative residual 1e-4
 * with the learned weights and with the plain omega_k on every level; the
 * learned ones stay (*kept = 1) only with fewer iterations, or as many and a
 * smaller true residual; otherwise every level falls back to damped Jacobi
 * (*kept = 0).  *kept = -1 when no judgement was made.  Any pointer may be
 * NULL. */
int32_t amg_learned_judge(const amg_hierarchy* h, int32_t* kept, int32_t* iters_plain, double* relres_plain,
                          int32_t* iters_learned, double* relres_learned);

/* (host) copy of omega_i / a_ii, the Jacobi scaling the cycle applies on level k. */
int32_t amg_export_jacobi(const amg_hierarchy* h, int32_t k, double* wdinv);

/* Release the hierarchy (NULL is ignored).  Its device memory returns to a
 * process-wide cache of large chunks that later setups reuse without
 * allocating; amg_release_cached_memory gives that cache back to HIP. */
void amg_destroy(amg_hierarchy* h);

/* Free every cached device chunk that no live hierarchy uses (hipFree);
 * returns the number of bytes released.  Live hierarchies are unaffected.
 * Call it after destroying hierarchies whose memory should return to the
 * device, and before the HIP runtime shuts down. */
size_t amg_release_cached_memory(void);

/* Number of levels L+1 of a hierarchy (the coarsest level is index L). */
int32_t amg_num_levels(const amg_hierarchy* h);

/* (host) size of level k: n_k, nnz(A_k), omega_k (0 on the coarsest level),
 * n_{k+1} (0 on the coarsest level) and the number of Algorithm 2 rounds.
 * Any output pointer may be NULL. */
int32_t amg_level_info(const amg_hierarchy* h, int32_t k, int32_t* n, int32_t* nnz,
                       double* omega, int32_t* n_coarse, int32_t* mis_rounds);

/* Copy level k to (host) buffers, for inspection and level-wise testing:
 * row_ptr[n+1], col_idx[nnz], val[nnz] of A_k; strong[nnz] the strength mask
 * C of Section 2.1.1 over A_k's pattern (0/1); state[n] the MIS(2) state of
 * Algorithm 2 (1 root, -1 other); agg[n] the aggregate index; pval[n] the
 * value of P_k's single nonzero per row (Algorithm 3); B[n] the near null
 * space vector B_k.  Setup-only arrays are absent on the coarsest level
 * (EINVAL if requested there).  Any pointer may be NULL.  Synchronises the
 * hierarchy's setup stream. */
int32_t amg_export_level(const amg_hierarchy* h, int32_t k, int32_t* row_ptr, int32_t* col_idx,
                         double* val, uint8_t* strong, int8_t* state, int32_t* agg,
                         double* pval, double* B);

/* y = A x (the sparse mat-vec of Section 3, "axpy" there), float64, with the
 * kernel families the solve uses: lanes_per_row in {1,2,4,8,16,32,64} selects
 * the CSR kernel with that many lanes per row, 0 picks the lane count from the
 * average row length, -1 selects the sliced-ELL kernel (the matrix is
 * converted into a temporary copy first; synchronises s), -2 the sliced-ELL
 * kernel reading 16-bit column offsets col - row (EINVAL when an offset lies
 * outside [-32768, 32767]; synchronises s).  Otherwise enqueue only. */
int32_t amg_spmv(const amg_csr* A, const double* x, double* y, int32_t lanes_per_row, hipStream_t s);

/* Node hash of the MIS(2) priorities (the random r_i of Algorithm 2 made
 * deterministic): out[i] = fmix32((i + stream * 0x9E3779B9) mod 2^32), the
 * MurmurHash3 32-bit finaliser; out: device uint32[n].  Enqueue only. */
int32_t amg_node_hash(int32_t n, uint32_t stream, uint32_t* out, hipStream_t s);

/* Galerkin product by aggregate index (Section 3.1, eq. galerkin) for a
 * given aggregation: (A_c)_IJ = sum over stored (i,j) with agg[i]=I,
 * agg[j]=J of (pval[i] * a_ij) * pval[j].  A, agg[n], pval[n]: device.
 * nnz_c: (host) receives nnz(A_c).  row_ptr_c[nc+1], col_c[cap], val_c[cap]:
 * (host) outputs, written only when cap >= nnz(A_c) (otherwise EINVAL with
 * *nnz_c set).  Synchronises s. */
int32_t amg_galerkin(const amg_csr* A, const int32_t* agg, const double* pval, int32_t nc,
                     int32_t* nnz_c, int32_t* row_ptr_c, int32_t* col_c, double* val_c,
                     int32_t cap, hipStream_t s);

/* amg_galerkin for callers that cannot allocate memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same product
 * by aggregate index (Section 3.1, eq. galerkin) with the same kernels, all of
 * their scratch in one static device array of the library (about 17 MiB per
 * device, held until the process ends); no hipMalloc, hipHostMalloc or other
 * allocating call.  Limits: A->n <= 131072 and A->nnz <= 1048576 (EINVAL
 * beyond).  Outputs are DEVICE arrays owned by the caller: row_ptr_c[nc+1]
 * (always written once the checks pass), col_c[cap] and val_c[cap] (written
 * only when cap >= nnz(A_c); otherwise EINVAL with *nnz_c set).  nnz_c: (host).
 * Input checks and errors as amg_galerkin.  Every call on one device shares
 * the array, so calls that overlap on one device (other streams or threads)
 * race; calls in sequence are independent.  Synchronises s. */
int32_t amg_galerkin_noalloc(const amg_csr* A, const int32_t* agg, const double* pval, int32_t nc,
                             int32_t* row_ptr_c, int32_t* col_c, double* val_c, int32_t cap, int32_t* nnz_c,
                             hipStream_t s);

/* (host) largest eigenvalue modulus of a real m-by-m upper Hessenberg matrix
 * H (row-major, m <= 8): the spectral estimate of Section 2.2.1 taken from
 * the Arnoldi Hessenberg matrix.  No device work. */
int32_t amg_hessenberg_radius(const double* H, int32_t m, double* rho);

/* (host) timing of the last setup and solve on this hierarchy, in ms, from
 * HIP events on the hierarchy's stream. */
int32_t amg_timings(const amg_hierarchy* h, double* setup_ms, double* solve_ms);

/* (host) parts of the last setup's time, in ms of host wall clock: the
 * per-level SpMV autotuner (near 0 when its results came from the cache of
 * an earlier setup with the same level sizes) and the capture of the outer
 * iteration into HIP graphs.  Both are inside amg_timings' setup_ms. */
int32_t amg_setup_phases(const amg_hierarchy* h, double* tune_ms, double* capture_ms);

/* (host) average duration in ms of the kernel selected by opt.probe, over the
 * samples taken since setup: HIP events recorded on the solve stream right
 * before and after that kernel (inside the replayed outer iteration), read at
 * host convergence checks whose last iteration ran the kernel.  *samples = 0
 * when no probe was selected or no sample was taken. */
int32_t amg_probe_timing(const amg_hierarchy* h, double* avg_ms, int32_t* samples);

#ifdef __cplusplus
}
#endif

#endif /* AMG_H */
