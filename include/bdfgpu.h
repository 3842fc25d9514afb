/*
 * bdfgpu: batched stiff-ODE BDF-Newton on AMD MI355X (gfx950).
 *
 * C ABI of the library.  Every argument is a plain pointer or size.
 *
 * Conventions (all entry points)
 *  - Memory.  Vector and matrix arguments are caller-owned DEVICE pointers
 *    unless stated "host".  The library never frees memory it did not
 *    allocate; memory it allocates (handle state, reduction scratch) it
 *    frees in the matching destroy call or at process exit.  This follows
 *    the ownership flag of the paper's SUNMemory structure (Section 3).
 *  - Layout.  Vectors are contiguous FP64.  When a vector holds many small
 *    systems it is cell-major: cell c owns entries [off_c, off_c + n_c)
 *    (grouping of independent systems, Section 2, Fig. blockdiag_jacobian).
 *    Dense blocks are contiguous column-major n x n blocks, block b at
 *    offset b*n*n.  Pivots are int32, 0-based: piv[b*n + k] is the row
 *    exchanged with row k at step k.
 *  - Streams.  Every call takes `stream`, a hipStream_t (NULL = the legacy
 *    default stream), and enqueues its work only there; vector, matrix and
 *    solver calls that work on the same data must share a stream
 *    (Sections 4.1 and 5).  Streaming operations return without waiting
 *    (Section 4.1, Listing lst:synchronize: the caller synchronises before
 *    touching results).  Reductions return their scalar through a HOST
 *    pointer and then have synchronised the stream (Section 4.1: reductions
 *    end with a transfer to the host), or, with flags &
 *    BDFGPU_RESULT_DEVICE, write a DEVICE pointer asynchronously.
 *  - Status.  0 success; > 0 recoverable (the caller may retry with a
 *    smaller step: singular pivot, Newton or error-test failure); < 0
 *    unrecoverable (codes below).  n == 0 is a no-op returning 0 (norms
 *    return 0).  bdfgpu_last_error() describes the last failure.
 *  - Concurrency.  Calls that use the library's internal reduction
 *    scratch (the nvec reductions) must not run concurrently on two streams
 *    of the same device.
 */
#ifndef BDFGPU_H
#define BDFGPU_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  > 0: the step could not be completed but a smaller step
 * may succeed (the paper's recoverable-failure semantics for task-local
 * nonlinear solves, Section 7); the integrator handle then keeps its last
 * accepted state (bdf_get_y, bdf_get_state) and stops: continue from that
 * state with bdf_set_state and a smaller h.  < 0: unrecoverable. */
#define BDFGPU_SUCCESS 0
#define BDFGPU_RECOVERABLE 1      /* recoverable failure (unspecified) */
#define BDFGPU_CONV_FAIL 2        /* Newton failed 10 times in one step */
#define BDFGPU_TEST_FAIL 3        /* error test failed 7 times in one step */
#define BDFGPU_ERR_ARG (-1)       /* bad argument */
#define BDFGPU_ERR_HIP (-2)       /* HIP runtime error */
#define BDFGPU_ERR_WORKSPACE (-3) /* caller workspace too small */
#define BDFGPU_ERR_TOO_MUCH_WORK (-4) /* max_steps reached before t_end */
#define BDFGPU_ERR_HMIN (-5)      /* step size fell below hmin (or below the
                                     resolution of t) */

#define BDFGPU_RESULT_DEVICE 1

/* Text of the last error recorded by any call on this thread's process. */
const char* bdfgpu_last_error(void);
/* Library version string. */
const char* bdfgpu_version(void);

/* ========================================================================
 * N_Vector operations (Section 2: streaming operations and reductions;
 * Section 4.1: reductions run fully on the GPU and end with one scalar
 * transfer; streaming operations are asynchronous).  The fused operations
 * below are defined by their plain formulas; arrays of coefficients and of
 * vector pointers are HOST arrays of length nv, the vectors themselves are
 * device arrays of length n.
 * ======================================================================== */

/* z = a x + b y.  z may alias x or y. */
int nvec_linear_sum(long n, double a, const double* x, double b,
                    const double* y, double* z, void* stream);
/* z = sum_j c[j] X[j], 1 <= nv <= 16.  z may alias X[0]. */
int nvec_linear_combination(int nv, const double* c, const double* const* X,
                            double* z, long n, void* stream);
/* Z[j] = a[j] x + Y[j], 1 <= nv <= 8.  Z[j] may alias Y[j]. */
int nvec_scale_add_multi(int nv, const double* a, const double* x,
                         const double* const* Y, double* const* Z, long n,
                         void* stream);
/* d[j] = sum_i x_i Y[j]_i, 1 <= nv <= 8.  d: host (sync) or device. */
int nvec_dot_prod_multi(int nv, const double* x, const double* const* Y,
                        double* d, long n, int flags, void* stream);
/* nvec_dot_prod_multi for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipFree or allocating library routine: its block
 * partials live in a static array of the library's device memory
 * (8192 blocks x 8 doubles = 512 KiB per device, held until the process
 * ends); the reduction grid never exceeds it, whatever n.  d is a DEVICE
 * array of nv doubles, written asynchronously on `stream`.  1 <= nv <= 8,
 * else BDFGPU_ERR_ARG.  All calls on one device share that array, which
 * keeps the last call's partials: calls that overlap on one GPU (two
 * streams, or two host threads) race and must be serialised by the caller.
 * n == 0 writes zeros. */
int nvec_dot_prod_multi_noalloc(int nv, const double* x, const double* const* Y,
                                double* d, long n, void* stream);
/* out = sqrt(sum_i (x_i w_i)^2 / n).  out: host (sync) or device. */
int nvec_wrms_norm(long n, const double* x, const double* w, double* out,
                   int flags, void* stream);
/* nrm[j] = sqrt(sum_i (X[j]_i W[j]_i)^2 / n), 1 <= nv <= 8: the WRMS norms
 * of several vectors in one pass (the vector-array form of the WRMS norm).
 * X, W: host arrays of nv device vectors; when every W[j] is the same
 * pointer that weight vector is read once.  nrm: host (sync) or device. */
int nvec_wrms_norm_multi(int nv, const double* const* X, const double* const* W,
                         double* nrm, long n, int flags, void* stream);
/* out = max_i |x_i|.  out: host (sync) or device. */
int nvec_max_norm(long n, const double* x, double* out, int flags, void* stream);
/* w_i = 1 / (rtol |y_i| + atol)  (error weights of the WRMS norm). */
int nvec_ewt(long n, double rtol, double atol, const double* y, double* w,
             void* stream);
/* z = c x. */
int nvec_scale(long n, double c, const double* x, double* z, void* stream);
/* z = c. */
int nvec_const(long n, double c, double* z, void* stream);

/* ========================================================================
 * Batched dense LU of block-diagonal matrices (Section 5: a direct solver
 * for block-diagonal systems whose blocks share one pattern; here every
 * block is dense, n <= 64).  getrf semantics: right-looking partial
 * pivoting, first maximal pivot, whole-row exchanges, division by the
 * pivot.  info[b] = k (1-based) if U(k,k) is exactly zero (first such k);
 * factoring continues; a singular block is not an error of the call.
 * ======================================================================== */

/* In place: A (nb blocks, n x n column-major) becomes L\U. */
int batched_lu_factor_f64(int nb, int n, double* A, int* piv, int* info,
                          void* stream);
/* In place: B (nb x n, block b at B + b*n) becomes the solution. */
int batched_lu_solve_f64(int nb, int n, const double* LU, const int* piv,
                         double* B, void* stream);
int batched_lu_factor_f32(int nb, int n, float* A, int* piv, int* info,
                          void* stream);
int batched_lu_solve_f32(int nb, int n, const float* LU, const int* piv,
                         float* B, void* stream);
/* Blocks of different sizes (block-diagonal matrices whose blocks are not
 * all alike) in one launch.  sizes, moff, voff: DEVICE arrays of nb
 * entries; block b is the sizes[b] x sizes[b] column-major block at
 * A + moff[b] (usually moff[b] = sum_{b'<b} sizes[b']^2), its pivots at
 * piv + voff[b] and its right-hand side / solution at B + voff[b]
 * (usually voff[b] = sum_{b'<b} sizes[b']).  nmax (host) bounds every size
 * and sets the lanes per block (the next power of two, <= 64); a block
 * whose size is outside 0..nmax gets info[b] = -1 and is left untouched.
 * Semantics per block as the uniform calls above. */
int batched_lu_factor_f64_var(int nb, int nmax, const int* sizes, const long* moff,
                              const long* voff, double* A, int* piv, int* info,
                              void* stream);
int batched_lu_solve_f64_var(int nb, int nmax, const int* sizes, const long* moff,
                             const long* voff, const double* LU, const int* piv,
                             double* B, void* stream);
int batched_lu_factor_f32_var(int nb, int nmax, const int* sizes, const long* moff,
                              const long* voff, float* A, int* piv, int* info,
                              void* stream);
int batched_lu_solve_f32_var(int nb, int nmax, const int* sizes, const long* moff,
                             const long* voff, const float* LU, const int* piv,
                             float* B, void* stream);
/* FP32 LU (LU32/piv32, from batched_lu_factor_f32 of M rounded to FP32)
 * plus FP64 iterative refinement: x0 = FP32 solve of b; then corrections
 * from the FP64 residual b - M x until |r|_inf <= sqrt(n) eps64 |M|_inf
 * |x|_inf, at most max_it corrections; a block that does not converge, or
 * whose corrections stop halving, is solved with FP64 LU of M instead.
 * status[b] = 0 refined, 1 fell back to FP64, 2 FP64 fallback singular.
 * sweeps[b] = corrections applied.  M, B unchanged; X receives x. */
int batched_lu_solve_refine(int nb, int n, const double* M, const float* LU32,
                            const int* piv32, const double* B, double* X,
                            int max_it, int* sweeps, int* status,
                            void* stream);

/* ========================================================================
 * Grouped BDF integrator over many independent mass-action systems.
 *
 * The systems ("cells") are grouped into one ODE with a block-diagonal
 * Jacobian (Section 2) and advanced with one step size and order; every
 * Newton iteration solves all cells' blocks at once and one failing cell
 * makes the whole step retry with a smaller step (Section 7, task-local
 * Newton and ensemble failure rule).  The method is a fixed-coefficient
 * Nordsieck BDF of orders 1..qmax (the paper names CVODE for this role but
 * does not state the method).  Integrator control lives on the device; the
 * host only enqueues attempts and reads the status every few attempts.
 *
 * Kinetics: r_k = kappa_k prod_s y_s^nu_ks, f_s = sum_k (mu_ks - nu_ks) r_k;
 * each reaction may have at most three reactant molecules, and three only
 * in classes of <= 12 species with FP64 LU or the Gauss-Jordan solve (the
 * paper's demonstration reaction has one, 2u + v -> 3u).
 * ======================================================================== */

#define BDFGPU_LS_LU64 0     /* FP64 LU per block */
#define BDFGPU_LS_LU32REF 1  /* FP32 LU + FP64 refinement, per-block fallback */
#define BDFGPU_LS_LEARNED 2  /* learned approximate inverse (options.precond),
                                per-cell and per-attempt fallback to FP64 LU;
                                cells of 13..31 species */
#define BDFGPU_LS_GMRES 4    /* Newton-Krylov: each Newton system solved over all
                                cells at once by right-preconditioned GMRES
                                scaled by the error weights (Krylov dimension 5,
                                classical Gram-Schmidt, tolerance 0.05 of the
                                Newton tolerance), with the cells' LU factors
                                at the last setup as block-Jacobi
                                preconditioner (refreshed every attempt, or per
                                the lazy rules); the global Newton with GMRES
                                of Section 7.  One lane per cell (<= 12
                                species), per-class launches, stream mode; the
                                host drives the Krylov iteration (one
                                synchronising reduction per inner-product
                                pass, as in Section 4.1) */
#define BDFGPU_LS_GJ 3       /* explicit block inverse by Gauss-Jordan
                                elimination with partial pivoting, applied as
                                a matrix-vector product in every Newton
                                iteration: the task-local block solve of the
                                paper's demonstration problem (Section 7).
                                Cells of <= 4 species one lane per cell,
                                larger cells (up to 64 species) one row per
                                lane of a segment; per-class launches (not
                                BDFGPU_LAUNCH_FUSED) */

#define BDFGPU_MODE_STREAM 0 /* kernels enqueued on the stream */
#define BDFGPU_MODE_GRAPH 1  /* one attempt captured in a hipGraph */

#define BDFGPU_LAUNCH_PER_CLASS 0 /* one launch per class of cells and phase */
#define BDFGPU_LAUNCH_FUSED 1     /* one persistent launch over every class per
                                     phase (blocks of uneven sizes together): the
                                     workgroups the device holds at once take the
                                     classes' blocks from a work queue in the
                                     handle's device memory, costliest blocks
                                     first; <= 8 classes, not with the learned
                                     preconditioner */
#define BDFGPU_LAUNCH_AUTO 2      /* bdf_create times the candidate launch modes and
                                     small-block mappings and keeps the fastest */

typedef struct {
  int ntopo;              /* number of network topologies */
  const int* topo_n;      /* host [ntopo]: species per topology (1..64) */
  const int* topo_R;      /* host [ntopo]: reactions per topology */
  const int* topo_off;    /* host [ntopo]: offset of topology t in nu/mu */
  const int* nu_all;      /* host: R_t x n_t row-major reactant counts */
  const int* mu_all;      /* host: R_t x n_t row-major product counts */
  long ncells;
  const int* cell_topo;   /* host [ncells]: topology of each cell */
  const double* rates;    /* device: R_c rate constants per cell, concatenated */
  const double* y0;       /* device: n_c initial values per cell, concatenated */
  double t0;
} bdf_problem;

typedef struct {
  double rtol, atol;      /* error weights 1/(rtol |y| + atol) */
  int qmax;               /* 1..5 */
  int maxcor;             /* Newton iterations per attempt (<= 4; 3 usual) */
  double h0;              /* first step; 0 = Hairer-Norsett-Wanner estimate */
  double hmin;
  int linsol;             /* BDFGPU_LS_* */
  int refine_max_it;      /* FP32 refinement corrections before FP64 */
  long max_steps;         /* per integrate call; 0 = unlimited */
  int mode;               /* BDFGPU_MODE_* */
  int attempts_per_sync;  /* attempts enqueued between status reads (>= 1) */
  int launch;             /* BDFGPU_LAUNCH_* */
  void* precond;          /* precond_handle* for BDFGPU_LS_LEARNED */
  int nonneg;             /* 1: each corrected solution is projected onto y >= 0
                             before the error test; the projection enters the
                             correction, so the history stays consistent.  A
                             project reading, not a method of the paper (its
                             N_Vector constraint-mask operation only flags
                             violations); it keeps bimolecular mass action
                             from running away after a component turns
                             negative.  Initial values must then be >= 0 */
  int map_small;          /* 0: classes of <= 12 species use one lane per cell
                             (block in registers); 1: a 16-lane segment per cell */
  int jit;                /* 1: bdf_create generates, for each one-lane-per-cell
                             class, a Newton kernel with the class's network
                             written out as straight-line code (the device-side
                             right-hand side and Jacobian callbacks a user
                             supplies, Section 6, here derived from nu and mu),
                             compiles it with hipcc
                             ($HIPCC, else /opt/rocm/bin/hipcc; about 4 s per
                             new network) into a shared library cached under
                             $BDFGPU_JIT_DIR (else $TMPDIR/bdfgpu-jit-<uid>)
                             and loads it; results are bitwise those of the
                             generic kernel.  0: generic kernels only.  Error
                             BDFGPU_ERR_HIP with the end of the compiler log if
                             compilation or loading fails. */
  int no_defer;           /* 0: with per-class launches of one-lane-per-cell
                             classes (FP64 or FP32-refined LU), an accepted
                             step's history update z_new = z(0) + l acor is
                             applied by the next attempt's Newton kernel as it
                             reads the history (and by the end of each
                             bdf_step / bdf_integrate / bdf_advance call), so
                             the history crosses HBM once per step; the order
                             selection's norms are summed per Newton iteration.
                             Results are those of the separate update.
                             1: a separate history-update kernel per attempt. */
  int per_cell;           /* 1: per-cell adaptive stepping.  Every cell is its
                             own ODE with its own step size, order, Newton
                             convergence test and error test, on WRMS norms
                             over its own species (the task-local integrators
                             of Section 7 taken down to single cells): a cell's
                             result is the grouped method's for a problem of
                             that one cell.  bdf_integrate advances every cell
                             to t_end; bdf_get_stats sums the cells' counters
                             (t: the earliest cell); bdf_get_cell_stats gives
                             them per cell.  Cells of <= 12 species, FP64 LU
                             or Gauss-Jordan, per-class launches; bdf_step,
                             bdf_advance and the state calls are refused.
                             max_steps bounds the attempts per cell. */
  int vc;                 /* 1: variable-coefficient BDF (CVODE's BDF takes its
                             coefficients from the step sizes, Section 1): the
                             corrector is the BDF formula on the actual past
                             grid, the error and order-change constants follow
                             from the history interpolating the last q + 1
                             accepted values, and order changes keep that
                             interpolation.  Constant steps give the fixed
                             coefficients.  Needs the deferred history update
                             (see no_defer) and not per_cell. */
  int lazy;               /* 1: the Newton matrix is kept over steps: its factors
                             (or inverse) are stored per cell (n^2 + n values)
                             and refreshed at the first attempt, after a Newton
                             failure, every 20 accepted steps and when gamma
                             has moved more than 30% from the stored factors'
                             gamma_s; a reuse scales each correction by
                             2 / (1 + gamma / gamma_s) and carries the
                             convergence-rate estimate over, and a Newton
                             failure on reused factors redoes the attempt with
                             fresh ones at the same step size.  Any class
                             size; needs FP64 LU, Gauss-Jordan or GMRES,
                             per-class launches (not BDFGPU_LAUNCH_FUSED) and
                             not per_cell. */
  int newton_per_launch;  /* Newton iterations per launch of the fused Newton
                             kernel, 1..maxcor (0: 2).  When the replay of a
                             launch's iterations leaves the attempt undecided,
                             the next launch continues from the stored iterate;
                             decisions and results do not depend on it.  The
                             learned preconditioner and GMRES run all maxcor
                             iterations in one launch. */
} bdf_options;

typedef struct {
  long nsteps, nattempts, nfevals, nsetups, nniters, nncfails, netfails;
  long nlinsolves, refine_sweeps, refine_fallbacks, nprojections;
  long hist_reads;        /* sum over attempts of q + 1 */
  long lp_cell_solves;    /* learned: per-cell corrections X r */
  long lp_fallback_cells; /* learned: cells moved to exact LU within an attempt */
  long lp_step_fallbacks; /* learned: attempts redone with exact LU */
  long order_hist[6];
  double t, h, hu, err_last;
  int q, qu, qwait, status;
  long nstale_retries;    /* lazy: attempts redone with fresh factors */
  long nliters;           /* GMRES iterations */
  long ncont;             /* Newton kernel launches that continued an attempt's
                             iterations (two iterations per launch) */
} bdf_stats;

typedef struct bdf_handle bdf_handle;

/* Copies the problem into library-owned device memory (internal layouts),
 * computes the first step, and returns a handle.  `stream` is used by
 * every later call on the handle. */
int bdf_create(const bdf_problem* p, const bdf_options* o, void* stream,
               bdf_handle** out);
/* Device bytes bdf_create_ws needs for this problem and these options (the
 * history, iterates, rates, network tables, reduction partials and control
 * block of every class; with BDFGPU_LAUNCH_AUTO the largest candidate).  No
 * device memory is touched and the problem's rates and y0 may be NULL; 0
 * for an invalid problem or options. */
size_t bdf_workspace_bytes(const bdf_problem* p, const bdf_options* o);
/* bdf_create with every piece of device state carved from the caller's
 * workspace ws (DEVICE memory, 256-byte aligned, ws_bytes >=
 * bdf_workspace_bytes) instead of hipMalloc: the caller owns the memory
 * and frees it after bdf_destroy, which frees only host-side handle memory
 * (the SUNMemory ownership rule of Section 3).  The library zeroes what it
 * needs.  BDFGPU_ERR_WORKSPACE if ws is NULL or too small.  (The
 * diagnostic calls bdf_eval_rhs_jac and bdf_capture_blocks still allocate
 * their own temporaries.) */
int bdf_create_ws(const bdf_problem* p, const bdf_options* o, void* ws,
                  size_t ws_bytes, void* stream, bdf_handle** out);
int bdf_destroy(bdf_handle* h);
/* Launch configuration in use (launch: BDFGPU_LAUNCH_PER_CLASS or _FUSED;
 * map_small as in bdf_options) and, after BDFGPU_LAUNCH_AUTO, the timed
 * ms per step of each candidate: ms_per_step[2 * launch + map_small]
 * (host array of 4; -1 where not tried or not possible). */
int bdf_get_tuning(bdf_handle* h, int* launch, int* map_small, double* ms_per_step);
/* One accepted internal step that does not pass t_end (the last step lands
 * on t_end exactly).  *tret = t after the step (host). */
int bdf_step(bdf_handle* h, double t_end, double* tret);
/* Steps until t == t_end exactly.  *tret = t (host). */
int bdf_integrate(bdf_handle* h, double t_end, double* tret);
/* At most nsteps accepted steps towards t_end (stops early at t_end).
 * *tret = t (host); *taken = steps accepted by this call. */
int bdf_advance(bdf_handle* h, double t_end, long nsteps, double* tret, long* taken);
/* Kernel timing with HIP events on the handle's stream (stream mode only):
 * on != 0 starts (and resets) timing of the three kernel groups of an
 * attempt: 0 predictor, Jacobian, block factorisation and all Newton
 * iterations (one fused launch per class), 1 learned mode only: predictor
 * and MLP inference, 2 history update.  ms[3] receives the summed
 * durations in milliseconds, counts[3] the number of timed launches (host
 * arrays). */
int bdf_set_profiling(bdf_handle* h, int on);
int bdf_get_kernel_times(bdf_handle* h, double* ms, long* counts);
/* Current solution z[0], cell-major, into the device array y (length N). */
int bdf_get_y(bdf_handle* h, double* y);
/* Counters and scalars (host struct). */
int bdf_get_stats(bdf_handle* h, bdf_stats* s);
/* Per-cell stepping only: per cell (user order), HOST arrays (any may be
 * NULL, not all): counts[5 c + k] = accepted steps, attempts, Newton
 * iterations, error-test failures, convergence failures; t[c] = time
 * reached; hu[c] = last accepted step size. */
int bdf_get_cell_stats(bdf_handle* h, int* counts, double* t, double* hu);
/* Total unknowns N and number of cells. */
long bdf_get_N(bdf_handle* h);
/* Integrator state for exact single-step comparisons: scalars (host
 * arrays: dvals = {t, h}, ivals = {q, qwait}) and history z[0..5] plus the
 * saved correction that the next order selection compares against (it is
 * refreshed by the accepted step whose successor selects the order), each
 * a device array of N values, cell-major. */
int bdf_get_state(bdf_handle* h, double* dvals, int* ivals, double* z6,
                  double* dprev);
int bdf_set_state(bdf_handle* h, const double* dvals, const int* ivals,
                  const double* z6, const double* dprev);
/* Training data for the learned preconditioner: for every stride-th cell
 * (at most max_blocks) of the handle's class of n species, the inputs
 * [y (n), log gamma] (FP64, device X_raw) and the block M = I - gamma J(y)
 * (device M, FP64, column-major) at the current solution y = z[0] and the
 * step size and order of the next attempt.  *got = blocks written. */
int bdf_capture_blocks(bdf_handle* h, int n, long stride, long max_blocks, double* X_raw,
                       double* M, long* got);
/* Mass-action right-hand side f(y) and Jacobian of every cell of the
 * handle's problem at the device state y (cell-major); J receives
 * column-major blocks.  Either output may be NULL. */
int bdf_eval_rhs_jac(bdf_handle* h, const double* y, double* f, double* J);

/* ========================================================================
 * Learned block preconditioner (not part of the paper: an approximate
 * inverse X ~ (I - gamma J)^-1 per cell from a small MLP, used by a modified
 * Newton iteration with per-cell fallback to the exact block LU).
 *
 * Network: x = standardised [y (n values), log gamma]; ReLU(W1 x + b1);
 * ReLU(W2 . + b2); out = W3 . + b3; X = I + reshape(out, n x n) row-major.
 * hid = 256.  All matrix products use BF16 operands (round to nearest even)
 * with FP32 accumulation; inference runs on MFMA.  Parameters are one FP32
 * array W1 (hid x (n+1)) | b1 | W2 (hid x hid) | b2 | W3 (n^2 x hid) | b3,
 * row-major, with FP64 Adam moments.  Training inputs: X_raw (ns x (n+1))
 * FP64 rows [y, log gamma]; blocks M (ns x n^2) FP64, column-major per
 * sample.  Loss: mean over samples of |X M - I|_F^2 / n^2.
 * ======================================================================== */
typedef struct precond_handle precond_handle;

int precond_create(int n, int hid, int batch_cap, precond_handle** out);
int precond_destroy(precond_handle* h);
long precond_num_params(precond_handle* h);
/* host arrays of precond_num_params floats; grads may be NULL */
int precond_set_params(precond_handle* h, const float* params_host);
int precond_get_params(precond_handle* h, float* params_host, float* grads_host);
/* input standardisation, host arrays of n+1 doubles */
int precond_set_normalization(precond_handle* h, const double* mean_host, const double* std_host);
int precond_get_normalization(precond_handle* h, double* mean_host, double* std_host);
/* mean and standard deviation of the ns device rows X (n+1 values each) */
int precond_fit_normalization(precond_handle* h, const double* X, long ns, void* stream);
/* loss (host, synchronising if loss != NULL) and gradients of one batch of
 * B <= batch_cap device samples; gradients stay in the handle */
int precond_loss_grad(precond_handle* h, int B, const double* X, const double* M, double* loss,
                      void* stream);
/* one Adam step (Kingma & Ba) with the handle's gradients */
int precond_adam(precond_handle* h, double lr, double b1, double b2, double eps, void* stream);
/* one epoch over the ns samples in the order of the device permutation
 * perm (mini-batches of `batch`, the tail shorter than a batch is skipped);
 * *mean_loss = mean batch loss */
int precond_train_epoch(precond_handle* h, long ns, const double* X, const double* M,
                        const int* perm, int batch, double lr, double* mean_loss, void* stream);
/* mean loss over ns device samples (no update) */
int precond_eval_loss(precond_handle* h, long ns, const double* X, const double* M, double* loss,
                      void* stream);
/* X = I + out for B device samples into out (B x n^2 FP32); use_mfma = 1
 * for the MFMA kernel, 0 for the vector-FMA kernel with the same rounding */
int precond_forward(precond_handle* h, long B, const double* X, float* out, int use_mfma,
                    void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BDFGPU_H */
