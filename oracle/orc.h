/*
 * Serial FP64 CPU oracle for the batched BDF-Newton hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this code; only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no source with the GPU
 * path.  It is deliberately plain: straightforward loops in the order the
 * definitions give, compiled without FMA contraction or fast-math.
 *
 * Conventions
 *  - Vectors are cell-major: cell c owns entries [off_c, off_c + n_c), the
 *    grouping of many small systems into one ODE with a block-diagonal
 *    Jacobian (Section 2, Fig. blockdiag_jacobian).
 *  - Dense blocks are column-major n x n: A[i + j*n] is row i, column j.
 *  - Pivots are 0-based: piv[k] is the row exchanged with row k at step k.
 *
 * Parity pins: every routine here is checked by tests against closed forms,
 * brute force or independent library routines, except the step-control
 * heuristics of the integrator, whose constants the paper does not give
 * (parity unpinned for those constants; the integrator's arithmetic is
 * pinned through exactness, convergence-order and exp(At) tests).
 */
#ifndef ORC_H
#define ORC_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- N_Vector operations (streaming and reductions) -------- */
void orc_nv_linear_sum(long n, double a, const double* x, double b,
                       const double* y, double* z);
void orc_nv_linear_combination(int nv, const double* c,
                               const double* const* X, double* z, long n);
void orc_nv_scale_add_multi(int nv, const double* a, const double* x,
                            const double* const* Y, double* const* Z, long n);
void orc_nv_dot_prod_multi(int nv, const double* x, const double* const* Y,
                           double* d, long n);
double orc_nv_wrms_norm(long n, const double* x, const double* w);
double orc_nv_max_norm(long n, const double* x);
void orc_nv_ewt(long n, double rtol, double atol, const double* y, double* w);
void orc_nv_scale(long n, double c, const double* x, double* z);
void orc_nv_const(long n, double c, double* z);

/* ---------------- dense LU per block ------------------------------------ */
int orc_lu_factor(int n, double* A, int* piv);
void orc_lu_solve(int n, const double* LU, const int* piv, double* b);
int orc_lu_factor_f32(int n, float* A, int* piv);
void orc_lu_solve_f32(int n, const float* LU, const int* piv, float* b);
/* FP64 iterative refinement on top of an FP32 LU (LU32/piv32) of M.
 * Returns 0 if the residual reached FP64 working accuracy, 1 if the block
 * must be solved in FP64 instead (x then undefined).
 * *sweeps = corrections applied. */
int orc_lu_refine_solve(int n, const double* M, const float* LU32,
                        const int* piv32, const double* b, double* x,
                        int max_it, int* sweeps);

/* Inverse of one block by Gauss-Jordan elimination on [A | I] (column-major
 * A, n x n), partial pivoting with the first maximal |a_ik| (rows below and
 * including k), division by the pivot; Ainv receives the inverse, row-major
 * (Ainv[i*n + j]).  Returns 0, or k+1 for the first exactly-zero pivot
 * (Ainv then undefined).  The explicit-inverse block solve of the paper's
 * demonstration problem (Section 7). */
int orc_gj_inverse(int n, const double* A, double* Ainv);

/* ---------------- mass-action kinetics ---------------------------------- */
void orc_ma_rhs(int n, int R, const int* nu, const int* mu,
                const double* kappa, const double* y, double* f);
void orc_ma_jac(int n, int R, const int* nu, const int* mu,
                const double* kappa, const double* y, double* J);

/* ---------------- small MLP (learned block preconditioner) -------------- */
float orc_bf16_round(float x);
/* 1 (default): BF16 rounding at every matrix-product input; 0: exact FP64
 * (used only to check the backward pass against finite differences) */
void orc_set_bf16(int on);
typedef struct {
  int nin, hid, nout;          /* 22, 256, 441 */
  const float* W1; const float* b1;   /* W1: hid x nin row-major */
  const float* W2; const float* b2;   /* W2: hid x hid */
  const float* W3; const float* b3;   /* W3: nout x hid */
  const double* in_mean;       /* nin */
  const double* in_std;        /* nin */
} orc_mlp;
/* forward for one sample x_raw (nin values, before standardisation);
 * out receives nout values (FP64 accumulation of BF16-rounded operands). */
void orc_mlp_forward(const orc_mlp* m, const double* x_raw, double* out);
/* loss and parameter gradients over a batch of B samples;
 * X_raw: B x nin, Mb: B blocks n x n column-major (n*n == nout).
 * Gradients are written into gW1.. (same shapes as the weights, FP64). */
double orc_mlp_loss_grad(const orc_mlp* m, int B, const double* X_raw,
                         const double* Mb, double* gW1, double* gb1,
                         double* gW2, double* gb2, double* gW3, double* gb3);
/* one Adam step on a flat parameter array (FP32 master weights). */
void orc_adam_step(long np, float* p, const double* g, double* m1, double* m2,
                   long t, double lr, double b1, double b2, double eps);

/* ---------------- grouped BDF integrator -------------------------------- */
typedef struct {
  int ntopo;
  const int* topo_n;      /* species per topology */
  const int* topo_R;      /* reactions per topology */
  const int* topo_off;    /* offset of topology t in nu_all/mu_all */
  const int* nu_all;      /* concatenated R_t x n_t row-major */
  const int* mu_all;
  long ncells;
  const int* cell_topo;   /* topology of each cell */
  const double* rates;    /* concatenated R_c per cell */
  const double* y0;       /* concatenated n_c per cell */
  double t0;
} orc_problem;

enum { ORC_LS_LU64 = 0, ORC_LS_LU32REF = 1, ORC_LS_LEARNED = 2, ORC_LS_GJ = 3, ORC_LS_GMRES = 4 };

typedef struct {
  double rtol, atol;
  int qmax;          /* 1..5 */
  int maxcor;        /* Newton iterations per attempt (3) */
  double h0;         /* 0: starting step from the Hairer-Norsett-Wanner rule */
  int linsol;        /* ORC_LS_* */
  int refine_max_it; /* FP32 refinement sweeps before FP64 fallback */
  long max_steps;    /* per integrate call */
  double hmin;
  const orc_mlp* mlp;  /* learned mode */
  int nonneg;        /* 1: corrected solutions projected onto y >= 0 */
  int fixed_step;    /* 1: accepted steps keep h and q (no step-size or order
                        selection); used only by the convergence-order pins */
  int vc;            /* 1: variable-coefficient BDF (coefficients from the past
                        step sizes; order changes keep the interpolation) */
  int lazy;          /* 1: Newton matrix kept over steps (LU64, GJ; with GMRES the
                        block-Jacobi preconditioner) */
} orc_options;

typedef struct {
  long nsteps, nattempts, nfevals, nsetups, nniters, nncfails, netfails;
  long nlinsolves, refine_sweeps, refine_fallbacks;
  long lp_cell_solves, lp_fallback_cells, lp_step_fallbacks;
  long order_hist[6];
  long nprojections;
  long nstale_retries;   /* attempts redone with fresh factors (lazy) */
  long nliters;          /* GMRES iterations */
  long lp_unconverged;   /* learned: cells (first iteration: attempts) that kept
                            an iteration from being accepted */
} orc_stats;

typedef struct orc_bdf orc_bdf;

orc_bdf* orc_bdf_create(const orc_problem* p, const orc_options* o);
void orc_bdf_destroy(orc_bdf* b);
long orc_bdf_N(const orc_bdf* b);
/* one accepted internal step not passing t_end; returns 0 or < 0 error */
int orc_bdf_step(orc_bdf* b, double t_end);
/* steps until t == t_end exactly; returns 0 or < 0 error */
int orc_bdf_integrate(orc_bdf* b, double t_end);
void orc_bdf_get_y(const orc_bdf* b, double* y);
void orc_bdf_get_stats(const orc_bdf* b, orc_stats* s);

/* integrator state for single-step parity checks */
typedef struct {
  double t, h, err_last;
  int q, qwait, qprime_pending, initialized;
  double hu; int qu;     /* last accepted step */
  /* order-selection estimates of the last accepted step (-1 when the step
   * did not select an order, or the order had no such neighbour) and the
   * growth factor that selection proposed before the hysteresis test */
  double err_qm1, err_qp1, eta_proposed;
  int q_proposed;
} orc_scalars;
void orc_bdf_get_scalars(const orc_bdf* b, orc_scalars* s);
/* computes the starting step and history (as the first step would) without
 * stepping; a no-op once initialised */
void orc_bdf_init(orc_bdf* b, double t_end);
void orc_bdf_set_scalars(orc_bdf* b, const orc_scalars* s);
/* history z[j] (j = 0..5) and previous correction; each N doubles */
void orc_bdf_get_history(const orc_bdf* b, double* z6, double* dprev);
void orc_bdf_set_history(orc_bdf* b, const double* z6, const double* dprev);
/* the BDF coefficient vector for order q (q+1 values) and the error
 * constant 1/((q+1) H_q H_{q+1}); exposed for the exactness pins */
void orc_bdf_coeffs(int q, double* l, double* tq);
/* variable coefficients: past accepted step sizes (most recent first, at
 * most 6) and the scale and step of the saved correction; for the pins */
void orc_bdf_set_past_steps(orc_bdf* b, int k, const double* tau, double dprev_c,
                            double dprev_h);
int orc_bdf_get_past_steps(const orc_bdf* b, double* tau, double* dprev_c, double* dprev_h);
/* lazy Newton matrix: gamma and step count of the last setup, carried
 * convergence-rate estimate */
void orc_bdf_get_lazy(const orc_bdf* b, double* gamma_s, long* nst_s, double* crate);
/* GMRES of the Newton-Krylov path on a block-diagonal system (blocks of
 * n[c], column-major M; block-Jacobi preconditioner from the LU factors LU,
 * piv): del with |W (r - M del)|_2 <= tol, W = diag(w); returns the
 * iterations taken (at most 5). */
int orc_gmres_solve(long ncells, const int* n, const double* M, const double* LU,
                    const int* piv, const double* w, const double* r, double tol, double* del);

#ifdef __cplusplus
}
#endif
#endif
