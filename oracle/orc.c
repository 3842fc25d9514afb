/*
 * Serial FP64 CPU oracle for the batched BDF-Newton hot path.
 * TEST INFRASTRUCTURE ONLY: loaded by tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 *
 * What each part follows
 *  - Vector operations: the streaming / reduction split of Section 2 and
 *    the reduction semantics of Section 4.1 (reductions produce one scalar).
 *    The fused operations (linear combination, scale-add-multi, multiple
 *    dot products, WRMS norm) are not defined in the paper; their plain
 *    definitions are written out here.  Reductions add in index order with
 *    Neumaier's compensated summation.
 *  - Dense LU: the batched block-diagonal direct solve of Section 5 (one
 *    shared pattern, one dense block per cell) as LAPACK getrf semantics:
 *    right-looking partial pivoting, first maximal pivot, whole-row swaps,
 *    division by the pivot.
 *  - The Newton iteration over all cells at once with a block-diagonal
 *    solve and whole-step retry on any failure: Section 7 (task-local
 *    nonlinear solver and ensemble failure rule).
 *  - The BDF integrator itself is not given by the paper (it only names
 *    CVODE); this is a fixed-coefficient Nordsieck BDF of orders 1..5 with
 *    CVODE-style weights, Newton and local error test.  Its constants are
 *    the readings listed in the design notes (parity unpinned for the
 *    step-control constants themselves).
 */
#include "orc.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Neumaier compensated summation (A. Neumaier, 1974)                       */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void ns_add(nsum* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}
static double ns_val(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* N_Vector operations                                                      */
/* ------------------------------------------------------------------------ */
void orc_nv_linear_sum(long n, double a, const double* x, double b,
                       const double* y, double* z) {
  for (long i = 0; i < n; ++i) {
    double xi = x[i], yi = y[i];
    z[i] = a * xi + b * yi;
  }
}

void orc_nv_linear_combination(int nv, const double* c,
                               const double* const* X, double* z, long n) {
  for (long i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s = s + c[j] * X[j][i];
    z[i] = s;
  }
}

void orc_nv_scale_add_multi(int nv, const double* a, const double* x,
                            const double* const* Y, double* const* Z, long n) {
  for (long i = 0; i < n; ++i) {
    double xi = x[i];
    for (int j = 0; j < nv; ++j) Z[j][i] = a[j] * xi + Y[j][i];
  }
}

void orc_nv_dot_prod_multi(int nv, const double* x, const double* const* Y,
                           double* d, long n) {
  for (int j = 0; j < nv; ++j) {
    nsum s = {0.0, 0.0};
    for (long i = 0; i < n; ++i) ns_add(&s, x[i] * Y[j][i]);
    d[j] = ns_val(&s);
  }
}

static double orc_nv_dot_prod_multi_1(long n, const double* x, const double* y) {
  const double* Y[1] = {y};
  double d;
  orc_nv_dot_prod_multi(1, x, Y, &d, n);
  return d;
}

double orc_nv_wrms_norm(long n, const double* x, const double* w) {
  if (n <= 0) return 0.0;
  nsum s = {0.0, 0.0};
  for (long i = 0; i < n; ++i) {
    double v = x[i] * w[i];
    ns_add(&s, v * v);
  }
  return sqrt(ns_val(&s) / (double)n);
}

double orc_nv_max_norm(long n, const double* x) {
  double m = 0.0;
  for (long i = 0; i < n; ++i)
    if (fabs(x[i]) > m) m = fabs(x[i]);
  return m;
}

void orc_nv_ewt(long n, double rtol, double atol, const double* y, double* w) {
  for (long i = 0; i < n; ++i) w[i] = 1.0 / (rtol * fabs(y[i]) + atol);
}

void orc_nv_scale(long n, double c, const double* x, double* z) {
  for (long i = 0; i < n; ++i) z[i] = c * x[i];
}

void orc_nv_const(long n, double c, double* z) {
  for (long i = 0; i < n; ++i) z[i] = c;
}

/* ------------------------------------------------------------------------ */
/* Dense LU, one block                                                      */
/* ------------------------------------------------------------------------ */
#define AT(A, i, j, n) (A)[(i) + (long)(j) * (n)]

int orc_lu_factor(int n, double* A, int* piv) {
  int info = 0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double amax = fabs(AT(A, k, k, n));
    for (int i = k + 1; i < n; ++i) {
      double v = fabs(AT(A, i, k, n));
      if (v > amax) { amax = v; p = i; }
    }
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        double t = AT(A, k, j, n);
        AT(A, k, j, n) = AT(A, p, j, n);
        AT(A, p, j, n) = t;
      }
    if (AT(A, k, k, n) == 0.0) {
      if (!info) info = k + 1;
      continue;
    }
    for (int i = k + 1; i < n; ++i) AT(A, i, k, n) = AT(A, i, k, n) / AT(A, k, k, n);
    for (int j = k + 1; j < n; ++j)
      for (int i = k + 1; i < n; ++i)
        AT(A, i, j, n) = AT(A, i, j, n) - AT(A, i, k, n) * AT(A, k, j, n);
  }
  return info;
}

void orc_lu_solve(int n, const double* LU, const int* piv, double* b) {
  for (int k = 0; k < n; ++k) {
    int p = piv[k];
    if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
  }
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int j = 0; j < i; ++j) s = s - AT(LU, i, j, n) * b[j];
    b[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s = s - AT(LU, i, j, n) * b[j];
    b[i] = s / AT(LU, i, i, n);
  }
}

int orc_lu_factor_f32(int n, float* A, int* piv) {
  int info = 0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    float amax = fabsf(AT(A, k, k, n));
    for (int i = k + 1; i < n; ++i) {
      float v = fabsf(AT(A, i, k, n));
      if (v > amax) { amax = v; p = i; }
    }
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        float t = AT(A, k, j, n);
        AT(A, k, j, n) = AT(A, p, j, n);
        AT(A, p, j, n) = t;
      }
    if (AT(A, k, k, n) == 0.0f) {
      if (!info) info = k + 1;
      continue;
    }
    for (int i = k + 1; i < n; ++i) AT(A, i, k, n) = AT(A, i, k, n) / AT(A, k, k, n);
    for (int j = k + 1; j < n; ++j)
      for (int i = k + 1; i < n; ++i)
        AT(A, i, j, n) = AT(A, i, j, n) - AT(A, i, k, n) * AT(A, k, j, n);
  }
  return info;
}

void orc_lu_solve_f32(int n, const float* LU, const int* piv, float* b) {
  for (int k = 0; k < n; ++k) {
    int p = piv[k];
    if (p != k) { float t = b[k]; b[k] = b[p]; b[p] = t; }
  }
  for (int i = 0; i < n; ++i) {
    float s = b[i];
    for (int j = 0; j < i; ++j) s = s - AT(LU, i, j, n) * b[j];
    b[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    float s = b[i];
    for (int j = i + 1; j < n; ++j) s = s - AT(LU, i, j, n) * b[j];
    b[i] = s / AT(LU, i, i, n);
  }
}

/* Gauss-Jordan elimination on the augmented matrix [A | I]: at step k the
 * pivot row (first maximal |a_ik|, i >= k) is exchanged into row k and
 * divided by its pivot, then a multiple of it is subtracted from every other
 * row, so that column k becomes the unit vector; after n steps the right
 * half holds the inverse.  Plain loops, division by the pivot. */
int orc_gj_inverse(int n, const double* A, double* Ainv) {
  double* W = (double*)malloc(sizeof(double) * (size_t)n * 2 * n);   /* row-major n x 2n */
  if (!W) return -1;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      W[i * 2 * n + j] = AT(A, i, j, n);
      W[i * 2 * n + n + j] = i == j ? 1.0 : 0.0;
    }
  int info = 0;
  for (int k = 0; k < n && !info; ++k) {
    int p = k;
    double amax = fabs(W[k * 2 * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = fabs(W[i * 2 * n + k]);
      if (v > amax) { amax = v; p = i; }
    }
    if (p != k)
      for (int j = 0; j < 2 * n; ++j) {
        double t = W[k * 2 * n + j];
        W[k * 2 * n + j] = W[p * 2 * n + j];
        W[p * 2 * n + j] = t;
      }
    double d = W[k * 2 * n + k];
    if (d == 0.0) { info = k + 1; break; }
    for (int j = 0; j < 2 * n; ++j) W[k * 2 * n + j] = W[k * 2 * n + j] / d;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      double f = W[i * 2 * n + k];
      for (int j = 0; j < 2 * n; ++j) W[i * 2 * n + j] = W[i * 2 * n + j] - f * W[k * 2 * n + j];
    }
  }
  if (!info)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Ainv[i * n + j] = W[i * 2 * n + n + j];
  free(W);
  return info;
}

/* Mixed-precision refinement for one block.
 * x0 = FP32 solve of b; then up to max_it corrections d = FP32 solve of the
 * FP64 residual r = b - M x.  Converged when the residual is at FP64
 * working accuracy, |r|_inf <= sqrt(n) * eps64 * |M|_inf * |x|_inf (the
 * residual test of LAPACK's mixed-precision dsgesv).  Not converged after
 * max_it corrections, or a correction that fails to halve (|d_k| >
 * 0.5 |d_{k-1}|, the sign that cond(M) * eps32 is near 1), means the block
 * must be solved in FP64 instead: returns 1 and leaves x undefined. */
int orc_lu_refine_solve(int n, const double* M, const float* LU32,
                        const int* piv32, const double* b, double* x,
                        int max_it, int* sweeps) {
  float* v = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double mnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s = s + fabs(AT(M, i, j, n));
    if (s > mnorm) mnorm = s;
  }
  for (int i = 0; i < n; ++i) v[i] = (float)b[i];
  orc_lu_solve_f32(n, LU32, piv32, v);
  for (int i = 0; i < n; ++i) x[i] = (double)v[i];
  const double eps64 = 2.220446049250313e-16;
  double dprev = 0.0;
  int it, status = 1;
  *sweeps = 0;
  for (it = 0; it <= max_it; ++it) {
    double rn = 0.0, xn = 0.0;
    for (int i = 0; i < n; ++i) {
      double s = b[i];
      for (int j = 0; j < n; ++j) s = s - AT(M, i, j, n) * x[j];
      r[i] = s;
      if (fabs(s) > rn) rn = fabs(s);
      if (fabs(x[i]) > xn) xn = fabs(x[i]);
    }
    if (!(rn == rn) || !(xn == xn)) break;           /* NaN */
    if (rn <= sqrt((double)n) * eps64 * mnorm * xn) { status = 0; break; }
    if (it == max_it) break;
    for (int i = 0; i < n; ++i) v[i] = (float)r[i];
    orc_lu_solve_f32(n, LU32, piv32, v);
    double dn = 0.0;
    for (int i = 0; i < n; ++i) {
      x[i] = x[i] + (double)v[i];
      if (fabs((double)v[i]) > dn) dn = fabs((double)v[i]);
    }
    *sweeps = it + 1;
    if (it >= 1 && dn > 0.5 * dprev) break;          /* stagnation */
    dprev = dn;
  }
  free(v);
  free(r);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Mass-action kinetics: r_k = kappa_k prod_s y_s^nu_ks,                     */
/* f_s = sum_k (mu_ks - nu_ks) r_k, J_sj = df_s/dy_j (analytic).             */
/* ------------------------------------------------------------------------ */
static double ipow(double y, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r = r * y;
  return r;
}

void orc_ma_rhs(int n, int R, const int* nu, const int* mu,
                const double* kappa, const double* y, double* f) {
  for (int s = 0; s < n; ++s) f[s] = 0.0;
  for (int k = 0; k < R; ++k) {
    double r = kappa[k];
    for (int s = 0; s < n; ++s) r = r * ipow(y[s], nu[k * n + s]);
    for (int s = 0; s < n; ++s) {
      int c = mu[k * n + s] - nu[k * n + s];
      if (c) f[s] = f[s] + (double)c * r;
    }
  }
}

void orc_ma_jac(int n, int R, const int* nu, const int* mu,
                const double* kappa, const double* y, double* J) {
  for (long i = 0; i < (long)n * n; ++i) J[i] = 0.0;
  for (int k = 0; k < R; ++k) {
    for (int j = 0; j < n; ++j) {
      int e = nu[k * n + j];
      if (!e) continue;
      double d = kappa[k] * (double)e * ipow(y[j], e - 1);
      for (int s = 0; s < n; ++s)
        if (s != j) d = d * ipow(y[s], nu[k * n + s]);
      for (int s = 0; s < n; ++s) {
        int c = mu[k * n + s] - nu[k * n + s];
        if (c) AT(J, s, j, n) = AT(J, s, j, n) + (double)c * d;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Small MLP with BF16 operands at every matrix product                     */
/* ------------------------------------------------------------------------ */
float orc_bf16_round(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) {
    if (u & 0x007fffffu) u |= 0x00400000u;
    u &= 0xffff0000u;
  } else {
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
  }
  float r;
  memcpy(&r, &u, 4);
  return r;
}

/* Rounding points can be switched off so that finite differences can check
 * the backward pass (rounding is passed straight through in the gradient). */
static int g_bf16_on = 1;
void orc_set_bf16(int on) { g_bf16_on = on; }

static double bf(double v) {
  return g_bf16_on ? (double)orc_bf16_round((float)v) : v;
}

typedef struct {
  double* xs;  /* nin  : standardised, BF16-rounded input */
  double* a1;  /* hid  : pre-activation 1 */
  double* h1;  /* hid  : BF16-rounded ReLU(a1) */
  double* a2;
  double* h2;
  double* out; /* nout */
} mlp_trace;

static void mlp_fwd(const orc_mlp* m, const double* x_raw, mlp_trace* t) {
  const int ni = m->nin, nh = m->hid, no = m->nout;
  for (int i = 0; i < ni; ++i) t->xs[i] = bf((x_raw[i] - m->in_mean[i]) / m->in_std[i]);
  for (int o = 0; o < nh; ++o) {
    double s = 0.0;
    for (int i = 0; i < ni; ++i) s = s + bf(m->W1[(long)o * ni + i]) * t->xs[i];
    s = s + (double)m->b1[o];
    t->a1[o] = s;
    t->h1[o] = bf(s > 0.0 ? s : 0.0);
  }
  for (int o = 0; o < nh; ++o) {
    double s = 0.0;
    for (int i = 0; i < nh; ++i) s = s + bf(m->W2[(long)o * nh + i]) * t->h1[i];
    s = s + (double)m->b2[o];
    t->a2[o] = s;
    t->h2[o] = bf(s > 0.0 ? s : 0.0);
  }
  for (int o = 0; o < no; ++o) {
    double s = 0.0;
    for (int i = 0; i < nh; ++i) s = s + bf(m->W3[(long)o * nh + i]) * t->h2[i];
    t->out[o] = s + (double)m->b3[o];
  }
}

static mlp_trace trace_alloc(const orc_mlp* m) {
  mlp_trace t;
  t.xs = (double*)calloc((size_t)m->nin, sizeof(double));
  t.a1 = (double*)calloc((size_t)m->hid, sizeof(double));
  t.h1 = (double*)calloc((size_t)m->hid, sizeof(double));
  t.a2 = (double*)calloc((size_t)m->hid, sizeof(double));
  t.h2 = (double*)calloc((size_t)m->hid, sizeof(double));
  t.out = (double*)calloc((size_t)m->nout, sizeof(double));
  return t;
}
static void trace_free(mlp_trace* t) {
  free(t->xs); free(t->a1); free(t->h1); free(t->a2); free(t->h2); free(t->out);
}

void orc_mlp_forward(const orc_mlp* m, const double* x_raw, double* out) {
  mlp_trace t = trace_alloc(m);
  mlp_fwd(m, x_raw, &t);
  memcpy(out, t.out, sizeof(double) * (size_t)m->nout);
  trace_free(&t);
}

/* Loss L = mean_b |X_b M_b - I|_F^2 / n^2 with X = I + reshape(out)
 * (row-major: X[i][j] = out[i*n + j]).  The rounding to BF16 of each matrix
 * product's inputs is passed straight through in the backward pass; the
 * backward products use the same BF16-rounded weights as the forward. */
double orc_mlp_loss_grad(const orc_mlp* m, int B, const double* X_raw,
                         const double* Mb, double* gW1, double* gb1,
                         double* gW2, double* gb2, double* gW3, double* gb3) {
  const int ni = m->nin, nh = m->hid, no = m->nout;
  int n = 0;
  while ((n + 1) * (n + 1) <= no) ++n;
  memset(gW1, 0, sizeof(double) * (size_t)nh * ni);
  memset(gb1, 0, sizeof(double) * (size_t)nh);
  memset(gW2, 0, sizeof(double) * (size_t)nh * nh);
  memset(gb2, 0, sizeof(double) * (size_t)nh);
  memset(gW3, 0, sizeof(double) * (size_t)no * nh);
  memset(gb3, 0, sizeof(double) * (size_t)no);
  mlp_trace t = trace_alloc(m);
  double* X = (double*)malloc(sizeof(double) * (size_t)no);
  double* E = (double*)malloc(sizeof(double) * (size_t)no);
  double* dout = (double*)malloc(sizeof(double) * (size_t)no);
  double* dh2 = (double*)malloc(sizeof(double) * (size_t)nh);
  double* dh1 = (double*)malloc(sizeof(double) * (size_t)nh);
  const double scale = 1.0 / ((double)no * (double)B);
  double L = 0.0;
  for (int b = 0; b < B; ++b) {
    const double* M = Mb + (long)b * no;
    mlp_fwd(m, X_raw + (long)b * ni, &t);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        X[i * n + j] = t.out[i * n + j] + (i == j ? 1.0 : 0.0);
    /* E = X M - I   (M column-major) */
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = s + X[i * n + k] * AT(M, k, j, n);
        E[i * n + j] = s - (i == j ? 1.0 : 0.0);
        L = L + E[i * n + j] * E[i * n + j] * scale;
      }
    /* dL/dX = 2 E M^T * scale */
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s = s + E[i * n + j] * AT(M, k, j, n);
        dout[i * n + k] = 2.0 * s * scale;
      }
    for (int o = 0; o < no; ++o) {
      gb3[o] += dout[o];
      for (int i = 0; i < nh; ++i) gW3[(long)o * nh + i] += dout[o] * t.h2[i];
    }
    for (int i = 0; i < nh; ++i) {
      double s = 0.0;
      for (int o = 0; o < no; ++o) s = s + bf(m->W3[(long)o * nh + i]) * dout[o];
      dh2[i] = t.a2[i] > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < nh; ++o) {
      gb2[o] += dh2[o];
      for (int i = 0; i < nh; ++i) gW2[(long)o * nh + i] += dh2[o] * t.h1[i];
    }
    for (int i = 0; i < nh; ++i) {
      double s = 0.0;
      for (int o = 0; o < nh; ++o) s = s + bf(m->W2[(long)o * nh + i]) * dh2[o];
      dh1[i] = t.a1[i] > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < nh; ++o) {
      gb1[o] += dh1[o];
      for (int i = 0; i < ni; ++i) gW1[(long)o * ni + i] += dh1[o] * t.xs[i];
    }
  }
  free(X); free(E); free(dout); free(dh2); free(dh1);
  trace_free(&t);
  return L;
}

/* Adam (Kingma & Ba, 2015) on FP32 master weights, moments in FP64. */
void orc_adam_step(long np, float* p, const double* g, double* m1, double* m2,
                   long t, double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t);
  double c2 = 1.0 - pow(b2, (double)t);
  for (long i = 0; i < np; ++i) {
    m1[i] = b1 * m1[i] + (1.0 - b1) * g[i];
    m2[i] = b2 * m2[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m1[i] / c1, vh = m2[i] / c2;
    p[i] = (float)((double)p[i] - lr * mh / (sqrt(vh) + eps));
  }
}

/* ------------------------------------------------------------------------ */
/* Grouped fixed-coefficient Nordsieck BDF                                  */
/* ------------------------------------------------------------------------ */
#define QMAX_ALL 5
#define MXNCF 10      /* Newton failures per step before giving up */
#define MXNEF 7       /* error-test failures per step before giving up */
#define CRDOWN 0.3    /* memory factor of the convergence-rate estimate */
#define RDIV 2.0      /* divergence factor */
#define NLS_COEF 0.1  /* Newton tolerance in WRMS units of the correction */
#define ETA_MAX 10.0  /* largest step growth */
#define ETA_MIN_EF 0.2
#define ETA_CF 0.25
#define ETA_RESTART 0.1
#define THRESH 1.5    /* hysteresis: smaller proposed growth keeps h, q */
#define BIAS_QM1 1.3
#define BIAS_Q 1.2
#define BIAS_QP1 1.4
#define ADDON 1e-6
#define LP_CELL_RATIO 0.9
#define MSBP 20       /* lazy setup: accepted steps between fresh Newton matrices */
#define DGMAX 0.3     /* lazy setup: largest |gamma / gamma_setup - 1| kept */
#define NTAU (QMAX_ALL + 1)
#define KRY_MAXL 5         /* GMRES: Krylov dimension, no restarts */
#define KRY_EPLIN 0.05     /* GMRES: tolerance factor on the Newton tolerance */

struct orc_bdf {
  orc_problem p;
  orc_options o;
  long N, nmat;
  long *yoff, *roff, *moff;
  int *cn, *cR;
  const int **cnu, **cmu;
  double* z[QMAX_ALL + 1];
  double* zp[QMAX_ALL + 1];
  double *dprev, *acor, *y, *w, *f, *r, *del, *tmp;
  double *M, *LU;
  float* LU32;
  int *piv, *piv32, *cellmode, *cellinfo;
  double *X, *dcell_prev;
  double t, h, err_last, hu;
  int q, qwait, qu, initialized;
  double err_qm1, err_qp1, eta_prop;
  int q_prop;
  /* variable coefficients: accepted step sizes, most recent first, and the
   * scale c of the previous correction (D = c acor, see vc_order_terms) */
  double tau[NTAU];
  int ntau;
  double dprev_c, dprev_h;
  /* lazy Newton matrix: stored factors valid, forced refresh, gamma and
   * step count of the last setup, convergence-rate estimate carried over */
  int m_valid, force_setup;
  long nst_s;
  double gamma_s, crate_keep;
  double* V;   /* GMRES: Krylov basis, KRY_MAXL + 1 vectors of N */
  orc_stats st;
};

static double harmonic(int q) {
  double s = 0.0;
  for (int i = 1; i <= q; ++i) s += 1.0 / (double)i;
  return s;
}

static double factorial(int q) {
  double s = 1.0;
  for (int i = 2; i <= q; ++i) s *= (double)i;
  return s;
}

void orc_bdf_coeffs(int q, double* l, double* tq) {
  /* coefficients of prod_{i=1..q} (1 + x/i), divided by H_q */
  double c[QMAX_ALL + 2];
  for (int j = 0; j <= QMAX_ALL + 1; ++j) c[j] = 0.0;
  c[0] = 1.0;
  for (int i = 1; i <= q; ++i)
    for (int j = i; j >= 1; --j) c[j] = c[j] + c[j - 1] / (double)i;
  double H = harmonic(q);
  for (int j = 0; j <= q; ++j) l[j] = c[j] / H;
  /* local error of order q from the correction: with an interpolating
   * history the correction is H_{q+1} times the (q+1)-th backward difference
   * and the truncation error is that difference over (q+1) H_q */
  if (tq) *tq = 1.0 / ((double)(q + 1) * H * harmonic(q + 1));
}

/* ---- variable-coefficient BDF (option vc) --------------------------------
 * Past accepted points t_{n-i} of an attempt of size h that reaches t_n sit
 * at s = -xi_i in units of h: xi_1 = 1 and xi_{i+1} = xi_i + tau_{i-1} / h
 * (tau_0 the last accepted step); points older than the known history are
 * taken one h apart, which is the start of an integration or a restart.
 * xi[1..k] are filled (xi[0] = 0). */
static void vc_xi(const orc_bdf* b, double h, int k, double* xi) {
  xi[0] = 0.0;
  xi[1] = 1.0;
  for (int i = 2; i <= k; ++i)
    xi[i] = xi[i - 1] + (i - 2 < b->ntau ? b->tau[i - 2] / h : 1.0);
}

/* c[j] = [s^j] prod_{i=1..k} (1 + s/xi_i) (degree k). */
static void poly_unit(const double* xi, int k, double* c) {
  for (int j = 0; j <= QMAX_ALL + 2; ++j) c[j] = 0.0;
  c[0] = 1.0;
  for (int i = 1; i <= k; ++i)
    for (int j = i; j >= 1; --j) c[j] = c[j] + c[j - 1] / xi[i];
}

/* c[j] = [s^j] s prod_{i=1..k} (s + xi_i) (degree k + 1, c[0] = 0). */
static void poly_through(const double* xi, int k, double* c) {
  for (int j = 0; j <= QMAX_ALL + 2; ++j) c[j] = 0.0;
  c[1] = 1.0;
  for (int i = 1; i <= k; ++i)
    for (int j = i + 1; j >= 1; --j) c[j] = c[j - 1] + xi[i] * c[j];
}

/* Variable-coefficient corrector of order q (reading: the step is the BDF
 * formula on the actual past grid).  The correction polynomial
 * prod_{i=1..q} (1 + s/xi_i) vanishes at the q previous accepted points,
 * so the corrected history keeps interpolating the last q + 1 accepted
 * values; normalised to slope 1 at s = 0: l_j = [s^j] prod / S_q with
 * S_k = sum_{i<=k} 1/xi_i.  With the history the interpolant of exact
 * values, the step's local error is the correction times
 * l_0 (1/xi_{q+1}) / S_{q+1} (the error polynomial of a degree-(q+1)
 * solution is a multiple of prod_{i=1..q+1} (s + xi_i)), so
 * tq = (1/xi_{q+1}) / (S_q S_{q+1}).  Constant steps (xi_i = i) give the
 * fixed coefficients. */
static void vc_coeffs(int q, const double* xi, double* l, double* tq) {
  double c[QMAX_ALL + 3];
  poly_unit(xi, q, c);
  double Sq = 0.0;
  for (int i = 1; i <= q; ++i) Sq = Sq + 1.0 / xi[i];
  for (int j = 0; j <= q; ++j) l[j] = c[j] / Sq;
  const double Sq1 = Sq + 1.0 / xi[q + 1];
  *tq = (1.0 / xi[q + 1]) / (Sq * Sq1);
}

orc_bdf* orc_bdf_create(const orc_problem* p, const orc_options* o) {
  if (o->lazy && o->linsol != ORC_LS_LU64 && o->linsol != ORC_LS_GJ && o->linsol != ORC_LS_GMRES)
    return NULL;
  orc_bdf* b = (orc_bdf*)calloc(1, sizeof(orc_bdf));
  b->p = *p;
  b->o = *o;
  long nc = p->ncells;
  b->yoff = (long*)calloc((size_t)nc + 1, sizeof(long));
  b->roff = (long*)calloc((size_t)nc + 1, sizeof(long));
  b->moff = (long*)calloc((size_t)nc + 1, sizeof(long));
  b->cn = (int*)calloc((size_t)nc + 1, sizeof(int));
  b->cR = (int*)calloc((size_t)nc + 1, sizeof(int));
  b->cnu = (const int**)calloc((size_t)nc + 1, sizeof(int*));
  b->cmu = (const int**)calloc((size_t)nc + 1, sizeof(int*));
  for (long c = 0; c < nc; ++c) {
    int t = p->cell_topo[c];
    b->cn[c] = p->topo_n[t];
    b->cR[c] = p->topo_R[t];
    b->cnu[c] = p->nu_all + p->topo_off[t];
    b->cmu[c] = p->mu_all + p->topo_off[t];
    b->yoff[c + 1] = b->yoff[c] + b->cn[c];
    b->roff[c + 1] = b->roff[c] + b->cR[c];
    b->moff[c + 1] = b->moff[c] + (long)b->cn[c] * b->cn[c];
  }
  b->N = b->yoff[nc];
  b->nmat = b->moff[nc];
  size_t N = (size_t)(b->N > 0 ? b->N : 1);
  for (int j = 0; j <= QMAX_ALL; ++j) {
    b->z[j] = (double*)calloc(N, sizeof(double));
    b->zp[j] = (double*)calloc(N, sizeof(double));
  }
  b->dprev = (double*)calloc(N, sizeof(double));
  b->acor = (double*)calloc(N, sizeof(double));
  b->y = (double*)calloc(N, sizeof(double));
  b->w = (double*)calloc(N, sizeof(double));
  b->f = (double*)calloc(N, sizeof(double));
  b->r = (double*)calloc(N, sizeof(double));
  b->del = (double*)calloc(N, sizeof(double));
  b->tmp = (double*)calloc(N, sizeof(double));
  size_t NM = (size_t)(b->nmat > 0 ? b->nmat : 1);
  b->M = (double*)calloc(NM, sizeof(double));
  b->LU = (double*)calloc(NM, sizeof(double));
  b->LU32 = (float*)calloc(NM, sizeof(float));
  b->piv = (int*)calloc(N, sizeof(int));
  b->piv32 = (int*)calloc(N, sizeof(int));
  b->cellmode = (int*)calloc((size_t)nc + 1, sizeof(int));
  b->cellinfo = (int*)calloc((size_t)nc + 1, sizeof(int));
  b->dcell_prev = (double*)calloc((size_t)nc + 1, sizeof(double));
  if (o->linsol == ORC_LS_LEARNED || o->linsol == ORC_LS_GJ)
    b->X = (double*)calloc(NM, sizeof(double));
  if (o->linsol == ORC_LS_GMRES) b->V = (double*)calloc((KRY_MAXL + 1) * N, sizeof(double));
  b->t = p->t0;
  b->err_qm1 = b->err_qp1 = -1.0;
  b->eta_prop = 1.0;
  memcpy(b->z[0], p->y0, sizeof(double) * (size_t)b->N);
  return b;
}

void orc_bdf_destroy(orc_bdf* b) {
  if (!b) return;
  free(b->yoff); free(b->roff); free(b->moff); free(b->cn); free(b->cR);
  free(b->cnu); free(b->cmu);
  for (int j = 0; j <= QMAX_ALL; ++j) { free(b->z[j]); free(b->zp[j]); }
  free(b->dprev); free(b->acor); free(b->y); free(b->w); free(b->f);
  free(b->r); free(b->del); free(b->tmp); free(b->M); free(b->LU);
  free(b->LU32); free(b->piv); free(b->piv32); free(b->cellmode);
  free(b->cellinfo); free(b->dcell_prev); free(b->X); free(b->V);
  free(b);
}

long orc_bdf_N(const orc_bdf* b) { return b->N; }

static void rhs_all(orc_bdf* b, const double* y, double* f) {
  for (long c = 0; c < b->p.ncells; ++c)
    orc_ma_rhs(b->cn[c], b->cR[c], b->cnu[c], b->cmu[c], b->p.rates + b->roff[c],
               y + b->yoff[c], f + b->yoff[c]);
  b->st.nfevals++;
}

static double wrms(const orc_bdf* b, const double* x) {
  return orc_nv_wrms_norm(b->N, x, b->w);
}

static void rescale(orc_bdf* b, double eta) {
  double fac = 1.0;
  for (int j = 1; j <= b->q; ++j) {
    fac = fac * eta;
    for (long i = 0; i < b->N; ++i) b->z[j][i] = b->z[j][i] * fac;
  }
}

/* Starting step: Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4,
 * with WRMS norms and p = 1. */
static double hnw_h0(orc_bdf* b, double t_end) {
  long N = b->N;
  orc_nv_ewt(N, b->o.rtol, b->o.atol, b->z[0], b->w);
  rhs_all(b, b->z[0], b->f);
  double d0 = wrms(b, b->z[0]);
  double d1 = wrms(b, b->f);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  if (h0 > t_end - b->t) h0 = t_end - b->t;
  for (long i = 0; i < N; ++i) b->tmp[i] = b->z[0][i] + h0 * b->f[i];
  rhs_all(b, b->tmp, b->r);
  for (long i = 0; i < N; ++i) b->r[i] = b->r[i] - b->f[i];
  double d2 = wrms(b, b->r) / h0;
  double dm = d1 > d2 ? d1 : d2;
  double h1 = dm <= 1e-15 ? (h0 * 1e-3 > 1e-6 ? h0 * 1e-3 : 1e-6)
                          : pow(0.01 / dm, 1.0 / 2.0);
  double h = 100.0 * h0 < h1 ? 100.0 * h0 : h1;
  return h;
}

static void initialize(orc_bdf* b, double t_end) {
  long N = b->N;
  double h = b->o.h0 > 0.0 ? b->o.h0 : hnw_h0(b, t_end);
  if (h > t_end - b->t) h = t_end - b->t;
  rhs_all(b, b->z[0], b->f);
  for (long i = 0; i < N; ++i) b->z[1][i] = h * b->f[i];
  for (int j = 2; j <= QMAX_ALL; ++j) memset(b->z[j], 0, sizeof(double) * (size_t)N);
  memset(b->dprev, 0, sizeof(double) * (size_t)N);
  b->h = h;
  b->q = 1;
  b->qwait = 2;
  b->ntau = 0;
  b->m_valid = 0;
  b->initialized = 1;
}

/* Fresh Jacobian at the predicted state and M = I - gamma J, per cell. */
static void build_M(orc_bdf* b, long c, double gamma) {
  int n = b->cn[c];
  double* M = b->M + b->moff[c];
  orc_ma_jac(n, b->cR[c], b->cnu[c], b->cmu[c], b->p.rates + b->roff[c],
             b->zp[0] + b->yoff[c], M);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      AT(M, i, j, n) = (i == j ? 1.0 : 0.0) - gamma * AT(M, i, j, n);
}

static int factor64(orc_bdf* b, long c) {
  int n = b->cn[c];
  memcpy(b->LU + b->moff[c], b->M + b->moff[c], sizeof(double) * (size_t)n * n);
  return orc_lu_factor(n, b->LU + b->moff[c], b->piv + b->yoff[c]);
}

/* Solve M del_c = r_c for one cell according to cellmode:
 * 0 FP64 LU, 1 FP32 LU + refinement, 2 learned X, 3 FP64 LU after fallback,
 * 5 Gauss-Jordan inverse. */
static int cell_solve(orc_bdf* b, long c) {
  int n = b->cn[c];
  long off = b->yoff[c];
  double* d = b->del + off;
  const double* r = b->r + off;
  int mode = b->cellmode[c];
  if (mode == 1) {
    int sw = 0;
    int st = orc_lu_refine_solve(n, b->M + b->moff[c], b->LU32 + b->moff[c],
                                 b->piv32 + off, r, d, b->o.refine_max_it, &sw);
    b->st.refine_sweeps += sw;
    if (st == 0) return 0;
    b->st.refine_fallbacks++;
    b->cellmode[c] = 3;
    if (factor64(b, c)) return 1;
    mode = 3;
  }
  if (mode == 2 || mode == 5) {   /* learned X, or the Gauss-Jordan inverse */
    const double* X = b->X + b->moff[c];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s = s + X[i * n + j] * r[j];
      d[i] = s;
    }
    if (mode == 2) b->st.lp_cell_solves++;
    return 0;
  }
  memcpy(d, r, sizeof(double) * (size_t)n);
  orc_lu_solve(n, b->LU + b->moff[c], b->piv + off, d);
  return 0;
}

static double cell_wrms(const orc_bdf* b, long c, const double* x) {
  return orc_nv_wrms_norm(b->cn[c], x + b->yoff[c], b->w + b->yoff[c]);
}

static int finite_cell(const orc_bdf* b, long c, const double* x) {
  for (int i = 0; i < b->cn[c]; ++i)
    if (!isfinite(x[b->yoff[c] + i])) return 0;
  return 1;
}

/* ---- Newton-Krylov (linsol GMRES) --------------------------------------
 * The Newton system M del = r is solved over all N unknowns at once by
 * GMRES (Saad & Schultz 1986) with right preconditioning and the error
 * weights as scaling (Brown & Hindmarsh 1989): with W = diag(w) it is
 * GMRES on W M P^{-1} W^{-1} for W r, and del = P^{-1} W^{-1} x.  P is
 * the block-Jacobi preconditioner: the LU factors of the cells' blocks of
 * M at the last setup (every attempt without lazy, so that P = M and one
 * iteration solves it).  The operator applies the current M = I - gamma J
 * with J at the predicted state.  Classical Gram-Schmidt (all inner
 * products of a new vector with the basis, then one update); Givens
 * rotations; at most KRY_MAXL iterations, no restart, stop when the scaled
 * residual's 2-norm is at most KRY_EPLIN * NLS_COEF * sqrt(N) (WRMS
 * KRY_EPLIN times the Newton tolerance).  Returns the iterations taken. */
typedef struct {
  long N, ncells;
  const int* cn;
  const long *yoff, *moff;
  const double* M;     /* current Newton matrix blocks (column-major) */
  const double* LU;    /* preconditioner: LU factors of the blocks */
  const int* piv;
  const double* w;     /* error weights (scaling) */
  double *V, *tmp;     /* (KRY_MAXL + 1) N and N doubles of workspace */
} kry_sys;

static void prec_solve(const kry_sys* k, double* x) {   /* x <- P^{-1} x, per cell */
  for (long c = 0; c < k->ncells; ++c)
    orc_lu_solve(k->cn[c], k->LU + k->moff[c], k->piv + k->yoff[c], x + k->yoff[c]);
}

static void apply_M(const kry_sys* k, const double* x, double* out) {   /* out = M x */
  for (long c = 0; c < k->ncells; ++c) {
    int n = k->cn[c];
    const double* M = k->M + k->moff[c];
    const double* xc = x + k->yoff[c];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s = s + AT(M, i, j, n) * xc[j];
      out[k->yoff[c] + i] = s;
    }
  }
}

/* del <- solution of M del = r to the scaled-residual tolerance tol (2-norm
 * of W (r - M del)); returns the iterations taken. */
static int gmres(const kry_sys* ks, const double* r, double tol, double* del) {
  const long N = ks->N;
  const double* w = ks->w;
  double* V = ks->V;
  double H[KRY_MAXL + 1][KRY_MAXL], cs[KRY_MAXL], sn[KRY_MAXL], g[KRY_MAXL + 1];
  for (long i = 0; i < N; ++i) V[i] = w[i] * r[i];
  double beta = sqrt(orc_nv_dot_prod_multi_1(N, V, V));
  memset(del, 0, sizeof(double) * (size_t)N);
  if (!(beta > tol)) return 0;
  for (long i = 0; i < N; ++i) V[i] = V[i] / beta;
  for (int j = 0; j <= KRY_MAXL; ++j) g[j] = 0.0;
  g[0] = beta;
  int k = 0, iters = 0;
  for (k = 0; k < KRY_MAXL; ++k) {
    double* vk = V + (long)k * N;
    double* wv = V + (long)(k + 1) * N;
    for (long i = 0; i < N; ++i) ks->tmp[i] = vk[i] / w[i];
    prec_solve(ks, ks->tmp);
    apply_M(ks, ks->tmp, wv);
    for (long i = 0; i < N; ++i) wv[i] = w[i] * wv[i];
    /* classical Gram-Schmidt: all inner products first, then one update */
    const double* Y[KRY_MAXL];
    for (int j = 0; j <= k; ++j) Y[j] = V + (long)j * N;
    double hk[KRY_MAXL + 1];
    orc_nv_dot_prod_multi(k + 1, wv, Y, hk, N);
    for (int j = 0; j <= k; ++j)
      for (long i = 0; i < N; ++i) wv[i] = wv[i] - hk[j] * Y[j][i];
    hk[k + 1] = sqrt(orc_nv_dot_prod_multi_1(N, wv, wv));
    iters++;
    const int breakdown = !(hk[k + 1] > 0.0);
    if (!breakdown)
      for (long i = 0; i < N; ++i) wv[i] = wv[i] / hk[k + 1];
    /* previous rotations on the new column, then one that zeroes h_{k+1,k} */
    for (int j = 0; j < k; ++j) {
      const double a = hk[j], c2 = hk[j + 1];
      hk[j] = cs[j] * a + sn[j] * c2;
      hk[j + 1] = -sn[j] * a + cs[j] * c2;
    }
    const double rr = sqrt(hk[k] * hk[k] + hk[k + 1] * hk[k + 1]);
    cs[k] = hk[k] / rr;
    sn[k] = hk[k + 1] / rr;
    hk[k] = rr;
    hk[k + 1] = 0.0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    for (int j = 0; j <= k; ++j) H[j][k] = hk[j];
    if (breakdown || fabs(g[k + 1]) <= tol) {
      k++;
      break;
    }
  }
  /* y = R^{-1} g, x = sum y_j v_j, del = P^{-1} W^{-1} x */
  double y[KRY_MAXL];
  for (int i = k - 1; i >= 0; --i) {
    double s2 = g[i];
    for (int j = i + 1; j < k; ++j) s2 = s2 - H[i][j] * y[j];
    y[i] = s2 / H[i][i];
  }
  for (int j = 0; j < k; ++j)
    for (long i = 0; i < N; ++i) del[i] = del[i] + y[j] * V[(long)j * N + i];
  for (long i = 0; i < N; ++i) del[i] = del[i] / w[i];
  prec_solve(ks, del);
  return iters;
}

static int newton_gmres(orc_bdf* b) {
  kry_sys ks = {b->N, b->p.ncells, b->cn, b->yoff, b->moff, b->M, b->LU, b->piv, b->w,
                b->V, b->tmp};
  const int it = gmres(&ks, b->r, KRY_EPLIN * NLS_COEF * sqrt((double)b->N), b->del);
  b->st.nliters += it;
  return it;
}

int orc_gmres_solve(long ncells, const int* n, const double* M, const double* LU,
                    const int* piv, const double* w, const double* r, double tol, double* del) {
  long* yoff = (long*)calloc((size_t)ncells + 1, sizeof(long));
  long* moff = (long*)calloc((size_t)ncells + 1, sizeof(long));
  for (long c = 0; c < ncells; ++c) {
    yoff[c + 1] = yoff[c] + n[c];
    moff[c + 1] = moff[c] + (long)n[c] * n[c];
  }
  const long N = yoff[ncells];
  double* V = (double*)calloc((size_t)(KRY_MAXL + 1) * (size_t)(N > 0 ? N : 1), sizeof(double));
  double* tmp = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
  kry_sys ks = {N, ncells, n, yoff, moff, M, LU, piv, w, V, tmp};
  const int it = gmres(&ks, r, tol, del);
  free(V); free(tmp); free(yoff); free(moff);
  return it;
}

/* Newton iteration on all cells at once (grouped; one global norm).
 * setup: fresh J, M = I - gamma J and its factors (else the stored factors
 * of an earlier gamma are reused and every correction is scaled by dscale);
 * *crate: the convergence-rate estimate, carried in and out.
 * Returns 0 converged, 1 failed (caller retries the step). */
static int newton(orc_bdf* b, double gamma, double l0, int force_lu, int setup, double dscale,
                  double* crate_io) {
  long N = b->N, nc = b->p.ncells;
  int ls = b->o.linsol;
  int setup_fail = 0;
  if (setup) b->st.nsetups++;
  if (ls == ORC_LS_GMRES) {
    /* the operator's M at every attempt; the preconditioner's factors at a
     * setup only */
    for (long c = 0; c < nc; ++c) {
      build_M(b, c, gamma);
      b->cellmode[c] = 0;
      if (setup && factor64(b, c)) setup_fail = 1;
    }
  } else if (!setup) {
    /* lazy reuse: cellmode (0 LU, 5 inverse) and the factors stay */
  } else if (ls == ORC_LS_LEARNED && !force_lu) {
    double xin[64];
    double lg = log(gamma);
    for (long c = 0; c < nc; ++c) {
      int n = b->cn[c];
      for (int i = 0; i < n; ++i) xin[i] = b->zp[0][b->yoff[c] + i];
      xin[n] = lg;
      double* X = b->X + b->moff[c];
      orc_mlp_forward(b->o.mlp, xin, X);
      for (int i = 0; i < n; ++i) X[i * n + i] += 1.0;
      b->cellmode[c] = 2;
      b->cellinfo[c] = 0;   /* M not built yet */
    }
  } else {
    for (long c = 0; c < nc; ++c) {
      build_M(b, c, gamma);
      b->cellinfo[c] = 1;
      if (ls == ORC_LS_LU32REF) {
        int n = b->cn[c];
        for (long i = 0; i < (long)n * n; ++i)
          b->LU32[b->moff[c] + i] = (float)b->M[b->moff[c] + i];
        int info = orc_lu_factor_f32(n, b->LU32 + b->moff[c], b->piv32 + b->yoff[c]);
        b->cellmode[c] = 1;
        if (info) {
          b->st.refine_fallbacks++;
          b->cellmode[c] = 3;
          if (factor64(b, c)) setup_fail = 1;
        }
      } else if (ls == ORC_LS_GJ) {
        /* explicit inverse; the solve is then X r (mode 5) */
        b->cellmode[c] = 5;
        if (orc_gj_inverse(b->cn[c], b->M + b->moff[c], b->X + b->moff[c])) setup_fail = 1;
      } else {
        b->cellmode[c] = 0;
        if (factor64(b, c)) setup_fail = 1;
      }
    }
  }
  if (setup_fail) return 1;
  memcpy(b->y, b->zp[0], sizeof(double) * (size_t)N);
  double crate = *crate_io, dold = 0.0;
  int rc = 1;
  for (int m = 0; m < b->o.maxcor; ++m) {
    rhs_all(b, b->y, b->f);
    for (long i = 0; i < N; ++i)
      b->r[i] = gamma * b->f[i] - l0 * b->zp[1][i] - (b->y[i] - b->zp[0][i]);
    if (ls == ORC_LS_GMRES) newton_gmres(b);
    for (long c = 0; c < nc && ls != ORC_LS_GMRES; ++c) {
      if (b->cellmode[c] == 2) {
        cell_solve(b, c);
        if (!finite_cell(b, c, b->del)) b->cellmode[c] = 4;  /* switch now */
      }
      if (b->cellmode[c] == 4) {   /* learned cell moved to exact LU */
        if (b->cellinfo[c] == 0) {
          build_M(b, c, gamma);
          b->cellinfo[c] = 1;
          b->st.lp_fallback_cells++;
          if (factor64(b, c)) return 1;
        }
        int n = b->cn[c];
        memcpy(b->del + b->yoff[c], b->r + b->yoff[c], sizeof(double) * (size_t)n);
        orc_lu_solve(n, b->LU + b->moff[c], b->piv + b->yoff[c], b->del + b->yoff[c]);
      } else if (b->cellmode[c] != 2) {
        if (cell_solve(b, c)) return 1;
      }
    }
    b->st.nlinsolves++;
    if (dscale != 1.0)
      for (long i = 0; i < N; ++i) b->del[i] = dscale * b->del[i];
    /* learned cells: a cell still solved with X that does not contract by
     * LP_CELL_RATIO switches to exact LU from the next iteration, and the
     * attempt cannot be accepted at that iteration; at the first iteration
     * no cell has a contraction rate yet, so a learned attempt is never
     * accepted there (reading: the grouped test alone would let a cell
     * whose X is poor pass on a small first correction X r) */
    long unconv = 0;
    if (ls == ORC_LS_LEARNED && !force_lu) {
      for (long c = 0; c < nc; ++c) {
        double dc = cell_wrms(b, c, b->del);
        if (b->cellmode[c] == 2 && m >= 1 && !(dc <= LP_CELL_RATIO * b->dcell_prev[c])) {
          b->cellmode[c] = 4;     /* exact LU from the next iteration on */
          unconv++;
        }
        b->dcell_prev[c] = dc;
      }
      if (m == 0) unconv = 1;
      b->st.lp_unconverged += unconv;
    }
    for (long i = 0; i < N; ++i) b->y[i] = b->y[i] + b->del[i];
    double d = wrms(b, b->del);
    b->st.nniters++;
    if (!isfinite(d)) break;
    if (m > 0) {
      double ratio = d / dold;
      crate = CRDOWN * crate > ratio ? CRDOWN * crate : ratio;
    }
    double dcon = d * (crate < 1.0 ? crate : 1.0);
    if (dcon <= NLS_COEF && unconv == 0) {
      rc = 0;
      break;
    }
    if (m + 1 == b->o.maxcor) break;
    if (m >= 1 && d > RDIV * dold) break;
    dold = d;
  }
  *crate_io = crate;
  return rc;
}

int orc_bdf_step(orc_bdf* b, double t_end) {
  long N = b->N;
  if (!b->initialized) initialize(b, t_end);
  if (b->t >= t_end) return 1;
  int ncf = 0, netf = 0, force_lu = 0;
  for (;;) {
    int q = b->q;
    if (b->t + b->h > t_end) {
      double eta = (t_end - b->t) / b->h;
      rescale(b, eta);
      b->h = t_end - b->t;
      b->qwait = q + 1;
    }
    if (b->h <= 4.0 * 2.220446049250313e-16 * fabs(b->t)) return -5;  /* t + h == t */
    int last = (b->t + b->h >= t_end);
    double l[QMAX_ALL + 1], tq, xi[QMAX_ALL + 3];
    if (b->o.vc) {
      vc_xi(b, b->h, q + 1, xi);
      vc_coeffs(q, xi, l, &tq);
    } else {
      orc_bdf_coeffs(q, l, &tq);
    }
    orc_nv_ewt(N, b->o.rtol, b->o.atol, b->z[0], b->w);
    for (int j = 0; j <= q; ++j) memcpy(b->zp[j], b->z[j], sizeof(double) * (size_t)N);
    for (int k = 1; k <= q; ++k)
      for (int j = q; j >= k; --j)
        for (long i = 0; i < N; ++i) b->zp[j - 1][i] = b->zp[j - 1][i] + b->zp[j][i];
    double gamma = b->h * l[0];
    b->st.nattempts++;
    /* lazy Newton matrix (reading): a fresh J and M at the first attempt,
     * after any Newton failure, every MSBP accepted steps and when gamma has
     * moved more than DGMAX from the gamma of the stored factors; otherwise
     * the stored factors of gamma_s are reused and each correction is
     * scaled by 2 / (1 + gamma / gamma_s), and the convergence-rate estimate
     * carries over from the previous attempt (it restarts at 1 after a
     * setup) */
    int setup = 1;
    double dscale = 1.0, crate = 1.0;
    if (b->o.lazy) {
      setup = !b->m_valid || b->force_setup || b->st.nsteps - b->nst_s >= MSBP ||
              fabs(gamma / b->gamma_s - 1.0) > DGMAX;
      if (setup) {
        b->gamma_s = gamma;
        b->nst_s = b->st.nsteps;
        b->m_valid = 1;
        b->force_setup = 0;
      } else {
        /* (the direct solve's correction scale; GMRES solves the current M) */
        dscale = b->o.linsol == ORC_LS_GMRES ? 1.0 : 2.0 / (1.0 + gamma / b->gamma_s);
        crate = b->crate_keep;
      }
    }
    int nst = newton(b, gamma, l[0], force_lu, setup, dscale, &crate);
    b->crate_keep = crate;
    if (nst) {
      if (b->o.linsol == ORC_LS_LEARNED && !force_lu) {
        force_lu = 1;
        b->st.lp_step_fallbacks++;
        continue;
      }
      if (b->o.lazy) {
        b->force_setup = 1;
        if (!setup) {   /* stale factors: redo the attempt with fresh ones */
          b->st.nstale_retries++;
          continue;
        }
      }
      force_lu = 0;
      ncf++;
      b->st.nncfails++;
      if (ncf >= MXNCF) return -4;
      if (b->h * ETA_CF < b->o.hmin) return -5;
      rescale(b, ETA_CF);
      b->h = b->h * ETA_CF;
      b->qwait = q + 1;
      continue;
    }
    if (b->o.nonneg) {
      /* y >= 0 by projection (a project reading: the paper states no such
       * step, and its constraint-mask vector operation only flags
       * violations): the corrected solution is projected onto the
       * constraint before the error test; the projection enters the
       * correction, so the whole history stays consistent with it */
      int any = 0;
      for (long i = 0; i < N; ++i)
        if (b->y[i] < 0.0) {
          b->y[i] = 0.0;
          any = 1;
        }
      if (any) b->st.nprojections++;
    }
    for (long i = 0; i < N; ++i) b->acor[i] = (b->y[i] - b->zp[0][i]) / l[0];
    double err = wrms(b, b->acor) * tq;
    b->err_last = err;
    if (err > 1.0) {
      force_lu = 0;
      netf++;
      b->st.netfails++;
      if (netf >= MXNEF) return -3;
      if (netf >= 3) {
        double hn = b->h * ETA_RESTART;
        if (hn < b->o.hmin) return -5;
        b->h = hn;
        b->q = 1;
        b->ntau = 0;   /* the new history knows no past points */
        rhs_all(b, b->z[0], b->f);
        for (long i = 0; i < N; ++i) b->z[1][i] = b->h * b->f[i];
        b->qwait = 2;
      } else {
        double eta = 0.9 * pow(err, -1.0 / (double)(q + 1));
        if (eta < ETA_MIN_EF) eta = ETA_MIN_EF;
        if (b->h * eta < b->o.hmin) return -5;
        rescale(b, eta);
        b->h = b->h * eta;
        b->qwait = q + 1;
      }
      continue;
    }
    /* accept: z[j] = z(0)[j] + l_j * acor; for j = 0 that is the corrected
     * solution y itself, which is stored as is */
    for (int j = 1; j <= q; ++j)
      for (long i = 0; i < N; ++i) b->z[j][i] = b->zp[j][i] + l[j] * b->acor[i];
    memcpy(b->z[0], b->y, sizeof(double) * (size_t)N);
    b->t = last ? t_end : b->t + b->h;
    b->hu = b->h;
    b->qu = q;
    for (int k = NTAU - 1; k > 0; --k) b->tau[k] = b->tau[k - 1];
    b->tau[0] = b->h;
    if (b->ntau < NTAU) b->ntau++;
    /* scale of this correction for the next order-(q+1) estimate:
     * acor c_n = h^{q+1} y^{(q+1)} / (q+1)! for a degree-(q+1) solution */
    double Sq1 = 0.0, pxi = 1.0;
    if (b->o.vc) {
      for (int i = 1; i <= q + 1; ++i) {
        Sq1 = Sq1 + 1.0 / xi[i];
        pxi = pxi * xi[i];
      }
    }
    const double cn = b->o.vc ? 1.0 / (pxi * Sq1) : 1.0;
    b->st.nsteps++;
    b->st.order_hist[q]++;
    b->qwait--;
    /* step size and order for the next step */
    double etaq = 1.0 / (pow(BIAS_Q * err, 1.0 / (double)(q + 1)) + ADDON);
    double eta = etaq;
    int qnew = q;
    b->err_qm1 = -1.0;
    b->err_qp1 = -1.0;
    if (b->o.fixed_step) {
      memcpy(b->dprev, b->acor, sizeof(double) * (size_t)N);
      b->dprev_c = cn;
      b->dprev_h = b->h;
      b->eta_prop = 1.0;
      b->q_prop = q;
      return 0;
    }
    if (b->qwait == 0) {
      b->qwait = 2;
      double etaqm1 = 0.0, etaqp1 = 0.0;
      if (q > 1) {
        /* error of an order-(q-1) step: z[q] times prod_{i<q} xi_i / S_{q-1}
         * (constant steps: (q-1)! / H_{q-1}) */
        double pr = factorial(q - 1), S = harmonic(q - 1);
        if (b->o.vc) {
          pr = 1.0;
          S = 0.0;
          for (int i = 1; i <= q - 1; ++i) {
            pr = pr * xi[i];
            S = S + 1.0 / xi[i];
          }
        }
        double e = wrms(b, b->z[q]) * pr / S;
        b->err_qm1 = e;
        etaqm1 = 1.0 / (pow(BIAS_QM1 * e, 1.0 / (double)q) + ADDON);
      }
      if (q < b->o.qmax) {
        /* error of an order-(q+1) step from the change of D = c acor
         * between the previous step and this one, the previous brought to
         * this h: (D_n - (h/h_prev)^{q+1} D_{n-1}) / (q+2) estimates
         * h^{q+2} y^{(q+2)} / (q+2)!; the order-(q+1) error is that times
         * prod_{i<=q+1} xi_i / S_{q+1}, i.e. |acor - kap acor_prev| /
         * ((q+2) S_{q+1}^2) (constant steps: kap = 1, S = H_{q+1}) */
        double kap = 1.0, S1 = harmonic(q + 1);
        if (b->o.vc) {
          kap = pow(b->h / b->dprev_h, (double)(q + 1)) * b->dprev_c / cn;
          S1 = Sq1;
        }
        for (long i = 0; i < N; ++i) b->tmp[i] = b->acor[i] - kap * b->dprev[i];
        double e = wrms(b, b->tmp) / ((double)(q + 2) * S1 * S1);
        b->err_qp1 = e;
        etaqp1 = 1.0 / (pow(BIAS_QP1 * e, 1.0 / (double)(q + 2)) + ADDON);
      }
      if (etaq >= etaqm1 && etaq >= etaqp1) {
        eta = etaq; qnew = q;
      } else if (etaqm1 >= etaqp1) {
        eta = etaqm1; qnew = q - 1;
      } else {
        eta = etaqp1; qnew = q + 1;
      }
    }
    b->eta_prop = eta;
    b->q_prop = qnew;
    if (eta >= THRESH) {
      if (eta > ETA_MAX) eta = ETA_MAX;
      if (qnew == q + 1 && b->o.vc) {
        /* raise keeping the interpolation of the past values: add
         * C s prod_{i<=q} (s + xi_i), which leaves the last q + 1 points,
         * with C such that the history also passes through y_{n-q-1}; the
         * previous history passed through it and differs from the new one
         * by acor Lambda(s), so C = acor Lambda(-xi_{q+1}) /
         * (xi_{q+1} prod_{i<=q} (xi_i - xi_{q+1})) */
        double lam = 0.0, pw = 1.0, den = xi[q + 1], e[QMAX_ALL + 3];
        for (int j = 0; j <= q; ++j) {
          lam = lam + l[j] * pw;
          pw = pw * -xi[q + 1];
        }
        for (int i = 1; i <= q; ++i) den = den * (xi[i] - xi[q + 1]);
        const double cr = lam / den;
        poly_through(xi, q, e);
        for (int j = 1; j <= q; ++j)
          for (long i = 0; i < N; ++i) b->z[j][i] = b->z[j][i] + (cr * e[j]) * b->acor[i];
        for (long i = 0; i < N; ++i) b->z[q + 1][i] = cr * b->acor[i];
      } else if (qnew == q + 1) {
        double c = 1.0 / (factorial(q + 1) * harmonic(q + 1));
        for (long i = 0; i < N; ++i) b->z[q + 1][i] = c * b->acor[i];
      } else if (qnew == q - 1 && b->o.vc) {
        /* lower the order keeping the interpolation: subtract
         * z[q] s prod_{i<q} (s + xi_i), which removes the s^q term and leaves
         * the last q points */
        double d[QMAX_ALL + 3];
        poly_through(xi, q - 1, d);
        for (int j = 1; j <= q - 1; ++j)
          for (long i = 0; i < N; ++i) b->z[j][i] = b->z[j][i] - d[j] * b->z[q][i];
      }
      b->q = qnew;
      rescale(b, eta);
      b->h = b->h * eta;
      b->qwait = b->q + 1;
    }
    memcpy(b->dprev, b->acor, sizeof(double) * (size_t)N);
    b->dprev_c = cn;
    b->dprev_h = b->hu;
    return 0;
  }
}

int orc_bdf_integrate(orc_bdf* b, double t_end) {
  long ns = 0;
  if (!b->initialized) initialize(b, t_end);
  while (b->t < t_end) {
    int s = orc_bdf_step(b, t_end);
    if (s < 0) return s;
    if (b->o.max_steps > 0 && ++ns >= b->o.max_steps && b->t < t_end) return -6;
  }
  return 0;
}

void orc_bdf_get_y(const orc_bdf* b, double* y) {
  memcpy(y, b->z[0], sizeof(double) * (size_t)b->N);
}

void orc_bdf_get_stats(const orc_bdf* b, orc_stats* s) { *s = b->st; }

void orc_bdf_get_scalars(const orc_bdf* b, orc_scalars* s) {
  s->t = b->t; s->h = b->h; s->err_last = b->err_last;
  s->q = b->q; s->qwait = b->qwait; s->qprime_pending = 0;
  s->initialized = b->initialized; s->hu = b->hu; s->qu = b->qu;
  s->err_qm1 = b->err_qm1; s->err_qp1 = b->err_qp1;
  s->eta_proposed = b->eta_prop; s->q_proposed = b->q_prop;
}

void orc_bdf_init(orc_bdf* b, double t_end) {
  if (!b->initialized) initialize(b, t_end);
}

void orc_bdf_set_scalars(orc_bdf* b, const orc_scalars* s) {
  b->t = s->t; b->h = s->h; b->err_last = s->err_last;
  b->q = s->q; b->qwait = s->qwait; b->initialized = s->initialized;
  b->hu = s->hu; b->qu = s->qu;
}

void orc_bdf_get_history(const orc_bdf* b, double* z6, double* dprev) {
  for (int j = 0; j <= QMAX_ALL; ++j)
    memcpy(z6 + (long)j * b->N, b->z[j], sizeof(double) * (size_t)b->N);
  memcpy(dprev, b->dprev, sizeof(double) * (size_t)b->N);
}

void orc_bdf_set_history(orc_bdf* b, const double* z6, const double* dprev) {
  for (int j = 0; j <= QMAX_ALL; ++j)
    memcpy(b->z[j], z6 + (long)j * b->N, sizeof(double) * (size_t)b->N);
  memcpy(b->dprev, dprev, sizeof(double) * (size_t)b->N);
  b->m_valid = 0;
}

void orc_bdf_set_past_steps(orc_bdf* b, int k, const double* tau, double dprev_c,
                            double dprev_h) {
  b->ntau = k < 0 ? 0 : (k > NTAU ? NTAU : k);
  for (int i = 0; i < b->ntau; ++i) b->tau[i] = tau[i];
  b->dprev_c = dprev_c;
  b->dprev_h = dprev_h;
}

int orc_bdf_get_past_steps(const orc_bdf* b, double* tau, double* dprev_c, double* dprev_h) {
  for (int i = 0; i < b->ntau; ++i) tau[i] = b->tau[i];
  *dprev_c = b->dprev_c;
  *dprev_h = b->dprev_h;
  return b->ntau;
}

void orc_bdf_get_lazy(const orc_bdf* b, double* gamma_s, long* nst_s, double* crate) {
  *gamma_s = b->gamma_s;
  *nst_s = b->nst_s;
  *crate = b->crate_keep;
}
