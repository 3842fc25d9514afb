// Device-resident controller of the grouped BDF integrator.
//
// The paper keeps integrator control on the host and data in device memory
// (Sections 2 and 6), with one synchronising transfer per reduction
// (Section 4.1).  On gfx950 the decisions of a step attempt (Newton
// convergence, local error test, step size and order) are a few dozen
// scalar operations on the norms that the step's kernels reduce anyway, so
// they run in the last workgroup of the kernel that produced the norms and
// the state lives in device memory.  An attempt is then a fixed sequence of
// launches with no host round trip, which a hipGraph can capture; the host
// reads the state only every few attempts.
//
// Method: fixed-coefficient Nordsieck BDF of order q <= 5 (the paper names
// CVODE for this role without stating its method).  History z[j] ~
// h^j y^(j)/j!; coefficient vector l_j = [x^j] prod_{i=1..q}(1 + x/i) / H_q;
// predictor z(0) = Pascal(z); corrector z_new[j] = z(0)[j] + l_j acor;
// Newton on M = I - gamma J, gamma = h l_0, with the whole step retried when
// any cell fails (Section 7, ensemble failure rule); local error
// acor / ((q+1) H_q H_{q+1}).  Rescaling by eta multiplies z[j] by eta^j;
// here that factor is kept pending in hs[j] and applied by the next kernel
// that reads the history.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/bdfgpu.h"

namespace bdfgpu {

enum Phase : int {
  PH_INIT1 = 0,
  PH_INIT2 = 1,
  PH_PREDICT = 2,
  PH_NEWTON = 3,
  PH_ACCEPT = 4,
  PH_DONE = 5,
  PH_PAUSE = 6,
  PH_ERROR = 7
};

constexpr int kQmaxAll = 5;
constexpr int kMaxCor = 4;        // Newton iterations per attempt, at most
constexpr int kRedPerIter = 8;     // reduced values per Newton iteration
constexpr int kMxNcf = 10;
constexpr int kMxNef = 7;
constexpr double kCrDown = 0.3;
constexpr double kRdiv = 2.0;
constexpr double kNlsCoef = 0.1;
constexpr double kEtaMax = 10.0;
constexpr double kEtaMinEf = 0.2;
constexpr double kEtaCf = 0.25;
constexpr double kEtaRestart = 0.1;
constexpr double kThresh = 1.5;
constexpr double kBiasQm1 = 1.3;
constexpr double kBiasQ = 1.2;
constexpr double kBiasQp1 = 1.4;
constexpr double kAddon = 1e-6;

struct Ctrl {
  double t, h, tend, hmin, h0user, hnw_h0;
  double hs[kQmaxAll + 2];   // pending history scale: true z[j] = stored z[j] * hs[j]
  double l[kQmaxAll + 2];    // corrector coefficients for the current q
  double tq, gamma, err, crate, dold, hu, craise, hnw_d1;
  double N;                  // total unknowns (for WRMS)
  int q, qmax, qwait, maxcor, qu;
  int phase, m, ncf, netf, last, restart, status, pad;
  int learned, force_lu;      // learned preconditioner; retry of an attempt with exact LU
  // Deferred history update (fuse = 1): an accepted attempt's update
  // z_new[j] = z(0)[j] + l_j acor is applied by the next attempt's Newton
  // kernel as it reads the history (or by the flush at the end of a drive),
  // so the history crosses HBM once per step instead of three times.  The
  // upd_* fields describe the accepted attempt: its iterate index, order,
  // coefficients, pending history scale and whether it also writes
  // z[q+1] = craise acor for a possible order raise.
  int fuse, upd, upd_m, upd_q, upd_raise, pad2;
  double upd_l[kQmaxAll + 2];
  double upd_hs[kQmaxAll + 2];
  double upd_craise;
  long step_limit;
  long nsteps, nattempts, nfevals, nsetups, nniters, nncfails, netfails;
  long nlinsolves, refine_sweeps, refine_fallbacks, nprojections;
  long hist_reads;          // sum over attempts of q + 1 (history vectors read)
  long lp_cell_solves, lp_fallback_cells, lp_step_fallbacks;
  long order_hist[6];
};

__host__ __device__ inline double harmonic(int q) {
  double s = 0.0;
  for (int i = 1; i <= q; ++i) s += 1.0 / (double)i;
  return s;
}

__host__ __device__ inline double factorial(int q) {
  double s = 1.0;
  for (int i = 2; i <= q; ++i) s *= (double)i;
  return s;
}

// l vector of order q and the local-error constant 1/((q+1) H_q H_{q+1}).
__device__ inline void set_coeffs(Ctrl* C) {
  const int q = C->q;
  double c[kQmaxAll + 2];
  for (int j = 0; j < kQmaxAll + 2; ++j) c[j] = 0.0;
  c[0] = 1.0;
  for (int i = 1; i <= q; ++i)
    for (int j = i; j >= 1; --j) c[j] = c[j] + c[j - 1] / (double)i;
  const double H = harmonic(q);
  for (int j = 0; j < kQmaxAll + 2; ++j) C->l[j] = j <= q ? c[j] / H : 0.0;
  C->tq = 1.0 / ((double)(q + 1) * H * harmonic(q + 1));
  C->craise = 1.0 / (factorial(q + 1) * harmonic(q + 1));
}

__device__ inline void rescale(Ctrl* C, double eta) {
  double f = 1.0;
  for (int j = 1; j <= C->q; ++j) {
    f = f * eta;
    C->hs[j] = C->hs[j] * f;
  }
}

__device__ inline void fail_error(Ctrl* C, int code);

__device__ inline void prepare_attempt(Ctrl* C) {
  if (C->h <= 4.0 * 2.220446049250313e-16 * fabs(C->t))   // t + h == t
    return fail_error(C, BDFGPU_ERR_HMIN);
  if (C->t + C->h > C->tend) {
    const double eta = (C->tend - C->t) / C->h;
    rescale(C, eta);
    C->h = C->tend - C->t;
    C->qwait = C->q + 1;
  }
  C->last = (C->t + C->h >= C->tend);
  set_coeffs(C);
  C->gamma = C->h * C->l[0];
  C->m = 0;
  C->crate = 1.0;
  C->dold = 0.0;
  C->phase = PH_PREDICT;
  C->nattempts++;
  C->nsetups++;
  C->hist_reads += C->q + 1;
}

__device__ inline void fail_error(Ctrl* C, int code) {
  C->status = code;
  C->phase = PH_ERROR;
}

__device__ inline void newton_failed(Ctrl* C) {
  if (C->learned && !C->force_lu) {
    // the learned attempt failed: redo it with exact LU before reducing h
    C->force_lu = 1;
    C->lp_step_fallbacks++;
    return prepare_attempt(C);
  }
  C->force_lu = 0;
  C->ncf++;
  C->nncfails++;
  if (C->ncf >= kMxNcf) return fail_error(C, BDFGPU_CONV_FAIL);
  if (C->h * kEtaCf < C->hmin) return fail_error(C, BDFGPU_ERR_HMIN);
  rescale(C, kEtaCf);
  C->h = C->h * kEtaCf;
  C->qwait = C->q + 1;
  prepare_attempt(C);
}

__device__ inline void error_test_failed(Ctrl* C, double err) {
  C->force_lu = 0;
  C->netf++;
  C->netfails++;
  if (C->netf >= kMxNef) return fail_error(C, BDFGPU_TEST_FAIL);
  if (C->netf >= 3) {
    const double hn = C->h * kEtaRestart;
    if (hn < C->hmin) return fail_error(C, BDFGPU_ERR_HMIN);
    C->h = hn;
    C->q = 1;
    C->restart = 1;          // next predictor sets z[1] = h f(z[0])
    for (int j = 0; j < kQmaxAll + 2; ++j) C->hs[j] = 1.0;
    C->qwait = 2;
  } else {
    double eta = 0.9 * pow(err, -1.0 / (double)(C->q + 1));
    if (eta < kEtaMinEf) eta = kEtaMinEf;
    if (C->h * eta < C->hmin) return fail_error(C, BDFGPU_ERR_HMIN);
    rescale(C, eta);
    C->h = C->h * eta;
    C->qwait = C->q + 1;
  }
  prepare_attempt(C);
}

// After the fused Newton kernel.  The kernel runs all maxcor iterations of
// the attempt for every cell (each cell's iterates depend only on its own
// block, gamma and the predicted state) and reduces, per iteration m, the
// sums s[8m + j]: j = 0 (delta w)^2, 1 ((y - z(0)[0]) w)^2 with y projected
// onto y >= 0 when constrained, 2 negative components, 3 refinement sweeps,
// 4 refinement fallbacks, 5 learned-inverse solves, 6 learned-to-LU
// switches; s[7] counts singular blocks.  The global convergence test is
// then replayed iteration by iteration exactly as a sequential Newton loop
// would take it, and C->m records the iteration whose iterate is the
// corrected solution.  Iterates past that point were computed but are
// unused, so the outcome equals that of stopping there.
__device__ inline void after_accept(Ctrl* C, const double* s);

__device__ inline void after_newton_all(Ctrl* C, const double* s) {
  if (C->restart) {   // the predictor re-evaluated f(z[0])
    C->nfevals++;
    C->restart = 0;
  }
  C->upd = 0;         // the Newton kernel applied any pending history update
  for (int m = 0; m < C->maxcor; ++m) {
    const double* t = s + kRedPerIter * m;
    C->nfevals++;
    C->nniters++;
    C->nlinsolves++;
    C->refine_sweeps += (long)t[3];
    C->refine_fallbacks += (long)t[4];
    if (C->learned) {
      C->lp_cell_solves += (long)t[5];
      C->lp_fallback_cells += (long)t[6];
    }
    if (m == 0 && s[7] > 0.0) return newton_failed(C);   // singular block in the setup
    const double d = sqrt(t[0] / C->N);
    if (!(d == d) || d > 1e300) return newton_failed(C);
    if (m > 0) {
      const double ratio = d / C->dold;
      C->crate = kCrDown * C->crate > ratio ? kCrDown * C->crate : ratio;
    }
    const double dcon = d * (C->crate < 1.0 ? C->crate : 1.0);
    if (dcon <= kNlsCoef) {
      C->m = m;
      if (t[2] > 0.0) C->nprojections++;
      const double err = sqrt(t[1] / C->N) / C->l[0] * C->tq;
      C->err = err;
      if (err <= 1.0) {
        if (C->fuse) {
          // the next Newton kernel applies the history update; the order
          // selection's sums came with this iteration's (slots 5 and 6)
          C->upd = 1;
          C->upd_m = m;
          C->upd_q = C->q;
          for (int j = 0; j < kQmaxAll + 2; ++j) {
            C->upd_l[j] = C->l[j];
            C->upd_hs[j] = C->hs[j];
          }
          C->upd_craise = C->craise;
          C->upd_raise = (C->qwait == 1 && C->q < kQmaxAll && C->q < C->qmax) ? 1 : 0;
          const double sacc[2] = {t[5], t[6]};
          return after_accept(C, sacc);
        }
        C->phase = PH_ACCEPT;
        return;
      }
      return error_test_failed(C, err);
    }
    if (m + 1 == C->maxcor) return newton_failed(C);
    if (m >= 1 && d > kRdiv * C->dold) return newton_failed(C);
    C->dold = d;
  }
  newton_failed(C);
}

// After the history update (or, with the deferred update, after the Newton
// kernel): sums of (z_new[q] w)^2 and ((acor - acor_prev) w)^2.
__device__ inline void after_accept(Ctrl* C, const double* s) {
  const int q = C->q;
  C->t = C->last ? C->tend : C->t + C->h;
  C->hu = C->h;
  C->qu = q;
  C->nsteps++;
  C->order_hist[q]++;
  C->qwait--;
  const double err = C->err;
  const double etaq = 1.0 / (pow(kBiasQ * err, 1.0 / (double)(q + 1)) + kAddon);
  double eta = etaq;
  int qnew = q;
  if (C->qwait == 0) {
    C->qwait = 2;
    double etaqm1 = 0.0, etaqp1 = 0.0;
    if (q > 1) {
      const double e = sqrt(s[0] / C->N) * factorial(q - 1) / harmonic(q - 1);
      etaqm1 = 1.0 / (pow(kBiasQm1 * e, 1.0 / (double)q) + kAddon);
    }
    if (q < C->qmax) {
      const double e = sqrt(s[1] / C->N) /
                       ((double)(q + 2) * harmonic(q + 1) * harmonic(q + 1));
      etaqp1 = 1.0 / (pow(kBiasQp1 * e, 1.0 / (double)(q + 2)) + kAddon);
    }
    if (etaq >= etaqm1 && etaq >= etaqp1) {
      eta = etaq;
      qnew = q;
    } else if (etaqm1 >= etaqp1) {
      eta = etaqm1;
      qnew = q - 1;
    } else {
      eta = etaqp1;
      qnew = q + 1;
    }
  }
  for (int j = 0; j < kQmaxAll + 2; ++j) C->hs[j] = 1.0;
  if (eta >= kThresh) {
    if (eta > kEtaMax) eta = kEtaMax;
    C->q = qnew;
    rescale(C, eta);
    C->h = C->h * eta;
    C->qwait = C->q + 1;
  }
  C->ncf = 0;
  C->netf = 0;
  C->force_lu = 0;
  if (C->t >= C->tend)
    C->phase = PH_DONE;
  else if (C->nsteps >= C->step_limit)
    C->phase = PH_PAUSE;
  else
    prepare_attempt(C);
}

// Starting step: Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4, with
// WRMS norms and p = 1, or the user's h0.  z[1] holds f(y0) and its pending
// scale becomes h, so z[1] = h f(y0).
__device__ inline void finish_init(Ctrl* C, double h) {
  C->h = h;
  for (int j = 0; j < kQmaxAll + 2; ++j) C->hs[j] = 1.0;
  C->hs[1] = h;
  C->q = 1;
  C->qwait = 2;
  C->restart = 0;
  if (C->nsteps >= C->step_limit)
    C->phase = PH_PAUSE;
  else
    prepare_attempt(C);
}

__device__ inline void after_init1(Ctrl* C, const double* s) {
  C->nfevals++;
  if (C->h0user > 0.0) {
    double h = C->h0user;
    if (h > C->tend - C->t) h = C->tend - C->t;
    return finish_init(C, h);
  }
  const double d0 = sqrt(s[0] / C->N), d1 = sqrt(s[1] / C->N);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  if (h0 > C->tend - C->t) h0 = C->tend - C->t;
  C->hnw_h0 = h0;
  C->hnw_d1 = d1;
  C->phase = PH_INIT2;
}

__device__ inline void after_init2(Ctrl* C, const double* s) {
  C->nfevals += 2;   // the second estimate evaluation and the history's f(y0)
  const double h0 = C->hnw_h0;
  const double d2 = sqrt(s[0] / C->N) / h0;
  const double dm = C->hnw_d1 > d2 ? C->hnw_d1 : d2;
  const double h1 = dm <= 1e-15 ? (h0 * 1e-3 > 1e-6 ? h0 * 1e-3 : 1e-6) : pow(0.01 / dm, 0.5);
  double h = 100.0 * h0 < h1 ? 100.0 * h0 : h1;
  if (h > C->tend - C->t) h = C->tend - C->t;
  finish_init(C, h);
}

}  // namespace bdfgpu
