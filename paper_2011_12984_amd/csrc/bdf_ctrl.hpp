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
//
// Variable coefficients (vc): the corrector is the BDF formula on the actual
// past grid.  Past accepted points sit at s = -xi_i (units of the attempt's
// h); the correction polynomial prod_{i<=q} (1 + s/xi_i), normalised to
// slope 1, vanishes at them, so the history keeps interpolating the last
// q + 1 accepted values, and the error and order-change constants follow
// from that (constant steps give the fixed ones).  Lazy Newton matrix
// (lazy): the factors of M are stored per cell and reused over steps while
// gamma stays within 30% of theirs, for at most 20 steps, with each
// correction scaled by 2 / (1 + gamma / gamma_s).
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
constexpr int kMsbp = 20;          // lazy: accepted steps between fresh Newton matrices
constexpr double kDgmax = 0.3;     // lazy: largest |gamma / gamma_s - 1| kept
constexpr int kNtau = kQmaxAll + 1;
constexpr int kKryMaxl = 5;        // GMRES: Krylov dimension (no restarts)
constexpr double kKryEplin = 0.05; // GMRES: tolerance factor on the Newton tolerance

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
  // variable coefficients: accepted step sizes (most recent first), the
  // attempt's xi_1..xi_{q+1} (xi[0] = 0), scale and step of the saved
  // correction, and kap, the factor on acor_prev in the order-(q+1) sum;
  // a lowering of the order applied with the deferred update:
  // z_new[j] -= upd_d[j] z_new[q] for j = 1..q-1
  int vc, ntau, upd_dec, lazy, setup, force_setup, m_valid, pad3;
  double tau[kNtau];
  double xi[kQmaxAll + 3];
  double dprev_c, dprev_h, kap;
  double upd_d[kQmaxAll + 2];
  // lazy Newton matrix: gamma and step count of the stored factors, the
  // correction scale of a reuse, the carried convergence-rate estimate
  double gamma_s, dscale, crate_keep;
  long nst_s, nstale_retries;
  int krylov, pad4;          // Newton-Krylov: GMRES solves the current M (no scaling)
  // Newton iterations per launch of the fused kernel (kiters <= maxcor):
  // a launch runs iterations m0 .. m0 + kiters - 1; when the replay of
  // their sums leaves the attempt undecided, m0 moves on and the next
  // launch continues from the stored iterate (the phase stays PH_PREDICT)
  int kiters, m0;
  long ncont;                // continuation launches
  long nliters;              // GMRES iterations
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
// With variable coefficients: xi_1 = 1, xi_{i+1} = xi_i + tau_{i-1} / h
// (points older than the known steps one h apart), l_j = [s^j] prod_{i<=q}
// (1 + s/xi_i) / S_q with S_k = sum_{i<=k} 1/xi_i, local-error constant
// (1/xi_{q+1}) / (S_q S_{q+1}); kap brings the saved correction to this
// step's scale: (h / h_prev)^{q+1} c_prev / c with c = 1 / (prod_{i<=q+1}
// xi_i S_{q+1}).
__device__ inline void set_coeffs(Ctrl* C) {
  const int q = C->q;
  double c[kQmaxAll + 2];
  for (int j = 0; j < kQmaxAll + 2; ++j) c[j] = 0.0;
  c[0] = 1.0;
  if (C->vc) {
    C->xi[0] = 0.0;
    C->xi[1] = 1.0;
    for (int i = 2; i <= kQmaxAll + 2; ++i)
      C->xi[i] = C->xi[i - 1] + (i - 2 < C->ntau ? C->tau[i - 2] / C->h : 1.0);
    for (int i = 1; i <= q; ++i)
      for (int j = i; j >= 1; --j) c[j] = c[j] + c[j - 1] / C->xi[i];
    double Sq = 0.0;
    for (int i = 1; i <= q; ++i) Sq = Sq + 1.0 / C->xi[i];
    for (int j = 0; j < kQmaxAll + 2; ++j) C->l[j] = j <= q ? c[j] / Sq : 0.0;
    const double Sq1 = Sq + 1.0 / C->xi[q + 1];
    C->tq = (1.0 / C->xi[q + 1]) / (Sq * Sq1);
    double pxi = 1.0;
    for (int i = 1; i <= q + 1; ++i) pxi = pxi * C->xi[i];
    const double cn = 1.0 / (pxi * Sq1);
    C->kap = C->dprev_h > 0.0 ? pow(C->h / C->dprev_h, (double)(q + 1)) * C->dprev_c / cn : 1.0;
    C->craise = 0.0;   // a raise is formed by after_accept
    return;
  }
  for (int i = 1; i <= q; ++i)
    for (int j = i; j >= 1; --j) c[j] = c[j] + c[j - 1] / (double)i;
  const double H = harmonic(q);
  for (int j = 0; j < kQmaxAll + 2; ++j) C->l[j] = j <= q ? c[j] / H : 0.0;
  C->tq = 1.0 / ((double)(q + 1) * H * harmonic(q + 1));
  C->craise = 1.0 / (factorial(q + 1) * harmonic(q + 1));
  C->kap = 1.0;
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
  C->m0 = 0;
  C->crate = 1.0;
  C->dold = 0.0;
  C->phase = PH_PREDICT;
  C->nattempts++;
  C->hist_reads += C->q + 1;
  C->setup = 1;
  C->dscale = 1.0;
  if (C->lazy) {
    const bool fresh = !C->m_valid || C->force_setup || C->nsteps - C->nst_s >= kMsbp ||
                       fabs(C->gamma / C->gamma_s - 1.0) > kDgmax;
    if (fresh) {
      C->gamma_s = C->gamma;
      C->nst_s = C->nsteps;
      C->m_valid = 1;
      C->force_setup = 0;
    } else {
      C->setup = 0;
      C->dscale = C->krylov ? 1.0 : 2.0 / (1.0 + C->gamma / C->gamma_s);
      C->crate = C->crate_keep;
    }
  }
  if (C->setup) C->nsetups++;
}

__device__ inline void fail_error(Ctrl* C, int code) {
  C->status = code;
  C->phase = PH_ERROR;
}

__device__ inline void newton_failed(Ctrl* C) {
  C->crate_keep = C->crate;
  if (C->lazy) {
    C->force_setup = 1;
    if (!C->setup) {   // reused factors: redo the attempt with fresh ones
      C->nstale_retries++;
      return prepare_attempt(C);
    }
  }
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
    C->ntau = 0;             // the new history knows no past points
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
  const int m0 = C->m0;
  const int m1 = m0 + C->kiters < C->maxcor ? m0 + C->kiters : C->maxcor;
  C->m0 = 0;
  for (int m = m0; m < m1; ++m) {
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
    // learned mode: no acceptance at the first iteration (no cell has a
    // contraction rate yet), nor at an iteration where a cell on its
    // approximate inverse did not contract (slot 7 of iterations >= 1)
    const bool lp_open = C->learned && !C->force_lu && (m == 0 || t[7] > 0.0);
    if (dcon <= kNlsCoef && !lp_open) {
      C->m = m;
      C->crate_keep = C->crate;
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
          C->upd_raise = (!C->vc && C->qwait == 1 && C->q < kQmaxAll && C->q < C->qmax) ? 1 : 0;
          C->upd_dec = 0;
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
  if (m1 < C->maxcor) {   // undecided: the next launch continues at m1
    C->m0 = m1;
    C->ncont++;
    return;
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
  double Sq1 = 0.0, pxi = 1.0;   // variable coefficients: S_{q+1}, prod xi
  if (C->vc) {
    for (int k = kNtau - 1; k > 0; --k) C->tau[k] = C->tau[k - 1];
    C->tau[0] = C->h;
    if (C->ntau < kNtau) C->ntau++;
    for (int i = 1; i <= q + 1; ++i) {
      Sq1 = Sq1 + 1.0 / C->xi[i];
      pxi = pxi * C->xi[i];
    }
    C->dprev_c = 1.0 / (pxi * Sq1);
    C->dprev_h = C->h;
  }
  const double err = C->err;
  const double etaq = 1.0 / (pow(kBiasQ * err, 1.0 / (double)(q + 1)) + kAddon);
  double eta = etaq;
  int qnew = q;
  if (C->qwait == 0) {
    C->qwait = 2;
    double etaqm1 = 0.0, etaqp1 = 0.0;
    if (q > 1) {
      // order q-1: |z[q]| prod_{i<q} xi_i / S_{q-1} ((q-1)! / H_{q-1} at
      // constant steps)
      double pr = factorial(q - 1), S = harmonic(q - 1);
      if (C->vc) {
        pr = 1.0;
        S = 0.0;
        for (int i = 1; i <= q - 1; ++i) {
          pr = pr * C->xi[i];
          S = S + 1.0 / C->xi[i];
        }
      }
      const double e = sqrt(s[0] / C->N) * pr / S;
      etaqm1 = 1.0 / (pow(kBiasQm1 * e, 1.0 / (double)q) + kAddon);
    }
    if (q < C->qmax) {
      // order q+1: |acor - kap acor_prev| / ((q+2) S_{q+1}^2)
      const double S1 = C->vc ? Sq1 : harmonic(q + 1);
      const double e = sqrt(s[1] / C->N) / ((double)(q + 2) * S1 * S1);
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
    if (C->vc && C->fuse && qnew == q + 1) {
      // raise keeping the interpolation: the update adds
      // cr acor s prod_{i<=q} (s + xi_i), cr = Lambda(-xi_{q+1}) /
      // (xi_{q+1} prod_{i<=q} (xi_i - xi_{q+1})), so the history also passes
      // through the accepted value before the last q + 1
      double lam = 0.0, pw = 1.0, den = C->xi[q + 1], e[kQmaxAll + 3];
      for (int j = 0; j <= q; ++j) {
        lam = lam + C->l[j] * pw;
        pw = pw * -C->xi[q + 1];
      }
      for (int i = 1; i <= q; ++i) den = den * (C->xi[i] - C->xi[q + 1]);
      const double cr = lam / den;
      for (int j = 0; j < kQmaxAll + 3; ++j) e[j] = 0.0;
      e[1] = 1.0;
      for (int i = 1; i <= q; ++i)
        for (int j = i + 1; j >= 1; --j) e[j] = e[j - 1] + C->xi[i] * e[j];
      for (int j = 1; j <= q; ++j) C->upd_l[j] = C->upd_l[j] + cr * e[j];
      C->upd_craise = cr;
      C->upd_raise = 1;
    } else if (C->vc && C->fuse && qnew == q - 1) {
      // lowering keeping the interpolation: subtract z[q] s prod_{i<q}
      // (s + xi_i), applied by the update after z_new is formed
      double d[kQmaxAll + 3];
      for (int j = 0; j < kQmaxAll + 3; ++j) d[j] = 0.0;
      d[1] = 1.0;
      for (int i = 1; i <= q - 1; ++i)
        for (int j = i + 1; j >= 1; --j) d[j] = d[j - 1] + C->xi[i] * d[j];
      for (int j = 0; j < kQmaxAll + 2; ++j) C->upd_d[j] = d[j];
      C->upd_dec = 1;
    }
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
  C->ntau = 0;
  C->m_valid = 0;
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
