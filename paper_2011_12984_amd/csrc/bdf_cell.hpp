// Per-cell adaptive stepping: every cell of a thread-per-cell class is its
// own ODE with its own step size, order and step count.
//
// The grouped integrator (bdf_ctrl.hpp) advances all cells with one h and q
// and global WRMS norms, so the stiffest cell sets everyone's step; the
// paper notes that grouping trades this for fewer, larger operations and
// lets every task run its own integrator instead (Section 7, task-local
// integrators; Fig. cvodestreams).  Here the task is a single cell: each
// lane runs the same method as the grouped controller (predictor, Newton
// with a fresh factorisation per attempt, local error test, step and order
// selection) on norms over its own species only, so one cell's result is
// exactly what the grouped method computes for a problem of that one cell.
// No reduction crosses cells: one launch is one attempt of every unfinished
// cell, and its decisions are taken in registers.  The history keeps a
// pending scale hsc per cell (true z[j] = stored z[j] * hsc^j) so that a
// rejected attempt writes nothing back.
#pragma once

#include "bdf_dev.hpp"

namespace bdfgpu {

// Per-cell control state, arrays of ncells (cell index c).
struct CellDev {
  double* t;       // time reached
  double* h;       // next step size
  double* hsc;     // pending history scale
  double* hu;      // last accepted step size
  int* iv;         // 4 per cell: q, qwait, ncf | netf << 8 | restart << 16, status
  int* cnt;        // 5 per cell: steps, attempts, Newton iterations, error-test and
                   // convergence failures
  double tend, h0user, hmin;
  int qmax, maxcor;
  int cap;                // attempts per cell in one launch
  long max_att;           // attempts per cell in all (0: unlimited)
  unsigned int* active;   // [slot]: cells still running after the launch
  int slot;
};

enum CellStatus : int { CELL_RUN = 0, CELL_DONE = 1 };

// Coefficients of order q (per lane), the same operations as set_coeffs.
__device__ __forceinline__ void cell_coeffs(int q, double (&l)[kQmaxAll + 2], double& tq,
                                            double& craise) {
  double c[kQmaxAll + 2];
#pragma unroll
  for (int j = 0; j < kQmaxAll + 2; ++j) c[j] = 0.0;
  c[0] = 1.0;
#pragma unroll
  for (int i = 1; i <= kQmaxAll; ++i)
    if (i <= q)
#pragma unroll
      for (int j = i; j >= 1; --j) c[j] = c[j] + c[j - 1] / (double)i;
  double H = 0.0, fq1 = 1.0;
#pragma unroll
  for (int i = 1; i <= kQmaxAll; ++i)
    if (i <= q) H += 1.0 / (double)i;
#pragma unroll
  for (int i = 2; i <= kQmaxAll + 1; ++i)
    if (i <= q + 1) fq1 *= (double)i;
  const double H1 = H + 1.0 / (double)(q + 1);
#pragma unroll
  for (int j = 0; j < kQmaxAll + 2; ++j) l[j] = j <= q ? c[j] / H : 0.0;
  tq = 1.0 / ((double)(q + 1) * H * H1);
  craise = 1.0 / (fq1 * H1);
}

__device__ __forceinline__ double harmonic_lane(int q) {
  double s = 0.0;
#pragma unroll
  for (int i = 1; i <= kQmaxAll; ++i)
    if (i <= q) s += 1.0 / (double)i;
  return s;
}

__device__ __forceinline__ double factorial_lane(int q) {
  double s = 1.0;
#pragma unroll
  for (int i = 2; i <= kQmaxAll; ++i)
    if (i <= q) s *= (double)i;
  return s;
}

// Starting step of every cell (Hairer, Norsett & Wanner, Solving ODEs I,
// Sec. II.4, WRMS norms over the cell's species, p = 1), or the user's h0;
// z[1] = h f(y0).
template <int NP, bool FULL>
__global__ void __launch_bounds__(kTpcThreads) k_cell_init(BdfDev D, CellDev P) {
  extern __shared__ double lds[];
  using TP = Tpc<NP, kTpcThreads>;
  const ClassDev& K = D.k;
  const int n = FULL ? NP : K.n;
  const long c = (long)blockIdx.x * kTpcThreads + threadIdx.x;
  if (c >= K.ncells) return;
  if (P.iv[4 * c + 3] != CELL_RUN || P.h[c] > 0.0) return;   // started already
  double* ycol = lds + threadIdx.x;
  double* kcol = lds + NP * kTpcThreads + threadIdx.x;
  for (int k = 0; k < K.R; ++k) kcol[k * kTpcThreads] = K.rates[TP::kidx(c, k, K.R)];
  double y0[NP], f0[NP], w[NP];
  tpc_load_vec<NP>(K.z[0], c, n, y0);
  TP::store_col(ycol, y0);
  NetTables::rhs<NP, kTpcThreads>(K.net, kcol, kTpcThreads, ycol, f0);
  const double t = P.t[c];
  double h;
  if (P.h0user > 0.0) {
    h = P.h0user;
    if (h > P.tend - t) h = P.tend - t;
  } else {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      w[i] = i < n ? 1.0 / (D.rtol * fabs(y0[i]) + D.atol) : 0.0;
      if (i < n) {
        s0 = fma(y0[i] * w[i], y0[i] * w[i], s0);
        s1 = fma(f0[i] * w[i], f0[i] * w[i], s1);
      }
    }
    const double d0 = sqrt(s0 / (double)n), d1 = sqrt(s1 / (double)n);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
    if (h0 > P.tend - t) h0 = P.tend - t;
    double y1[NP], f1[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) y1[i] = y0[i] + h0 * f0[i];
    TP::store_col(ycol, y1);
    NetTables::rhs<NP, kTpcThreads>(K.net, kcol, kTpcThreads, ycol, f1);
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double d = (f1[i] - f0[i]) * w[i];
      if (i < n) s2 = fma(d, d, s2);
    }
    const double d2 = sqrt(s2 / (double)n) / h0;
    const double dm = d1 > d2 ? d1 : d2;
    const double h1 =
        dm <= 1e-15 ? (h0 * 1e-3 > 1e-6 ? h0 * 1e-3 : 1e-6) : pow(0.01 / dm, 0.5);
    h = 100.0 * h0 < h1 ? 100.0 * h0 : h1;
    if (h > P.tend - t) h = P.tend - t;
  }
#pragma unroll
  for (int i = 0; i < NP; ++i)
    if (i < n) K.z[1][TP::idx(c, i, n)] = f0[i] * h;
  P.h[c] = h;
  P.hsc[c] = 1.0;
  P.iv[4 * c + 0] = 1;   // q
  P.iv[4 * c + 1] = 2;   // qwait
  P.iv[4 * c + 2] = 0;
  P.cnt[5 * c + 1] = 0;
}

// Up to P.cap attempts of every unfinished cell: each one prepares (tstop
// clamp, coefficients), predicts, builds J and the LU at the predicted state,
// runs Newton with the cell's own convergence test and the error test, then
// either updates the history with step and order selection or sets the
// cell's retry parameters.  A lane stops at its cell's end (or failure); the
// wave stops when all its lanes have, so a few slow cells keep only their
// own waves busy.
// LS: 0 FP64 LU, 3 Gauss-Jordan inverse (NP <= 4).
template <int NP, bool FULL, int LS>
__global__ void __launch_bounds__(kTpcThreads) k_cell_attempt(BdfDev D, CellDev P) {
  extern __shared__ double lds[];
  using TP = Tpc<NP, kTpcThreads>;
  constexpr int TB = kTpcThreads;
  const ClassDev& K = D.k;
  const NetDev& nd = K.net;
  const int n = FULL ? NP : K.n, R = K.R;
  const long c = (long)blockIdx.x * TB + threadIdx.x;
  const bool in = c < K.ncells;
  int status = in ? P.iv[4 * c + 3] : CELL_DONE;
  const bool run = status == CELL_RUN;
  if (__ballot(run) == 0) return;
  double* ycol = lds + threadIdx.x;
  double* kcol = lds + NP * TB + threadIdx.x;
  if (run)
    for (int k = 0; k < R; ++k) kcol[k * TB] = K.rates[TP::kidx(c, k, R)];
  double t = 0.0, h = 1.0, hsc = 1.0;
  int q = 1, qwait = 2, ncf = 0, netf = 0, restart = 0;
  int nst = 0, nat = 0, nit = 0, nef = 0, ncfs = 0;
  if (run) {
    t = P.t[c];
    h = P.h[c];
    hsc = P.hsc[c];
    q = P.iv[4 * c + 0];
    qwait = P.iv[4 * c + 1];
    const int fl = P.iv[4 * c + 2];
    ncf = fl & 0xff;
    netf = (fl >> 8) & 0xff;
    restart = (fl >> 16) & 1;
    nst = P.cnt[5 * c + 0];
    nat = P.cnt[5 * c + 1];
    nit = P.cnt[5 * c + 2];
    nef = P.cnt[5 * c + 3];
    ncfs = P.cnt[5 * c + 4];
  }
  for (int att = 0; att < P.cap; ++att) {
    if (status == CELL_RUN && P.max_att > 0 && nat >= P.max_att) status = BDFGPU_ERR_TOO_MUCH_WORK;
    if (status == CELL_RUN && h <= 4.0 * 2.220446049250313e-16 * fabs(t)) status = BDFGPU_ERR_HMIN;
    if (!__any(status == CELL_RUN)) break;
    const bool act = status == CELL_RUN;   // this lane attempts a step
    // prepare: land exactly on tend
    if (act && t + h > P.tend) {
      const double eta = (P.tend - t) / h;
      hsc *= eta;
      h = P.tend - t;
      qwait = q + 1;
    }
    const bool last = t + h >= P.tend;
    double l[kQmaxAll + 2], tq, craise;
    cell_coeffs(q, l, tq, craise);
    const double gamma = h * l[0];
    const double l0 = l[0];
    // history (every row: the orders differ across the wave), scaled
    double zs[kQmaxAll + 1][NP];
    double f[NP];
    {
      double sj = 1.0;
  #pragma unroll
      for (int j = 0; j <= kQmaxAll; ++j) {
        double v[NP];
        tpc_load_vec<NP>(K.z[j], c < K.ncells ? c : 0, n, v);
  #pragma unroll
        for (int i = 0; i < NP; ++i) zs[j][i] = (act && j <= q) ? v[i] * sj : 0.0;
        sj *= hsc;
      }
    }
    double w[NP];
  #pragma unroll
    for (int i = 0; i < NP; ++i) w[i] = i < n ? 1.0 / (D.rtol * fabs(zs[0][i]) + D.atol) : 0.0;
    if (__any(act && restart)) {
      // restart at order 1 after repeated error-test failures: z[1] = h f(z[0])
      // (written back, as the grouped predictor does; the history's scale is 1)
      TP::store_col(ycol, zs[0]);
      NetTables::rhs<NP, TB>(nd, kcol, TB, ycol, f);
      if (act && restart) {
  #pragma unroll
        for (int i = 0; i < NP; ++i) {
          zs[1][i] = i < n ? h * f[i] : 0.0;
          if (i < n) K.z[1][TP::idx(c, i, n)] = zs[1][i];
        }
      }
    }
    restart = 0;
  #pragma unroll
    for (int k = 1; k <= kQmaxAll; ++k)
  #pragma unroll
      for (int j = kQmaxAll; j >= k; --j)
        if (k <= q && j <= q)
  #pragma unroll
          for (int i = 0; i < NP; ++i) zs[j - 1][i] = zs[j - 1][i] + zs[j][i];
    double zp0[NP], cv[NP];
  #pragma unroll
    for (int i = 0; i < NP; ++i) {
      zp0[i] = zs[0][i];
      cv[i] = zs[0][i] - l0 * zs[1][i];
    }
    TP::store_col(ycol, zp0);
    double A[NP][NP], rowsum[NP];
    int piv[NP];
    constexpr int NX = LS == 3 ? NP : 1;   // LS 3: the block's explicit inverse
    double Xi[NX][NX];
    NetTables::build_M<NP, TB, double, false>(nd, kcol, TB, ycol, gamma, A, rowsum);
    int info;
    if constexpr (LS == 3)
      info = TpcGJ<NP>::invert(A, Xi);
    else
      info = TpcLU<NP, double>::factor(A, piv);
    double y[NP];
  #pragma unroll
    for (int i = 0; i < NP; ++i) y[i] = zp0[i];
    // Newton: converged, failed, or undecided; a lane stops iterating at its
    // decision (its iterate then stays)
    bool conv = false, fail = act && info != 0;
    if (fail) nit++;   // the grouped count includes the iteration a singular setup fails
    double crate = 1.0, dold = 0.0;
    for (int m = 0; m < P.maxcor; ++m) {
      const bool go = act && !conv && !fail;
      if (!__any(go)) break;
      TP::store_col(ycol, y);
      NetTables::rhs<NP, TB>(nd, kcol, TB, ycol, f);
      double del[NP];
  #pragma unroll
      for (int i = 0; i < NP; ++i) del[i] = fma(gamma, f[i], cv[i] - y[i]);
      if constexpr (LS == 3) {
        double rr[NP];
  #pragma unroll
        for (int i = 0; i < NP; ++i) rr[i] = del[i];
        TpcGJ<NP>::apply(Xi, rr, del);
      } else {
        TpcLU<NP, double>::solve(A, piv, del);
      }
      if (go) {
        nit++;
        double sd = 0.0;
  #pragma unroll
        for (int i = 0; i < NP; ++i) {
          if (i < n) {
            y[i] += del[i];
            const double a = del[i] * w[i];
            sd = fma(a, a, sd);
          }
        }
        const double d = sqrt(sd / (double)n);
        if (!(d == d) || d > 1e300) {
          fail = true;
        } else {
          if (m > 0) {
            const double ratio = d / dold;
            crate = kCrDown * crate > ratio ? kCrDown * crate : ratio;
          }
          const double dcon = d * (crate < 1.0 ? crate : 1.0);
          if (dcon <= kNlsCoef) {
            conv = true;
          } else if (m + 1 == P.maxcor || (m >= 1 && d > kRdiv * dold)) {
            fail = true;
          }
          dold = d;
        }
      }
    }
    if (act && !conv) fail = true;
    if (act) nat++;
    // decisions
    double acor[NP];
    double err = 0.0;
    if (act && conv) {
      double sa = 0.0;
  #pragma unroll
      for (int i = 0; i < NP; ++i) {
        const double yp = (D.nonneg && y[i] < 0.0) ? 0.0 : y[i];
        y[i] = yp;
        acor[i] = i < n ? (yp - zp0[i]) / l0 : 0.0;
        const double b = i < n ? (yp - zp0[i]) * w[i] : 0.0;
        sa = fma(b, b, sa);
      }
      err = sqrt(sa / (double)n) / l0 * tq;
    }
    bool accept = act && conv && err <= 1.0;
    if (act && fail) {
      ncf++;
      ncfs++;
      if (ncf >= kMxNcf) {
        status = BDFGPU_CONV_FAIL;
      } else if (h * kEtaCf < P.hmin) {
        status = BDFGPU_ERR_HMIN;
      } else {
        hsc *= kEtaCf;
        h *= kEtaCf;
        qwait = q + 1;
      }
    } else if (act && !accept) {
      netf++;
      nef++;
      if (netf >= kMxNef) {
        status = BDFGPU_TEST_FAIL;
      } else if (netf >= 3) {
        const double hn = h * kEtaRestart;
        if (hn < P.hmin) {
          status = BDFGPU_ERR_HMIN;
        } else {
          h = hn;
          q = 1;
          restart = 1;
          hsc = 1.0;
          qwait = 2;
        }
      } else {
        double eta = 0.9 * pow(err, -1.0 / (double)(q + 1));
        if (eta < kEtaMinEf) eta = kEtaMinEf;
        if (h * eta < P.hmin) {
          status = BDFGPU_ERR_HMIN;
        } else {
          hsc *= eta;
          h *= eta;
          qwait = q + 1;
        }
      }
    }
    // accepted: history update z_new[j] = z(0)[j] + l_j acor from the history
    // read again (the predicted rows were not kept through the iterations),
    // step and order selection
    const bool sel = accept && qwait == 1;
    const bool raise = sel && q < kQmaxAll && q < P.qmax;
    double dp[NP];
    if (__any(raise)) tpc_load_vec<NP>(K.dprev, c < K.ncells ? c : 0, n, dp);
    if (__any(accept)) {
      double zu[kQmaxAll + 1][NP];
      {
        double sj = 1.0;
  #pragma unroll
        for (int j = 0; j <= kQmaxAll; ++j) {
          double v[NP];
          tpc_load_vec<NP>(K.z[j], c < K.ncells ? c : 0, n, v);
  #pragma unroll
          for (int i = 0; i < NP; ++i) zu[j][i] = (accept && j <= q) ? v[i] * sj : 0.0;
          sj *= hsc;
        }
      }
  #pragma unroll
      for (int k = 1; k <= kQmaxAll; ++k)
  #pragma unroll
        for (int j = kQmaxAll; j >= k; --j)
          if (k <= q && j <= q)
  #pragma unroll
            for (int i = 0; i < NP; ++i) zu[j - 1][i] = zu[j - 1][i] + zu[j][i];
      if (accept) {
      double szq = 0.0, sdd = 0.0;
  #pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (i < n) {
          const long id = TP::idx(c, i, n);
          K.z[0][id] = y[i];
          double znq = y[i];
  #pragma unroll
          for (int j = 1; j <= kQmaxAll; ++j) {
            if (j <= q) {
              const double zn = fma(l[j], acor[i], zu[j][i]);
              K.z[j][id] = zn;
              if (j == q) znq = zn;
            }
          }
          if (raise) {
            K.z[q + 1][id] = craise * acor[i];
            const double b = (acor[i] - dp[i]) * w[i];
            sdd = fma(b, b, sdd);
          }
          if (qwait == 2) K.dprev[id] = acor[i];
          const double a = znq * w[i];
          szq = fma(a, a, szq);
        }
      }
      t = last ? P.tend : t + h;
      P.hu[c] = h;
      nst++;
      qwait--;
      const double etaq = 1.0 / (pow(kBiasQ * err, 1.0 / (double)(q + 1)) + kAddon);
      double eta = etaq;
      int qnew = q;
      if (qwait == 0) {
        qwait = 2;
        double etaqm1 = 0.0, etaqp1 = 0.0;
        if (q > 1) {
          const double e = sqrt(szq / (double)n) * factorial_lane(q - 1) / harmonic_lane(q - 1);
          etaqm1 = 1.0 / (pow(kBiasQm1 * e, 1.0 / (double)q) + kAddon);
        }
        if (q < P.qmax) {
          const double hq1 = harmonic_lane(q + 1);
          const double e = sqrt(sdd / (double)n) / ((double)(q + 2) * hq1 * hq1);
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
      hsc = 1.0;
      if (eta >= kThresh) {
        if (eta > kEtaMax) eta = kEtaMax;
        q = qnew;
        hsc = eta;
        h = h * eta;
        qwait = q + 1;
      }
      ncf = 0;
      netf = 0;
      if (t >= P.tend) status = CELL_DONE;
      }
    }
  }
  if (run) {
    P.t[c] = t;
    P.h[c] = h;
    P.hsc[c] = hsc;
    P.iv[4 * c + 0] = q;
    P.iv[4 * c + 1] = qwait;
    P.iv[4 * c + 2] = ncf | (netf << 8) | (restart << 16);
    P.iv[4 * c + 3] = status;
    P.cnt[5 * c + 0] = nst;
    P.cnt[5 * c + 1] = nat;
    P.cnt[5 * c + 2] = nit;
    P.cnt[5 * c + 3] = nef;
    P.cnt[5 * c + 4] = ncfs;
  }
  // cells still running after this attempt
  const unsigned long long still = __ballot(in && status == CELL_RUN);
  if (threadIdx.x == 0 && still) atomicAdd(P.active + P.slot, (unsigned int)__popcll(still));
}

}  // namespace bdfgpu
