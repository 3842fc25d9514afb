// Per-cell kernels of the grouped BDF step on gfx950.
//
// One step attempt runs: predictor + first Newton iteration, further Newton
// iterations, then the history update.  Every kernel re-evaluates the
// mass-action Jacobian at the predicted state and re-factors M = I - gamma J
// of its cells in registers instead of storing the factors: a 10 x 10 FP64
// factorisation costs ~700 flops but storing and re-reading it would cost
// 1.6 kB of HBM traffic per cell and iteration.  HBM then carries only the
// vectors of the method.
//
// Two mappings of cells to lanes:
//  * thread per cell (TPC, n <= 12): the block lives in one lane's
//    registers; vectors use a tiled layout (64 cells per tile, species-major
//    inside the tile) so that every load and store is a full 512-byte
//    wavefront access.
//  * segment per cell (SPC, 12 < n <= 64): one lane per row of the block in
//    a segment of 16, 32 or 64 lanes (see spc.hpp); vectors are cell-major.
#pragma once

#include <hip/hip_runtime.h>

#include "bdf_ctrl.hpp"
#include "common.hpp"
#include "spc.hpp"

namespace bdfgpu {

// Shared network of one class of cells: r_k = kappa_k * y[ra_k] * y[rb_k]
// (missing reactant = -1), f = S r, and for the Jacobian a list per column a
// of (reaction k, partner species p or -1, multiplicity m): dr_k/dy_a =
// m kappa_k y_p.
struct NetDev {
  int n, R, np;          // species, reactions, padded row length of S
  const double* S;       // [R][np] net stoichiometry mu - nu
  const int* ra;         // [R]
  const int* rb;         // [R]
  const int* jst;        // [np + 1] start of each column's list
  const int* jk;         // [nent]
  const int* jp;         // [nent]
  const double* jm;      // [nent]
};

struct ClassDev {
  long ncells;
  int n, R;
  double* z[kQmaxAll + 1];
  double* dprev;
  double* zp0;
  double* cv;            // z(0)[0] - l0 z(0)[1]
  double* y;             // Newton iterate
  const double* rates;
  NetDev net;
  long blk0;             // first block of this class in the phase reduction
  int refine_max_it;
  // learned preconditioner
  float* X;              // per cell n x n approximate inverse (row-major)
  double* xin;           // per cell MLP inputs [z(0)[0], log gamma]
  int* lpmode;           // per cell: 2 learned, 3 switching to LU, 4 / 0 exact LU
  double* dcprev;        // per cell WRMS of the previous correction
};

struct BdfDev {
  Ctrl* C;
  double* partials;
  unsigned int* counter;
  unsigned int nblocks_total;
  double rtol, atol;
  int nonneg;
  ClassDev k;
};

constexpr int kRedVals = 8;
constexpr int kCellThreads = 256;

// Block-level reduction of the kRedVals partial sums of one kernel, then the
// device controller in the last block across all launches of the phase.
template <typename F>
__device__ __forceinline__ void reduce_and_control(const BdfDev& D, double (&v)[kRedVals],
                                                   double* sh, F&& control) {
  block_sum<kRedVals>(v, sh);
  double tot[kRedVals];
  const unsigned int gb = (unsigned int)(D.k.blk0 + blockIdx.x);
  // the ticket/last-block protocol, with a global block index
  __shared__ int am_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kRedVals; ++k) D.partials[(size_t)gb * kRedVals + k] = v[k];
    __threadfence();
    const unsigned int t = atomicAdd(D.counter, 1u);
    am_last = (t == D.nblocks_total - 1);
  }
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  double acc[kRedVals];
#pragma unroll
  for (int k = 0; k < kRedVals; ++k) acc[k] = 0.0;
  for (unsigned int b = threadIdx.x; b < D.nblocks_total; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kRedVals; ++k)
      acc[k] += __hip_atomic_load(&D.partials[(size_t)b * kRedVals + k], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum<kRedVals>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kRedVals; ++k) tot[k] = acc[k];
    *D.counter = 0u;
    control(D.C, tot);
  }
}

// ===========================================================================
// Thread per cell
// ===========================================================================
template <int NP>
struct Tpc {
  // tiled index of species i of cell c (n species per cell)
  __device__ static __forceinline__ long idx(long c, int i, int n) {
    return (c >> 6) * 64L * n + (long)i * 64 + (c & 63);
  }
  __device__ static __forceinline__ long kidx(long c, int k, int R) {
    return (c >> 6) * 64L * R + (long)k * 64 + (c & 63);
  }

  // ycol: this thread's LDS column (stride kCellThreads) holding the state
  __device__ static void rhs(const NetDev& nd, const double* kap, const double* ycol,
                             double (&f)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) f[i] = 0.0;
    for (int k = 0; k < nd.R; ++k) {
      const int a = nd.ra[k], b = nd.rb[k];
      double r = kap[(long)k * 64];
      if (a >= 0) r *= ycol[a * kCellThreads];
      if (b >= 0) r *= ycol[b * kCellThreads];
      const double* Sk = nd.S + (long)k * nd.np;
#pragma unroll
      for (int i = 0; i < NP; ++i) f[i] = fma(Sk[i], r, f[i]);
    }
  }

  __device__ static void jac(const NetDev& nd, const double* kap, const double* ycol,
                             double (&J)[NP][NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = 0; j < NP; ++j) J[i][j] = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const int e0 = nd.jst[a], e1 = nd.jst[a + 1];
      for (int e = e0; e < e1; ++e) {
        const int k = nd.jk[e], p = nd.jp[e];
        double g = kap[(long)k * 64] * nd.jm[e];
        if (p >= 0) g *= ycol[p * kCellThreads];
        const double* Sk = nd.S + (long)k * nd.np;
#pragma unroll
        for (int i = 0; i < NP; ++i) J[i][a] = fma(Sk[i], g, J[i][a]);
      }
    }
  }

  template <typename T>
  __device__ static int factor(T (&A)[NP][NP], int (&piv)[NP]) {
    int info = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      int p = k;
      T amax = sabs(A[k][k]);
#pragma unroll
      for (int i = k + 1; i < NP; ++i) {
        const T v = sabs(A[i][k]);
        const bool gt = v > amax;
        amax = gt ? v : amax;
        p = gt ? i : p;
      }
      piv[k] = p;
#pragma unroll
      for (int i = k + 1; i < NP; ++i) {
        const bool sw = (p == i);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
          const T t = A[k][j];
          A[k][j] = sw ? A[i][j] : t;
          A[i][j] = sw ? t : A[i][j];
        }
      }
      const T d = A[k][k];
      const bool z = (d == T(0));
      if (z && !info) info = k + 1;
      const T dd = z ? T(1) : d;
#pragma unroll
      for (int i = k + 1; i < NP; ++i) {
        const T l = z ? A[i][k] : A[i][k] / dd;
        A[i][k] = l;
#pragma unroll
        for (int j = k + 1; j < NP; ++j) A[i][j] = fma(-l, A[k][j], A[i][j]);
      }
    }
    return info;
  }

  template <typename T>
  __device__ static void solve(const T (&A)[NP][NP], const int (&piv)[NP], T (&b)[NP]) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int p = piv[k];
#pragma unroll
      for (int i = k + 1; i < NP; ++i) {
        const bool sw = (p == i);
        const T t = b[k];
        b[k] = sw ? b[i] : t;
        b[i] = sw ? t : b[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = 0; j < i; ++j) b[i] = fma(-A[i][j], b[j], b[i]);
#pragma unroll
    for (int i = NP - 1; i >= 0; --i) {
#pragma unroll
      for (int j = i + 1; j < NP; ++j) b[i] = fma(-A[i][j], b[j], b[i]);
      b[i] = b[i] / A[i][i];
    }
  }

  // Column a of J at the state held in ycol (a is a compile-time constant
  // after unrolling at the call site).
  __device__ static __forceinline__ void jac_col(const NetDev& nd, const double* kap,
                                                 const double* ycol, int a, double (&col)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) col[i] = 0.0;
    const int e0 = nd.jst[a], e1 = nd.jst[a + 1];
    for (int e = e0; e < e1; ++e) {
      const int k = nd.jk[e], p = nd.jp[e];
      double g = kap[(long)k * 64] * nd.jm[e];
      if (p >= 0) g *= ycol[p * kCellThreads];
      const double* Sk = nd.S + (long)k * nd.np;
#pragma unroll
      for (int i = 0; i < NP; ++i) col[i] = fma(Sk[i], g, col[i]);
    }
  }

  // M = I - gamma J, assembled one column at a time so that J never needs
  // registers of its own.
  __device__ static void build_M(const NetDev& nd, const double* kap, const double* ycol,
                                 double gamma, double (&M)[NP][NP]) {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      double col[NP];
      jac_col(nd, kap, ycol, a, col);
#pragma unroll
      for (int i = 0; i < NP; ++i) M[i][a] = (i == a ? 1.0 : 0.0) - gamma * col[i];
    }
  }

  // out = (I - gamma J) x without forming J: J x = sum_k S_k (grad r_k . x).
  // x must also be in the LDS column xcol (reactant lookups by index).
  __device__ static void mvp(const NetDev& nd, const double* kap, const double* ycol,
                             const double* xcol, double gamma, const double (&x)[NP],
                             double (&out)[NP]) {
    double jx[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) jx[i] = 0.0;
    for (int k = 0; k < nd.R; ++k) {
      const int a = nd.ra[k], b = nd.rb[k];
      if (a < 0) continue;
      const double kk = kap[(long)k * 64];
      double d;
      if (b < 0)
        d = kk * xcol[a * kCellThreads];
      else
        d = kk * fma(xcol[a * kCellThreads], ycol[b * kCellThreads],
                     ycol[a * kCellThreads] * xcol[b * kCellThreads]);
      const double* Sk = nd.S + (long)k * nd.np;
#pragma unroll
      for (int i = 0; i < NP; ++i) jx[i] = fma(Sk[i], d, jx[i]);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) out[i] = fma(-gamma, jx[i], x[i]);
  }

  // Solve (I - gamma J) x = r, J at the state in ycol.  LS 0: FP64 LU.
  // LS 1: FP32 LU, FP64 residuals from the matrix-free product (so the FP64
  // matrix is never live beside the FP32 factors), FP64 LU fallback.
  // xcol is scratch.  Returns info (singular block).
  template <int LS>
  __device__ static int linsolve(const NetDev& nd, const double* kap, const double* ycol,
                                 double* xcol, double gamma, const double (&r)[NP],
                                 double (&x)[NP], int max_it, int& sweeps, int& fallback) {
    sweeps = 0;
    fallback = 0;
    if (LS == 1) {
      bool ok = false;
      {
        float L[NP][NP];
        double rowsum[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) rowsum[i] = 0.0;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          double col[NP];
          jac_col(nd, kap, ycol, a, col);
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const double m = (i == a ? 1.0 : 0.0) - gamma * col[i];
            L[i][a] = (float)m;
            rowsum[i] += fabs(m);
          }
        }
        double mnorm = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) mnorm = fmax(mnorm, rowsum[i]);
        int pv[NP];
        const int inf32 = factor<float>(L, pv);
        if (!inf32) {
          float v[NP];
#pragma unroll
          for (int i = 0; i < NP; ++i) v[i] = (float)r[i];
          solve<float>(L, pv, v);
#pragma unroll
          for (int i = 0; i < NP; ++i) x[i] = (double)v[i];
          const double eps64 = 2.220446049250313e-16;
          double dprev = 0.0;
          for (int it = 0; it <= max_it; ++it) {
            tpc_store_col_(xcol, x);
            double mx[NP];
            mvp(nd, kap, ycol, xcol, gamma, x, mx);
            double rn = 0.0, xn = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
              mx[i] = r[i] - mx[i];
              rn = fmax(rn, fabs(mx[i]));
              xn = fmax(xn, fabs(x[i]));
            }
            if (!(rn == rn) || !(xn == xn)) break;
            if (rn <= sqrt((double)NP) * eps64 * mnorm * xn) {
              ok = true;
              break;
            }
            if (it == max_it) break;
#pragma unroll
            for (int i = 0; i < NP; ++i) v[i] = (float)mx[i];
            solve<float>(L, pv, v);
            double dn = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
              x[i] += (double)v[i];
              dn = fmax(dn, fabs((double)v[i]));
            }
            sweeps = it + 1;
            if (it >= 1 && dn > 0.5 * dprev) break;
            dprev = dn;
          }
        }
      }
      if (ok) return 0;
      fallback = 1;
    }
    double M[NP][NP];
    build_M(nd, kap, ycol, gamma, M);
    int pv64[NP];
    const int inf = factor<double>(M, pv64);
#pragma unroll
    for (int i = 0; i < NP; ++i) x[i] = r[i];
    solve<double>(M, pv64, x);
    return inf;
  }

  __device__ static __forceinline__ void tpc_store_col_(double* col, const double (&v)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) col[i * kCellThreads] = v[i];
  }
};

template <int NP>
__device__ __forceinline__ void tpc_store_col(double* ycol, const double (&v)[NP]) {
#pragma unroll
  for (int i = 0; i < NP; ++i) ycol[i * kCellThreads] = v[i];
}

// Predictor + first Newton iteration (FIRST = 1) or Newton iteration
// mslot >= 1 (FIRST = 0); the two are separate kernels so that profiles
// attribute their time separately.  Register budget: the state vectors live
// in two per-thread LDS columns, so only M (or the FP32 factors) and the
// right-hand side are live through the factorisation.
template <int NP, int LS, int FIRST>
__global__ void __launch_bounds__(kCellThreads) k_tpc_newton(BdfDev D, int mslot) {
  __shared__ double s_y[NP * kCellThreads];
  __shared__ double s_x[NP * kCellThreads];
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  const int phase = C->phase;
  if (FIRST ? phase != PH_PREDICT : (phase != PH_NEWTON || C->m != mslot)) return;
  const ClassDev& K = D.k;
  const NetDev& nd = K.net;
  const int n = K.n;
  const long c = (long)blockIdx.x * kCellThreads + threadIdx.x;
  const bool act = c < K.ncells;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (act) {
    const double* kap = K.rates + Tpc<NP>::kidx(c, 0, K.R);
    double* ycol = s_y + threadIdx.x;   // z(0)[0]: J is evaluated here
    double* xcol = s_x + threadIdx.x;   // Newton iterate, then scratch
    const double gamma = C->gamma;
    double r[NP];
    if (FIRST) {
      const double l0 = C->l[0];
      const int q = C->q;
      double zs[kQmaxAll + 1][NP];
#pragma unroll
      for (int j = 0; j <= kQmaxAll; ++j) {
        const double hsj = C->hs[j];
#pragma unroll
        for (int i = 0; i < NP; ++i)
          zs[j][i] = (j <= q && i < n) ? K.z[j][Tpc<NP>::idx(c, i, n)] * hsj : 0.0;
      }
      if (C->restart) {
        double f0[NP];
        tpc_store_col<NP>(ycol, zs[0]);
        Tpc<NP>::rhs(nd, kap, ycol, f0);
        const double h = C->h;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          zs[1][i] = h * f0[i];
          if (i < n) K.z[1][Tpc<NP>::idx(c, i, n)] = zs[1][i];
        }
      }
      // Pascal triangle: z(0)[j] = sum_{k >= j} C(k, j) z[k]
#pragma unroll
      for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
        for (int j = kQmaxAll; j >= k; --j)
          if (k <= q && j <= q)
#pragma unroll
            for (int i = 0; i < NP; ++i) zs[j - 1][i] = zs[j - 1][i] + zs[j][i];
      double dcy[NP];   // z(0)[0] - l0 z(0)[1] - y, with y = z(0)[0]
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const double cvi = zs[0][i] - l0 * zs[1][i];
        ycol[i * kCellThreads] = zs[0][i];
        dcy[i] = cvi - zs[0][i];
        if (i < n) {
          const long id = Tpc<NP>::idx(c, i, n);
          K.zp0[id] = zs[0][i];
          K.cv[id] = cvi;
        }
      }
      double f[NP];
      Tpc<NP>::rhs(nd, kap, ycol, f);
#pragma unroll
      for (int i = 0; i < NP; ++i) r[i] = fma(gamma, f[i], dcy[i]);
    } else {
      double dcy[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const bool in = i < n;
        const long id = Tpc<NP>::idx(c, i, n);
        const double yi = in ? K.y[id] : 0.0;
        xcol[i * kCellThreads] = yi;
        ycol[i * kCellThreads] = in ? K.zp0[id] : 0.0;
        dcy[i] = (in ? K.cv[id] : 0.0) - yi;
      }
      double f[NP];
      Tpc<NP>::rhs(nd, kap, xcol, f);
#pragma unroll
      for (int i = 0; i < NP; ++i) r[i] = fma(gamma, f[i], dcy[i]);
    }
    double del[NP];
    int sweeps, fb;
    const int info =
        Tpc<NP>::template linsolve<LS>(nd, kap, ycol, xcol, gamma, r, del, K.refine_max_it,
                                       sweeps, fb);
    double sd = 0.0, sa = 0.0, neg = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < n) {
        const long id = Tpc<NP>::idx(c, i, n);
        const double zp0 = ycol[i * kCellThreads];
        const double yold = FIRST ? zp0 : K.y[id];
        const double ynew = yold + del[i];
        K.y[id] = ynew;
        const double w = 1.0 / (D.rtol * fabs(K.z[0][id]) + D.atol);
        const bool ng = D.nonneg && ynew < 0.0;
        neg += ng ? 1.0 : 0.0;
        const double yp = ng ? 0.0 : ynew;
        const double a = del[i] * w, b = (yp - zp0) * w;
        sd = fma(a, a, sd);
        sa = fma(b, b, sa);
      }
    }
    red[0] = sd;
    red[1] = sa;
    red[2] = info ? 1.0 : 0.0;
    red[3] = (double)sweeps;
    red[4] = (double)fb;
    red[5] = neg;
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_newton(Cc, s); });
}

template <int NP>
__global__ void __launch_bounds__(kCellThreads) k_tpc_accept(BdfDev D) {
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  if (C->phase != PH_ACCEPT) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const long c = (long)blockIdx.x * kCellThreads + threadIdx.x;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells) {
    const int q = C->q;
    const double l0 = C->l[0];
    const bool raise = (C->qwait == 1 && q < C->qmax);
    double zs[kQmaxAll + 1][NP];
#pragma unroll
    for (int j = 0; j <= kQmaxAll; ++j) {
      const double hsj = C->hs[j];
#pragma unroll
      for (int i = 0; i < NP; ++i)
        zs[j][i] = (j <= q && i < n) ? K.z[j][Tpc<NP>::idx(c, i, n)] * hsj : 0.0;
    }
    double w[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) w[i] = i < n ? 1.0 / (D.rtol * fabs(zs[0][i]) + D.atol) : 0.0;
#pragma unroll
    for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
      for (int j = kQmaxAll; j >= k; --j)
        if (k <= q && j <= q)
#pragma unroll
          for (int i = 0; i < NP; ++i) zs[j - 1][i] = zs[j - 1][i] + zs[j][i];
    double szq = 0.0, sdd = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < n) {
        const long id = Tpc<NP>::idx(c, i, n);
        const double yv = K.y[id];
        const double yp = D.nonneg && yv < 0.0 ? 0.0 : yv;
        const double acor = (yp - zs[0][i]) / l0;
        const double dp = K.dprev[id];
        double znq = yp;
        K.z[0][id] = yp;   // z(0)[0] + l0 acor is the corrected solution itself
#pragma unroll
        for (int j = 1; j <= kQmaxAll; ++j) {
          if (j <= q) {
            const double zn = fma(C->l[j], acor, zs[j][i]);
            K.z[j][id] = zn;
            if (j == q) znq = zn;
          }
        }
        if (raise) K.z[q + 1][id] = C->craise * acor;
        K.dprev[id] = acor;
        const double a = znq * w[i], b = (acor - dp) * w[i];
        szq = fma(a, a, szq);
        sdd = fma(b, b, sdd);
      }
    }
    red[0] = szq;
    red[1] = sdd;
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_accept(Cc, s); });
}

// Starting step, part 1: f(y0) into z[1] (scaled later by h), norms of y0, f0.
template <int NP>
__global__ void __launch_bounds__(kCellThreads) k_tpc_init1(BdfDev D) {
  __shared__ double s_y[NP * kCellThreads];
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  if (C->phase != PH_INIT1) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const long c = (long)blockIdx.x * kCellThreads + threadIdx.x;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells) {
    const double* kap = K.rates + Tpc<NP>::kidx(c, 0, K.R);
    double* ycol = s_y + threadIdx.x;
    double y[NP], f[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) y[i] = i < n ? K.z[0][Tpc<NP>::idx(c, i, n)] : 0.0;
    tpc_store_col<NP>(ycol, y);
    Tpc<NP>::rhs(K.net, kap, ycol, f);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < n) {
        K.z[1][Tpc<NP>::idx(c, i, n)] = f[i];
        const double w = 1.0 / (D.rtol * fabs(y[i]) + D.atol);
        s0 = fma(y[i] * w, y[i] * w, s0);
        s1 = fma(f[i] * w, f[i] * w, s1);
      }
    }
    red[0] = s0;
    red[1] = s1;
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_init1(Cc, s); });
}

template <int NP>
__global__ void __launch_bounds__(kCellThreads) k_tpc_init2(BdfDev D) {
  __shared__ double s_y[NP * kCellThreads];
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  if (C->phase != PH_INIT2) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const long c = (long)blockIdx.x * kCellThreads + threadIdx.x;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells) {
    const double* kap = K.rates + Tpc<NP>::kidx(c, 0, K.R);
    double* ycol = s_y + threadIdx.x;
    const double h0 = C->hnw_h0;
    double y1[NP], f0[NP], f1[NP], w[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const bool in = i < n;
      const long id = Tpc<NP>::idx(c, i, n);
      const double y0 = in ? K.z[0][id] : 0.0;
      f0[i] = in ? K.z[1][id] : 0.0;
      w[i] = in ? 1.0 / (D.rtol * fabs(y0) + D.atol) : 0.0;
      y1[i] = y0 + h0 * f0[i];
    }
    tpc_store_col<NP>(ycol, y1);
    Tpc<NP>::rhs(K.net, kap, ycol, f1);
    double s0 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double d = (f1[i] - f0[i]) * w[i];
      s0 = fma(d, d, s0);
    }
    red[0] = s0;
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_init2(Cc, s); });
}

// ===========================================================================
// Segment per cell
// ===========================================================================
template <int SEG>
struct Spc {
  static constexpr int CPB = kCellThreads / SEG;   // cells per block

  // lane i: f_i and row i of J at the segment's state in ys (LDS, SEG values)
  __device__ static void rhs_row(const NetDev& nd, const double* kap, const double* ys, int i,
                                 double& f) {
    f = 0.0;
    for (int k = 0; k < nd.R; ++k) {
      const int a = nd.ra[k], b = nd.rb[k];
      double r = kap[k];
      if (a >= 0) r *= ys[a];
      if (b >= 0) r *= ys[b];
      f = fma(nd.S[(long)k * nd.np + i], r, f);
    }
  }

  __device__ static void jac_row(const NetDev& nd, const double* kap, const double* ys, int i,
                                 double (&J)[SEG]) {
#pragma unroll
    for (int a = 0; a < SEG; ++a) {
      double acc = 0.0;
      if (a < nd.n) {
        const int e0 = nd.jst[a], e1 = nd.jst[a + 1];
        for (int e = e0; e < e1; ++e) {
          const int k = nd.jk[e], p = nd.jp[e];
          double g = kap[k] * nd.jm[e];
          if (p >= 0) g *= ys[p];
          acc = fma(nd.S[(long)k * nd.np + i], g, acc);
        }
      }
      J[a] = acc;
    }
  }
};

struct SpcShared {
  double ys[kCellThreads];
  double prow[kCellThreads];
  float prow32[kCellThreads];
  int wl[kCellThreads];
  int wl32[kCellThreads];
  double red[(kCellThreads / 64) * kRedVals];
};

// Solve M x = r for the segment's block; lane i holds row i of M and r_i.
template <int SEG, int LS>
__device__ __forceinline__ double spc_linsolve(double (&Mrow)[SEG], double r, int i, int n,
                                               int seg_base, SpcShared& sh, int sb, int max_it,
                                               int& info, int& sweeps, int& fallback) {
  sweeps = 0;
  fallback = 0;
  double x = 0.0;
  bool ok = false;
  if (LS == 1) {
    float L[SEG];
#pragma unroll
    for (int j = 0; j < SEG; ++j) L[j] = (float)Mrow[j];
    int pos32, piv32;
    const int inf32 = SpcLU<SEG, float>::factor(L, i, n, pos32, piv32, sh.prow32 + sb, sh.wl32 + sb);
    if (!inf32) {
      double rs = 0.0;
#pragma unroll
      for (int j = 0; j < SEG; ++j) rs += fabs(Mrow[j]);
      const double mnorm = seg_max<SEG>(rs);
      x = (double)SpcLU<SEG, float>::solve(L, i, seg_base, n, pos32, sh.wl32 + sb, (float)r);
      const double eps64 = 2.220446049250313e-16;
      double dprev = 0.0;
      for (int it = 0; it <= max_it; ++it) {
        double res = r;
#pragma unroll
        for (int j = 0; j < SEG; ++j) res = fma(-Mrow[j], __shfl(x, seg_base + j, 64), res);
        const double rn = seg_max<SEG>(fabs(res));
        const double xn = seg_max<SEG>(fabs(x));
        if (!(rn == rn) || !(xn == xn)) break;
        if (rn <= sqrt((double)n) * eps64 * mnorm * xn) {
          ok = true;
          break;
        }
        if (it == max_it) break;
        const double d =
            (double)SpcLU<SEG, float>::solve(L, i, seg_base, n, pos32, sh.wl32 + sb, (float)res);
        x += d;
        const double dn = seg_max<SEG>(fabs(d));
        sweeps = it + 1;
        if (it >= 1 && dn > 0.5 * dprev) break;
        dprev = dn;
      }
    }
    if (!ok) fallback = 1;
  }
  info = 0;
  if (!ok) {
    int pos, piv;
    info = SpcLU<SEG, double>::factor(Mrow, i, n, pos, piv, sh.prow + sb, sh.wl + sb);
    x = SpcLU<SEG, double>::solve(Mrow, i, seg_base, n, pos, sh.wl + sb, r);
  }
  return x;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Predictor for one segment-per-cell lane: returns z(0)[0] and z(0)[0] -
// l0 z(0)[1] of row i (Pascal triangle on the pending-scaled history).
template <int SEG>
__device__ __forceinline__ void spc_predict_row(const BdfDev& D, const Ctrl* C, SpcShared& sh,
                                                int sb, int i, bool act, bool row, long id,
                                                const double* kap, double& zp0, double& cv) {
  const ClassDev& K = D.k;
  const int q = C->q;
  double zs[kQmaxAll + 1];
#pragma unroll
  for (int j = 0; j <= kQmaxAll; ++j) zs[j] = (row && j <= q) ? K.z[j][id] * C->hs[j] : 0.0;
  if (C->restart) {
    sh.ys[threadIdx.x] = zs[0];
    wave_sync_lds();
    double f0 = 0.0;
    if (act) Spc<SEG>::rhs_row(K.net, kap, sh.ys + sb, i, f0);
    zs[1] = row ? C->h * f0 : 0.0;
    if (row) K.z[1][id] = zs[1];
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
    for (int j = kQmaxAll; j >= k; --j)
      if (k <= q && j <= q) zs[j - 1] = zs[j - 1] + zs[j];
  zp0 = zs[0];
  cv = zs[0] - C->l[0] * zs[1];
}

// Learned mode: predictor only, plus the MLP inputs [z(0)[0], log gamma]
// of every cell and the per-cell solver mode of the attempt.
template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_predict(BdfDev D) {
  __shared__ SpcShared sh;
  Ctrl* C = D.C;
  if (C->phase != PH_PREDICT) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const int i = threadIdx.x & (SEG - 1);
  const int sb = threadIdx.x & ~(SEG - 1);
  const long c = (long)blockIdx.x * Spc<SEG>::CPB + threadIdx.x / SEG;
  const bool act = c < K.ncells;
  const bool row = act && i < n;
  const long id = c * n + i;
  const double* kap = K.rates + (act ? c : 0) * (long)K.R;
  double zp0, cv;
  spc_predict_row<SEG>(D, C, sh, sb, i, act, row, id, kap, zp0, cv);
  if (row) {
    K.zp0[id] = zp0;
    K.cv[id] = cv;
    K.y[id] = zp0;
    K.xin[c * (n + 1) + i] = zp0;
  }
  if (act && i == 0) {
    K.xin[c * (n + 1) + n] = log(C->gamma);
    K.lpmode[c] = C->force_lu ? 0 : 2;
    K.dcprev[c] = 0.0;
  }
}

// Newton iteration for segment-per-cell classes.  FIRST = 1: the attempt's
// first iteration (with the predictor unless LS == 2, whose predictor ran
// in k_spc_predict).  LS: 0 FP64 LU, 1 FP32 LU + refinement, 2 learned
// approximate inverse with per-cell fallback to FP64 LU.
template <int SEG, int LS, int FIRST>
__global__ void __launch_bounds__(kCellThreads) k_spc_newton(BdfDev D, int mslot) {
  __shared__ SpcShared sh;
  Ctrl* C = D.C;
  const int phase = C->phase;
  if (FIRST ? phase != PH_PREDICT : (phase != PH_NEWTON || C->m != mslot)) return;
  const ClassDev& K = D.k;
  const NetDev& nd = K.net;
  const int n = K.n;
  const int lane = threadIdx.x & 63;
  const int i = lane & (SEG - 1);
  const int seg_base = lane & ~(SEG - 1);
  const int sb = threadIdx.x & ~(SEG - 1);
  const long c = (long)blockIdx.x * Spc<SEG>::CPB + threadIdx.x / SEG;
  const bool act = c < K.ncells;           // uniform over the segment
  const bool row = act && i < n;
  const long id = c * n + i;
  const double* kap = K.rates + (act ? c : 0) * (long)K.R;
  const double gamma = C->gamma;
  const int m = FIRST ? 0 : mslot;
  double y = 0.0, zp0 = 0.0, cv = 0.0, w = 0.0;
  if (FIRST && LS != 2) {
    spc_predict_row<SEG>(D, C, sh, sb, i, act, row, id, kap, zp0, cv);
    y = zp0;
    w = row ? 1.0 / (D.rtol * fabs(K.z[0][id]) + D.atol) : 0.0;
  } else if (row) {
    y = K.y[id];
    zp0 = K.zp0[id];
    cv = K.cv[id];
    w = 1.0 / (D.rtol * fabs(K.z[0][id]) + D.atol);
  }
  // f at the iterate
  __builtin_amdgcn_wave_barrier();
  sh.ys[threadIdx.x] = y;
  wave_sync_lds();
  double f = 0.0;
  if (act) Spc<SEG>::rhs_row(nd, kap, sh.ys + sb, i, f);
  const double r = row ? fma(gamma, f, cv - y) : 0.0;
  int mode = 0;                           // 0/4 exact LU, 2 learned, 3 switching
  if (LS == 2 && act) mode = K.lpmode[c];
  double del = 0.0;
  int info = 0, sweeps = 0, fb = 0;
  double lp_solves = 0.0, lp_fb = 0.0;
  bool use_lu = (LS != 2) || mode != 2;
  if (LS == 2 && mode == 2) {
    // correction = X r with the cell's approximate inverse (row i of X)
    __builtin_amdgcn_wave_barrier();
    sh.ys[threadIdx.x] = r;
    wave_sync_lds();
    if (row) {
      const float* Xr = K.X + c * (long)n * n + (long)i * n;
      double s = 0.0;
      for (int j = 0; j < n; ++j) s = fma((double)Xr[j], sh.ys[sb + j], s);
      del = s;
    }
    const double bad = seg_max<SEG>(row && !(fabs(del) <= 1.79e308) ? 1.0 : 0.0);
    lp_solves = 1.0;
    if (bad > 0.0) {
      mode = 3;
      use_lu = true;
    }
  }
  if (use_lu) {
    double Mrow[SEG];
    __builtin_amdgcn_wave_barrier();
    sh.ys[threadIdx.x] = zp0;
    wave_sync_lds();
    if (act) Spc<SEG>::jac_row(nd, kap, sh.ys + sb, i, Mrow);
    else
#pragma unroll
      for (int j = 0; j < SEG; ++j) Mrow[j] = 0.0;
#pragma unroll
    for (int j = 0; j < SEG; ++j) Mrow[j] = (i == j ? 1.0 : 0.0) - gamma * Mrow[j];
    if (!row)
#pragma unroll
      for (int j = 0; j < SEG; ++j) Mrow[j] = (i == j ? 1.0 : 0.0);
    del = spc_linsolve<SEG, LS == 1 ? 1 : 0>(Mrow, r, i, act ? n : 0, seg_base, sh, sb,
                                              K.refine_max_it, info, sweeps, fb);
    if (LS == 2 && mode == 3) {
      lp_fb = 1.0;
      mode = 4;
    }
  }
  if (LS == 2) {
    const double dc2 = seg_sum<SEG>(row ? (del * w) * (del * w) : 0.0);
    const double dc = sqrt(dc2 / (double)n);
    if (act) {
      if (mode == 2 && m >= 1 && dc > 0.9 * K.dcprev[c]) mode = 3;
      __builtin_amdgcn_wave_barrier();
      if (i == 0) {
        K.lpmode[c] = mode;
        K.dcprev[c] = dc;
      }
    }
  }
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (row) {
    y += del;
    K.y[id] = y;
    if (FIRST && LS != 2) {
      K.zp0[id] = zp0;
      K.cv[id] = cv;
    }
    const bool ng = D.nonneg && y < 0.0;
    const double a = del * w, b = ((ng ? 0.0 : y) - zp0) * w;
    red[0] = a * a;
    red[1] = b * b;
    red[5] = ng ? 1.0 : 0.0;
  }
  if (act && i == 0) {
    red[2] = info ? 1.0 : 0.0;
    red[3] = (double)sweeps;
    red[4] = (double)fb;
    red[6] = lp_solves;
    red[7] = lp_fb;
  }
  reduce_and_control(D, red, sh.red, [](Ctrl* Cc, const double* s) { after_newton(Cc, s); });
}

template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_accept(BdfDev D) {
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  if (C->phase != PH_ACCEPT) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const int i = threadIdx.x & (SEG - 1);
  const long c = (long)blockIdx.x * Spc<SEG>::CPB + threadIdx.x / SEG;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells && i < n) {
    const long id = c * n + i;
    const int q = C->q;
    const double l0 = C->l[0];
    double zs[kQmaxAll + 1];
#pragma unroll
    for (int j = 0; j <= kQmaxAll; ++j) zs[j] = j <= q ? K.z[j][id] * C->hs[j] : 0.0;
    const double w = 1.0 / (D.rtol * fabs(zs[0]) + D.atol);
#pragma unroll
    for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
      for (int j = kQmaxAll; j >= k; --j)
        if (k <= q && j <= q) zs[j - 1] = zs[j - 1] + zs[j];
    const double yv = K.y[id];
    const double yp = D.nonneg && yv < 0.0 ? 0.0 : yv;
    const double acor = (yp - zs[0]) / l0;
    const double dp = K.dprev[id];
    double znq = yp;
    K.z[0][id] = yp;   // z(0)[0] + l0 acor is the corrected solution itself
#pragma unroll
    for (int j = 1; j <= kQmaxAll; ++j) {
      if (j <= q) {
        const double zn = fma(C->l[j], acor, zs[j]);
        K.z[j][id] = zn;
        if (j == q) znq = zn;
      }
    }
    if (C->qwait == 1 && q < C->qmax) K.z[q + 1][id] = C->craise * acor;
    K.dprev[id] = acor;
    const double a = znq * w, b = (acor - dp) * w;
    red[0] = a * a;
    red[1] = b * b;
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_accept(Cc, s); });
}

template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_init1(BdfDev D) {
  __shared__ double s_y[kCellThreads];
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  if (C->phase != PH_INIT1) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const int i = threadIdx.x & (SEG - 1);
  const int sb = threadIdx.x & ~(SEG - 1);
  const long c = (long)blockIdx.x * Spc<SEG>::CPB + threadIdx.x / SEG;
  const bool act = c < K.ncells;
  const bool row = act && i < n;
  const long id = c * n + i;
  const double y = row ? K.z[0][id] : 0.0;
  s_y[threadIdx.x] = y;
  __syncthreads();
  double f = 0.0;
  if (act) Spc<SEG>::rhs_row(K.net, K.rates + c * (long)K.R, s_y + sb, i, f);
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (row) {
    K.z[1][id] = f;
    const double w = 1.0 / (D.rtol * fabs(y) + D.atol);
    red[0] = (y * w) * (y * w);
    red[1] = (f * w) * (f * w);
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_init1(Cc, s); });
}

template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_init2(BdfDev D) {
  __shared__ double s_y[kCellThreads];
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  if (C->phase != PH_INIT2) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const int i = threadIdx.x & (SEG - 1);
  const int sb = threadIdx.x & ~(SEG - 1);
  const long c = (long)blockIdx.x * Spc<SEG>::CPB + threadIdx.x / SEG;
  const bool act = c < K.ncells;
  const bool row = act && i < n;
  const long id = c * n + i;
  const double h0 = C->hnw_h0;
  const double y0 = row ? K.z[0][id] : 0.0;
  const double f0 = row ? K.z[1][id] : 0.0;
  s_y[threadIdx.x] = y0 + h0 * f0;
  __syncthreads();
  double f1 = 0.0;
  if (act) Spc<SEG>::rhs_row(K.net, K.rates + c * (long)K.R, s_y + sb, i, f1);
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (row) {
    const double w = 1.0 / (D.rtol * fabs(y0) + D.atol);
    const double d = (f1 - f0) * w;
    red[0] = d * d;
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_init2(Cc, s); });
}

}  // namespace bdfgpu
