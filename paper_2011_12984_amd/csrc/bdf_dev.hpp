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

constexpr int kRedVals = 6;
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

  // Solve M x = r.  LS 0: FP64 LU of M.  LS 1: FP32 LU + FP64 refinement
  // with FP64 fallback.  M is destroyed.  Returns info (singular).
  template <int LS>
  __device__ static int linsolve(double (&M)[NP][NP], const double (&r)[NP], double (&x)[NP],
                                 int max_it, int& sweeps, int& fallback) {
    sweeps = 0;
    fallback = 0;
    if (LS == 1) {
      float L[NP][NP];
      int pv[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = 0; j < NP; ++j) L[i][j] = (float)M[i][j];
      const int inf32 = factor<float>(L, pv);
      bool ok = false;
      if (!inf32) {
        double mnorm = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < NP; ++j) s += fabs(M[i][j]);
          mnorm = fmax(mnorm, s);
        }
        float v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = (float)r[i];
        solve<float>(L, pv, v);
#pragma unroll
        for (int i = 0; i < NP; ++i) x[i] = (double)v[i];
        const double eps64 = 2.220446049250313e-16;
        double dprev = 0.0;
        for (int it = 0; it <= max_it; ++it) {
          double res[NP];
          double rn = 0.0, xn = 0.0;
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            double s = r[i];
#pragma unroll
            for (int j = 0; j < NP; ++j) s = fma(-M[i][j], x[j], s);
            res[i] = s;
            rn = fmax(rn, fabs(s));
            xn = fmax(xn, fabs(x[i]));
          }
          if (!(rn == rn) || !(xn == xn)) break;
          if (rn <= sqrt((double)NP) * eps64 * mnorm * xn) {
            ok = true;
            break;
          }
          if (it == max_it) break;
#pragma unroll
          for (int i = 0; i < NP; ++i) v[i] = (float)res[i];
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
      if (ok) return 0;
      fallback = 1;
    }
    int pv64[NP];
    const int inf = factor<double>(M, pv64);
#pragma unroll
    for (int i = 0; i < NP; ++i) x[i] = r[i];
    solve<double>(M, pv64, x);
    return inf;
  }
};

template <int NP>
__device__ __forceinline__ void tpc_store_col(double* ycol, const double (&v)[NP]) {
#pragma unroll
  for (int i = 0; i < NP; ++i) ycol[i * kCellThreads] = v[i];
}

// Predictor + first Newton iteration (FIRST = 1) or Newton iteration
// mslot >= 1 (FIRST = 0); the two are separate kernels so that profiles
// attribute their time separately.
template <int NP, int LS, int FIRST>
__global__ void __launch_bounds__(kCellThreads) k_tpc_newton(BdfDev D, int mslot) {
  __shared__ double s_y[NP * kCellThreads];
  __shared__ double s_red[(kCellThreads / 64) * kRedVals];
  Ctrl* C = D.C;
  const int phase = C->phase;
  if (FIRST ? phase != PH_PREDICT : (phase != PH_NEWTON || C->m != mslot)) return;
  const ClassDev& K = D.k;
  const NetDev& nd = K.net;
  const int n = K.n;
  const long c = (long)blockIdx.x * kCellThreads + threadIdx.x;
  const bool act = c < K.ncells;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (act) {
    const double* kap = K.rates + Tpc<NP>::kidx(c, 0, K.R);
    double* ycol = s_y + threadIdx.x;
    const double gamma = C->gamma, l0 = C->l[0];
    const int q = C->q;
    double y[NP], zp0[NP], cv[NP], w[NP];
    if (FIRST) {
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
#pragma unroll
      for (int i = 0; i < NP; ++i) w[i] = i < n ? 1.0 / (D.rtol * fabs(zs[0][i]) + D.atol) : 0.0;
      // Pascal triangle: z(0)[j] = sum_{k >= j} C(k, j) z[k]
#pragma unroll
      for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
        for (int j = kQmaxAll; j >= k; --j)
          if (k <= q && j <= q)
#pragma unroll
            for (int i = 0; i < NP; ++i) zs[j - 1][i] = zs[j - 1][i] + zs[j][i];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        zp0[i] = zs[0][i];
        y[i] = zs[0][i];
        cv[i] = zs[0][i] - l0 * zs[1][i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const bool in = i < n;
        const long id = Tpc<NP>::idx(c, i, n);
        y[i] = in ? K.y[id] : 0.0;
        zp0[i] = in ? K.zp0[id] : 0.0;
        cv[i] = in ? K.cv[id] : 0.0;
        w[i] = in ? 1.0 / (D.rtol * fabs(K.z[0][id]) + D.atol) : 0.0;
      }
    }
    double M[NP][NP], f[NP];
    tpc_store_col<NP>(ycol, zp0);
    Tpc<NP>::jac(nd, kap, ycol, M);
    if (!FIRST) tpc_store_col<NP>(ycol, y);
    Tpc<NP>::rhs(nd, kap, ycol, f);
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = 0; j < NP; ++j) M[i][j] = (i == j ? 1.0 : 0.0) - gamma * M[i][j];
    double r[NP], del[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) r[i] = fma(gamma, f[i], cv[i] - y[i]);
    int sweeps, fb;
    const int info = Tpc<NP>::template linsolve<LS>(M, r, del, K.refine_max_it, sweeps, fb);
    double sd = 0.0, sa = 0.0, neg = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      y[i] += del[i];
      const bool ng = D.nonneg && y[i] < 0.0;
      neg += ng ? 1.0 : 0.0;
      const double yp = ng ? 0.0 : y[i];
      const double a = del[i] * w[i], b = (yp - zp0[i]) * w[i];
      sd = fma(a, a, sd);
      sa = fma(b, b, sa);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < n) {
        const long id = Tpc<NP>::idx(c, i, n);
        K.y[id] = y[i];
        if (FIRST) {
          K.zp0[id] = zp0[i];
          K.cv[id] = cv[i];
        }
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
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
  const double gamma = C->gamma, l0 = C->l[0];
  const int q = C->q;
  double y = 0.0, zp0 = 0.0, cv = 0.0, w = 0.0;
  if (FIRST) {
    double zs[kQmaxAll + 1];
#pragma unroll
    for (int j = 0; j <= kQmaxAll; ++j) zs[j] = (row && j <= q) ? K.z[j][id] * C->hs[j] : 0.0;
    if (C->restart) {
      sh.ys[threadIdx.x] = zs[0];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double f0 = 0.0;
      if (act) Spc<SEG>::rhs_row(nd, kap, sh.ys + sb, i, f0);
      zs[1] = row ? C->h * f0 : 0.0;
      if (row) K.z[1][id] = zs[1];
      __builtin_amdgcn_wave_barrier();
    }
    w = row ? 1.0 / (D.rtol * fabs(zs[0]) + D.atol) : 0.0;
#pragma unroll
    for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
      for (int j = kQmaxAll; j >= k; --j)
        if (k <= q && j <= q) zs[j - 1] = zs[j - 1] + zs[j];
    zp0 = zs[0];
    y = zs[0];
    cv = zs[0] - l0 * zs[1];
  } else if (row) {
    y = K.y[id];
    zp0 = K.zp0[id];
    cv = K.cv[id];
    w = 1.0 / (D.rtol * fabs(K.z[0][id]) + D.atol);
  }
  double Mrow[SEG];
  sh.ys[threadIdx.x] = zp0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (act) Spc<SEG>::jac_row(nd, kap, sh.ys + sb, i, Mrow);
  else
#pragma unroll
    for (int j = 0; j < SEG; ++j) Mrow[j] = 0.0;
  double f = 0.0;
  if (!FIRST) {
    __builtin_amdgcn_wave_barrier();
    sh.ys[threadIdx.x] = y;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (act) Spc<SEG>::rhs_row(nd, kap, sh.ys + sb, i, f);
#pragma unroll
  for (int j = 0; j < SEG; ++j) Mrow[j] = (i == j ? 1.0 : 0.0) - gamma * Mrow[j];
  if (!row) {
#pragma unroll
    for (int j = 0; j < SEG; ++j) Mrow[j] = (i == j ? 1.0 : 0.0);
    f = 0.0;
  }
  const double r = row ? fma(gamma, f, cv - y) : 0.0;
  int info, sweeps, fb;
  const double del = spc_linsolve<SEG, LS>(Mrow, r, i, act ? n : 0, seg_base, sh, sb,
                                           K.refine_max_it, info, sweeps, fb);
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (row) {
    y += del;
    K.y[id] = y;
    if (FIRST) {
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
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (row) {
    const double w = 1.0 / (D.rtol * fabs(y0) + D.atol);
    const double d = (f1 - f0) * w;
    red[0] = d * d;
  }
  reduce_and_control(D, red, s_red, [](Ctrl* Cc, const double* s) { after_init2(Cc, s); });
}

}  // namespace bdfgpu
