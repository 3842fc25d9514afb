// Newton-Krylov kernels (linsol GMRES), thread per cell.
//
// The Newton system M del = r of an attempt is solved over all unknowns at
// once by right-preconditioned GMRES scaled by the error weights w (the
// paper's global Newton with GMRES and the task-local block solver as
// preconditioner, Section 7; Krylov solvers, Section 5): GMRES on
// W M P^{-1} W^{-1} for W r, del = P^{-1} W^{-1} x.  The preconditioner P
// is the cells' LU factors of M at the last setup, stored per cell.  The
// host runs the Krylov iteration (the paper's host-side control with one
// synchronising reduction per inner product, Section 4.1) and these
// kernels do the vector work, each ending in per-block partial sums:
//
//   predict  z(0) = Pascal(z), cv = z(0)[0] - l0 z(0)[1], w, y = z(0)[0];
//            at a setup also M at z(0)[0] and its LU factors (P)
//   resid    v0 = w (gamma f(y) + cv - y);              sums |v0|^2
//   apply k  v_k *= 1/h (normalise), u = W M P^{-1} W^{-1} v_k -> V[k+1];
//            sums <u, v_j> for j <= k (classical Gram-Schmidt: all inner
//            products of the new vector in one pass, N_VDotProdMulti)
//   orth k   V[k+1] -= sum_j h_j v_j;                     sums |V[k+1]|^2
//   update   del = P^{-1} W^{-1} sum_j y_j v_j, y += del, iterate -> ys[m];
//            sums (del w)^2, ((y - z(0)[0]) w)^2 (y >= 0 projected when
//            constrained), negative components
//
// The operator applies M = I - gamma J with J at z(0)[0], formed per cell
// in registers.  Basis vectors live in one allocation, V[j] = V + j vstride,
// in the tiled layout of the state.
#include "bdf_dev.hpp"

namespace bdfgpu {

constexpr int kKryRed = 8;   // partial sums per block

template <int NP>
__device__ __forceinline__ double kld(const double* v, long c, int i, int n) {
  const int ii = i < n ? i : n - 1;
  const double x = v[Tpc<NP>::idx(c, ii, n)];
  return i < n ? x : 0.0;
}

template <int NP>
__device__ __forceinline__ void kst(double* v, long c, int n, const double (&x)[NP]) {
#pragma unroll
  for (int i = 0; i < NP; ++i)
    if (i < n) v[Tpc<NP>::idx(c, i, n)] = x[i];
}

// rates of cell c into the LDS columns kcol (stride kTpcThreads)
template <int NP>
__device__ __forceinline__ void kry_rates(const ClassDev& K, long c, double* kcol) {
  const int R = K.R;
  for (int k0 = 0; k0 < R; k0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = K.rates[Tpc<NP>::kidx(c, k0 + u < R ? k0 + u : R - 1, R)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < R) kcol[(k0 + u) * kTpcThreads] = v[u];
  }
}

// LDS: R rate columns, NP state columns, then the reduction scratch
__host__ inline size_t kry_lds(int np, int R) {
  return sizeof(double) * ((size_t)kTpcThreads * (size_t)(R + np) +
                           (size_t)(kTpcThreads / 64) * kKryRed);
}

template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_kry_predict(BdfDev D) {
  extern __shared__ double lds[];
  const Ctrl* C = D.C;
  if (C->phase != PH_PREDICT) return;
  const ClassDev& K = D.k;
  const int n = K.n, R = K.R;
  const long c = (long)blockIdx.x * kTpcThreads + threadIdx.x;
  double* kcol = lds + threadIdx.x;
  double* ycol = lds + (size_t)R * kTpcThreads + threadIdx.x;
  double* s_red = lds + (size_t)(R + NP) * kTpcThreads;
  double red[kKryRed];
#pragma unroll
  for (int k = 0; k < kKryRed; ++k) red[k] = 0.0;
  if (c < K.ncells) {
    kry_rates<NP>(K, c, kcol);
    const int q = C->q;
    double zs[kQmaxAll + 1][NP];
    tpc_load_hist<NP>(K, C, c, n, q, zs);
    double w[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) w[i] = i < n ? 1.0 / (D.rtol * fabs(zs[0][i]) + D.atol) : 0.0;
    if (C->restart) {   // z[1] = h f(z[0]) after a restart at order 1
      double f0[NP];
      Tpc<NP>::store_col(ycol, zs[0]);
      NetTables::rhs<NP, kTpcThreads>(K.net, kcol, kTpcThreads, ycol, f0);
#pragma unroll
      for (int i = 0; i < NP; ++i) zs[1][i] = C->h * f0[i];
      kst<NP>(K.z[1], c, n, zs[1]);
    }
#pragma unroll
    for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
      for (int j = kQmaxAll; j >= k; --j)
        if (k <= q && j <= q)
#pragma unroll
          for (int i = 0; i < NP; ++i) zs[j - 1][i] = zs[j - 1][i] + zs[j][i];
    const double l0 = C->l[0];
    double cv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) cv[i] = zs[0][i] - l0 * zs[1][i];
    kst<NP>(K.zp0, c, n, zs[0]);
    kst<NP>(K.cv, c, n, cv);
    kst<NP>(K.wt, c, n, w);
    kst<NP>(K.yk, c, n, zs[0]);
    if (C->setup) {   // the preconditioner: LU of M at z(0)[0]
      Tpc<NP>::store_col(ycol, zs[0]);
      double A[NP][NP], rowsum[NP];
      int piv[NP];
      double Xi[1][1];
      NetTables::build_M<NP, kTpcThreads, double, false>(K.net, kcol, kTpcThreads, ycol,
                                                         C->gamma, A, rowsum);
      const int info = TpcLU<NP, double>::factor(A, piv);
      tpc_store_factors<NP, 0>(K, c, A, piv, Xi);
      red[0] = info != 0 ? 1.0 : 0.0;
    }
  }
  block_partials<kKryRed>(D, (unsigned int)(K.blk0 + blockIdx.x), red, s_red);
}

template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_kry_resid(BdfDev D) {
  extern __shared__ double lds[];
  const Ctrl* C = D.C;
  if (C->phase != PH_PREDICT) return;
  const ClassDev& K = D.k;
  const int n = K.n, R = K.R;
  const long c = (long)blockIdx.x * kTpcThreads + threadIdx.x;
  double* kcol = lds + threadIdx.x;
  double* ycol = lds + (size_t)R * kTpcThreads + threadIdx.x;
  double* s_red = lds + (size_t)(R + NP) * kTpcThreads;
  double red[kKryRed];
#pragma unroll
  for (int k = 0; k < kKryRed; ++k) red[k] = 0.0;
  if (c < K.ncells) {
    kry_rates<NP>(K, c, kcol);
    double y[NP], cv[NP], w[NP], f[NP], v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      y[i] = kld<NP>(K.yk, c, i, n);
      cv[i] = kld<NP>(K.cv, c, i, n);
      w[i] = kld<NP>(K.wt, c, i, n);
    }
    Tpc<NP>::store_col(ycol, y);
    NetTables::rhs<NP, kTpcThreads>(K.net, kcol, kTpcThreads, ycol, f);
    const double gamma = C->gamma;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      v[i] = w[i] * fma(gamma, f[i], cv[i] - y[i]);
      s = fma(v[i], v[i], s);
    }
    kst<NP>(K.V, c, n, v);
    red[0] = s;
  }
  block_partials<kKryRed>(D, (unsigned int)(K.blk0 + blockIdx.x), red, s_red);
}

// u = W M P^{-1} W^{-1} v_k after normalising v_k by inv; inner products of
// u with v_0..v_k.  KK = k (a compile-time constant, so that the basis
// loads go out together).
template <int NP, int KK>
__device__ __forceinline__ void kry_apply_body(const BdfDev& D, double inv, double* lds) {
  const Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const int n = K.n, R = K.R;
  const long c = (long)blockIdx.x * kTpcThreads + threadIdx.x;
  const long vs = K.vstride;
  double* kcol = lds + threadIdx.x;
  double* ycol = lds + (size_t)R * kTpcThreads + threadIdx.x;
  double* s_red = lds + (size_t)(R + NP) * kTpcThreads;
  double red[kKryRed];
#pragma unroll
  for (int k = 0; k < kKryRed; ++k) red[k] = 0.0;
  if (c < K.ncells) {
    kry_rates<NP>(K, c, kcol);
    double vk[NP], w[NP], z0[NP], t[NP];
    double* Vk = K.V + KK * vs;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      vk[i] = kld<NP>(Vk, c, i, n) * inv;
      w[i] = kld<NP>(K.wt, c, i, n);
      z0[i] = kld<NP>(K.zp0, c, i, n);
    }
    kst<NP>(Vk, c, n, vk);
    double A[NP][NP], Xi[1][1];
    int piv[NP];
    tpc_load_factors<NP, 0>(K, c, A, piv, Xi);
#pragma unroll
    for (int i = 0; i < NP; ++i) t[i] = i < n ? vk[i] / w[i] : 0.0;
    TpcLU<NP, double>::solve(A, piv, t);
    // M = I - gamma J at z(0)[0]; u = W (M t), each row summed in column order
    Tpc<NP>::store_col(ycol, z0);
    double rowsum[NP];
    NetTables::build_M<NP, kTpcThreads, double, false>(K.net, kcol, kTpcThreads, ycol, C->gamma,
                                                       A, rowsum);
    double u[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) s = fma(A[i][j], t[j], s);
      u[i] = i < n ? w[i] * s : 0.0;
    }
    kst<NP>(K.V + (KK + 1) * vs, c, n, u);
    double vj[KK > 0 ? KK : 1][NP];
#pragma unroll
    for (int j = 0; j < KK; ++j)
#pragma unroll
      for (int i = 0; i < NP; ++i) vj[j][i] = kld<NP>(K.V + j * vs, c, i, n);
#pragma unroll
    for (int j = 0; j < KK; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) s = fma(u[i], vj[j][i], s);
      red[j] = s;
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) s = fma(u[i], vk[i], s);
    red[KK] = s;
  }
  block_partials<kKryRed>(D, (unsigned int)(K.blk0 + blockIdx.x), red, s_red);
}

template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_kry_apply(BdfDev D, int k, double inv) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_PREDICT) return;
  switch (k) {
    case 0: kry_apply_body<NP, 0>(D, inv, lds); break;
    case 1: kry_apply_body<NP, 1>(D, inv, lds); break;
    case 2: kry_apply_body<NP, 2>(D, inv, lds); break;
    case 3: kry_apply_body<NP, 3>(D, inv, lds); break;
    default: kry_apply_body<NP, 4>(D, inv, lds); break;
  }
}

struct KryCoef {
  double v[kKryMaxl + 1];
};

// V[k+1] -= sum_{j<=k} h_j v_j; |V[k+1]|^2
template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_kry_orth(BdfDev D, int k, KryCoef h) {
  __shared__ double s_red[(kTpcThreads / 64) * kKryRed];
  if (D.C->phase != PH_PREDICT) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const long c = (long)blockIdx.x * kTpcThreads + threadIdx.x;
  const long vs = K.vstride;
  double red[kKryRed];
#pragma unroll
  for (int j = 0; j < kKryRed; ++j) red[j] = 0.0;
  if (c < K.ncells) {
    double u[NP];
    double* Vn = K.V + (k + 1) * vs;
#pragma unroll
    for (int i = 0; i < NP; ++i) u[i] = kld<NP>(Vn, c, i, n);
#pragma unroll
    for (int j = 0; j <= kKryMaxl - 1; ++j) {
      if (j <= k) {
        const double hj = h.v[j];
#pragma unroll
        for (int i = 0; i < NP; ++i) u[i] = fma(-hj, kld<NP>(K.V + j * vs, c, i, n), u[i]);
      }
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) s = fma(u[i], u[i], s);
    kst<NP>(Vn, c, n, u);
    red[0] = s;
  }
  block_partials<kKryRed>(D, (unsigned int)(K.blk0 + blockIdx.x), red, s_red);
}

// del = P^{-1} W^{-1} sum_{j<kend} y_j v_j; y += del; the iterate of Newton
// iteration m; the Newton and error-test sums
template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_kry_update(BdfDev D, int m, int kend, KryCoef y) {
  __shared__ double s_red[(kTpcThreads / 64) * kKryRed];
  const Ctrl* C = D.C;
  if (C->phase != PH_PREDICT) return;
  const ClassDev& K = D.k;
  const int n = K.n;
  const long c = (long)blockIdx.x * kTpcThreads + threadIdx.x;
  const long vs = K.vstride;
  double red[kKryRed];
#pragma unroll
  for (int j = 0; j < kKryRed; ++j) red[j] = 0.0;
  if (c < K.ncells) {
    double x[NP], w[NP], yv[NP], z0[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      x[i] = 0.0;
      w[i] = kld<NP>(K.wt, c, i, n);
      yv[i] = kld<NP>(K.yk, c, i, n);
      z0[i] = kld<NP>(K.zp0, c, i, n);
    }
    if (kend > 0) {
#pragma unroll
      for (int j = 0; j < kKryMaxl; ++j) {
        if (j < kend) {
          const double yj = y.v[j];
#pragma unroll
          for (int i = 0; i < NP; ++i) x[i] = fma(yj, kld<NP>(K.V + j * vs, c, i, n), x[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < NP; ++i) x[i] = i < n ? x[i] / w[i] : 0.0;
      double A[NP][NP], Xi[1][1];
      int piv[NP];
      tpc_load_factors<NP, 0>(K, c, A, piv, Xi);
      TpcLU<NP, double>::solve(A, piv, x);
    }
    double sd = 0.0, sa = 0.0, neg = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < n) {
        yv[i] += x[i];
        const bool ng = D.nonneg && yv[i] < 0.0;
        neg += ng ? 1.0 : 0.0;
        const double a = x[i] * w[i], b = ((ng ? 0.0 : yv[i]) - z0[i]) * w[i];
        sd = fma(a, a, sd);
        sa = fma(b, b, sa);
      }
    }
    kst<NP>(K.yk, c, n, yv);
    kst<NP>(K.ys[m], c, n, yv);
    red[0] = sd;
    red[1] = sa;
    red[2] = neg;
  }
  block_partials<kKryRed>(D, (unsigned int)(K.blk0 + blockIdx.x), red, s_red);
}

// Sum of the first K partials of nb blocks, fixed order: thread t adds
// blocks t, t + 256, ...; then a tree over the threads.
__global__ void __launch_bounds__(256) k_kry_sum(const double* partials, unsigned int nb,
                                                 double* out) {
  __shared__ double sh[256][kKryRed];
  double v[kKryRed];
#pragma unroll
  for (int k = 0; k < kKryRed; ++k) v[k] = 0.0;
  for (unsigned int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
    for (int k = 0; k < kKryRed; ++k) v[k] += partials[(size_t)b * kRedMax + k];
#pragma unroll
  for (int k = 0; k < kKryRed; ++k) sh[threadIdx.x][k] = v[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int k = 0; k < kKryRed; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x < kKryRed) out[threadIdx.x] = sh[0][threadIdx.x];
}

// The controller's Newton decision on the sums the host assembled.
__global__ void k_kry_control(Ctrl* C, const double* sums, long liters) {
  if (C->phase != PH_PREDICT) return;
  C->nliters += liters;
  after_newton_all(C, sums);
}

template <int NP>
static void kry_go(int which, const BdfDev& D, unsigned int grid, hipStream_t s, int k,
                   double a, const double* coef) {
  const size_t lds = kry_lds(NP, D.k.R);
  KryCoef h;
  for (int j = 0; j <= kKryMaxl; ++j) h.v[j] = coef ? coef[j] : 0.0;
  switch (which) {
    case 0: hipLaunchKernelGGL(k_kry_predict<NP>, dim3(grid), dim3(kTpcThreads), lds, s, D); break;
    case 1: hipLaunchKernelGGL(k_kry_resid<NP>, dim3(grid), dim3(kTpcThreads), lds, s, D); break;
    case 2:
      hipLaunchKernelGGL(k_kry_apply<NP>, dim3(grid), dim3(kTpcThreads), lds, s, D, k, a);
      break;
    case 3: hipLaunchKernelGGL(k_kry_orth<NP>, dim3(grid), dim3(kTpcThreads), 0, s, D, k, h); break;
    default:
      hipLaunchKernelGGL(k_kry_update<NP>, dim3(grid), dim3(kTpcThreads), 0, s, D, k, (int)a, h);
      break;
  }
}

// which: 0 predict, 1 resid, 2 apply (k, a = 1/norm), 3 orth (k, coef =
// h), 4 update (k = Newton iteration, a = basis size, coef = y)
void launch_kry(int np, int which, const BdfDev& D, unsigned int grid, hipStream_t s, int k,
                double a, const double* coef) {
  switch (np) {
    case 3: kry_go<3>(which, D, grid, s, k, a, coef); break;
    case 4: kry_go<4>(which, D, grid, s, k, a, coef); break;
    case 6: kry_go<6>(which, D, grid, s, k, a, coef); break;
    case 8: kry_go<8>(which, D, grid, s, k, a, coef); break;
    case 10: kry_go<10>(which, D, grid, s, k, a, coef); break;
    default: kry_go<12>(which, D, grid, s, k, a, coef); break;
  }
}

void launch_kry_sum(const double* partials, unsigned int nb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_kry_sum, dim3(1), dim3(256), 0, s, partials, nb, out);
}

void launch_kry_control(Ctrl* C, const double* sums, long liters, hipStream_t s) {
  hipLaunchKernelGGL(k_kry_control, dim3(1), dim3(1), 0, s, C, sums, liters);
}

}  // namespace bdfgpu
