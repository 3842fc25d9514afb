// Per-cell kernels of the grouped BDF step on gfx950.
//
// One step attempt is two launches over every class of cells:
//  * k_*_newton: predictor, evaluation of J at the predicted state, one
//    factorisation of M = I - gamma J per cell, then all maxcor Newton
//    iterations with that factorisation.  A cell's iterates depend only on
//    its own block, gamma and the predicted state, so the iterations need no
//    global synchronisation; each iteration's norms are reduced separately
//    and the controller replays the global convergence test on them
//    (after_newton_all).  The factors never leave registers, and the state
//    is read from HBM once per attempt instead of once per iteration.
//  * k_*_accept: history update from the iterate the controller picked,
//    with the norms for the order selection.
//
// Two mappings of cells to lanes:
//  * thread per cell (TPC, n <= 12): the block lives in one lane's
//    registers; vectors use a tiled layout (64 cells per tile, species-major
//    inside the tile) so that every load and store is a full 512-byte
//    wavefront access.  Reaction rates and the evaluation point sit in LDS
//    columns so that the network's species and reaction indices (uniform
//    over the wave, unknown at compile time) can address them.
//  * segment per cell (SPC, 12 < n <= 64): one lane per row of the block in
//    a segment of 16, 32 or 64 lanes (see spc.hpp); vectors are cell-major.
#pragma once

#include <hip/hip_runtime.h>

#include "bdf_ctrl.hpp"
#include "common.hpp"
#include "spc.hpp"

namespace bdfgpu {

// Shared network of one class of cells: r_k = kappa_k * y[ra_k] * y[rb_k] *
// y[rc_k] (missing reactant = -1; a third reactant only in thread-per-cell
// classes), f = S r, and for the Jacobian a list per column a of (reaction
// k, partner species p and p2 or -1, multiplicity m): dr_k/dy_a =
// m kappa_k y_p y_p2.
struct NetDev {
  int n, R, np;          // species, reactions, padded row length of S
  const double* S;       // [R][np] net stoichiometry mu - nu
  const int* ra;         // [R]
  const int* rb;         // [R]
  const int* rc;         // [R]
  const int* jst;        // [np + 1] start of each column's list
  const int* jk;         // [nent]
  const int* jp;         // [nent]
  const int* jp2;        // [nent]
  const double* jm;      // [nent]
};

struct ClassDev {
  long ncells;
  int n, R;
  double* z[kQmaxAll + 1];
  double* dprev;
  double* ys[kMaxCor];   // Newton iterate after iteration m
  double* zp0;           // learned mode: z(0)[0] from the predictor kernel
  double* cv;            // learned mode: z(0)[0] - l0 z(0)[1]
  const double* rates;
  NetDev net;
  long blk0;             // first block of this class in the phase reduction
  int refine_max_it;
  // learned preconditioner
  float* X;              // per cell n x n approximate inverse (row-major)
  double* xin;           // per cell MLP inputs [z(0)[0], log gamma]
  // lazy Newton matrix (thread-per-cell classes): per cell the NP x NP
  // factors (or inverse) and NP pivots, tiled like the state: entry k of
  // cell c at (c/64) 64 K + 64 k + c%64 with K = NP^2 (NP for pivots)
  double* lu;
  int* lpiv;
  // Newton-Krylov: weights, current iterate, Krylov basis V[j] = V + j vstride
  double* wt;
  double* yk;
  double* V;
  long vstride;
};

struct BdfDev {
  Ctrl* C;
  double* partials;      // [nblocks_total][kRedMax]
  unsigned int nblocks_total;
  double rtol, atol;
  int nonneg;
  int defer;             // deferred history update (host copy of Ctrl::fuse, for LDS sizing)
  int lazy;              // stored Newton-matrix factors (host copy of Ctrl::lazy)
  int vc;                // variable coefficients (host copy of Ctrl::vc)
  ClassDev k;
};

constexpr int kRedVals = 8;                        // init and accept kernels
constexpr int kRedNewton = kRedPerIter * kMaxCor;  // fused Newton kernels
constexpr int kRedMax = kRedNewton;
constexpr int kRedGroup = 256;                     // blocks per first-level group
constexpr int kCellThreads = 256;                  // SPC blocks
constexpr int kTpcThreads = 64;                    // TPC blocks (one wave)
constexpr int kAcceptChunk = 16;                  // species per chunk of the TPC history update

// Sum K values over the 64 lanes of a wave with K - 1 + (6 - log2 K)
// exchanges instead of 6 K: each exchange step halves the number of values
// a lane keeps.  On return lane l holds, in v[0], the total of value
// index red_index<K>(l).  The order of additions is fixed.
template <int K>
__device__ __forceinline__ int red_index(int lane) {
  int k = 0;
  int cnt = K, bit = 32;
  while (cnt > 1) {
    cnt >>= 1;
    if (lane & bit) k += cnt;
    bit >>= 1;
  }
  return k;
}

template <int K, int CNT, int BIT>
__device__ __forceinline__ void reduce_scatter_step(double (&v)[K], int lane) {
  if constexpr (BIT >= 1) {
    if constexpr (CNT > 1) {
      constexpr int HALF = CNT / 2;
      const bool upper = (lane & BIT) != 0;
#pragma unroll
      for (int i = 0; i < HALF; ++i) {
        const double send = upper ? v[i] : v[i + HALF];
        const double keep = upper ? v[i + HALF] : v[i];
        v[i] = keep + __shfl_xor(send, BIT, 64);
      }
      reduce_scatter_step<K, HALF, BIT / 2>(v, lane);
    } else {
      v[0] = v[0] + __shfl_xor(v[0], BIT, 64);
      reduce_scatter_step<K, 1, BIT / 2>(v, lane);
    }
  }
}

template <int K>
__device__ __forceinline__ void wave_reduce_scatter(double (&v)[K]) {
  reduce_scatter_step<K, K, 32>(v, threadIdx.x & 63);
}

// Block reduction of K partial sums, stored with plain stores at
// partials[gb][0..K) (gb: the block's index among all blocks of every
// launch of the phase).  The sums over blocks and the controller run in the
// two small kernels that follow the phase (k_reduce_groups, k_control):
// publishing a block's partials to the last block of the same launch would
// need a device-scope release fence per block, which writes back the L2's
// dirty lines and makes write-heavy kernels many times slower on gfx950;
// the kernel boundary publishes everything once.
template <int K>
__device__ __forceinline__ void block_partials(const BdfDev& D, unsigned int gb, double (&v)[K],
                                               double* sh) {
  static_assert(K <= kRedMax && (K & (K - 1)) == 0 && K <= 64, "reduction width");
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  wave_reduce_scatter<K>(v);
  // lanes 0 .. K-1 (stepping by 64 / K) hold distinct indices
  if ((lane & ((64 / K) - 1)) == 0) sh[wid * K + red_index<K>(lane)] = v[0];
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w * K + threadIdx.x];
    D.partials[(size_t)gb * kRedMax + threadIdx.x] = s;
  }
}

// First level: group g sums the partials of blocks [g*kRedGroup, ...) in a
// fixed order: thread b loads block b's K values (all loads in flight at
// once), then a fixed reduction tree over the block.
template <int K>
__global__ void __launch_bounds__(kRedGroup) k_reduce_groups(const Ctrl* C, int want,
                                                              const double* partials,
                                                              unsigned int nblocks,
                                                              double* gpartials) {
  if (C->phase != want) return;
  __shared__ double sh[(kRedGroup / 64) * K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned int b = blockIdx.x * kRedGroup + threadIdx.x;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = b < nblocks ? partials[(size_t)b * kRedMax + k] : 0.0;
  wave_reduce_scatter<K>(v);
  if ((lane & ((64 / K) - 1)) == 0) sh[wid * K + red_index<K>(lane)] = v[0];
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kRedGroup / 64; ++w) t += sh[w * K + threadIdx.x];
    gpartials[(size_t)blockIdx.x * kRedMax + threadIdx.x] = t;
  }
}

// Second level and the controller (one block of 256 threads; thread t adds
// groups t, t + 256, ... in order, then the fixed tree).  WHICH: 0 starting
// step part 1, 1 part 2, 2 fused Newton, 3 history update.
template <int K, int WHICH>
__global__ void __launch_bounds__(256) k_control(Ctrl* C, int want, const double* gpartials,
                                                  unsigned int ngroups) {
  if (C->phase != want) return;
  __shared__ double sh[4 * K];
  __shared__ double tot[K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (unsigned int b = threadIdx.x; b < ngroups; b += 256)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += gpartials[(size_t)b * kRedMax + k];
  wave_reduce_scatter<K>(v);
  if ((lane & ((64 / K) - 1)) == 0) sh[wid * K + red_index<K>(lane)] = v[0];
  __syncthreads();
  if (threadIdx.x < K) tot[threadIdx.x] = sh[threadIdx.x] + sh[K + threadIdx.x] +
                                          sh[2 * K + threadIdx.x] + sh[3 * K + threadIdx.x];
  // the controller is serial scalar code with many dependent accesses to the
  // control block: it runs on a copy in LDS, copied in and out by the block
  static_assert(sizeof(Ctrl) % sizeof(long) == 0, "Ctrl is copied in 8-byte words");
  constexpr int kWords = (int)(sizeof(Ctrl) / sizeof(long));
  __shared__ long cw[kWords];
  const long* cg = reinterpret_cast<const long*>(C);
  for (int t = threadIdx.x; t < kWords; t += blockDim.x) cw[t] = cg[t];
  __syncthreads();
  if (threadIdx.x == 0) {
    Ctrl* L = reinterpret_cast<Ctrl*>(cw);
    if (WHICH == 0) after_init1(L, tot);
    else if (WHICH == 1) after_init2(L, tot);
    else if (WHICH == 2) after_newton_all(L, tot);
    else after_accept(L, tot);
  }
  __syncthreads();
  long* cgw = reinterpret_cast<long*>(C);
  for (int t = threadIdx.x; t < kWords; t += blockDim.x) cgw[t] = cw[t];
}

// ===========================================================================
// Thread per cell
// ===========================================================================

// Dense LU of one lane's NP x NP block in registers, partial pivoting with
// the pivot rule of LAPACK getrf (first maximal |a_ik|).  Row exchanges
// touch only the trailing columns k..NP-1 and the multipliers stay where
// they were computed, as in LINPACK's factor/solve pair: the solve applies
// exchange k just before elimination step k, which performs the same
// floating-point operations on the same values as exchanging whole rows.
// This saves the exchanges of the multiplier columns, and an exchange is
// skipped altogether when no lane of the wave pivots on that row.  The
// diagonal holds reciprocal pivots.  The recursion over k keeps every
// register index a compile-time constant.
// Marks a wave-uniform branch whose body must not be turned into selects:
// row exchanges are rare, and executing their selects unconditionally (as
// the compiler otherwise does for short bodies) costs every wave the full
// exchange code of every row pair.
__device__ __forceinline__ void keep_branch() { asm volatile(""); }

template <int NP, typename T>
struct TpcLU {
  template <int K>
  __device__ static __forceinline__ void step(T (&A)[NP][NP], int (&piv)[NP], int& info) {
    if constexpr (K < NP) {
      int p = K;
      T amax = sabs(A[K][K]);
#pragma unroll
      for (int i = K + 1; i < NP; ++i) {
        const T v = sabs(A[i][K]);
        const bool gt = v > amax;
        amax = gt ? v : amax;
        p = gt ? i : p;
      }
      piv[K] = p;
#pragma unroll
      for (int i = K + 1; i < NP; ++i) {
        if (__any(p == i)) {
          keep_branch();
          const bool sw = (p == i);
#pragma unroll
          for (int j = K; j < NP; ++j) {
            const T t = A[K][j];
            A[K][j] = sw ? A[i][j] : t;
            A[i][j] = sw ? t : A[i][j];
          }
        }
      }
      const T d = A[K][K];
      const bool z = (d == T(0));
      if (z && !info) info = K + 1;
      // a zero pivot leaves the column as it is: rinv is then exactly 1
      const T rinv = T(1) / (z ? T(1) : d);
      A[K][K] = rinv;
#pragma unroll
      for (int i = K + 1; i < NP; ++i) {
        const T l = A[i][K] * rinv;
        A[i][K] = l;
#pragma unroll
        for (int j = K + 1; j < NP; ++j) A[i][j] = fma(-l, A[K][j], A[i][j]);
      }
      __builtin_amdgcn_sched_barrier(0);
      step<K + 1>(A, piv, info);
    }
  }

  __device__ static __forceinline__ int factor(T (&A)[NP][NP], int (&piv)[NP]) {
    int info = 0;
    step<0>(A, piv, info);
    return info;
  }

  __device__ static __forceinline__ void solve(const T (&A)[NP][NP], const int (&piv)[NP],
                                               T (&b)[NP]) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int p = piv[k];
#pragma unroll
      for (int i = k + 1; i < NP; ++i) {
        if (__any(p == i)) {
          keep_branch();
          const bool sw = (p == i);
          const T t = b[k];
          b[k] = sw ? b[i] : t;
          b[i] = sw ? t : b[i];
        }
      }
#pragma unroll
      for (int i = k + 1; i < NP; ++i) b[i] = fma(-A[i][k], b[k], b[i]);
    }
#pragma unroll
    for (int i = NP - 1; i >= 0; --i) {
#pragma unroll
      for (int j = i + 1; j < NP; ++j) b[i] = fma(-A[i][j], b[j], b[i]);
      b[i] = b[i] * A[i][i];
    }
  }
};

// Explicit inverse of one lane's NP x NP block (NP <= 4) by Gauss-Jordan
// elimination on [A | I]: at step K the first maximal |a_iK| (i >= K) is
// exchanged into row K (columns left of K are unit columns there, so only
// columns K.. of A and all of X move), row K is divided by its pivot and
// its multiples are subtracted from every other row.  X receives A^-1
// (X[i][j] = (A^-1)_ij); A is destroyed.  The explicit-inverse block solve
// of the paper's demonstration problem (Section 7).  Returns the first
// exactly-zero pivot (1-based) or 0; a zero pivot leaves that step's column
// as it is.
template <int NP>
struct TpcGJ {
  template <int K>
  __device__ static __forceinline__ void step(double (&A)[NP][NP], double (&X)[NP][NP], int& info) {
    if constexpr (K < NP) {
      int p = K;
      double amax = sabs(A[K][K]);
#pragma unroll
      for (int i = K + 1; i < NP; ++i) {
        const double v = sabs(A[i][K]);
        const bool gt = v > amax;
        amax = gt ? v : amax;
        p = gt ? i : p;
      }
#pragma unroll
      for (int i = K + 1; i < NP; ++i) {
        if (__any(p == i)) {
          keep_branch();
          const bool sw = (p == i);
#pragma unroll
          for (int j = K; j < NP; ++j) {
            const double t = A[K][j];
            A[K][j] = sw ? A[i][j] : t;
            A[i][j] = sw ? t : A[i][j];
          }
#pragma unroll
          for (int j = 0; j < NP; ++j) {
            const double t = X[K][j];
            X[K][j] = sw ? X[i][j] : t;
            X[i][j] = sw ? t : X[i][j];
          }
        }
      }
      const double d0 = A[K][K];
      const bool z = (d0 == 0.0);
      if (z && !info) info = K + 1;
      const double d = z ? 1.0 : d0;
#pragma unroll
      for (int j = K + 1; j < NP; ++j) A[K][j] = A[K][j] / d;
#pragma unroll
      for (int j = 0; j < NP; ++j) X[K][j] = X[K][j] / d;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (i == K) continue;
        const double f = A[i][K];
#pragma unroll
        for (int j = K + 1; j < NP; ++j) A[i][j] = fma(-f, A[K][j], A[i][j]);
#pragma unroll
        for (int j = 0; j < NP; ++j) X[i][j] = fma(-f, X[K][j], X[i][j]);
      }
      step<K + 1>(A, X, info);
    }
  }

  __device__ static __forceinline__ int invert(double (&A)[NP][NP], double (&X)[NP][NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = 0; j < NP; ++j) X[i][j] = i == j ? 1.0 : 0.0;
    int info = 0;
    step<0>(A, X, info);
    return info;
  }

  // out = X r, each row summed in column order
  __device__ static __forceinline__ void apply(const double (&X)[NP][NP], const double (&r)[NP],
                                               double (&out)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) s = fma(X[i][j], r[j], s);
      out[i] = s;
    }
  }
};

template <int NP, int TB = kTpcThreads>
struct Tpc {
  static constexpr int T = TB;            // LDS column stride (threads per block)
  // tiled index of species i of cell c (n species per cell)
  __device__ static __forceinline__ long idx(long c, int i, int n) {
    return (c >> 6) * 64L * n + (long)i * 64 + (c & 63);
  }
  __device__ static __forceinline__ long kidx(long c, int k, int R) {
    return (c >> 6) * 64L * R + (long)k * 64 + (c & 63);
  }

  // f at the state in ycol (LDS column, stride T); rates in kcol with
  // stride ks (an LDS column, or the tiled rates in global memory).
  __device__ static __forceinline__ void rhs(const NetDev& nd, const double* kcol, int ks, const double* ycol,
                             double (&f)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) f[i] = 0.0;
#pragma unroll 2
    for (int k = 0; k < nd.R; ++k) {
      const int a = nd.ra[k], b = nd.rb[k], c3 = nd.rc[k];
      double r = kcol[k * ks];
      if (a >= 0) r *= ycol[a * T];
      if (b >= 0) r *= ycol[b * T];
      if (c3 >= 0) r *= ycol[c3 * T];
      const double* Sk = nd.S + (long)k * nd.np;
#pragma unroll
      for (int i = 0; i < NP; ++i) f[i] = fma(Sk[i], r, f[i]);
    }
  }

  // Column a of J at the state in ycol (a is a compile-time constant after
  // unrolling at the call site).
  __device__ static __forceinline__ void jac_col(const NetDev& nd, const double* kcol, int ks,
                                                 const double* ycol, int a, double (&col)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) col[i] = 0.0;
    const int e0 = nd.jst[a], e1 = nd.jst[a + 1];
#pragma unroll 2
    for (int e = e0; e < e1; ++e) {
      const int k = nd.jk[e], p = nd.jp[e], p2 = nd.jp2[e];
      double g = kcol[k * ks] * nd.jm[e];
      if (p >= 0) g *= ycol[p * T];
      if (p2 >= 0) g *= ycol[p2 * T];
      const double* Sk = nd.S + (long)k * nd.np;
#pragma unroll
      for (int i = 0; i < NP; ++i) col[i] = fma(Sk[i], g, col[i]);
    }
  }

  // M = I - gamma J, assembled one column at a time; ROWSUM: also the row
  // sums of |M| (for the FP32 refinement's stopping test).
  template <typename TT, bool ROWSUM>
  __device__ static __forceinline__ void build_M(const NetDev& nd, const double* kcol, int ks,
                                                 const double* ycol, double gamma,
                                                 TT (&M)[NP][NP], double (&rowsum)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) rowsum[i] = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      double col[NP];
      jac_col(nd, kcol, ks, ycol, a, col);
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const double m = fma(-gamma, col[i], i == a ? 1.0 : 0.0);
        M[i][a] = (TT)m;
        if (ROWSUM) rowsum[i] += fabs(m);
      }
    }
  }

  // out = (I - gamma J) x without forming J: J x = sum_k S_k (grad r_k . x).
  // x must also be in the LDS column xcol (reactant lookups by index).
  __device__ static __forceinline__ void mvp(const NetDev& nd, const double* kcol, int ks, const double* ycol,
                             const double* xcol, double gamma, const double (&x)[NP],
                             double (&out)[NP]) {
    double jx[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) jx[i] = 0.0;
#pragma unroll 2
    for (int k = 0; k < nd.R; ++k) {
      const int a = nd.ra[k], b = nd.rb[k];
      if (a < 0) continue;
      const double kk = kcol[k * ks];
      double d;
      if (b < 0)
        d = kk * xcol[a * T];
      else
        d = kk * fma(xcol[a * T], ycol[b * T], ycol[a * T] * xcol[b * T]);
      const double* Sk = nd.S + (long)k * nd.np;
#pragma unroll
      for (int i = 0; i < NP; ++i) jx[i] = fma(Sk[i], d, jx[i]);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) out[i] = fma(-gamma, jx[i], x[i]);
  }

  __device__ static __forceinline__ void store_col(double* col, const double (&v)[NP]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) col[i * T] = v[i];
  }
};

// Network evaluation policy of the thread-per-cell Newton kernel: f, M =
// I - gamma J and (I - gamma J) x for the cell's network.  NetTables reads
// the network from the NetDev tables at run time (any network); a class can
// instead bring a policy generated for its own network (straight-line code
// with the species and reaction indices as constants), which must compute
// the same operations in the same order so that both give identical bits.
struct NetTables {
  template <int NP, int T>
  __device__ static __forceinline__ void rhs(const NetDev& nd, const double* kcol, int ks,
                                             const double* ycol, double (&f)[NP]) {
    Tpc<NP, T>::rhs(nd, kcol, ks, ycol, f);
  }
  template <int NP, int T, typename TT, bool ROWSUM>
  __device__ static __forceinline__ void build_M(const NetDev& nd, const double* kcol, int ks,
                                                 const double* ycol, double gamma,
                                                 TT (&M)[NP][NP], double (&rowsum)[NP]) {
    Tpc<NP, T>::template build_M<TT, ROWSUM>(nd, kcol, ks, ycol, gamma, M, rowsum);
  }
  template <int NP, int T>
  __device__ static __forceinline__ void mvp(const NetDev& nd, const double* kcol, int ks,
                                             const double* ycol, const double* xcol, double gamma,
                                             const double (&x)[NP], double (&out)[NP]) {
    Tpc<NP, T>::mvp(nd, kcol, ks, ycol, xcol, gamma, x, out);
  }
};

// History loads.  A load under a runtime condition compiles to a branch with
// a wait for that one load, which serialises the HBM round trips; so the
// order q selects a compile-time variant, padded species read a clamped
// (valid) address, and the results are selected afterwards.
template <int NP, int Q>
__device__ __forceinline__ void tpc_load_hist_q(const ClassDev& K, const Ctrl* C, long c, int n,
                                                double (&zs)[kQmaxAll + 1][NP]) {
#pragma unroll
  for (int j = 0; j <= kQmaxAll; ++j) {
    if (j <= Q) {
      const double hsj = C->hs[j];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const int ii = i < n ? i : n - 1;
        const double v = K.z[j][Tpc<NP>::idx(c, ii, n)];
        zs[j][i] = i < n ? v * hsj : 0.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NP; ++i) zs[j][i] = 0.0;
    }
  }
}

template <int NP>
__device__ __forceinline__ void tpc_load_hist(const ClassDev& K, const Ctrl* C, long c, int n,
                                              int q, double (&zs)[kQmaxAll + 1][NP]) {
  switch (q) {
    case 1: tpc_load_hist_q<NP, 1>(K, C, c, n, zs); break;
    case 2: tpc_load_hist_q<NP, 2>(K, C, c, n, zs); break;
    case 3: tpc_load_hist_q<NP, 3>(K, C, c, n, zs); break;
    case 4: tpc_load_hist_q<NP, 4>(K, C, c, n, zs); break;
    default: tpc_load_hist_q<NP, 5>(K, C, c, n, zs); break;
  }
}

// One species vector of a TPC cell, clamped loads (see above).
template <int NP>
__device__ __forceinline__ void tpc_load_vec(const double* v, long c, int n, double (&out)[NP]) {
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int ii = i < n ? i : n - 1;
    const double x = v[Tpc<NP>::idx(c, ii, n)];
    out[i] = i < n ? x : 0.0;
  }
}

// Deferred history update (Ctrl::fuse): the accepted previous attempt, of
// order UQ, left its corrected solution in iterate upd_m; z_new[j] =
// z(0)[j] + l_j acor is formed from the stored history (pending scale
// upd_hs) exactly as the separate history-update kernel forms it, written
// back (with z[UQ+1] = craise acor when that step could raise the order),
// and returned unscaled in zs (rows 0..UQ+1), with acor.  All loads go out
// in one batch.
template <int NP, int UQ, bool VC>
__device__ __forceinline__ void tpc_apply_update_q(const BdfDev& D, long c, int n,
                                                   double (&zs)[kQmaxAll + 1][NP],
                                                   double (&acor)[NP]) {
  const Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const double* ysrc = K.ys[C->upd_m];
  double yv[NP];
#pragma unroll
  for (int j = 0; j <= kQmaxAll; ++j) {
    if (j <= UQ) {
      const double hsj = C->upd_hs[j];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const int ii = i < n ? i : n - 1;
        const double v = K.z[j][Tpc<NP>::idx(c, ii, n)];
        zs[j][i] = i < n ? v * hsj : 0.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NP; ++i) zs[j][i] = 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int ii = i < n ? i : n - 1;
    const double v = ysrc[Tpc<NP>::idx(c, ii, n)];
    yv[i] = i < n ? v : 0.0;
  }
  const double l0 = C->upd_l[0];
  const bool raise = UQ < kQmaxAll && C->upd_raise;
  const double craise = C->upd_craise;
  double lj[UQ + 1];
#pragma unroll
  for (int j = 0; j <= UQ; ++j) lj[j] = C->upd_l[j];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
#pragma unroll
    for (int k = 1; k <= UQ; ++k)
#pragma unroll
      for (int j = UQ; j >= k; --j) zs[j - 1][i] = zs[j - 1][i] + zs[j][i];
    const double yp = D.nonneg && yv[i] < 0.0 ? 0.0 : yv[i];
    const double a = i < n ? (yp - zs[0][i]) / l0 : 0.0;
    acor[i] = a;
    zs[0][i] = i < n ? yp : 0.0;
#pragma unroll
    for (int j = 1; j <= UQ; ++j) zs[j][i] = i < n ? fma(lj[j], a, zs[j][i]) : 0.0;
    if constexpr (UQ < kQmaxAll) zs[UQ + 1][i] = (raise && i < n) ? craise * a : 0.0;
  }
  if constexpr (VC) {
    if (C->upd_dec) {   // variable coefficients: order lowered to UQ - 1
#pragma unroll
      for (int j = 1; j < UQ; ++j) {
        const double dj = C->upd_d[j];
#pragma unroll
        for (int i = 0; i < NP; ++i) zs[j][i] = fma(-dj, zs[UQ][i], zs[j][i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    if (i < n) {
      const long id = Tpc<NP>::idx(c, i, n);
#pragma unroll
      for (int j = 0; j <= UQ; ++j) K.z[j][id] = zs[j][i];
      if constexpr (UQ < kQmaxAll) {
        if (raise) K.z[UQ + 1][id] = zs[UQ + 1][i];
      }
    }
  }
}

// VC: variable coefficients (an order lowering may come with the update)
template <int NP, bool VC>
__device__ __forceinline__ void tpc_apply_update(const BdfDev& D, long c, int n,
                                                 double (&zs)[kQmaxAll + 1][NP],
                                                 double (&acor)[NP]) {
  switch (D.C->upd_q) {
    case 1: tpc_apply_update_q<NP, 1, VC>(D, c, n, zs, acor); break;
    case 2: tpc_apply_update_q<NP, 2, VC>(D, c, n, zs, acor); break;
    case 3: tpc_apply_update_q<NP, 3, VC>(D, c, n, zs, acor); break;
    case 4: tpc_apply_update_q<NP, 4, VC>(D, c, n, zs, acor); break;
    default: tpc_apply_update_q<NP, 5, VC>(D, c, n, zs, acor); break;
  }
}

// Lazy Newton matrix: a cell's factors (LU with pivots, or the inverse),
// tiled as described at ClassDev::lu; every load goes out before the first
// use.
template <int NP, int LS, class TF>
__device__ __forceinline__ void tpc_store_factors(const ClassDev& K, long c,
                                                  const TF (&A)[NP][NP], const int (&piv)[NP],
                                                  const double (&Xi)[LS == 3 ? NP : 1]
                                                                    [LS == 3 ? NP : 1]) {
  const long base = (c >> 6) * 64L * NP * NP + (c & 63);
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const long k = (long)(i * NP + j) * 64;
      if constexpr (LS == 3)
        K.lu[base + k] = Xi[i][j];
      else
        K.lu[base + k] = (double)A[i][j];
    }
  if constexpr (LS != 3) {
    const long pb = (c >> 6) * 64L * NP + (c & 63);
#pragma unroll
    for (int i = 0; i < NP; ++i) K.lpiv[pb + i * 64] = piv[i];
  }
}

template <int NP, int LS, class TF>
__device__ __forceinline__ void tpc_load_factors(const ClassDev& K, long c, TF (&A)[NP][NP],
                                                 int (&piv)[NP],
                                                 double (&Xi)[LS == 3 ? NP : 1]
                                                             [LS == 3 ? NP : 1]) {
  const long base = (c >> 6) * 64L * NP * NP + (c & 63);
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const long k = (long)(i * NP + j) * 64;
      if constexpr (LS == 3)
        Xi[i][j] = K.lu[base + k];
      else
        A[i][j] = (TF)K.lu[base + k];
    }
  if constexpr (LS != 3) {
    const long pb = (c >> 6) * 64L * NP + (c & 63);
#pragma unroll
    for (int i = 0; i < NP; ++i) piv[i] = K.lpiv[pb + i * 64];
  }
}

// Dynamic LDS of the TPC kernels (tb threads per block): the fused Newton
// kernel keeps NP columns for the evaluation point, NP for the refinement
// iterate (LS 1) and R for the rates, then the reduction scratch; the
// starting-step kernels NP columns and the scratch; the history update only
// the scratch.
// With the deferred history update (defer) two more columns follow the
// scratch: z(0)[q] and the previous step's correction, for the order
// selection's sums.
__host__ __device__ inline size_t tpc_newton_lds(int np, int R, int ls, int tb, bool defer = false) {
  return sizeof(double) *
         ((size_t)tb * (size_t)(np * (ls == 1 ? 2 : 1) + R + (defer ? 2 * np : 0)) +
          (size_t)(tb / 64) * kRedNewton);
}
__host__ __device__ inline size_t tpc_init_lds(int np, int tb) {
  return sizeof(double) * ((size_t)tb * np + (size_t)(tb / 64) * kRedVals);
}
__host__ __device__ inline size_t tpc_accept_lds(int tb) {
  return sizeof(double) * (size_t)(tb / 64) * kRedVals;
}

// Fused predictor + Newton iterations, thread per cell.  LS 0: FP64 LU kept
// in registers.  LS 1: FP32 LU kept in registers; each solve is refined with
// FP64 residuals from the matrix-free product (I - gamma J) x; a cell whose
// refinement fails switches to FP64 LU, re-assembled and factored at every
// later iteration of the attempt (rare: the FP64 factors would double the
// register footprint if they were kept beside the FP32 ones).
//
// RC: rates loaded in the same batch as the history (a kernel generated for
// one network passes its R); the rest follow in chunks of 8.  Every wave
// issues these loads before it waits on any of them, so their HBM round
// trips overlap; at one wave per SIMD a serial round trip costs the SIMD.
//
// FULL: the class's species fill the padded size (n == NP), so n is a
// compile-time constant: the padding selects and clamped addresses vanish
// and every tiled address is a constant offset from the cell's base.
// MODE: bit 0 lazy Newton matrix (stored factors), bit 1 variable
// coefficients; each combination is its own kernel so that the plain one
// carries none of their code.
template <int NP, int LS, int TB, class Net = NetTables, int RC = 24, bool FULL = false,
          int MODE = 0>
__device__ __forceinline__ void tpc_newton_body(const BdfDev& D, long blk, double* lds) {
  constexpr bool LZ = (MODE & 1) != 0, VC = (MODE & 2) != 0;
  static_assert(!LZ || LS == 0 || LS == 3, "stored factors: FP64 LU or the inverse");
  using TP = Tpc<NP, TB>;
  Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const NetDev& nd = K.net;
  const int n = FULL ? NP : K.n, R = K.R;
  const long c = blk * TB + threadIdx.x;
  const bool act = c < K.ncells;
  constexpr int F = LS == 1 ? 2 : 1;
  double* ycol = lds + threadIdx.x;                 // evaluation point
  double* xcol = lds + NP * TB + threadIdx.x;       // LS 1 iterate
  double* kcol = lds + F * NP * TB + threadIdx.x;   // rates
  double* s_red = lds + (size_t)(F * NP + R) * TB;
  double* qcol = s_red + (TB / 64) * kRedNewton + threadIdx.x;   // deferred update: z(0)[q]
  double* pcol = qcol + NP * TB;                                 // and the previous acor
  double red[kRedNewton];
#pragma unroll
  for (int k = 0; k < kRedNewton; ++k) red[k] = 0.0;
  if (act) {
    const int r0 = R < RC ? R : RC;   // rates in the first batch
    double rv[RC];
    if (r0 > 0) {
#pragma unroll
      for (int u = 0; u < RC; ++u) rv[u] = K.rates[TP::kidx(c, u < r0 ? u : r0 - 1, R)];
    }
    const double gamma = C->gamma;
    const double l0 = C->l[0];
    const int q = C->q;
    const int maxcor = C->maxcor;
    // this launch's iterations (a continuation starts at m0 > 0 from the
    // stored iterate of iteration m0 - 1)
    const int m0 = C->m0;
    const int m1 = m0 + C->kiters < maxcor ? m0 + C->kiters : maxcor;
    // deferred update: if accepted, this step selects the order (qwait == 1),
    // so each iteration also sums the selection's norms
    const bool sel = C->fuse && C->qwait == 1;
    const bool selp1 = sel && q < C->qmax && q < kQmaxAll;
    double zp0[NP], cv[NP], w[NP];
    {
      double zs[kQmaxAll + 1][NP];
      double acp[NP];
      if (C->fuse && C->upd) {
        tpc_apply_update<NP, VC>(D, c, n, zs, acp);
        // a continuation launch of this attempt reads acor_prev back for
        // the order selection's sums
        if (selp1) {
#pragma unroll
          for (int i = 0; i < NP; ++i)
            if (i < n) K.dprev[TP::idx(c, i, n)] = acp[i];
        }
#pragma unroll
        for (int j = 0; j <= kQmaxAll; ++j) {
          const double hsj = C->hs[j];
#pragma unroll
          for (int i = 0; i < NP; ++i) zs[j][i] = j <= q ? zs[j][i] * hsj : 0.0;
        }
      } else {
        tpc_load_hist<NP>(K, C, c, n, q, zs);
        if (selp1) tpc_load_vec<NP>(K.dprev, c, n, acp);
      }
#pragma unroll
      for (int u = 0; u < RC; ++u)
        if (u < r0) kcol[u * TB] = rv[u];
      for (int k0 = RC; k0 < R; k0 += 8) {   // 8 loads in flight per chunk
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = K.rates[TP::kidx(c, k0 + u < R ? k0 + u : R - 1, R)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (k0 + u < R) kcol[(k0 + u) * TB] = v[u];
      }
#pragma unroll
      for (int i = 0; i < NP; ++i) w[i] = i < n ? 1.0 / (D.rtol * fabs(zs[0][i]) + D.atol) : 0.0;
      if (C->restart) {
        double f0[NP];
        TP::store_col(ycol, zs[0]);
        Net::template rhs<NP, TB>(nd, kcol, TB, ycol, f0);
        const double h = C->h;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          zs[1][i] = h * f0[i];
          if (i < n) K.z[1][TP::idx(c, i, n)] = zs[1][i];
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
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        zp0[i] = zs[0][i];
        cv[i] = zs[0][i] - l0 * zs[1][i];
      }
      if (sel) {
        // z(0)[q] (the top row, which the predictor leaves unchanged)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double v = 0.0;
#pragma unroll
          for (int j = 1; j <= kQmaxAll; ++j) v = j == q ? zs[j][i] : v;
          qcol[i * TB] = v;
          if (selp1) pcol[i * TB] = acp[i];
        }
      }
    }
    TP::store_col(ycol, zp0);
    using TF = typename std::conditional<LS == 1, float, double>::type;
    TF A[NP][NP];
    int piv[NP];
    double rowsum[NP];
    constexpr int NX = LS == 3 ? NP : 1;   // LS 3: the block's explicit inverse
    double Xi[NX][NX];
    double mnorm = 0.0;
    int info = 0;
    // LZ (lazy Newton matrix): reuse the stored factors unless this attempt
    // sets up (uniform over the grid)
    const bool reuse = LZ && !C->setup;
    if (reuse) {
      tpc_load_factors<NP, LS>(K, c, A, piv, Xi);
    } else {
      Net::template build_M<NP, TB, TF, LS == 1>(nd, kcol, TB, ycol, gamma, A, rowsum);
#pragma unroll
      for (int i = 0; i < NP; ++i) mnorm = fmax(mnorm, rowsum[i]);
      if constexpr (LS == 3)
        info = TpcGJ<NP>::invert(A, Xi);
      else
        info = TpcLU<NP, TF>::factor(A, piv);
      if constexpr (LZ) tpc_store_factors<NP, LS>(K, c, A, piv, Xi);
    }
    const double dscale = C->dscale;
    bool fp64 = (LS == 1) && info != 0;   // LS 1: FP32 factor singular -> FP64 LU
    bool sing = (LS == 0 || LS == 3) && info != 0;
    red[4] = fp64 && m0 == 0 ? 1.0 : 0.0;   // counted with the first iteration
    double y[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) y[i] = zp0[i];
    if (m0 > 0) {
      const double* yp = K.ys[m0 - 1];
#pragma unroll
      for (int i = 0; i < NP; ++i)
        if (i < n) y[i] = yp[TP::idx(c, i, n)];
    }
    double* yev = LS == 1 ? xcol : ycol;   // LS 1 keeps z(0)[0] in ycol for J
    for (int m = m0; m < m1; ++m) {
      TP::store_col(yev, y);
      double r[NP];
      Net::template rhs<NP, TB>(nd, kcol, TB, yev, r);
#pragma unroll
      for (int i = 0; i < NP; ++i) r[i] = fma(gamma, r[i], cv[i] - y[i]);
      double del[NP];
      int sweeps = 0, fb = 0;
      if constexpr (LS == 0) {
#pragma unroll
        for (int i = 0; i < NP; ++i) del[i] = r[i];
        TpcLU<NP, TF>::solve(A, piv, del);
        if (reuse) {
#pragma unroll
          for (int i = 0; i < NP; ++i) del[i] = dscale * del[i];
        }
      } else if constexpr (LS == 3) {
        TpcGJ<NP>::apply(Xi, r, del);
        if (reuse) {
#pragma unroll
          for (int i = 0; i < NP; ++i) del[i] = dscale * del[i];
        }
      } else {
        bool ok = false;
        if (!fp64) {
          float v[NP];
#pragma unroll
          for (int i = 0; i < NP; ++i) v[i] = (float)r[i];
          TpcLU<NP, TF>::solve(A, piv, v);
#pragma unroll
          for (int i = 0; i < NP; ++i) del[i] = (double)v[i];
          const double eps64 = 2.220446049250313e-16;
          double dprv = 0.0;
          for (int it = 0; it <= K.refine_max_it; ++it) {
            TP::store_col(xcol, del);
            double mx[NP];
            Net::template mvp<NP, TB>(nd, kcol, TB, ycol, xcol, gamma, del, mx);
            double rn = 0.0, xn = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
              mx[i] = r[i] - mx[i];
              rn = fmax(rn, fabs(mx[i]));
              xn = fmax(xn, fabs(del[i]));
            }
            if (!(rn == rn) || !(xn == xn)) break;
            if (rn <= sqrt((double)NP) * eps64 * mnorm * xn) {
              ok = true;
              break;
            }
            if (it == K.refine_max_it) break;
#pragma unroll
            for (int i = 0; i < NP; ++i) v[i] = (float)mx[i];
            TpcLU<NP, TF>::solve(A, piv, v);
            double dn = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
              del[i] += (double)v[i];
              dn = fmax(dn, fabs((double)v[i]));
            }
            sweeps = it + 1;
            if (it >= 1 && dn > 0.5 * dprv) break;
            dprv = dn;
          }
          if (!ok) {
            fp64 = true;
            fb = 1;
          }
        }
        if (!ok) {
          double M[NP][NP], rs[NP];
          Net::template build_M<NP, TB, double, false>(nd, kcol, TB, ycol, gamma, M, rs);
          int pv[NP];
          if (TpcLU<NP, double>::factor(M, pv)) sing = true;
#pragma unroll
          for (int i = 0; i < NP; ++i) del[i] = r[i];
          TpcLU<NP, double>::solve(M, pv, del);
        }
      }
      double sd = 0.0, sa = 0.0, neg = 0.0, sq = 0.0, sp = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (i < n) {
          y[i] += del[i];
          K.ys[m][TP::idx(c, i, n)] = y[i];
          const bool ng = D.nonneg && y[i] < 0.0;
          neg += ng ? 1.0 : 0.0;
          const double a = del[i] * w[i], b = ((ng ? 0.0 : y[i]) - zp0[i]) * w[i];
          sd = fma(a, a, sd);
          sa = fma(b, b, sa);
        }
      }
      if (sel) {
        // the order selection's sums if this iterate is accepted: the new
        // z[q] = z(0)[q] + l_q acor and acor - acor_prev, as the history
        // update forms them
        const double lq = C->l[q];
        const double kap = VC ? C->kap : 1.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          if (i < n) {
            const double yp = D.nonneg && y[i] < 0.0 ? 0.0 : y[i];
            const double ac = (yp - zp0[i]) / l0;
            const double zq = fma(lq, ac, qcol[i * TB]) * w[i];
            sq = fma(zq, zq, sq);
            if (selp1) {
              double e;
              if constexpr (VC)
                e = (ac - kap * pcol[i * TB]) * w[i];
              else
                e = (ac - pcol[i * TB]) * w[i];
              sp = fma(e, e, sp);
            }
          }
        }
      }
      // m is not a compile-time constant: accumulate into every slot with
      // a select so that red[] stays in registers
#pragma unroll
      for (int mm = 0; mm < kMaxCor; ++mm) {
        const bool hit = (mm == m);
        red[kRedPerIter * mm + 0] += hit ? sd : 0.0;
        red[kRedPerIter * mm + 1] += hit ? sa : 0.0;
        red[kRedPerIter * mm + 2] += hit ? neg : 0.0;
        red[kRedPerIter * mm + 3] += hit ? (double)sweeps : 0.0;
        red[kRedPerIter * mm + 4] += hit ? (double)fb : 0.0;
        red[kRedPerIter * mm + 5] += hit ? sq : 0.0;
        red[kRedPerIter * mm + 6] += hit ? sp : 0.0;
      }
    }
    red[7] = sing ? 1.0 : 0.0;
  }
  block_partials<kRedNewton>(D, (unsigned int)(D.k.blk0 + blk), red, s_red);
}

template <int NP, int LS, bool FULL = false, int MODE = 0>
__global__ void __launch_bounds__(kTpcThreads) k_tpc_newton(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_PREDICT) return;
  tpc_newton_body<NP, LS, kTpcThreads, NetTables, 24, FULL, MODE>(D, blockIdx.x, lds);
}

// History update after an accepted attempt: z_new[j] = z(0)[j] + l_j acor
// from the iterate of iteration C->m.  acor_prev is read only when the
// order selection of this step needs it and written only when the next
// step's does (the step after one with qwait == 2 is the only one that
// reads it).
// History update of one cell at order Q (a compile-time constant, so the
// loads, Pascal sums and stores carry no run-time order tests), CH species
// at a time: each chunk's loads go out together, then its prediction,
// correction and stores.  Chunks of 2..5 species hold fewer registers and
// run more waves per SIMD, but at 10 species one chunk (all rows of the
// history in flight) measured as fast or slightly faster, so kAcceptChunk
// covers every thread-per-cell size.  Per element the operations, and the
// order of the two norm sums over species, do not depend on CH.
template <int NP, int TB, int Q, int CH>
__device__ __forceinline__ void tpc_accept_q(const BdfDev& D, long c, const double* ysrc, double& szq,
                                             double& sdd) {
  const Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const int n = K.n;
  const double l0 = C->l[0];
  const bool select = C->qwait == 1;
  const bool raise = Q < kQmaxAll && select && Q < C->qmax;
  const bool keep = C->qwait == 2;
  double hs[Q + 1], lj[Q + 1];
#pragma unroll
  for (int j = 0; j <= Q; ++j) {
    hs[j] = C->hs[j];
    lj[j] = C->l[j];
  }
  const double craise = C->craise;
#pragma unroll
  for (int i0 = 0; i0 < NP; i0 += CH) {
    double zs[Q + 1][CH], yv[CH], dp[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u;
      const int ii = i < n ? i : n - 1;
      const long id = Tpc<NP, TB>::idx(c, ii, n);
#pragma unroll
      for (int j = 0; j <= Q; ++j) {
        const double v = i < NP ? K.z[j][id] : 0.0;
        zs[j][u] = i < n ? v * hs[j] : 0.0;
      }
      const double y = i < NP ? ysrc[id] : 0.0;
      yv[u] = i < n ? y : 0.0;
    }
    if (raise) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int i = i0 + u;
        const double x = i < NP ? K.dprev[Tpc<NP, TB>::idx(c, i < n ? i : n - 1, n)] : 0.0;
        dp[u] = i < n ? x : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u;
      if (i < NP && i < n) {
        const double w = 1.0 / (D.rtol * fabs(zs[0][u]) + D.atol);
        // Pascal triangle: z(0)[j] = sum_{k >= j} C(k, j) z[k]
#pragma unroll
        for (int k = 1; k <= Q; ++k)
#pragma unroll
          for (int j = Q; j >= k; --j) zs[j - 1][u] = zs[j - 1][u] + zs[j][u];
        const long id = Tpc<NP, TB>::idx(c, i, n);
        const double yp = D.nonneg && yv[u] < 0.0 ? 0.0 : yv[u];
        const double acor = (yp - zs[0][u]) / l0;
        double znq = yp;
        K.z[0][id] = yp;   // z(0)[0] + l0 acor is the corrected solution itself
#pragma unroll
        for (int j = 1; j <= Q; ++j) {
          const double zn = fma(lj[j], acor, zs[j][u]);
          K.z[j][id] = zn;
          if (j == Q) znq = zn;
        }
        if constexpr (Q < kQmaxAll) {
          if (raise) {
            K.z[Q + 1][id] = craise * acor;
            const double b = (acor - dp[u]) * w;
            sdd = fma(b, b, sdd);
          }
        }
        if (keep) K.dprev[id] = acor;
        const double a = znq * w;
        szq = fma(a, a, szq);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int NP, int TB>
__device__ __forceinline__ void tpc_accept_body(const BdfDev& D, long blk, double* lds) {
  constexpr int CH = kAcceptChunk < NP ? kAcceptChunk : NP;
  double* s_red = lds;
  const ClassDev& K = D.k;
  const long c = blk * TB + threadIdx.x;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells) {
    double szq = 0.0, sdd = 0.0;
    // the iterate to accept (looked up here, once: indexing the pointer
    // array inside the order-specialised bodies made the compiler copy the
    // kernel arguments to scratch)
    const double* ysrc = K.ys[D.C->m];
    switch (D.C->q) {
      case 1: tpc_accept_q<NP, TB, 1, CH>(D, c, ysrc, szq, sdd); break;
      case 2: tpc_accept_q<NP, TB, 2, CH>(D, c, ysrc, szq, sdd); break;
      case 3: tpc_accept_q<NP, TB, 3, CH>(D, c, ysrc, szq, sdd); break;
      case 4: tpc_accept_q<NP, TB, 4, CH>(D, c, ysrc, szq, sdd); break;
      default: tpc_accept_q<NP, TB, 5, CH>(D, c, ysrc, szq, sdd); break;
    }
    red[0] = szq;
    red[1] = sdd;
  }
  block_partials<kRedVals>(D, (unsigned int)(D.k.blk0 + blk), red, s_red);
}

template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_tpc_accept(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_ACCEPT) return;
  tpc_accept_body<NP, kTpcThreads>(D, blockIdx.x, lds);
}

// Applies a pending deferred history update (end of a drive, before the
// host reads the state) and saves acor for the next order selection.
template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_tpc_flush(BdfDev D) {
  if (!D.C->upd) return;
  const long c = (long)blockIdx.x * kTpcThreads + threadIdx.x;
  const ClassDev& K = D.k;
  if (c >= K.ncells) return;
  const int n = K.n;
  double zs[kQmaxAll + 1][NP], acor[NP];
  if (n == NP)   // (rare: the end of a drive; one variant serves every mode)
    tpc_apply_update<NP, true>(D, c, NP, zs, acor);
  else
    tpc_apply_update<NP, true>(D, c, n, zs, acor);
#pragma unroll
  for (int i = 0; i < NP; ++i)
    if (i < n) K.dprev[Tpc<NP>::idx(c, i, n)] = acor[i];
}

// Starting step, part 1: f(y0) into z[1] (scaled later by h), norms of y0, f0.
template <int NP, int TB>
__device__ __forceinline__ void tpc_init1_body(const BdfDev& D, long blk, double* lds) {
  double* s_y = lds;
  double* s_red = lds + NP * TB;
  Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const int n = K.n;
  const long c = blk * TB + threadIdx.x;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells) {
    const double* kap = K.rates + Tpc<NP, TB>::kidx(c, 0, K.R);
    double* ycol = s_y + threadIdx.x;
    double y[NP], f[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) y[i] = i < n ? K.z[0][Tpc<NP, TB>::idx(c, i, n)] : 0.0;
    Tpc<NP, TB>::store_col(ycol, y);
    Tpc<NP, TB>::rhs(K.net, kap, 64, ycol, f);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < n) {
        K.z[1][Tpc<NP, TB>::idx(c, i, n)] = f[i];
        const double w = 1.0 / (D.rtol * fabs(y[i]) + D.atol);
        s0 = fma(y[i] * w, y[i] * w, s0);
        s1 = fma(f[i] * w, f[i] * w, s1);
      }
    }
    red[0] = s0;
    red[1] = s1;
  }
  block_partials<kRedVals>(D, (unsigned int)(D.k.blk0 + blk), red, s_red);
}

template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_tpc_init1(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_INIT1) return;
  tpc_init1_body<NP, kTpcThreads>(D, blockIdx.x, lds);
}

template <int NP, int TB>
__device__ __forceinline__ void tpc_init2_body(const BdfDev& D, long blk, double* lds) {
  double* s_y = lds;
  double* s_red = lds + NP * TB;
  Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const int n = K.n;
  const long c = blk * TB + threadIdx.x;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells) {
    const double* kap = K.rates + Tpc<NP, TB>::kidx(c, 0, K.R);
    double* ycol = s_y + threadIdx.x;
    const double h0 = C->hnw_h0;
    double y1[NP], f0[NP], f1[NP], w[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const bool in = i < n;
      const long id = Tpc<NP, TB>::idx(c, i, n);
      const double y0 = in ? K.z[0][id] : 0.0;
      f0[i] = in ? K.z[1][id] : 0.0;
      w[i] = in ? 1.0 / (D.rtol * fabs(y0) + D.atol) : 0.0;
      y1[i] = y0 + h0 * f0[i];
    }
    Tpc<NP, TB>::store_col(ycol, y1);
    Tpc<NP, TB>::rhs(K.net, kap, 64, ycol, f1);
    double s0 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double d = (f1[i] - f0[i]) * w[i];
      s0 = fma(d, d, s0);
    }
    red[0] = s0;
  }
  block_partials<kRedVals>(D, (unsigned int)(D.k.blk0 + blk), red, s_red);
}

template <int NP>
__global__ void __launch_bounds__(kTpcThreads) k_tpc_init2(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_INIT2) return;
  tpc_init2_body<NP, kTpcThreads>(D, blockIdx.x, lds);
}

}  // namespace bdfgpu
