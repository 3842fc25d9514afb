// Segment-per-cell step kernels: one block of 13..64 species (or, with
// map_small, any size) per segment of SEG lanes, one row of the block per
// lane (the row-distributed LU of spc.hpp).  Thread-per-cell kernels, the
// controller and the shared device structures are in bdf_dev.hpp.
#pragma once

#include "bdf_dev.hpp"

namespace bdfgpu {

// ===========================================================================
// Segment per cell
// ===========================================================================
// The network tables through the constant address space: they are not
// written while a kernel runs, and every lane of a wave reads the same entry,
// so the loads go through the scalar cache (read only) instead of one vector
// load per entry with its full memory latency in the reaction loops.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* ro(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// Reactions of a segment class rounded up to the group of rhs_row.
__host__ __device__ inline int spc_rpad(int R) { return R > 0 ? (R + 7) / 8 * 8 : 8; }

template <int SEG>
struct Spc {
  static constexpr int CPB = kCellThreads / SEG;   // cells per block

  // lane i: f_i at the segment's state in ys (LDS, SEG values); kap: the
  // cell's rates, St: the stoichiometry staged in LDS as St[k * SEG + i]
  // (FP32 holds the small integer entries exactly), both zero-padded to R
  // rounded up to 8 (spc_stage), with the reactant tables padded alike
  // (index -1).  Reactions go in groups of 8 whose reactant indices are
  // loaded together (scalar loads, then one wait); an absent reactant is
  // selected out, not branched over.
  __device__ static __forceinline__ void rhs_row(const NetDev& nd, const double* kap,
                                                 const float* St, const double* ys, int i,
                                                 double& f) {
    const auto* ra = ro(nd.ra);
    const auto* rb = ro(nd.rb);
    const int R = nd.R;
    double acc = 0.0;
    for (int k0 = 0; k0 < R; k0 += 8) {
      int a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = ra[k0 + u];
        b[u] = rb[k0 + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double ya = ys[a[u] < 0 ? 0 : a[u]];
        const double yb = ys[b[u] < 0 ? 0 : b[u]];
        double r = kap[k0 + u];
        r = a[u] < 0 ? r : r * ya;
        r = b[u] < 0 ? r : r * yb;
        acc = fma((double)St[(k0 + u) * SEG + i], r, acc);
      }
    }
    f = acc;
  }

  // Row i of J: column a sums its table entries in groups of 4 (each
  // column's list is padded to a multiple of 4 with zero-multiplicity
  // entries), loaded together as rhs_row does for the reactions.
  template <int NC>
  __device__ static __forceinline__ void jac_row(const NetDev& nd, const double* kap,
                                                 const float* St, const double* ys, int i,
                                                 double (&J)[NC]) {
    jac_cols<NC>(nd, kap, St, ys, i, [&](int a, double v) { J[a] = v; });
  }

  // The same, handing each entry J_ia to put(a, J_ia) as it is formed (a
  // compile-time index once the column loop is unrolled), so that a caller
  // can convert the row without holding it in FP64.
  template <int NC, typename F>
  __device__ static __forceinline__ void jac_cols(const NetDev& nd, const double* kap,
                                                  const float* St, const double* ys, int i,
                                                  F&& put) {
    const auto* jst = ro(nd.jst);
    const auto* jk = ro(nd.jk);
    const auto* jp = ro(nd.jp);
    const auto* jm = ro(nd.jm);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double acc = 0.0;
      if (a < nd.n) {
        const int e0 = jst[a], e1 = jst[a + 1];
        for (int e = e0; e < e1; e += 4) {
          int k[4], p[4];
          double m[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            k[u] = jk[e + u];
            p[u] = jp[e + u];
            m[u] = jm[e + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double yp = ys[p[u] < 0 ? 0 : p[u]];
            double g = kap[k[u]] * m[u];
            g = p[u] < 0 ? g : g * yp;
            acc = fma((double)St[k[u] * SEG + i], g, acc);
          }
        }
      }
      put(a, acc);
    }
  }

  // Lane i: (J x)_i without the matrix, J at the state whose values ys holds
  // and x in xs (LDS, SEG values each).  Each reaction's derivative along x,
  // kappa (x_a y_b + y_a x_b) (an absent reactant contributes a factor 1 and
  // no derivative), is formed once, the segment's lanes taking reactions i,
  // i + SEG, ..., and kept in g (LDS, R rounded up to 8 values for this
  // segment); then every row sums its stoichiometry against them in reaction
  // order, as rhs_row does against the rates.
  __device__ static __forceinline__ double jx_row(const NetDev& nd, const double* kap,
                                                  const float* St, const double* ys,
                                                  const double* xs, double* g, int i) {
    const auto* ra = ro(nd.ra);
    const auto* rb = ro(nd.rb);
    const int R = nd.R, Rp = spc_rpad(R);
    __builtin_amdgcn_wave_barrier();
    for (int k = i; k < Rp; k += SEG) {
      const int a = k < R ? ra[k] : -1;
      const int b = k < R ? rb[k] : -1;
      const double xa = a < 0 ? 0.0 : xs[a], ya = a < 0 ? 1.0 : ys[a];
      const double xb = b < 0 ? 0.0 : xs[b], yb = b < 0 ? 1.0 : ys[b];
      g[k] = kap[k] * fma(xa, yb, ya * xb);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double acc = 0.0;
    for (int k0 = 0; k0 < R; k0 += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fma((double)St[(k0 + u) * SEG + i], g[k0 + u], acc);
    }
    return acc;
  }
};

struct SpcShared {
  double ys[kCellThreads];
  double prow[kCellThreads];
  float prow32[kCellThreads];
  int wl[kCellThreads];
  int wl32[kCellThreads];
  double red[(kCellThreads / 64) * kRedNewton];
  double wsum[(kCellThreads / 64) * kRedNewton];   // per-wave Newton sums
};

// v summed over the wave (every lane gets the same bits) and added by lane 0
// to *s; all 64 lanes must be active.
__device__ __forceinline__ void wave_add(double v, double* s) {
  v += lane_pair_t<0>(v);
  v += lane_pair_t<1>(v);
  v += lane_pair_t<2>(v);
  v += lane_pair_t<3>(v);
  v += lane_pair_t<4>(v);
  v += lane_pair_t<5>(v);
  if ((threadIdx.x & 63) == 0) *s += v;
}

// Dynamic LDS of the SPC kernels: the shared scratch, then the rates of the
// block's cells (CPB x Rp, FP64), then the stoichiometry (Rp x SEG; its
// entries are small integers, exact in FP32), Rp = R rounded up to 8 with
// zero rates and stoichiometry past R, then the reaction derivatives of the
// matrix-free Jacobian products (CPB x Rp, FP64).
__host__ __device__ inline size_t spc_lds_bytes(int seg, int R) {
  const size_t r = (size_t)spc_rpad(R);
  return sizeof(SpcShared) + 2 * sizeof(double) * (size_t)(kCellThreads / seg) * r +
         sizeof(float) * r * seg;
}

// This segment's Rp values of the derivative area (after the stoichiometry).
template <int SEG>
__device__ __forceinline__ double* spc_gk(const float* St, int R, int cb) {
  const int Rp = spc_rpad(R);
  return reinterpret_cast<double*>(const_cast<float*>(St) + (size_t)Rp * SEG) + (size_t)cb * Rp;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Carve the dynamic LDS and stage the rates of the block's cells (cell c at
// lk + c Rp, zero past R) and the class stoichiometry (zero rows past R).
template <int SEG>
__device__ __forceinline__ void spc_stage(const ClassDev& K, long blk, double* lds,
                                          SpcShared*& sh, double*& lk, float*& St) {
  sh = reinterpret_cast<SpcShared*>(lds);
  lk = lds + sizeof(SpcShared) / sizeof(double);
  const int R = K.R, Rp = spc_rpad(R);
  St = reinterpret_cast<float*>(lk + (size_t)Spc<SEG>::CPB * Rp);
  const long c0 = blk * Spc<SEG>::CPB;
  const long nc = K.ncells - c0 < Spc<SEG>::CPB ? K.ncells - c0 : Spc<SEG>::CPB;
  for (int t = threadIdx.x; t < Spc<SEG>::CPB * Rp; t += blockDim.x) {
    const int cl = t / Rp, k = t - cl * Rp;
    lk[t] = (cl < nc && k < R) ? K.rates[(c0 + cl) * R + k] : 0.0;
  }
  const int np = K.net.np;
  for (int t = threadIdx.x; t < Rp * SEG; t += blockDim.x) {
    const int k = t / SEG, i = t - k * SEG;
    St[t] = (k < R && i < np) ? (float)K.net.S[(long)k * np + i] : 0.0f;
  }
  __syncthreads();
}

// History of one SPC lane: clamped index for padding lanes, compile-time
// order (see the TPC history loads).
template <int Q>
__device__ __forceinline__ void spc_load_hist_q(const ClassDev& K, const Ctrl* C, long ids,
                                                bool row, double (&zs)[kQmaxAll + 1]) {
#pragma unroll
  for (int j = 0; j <= kQmaxAll; ++j) {
    if (j <= Q) {
      const double v = K.z[j][ids];
      zs[j] = row ? v * C->hs[j] : 0.0;
    } else {
      zs[j] = 0.0;
    }
  }
}

__device__ __forceinline__ void spc_load_hist(const ClassDev& K, const Ctrl* C, long ids, bool row,
                                              int q, double (&zs)[kQmaxAll + 1]) {
  switch (q) {
    case 1: spc_load_hist_q<1>(K, C, ids, row, zs); break;
    case 2: spc_load_hist_q<2>(K, C, ids, row, zs); break;
    case 3: spc_load_hist_q<3>(K, C, ids, row, zs); break;
    case 4: spc_load_hist_q<4>(K, C, ids, row, zs); break;
    default: spc_load_hist_q<5>(K, C, ids, row, zs); break;
  }
}

// Predictor for one segment-per-cell lane: z(0)[0] and z(0)[0] - l0 z(0)[1]
// of row i (Pascal triangle on the pending-scaled history), and the error
// weight from z[0].
template <int SEG>
__device__ __forceinline__ void spc_predict_row(const BdfDev& D, const Ctrl* C, SpcShared& sh,
                                                int sb, int i, bool act, bool row, long id,
                                                const double* kap, const float* St,
                                                double& zp0, double& cv, double& w) {
  const ClassDev& K = D.k;
  const int q = C->q;
  double zs[kQmaxAll + 1];
  spc_load_hist(K, C, row ? id : 0, row, q, zs);
  w = row ? 1.0 / (D.rtol * fabs(zs[0]) + D.atol) : 0.0;
  if (C->restart) {
    __builtin_amdgcn_wave_barrier();
    sh.ys[threadIdx.x] = zs[0];
    wave_sync_lds();
    double f0 = 0.0;
    if (act) Spc<SEG>::rhs_row(K.net, kap, St, sh.ys + sb, i, f0);
    zs[1] = row ? C->h * f0 : 0.0;
    if (row) K.z[1][id] = zs[1];
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
// of every cell.
template <int SEG>
__device__ __forceinline__ void spc_predict_body(const BdfDev& D, long blk, double* lds) {
  Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const int n = K.n;
  const int i = threadIdx.x & (SEG - 1);
  const int sb = threadIdx.x & ~(SEG - 1);
  const int cb = threadIdx.x / SEG;
  const long c = blk * Spc<SEG>::CPB + cb;
  const bool act = c < K.ncells;
  const bool row = act && i < n;
  const long id = c * n + i;
  SpcShared* shp;
  double* lk;
  float* St;
  spc_stage<SEG>(K, blk, lds, shp, lk, St);
  const double* kap = lk + cb * spc_rpad(K.R);
  double zp0, cv, w;
  spc_predict_row<SEG>(D, C, *shp, sb, i, act, row, id, kap, St, zp0, cv, w);
  if (row) {
    K.zp0[id] = zp0;
    K.cv[id] = cv;
    K.xin[c * (n + 1) + i] = zp0;
  }
  if (act && i == 0) K.xin[c * (n + 1) + n] = log(C->gamma);
}

template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_predict(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_PREDICT) return;
  spc_predict_body<SEG>(D, blockIdx.x, lds);
}

// Lazy Newton matrix on segment classes: per cell c, lane i's row as the
// factorisation left it (row i of L\U for LU; for Gauss-Jordan the inverse
// row that lane holds) in column order, and its position in the permuted
// matrix, at K.lu[c NC^2 + j NC + i] (column j of the lane-held rows
// contiguous, so each column is one coalesced access per segment) and
// K.lpiv[c NC + i].  Only the lanes holding rows (i < NC) store or load.
template <int SEG, int NC>
__device__ __forceinline__ void spc_store_factors(const ClassDev& K, long c, int i, bool act,
                                                  const double (&Mrow)[NC], int pos) {
  if (!act || i >= NC) return;
  double* base = K.lu + c * (long)(NC * NC) + i;
#pragma unroll
  for (int j = 0; j < NC; ++j) base[j * NC] = Mrow[j];
  K.lpiv[c * NC + i] = pos;
}

// Lazy Gauss-Jordan inverse: lane i's row from SpcGJ::invert (the inverse
// row of unknown pos, columns in position order) stored as the plain
// inverse, X[pos][wl[j]] at K.lu[c NC^2 + wl[j] NC + pos], so that the reuse
// kernel loads row i of X in natural order like spc_load_factors.
template <int SEG, int NC>
__device__ __forceinline__ void spc_store_inverse(const ClassDev& K, long c, int i, bool act,
                                                  const double (&S)[NC], int pos, const int* wl) {
  if (!act || i >= NC) return;
  double* base = K.lu + c * (long)(NC * NC) + pos;
#pragma unroll
  for (int j = 0; j < NC; ++j) base[(long)wl[j] * NC] = S[j];
}

// Reload what spc_store_factors stored and rebuild the position -> lane map
// wl of the segment; lanes without a row keep the identity row (zeros).
template <int SEG, int NC>
__device__ __forceinline__ void spc_load_factors(const ClassDev& K, long c, int i, bool act,
                                                 double (&Mrow)[NC], int& pos, int* wl) {
  const bool has = act && i < NC;
  const double* base = K.lu + (has ? c * (long)(NC * NC) + i : 0);
#pragma unroll
  for (int j = 0; j < NC; ++j) Mrow[j] = has ? base[j * NC] : (i == j ? 1.0 : 0.0);
  pos = has ? K.lpiv[c * NC + i] : i;
  __builtin_amdgcn_wave_barrier();
  if (has) wl[pos] = i;
  wave_sync_lds();
}

// Fused Newton iterations, segment per cell.  LS 0: FP64 LU factored once.
// LS 3: explicit inverse by Gauss-Jordan elimination, applied as a
// matrix-vector product (no serial substitution chain).
// LS 1: FP32 LU factored once, each solve refined with FP64 residuals
// r - M x = r - x + gamma J x, the product with J formed without the matrix
// (Spc::jx_row), so that no FP64 row stays in registers; a cell whose FP32
// factor is singular, or whose refinement fails, is solved with FP64 LU from
// then on, its M formed and factored again at each iteration that needs it
// (a rare path, kept off the registers of the refined one).  LS 2: correction X r with the cell's
// learned approximate inverse (X from the MLP, computed after the predictor
// kernel); a cell switches to FP64 LU for the rest of the attempt when X r
// is not finite, or from the second iteration on when its correction norm
// does not fall below 0.9 times the previous one.
// NC: columns held per lane (n rounded up to a multiple of 8, at most SEG).
// LZ (LS 0 and 3), the lazy Newton matrix in two kernels so that the reuse
// kernel carries no factorisation (and needs far fewer registers): 1 forms,
// factors (inverts) and stores M (a setup attempt), 2 reloads the stored
// factors (inverse) and scales each correction by C->dscale; the caller
// launches the one that C->setup asks for or both (the other returns at
// once).
template <int SEG, int LS, int NC = SEG, int LZ = 0>
__device__ __forceinline__ void spc_newton_body(const BdfDev& D, long blk, double* lds) {
  static_assert(LZ == 0 || LS == 0 || LS == 3, "stored factors: FP64 LU or the inverse");
  Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const NetDev& nd = K.net;
  const int n = K.n;
  const int lane = threadIdx.x & 63;
  const int i = lane & (SEG - 1);
  const int seg_base = lane & ~(SEG - 1);
  const int sb = threadIdx.x & ~(SEG - 1);
  const int cb = threadIdx.x / SEG;
  const long c = blk * Spc<SEG>::CPB + cb;
  const bool act = c < K.ncells;           // uniform over the segment
  const bool row = act && i < n;
  const long id = c * n + i;
  SpcShared* shp;
  double* lk;
  float* St;
  spc_stage<SEG>(K, blk, lds, shp, lk, St);
  SpcShared& sh = *shp;
  // Each iteration's norms: with the FP32 and learned solvers they are
  // summed over the wave at once and kept in LDS (the iteration number is
  // not a compile-time index, and per-lane accumulators for every iteration
  // cost registers those kernels need to run two or three waves per SIMD);
  // so do the lazy kernels, whose reuse kernel gains a wave from it; the
  // eager FP64 kernel, which gains none, keeps per-lane sums.
  constexpr bool kLdsSums = LS != 0 || LZ != 0;
  double* wsum = sh.wsum + (threadIdx.x >> 6) * kRedNewton;
  if (kLdsSums && lane < kRedNewton) wsum[lane] = 0.0;
  double red[kRedNewton];
#pragma unroll
  for (int k = 0; k < kRedNewton; ++k) red[k] = 0.0;
  const double* kap = lk + cb * spc_rpad(K.R);
  const double gamma = C->gamma;
  const int maxcor = C->maxcor;
  // this launch's iterations (a continuation starts at m0 > 0 from the
  // stored iterate of iteration m0 - 1)
  const int m0 = C->m0;
  const int m1 = m0 + C->kiters < maxcor ? m0 + C->kiters : maxcor;
  double zp0 = 0.0, cv = 0.0, w = 0.0;
  if (LS != 2) {
    spc_predict_row<SEG>(D, C, sh, sb, i, act, row, id, kap, St, zp0, cv, w);
  } else if (row) {
    zp0 = K.zp0[id];
    cv = K.cv[id];
    w = 1.0 / (D.rtol * fabs(K.z[0][id]) + D.atol);
  }
  // M = I - gamma J(z(0)[0]), row i in this lane (identity rows past n)
  double Mrow[NC];
  auto assemble = [&]() {
    __builtin_amdgcn_wave_barrier();
    sh.ys[threadIdx.x] = zp0;
    wave_sync_lds();
    if (act)
      Spc<SEG>::template jac_row<NC>(nd, kap, St, sh.ys + sb, i, Mrow);
    else
#pragma unroll
      for (int j = 0; j < NC; ++j) Mrow[j] = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) Mrow[j] = (i == j ? 1.0 : 0.0) - gamma * Mrow[j];
    if (!row)
#pragma unroll
      for (int j = 0; j < NC; ++j) Mrow[j] = (i == j ? 1.0 : 0.0);
  };
  const int nn = act ? n : 0;
  int pos = i, piv = i, info = 0;
  // LS 1 state
  float L[LS == 1 ? NC : 1];
  int pos32 = i, piv32 = i, src32 = i;
  float dinv32 = 1.0f;
  bool fp64 = LS == 0, sing32 = false;
  double mnorm = 0.0;
  // LS 2 state
  int mode = 0;                           // 2 learned, 3 switching to LU, 4 LU
  bool factored = false;
  double dcprev = 0.0;
  constexpr bool reuse = LZ == 2;
  if constexpr (LS == 0) {
    if constexpr (reuse) {
      spc_load_factors<SEG, NC>(K, c, i, act, Mrow, pos, sh.wl + sb);
    } else {
      assemble();
      info = SpcLU<SEG, double, NC>::factor(Mrow, i, nn, pos, piv, sh.prow + sb, sh.wl + sb);
      if constexpr (LZ == 1) spc_store_factors<SEG, NC>(K, c, i, act, Mrow, pos);
    }
    factored = true;
  } else if constexpr (LS == 3) {
    if constexpr (reuse) {   // row i of the stored inverse, natural order
      const bool has = act && i < NC;
      const double* base = K.lu + (has ? c * (long)(NC * NC) + i : 0);
#pragma unroll
      for (int j = 0; j < NC; ++j) Mrow[j] = has ? base[j * NC] : 0.0;
    } else {
      assemble();
      info = SpcGJ<SEG, NC>::invert(Mrow, i, nn, pos, sh.prow + sb, sh.wl + sb);
      if constexpr (LZ == 1) spc_store_inverse<SEG, NC>(K, c, i, act, Mrow, pos, sh.wl + sb);
    }
    factored = true;
  } else if constexpr (LS == 1) {
    // M as assemble() forms it, converted to FP32 entry by entry
    double rs = 0.0;
    auto put = [&](int a, double v) {
      const double e = i == a ? 1.0 : 0.0;
      const double mv = row ? e - gamma * v : e;
      rs += fabs(mv);
      L[a] = (float)mv;
    };
    __builtin_amdgcn_wave_barrier();
    sh.ys[threadIdx.x] = zp0;
    wave_sync_lds();
    if (act)
      Spc<SEG>::template jac_cols<NC>(nd, kap, St, sh.ys + sb, i, put);
    else
#pragma unroll
      for (int j = 0; j < NC; ++j) put(j, 0.0);
    mnorm = seg_max<SEG>(rs);
    const int inf32 =
        SpcLU<SEG, float, NC>::factor(L, i, nn, pos32, piv32, sh.prow32 + sb, sh.wl32 + sb);
    // a singular FP32 factor sends the segment's wave to FP64 LU (below)
    sing32 = inf32 != 0;
    fp64 = __any(sing32) != 0;
    // rows to position order: each right-hand side is read from lane src32
    src32 = SpcLU<SEG, float, NC>::position_source(i, nn, sh.wl32 + sb);
    SpcLU<SEG, float, NC>::to_position_order(L, seg_base, src32);
    dinv32 = SpcLU<SEG, float, NC>::pivot_reciprocal(L, i);
    // J's evaluation point for the matrix-free residuals (this segment's
    // part of prow, which only an FP64 factorisation, after which the
    // segment no longer refines, writes)
    sh.prow[threadIdx.x] = zp0;
  } else {
    mode = (act && !C->force_lu) ? 2 : 4;
    if (mode == 4) {
      assemble();
      info = SpcLU<SEG, double, NC>::factor(Mrow, i, nn, pos, piv, sh.prow + sb, sh.wl + sb);
      factored = true;
    }
  }
  float Xrow[LS == 2 ? NC : 1];
  if constexpr (LS == 2) {
#pragma unroll
    for (int j = 0; j < NC; ++j)
      Xrow[j] = K.X[(row ? c * (long)n * n + (long)i * n : 0) + (j < n ? j : 0)];
#pragma unroll
    for (int j = 0; j < NC; ++j) Xrow[j] = (mode == 2 && row && j < n) ? Xrow[j] : 0.0f;
  }
  if (LS == 1 && sing32 && act && i == 0) wsum[4] = 1.0;   // FP32 factor singular at setup
  double y = zp0;
  if (m0 > 0 && row) y = K.ys[m0 - 1][id];
  // LS 1: the FP32-refined iterations run on their own path (P 1).  When a
  // cell of the wave needs FP64 LU (a singular FP32 factor, or a refinement
  // that fails), the whole wave leaves it for a path that holds the FP64
  // factors and no FP32 ones (P 2), redoing the iteration whose refinement
  // failed; the cells that needed it count as fallbacks (with their sweeps)
  // at that iteration, the others of the wave are solved by FP64 LU too.
  int sweeps_p = 0, fb_p = 0;
  auto iterate = [&](int m, auto path) -> bool {
    constexpr int P = decltype(path)::value;
    __builtin_amdgcn_wave_barrier();
    sh.ys[threadIdx.x] = y;
    wave_sync_lds();
    double f = 0.0;
    if (act) Spc<SEG>::rhs_row(nd, kap, St, sh.ys + sb, i, f);
    const double r = row ? fma(gamma, f, cv - y) : 0.0;
    double del = 0.0;
    int sweeps = sweeps_p, fb = fb_p;
    sweeps_p = 0;
    fb_p = 0;
    double lp_solves = 0.0, lp_fb = 0.0, lp_unconv = 0.0;
    if constexpr (LS == 0) {
      del = SpcLU<SEG, double, NC>::solve(Mrow, i, seg_base, nn, pos, sh.wl + sb, r);
      if constexpr (reuse) del *= C->dscale;
    } else if constexpr (LS == 3) {
      if constexpr (reuse)
        del = C->dscale * SpcGJ<SEG, NC>::apply_natural(Mrow, i, r, seg_base, sh.prow + sb);
      else
        del = SpcGJ<SEG, NC>::apply(Mrow, i, pos, r, sh.prow + sb);
    } else if constexpr (LS == 1 && P == 2) {
      del = SpcLU<SEG, double, NC>::solve(Mrow, i, seg_base, nn, pos, sh.wl + sb, r);
    } else if constexpr (LS == 1) {
      bool ok = false;
      if (!fp64) {
        double x = (double)SpcLU<SEG, float, NC>::solve_ordered(
            L, i, seg_base, nn, dinv32, (float)__shfl(r, seg_base + src32, 64));
        const double eps64 = 2.220446049250313e-16;
        double dprv = 0.0;
        double* gk = spc_gk<SEG>(St, K.R, cb);
        for (int it = 0; it <= K.refine_max_it; ++it) {
          __builtin_amdgcn_wave_barrier();
          sh.ys[threadIdx.x] = x;
          wave_sync_lds();
          const double jx = Spc<SEG>::jx_row(nd, kap, St, sh.prow + sb, sh.ys + sb, gk, i);
          const double res = row ? fma(gamma, jx, r - x) : r - x;
          const double rn = seg_max<SEG>(fabs(res));
          const double xn = seg_max<SEG>(fabs(x));
          if (!(rn == rn) || !(xn == xn)) break;
          if (rn <= sqrt((double)n) * eps64 * mnorm * xn) {
            ok = true;
            break;
          }
          if (it == K.refine_max_it) break;
          const double d = (double)SpcLU<SEG, float, NC>::solve_ordered(
              L, i, seg_base, nn, dinv32, (float)__shfl(res, seg_base + src32, 64));
          x += d;
          const double dn = seg_max<SEG>(fabs(d));
          sweeps = it + 1;
          if (it >= 1 && dn > 0.5 * dprv) break;
          dprv = dn;
        }
        del = x;
        if (__any(!ok)) {   // uniform over the wave
          sweeps_p = sweeps;
          fb_p = ok ? 0 : 1;
          return false;
        }
      }
    } else {
      if (mode == 2) {
        // correction = X r with row i of the cell's approximate inverse
        double sx = 0.0;
#pragma unroll
        for (int j = 0; j < NC; ++j) sx = fma((double)Xrow[j], __shfl(r, seg_base + j, 64), sx);
        del = row ? sx : 0.0;
        const double bad = seg_max<SEG>(row && !(fabs(del) <= 1.79e308) ? 1.0 : 0.0);
        lp_solves = act ? 1.0 : 0.0;
        if (bad > 0.0) mode = 3;
      }
      if (mode != 2) {
        if (!factored) {
          assemble();
          info = SpcLU<SEG, double, NC>::factor(Mrow, i, nn, pos, piv, sh.prow + sb, sh.wl + sb);
          factored = true;
        }
        del = SpcLU<SEG, double, NC>::solve(Mrow, i, seg_base, nn, pos, sh.wl + sb, r);
        if (mode == 3) {
          lp_fb = 1.0;
          mode = 4;
        }
      }
      // a cell still on X that does not contract by 0.9 moves to LU from
      // the next iteration and keeps this iteration from being accepted
      // (counted in slot 7 of the iteration)
      const double dc = sqrt(seg_sum<SEG>(row ? (del * w) * (del * w) : 0.0) / (double)n);
      if (mode == 2 && m >= 1 && !(dc <= 0.9 * dcprev)) {
        mode = 3;
        lp_unconv = 1.0;
      }
      dcprev = dc;
    }
    double sd = 0.0, sa = 0.0, neg = 0.0;
    if (row) {
      y += del;
      K.ys[m][id] = y;
      const bool ng = D.nonneg && y < 0.0;
      const double a = del * w, b = ((ng ? 0.0 : y) - zp0) * w;
      sd = a * a;
      sa = b * b;
      neg = ng ? 1.0 : 0.0;
    }
    const bool lead = act && i == 0;
    if constexpr (kLdsSums) {
      double* ws = wsum + kRedPerIter * m;
      wave_add(sd, ws + 0);
      wave_add(sa, ws + 1);
      wave_add(neg, ws + 2);
      if constexpr (LS == 1) {
        wave_add(lead ? (double)sweeps : 0.0, ws + 3);
        wave_add(lead ? (double)fb : 0.0, ws + 4);
      }
      if constexpr (LS == 2) {
        wave_add(lead ? lp_solves : 0.0, ws + 5);
        wave_add(lead ? lp_fb : 0.0, ws + 6);
        if (m >= 1) wave_add(lead ? lp_unconv : 0.0, ws + 7);
      }
    } else {
#pragma unroll
      for (int mm = 0; mm < kMaxCor; ++mm) {
        const bool hit = (mm == m);
        red[kRedPerIter * mm + 0] += hit ? sd : 0.0;
        red[kRedPerIter * mm + 1] += hit ? sa : 0.0;
        red[kRedPerIter * mm + 2] += hit ? neg : 0.0;
      }
    }
    return true;
  };
  if constexpr (LS == 1) {
    int m = m0;
    if (!fp64)
      for (; m < m1; ++m)
        if (!iterate(m, std::integral_constant<int, 1>{})) break;
    if (m < m1) {   // uniform over the wave
      assemble();
      info = SpcLU<SEG, double, NC>::factor(Mrow, i, nn, pos, piv, sh.prow + sb, sh.wl + sb);
      for (; m < m1; ++m) iterate(m, std::integral_constant<int, 2>{});
    }
  } else {
    for (int m = m0; m < m1; ++m) iterate(m, std::integral_constant<int, 0>{});
  }
  if constexpr (kLdsSums) {
#pragma unroll
    for (int k = 0; k < kRedNewton; ++k) red[k] = lane == 0 ? wsum[k] : 0.0;
  }
  // a singular FP64 factorisation fails the attempt (LS 1: only the FP64
  // fallback can be singular; the FP32 factor then falls back)
  red[7] = (act && i == 0 && info) ? 1.0 : 0.0;
  block_partials<kRedNewton>(D, (unsigned int)(K.blk0 + blk), red, sh.red);
}

template <int SEG, int LS, int NC = SEG, int LZ = 0>
__global__ void __launch_bounds__(kCellThreads) k_spc_newton(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_PREDICT) return;
  if (LZ != 0 && (D.C->setup != 0) != (LZ == 1)) return;   // the other lazy kernel's attempt
  spc_newton_body<SEG, LS, NC, LZ>(D, blockIdx.x, lds);
}

// The same kernel asked to fit W waves per SIMD (512 / W registers), for
// instantiations that need only a few registers more than that, or whose
// excess belongs to a rarely taken path (the FP64 fallback of the
// FP32-refined solver), around which the compiler places the spills.
template <int SEG, int LS, int NC, int W, int LZ = 0>
__global__ void __launch_bounds__(kCellThreads) __attribute__((amdgpu_waves_per_eu(W)))
k_spc_newton_w(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_PREDICT) return;
  if (LZ != 0 && (D.C->setup != 0) != (LZ == 1)) return;
  spc_newton_body<SEG, LS, NC, LZ>(D, blockIdx.x, lds);
}

__host__ __device__ inline size_t spc_accept_lds() {
  return sizeof(double) * (size_t)(kCellThreads / 64) * kRedVals;
}

template <int SEG>
__device__ __forceinline__ void spc_accept_body(const BdfDev& D, long blk, double* lds) {
  double* s_red = lds;
  Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const int n = K.n;
  const int i = threadIdx.x & (SEG - 1);
  const long c = blk * Spc<SEG>::CPB + threadIdx.x / SEG;
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (c < K.ncells && i < n) {
    const long id = c * n + i;
    const int q = C->q;
    const double l0 = C->l[0];
    const bool select = C->qwait == 1;
    const bool raise = select && q < C->qmax;
    const bool keep = C->qwait == 2;
    double zs[kQmaxAll + 1];
    spc_load_hist(K, C, id, true, q, zs);
    const double yv = K.ys[C->m][id];
    const double dp = raise ? K.dprev[id] : 0.0;
    const double w = 1.0 / (D.rtol * fabs(zs[0]) + D.atol);
#pragma unroll
    for (int k = 1; k <= kQmaxAll; ++k)
#pragma unroll
      for (int j = kQmaxAll; j >= k; --j)
        if (k <= q && j <= q) zs[j - 1] = zs[j - 1] + zs[j];
    const double yp = D.nonneg && yv < 0.0 ? 0.0 : yv;
    const double acor = (yp - zs[0]) / l0;
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
    if (raise) {
      K.z[q + 1][id] = C->craise * acor;
      const double b = (acor - dp) * w;
      red[1] = b * b;
    }
    if (keep) K.dprev[id] = acor;
    const double a = znq * w;
    red[0] = a * a;
  }
  block_partials<kRedVals>(D, (unsigned int)(K.blk0 + blk), red, s_red);
}

template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_accept(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_ACCEPT) return;
  spc_accept_body<SEG>(D, blockIdx.x, lds);
}

// Starting step, part 1 (f(y0) into z[1], norms of y0 and f0) and part 2
// (norm of f(y0 + h0 f0) - f0).
template <int SEG, int PART>
__device__ __forceinline__ void spc_init_body(const BdfDev& D, long blk, double* lds) {
  Ctrl* C = D.C;
  const ClassDev& K = D.k;
  const int n = K.n;
  const int i = threadIdx.x & (SEG - 1);
  const int sb = threadIdx.x & ~(SEG - 1);
  const int cb = threadIdx.x / SEG;
  const long c = blk * Spc<SEG>::CPB + cb;
  const bool act = c < K.ncells;
  const bool row = act && i < n;
  const long id = c * n + i;
  SpcShared* shp;
  double* lk;
  float* St;
  spc_stage<SEG>(K, blk, lds, shp, lk, St);
  SpcShared& sh = *shp;
  const double* kap = lk + cb * spc_rpad(K.R);
  const double y0 = row ? K.z[0][id] : 0.0;
  const double f0 = (PART == 2 && row) ? K.z[1][id] : 0.0;
  sh.ys[threadIdx.x] = PART == 1 ? y0 : y0 + C->hnw_h0 * f0;
  __syncthreads();
  double f = 0.0;
  if (act) Spc<SEG>::rhs_row(K.net, kap, St, sh.ys + sb, i, f);
  double red[kRedVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (row) {
    const double w = 1.0 / (D.rtol * fabs(y0) + D.atol);
    if (PART == 1) {
      K.z[1][id] = f;
      red[0] = (y0 * w) * (y0 * w);
      red[1] = (f * w) * (f * w);
    } else {
      const double d = (f - f0) * w;
      red[0] = d * d;
    }
  }
  block_partials<kRedVals>(D, (unsigned int)(K.blk0 + blk), red, sh.red);
}

template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_init1(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_INIT1) return;
  spc_init_body<SEG, 1>(D, blockIdx.x, lds);
}

template <int SEG>
__global__ void __launch_bounds__(kCellThreads) k_spc_init2(BdfDev D) {
  extern __shared__ double lds[];
  if (D.C->phase != PH_INIT2) return;
  spc_init_body<SEG, 2>(D, blockIdx.x, lds);
}

}  // namespace bdfgpu
