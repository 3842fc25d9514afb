// Batched dense LU factor / solve / mixed-precision refinement entry points.
//
// The paper's direct solver for block-diagonal systems (Section 5) factors
// every block of a block-diagonal matrix whose blocks share one pattern; the
// many-small-systems use case makes the blocks small and dense (Section 2),
// so here each block is one SEG-lane segment of a wavefront with one row per
// lane (see spc.hpp).  Sizes that are not a power of two are padded with
// identity rows and columns inside registers, which leaves the leading
// n x n factors, pivots and solutions exactly those of the unpadded block.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"
#include "spc.hpp"

namespace bdfgpu {

constexpr int kLuThreads = 256;

template <int SEG, typename T>
__global__ void __launch_bounds__(kLuThreads) k_lu_factor(int nb, int n, T* A, int* piv,
                                                          int* info) {
  __shared__ T s_prow[kLuThreads];
  __shared__ int s_wl[kLuThreads];
  const int lane = threadIdx.x & 63;
  const int r = lane & (SEG - 1);
  const int sbase = threadIdx.x & ~(SEG - 1);   // this segment's LDS slots
  const long b = ((long)blockIdx.x * blockDim.x + threadIdx.x) / SEG;
  const bool valid = b < nb;
  const long base = b * (long)n * n;
  T row[SEG];
#pragma unroll
  for (int j = 0; j < SEG; ++j)
    row[j] = (valid && r < n && j < n) ? A[base + r + (long)j * n] : (r == j ? T(1) : T(0));
  int pos, pv;
  const int inf = SpcLU<SEG, T>::factor(row, r, valid ? n : 0, pos, pv, s_prow + sbase,
                                        s_wl + sbase);
  if (valid && r < n && pos < n) {
#pragma unroll
    for (int j = 0; j < SEG; ++j)
      if (j < n) A[base + pos + (long)j * n] = row[j];
    piv[b * n + r] = pv;
  }
  if (valid && r == 0) info[b] = inf;
}

template <int SEG, typename T>
__global__ void __launch_bounds__(kLuThreads) k_lu_solve(int nb, int n, const T* LU,
                                                         const int* piv, T* B) {
  const int lane = threadIdx.x & 63;
  const int r = lane & (SEG - 1);
  const int seg_base = lane & ~(SEG - 1);
  const long b = ((long)blockIdx.x * blockDim.x + threadIdx.x) / SEG;
  const bool valid = b < nb;
  const long base = b * (long)n * n;
  T row[SEG];
#pragma unroll
  for (int j = 0; j < SEG; ++j)
    row[j] = (valid && r < n && j < n) ? LU[base + r + (long)j * n] : (r == j ? T(1) : T(0));
  T val = (valid && r < n) ? B[b * n + r] : T(0);
  const T x = SpcLU<SEG, T>::solve_stored(row, r, seg_base, valid ? piv + b * n : piv,
                                          valid ? n : 0, val);
  if (valid && r < n) B[b * n + r] = x;
}

template <int SEG>
__global__ void __launch_bounds__(kLuThreads) k_lu_refine(int nb, int n, const double* M,
                                                          const float* LU32, const int* piv32,
                                                          const double* B, double* X,
                                                          int max_it, int* sweeps,
                                                          int* status) {
  __shared__ double s_prow[kLuThreads];
  __shared__ int s_wl[kLuThreads];
  const int sbase = threadIdx.x & ~(SEG - 1);
  const int lane = threadIdx.x & 63;
  const int r = lane & (SEG - 1);
  const int seg_base = lane & ~(SEG - 1);
  const long b = ((long)blockIdx.x * blockDim.x + threadIdx.x) / SEG;
  const bool valid = b < nb;
  const long base = b * (long)n * n;
  double rowM[SEG];
  float rowL[SEG];
#pragma unroll
  for (int j = 0; j < SEG; ++j) {
    const bool in = valid && r < n && j < n;
    rowM[j] = in ? M[base + r + (long)j * n] : (r == j ? 1.0 : 0.0);
    rowL[j] = in ? LU32[base + r + (long)j * n] : (r == j ? 1.0f : 0.0f);
  }
  const double bv = (valid && r < n) ? B[b * n + r] : 0.0;
  const int* pv = valid ? piv32 + b * n : piv32;
  const int ne = valid ? n : 0;
  double rs = 0.0;
#pragma unroll
  for (int j = 0; j < SEG; ++j) rs += fabs(rowM[j]);
  const double mnorm = seg_max<SEG>(r < n ? rs : 0.0);
  double x = (double)SpcLU<SEG, float>::solve_stored(rowL, r, seg_base, pv, ne, (float)bv);
  const double eps64 = 2.220446049250313e-16;
  double dprev = 0.0;
  int st = 1, sw = 0;
  for (int it = 0; it <= max_it; ++it) {
    double res = bv;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const double xj = __shfl(x, seg_base + j, 64);
      res = fma(-rowM[j], xj, res);
    }
    const double rn = seg_max<SEG>(r < n ? fabs(res) : 0.0);
    const double xn = seg_max<SEG>(r < n ? fabs(x) : 0.0);
    if (!(rn == rn) || !(xn == xn)) break;
    if (rn <= sqrt((double)n) * eps64 * mnorm * xn) {
      st = 0;
      break;
    }
    if (it == max_it) break;
    const double d =
        (double)SpcLU<SEG, float>::solve_stored(rowL, r, seg_base, pv, ne, (float)res);
    x += d;
    const double dn = seg_max<SEG>(r < n ? fabs(d) : 0.0);
    sw = it + 1;
    if (it >= 1 && dn > 0.5 * dprev) break;
    dprev = dn;
  }
  if (st) {
    int pos, pvv;
    const int inf = SpcLU<SEG, double>::factor(rowM, r, ne, pos, pvv, s_prow + sbase,
                                               s_wl + sbase);
    x = SpcLU<SEG, double>::solve(rowM, r, seg_base, ne, pos, s_wl + sbase, bv);
    if (inf) st = 2;
  }
  if (valid && r < n) X[b * n + r] = x;
  if (valid && r == 0) {
    sweeps[b] = sw;
    status[b] = st;
  }
}

// Blocks of different sizes in one launch: block b is sizes[b] x sizes[b]
// (<= nmax <= SEG) at A + moff[b], its pivots and right-hand side at
// voff[b].  A block whose size is outside 0..nmax gets info = -1 and is
// left untouched.
template <int SEG, typename T>
__global__ void __launch_bounds__(kLuThreads) k_lu_factor_var(int nb, int nmax, const int* sizes,
                                                              const long* moff, const long* voff,
                                                              T* A, int* piv, int* info) {
  __shared__ T s_prow[kLuThreads];
  __shared__ int s_wl[kLuThreads];
  const int lane = threadIdx.x & 63;
  const int r = lane & (SEG - 1);
  const int sbase = threadIdx.x & ~(SEG - 1);
  const long b = ((long)blockIdx.x * blockDim.x + threadIdx.x) / SEG;
  const int nraw = b < nb ? sizes[b] : 0;
  const bool bad = nraw < 0 || nraw > nmax;
  const int n = bad ? 0 : nraw;
  const long base = n > 0 ? moff[b] : 0;
  const long vb = n > 0 ? voff[b] : 0;
  T row[SEG];
#pragma unroll
  for (int j = 0; j < SEG; ++j)
    row[j] = (r < n && j < n) ? A[base + r + (long)j * n] : (r == j ? T(1) : T(0));
  int pos, pv;
  const int inf = SpcLU<SEG, T>::factor(row, r, n, pos, pv, s_prow + sbase, s_wl + sbase);
  if (r < n && pos < n) {
#pragma unroll
    for (int j = 0; j < SEG; ++j)
      if (j < n) A[base + pos + (long)j * n] = row[j];
    piv[vb + r] = pv;
  }
  if (b < nb && r == 0) info[b] = bad ? -1 : inf;
}

template <int SEG, typename T>
__global__ void __launch_bounds__(kLuThreads) k_lu_solve_var(int nb, int nmax, const int* sizes,
                                                             const long* moff, const long* voff,
                                                             const T* LU, const int* piv, T* B) {
  const int lane = threadIdx.x & 63;
  const int r = lane & (SEG - 1);
  const int seg_base = lane & ~(SEG - 1);
  const long b = ((long)blockIdx.x * blockDim.x + threadIdx.x) / SEG;
  const int nraw = b < nb ? sizes[b] : 0;
  const int n = (nraw < 0 || nraw > nmax) ? 0 : nraw;
  const long base = n > 0 ? moff[b] : 0;
  const long vb = n > 0 ? voff[b] : 0;
  T row[SEG];
#pragma unroll
  for (int j = 0; j < SEG; ++j)
    row[j] = (r < n && j < n) ? LU[base + r + (long)j * n] : (r == j ? T(1) : T(0));
  T val = r < n ? B[vb + r] : T(0);
  const T x = SpcLU<SEG, T>::solve_stored(row, r, seg_base, piv + vb, n, val);
  if (r < n) B[vb + r] = x;
}

static int seg_for(int n) {
  return n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : n <= 64 ? 64 : 0;
}

static unsigned int lu_blocks(long nb, int seg) {
  const long cpb = kLuThreads / seg;
  return (unsigned int)((nb + cpb - 1) / cpb);
}

template <typename T>
static int lu_factor_var(const char* name, int nb, int nmax, const int* sizes, const long* moff,
                         const long* voff, T* A, int* piv, int* info, void* stream) {
  if (nb < 0 || nmax < 0 || nmax > 64 ||
      (nb > 0 && nmax > 0 && (!sizes || !moff || !voff || !A || !piv || !info)))
    return arg_error(name);
  if (nb == 0) return 0;
  const int seg = nmax == 0 ? 2 : seg_for(nmax);
  hipStream_t s = as_stream(stream);
  dim3 g(lu_blocks(nb, seg)), blk(kLuThreads);
  switch (seg) {
    case 2: hipLaunchKernelGGL((k_lu_factor_var<2, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, A, piv, info); break;
    case 4: hipLaunchKernelGGL((k_lu_factor_var<4, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, A, piv, info); break;
    case 8: hipLaunchKernelGGL((k_lu_factor_var<8, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, A, piv, info); break;
    case 16: hipLaunchKernelGGL((k_lu_factor_var<16, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, A, piv, info); break;
    case 32: hipLaunchKernelGGL((k_lu_factor_var<32, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, A, piv, info); break;
    default: hipLaunchKernelGGL((k_lu_factor_var<64, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, A, piv, info); break;
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

template <typename T>
static int lu_solve_var(const char* name, int nb, int nmax, const int* sizes, const long* moff,
                        const long* voff, const T* LU, const int* piv, T* B, void* stream) {
  if (nb < 0 || nmax < 0 || nmax > 64 ||
      (nb > 0 && nmax > 0 && (!sizes || !moff || !voff || !LU || !piv || !B)))
    return arg_error(name);
  if (nb == 0 || nmax == 0) return 0;
  const int seg = seg_for(nmax);
  hipStream_t s = as_stream(stream);
  dim3 g(lu_blocks(nb, seg)), blk(kLuThreads);
  switch (seg) {
    case 2: hipLaunchKernelGGL((k_lu_solve_var<2, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, LU, piv, B); break;
    case 4: hipLaunchKernelGGL((k_lu_solve_var<4, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, LU, piv, B); break;
    case 8: hipLaunchKernelGGL((k_lu_solve_var<8, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, LU, piv, B); break;
    case 16: hipLaunchKernelGGL((k_lu_solve_var<16, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, LU, piv, B); break;
    case 32: hipLaunchKernelGGL((k_lu_solve_var<32, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, LU, piv, B); break;
    default: hipLaunchKernelGGL((k_lu_solve_var<64, T>), g, blk, 0, s, nb, nmax, sizes, moff, voff, LU, piv, B); break;
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace bdfgpu

using namespace bdfgpu;

extern "C" {

int batched_lu_factor_f64(int nb, int n, double* A, int* piv, int* info, void* stream) {
  if (nb < 0 || n < 0 || n > 64 || (nb > 0 && n > 0 && (!A || !piv || !info)))
    return arg_error("batched_lu_factor_f64: bad argument (n must be <= 64)");
  if (nb == 0 || n == 0) return 0;
  const int seg = seg_for(n);
  hipStream_t s = as_stream(stream);
  dim3 g(lu_blocks(nb, seg)), blk(kLuThreads);
  switch (seg) {
    case 2: hipLaunchKernelGGL((k_lu_factor<2, double>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 4: hipLaunchKernelGGL((k_lu_factor<4, double>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 8: hipLaunchKernelGGL((k_lu_factor<8, double>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 16: hipLaunchKernelGGL((k_lu_factor<16, double>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 32: hipLaunchKernelGGL((k_lu_factor<32, double>), g, blk, 0, s, nb, n, A, piv, info); break;
    default: hipLaunchKernelGGL((k_lu_factor<64, double>), g, blk, 0, s, nb, n, A, piv, info); break;
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int batched_lu_factor_f32(int nb, int n, float* A, int* piv, int* info, void* stream) {
  if (nb < 0 || n < 0 || n > 64 || (nb > 0 && n > 0 && (!A || !piv || !info)))
    return arg_error("batched_lu_factor_f32: bad argument (n must be <= 64)");
  if (nb == 0 || n == 0) return 0;
  const int seg = seg_for(n);
  hipStream_t s = as_stream(stream);
  dim3 g(lu_blocks(nb, seg)), blk(kLuThreads);
  switch (seg) {
    case 2: hipLaunchKernelGGL((k_lu_factor<2, float>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 4: hipLaunchKernelGGL((k_lu_factor<4, float>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 8: hipLaunchKernelGGL((k_lu_factor<8, float>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 16: hipLaunchKernelGGL((k_lu_factor<16, float>), g, blk, 0, s, nb, n, A, piv, info); break;
    case 32: hipLaunchKernelGGL((k_lu_factor<32, float>), g, blk, 0, s, nb, n, A, piv, info); break;
    default: hipLaunchKernelGGL((k_lu_factor<64, float>), g, blk, 0, s, nb, n, A, piv, info); break;
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int batched_lu_solve_f64(int nb, int n, const double* LU, const int* piv, double* B,
                         void* stream) {
  if (nb < 0 || n < 0 || n > 64 || (nb > 0 && n > 0 && (!LU || !piv || !B)))
    return arg_error("batched_lu_solve_f64: bad argument (n must be <= 64)");
  if (nb == 0 || n == 0) return 0;
  const int seg = seg_for(n);
  hipStream_t s = as_stream(stream);
  dim3 g(lu_blocks(nb, seg)), blk(kLuThreads);
  switch (seg) {
    case 2: hipLaunchKernelGGL((k_lu_solve<2, double>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 4: hipLaunchKernelGGL((k_lu_solve<4, double>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 8: hipLaunchKernelGGL((k_lu_solve<8, double>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 16: hipLaunchKernelGGL((k_lu_solve<16, double>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 32: hipLaunchKernelGGL((k_lu_solve<32, double>), g, blk, 0, s, nb, n, LU, piv, B); break;
    default: hipLaunchKernelGGL((k_lu_solve<64, double>), g, blk, 0, s, nb, n, LU, piv, B); break;
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int batched_lu_solve_f32(int nb, int n, const float* LU, const int* piv, float* B,
                         void* stream) {
  if (nb < 0 || n < 0 || n > 64 || (nb > 0 && n > 0 && (!LU || !piv || !B)))
    return arg_error("batched_lu_solve_f32: bad argument (n must be <= 64)");
  if (nb == 0 || n == 0) return 0;
  const int seg = seg_for(n);
  hipStream_t s = as_stream(stream);
  dim3 g(lu_blocks(nb, seg)), blk(kLuThreads);
  switch (seg) {
    case 2: hipLaunchKernelGGL((k_lu_solve<2, float>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 4: hipLaunchKernelGGL((k_lu_solve<4, float>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 8: hipLaunchKernelGGL((k_lu_solve<8, float>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 16: hipLaunchKernelGGL((k_lu_solve<16, float>), g, blk, 0, s, nb, n, LU, piv, B); break;
    case 32: hipLaunchKernelGGL((k_lu_solve<32, float>), g, blk, 0, s, nb, n, LU, piv, B); break;
    default: hipLaunchKernelGGL((k_lu_solve<64, float>), g, blk, 0, s, nb, n, LU, piv, B); break;
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int batched_lu_solve_refine(int nb, int n, const double* M, const float* LU32, const int* piv32,
                            const double* B, double* X, int max_it, int* sweeps, int* status,
                            void* stream) {
  if (nb < 0 || n < 0 || n > 64 || max_it < 0 ||
      (nb > 0 && n > 0 && (!M || !LU32 || !piv32 || !B || !X || !sweeps || !status)))
    return arg_error("batched_lu_solve_refine: bad argument (n must be <= 64)");
  if (nb == 0 || n == 0) return 0;
  const int seg = seg_for(n);
  hipStream_t s = as_stream(stream);
  dim3 g(lu_blocks(nb, seg)), blk(kLuThreads);
  switch (seg) {
    case 2: hipLaunchKernelGGL(k_lu_refine<2>, g, blk, 0, s, nb, n, M, LU32, piv32, B, X, max_it, sweeps, status); break;
    case 4: hipLaunchKernelGGL(k_lu_refine<4>, g, blk, 0, s, nb, n, M, LU32, piv32, B, X, max_it, sweeps, status); break;
    case 8: hipLaunchKernelGGL(k_lu_refine<8>, g, blk, 0, s, nb, n, M, LU32, piv32, B, X, max_it, sweeps, status); break;
    case 16: hipLaunchKernelGGL(k_lu_refine<16>, g, blk, 0, s, nb, n, M, LU32, piv32, B, X, max_it, sweeps, status); break;
    case 32: hipLaunchKernelGGL(k_lu_refine<32>, g, blk, 0, s, nb, n, M, LU32, piv32, B, X, max_it, sweeps, status); break;
    default: hipLaunchKernelGGL(k_lu_refine<64>, g, blk, 0, s, nb, n, M, LU32, piv32, B, X, max_it, sweeps, status); break;
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int batched_lu_factor_f64_var(int nb, int nmax, const int* sizes, const long* moff,
                              const long* voff, double* A, int* piv, int* info, void* stream) {
  return lu_factor_var<double>("batched_lu_factor_f64_var: bad argument (nmax <= 64)", nb, nmax,
                               sizes, moff, voff, A, piv, info, stream);
}

int batched_lu_factor_f32_var(int nb, int nmax, const int* sizes, const long* moff,
                              const long* voff, float* A, int* piv, int* info, void* stream) {
  return lu_factor_var<float>("batched_lu_factor_f32_var: bad argument (nmax <= 64)", nb, nmax,
                              sizes, moff, voff, A, piv, info, stream);
}

int batched_lu_solve_f64_var(int nb, int nmax, const int* sizes, const long* moff,
                             const long* voff, const double* LU, const int* piv, double* B,
                             void* stream) {
  return lu_solve_var<double>("batched_lu_solve_f64_var: bad argument (nmax <= 64)", nb, nmax,
                              sizes, moff, voff, LU, piv, B, stream);
}

int batched_lu_solve_f32_var(int nb, int nmax, const int* sizes, const long* moff,
                             const long* voff, const float* LU, const int* piv, float* B,
                             void* stream) {
  return lu_solve_var<float>("batched_lu_solve_f32_var: bad argument (nmax <= 64)", nb, nmax,
                             sizes, moff, voff, LU, piv, B, stream);
}

}  // extern "C"
