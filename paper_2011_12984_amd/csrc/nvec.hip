// N_Vector operations for gfx950: streaming kernels and two-pass reductions
// (wavefront shuffle and LDS to one partial per block, then one finishing
// block that sums the partials in block order).
//
// The paper groups vector operations into streaming operations and
// reductions (Section 2); reductions are completed on the GPU and the scalar
// returned by one transfer (Section 4.1).  The fused operations (linear
// combination, scale-add-multi, multiple dot products, WRMS norm) are
// memory-bound: each reads every input once and writes every output once,
// with 16-byte loads and stores, so their speed is set by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "common.hpp"

namespace bdfgpu {

static thread_local std::string g_last_error;
static std::mutex g_err_mu;
static std::string g_last_error_global;

void set_last_error(const char* msg, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s (%s:%d)", msg, file, line);
  std::lock_guard<std::mutex> lk(g_err_mu);
  g_last_error_global = buf;
}

int arg_error(const char* msg) {
  std::lock_guard<std::mutex> lk(g_err_mu);
  g_last_error_global = msg;
  return BDFGPU_ERR_ARG;
}

// ---------------------------------------------------------------------------
// Per-device reduction scratch: per-block partials, a device result slot
// and a pinned host result buffer.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 8192;   // upper bound on blocks of a reduction
constexpr int kRedK = 8;           // values per block
constexpr int kMaxDev = 64;

struct RedScratch {
  double* partials = nullptr;
  double* dres = nullptr;
  double* hres = nullptr;
};
static RedScratch g_red[kMaxDev];
static std::mutex g_red_mu;

// Reduction scratch that needs no allocation, for nvec_dot_prod_multi_noalloc:
// block partials in the library's static device memory (kRedBlocks x kRedK
// doubles = 512 KiB, held by every device the library runs on until the
// process ends).  Host code uses only the per-device address obtained with
// hipGetSymbolAddress, never the array's name.
static __device__ __align__(256) double scratch[kRedBlocks * kRedK];
static double* g_scratch_ptr[kMaxDev];
static std::mutex g_scratch_mu;

static int get_static_scratch(double** out) {
  int dev = 0;
  BDF_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return arg_error("device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BDF_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return arg_error("static reduction scratch has no device address");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

static int get_red_scratch(RedScratch** out) {
  int dev = 0;
  BDF_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return arg_error("device index out of range");
  std::lock_guard<std::mutex> lk(g_red_mu);
  RedScratch& r = g_red[dev];
  if (!r.partials) {
    BDF_HIP_TRY(hipMalloc(&r.partials, sizeof(double) * kRedBlocks * kRedK));
    BDF_HIP_TRY(hipMalloc(&r.dres, sizeof(double) * kRedK));
    BDF_HIP_TRY(hipHostMalloc(&r.hres, sizeof(double) * kRedK, hipHostMallocDefault));
    BDF_HIP_TRY(hipDeviceSynchronize());
  }
  *out = &r;
  return 0;
}

typedef double dbl2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ dbl2 ntload(const double* p, long i) {
  return __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(p) + i);
}
__device__ __forceinline__ void ntstore(double* p, long i, dbl2 v) {
  __builtin_nontemporal_store(v, reinterpret_cast<dbl2*>(p) + i);
}

static inline bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Launch shape for memory-bound kernels on 16-byte units.  A block of 256
// threads owns tiles of kTile = 256 * kU units of every vector; wave w owns
// 64 * kU consecutive units of the tile and lane l touches units l, l + 64,
// ..., so each wave reads 4 KB contiguous from every vector per tile and
// keeps all of its loads in flight at once.  In a sweep on MI355X this shape
// beat one unit per thread by 10-25% for operations on many vectors (a dot
// product of one vector against eight: 5.9 -> 7.0 TB/s).  Streaming kernels
// take one tile per block; reductions a bounded grid that loops over tiles,
// so that the block partials stay few.
constexpr int kStreamThreads = 256;
constexpr int kU = 4;
constexpr long kTile = (long)kStreamThreads * kU;

static long ntiles_of(long nunits) { return (nunits + kTile - 1) / kTile; }
static unsigned int stream_blocks(long nunits) {
  return (unsigned int)std::max(1L, std::min(ntiles_of(nunits), 1L << 24));
}
// first unit of this thread in tile t
__device__ __forceinline__ long tile_base(long t) {
  return (t * kStreamThreads + (long)(threadIdx.x >> 6) * 64) * kU + (threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// Streaming kernels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_linear_sum2(long n2, double a, const double* __restrict__ x,
                                                     double b, const double* __restrict__ y,
                                                     double* __restrict__ z) {
  const long nt = (n2 + kTile - 1) / kTile;
  for (long t = blockIdx.x; t < nt; t += gridDim.x) {
    const long i0 = tile_base(t);
    if (i0 + (kU - 1) * 64 < n2) {
      dbl2 xv[kU], yv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        xv[u] = ntload(x, i0 + u * 64);
        yv[u] = ntload(y, i0 + u * 64);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        dbl2 o;
        o.x = a * xv[u].x + b * yv[u].x;
        o.y = a * xv[u].y + b * yv[u].y;
        ntstore(z, i0 + u * 64, o);
      }
    } else {
      for (int u = 0; u < kU; ++u) {
        const long i = i0 + u * 64;
        if (i >= n2) break;
        const dbl2 xv = ntload(x, i), yv = ntload(y, i);
        dbl2 o;
        o.x = a * xv.x + b * yv.x;
        o.y = a * xv.y + b * yv.y;
        ntstore(z, i, o);
      }
    }
  }
}

__global__ void k_linear_sum1(long n, long start, double a, const double* x,
                              double b, const double* y, double* z) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = start + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    z[i] = a * x[i] + b * y[i];
}

struct LcArgs {
  const double* X[16];
  double c[16];
};

__device__ __forceinline__ dbl2 lc_unit(const LcArgs& A, const dbl2* v, int nv) {
  dbl2 o;
  o.x = A.c[0] * v[0].x;
  o.y = A.c[0] * v[0].y;
  for (int j = 1; j < nv; ++j) {
    o.x = fma(A.c[j], v[j].x, o.x);
    o.y = fma(A.c[j], v[j].y, o.y);
  }
  return o;
}

template <int NV>
__global__ void __launch_bounds__(256) k_linear_combination2(long n2, LcArgs A, double* __restrict__ z) {
  const long nt = (n2 + kTile - 1) / kTile;
  for (long t = blockIdx.x; t < nt; t += gridDim.x) {
    const long i0 = tile_base(t);
    if (i0 + (kU - 1) * 64 < n2) {
      dbl2 v[kU][NV];
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u][j] = ntload(A.X[j], i0 + u * 64);
      // every load of the tile is issued before the first sum waits on one
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        dbl2 o;
        o.x = A.c[0] * v[u][0].x;
        o.y = A.c[0] * v[u][0].y;
#pragma unroll
        for (int j = 1; j < NV; ++j) {
          o.x = fma(A.c[j], v[u][j].x, o.x);
          o.y = fma(A.c[j], v[u][j].y, o.y);
        }
        ntstore(z, i0 + u * 64, o);
      }
    } else {
      for (int u = 0; u < kU; ++u) {
        const long i = i0 + u * 64;
        if (i >= n2) break;
        dbl2 v[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = ntload(A.X[j], i);
        ntstore(z, i, lc_unit(A, v, NV));
      }
    }
  }
}

// Long-run form for many vectors: a lane owns kLcU units spaced 64 apart, so a wave sums 64 * kLcU
// consecutive units (32 KB of every vector) and walks the vectors one at a time, loading vector
// j + 1 while it adds vector j.  Each vector is then read in 32 KB runs instead of the 4 KB runs of
// the tile form, and the registers no longer grow with the number of vectors (186 VGPRs, two
// waves per SIMD).  In a sweep on MI355X at 16 vectors of 2^26 doubles it took 1.49-1.50 ms
// against 1.53-1.54 for the tile form; at 8 units per lane or with more vectors in flight it
// was slower.  Whole chunks only; the caller hands the rest to the tile form.
constexpr int kLcU = 32;
constexpr long kLcChunk = (long)kStreamThreads * kLcU;

template <int NV>
__global__ void __launch_bounds__(256) k_linear_combination_runs(long n2, LcArgs A,
                                                                 double* __restrict__ z) {
  const long i0 = ((long)blockIdx.x * kStreamThreads + (long)(threadIdx.x >> 6) * 64) * kLcU +
                  (threadIdx.x & 63);
  if (i0 + (kLcU - 1) * 64 >= n2) return;   // the grid covers whole chunks only
  dbl2 acc[kLcU], cur[kLcU], nxt[kLcU];
#pragma unroll
  for (int u = 0; u < kLcU; ++u) cur[u] = ntload(A.X[0], i0 + u * 64);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j + 1 < NV) {
#pragma unroll
      for (int u = 0; u < kLcU; ++u) nxt[u] = ntload(A.X[j + 1], i0 + u * 64);
    }
#pragma unroll
    for (int u = 0; u < kLcU; ++u) {
      if (j == 0) {
        acc[u] = A.c[0] * cur[u];
      } else {
        acc[u].x = fma(A.c[j], cur[u].x, acc[u].x);
        acc[u].y = fma(A.c[j], cur[u].y, acc[u].y);
      }
    }
#pragma unroll
    for (int u = 0; u < kLcU; ++u) cur[u] = nxt[u];
  }
#pragma unroll
  for (int u = 0; u < kLcU; ++u) ntstore(z, i0 + u * 64, acc[u]);
}

__global__ void k_linear_combination1(int nv, long n, long start, LcArgs A, double* z) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = start + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double s = A.c[0] * A.X[0][i];
    for (int j = 1; j < nv; ++j) s = fma(A.c[j], A.X[j][i], s);
    z[i] = s;
  }
}

struct SamArgs {
  const double* Y[8];
  double* Z[8];
  double a[8];
};

template <int NV>
__global__ void __launch_bounds__(256) k_scale_add_multi2(long n2, const double* __restrict__ x,
                                                          SamArgs A) {
  const long nt = (n2 + kTile - 1) / kTile;
  for (long t = blockIdx.x; t < nt; t += gridDim.x) {
    const long i0 = tile_base(t);
    if (i0 + (kU - 1) * 64 < n2) {
      dbl2 xv[kU], yv[kU][NV];
#pragma unroll
      for (int u = 0; u < kU; ++u) xv[u] = ntload(x, i0 + u * 64);
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int u = 0; u < kU; ++u) yv[u][j] = ntload(A.Y[j], i0 + u * 64);
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          dbl2 o;
          o.x = fma(A.a[j], xv[u].x, yv[u][j].x);
          o.y = fma(A.a[j], xv[u].y, yv[u][j].y);
          ntstore(A.Z[j], i0 + u * 64, o);
        }
    } else {
      for (int u = 0; u < kU; ++u) {
        const long i = i0 + u * 64;
        if (i >= n2) break;
        const dbl2 xv = ntload(x, i);
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          const dbl2 yv = ntload(A.Y[j], i);
          dbl2 o;
          o.x = fma(A.a[j], xv.x, yv.x);
          o.y = fma(A.a[j], xv.y, yv.y);
          ntstore(A.Z[j], i, o);
        }
      }
    }
  }
}

__global__ void k_scale_add_multi1(int nv, long n, long start, const double* x, SamArgs A) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = start + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double xv = x[i];
    for (int j = 0; j < nv; ++j) A.Z[j][i] = fma(A.a[j], xv, A.Y[j][i]);
  }
}

// One-input (or no-input) element maps: one 16-byte unit per thread with
// non-temporal loads and stores over aligned vectors (a plain copy in this
// shape streams at about 6.5 TB/s on MI355X), the odd tail or unaligned
// vectors element by element from `start`.
constexpr int kMapThreads = 256;
static unsigned int map_blocks(long units) {
  return (unsigned int)std::max(1L, std::min((units + kMapThreads - 1) / kMapThreads, 1L << 24));
}

__global__ void __launch_bounds__(kMapThreads) k_ewt2(long n2, double rtol, double atol,
                                                      const double* y, double* w) {
  const long stride = (long)gridDim.x * kMapThreads;
  for (long i = (long)blockIdx.x * kMapThreads + threadIdx.x; i < n2; i += stride) {
    const dbl2 v = ntload(y, i);
    dbl2 o;
    o.x = 1.0 / (rtol * fabs(v.x) + atol);
    o.y = 1.0 / (rtol * fabs(v.y) + atol);
    ntstore(w, i, o);
  }
}

__global__ void k_ewt(long n, long start, double rtol, double atol, const double* y, double* w) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = start + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    w[i] = 1.0 / (rtol * fabs(y[i]) + atol);
}

__global__ void __launch_bounds__(kMapThreads) k_scale2(long n2, double c, const double* x,
                                                        double* z) {
  const long stride = (long)gridDim.x * kMapThreads;
  for (long i = (long)blockIdx.x * kMapThreads + threadIdx.x; i < n2; i += stride) {
    dbl2 v = ntload(x, i);
    v.x = c * v.x;
    v.y = c * v.y;
    ntstore(z, i, v);
  }
}

__global__ void k_scale(long n, long start, double c, const double* x, double* z) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = start + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    z[i] = c * x[i];
}

__global__ void __launch_bounds__(kMapThreads) k_const2(long n2, double c, double* __restrict__ z) {
  const long stride = (long)gridDim.x * kMapThreads;
  dbl2 v;
  v.x = c;
  v.y = c;
  for (long i = (long)blockIdx.x * kMapThreads + threadIdx.x; i < n2; i += stride) ntstore(z, i, v);
}

__global__ void k_const(long n, long start, double c, double* z) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = start + (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) z[i] = c;
}

// ---------------------------------------------------------------------------
// Reductions.  Per-thread FP64 partials -> wave shuffle -> LDS -> one
// partial per block (plain stores) -> k_finish: one block sums the partials
// in block order.  No float atomics and no per-block device-scope fence
// (each would write back the L2); deterministic for a given launch shape.
// ---------------------------------------------------------------------------
struct DotArgs {
  const double* Y[8];
};

template <int K>
__device__ __forceinline__ void store_block_partials(double (&acc)[K], double* sh,
                                                     double* partials) {
  block_sum<K>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) partials[(size_t)blockIdx.x * kRedK + k] = acc[k];
}

template <int NV>
__global__ void __launch_bounds__(256) k_dot_prod_multi(long n, const double* __restrict__ x,
                                                        DotArgs A, double* partials) {
  __shared__ double sh[4 * NV];
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  const long n2 = n >> 1;
  const long nt = (n2 + kTile - 1) / kTile;
  for (long t = blockIdx.x; t < nt; t += gridDim.x) {
    const long i0 = tile_base(t);
    if (i0 + (kU - 1) * 64 < n2) {
      dbl2 xv[kU], yv[kU][NV];
#pragma unroll
      for (int u = 0; u < kU; ++u) xv[u] = ntload(x, i0 + u * 64);
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int u = 0; u < kU; ++u) yv[u][j] = ntload(A.Y[j], i0 + u * 64);
      // every load of the tile is issued before the first sum waits on one
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kU; ++u)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          acc[j] = fma(xv[u].x, yv[u][j].x, acc[j]);
          acc[j] = fma(xv[u].y, yv[u][j].y, acc[j]);
        }
    } else {
      for (int u = 0; u < kU; ++u) {
        const long i = i0 + u * 64;
        if (i >= n2) break;
        const dbl2 xv = ntload(x, i);
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          const dbl2 yv = ntload(A.Y[j], i);
          acc[j] = fma(xv.x, yv.x, acc[j]);
          acc[j] = fma(xv.y, yv.y, acc[j]);
        }
      }
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = fma(x[n - 1], A.Y[j][n - 1], acc[j]);
  }
  store_block_partials<NV>(acc, sh, partials);
}

__global__ void __launch_bounds__(256) k_wrms(long n, const double* __restrict__ x,
                                              const double* __restrict__ w, double* partials) {
  __shared__ double sh[4];
  double acc[1] = {0.0};
  const long n2 = n >> 1;
  const long nt = (n2 + kTile - 1) / kTile;
  for (long t = blockIdx.x; t < nt; t += gridDim.x) {
    const long i0 = tile_base(t);
    if (i0 + (kU - 1) * 64 < n2) {
      dbl2 xv[kU], wv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        xv[u] = ntload(x, i0 + u * 64);
        wv[u] = ntload(w, i0 + u * 64);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const double a = xv[u].x * wv[u].x, b = xv[u].y * wv[u].y;
        acc[0] = fma(a, a, acc[0]);
        acc[0] = fma(b, b, acc[0]);
      }
    } else {
      for (int u = 0; u < kU; ++u) {
        const long i = i0 + u * 64;
        if (i >= n2) break;
        const dbl2 xv = ntload(x, i), wv = ntload(w, i);
        const double a = xv.x * wv.x, b = xv.y * wv.y;
        acc[0] = fma(a, a, acc[0]);
        acc[0] = fma(b, b, acc[0]);
      }
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double a = x[n - 1] * w[n - 1];
    acc[0] = fma(a, a, acc[0]);
  }
  store_block_partials<1>(acc, sh, partials);
}

// WRMS norms of nv vectors, each with its weight vector (SHW: one weight
// vector shared by all, read once): sums of (x_ji w_ji)^2 per vector.
struct WrmsArgs {
  const double* X[8];
  const double* W[8];
};

template <int NV, bool SHW>
__global__ void __launch_bounds__(256) k_wrms_multi(long n, WrmsArgs A, double* partials) {
  __shared__ double sh[4 * NV];
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  constexpr int NW = SHW ? 1 : NV;
  const long n2 = n >> 1;
  const long nt = (n2 + kTile - 1) / kTile;
  for (long t = blockIdx.x; t < nt; t += gridDim.x) {
    const long i0 = tile_base(t);
    if (i0 + (kU - 1) * 64 < n2) {
      dbl2 xv[kU][NV], wv[kU][NW];
#pragma unroll
      for (int j = 0; j < NW; ++j)
#pragma unroll
        for (int u = 0; u < kU; ++u) wv[u][j] = ntload(A.W[j], i0 + u * 64);
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int u = 0; u < kU; ++u) xv[u][j] = ntload(A.X[j], i0 + u * 64);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kU; ++u)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          const dbl2 w = wv[u][SHW ? 0 : j];
          const double a = xv[u][j].x * w.x, b = xv[u][j].y * w.y;
          acc[j] = fma(a, a, acc[j]);
          acc[j] = fma(b, b, acc[j]);
        }
    } else {
      for (int u = 0; u < kU; ++u) {
        const long i = i0 + u * 64;
        if (i >= n2) break;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          const dbl2 xv = ntload(A.X[j], i), w = ntload(A.W[SHW ? 0 : j], i);
          const double a = xv.x * w.x, b = xv.y * w.y;
          acc[j] = fma(a, a, acc[j]);
          acc[j] = fma(b, b, acc[j]);
        }
      }
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double a = A.X[j][n - 1] * A.W[SHW ? 0 : j][n - 1];
      acc[j] = fma(a, a, acc[j]);
    }
  }
  store_block_partials<NV>(acc, sh, partials);
}

template <int NV>
__global__ void __launch_bounds__(256) k_wrms_multi_u(long n, WrmsArgs A, double* partials) {
  __shared__ double sh[4 * NV];
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const double a = A.X[j][i] * A.W[j][i];
      acc[j] = fma(a, a, acc[j]);
    }
  }
  store_block_partials<NV>(acc, sh, partials);
}

// scalar-load variants for vectors that are not 16-byte aligned
template <int NV>
__global__ void __launch_bounds__(256) k_dot_prod_multi_u(long n, const double* x, DotArgs A,
                                                          double* partials) {
  __shared__ double sh[4 * NV];
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double xv = x[i];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = fma(xv, A.Y[j][i], acc[j]);
  }
  store_block_partials<NV>(acc, sh, partials);
}

__global__ void __launch_bounds__(256) k_wrms_u(long n, const double* x, const double* w,
                                                double* partials) {
  __shared__ double sh[4];
  double acc[1] = {0.0};
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double a = x[i] * w[i];
    acc[0] = fma(a, a, acc[0]);
  }
  store_block_partials<1>(acc, sh, partials);
}

__global__ void __launch_bounds__(256) k_maxnorm(long n, const double* x, double* partials) {
  __shared__ double sh[4];
  double m = 0.0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    m = fmax(m, fabs(x[i]));
  m = wave_max(m);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) v = fmax(v, sh[k]);
    partials[(size_t)blockIdx.x * kRedK] = v;
  }
}

// One block of 1024 threads: value k of the result is the sum (op 0), the
// square root of the mean (op 1, WRMS: divided by n) or the maximum (op 2)
// over the nb block partials.  Thread t takes partials t, t + 1024, ... in
// order (all nv values at once), then a fixed tree over the block.
__global__ void __launch_bounds__(1024) k_finish(int nv, unsigned int nb, int op, long n,
                                                 const double* partials, double* out) {
  __shared__ double sh[16 * kRedK];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v[kRedK];
#pragma unroll
  for (int k = 0; k < kRedK; ++k) v[k] = 0.0;
  for (unsigned int b = threadIdx.x; b < nb; b += 1024) {
#pragma unroll
    for (int k = 0; k < kRedK; ++k) {
      if (k < nv) {
        const double x = partials[(size_t)b * kRedK + k];
        v[k] = op == 2 ? fmax(v[k], x) : v[k] + x;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kRedK; ++k) {
    if (k < nv) {
      const double r = op == 2 ? wave_max(v[k]) : wave_sum(v[k]);
      if (lane == 0) sh[wid * kRedK + k] = r;
    }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int k = threadIdx.x;
    double a = 0.0;
    for (int w = 0; w < 16; ++w) a = op == 2 ? fmax(a, sh[w * kRedK + k]) : a + sh[w * kRedK + k];
    out[k] = op == 1 ? sqrt(a / (double)n) : a;
  }
}

// Grid of a reduction over nunits units handled kTile per block and tile
// (aligned kernels) or one per thread (scalar kernels, per_thread = true).
static unsigned int red_blocks(long nunits, bool per_thread = false) {
  long want = per_thread ? (nunits + kStreamThreads - 1) / kStreamThreads : ntiles_of(nunits);
  return (unsigned int)std::max(1L, std::min(want, (long)kRedBlocks));
}

// Where k_finish writes: the caller's device array directly, or the device
// slot that finish_reduction then copies to the host.
static double* finish_target(RedScratch* r, double* out, int flags) {
  return (flags & BDFGPU_RESULT_DEVICE) ? out : r->dres;
}

// Finish a reduction whose k_finish wrote to its finish_target: a device
// result is already in place; a host result is copied back and waited for.
static int finish_reduction(RedScratch* r, int nv, double* out, int flags, hipStream_t s) {
  if (flags & BDFGPU_RESULT_DEVICE) return 0;
  BDF_HIP_TRY(hipMemcpyAsync(r->hres, r->dres, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
  BDF_HIP_TRY(hipStreamSynchronize(s));
  memcpy(out, r->hres, sizeof(double) * nv);
  return 0;
}

// Blocks of the dot-product kernels for n elements (aligned: 16-byte units).
static unsigned int dot_grid(long n, bool al) {
  return al ? red_blocks(n >> 1) : red_blocks(n, true);
}

// Multiple dot products: block partials into `partials` (at most kRedBlocks
// blocks of kRedK values), then k_finish sums them into the device array out.
static hipError_t launch_dot(int nv, const double* x, const DotArgs& A, bool al, long n,
                             double* partials, double* out, hipStream_t s) {
  dim3 g(dot_grid(n, al)), b(256);
  if (al) {
    switch (nv) {
#define DP_CASE(K) case K: hipLaunchKernelGGL(k_dot_prod_multi<K>, g, b, 0, s, n, x, A, partials); break;
      DP_CASE(1) DP_CASE(2) DP_CASE(3) DP_CASE(4) DP_CASE(5) DP_CASE(6) DP_CASE(7) DP_CASE(8)
#undef DP_CASE
    }
  } else {
    switch (nv) {
#define DP_CASE(K) case K: hipLaunchKernelGGL(k_dot_prod_multi_u<K>, g, b, 0, s, n, x, A, partials); break;
      DP_CASE(1) DP_CASE(2) DP_CASE(3) DP_CASE(4) DP_CASE(5) DP_CASE(6) DP_CASE(7) DP_CASE(8)
#undef DP_CASE
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, nv, g.x, 0, n, partials, out);
  return hipGetLastError();
}

// out[0..k) = 0 (a kernel rather than a memset, so that it can be captured)
__global__ void k_zero(int k, double* out) {
  if ((int)threadIdx.x < k) out[threadIdx.x] = 0.0;
}

}  // namespace bdfgpu

using namespace bdfgpu;

extern "C" {

const char* bdfgpu_last_error(void) {
  std::lock_guard<std::mutex> lk(g_err_mu);
  static thread_local std::string copy;
  copy = g_last_error_global;
  return copy.c_str();
}

const char* bdfgpu_version(void) { return "bdfgpu 0.1 gfx950"; }

int nvec_linear_sum(long n, double a, const double* x, double b, const double* y, double* z,
                    void* stream) {
  if (n < 0 || (n > 0 && (!x || !y || !z))) return arg_error("nvec_linear_sum: bad argument");
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  long n2 = 0;
  if (aligned16(x) && aligned16(y) && aligned16(z)) {
    n2 = n >> 1;
    if (n2)
      hipLaunchKernelGGL(k_linear_sum2, dim3(stream_blocks(n2)), dim3(kStreamThreads), 0, s, n2, a,
                         x, b, y, z);
  }
  if (2 * n2 < n)
    hipLaunchKernelGGL(k_linear_sum1, dim3(stream_blocks(n - 2 * n2)), dim3(kStreamThreads), 0, s,
                       n, 2 * n2, a, x, b, y, z);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int nvec_linear_combination(int nv, const double* c, const double* const* X, double* z, long n,
                            void* stream) {
  if (nv < 1 || nv > 16 || n < 0 || !c || !X) return arg_error("nvec_linear_combination: bad nv/args");
  if (n == 0) return 0;
  LcArgs A;
  memset(&A, 0, sizeof(A));
  bool al = aligned16(z);
  for (int j = 0; j < nv; ++j) {
    if (!X[j]) return arg_error("nvec_linear_combination: null vector");
    A.X[j] = X[j];
    A.c[j] = c[j];
    al = al && aligned16(X[j]);
  }
  hipStream_t s = as_stream(stream);
  long n2 = 0;
  if (al) {
    n2 = n >> 1;
    // 12 or more vectors: whole 8192-unit chunks in the long-run form, the rest in the tile form
    // on pointers advanced past them (16-byte alignment is kept)
    const long nchunks = nv >= 12 ? std::min(n2 / kLcChunk, 1L << 24) : 0;
    if (nchunks) {
      dim3 g((unsigned int)nchunks), b(kStreamThreads);
      switch (nv) {
#define LC_CASE(K) case K: hipLaunchKernelGGL(k_linear_combination_runs<K>, g, b, 0, s, n2, A, z); break;
        LC_CASE(12) LC_CASE(13) LC_CASE(14) LC_CASE(15) LC_CASE(16)
#undef LC_CASE
      }
    }
    const long done = nchunks * kLcChunk, rest = n2 - done;
    LcArgs R = A;
    for (int j = 0; j < nv; ++j) R.X[j] = A.X[j] + 2 * done;
    double* zr = z + 2 * done;
    dim3 g(stream_blocks(rest)), b(kStreamThreads);
    if (rest) switch (nv) {
#define LC_CASE(K) case K: hipLaunchKernelGGL(k_linear_combination2<K>, g, b, 0, s, rest, R, zr); break;
      LC_CASE(1) LC_CASE(2) LC_CASE(3) LC_CASE(4) LC_CASE(5) LC_CASE(6) LC_CASE(7) LC_CASE(8)
      LC_CASE(9) LC_CASE(10) LC_CASE(11) LC_CASE(12) LC_CASE(13) LC_CASE(14) LC_CASE(15) LC_CASE(16)
#undef LC_CASE
    }
  }
  if (2 * n2 < n)
    hipLaunchKernelGGL(k_linear_combination1, dim3(stream_blocks(n - 2 * n2)), dim3(kStreamThreads),
                       0, s, nv, n, 2 * n2, A, z);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int nvec_scale_add_multi(int nv, const double* a, const double* x, const double* const* Y,
                         double* const* Z, long n, void* stream) {
  if (nv < 1 || nv > 8 || n < 0 || !a || !Y || !Z || (n > 0 && !x))
    return arg_error("nvec_scale_add_multi: bad nv/args");
  if (n == 0) return 0;
  SamArgs A;
  memset(&A, 0, sizeof(A));
  bool al = aligned16(x);
  for (int j = 0; j < nv; ++j) {
    if (!Y[j] || !Z[j]) return arg_error("nvec_scale_add_multi: null vector");
    A.Y[j] = Y[j];
    A.Z[j] = Z[j];
    A.a[j] = a[j];
    al = al && aligned16(Y[j]) && aligned16(Z[j]);
  }
  hipStream_t s = as_stream(stream);
  long n2 = 0;
  if (al) {
    n2 = n >> 1;
    dim3 g(stream_blocks(n2)), b(kStreamThreads);
    if (n2) switch (nv) {
#define SAM_CASE(K) case K: hipLaunchKernelGGL(k_scale_add_multi2<K>, g, b, 0, s, n2, x, A); break;
      SAM_CASE(1) SAM_CASE(2) SAM_CASE(3) SAM_CASE(4) SAM_CASE(5) SAM_CASE(6) SAM_CASE(7) SAM_CASE(8)
#undef SAM_CASE
    }
  }
  if (2 * n2 < n)
    hipLaunchKernelGGL(k_scale_add_multi1, dim3(stream_blocks(n - 2 * n2)), dim3(kStreamThreads), 0,
                       s, nv, n, 2 * n2, x, A);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int nvec_dot_prod_multi(int nv, const double* x, const double* const* Y, double* d, long n,
                        int flags, void* stream) {
  if (nv < 1 || nv > 8 || n < 0 || !Y || !d || (n > 0 && !x))
    return arg_error("nvec_dot_prod_multi: bad nv/args");
  hipStream_t s = as_stream(stream);
  if (n == 0) {
    if (flags & BDFGPU_RESULT_DEVICE) {
      BDF_HIP_TRY(hipMemsetAsync(d, 0, sizeof(double) * nv, s));
    } else {
      for (int j = 0; j < nv; ++j) d[j] = 0.0;
    }
    return 0;
  }
  RedScratch* r = nullptr;
  int st = get_red_scratch(&r);
  if (st) return st;
  DotArgs A;
  memset(&A, 0, sizeof(A));
  bool al = aligned16(x);
  for (int j = 0; j < nv; ++j) {
    if (!Y[j]) return arg_error("nvec_dot_prod_multi: null vector");
    A.Y[j] = Y[j];
    al = al && aligned16(Y[j]);
  }
  BDF_HIP_TRY(launch_dot(nv, x, A, al, n, r->partials, finish_target(r, d, flags), s));
  return finish_reduction(r, nv, d, flags, s);
}

int nvec_dot_prod_multi_noalloc(int nv, const double* x, const double* const* Y, double* d,
                                long n, void* stream) {
  if (nv < 1 || nv > kRedK || n < 0 || !Y || !d || (n > 0 && !x))
    return arg_error("nvec_dot_prod_multi_noalloc: bad argument (1 <= nv <= 8, device d)");
  hipStream_t s = as_stream(stream);
  if (n == 0) {
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, nv, d);
    BDF_HIP_TRY(hipGetLastError());
    return 0;
  }
  double* partials = nullptr;
  int st = get_static_scratch(&partials);
  if (st) return st;
  DotArgs A;
  memset(&A, 0, sizeof(A));
  bool al = aligned16(x);
  for (int j = 0; j < nv; ++j) {
    if (!Y[j]) return arg_error("nvec_dot_prod_multi_noalloc: null vector");
    A.Y[j] = Y[j];
    al = al && aligned16(Y[j]);
  }
  if (dot_grid(n, al) > (unsigned int)kRedBlocks)
    return arg_error("nvec_dot_prod_multi_noalloc: reduction grid exceeds the static scratch");
  BDF_HIP_TRY(launch_dot(nv, x, A, al, n, partials, d, s));
  return 0;
}

int nvec_wrms_norm(long n, const double* x, const double* w, double* out, int flags,
                   void* stream) {
  if (n < 0 || !out || (n > 0 && (!x || !w))) return arg_error("nvec_wrms_norm: bad argument");
  hipStream_t s = as_stream(stream);
  if (n == 0) {
    if (flags & BDFGPU_RESULT_DEVICE) {
      BDF_HIP_TRY(hipMemsetAsync(out, 0, sizeof(double), s));
    } else {
      *out = 0.0;
    }
    return 0;
  }
  RedScratch* r = nullptr;
  int st = get_red_scratch(&r);
  if (st) return st;
  bool al = aligned16(x) && aligned16(w);
  dim3 g(al ? red_blocks(n >> 1) : red_blocks(n, true)), b(256);
  if (al)
    hipLaunchKernelGGL(k_wrms, g, b, 0, s, n, x, w, r->partials);
  else
    hipLaunchKernelGGL(k_wrms_u, g, b, 0, s, n, x, w, r->partials);
  BDF_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, 1, g.x, 1, n, r->partials,
                     finish_target(r, out, flags));
  BDF_HIP_TRY(hipGetLastError());
  return finish_reduction(r, 1, out, flags, s);
}

int nvec_wrms_norm_multi(int nv, const double* const* X, const double* const* Wt, double* nrm,
                         long n, int flags, void* stream) {
  if (nv < 1 || nv > 8 || n < 0 || !X || !Wt || !nrm)
    return arg_error("nvec_wrms_norm_multi: bad argument (1 <= nv <= 8)");
  hipStream_t s = as_stream(stream);
  if (n == 0) {
    if (flags & BDFGPU_RESULT_DEVICE) {
      hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, nv, nrm);
      BDF_HIP_TRY(hipGetLastError());
    } else {
      for (int j = 0; j < nv; ++j) nrm[j] = 0.0;
    }
    return 0;
  }
  RedScratch* r = nullptr;
  int st = get_red_scratch(&r);
  if (st) return st;
  WrmsArgs A;
  memset(&A, 0, sizeof(A));
  bool al = true, shw = true;
  for (int j = 0; j < nv; ++j) {
    if (!X[j] || !Wt[j]) return arg_error("nvec_wrms_norm_multi: null vector");
    A.X[j] = X[j];
    A.W[j] = Wt[j];
    al = al && aligned16(X[j]) && aligned16(Wt[j]);
    shw = shw && Wt[j] == Wt[0];
  }
  dim3 g(al ? red_blocks(n >> 1) : red_blocks(n, true)), b(256);
  if (al && shw) {
    switch (nv) {
#define WM_CASE(K) case K: hipLaunchKernelGGL((k_wrms_multi<K, true>), g, b, 0, s, n, A, r->partials); break;
      WM_CASE(1) WM_CASE(2) WM_CASE(3) WM_CASE(4) WM_CASE(5) WM_CASE(6) WM_CASE(7) WM_CASE(8)
#undef WM_CASE
    }
  } else if (al) {
    switch (nv) {
#define WM_CASE(K) case K: hipLaunchKernelGGL((k_wrms_multi<K, false>), g, b, 0, s, n, A, r->partials); break;
      WM_CASE(1) WM_CASE(2) WM_CASE(3) WM_CASE(4) WM_CASE(5) WM_CASE(6) WM_CASE(7) WM_CASE(8)
#undef WM_CASE
    }
  } else {
    switch (nv) {
#define WM_CASE(K) case K: hipLaunchKernelGGL(k_wrms_multi_u<K>, g, b, 0, s, n, A, r->partials); break;
      WM_CASE(1) WM_CASE(2) WM_CASE(3) WM_CASE(4) WM_CASE(5) WM_CASE(6) WM_CASE(7) WM_CASE(8)
#undef WM_CASE
    }
  }
  BDF_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, nv, g.x, 1, n, r->partials,
                     finish_target(r, nrm, flags));
  BDF_HIP_TRY(hipGetLastError());
  return finish_reduction(r, nv, nrm, flags, s);
}

int nvec_max_norm(long n, const double* x, double* out, int flags, void* stream) {
  if (n < 0 || !out || (n > 0 && !x)) return arg_error("nvec_max_norm: bad argument");
  hipStream_t s = as_stream(stream);
  if (n == 0) {
    if (flags & BDFGPU_RESULT_DEVICE) {
      BDF_HIP_TRY(hipMemsetAsync(out, 0, sizeof(double), s));
    } else {
      *out = 0.0;
    }
    return 0;
  }
  RedScratch* r = nullptr;
  int st = get_red_scratch(&r);
  if (st) return st;
  const unsigned int gm = red_blocks(n, true);
  hipLaunchKernelGGL(k_maxnorm, dim3(gm), dim3(256), 0, s, n, x, r->partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, 1, gm, 2, n, r->partials,
                     finish_target(r, out, flags));
  BDF_HIP_TRY(hipGetLastError());
  return finish_reduction(r, 1, out, flags, s);
}

int nvec_ewt(long n, double rtol, double atol, const double* y, double* w, void* stream) {
  if (n < 0 || (n > 0 && (!y || !w))) return arg_error("nvec_ewt: bad argument");
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  const long n2 = (aligned16(y) && aligned16(w)) ? n >> 1 : 0;
  if (n2)
    hipLaunchKernelGGL(k_ewt2, dim3(map_blocks(n2)), dim3(kMapThreads), 0, s, n2, rtol, atol, y, w);
  if (2 * n2 < n)
    hipLaunchKernelGGL(k_ewt, dim3(map_blocks(n - 2 * n2)), dim3(kMapThreads), 0, s, n, 2 * n2,
                       rtol, atol, y, w);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int nvec_scale(long n, double c, const double* x, double* z, void* stream) {
  if (n < 0 || (n > 0 && (!x || !z))) return arg_error("nvec_scale: bad argument");
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  const long n2 = (aligned16(x) && aligned16(z)) ? n >> 1 : 0;
  if (n2) hipLaunchKernelGGL(k_scale2, dim3(map_blocks(n2)), dim3(kMapThreads), 0, s, n2, c, x, z);
  if (2 * n2 < n)
    hipLaunchKernelGGL(k_scale, dim3(map_blocks(n - 2 * n2)), dim3(kMapThreads), 0, s, n, 2 * n2,
                       c, x, z);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int nvec_const(long n, double c, double* z, void* stream) {
  if (n < 0 || (n > 0 && !z)) return arg_error("nvec_const: bad argument");
  if (n == 0) return 0;
  hipStream_t s = as_stream(stream);
  const long n2 = aligned16(z) ? n >> 1 : 0;
  if (n2) hipLaunchKernelGGL(k_const2, dim3(map_blocks(n2)), dim3(kMapThreads), 0, s, n2, c, z);
  if (2 * n2 < n)
    hipLaunchKernelGGL(k_const, dim3(map_blocks(n - 2 * n2)), dim3(kMapThreads), 0, s, n, 2 * n2,
                       c, z);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

}  // extern "C"
