// Shared device/host helpers for the gfx950 kernels of the batched BDF path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "../../include/bdfgpu.h"

namespace bdfgpu {

#define BDF_HIP_TRY(expr)                                                    \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      bdfgpu::set_last_error(hipGetErrorString(e_), __FILE__, __LINE__);     \
      return BDFGPU_ERR_HIP;                                                 \
    }                                                                        \
  } while (0)

void set_last_error(const char* msg, const char* file, int line);
// Records msg as the last error and returns BDFGPU_ERR_ARG.
int arg_error(const char* msg);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Wave and block reductions (fixed order: results are deterministic for a
// given launch shape)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Sum K values over the block.  `sh` must hold (blockDim.x / 64) * K doubles.
// Result valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[wid * K + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[w * K + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

inline unsigned int ceil_div(long a, long b) { return (unsigned int)((a + b - 1) / b); }

}  // namespace bdfgpu
