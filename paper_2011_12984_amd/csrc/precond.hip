// Learned block preconditioner: a small MLP that maps a cell's state and
// log(gamma) to an approximate inverse X ~ (I - gamma J)^-1, trained on the
// GPU with the kernels below.
//
// Network: x = standardised [y (n), log gamma] -> ReLU(W1 x + b1) ->
// ReLU(W2 . + b2) -> W3 . + b3 = out, X = I + reshape(out) (row-major).
// Every matrix product takes BF16 operands (weights and activations rounded
// to nearest even from FP32) and accumulates in FP32.  Inference uses
// gfx950 MFMA (v_mfma_f32_32x32x16_bf16); training uses FP32 vector kernels
// with the same rounding points, and FP32 master weights with Adam.
//
// Loss: mean over the batch of |X M - I|_F^2 / n^2, so the relative error of
// a preconditioned Newton correction X r against the exact M^-1 r is bounded
// by |X M - I|.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace bdfgpu {

// ---------------------------------------------------------------------------
// BF16 helpers (round to nearest even, NaN kept quiet)
// ---------------------------------------------------------------------------
__host__ __device__ inline unsigned short f2bf(float x) {
  unsigned int u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) {
    if (u & 0x007fffffu) u |= 0x00400000u;
    return (unsigned short)(u >> 16);
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__host__ __device__ inline float bf2f(unsigned short b) {
  unsigned int u = ((unsigned int)b) << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__device__ __forceinline__ float bfr(float x) { return bf2f(f2bf(x)); }

struct Precond {
  int n, nin, hid, nout;
  long np;                       // total parameters
  float* params = nullptr;       // FP32 master: W1 | b1 | W2 | b2 | W3 | b3
  float* grads = nullptr;
  double* m1 = nullptr;
  double* m2 = nullptr;
  long adam_t = 0;
  double* in_mean = nullptr;     // nin
  double* in_std = nullptr;
  // padded BF16 copies for the MFMA forward
  unsigned short* w1b = nullptr; // hid x 32
  unsigned short* w2b = nullptr; // hid x hid
  unsigned short* w3b = nullptr; // nout_pad x hid
  int nout_pad;
  bool dirty = true;
  // training scratch for one batch
  int bcap = 0;
  float *xs = nullptr, *a1 = nullptr, *h1 = nullptr, *a2 = nullptr, *h2 = nullptr, *out = nullptr;
  float *dout = nullptr, *dh = nullptr, *dh2 = nullptr;
  double* lossbuf = nullptr;
  double* statpart = nullptr;    // kStatBlocks x nin partial column sums
  double* bx = nullptr;          // gathered batch inputs
  double* bm = nullptr;          // gathered batch blocks
  std::vector<void*> allocs;
  long off_W1, off_b1, off_W2, off_b2, off_W3, off_b3;
};

static int pc_alloc(Precond* p, void** ptr, size_t bytes) {
  BDF_HIP_TRY(hipMalloc(ptr, bytes < 16 ? 16 : bytes));
  p->allocs.push_back(*ptr);
  return 0;
}

// ---------------------------------------------------------------------------
// Training kernels (FP32 vector arithmetic)
// ---------------------------------------------------------------------------

// C[M x N] (ldc) = alpha * op(A) op(B) (+ C if accumulate), row-major
// operands; op(A)[m][k] = ta ? A[k*lda + m] : A[m*lda + k]; likewise B.
// ra, rb: round the A, B elements to BF16 before the product.
constexpr int kGT = 64, kGK = 16;
__global__ void __launch_bounds__(256) k_gemm_f32(int M, int N, int K, const float* A, int lda,
                                                  int ta, const float* B, int ldb, int tb,
                                                  float* C, int ldc, int ra, int rb,
                                                  int accumulate) {
  __shared__ float sA[kGK][kGT + 1];
  __shared__ float sB[kGK][kGT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int k0 = 0; k0 < K; k0 += kGK) {
    for (int e = threadIdx.x; e < kGK * kGT; e += 256) {
      const int kk = e / kGT, mm = e % kGT;
      const int m = m0 + mm, k = k0 + kk;
      float a = 0.f;
      if (m < M && k < K) a = ta ? A[(long)k * lda + m] : A[(long)m * lda + k];
      sA[kk][mm] = ra ? bfr(a) : a;
      const int nn = mm, n = n0 + nn;
      float b = 0.f;
      if (n < N && k < K) b = tb ? B[(long)n * ldb + k] : B[(long)k * ldb + n];
      sB[kk][nn] = rb ? bfr(b) : b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= N) continue;
      float v = acc[i][j];
      if (accumulate) v += C[(long)m * ldc + n];
      C[(long)m * ldc + n] = v;
    }
  }
}

// standardise raw inputs (FP64) and round to BF16: xs[b][i]
__global__ void k_standardise(int B, int nin, const double* X, const double* mean,
                              const double* stdv, float* xs) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * nin) return;
  const int i = (int)(t % nin);
  xs[t] = bfr((float)((X[t] - mean[i]) / stdv[i]));
}

// a = pre-activation (+ bias), h = BF16(ReLU(a))
__global__ void k_bias_relu(int B, int N, float* a, const float* bias, float* h) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * N) return;
  const float v = a[t] + bias[t % N];
  a[t] = v;
  h[t] = bfr(v > 0.f ? v : 0.f);
}

__global__ void k_bias_add(int B, int N, float* a, const float* bias) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * N) return;
  a[t] += bias[t % N];
}

// Per sample: X = I + out (row-major n x n), M column-major; E = X M - I;
// loss += |E|^2 * scale; dout = 2 E M^T * scale.  One 64-thread block per
// sample; FP64 arithmetic for the small products.
__global__ void __launch_bounds__(64) k_loss_grad(int B, int n, const float* out, const double* M,
                                                  float* dout, double* loss_part, double scale) {
  const int b = blockIdx.x;
  const int nn = n * n;
  __shared__ double sX[32 * 32];
  __shared__ double sE[32 * 32];
  __shared__ double sL[64];
  const float* o = out + (long)b * nn;
  const double* Mb = M + (long)b * nn;
  for (int e = threadIdx.x; e < nn; e += 64) {
    const int i = e / n, j = e % n;
    sX[i * n + j] = (double)o[e] + (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  double l = 0.0;
  for (int e = threadIdx.x; e < nn; e += 64) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += sX[i * n + k] * Mb[k + j * n];
    s -= (i == j ? 1.0 : 0.0);
    sE[i * n + j] = s;
    l += s * s * scale;
  }
  sL[threadIdx.x] = l;
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += 64) {
    const int i = e / n, k = e % n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += sE[i * n + j] * Mb[k + j * n];
    dout[(long)b * nn + e] = (float)(2.0 * s * scale);
  }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 64; ++k) t += sL[k];
    loss_part[b] = t;
  }
}

// column sums: g[n] (+)= sum_b D[b][n]
// g[j] = sum_b D[b][j] (bias gradients).  A block of 1024 threads takes
// 64 columns; thread (slice s, column j) sums rows s, s + 16, ... in order,
// then the 16 slices are summed in order.
__global__ void __launch_bounds__(1024) k_colsum(int B, int N, const float* D, float* g) {
  __shared__ float sh[16][64];
  const int cj = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + cj;
  float a = 0.f;
  if (j < N)
    for (int b = sl; b < B; b += 16) a += D[(long)b * N + j];
  sh[sl][cj] = a;
  __syncthreads();
  if (sl == 0 && j < N) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += sh[k][cj];
    g[j] = t;
  }
}

// dh = dh * (a > 0)
__global__ void k_relu_bwd(long total, float* dh, const float* a) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < total && !(a[t] > 0.f)) dh[t] = 0.f;
}

__global__ void k_sum_loss(int B, const double* part, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += part[b];
    out[0] = s;
  }
}

// Adam (Kingma & Ba) on FP32 master weights with FP64 moments.
__global__ void k_adam(long np, float* p, const float* g, double* m1, double* m2, double lr,
                       double b1, double b2, double eps, double c1, double c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const double gi = (double)g[i];
  const double a = b1 * m1[i] + (1.0 - b1) * gi;
  const double v = b2 * m2[i] + (1.0 - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  p[i] = (float)((double)p[i] - lr * (a / c1) / (sqrt(v / c2) + eps));
}

// gather rows of a batch: dst[b][*] = src[perm[b]][*]
__global__ void k_gather(int B, int w, const double* src, const int* perm, double* dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * w) return;
  const long b = t / w;
  const int i = (int)(t - b * w);
  dst[t] = src[(long)perm[b] * w + i];
}

// per-column mean and standard deviation over ns samples (one thread per
// column, FP64 two-pass)
// Column statistics of an ns x w FP64 matrix (w <= 32) in two passes, each
// a per-block partial over a fixed chunk of rows (pass 0: sum of x; pass 1:
// sum of (x - mean)^2) and one finishing block that sums the partials in
// block order.  Thread t of a block takes column t % w of rows t / w,
// t / w + 256 / w, ...; the block then sums its rows per column in order.
constexpr int kStatBlocks = 1024;
__global__ void __launch_bounds__(256) k_col_partial(long ns, int w, int pass, const double* X,
                                                     const double* mean, double* part) {
  __shared__ double sh[256];
  const int t = threadIdx.x, rpi = 256 / w, c = t % w, rl = t / w;
  const long chunk = (ns + gridDim.x - 1) / gridDim.x;
  const long r0 = (long)blockIdx.x * chunk;
  const long r1 = r0 + chunk < ns ? r0 + chunk : ns;
  double acc = 0.0;
  if (rl < rpi) {
    const double mu = pass ? mean[c] : 0.0;
    for (long r = r0 + rl; r < r1; r += rpi) {
      const double v = X[r * w + c];
      acc += pass ? (v - mu) * (v - mu) : v;
    }
  }
  sh[t] = acc;
  __syncthreads();
  if (t < w) {
    double a = 0.0;
    for (int j = 0; j < rpi; ++j) a += sh[j * w + t];
    part[(long)blockIdx.x * w + t] = a;
  }
}

__global__ void k_col_finish(int nb, long ns, int w, int pass, const double* part, double* mean,
                             double* stdv) {
  const int c = threadIdx.x;
  if (c >= w) return;
  double a = 0.0;
  for (int b = 0; b < nb; ++b) a += part[(long)b * w + c];
  if (pass == 0) {
    mean[c] = a / (double)ns;
  } else {
    const double sd = sqrt(a / (double)(ns > 1 ? ns : 1));
    stdv[c] = sd > 1e-12 ? sd : 1.0;
  }
}

// FP32 master weights -> padded BF16 copies for inference
__global__ void k_pack_bf16(int rows, int cols, int rows_pad, int cols_pad, const float* W,
                            unsigned short* Wb) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)rows_pad * cols_pad) return;
  const int r = (int)(t / cols_pad), c = (int)(t % cols_pad);
  Wb[t] = (r < rows && c < cols) ? f2bf(W[(long)r * cols + c]) : (unsigned short)0;
}

// ---------------------------------------------------------------------------
// Inference.  Two paths with the same rounding points: a vector-FMA path
// (reference) and the MFMA path.  Inputs: raw x (B x nin, FP64).  Output:
// X = I + out (B x nout, FP32, row-major n x n per sample).
// ---------------------------------------------------------------------------

// vector path: one thread per (sample, output) of each layer
__global__ void k_fwd_layer_vec(int B, int K, int N, const float* in, const float* W,
                                const float* bias, float* outp, int relu_bf16, int add_eye, int n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * N) return;
  const long b = t / N;
  const int o = (int)(t - b * N);
  float s = 0.f;
  for (int k = 0; k < K; ++k) s = fmaf(bfr(W[(long)o * K + k]), in[b * K + k], s);
  s += bias[o];
  if (relu_bf16) s = bfr(s > 0.f ? s : 0.f);
  if (add_eye && (o / n) == (o % n)) s += 1.0f;
  outp[t] = s;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kMlpHid = 256;
constexpr int kMlpRowPad = kMlpHid + 8;   // LDS row stride (bf16 elements)

// MFMA path.  One wavefront owns 32 samples end to end; its activations
// (32 x 256 BF16) stay in LDS.  v_mfma_f32_32x32x16_bf16 lane layout:
// A: lane l holds A[l % 32][8 (l / 32) + 0..7]; B: lane l holds
// B[8 (l / 32) + 0..7][l % 32]; C: lane l holds column l % 32, rows
// 8 (v / 4) + 4 (l / 32) + v % 4 for v = 0..15.
// Two waves per SIMD (256 registers, the accumulators in VGPRs, a few
// spills around the output stores): 2.26 -> 2.06 ms per 2^20 samples against
// one wave per SIMD with the accumulators in AGPRs.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_mlp_fwd_mfma(long B, int n, const double* X,
                                                      const double* mean, const double* stdv,
                                                      const unsigned short* w1b, const float* b1,
                                                      const unsigned short* w2b, const float* b2,
                                                      const unsigned short* w3b, const float* b3,
                                                      int nout, int nout_pad, float* out,
                                                      const int* gphase, int want,
                                                      const int* gskip) {
  __shared__ unsigned short act[4][32 * kMlpRowPad];
  // optional gate on integrator state (device memory): run only in phase
  // `want` and when not skipped
  if (gphase && (*gphase != want || *gskip != 0)) return;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const long s0 = ((long)blockIdx.x * 4 + wave) * 32;     // first sample of this wave
  unsigned short* A = act[wave];
  const int nin = n + 1;
  // input: 32 samples x 32 (zero padded) standardised BF16 values
  for (int e = l; e < 32 * 32; e += 64) {
    const int r = e >> 5, c = e & 31;
    const long s = s0 + r;
    float v = 0.f;
    if (s < B && c < nin) v = (float)((X[s * nin + c] - mean[c]) / stdv[c]);
    A[r * kMlpRowPad + c] = f2bf(v);
  }
  __syncthreads();
  const int row = l & 31, kh = l >> 5;
  // The block's four waves split each layer's output tiles and compute
  // them for all 128 samples of the block (every wave's activations are in
  // LDS), so every weight fragment loaded from L2 feeds four MFMAs.  Each
  // output's MFMA sequence over k is the one a single wave would run.
  unsigned short* Ap[4] = {act[0], act[1], act[2], act[3]};
  // ---- layer 1 (K = 32) and layer 2 (K = 256): 8 output tiles, 2 per wave
  for (int layer = 0; layer < 2; ++layer) {
    const int K = layer == 0 ? 32 : kMlpHid;
    const unsigned short* W = layer == 0 ? w1b : w2b;
    const float* bias = layer == 0 ? b1 : b2;
    f32x16 acc[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][g][v] = 0.f;
    // weight fragments of the next k step are loaded while this step's
    // MFMAs run (without the overlap every MFMA waited for its own load)
    const unsigned short* Wl = W + (long)(wave * 2 * 32 + row) * K + 8 * kh;
    bf16x8 bcur[2], bnext[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) bcur[t] = *reinterpret_cast<const bf16x8*>(&Wl[(long)t * 32 * K]);
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x8 a[4];
#pragma unroll
      for (int g = 0; g < 4; ++g)
        a[g] = *reinterpret_cast<const bf16x8*>(&Ap[g][row * kMlpRowPad + k0 + 8 * kh]);
      const int kn = k0 + 16 < K ? k0 + 16 : k0;   // (the last step reloads its own)
#pragma unroll
      for (int t = 0; t < 2; ++t)
        bnext[t] = *reinterpret_cast<const bf16x8*>(&Wl[(long)t * 32 * K + kn]);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int g = 0; g < 4; ++g)
          acc[t][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[g], bcur[t], acc[t][g], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < 2; ++t) bcur[t] = bnext[t];
    }
    __syncthreads();   // every lane finished reading this layer's input
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int col = (wave * 2 + t) * 32 + row;
      const float bb = bias[col];
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int r = 8 * (v >> 2) + 4 * kh + (v & 3);
          const float x = acc[t][g][v] + bb;
          Ap[g][r * kMlpRowPad + col] = f2bf(x > 0.f ? x : 0.f);
        }
    }
    __syncthreads();
  }
  // ---- layer 3 (K = 256, nout_pad / 32 output tiles, split in four
  // contiguous ranges; tiles two at a time, the next k step's weight
  // fragments loading during the current MFMAs)
  const int ntile = nout_pad / 32;
  const int tb = ntile * wave / 4, te = ntile * (wave + 1) / 4;
  for (int t0 = tb; t0 < te; t0 += 2) {
    f32x16 acc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[u][g][v] = 0.f;
    // a second tile past this wave's range reads the first tile's rows (in
    // bounds); its MFMAs are skipped
    const bool two = t0 + 1 < te;
    const unsigned short* W0 = w3b + (long)(t0 * 32 + row) * kMlpHid + 8 * kh;
    const unsigned short* W1 = two ? W0 + 32L * kMlpHid : W0;
    bf16x8 c0 = *reinterpret_cast<const bf16x8*>(W0);
    bf16x8 c1 = *reinterpret_cast<const bf16x8*>(W1);
    for (int k0 = 0; k0 < kMlpHid; k0 += 16) {
      bf16x8 a[4];
#pragma unroll
      for (int g = 0; g < 4; ++g)
        a[g] = *reinterpret_cast<const bf16x8*>(&Ap[g][row * kMlpRowPad + k0 + 8 * kh]);
      const int kn = k0 + 16 < kMlpHid ? k0 + 16 : k0;
      const bf16x8 n0 = *reinterpret_cast<const bf16x8*>(W0 + kn);
      const bf16x8 n1 = *reinterpret_cast<const bf16x8*>(W1 + kn);
#pragma unroll
      for (int g = 0; g < 4; ++g)
        acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[g], c0, acc[0][g], 0, 0, 0);
      if (two) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
          acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[g], c1, acc[1][g], 0, 0, 0);
      }
      c0 = n0;
      c1 = n1;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int col = (t0 + u) * 32 + row;
      if (col >= nout || (u == 1 && !two)) continue;
      const float bb = b3[col];
      const bool diag = (col / n) == (col % n);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const long sg = ((long)blockIdx.x * 4 + g) * 32;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const long s = sg + 8 * (v >> 2) + 4 * kh + (v & 3);
          if (s < B) out[s * nout + col] = acc[u][g][v] + bb + (diag ? 1.0f : 0.0f);
        }
      }
    }
  }
}

static int refresh_inference_weights(Precond* p, hipStream_t s) {
  if (!p->dirty) return 0;
  const float* P = p->params;
  hipLaunchKernelGGL(k_pack_bf16, dim3(ceil_div((long)p->hid * 32, 256)), dim3(256), 0, s, p->hid,
                     p->nin, p->hid, 32, P + p->off_W1, p->w1b);
  hipLaunchKernelGGL(k_pack_bf16, dim3(ceil_div((long)p->hid * p->hid, 256)), dim3(256), 0, s,
                     p->hid, p->hid, p->hid, p->hid, P + p->off_W2, p->w2b);
  hipLaunchKernelGGL(k_pack_bf16, dim3(ceil_div((long)p->nout_pad * p->hid, 256)), dim3(256), 0,
                     s, p->nout, p->hid, p->nout_pad, p->hid, P + p->off_W3, p->w3b);
  BDF_HIP_TRY(hipGetLastError());
  p->dirty = false;
  return 0;
}

int precond_infer(Precond* p, long B, const double* X, float* out, int use_mfma, hipStream_t s,
                  const int* gphase = nullptr, int want = 0, const int* gskip = nullptr) {
  if (B <= 0) return 0;
  int st = refresh_inference_weights(p, s);
  if (st) return st;
  const float* P = p->params;
  if (use_mfma) {
    hipLaunchKernelGGL(k_mlp_fwd_mfma, dim3(ceil_div(B, 128)), dim3(256), 0, s, B, p->n, X,
                       p->in_mean, p->in_std, p->w1b, P + p->off_b1, p->w2b, P + p->off_b2,
                       p->w3b, P + p->off_b3, p->nout, p->nout_pad, out, gphase, want, gskip);
    BDF_HIP_TRY(hipGetLastError());
    return 0;
  }
  // vector path, in chunks that fit the batch scratch
  const long chunk = p->bcap;
  for (long b0 = 0; b0 < B; b0 += chunk) {
    const int bb = (int)std::min<long>(chunk, B - b0);
    hipLaunchKernelGGL(k_standardise, dim3(ceil_div((long)bb * p->nin, 256)), dim3(256), 0, s, bb,
                       p->nin, X + b0 * p->nin, p->in_mean, p->in_std, p->xs);
    hipLaunchKernelGGL(k_fwd_layer_vec, dim3(ceil_div((long)bb * p->hid, 256)), dim3(256), 0, s,
                       bb, p->nin, p->hid, p->xs, P + p->off_W1, P + p->off_b1, p->h1, 1, 0, p->n);
    hipLaunchKernelGGL(k_fwd_layer_vec, dim3(ceil_div((long)bb * p->hid, 256)), dim3(256), 0, s,
                       bb, p->hid, p->hid, p->h1, P + p->off_W2, P + p->off_b2, p->h2, 1, 0, p->n);
    hipLaunchKernelGGL(k_fwd_layer_vec, dim3(ceil_div((long)bb * p->nout, 256)), dim3(256), 0, s,
                       bb, p->hid, p->nout, p->h2, P + p->off_W3, P + p->off_b3,
                       out + b0 * p->nout, 0, 1, p->n);
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

// C = op(A) op(B); rbw: round the B operand (the weights) to BF16.
static void gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, int ta,
                 const float* B, int ldb, int tb, float* C, int ldc, int rbw, int acc) {
  dim3 g(ceil_div(N, kGT), ceil_div(M, kGT)), b(256);
  hipLaunchKernelGGL(k_gemm_f32, g, b, 0, s, M, N, K, A, lda, ta, B, ldb, tb, C, ldc, 0, rbw, acc);
}

// Loss and gradients of one batch (bx: B x nin raw inputs, bm: B blocks).
static int loss_grad(Precond* p, int B, const double* bx, const double* bm, hipStream_t s) {
  const int nin = p->nin, H = p->hid, NO = p->nout;
  float* P = p->params;
  float* Gd = p->grads;
  hipLaunchKernelGGL(k_standardise, dim3(ceil_div((long)B * nin, 256)), dim3(256), 0, s, B, nin,
                     bx, p->in_mean, p->in_std, p->xs);
  // forward with BF16 operands (weights rounded on load; activations are
  // already BF16 values)
  gemm(s, B, H, nin, p->xs, nin, 0, P + p->off_W1, nin, 1, p->a1, H, 1, 0);
  hipLaunchKernelGGL(k_bias_relu, dim3(ceil_div((long)B * H, 256)), dim3(256), 0, s, B, H, p->a1,
                     P + p->off_b1, p->h1);
  gemm(s, B, H, H, p->h1, H, 0, P + p->off_W2, H, 1, p->a2, H, 1, 0);
  hipLaunchKernelGGL(k_bias_relu, dim3(ceil_div((long)B * H, 256)), dim3(256), 0, s, B, H, p->a2,
                     P + p->off_b2, p->h2);
  gemm(s, B, NO, H, p->h2, H, 0, P + p->off_W3, H, 1, p->out, NO, 1, 0);
  hipLaunchKernelGGL(k_bias_add, dim3(ceil_div((long)B * NO, 256)), dim3(256), 0, s, B, NO, p->out,
                     P + p->off_b3);
  const double scale = 1.0 / ((double)NO * (double)B);
  hipLaunchKernelGGL(k_loss_grad, dim3(B), dim3(64), 0, s, B, p->n, p->out, bm, p->dout,
                     p->lossbuf + 1, scale);
  hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, s, B, p->lossbuf + 1, p->lossbuf);
  // backward (FP32; products with the BF16-rounded weights used forward)
  gemm(s, NO, H, B, p->dout, NO, 1, p->h2, H, 0, Gd + p->off_W3, H, 0, 0);       // gW3 = dout^T h2
  hipLaunchKernelGGL(k_colsum, dim3(ceil_div(NO, 64)), dim3(1024), 0, s, B, NO, p->dout,
                     Gd + p->off_b3);
  gemm(s, B, H, NO, p->dout, NO, 0, P + p->off_W3, H, 0, p->dh2, H, 1, 0);      // dh2 = dout W3
  hipLaunchKernelGGL(k_relu_bwd, dim3(ceil_div((long)B * H, 256)), dim3(256), 0, s, (long)B * H,
                     p->dh2, p->a2);
  gemm(s, H, H, B, p->dh2, H, 1, p->h1, H, 0, Gd + p->off_W2, H, 0, 0);          // gW2
  hipLaunchKernelGGL(k_colsum, dim3(ceil_div(H, 64)), dim3(1024), 0, s, B, H, p->dh2,
                     Gd + p->off_b2);
  gemm(s, B, H, H, p->dh2, H, 0, P + p->off_W2, H, 0, p->dh, H, 1, 0);          // dh1
  hipLaunchKernelGGL(k_relu_bwd, dim3(ceil_div((long)B * H, 256)), dim3(256), 0, s, (long)B * H,
                     p->dh, p->a1);
  gemm(s, H, nin, B, p->dh, H, 1, p->xs, nin, 0, Gd + p->off_W1, nin, 0, 0);     // gW1
  hipLaunchKernelGGL(k_colsum, dim3(ceil_div(H, 64)), dim3(1024), 0, s, B, H, p->dh,
                     Gd + p->off_b1);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

static int adam(Precond* p, double lr, double b1, double b2, double eps, hipStream_t s) {
  p->adam_t++;
  const double c1 = 1.0 - pow(b1, (double)p->adam_t), c2 = 1.0 - pow(b2, (double)p->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(ceil_div(p->np, 256)), dim3(256), 0, s, p->np, p->params,
                     p->grads, p->m1, p->m2, lr, b1, b2, eps, c1, c2);
  BDF_HIP_TRY(hipGetLastError());
  p->dirty = true;
  return 0;
}

}  // namespace bdfgpu

using namespace bdfgpu;

struct precond_handle {
  Precond p;
};

namespace bdfgpu {
// Used by the integrator: MLP inference for one class, gated on the
// controller's phase so that it can sit in a captured attempt sequence.
int precond_launch_gated(precond_handle* h, long B, const double* X, float* out,
                         const int* gphase, int want, const int* gskip, hipStream_t s) {
  // the weights are refreshed before capture by precond_prepare_inference
  return precond_infer(&h->p, B, X, out, 1, s, gphase, want, gskip);
}
int precond_dim(precond_handle* h) { return h ? h->p.n : -1; }
int precond_prepare_inference(precond_handle* h, hipStream_t s) {
  return refresh_inference_weights(&h->p, s);
}
}  // namespace bdfgpu

extern "C" {

int precond_create(int n, int hid, int batch_cap, precond_handle** out) {
  if (!out || n < 1 || n > 31 || hid != kMlpHid || batch_cap < 1)
    return arg_error("precond_create: n must be 1..31, hid 256, batch_cap >= 1");
  precond_handle* h = new precond_handle();
  Precond* p = &h->p;
  p->n = n;
  p->nin = n + 1;
  p->hid = hid;
  p->nout = n * n;
  p->nout_pad = ((p->nout + 31) / 32) * 32;
  p->off_W1 = 0;
  p->off_b1 = p->off_W1 + (long)hid * p->nin;
  p->off_W2 = p->off_b1 + hid;
  p->off_b2 = p->off_W2 + (long)hid * hid;
  p->off_W3 = p->off_b2 + hid;
  p->off_b3 = p->off_W3 + (long)p->nout * hid;
  p->np = p->off_b3 + p->nout;
  p->bcap = batch_cap;
  int st = 0;
  const size_t B = (size_t)batch_cap;
  if ((st = pc_alloc(p, (void**)&p->params, sizeof(float) * p->np)) ||
      (st = pc_alloc(p, (void**)&p->grads, sizeof(float) * p->np)) ||
      (st = pc_alloc(p, (void**)&p->m1, sizeof(double) * p->np)) ||
      (st = pc_alloc(p, (void**)&p->m2, sizeof(double) * p->np)) ||
      (st = pc_alloc(p, (void**)&p->in_mean, sizeof(double) * p->nin)) ||
      (st = pc_alloc(p, (void**)&p->in_std, sizeof(double) * p->nin)) ||
      (st = pc_alloc(p, (void**)&p->w1b, 2 * (size_t)hid * 32)) ||
      (st = pc_alloc(p, (void**)&p->w2b, 2 * (size_t)hid * hid)) ||
      (st = pc_alloc(p, (void**)&p->w3b, 2 * (size_t)p->nout_pad * hid)) ||
      (st = pc_alloc(p, (void**)&p->xs, sizeof(float) * B * p->nin)) ||
      (st = pc_alloc(p, (void**)&p->a1, sizeof(float) * B * hid)) ||
      (st = pc_alloc(p, (void**)&p->h1, sizeof(float) * B * hid)) ||
      (st = pc_alloc(p, (void**)&p->a2, sizeof(float) * B * hid)) ||
      (st = pc_alloc(p, (void**)&p->h2, sizeof(float) * B * hid)) ||
      (st = pc_alloc(p, (void**)&p->out, sizeof(float) * B * p->nout)) ||
      (st = pc_alloc(p, (void**)&p->dout, sizeof(float) * B * p->nout)) ||
      (st = pc_alloc(p, (void**)&p->dh, sizeof(float) * B * hid)) ||
      (st = pc_alloc(p, (void**)&p->dh2, sizeof(float) * B * hid)) ||
      (st = pc_alloc(p, (void**)&p->lossbuf, sizeof(double) * (B + 1))) ||
      (st = pc_alloc(p, (void**)&p->statpart, sizeof(double) * kStatBlocks * p->nin)) ||
      (st = pc_alloc(p, (void**)&p->bx, sizeof(double) * B * p->nin)) ||
      (st = pc_alloc(p, (void**)&p->bm, sizeof(double) * B * p->nout))) {
    precond_destroy(h);
    return st;
  }
  BDF_HIP_TRY(hipMemset(p->params, 0, sizeof(float) * p->np));
  BDF_HIP_TRY(hipMemset(p->m1, 0, sizeof(double) * p->np));
  BDF_HIP_TRY(hipMemset(p->m2, 0, sizeof(double) * p->np));
  std::vector<double> ones(p->nin, 1.0);
  BDF_HIP_TRY(hipMemset(p->in_mean, 0, sizeof(double) * p->nin));
  BDF_HIP_TRY(hipMemcpy(p->in_std, ones.data(), sizeof(double) * p->nin, hipMemcpyHostToDevice));
  *out = h;
  return 0;
}

int precond_destroy(precond_handle* h) {
  if (!h) return 0;
  (void)hipDeviceSynchronize();
  for (void* a : h->p.allocs) (void)hipFree(a);
  delete h;
  return 0;
}

long precond_num_params(precond_handle* h) { return h ? h->p.np : -1; }

int precond_set_params(precond_handle* h, const float* params_host) {
  if (!h || !params_host) return arg_error("precond_set_params: bad argument");
  BDF_HIP_TRY(hipMemcpy(h->p.params, params_host, sizeof(float) * h->p.np, hipMemcpyHostToDevice));
  BDF_HIP_TRY(hipMemset(h->p.m1, 0, sizeof(double) * h->p.np));
  BDF_HIP_TRY(hipMemset(h->p.m2, 0, sizeof(double) * h->p.np));
  h->p.adam_t = 0;
  h->p.dirty = true;
  return 0;
}

int precond_get_params(precond_handle* h, float* params_host, float* grads_host) {
  if (!h) return arg_error("precond_get_params: null handle");
  BDF_HIP_TRY(hipDeviceSynchronize());
  if (params_host)
    BDF_HIP_TRY(hipMemcpy(params_host, h->p.params, sizeof(float) * h->p.np, hipMemcpyDeviceToHost));
  if (grads_host)
    BDF_HIP_TRY(hipMemcpy(grads_host, h->p.grads, sizeof(float) * h->p.np, hipMemcpyDeviceToHost));
  return 0;
}

int precond_set_normalization(precond_handle* h, const double* mean_host, const double* std_host) {
  if (!h || !mean_host || !std_host) return arg_error("precond_set_normalization: bad argument");
  BDF_HIP_TRY(hipMemcpy(h->p.in_mean, mean_host, sizeof(double) * h->p.nin, hipMemcpyHostToDevice));
  BDF_HIP_TRY(hipMemcpy(h->p.in_std, std_host, sizeof(double) * h->p.nin, hipMemcpyHostToDevice));
  return 0;
}

int precond_get_normalization(precond_handle* h, double* mean_host, double* std_host) {
  if (!h || !mean_host || !std_host) return arg_error("precond_get_normalization: bad argument");
  BDF_HIP_TRY(hipDeviceSynchronize());
  BDF_HIP_TRY(hipMemcpy(mean_host, h->p.in_mean, sizeof(double) * h->p.nin, hipMemcpyDeviceToHost));
  BDF_HIP_TRY(hipMemcpy(std_host, h->p.in_std, sizeof(double) * h->p.nin, hipMemcpyDeviceToHost));
  return 0;
}

int precond_fit_normalization(precond_handle* h, const double* X, long ns, void* stream) {
  if (!h || !X || ns < 1) return arg_error("precond_fit_normalization: bad argument");
  hipStream_t s = as_stream(stream);
  const int w = h->p.nin;
  const int nb = (int)std::min<long>(kStatBlocks, ns);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_col_partial, dim3(nb), dim3(256), 0, s, ns, w, pass, X, h->p.in_mean,
                       h->p.statpart);
    hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(64), 0, s, nb, ns, w, pass, h->p.statpart,
                       h->p.in_mean, h->p.in_std);
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

int precond_loss_grad(precond_handle* h, int B, const double* X, const double* M, double* loss,
                      void* stream) {
  if (!h || B < 1 || B > h->p.bcap || !X || !M) return arg_error("precond_loss_grad: bad argument");
  hipStream_t s = as_stream(stream);
  int st = loss_grad(&h->p, B, X, M, s);
  if (st) return st;
  if (loss) {
    BDF_HIP_TRY(hipMemcpyAsync(loss, h->p.lossbuf, sizeof(double), hipMemcpyDeviceToHost, s));
    BDF_HIP_TRY(hipStreamSynchronize(s));
  }
  return 0;
}

int precond_adam(precond_handle* h, double lr, double b1, double b2, double eps, void* stream) {
  if (!h) return arg_error("precond_adam: null handle");
  return adam(&h->p, lr, b1, b2, eps, as_stream(stream));
}

int precond_train_epoch(precond_handle* h, long ns, const double* X, const double* M,
                        const int* perm, int batch, double lr, double* mean_loss, void* stream) {
  if (!h || ns < 1 || !X || !M || !perm || batch < 1 || batch > h->p.bcap)
    return arg_error("precond_train_epoch: bad argument");
  Precond* p = &h->p;
  hipStream_t s = as_stream(stream);
  double total = 0.0;
  long nb = 0;
  std::vector<double> losses;
  for (long b0 = 0; b0 + batch <= ns; b0 += batch) {
    hipLaunchKernelGGL(k_gather, dim3(ceil_div((long)batch * p->nin, 256)), dim3(256), 0, s, batch,
                       p->nin, X, perm + b0, p->bx);
    hipLaunchKernelGGL(k_gather, dim3(ceil_div((long)batch * p->nout, 256)), dim3(256), 0, s, batch,
                       p->nout, M, perm + b0, p->bm);
    int st = loss_grad(p, batch, p->bx, p->bm, s);
    if (st) return st;
    double l = 0.0;
    BDF_HIP_TRY(hipMemcpyAsync(&l, p->lossbuf, sizeof(double), hipMemcpyDeviceToHost, s));
    st = adam(p, lr, 0.9, 0.999, 1e-8, s);
    if (st) return st;
    BDF_HIP_TRY(hipStreamSynchronize(s));
    total += l;
    nb++;
  }
  if (mean_loss) *mean_loss = nb ? total / (double)nb : 0.0;
  return 0;
}

int precond_eval_loss(precond_handle* h, long ns, const double* X, const double* M, double* loss,
                      void* stream) {
  if (!h || ns < 1 || !X || !M || !loss) return arg_error("precond_eval_loss: bad argument");
  Precond* p = &h->p;
  hipStream_t s = as_stream(stream);
  double total = 0.0;
  for (long b0 = 0; b0 < ns; b0 += p->bcap) {
    const int B = (int)std::min<long>(p->bcap, ns - b0);
    int st = loss_grad(p, B, X + b0 * p->nin, M + b0 * p->nout, s);
    if (st) return st;
    double l = 0.0;
    BDF_HIP_TRY(hipMemcpyAsync(&l, p->lossbuf, sizeof(double), hipMemcpyDeviceToHost, s));
    BDF_HIP_TRY(hipStreamSynchronize(s));
    total += l * (double)B;
  }
  *loss = total / (double)ns;
  return 0;
}

int precond_forward(precond_handle* h, long B, const double* X, float* out, int use_mfma,
                    void* stream) {
  if (!h || B < 0 || (B > 0 && (!X || !out))) return arg_error("precond_forward: bad argument");
  return precond_infer(&h->p, B, X, out, use_mfma, as_stream(stream));
}

}  // extern "C"
