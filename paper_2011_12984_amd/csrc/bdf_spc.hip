// Segment-per-cell instantiations of the BDF step kernels (blocks of 13 to
// 64 species in segments of 16, 32 or 64 lanes; the Newton kernel also by
// the row width each lane holds, and with FP64 LU or the Gauss-Jordan
// inverse also with stored factors for the lazy Newton matrix).
#include "bdf_spc_dev.hpp"

namespace bdfgpu {

// Dynamic LDS above 64 KiB is requested explicitly (once per kernel).
template <typename KF>
static void raise_lds(KF* kern, size_t lds, size_t& raised) {
  if (lds > raised &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)
    raised = lds;
}

// Waves per SIMD asked of the segment Newton kernel (0: as many as its
// registers allow).  Learned mode at 24 columns needs more registers than
// two waves allow, mostly for a path that rarely runs (the LU fallback); the
// FP32-refined 48- and 64-column kernels fit three waves with their spills
// on the FP64 path; the FP32-refined 24- and 32-column kernels sit a few
// registers above four and three waves, the FP64 LU and Gauss-Jordan
// 64-column kernels a few above two.
template <int SEG, int LS, int NC>
constexpr int newton_waves() {
  if (SEG == 32 && LS == 2 && NC == 24) return 2;
  if (SEG == 64 && LS == 1 && (NC == 48 || NC == 64)) return 3;
  if (SEG == 32 && LS == 1 && NC == 24) return 4;
  if (SEG == 32 && LS == 1 && NC == 32) return 3;
  if (SEG == 64 && (LS == 0 || LS == 3) && NC == 64) return 2;   // FP64 LU, inverse: ~280
  return 0;
}

// Waves per SIMD asked of the lazy reuse kernel (0: as its registers allow):
// the 48- and 64-column ones and the 32-column inverse sit a few registers
// above three.
template <int SEG, int LS, int NC>
constexpr int reuse_waves() {
  return ((SEG == 64 && (NC == 64 || NC == 48)) || (SEG == 32 && NC == 32 && LS == 3)) ? 3 : 0;
}

// ... and of the lazy setup kernel: the 64-column one sits a few registers
// above two.
template <int SEG, int LS, int NC>
constexpr int setup_waves() {
  return (SEG == 64 && NC == 64) ? 2 : 0;
}

template <int SEG, int LS, int NC>
static void go_newton(const BdfDev& D, dim3 g, dim3 b, size_t lds, hipStream_t s) {
  static size_t raised = 65536;
  constexpr int w = newton_waves<SEG, LS, NC>();
  if constexpr (LS == 0 || LS == 3) {
    if (D.lazy) {   // lazy Newton matrix: the setup kernel, then the reuse kernel
      static size_t raised_s = 65536, raised_r = 65536;
      constexpr int sw = setup_waves<SEG, LS, NC>();
      if constexpr (sw > 0) {
        raise_lds(&k_spc_newton_w<SEG, LS, NC, sw, 1>, lds, raised_s);
        hipLaunchKernelGGL((k_spc_newton_w<SEG, LS, NC, sw, 1>), g, b, lds, s, D);
      } else {
        raise_lds(&k_spc_newton<SEG, LS, NC, 1>, lds, raised_s);
        hipLaunchKernelGGL((k_spc_newton<SEG, LS, NC, 1>), g, b, lds, s, D);
      }
      constexpr int rw = reuse_waves<SEG, LS, NC>();
      if constexpr (rw > 0) {
        raise_lds(&k_spc_newton_w<SEG, LS, NC, rw, 2>, lds, raised_r);
        hipLaunchKernelGGL((k_spc_newton_w<SEG, LS, NC, rw, 2>), g, b, lds, s, D);
      } else {
        raise_lds(&k_spc_newton<SEG, LS, NC, 2>, lds, raised_r);
        hipLaunchKernelGGL((k_spc_newton<SEG, LS, NC, 2>), g, b, lds, s, D);
      }
      return;
    }
  }
  if constexpr (w > 0) {
    raise_lds(&k_spc_newton_w<SEG, LS, NC, w>, lds, raised);
    hipLaunchKernelGGL((k_spc_newton_w<SEG, LS, NC, w>), g, b, lds, s, D);
  } else {
    raise_lds(&k_spc_newton<SEG, LS, NC>, lds, raised);
    hipLaunchKernelGGL((k_spc_newton<SEG, LS, NC>), g, b, lds, s, D);
  }
}

// Row width of the Newton kernel: n rounded up to a multiple of 8, within
// the widths instantiated for the segment.
template <int SEG, int LS>
static void newton_nc(const BdfDev& D, dim3 g, dim3 b, size_t lds, hipStream_t s) {
  const int nc = (D.k.n + 7) / 8 * 8;
  if constexpr (SEG == 16) {
    if (nc <= 8) return go_newton<16, LS, 8>(D, g, b, lds, s);
    return go_newton<16, LS, 16>(D, g, b, lds, s);
  } else if constexpr (SEG == 32) {
    if (nc <= 24) return go_newton<32, LS, 24>(D, g, b, lds, s);
    return go_newton<32, LS, 32>(D, g, b, lds, s);
  } else {
    if (nc <= 40) return go_newton<64, LS, 40>(D, g, b, lds, s);
    if (nc <= 48) return go_newton<64, LS, 48>(D, g, b, lds, s);
    if (nc <= 56) return go_newton<64, LS, 56>(D, g, b, lds, s);
    return go_newton<64, LS, 64>(D, g, b, lds, s);
  }
}

template <int SEG>
static void spc_go(int ls, int which, const BdfDev& D, unsigned int grid, hipStream_t s) {
  const dim3 g(grid), b(kCellThreads);
  const size_t lds = spc_lds_bytes(SEG, D.k.R);
  switch (which) {
    case 0: hipLaunchKernelGGL(k_spc_init1<SEG>, g, b, lds, s, D); break;
    case 1: hipLaunchKernelGGL(k_spc_init2<SEG>, g, b, lds, s, D); break;
    case 2:
      if (ls == 1)
        newton_nc<SEG, 1>(D, g, b, lds, s);
      else if (ls == 2)
        newton_nc<SEG, 2>(D, g, b, lds, s);
      else if (ls == 3)
        newton_nc<SEG, 3>(D, g, b, lds, s);
      else
        newton_nc<SEG, 0>(D, g, b, lds, s);
      break;
    case 4: hipLaunchKernelGGL(k_spc_predict<SEG>, g, b, lds, s, D); break;
    default: hipLaunchKernelGGL(k_spc_accept<SEG>, g, b, spc_accept_lds(), s, D); break;
  }
}

int spc_seg(int n) { return n <= 16 ? 16 : n <= 32 ? 32 : n <= 64 ? 64 : 0; }

void launch_spc(int seg, int ls, int which, const BdfDev& D, unsigned int grid, hipStream_t s) {
  switch (seg) {
    case 16: spc_go<16>(ls, which, D, grid, s); break;
    case 32: spc_go<32>(ls, which, D, grid, s); break;
    default: spc_go<64>(ls, which, D, grid, s); break;
  }
}

}  // namespace bdfgpu
