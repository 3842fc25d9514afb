// Segment-per-cell instantiations of the BDF step kernels (blocks of 13 to
// 64 species in segments of 16, 32 or 64 lanes).
#include "bdf_dev.hpp"

namespace bdfgpu {

// Dynamic LDS above 64 KiB is requested explicitly (once per kernel).
template <typename KF>
static void raise_lds(KF* kern, size_t lds, size_t& raised) {
  if (lds > raised &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)
    raised = lds;
}

template <int SEG>
static void spc_go(int ls, int which, const BdfDev& D, unsigned int grid, hipStream_t s) {
  const dim3 g(grid), b(kCellThreads);
  const size_t lds = spc_lds_bytes(SEG, D.k.R);
  switch (which) {
    case 0: hipLaunchKernelGGL(k_spc_init1<SEG>, g, b, lds, s, D); break;
    case 1: hipLaunchKernelGGL(k_spc_init2<SEG>, g, b, lds, s, D); break;
    case 2:
      if (ls == 1) {
        static size_t r1 = 65536;
        raise_lds(&k_spc_newton<SEG, 1>, lds, r1);
        hipLaunchKernelGGL((k_spc_newton<SEG, 1>), g, b, lds, s, D);
      } else if (ls == 2) {
        static size_t r2 = 65536;
        raise_lds(&k_spc_newton<SEG, 2>, lds, r2);
        hipLaunchKernelGGL((k_spc_newton<SEG, 2>), g, b, lds, s, D);
      } else {
        static size_t r0 = 65536;
        raise_lds(&k_spc_newton<SEG, 0>, lds, r0);
        hipLaunchKernelGGL((k_spc_newton<SEG, 0>), g, b, lds, s, D);
      }
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
