// Thread-per-cell instantiations of the BDF step kernels (blocks of up to
// 12 species; other sizes are padded to the next instantiated size).
#include "bdf_dev.hpp"

namespace bdfgpu {

void launch_tpc_newton_mode(int np, int ls, int mode, const BdfDev& D, unsigned int grid,
                            size_t lds, hipStream_t s);

// Dynamic LDS above 64 KiB (gfx950 has 160 KiB per workgroup) is requested
// explicitly; the first launch that needs it raises the kernel's limit.
template <int NP, int LS, bool FULL>
static void go_newton_v(const BdfDev& D, dim3 g, dim3 b, size_t lds, hipStream_t s) {
  static size_t raised = 65536;
  if (lds > raised &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tpc_newton<NP, LS, FULL>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)
    raised = lds;
  hipLaunchKernelGGL((k_tpc_newton<NP, LS, FULL>), g, b, lds, s, D);
}

// classes whose species fill the padded size get the variant with n fixed;
// the lazy Newton matrix and variable coefficients have kernels of their
// own (bdf_tpc_modes.hip)
template <int NP, int LS>
static void go_newton(const BdfDev& D, dim3 g, dim3 b, size_t lds, hipStream_t s) {
  const int mode = (D.lazy ? 1 : 0) | (D.vc ? 2 : 0);
  if (mode) return launch_tpc_newton_mode(NP, LS, mode, D, g.x, lds, s);
  if (D.k.n == NP)
    go_newton_v<NP, LS, true>(D, g, b, lds, s);
  else
    go_newton_v<NP, LS, false>(D, g, b, lds, s);
}

template <int NP>
static void tpc_go(int ls, int which, const BdfDev& D, unsigned int grid, hipStream_t s) {
  const dim3 g(grid), b(kTpcThreads);
  const size_t ilds = tpc_init_lds(NP, kTpcThreads);
  switch (which) {
    case 0: hipLaunchKernelGGL(k_tpc_init1<NP>, g, b, ilds, s, D); break;
    case 1: hipLaunchKernelGGL(k_tpc_init2<NP>, g, b, ilds, s, D); break;
    case 2: {
      const size_t lds = tpc_newton_lds(NP, D.k.R, ls, kTpcThreads, D.defer);
      if (ls == 1)
        go_newton<NP, 1>(D, g, b, lds, s);
      else if (ls == 3) {
        if constexpr (NP <= 4) go_newton<NP, 3>(D, g, b, lds, s);   // (bdf_create enforces NP <= 4)
      } else
        go_newton<NP, 0>(D, g, b, lds, s);
      break;
    }
    case 3: hipLaunchKernelGGL(k_tpc_accept<NP>, g, b, tpc_accept_lds(kTpcThreads), s, D); break;
    default: hipLaunchKernelGGL(k_tpc_flush<NP>, g, b, 0, s, D); break;
  }
}

int tpc_padded(int n) {
  return n <= 3 ? 3 : n <= 4 ? 4 : n <= 6 ? 6 : n <= 8 ? 8 : n <= 10 ? 10 : n <= 12 ? 12 : 0;
}

void launch_tpc(int np, int ls, int which, const BdfDev& D, unsigned int grid, hipStream_t s) {
  switch (np) {
    case 3: tpc_go<3>(ls, which, D, grid, s); break;
    case 4: tpc_go<4>(ls, which, D, grid, s); break;
    case 6: tpc_go<6>(ls, which, D, grid, s); break;
    case 8: tpc_go<8>(ls, which, D, grid, s); break;
    case 10: tpc_go<10>(ls, which, D, grid, s); break;
    default: tpc_go<12>(ls, which, D, grid, s); break;
  }
}

}  // namespace bdfgpu
