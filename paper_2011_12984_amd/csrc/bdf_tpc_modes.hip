// Thread-per-cell Newton kernels with the lazy Newton matrix (mode bit 0)
// and variable coefficients (mode bit 1); the plain kernels are in
// bdf_tpc.hip.  Kept apart so that the two units compile in parallel.
#include "bdf_dev.hpp"

namespace bdfgpu {

template <int NP, int LS, bool FULL, int MODE>
static void go_mode_v(const BdfDev& D, unsigned int grid, size_t lds, hipStream_t s) {
  static size_t raised = 65536;
  if (lds > raised &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tpc_newton<NP, LS, FULL, MODE>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)
    raised = lds;
  hipLaunchKernelGGL((k_tpc_newton<NP, LS, FULL, MODE>), dim3(grid), dim3(kTpcThreads), lds, s,
                     D);
}

template <int NP, int LS, int MODE>
static void go_mode(const BdfDev& D, unsigned int grid, size_t lds, hipStream_t s) {
  if (D.k.n == NP)
    go_mode_v<NP, LS, true, MODE>(D, grid, lds, s);
  else
    go_mode_v<NP, LS, false, MODE>(D, grid, lds, s);
}

// ls 1 (FP32 LU) has no stored-factor form: bdf_create refuses lazy with it
template <int NP, int LS>
static void go_modes(int mode, const BdfDev& D, unsigned int grid, size_t lds, hipStream_t s) {
  if constexpr (LS == 1) {
    go_mode<NP, LS, 2>(D, grid, lds, s);
  } else {
    switch (mode) {
      case 1: go_mode<NP, LS, 1>(D, grid, lds, s); break;
      case 2: go_mode<NP, LS, 2>(D, grid, lds, s); break;
      default: go_mode<NP, LS, 3>(D, grid, lds, s); break;
    }
  }
}

template <int NP>
static void go_np(int ls, int mode, const BdfDev& D, unsigned int grid, size_t lds,
                  hipStream_t s) {
  if (ls == 1) return go_modes<NP, 1>(mode, D, grid, lds, s);
  if constexpr (NP <= 4) {
    if (ls == 3) return go_modes<NP, 3>(mode, D, grid, lds, s);   // (bdf_create: NP <= 4)
  }
  go_modes<NP, 0>(mode, D, grid, lds, s);
}

void launch_tpc_newton_mode(int np, int ls, int mode, const BdfDev& D, unsigned int grid,
                            size_t lds, hipStream_t s) {
  switch (np) {
    case 3: go_np<3>(ls, mode, D, grid, lds, s); break;
    case 4: go_np<4>(ls, mode, D, grid, lds, s); break;
    case 6: go_np<6>(ls, mode, D, grid, lds, s); break;
    case 8: go_np<8>(ls, mode, D, grid, lds, s); break;
    case 10: go_np<10>(ls, mode, D, grid, lds, s); break;
    default: go_np<12>(ls, mode, D, grid, lds, s); break;
  }
}

}  // namespace bdfgpu
