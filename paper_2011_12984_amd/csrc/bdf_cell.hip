// Per-cell adaptive stepping: instantiations of the per-cell starting-step
// and attempt kernels for the thread-per-cell block sizes.
#include "bdf_cell.hpp"

namespace bdfgpu {

// control state of a fresh class: t = t0, not started (h = 0), q = 1
__global__ void k_cell_setup(long ncells, double t0, double* t, double* h, double* hsc,
                             double* hu, int* iv, int* cnt) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  t[c] = t0;
  h[c] = 0.0;
  hsc[c] = 1.0;
  hu[c] = 0.0;
  iv[4 * c + 0] = 1;
  iv[4 * c + 1] = 2;
  iv[4 * c + 2] = 0;
  iv[4 * c + 3] = CELL_RUN;
  for (int k = 0; k < 5; ++k) cnt[5 * c + k] = 0;
}

// cells that reached an earlier end time run again towards a later one
__global__ void k_cell_resume(long ncells, double tend, const double* t, int* iv) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  if (iv[4 * c + 3] == CELL_DONE && t[c] < tend) iv[4 * c + 3] = CELL_RUN;
}

__global__ void k_zero_u32(unsigned int* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

template <int NP, bool FULL, int LS>
static void cell_go_v(int which, const BdfDev& D, const CellDev& P, unsigned int grid,
                      hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)kTpcThreads * (size_t)(NP + D.k.R);
  static size_t raised[2] = {65536, 65536};
  const void* fn = which == 0 ? reinterpret_cast<const void*>(&k_cell_init<NP, FULL>)
                              : reinterpret_cast<const void*>(&k_cell_attempt<NP, FULL, LS>);
  if (lds > raised[which] &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)
    raised[which] = lds;
  if (which == 0)
    hipLaunchKernelGGL((k_cell_init<NP, FULL>), dim3(grid), dim3(kTpcThreads), lds, s, D, P);
  else
    hipLaunchKernelGGL((k_cell_attempt<NP, FULL, LS>), dim3(grid), dim3(kTpcThreads), lds, s,
                       D, P);
}

template <int NP, int LS>
static void cell_go(int which, const BdfDev& D, const CellDev& P, unsigned int grid,
                    hipStream_t s) {
  if (D.k.n == NP)
    cell_go_v<NP, true, LS>(which, D, P, grid, s);
  else
    cell_go_v<NP, false, LS>(which, D, P, grid, s);
}

template <int NP>
static void cell_go_ls(int ls, int which, const BdfDev& D, const CellDev& P, unsigned int grid,
                       hipStream_t s) {
  if constexpr (NP <= 4) {
    if (ls == 3) return cell_go<NP, 3>(which, D, P, grid, s);   // (bdf_create enforces NP <= 4)
  }
  cell_go<NP, 0>(which, D, P, grid, s);
}

// which: 0 starting step, 1 a batch of attempts; ls: 0 FP64 LU, 3 Gauss-Jordan
void launch_cell(int np, int ls, int which, const BdfDev& D, const CellDev& P, unsigned int grid,
                 hipStream_t s) {
  switch (np) {
    case 3: cell_go_ls<3>(ls, which, D, P, grid, s); break;
    case 4: cell_go_ls<4>(ls, which, D, P, grid, s); break;
    case 6: cell_go_ls<6>(ls, which, D, P, grid, s); break;
    case 8: cell_go_ls<8>(ls, which, D, P, grid, s); break;
    case 10: cell_go_ls<10>(ls, which, D, P, grid, s); break;
    default: cell_go_ls<12>(ls, which, D, P, grid, s); break;
  }
}

}  // namespace bdfgpu
