// One persistent launch for every class of cells (blocks of uneven sizes):
// a grid sized to what the device holds at once takes work items from a
// queue in device memory, one class block per item (thread per cell with
// 256-cell blocks, or a segment per cell), the classes with the costliest
// blocks first, until the queue is empty.  Each item writes its block
// partials where the per-class launches would, so the phase reduction and
// the decisions are the same whichever workgroup ran it.
#include "bdf_dev.hpp"
#include "bdf_multi.hpp"

namespace bdfgpu {

template <int WHICH, int LS>
__device__ __forceinline__ void multi_body(const BdfDev& D, int kind, long blk, double* lds) {
  constexpr int TB = kCellThreads;
  switch (kind) {
#define TPC_CASE(K, NP)                                                   \
  case K:                                                                 \
    if (WHICH == 0) tpc_init1_body<NP, TB>(D, blk, lds);                  \
    else if (WHICH == 1) tpc_init2_body<NP, TB>(D, blk, lds);             \
    else if (WHICH == 2) tpc_newton_body<NP, LS, TB>(D, blk, lds);        \
    else tpc_accept_body<NP, TB>(D, blk, lds);                            \
    break;
    TPC_CASE(KIND_TPC3, 3)
    TPC_CASE(KIND_TPC4, 4)
    TPC_CASE(KIND_TPC6, 6)
    TPC_CASE(KIND_TPC8, 8)
    TPC_CASE(KIND_TPC10, 10)
    TPC_CASE(KIND_TPC12, 12)
#undef TPC_CASE
#define SPC_CASE(K, SEG)                                                  \
  case K:                                                                 \
    if (WHICH == 0) spc_init_body<SEG, 1>(D, blk, lds);                   \
    else if (WHICH == 1) spc_init_body<SEG, 2>(D, blk, lds);              \
    else if (WHICH == 2) spc_newton_body<SEG, LS>(D, blk, lds);           \
    else spc_accept_body<SEG>(D, blk, lds);                               \
    break;
    SPC_CASE(KIND_SPC16, 16)
    SPC_CASE(KIND_SPC32, 32)
    SPC_CASE(KIND_SPC64, 64)
#undef SPC_CASE
    default: break;
  }
}

// Every workgroup leaves once the queue is past its last item (the counter
// only grows), so the grid drains whatever the item count.
template <int WHICH, int LS>
__global__ void __launch_bounds__(kCellThreads) k_multi(MultiDev M) {
  extern __shared__ double lds[];
  __shared__ unsigned int s_item;
  const int want = WHICH == 0 ? PH_INIT1 : WHICH == 1 ? PH_INIT2 : WHICH == 2 ? PH_PREDICT
                                                                               : PH_ACCEPT;
  if (M.base.C->phase != want) return;
  for (;;) {
    __syncthreads();   // the previous item is done with the LDS and s_item
    if (threadIdx.x == 0) s_item = atomicAdd(M.queue, 1u);
    __syncthreads();
    const long it = (long)s_item;
    if (it >= M.total) break;
    int j = 0;
    while (j + 1 < M.ncls && it >= M.qend[j]) ++j;
    const int cl = M.qcls[j];
    BdfDev D = M.base;
    D.k = M.k[cl];
    D.k.blk0 = cl ? M.bend[cl - 1] : 0;
    multi_body<WHICH, LS>(D, M.kind[cl], it - (j ? M.qend[j - 1] : 0), lds);
  }
}

__global__ void k_queue_reset(unsigned int* q) {
  if (threadIdx.x == 0) *q = 0u;
}

int multi_kind(int map_tpc, int np) {
  if (map_tpc) {
    switch (np) {
      case 3: return KIND_TPC3;
      case 4: return KIND_TPC4;
      case 6: return KIND_TPC6;
      case 8: return KIND_TPC8;
      case 10: return KIND_TPC10;
      default: return KIND_TPC12;
    }
  }
  return np == 16 ? KIND_SPC16 : np == 32 ? KIND_SPC32 : KIND_SPC64;
}

size_t multi_lds(int kind, int np, int R, int ls, int which) {
  if (kind <= KIND_TPC12) {
    if (which == 2) return tpc_newton_lds(np, R, ls, kCellThreads);
    if (which == 3) return tpc_accept_lds(kCellThreads);
    return tpc_init_lds(np, kCellThreads);
  }
  if (which == 3) return spc_accept_lds();
  return spc_lds_bytes(np, R);
}

long multi_blocks(int kind, int np, long ncells) {
  const long cpb = kind <= KIND_TPC12 ? kCellThreads : kCellThreads / np;
  return std::max<long>(1, (ncells + cpb - 1) / cpb);
}

// Relative work of one block of a class, for the queue order: cells per
// block times the cube of the row width its cells are factored at.
double multi_block_cost(int kind, int np) {
  const double cpb = kind <= KIND_TPC12 ? (double)kCellThreads : (double)(kCellThreads / np);
  return cpb * (double)np * (double)np * (double)np;
}

// dynamic LDS above 64 KiB (gfx950 has 160 KiB per workgroup) is requested
// explicitly; the first use that needs it raises the limit
template <int WHICH, int LS>
static void raise_lds(size_t lds) {
  static size_t raised = 65536;
  if (lds > raised) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_multi<WHICH, LS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess)
      raised = lds;
  }
}

// Workgroups the device holds at once: per-CU occupancy of the kernel at
// this LDS size times the CU count (0 if the runtime cannot tell).
template <int WHICH, int LS>
static unsigned int resident(size_t lds) {
  raise_lds<WHICH, LS>(lds);
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_multi<WHICH, LS>, kCellThreads,
                                                   lds) != hipSuccess)
    return 0;
  return (unsigned int)std::max(0, per) * (unsigned int)std::max(0, ncu);
}

unsigned int multi_grid(int ls, int which, size_t lds) {
  switch (which) {
    case 0: return resident<0, 0>(lds);
    case 1: return resident<1, 0>(lds);
    case 2: return ls == 1 ? resident<2, 1>(lds) : resident<2, 0>(lds);
    default: return resident<3, 0>(lds);
  }
}

template <int WHICH, int LS>
static void go(const MultiDev& M, dim3 g, dim3 b, size_t lds, hipStream_t s) {
  raise_lds<WHICH, LS>(lds);
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, M.queue);
  hipLaunchKernelGGL((k_multi<WHICH, LS>), g, b, lds, s, M);
}

// grid: the persistent grid (the resident workgroups, at most one per item).
void launch_multi(int ls, int which, const MultiDev& M, unsigned int grid, size_t lds,
                  hipStream_t s) {
  const dim3 g(std::max(1u, grid)), b(kCellThreads);
  switch (which) {
    case 0: go<0, 0>(M, g, b, lds, s); break;
    case 1: go<1, 0>(M, g, b, lds, s); break;
    case 2:
      if (ls == 1)
        go<2, 1>(M, g, b, lds, s);
      else
        go<2, 0>(M, g, b, lds, s);
      break;
    default: go<3, 0>(M, g, b, lds, s); break;
  }
}

}  // namespace bdfgpu
