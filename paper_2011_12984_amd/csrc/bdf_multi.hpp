// Descriptor of a single launch over every class of cells.
#pragma once

#include "bdf_spc_dev.hpp"

namespace bdfgpu {

constexpr int kMaxClasses = 8;

enum Kind : int {
  KIND_TPC3 = 0,
  KIND_TPC4,
  KIND_TPC6,
  KIND_TPC8,
  KIND_TPC10,
  KIND_TPC12,
  KIND_SPC16,
  KIND_SPC32,
  KIND_SPC64
};

struct MultiDev {
  BdfDev base;                 // controller, reduction buffers, tolerances
  ClassDev k[kMaxClasses];
  long bend[kMaxClasses];      // one past each class's last block in the grid
  int kind[kMaxClasses];
  int ncls;
};

int multi_kind(int map_tpc, int np);
size_t multi_lds(int kind, int np, int R, int ls, int which);
long multi_blocks(int kind, int np, long ncells);
void launch_multi(int ls, int which, const MultiDev& M, unsigned int grid, size_t lds,
                  hipStream_t s);

}  // namespace bdfgpu
