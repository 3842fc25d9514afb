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
  long bend[kMaxClasses];      // one past each class's last block in the phase reduction
  int kind[kMaxClasses];
  int ncls;
  // work queue: items 0 .. total-1 are the classes' blocks, class qcls[0]'s
  // first (the costliest per block), then qcls[1]'s, ...; qend[j] is one
  // past the last item of qcls[j]
  unsigned int* queue;         // next item (set to 0 before every launch)
  long total;
  int qcls[kMaxClasses];
  long qend[kMaxClasses];
};

int multi_kind(int map_tpc, int np);
size_t multi_lds(int kind, int np, int R, int ls, int which);
long multi_blocks(int kind, int np, long ncells);
double multi_block_cost(int kind, int np);
unsigned int multi_grid(int ls, int which, size_t lds);
void launch_multi(int ls, int which, const MultiDev& M, unsigned int grid, size_t lds,
                  hipStream_t s);

}  // namespace bdfgpu
