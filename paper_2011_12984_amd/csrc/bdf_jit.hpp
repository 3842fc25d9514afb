// Network-specialised thread-per-cell Newton kernels: source generation,
// compilation with hipcc into a shared library (cached on disk), loading.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace bdfgpu {

struct BdfDev;
// Launches the generated Newton kernel of one class: grid blocks of
// kTpcThreads, lds bytes of dynamic LDS, on stream s.
typedef void (*NetLaunch)(const BdfDev* D, unsigned int grid, unsigned int lds, hipStream_t s);

// HIP source of the fused Newton kernel bdf_newton_net_np<np>_ls<ls> for one
// mass-action network: nu, mu are the R x n reactant and product
// stoichiometries (row-major, at most two reactant molecules per reaction),
// np the padded block size of the thread-per-cell kernels, ls the linear
// solver (0 FP64 LU, 1 FP32 LU + refinement).  f, J and (I - gamma J) x are
// straight-line code over the network's nonzeros, in the same operations
// and order as the table-driven kernel, so both give identical bits.  The
// source also defines the extern "C" launcher bdf_newton_net_launch.
// mode: bit 0 lazy Newton matrix, bit 1 variable coefficients
std::string net_newton_source(const int* nu, const int* mu, int n, int R, int np, int ls,
                              int mode);

// Compiles src with hipcc ($HIPCC, else /opt/rocm/bin/hipcc) into
// net.so under $BDFGPU_JIT_DIR (else $TMPDIR/bdfgpu-jit-<uid>) in a
// directory named by a hash of the source, headers and flags, unless it is
// there already, then loads it and returns its launcher; a process compiles
// and loads each source once.  0 on success, else a BDFGPU_ERR_* code with
// the end of the compiler log as the last error.
int jit_newton(const std::string& src, NetLaunch* fn);

}  // namespace bdfgpu
