// Host side of the grouped BDF integrator: problem setup, internal layouts,
// attempt sequencing and hipGraph capture.
//
// Cells are grouped by network topology into classes; every class gets its
// own storage in the layout of its cell-to-lane mapping (tiled for thread
// per cell, cell-major for segment per cell).  One step attempt is the fixed
// launch sequence fused predictor + Newton, then history update, over all
// classes (learned mode: predictor and MLP inference first); kernels whose
// phase is not current return at once, so the same sequence serves every
// outcome and can be captured once into a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <vector>

#include <chrono>

#include "bdf_cell.hpp"
#include "bdf_spc_dev.hpp"
#include "bdf_jit.hpp"
#include "bdf_multi.hpp"
#include "common.hpp"

namespace bdfgpu {

int tpc_padded(int n);
int spc_seg(int n);
void launch_tpc(int np, int ls, int which, const BdfDev& D, unsigned int grid, hipStream_t s);
void launch_spc(int seg, int ls, int which, const BdfDev& D, unsigned int grid, hipStream_t s);
void launch_cell(int np, int ls, int which, const BdfDev& D, const CellDev& P, unsigned int grid,
                 hipStream_t s);
void launch_kry(int np, int which, const BdfDev& D, unsigned int grid, hipStream_t s, int k,
                double a, const double* coef);
void launch_kry_sum(const double* partials, unsigned int nb, double* out, hipStream_t s);
void launch_kry_control(Ctrl* C, const double* sums, long liters, hipStream_t s);
__global__ void k_cell_setup(long ncells, double t0, double* t, double* h, double* hsc,
                             double* hu, int* iv, int* cnt);
__global__ void k_cell_resume(long ncells, double tend, const double* t, int* iv);
__global__ void k_zero_u32(unsigned int* p, int n);

int precond_launch_gated(precond_handle* h, long B, const double* X, float* out,
                         const int* gphase, int want, const int* gskip, hipStream_t s);
int precond_dim(precond_handle* h);
int precond_prepare_inference(precond_handle* h, hipStream_t s);

enum { MAP_TPC = 0, MAP_SPC = 1 };

struct ClassHost {
  int topo, n, R, map, np;      // np: TPC padded size or SPC segment
  long ncells;
  unsigned int grid;            // blocks of the class's own launches
  long blk0;
  int kind;                     // mapping in the single launch over all classes
  long mblocks, mblk0;          // blocks and first block in that launch
  long* d_yoff = nullptr;       // user-layout offset of each class cell's y
  long* d_roff = nullptr;       // user-layout offset of each class cell's rates
  NetLaunch jit = nullptr;      // network-specialised Newton kernel, if any
  ClassDev dev;
  std::vector<long> members;    // user indices of the class's cells
  CellDev cell;                 // per-cell stepping: control state of each cell
};

__global__ void k_clear_upd(Ctrl* C) { C->upd = 0; }

__global__ void k_resume(Ctrl* C, double tend, long inc) {
  C->tend = tend;
  const long lim = C->nsteps + inc;
  C->step_limit = lim < C->nsteps ? LONG_MAX : lim;
  if (C->phase == PH_PAUSE || C->phase == PH_DONE) {
    if (C->t < tend)
      prepare_attempt(C);
    else
      C->phase = PH_DONE;
  }
}

// user layout <-> class layout.  tiled: element i of class cell c at
// (c/64)*64*w + i*64 + c%64, else c*w + i.
__global__ void k_to_class(long ncells, int w, int tiled, const long* off, const double* src,
                           double* dst, double scale) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * w) return;
  const long c = t / w;
  const int i = (int)(t - c * w);
  const long d = tiled ? (c >> 6) * 64L * w + (long)i * 64 + (c & 63) : c * w + i;
  dst[d] = src[off[c] + i] * scale;
}

__global__ void k_from_class(long ncells, int w, int tiled, const long* off, const double* src,
                             double* dst, double scale) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * w) return;
  const long c = t / w;
  const int i = (int)(t - c * w);
  const long d = tiled ? (c >> 6) * 64L * w + (long)i * 64 + (c & 63) : c * w + i;
  dst[off[c] + i] = src[d] * scale;
}

// f and J of every class cell at a user-layout state (test and inspection
// path, one thread per cell, plain loops).
__global__ void k_eval_rhs_jac(long ncells, NetDev nd, const long* yoff, const long* roff,
                               const long* joff, const double* rates, const double* y,
                               double* f, double* J) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const double* yc = y + yoff[c];
  const double* kc = rates + roff[c];
  const int n = nd.n;
  if (f)
    for (int i = 0; i < n; ++i) f[yoff[c] + i] = 0.0;
  if (J)
    for (int i = 0; i < n * n; ++i) J[joff[c] + i] = 0.0;
  for (int k = 0; k < nd.R; ++k) {
    const int a = nd.ra[k], b = nd.rb[k], d = nd.rc[k];
    double r = kc[k];
    if (a >= 0) r *= yc[a];
    if (b >= 0) r *= yc[b];
    if (d >= 0) r *= yc[d];
    if (f)
      for (int i = 0; i < n; ++i) f[yoff[c] + i] += nd.S[(long)k * nd.np + i] * r;
  }
  if (J)
    for (int a = 0; a < n; ++a)
      for (int e = nd.jst[a]; e < nd.jst[a + 1]; ++e) {
        const int k = nd.jk[e], p = nd.jp[e], p2 = nd.jp2[e];
        double g = kc[k] * nd.jm[e];
        if (p >= 0) g *= yc[p];
        if (p2 >= 0) g *= yc[p2];
        for (int i = 0; i < n; ++i) J[joff[c] + i + (long)a * n] += nd.S[(long)k * nd.np + i] * g;
      }
}

// Training samples for the learned preconditioner: inputs [y, log gamma]
// and M = I - gamma J(y) (column-major) of every stride-th class cell.
__global__ void k_capture(long nsamp, long stride, int n, int tiled, NetDev nd,
                          const double* z0, const double* rates, double gamma, double* Xraw,
                          double* Mout) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsamp) return;
  const long c = k * stride;
  double y[64];
  for (int i = 0; i < n; ++i)
    y[i] = z0[tiled ? (c >> 6) * 64L * n + (long)i * 64 + (c & 63) : c * n + i];
  for (int i = 0; i < n; ++i) Xraw[k * (n + 1) + i] = y[i];
  Xraw[k * (n + 1) + n] = log(gamma);
  double* Mk = Mout + k * (long)n * n;
  for (int e = 0; e < n * n; ++e) Mk[e] = 0.0;
  for (int a = 0; a < n; ++a)
    for (int e = nd.jst[a]; e < nd.jst[a + 1]; ++e) {
      const int kk = nd.jk[e], p = nd.jp[e], p2 = nd.jp2[e];
      const double kap = rates[tiled ? (c >> 6) * 64L * nd.R + (long)kk * 64 + (c & 63)
                                     : c * nd.R + kk];
      double g = kap * nd.jm[e];
      if (p >= 0) g *= y[p];
      if (p2 >= 0) g *= y[p2];
      for (int i = 0; i < n; ++i) Mk[i + (long)a * n] += nd.S[(long)kk * nd.np + i] * g;
    }
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i)
      Mk[i + (long)a * n] = (i == a ? 1.0 : 0.0) - gamma * Mk[i + (long)a * n];
}

}  // namespace bdfgpu

using namespace bdfgpu;

struct bdf_handle {
  hipStream_t s = nullptr;
  hipStream_t cap = nullptr;     // capture stream for graph mode
  bdf_options o;
  long N = 0, ncells = 0;
  std::vector<ClassHost> cls;
  Ctrl* dC = nullptr;
  Ctrl* hC = nullptr;            // pinned mirror
  double* partials = nullptr;
  double* gpartials = nullptr;
  unsigned int nblocks_total = 0;  // per-class launches
  unsigned int nblocks_multi = 0;  // single launch over all classes: work items
  unsigned int* d_queue = nullptr;  // its work-queue counter
  unsigned int multi_grid[4] = {0, 0, 0, 0};   // its persistent grid per phase
  int qcls[kMaxClasses] = {0};      // classes in queue order, costliest blocks first
  long qend[kMaxClasses] = {0};
  bool fused = false;              // launch mode in use
  bool defer = false;              // deferred history update (Ctrl::fuse)
  bool fusable = false;
  size_t multi_lds[4] = {0, 0, 0, 0};
  // autotuning record: candidate (launch, map_small) -> ms per step (-1 if
  // not tried) and the choice
  double tune_ms[4] = {-1, -1, -1, -1};
  int tune_launch = 0, tune_map_small = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<void*> allocs;
  std::vector<long> h_joff;      // per class: user offsets of J blocks (for eval)
  std::vector<long*> d_joff;
  // kernel timing (stream mode): event pairs around each kernel group
  bool prof = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_key;       // group of each pending pair
  size_t ev_used = 0;            // pairs recorded since the last fold
  double prof_ms[3] = {0, 0, 0};
  long prof_cnt[3] = {0, 0, 0};
  // device state in caller memory (bdf_create_ws) or counted only
  // (bdf_workspace_bytes: a dry run of the creation that touches no device)
  char* ws = nullptr;
  size_t ws_size = 0, ws_used = 0;
  bool dry = false;
  // per-cell stepping: counts of cells still running after each attempt of
  // a batch (device) and the pinned copy of the last one
  bool per_cell = false;
  unsigned int* d_active = nullptr;
  unsigned int* h_active = nullptr;
  // Newton-Krylov: host-driven GMRES; reduced sums (device, pinned host)
  // and the per-iteration Newton sums handed to the controller
  bool krylov = false;
  double* d_kry = nullptr;
  double* h_kry = nullptr;
  double* d_ksums = nullptr;
};

constexpr int kCellSlots = 1;       // per-cell mode: count of running cells
constexpr int kCellAttempts = 128;  // per-cell mode: attempts per cell in one launch

constexpr size_t kWsAlign = 256;

// Device memory of the handle: from the caller's workspace when one was
// given (256-byte aligned pieces, in creation order), else hipMalloc'd and
// freed by bdf_destroy.
static int dalloc(bdf_handle* h, void** p, size_t bytes) {
  bytes = bytes < 16 ? 16 : bytes;
  if (h->dry || h->ws) {
    const size_t off = (h->ws_used + kWsAlign - 1) / kWsAlign * kWsAlign;
    if (!h->dry && off + bytes > h->ws_size) {
      set_last_error("bdf_create_ws: workspace too small (see bdf_workspace_bytes)", __FILE__,
                     __LINE__);
      return BDFGPU_ERR_WORKSPACE;
    }
    h->ws_used = off + bytes;
    *p = h->dry ? nullptr : h->ws + off;
    return 0;
  }
  BDF_HIP_TRY(hipMalloc(p, bytes));
  h->allocs.push_back(*p);
  return 0;
}

// zero-filled device memory (nothing in a dry run)
static int dalloc_zero(bdf_handle* h, void** p, size_t bytes) {
  int st = dalloc(h, p, bytes);
  if (st || h->dry) return st;
  BDF_HIP_TRY(hipMemsetAsync(*p, 0, bytes < 16 ? 16 : bytes, h->s));
  return 0;
}

template <typename T>
static int upload(bdf_handle* h, T** d, const std::vector<T>& v) {
  int st = dalloc(h, reinterpret_cast<void**>(d), sizeof(T) * std::max<size_t>(1, v.size()));
  if (st) return st;
  if (!v.empty() && !h->dry)
    BDF_HIP_TRY(hipMemcpy(*d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return 0;
}

static BdfDev make_dev(bdf_handle* h, const ClassHost& c) {
  BdfDev D;
  D.C = h->dC;
  D.partials = h->partials;
  D.nblocks_total = h->fused ? h->nblocks_multi : h->nblocks_total;
  D.rtol = h->o.rtol;
  D.atol = h->o.atol;
  D.nonneg = h->o.nonneg ? 1 : 0;
  D.defer = h->defer ? 1 : 0;
  D.lazy = h->o.lazy ? 1 : 0;
  D.vc = h->o.vc ? 1 : 0;
  D.k = c.dev;
  D.k.blk0 = c.blk0;
  return D;
}

static void launch_phase_kernels(bdf_handle* h, int which, hipStream_t s);

// Sums of the phase's block partials and the controller (which 0..3).
static void launch_control(bdf_handle* h, int which, hipStream_t s) {
  static const int want[4] = {PH_INIT1, PH_INIT2, PH_PREDICT, PH_ACCEPT};
  const unsigned int nb = h->fused ? h->nblocks_multi : h->nblocks_total;
  const unsigned int ng = (nb + kRedGroup - 1) / kRedGroup;
  const int K = which == 2 ? kRedNewton : kRedVals;
  if (K == kRedNewton)
    hipLaunchKernelGGL(k_reduce_groups<kRedNewton>, dim3(ng), dim3(256), 0, s, h->dC, want[which],
                       h->partials, nb, h->gpartials);
  else
    hipLaunchKernelGGL(k_reduce_groups<kRedVals>, dim3(ng), dim3(256), 0, s, h->dC, want[which],
                       h->partials, nb, h->gpartials);
  switch (which) {
    case 0:
      hipLaunchKernelGGL((k_control<kRedVals, 0>), dim3(1), dim3(256), 0, s, h->dC, want[0],
                         h->gpartials, ng);
      break;
    case 1:
      hipLaunchKernelGGL((k_control<kRedVals, 1>), dim3(1), dim3(256), 0, s, h->dC, want[1],
                         h->gpartials, ng);
      break;
    case 2:
      hipLaunchKernelGGL((k_control<kRedNewton, 2>), dim3(1), dim3(256), 0, s, h->dC, want[2],
                         h->gpartials, ng);
      break;
    default:
      hipLaunchKernelGGL((k_control<kRedVals, 3>), dim3(1), dim3(256), 0, s, h->dC, want[3],
                         h->gpartials, ng);
      break;
  }
}

static void launch_phase(bdf_handle* h, int which, hipStream_t s) {
  launch_phase_kernels(h, which, s);
  if (which <= 3) launch_control(h, which, s);
}

static void launch_phase_kernels(bdf_handle* h, int which, hipStream_t s) {
  if (h->fused && which <= 3) {
    MultiDev M;
    memset(&M, 0, sizeof(M));
    M.ncls = (int)h->cls.size();
    for (int k = 0; k < M.ncls; ++k) {
      const ClassHost& c = h->cls[k];
      M.k[k] = c.dev;
      M.kind[k] = c.kind;
      M.bend[k] = c.mblk0 + c.mblocks;
      M.qcls[k] = h->qcls[k];
      M.qend[k] = h->qend[k];
    }
    M.queue = h->d_queue;
    M.total = h->nblocks_multi;
    M.base = make_dev(h, h->cls[0]);
    launch_multi(h->o.linsol, which, M, h->multi_grid[which], h->multi_lds[which], s);
    return;
  }
  for (const ClassHost& c : h->cls) {
    if (which == 5 && c.map != MAP_TPC) continue;   // flush: thread-per-cell classes only
    BdfDev D = make_dev(h, c);
    if (c.map == MAP_TPC && which == 2 && c.jit) {
      c.jit(&D, c.grid,
            (unsigned int)tpc_newton_lds(c.np, c.R, h->o.linsol, kTpcThreads, h->defer), s);
    } else if (c.map == MAP_TPC)
      launch_tpc(c.np, h->o.linsol, which, D, c.grid, s);
    else
      launch_spc(c.np, h->o.linsol, which, D, c.grid, s);
  }
}

static void prof_mark(bdf_handle* h, int key, bool begin, hipStream_t s) {
  if (!h->prof) return;
  if (begin) {
    if (2 * (h->ev_used + 1) > h->ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
      h->ev.push_back(a);
      h->ev.push_back(b);
      h->ev_key.push_back(key);
    }
    h->ev_key[h->ev_used] = key;
    (void)hipEventRecord(h->ev[2 * h->ev_used], s);
  } else {
    (void)hipEventRecord(h->ev[2 * h->ev_used + 1], s);
    h->ev_used++;
  }
}

// after a stream synchronisation: add up the recorded pairs
static void prof_fold(bdf_handle* h) {
  for (size_t i = 0; i < h->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) == hipSuccess) {
      h->prof_ms[h->ev_key[i]] += ms;
      h->prof_cnt[h->ev_key[i]]++;
    }
  }
  h->ev_used = 0;
}

static void enqueue_attempt(bdf_handle* h, hipStream_t s) {
  if (h->o.linsol == BDFGPU_LS_LEARNED) {
    // predictor, then the MLP's approximate inverses (skipped when the
    // attempt is being redone with exact LU), then the Newton iterations
    prof_mark(h, 1, true, s);
    launch_phase(h, 4, s);
    for (const ClassHost& c : h->cls)
      (void)precond_launch_gated(reinterpret_cast<precond_handle*>(h->o.precond), c.ncells,
                                 c.dev.xin, c.dev.X, &h->dC->phase, PH_PREDICT,
                                 &h->dC->force_lu, s);
    prof_mark(h, 1, false, s);
  }
  prof_mark(h, 0, true, s);
  launch_phase_kernels(h, 2, s);
  prof_mark(h, 0, false, s);
  launch_control(h, 2, s);
  if (h->defer) return;   // the next Newton kernel updates the history
  prof_mark(h, 2, true, s);
  launch_phase_kernels(h, 3, s);
  prof_mark(h, 2, false, s);
  launch_control(h, 3, s);
}

// Deferred history update: apply the last accepted attempt's update before
// the host reads or replaces the state (the flush kernels return at once
// when none is pending), then clear the pending flag.
static int flush_update(bdf_handle* h) {
  if (!h->defer) return 0;
  launch_phase_kernels(h, 5, h->s);
  hipLaunchKernelGGL(k_clear_upd, dim3(1), dim3(1), 0, h->s, h->dC);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

static int read_ctrl(bdf_handle* h) {
  BDF_HIP_TRY(hipMemcpyAsync(h->hC, h->dC, sizeof(Ctrl), hipMemcpyDeviceToHost, h->s));
  BDF_HIP_TRY(hipStreamSynchronize(h->s));
  return 0;
}

static int build_graph(bdf_handle* h) {
  if (h->o.linsol == BDFGPU_LS_LEARNED) {
    int st = precond_prepare_inference(reinterpret_cast<precond_handle*>(h->o.precond), h->s);
    if (st) return st;
    BDF_HIP_TRY(hipStreamSynchronize(h->s));
  }
  BDF_HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  BDF_HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
  enqueue_attempt(h, h->cap);
  BDF_HIP_TRY(hipStreamEndCapture(h->cap, &h->graph));
  BDF_HIP_TRY(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
  return 0;
}

// One pass of a Krylov kernel over every class, its block partials summed
// on the device and read back (8 values).
static int kry_phase(bdf_handle* h, int which, int k, double a, const double* coef, double* out) {
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    launch_kry(c.np, which, make_dev(h, c), c.grid, h->s, k, a, coef);
  }
  launch_kry_sum(h->partials, h->nblocks_total, h->d_kry, h->s);
  BDF_HIP_TRY(hipMemcpyAsync(h->h_kry, h->d_kry, sizeof(double) * 8, hipMemcpyDeviceToHost, h->s));
  BDF_HIP_TRY(hipStreamSynchronize(h->s));
  for (int j = 0; j < 8; ++j) out[j] = h->h_kry[j];
  return 0;
}

// The Newton iterations of one attempt with GMRES (the controller's state
// read just before, phase PH_PREDICT): predictor and preconditioner setup,
// then per Newton iteration the residual, the Krylov iterations and the
// update; the Newton sums go to the controller, which takes the decision.
// The host stops at the iteration where the controller will decide (the
// same test on the same sums); iterations not run get NaN sums, which the
// controller would treat as a failure if it ever read them.
static int kry_attempt(bdf_handle* h) {
  const Ctrl C0 = *h->hC;
  double o[8], sums[kRedNewton];
  for (int j = 0; j < kRedNewton; ++j) sums[j] = 0.0;
  int st = kry_phase(h, 0, 0, 0.0, nullptr, o);
  if (st) return st;
  sums[7] = o[0];   // singular blocks in the setup
  const double N = C0.N;
  const double tol = kKryEplin * kNlsCoef * sqrt(N);
  long liters = 0;
  double crate = C0.crate, dold = 0.0;
  int mlast = 0;
  for (int m = 0; m < C0.maxcor; ++m) {
    mlast = m;
    if (m == 0 && sums[7] > 0.0) break;
    if ((st = kry_phase(h, 1, 0, 0.0, nullptr, o))) return st;
    const double beta = sqrt(o[0]);
    double g[kKryMaxl + 1], cs[kKryMaxl], sn[kKryMaxl], H[kKryMaxl][kKryMaxl], y[kKryMaxl + 1];
    for (int j = 0; j <= kKryMaxl; ++j) g[j] = y[j] = 0.0;
    int kend = 0;
    if (beta > tol) {
      g[0] = beta;
      double inv = 1.0 / beta;
      int k = 0;
      for (k = 0; k < kKryMaxl; ++k) {
        double hk[kKryMaxl + 1];
        if ((st = kry_phase(h, 2, k, inv, nullptr, o))) return st;
        for (int j = 0; j <= k; ++j) hk[j] = o[j];
        if ((st = kry_phase(h, 3, k, 0.0, hk, o))) return st;
        hk[k + 1] = sqrt(o[0]);
        liters++;
        const bool breakdown = !(hk[k + 1] > 0.0);
        inv = breakdown ? 0.0 : 1.0 / hk[k + 1];
        for (int j = 0; j < k; ++j) {
          const double a = hk[j], c2 = hk[j + 1];
          hk[j] = cs[j] * a + sn[j] * c2;
          hk[j + 1] = -sn[j] * a + cs[j] * c2;
        }
        const double rr = sqrt(hk[k] * hk[k] + hk[k + 1] * hk[k + 1]);
        cs[k] = hk[k] / rr;
        sn[k] = hk[k + 1] / rr;
        hk[k] = rr;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        for (int j = 0; j <= k; ++j) H[j][k] = hk[j];
        if (breakdown || fabs(g[k + 1]) <= tol) {
          k++;
          break;
        }
      }
      kend = k;
      for (int i = kend - 1; i >= 0; --i) {
        double s2 = g[i];
        for (int j = i + 1; j < kend; ++j) s2 = s2 - H[i][j] * y[j];
        y[i] = s2 / H[i][i];
      }
    }
    if ((st = kry_phase(h, 4, m, (double)kend, y, o))) return st;
    sums[kRedPerIter * m + 0] = o[0];
    sums[kRedPerIter * m + 1] = o[1];
    sums[kRedPerIter * m + 2] = o[2];
    // the controller's test (after_newton_all), to know where it stops
    const double d = sqrt(o[0] / N);
    if (!(d == d) || d > 1e300) break;
    if (m > 0) {
      const double ratio = d / dold;
      crate = kCrDown * crate > ratio ? kCrDown * crate : ratio;
    }
    if (d * (crate < 1.0 ? crate : 1.0) <= kNlsCoef) break;
    if (m >= 1 && d > kRdiv * dold) break;
    dold = d;
  }
  for (int m = mlast + 1; m < kMaxCor; ++m) sums[kRedPerIter * m] = NAN;
  BDF_HIP_TRY(hipMemcpyAsync(h->d_ksums, sums, sizeof(sums), hipMemcpyHostToDevice, h->s));
  launch_kry_control(h->dC, h->d_ksums, liters, h->s);
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

// Newton-Krylov: one attempt at a time, the host driving the Krylov
// iterations, then the history update and its controller step.
static int drive_krylov(bdf_handle* h, double* tret) {
  long last_progress = -1;
  for (;;) {
    int st = read_ctrl(h);
    if (st) return st;
    const int ph = h->hC->phase;
    if (ph == PH_ERROR) {
      if (tret) *tret = h->hC->t;
      set_last_error("integrator failure (see status code)", __FILE__, __LINE__);
      return h->hC->status;
    }
    if (ph == PH_DONE || ph == PH_PAUSE) break;
    const long progress = h->hC->nattempts + h->hC->nsteps + h->hC->ncont;
    if (progress == last_progress) {
      set_last_error("integrator made no progress (phase stuck)", __FILE__, __LINE__);
      return BDFGPU_ERR_HIP;
    }
    last_progress = progress;
    if (ph == PH_PREDICT && (st = kry_attempt(h))) return st;
    launch_phase_kernels(h, 3, h->s);
    launch_control(h, 3, h->s);
    BDF_HIP_TRY(hipGetLastError());
  }
  if (tret) *tret = h->hC->t;
  return 0;
}

// Run attempts until the controller leaves the active phases.
static int drive(bdf_handle* h, double tend, long inc, double* tret) {
  if (h->o.linsol == BDFGPU_LS_LEARNED) {
    int st = precond_prepare_inference(reinterpret_cast<precond_handle*>(h->o.precond), h->s);
    if (st) return st;
  }
  hipLaunchKernelGGL(k_resume, dim3(1), dim3(1), 0, h->s, h->dC, tend, inc);
  BDF_HIP_TRY(hipGetLastError());
  launch_phase(h, 0, h->s);   // starting-step estimate (no-ops once done)
  launch_phase(h, 1, h->s);
  BDF_HIP_TRY(hipGetLastError());
  if (h->krylov) return drive_krylov(h, tret);
  const int per = std::max(1, h->o.attempts_per_sync);
  long last_progress = -1;
  for (;;) {
    for (int a = 0; a < per; ++a) {
      if (h->gexec) {
        BDF_HIP_TRY(hipGraphLaunch(h->gexec, h->s));
      } else {
        enqueue_attempt(h, h->s);
      }
    }
    BDF_HIP_TRY(hipGetLastError());
    int st = read_ctrl(h);
    if (st) return st;
    prof_fold(h);
    const int ph = h->hC->phase;
    if (ph == PH_ERROR) {
      if ((st = flush_update(h))) return st;
      BDF_HIP_TRY(hipStreamSynchronize(h->s));
      if (tret) *tret = h->hC->t;
      set_last_error("integrator failure (see status code)", __FILE__, __LINE__);
      return h->hC->status;
    }
    if (ph == PH_DONE || ph == PH_PAUSE) {
      if ((st = flush_update(h))) return st;
      BDF_HIP_TRY(hipStreamSynchronize(h->s));
      break;
    }
    const long progress = h->hC->nattempts + h->hC->nsteps + h->hC->ncont;
    if (progress == last_progress) {
      set_last_error("integrator made no progress (phase stuck)", __FILE__, __LINE__);
      return BDFGPU_ERR_HIP;
    }
    last_progress = progress;
  }
  if (tret) *tret = h->hC->t;
  return 0;
}

// Per-cell stepping: starting steps of the cells not started yet, then
// batches of attempts (every unfinished cell of every class one attempt per
// launch) until no cell is running; the count of running cells after the
// batch's last attempt is the only host read.  Returns the first failing
// cell's status (in class order), if any.
static int cell_dev(bdf_handle* h, const ClassHost& c, double tend, int slot, CellDev* P) {
  *P = c.cell;
  P->tend = tend;
  P->active = h->d_active;
  P->slot = slot;
  P->cap = kCellAttempts;
  P->max_att = h->o.max_steps;
  return 0;
}

static int drive_cells(bdf_handle* h, double tend, double* tret) {
  CellDev P;
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    cell_dev(h, c, tend, 0, &P);
    hipLaunchKernelGGL(k_cell_resume, dim3(ceil_div(c.ncells, 256)), dim3(256), 0, h->s,
                       c.ncells, tend, c.cell.t, c.cell.iv);
    launch_cell(c.np, h->o.linsol, 0, make_dev(h, c), P, c.grid, h->s);
  }
  BDF_HIP_TRY(hipGetLastError());
  // each launch runs up to kCellAttempts attempts per cell; the host reads
  // the number of cells still running after each launch
  for (;;) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, h->s, h->d_active, 1);
    for (const ClassHost& c : h->cls) {
      if (c.ncells == 0) continue;
      cell_dev(h, c, tend, 0, &P);
      launch_cell(c.np, h->o.linsol, 1, make_dev(h, c), P, c.grid, h->s);
    }
    BDF_HIP_TRY(hipGetLastError());
    BDF_HIP_TRY(hipMemcpyAsync(h->h_active, h->d_active, sizeof(unsigned int),
                               hipMemcpyDeviceToHost, h->s));
    BDF_HIP_TRY(hipStreamSynchronize(h->s));
    if (*h->h_active == 0) break;
  }
  if (tret) *tret = tend;
  // the first failed cell's status
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    std::vector<int> iv(4 * c.ncells);
    BDF_HIP_TRY(hipMemcpy(iv.data(), c.cell.iv, sizeof(int) * iv.size(), hipMemcpyDeviceToHost));
    for (long i = 0; i < c.ncells; ++i) {
      const int stc = iv[4 * i + 3];
      if (stc != CELL_DONE && stc != CELL_RUN) {
        set_last_error("per-cell stepping: a cell failed (see status code)", __FILE__, __LINE__);
        return stc;
      }
    }
  }
  return 0;
}

extern "C" {

static int create_impl(const bdf_problem* p, const bdf_options* o, void* stream, void* ws,
                       size_t ws_bytes, bool dry, bdf_handle** out) {
  if (!p || !o || !out) return arg_error("bdf_create: null argument");
  if (p->ncells < 0 || p->ntopo < 1 || !p->topo_n || !p->topo_R || !p->topo_off ||
      !p->nu_all || !p->mu_all ||
      (p->ncells > 0 && (!p->cell_topo || (!dry && (!p->rates || !p->y0)))))
    return arg_error("bdf_create: bad problem description");
  if (o->qmax < 1 || o->qmax > kQmaxAll || o->maxcor < 1 || o->maxcor > kMaxCor ||
      o->newton_per_launch < 0 || !(o->rtol >= 0.0) || !(o->atol > 0.0) ||
      (o->linsol != BDFGPU_LS_LU64 && o->linsol != BDFGPU_LS_LU32REF &&
       o->linsol != BDFGPU_LS_LEARNED && o->linsol != BDFGPU_LS_GJ &&
       o->linsol != BDFGPU_LS_GMRES) ||
      (o->linsol == BDFGPU_LS_LEARNED && !o->precond))
    return arg_error("bdf_create: bad options (qmax 1..5, maxcor 1..4, atol > 0, linsol, precond)");
  if (o->per_cell && ((o->linsol != BDFGPU_LS_LU64 && o->linsol != BDFGPU_LS_GJ) ||
                      o->launch == BDFGPU_LAUNCH_FUSED || o->map_small))
    return arg_error("bdf_create: per-cell stepping needs FP64 LU or the Gauss-Jordan solve, "
                     "per-class launches and one lane per cell");
  if (o->linsol == BDFGPU_LS_GJ && o->launch == BDFGPU_LAUNCH_FUSED)
    return arg_error("bdf_create: the Gauss-Jordan solve needs per-class launches");
  if (o->vc && (o->per_cell || o->no_defer))
    return arg_error("bdf_create: variable coefficients need the deferred history update and "
                     "grouped stepping");
  if (o->lazy && (o->per_cell || o->launch == BDFGPU_LAUNCH_FUSED))
    return arg_error("bdf_create: the lazy Newton matrix needs grouped stepping and per-class "
                     "launches");
  if (o->lazy && o->linsol != BDFGPU_LS_LU64 && o->linsol != BDFGPU_LS_GJ &&
      o->linsol != BDFGPU_LS_GMRES)
    return arg_error("bdf_create: the lazy Newton matrix needs FP64 LU, the Gauss-Jordan solve "
                     "or GMRES");
  if (o->linsol == BDFGPU_LS_GMRES &&
      (o->per_cell || o->vc || o->map_small || o->launch == BDFGPU_LAUNCH_FUSED ||
       o->launch == BDFGPU_LAUNCH_AUTO || o->mode == BDFGPU_MODE_GRAPH))
    return arg_error("bdf_create: GMRES needs grouped stepping with fixed coefficients, one lane "
                     "per cell, per-class launches and stream mode");
  *out = nullptr;
  bdf_handle* h = new bdf_handle();
  h->s = as_stream(stream);
  h->per_cell = o->per_cell != 0;
  h->krylov = o->linsol == BDFGPU_LS_GMRES;
  h->ws = static_cast<char*>(ws);
  h->ws_size = ws_bytes;
  h->dry = dry;
  h->o = *o;
  if (h->o.refine_max_it <= 0) h->o.refine_max_it = 5;
  h->ncells = p->ncells;
  // per-cell user offsets
  std::vector<long> yoff(p->ncells + 1, 0), roff(p->ncells + 1, 0);
  for (long c = 0; c < p->ncells; ++c) {
    const int t = p->cell_topo[c];
    if (t < 0 || t >= p->ntopo) {
      delete h;
      return arg_error("bdf_create: cell_topo out of range");
    }
    yoff[c + 1] = yoff[c] + p->topo_n[t];
    roff[c + 1] = roff[c] + p->topo_R[t];
  }
  h->N = yoff[p->ncells];
  // classes: one per topology that has cells
  std::map<int, std::vector<long>> members;
  for (long c = 0; c < p->ncells; ++c) members[p->cell_topo[c]].push_back(c);
  long blk = 0, mblk = 0;
  int st = 0;
  // per-workgroup LDS limit (160 KiB on gfx950; 64 KiB assumed if unknown)
  // (a dry run without a usable device assumes gfx950's 160 KiB)
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    if (!dry) BDF_HIP_TRY(hipGetDevice(&dev));
    lds_max = 160 * 1024;
  } else if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                 hipSuccess ||
             lds_max < 65536) {
    lds_max = 65536;
  }
  for (auto& kv : members) {
    const int t = kv.first;
    const int n = p->topo_n[t], R = p->topo_R[t];
    if (n < 1 || n > 64 || R < 0) {
      bdf_destroy(h);
      return arg_error("bdf_create: species per cell must be 1..64");
    }
    const int* nu = p->nu_all + p->topo_off[t];
    const int* mu = p->mu_all + p->topo_off[t];
    ClassHost ch;
    ch.topo = t;
    ch.n = n;
    ch.R = R;
    ch.ncells = (long)kv.second.size();
    ch.members = kv.second;
    // thread per cell while the rates and evaluation point fit the LDS of a
    // block (and, with the Gauss-Jordan inverse, for <= 4 species), else
    // segment per cell
    ch.map = (!o->map_small && n <= 12 && (o->linsol != BDFGPU_LS_GJ || n <= 4) &&
              tpc_newton_lds(tpc_padded(n), R, o->linsol, kTpcThreads) <= (size_t)lds_max)
                 ? MAP_TPC
                 : MAP_SPC;
    if (o->per_cell && ch.map != MAP_TPC) {
      bdf_destroy(h);
      return arg_error("bdf_create: per-cell stepping needs cells of <= 12 species (<= 4 with "
                       "the Gauss-Jordan solve)");
    }
    if (ch.map == MAP_SPC && spc_lds_bytes(spc_seg(n), R) > (size_t)lds_max) {
      bdf_destroy(h);
      return arg_error("bdf_create: too many reactions for the block's LDS");
    }
    if (o->linsol == BDFGPU_LS_LEARNED &&
        (ch.map != MAP_SPC || n > 31 ||
         precond_dim(reinterpret_cast<precond_handle*>(o->precond)) != n)) {
      bdf_destroy(h);
      return arg_error("bdf_create: the learned preconditioner needs 13..31 species per cell "
                       "and a network of the preconditioner's size");
    }
    ch.np = ch.map == MAP_TPC ? tpc_padded(n) : spc_seg(n);
    // network-specialised Newton kernel
    if (o->jit && ch.map == MAP_TPC && !dry && o->linsol != BDFGPU_LS_GMRES) {
      st = jit_newton(net_newton_source(nu, mu, n, R, ch.np, o->linsol,
                                        (o->lazy ? 1 : 0) | (o->vc ? 2 : 0)),
                      &ch.jit);
      if (st) {
        bdf_destroy(h);
        return st;
      }
    }
    const int cpb = ch.map == MAP_TPC ? kTpcThreads : kCellThreads / ch.np;
    ch.grid = (unsigned int)std::max<long>(1, (ch.ncells + cpb - 1) / cpb);
    ch.blk0 = blk;
    blk += ch.grid;
    ch.kind = multi_kind(ch.map == MAP_TPC, ch.np);
    ch.mblocks = multi_blocks(ch.kind, ch.np, ch.ncells);
    ch.mblk0 = mblk;
    mblk += ch.mblocks;
    // network tables
    const int np = ch.np;
    std::vector<double> S((size_t)R * np, 0.0);
    std::vector<int> ra(R, -1), rb(R, -1), rc(R, -1);
    // Jacobian entries per column: (reaction, partner, second partner,
    // multiplicity), reactions ascending
    struct JEnt {
      int k, p, p2;
      double m;
    };
    std::vector<std::vector<JEnt>> cols(np);
    bool third = false;
    for (int k = 0; k < R; ++k) {
      int order = 0;
      std::vector<int> reac;
      for (int s2 = 0; s2 < n; ++s2) {
        const int e = nu[k * n + s2];
        if (e < 0 || mu[k * n + s2] < 0) {
          bdf_destroy(h);
          return arg_error("bdf_create: negative stoichiometry");
        }
        for (int r = 0; r < e; ++r) reac.push_back(s2);
        order += e;
        S[(size_t)k * np + s2] = (double)(mu[k * n + s2] - nu[k * n + s2]);
      }
      if (order > 3) {
        bdf_destroy(h);
        return arg_error("bdf_create: reactions may have at most three reactant molecules");
      }
      third = third || order == 3;
      if (order >= 1) ra[k] = reac[0];
      if (order >= 2) rb[k] = reac[1];
      if (order == 3) rc[k] = reac[2];
      // d r / d y_a = e_a kappa prod(other reactant molecules), once per
      // distinct reactant a (reac is sorted)
      for (int i = 0; i < order; ++i) {
        if (i > 0 && reac[i] == reac[i - 1]) continue;
        const int a = reac[i];
        int e = 0;
        std::vector<int> others;
        bool dropped = false;
        for (int r : reac) {
          if (r == a) {
            ++e;
            if (!dropped) {
              dropped = true;
              continue;
            }
          }
          others.push_back(r);
        }
        cols[a].push_back({k, others.size() > 0 ? others[0] : -1,
                           others.size() > 1 ? others[1] : -1, (double)e});
      }
    }
    if (third && (ch.map != MAP_TPC || o->linsol == BDFGPU_LS_LU32REF ||
                  o->linsol == BDFGPU_LS_LEARNED)) {
      bdf_destroy(h);
      return arg_error("bdf_create: three-molecule reactions need one lane per cell (<= 12 "
                       "species) and FP64 LU or the Gauss-Jordan solve");
    }
    // segment kernels read the tables in groups (reactions by 8, each
    // column's entries by 4): padding reactions have no reactant, padding
    // entries a zero multiplicity
    const bool pad = ch.map == MAP_SPC;
    if (pad) {
      ra.resize((size_t)(R + 7) / 8 * 8, -1);
      rb.resize((size_t)(R + 7) / 8 * 8, -1);
      rc.resize((size_t)(R + 7) / 8 * 8, -1);
    }
    std::vector<int> jst(np + 1, 0), jk, jp, jp2;
    std::vector<double> jm;
    for (int a = 0; a < np; ++a) {
      jst[a] = (int)jk.size();
      for (auto& e : cols[a]) {
        jk.push_back(e.k);
        jp.push_back(e.p);
        jp2.push_back(e.p2);
        jm.push_back(e.m);
      }
      while (pad && (jk.size() - (size_t)jst[a]) % 4 != 0) {
        jk.push_back(0);
        jp.push_back(-1);
        jp2.push_back(-1);
        jm.push_back(0.0);
      }
    }
    jst[np] = (int)jk.size();
    NetDev nd;
    nd.n = n;
    nd.R = R;
    nd.np = np;
    if ((st = upload(h, const_cast<double**>(&nd.S), S)) || (st = upload(h, const_cast<int**>(&nd.ra), ra)) ||
        (st = upload(h, const_cast<int**>(&nd.rb), rb)) || (st = upload(h, const_cast<int**>(&nd.rc), rc)) ||
        (st = upload(h, const_cast<int**>(&nd.jst), jst)) ||
        (st = upload(h, const_cast<int**>(&nd.jk), jk)) || (st = upload(h, const_cast<int**>(&nd.jp), jp)) ||
        (st = upload(h, const_cast<int**>(&nd.jp2), jp2)) ||
        (st = upload(h, const_cast<double**>(&nd.jm), jm))) {
      bdf_destroy(h);
      return st;
    }
    // vectors
    const bool tiled = ch.map == MAP_TPC;
    const long cap_cells = tiled ? ((ch.ncells + 63) / 64) * 64 : ch.ncells;
    const size_t vbytes = sizeof(double) * (size_t)std::max<long>(1, cap_cells * n);
    ClassDev& K = ch.dev;
    memset(&K, 0, sizeof(K));
    K.ncells = ch.ncells;
    K.n = n;
    K.R = R;
    K.net = nd;
    K.refine_max_it = h->o.refine_max_it;
    for (int j = 0; j <= kQmaxAll; ++j)
      if ((st = dalloc_zero(h, (void**)&K.z[j], vbytes))) { bdf_destroy(h); return st; }
    if ((st = dalloc_zero(h, (void**)&K.dprev, vbytes))) {
      bdf_destroy(h);
      return st;
    }
    for (int m = 0; m < o->maxcor; ++m)
      if ((st = dalloc(h, (void**)&K.ys[m], vbytes))) {
        bdf_destroy(h);
        return st;
      }
    if (h->krylov && tiled) {   // predicted state, weights, iterate, Krylov basis
      K.vstride = cap_cells * n;
      if ((st = dalloc(h, (void**)&K.zp0, vbytes)) || (st = dalloc(h, (void**)&K.cv, vbytes)) ||
          (st = dalloc(h, (void**)&K.wt, vbytes)) || (st = dalloc(h, (void**)&K.yk, vbytes)) ||
          (st = dalloc_zero(h, (void**)&K.V, vbytes * (kKryMaxl + 1)))) {
        bdf_destroy(h);
        return st;
      }
    }
    if (o->lazy || (h->krylov && tiled)) {   // stored factors of M (or its inverse), pivots
      // thread per cell: NP x NP tiled like the state; segment per cell:
      // NC x NC per cell with NC = n rounded up to 8, the kernel's row width
      const size_t w = tiled ? (size_t)ch.np : (size_t)((n + 7) / 8 * 8);
      if ((st = dalloc(h, (void**)&K.lu, sizeof(double) * std::max<long>(1, cap_cells) * w * w)) ||
          (st = dalloc(h, (void**)&K.lpiv, sizeof(int) * std::max<long>(1, cap_cells) * w))) {
        bdf_destroy(h);
        return st;
      }
    }
    if (o->linsol == BDFGPU_LS_LEARNED) {
      const long nc = std::max<long>(1, ch.ncells);
      if ((st = dalloc(h, (void**)&K.X, sizeof(float) * nc * n * n)) ||
          (st = dalloc(h, (void**)&K.xin, sizeof(double) * nc * (n + 1))) ||
          (st = dalloc(h, (void**)&K.zp0, vbytes)) || (st = dalloc(h, (void**)&K.cv, vbytes))) {
        bdf_destroy(h);
        return st;
      }
    }
    double* rates = nullptr;
    if ((st = dalloc_zero(h, (void**)&rates,
                          sizeof(double) * (size_t)std::max<long>(1, cap_cells * R)))) {
      bdf_destroy(h);
      return st;
    }
    K.rates = rates;
    std::vector<long> cy(ch.ncells), cr(ch.ncells);
    for (long i = 0; i < ch.ncells; ++i) {
      cy[i] = yoff[kv.second[i]];
      cr[i] = roff[kv.second[i]];
    }
    if ((st = upload(h, &ch.d_yoff, cy)) || (st = upload(h, &ch.d_roff, cr))) {
      bdf_destroy(h);
      return st;
    }
    if (o->per_cell) {
      CellDev& P = ch.cell;
      memset(&P, 0, sizeof(P));
      const size_t nc = (size_t)std::max<long>(1, ch.ncells);
      if ((st = dalloc(h, (void**)&P.t, sizeof(double) * nc)) ||
          (st = dalloc(h, (void**)&P.h, sizeof(double) * nc)) ||
          (st = dalloc(h, (void**)&P.hsc, sizeof(double) * nc)) ||
          (st = dalloc(h, (void**)&P.hu, sizeof(double) * nc)) ||
          (st = dalloc(h, (void**)&P.iv, sizeof(int) * 4 * nc)) ||
          (st = dalloc(h, (void**)&P.cnt, sizeof(int) * 5 * nc))) {
        bdf_destroy(h);
        return st;
      }
      P.h0user = o->h0;
      P.hmin = o->hmin;
      P.qmax = o->qmax;
      P.maxcor = o->maxcor;
      if (!dry && ch.ncells > 0)
        hipLaunchKernelGGL(k_cell_setup, dim3(ceil_div(ch.ncells, 256)), dim3(256), 0, h->s,
                           ch.ncells, p->t0, P.t, P.h, P.hsc, P.hu, P.iv, P.cnt);
    }
    if (ch.ncells > 0 && !dry) {
      const unsigned int gy = ceil_div(ch.ncells * n, 256), gr = ceil_div(ch.ncells * (long)R, 256);
      hipLaunchKernelGGL(k_to_class, dim3(gy), dim3(256), 0, h->s, ch.ncells, n, (int)tiled,
                         ch.d_yoff, p->y0, K.z[0], 1.0);
      if (R > 0)
        hipLaunchKernelGGL(k_to_class, dim3(gr), dim3(256), 0, h->s, ch.ncells, R, (int)tiled,
                           ch.d_roff, p->rates, rates, 1.0);
      BDF_HIP_TRY(hipGetLastError());
    }
    h->cls.push_back(ch);
  }
  h->nblocks_total = (unsigned int)blk;
  h->nblocks_multi = (unsigned int)mblk;
  // one launch over all classes: at most kMaxClasses classes, no learned
  // mode, LDS within one workgroup's limit
  h->fusable = h->cls.size() >= 1 && h->cls.size() <= (size_t)kMaxClasses &&
               o->linsol != BDFGPU_LS_LEARNED;
  for (int w = 0; w < 4 && h->fusable; ++w) {
    size_t mx = 0;
    for (const ClassHost& c : h->cls) mx = std::max(mx, multi_lds(c.kind, c.np, c.R, o->linsol, w));
    h->multi_lds[w] = mx;
    if (mx > (size_t)lds_max) h->fusable = false;
  }
  if (h->fusable) {   // queue order: classes by the work of one block, costliest first
    const int nc = (int)h->cls.size();
    for (int k = 0; k < nc; ++k) h->qcls[k] = k;
    std::stable_sort(h->qcls, h->qcls + nc, [&](int a, int b) {
      return multi_block_cost(h->cls[a].kind, h->cls[a].np) >
             multi_block_cost(h->cls[b].kind, h->cls[b].np);
    });
    long e = 0;
    for (int k = 0; k < nc; ++k) h->qend[k] = (e += h->cls[h->qcls[k]].mblocks);
  }
  if (o->launch == BDFGPU_LAUNCH_FUSED && !h->fusable) {
    bdf_destroy(h);
    return arg_error("bdf_create: one launch over all classes needs <= 8 classes, no learned "
                     "preconditioner and per-block LDS within the device limit");
  }
  h->fused = o->launch == BDFGPU_LAUNCH_FUSED;
  // deferred history update: per-class launches of thread-per-cell classes
  // with FP64 or FP32-refined LU
  h->defer = !o->no_defer && !h->fused && o->linsol != BDFGPU_LS_LEARNED && !h->cls.empty() &&
             !o->per_cell;
  for (const ClassHost& c : h->cls)
    if (c.map != MAP_TPC) h->defer = false;
  if (h->krylov) {
    h->defer = false;   // the separate history update follows the Krylov Newton iterations
    for (const ClassHost& c : h->cls)
      if (c.map != MAP_TPC) {
        bdf_destroy(h);
        return arg_error("bdf_create: GMRES needs one lane per cell (<= 12 species)");
      }
    if ((st = dalloc(h, (void**)&h->d_kry, sizeof(double) * 8)) ||
        (st = dalloc(h, (void**)&h->d_ksums, sizeof(double) * kRedNewton))) {
      bdf_destroy(h);
      return st;
    }
  }
  if (o->vc && !h->defer && !h->krylov) {
    bdf_destroy(h);
    return arg_error("bdf_create: variable coefficients need the deferred history update: one "
                     "lane per cell for every class (<= 12 species), per-class launches, no "
                     "learned preconditioner");
  }
  const long bmax = std::max(blk, mblk);
  const long ngroups = std::max<long>(1, (bmax + kRedGroup - 1) / kRedGroup);
  if ((st = dalloc(h, (void**)&h->partials, sizeof(double) * kRedMax * std::max<long>(1, bmax))) ||
      (st = dalloc(h, (void**)&h->gpartials, sizeof(double) * kRedMax * ngroups)) ||
      (st = dalloc(h, (void**)&h->dC, sizeof(Ctrl)))) {
    bdf_destroy(h);
    return st;
  }
  if (o->per_cell &&
      (st = dalloc(h, (void**)&h->d_active, sizeof(unsigned int) * kCellSlots))) {
    bdf_destroy(h);
    return st;
  }
  if (h->fusable && (st = dalloc(h, (void**)&h->d_queue, sizeof(unsigned int)))) {
    bdf_destroy(h);
    return st;
  }
  if (dry) {   // sizes counted: nothing was allocated or launched
    *out = h;
    return 0;
  }
  if (h->fusable)
    for (int w = 0; w < 4; ++w) {
      const unsigned int r = multi_grid(o->linsol, w, h->multi_lds[w]);
      h->multi_grid[w] = r == 0 ? h->nblocks_multi : std::min(r, h->nblocks_multi);
    }
  if (o->per_cell)
    BDF_HIP_TRY(hipHostMalloc((void**)&h->h_active, sizeof(unsigned int), hipHostMallocDefault));
  if (h->krylov)
    BDF_HIP_TRY(hipHostMalloc((void**)&h->h_kry, sizeof(double) * 8, hipHostMallocDefault));
  BDF_HIP_TRY(hipHostMalloc((void**)&h->hC, sizeof(Ctrl), hipHostMallocDefault));
  Ctrl C;
  memset(&C, 0, sizeof(C));
  C.t = p->t0;
  C.tend = p->t0;
  C.hmin = o->hmin;
  C.h0user = o->h0;
  for (int j = 0; j < kQmaxAll + 2; ++j) C.hs[j] = 1.0;
  C.N = (double)h->N;
  C.q = 1;
  C.qmax = o->qmax;
  C.qwait = 2;
  C.maxcor = o->maxcor;
  C.phase = h->N > 0 ? PH_INIT1 : PH_DONE;
  C.learned = o->linsol == BDFGPU_LS_LEARNED ? 1 : 0;
  C.fuse = h->defer ? 1 : 0;
  C.vc = o->vc ? 1 : 0;
  C.lazy = o->lazy ? 1 : 0;
  C.krylov = h->krylov ? 1 : 0;
  // two Newton iterations per fused launch unless asked otherwise (a third,
  // when the replay of the first two leaves the attempt undecided, in a
  // continuation launch); the
  // learned mode keeps per-cell state across its iterations and the GMRES
  // path drives its iterations from the host, so they run all in one
  C.kiters = (C.learned || C.krylov) ? o->maxcor
             : o->newton_per_launch > 0 ? std::min(o->newton_per_launch, o->maxcor)
                                        : std::min(2, o->maxcor);
  C.kap = 1.0;
  C.dscale = 1.0;
  C.setup = 1;
  C.step_limit = LONG_MAX;
  BDF_HIP_TRY(hipMemcpyAsync(h->dC, &C, sizeof(Ctrl), hipMemcpyHostToDevice, h->s));
  BDF_HIP_TRY(hipStreamSynchronize(h->s));
  if (o->mode == BDFGPU_MODE_GRAPH && h->N > 0 && !o->per_cell) {
    st = build_graph(h);
    if (st) {
      bdf_destroy(h);
      return st;
    }
  }
  *out = h;
  return 0;
}

// Autotuning by trial: every candidate launch configuration (per-class
// launches or one launch over all classes; thread per cell or a 16-lane
// segment per cell for classes of <= 12 species) is built from the same
// problem, stepped a few times from the initial state and timed; the
// fastest is then built for the caller.
static constexpr int kTuneWarm = 4, kTuneSteps = 12;

static int create_tuned(const bdf_problem* p, const bdf_options* o, void* stream, void* ws,
                        size_t ws_bytes, bdf_handle** out) {
  if (!p || !o || !out) return arg_error("bdf_create: null argument");
  if (o->launch != BDFGPU_LAUNCH_AUTO) return create_impl(p, o, stream, ws, ws_bytes, false, out);
  bool small = false;
  for (long c = 0; c < p->ncells && !small; ++c) {
    const int t = p->cell_topo ? p->cell_topo[c] : -1;
    if (t >= 0 && t < p->ntopo && p->topo_n[t] <= 12) small = true;
  }
  double ms[4] = {-1.0, -1.0, -1.0, -1.0};
  double best = 1e300;
  int bl = 0, bm = 0;
  for (int launch = 0; launch < 2; ++launch)
    for (int msm = 0; msm < (small ? 2 : 1); ++msm) {
      bdf_options o2 = *o;
      o2.launch = launch;
      o2.map_small = msm;
      o2.mode = BDFGPU_MODE_STREAM;
      bdf_handle* t = nullptr;
      int st = create_impl(p, &o2, stream, ws, ws_bytes, false, &t);
      if (st) {
        if (launch == 1) continue;   // no single launch for this problem
        return st;
      }
      double tr = 0.0;
      long taken = 0;
      st = bdf_advance(t, 1e300, kTuneWarm, &tr, &taken);
      double dt = 1e300;
      if (st == 0) {
        (void)hipStreamSynchronize(t->s);
        const auto t0 = std::chrono::steady_clock::now();
        st = bdf_advance(t, 1e300, kTuneSteps, &tr, &taken);
        (void)hipStreamSynchronize(t->s);
        const auto t1 = std::chrono::steady_clock::now();
        if (st == 0 && taken > 0)
          dt = std::chrono::duration<double, std::milli>(t1 - t0).count() / (double)taken;
      }
      bdf_destroy(t);
      ms[2 * launch + msm] = dt < 1e300 ? dt : -1.0;
      if (dt < best) {
        best = dt;
        bl = launch;
        bm = msm;
      }
    }
  bdf_options o3 = *o;
  o3.launch = bl;
  o3.map_small = bm;
  int st = create_impl(p, &o3, stream, ws, ws_bytes, false, out);
  if (st) return st;
  for (int k = 0; k < 4; ++k) (*out)->tune_ms[k] = ms[k];
  (*out)->tune_launch = bl;
  (*out)->tune_map_small = bm;
  return 0;
}

int bdf_create(const bdf_problem* p, const bdf_options* o, void* stream, bdf_handle** out) {
  return create_tuned(p, o, stream, nullptr, 0, out);
}

int bdf_create_ws(const bdf_problem* p, const bdf_options* o, void* ws, size_t ws_bytes,
                  void* stream, bdf_handle** out) {
  if (!ws && ws_bytes > 0) return arg_error("bdf_create_ws: null workspace");
  if (!ws) {
    if (out) *out = nullptr;
    set_last_error("bdf_create_ws: no workspace (see bdf_workspace_bytes)", __FILE__, __LINE__);
    return BDFGPU_ERR_WORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(ws) % kWsAlign != 0)
    return arg_error("bdf_create_ws: workspace must be 256-byte aligned");
  return create_tuned(p, o, stream, ws, ws_bytes, out);
}

size_t bdf_workspace_bytes(const bdf_problem* p, const bdf_options* o) {
  if (!p || !o) return 0;
  size_t need = 0;
  auto count = [&](const bdf_options& oc) -> bool {
    bdf_handle* t = nullptr;
    if (create_impl(p, &oc, nullptr, nullptr, 0, true, &t) != 0) return false;
    need = std::max(need, t->ws_used);
    bdf_destroy(t);
    return true;
  };
  if (o->launch != BDFGPU_LAUNCH_AUTO) return count(*o) ? need : 0;
  // the autotuner builds every candidate in the same workspace, one at a time
  bool ok = false;
  for (int launch = 0; launch < 2; ++launch)
    for (int msm = 0; msm < 2; ++msm) {
      bdf_options oc = *o;
      oc.launch = launch;
      oc.map_small = msm;
      oc.mode = BDFGPU_MODE_STREAM;
      ok = count(oc) || ok;
    }
  return ok ? need : 0;
}

int bdf_get_tuning(bdf_handle* h, int* launch, int* map_small, double* ms_per_step) {
  if (!h || !launch || !map_small || !ms_per_step) return arg_error("bdf_get_tuning: bad argument");
  *launch = h->fused ? 1 : 0;
  *map_small = h->o.map_small;
  for (int k = 0; k < 4; ++k) ms_per_step[k] = h->tune_ms[k];
  return 0;
}

int bdf_destroy(bdf_handle* h) {
  if (!h) return 0;
  if (h->s) (void)hipStreamSynchronize(h->s);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->hC) (void)hipHostFree(h->hC);
  if (h->h_active) (void)hipHostFree(h->h_active);
  if (h->h_kry) (void)hipHostFree(h->h_kry);
  delete h;
  return 0;
}

long bdf_get_N(bdf_handle* h) { return h ? h->N : -1; }

int bdf_step(bdf_handle* h, double t_end, double* tret) {
  if (!h) return arg_error("bdf_step: null handle");
  if (h->per_cell) return arg_error("bdf_step: per-cell stepping integrates to t_end only");
  if (h->N == 0) {
    if (tret) *tret = t_end;
    return 0;
  }
  return drive(h, t_end, 1, tret);
}

int bdf_advance(bdf_handle* h, double t_end, long nsteps, double* tret, long* taken) {
  if (!h || nsteps < 0) return arg_error("bdf_advance: bad argument");
  if (h->per_cell) return arg_error("bdf_advance: per-cell stepping integrates to t_end only");
  if (taken) *taken = 0;
  if (h->N == 0 || nsteps == 0) {
    if (tret) *tret = h->N == 0 ? t_end : h->hC->t;
    return 0;
  }
  int st = read_ctrl(h);
  if (st) return st;
  const long before = h->hC->nsteps;
  st = drive(h, t_end, nsteps, tret);
  if (taken) *taken = h->hC->nsteps - before;
  return st;
}

int bdf_set_profiling(bdf_handle* h, int on) {
  if (!h) return arg_error("bdf_set_profiling: null handle");
  if (on && h->gexec) return arg_error("bdf_set_profiling: not available in graph mode");
  h->prof = on != 0;
  h->ev_used = 0;
  for (int k = 0; k < 3; ++k) {
    h->prof_ms[k] = 0.0;
    h->prof_cnt[k] = 0;
  }
  return 0;
}

int bdf_get_kernel_times(bdf_handle* h, double* ms, long* counts) {
  if (!h || !ms || !counts) return arg_error("bdf_get_kernel_times: bad argument");
  for (int k = 0; k < 3; ++k) {
    ms[k] = h->prof_ms[k];
    counts[k] = h->prof_cnt[k];
  }
  return 0;
}

int bdf_integrate(bdf_handle* h, double t_end, double* tret) {
  if (!h) return arg_error("bdf_integrate: null handle");
  if (h->N == 0) {
    if (tret) *tret = t_end;
    return 0;
  }
  if (h->per_cell) return drive_cells(h, t_end, tret);
  const long inc = h->o.max_steps > 0 ? h->o.max_steps : LONG_MAX / 4;
  int st = drive(h, t_end, inc, tret);
  if (st) return st;
  if (h->hC->phase == PH_PAUSE && h->hC->t < t_end) {
    set_last_error("max_steps reached before t_end", __FILE__, __LINE__);
    return BDFGPU_ERR_TOO_MUCH_WORK;
  }
  return 0;
}

int bdf_get_y(bdf_handle* h, double* y) {
  if (!h || (!y && h->N > 0)) return arg_error("bdf_get_y: bad argument");
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    hipLaunchKernelGGL(k_from_class, dim3(ceil_div(c.ncells * c.n, 256)), dim3(256), 0, h->s,
                       c.ncells, c.n, (int)(c.map == MAP_TPC), c.d_yoff, c.dev.z[0], y, 1.0);
  }
  BDF_HIP_TRY(hipGetLastError());
  return 0;
}

// Per-cell mode: sums of the cells' counters; t = the earliest cell time,
// h and q of the first cell, status = the first failed cell's.
static int cell_stats_sum(bdf_handle* h, bdf_stats* s) {
  memset(s, 0, sizeof(*s));
  double tmin = 1e300;
  bool first = true;
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    std::vector<int> cnt(5 * c.ncells), iv(4 * c.ncells);
    std::vector<double> t(c.ncells), hh(c.ncells);
    BDF_HIP_TRY(hipMemcpy(cnt.data(), c.cell.cnt, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost));
    BDF_HIP_TRY(hipMemcpy(iv.data(), c.cell.iv, sizeof(int) * iv.size(), hipMemcpyDeviceToHost));
    BDF_HIP_TRY(hipMemcpy(t.data(), c.cell.t, sizeof(double) * t.size(), hipMemcpyDeviceToHost));
    BDF_HIP_TRY(hipMemcpy(hh.data(), c.cell.h, sizeof(double) * hh.size(), hipMemcpyDeviceToHost));
    for (long i = 0; i < c.ncells; ++i) {
      s->nsteps += cnt[5 * i + 0];
      s->nattempts += cnt[5 * i + 1];
      s->nniters += cnt[5 * i + 2];
      s->netfails += cnt[5 * i + 3];
      s->nncfails += cnt[5 * i + 4];
      tmin = std::min(tmin, t[i]);
      const int stc = iv[4 * i + 3];
      if (stc != CELL_DONE && stc != CELL_RUN && s->status == 0) s->status = stc;
      if (first) {
        s->h = hh[i];
        s->q = iv[4 * i + 0];
        first = false;
      }
    }
  }
  s->nsetups = s->nattempts;
  s->nlinsolves = s->nniters;
  s->nfevals = s->nniters;
  s->t = tmin < 1e300 ? tmin : 0.0;
  return 0;
}

int bdf_get_cell_stats(bdf_handle* h, int* counts, double* t, double* hu) {
  if (!h || (!counts && !t && !hu)) return arg_error("bdf_get_cell_stats: bad argument");
  if (!h->per_cell) return arg_error("bdf_get_cell_stats: the handle does not step per cell");
  BDF_HIP_TRY(hipStreamSynchronize(h->s));
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    std::vector<int> cnt(5 * c.ncells);
    std::vector<double> tt(c.ncells), hh(c.ncells);
    BDF_HIP_TRY(hipMemcpy(cnt.data(), c.cell.cnt, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost));
    BDF_HIP_TRY(hipMemcpy(tt.data(), c.cell.t, sizeof(double) * tt.size(), hipMemcpyDeviceToHost));
    BDF_HIP_TRY(hipMemcpy(hh.data(), c.cell.hu, sizeof(double) * hh.size(), hipMemcpyDeviceToHost));
    for (long i = 0; i < c.ncells; ++i) {
      const long u = c.members[i];
      if (counts)
        for (int k = 0; k < 5; ++k) counts[5 * u + k] = cnt[5 * i + k];
      if (t) t[u] = tt[i];
      if (hu) hu[u] = hh[i];
    }
  }
  return 0;
}

int bdf_get_stats(bdf_handle* h, bdf_stats* s) {
  if (!h || !s) return arg_error("bdf_get_stats: bad argument");
  if (h->per_cell) {
    BDF_HIP_TRY(hipStreamSynchronize(h->s));
    return cell_stats_sum(h, s);
  }
  int st = read_ctrl(h);
  if (st) return st;
  const Ctrl& C = *h->hC;
  memset(s, 0, sizeof(*s));
  s->nsteps = C.nsteps;
  s->nattempts = C.nattempts;
  s->nfevals = C.nfevals;
  s->nsetups = C.nsetups;
  s->nniters = C.nniters;
  s->nncfails = C.nncfails;
  s->netfails = C.netfails;
  s->nlinsolves = C.nlinsolves;
  s->refine_sweeps = C.refine_sweeps;
  s->refine_fallbacks = C.refine_fallbacks;
  s->nprojections = C.nprojections;
  s->hist_reads = C.hist_reads;
  s->lp_cell_solves = C.lp_cell_solves;
  s->lp_fallback_cells = C.lp_fallback_cells;
  s->lp_step_fallbacks = C.lp_step_fallbacks;
  s->ncont = C.ncont;
  for (int j = 0; j < 6; ++j) s->order_hist[j] = C.order_hist[j];
  s->t = C.t;
  s->h = C.h;
  s->hu = C.hu;
  s->err_last = C.err;
  s->q = C.q;
  s->qu = C.qu;
  s->qwait = C.qwait;
  s->status = C.status;
  s->nstale_retries = C.nstale_retries;
  s->nliters = C.nliters;
  return 0;
}

int bdf_get_state(bdf_handle* h, double* dvals, int* ivals, double* z6, double* dprev) {
  if (!h || !dvals || !ivals || (h->N > 0 && (!z6 || !dprev)))
    return arg_error("bdf_get_state: bad argument");
  if (h->per_cell) return arg_error("bdf_get_state: not available with per-cell stepping");
  int st = read_ctrl(h);
  if (st) return st;
  const Ctrl C = *h->hC;
  dvals[0] = C.t;
  dvals[1] = C.h;
  ivals[0] = C.q;
  ivals[1] = C.qwait;
  BDF_HIP_TRY(hipMemsetAsync(z6, 0, sizeof(double) * 6 * h->N, h->s));
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    const dim3 g(ceil_div(c.ncells * c.n, 256));
    const int tiled = c.map == MAP_TPC;
    for (int j = 0; j <= C.q && j <= kQmaxAll; ++j)
      hipLaunchKernelGGL(k_from_class, g, dim3(256), 0, h->s, c.ncells, c.n, tiled, c.d_yoff,
                         c.dev.z[j], z6 + (long)j * h->N, C.hs[j]);
    hipLaunchKernelGGL(k_from_class, g, dim3(256), 0, h->s, c.ncells, c.n, tiled, c.d_yoff,
                       c.dev.dprev, dprev, 1.0);
  }
  BDF_HIP_TRY(hipGetLastError());
  BDF_HIP_TRY(hipStreamSynchronize(h->s));
  return 0;
}

int bdf_set_state(bdf_handle* h, const double* dvals, const int* ivals, const double* z6,
                  const double* dprev) {
  if (!h || !dvals || !ivals || (h->N > 0 && (!z6 || !dprev)))
    return arg_error("bdf_set_state: bad argument");
  if (h->per_cell) return arg_error("bdf_set_state: not available with per-cell stepping");
  if (ivals[0] < 1 || ivals[0] > h->o.qmax) return arg_error("bdf_set_state: q out of range");
  int st = read_ctrl(h);
  if (st) return st;
  Ctrl C = *h->hC;
  C.t = dvals[0];
  C.h = dvals[1];
  C.q = ivals[0];
  C.qwait = ivals[1];
  for (int j = 0; j < kQmaxAll + 2; ++j) C.hs[j] = 1.0;
  C.restart = 0;
  C.upd = 0;   // the given history replaces any pending update
  C.ntau = 0;      // variable coefficients: no known past points
  C.m_valid = 0;   // lazy: no stored factors for this state
  C.ncf = 0;
  C.netf = 0;
  C.phase = PH_PAUSE;
  for (const ClassHost& c : h->cls) {
    if (c.ncells == 0) continue;
    const dim3 g(ceil_div(c.ncells * c.n, 256));
    const int tiled = c.map == MAP_TPC;
    for (int j = 0; j <= kQmaxAll; ++j)
      hipLaunchKernelGGL(k_to_class, g, dim3(256), 0, h->s, c.ncells, c.n, tiled, c.d_yoff,
                         z6 + (long)j * h->N, c.dev.z[j], 1.0);
    hipLaunchKernelGGL(k_to_class, g, dim3(256), 0, h->s, c.ncells, c.n, tiled, c.d_yoff, dprev,
                       c.dev.dprev, 1.0);
  }
  BDF_HIP_TRY(hipGetLastError());
  BDF_HIP_TRY(hipMemcpyAsync(h->dC, &C, sizeof(Ctrl), hipMemcpyHostToDevice, h->s));
  BDF_HIP_TRY(hipStreamSynchronize(h->s));
  return 0;
}

int bdf_capture_blocks(bdf_handle* h, int n, long stride, long max_blocks, double* X_raw,
                       double* M, long* got) {
  if (!h || stride < 1 || max_blocks < 0 || !got || (max_blocks > 0 && (!X_raw || !M)))
    return arg_error("bdf_capture_blocks: bad argument");
  *got = 0;
  const ClassHost* cl = nullptr;
  for (const ClassHost& c : h->cls)
    if (c.n == n) cl = &c;
  if (!cl) return arg_error("bdf_capture_blocks: no class with that many species");
  int st = read_ctrl(h);
  if (st) return st;
  const Ctrl& C = *h->hC;
  const double gamma = C.h / harmonic(C.q);   // h l_0 with l_0 = 1 / H_q
  const long ns = std::min(max_blocks, (cl->ncells + stride - 1) / stride);
  if (ns <= 0) return 0;
  hipLaunchKernelGGL(k_capture, dim3(ceil_div(ns, 64)), dim3(64), 0, h->s, ns, stride, n,
                     (int)(cl->map == MAP_TPC), cl->dev.net, cl->dev.z[0], cl->dev.rates, gamma,
                     X_raw, M);
  BDF_HIP_TRY(hipGetLastError());
  BDF_HIP_TRY(hipStreamSynchronize(h->s));
  *got = ns;
  return 0;
}

int bdf_eval_rhs_jac(bdf_handle* h, const double* y, double* f, double* J) {
  if (!h || (h->N > 0 && !y)) return arg_error("bdf_eval_rhs_jac: bad argument");
  // J offsets per class cell (user order of cells, blocks n_c^2)
  if (h->d_joff.empty()) {
    // recover the global cell order from the per-class y offsets
    std::vector<std::pair<long, std::pair<int, long>>> order;   // (yoff, (class, idx))
    std::vector<std::vector<long>> cy(h->cls.size());
    for (size_t k = 0; k < h->cls.size(); ++k) {
      const ClassHost& c = h->cls[k];
      cy[k].resize(c.ncells);
      if (c.ncells)
        BDF_HIP_TRY(hipMemcpy(cy[k].data(), c.d_yoff, sizeof(long) * c.ncells, hipMemcpyDeviceToHost));
      for (long i = 0; i < c.ncells; ++i) order.push_back({cy[k][i], {(int)k, i}});
    }
    std::sort(order.begin(), order.end());
    std::vector<std::vector<long>> jo(h->cls.size());
    for (size_t k = 0; k < h->cls.size(); ++k) jo[k].resize(h->cls[k].ncells);
    long acc = 0;
    for (auto& e : order) {
      const int k = e.second.first;
      jo[k][e.second.second] = acc;
      acc += (long)h->cls[k].n * h->cls[k].n;
    }
    for (size_t k = 0; k < h->cls.size(); ++k) {
      long* d = nullptr;
      BDF_HIP_TRY(hipMalloc(&d, sizeof(long) * std::max<size_t>(1, jo[k].size())));
      h->allocs.push_back(d);
      if (!jo[k].empty())
        BDF_HIP_TRY(hipMemcpy(d, jo[k].data(), sizeof(long) * jo[k].size(), hipMemcpyHostToDevice));
      h->d_joff.push_back(d);
    }
  }
  for (size_t k = 0; k < h->cls.size(); ++k) {
    const ClassHost& c = h->cls[k];
    if (c.ncells == 0) continue;
    // rates back to user layout are not kept; evaluate from the class copy
    // through a temporary cell-major copy of the rates
    double* rtmp = nullptr;
    BDF_HIP_TRY(hipMalloc(&rtmp, sizeof(double) * std::max<long>(1, c.ncells * c.R)));
    std::vector<long> ro(c.ncells);
    for (long i = 0; i < c.ncells; ++i) ro[i] = i * c.R;
    long* dro = nullptr;
    BDF_HIP_TRY(hipMalloc(&dro, sizeof(long) * std::max<long>(1, c.ncells)));
    BDF_HIP_TRY(hipMemcpy(dro, ro.data(), sizeof(long) * c.ncells, hipMemcpyHostToDevice));
    if (c.R > 0)
      hipLaunchKernelGGL(k_from_class, dim3(ceil_div(c.ncells * (long)c.R, 256)), dim3(256), 0,
                         h->s, c.ncells, c.R, (int)(c.map == MAP_TPC), dro, c.dev.rates, rtmp,
                         1.0);
    hipLaunchKernelGGL(k_eval_rhs_jac, dim3(ceil_div(c.ncells, 128)), dim3(128), 0, h->s,
                       c.ncells, c.dev.net, c.d_yoff, dro, h->d_joff[k], rtmp, y, f, J);
    BDF_HIP_TRY(hipGetLastError());
    BDF_HIP_TRY(hipStreamSynchronize(h->s));
    (void)hipFree(rtmp);
    (void)hipFree(dro);
  }
  return 0;
}

}  // extern "C"
