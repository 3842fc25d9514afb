// Network-specialised thread-per-cell Newton kernels.
//
// The table-driven kernel reads each reaction's species indices from the
// network tables at run time; every index lookup is a scalar load followed
// by a dependent LDS read of the state, and the scalar and LDS loads share
// one wait counter, so the lookups serialise.  For a given network the
// indices are constants: the generated policy below evaluates f, M = I -
// gamma J and (I - gamma J) x as straight-line code over the network's
// nonzeros (a reaction touches at most four species), with the state read
// from the LDS column at constant offsets.  It performs the same floating
// point operations in the same order as NetTables (zero terms dropped: they
// add +-0 exactly), with contraction off, so both kernels give identical
// bits; the rest of the kernel is the shared tpc_newton_body.
//
// The source and a launcher are compiled with hipcc into a small shared
// library that is loaded with dlopen, the way the prebuilt kernels are
// loaded.  (The same machine code loaded as a hipRTC module ran 15% slower
// on MI355X, with identical kernel descriptor and metadata.)  Libraries are
// cached on disk by a hash of everything that goes into them.
#include "bdf_jit.hpp"

#include <dlfcn.h>
#include <fcntl.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cerrno>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <utility>
#include <vector>

extern char** environ;

#include "common.hpp"

// kJitHeaderNames / kJitHeaderTexts / kJitHeaders: the device headers,
// embedded at build time so that the generated kernels compile against the
// same templates as the prebuilt ones
#include "jit_headers.inc"

namespace bdfgpu {

namespace {

struct Reaction {
  int a = -1, b = -1, c = -1;   // reactant species (a <= b <= c), -1 if absent
  std::vector<int> s;           // net stoichiometry mu - nu, length n
  std::vector<int> reac;        // reactant molecules, sorted
};

std::vector<Reaction> reactions(const int* nu, const int* mu, int n, int R) {
  std::vector<Reaction> out(R);
  for (int k = 0; k < R; ++k) {
    std::vector<int> reac;
    out[k].s.assign(n, 0);
    for (int i = 0; i < n; ++i) {
      for (int e = 0; e < nu[k * n + i]; ++e) reac.push_back(i);
      out[k].s[i] = mu[k * n + i] - nu[k * n + i];
    }
    if (reac.size() >= 1) out[k].a = reac[0];
    if (reac.size() >= 2) out[k].b = reac[1];
    if (reac.size() >= 3) out[k].c = reac[2];
    out[k].reac = reac;
  }
  return out;
}

// dst += S v with the rounding of fma(S, v, dst)
void emit_update(std::ostringstream& o, const std::string& dst, int S, const char* v,
                 const char* ind) {
  if (S == 1)
    o << ind << dst << " = " << dst << " + " << v << ";\n";
  else if (S == -1)
    o << ind << dst << " = " << dst << " - " << v << ";\n";
  else
    o << ind << dst << " = fma(" << S << ".0, " << v << ", " << dst << ");\n";
}

}  // namespace

std::string net_newton_source(const int* nu, const int* mu, int n, int R, int np, int ls,
                              int mode) {
  const std::vector<Reaction> rx = reactions(nu, mu, n, R);
  std::vector<bool> react(n, false);
  for (const Reaction& r : rx)
    for (int x : r.reac) react[x] = true;
  // Jacobian entries per column a in the order of the network tables:
  // reaction k ascending; (k, partners or -1, multiplicity): once per
  // distinct reactant a, dr/dy_a = e_a kappa prod(the other molecules)
  struct Ent {
    int k, p, p2;
    double m;
  };
  std::vector<std::vector<Ent>> cols(n);
  for (int k = 0; k < R; ++k) {
    const std::vector<int>& rc = rx[k].reac;
    for (size_t i = 0; i < rc.size(); ++i) {
      if (i > 0 && rc[i] == rc[i - 1]) continue;
      const int a = rc[i];
      int e = 0;
      std::vector<int> others;
      bool dropped = false;
      for (int x : rc) {
        if (x == a) {
          ++e;
          if (!dropped) {
            dropped = true;
            continue;
          }
        }
        others.push_back(x);
      }
      cols[a].push_back({k, others.size() > 0 ? others[0] : -1, others.size() > 1 ? others[1] : -1,
                         (double)e});
    }
  }

  std::ostringstream o;
  o << "// generated: Newton kernel for a network of " << n << " species and " << R
    << " reactions\n#include <hip/hip_runtime.h>\n\n#include \"bdf_dev.hpp\"\n\n"
       "namespace bdfgpu {\nstruct NetGen {\n";

  // f
  o << "  template <int NP, int T>\n"
       "  __device__ static __forceinline__ void rhs(const NetDev&, const double* kcol, int ks,\n"
       "                                             const double* ycol, double (&f)[NP]) {\n"
       "#pragma clang fp contract(off)\n"
       "#pragma unroll\n"
       "    for (int i = 0; i < NP; ++i) f[i] = 0.0;\n";
  for (int i = 0; i < n; ++i)
    if (react[i]) o << "    const double y" << i << " = ycol[" << i << " * T];\n";
  for (int k = 0; k < R; ++k) {
    const Reaction& r = rx[k];
    o << "    {\n      double r = kcol[" << k << " * ks];\n";
    if (r.a >= 0) o << "      r *= y" << r.a << ";\n";
    if (r.b >= 0) o << "      r *= y" << r.b << ";\n";
    if (r.c >= 0) o << "      r *= y" << r.c << ";\n";
    for (int i = 0; i < n; ++i)
      if (r.s[i] != 0) emit_update(o, "f[" + std::to_string(i) + "]", r.s[i], "r", "      ");
    o << "    }\n";
  }
  o << "  }\n\n";

  // M = I - gamma J, column by column
  o << "  template <int NP, int T, typename TT, bool ROWSUM>\n"
       "  __device__ static __forceinline__ void build_M(const NetDev&, const double* kcol, int ks,\n"
       "                                                 const double* ycol, double gamma,\n"
       "                                                 TT (&M)[NP][NP], double (&rowsum)[NP]) {\n"
       "#pragma clang fp contract(off)\n"
       "#pragma unroll\n"
       "    for (int i = 0; i < NP; ++i) rowsum[i] = 0.0;\n";
  for (int i = 0; i < n; ++i)
    if (react[i]) o << "    const double y" << i << " = ycol[" << i << " * T];\n";
  for (int a = 0; a < np; ++a) {
    std::vector<bool> touched(np, false);
    if (a < n)
      for (const Ent& e : cols[a])
        for (int i = 0; i < n; ++i)
          if (rx[e.k].s[i] != 0) touched[i] = true;
    o << "    {\n";
    for (int i = 0; i < np; ++i)
      if (touched[i]) o << "      double c" << i << " = 0.0;\n";
    if (a < n)
      for (const Ent& e : cols[a]) {
        o << "      {\n        double g = kcol[" << e.k << " * ks] * " << (int)e.m << ".0;\n";
        if (e.p >= 0) o << "        g *= y" << e.p << ";\n";
        if (e.p2 >= 0) o << "        g *= y" << e.p2 << ";\n";
        for (int i = 0; i < n; ++i)
          if (rx[e.k].s[i] != 0) emit_update(o, "c" + std::to_string(i), rx[e.k].s[i], "g", "        ");
        o << "      }\n";
      }
    for (int i = 0; i < np; ++i) {
      const char* d = i == a ? "1.0" : "0.0";
      if (touched[i]) {
        o << "      {\n        const double m = fma(-gamma, c" << i << ", " << d << ");\n"
          << "        M[" << i << "][" << a << "] = (TT)m;\n"
          << "        if (ROWSUM) rowsum[" << i << "] += fabs(m);\n      }\n";
      } else {
        o << "      M[" << i << "][" << a << "] = (TT)" << d << ";\n";
        if (i == a) o << "      if (ROWSUM) rowsum[" << i << "] += 1.0;\n";
      }
    }
    o << "    }\n";
  }
  o << "  }\n\n";

  // (I - gamma J) x
  o << "  template <int NP, int T>\n"
       "  __device__ static __forceinline__ void mvp(const NetDev&, const double* kcol, int ks,\n"
       "                                             const double* ycol, const double* xcol,\n"
       "                                             double gamma, const double (&x)[NP],\n"
       "                                             double (&out)[NP]) {\n"
       "#pragma clang fp contract(off)\n"
       "    double jx[NP];\n"
       "#pragma unroll\n"
       "    for (int i = 0; i < NP; ++i) jx[i] = 0.0;\n";
  for (int i = 0; i < n; ++i)
    if (react[i])
      o << "    const double y" << i << " = ycol[" << i << " * T], x" << i << " = xcol[" << i
        << " * T];\n";
  for (int k = 0; k < R; ++k) {
    const Reaction& r = rx[k];
    if (r.a < 0) continue;
    o << "    {\n      const double kk = kcol[" << k << " * ks];\n";
    if (r.b < 0)
      o << "      const double d = kk * x" << r.a << ";\n";
    else if (r.c < 0)
      o << "      const double d = kk * fma(x" << r.a << ", y" << r.b << ", y" << r.a << " * x"
        << r.b << ");\n";
    else   // three molecules (the FP32-refined solve, which uses this, refuses them)
      o << "      const double d = kk * (x" << r.a << " * y" << r.b << " * y" << r.c << " + y"
        << r.a << " * x" << r.b << " * y" << r.c << " + y" << r.a << " * y" << r.b << " * x"
        << r.c << ");\n";
    for (int i = 0; i < n; ++i)
      if (r.s[i] != 0) emit_update(o, "jx[" + std::to_string(i) + "]", r.s[i], "d", "      ");
    o << "    }\n";
  }
  o << "#pragma unroll\n"
       "    for (int i = 0; i < NP; ++i) out[i] = fma(-gamma, jx[i], x[i]);\n"
       "  }\n};\n}  // namespace bdfgpu\n\n";

  // named by block size and solver so that profiles keep the variants apart
  const std::string kname = "bdf_newton_net_np" + std::to_string(np) + "_ls" + std::to_string(ls) +
                            (mode ? "_m" + std::to_string(mode) : std::string());
  o << "__global__ void __launch_bounds__(bdfgpu::kTpcThreads) " << kname
    << "(bdfgpu::BdfDev D) {\n"
       "  extern __shared__ double lds[];\n"
       "  if (D.C->phase != bdfgpu::PH_PREDICT) return;\n"
       "  bdfgpu::tpc_newton_body<"
    << np << ", " << ls << ", bdfgpu::kTpcThreads, bdfgpu::NetGen, " << (R < 1 ? 1 : R > 24 ? 24 : R)
    << ", " << (n == np ? "true" : "false") << ", " << mode
    << ">(D, blockIdx.x, lds);\n}\n\n"
       "// dynamic LDS above 64 KiB is requested once per process\n"
       "extern \"C\" void bdf_newton_net_launch(const bdfgpu::BdfDev* D, unsigned int grid,\n"
       "                                      unsigned int lds, hipStream_t s) {\n"
       "  static unsigned int raised = 65536;\n"
       "  if (lds > raised && hipFuncSetAttribute(reinterpret_cast<const void*>(&"
    << kname
    << "),\n"
       "                                          hipFuncAttributeMaxDynamicSharedMemorySize,\n"
       "                                          (int)lds) == hipSuccess)\n"
       "    raised = lds;\n"
       "  hipLaunchKernelGGL("
    << kname << ", dim3(grid), dim3(bdfgpu::kTpcThreads), lds, s, *D);\n}\n";
  return o.str();
}

namespace {

std::mutex g_jit_mu;
std::map<std::string, NetLaunch> g_jit_cache;   // source -> launcher

const char* const kHipccFlags[] = {"-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
                                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                   "-Wno-unused-command-line-argument", "-Wno-unused-variable"};

uint64_t fnv1a(uint64_t h, const std::string& s) {
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

bool mkdirs(const std::string& path) {
  std::string cur;
  std::stringstream ss(path);
  std::string part;
  if (!path.empty() && path[0] == '/') cur = "/";
  while (std::getline(ss, part, '/')) {
    if (part.empty()) continue;
    cur += part + "/";
    if (mkdir(cur.c_str(), 0700) != 0 && errno != EEXIST) return false;
  }
  return true;
}

bool write_file(const std::string& path, const std::string& text) {
  const std::string tmp = path + ".tmp" + std::to_string(getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return false;
    f << text;
    if (!f) return false;
  }
  return rename(tmp.c_str(), path.c_str()) == 0;
}

std::string cache_root() {
  if (const char* d = getenv("BDFGPU_JIT_DIR")) return d;
  const char* t = getenv("TMPDIR");
  return std::string(t && *t ? t : "/tmp") + "/bdfgpu-jit-" + std::to_string(getuid());
}

std::string hipcc_path() {
  if (const char* c = getenv("HIPCC")) return c;
  return "/opt/rocm/bin/hipcc";
}

// Runs hipcc on dir/pkg/csrc/net.hip as a child process (stdout and stderr
// into dir/build.log); 0 on success.
int run_hipcc(const std::string& dir, const std::string& out) {
  const std::string cc = hipcc_path();
  if (access(cc.c_str(), X_OK) != 0) return -1;
  std::vector<std::string> args = {cc};
  for (const char* f : kHipccFlags) args.push_back(f);
  args.push_back(dir + "/pkg/csrc/net.hip");
  args.push_back("-o");
  args.push_back(out);
  std::vector<char*> argv;
  for (std::string& a : args) argv.push_back(&a[0]);
  argv.push_back(nullptr);
  posix_spawn_file_actions_t fa;
  posix_spawn_file_actions_init(&fa);
  const std::string log = dir + "/build.log";
  posix_spawn_file_actions_addopen(&fa, 1, log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
  posix_spawn_file_actions_adddup2(&fa, 1, 2);
  pid_t pid = 0;
  const int rc = posix_spawn(&pid, cc.c_str(), &fa, nullptr, argv.data(), environ);
  posix_spawn_file_actions_destroy(&fa);
  if (rc != 0) return -1;
  int status = 0;
  while (waitpid(pid, &status, 0) < 0)
    if (errno != EINTR) return -1;
  return WIFEXITED(status) && WEXITSTATUS(status) == 0 ? 0 : -1;
}

std::string read_tail(const std::string& path, size_t n) {
  std::ifstream f(path);
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  return t.size() > n ? t.substr(t.size() - n) : t;
}

}  // namespace

int jit_newton(const std::string& src, NetLaunch* fn) {
  std::lock_guard<std::mutex> lk(g_jit_mu);
  auto it = g_jit_cache.find(src);
  if (it != g_jit_cache.end()) {
    *fn = it->second;
    return 0;
  }
  // everything that goes into the library: source, headers, flags
  uint64_t h = fnv1a(1469598103934665603ull, src);
  for (int i = 0; i < kJitHeaders; ++i) {
    h = fnv1a(h, kJitHeaderNames[i]);
    h = fnv1a(h, kJitHeaderTexts[i]);
  }
  for (const char* f : kHipccFlags) h = fnv1a(h, f);
  char hex[17];
  snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)h);
  const std::string dir = cache_root() + "/" + hex;
  const std::string lib = dir + "/net.so";
  if (access(lib.c_str(), R_OK) != 0) {
    // headers under the relative paths their #include lines use
    if (!mkdirs(dir + "/pkg/csrc") || !mkdirs(dir + "/include"))
      return arg_error("jit: cannot create the kernel cache directory (BDFGPU_JIT_DIR)");
    for (int i = 0; i < kJitHeaders; ++i) {
      const std::string name = kJitHeaderNames[i];
      const std::string path = name.rfind("../../", 0) == 0 ? dir + "/" + name.substr(6)
                                                            : dir + "/pkg/csrc/" + name;
      if (!write_file(path, kJitHeaderTexts[i])) return arg_error("jit: cannot write headers");
    }
    if (!write_file(dir + "/pkg/csrc/net.hip", src)) return arg_error("jit: cannot write source");
    const std::string tmp = lib + ".tmp" + std::to_string(getpid());
    if (run_hipcc(dir, tmp) != 0) {
      const std::string msg = "jit: hipcc (" + hipcc_path() + ") failed: " +
                              read_tail(dir + "/build.log", 400);
      set_last_error(msg.c_str(), __FILE__, __LINE__);
      return BDFGPU_ERR_HIP;
    }
    if (rename(tmp.c_str(), lib.c_str()) != 0) return arg_error("jit: cannot place the library");
  }
  // the library stays loaded until the process ends: handles of any age use it
  void* so = dlopen(lib.c_str(), RTLD_NOW | RTLD_LOCAL);
  if (!so) {
    const std::string msg = std::string("jit: dlopen failed: ") + dlerror();
    set_last_error(msg.c_str(), __FILE__, __LINE__);
    return BDFGPU_ERR_HIP;
  }
  NetLaunch f = reinterpret_cast<NetLaunch>(dlsym(so, "bdf_newton_net_launch"));
  if (!f) return arg_error("jit: launcher symbol missing");
  g_jit_cache.emplace(src, f);
  *fn = f;
  return 0;
}

}  // namespace bdfgpu
