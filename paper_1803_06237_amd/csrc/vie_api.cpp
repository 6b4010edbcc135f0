// C ABI of the voxel J-VIE solver: plan lifetime, contrast, matvec and the
// GMRES / flexible-GMRES drivers.  See include/vie.h for the contract.
#include "../../include/vie.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <algorithm>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "krylov.hpp"
#include "vie_internal.hpp"

namespace vie {
template <typename T>
hipError_t allow_lds(size_t bytes);
hipError_t net_apply(vie_net_s* N, const double2* r, const double2* w, const double2* chi, double2* z);
const int* net_grid(vie_net_s* N);
void net_set_stream(vie_net_s* N, hipStream_t s);
}

using namespace vie;

namespace {

thread_local std::string g_thread_error;

// Host Toeplitz tables depend only on (grid, kappa); plans of one process share them.
std::shared_ptr<const std::vector<std::complex<double>>> cached_table(const int n[3], double kappa) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, double>, std::shared_ptr<const std::vector<std::complex<double>>>> cache;
  const auto key = std::make_tuple(n[0], n[1], n[2], kappa);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  auto t = std::make_shared<std::vector<std::complex<double>>>((size_t)6 * n[0] * n[1] * n[2]);
  vie::green_table(n, kappa, t->data(), 0);
  std::lock_guard<std::mutex> lk(mu);
  if (cache.size() >= 16) cache.clear();
  cache[key] = t;
  return t;
}

std::shared_ptr<const std::vector<std::complex<double>>> cached_curl_table(const int n[3], double kappa) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, double>, std::shared_ptr<const std::vector<std::complex<double>>>> cache;
  const auto key = std::make_tuple(n[0], n[1], n[2], kappa);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  auto t = std::make_shared<std::vector<std::complex<double>>>((size_t)3 * n[0] * n[1] * n[2]);
  vie::curl_table(n, kappa, t->data(), 0);
  std::lock_guard<std::mutex> lk(mu);
  if (cache.size() >= 16) cache.clear();
  cache[key] = t;
  return t;
}

template <typename T>
struct GmresWs {
  long n = 0;
  int m = 0;
  bool flex = false;
  cx<T>* V = nullptr;
  cx<T>* Z = nullptr;
  double2* partial = nullptr;
  double2* h1 = nullptr;
  double2* h2 = nullptr;
  double2* sumsq = nullptr;
  double2* H = nullptr;
  double2* sn = nullptr;
  double2* g = nullptr;
  double2* y = nullptr;
  double* cs = nullptr;
  double* state = nullptr;
  double* state_h = nullptr;
  int* gate = nullptr;   // second Gram-Schmidt sweep needed (device flag)
  hipEvent_t ev[2] = {nullptr, nullptr};   // step j's state copied to state_h + 4 (j & 1)
  bool borrowed = false;  // pointers lent by the caller (static scratch): never freed or resized

  void release() {
    if (borrowed) return;
    for (void* p : {(void*)V, (void*)Z, (void*)partial, (void*)h1, (void*)h2, (void*)sumsq, (void*)H, (void*)sn,
                    (void*)g, (void*)y, (void*)cs, (void*)state, (void*)gate})
      if (p) (void)hipFree(p);
    if (state_h) (void)hipHostFree(state_h);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    *this = GmresWs();
  }
  hipError_t ensure(long n_, int m_, bool flex_) {
    if (n_ == n && m_ == m && flex_ == flex && V) return hipSuccess;
    if (borrowed) return hipErrorInvalidValue;
    release();
    n = n_;
    m = m_;
    flex = flex_;
    const long nb = partial_blocks(n);
    hipError_t e;
    if ((e = dmalloc(&V, sizeof(cx<T>) * (size_t)n * (m + 1)))) return e;
    if (flex && (e = dmalloc(&Z, sizeof(cx<T>) * (size_t)n * m))) return e;
    if ((e = dmalloc(&partial, sizeof(double2) * (size_t)nb * (m + 1)))) return e;
    if ((e = dmalloc(&h1, sizeof(double2) * (m + 2)))) return e;
    if ((e = dmalloc(&h2, sizeof(double2) * (m + 2)))) return e;
    if ((e = dmalloc(&sumsq, sizeof(double2) * 2))) return e;
    if ((e = dmalloc(&gate, sizeof(int)))) return e;
    if ((e = dmalloc(&H, sizeof(double2) * (size_t)(m + 1) * m))) return e;
    if ((e = dmalloc(&sn, sizeof(double2) * (m + 1)))) return e;
    if ((e = dmalloc(&g, sizeof(double2) * (m + 1)))) return e;
    if ((e = dmalloc(&y, sizeof(double2) * (m + 1)))) return e;
    if ((e = dmalloc(&cs, sizeof(double) * (m + 1)))) return e;
    if ((e = dmalloc(&state, sizeof(double) * 4))) return e;
    if ((e = hipHostMalloc(&state_h, sizeof(double) * 8, hipHostMallocDefault))) return e;
    for (hipEvent_t& ev_i : ev)
      if ((e = hipEventCreateWithFlags(&ev_i, hipEventDisableTiming))) return e;
    return hipSuccess;
  }
};

}  // namespace

struct vie_plan_s {
  Geom g{};
  double h = 0, k0 = 0, eps_b = 0, kappa = 0;
  unsigned flags = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  Tune t64{}, t32{};
  double2* goct64 = nullptr;
  float2* goct32 = nullptr;
  double2* chi64 = nullptr;
  float2* chi32 = nullptr;
  double2* U64 = nullptr;
  float2* U32 = nullptr;
  double2* tw64[3] = {nullptr, nullptr, nullptr};
  float2* tw32[3] = {nullptr, nullptr, nullptr};
  double2* rvec = nullptr;     // FP64 scratch vector (residuals)
  float2* v32a = nullptr;      // FP32 scratch vectors (mixed tier)
  float2* v32b = nullptr;
  // support of the contrast (voxel columns with chi != 0 on some slice); the
  // solver keeps its Krylov vectors compressed to these columns
  int* colflag = nullptr;      // device, n1 n2 flags
  int* scol = nullptr;         // device, ns column indices i1 n2 + i2, increasing
  int ns = 0;
  double2* fx = nullptr;       // full FP64 operator input, zero off the support
  double2* fy = nullptr;       // full FP64 operator output
  double2* fw = nullptr;       // full FP64 base vector (learned-circulant tier)
  float2* fx32 = nullptr;      // the same in FP32 (mixed tier)
  float2* fy32 = nullptr;
  double2* bc = nullptr;       // compressed right-hand side and solution
  double2* xc = nullptr;
  double2* partial_full = nullptr;   // reduction scratch for full-length norms
  double2* sumsq_full = nullptr;
  int* flag = nullptr;
  bool has_contrast = false;
  vie_net_s* net = nullptr;    // learned preconditioner (not owned)
  vie::Circ* circ = nullptr;   // block-circulant preconditioner of the current contrast
  // JM-VIE (vie_jm_enable): spectrum of K = curl S on the octant, magnetic
  // contrast (mu_r - 1)/mu_r, the magnetic half's z-pass intermediate, the full
  // cross-section spectra of the six components, FP32 vectors of the mixed tier
  bool jm = false;
  double2* koct64 = nullptr;
  float2* koct32 = nullptr;
  double2* chim64 = nullptr;
  float2* chim32 = nullptr;
  double2* Um64 = nullptr;
  float2* Um32 = nullptr;
  double2* S64 = nullptr;
  float2* S32 = nullptr;
  float2* jm32a = nullptr;
  float2* jm32b = nullptr;
  bool jm_fused64 = false;   // cross-section pass with the spectra in LDS (else through S64 / S32)
  bool jm_fused32 = false;
  std::shared_ptr<const std::vector<std::complex<double>>> table;   // host Toeplitz table
  GmresWs<double> ws64;
  GmresWs<float> ws32;
  GmresWs<double> ws64i;       // inner FP64-Arnoldi solves of the mixed tier (precision 5)
  // created by vie_plan for vie_solve_noalloc, which may not create them itself
  hipEvent_t nev[2] = {nullptr, nullptr};
  double* npin = nullptr;      // pinned host slot, 8 doubles
  std::string err;
};

namespace {

int fail(vie_plan_s* p, int code, const std::string& msg) {
  if (p) p->err = msg;
  else g_thread_error = msg;
  return code;
}

int hipfail(vie_plan_s* p, hipError_t e, const char* where) {
  return fail(p, VIE_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPTRY(p, expr)                                     \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return hipfail((p), _e, #expr);   \
  } while (0)

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

template <typename T>
bool pick_tune(const Geom& g, size_t budget, size_t zbudget, Tune* t) {
  const size_t cs = sizeof(cx<T>);
  int tp = 16;
  const int n1p = 1 << ilog2(g.n1);
  if (tp > n1p) tp = n1p;
  while (tp > 1 && (size_t)tp * (g.M3 + 1) * cs > zbudget) tp >>= 1;
  if ((size_t)tp * (g.M3 + 1) * cs > budget) return false;
  t->tp = tp;
  int zt = (tp * g.M3 + 15) / 16;
  zt = ((zt + 63) / 64) * 64;
  if (zt < 64) zt = 64;
  if (zt > 1024) return false;
  t->zthreads = zt < 256 ? (tp * g.M3 >= 256 ? 256 : zt) : zt;
  // generic xy pass (cross-sections other than 64 x 64): column chunk cc within
  // the LDS budget, at most 8 values per thread per transform stage
  int cc = g.M1 < 16 ? g.M1 : 16;
  while (cc > 1 && xy_lds_bytes<T>(g, cc) > budget) cc >>= 1;
  if (xy_lds_bytes<T>(g, cc) > budget) return false;
  t->cc = cc;
  int need = 3 * g.n2 * g.M1;
  if (3 * g.M2 * cc > need) need = 3 * g.M2 * cc;
  int xt = (need + 7) / 8;
  xt = ((xt + 63) / 64) * 64;
  if (xt < 512) xt = 512;
  if (xt > 1024) return false;
  t->xythreads = xt;
  const size_t z4 = z4_lds_bytes<T>(g.M3);
  t->z4 = (z4 > 0 && z4 <= budget) ? 1 : 0;
  t->xyv = sizeof(T) == 8 ? 1 : 0;
  t->zp = 0;
  return true;
}

// ---- plan-time tuning of launch shapes ----------------------------------------
// Candidates: the four-step z passes' pencils per workgroup (the forward and the
// inverse pass share the choice) and the 64 x 64 xy pass variant.  Each candidate
// runs two untimed and five timed whole products (all three passes) between HIP
// events; the fastest wins.  Results are kept per (device, grid, precision) for
// the life of the process and in the tuner cache file.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, Tune> g_tune_cache;

template <typename T>
hipError_t time_passes(const Geom& g, const Tune& t, int w0, int w1, const void* x, void* y, void* U,
                       const void* goct, const void* chi, const void* const tw[3], hipStream_t s, float* ms) {
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0))) return e;
  if ((e = hipEventCreate(&e1))) return e;
  for (int r = 0; r < 7 && !e; ++r) {
    if (r == 2) e = hipEventRecord(e0, s);
    for (int w = w0; w <= w1 && !e; ++w) e = launch_pass<T>(w, g, t, x, y, nullptr, 0, U, goct, chi, tw, s);
  }
  if (!e) e = hipEventRecord(e1, s);
  if (!e) e = hipEventSynchronize(e1);
  if (!e) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

// Persistent tuner cache: one line "arch n1 n2 n3 value_bytes z4 zp xyv" per tuned
// shape, in the file named by VIE_TUNE_CACHE (empty: no file), by default
// $XDG_CACHE_HOME/vie-mi355x/tune.txt or $HOME/.cache/vie-mi355x/tune.txt.  A
// process reads it before timing candidates and appends what it tunes; the last
// line for a key wins.  Lines are appended with one write each.
std::string tune_cache_path() {
  if (const char* v = std::getenv("VIE_TUNE_CACHE")) return v;
  std::string dir;
  if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = x;
  else if (const char* h = std::getenv("HOME"); h && *h) dir = std::string(h) + "/.cache";
  else return "";
  return dir + "/vie-mi355x/tune.txt";
}

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return (colon == std::string::npos ? a : a.substr(0, colon)) + "-cu" + std::to_string(prop.multiProcessorCount);
}

bool tune_cache_lookup(const std::string& arch, const Geom& g, int vb, Tune* t) {
  const std::string path = tune_cache_path();
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char a[128];
  int n1, n2, n3, b, z4, zp, xyv;
  bool found = false;
  Tune best = *t;
  while (std::fscanf(f, "%127s %d %d %d %d %d %d %d", a, &n1, &n2, &n3, &b, &z4, &zp, &xyv) == 8) {
    if (arch == a && n1 == g.n1 && n2 == g.n2 && n3 == g.n3 && b == vb) {
      best.z4 = z4;
      best.zp = zp;
      best.xyv = xyv;
      found = true;
    }
  }
  std::fclose(f);
  // only shapes this build can launch
  if (found) {
    int opts[8];
    const int n = vb == 16 ? z4_pencil_options<double>(g.M3, opts, 8) : z4_pencil_options<float>(g.M3, opts, 8);
    bool ok = best.xyv >= 0 && best.xyv <= 2 && (best.z4 == 0 || best.z4 == 1) && (t->z4 || !best.z4);
    if (best.z4) {
      bool hit = false;
      for (int i = 0; i < n; ++i) hit = hit || opts[i] == best.zp;
      ok = ok && hit;
    }
    if (ok) *t = best;
    return ok;
  }
  return false;
}

void tune_cache_store(const std::string& arch, const Geom& g, int vb, const Tune& t) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    // create the directory chain (errors ignored: the cache is optional)
    for (size_t i = 1; i <= slash; ++i)
      if (path[i] == '/' || i == slash) (void)::mkdir(path.substr(0, i == slash ? slash : i).c_str(), 0755);
  }
  char line[256];
  const int len = std::snprintf(line, sizeof line, "%s %d %d %d %d %d %d %d\n", arch.c_str(), g.n1, g.n2, g.n3, vb,
                                t.z4, t.zp, t.xyv);
  const int fd = ::open(path.c_str(), O_WRONLY | O_CREAT | O_APPEND, 0644);
  if (fd < 0) return;
  (void)!::write(fd, line, (size_t)len);
  ::close(fd);
}

template <typename T>
hipError_t autotune(const Geom& g, int device, Tune* t, void* U, const void* goct, const void* chi,
                    const void* const tw[3], hipStream_t s) {
  const auto key = std::make_tuple(device, g.n1, g.n2, g.n3, (int)sizeof(T));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *t = it->second;
      return hipSuccess;
    }
  }
  // the suffix names the candidate set: lines written for an older set are not read
  const std::string arch = device_arch(device) + "/xy6432";
  if (tune_cache_lookup(arch, g, (int)sizeof(cx<T>), t)) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = *t;
    return hipSuccess;
  }
  const size_t bytes = sizeof(cx<T>) * 3 * (size_t)g.N;
  void* x = nullptr;
  void* y = nullptr;
  hipError_t e = dmalloc(&x, bytes);
  if (!e) e = dmalloc(&y, bytes);
  if (!e) e = hipMemsetAsync(x, 0, bytes, s);
  // Every candidate is timed in three interleaved rounds and keeps its best
  // round: single rounds let launch noise decide between shapes within 1 % of
  // each other, and the choice then changed from one process to the next.
  constexpr int kRounds = 3;
  // Candidates: the four-step pencil counts and the generic LDS z passes (the
  // 64-value shapes of long pencils run at low occupancy in FP64), crossed with
  // the xy variants of 64 x 64 planes.  They are timed jointly, as whole
  // back-to-back products: the z pass's write pattern decides what the xy pass
  // finds in L2 and the Infinity Cache, so a pass timed alone, or with events
  // between the passes, can rank the shapes differently (FP64 32x32x512: with
  // events between the passes 8 pencils per workgroup look 7 us faster than 4;
  // back to back, 4 stay ahead).
  std::vector<Tune> cand;
  {
    std::vector<Tune> zc;
    if (t->z4) {
      int opts[8];
      const int n = z4_pencil_options<T>(g.M3, opts, 8);
      for (int i = 0; i < n; ++i) {
        Tune c = *t;
        c.zp = opts[i];
        zc.push_back(c);
      }
      Tune c = *t;
      c.z4 = 0;
      c.zp = 0;
      zc.push_back(c);
    } else {
      zc.push_back(*t);
    }
    const int nv = xy_variants(g);
    for (const Tune& z : zc)
      for (int v = 0; v < nv; ++v) {
        Tune c = z;
        if (nv > 1) c.xyv = v;
        cand.push_back(c);
      }
  }
  if (cand.size() > 1) {
    std::vector<float> best(cand.size(), INFINITY);
    for (int r = 0; r < kRounds && !e; ++r) {
      for (size_t i = 0; i < cand.size() && !e; ++i) {
        float ms = 0;
        e = time_passes<T>(g, cand[i], 0, 2, x, y, U, goct, chi, tw, s, &ms);
        if (!e && ms < best[i]) best[i] = ms;
      }
    }
    size_t bi = 0;
    for (size_t i = 1; i < cand.size(); ++i)
      if (best[i] < best[bi]) bi = i;
    if (!e) *t = cand[bi];
  }
  if (x) (void)hipFree(x);
  if (y) (void)hipFree(y);
  if (!e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = *t;
    tune_cache_store(arch, g, (int)sizeof(cx<T>), *t);
  }
  return e;
}

template <typename T>
hipError_t make_twiddles(int M, cx<T>** out) {
  std::vector<cx<T>> h(M);
  for (int k = 0; k < M; ++k) {
    long double a = -2.0L * 3.14159265358979323846264338327950288L * k / M;
    h[k] = cx<T>{(T)std::cos(a), (T)std::sin(a)};
  }
  hipError_t e = dmalloc(out, sizeof(cx<T>) * M);
  if (e) return e;
  return hipMemcpy(*out, h.data(), sizeof(cx<T>) * M, hipMemcpyHostToDevice);
}

// ---- operator wrappers used by the solvers ---------------------------------
struct Op64 {
  vie_plan_s* p;
  hipError_t apply(const double2* x, double2* y) {
    const void* tw[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    return launch_matvec<double>(p->g, p->t64, x, y, nullptr, 0, p->U64, p->goct64, p->chi64, tw, p->stream);
  }
  hipError_t residual(const double2* x, const double2* b, double2* r) {
    const void* tw[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    return launch_matvec<double>(p->g, p->t64, x, r, b, 1, p->U64, p->goct64, p->chi64, tw, p->stream);
  }
};
struct Op32 {
  vie_plan_s* p;
  hipError_t apply(const float2* x, float2* y) {
    const void* tw[3] = {p->tw32[0], p->tw32[1], p->tw32[2]};
    return launch_matvec<float>(p->g, p->t32, x, y, nullptr, 0, p->U32, p->goct32, p->chi32, tw, p->stream);
  }
  hipError_t residual(const float2* x, const float2* b, float2* r) {
    const void* tw[3] = {p->tw32[0], p->tw32[1], p->tw32[2]};
    return launch_matvec<float>(p->g, p->t32, x, r, b, 1, p->U32, p->goct32, p->chi32, tw, p->stream);
  }
};

// The operator on support-compressed vectors: scatter into a full vector that is
// zero off the support, FFT product, gather the support back.
struct Op64c {
  vie_plan_s* p;
  Support u;
  double2* fx;   // full-length input (zero off the support) and output
  double2* fy;
  hipError_t full(const double2* xc) {
    hipError_t e = scatter<double>(u, xc, fx, p->stream);
    if (e) return e;
    const void* tw[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    return launch_matvec<double>(p->g, p->t64, fx, fy, nullptr, 0, p->U64, p->goct64, p->chi64, tw, p->stream);
  }
  hipError_t apply(const double2* xc, double2* yc) {
    hipError_t e = full(xc);
    return e ? e : gather<double>(u, fy, yc, nullptr, p->stream);
  }
  hipError_t residual(const double2* xc, const double2* bc, double2* rc) {
    hipError_t e = full(xc);
    return e ? e : gather<double>(u, fy, rc, bc, p->stream);
  }
};
struct Op32c {
  vie_plan_s* p;
  Support u;
  hipError_t full(const float2* xc) {
    hipError_t e = scatter<float>(u, xc, p->fx32, p->stream);
    if (e) return e;
    const void* tw[3] = {p->tw32[0], p->tw32[1], p->tw32[2]};
    return launch_matvec<float>(p->g, p->t32, p->fx32, p->fy32, nullptr, 0, p->U32, p->goct32, p->chi32, tw,
                                p->stream);
  }
  hipError_t apply(const float2* xc, float2* yc) {
    hipError_t e = full(xc);
    return e ? e : gather<float>(u, p->fy32, yc, nullptr, p->stream);
  }
  hipError_t residual(const float2* xc, const float2* bc, float2* rc) {
    hipError_t e = full(xc);
    return e ? e : gather<float>(u, p->fy32, rc, bc, p->stream);
  }
};

// The FP32 product on FP64 support-compressed vectors: the inner solve of the mixed
// tier with FP64 Arnoldi (precision 5).  x is rounded to FP32, the FP32 product runs
// on the full grid, the gathered result is widened back to FP64.
struct Op32in64c {
  vie_plan_s* p;
  Support u;
  long n;
  hipError_t apply(const double2* xc, double2* yc) {
    hipError_t e = convert<double, float>(xc, p->v32a, n, p->stream);
    if (e) return e;
    if ((e = scatter<float>(u, p->v32a, p->fx32, p->stream))) return e;
    const void* tw[3] = {p->tw32[0], p->tw32[1], p->tw32[2]};
    if ((e = launch_matvec<float>(p->g, p->t32, p->fx32, p->fy32, nullptr, 0, p->U32, p->goct32, p->chi32, tw,
                                  p->stream)))
      return e;
    if ((e = gather<float>(u, p->fy32, p->v32b, nullptr, p->stream))) return e;
    return convert<float, double>(p->v32b, yc, n, p->stream);
  }
  // the inner solve starts from zero and never confirms a true residual
  hipError_t residual(const double2*, const double2*, double2*) { return hipErrorNotSupported; }
};

// The JM-VIE operator on full 6N vectors (electric, then magnetic in impedance units).
struct OpJM64 {
  vie_plan_s* p;
  hipError_t run(const double2* x, double2* y, const double2* b, int mode) {
    const void* tw[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    return launch_jm_matvec<double>(p->g, p->t64, x, y, b, mode, p->U64, p->Um64, p->S64, p->goct64, p->koct64,
                                    p->chi64, p->chim64, p->kappa, p->jm_fused64, tw, p->stream);
  }
  hipError_t apply(const double2* x, double2* y) { return run(x, y, nullptr, 0); }
  hipError_t residual(const double2* x, const double2* b, double2* r) { return run(x, r, b, 1); }
};
struct OpJM32 {
  vie_plan_s* p;
  hipError_t run(const float2* x, float2* y, const float2* b, int mode) {
    const void* tw[3] = {p->tw32[0], p->tw32[1], p->tw32[2]};
    return launch_jm_matvec<float>(p->g, p->t32, x, y, b, mode, p->U32, p->Um32, p->S32, p->goct32, p->koct32,
                                   p->chi32, p->chim32, p->kappa, p->jm_fused32, tw, p->stream);
  }
  hipError_t apply(const float2* x, float2* y) { return run(x, y, nullptr, 0); }
  hipError_t residual(const float2* x, const float2* b, float2* r) { return run(x, r, b, 1); }
};

struct Stats {
  int iters = 0, restarts = 0, matvecs = 0, inner = 0, fallback = 0;
  double est = 0, rel_true = INFINITY;
  int stall_k = 0;   // in: stop after this many restarts without progress (0: never)
  int stalled = 0;   // out: stopped by that rule
};

// least relative decrease of the true residual per restart that counts as progress
constexpr double kStallDrop = 1e-3;

struct NoPrecond {
  hipError_t operator()(const void*, void*, Stats&) { return hipSuccess; }
};

hipError_t read_scalar(const double2* d, double* out, double* pinned, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(pinned, d, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e) return e;
  if ((e = hipStreamSynchronize(s))) return e;
  *out = pinned[0];
  return hipSuccess;
}

// GMRES(m) (flexible when a preconditioner is given) on basis type T.
// check_true: confirm convergence with the true residual and restart until then.
template <typename T, typename OP, typename PC>
int gmres_core(vie_plan_s* p, GmresWs<T>& W, OP& A, PC* M, long n, const cx<T>* b, cx<T>* x, double tol, int m,
               int maxit, bool use_x0, bool check_true, Stats& st) {
  using K = KrylovOps<T>;
  hipStream_t s = p->stream;
  HIPTRY(p, W.ensure(n, m, M != nullptr));
  double bsq = 0;
  HIPTRY(p, K::nrm2sq(b, n, W.partial, W.sumsq, s));
  HIPTRY(p, read_scalar(W.sumsq, &bsq, W.state_h, s));
  if (!std::isfinite(bsq)) return fail(p, VIE_EINVAL, "right-hand side is not finite");
  const double bnorm = std::sqrt(bsq);
  if (bnorm == 0.0) {
    HIPTRY(p, K::zero(x, n, s));
    st.rel_true = 0;
    return VIE_OK;
  }
  cx<T>* V0 = W.V;
  if (use_x0) {
    HIPTRY(p, A.residual(x, b, V0));
    st.matvecs++;
  } else {
    HIPTRY(p, K::zero(x, n, s));
    HIPTRY(p, hipMemcpyAsync(V0, b, sizeof(cx<T>) * n, hipMemcpyDeviceToDevice, s));
  }
  double beta2 = 0;
  HIPTRY(p, K::nrm2sq(V0, n, W.partial, W.sumsq, s));
  HIPTRY(p, read_scalar(W.sumsq, &beta2, W.state_h, s));
  double rel = std::sqrt(beta2) / bnorm;
  st.est = rel;
  int status = VIE_ENOCONV;
  const int ldh = m + 1;
  // stagnation: the true residual of each restart against the best so far
  double best = rel;
  int since = 0, cycles = 0;
  while (true) {
    if (!std::isfinite(rel)) return fail(p, VIE_ENUMERIC, "non-finite residual");
    if (rel <= tol) {
      status = VIE_OK;
      break;
    }
    if (st.iters >= maxit) break;
    if (check_true && st.stall_k > 0 && cycles > 0) {
      if (rel < best * (1.0 - kStallDrop)) {
        best = rel;
        since = 0;
      } else if (++since >= st.stall_k) {
        st.stalled = 1;
        break;
      }
    }
    ++cycles;
    HIPTRY(p, K::set_g(W.g, m, W.sumsq, s));
    HIPTRY(p, K::scale(V0, V0, n, W.sumsq, s));
    // One Arnoldi step queued on the stream, ending with a copy of its state
    // (residual estimate, breakdown, non-finite flags) to pinned slot j & 1.
    auto step = [&](int j) -> hipError_t {
      cx<T>* Vj = W.V + (long)j * n;
      cx<T>* w = W.V + (long)(j + 1) * n;
      const cx<T>* z = Vj;
      hipError_t e;
      if (M) {
        cx<T>* Zj = W.Z + (long)j * n;
        if ((e = (*M)(Vj, Zj, st))) return e;
        z = Zj;
      }
      if ((e = A.apply(z, w))) return e;
      st.matvecs++;
      if ((e = K::mdot(W.V, n, j + 1, w, n, W.partial, W.h1, 0, s))) return e;
      if (j + 1 <= 512) {
        // the multi-axpy also sums |w'|^2 per block; one block reduces and takes
        // the second-sweep decision (decided on the device)
        const int nbm = maxpy_blocks(n);
        if ((e = K::template maxpy_nrm<T>(W.V, n, j + 1, W.h1, -1.0, w, n, W.partial, s))) return e;
        if ((e = K::reduce_dgks(W.partial, nbm, W.sumsq, W.h1, j + 1, W.gate, W.h2, s))) return e;
        if ((e = K::mdot(W.V, n, j + 1, w, n, W.partial, W.h2, 0, s, W.gate))) return e;
        if ((e = K::template maxpy_nrm<T>(W.V, n, j + 1, W.h2, -1.0, w, n, W.partial, s, W.gate))) return e;
        if ((e = K::reduce(W.partial, nbm, W.sumsq, s, W.gate))) return e;
      } else {
        if ((e = K::template maxpy<T>(W.V, n, j + 1, W.h1, -1.0, w, n, s))) return e;
        if ((e = K::nrm2sq(w, n, W.partial, W.sumsq, s))) return e;
        // second sweep only where the first cancelled too much (decided on the device)
        if ((e = K::dgks(W.h1, j + 1, W.sumsq, W.gate, W.h2, s))) return e;
        if ((e = K::mdot(W.V, n, j + 1, w, n, W.partial, W.h2, 0, s, W.gate))) return e;
        if ((e = K::template maxpy<T>(W.V, n, j + 1, W.h2, -1.0, w, n, s, W.gate))) return e;
        if ((e = K::nrm2sq(w, n, W.partial, W.sumsq, s, W.gate))) return e;
      }
      if ((e = K::scale(w, w, n, W.sumsq, s))) return e;
      if ((e = K::arnoldi_update(W.h1, W.h2, W.sumsq, W.H, ldh, W.cs, W.sn, W.g, j, bnorm, W.state, s))) return e;
      if ((e = hipMemcpyAsync(W.state_h + 4 * (j & 1), W.state, 3 * sizeof(double), hipMemcpyDeviceToHost, s)))
        return e;
      return hipEventRecord(W.ev[j & 1], s);
    };
    // Without a preconditioner the steps are pipelined: step j + 1 is queued
    // before the host waits for step j's state, so the device does not idle
    // through the host round trip.  A step queued after convergence is
    // discarded: it writes only V_{j+2}, Hessenberg column j + 1 and g_{j+1},
    // g_{j+2}, none of which the solution with k = j + 1 columns reads.  (The
    // flexible variant's preconditioner synchronises by itself.)
    const bool pipe = M == nullptr;
    int k = 0;
    if (pipe) HIPTRY(p, step(0));
    for (int j = 0; j < m; ++j) {
      if (!pipe) HIPTRY(p, step(j));
      else if (j + 1 < m && st.iters + 2 <= maxit) HIPTRY(p, step(j + 1));
      HIPTRY(p, hipEventSynchronize(W.ev[j & 1]));
      const double* sh = W.state_h + 4 * (j & 1);
      st.iters++;
      k = j + 1;
      st.est = sh[0];
      if (sh[2] != 0.0) {
        (void)hipStreamSynchronize(s);
        return fail(p, VIE_ENUMERIC, "non-finite value in Arnoldi step");
      }
      if (sh[0] <= tol || sh[1] == 0.0 || st.iters >= maxit) break;
    }
    HIPTRY(p, K::trisolve(W.H, ldh, W.g, k, W.y, s));
    HIPTRY(p, K::template maxpy<T>(M ? W.Z : W.V, n, k, W.y, 1.0, x, n, s));
    st.restarts++;
    if (!check_true) {
      status = st.est <= tol ? VIE_OK : VIE_ENOCONV;
      HIPTRY(p, hipStreamSynchronize(s));
      break;
    }
    HIPTRY(p, A.residual(x, b, V0));
    st.matvecs++;
    HIPTRY(p, K::nrm2sq(V0, n, W.partial, W.sumsq, s));
    HIPTRY(p, read_scalar(W.sumsq, &beta2, W.state_h, s));
    rel = std::sqrt(beta2) / bnorm;
    st.rel_true = rel;
  }
  if (check_true) st.rel_true = rel;
  return status;
}

}  // namespace

int vie::plan_export(vie_plan_t p, Geom* g, Tune* t64, Tune* t32, void** U64, void** U32, void** goct64,
                     void** goct32, void** chi64, void** chi32, const void** tw64, const void** tw32,
                     hipStream_t* stream, int* has_contrast) {
  if (!p) return VIE_EINVAL;
  *g = p->g;
  *t64 = p->t64;
  *t32 = p->t32;
  *U64 = p->U64;
  *U32 = p->U32;
  *goct64 = p->goct64;
  *goct32 = p->goct32;
  *chi64 = p->chi64;
  *chi32 = p->chi32;
  for (int d = 0; d < 3; ++d) {
    tw64[d] = p->tw64[d];
    tw32[d] = p->tw32[d];
  }
  *stream = p->stream;
  *has_contrast = p->has_contrast ? 1 : 0;
  return VIE_OK;
}

vie::Circ* vie::plan_circ(vie_plan_t p) { return p ? p->circ : nullptr; }

int vie::plan_support(vie_plan_t p, const int** col, int* ns) {
  if (!p || !p->has_contrast) return VIE_ESTATE;
  *col = p->scol;
  *ns = p->ns;
  return VIE_OK;
}

hipError_t vie::dmalloc_bytes(void** p, size_t bytes) {
  static const bool nanfill = [] {
    const char* v = std::getenv("VIE_DEBUG_NANFILL");
    return v && v[0] == '1';
  }();
  hipError_t e = hipMalloc(p, bytes);
  if (e || !nanfill || bytes == 0) return e;
  if ((e = hipMemset(*p, 0xFF, bytes))) return e;
  return hipDeviceSynchronize();
}

size_t vie::lds_budget(int device) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v <= 0)
    v = 65536;
  return (size_t)v;
}

// ---- static scratch of the allocation-free entry point ------------------------
// vie_solve_noalloc takes every device buffer beyond its inputs and outputs from
// this array: the full-length operator vectors, the compressed right-hand side and
// solution, the reduction partials and the Krylov workspace.  Each GPU holds its
// own copy for the life of the process.  Host code never uses the array's name as
// an address: vie_plan looks its device address up once per device (with that
// device current) and every use goes through that pointer.
namespace {
constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

void scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
  g_scratch_done[device] = true;
}

// Bump allocation inside the scratch array, 256-byte aligned.
struct ScratchCarver {
  unsigned char* base;
  size_t used = 0;
  template <typename P>
  P* take(size_t count) {
    used = (used + 255) & ~(size_t)255;
    P* r = reinterpret_cast<P*>(base + used);
    used += sizeof(P) * (count ? count : 1);
    return r;
  }
};
}  // namespace

extern "C" {

const char* vie_version(void) { return "vie-mi355x 0.1 (gfx950)"; }

const char* vie_last_error(vie_plan_t plan) { return plan ? plan->err.c_str() : g_thread_error.c_str(); }

int vie_green_table(const int grid[3], double kappa, vie_c128* out, int nthreads) {
  if (!grid || !out) return fail(nullptr, VIE_EINVAL, "null argument");
  for (int d = 0; d < 3; ++d)
    if (grid[d] < 1 || grid[d] > 4096) return fail(nullptr, VIE_EINVAL, "grid size out of range");
  if (!std::isfinite(kappa)) return fail(nullptr, VIE_EINVAL, "kappa not finite");
  vie::green_table(grid, kappa, reinterpret_cast<std::complex<double>*>(out), nthreads);
  return VIE_OK;
}

int vie_plan(vie_plan_t* out, const int grid[3], double h, double k0, double eps_b, unsigned flags,
             void* hip_stream) {
  if (!out || !grid) return fail(nullptr, VIE_EINVAL, "null argument");
  *out = nullptr;
  if (!(h > 0) || !(k0 > 0) || !(eps_b > 0) || !std::isfinite(h) || !std::isfinite(k0) || !std::isfinite(eps_b))
    return fail(nullptr, VIE_EINVAL, "h, k0 and eps_b must be positive and finite");
  const int lim[3] = {32, 32, 2048};
  for (int d = 0; d < 3; ++d)
    if (grid[d] < 1 || grid[d] > lim[d]) return fail(nullptr, VIE_EINVAL, "grid outside n1,n2 <= 32, n3 <= 2048");
  auto* p = new vie_plan_s();
  p->h = h;
  p->k0 = k0;
  p->eps_b = eps_b;
  p->kappa = k0 * std::sqrt(eps_b) * h;
  p->flags = flags;
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  Geom& g = p->g;
  g.n1 = grid[0];
  g.n2 = grid[1];
  g.n3 = grid[2];
  int Ms[3];
  for (int d = 0; d < 3; ++d) {
    int M = 1;
    while (M < 2 * grid[d] - 1) M <<= 1;
    Ms[d] = M;
  }
  g.M1 = Ms[0];
  g.M2 = Ms[1];
  g.M3 = Ms[2];
  g.L1 = ilog2(g.M1);
  g.L2 = ilog2(g.M2);
  g.L3 = ilog2(g.M3);
  g.H1 = g.M1 / 2 + 1;
  g.H2 = g.M2 / 2 + 1;
  g.H3 = g.M3 / 2 + 1;
  g.N = (long)g.n1 * g.n2 * g.n3;
  auto bail = [&](int code) {
    vie_destroy(p);
    return code;
  };
  hipError_t e;
  if ((e = hipGetDevice(&p->device))) return bail(hipfail(nullptr, e, "hipGetDevice"));
  scratch_init(p->device);
  for (hipEvent_t& ev : p->nev)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming))) return bail(hipfail(nullptr, e, "hipEventCreate"));
  if ((e = hipHostMalloc(&p->npin, sizeof(double) * 8, hipHostMallocDefault)))
    return bail(hipfail(nullptr, e, "hipHostMalloc"));
  const size_t budget = lds_budget(p->device);
  const size_t zbudget = budget < 65536 ? budget : 65536;
  if (!pick_tune<double>(g, budget, zbudget, &p->t64) || !pick_tune<float>(g, budget, zbudget, &p->t32))
    return bail(fail(nullptr, VIE_EINVAL, "grid does not fit the LDS budget"));
  if ((e = allow_lds<double>(budget)) || (e = allow_lds<float>(budget)))
    return bail(hipfail(nullptr, e, "hipFuncSetAttribute"));
  // host table
  const auto table = cached_table(grid, p->kappa);
  p->table = table;
  const bool f32 = (flags & VIE_WITH_FP32) != 0;
  const long H = (long)g.H1 * g.H2 * g.H3;
  const long P = (long)g.M1 * g.M2 * g.M3;
  double2* table_dev = nullptr;
  double2* full = nullptr;
  auto cleanup_tmp = [&]() {
    if (table_dev) (void)hipFree(table_dev);
    if (full) (void)hipFree(full);
  };
#define PLANTRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) {                             \
      cleanup_tmp();                                    \
      return bail(hipfail(nullptr, _e, #expr));         \
    }                                                   \
  } while (0)
  for (int d = 0; d < 3; ++d) {
    PLANTRY(make_twiddles<double>(Ms[d], &p->tw64[d]));
    PLANTRY(make_twiddles<float>(Ms[d], &p->tw32[d]));
  }
  PLANTRY(dmalloc(&p->goct64, sizeof(double2) * 6 * H));
  if (f32) PLANTRY(dmalloc(&p->goct32, sizeof(float2) * 6 * H));
  PLANTRY(dmalloc(&p->chi64, sizeof(double2) * g.N));
  PLANTRY(dmalloc(&p->chi32, sizeof(float2) * g.N));
  PLANTRY(dmalloc(&p->U64, sizeof(double2) * 3 * (size_t)g.n1 * g.n2 * g.M3));
  if (f32) PLANTRY(dmalloc(&p->U32, sizeof(float2) * 3 * (size_t)g.n1 * g.n2 * g.M3));
  PLANTRY(dmalloc(&p->rvec, sizeof(double2) * 3 * g.N));
  PLANTRY(dmalloc(&p->flag, sizeof(int)));
  PLANTRY(dmalloc(&p->colflag, sizeof(int) * (size_t)g.n1 * g.n2));
  PLANTRY(dmalloc(&p->scol, sizeof(int) * (size_t)g.n1 * g.n2));
  PLANTRY(dmalloc(&table_dev, sizeof(double2) * 6 * g.N));
  PLANTRY(dmalloc(&full, sizeof(double2) * P));
  PLANTRY(hipMemcpyAsync(table_dev, table->data(), sizeof(double2) * 6 * g.N, hipMemcpyHostToDevice, p->stream));
  {
    const double2* tw[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    PLANTRY(launch_spectrum(g, table_dev, full, p->goct64, p->goct32, tw, p->stream));
  }
  PLANTRY(hipStreamSynchronize(p->stream));
  cleanup_tmp();
  table_dev = full = nullptr;
  if (!(flags & VIE_NO_AUTOTUNE)) {
    // launch-shape tuning on the plan's own buffers; the contrast is zeroed first
    // (set_contrast overwrites it)
    const void* tw64[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    const void* tw32[3] = {p->tw32[0], p->tw32[1], p->tw32[2]};
    PLANTRY(hipMemsetAsync(p->chi64, 0, sizeof(double2) * g.N, p->stream));
    PLANTRY(hipMemsetAsync(p->chi32, 0, sizeof(float2) * g.N, p->stream));
    PLANTRY(autotune<double>(g, p->device, &p->t64, p->U64, p->goct64, p->chi64, tw64, p->stream));
    if (f32) PLANTRY(autotune<float>(g, p->device, &p->t32, p->U32, p->goct32, p->chi32, tw32, p->stream));
  }
#undef PLANTRY
  *out = p;
  return VIE_OK;
}

int vie_set_contrast(vie_plan_t p, const vie_c128* eps) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!eps) return fail(p, VIE_EINVAL, "null eps");
  if (p->circ) {
    HIPTRY(p, hipStreamSynchronize(p->stream));
    circ_destroy(p->circ);
    p->circ = nullptr;
  }
  HIPTRY(p, hipMemsetAsync(p->flag, 0, sizeof(int), p->stream));
  HIPTRY(p, launch_contrast(p->g.N, reinterpret_cast<const double2*>(eps), p->eps_b, p->chi64, p->chi32, p->flag,
                            p->stream));
  int bad = 0;
  HIPTRY(p, hipMemcpyAsync(&bad, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPTRY(p, hipStreamSynchronize(p->stream));
  if (bad) {
    p->has_contrast = false;
    return fail(p, VIE_EINVAL, "eps has a non-finite or zero value");
  }
  // support columns, in increasing i1 n2 + i2 order
  const long n12 = (long)p->g.n1 * p->g.n2;
  std::vector<int> flags(n12), cols;
  HIPTRY(p, column_flags(p->chi64, n12, p->g.n3, p->colflag, p->stream));
  HIPTRY(p, hipMemcpyAsync(flags.data(), p->colflag, sizeof(int) * n12, hipMemcpyDeviceToHost, p->stream));
  HIPTRY(p, hipStreamSynchronize(p->stream));
  for (long c = 0; c < n12; ++c)
    if (flags[c]) cols.push_back((int)c);
  p->ns = (int)cols.size();
  if (p->ns) HIPTRY(p, hipMemcpy(p->scol, cols.data(), sizeof(int) * cols.size(), hipMemcpyHostToDevice));
  p->has_contrast = true;
  return VIE_OK;
}

int vie_get_contrast(vie_plan_t p, vie_c128* chi) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!chi) return fail(p, VIE_EINVAL, "null chi");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  HIPTRY(p, hipMemcpyAsync(chi, p->chi64, sizeof(double2) * p->g.N, hipMemcpyDeviceToDevice, p->stream));
  return VIE_OK;
}

int vie_rhs(vie_plan_t p, const vie_c128* e_inc, vie_c128* b) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!e_inc || !b) return fail(p, VIE_EINVAL, "null vector");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  HIPTRY(p, launch_rhs(p->g.N, std::pow(p->h, 1.5), p->chi64, reinterpret_cast<const double2*>(e_inc),
                       reinterpret_cast<double2*>(b), p->stream));
  return VIE_OK;
}

int vie_matvec(vie_plan_t p, const vie_c128* x, vie_c128* y) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!x || !y || (const void*)x == (const void*)y) return fail(p, VIE_EINVAL, "x, y null or aliased");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  Op64 A{p};
  HIPTRY(p, A.apply(reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y)));
  return VIE_OK;
}

int vie_matvec_c64(vie_plan_t p, const vie_c64* x, vie_c64* y) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!x || !y || (const void*)x == (const void*)y) return fail(p, VIE_EINVAL, "x, y null or aliased");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  if (!p->goct32) return fail(p, VIE_ESTATE, "plan built without VIE_WITH_FP32");
  Op32 A{p};
  HIPTRY(p, A.apply(reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(y)));
  return VIE_OK;
}

int vie_residual(vie_plan_t p, const vie_c128* x, const vie_c128* b, vie_c128* r) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!x || !b || !r || (const void*)x == (const void*)r) return fail(p, VIE_EINVAL, "bad vectors");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  Op64 A{p};
  HIPTRY(p, A.residual(reinterpret_cast<const double2*>(x), reinterpret_cast<const double2*>(b),
                       reinterpret_cast<double2*>(r)));
  return VIE_OK;
}

namespace {

// Solve-time buffers of vie_solve: the plan's own (allocated on first use) or
// carved from the static scratch array (vie_solve_noalloc).
struct SolveBufs {
  double2* fx;            // full FP64 operator input, zero off the support (3N)
  double2* fy;            // full FP64 operator output (3N)
  double2* fw;            // full FP64 base vector of the learned-circulant tier (3N; null elsewhere)
  double2* bc;            // compressed right-hand side (3N at most)
  double2* xc;            // compressed solution (3N at most)
  double2* partial_full;  // reduction partials of full-length norms
  double2* sumsq_full;    // 2 values
  GmresWs<double>* ws;    // FP64 Krylov workspace
};

// argument checks and defaults shared by vie_solve and vie_solve_noalloc
int solve_options(vie_plan_s* p, const vie_c128* b, vie_c128* x, double tol, const vie_solve_opts* opts,
                  vie_solve_opts& o) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!b || !x || (const void*)b == (const void*)x) return fail(p, VIE_EINVAL, "b, x null or aliased");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(p, VIE_EINVAL, "tol must be positive");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  o = vie_solve_opts{50, 10000, 0, 0, 20, 1e-4, 0, 0};
  if (opts) o = *opts;
  if (o.restart <= 0) o.restart = 50;
  if (o.maxit <= 0) o.maxit = 10000;
  if (o.inner_restart <= 0) o.inner_restart = 20;
  if (!(o.inner_tol > 0)) o.inner_tol = 1e-4;
  if (o.restart > 4096 || o.inner_restart > 4096) return fail(p, VIE_EINVAL, "restart too large");
  if (o.precision < 0 || o.precision > 5) return fail(p, VIE_EINVAL, "unknown precision tier");
  if ((o.precision == 1 || o.precision == 5) && !p->goct32)
    return fail(p, VIE_ESTATE, "mixed tier needs a plan built with VIE_WITH_FP32");
  if ((o.precision == 2 || o.precision == 4) && !p->net)
    return fail(p, VIE_ESTATE, "no preconditioner attached (vie_set_preconditioner)");
  if ((o.precision == 3 || o.precision == 4) && !p->circ)
    return fail(p, VIE_ESTATE, "no circulant preconditioner (vie_circulant_build)");
  if ((o.precision == 3 || o.precision == 4) && circ_info(p->circ).s != p->ns)
    return fail(p, VIE_ESTATE, "circulant preconditioner built for another support");
  return VIE_OK;
}

int solve_impl(vie_plan_s* p, const vie_c128* b, vie_c128* x, double tol, const vie_solve_opts& o,
               vie_solve_info* info, const SolveBufs& B, std::chrono::steady_clock::time_point t0) {
  hipStream_t s = p->stream;
  const long nfull = 3 * p->g.N;
  const double2* bd = reinterpret_cast<const double2*>(b);
  double2* xd = reinterpret_cast<double2*>(x);
  Stats st;
  st.stall_k = o.stall_restarts > 0 ? o.stall_restarts : 0;
  int status = VIE_OK;
  auto report = [&](int code) {
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) {
      info->iters = st.iters;
      info->inner_iters = st.inner;
      info->restarts = st.restarts;
      info->matvecs = st.matvecs;
      info->status = code;
      info->rel_res_true = st.rel_true;
      info->rel_res_est = st.est;
      info->seconds = secs;
      info->fallback = st.fallback;
      info->stalled = st.stalled;
    }
    if (code == VIE_ENOCONV && p->err.empty()) p->err = "tolerance not reached within maxit";
    return code;
  };
  // Off the support A is the identity, so x = b there; on it the system is
  // A_SS x_S = b_S - (A b_off)_S with b_off = b off the support.
  auto x_is_b = [&]() { return hipMemcpyAsync(xd, bd, sizeof(double2) * nfull, hipMemcpyDeviceToDevice, s); };
  if (p->ns == 0) {
    HIPTRY(p, x_is_b());
    HIPTRY(p, hipStreamSynchronize(s));
    st.rel_true = st.est = 0;
    return report(VIE_OK);
  }
  const Support u{p->scol, p->ns, (long)p->g.n1 * p->g.n2, p->g.n3};
  const long n = u.size();
  using K = KrylovOps<double>;
  HIPTRY(p, K::zero(B.fx, nfull, s));
  if (p->fx32) HIPTRY(p, KrylovOps<float>::zero(p->fx32, nfull, s));
  double tmp_h[1];
  auto read_norm2 = [&](const double2* v, long len, double* out) -> hipError_t {
    hipError_t e = K::nrm2sq(v, len, B.partial_full, B.sumsq_full, s);
    if (e) return e;
    e = hipMemcpyAsync(tmp_h, B.sumsq_full, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e) return e;
    e = hipStreamSynchronize(s);
    *out = tmp_h[0];
    return e;
  };
  double bsq_on = 0, bsq_off = 0, bcsq = 0;
  HIPTRY(p, gather<double>(u, bd, B.bc, nullptr, s));
  HIPTRY(p, read_norm2(B.bc, n, &bsq_on));
  HIPTRY(p, hipMemcpyAsync(p->rvec, bd, sizeof(double2) * nfull, hipMemcpyDeviceToDevice, s));
  HIPTRY(p, zero_support<double>(u, p->rvec, s));
  HIPTRY(p, read_norm2(p->rvec, nfull, &bsq_off));
  if (!std::isfinite(bsq_on) || !std::isfinite(bsq_off)) return fail(p, VIE_EINVAL, "right-hand side is not finite");
  if (bsq_off > 0) {
    const void* tw[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    HIPTRY(p, launch_matvec<double>(p->g, p->t64, p->rvec, B.fy, nullptr, 0, p->U64, p->goct64, p->chi64, tw, s));
    st.matvecs++;
    HIPTRY(p, gather<double>(u, B.fy, B.bc, B.bc, s));
    HIPTRY(p, read_norm2(B.bc, n, &bcsq));
  } else {
    bcsq = bsq_on;
  }
  const double bnorm = std::sqrt(bsq_on + bsq_off);
  if (bnorm == 0.0 || bcsq == 0.0) {
    // b = 0, or b off the support only: x = b solves exactly
    HIPTRY(p, x_is_b());
    HIPTRY(p, hipStreamSynchronize(s));
    st.rel_true = st.est = 0;
    return report(VIE_OK);
  }
  const double ratio = std::sqrt(bcsq) / bnorm;   // ||b_c|| / ||b||
  const double tolc = tol / ratio;
  if (o.use_x0) HIPTRY(p, gather<double>(u, xd, B.xc, nullptr, s));
  Op64c A{p, u, B.fx, B.fy};
  // mixed tiers: an outer FGMRES that stalled hands its iterate to FP64 GMRES for
  // the rest of the iteration budget (same stall rule)
  auto mixed_fallback = [&](int code) -> int {
    if (code != VIE_ENOCONV || !st.stalled || st.iters >= o.maxit) return code;
    st.stalled = 0;
    st.fallback = 1;
    return gmres_core<double, Op64c, NoPrecond>(p, *B.ws, A, nullptr, n, B.bc, B.xc, tolc, o.restart, o.maxit,
                                                true, true, st);
  };
  if (o.precision == 0) {
    status = gmres_core<double, Op64c, NoPrecond>(p, *B.ws, A, nullptr, n, B.bc, B.xc, tolc, o.restart, o.maxit,
                                                  o.use_x0 != 0, true, st);
  } else if (o.precision == 1) {
    Op32c A32{p, u};
    // right preconditioner: z = inner FP32 GMRES solve of A z = v
    auto inner = [&](const void* v, void* z, Stats& outer) -> hipError_t {
      hipError_t e = convert<double, float>(reinterpret_cast<const double2*>(v), p->v32a, n, s);
      if (e) return e;
      Stats si;
      int rc = gmres_core<float, Op32c, NoPrecond>(p, p->ws32, A32, nullptr, n, p->v32a, p->v32b, o.inner_tol,
                                                    o.inner_restart, o.inner_restart, false, false, si);
      outer.inner += si.iters;
      if (rc != VIE_OK && rc != VIE_ENOCONV) return hipErrorUnknown;
      return convert<float, double>(p->v32b, reinterpret_cast<double2*>(z), n, s);
    };
    struct Pc {
      decltype(inner)& f;
      hipError_t operator()(const void* v, void* z, Stats& st_) { return f(v, z, st_); }
    } pc{inner};
    status = gmres_core<double, Op64c, Pc>(p, *B.ws, A, &pc, n, B.bc, B.xc, tolc, o.restart, o.maxit,
                                           o.use_x0 != 0, true, st);
    status = mixed_fallback(status);
  } else if (o.precision == 5) {
    // mixed tier with FP64 inner Arnoldi: the inner GMRES keeps its Krylov vectors,
    // Gram-Schmidt and Hessenberg data in FP64 and only its products run in FP32
    Op32in64c A32{p, u, n};
    auto inner = [&](const void* v, void* z, Stats& outer) -> hipError_t {
      Stats si;
      int rc = gmres_core<double, Op32in64c, NoPrecond>(p, p->ws64i, A32, nullptr, n,
                                                         reinterpret_cast<const double2*>(v),
                                                         reinterpret_cast<double2*>(z), o.inner_tol,
                                                         o.inner_restart, o.inner_restart, false, false, si);
      outer.inner += si.iters;
      return (rc != VIE_OK && rc != VIE_ENOCONV) ? hipErrorUnknown : hipSuccess;
    };
    struct Pc {
      decltype(inner)& f;
      hipError_t operator()(const void* v, void* z, Stats& st_) { return f(v, z, st_); }
    } pc{inner};
    status = gmres_core<double, Op64c, Pc>(p, *B.ws, A, &pc, n, B.bc, B.xc, tolc, o.restart, o.maxit,
                                           o.use_x0 != 0, true, st);
    status = mixed_fallback(status);
  } else if (o.precision == 2 || o.precision == 4) {
    // learned tiers.  Precision 2: z = net(v) (the network's correction of v);
    // precision 4: z = W^{-1} v + net(v, W^{-1} v) (the network's correction of the
    // block circulant).  x0 = the preconditioner applied to b.  The method without
    // the network takes over for the rest of the solve -- plain GMRES (2) or the
    // circulant FGMRES (4) -- when a restart cycle reduces the true residual by less
    // than half, when the guess is not finite (x0 = 0 then), or when a network
    // output makes an Arnoldi step non-finite (the iterate of that cycle's start is
    // restored: gmres_core leaves x untouched when it stops inside a cycle).
    net_set_stream(p->net, s);
    int napply = 0;
    const bool on_circ = o.precision == 4;
    if (on_circ) HIPTRY(p, K::zero(B.fw, nfull, s));
    struct Pc {
      vie_plan_s* p;
      Support u;
      int* count;
      double2* fx;
      double2* fw;
      double2* fy;
      bool on_circ;
      hipError_t operator()(const void* v, void* z, Stats&) {
        ++*count;
        const double2* vc = reinterpret_cast<const double2*>(v);
        double2* zc = reinterpret_cast<double2*>(z);
        hipError_t e = scatter<double>(u, vc, fx, p->stream);
        if (e) return e;
        if (on_circ) {
          if ((e = circ_apply_rows(p->circ, vc, zc, p->stream))) return e;
          if ((e = scatter<double>(u, zc, fw, p->stream))) return e;
        }
        if ((e = net_apply(p->net, fx, on_circ ? fw : nullptr, p->chi64, fy))) return e;
        return gather<double>(u, fy, zc, nullptr, p->stream);
      }
    } pc{p, u, &napply, B.fx, B.fw, B.fy, on_circ};
    struct CircPc {
      vie_plan_s* p;
      hipError_t operator()(const void* v, void* z, Stats& s_) {
        ++s_.inner;
        return circ_apply_rows(p->circ, reinterpret_cast<const double2*>(v), reinterpret_cast<double2*>(z),
                               p->stream);
      }
    } cpc{p};
    bool fell_back = false;
    bool have_x0 = o.use_x0 != 0;
    if (!o.use_x0) {
      HIPTRY(p, pc(B.bc, B.xc, st));
      double xsq = 0;
      HIPTRY(p, read_norm2(B.xc, n, &xsq));
      if (std::isfinite(xsq)) {
        have_x0 = true;
      } else {
        HIPTRY(p, K::zero(B.xc, n, s));
        fell_back = true;
      }
    }
    double prev = INFINITY;
    status = VIE_ENOCONV;
    int circ_applies = 0;
    while (st.iters < o.maxit) {
      const int budget = fell_back ? o.maxit : std::min(o.maxit, st.iters + o.restart);
      if (fell_back) {
        Stats before = st;
        if (on_circ)
          status = gmres_core<double, Op64c, CircPc>(p, *B.ws, A, &cpc, n, B.bc, B.xc, tolc, o.restart, budget,
                                                     have_x0, true, st);
        else
          status = gmres_core<double, Op64c, NoPrecond>(p, *B.ws, A, nullptr, n, B.bc, B.xc, tolc, o.restart,
                                                        budget, have_x0, true, st);
        circ_applies += st.inner - before.inner;
        break;
      }
      // the cycle's starting iterate, kept in the full-length scratch vector
      HIPTRY(p, hipMemcpyAsync(p->rvec, B.xc, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
      status = gmres_core<double, Op64c, Pc>(p, *B.ws, A, &pc, n, B.bc, B.xc, tolc, o.restart, budget, have_x0,
                                             true, st);
      have_x0 = true;
      if (status == VIE_ENUMERIC) {
        HIPTRY(p, hipMemcpyAsync(B.xc, p->rvec, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
        p->err.clear();
        fell_back = true;
        continue;
      }
      if (status != VIE_ENOCONV) break;
      if (!(st.rel_true < 0.5 * prev)) fell_back = true;
      prev = st.rel_true;
    }
    st.inner = napply + circ_applies;
    st.fallback = fell_back ? 1 : 0;
  } else {
    // FP64 FGMRES right-preconditioned by the block circulant: z = W^{-1} v
    struct Pc {
      vie_plan_s* p;
      hipError_t operator()(const void* v, void* z, Stats& s_) {
        ++s_.inner;
        return circ_apply_rows(p->circ, reinterpret_cast<const double2*>(v), reinterpret_cast<double2*>(z),
                               p->stream);
      }
    } pc{p};
    status = gmres_core<double, Op64c, Pc>(p, *B.ws, A, &pc, n, B.bc, B.xc, tolc, o.restart, o.maxit,
                                           o.use_x0 != 0, true, st);
  }
  if (status == VIE_OK || status == VIE_ENOCONV) {
    HIPTRY(p, x_is_b());
    HIPTRY(p, scatter<double>(u, B.xc, xd, s));
    HIPTRY(p, hipStreamSynchronize(s));
  }
  st.rel_true *= ratio;
  st.est *= ratio;
  return report(status);
}

}  // namespace

int vie_solve(vie_plan_t p, const vie_c128* b, vie_c128* x, double tol, const vie_solve_opts* opts,
              vie_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  vie_solve_opts o;
  const int rc = solve_options(p, b, x, tol, opts, o);
  if (rc != VIE_OK) return rc;
  const long nfull = 3 * p->g.N;
  if (!p->fx) {
    HIPTRY(p, dmalloc(&p->fx, sizeof(double2) * nfull));
    HIPTRY(p, dmalloc(&p->fy, sizeof(double2) * nfull));
    HIPTRY(p, dmalloc(&p->bc, sizeof(double2) * nfull));
    HIPTRY(p, dmalloc(&p->xc, sizeof(double2) * nfull));
    HIPTRY(p, dmalloc(&p->partial_full, sizeof(double2) * (partial_blocks(nfull) + 1)));
    HIPTRY(p, dmalloc(&p->sumsq_full, sizeof(double2) * 2));
  }
  if ((o.precision == 1 || o.precision == 5) && !p->fx32) {
    HIPTRY(p, dmalloc(&p->fx32, sizeof(float2) * nfull));
    HIPTRY(p, dmalloc(&p->fy32, sizeof(float2) * nfull));
    HIPTRY(p, dmalloc(&p->v32a, sizeof(float2) * nfull));
    HIPTRY(p, dmalloc(&p->v32b, sizeof(float2) * nfull));
  }
  if (o.precision == 4 && !p->fw) HIPTRY(p, dmalloc(&p->fw, sizeof(double2) * nfull));
  const SolveBufs B{p->fx, p->fy, p->fw, p->bc, p->xc, p->partial_full, p->sumsq_full, &p->ws64};
  return solve_impl(p, b, x, tol, o, info, B, t0);
}

int vie_solve_noalloc(vie_plan_t p, const vie_c128* b, vie_c128* x, double tol, const vie_solve_opts* opts,
                      vie_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  vie_solve_opts o;
  const int rc = solve_options(p, b, x, tol, opts, o);
  if (rc != VIE_OK) return rc;
  if (o.precision != 0 && o.precision != 3)
    return fail(p, VIE_EINVAL, "vie_solve_noalloc: precision 0 (GMRES) or 3 (circulant FGMRES) only");
  if (p->device < 0 || p->device >= kMaxDevices || !g_scratch_ptr[p->device])
    return fail(p, VIE_EDEVICE,
                std::string("vie_solve_noalloc: no scratch address for this device (hipGetSymbolAddress: ") +
                    (p->device >= 0 && p->device < kMaxDevices ? hipGetErrorString(g_scratch_err[p->device])
                                                               : "device index out of range") +
                    ")");
  const long nfull = 3 * p->g.N;
  const long n = 3L * p->ns * p->g.n3;   // support-compressed length
  const int m = o.restart;
  const bool flex = o.precision == 3;
  ScratchCarver c{static_cast<unsigned char*>(g_scratch_ptr[p->device])};
  SolveBufs B;
  B.fx = c.take<double2>(nfull);
  B.fy = c.take<double2>(nfull);
  B.fw = nullptr;
  B.bc = c.take<double2>(n);
  B.xc = c.take<double2>(n);
  B.partial_full = c.take<double2>(partial_blocks(nfull) + 1);
  B.sumsq_full = c.take<double2>(2);
  GmresWs<double> ws;
  ws.borrowed = true;
  ws.n = n;
  ws.m = m;
  ws.flex = flex;
  ws.V = c.take<double2>((size_t)n * (m + 1));
  ws.Z = flex ? c.take<double2>((size_t)n * m) : nullptr;
  ws.partial = c.take<double2>((size_t)partial_blocks(n) * (m + 1));
  ws.h1 = c.take<double2>(m + 2);
  ws.h2 = c.take<double2>(m + 2);
  ws.sumsq = c.take<double2>(2);
  ws.gate = c.take<int>(1);
  ws.H = c.take<double2>((size_t)(m + 1) * m);
  ws.sn = c.take<double2>(m + 1);
  ws.g = c.take<double2>(m + 1);
  ws.y = c.take<double2>(m + 1);
  ws.cs = c.take<double>(m + 1);
  ws.state = c.take<double>(4);
  ws.state_h = p->npin;
  ws.ev[0] = p->nev[0];
  ws.ev[1] = p->nev[1];
  if (c.used > kScratchBytes)
    return fail(p, VIE_EINVAL,
                "vie_solve_noalloc: this grid, support and restart need " + std::to_string(c.used) +
                    " bytes of scratch; the limit is " + std::to_string(kScratchBytes));
  B.ws = &ws;
  return solve_impl(p, b, x, tol, o, info, B, t0);
}

int vie_profile_matvec(vie_plan_t p, int precision, const void* x, void* y, int reps, double pass_ms[3],
                       double* total_ms) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!x || !y || x == y || reps < 1 || !pass_ms) return fail(p, VIE_EINVAL, "bad arguments");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  if (precision == 1 && !p->goct32) return fail(p, VIE_ESTATE, "plan built without VIE_WITH_FP32");
  if (precision != 0 && precision != 1) return fail(p, VIE_EINVAL, "precision must be 0 or 1");
  std::vector<hipEvent_t> ev((size_t)reps * 4);
  for (auto& e : ev) HIPTRY(p, hipEventCreate(&e));
  const void* tw64[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
  const void* tw32[3] = {p->tw32[0], p->tw32[1], p->tw32[2]};
  for (int r = 0; r < reps; ++r) {
    HIPTRY(p, hipEventRecord(ev[4 * r], p->stream));
    for (int w = 0; w < 3; ++w) {
      if (precision == 0)
        HIPTRY(p, launch_pass<double>(w, p->g, p->t64, x, y, nullptr, 0, p->U64, p->goct64, p->chi64, tw64,
                                      p->stream));
      else
        HIPTRY(p, launch_pass<float>(w, p->g, p->t32, x, y, nullptr, 0, p->U32, p->goct32, p->chi32, tw32,
                                     p->stream));
      HIPTRY(p, hipEventRecord(ev[4 * r + w + 1], p->stream));
    }
  }
  HIPTRY(p, hipStreamSynchronize(p->stream));
  double acc[3] = {0, 0, 0}, tot = 0;
  for (int r = 0; r < reps; ++r) {
    for (int w = 0; w < 3; ++w) {
      float ms = 0;
      HIPTRY(p, hipEventElapsedTime(&ms, ev[4 * r + w], ev[4 * r + w + 1]));
      acc[w] += ms;
    }
    float ms = 0;
    HIPTRY(p, hipEventElapsedTime(&ms, ev[4 * r], ev[4 * r + 3]));
    tot += ms;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (int w = 0; w < 3; ++w) pass_ms[w] = acc[w] / reps;
  if (total_ms) *total_ms = tot / reps;
  return VIE_OK;
}

int vie_set_preconditioner(vie_plan_t p, vie_net_t net) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (net) {
    const int* g = net_grid(net);
    if (g[0] != p->g.n1 || g[1] != p->g.n2 || g[2] != p->g.n3)
      return fail(p, VIE_EINVAL, "network grid differs from the plan's grid");
  }
  p->net = net;
  return VIE_OK;
}

int vie_get_tune(vie_plan_t p, int precision, int* xy_variant, int* z_pencils) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (precision != 0 && precision != 1) return fail(p, VIE_EINVAL, "precision must be 0 or 1");
  const Tune& t = precision == 0 ? p->t64 : p->t32;
  int opts[8];
  const int n = precision == 0 ? z4_pencil_options<double>(p->g.M3, opts, 8)
                               : z4_pencil_options<float>(p->g.M3, opts, 8);
  if (xy_variant) *xy_variant = xy_variants(p->g) > 1 ? t.xyv : -1;
  if (z_pencils) *z_pencils = t.z4 && n ? (t.zp ? t.zp : opts[0]) : 0;
  return VIE_OK;
}

int vie_set_tune(vie_plan_t p, int precision, int xy_variant, int z_pencils) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (precision != 0 && precision != 1) return fail(p, VIE_EINVAL, "precision must be 0 or 1");
  if (xy_variant < 0 || xy_variant > 2) return fail(p, VIE_EINVAL, "xy_variant must be 0, 1 or 2");
  int opts[8];
  const int n = precision == 0 ? z4_pencil_options<double>(p->g.M3, opts, 8)
                               : z4_pencil_options<float>(p->g.M3, opts, 8);
  Tune& t = precision == 0 ? p->t64 : p->t32;
  if (z_pencils > 0) {
    bool ok = false;
    for (int i = 0; i < n; ++i) ok = ok || opts[i] == z_pencils;
    if (!ok) return fail(p, VIE_EINVAL, "z_pencils is not a candidate for this grid");
  } else if (z_pencils < -1) {
    return fail(p, VIE_EINVAL, "z_pencils must be -1, 0 or a candidate");
  }
  HIPTRY(p, hipStreamSynchronize(p->stream));
  t.xyv = xy_variant;
  t.z4 = (z_pencils >= 0 && n > 0) ? 1 : 0;
  t.zp = z_pencils > 0 ? z_pencils : 0;
  return VIE_OK;
}

int vie_circulant_build(vie_plan_t p, unsigned flags, vie_circulant_info* info) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (flags & ~1u) return fail(p, VIE_EINVAL, "unknown circulant flags");
  if (!p->has_contrast) return fail(p, VIE_ESTATE, "set_contrast first");
  if (p->circ) {
    HIPTRY(p, hipStreamSynchronize(p->stream));
    circ_destroy(p->circ);
    p->circ = nullptr;
  }
  std::string err;
  CircInfo ci{};
  const int rc = circ_build(&p->circ, p->g, p->table->data(), p->chi64, (flags & VIE_CIRC_FP64) != 0, p->stream, err,
                            &ci);
  if (rc != VIE_OK) return fail(p, rc, err);
  if (info) {
    info->support_columns = ci.s;
    info->block_size = ci.m;
    info->blocks = ci.s ? ci.P : 0;
    info->first_slice = ci.z0;
    info->fp64 = ci.fp64;
    info->bytes = ci.bytes;
    info->seconds = ci.seconds;
  }
  return VIE_OK;
}

int vie_circulant_apply(vie_plan_t p, const vie_c128* r, vie_c128* z) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!r || !z || (const void*)r == (const void*)z) return fail(p, VIE_EINVAL, "r, z null or aliased");
  if (!p->circ) return fail(p, VIE_ESTATE, "no circulant preconditioner (vie_circulant_build)");
  HIPTRY(p, circ_apply(p->circ, reinterpret_cast<const double2*>(r), reinterpret_cast<double2*>(z), p->stream));
  return VIE_OK;
}

int vie_curl_table(const int grid[3], double kappa, vie_c128* out, int nthreads) {
  if (!grid || !out) return fail(nullptr, VIE_EINVAL, "null argument");
  for (int d = 0; d < 3; ++d)
    if (grid[d] < 1 || grid[d] > 4096) return fail(nullptr, VIE_EINVAL, "grid size out of range");
  if (!std::isfinite(kappa)) return fail(nullptr, VIE_EINVAL, "kappa not finite");
  vie::curl_table(grid, kappa, reinterpret_cast<std::complex<double>*>(out), nthreads);
  return VIE_OK;
}

int vie_jm_enable(vie_plan_t p) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (p->jm) return VIE_OK;
  const Geom& g = p->g;
  if (g.M1 * g.M2 > 64 * 64) return fail(p, VIE_EINVAL, "cross-section too large for the JM kernels");
  const bool f32 = p->goct32 != nullptr;
  const int n[3] = {g.n1, g.n2, g.n3};
  const auto kt = cached_curl_table(n, p->kappa);
  const long H = (long)g.H1 * g.H2 * g.H3;
  const long P = (long)g.M1 * g.M2 * g.M3;
  const size_t nU = 3 * (size_t)g.n1 * g.n2 * g.M3;
  double2* kdev = nullptr;
  double2* full = nullptr;
  auto done = [&](int code) {
    if (kdev) (void)hipFree(kdev);
    if (full) (void)hipFree(full);
    if (code != VIE_OK) {
      // leave the plan as before the call: no JM buffer survives a failure
      (void)hipStreamSynchronize(p->stream);
      for (void** q : {(void**)&p->koct64, (void**)&p->koct32, (void**)&p->chim64, (void**)&p->chim32,
                       (void**)&p->Um64, (void**)&p->Um32, (void**)&p->S64, (void**)&p->S32}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
      }
      p->jm_fused64 = p->jm_fused32 = false;
    }
    return code;
  };
#define JMTRY(expr)                                              \
  do {                                                           \
    hipError_t _e = (expr);                                      \
    if (_e != hipSuccess) return done(hipfail(p, _e, #expr));    \
  } while (0)
  JMTRY(allow_lds_jm<double>());
  JMTRY(allow_lds_jm<float>());
  JMTRY(dmalloc(&p->koct64, sizeof(double2) * 3 * H));
  if (f32) JMTRY(dmalloc(&p->koct32, sizeof(float2) * 3 * H));
  JMTRY(dmalloc(&p->chim64, sizeof(double2) * g.N));
  JMTRY(dmalloc(&p->chim32, sizeof(float2) * g.N));
  JMTRY(hipMemsetAsync(p->chim64, 0, sizeof(double2) * g.N, p->stream));
  JMTRY(hipMemsetAsync(p->chim32, 0, sizeof(float2) * g.N, p->stream));
  JMTRY(dmalloc(&p->Um64, sizeof(double2) * nU));
  p->jm_fused64 = jm_fused_shape<double>(g, nullptr, nullptr);
  p->jm_fused32 = f32 && jm_fused_shape<float>(g, nullptr, nullptr);
  if (!p->jm_fused64) JMTRY(dmalloc(&p->S64, sizeof(double2) * jm_spectrum_values(g)));
  if (f32) {
    JMTRY(dmalloc(&p->Um32, sizeof(float2) * nU));
    if (!p->jm_fused32) JMTRY(dmalloc(&p->S32, sizeof(float2) * jm_spectrum_values(g)));
  }
  JMTRY(dmalloc(&kdev, sizeof(double2) * 3 * g.N));
  JMTRY(dmalloc(&full, sizeof(double2) * P));
  JMTRY(hipMemcpyAsync(kdev, kt->data(), sizeof(double2) * 3 * g.N, hipMemcpyHostToDevice, p->stream));
  {
    const double2* tw[3] = {p->tw64[0], p->tw64[1], p->tw64[2]};
    JMTRY(launch_curl_spectrum(g, kdev, full, p->koct64, p->koct32, tw, p->stream));
  }
  JMTRY(hipStreamSynchronize(p->stream));
#undef JMTRY
  p->jm = true;
  return done(VIE_OK);
}

int vie_jm_set_route(vie_plan_t p, int precision, int fused) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm) return fail(p, VIE_ESTATE, "vie_jm_enable first");
  if (precision != 0 && precision != 1) return fail(p, VIE_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  if (precision == 1 && !p->goct32) return fail(p, VIE_ESTATE, "plan made without VIE_WITH_FP32");
  const bool fits = precision == 0 ? jm_fused_shape<double>(p->g, nullptr, nullptr)
                                   : jm_fused_shape<float>(p->g, nullptr, nullptr);
  if (fused && !fits) return fail(p, VIE_EINVAL, "the fused cross-section pass does not fit this grid");
  if (!fused) {
    void** S = precision == 0 ? (void**)&p->S64 : (void**)&p->S32;
    const size_t cs = precision == 0 ? sizeof(double2) : sizeof(float2);
    if (!*S) HIPTRY(p, dmalloc(S, cs * jm_spectrum_values(p->g)));
  }
  (precision == 0 ? p->jm_fused64 : p->jm_fused32) = fused != 0;
  return VIE_OK;
}

int vie_jm_get_route(vie_plan_t p, int precision, int* fused) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm) return fail(p, VIE_ESTATE, "vie_jm_enable first");
  if (precision != 0 && precision != 1) return fail(p, VIE_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  if (!fused) return fail(p, VIE_EINVAL, "null output");
  *fused = precision == 0 ? p->jm_fused64 : p->jm_fused32;
  return VIE_OK;
}

int vie_jm_set_permeability(vie_plan_t p, const vie_c128* mu_r) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm) return fail(p, VIE_ESTATE, "vie_jm_enable first");
  if (!mu_r) return fail(p, VIE_EINVAL, "null mu_r");
  HIPTRY(p, hipMemsetAsync(p->flag, 0, sizeof(int), p->stream));
  // (mu_r - 1)/mu_r = 1 - 1/mu_r: the contrast kernel with a unit background
  HIPTRY(p, launch_contrast(p->g.N, reinterpret_cast<const double2*>(mu_r), 1.0, p->chim64, p->chim32, p->flag,
                            p->stream));
  int bad = 0;
  HIPTRY(p, hipMemcpyAsync(&bad, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPTRY(p, hipStreamSynchronize(p->stream));
  if (bad) return fail(p, VIE_EINVAL, "mu_r has a zero or non-finite entry");
  return VIE_OK;
}

int vie_jm_rhs(vie_plan_t p, const vie_c128* e_inc, const vie_c128* etah_inc, vie_c128* b) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm || !p->has_contrast) return fail(p, VIE_ESTATE, "vie_jm_enable and set_contrast first");
  if (!e_inc || !etah_inc || !b) return fail(p, VIE_EINVAL, "null vector");
  const double sc = std::pow(p->h, 1.5);
  double2* bd = reinterpret_cast<double2*>(b);
  HIPTRY(p, launch_rhs(p->g.N, sc, p->chi64, reinterpret_cast<const double2*>(e_inc), bd, p->stream));
  HIPTRY(p, launch_rhs(p->g.N, sc, p->chim64, reinterpret_cast<const double2*>(etah_inc), bd + 3 * p->g.N,
                       p->stream));
  return VIE_OK;
}

int vie_jm_matvec(vie_plan_t p, const vie_c128* x, vie_c128* y) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm || !p->has_contrast) return fail(p, VIE_ESTATE, "vie_jm_enable and set_contrast first");
  if (!x || !y || (const void*)x == (const void*)y) return fail(p, VIE_EINVAL, "x, y null or aliased");
  OpJM64 A{p};
  HIPTRY(p, A.apply(reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y)));
  return VIE_OK;
}

int vie_jm_matvec_c64(vie_plan_t p, const vie_c64* x, vie_c64* y) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm || !p->has_contrast) return fail(p, VIE_ESTATE, "vie_jm_enable and set_contrast first");
  if (!p->Um32) return fail(p, VIE_ESTATE, "FP32 product needs a plan built with VIE_WITH_FP32");
  if (!x || !y || (const void*)x == (const void*)y) return fail(p, VIE_EINVAL, "x, y null or aliased");
  OpJM32 A{p};
  HIPTRY(p, A.apply(reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(y)));
  return VIE_OK;
}

int vie_jm_residual(vie_plan_t p, const vie_c128* x, const vie_c128* b, vie_c128* r) {
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm || !p->has_contrast) return fail(p, VIE_ESTATE, "vie_jm_enable and set_contrast first");
  if (!x || !b || !r || (const void*)x == (const void*)r || (const void*)b == (const void*)r)
    return fail(p, VIE_EINVAL, "x, b, r null or aliased");
  OpJM64 A{p};
  HIPTRY(p, A.residual(reinterpret_cast<const double2*>(x), reinterpret_cast<const double2*>(b),
                       reinterpret_cast<double2*>(r)));
  return VIE_OK;
}

int vie_jm_solve(vie_plan_t p, const vie_c128* b, vie_c128* x, double tol, const vie_solve_opts* opts,
                 vie_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return fail(nullptr, VIE_EINVAL, "null plan");
  if (!p->jm || !p->has_contrast) return fail(p, VIE_ESTATE, "vie_jm_enable and set_contrast first");
  if (!b || !x || (const void*)b == (const void*)x) return fail(p, VIE_EINVAL, "b, x null or aliased");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(p, VIE_EINVAL, "tol must be positive");
  vie_solve_opts o{50, 10000, 0, 0, 20, 1e-4, 0, 0};
  if (opts) o = *opts;
  if (o.restart <= 0) o.restart = 50;
  if (o.maxit <= 0) o.maxit = 10000;
  if (o.inner_restart <= 0) o.inner_restart = 20;
  if (!(o.inner_tol > 0)) o.inner_tol = 1e-4;
  if (o.restart > 4096 || o.inner_restart > 4096) return fail(p, VIE_EINVAL, "restart too large");
  if (o.precision != 0 && o.precision != 1) return fail(p, VIE_EINVAL, "JM solves take precision 0 or 1");
  if (o.precision == 1 && !p->Um32) return fail(p, VIE_ESTATE, "mixed tier needs a plan built with VIE_WITH_FP32");
  hipStream_t s = p->stream;
  const long n = 6 * p->g.N;
  const double2* bd = reinterpret_cast<const double2*>(b);
  double2* xd = reinterpret_cast<double2*>(x);
  Stats st;
  OpJM64 A{p};
  int status;
  if (o.precision == 0) {
    status = gmres_core<double, OpJM64, NoPrecond>(p, p->ws64, A, nullptr, n, bd, xd, tol, o.restart, o.maxit,
                                                   o.use_x0 != 0, true, st);
  } else {
    if (!p->jm32a) {
      HIPTRY(p, dmalloc(&p->jm32a, sizeof(float2) * n));
      HIPTRY(p, dmalloc(&p->jm32b, sizeof(float2) * n));
    }
    OpJM32 A32{p};
    // right preconditioner: z = inner FP32 GMRES solve of A z = v
    auto inner = [&](const void* v, void* z, Stats& outer) -> hipError_t {
      hipError_t e = convert<double, float>(reinterpret_cast<const double2*>(v), p->jm32a, n, s);
      if (e) return e;
      Stats si;
      int rc = gmres_core<float, OpJM32, NoPrecond>(p, p->ws32, A32, nullptr, n, p->jm32a, p->jm32b, o.inner_tol,
                                                     o.inner_restart, o.inner_restart, false, false, si);
      outer.inner += si.iters;
      if (rc != VIE_OK && rc != VIE_ENOCONV) return hipErrorUnknown;
      return convert<float, double>(p->jm32b, reinterpret_cast<double2*>(z), n, s);
    };
    struct Pc {
      decltype(inner)& f;
      hipError_t operator()(const void* v, void* z, Stats& st_) { return f(v, z, st_); }
    } pc{inner};
    status = gmres_core<double, OpJM64, Pc>(p, p->ws64, A, &pc, n, bd, xd, tol, o.restart, o.maxit, o.use_x0 != 0,
                                            true, st);
  }
  if (status == VIE_OK || status == VIE_ENOCONV) HIPTRY(p, hipStreamSynchronize(s));
  if (info) {
    info->iters = st.iters;
    info->inner_iters = st.inner;
    info->restarts = st.restarts;
    info->matvecs = st.matvecs;
    info->status = status;
    info->rel_res_true = st.rel_true;
    info->rel_res_est = st.est;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->fallback = 0;
    info->stalled = 0;
  }
  if (status == VIE_ENOCONV && p->err.empty()) p->err = "tolerance not reached within maxit";
  return status;
}

void vie_destroy(vie_plan_t p) {
  if (!p) return;
  if (p->circ) {
    (void)hipStreamSynchronize(p->stream);
    circ_destroy(p->circ);
  }
  p->ws64.release();
  p->ws32.release();
  p->ws64i.release();
  for (hipEvent_t ev : p->nev)
    if (ev) (void)hipEventDestroy(ev);
  if (p->npin) (void)hipHostFree(p->npin);
  for (void* q : {(void*)p->goct64, (void*)p->goct32, (void*)p->chi64, (void*)p->chi32, (void*)p->U64,
                  (void*)p->U32, (void*)p->rvec, (void*)p->v32a, (void*)p->v32b, (void*)p->flag, (void*)p->colflag,
                  (void*)p->scol, (void*)p->fx, (void*)p->fy, (void*)p->fw, (void*)p->fx32, (void*)p->fy32, (void*)p->bc,
                  (void*)p->xc, (void*)p->partial_full, (void*)p->sumsq_full, (void*)p->koct64,
                  (void*)p->koct32, (void*)p->chim64, (void*)p->chim32, (void*)p->Um64, (void*)p->Um32,
                  (void*)p->S64, (void*)p->S32, (void*)p->jm32a, (void*)p->jm32b})
    if (q) (void)hipFree(q);
  for (int d = 0; d < 3; ++d) {
    if (p->tw64[d]) (void)hipFree(p->tw64[d]);
    if (p->tw32[d]) (void)hipFree(p->tw32[d]);
  }
  delete p;
}

}  // extern "C"
