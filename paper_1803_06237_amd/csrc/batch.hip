// Batched solves: many systems (uneven grids, each its own plan) advanced in
// lockstep by GMRES(m) or, for the mixed tier, FP64 flexible GMRES(m) whose
// preconditioner is a fixed number of FP32 GMRES steps (Section V-D solves the
// discrete J-VIE with GMRES; the batching, the tiers and the graph capture are
// this library's design).
//
// Every kernel covers the whole batch in one launch: the work of system s is the
// item range [prefix[s], prefix[s+1]) and each workgroup walks items with a grid
// stride.  Convergence is tracked on the device: a system whose residual
// estimate reaches tol clears its flag and every later kernel of the cycle skips
// it, so a whole restart cycle needs no host synchronisation and is captured
// once as a HIP graph and replayed.  The host synchronises once per cycle to
// read the true residuals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "fft_device.hpp"
#include "krylov.hpp"
#include "vie_internal.hpp"

namespace vie {

namespace {

constexpr int kT = 256;
constexpr int kE = 8;
constexpr int kC = kT * kE;   // elements per chunk

__device__ __forceinline__ double2 d2(double2 v) { return v; }
__device__ __forceinline__ double2 d2(float2 v) { return double2{(double)v.x, (double)v.y}; }
template <typename V> __device__ __forceinline__ V fromd(double2 v);
template <> __device__ __forceinline__ double2 fromd<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 fromd<float2>(double2 v) { return float2{(float)v.x, (float)v.y}; }

__device__ __forceinline__ int find_item(const int* prefix, int nsys, int item) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int NV>
__device__ __forceinline__ void bsum(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i)
    for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_down(v[i], o, 64);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 0; i < NV; ++i) {
      double s = 0;
      for (int w = 0; w < kT / 64; ++w) s += lds[w * NV + i];
      v[i] = s;
    }
  __syncthreads();
}

}  // namespace

// Per-system Krylov state (device memory).
struct KDesc {
  void* V;          // (m + 1) * n basis vectors
  void* Z;          // m * n preconditioned vectors (flexible) or null
  void* x;          // solution
  const void* b;    // right-hand side
  void* r;          // residual buffer (cycle start vector)
  long n;
  int nchunk;
  double2* partial; // (m + 1) * nchunk
  double2* h1;
  double2* h2;
  double2* sumsq;   // [0] ||w||^2 of the current vector, [1] ||b||^2
  double2* H;       // (m + 1) * m, column-major
  double* cs;
  double2* sn;
  double2* g;
  double2* y;
  int* act;         // active in the current step
  const int* act0;  // active for the cycle
  int* kdone;       // Arnoldi steps of the current cycle
  int* iters;       // accumulated steps
  double* est;      // residual estimate |g_{k}| / ||b||
  double tol;
};

// Support compression of one system: Krylov vectors hold the 3 s n3 values of the
// support columns, comp[(a s + p) n3 + i3] = full[a][col[p]][i3], and the product
// runs on the full-length buffers fx (zero off the support) and fy.
struct SDesc {
  const int* col;   // s increasing column indices i1 n2 + i2
  int s;
  int n3;
  long n12;
  void* fx;
  void* fy;
};

// vector selector: 0 -> V_j, 1 -> Z_j, 2 -> x, 3 -> b, 4 -> r
template <typename T>
__device__ __forceinline__ cx<T>* vsel(const KDesc& D, int which, int j) {
  switch (which) {
    case 0: return (cx<T>*)D.V + (long)j * D.n;
    case 1: return (cx<T>*)D.Z + (long)j * D.n;
    case 2: return (cx<T>*)D.x;
    case 3: return (cx<T>*)D.b;
    default: return (cx<T>*)D.r;
  }
}

// partial[i * nchunk + chunk] = V_i^H w over the chunk, i <= j, w = V_{j+1}
template <typename T>
__global__ __launch_bounds__(kT) void k_b_mdot(const KDesc* __restrict__ d, const int* __restrict__ prefix, int nsys,
                                               int total, int j) {
  __shared__ double lds[(kT / 64) * 8];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& D = d[s];
    if (*D.act == 0) continue;
    const int chunk = item - prefix[s];
    const long e0 = (long)chunk * kC + threadIdx.x;
    const cx<T>* w = (const cx<T>*)D.V + (long)(j + 1) * D.n;
    double2 wv[kE];
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      wv[k] = e < D.n ? d2(w[e]) : double2{0.0, 0.0};
    }
    for (int i0 = 0; i0 <= j; i0 += 4) {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (i0 + q <= j) {
          const cx<T>* Vi = (const cx<T>*)D.V + (long)(i0 + q) * D.n;
#pragma unroll
          for (int k = 0; k < kE; ++k) {
            const long e = e0 + (long)k * kT;
            if (e < D.n) {
              const double2 a = d2(Vi[e]);
              acc[2 * q] += a.x * wv[k].x + a.y * wv[k].y;
              acc[2 * q + 1] += a.x * wv[k].y - a.y * wv[k].x;
            }
          }
        }
      }
      bsum<8>(acc, lds);
      if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q)
          if (i0 + q <= j) D.partial[(long)(i0 + q) * D.nchunk + chunk] = double2{acc[2 * q], acc[2 * q + 1]};
    }
  }
}

// h[i] = sum over chunks of partial[i], i < count; items (s, i)
__global__ __launch_bounds__(kT) void k_b_reduce(const KDesc* __restrict__ d, int nsys, int count, int which) {
  __shared__ double lds[(kT / 64) * 2];
  for (int item = blockIdx.x; item < nsys * count; item += gridDim.x) {
    const int s = item / count, i = item % count;
    const KDesc& D = d[s];
    if (*D.act == 0) continue;
    double v[2] = {0.0, 0.0};
    for (int c = threadIdx.x; c < D.nchunk; c += kT) {
      const double2 p = D.partial[(long)i * D.nchunk + c];
      v[0] += p.x;
      v[1] += p.y;
    }
    bsum<2>(v, lds);
    if (threadIdx.x == 0) {
      double2* out = which == 0 ? D.h1 : (which == 1 ? D.h2 : D.sumsq);
      out[i] = double2{v[0], v[1]};
    }
  }
}

// w = V_{j+1} -= sum_{i <= j} h_i V_i   (which = 0: h1, 1: h2)
template <typename T>
__global__ __launch_bounds__(kT) void k_b_orth(const KDesc* __restrict__ d, const int* __restrict__ prefix, int nsys,
                                               int total, int j, int which) {
  __shared__ double2 c[512];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& D = d[s];
    if (*D.act == 0) continue;
    const double2* h = which == 0 ? D.h1 : D.h2;
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += kT) c[i] = h[i];
    __syncthreads();
    const long e0 = (long)(item - prefix[s]) * kC + threadIdx.x;
    cx<T>* w = (cx<T>*)D.V + (long)(j + 1) * D.n;
    double2 acc[kE];
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      acc[k] = e < D.n ? d2(w[e]) : double2{0.0, 0.0};
    }
    for (int i = 0; i <= j; ++i) {
      const double2 ci = c[i];
      const cx<T>* Vi = (const cx<T>*)D.V + (long)i * D.n;
#pragma unroll
      for (int k = 0; k < kE; ++k) {
        const long e = e0 + (long)k * kT;
        if (e < D.n) {
          const double2 a = d2(Vi[e]);
          acc[k].x -= ci.x * a.x - ci.y * a.y;
          acc[k].y -= ci.x * a.y + ci.y * a.x;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      if (e < D.n) w[e] = fromd<cx<T>>(acc[k]);
    }
  }
}

// partial[chunk] = ||v||^2 over the chunk, v selected by (which, j); act_sel: 0 -> act, 1 -> act0
template <typename T>
__global__ __launch_bounds__(kT) void k_b_nrm2(const KDesc* __restrict__ d, const int* __restrict__ prefix, int nsys,
                                               int total, int which, int j, int act_sel) {
  __shared__ double lds[(kT / 64) * 2];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& D = d[s];
    if ((act_sel ? *D.act0 : *D.act) == 0) continue;
    const int chunk = item - prefix[s];
    const long e0 = (long)chunk * kC + threadIdx.x;
    const cx<T>* v = vsel<T>(D, which, j);
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      if (e < D.n) {
        const double2 a = d2(v[e]);
        acc[0] += a.x * a.x + a.y * a.y;
      }
    }
    bsum<2>(acc, lds);
    if (threadIdx.x == 0) D.partial[chunk] = double2{acc[0], 0.0};
  }
}

// sumsq[slot] = sum of partial[0..nchunk)
__global__ __launch_bounds__(kT) void k_b_nrm2_fin(const KDesc* __restrict__ d, int nsys, int slot, int act_sel) {
  __shared__ double lds[(kT / 64) * 2];
  for (int s = blockIdx.x; s < nsys; s += gridDim.x) {
    const KDesc& D = d[s];
    if ((act_sel ? *D.act0 : *D.act) == 0) continue;
    double v[2] = {0.0, 0.0};
    for (int c = threadIdx.x; c < D.nchunk; c += kT) v[0] += D.partial[c].x;
    bsum<2>(v, lds);
    if (threadIdx.x == 0) D.sumsq[slot] = double2{v[0], 0.0};
  }
}

// dst = src / sqrt(sumsq[0])
template <typename T>
__global__ __launch_bounds__(kT) void k_b_scale(const KDesc* __restrict__ d, const int* __restrict__ prefix, int nsys,
                                                int total, int wsrc, int jsrc, int jdst, int act_sel) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& D = d[s];
    if ((act_sel ? *D.act0 : *D.act) == 0) continue;
    const double nr = sqrt(D.sumsq[0].x);
    const double f = nr > 0.0 ? 1.0 / nr : 0.0;
    const cx<T>* src = vsel<T>(D, wsrc, jsrc);
    cx<T>* dst = (cx<T>*)D.V + (long)jdst * D.n;
    const long e0 = (long)(item - prefix[s]) * kC + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      if (e < D.n) {
        const double2 a = d2(src[e]);
        dst[e] = fromd<cx<T>>(double2{a.x * f, a.y * f});
      }
    }
  }
}

// cycle start: g = (beta, 0, ...), step flags from the cycle flags
__global__ void k_b_init(const KDesc* __restrict__ d, int nsys, int m) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
    const KDesc& D = d[s];
    *D.act = *D.act0;
    *D.kdone = 0;
    if (*D.act0 == 0) continue;
    for (int i = 0; i <= m; ++i) D.g[i] = double2{0.0, 0.0};
    D.g[0] = double2{sqrt(D.sumsq[0].x), 0.0};
  }
}

// Hessenberg column j, Givens rotations, residual estimate and step mask.
__global__ void k_b_givens(const KDesc* __restrict__ d, int nsys, int j, int m) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
    const KDesc& D = d[s];
    if (*D.act == 0) continue;
    double2* h = D.H + (long)j * (m + 1);
    for (int i = 0; i <= j; ++i) h[i] = double2{D.h1[i].x + D.h2[i].x, D.h1[i].y + D.h2[i].y};
    const double hn = sqrt(D.sumsq[0].x);
    h[j + 1] = double2{hn, 0.0};
    for (int i = 0; i < j; ++i) {
      const double2 a = h[i], bb = h[i + 1];
      const double c = D.cs[i];
      const double2 sn = D.sn[i];
      h[i] = double2{c * a.x + (sn.x * bb.x - sn.y * bb.y), c * a.y + (sn.x * bb.y + sn.y * bb.x)};
      h[i + 1] = double2{-(sn.x * a.x + sn.y * a.y) + c * bb.x, -(sn.x * a.y - sn.y * a.x) + c * bb.y};
    }
    const double2 a = h[j], bb = h[j + 1];
    const double na = hypot(a.x, a.y), nb = hypot(bb.x, bb.y);
    double c;
    double2 sn, r;
    if (nb == 0.0) {
      c = 1.0;
      sn = double2{0.0, 0.0};
      r = a;
    } else if (na == 0.0) {
      c = 0.0;
      sn = double2{1.0, 0.0};
      r = bb;
    } else {
      const double t = hypot(na, nb);
      const double2 ph = double2{a.x / na, a.y / na};
      c = na / t;
      sn = double2{(ph.x * bb.x + ph.y * bb.y) / t, (ph.y * bb.x - ph.x * bb.y) / t};
      r = double2{ph.x * t, ph.y * t};
    }
    D.cs[j] = c;
    D.sn[j] = sn;
    h[j] = r;
    h[j + 1] = double2{0.0, 0.0};
    const double2 gj = D.g[j];
    D.g[j + 1] = double2{-(sn.x * gj.x + sn.y * gj.y), -(sn.x * gj.y - sn.y * gj.x)};
    D.g[j] = double2{c * gj.x, c * gj.y};
    const double bn = sqrt(D.sumsq[1].x);
    const double est = hypot(D.g[j + 1].x, D.g[j + 1].y) / (bn > 0 ? bn : 1.0);
    *D.est = est;
    *D.kdone = j + 1;
    *D.iters += 1;
    if (!(est > D.tol) || hn == 0.0 || !isfinite(est)) *D.act = 0;
  }
}

// y = R^{-1} g over the kdone leading columns
__global__ void k_b_trisolve(const KDesc* __restrict__ d, int nsys, int m) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
    const KDesc& D = d[s];
    if (*D.act0 == 0) continue;
    const int k = *D.kdone;
    for (int i = k - 1; i >= 0; --i) {
      double2 acc = D.g[i];
      for (int l = i + 1; l < k; ++l) {
        const double2 hil = D.H[(long)l * (m + 1) + i], yl = D.y[l];
        acc.x -= hil.x * yl.x - hil.y * yl.y;
        acc.y -= hil.x * yl.y + hil.y * yl.x;
      }
      const double2 dd = D.H[(long)i * (m + 1) + i];
      const double q = dd.x * dd.x + dd.y * dd.y;
      D.y[i] = q > 0 ? double2{(acc.x * dd.x + acc.y * dd.y) / q, (acc.y * dd.x - acc.x * dd.y) / q}
                     : double2{0.0, 0.0};
    }
  }
}

// x += sum_{i < kdone} y_i basis_i (basis = Z if flexible else V)
template <typename T>
__global__ __launch_bounds__(kT) void k_b_update(const KDesc* __restrict__ d, const int* __restrict__ prefix, int nsys,
                                                 int total) {
  __shared__ double2 c[512];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& D = d[s];
    if (*D.act0 == 0) continue;
    const int k = *D.kdone;
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += kT) c[i] = D.y[i];
    __syncthreads();
    const cx<T>* basis = (const cx<T>*)(D.Z ? D.Z : D.V);
    cx<T>* x = (cx<T>*)D.x;
    const long e0 = (long)(item - prefix[s]) * kC + threadIdx.x;
#pragma unroll
    for (int kk = 0; kk < kE; ++kk) {
      const long e = e0 + (long)kk * kT;
      if (e >= D.n) continue;
      double2 acc = d2(x[e]);
      for (int i = 0; i < k; ++i) {
        const double2 a = d2(basis[(long)i * D.n + e]);
        acc.x += c[i].x * a.x - c[i].y * a.y;
        acc.y += c[i].x * a.y + c[i].y * a.x;
      }
      x[e] = fromd<cx<T>>(acc);
    }
  }
}

// dst(vector of Dd selected by (wd, jd)) = src(vector of Ds selected by (ws, js)), type converted;
// skipped when the source system's step flag is off.  zero = 1 writes zeros instead.
template <typename TS, typename TD>
__global__ __launch_bounds__(kT) void k_b_copy(const KDesc* __restrict__ ds, const KDesc* __restrict__ dd,
                                               const int* __restrict__ prefix, int nsys, int total, int ws, int js,
                                               int wd, int jd, int zero, int act_sel) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& S = ds[s];
    const KDesc& Dd = dd[s];
    if ((act_sel ? *S.act0 : *S.act) == 0) continue;
    const cx<TS>* src = vsel<TS>(S, ws, js);
    cx<TD>* dst = vsel<TD>(Dd, wd, jd);
    const long e0 = (long)(item - prefix[s]) * kC + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      if (e < Dd.n) dst[e] = zero ? cx<TD>{(TD)0, (TD)0} : fromd<cx<TD>>(d2(src[e]));
    }
  }
}

__device__ __forceinline__ long full_index(const SDesc& S, long e) {
  const long row = e / S.n3;
  const int t = (int)(e - row * S.n3);
  const int a = (int)(row / S.s), p = (int)(row - (long)a * S.s);
  return ((long)a * S.n12 + S.col[p]) * S.n3 + t;
}

// fx on the support = the compressed vector selected by (which, j); the entries
// off the support stay as they are (zero)
template <typename T>
__global__ __launch_bounds__(kT) void k_b_scatter(const KDesc* __restrict__ d, const SDesc* __restrict__ sd,
                                                  const int* __restrict__ prefix, int nsys, int total, int which,
                                                  int j, int act_sel) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& D = d[s];
    if ((act_sel ? *D.act0 : *D.act) == 0) continue;
    const SDesc& S = sd[s];
    const cx<T>* src = vsel<T>(D, which, j);
    cx<T>* fx = (cx<T>*)S.fx;
    const long e0 = (long)(item - prefix[s]) * kC + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      if (e < D.n) fx[full_index(S, e)] = src[e];
    }
  }
}

// the compressed vector selected by (which, j) = fy on the support; sub = 1:
// = b - fy on the support (the residual of the cycle start)
template <typename T>
__global__ __launch_bounds__(kT) void k_b_gather(const KDesc* __restrict__ d, const SDesc* __restrict__ sd,
                                                 const int* __restrict__ prefix, int nsys, int total, int which,
                                                 int j, int sub, int act_sel) {
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_item(prefix, nsys, item);
    const KDesc& D = d[s];
    if ((act_sel ? *D.act0 : *D.act) == 0) continue;
    const SDesc& S = sd[s];
    cx<T>* dst = vsel<T>(D, which, j);
    const cx<T>* b = (const cx<T>*)D.b;
    const cx<T>* fy = (const cx<T>*)S.fy;
    const long e0 = (long)(item - prefix[s]) * kC + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const long e = e0 + (long)k * kT;
      if (e < D.n) {
        const cx<T> v = fy[full_index(S, e)];
        dst[e] = sub ? cx<T>{b[e].x - v.x, b[e].y - v.y} : v;
      }
    }
  }
}

}  // namespace vie

// =============================================================================
// host side
// =============================================================================
using namespace vie;

namespace {

struct SysPlan {            // what the batch needs from a plan
  Geom g;
  Tune t64, t32;
  void *U64, *U32, *goct64, *goct32, *chi64, *chi32;
  const void* tw64[3];
  const void* tw32[3];
};

template <typename T>
struct BatchLevel {         // one Krylov level (outer FP64 or inner FP32) for the whole batch
  int nsys = 0, m = 0;
  bool flex = false;
  std::vector<KDesc> h;
  KDesc* d = nullptr;
  std::vector<int> cpre;    // chunk prefix
  int* d_cpre = nullptr;
  int ctotal = 0;
  std::vector<void*> allocs;

  hipError_t alloc(void** p, size_t bytes) {
    hipError_t e = dmalloc(p, bytes);
    if (!e) allocs.push_back(*p);
    return e;
  }
  void release() {
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    d = nullptr;
    d_cpre = nullptr;
  }
};

// matvec descriptors for one level: step (V_j or Z_j -> V_{j+1}) and residual (x -> r),
// both on the full-length buffers of the support descriptors
struct PassSet {
  std::vector<SDesc> h_sd;        // per system, filled before build_passes
  SDesc* d_sd = nullptr;
  PassDesc* d_step = nullptr;
  PassDesc* d_res = nullptr;
  std::vector<PassDesc> h_step, h_res;
  // z-pass groups: systems sharing a four-step shape, launched together
  struct Group {
    int A, B, P;
    std::vector<int> sys;
    int* d_zpre = nullptr;
    int ztotal = 0;
    PassDesc* d_step = nullptr;
    PassDesc* d_res = nullptr;
  };
  std::vector<Group> zgroups;
  std::vector<int> zsingle;      // systems on the generic z kernels
  std::vector<int> xy_sys;       // systems on the batched xy64 kernel
  int* d_xypre = nullptr;
  int xytotal = 0;
  PassDesc* d_xy = nullptr;       // step flags
  PassDesc* d_xy_res = nullptr;   // cycle flags (residual products)
  std::vector<int> xysingle;
};

}  // namespace

struct vie_batch_s {
  int nsys;
  hipStream_t stream;
  std::vector<SysPlan> sp;
  BatchLevel<double> outer;
  BatchLevel<float> inner;
  PassSet p64, p32;
  bool mixed;
  bool circ_tier = false;         // FP64 FGMRES preconditioned by each plan's block circulant
  std::vector<Circ*> circ;        // per system (systems of one plan share it)
  std::vector<int> on;            // host copy of the cycle flags
  std::vector<void*> allocs;
  hipGraphExec_t graph = nullptr;
  std::string err;
};

namespace {

template <typename T>
hipError_t build_level(BatchLevel<T>& L, const std::vector<long>& n, int m, bool flex, double tol,
                       const std::vector<const void*>& b, const std::vector<void*>& x, int* act_cycle,
                       const int* act_cycle_src) {
  L.nsys = (int)n.size();
  L.m = m;
  L.flex = flex;
  L.h.resize(L.nsys);
  L.cpre.assign(L.nsys + 1, 0);
  hipError_t e;
  int* flags = nullptr;   // per system: act, kdone, iters
  if ((e = L.alloc((void**)&flags, sizeof(int) * 3 * L.nsys))) return e;
  if ((e = hipMemset(flags, 0, sizeof(int) * 3 * L.nsys))) return e;
  double* est = nullptr;
  if ((e = L.alloc((void**)&est, sizeof(double) * L.nsys))) return e;
  for (int s = 0; s < L.nsys; ++s) {
    KDesc& D = L.h[s];
    std::memset(&D, 0, sizeof(D));
    D.n = n[s];
    D.nchunk = (int)((n[s] + kC - 1) / kC);
    L.cpre[s + 1] = L.cpre[s] + D.nchunk;
    // (a system without support has length 0 and no chunks; its buffers keep one
    // element so every pointer is valid)
    const size_t len = n[s] > 0 ? (size_t)n[s] : 1;
    const size_t nch = D.nchunk > 0 ? (size_t)D.nchunk : 1;
    if ((e = L.alloc(&D.V, sizeof(cx<T>) * len * (m + 1)))) return e;
    if (flex && (e = L.alloc(&D.Z, sizeof(cx<T>) * len * m))) return e;
    D.x = x[s];
    D.b = b[s];
    if ((e = L.alloc(&D.r, sizeof(cx<T>) * len))) return e;
    if ((e = L.alloc((void**)&D.partial, sizeof(double2) * (size_t)(m + 1) * nch))) return e;
    double2* small = nullptr;
    const size_t per = (size_t)(m + 2) * 2 + 2 + (size_t)(m + 1) * m + 3 * (size_t)(m + 1);
    if ((e = L.alloc((void**)&small, sizeof(double2) * per))) return e;
    D.h1 = small;
    D.h2 = D.h1 + (m + 2);
    D.sumsq = D.h2 + (m + 2);
    D.H = D.sumsq + 2;
    D.sn = D.H + (size_t)(m + 1) * m;
    D.g = D.sn + (m + 1);
    D.y = D.g + (m + 1);
    if ((e = L.alloc((void**)&D.cs, sizeof(double) * (m + 1)))) return e;
    D.act = flags + s;
    D.kdone = flags + L.nsys + s;
    D.iters = flags + 2 * L.nsys + s;
    D.act0 = act_cycle_src ? act_cycle_src + s : act_cycle + s;
    D.est = est + s;
    D.tol = tol;
  }
  L.ctotal = L.cpre[L.nsys];
  if ((e = L.alloc((void**)&L.d, sizeof(KDesc) * L.nsys))) return e;
  if ((e = hipMemcpy(L.d, L.h.data(), sizeof(KDesc) * L.nsys, hipMemcpyHostToDevice))) return e;
  if ((e = L.alloc((void**)&L.d_cpre, sizeof(int) * (L.nsys + 1)))) return e;
  return hipMemcpy(L.d_cpre, L.cpre.data(), sizeof(int) * (L.nsys + 1), hipMemcpyHostToDevice);
}

template <typename T>
hipError_t build_passes(vie_batch_s* B, PassSet& PS, const BatchLevel<T>& L, std::vector<void*>& allocs) {
  const bool dbl = sizeof(T) == 8;
  auto alloc = [&](void** p, size_t bytes) {
    hipError_t e = dmalloc(p, bytes);
    if (!e) allocs.push_back(*p);
    return e;
  };
  hipError_t e;
  const int n = B->nsys;
  PS.h_step.resize(n);
  PS.h_res.resize(n);
  for (int s = 0; s < n; ++s) {
    const SysPlan& P = B->sp[s];
    const KDesc& D = L.h[s];
    PassDesc pd{};
    pd.g = P.g;
    pd.U = dbl ? P.U64 : P.U32;
    pd.goct = dbl ? P.goct64 : P.goct32;
    pd.chi = dbl ? P.chi64 : P.chi32;
    pd.twz = dbl ? P.tw64[2] : P.tw32[2];
    pd.twx = dbl ? P.tw64[0] : P.tw32[0];
    // the products read fx and write fy; the batched scatter and gather around
    // them move the compressed Krylov vectors
    pd.active = D.act;
    pd.xb = PS.h_sd[s].fx;
    pd.xs = 0;
    pd.yb = PS.h_sd[s].fy;
    pd.ys = 0;
    pd.b = nullptr;
    PS.h_step[s] = pd;
    pd.active = D.act0;
    PS.h_res[s] = pd;
  }
  if ((e = alloc((void**)&PS.d_sd, sizeof(SDesc) * n))) return e;
  if ((e = hipMemcpy(PS.d_sd, PS.h_sd.data(), sizeof(SDesc) * n, hipMemcpyHostToDevice))) return e;
  // z groups
  for (int s = 0; s < n; ++s) {
    int A, Bv, Pp;
    const Tune& t = dbl ? B->sp[s].t64 : B->sp[s].t32;
    if (t.z4 && z4_shape<T>(B->sp[s].g.M3, &A, &Bv, &Pp)) {
      auto it = std::find_if(PS.zgroups.begin(), PS.zgroups.end(),
                             [&](const PassSet::Group& G) { return G.A == A && G.B == Bv && G.P == Pp; });
      if (it == PS.zgroups.end()) {
        PS.zgroups.push_back(PassSet::Group{A, Bv, Pp, {}, nullptr, 0, nullptr, nullptr});
        it = PS.zgroups.end() - 1;
      }
      it->sys.push_back(s);
    } else {
      PS.zsingle.push_back(s);
    }
    if (B->sp[s].g.M1 == 64 && B->sp[s].g.M2 == 64) PS.xy_sys.push_back(s);
    else PS.xysingle.push_back(s);
  }
  for (auto& G : PS.zgroups) {
    std::vector<int> pre(G.sys.size() + 1, 0);
    std::vector<PassDesc> st, rs;
    for (size_t i = 0; i < G.sys.size(); ++i) {
      const Geom& g = B->sp[G.sys[i]].g;
      pre[i + 1] = pre[i] + 3 * g.n2 * ((g.n1 + G.P - 1) / G.P);
      PassDesc a = PS.h_step[G.sys[i]], r = PS.h_res[G.sys[i]];
      a.P = r.P = G.P;
      st.push_back(a);
      rs.push_back(r);
    }
    G.ztotal = pre.back();
    if ((e = alloc((void**)&G.d_zpre, sizeof(int) * pre.size()))) return e;
    if ((e = hipMemcpy(G.d_zpre, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice))) return e;
    if ((e = alloc((void**)&G.d_step, sizeof(PassDesc) * st.size()))) return e;
    if ((e = hipMemcpy(G.d_step, st.data(), sizeof(PassDesc) * st.size(), hipMemcpyHostToDevice))) return e;
    if ((e = alloc((void**)&G.d_res, sizeof(PassDesc) * rs.size()))) return e;
    if ((e = hipMemcpy(G.d_res, rs.data(), sizeof(PassDesc) * rs.size(), hipMemcpyHostToDevice))) return e;
  }
  if (!PS.xy_sys.empty()) {
    std::vector<int> pre(PS.xy_sys.size() + 1, 0);
    std::vector<PassDesc> st, rs;
    for (size_t i = 0; i < PS.xy_sys.size(); ++i) {
      const Geom& g = B->sp[PS.xy_sys[i]].g;
      pre[i + 1] = pre[i] + (g.M3 == 1 ? 1 : g.M3 / 2);
      st.push_back(PS.h_step[PS.xy_sys[i]]);
      rs.push_back(PS.h_res[PS.xy_sys[i]]);
    }
    PS.xytotal = pre.back();
    if ((e = alloc((void**)&PS.d_xypre, sizeof(int) * pre.size()))) return e;
    if ((e = hipMemcpy(PS.d_xypre, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice))) return e;
    if ((e = alloc((void**)&PS.d_xy, sizeof(PassDesc) * st.size()))) return e;
    if ((e = hipMemcpy(PS.d_xy, st.data(), sizeof(PassDesc) * st.size(), hipMemcpyHostToDevice))) return e;
    if ((e = alloc((void**)&PS.d_xy_res, sizeof(PassDesc) * rs.size()))) return e;
    if ((e = hipMemcpy(PS.d_xy_res, rs.data(), sizeof(PassDesc) * rs.size(), hipMemcpyHostToDevice))) return e;
  }
  return hipSuccess;
}

// Batched matvec on compressed vectors: residual = false: V_{j+1} = A (V_j or
// Z_j), systems gated by their step flags; true: r = b - A x, gated by the cycle
// flags.  Scatter into fx, the three passes fx -> fy, gather from fy.
template <typename T>
hipError_t batch_matvec(vie_batch_s* B, PassSet& PS, const BatchLevel<T>& L, bool residual, int j) {
  hipStream_t s = B->stream;
  hipError_t e;
  const int mode = 0;
  const int jx = 0, jy = 0;
  const bool dbl = sizeof(T) == 8;
  const int act_sel = residual ? 1 : 0;
  const int gsz = L.ctotal < 4096 ? (L.ctotal > 0 ? L.ctotal : 1) : 4096;
  hipLaunchKernelGGL((k_b_scatter<T>), dim3(gsz), dim3(kT), 0, s, L.d, PS.d_sd, L.d_cpre, L.nsys, L.ctotal,
                     residual ? 2 : (L.flex ? 1 : 0), residual ? 0 : j, act_sel);
  if ((e = hipGetLastError())) return e;
  for (int which = 0; which < 3; ++which) {
    if (which == 1) {
      if (PS.xytotal > 0 &&
          (e = launch_pass_batch<T>(1, 0, residual ? PS.d_xy_res : PS.d_xy, PS.d_xypre, (int)PS.xy_sys.size(), PS.xytotal, 0, 0, 0, 0, 0, s)))
        return e;
      for (int sidx : PS.xysingle) {
        const SysPlan& P = B->sp[sidx];
        const void* tw[3] = {dbl ? P.tw64[0] : P.tw32[0], dbl ? P.tw64[1] : P.tw32[1], dbl ? P.tw64[2] : P.tw32[2]};
        if ((e = launch_pass<T>(1, P.g, dbl ? P.t64 : P.t32, nullptr, nullptr, nullptr, 0, dbl ? P.U64 : P.U32,
                                dbl ? P.goct64 : P.goct32, dbl ? P.chi64 : P.chi32, tw, s)))
          return e;
      }
      continue;
    }
    for (auto& G : PS.zgroups)
      if ((e = launch_pass_batch<T>(which, mode, residual ? G.d_res : G.d_step, G.d_zpre, (int)G.sys.size(),
                                    G.ztotal, G.A, G.B, G.P, jx, jy, s)))
        return e;
    for (int sidx : PS.zsingle) {
      const SysPlan& P = B->sp[sidx];
      const PassDesc& pd = residual ? PS.h_res[sidx] : PS.h_step[sidx];
      const void* xp = (const cx<T>*)pd.xb + (long)jx * pd.xs;
      void* yp = (cx<T>*)pd.yb + (long)jy * pd.ys;
      const void* tw[3] = {dbl ? P.tw64[0] : P.tw32[0], dbl ? P.tw64[1] : P.tw32[1], dbl ? P.tw64[2] : P.tw32[2]};
      if ((e = launch_pass<T>(which, P.g, dbl ? P.t64 : P.t32, xp, yp, pd.b, mode, dbl ? P.U64 : P.U32,
                              dbl ? P.goct64 : P.goct32, dbl ? P.chi64 : P.chi32, tw, s)))
        return e;
    }
  }
  hipLaunchKernelGGL((k_b_gather<T>), dim3(gsz), dim3(kT), 0, s, L.d, PS.d_sd, L.d_cpre, L.nsys, L.ctotal,
                     residual ? 4 : 0, residual ? 0 : j + 1, residual ? 1 : 0, act_sel);
  return hipGetLastError();
}

inline int grid_for(int total) { return total < 4096 ? (total > 0 ? total : 1) : 4096; }

// Norm of a vector of every cycle-active system into sumsq[slot].
template <typename T>
hipError_t batch_norm(hipStream_t s, const BatchLevel<T>& L, int which, int j, int slot, int act_sel) {
  hipLaunchKernelGGL((k_b_nrm2<T>), dim3(grid_for(L.ctotal)), dim3(kT), 0, s, L.d, L.d_cpre, L.nsys, L.ctotal, which,
                     j, act_sel);
  hipLaunchKernelGGL(k_b_nrm2_fin, dim3(L.nsys), dim3(kT), 0, s, L.d, L.nsys, slot, act_sel);
  return hipGetLastError();
}

template <typename T>
hipError_t enqueue_cycle(vie_batch_s* B, BatchLevel<T>& L, PassSet& PS, int inner_steps);

// Inner FP32 GMRES for outer step j: b32 = V64_j, x32 = 0, inner_steps Arnoldi
// steps (masked at inner tol), x32 update, Z64_j = x32.
hipError_t enqueue_inner(vie_batch_s* B, int j) {
  hipStream_t s = B->stream;
  BatchLevel<float>& I = B->inner;
  BatchLevel<double>& O = B->outer;
  // inner rhs and zero start (inner cycle flags alias the outer step flags)
  hipLaunchKernelGGL((k_b_copy<double, float>), dim3(grid_for(O.ctotal)), dim3(kT), 0, s, O.d, I.d, O.d_cpre, O.nsys,
                     O.ctotal, 0, j, 3, 0, 0, 0);
  hipLaunchKernelGGL((k_b_copy<float, float>), dim3(grid_for(I.ctotal)), dim3(kT), 0, s, I.d, I.d, I.d_cpre, I.nsys,
                     I.ctotal, 3, 0, 2, 0, 1, 1);
  hipError_t e;
  if ((e = batch_norm<float>(s, I, 3, 0, 1, 1))) return e;       // ||b||^2 -> sumsq[1]
  if ((e = batch_norm<float>(s, I, 3, 0, 0, 1))) return e;       // beta^2 -> sumsq[0]
  hipLaunchKernelGGL((k_b_scale<float>), dim3(grid_for(I.ctotal)), dim3(kT), 0, s, I.d, I.d_cpre, I.nsys, I.ctotal, 3,
                     0, 0, 1);
  if ((e = enqueue_cycle<float>(B, I, B->p32, 0))) return e;
  hipLaunchKernelGGL((k_b_copy<float, double>), dim3(grid_for(I.ctotal)), dim3(kT), 0, s, I.d, O.d, I.d_cpre, I.nsys,
                     I.ctotal, 2, 0, 1, j, 0, 1);
  return hipGetLastError();
}

// One restart cycle (V_0 already holds r / beta and sumsq[0] = beta^2):
// init, m Arnoldi steps with CGS2, triangular solve, x update.
template <typename T>
hipError_t enqueue_cycle(vie_batch_s* B, BatchLevel<T>& L, PassSet& PS, int) {
  hipStream_t s = B->stream;
  hipError_t e;
  hipLaunchKernelGGL(k_b_init, dim3((L.nsys + 63) / 64), dim3(64), 0, s, L.d, L.nsys, L.m);
  for (int j = 0; j < L.m; ++j) {
    if (L.flex && B->mixed) {
      if ((e = enqueue_inner(B, j))) return e;
    } else if (L.flex && B->circ_tier) {
      // Z_j = W^{-1} V_j for the systems active in this cycle, one after the other
      // on the batch stream (systems that share a plan share its work buffers)
      for (int i = 0; i < L.nsys; ++i) {
        if (!B->on[i]) continue;
        const KDesc& D = L.h[i];
        if ((e = circ_apply_rows(B->circ[i], (const double2*)D.V + (long)j * D.n, (double2*)D.Z + (long)j * D.n,
                                 s)))
          return e;
      }
    }
    if ((e = batch_matvec<T>(B, PS, L, false, j))) return e;
    const int g = grid_for(L.ctotal);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL((k_b_mdot<T>), dim3(g), dim3(kT), 0, s, L.d, L.d_cpre, L.nsys, L.ctotal, j);
      hipLaunchKernelGGL(k_b_reduce, dim3(grid_for(L.nsys * (j + 1))), dim3(kT), 0, s, L.d, L.nsys, j + 1, pass);
      hipLaunchKernelGGL((k_b_orth<T>), dim3(g), dim3(kT), 0, s, L.d, L.d_cpre, L.nsys, L.ctotal, j, pass);
    }
    if ((e = batch_norm<T>(s, L, 0, j + 1, 0, 0))) return e;
    hipLaunchKernelGGL((k_b_scale<T>), dim3(g), dim3(kT), 0, s, L.d, L.d_cpre, L.nsys, L.ctotal, 0, j + 1, j + 1, 0);
    hipLaunchKernelGGL(k_b_givens, dim3((L.nsys + 63) / 64), dim3(64), 0, s, L.d, L.nsys, j, L.m);
  }
  hipLaunchKernelGGL(k_b_trisolve, dim3((L.nsys + 63) / 64), dim3(64), 0, s, L.d, L.nsys, L.m);
  hipLaunchKernelGGL((k_b_update<T>), dim3(grid_for(L.ctotal)), dim3(kT), 0, s, L.d, L.d_cpre, L.nsys, L.ctotal);
  return hipGetLastError();
}

}  // namespace

extern "C" int vie_solve_batch(vie_plan_t const* plans, const vie_c128* const* rhs, vie_c128* const* x, int count,
                               double tol, const vie_solve_opts* opts, vie_solve_info* infos) {
  if (!plans || !rhs || !x || count < 1 || !(tol > 0)) return VIE_EINVAL;
  vie_solve_opts o{50, 10000, 0, 0, 20, 1e-4, 1, 0};
  if (opts) o = *opts;
  hipStream_t user_stream = nullptr;
  if (o.restart <= 0) o.restart = 50;
  if (o.maxit <= 0) o.maxit = 10000;
  if (o.inner_restart <= 0) o.inner_restart = 20;
  if (!(o.inner_tol > 0)) o.inner_tol = 1e-4;
  if (o.restart > 500 || o.inner_restart > 500) return VIE_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  vie_batch_s B;
  B.nsys = count;
  B.sp.resize(count);
  if (o.precision < 0 || o.precision > 3 || o.precision == 2) return VIE_EINVAL;
  B.mixed = o.precision == 1;
  B.circ_tier = o.precision == 3;
  if (B.circ_tier) o.use_graph = 0;   // the active set is chosen on the host per cycle
  B.circ.assign(count, nullptr);
  std::vector<long> n(count), nfull(count);
  std::vector<Support> sup(count);
  for (int s = 0; s < count; ++s) {
    SysPlan& P = B.sp[s];
    hipStream_t st;
    int hc = 0;
    if (!plans[s] || !rhs[s] || !x[s]) return VIE_EINVAL;
    int rc = plan_export(plans[s], &P.g, &P.t64, &P.t32, &P.U64, &P.U32, &P.goct64, &P.goct32, &P.chi64, &P.chi32,
                         P.tw64, P.tw32, &st, &hc);
    if (rc) return rc;
    if (!hc) return VIE_ESTATE;
    if (B.mixed && !P.goct32) return VIE_ESTATE;
    if (B.circ_tier && !(B.circ[s] = plan_circ(plans[s]))) return VIE_ESTATE;
    if (s == 0) user_stream = st;
    const int* col = nullptr;
    int ns = 0;
    if ((rc = plan_support(plans[s], &col, &ns))) return rc;
    sup[s] = Support{col, ns, (long)P.g.n1 * P.g.n2, P.g.n3};
    nfull[s] = 3 * P.g.N;
    n[s] = sup[s].size();   // Krylov vectors hold the support columns only
  }
  // the batch runs on a stream of its own (graph capture needs a non-default
  // stream), ordered after the caller's stream, and returns synchronised
  if (hipStreamSynchronize(user_stream) != hipSuccess) return VIE_EDEVICE;
  if (hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking) != hipSuccess) return VIE_EDEVICE;
  hipStream_t s = B.stream;
  std::vector<const void*> bptr(count);
  std::vector<void*> xptr(count);
  int status = VIE_OK;
  int* act = nullptr;    // cycle flags (outer)
  int* hflags = nullptr;
  std::vector<void*> extra;
  auto cleanup = [&]() {
    if (B.graph) (void)hipGraphExecDestroy(B.graph);
    B.outer.release();
    B.inner.release();
    for (void* q : extra) (void)hipFree(q);
    for (void* q : B.allocs) (void)hipFree(q);
    if (hflags) (void)hipHostFree(hflags);
    (void)hipStreamSynchronize(B.stream);
    (void)hipStreamDestroy(B.stream);
  };
#define BTRY(expr)                  \
  do {                              \
    hipError_t _e = (expr);         \
    if (_e != hipSuccess) {         \
      cleanup();                    \
      return VIE_EDEVICE;           \
    }                               \
  } while (0)
  BTRY(dmalloc(&act, sizeof(int) * count));
  extra.push_back(act);
  // every system gets its own intermediate buffers, so one plan may serve
  // several right-hand sides of the batch
  for (int i = 0; i < count; ++i) {
    SysPlan& P = B.sp[i];
    const size_t u = (size_t)3 * P.g.n1 * P.g.n2 * P.g.M3;
    BTRY(dmalloc(&P.U64, sizeof(double2) * u));
    extra.push_back(P.U64);
    if (B.mixed) {
      BTRY(dmalloc(&P.U32, sizeof(float2) * u));
      extra.push_back(P.U32);
    }
  }
  BTRY(hipHostMalloc(&hflags, sizeof(int) * count * 4 + sizeof(double) * count * 4, hipHostMallocDefault));
  // Support compression (as in vie_solve): off the support A is the identity, so
  // x = b there; on it the system is A_SS x_S = b_S - (A b_off)_S with b_off = b
  // off the support.  Per system: full-length product buffers fx (zero off the
  // support) and fy, the compressed right-hand side bc and solution xc.
  B.p64.h_sd.resize(count);
  B.p32.h_sd.resize(count);
  long nmax = 1;
  for (int i = 0; i < count; ++i) {
    const size_t len = n[i] > 0 ? (size_t)n[i] : 1;
    void *fx = nullptr, *fy = nullptr, *bc = nullptr, *xc = nullptr;
    BTRY(dmalloc(&fx, sizeof(double2) * nfull[i]));
    extra.push_back(fx);
    BTRY(dmalloc(&fy, sizeof(double2) * nfull[i]));
    extra.push_back(fy);
    BTRY(dmalloc(&bc, sizeof(double2) * len));
    extra.push_back(bc);
    BTRY(dmalloc(&xc, sizeof(double2) * len));
    extra.push_back(xc);
    B.p64.h_sd[i] = SDesc{sup[i].col, sup[i].s, sup[i].n3, sup[i].n12, fx, fy};
    bptr[i] = bc;
    xptr[i] = xc;
    if (B.mixed) {
      void *fx32 = nullptr, *fy32 = nullptr;
      BTRY(dmalloc(&fx32, sizeof(float2) * nfull[i]));
      extra.push_back(fx32);
      BTRY(dmalloc(&fy32, sizeof(float2) * nfull[i]));
      extra.push_back(fy32);
      BTRY(hipMemsetAsync(fx32, 0, sizeof(float2) * nfull[i], s));
      B.p32.h_sd[i] = SDesc{sup[i].col, sup[i].s, sup[i].n3, sup[i].n12, fx32, fy32};
    }
    nmax = std::max(nmax, nfull[i]);
  }
  // norms: sq[3 i] = ||b_S||^2, sq[3 i + 1] = ||b_off||^2, sq[3 i + 2] = ||b_c||^2
  double2* dsq = nullptr;
  double2* part = nullptr;
  BTRY(dmalloc(&dsq, sizeof(double2) * 3 * count));
  extra.push_back(dsq);
  BTRY(dmalloc(&part, sizeof(double2) * partial_blocks(nmax)));
  extra.push_back(part);
  BTRY(hipMemsetAsync(dsq, 0, sizeof(double2) * 3 * count, s));
  using K = KrylovOps<double>;
  for (int i = 0; i < count; ++i) {
    double2* fx = (double2*)B.p64.h_sd[i].fx;
    BTRY(hipMemcpyAsync(fx, rhs[i], sizeof(double2) * nfull[i], hipMemcpyDeviceToDevice, s));
    if (sup[i].s > 0) {
      BTRY(gather<double>(sup[i], (const double2*)rhs[i], (double2*)bptr[i], nullptr, s));
      BTRY(K::nrm2sq((const double2*)bptr[i], n[i], part, dsq + 3 * i, s));
      BTRY(zero_support<double>(sup[i], fx, s));
    }
    BTRY(K::nrm2sq(fx, nfull[i], part, dsq + 3 * i + 1, s));
  }
  std::vector<double2> hsq(3 * count);
  BTRY(hipMemcpyAsync(hsq.data(), dsq, sizeof(double2) * 3 * count, hipMemcpyDeviceToHost, s));
  BTRY(hipStreamSynchronize(s));
  std::vector<int> boff(count, 0);
  for (int i = 0; i < count; ++i) {
    if (!std::isfinite(hsq[3 * i].x) || !std::isfinite(hsq[3 * i + 1].x)) {
      cleanup();
      return VIE_EINVAL;   // right-hand side not finite
    }
    boff[i] = sup[i].s > 0 && hsq[3 * i + 1].x > 0;
    if (!boff[i]) continue;
    const SysPlan& P = B.sp[i];
    const SDesc& S = B.p64.h_sd[i];
    BTRY(launch_matvec<double>(P.g, P.t64, S.fx, S.fy, nullptr, 0, P.U64, P.goct64, P.chi64, P.tw64, s));
    BTRY(gather<double>(sup[i], (const double2*)S.fy, (double2*)bptr[i], (const double2*)bptr[i], s));
    BTRY(K::nrm2sq((const double2*)bptr[i], n[i], part, dsq + 3 * i + 2, s));
  }
  for (int i = 0; i < count; ++i) BTRY(hipMemsetAsync(B.p64.h_sd[i].fx, 0, sizeof(double2) * nfull[i], s));
  BTRY(hipMemcpyAsync(hsq.data(), dsq, sizeof(double2) * 3 * count, hipMemcpyDeviceToHost, s));
  BTRY(hipStreamSynchronize(s));
  // ||r|| / ||b|| = (||r_c|| / ||b_c||) * ratio with ratio = ||b_c|| / ||b||
  std::vector<double> ratio(count, 0.0), tolc(count, tol);
  for (int i = 0; i < count; ++i) {
    const double bnorm = std::sqrt(hsq[3 * i].x + hsq[3 * i + 1].x);
    const double bcsq = boff[i] ? hsq[3 * i + 2].x : hsq[3 * i].x;
    if (bnorm > 0 && bcsq > 0) {
      ratio[i] = std::sqrt(bcsq) / bnorm;
      tolc[i] = tol / ratio[i];
    }
  }
  BTRY(build_level<double>(B.outer, n, o.restart, B.mixed || B.circ_tier, tol, bptr, xptr, act, nullptr));
  for (int i = 0; i < count; ++i) B.outer.h[i].tol = tolc[i];
  BTRY(hipMemcpy(B.outer.d, B.outer.h.data(), sizeof(KDesc) * count, hipMemcpyHostToDevice));
  if (B.mixed) {
    std::vector<const void*> ib(count);
    std::vector<void*> ix(count);
    for (int i = 0; i < count; ++i) {
      void *bb = nullptr, *xx = nullptr;
      const size_t len = n[i] > 0 ? (size_t)n[i] : 1;
      BTRY(dmalloc(&bb, sizeof(float2) * len));
      extra.push_back(bb);
      BTRY(dmalloc(&xx, sizeof(float2) * len));
      extra.push_back(xx);
      ib[i] = bb;
      ix[i] = xx;
    }
    // inner cycle flags alias the outer step flags (an outer system that stopped
    // needs no preconditioning); the inner level has its own step flags
    BTRY(build_level<float>(B.inner, n, o.inner_restart, false, o.inner_tol, ib, ix, nullptr, nullptr));
    for (int i = 0; i < count; ++i) B.inner.h[i].act0 = B.outer.h[i].act;
    BTRY(hipMemcpy(B.inner.d, B.inner.h.data(), sizeof(KDesc) * count, hipMemcpyHostToDevice));
    BTRY(build_passes<float>(&B, B.p32, B.inner, B.allocs));
  }
  BTRY(build_passes<double>(&B, B.p64, B.outer, B.allocs));
  BatchLevel<double>& O = B.outer;
  // all systems on for the set-up reductions
  std::vector<int> on(count, 1);
  BTRY(hipMemcpyAsync(act, on.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
  BTRY(batch_norm<double>(s, O, 3, 0, 1, 1));          // ||b_c||^2
  if (o.use_x0) {
    for (int i = 0; i < count; ++i)
      if (sup[i].s > 0) BTRY(gather<double>(sup[i], (const double2*)x[i], (double2*)xptr[i], nullptr, s));
    BTRY(batch_matvec<double>(&B, B.p64, O, true, 0));  // r = b - A x
  } else {
    hipLaunchKernelGGL((k_b_copy<double, double>), dim3(grid_for(O.ctotal)), dim3(kT), 0, s, O.d, O.d, O.d_cpre,
                       count, O.ctotal, 3, 0, 2, 0, 1, 1);   // x = 0
    hipLaunchKernelGGL((k_b_copy<double, double>), dim3(grid_for(O.ctotal)), dim3(kT), 0, s, O.d, O.d, O.d_cpre,
                       count, O.ctotal, 3, 0, 4, 0, 0, 1);   // r = b
  }
  std::vector<int> iters(count, 0), inner_it(count, 0), restarts(count, 0), matvecs(count, 0);
  std::vector<double> bn(count), rel(count), est(count);
  std::vector<double2> sq(2 * count);
  bool graph_built = false;
  int cycles = 0;
  while (true) {
    // residual norms of the cycle start: sumsq[0] = ||r||^2
    BTRY(batch_norm<double>(s, O, 4, 0, 0, 1));
    for (int i = 0; i < count; ++i)
      BTRY(hipMemcpyAsync(&sq[2 * i], O.h[i].sumsq, sizeof(double2) * 2, hipMemcpyDeviceToHost, s));
    BTRY(hipMemcpyAsync(hflags, O.h[0].iters - 2 * count, sizeof(int) * 3 * count, hipMemcpyDeviceToHost, s));
    BTRY(hipStreamSynchronize(s));
    int nact = 0;
    for (int i = 0; i < count; ++i) {
      bn[i] = std::sqrt(sq[2 * i + 1].x);
      rel[i] = bn[i] > 0 ? std::sqrt(sq[2 * i].x) / bn[i] * ratio[i] : 0.0;
      iters[i] = hflags[2 * count + i];
      on[i] = (std::isfinite(rel[i]) && rel[i] > tol && iters[i] < o.maxit) ? 1 : 0;
      if (!std::isfinite(rel[i])) status = VIE_ENUMERIC;
      nact += on[i];
    }
    if (nact == 0 || status == VIE_ENUMERIC) break;
    B.on = on;
    BTRY(hipMemcpyAsync(act, on.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    // V_0 = r / beta for the active systems
    hipLaunchKernelGGL((k_b_scale<double>), dim3(grid_for(O.ctotal)), dim3(kT), 0, s, O.d, O.d_cpre, count, O.ctotal,
                       4, 0, 0, 1);
    if (o.use_graph) {
      if (!graph_built) {
        hipGraph_t gr;
        BTRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t ce = enqueue_cycle<double>(&B, O, B.p64, 0);
        hipError_t ee = hipStreamEndCapture(s, &gr);
        if (ce || ee) {
          cleanup();
          return VIE_EDEVICE;
        }
        BTRY(hipGraphInstantiate(&B.graph, gr, nullptr, nullptr, 0));
        (void)hipGraphDestroy(gr);
        graph_built = true;
      }
      BTRY(hipGraphLaunch(B.graph, s));
    } else {
      BTRY(enqueue_cycle<double>(&B, O, B.p64, 0));
    }
    ++cycles;
    for (int i = 0; i < count; ++i)
      if (on[i]) restarts[i]++;
    // true residual r = b - A x of the active systems
    BTRY(batch_matvec<double>(&B, B.p64, O, true, 0));
    if (cycles > 100000) break;
  }
  // x = b off the support, xc on it
  for (int i = 0; i < count; ++i) {
    BTRY(hipMemcpyAsync(x[i], rhs[i], sizeof(double2) * nfull[i], hipMemcpyDeviceToDevice, s));
    if (sup[i].s > 0) BTRY(scatter<double>(sup[i], (const double2*)xptr[i], (double2*)x[i], s));
  }
  // report
  std::vector<int> inn(count, 0);
  BTRY(hipStreamSynchronize(s));
  if (B.mixed) {
    // flags of the inner level: [act | kdone | iters], nsys each
    std::vector<int> all(3 * count);
    BTRY(hipMemcpy(all.data(), B.inner.h[0].act, sizeof(int) * 3 * count, hipMemcpyDeviceToHost));
    for (int i = 0; i < count; ++i) inn[i] = all[2 * count + i];
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = status;
  for (int i = 0; i < count; ++i) {
    const int st = status == VIE_ENUMERIC ? VIE_ENUMERIC : (rel[i] <= tol ? VIE_OK : VIE_ENOCONV);
    if (st != VIE_OK && worst == VIE_OK) worst = st;
    if (infos) {
      infos[i].iters = iters[i];
      infos[i].inner_iters = inn[i];
      infos[i].restarts = restarts[i];
      infos[i].matvecs = iters[i] + restarts[i] + (o.use_x0 ? 1 : 0) + boff[i];
      infos[i].status = st;
      infos[i].rel_res_true = rel[i];
      infos[i].rel_res_est = rel[i];
      infos[i].seconds = secs;
      infos[i].fallback = 0;
      infos[i].stalled = 0;
    }
  }
  cleanup();
#undef BTRY
  return worst;
}
