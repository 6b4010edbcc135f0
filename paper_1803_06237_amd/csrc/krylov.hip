// GMRES(m) and flexible GMRES(m) on the device (Section V-D: the discrete J-VIE
// is solved by GMRES with matrix-vector products only).
//
// Arnoldi uses classical Gram-Schmidt with a selective second sweep: a fused
// multi-dot h = V^H w over all basis vectors followed by a multi-axpy
// w -= V h, repeated once when the first sweep cancelled more than the
// criterion of Daniel, Gragg, Kaufman and Stewart allows (decided on the device).  The Hessenberg matrix is kept in upper-triangular form with complex
// Givens rotations by one device thread; the host reads only the residual
// estimate |g_{j+1}| / ||b|| after each step.  Reductions are two-stage and in
// a fixed order, so results are bitwise reproducible run to run.  All
// reductions and Hessenberg data are FP64; basis vectors are FP64 (cx<double>)
// or FP32 (cx<float>, the inner solve of the mixed tier).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "fft_device.hpp"
#include "krylov.hpp"

namespace vie {

constexpr int kThreads = 256;
constexpr int kEPT = 2;                     // elements per thread held in registers (reductions)
constexpr int kChunk = kThreads * kEPT;     // elements per block (reductions)
constexpr int kGroup = 4;                   // basis vectors per block of the multi-dot

__device__ __forceinline__ double2 to_d(double2 v) { return v; }
__device__ __forceinline__ double2 to_d(float2 v) { return double2{(double)v.x, (double)v.y}; }
template <typename V> __device__ __forceinline__ V from_d(double2 v);
template <> __device__ __forceinline__ double2 from_d<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d<float2>(double2 v) { return float2{(float)v.x, (float)v.y}; }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block-wide sum of NV double values per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < NV; ++i) {
      double s = 0;
      for (int w = 0; w < kThreads / 64; ++w) s += lds[w * NV + i];
      v[i] = s;
    }
  }
  __syncthreads();
}

// partial[i * nblk + blk] = sum over the block's chunk of conj(V_i) w, for the
// kGroup vectors i of blockIdx.y (nblk = gridDim.x element chunks)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mdot(const cx<T>* __restrict__ V, long ldv, int nv,
                                                    const cx<T>* __restrict__ w, long n,
                                                    double2* __restrict__ partial, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double lds[(kThreads / 64) * 2 * kGroup];
  const long e0 = (long)blockIdx.x * kChunk + threadIdx.x;
  double2 wv[kEPT];
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const long e = e0 + (long)k * kThreads;
    wv[k] = e < n ? to_d(w[e]) : double2{0.0, 0.0};
  }
  {
    const int i0 = blockIdx.y * kGroup;
    double acc[2 * kGroup];
#pragma unroll
    for (int q = 0; q < 2 * kGroup; ++q) acc[q] = 0.0;
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
      if (i0 + q < nv) {
        const cx<T>* Vi = V + (long)(i0 + q) * ldv;
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
          const long e = e0 + (long)k * kThreads;
          if (e < n) {
            const double2 a = to_d(Vi[e]);
            acc[2 * q] += a.x * wv[k].x + a.y * wv[k].y;
            acc[2 * q + 1] += a.x * wv[k].y - a.y * wv[k].x;
          }
        }
      }
    }
    block_sum<2 * kGroup>(acc, lds);
    if (threadIdx.x == 0)
      for (int q = 0; q < kGroup; ++q)
        if (i0 + q < nv) partial[(long)(i0 + q) * gridDim.x + blockIdx.x] = double2{acc[2 * q], acc[2 * q + 1]};
  }
}

// out[i] (+)= sum_b partial[i * nblk + b], one workgroup per i, fixed order
__global__ __launch_bounds__(kThreads) void k_reduce(const double2* __restrict__ partial, int nblk,
                                                      double2* __restrict__ out, int accumulate,
                                                      const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double lds[(kThreads / 64) * 2];
  const int i = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
    const double2 p = partial[(long)i * nblk + b];
    v[0] += p.x;
    v[1] += p.y;
  }
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) {
    if (accumulate) out[i] = double2{out[i].x + v[0], out[i].y + v[1]};
    else out[i] = double2{v[0], v[1]};
  }
}

// w += sign * sum_i coef[i] V_i, one element per thread (loads of the nv vectors
// are independent, so they overlap)
template <typename T, typename TW>
__global__ __launch_bounds__(kThreads) void k_maxpy(const cx<T>* __restrict__ V, long ldv, int nv,
                                                     const double2* __restrict__ coef, double sign,
                                                     cx<TW>* __restrict__ w, long n, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double2 c[512];
  for (int i = threadIdx.x; i < nv && i < 512; i += kThreads) c[i] = double2{sign * coef[i].x, sign * coef[i].y};
  __syncthreads();
  const long e = (long)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n) return;
  double2 acc = to_d(w[e]);
  const cx<T>* Ve = V + e;
#pragma unroll 4
  for (int i = 0; i < nv; ++i) {
    const double2 ci = c[i];
    const double2 a = to_d(Ve[(long)i * ldv]);
    acc.x += ci.x * a.x - ci.y * a.y;
    acc.y += ci.x * a.y + ci.y * a.x;
  }
  w[e] = from_d<cx<TW>>(acc);
}

// partial[blk] = sum |w|^2 over the block's chunk
template <typename T>
__global__ __launch_bounds__(kThreads) void k_nrm2_partial(const cx<T>* __restrict__ w, long n,
                                                            double2* __restrict__ partial,
                                                            const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double lds[(kThreads / 64) * 2];
  const long e0 = (long)blockIdx.x * kChunk + threadIdx.x;
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kEPT; ++k) {
    const long e = e0 + (long)k * kThreads;
    if (e < n) {
      const double2 a = to_d(w[e]);
      v[0] += a.x * a.x + a.y * a.y;
    }
  }
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = double2{v[0], 0.0};
}

// dst = src * (1/norm) where norm = sqrt(sumsq->x); dst may alias src
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale(const cx<T>* src, cx<T>* dst, long n,
                                                     const double2* __restrict__ sumsq) {
  const double nr = sqrt(sumsq->x);
  const double s = nr > 0.0 ? 1.0 / nr : 0.0;
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < n; e += (long)gridDim.x * kThreads) {
    const double2 a = to_d(src[e]);
    dst[e] = from_d<cx<T>>(double2{a.x * s, a.y * s});
  }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(kThreads) void k_copy(const cx<TS>* __restrict__ src, cx<TD>* __restrict__ dst,
                                                    long n) {
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < n; e += (long)gridDim.x * kThreads)
    dst[e] = from_d<cx<TD>>(to_d(src[e]));
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero(cx<T>* __restrict__ dst, long n) {
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < n; e += (long)gridDim.x * kThreads)
    dst[e] = cx<T>{(T)0, (T)0};
}

// w += sign * sum_i coef[i] V_i (nv <= 512) and, of the stored result, the block
// partial sums of |w|^2: partial[blk] (blocks of kThreads elements).  Saves the
// separate norm pass over w.
template <typename T, typename TW>
__global__ __launch_bounds__(kThreads) void k_maxpy_nrm(const cx<T>* __restrict__ V, long ldv, int nv,
                                                         const double2* __restrict__ coef, double sign,
                                                         cx<TW>* __restrict__ w, long n,
                                                         double2* __restrict__ partial,
                                                         const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ double2 c[512];
  __shared__ double lds[kThreads / 64];
  for (int i = threadIdx.x; i < nv && i < 512; i += kThreads) c[i] = double2{sign * coef[i].x, sign * coef[i].y};
  __syncthreads();
  const long e = (long)blockIdx.x * kThreads + threadIdx.x;
  double v[1] = {0.0};
  if (e < n) {
    double2 acc = to_d(w[e]);
    const cx<T>* Ve = V + e;
#pragma unroll 4
    for (int i = 0; i < nv; ++i) {
      const double2 ci = c[i];
      const double2 a = to_d(Ve[(long)i * ldv]);
      acc.x += ci.x * a.x - ci.y * a.y;
      acc.y += ci.x * a.y + ci.y * a.x;
    }
    const cx<TW> out = from_d<cx<TW>>(acc);
    w[e] = out;
    const double2 o = to_d(out);
    v[0] = o.x * o.x + o.y * o.y;
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = double2{v[0], 0.0};
}

// First-sweep norm and the second-sweep decision in one block: sumsq = sum of
// the partials (||w'||^2), then the criterion below on ||h||^2.
__global__ __launch_bounds__(kThreads) void k_reduce_dgks(const double2* __restrict__ partial, int nblk,
                                                           double2* __restrict__ sumsq,
                                                           const double2* __restrict__ h, int nv,
                                                           int* __restrict__ gate, double2* __restrict__ h2) {
  __shared__ double lds[(kThreads / 64) * 2];
  __shared__ int s_again;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kThreads) v[0] += partial[b].x;
  for (int i = threadIdx.x; i < nv; i += kThreads) v[1] += h[i].x * h[i].x + h[i].y * h[i].y;
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) {
    sumsq[0] = double2{v[0], 0.0};
    const int again = (v[0] >= v[1]) ? 0 : 1;
    *gate = again;
    s_again = again;
  }
  __syncthreads();
  if (!s_again)
    for (int i = threadIdx.x; i < nv; i += kThreads) h2[i] = double2{0.0, 0.0};
}

// Selective second Gram-Schmidt sweep (Daniel, Gragg, Kaufman and Stewart's
// criterion with eta = 1/sqrt(2)): after the first sweep w' = w - V h, and for
// an orthonormal V, ||w||^2 = ||w'||^2 + ||h||^2, so ||w'|| < eta ||w|| holds
// exactly when ||w'||^2 < ||h||^2.  Then *gate = 1 and the second sweep runs;
// otherwise *gate = 0, its kernels return at once and h2 is zeroed here (the
// Hessenberg column is h1 + h2).  A non-finite norm keeps the second sweep.
__global__ void k_dgks(const double2* __restrict__ h, int nv, const double2* __restrict__ sumsq,
                       int* __restrict__ gate, double2* __restrict__ h2) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nv; i += 64) v += h[i].x * h[i].x + h[i].y * h[i].y;
  v = wave_sum(v);
  const double hh = __shfl(v, 0, 64);
  const int again = (sumsq[0].x >= hh) ? 0 : 1;
  if (threadIdx.x == 0) *gate = again;
  if (!again)
    for (int i = threadIdx.x; i < nv; i += 64) h2[i] = double2{0.0, 0.0};
}

// One Arnoldi step's Hessenberg bookkeeping (single thread).
// h1[0..j] + h2[0..j] = projections of the two Gram-Schmidt sweeps,
// sumsq->x = ||w||^2 after orthogonalisation.
// H is column-major with leading dimension m+1.  state[0] = residual estimate
// |g_{j+1}| / bnorm, state[1] = ||w|| (breakdown when 0), state[2] = 1 if any
// value is non-finite.
__global__ void k_arnoldi_update(const double2* __restrict__ h1, const double2* __restrict__ h2,
                                 const double2* __restrict__ sumsq,
                                 double2* __restrict__ H, int ldh, double* __restrict__ cs,
                                 double2* __restrict__ sn, double2* __restrict__ gvec, int j, double bnorm,
                                 double* __restrict__ state) {
  // the new column h = h1 + h2 is staged in LDS by the whole block; one thread
  // then sweeps the previous rotations down it with the running entry in a
  // register (the loads of h, cs, sn do not depend on the sweep, so they are
  // issued ahead of it), and the block writes the column back
  extern __shared__ unsigned char smem_raw[];
  double2* hs = reinterpret_cast<double2*>(smem_raw);   // j + 2 entries
  for (int i = threadIdx.x; i <= j; i += blockDim.x) hs[i] = double2{h1[i].x + h2[i].x, h1[i].y + h2[i].y};
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hn = sqrt(sumsq->x);
    // previous rotations: [c s; -conj(s) c] on (h_i, h_{i+1})
    double2 a = hs[0];
    for (int i = 0; i < j; ++i) {
      const double2 b = hs[i + 1];
      const double c = cs[i];
      const double2 s = sn[i];
      hs[i] = double2{c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x)};
      a = double2{-(s.x * a.x + s.y * a.y) + c * b.x, -(s.x * a.y - s.y * a.x) + c * b.y};
    }
    // new rotation zeroing h_{j+1} = ||w||
    const double2 b = double2{hn, 0.0};
    const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
    double c;
    double2 sv, r;
    if (nb == 0.0) {
      c = 1.0;
      sv = double2{0.0, 0.0};
      r = a;
    } else if (na == 0.0) {
      c = 0.0;
      sv = double2{1.0, 0.0};
      r = b;
    } else {
      const double t = hypot(na, nb);
      const double2 ph = double2{a.x / na, a.y / na};
      c = na / t;
      // s = ph * conj(b) / t
      sv = double2{(ph.x * b.x + ph.y * b.y) / t, (ph.y * b.x - ph.x * b.y) / t};
      r = double2{ph.x * t, ph.y * t};
    }
    cs[j] = c;
    sn[j] = sv;
    hs[j] = r;
    hs[j + 1] = double2{0.0, 0.0};
    const double2 gj = gvec[j];
    // g_{j+1} = -conj(s) g_j ; g_j = c g_j
    const double2 gn = double2{-(sv.x * gj.x + sv.y * gj.y), -(sv.x * gj.y - sv.y * gj.x)};
    gvec[j + 1] = gn;
    gvec[j] = double2{c * gj.x, c * gj.y};
    const double est = hypot(gn.x, gn.y) / bnorm;
    state[0] = est;
    state[1] = hn;
    state[2] = (isfinite(est) && isfinite(hn) && isfinite(r.x) && isfinite(r.y)) ? 0.0 : 1.0;
  }
  __syncthreads();
  double2* h = H + (long)j * ldh;
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) h[i] = hs[i];
}

// y = R^{-1} g for the leading k x k upper triangle of H (single thread)
__global__ void k_trisolve(const double2* __restrict__ H, int ldh, const double2* __restrict__ gvec, int k,
                           double2* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double2 s = gvec[i];
    for (int l = i + 1; l < k; ++l) {
      const double2 hil = H[(long)l * ldh + i], yl = y[l];
      s.x -= hil.x * yl.x - hil.y * yl.y;
      s.y -= hil.x * yl.y + hil.y * yl.x;
    }
    const double2 d = H[(long)i * ldh + i];
    const double dd = d.x * d.x + d.y * d.y;
    y[i] = double2{(s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd};
  }
}

__global__ void k_set_g(double2* gvec, int m, const double2* sumsq) {
  for (int i = threadIdx.x; i <= m; i += blockDim.x) gvec[i] = double2{0.0, 0.0};
  if (threadIdx.x == 0) gvec[0] = double2{sqrt(sumsq->x), 0.0};
}

// ---- support compression ------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(const cx<T>* __restrict__ full, cx<T>* comp, const cx<T>* sub,
                                                      const int* __restrict__ col, int s, long n12, int n3) {
  const long total = 3L * s * n3;
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < total; e += (long)gridDim.x * kThreads) {
    const long row = e / n3;
    const int t = (int)(e - row * n3);
    const int a = (int)(row / s), p = (int)(row - (long)a * s);
    const cx<T> v = full[((long)a * n12 + col[p]) * n3 + t];
    comp[e] = sub ? cx<T>{sub[e].x - v.x, sub[e].y - v.y} : v;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter(const cx<T>* __restrict__ comp, cx<T>* __restrict__ full,
                                                       const int* __restrict__ col, int s, long n12, int n3,
                                                       int zero) {
  const long total = 3L * s * n3;
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < total; e += (long)gridDim.x * kThreads) {
    const long row = e / n3;
    const int t = (int)(e - row * n3);
    const int a = (int)(row / s), p = (int)(row - (long)a * s);
    full[((long)a * n12 + col[p]) * n3 + t] = zero ? cx<T>{(T)0, (T)0} : comp[e];
  }
}

__global__ __launch_bounds__(kThreads) void k_column_flags(const double2* __restrict__ chi, long n12, int n3,
                                                            int* __restrict__ flags) {
  const long c = (long)blockIdx.x * kThreads + threadIdx.x;
  if (c >= n12) return;
  const double2* z = chi + c * n3;
  int any = 0;
  for (int t = 0; t < n3; ++t) any |= (z[t].x != 0.0 || z[t].y != 0.0) ? 1 : 0;
  flags[c] = any;
}

// ------------------------------------------------------------------ host-side helpers

static inline int nblocks(long n) { return (int)((n + kChunk - 1) / kChunk); }

template <typename T>
hipError_t KrylovOps<T>::nrm2sq(const cx<T>* w, long n, double2* partial, double2* out, hipStream_t s,
                                const int* gate) {
  const int nb = nblocks(n);
  hipLaunchKernelGGL((k_nrm2_partial<T>), dim3(nb), dim3(kThreads), 0, s, w, n, partial, gate);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, partial, nb, out, 0, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::mdot(const cx<T>* V, long ldv, int nv, const cx<T>* w, long n, double2* partial,
                              double2* out, int accumulate, hipStream_t s, const int* gate) {
  const int nb = nblocks(n);
  hipLaunchKernelGGL((k_mdot<T>), dim3(nb, (nv + kGroup - 1) / kGroup), dim3(kThreads), 0, s, V, ldv, nv, w, n,
                     partial, gate);
  hipLaunchKernelGGL(k_reduce, dim3(nv), dim3(kThreads), 0, s, partial, nb, out, accumulate, gate);
  return hipGetLastError();
}

template <typename T>
template <typename TW>
hipError_t KrylovOps<T>::maxpy(const cx<T>* V, long ldv, int nv, const double2* coef, double sign, cx<TW>* w,
                               long n, hipStream_t s, const int* gate) {
  for (int i0 = 0; i0 < nv; i0 += 512) {
    const int cnt = nv - i0 < 512 ? nv - i0 : 512;
    hipLaunchKernelGGL((k_maxpy<T, TW>), dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       V + (long)i0 * ldv, ldv, cnt,
                       coef + i0, sign, w, n, gate);
  }
  return hipGetLastError();
}

template <typename T>
template <typename TW>
hipError_t KrylovOps<T>::maxpy_nrm(const cx<T>* V, long ldv, int nv, const double2* coef, double sign, cx<TW>* w,
                                   long n, double2* partial, hipStream_t s, const int* gate) {
  if (nv > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_maxpy_nrm<T, TW>), dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, V,
                     ldv, nv, coef, sign, w, n, partial, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::reduce_dgks(const double2* partial, int nblk, double2* sumsq, const double2* h1, int nv,
                                     int* gate, double2* h2, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_dgks, dim3(1), dim3(kThreads), 0, s, partial, nblk, sumsq, h1, nv, gate, h2);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::reduce(const double2* partial, int nblk, double2* out, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, partial, nblk, out, 0, gate);
  return hipGetLastError();
}

int maxpy_blocks(long n) { return (int)((n + kThreads - 1) / kThreads); }

template <typename T>
hipError_t KrylovOps<T>::dgks(const double2* h1, int nv, const double2* sumsq, int* gate, double2* h2,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_dgks, dim3(1), dim3(64), 0, s, h1, nv, sumsq, gate, h2);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::scale(const cx<T>* src, cx<T>* dst, long n, const double2* sumsq, hipStream_t s) {
  hipLaunchKernelGGL((k_scale<T>), dim3(2048), dim3(kThreads), 0, s, src, dst, n, sumsq);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::zero(cx<T>* dst, long n, hipStream_t s) {
  hipLaunchKernelGGL((k_zero<T>), dim3(2048), dim3(kThreads), 0, s, dst, n);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::arnoldi_update(const double2* h1, const double2* h2, const double2* sumsq, double2* H,
                                        int ldh, double* cs, double2* sn, double2* g, int j, double bnorm,
                                        double* state, hipStream_t s) {
  // up to 4097 staged values (restart <= 4096): a little above the default 64 KiB
  static const hipError_t lds_ok = hipFuncSetAttribute((const void*)k_arnoldi_update,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 4098 * 16);
  if (lds_ok != hipSuccess) return lds_ok;
  hipLaunchKernelGGL(k_arnoldi_update, dim3(1), dim3(64), (size_t)(j + 2) * sizeof(double2), s, h1, h2, sumsq, H,
                     ldh, cs, sn, g, j, bnorm, state);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::trisolve(const double2* H, int ldh, const double2* g, int k, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(64), 0, s, H, ldh, g, k, y);
  return hipGetLastError();
}

template <typename T>
hipError_t KrylovOps<T>::set_g(double2* g, int m, const double2* sumsq, hipStream_t s) {
  hipLaunchKernelGGL(k_set_g, dim3(1), dim3(256), 0, s, g, m, sumsq);
  return hipGetLastError();
}

template <typename TS, typename TD>
hipError_t convert(const cx<TS>* src, cx<TD>* dst, long n, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<TS, TD>), dim3(2048), dim3(kThreads), 0, s, src, dst, n);
  return hipGetLastError();
}

template struct KrylovOps<double>;
template struct KrylovOps<float>;
template hipError_t KrylovOps<double>::maxpy_nrm<double>(const cx<double>*, long, int, const double2*, double,
                                                         cx<double>*, long, double2*, hipStream_t, const int*);
template hipError_t KrylovOps<float>::maxpy_nrm<float>(const cx<float>*, long, int, const double2*, double,
                                                       cx<float>*, long, double2*, hipStream_t, const int*);
template hipError_t KrylovOps<double>::maxpy<double>(const cx<double>*, long, int, const double2*, double,
                                                     cx<double>*, long, hipStream_t, const int*);
template hipError_t KrylovOps<float>::maxpy<float>(const cx<float>*, long, int, const double2*, double,
                                                   cx<float>*, long, hipStream_t, const int*);
template hipError_t convert<double, float>(const cx<double>*, cx<float>*, long, hipStream_t);
template hipError_t convert<float, double>(const cx<float>*, cx<double>*, long, hipStream_t);
template hipError_t convert<double, double>(const cx<double>*, cx<double>*, long, hipStream_t);

int partial_blocks(long n) { return nblocks(n); }

static inline int grid_for(long n) {
  const long b = (n + kThreads - 1) / kThreads;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

template <typename T>
hipError_t gather(const Support& u, const cx<T>* full, cx<T>* comp, const cx<T>* sub, hipStream_t s) {
  if (u.s == 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather<T>), dim3(grid_for(u.size())), dim3(kThreads), 0, s, full, comp, sub, u.col, u.s,
                     u.n12, u.n3);
  return hipGetLastError();
}

template <typename T>
hipError_t scatter(const Support& u, const cx<T>* comp, cx<T>* full, hipStream_t s) {
  if (u.s == 0) return hipSuccess;
  hipLaunchKernelGGL((k_scatter<T>), dim3(grid_for(u.size())), dim3(kThreads), 0, s, comp, full, u.col, u.s, u.n12,
                     u.n3, 0);
  return hipGetLastError();
}

template <typename T>
hipError_t zero_support(const Support& u, cx<T>* full, hipStream_t s) {
  if (u.s == 0) return hipSuccess;
  hipLaunchKernelGGL((k_scatter<T>), dim3(grid_for(u.size())), dim3(kThreads), 0, s, nullptr, full, u.col, u.s,
                     u.n12, u.n3, 1);
  return hipGetLastError();
}

hipError_t column_flags(const double2* chi, long n12, int n3, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_column_flags, dim3((unsigned)((n12 + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, chi,
                     n12, n3, flags);
  return hipGetLastError();
}

template hipError_t gather<double>(const Support&, const cx<double>*, cx<double>*, const cx<double>*, hipStream_t);
template hipError_t gather<float>(const Support&, const cx<float>*, cx<float>*, const cx<float>*, hipStream_t);
template hipError_t scatter<double>(const Support&, const cx<double>*, cx<double>*, hipStream_t);
template hipError_t scatter<float>(const Support&, const cx<float>*, cx<float>*, hipStream_t);
template hipError_t zero_support<double>(const Support&, cx<double>*, hipStream_t);
template hipError_t zero_support<float>(const Support&, cx<float>*, hipStream_t);

}  // namespace vie
