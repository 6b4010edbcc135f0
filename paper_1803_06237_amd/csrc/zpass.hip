// Passes 1 and 3 of the matvec (zero-padded z FFT / inverse z FFT with crop and
// contrast) as four-step transforms held in registers.
//
// Length M3 = A * B.  Each pencil is handled by A threads.  Thread a holds
// x[a + A b] (b < B), takes a B-point DFT over b in registers, multiplies by
// W_M3^(a k1), and one LDS exchange hands the values of frequency k1 of all A
// threads to the thread that owns task k1 (tasks k1 = a + A t, t < B / A),
// which finishes with an A-point DFT: X[k1 + B k2], k2 < A.  The inverse is the
// same with conjugate twiddles.  The zero padding (x[n] = 0 for n >= n3) and
// the crop (only n < n3 kept) come for free from the index ranges.
//
// A block handles P pencils of consecutive i1 at fixed (component, i2), so the
// kz-plane-major intermediate U[kz][c][i2][i1] is written and read in runs of P
// elements through an LDS staging array [kz][P + 1] (padded against bank
// conflicts); the z-contiguous vectors x, y, chi are accessed directly.
//
// The exchange moves the real parts, then the imaginary parts, and the staging
// array holds one half of the kz range at a time.  That halves the LDS of a
// pencil (8 KiB at M3 = 1024 in FP64), so a CU holds twice as many pencils: at
// 32 x 32 x 512 every pencil of a pass is resident at once instead of in one
// and a half rounds of workgroups.
#include <hip/hip_runtime.h>

#include "block_maps.hpp"
#include "dft_reg.hpp"
#include "vie_internal.hpp"

namespace vie {

namespace {
// exchange slot of (pencil p, frequency k1, source thread a): rotated so that
// the A reads of one thread and the A writes of one frequency hit distinct banks
template <int A>
__device__ __forceinline__ int xslot(int p, int M, int k1, int a) {
  return p * M + k1 * A + ((a + k1) & (A - 1));
}
// Pencils exchange real and imaginary parts separately and stage half of the
// kz range at a time (both precisions: it halves the LDS of a workgroup, so
// twice as many are resident; FP32 forward pass 21.4 -> 15.6 us at 32x32x512)
template <typename T>
constexpr bool z4_split() {
  return true;
}

// Thread a of pencil p hands v[k1] to the owner of frequency k1; afterwards
// w[t A + j] holds frequency a + A t of thread j (t < B / A).  S must be free on
// entry; the caller synchronises before reusing it.
template <typename T, int A, int B>
__device__ __forceinline__ void z4_exchange(const cx<T>* v, cx<T>* w, cx<T>* S, int p, int a, bool on) {
  constexpr int M = A * B;
  if constexpr (z4_split<T>()) {
    T* Sd = reinterpret_cast<T*>(S);
    if (on) {
#pragma unroll
      for (int k1 = 0; k1 < B; ++k1) Sd[xslot<A>(p, M, k1, a)] = v[k1].x;
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int t = 0; t < B / A; ++t)
#pragma unroll
        for (int j = 0; j < A; ++j) w[t * A + j].x = Sd[xslot<A>(p, M, a + A * t, j)];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int k1 = 0; k1 < B; ++k1) Sd[xslot<A>(p, M, k1, a)] = v[k1].y;
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int t = 0; t < B / A; ++t)
#pragma unroll
        for (int j = 0; j < A; ++j) w[t * A + j].y = Sd[xslot<A>(p, M, a + A * t, j)];
    }
  } else {
    if (on) {
#pragma unroll
      for (int k1 = 0; k1 < B; ++k1) S[xslot<A>(p, M, k1, a)] = v[k1];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int t = 0; t < B / A; ++t)
#pragma unroll
        for (int j = 0; j < A; ++j) w[t * A + j] = S[xslot<A>(p, M, a + A * t, j)];
    }
  }
}
}  // namespace

// LDS of a workgroup of P pencils of length M
template <typename T>
size_t z4_lds_for(int M, int P) {
  return (size_t)(z4_split<T>() ? M / 2 : M) * (P + 1) * sizeof(cx<T>);
}

template <typename T, int A, int B>
__device__ __forceinline__ void zfwd4_body(gptr<const cx<T>> __restrict__ x, gptr<cx<T>> __restrict__ U,
                                           const Geom& g, int P, gptr<const cx<T>> __restrict__ tw, int blk,
                                           cx<T>* S, int tid) {
  constexpr int M = A * B;
  const PencilBlock pb = pencil_block(blk, g.n1, g.n2, P);
  const int i2 = pb.i2, c = pb.c, i1_0 = pb.i1_0, np = pb.np;
  const int p = tid / A, a = tid % A;
  const int ld = P + 1;
  cx<T> v[B];
  if (p < np) {
    gptr<const cx<T>> src = x + (((long)c * g.n1 + i1_0 + p) * g.n2 + i2) * g.n3;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int n = a + A * b;
      v[b] = cx<T>{(T)0, (T)0};
      if (b < B / 2 && n < g.n3) v[b] = src[n];   // n >= M/2 >= n3 is padding
    }
    dft_reg<T, false, B>(v);
#pragma unroll
    for (int k1 = 1; k1 < B; ++k1) v[k1] = cmul(v[k1], tw[a * k1]);
  }
  cx<T> w[B];
  z4_exchange<T, A, B>(v, w, S, p, a, p < np);
  if (p < np) {
#pragma unroll
    for (int t = 0; t < B / A; ++t) dft_reg<T, false, A>(w + t * A);
  }
  __syncthreads();
  // w[t A + k2] is X[kz] at kz = a + A t + B k2; staged H kz-ranges of M / H
  constexpr int H = z4_split<T>() ? 2 : 1;
  const long plane = 3L * g.n1 * g.n2;
  gptr<cx<T>> dst = U + ((long)c * g.n2 + i2) * g.n1 + i1_0;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    if (p < np) {
#pragma unroll
      for (int t = 0; t < B / A; ++t)
#pragma unroll
        for (int k2 = 0; k2 < A / H; ++k2) S[(a + A * t + B * k2) * ld + p] = w[t * A + h * (A / H) + k2];
    }
    __syncthreads();
    gptr<cx<T>> dh = dst + (long)h * (M / H) * plane;
    if (np == P) {
      // full block: thread t owns pencil t % P at planes t / P + A k, k < B / H;
      // eight values in flight per batch, no divisions
      const int pp = tid % P, kz0 = tid / P;
#pragma unroll
      for (int k0 = 0; k0 < B / H; k0 += 8) {
        cx<T> tmp[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) tmp[k] = S[(kz0 + A * (k0 + k)) * ld + pp];
#pragma unroll
        for (int k = 0; k < 8; ++k) dh[(long)(kz0 + A * (k0 + k)) * plane + pp] = tmp[k];
      }
    } else {
      for (int t = tid; t < np * (M / H); t += blockDim.x) {
        const int pp = t % np, kz = t / np;
        dh[kz * plane + pp] = S[kz * ld + pp];
      }
    }
    __syncthreads();
  }
}

template <typename T, int A, int B>
__global__ __launch_bounds__(256) void k_zfwd4(const cx<T>* __restrict__ x, cx<T>* __restrict__ U, Geom g,
                                                int P, const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  zfwd4_body<T, A, B>((gptr<const cx<T>>)x, (gptr<cx<T>>)U, g, P, (gptr<const cx<T>>)tw,
                      xcd_group(blockIdx.x, gridDim.x, P, (int)sizeof(cx<T>)), reinterpret_cast<cx<T>*>(smem_raw), threadIdx.x);
}

template <typename T, int A, int B, int MODE>
__device__ __forceinline__ void zinv4_body(gptr<const cx<T>> __restrict__ U, gptr<const cx<T>> __restrict__ x,
                                           gptr<cx<T>> __restrict__ y, gptr<const cx<T>> __restrict__ bvec,
                                           gptr<const cx<T>> __restrict__ chi, const Geom& g, int P,
                                           gptr<const cx<T>> __restrict__ tw, int blk, cx<T>* S, int tid) {
  constexpr int M = A * B;
  const PencilBlock pb = pencil_block(blk, g.n1, g.n2, P);
  const int i2 = pb.i2, c = pb.c, i1_0 = pb.i1_0, np = pb.np;
  const int p = tid / A, a = tid % A;
  const int ld = P + 1;
  const long plane = 3L * g.n1 * g.n2;
  gptr<const cx<T>> src = U + ((long)c * g.n2 + i2) * g.n1 + i1_0;
  // staged H kz-ranges of M / H; range h holds v[b] for b in [h B / H, (h + 1) B / H)
  constexpr int H = z4_split<T>() ? 2 : 1;
  cx<T> v[B];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    gptr<const cx<T>> sh = src + (long)h * (M / H) * plane;
    if (np == P) {
      // full block: thread t owns pencil t % P at planes t / P + A k, k < B / H;
      // eight loads in flight per batch (one at a time would expose every
      // latency), no divisions
      const int pp = tid % P, kz0 = tid / P;
#pragma unroll
      for (int k0 = 0; k0 < B / H; k0 += 8) {
        cx<T> tmp[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) tmp[k] = sh[(long)(kz0 + A * (k0 + k)) * plane + pp];
#pragma unroll
        for (int k = 0; k < 8; ++k) S[(kz0 + A * (k0 + k)) * ld + pp] = tmp[k];
      }
    } else {
      for (int t = tid; t < np * (M / H); t += blockDim.x) {
        const int pp = t % np, kz = t / np;
        S[kz * ld + pp] = sh[kz * plane + pp];
      }
    }
    __syncthreads();
    if (p < np) {
#pragma unroll
      for (int b = 0; b < B / H; ++b) v[h * (B / H) + b] = S[(a + A * b) * ld + p];
    }
    __syncthreads();
  }
  if (p < np) {
    dft_reg<T, true, B>(v);
#pragma unroll
    for (int k1 = 1; k1 < B; ++k1) v[k1] = cmulc(v[k1], tw[a * k1]);
  }
  cx<T> w[B];
  z4_exchange<T, A, B>(v, w, S, p, a, p < np);
  if (p < np) {
    const long vox = ((long)(i1_0 + p) * g.n2 + i2) * g.n3;
    const long off = (long)c * g.N + vox;
#pragma unroll
    for (int t = 0; t < B / A; ++t) {
      const int k1 = a + A * t;
      cx<T>* z = w + t * A;
      dft_reg<T, true, A>(z);
      // Pin the kept outputs in registers here.  Otherwise the compiler sinks
      // their arithmetic into the conditional stores below, which keeps the
      // transform's intermediates live across all of them (280 instead of 168
      // VGPRs in FP64 at A = 32: one wave per SIMD instead of three).
#pragma unroll
      for (int k2 = 0; k2 < A / 2; ++k2) asm volatile("" : "+v"(z[k2].x), "+v"(z[k2].y));
#pragma unroll
      for (int k2 = 0; k2 < A / 2; ++k2) {
        const int n = k1 + B * k2;
        if (n < g.n3) {   // n >= M/2 >= n3 is cropped
          const cx<T> r = csub(x[off + n], cmul(chi[vox + n], z[k2]));
          y[off + n] = MODE == 0 ? r : csub(bvec[off + n], r);
        }
      }
    }
  }
  __syncthreads();
}

template <typename T, int A, int B, int MODE>
__global__ __launch_bounds__(256) void k_zinv4(const cx<T>* __restrict__ U, const cx<T>* __restrict__ x,
                                                cx<T>* __restrict__ y, const cx<T>* __restrict__ bvec,
                                                const cx<T>* __restrict__ chi, Geom g, int P,
                                                const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  zinv4_body<T, A, B, MODE>((gptr<const cx<T>>)U, (gptr<const cx<T>>)x, (gptr<cx<T>>)y, (gptr<const cx<T>>)bvec,
                            (gptr<const cx<T>>)chi, g, P, (gptr<const cx<T>>)tw, xcd_group(blockIdx.x, gridDim.x, P, (int)sizeof(cx<T>)),
                            reinterpret_cast<cx<T>*>(smem_raw), threadIdx.x);
}

// Launch: returns hipErrorNotSupported when (M3, precision) has no four-step
// instance, so the caller falls back to the generic LDS Stockham passes.
template <typename T>
struct ZShape {
  int A, B, P;
};

// Pencil counts P tried by the plan-time tuner, default first; each keeps the
// workgroup (A P threads) within the kernels' 256 and its LDS (z4_lds_for)
// within 160 KiB.
template <typename T>
int z4_pencil_options(int M3, int* out, int cap) {
  const bool dbl = sizeof(T) == 8;
  int opts[6] = {0, 0, 0, 0, 0, 0}, n = 0;
  if (M3 == 512) {                                   // A = 16
    if (dbl) { opts[0] = 8; opts[1] = 4; opts[2] = 16; opts[3] = 2; n = 4; }
    else { opts[0] = 16; opts[1] = 8; opts[2] = 4; opts[3] = 2; n = 4; }
  } else if (M3 == 1024) {                           // A = 32
    if (dbl) { opts[0] = 4; opts[1] = 2; opts[2] = 8; n = 3; }
    else { opts[0] = 8; opts[1] = 4; opts[2] = 2; n = 3; }
  } else if (M3 == 2048) {                           // A = 32, 64 values per thread
    if (dbl) { opts[0] = 2; opts[1] = 4; opts[2] = 1; n = 3; }
    else { opts[0] = 4; opts[1] = 2; n = 2; }
  } else if (M3 == 4096) {                           // A = 64, 64 values per thread
    if (dbl) { opts[0] = 2; opts[1] = 1; n = 2; }
    else { opts[0] = 2; opts[1] = 4; opts[2] = 1; n = 3; }
  }
  for (int i = 0; i < n && i < cap; ++i) out[i] = opts[i];
  return n;
}

template <typename T>
static bool zshape(int M3, ZShape<T>* s, int P = 0) {
  int opts[8];
  const int n = z4_pencil_options<T>(M3, opts, 8);
  if (n == 0) return false;
  bool ok = P == 0;
  for (int i = 0; i < n; ++i) ok = ok || opts[i] == P;
  if (!ok) return false;
  const int p = P ? P : opts[0];
  if (M3 == 512) *s = {16, 32, p};
  else if (M3 == 1024) *s = {32, 32, p};
  else if (M3 == 2048) *s = {32, 64, p};
  else *s = {64, 64, p};
  return true;
}

template <typename T>
size_t z4_lds_bytes(int M3, int P) {
  ZShape<T> s;
  if (!zshape<T>(M3, &s, P)) return 0;
  return z4_lds_for<T>(M3, s.P);
}

template <typename T>
hipError_t launch_z4(int which, const Geom& g, int P, const void* x, void* y, const void* b, int mode, void* U,
                     const void* chi, const void* twz, hipStream_t st) {
  using C = cx<T>;
  ZShape<T> s;
  if (!zshape<T>(g.M3, &s, P)) return hipErrorNotSupported;
  const int nb1 = (g.n1 + s.P - 1) / s.P;
  const dim3 grid(3 * g.n2 * nb1), block(s.A * s.P);
  const size_t lds = z4_lds_for<T>(g.M3, s.P);
#define VIE_Z4(AA, BB)                                                                                        \
  if (s.A == AA && s.B == BB) {                                                                               \
    if (which == 0)                                                                                           \
      hipLaunchKernelGGL((k_zfwd4<T, AA, BB>), grid, block, lds, st, (const C*)x, (C*)U, g, s.P, (const C*)twz); \
    else if (mode == 0)                                                                                       \
      hipLaunchKernelGGL((k_zinv4<T, AA, BB, 0>), grid, block, lds, st, (const C*)U, (const C*)x, (C*)y,      \
                         (const C*)nullptr, (const C*)chi, g, s.P, (const C*)twz);                             \
    else                                                                                                      \
      hipLaunchKernelGGL((k_zinv4<T, AA, BB, 1>), grid, block, lds, st, (const C*)U, (const C*)x, (C*)y,      \
                         (const C*)b, (const C*)chi, g, s.P, (const C*)twz);                                   \
    return hipGetLastError();                                                                                 \
  }
  VIE_Z4(16, 32)
  VIE_Z4(32, 32)
  VIE_Z4(32, 64)
  VIE_Z4(64, 64)
#undef VIE_Z4
  return hipErrorNotSupported;
}

__device__ __forceinline__ int find_sys(const int* prefix, int nsys, int item) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Persistent batched z passes: each workgroup walks the (system, pencil block)
// items of the batch with a grid stride.
template <typename T, int A, int B>
__global__ __launch_bounds__(256) void k_zfwd4_batch(const PassDesc* __restrict__ d, const int* __restrict__ prefix,
                                                     int nsys, int total, int jx, int jy) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* S = reinterpret_cast<cx<T>*>(smem_raw);
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(prefix, nsys, item);
    const PassDesc& D = d[s];
    if (D.active && *D.active == 0) continue;
    zfwd4_body<T, A, B>((gptr<const cx<T>>)(const cx<T>*)D.xb + (long)jx * D.xs, (gptr<cx<T>>)(cx<T>*)D.U, D.g, D.P,
                        (gptr<const cx<T>>)(const cx<T>*)D.twz, item - prefix[s], S, opaque_tid());
  }
}

template <typename T, int A, int B, int MODE>
__global__ __launch_bounds__(256) void k_zinv4_batch(const PassDesc* __restrict__ d, const int* __restrict__ prefix,
                                                     int nsys, int total, int jx, int jy) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* S = reinterpret_cast<cx<T>*>(smem_raw);
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int s = find_sys(prefix, nsys, item);
    const PassDesc& D = d[s];
    if (D.active && *D.active == 0) continue;
    zinv4_body<T, A, B, MODE>((gptr<const cx<T>>)(const cx<T>*)D.U, (gptr<const cx<T>>)(const cx<T>*)D.xb + (long)jx * D.xs,
                              (gptr<cx<T>>)(cx<T>*)D.yb + (long)jy * D.ys, (gptr<const cx<T>>)(const cx<T>*)D.b,
                              (gptr<const cx<T>>)(const cx<T>*)D.chi, D.g, D.P, (gptr<const cx<T>>)(const cx<T>*)D.twz,
                              item - prefix[s], S, opaque_tid());
  }
}

template <typename T>
bool z4_shape(int M3, int* A, int* B, int* P) {
  ZShape<T> s;
  if (!zshape<T>(M3, &s)) return false;
  *A = s.A;
  *B = s.B;
  *P = s.P;
  return true;
}

template <typename T>
hipError_t launch_z4_batch(int which, int mode, const PassDesc* d, const int* prefix, int nsys, int total, int A,
                           int B, int P, int jx, int jy, hipStream_t st) {
  const size_t lds = z4_lds_for<T>(A * B, P);
  const dim3 grid(total < 4096 ? total : 4096), block(A * P);
#define VIE_Z4B(AA, BB)                                                                                      \
  if (A == AA && B == BB) {                                                                                  \
    if (which == 0)                                                                                          \
      hipLaunchKernelGGL((k_zfwd4_batch<T, AA, BB>), grid, block, lds, st, d, prefix, nsys, total, jx, jy);  \
    else if (mode == 0)                                                                                      \
      hipLaunchKernelGGL((k_zinv4_batch<T, AA, BB, 0>), grid, block, lds, st, d, prefix, nsys, total, jx, jy); \
    else                                                                                                     \
      hipLaunchKernelGGL((k_zinv4_batch<T, AA, BB, 1>), grid, block, lds, st, d, prefix, nsys, total, jx, jy); \
    return hipGetLastError();                                                                                \
  }
  VIE_Z4B(16, 32)
  VIE_Z4B(32, 32)
  VIE_Z4B(32, 64)
  VIE_Z4B(64, 64)
#undef VIE_Z4B
  return hipErrorNotSupported;
}

template <typename T>
hipError_t allow_lds_z4() {
  hipError_t e;
  const int big = 160 * 1024;
#define VIE_ALLOW(AA, BB)                                                                                   \
  if ((e = hipFuncSetAttribute((const void*)k_zfwd4<T, AA, BB>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) \
    return e;                                                                                                 \
  if ((e = hipFuncSetAttribute((const void*)k_zinv4<T, AA, BB, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,    \
                               big)))                                                                         \
    return e;                                                                                                 \
  if ((e = hipFuncSetAttribute((const void*)k_zinv4<T, AA, BB, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,    \
                               big)))                                                                         \
    return e;
  VIE_ALLOW(16, 32)
  VIE_ALLOW(32, 32)
  VIE_ALLOW(32, 64)
  VIE_ALLOW(64, 64)
#undef VIE_ALLOW
#define VIE_ALLOWB(AA, BB)                                                                                         \
  if ((e = hipFuncSetAttribute((const void*)k_zfwd4_batch<T, AA, BB>,                                           \
                               hipFuncAttributeMaxDynamicSharedMemorySize, big)))                                \
    return e;                                                                                                      \
  if ((e = hipFuncSetAttribute((const void*)k_zinv4_batch<T, AA, BB, 0>,                                        \
                               hipFuncAttributeMaxDynamicSharedMemorySize, big)))                                \
    return e;                                                                                                      \
  if ((e = hipFuncSetAttribute((const void*)k_zinv4_batch<T, AA, BB, 1>,                                        \
                               hipFuncAttributeMaxDynamicSharedMemorySize, big)))                                \
    return e;
  VIE_ALLOWB(16, 32)
  VIE_ALLOWB(32, 32)
  VIE_ALLOWB(32, 64)
  VIE_ALLOWB(64, 64)
#undef VIE_ALLOWB
  return hipSuccess;
}

template hipError_t launch_z4<double>(int, const Geom&, int, const void*, void*, const void*, int, void*,
                                      const void*, const void*, hipStream_t);
template hipError_t launch_z4<float>(int, const Geom&, int, const void*, void*, const void*, int, void*,
                                     const void*, const void*, hipStream_t);
template int z4_pencil_options<double>(int, int*, int);
template int z4_pencil_options<float>(int, int*, int);
template hipError_t allow_lds_z4<double>();
template hipError_t allow_lds_z4<float>();
template size_t z4_lds_bytes<double>(int, int);
template bool z4_shape<double>(int, int*, int*, int*);
template bool z4_shape<float>(int, int*, int*, int*);
template hipError_t launch_z4_batch<double>(int, int, const PassDesc*, const int*, int, int, int, int, int, int, int,
                                            hipStream_t);
template hipError_t launch_z4_batch<float>(int, int, const PassDesc*, const int*, int, int, int, int, int, int, int,
                                           hipStream_t);
template size_t z4_lds_bytes<float>(int, int);

}  // namespace vie
