// Pass 2 of the matvec for the 64 x 32 circulant cross-section (16 < n1 <= 32,
// 8 < n2 <= 16; the paper's 500 x 200 nm strip at h = 50/3 nm is 30 x 12): per
// kz plane, zero-padded 2-D FFT of the three current components, the 3x3
// symmetric product with the Green spectrum, inverse 2-D FFT and crop (Section
// III-A: N is block Toeplitz, its product a circular convolution).
//
// One plane per workgroup of 256 threads, every transform in registers:
//  A: the 3 n2 forward x transforms (64 points, inputs x < 32) by groups of 8
//     lanes, each a radix-8 x 8 four-step DFT: lane a holds x[a + 8 b], 8-point
//     DFT over b, twiddle W64^(a k), 8 x 8 transpose across the group through
//     LDS, 8-point DFT; lane a then holds X[a + 8 m].  Group q takes row q of
//     component 0 and 2 (q < 16) or row q - 16 of component 1, and the row's own
//     64-value slot of the hand-off buffer serves as its exchange area.
//  B: the 64 columns (kx) by groups of 4 lanes, all three components: 32-point
//     DFT as 8-point DFT over b of y = a + 4 b (inputs y < 16), twiddle
//     W32^(a k1), 4 x 8 exchange through the group's own 32-value area, 4-point
//     DFT over a, giving Y[k1 + 8 k2] with k1 in {2 a', 2 a' + 1} on lane a';
//     the Green product; the inverse in the mirrored order, keeping y < 16.
//  C: the 3 n2 inverse x transforms as in A, crop to x < n1, store.
// LDS: the hand-off (3 x 16 rows of 64 x-frequencies) and, in variant 1, 64
// column exchange areas of 32 values (80 KiB in FP64, 40 KiB in FP32); variant 2
// exchanges in the column's own hand-off entries of components 0 and 1, free
// once the column is in registers (48 KiB, 24 KiB).
// The layouts (xy6432_maps.hpp) were chosen by enumerating the accesses of one
// LDS pass (256 bytes: 16 lanes of 16-byte or 32 lanes of 8-byte values), and
// the host check in maps_check.cpp repeats that enumeration: every access is
// free of bank conflicts except variant 1's column exchange in FP32 (two-way).
// Hand-off element
// (c, y, kx) at row (c, y), column kx ^ 10 (y & 3); column exchange element
// (a, k) of group g at ((k + (g & 3)) & 7) 4 + (a ^ ((k >> 1) & 3)) of its area
// (variant 1) or at hand-off entry (k & 1, 4 (k >> 1) + ((a + (k >> 1)) & 3), g)
// (variant 2: the four lanes of a group always differ in y & 3); row exchange
// element (i, j) of group q at (i ^ (q & 3)) 8 + ((i + j) & 7).
// Planes kz and M3 - kz use the same slab of the folded Green spectrum and go to
// workgroups b and b + 8 (same XCD).
#include <hip/hip_runtime.h>

#include "block_maps.hpp"
#include "fft_device.hpp"
#include "vie_internal.hpp"
#include "xy6432_maps.hpp"

namespace vie {

namespace {

constexpr int kHandVals = kXy32HandVals;
constexpr int kColX = kXy32ColX;
constexpr int kLdsVals = kHandVals + 64 * kColX;
constexpr int kThreads = 256;

__device__ __forceinline__ int hand(int c, int y, int kx) { return xy32_hand(c, y, kx); }

// 64-point DFT of a group of 8 lanes (lane a holds x[a + 8 b] in, X[a + 8 m] out);
// X is the group's 64-value exchange area.  The area belongs to one wave, whose LDS
// accesses complete in program order, so wave barriers order the exchange.
template <typename T, bool INV>
__device__ __forceinline__ void row64(cx<T>* v, const cx<T>* w, int a, cx<T>* X, int f) {
  dft8<T, INV>(v);
#pragma unroll
  for (int k = 1; k < 8; ++k) v[k] = INV ? cmulc(v[k], w[k]) : cmul(v[k], w[k]);
#pragma unroll
  for (int k = 0; k < 8; ++k) X[xy32_rowx(k, a, f)] = v[k];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = X[xy32_rowx(a, j, f)];
  __builtin_amdgcn_wave_barrier();
  dft8<T, INV>(v);
}

// The value as the compiler must materialise it here: without this, parts of the
// Green product were carried into the inverse transforms as separate terms, which
// raised the register need of the column stage by about half.
template <typename T>
__device__ __forceinline__ void pin(cx<T>& v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y));
}


template <typename T, bool COMPACT>
__device__ __forceinline__ void xy6432_plane(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
                                             const cx<T>* __restrict__ tw64, const cx<T>* __restrict__ tw32, int kz,
                                             cx<T>* R) {
  const int n1 = g.n1, n2 = g.n2;
  const cx<T> zero{(T)0, (T)0};
  cx<T>* P = U + (long)kz * 3 * n1 * n2;

  // ---------------- A: forward x transforms
  // (each stage takes a fresh opaque thread index, so that its per-lane LDS
  // address terms are computed where they are used instead of all at the start)
  {
    const int t = opaque_tid();
    const int a = t & 7, q = t >> 3;
    cx<T> w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = tw64[a * k];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (i == 1 && q >= 16) break;
      int c, y;
      xy32_row_task(q, i, &c, &y);
      if (y >= n2) continue;
      cx<T> v[8];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int x = a + 8 * b;
        v[b] = x < n1 ? P[(c * n2 + y) * n1 + x] : zero;
      }
#pragma unroll
      for (int b = 4; b < 8; ++b) v[b] = zero;
      row64<T, false>(v, w, a, R + (c * 16 + y) * 64, q & 3);
#pragma unroll
      for (int m = 0; m < 8; ++m) R[hand(c, y, a + 8 * m)] = v[m];
    }
  }
  __syncthreads();

  // ---------------- B: columns kx = group, forward, Green product, inverse
  {
    const int t = opaque_tid();
    const int a = t & 3, kx = t >> 2, r = kx & 3;
    // exchange element (aa, k) of this column: its own area, or (COMPACT) a slot of
    // the column's own hand-off entries, free once the column is in registers
    auto xs = [&](int aa, int k) -> int {
      if (COMPACT) return xy32_cslot(aa, k, kx);
      return kHandVals + kx * kColX + xy32_colx(aa, k, r);
    };
    cx<T> v[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int y = a + 4 * b;
        v[c][b] = y < n2 ? R[hand(c, y, kx)] : zero;
      }
#pragma unroll
      for (int b = 4; b < 8; ++b) v[c][b] = zero;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dft8<T, false>(v[c]);                                  // Z[a][k1]
#pragma unroll
      for (int k = 1; k < 8; ++k) v[c][k] = cmul(v[c][k], tw32[a * k]);
#pragma unroll
      for (int k = 0; k < 8; ++k) R[xs(a, k)] = v[c][k];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int s = 0; s < 4; ++s) v[c][e * 4 + s] = R[xs(s, 2 * a + e)];
      __builtin_amdgcn_wave_barrier();
      dft4<T, false>(v[c]);                                  // v[e 4 + m] = Y[2 a + e + 8 m]
      dft4<T, false>(v[c] + 4);
      // components one after the other: interleaving their transforms runs the
      // kernel out of registers
      __builtin_amdgcn_sched_barrier(0);
    }
    // Green product at (kx, ky), spectrum folded to the stored octant
    const int k3 = kz <= g.M3 / 2 ? kz : g.M3 - kz;
    const T s3 = kz <= g.M3 / 2 ? (T)1 : (T)-1;
    const int k1 = kx <= 32 ? kx : 64 - kx;
    const T s1 = kx <= 32 ? (T)1 : (T)-1;
    const cx<T>* G3 = goct + ((long)k3 * g.H2 * g.H1 + k1) * 6;
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int ky = 2 * a + e + 8 * m;
        const int k2 = ky <= 16 ? ky : 32 - ky;
        const T s2 = ky <= 16 ? (T)1 : (T)-1;
        const cx<T>* Gp = G3 + (long)k2 * g.H1 * 6;
        const cx<T> gxx = Gp[0], gyy = Gp[3], gzz = Gp[5];
        const cx<T> gxy = cscale(Gp[1], s1 * s2), gxz = cscale(Gp[2], s1 * s3), gyz = cscale(Gp[4], s2 * s3);
        const int i = e * 4 + m;
        const cx<T> ux = v[0][i], uy = v[1][i], uz = v[2][i];
        v[0][i] = cadd(cadd(cmul(gxx, ux), cmul(gxy, uy)), cmul(gxz, uz));
        v[1][i] = cadd(cadd(cmul(gxy, ux), cmul(gyy, uy)), cmul(gyz, uz));
        v[2][i] = cadd(cadd(cmul(gxz, ux), cmul(gyz, uy)), cmul(gzz, uz));
        pin<T>(v[0][i]);
        pin<T>(v[1][i]);
        pin<T>(v[2][i]);
        // one point's spectrum loads in flight at a time: hoisting all eight
        // points' loads (48 values) ran the kernel out of registers
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dft4<T, true>(v[c]);                                   // v[e 4 + s] = T[k1 = 2 a + e][s]
      dft4<T, true>(v[c] + 4);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k1v = 2 * a + e;
          R[xs(s, k1v)] = s == 0 ? v[c][e * 4] : cmulc(v[c][e * 4 + s], tw32[s * k1v]);
        }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int k = 0; k < 8; ++k) v[c][k] = R[xs(a, k)];
      __builtin_amdgcn_wave_barrier();
      dft8<T, true>(v[c]);                                   // v[b] = column value at y = a + 4 b
      __builtin_amdgcn_sched_barrier(0);
    }
    // stored after all three inverse transforms: the compact exchange reuses the
    // column's entries of components 0 and 1
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int y = a + 4 * b;
        if (y < n2) R[hand(c, y, kx)] = v[c][b];
      }
  }
  __syncthreads();

  // ---------------- C: inverse x transforms, crop, store
  {
    const int t = opaque_tid();
    const int a = t & 7, q = t >> 3;
    cx<T> w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = tw64[a * k];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (i == 1 && q >= 16) break;
      int c, y;
      xy32_row_task(q, i, &c, &y);
      if (y >= n2) continue;
      cx<T> v[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) v[m] = R[hand(c, y, a + 8 * m)];
      row64<T, true>(v, w, a, R + (c * 16 + y) * 64, q & 3);   // v[b] = row value at x = a + 8 b
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int x = a + 8 * b;
        if (x < n1) P[(c * n2 + y) * n1 + x] = v[b];
      }
    }
  }
}

// Variants: V = 1 gives every column group its own exchange area (80 KiB of LDS
// in FP64: two workgroups per CU; 40 KiB in FP32: four); V = 2 exchanges in the
// column's own hand-off entries (48 KiB in FP64: three workgroups per CU; 24 KiB
// in FP32: five, bounded by registers).  The launch bound holds the compiler to the
// registers of that many waves per SIMD.
template <typename T, int V> constexpr int kWaves = sizeof(T) == 8 ? (V == 1 ? 2 : 3) : (V == 1 ? 4 : 5);
template <int V> constexpr int kLdsOf = V == 1 ? kLdsVals : kHandVals;

template <typename T, int V>
__global__ __launch_bounds__(kThreads, (kWaves<T, V>)) void k_xy6432(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, Geom g,
                                                     const cx<T>* __restrict__ tw64, const cx<T>* __restrict__ tw32) {
  extern __shared__ unsigned char smem_raw[];
  xy6432_plane<T, V == 2>(U, goct, g, tw64, tw32, paired_plane(blockIdx.x, g.M3),
                          reinterpret_cast<cx<T>*>(smem_raw));
}

}  // namespace

template <typename T>
hipError_t launch_xy6432(const Geom& g, int V, void* U, const void* goct, const void* tw1, const void* tw2,
                         hipStream_t s) {
  if (g.M1 != 64 || g.M2 != 32 || g.n1 > 32 || g.n2 > 16 || (V != 1 && V != 2)) return hipErrorInvalidValue;
  if (V == 1)
    hipLaunchKernelGGL((k_xy6432<T, 1>), dim3(g.M3), dim3(kThreads), kLdsOf<1> * sizeof(cx<T>), s, (cx<T>*)U,
                       (const cx<T>*)goct, g, (const cx<T>*)tw1, (const cx<T>*)tw2);
  else
    hipLaunchKernelGGL((k_xy6432<T, 2>), dim3(g.M3), dim3(kThreads), kLdsOf<2> * sizeof(cx<T>), s, (cx<T>*)U,
                       (const cx<T>*)goct, g, (const cx<T>*)tw1, (const cx<T>*)tw2);
  return hipGetLastError();
}

template <typename T>
hipError_t allow_lds_xy6432() {
  const auto attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipFuncSetAttribute((const void*)k_xy6432<T, 1>, attr, (int)(kLdsOf<1> * sizeof(cx<T>)));
  return e ? e : hipFuncSetAttribute((const void*)k_xy6432<T, 2>, attr, (int)(kLdsOf<2> * sizeof(cx<T>)));
}

template hipError_t launch_xy6432<double>(const Geom&, int, void*, const void*, const void*, const void*,
                                          hipStream_t);
template hipError_t launch_xy6432<float>(const Geom&, int, void*, const void*, const void*, const void*,
                                         hipStream_t);
template hipError_t allow_lds_xy6432<double>();
template hipError_t allow_lds_xy6432<float>();

}  // namespace vie
