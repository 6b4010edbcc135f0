// Pass 2 of the matvec for the 64 x 64 circulant cross-section (16 < n1, n2 <= 32):
// per kz plane, zero-padded 2-D FFT of the three current components, the 3x3
// symmetric product with the Green spectrum, inverse 2-D FFT and crop
// (Section III-A: N is block Toeplitz, its product a circular convolution).
//
// Each 64-point transform is a four-step radix-8 x 8 DFT done in registers by
// a group of 8 lanes: lane a holds x[a + 8 b] (b = 0..7), takes an 8-point DFT
// over b, twiddles by W64^(a k), and an 8 x 8 transpose across the group's
// lanes through LDS hands lane k the values k of all eight lanes for the second
// 8-point DFT; lane a then holds X[a + 8 m].
// Inputs are only 32 long (the upper half is the zero padding) and only the
// first 32 outputs of each inverse transform are kept (the crop).
//
// Two variants, picked per grid and precision by timing at plan time:
//  V = 0 (full plane): the rows of all 64 x-frequencies of the three components
//   stay in LDS (3 x 32 x 64 values, 96 KiB FP64) and the same region serves the
//   8 x 8 exchanges between workgroup barriers: rows forward; columns forward,
//   Green product and inverse in two halves of kx; rows inverse, crop, store.
//  V = 1 (x-frequency halves): the 64 x-frequencies are processed in two halves
//   (|kx| <= 16 and |kx| >= 16 after folding, so each half reads its own part of
//   the spectrum slab) so that the row-to-column hand-off needs 3 x 32 x 32
//   values of LDS, and each
//   group of 8 lanes exchanges through its own 64-value LDS area without
//   workgroup barriers (80 KiB FP64 in all, two workgroups per CU):
//   A_h: rows (x) forward for row y = group, all 3 components; the 32
//        frequencies of half h go to LDS;
//   B_h: columns (y) forward, Green product, columns inverse for one column
//        of the half per group, in place in LDS;
//   C_h: rows inverse from the 32 frequencies of half h (the rest taken as
//        zero); half 0 parks its partial row in the plane's own storage (after
//        reading the row input again for A_1) and half 1 adds to it.
//  V = 2 (wide): 512 threads (64 groups, two waves per SIMD) and the whole
//   160 KiB of LDS in FP64: the rows of all 64 x-frequencies of the three
//   components (96 KiB) plus a private 64-value exchange area per group, so no
//   row transform is done twice and no partial row leaves the CU:
//   A: the 96 forward row transforms (32 rows x 3 components) over the 64
//      groups (groups g < 32 take components 0 and 2 of row g, the others
//      component 1 of row g - 32);
//   B: one column (kx = g) per group: forward, Green product, inverse;
//   C: the 96 inverse row transforms as in A, crop, store.
// Planes kz and M3 - kz use the same slab of the folded Green spectrum: the
// single-system kernel puts them on workgroups b and b + 8 (same XCD), the
// batched kernel transforms the pair in one workgroup.
// LDS layouts avoid bank conflicts.  The LDS serves a wave in passes of 256 bytes
// (16 lanes of 16-byte values in FP64, 32 lanes of 8-byte values in FP32), so
// the 2 or 4 lane groups of a pass must use disjoint banks as well as the 8
// lanes of a group: hand-off element (c, y, j) sits in row (c, y) at column
// j ^ (y & 7) ^ 8 (y & 3), and the exchange area of group q stores its row i in
// slot i ^ (q & 3), rotated by i.
#include <hip/hip_runtime.h>

#include "block_maps.hpp"
#include "fft_device.hpp"
#include "vie_internal.hpp"

namespace vie {

namespace {

__device__ __forceinline__ int hpos(int c, int y, int j) {
  return (c * 32 + y) * 32 + (j ^ (y & 7) ^ ((y & 3) << 3));
}

constexpr int kRowVals = 3 * 32 * 32;               // row/column hand-off of one half
constexpr int kXyLdsVals = kRowVals + 32 * 64;      // + 32 groups x 64 exchange values
constexpr int kFullLdsVals = 3 * 32 * 64;           // full-plane variant: rows of all 64 frequencies
constexpr int kWideLdsVals = kFullLdsVals + 64 * 64; // wide variant: + 64 groups x 64 exchange values
// x-frequency halves of the V = 1 variant, as the m of kx = a + 8 m (a = lane):
// half 0 = m in {0, 1, 6, 7} (kx < 16 or kx >= 48, folded |kx| <= 16), half 1 =
// m in {2, 3, 4, 5} (16 <= kx < 48, folded |kx| >= 16), so that the two halves
// read disjoint parts of the folded spectrum slab.
__constant__ constexpr int kHalf0[4] = {0, 1, 6, 7};

// full-plane variant: element (c, y, kx) of the row buffer, and the 8 x 8 exchange
// block of group gr (64 values) with element (i, j) rotated as in xpos
__device__ __forceinline__ int rpos(int c, int y, int kx) {
  return (c * 32 + y) * 64 + (kx ^ (y & 7) ^ ((y & 3) << 3));
}
__device__ __forceinline__ int gpos(int gr, int i, int j) { return gr * 64 + (i ^ (gr & 3)) * 8 + ((i + j) & 7); }

template <typename T, bool INV>
__device__ __forceinline__ void twiddle8(cx<T>* v, const cx<T>* w) {
#pragma unroll
  for (int k = 1; k < 8; ++k) v[k] = INV ? cmulc(v[k], w[k]) : cmul(v[k], w[k]);
}

// Exchange area of one group of 8 lanes (64 values): element (i, j) stored in
// slot i ^ f (f = group & 3) and rotated by i, so that the lanes of a group and
// the groups of an LDS pass touch distinct banks.
__device__ __forceinline__ int xpos(int i, int j, int f) { return (i ^ f) * 8 + ((i + j) & 7); }

// 8 x 8 transpose across the 8 lanes of a group through the group's own 64-value
// LDS area X: lane a's v[k] becomes lane k's v[a].  The area belongs to one wave,
// whose LDS accesses complete in program order, so no workgroup barrier is needed.
template <typename T>
__device__ __forceinline__ void transpose8(cx<T>* v, int a, cx<T>* X, int f) {
#pragma unroll
  for (int k = 0; k < 8; ++k) X[xpos(k, a, f)] = v[k];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = X[xpos(a, j, f)];
  __builtin_amdgcn_wave_barrier();
}

// 64-point transform of the group: in, lane a holds x[a + 8 b]; out, lane a holds X[a + 8 m]
template <typename T, bool INV>
__device__ __forceinline__ void fft64(cx<T>* v, const cx<T>* w, int a, cx<T>* X, int f) {
  dft8<T, INV>(v);
  twiddle8<T, INV>(v, w);
  transpose8<T>(v, a, X, f);
  dft8<T, INV>(v);
}

}  // namespace

template <typename T>
__device__ __forceinline__ void xy64_full(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
                                            const cx<T>* __restrict__ tw64, int kz_first, int nplanes, int kz_second,
                                            cx<T>* R) {
  const int tid = threadIdx.x;
  const int a = tid & 7;
  const int q = tid >> 3;                            // 0..31
  const int n1 = g.n1, n2 = g.n2;
  // W64^(a k), k = 0..7
  cx<T> w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = tw64[a * k];
  for (int pi = 0; pi < nplanes; ++pi) {
  const int kz = pi == 0 ? kz_first : kz_second;
  cx<T>* P = U + (long)kz * 3 * n1 * n2;

  // ---------------- stage A: forward FFT along x for row y = q, all components
  cx<T> v[3][8];
  {
    const int y = q;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int x = a + 8 * b;
        v[c][b] = (x < n1 && y < n2) ? P[(c * n2 + y) * n1 + x] : cx<T>{(T)0, (T)0};
      }
#pragma unroll
      for (int b = 4; b < 8; ++b) v[c][b] = cx<T>{(T)0, (T)0};
      dft8<T, false>(v[c]);
      twiddle8<T, false>(v[c], w);
#pragma unroll
      for (int k = 0; k < 8; ++k) R[gpos(c * 32 + y, k, a)] = v[c][k];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[gpos(c * 32 + y, a, j)];
      dft8<T, false>(v[c]);    // v[c][m] = X[kx = a + 8 m]
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 8; ++m) R[rpos(c, y, a + 8 * m)] = v[c][m];
    __syncthreads();
  }

  // ---------------- stage B: columns; task (kx = q + 32 h, a) for half h
  cx<T> in[2][3][4];     // column inputs y = a + 8 b, b < 4
  cx<T> out[2][3][4];    // column outputs y = a + 8 b, b < 4
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int kx = q + 32 * h;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 4; ++b) in[h][c][b] = R[rpos(c, a + 8 * b, kx)];
  }
  __syncthreads();
  const int k3 = kz <= g.M3 / 2 ? kz : g.M3 - kz;
  const T s3 = kz <= g.M3 / 2 ? (T)1 : (T)-1;
  const cx<T>* G3 = goct + (long)k3 * g.H2 * g.H1 * 6;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int kx = q + 32 * h;
    // forward: DFT over b, twiddle, exchange (group = (c, q)), DFT over a
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int b = 0; b < 4; ++b) v[c][b] = in[h][c][b];
#pragma unroll
      for (int b = 4; b < 8; ++b) v[c][b] = cx<T>{(T)0, (T)0};
      dft8<T, false>(v[c]);
      twiddle8<T, false>(v[c], w);
#pragma unroll
      for (int k = 0; k < 8; ++k) R[gpos(c * 32 + q, k, a)] = v[c][k];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[gpos(c * 32 + q, a, j)];
      dft8<T, false>(v[c]);    // v[c][m] = Y[ky = a + 8 m]
    }
    // Green product at (kx, ky), spectrum folded to the stored octant
    const int k1 = kx <= 32 ? kx : 64 - kx;
    const T s1 = kx <= 32 ? (T)1 : (T)-1;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int ky = a + 8 * m;
      const int k2 = ky <= 32 ? ky : 64 - ky;
      const T s2 = ky <= 32 ? (T)1 : (T)-1;
      const cx<T>* Gp = G3 + ((long)k2 * g.H1 + k1) * 6;
      const cx<T> gxx = Gp[0], gyy = Gp[3], gzz = Gp[5];
      const cx<T> gxy = cscale(Gp[1], s1 * s2), gxz = cscale(Gp[2], s1 * s3), gyz = cscale(Gp[4], s2 * s3);
      const cx<T> ux = v[0][m], uy = v[1][m], uz = v[2][m];
      v[0][m] = cadd(cadd(cmul(gxx, ux), cmul(gxy, uy)), cmul(gxz, uz));
      v[1][m] = cadd(cadd(cmul(gxy, ux), cmul(gyy, uy)), cmul(gyz, uz));
      v[2][m] = cadd(cadd(cmul(gxz, ux), cmul(gyz, uy)), cmul(gzz, uz));
    }
    // inverse: thread holds Y[a + 8 m]; DFT over m, twiddle conj, exchange, DFT over a
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dft8<T, true>(v[c]);
      twiddle8<T, true>(v[c], w);
#pragma unroll
      for (int k = 0; k < 8; ++k) R[gpos(c * 32 + q, k, a)] = v[c][k];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[gpos(c * 32 + q, a, j)];
      dft8<T, true>(v[c]);     // v[c][b] = column value at y = a + 8 b
#pragma unroll
      for (int b = 0; b < 4; ++b) out[h][c][b] = v[c][b];
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int kx = q + 32 * h;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 4; ++b) R[rpos(c, a + 8 * b, kx)] = out[h][c][b];
  }
  __syncthreads();

  // ---------------- stage C: inverse FFT along x for row y = q, crop, store
  {
    const int y = q;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int m = 0; m < 8; ++m) v[c][m] = R[rpos(c, y, a + 8 * m)];
      dft8<T, true>(v[c]);
      twiddle8<T, true>(v[c], w);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 8; ++k) R[gpos(c * 32 + y, k, a)] = v[c][k];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[gpos(c * 32 + y, a, j)];
      dft8<T, true>(v[c]);     // v[c][b] = row value at x = a + 8 b
      if (y < n2) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int x = a + 8 * b;
          if (x < n1) P[(c * n2 + y) * n1 + x] = v[c][b];
        }
      }
    }
  }
  __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ void xy64_half(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
                                          const cx<T>* __restrict__ tw64, int kz_first, int nplanes, int kz_second,
                                          cx<T>* R) {
  const int tid = threadIdx.x;
  const int a = tid & 7;
  const int q = tid >> 3;                            // group: row y in A and C, column in B
  const int n1 = g.n1, n2 = g.n2;
  cx<T>* X = R + kRowVals + q * 64;                  // this group's exchange area
  const int f = q & 3;
  cx<T> w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = tw64[a * k];
  const cx<T> zero{(T)0, (T)0};
  for (int pi = 0; pi < nplanes; ++pi) {
    const int kz = pi == 0 ? kz_first : kz_second;
    cx<T>* P = U + (long)kz * 3 * n1 * n2;
    const int k3 = kz <= g.M3 / 2 ? kz : g.M3 - kz;
    const T s3 = kz <= g.M3 / 2 ? (T)1 : (T)-1;
    const cx<T>* G3 = goct + (long)k3 * g.H2 * g.H1 * 6;
    const int y = q;
    const bool row_ok = y < n2;
    cx<T> in[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int x = a + 8 * b;
        in[c][b] = (x < n1 && row_ok) ? P[(c * n2 + y) * n1 + x] : zero;
      }
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      const bool first = h == 0;
      // ---- A_h: forward x transform of row y, frequencies of half h to LDS
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<T> v[8];
#pragma unroll
        for (int b = 0; b < 4; ++b) v[b] = in[c][b];
#pragma unroll
        for (int b = 4; b < 8; ++b) v[b] = zero;
        fft64<T, false>(v, w, a, X, f);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const cx<T> h0 = v[kHalf0[j]], h1 = v[j + 2];
          R[hpos(c, y, a + 8 * j)] = cx<T>{first ? h0.x : h1.x, first ? h0.y : h1.y};
        }
      }
      __syncthreads();
      // ---- B_h: LDS column q = a' + 8 j holds kx = a' + 8 m with m the j-th of the half
      {
        const int jq = q >> 3;
        const int kx = (q & 7) + 8 * (first ? (jq < 2 ? jq : jq + 4) : jq + 2);
        cx<T> v[3][8];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
          for (int b = 0; b < 4; ++b) v[c][b] = R[hpos(c, a + 8 * b, q)];
#pragma unroll
          for (int b = 4; b < 8; ++b) v[c][b] = zero;
          fft64<T, false>(v[c], w, a, X, f);  // v[c][m] = Y[ky = a + 8 m]
        }
        const int k1 = kx <= 32 ? kx : 64 - kx;
        const T s1 = kx <= 32 ? (T)1 : (T)-1;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int ky = a + 8 * m;
          const int k2 = ky <= 32 ? ky : 64 - ky;
          const T s2 = ky <= 32 ? (T)1 : (T)-1;
          const cx<T>* Gp = G3 + ((long)k2 * g.H1 + k1) * 6;
          const cx<T> gxx = Gp[0], gyy = Gp[3], gzz = Gp[5];
          const cx<T> gxy = cscale(Gp[1], s1 * s2), gxz = cscale(Gp[2], s1 * s3), gyz = cscale(Gp[4], s2 * s3);
          const cx<T> ux = v[0][m], uy = v[1][m], uz = v[2][m];
          v[0][m] = cadd(cadd(cmul(gxx, ux), cmul(gxy, uy)), cmul(gxz, uz));
          v[1][m] = cadd(cadd(cmul(gxy, ux), cmul(gyy, uy)), cmul(gyz, uz));
          v[2][m] = cadd(cadd(cmul(gxz, ux), cmul(gyz, uy)), cmul(gzz, uz));
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          fft64<T, true>(v[c], w, a, X, f);   // v[c][b] = column value at y = a + 8 b
#pragma unroll
          for (int b = 0; b < 4; ++b) R[hpos(c, a + 8 * b, q)] = v[c][b];
        }
      }
      __syncthreads();
      // ---- C_h: inverse x transform of row y from the frequencies of half h.  The
      // row's input is read again first (for A_1; unconditional, so that in[] is not
      // carried across the column stage), then half 0 parks its partial result in
      // the row's place and half 1 adds to it.
      // (in half 1 the same loads bring the parked partial rows, all 12 at once)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int x = a + 8 * b;
          in[c][b] = (x < n1 && row_ok) ? P[(c * n2 + y) * n1 + x] : zero;
        }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<T> v[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const cx<T> t = R[hpos(c, y, a + 8 * j)];
          const cx<T> in0{first ? t.x : (T)0, first ? t.y : (T)0};
          const cx<T> in1{first ? (T)0 : t.x, first ? (T)0 : t.y};
          v[kHalf0[j]] = in0;
          v[j + 2] = in1;
        }
        fft64<T, true>(v, w, a, X, f);        // v[b] = row value at x = a + 8 b
        if (row_ok) {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int x = a + 8 * b;
            if (x < n1) P[(c * n2 + y) * n1 + x] = first ? v[b] : cadd(in[c][b], v[b]);
          }
        }
      }
      __syncthreads();
    }
  }
}


// Inputs of the two row tasks of group q for plane P (zero outside the grid),
// from clamped, always valid addresses: no branches, one memory latency.
template <typename T>
__device__ __forceinline__ void wide_load_rows(const cx<T>* P, int q, int a, int n1, int n2, cx<T> (&in)[2][4]) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int ft = q + 64 * t < 96 ? q + 64 * t : q;
    const int c = ft >> 5, y = ft & 31;
    const int yc = y < n2 ? y : n2 - 1;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int x = a + 8 * b;
      const cx<T> v = P[(c * n2 + yc) * n1 + (x < n1 ? x : n1 - 1)];
      const bool ok = x < n1 && y < n2;
      in[t][b] = cx<T>{ok ? v.x : (T)0, ok ? v.y : (T)0};
    }
  }
}

// Green values of column kx (folded index k1) at ky = a + 8 m: the six entries
// of the folded octant
template <typename T>
__device__ __forceinline__ void wide_load_green(const cx<T>* G3, const Geom& g, int k1, int a, int m, cx<T>* out) {
  const int ky = a + 8 * m;
  const int k2 = ky <= 32 ? ky : 64 - ky;
  const cx<T>* Gp = G3 + ((long)k2 * g.H1 + k1) * 6;
#pragma unroll
  for (int e = 0; e < 6; ++e) out[e] = Gp[e];
}

template <typename T>
__device__ __forceinline__ void xy64_wide(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
                                          const cx<T>* __restrict__ tw64, int kz_first, int nplanes, int kz_second,
                                          cx<T>* R) {
  const int n1 = g.n1, n2 = g.n2;
  cx<T> w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = tw64[(threadIdx.x & 7) * k];
  const cx<T> zero{(T)0, (T)0};
  for (int pi = 0; pi < nplanes; ++pi) {
    // thread indices taken afresh per plane (see opaque_tid)
    const int tid = nplanes > 1 ? opaque_tid() : (int)threadIdx.x;
    const int a = tid & 7;
    const int q = tid >> 3;                          // 0..63
    const int f = q & 3;
    cx<T>* X = R + kFullLdsVals + q * 64;            // this group's exchange area
    const int kx = q;                                // column of stage B
    const int k1 = kx <= 32 ? kx : 64 - kx;
    const T s1 = kx <= 32 ? (T)1 : (T)-1;
    const int kz = pi == 0 ? kz_first : kz_second;
    cx<T>* P = U + (long)kz * 3 * n1 * n2;
    const int k3 = kz <= g.M3 / 2 ? kz : g.M3 - kz;
    const T s3 = kz <= g.M3 / 2 ? (T)1 : (T)-1;
    const cx<T>* G3 = goct + (long)k3 * g.H2 * g.H1 * 6;
    cx<T> in[2][4];
    wide_load_rows<T>(P, q, a, n1, n2, in);
    // ---- A: forward x transforms; row task ft = q + 64 t (t = 0, 1) is
    // (component ft / 32, row ft % 32) while ft < 96
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int ft = q + 64 * t;
      if (ft < 96) {
        const int c = ft >> 5, y = ft & 31;
        cx<T> v[8];
#pragma unroll
        for (int b = 0; b < 4; ++b) v[b] = in[t][b];
#pragma unroll
        for (int b = 4; b < 8; ++b) v[b] = zero;
        fft64<T, false>(v, w, a, X, f);           // v[m] = X[kx = a + 8 m]
#pragma unroll
        for (int m = 0; m < 8; ++m) R[rpos(c, y, a + 8 * m)] = v[m];
      }
    }
    __syncthreads();
    // ---- B: column kx = q of all three components.  The Green values of ky =
    // a + 8 m come through a ring of two batches: the first two are loaded
    // before the forward transforms, batch m + 2 as batch m is used.
    {
      constexpr int kRing = 2;
      cx<T> G[kRing][6];
#pragma unroll
      for (int m = 0; m < kRing; ++m) wide_load_green<T>(G3, g, k1, a, m, G[m]);
      cx<T> v[3][8];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int b = 0; b < 4; ++b) v[c][b] = R[rpos(c, a + 8 * b, kx)];
#pragma unroll
        for (int b = 4; b < 8; ++b) v[c][b] = zero;
        fft64<T, false>(v[c], w, a, X, f);        // v[c][m] = Y[ky = a + 8 m]
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int ky = a + 8 * m;
        const T s2 = ky <= 32 ? (T)1 : (T)-1;
        cx<T>* Gm = G[m % kRing];
        const cx<T> gxx = Gm[0], gyy = Gm[3], gzz = Gm[5];
        const cx<T> gxy = cscale(Gm[1], s1 * s2), gxz = cscale(Gm[2], s1 * s3), gyz = cscale(Gm[4], s2 * s3);
        const cx<T> ux = v[0][m], uy = v[1][m], uz = v[2][m];
        v[0][m] = cadd(cadd(cmul(gxx, ux), cmul(gxy, uy)), cmul(gxz, uz));
        v[1][m] = cadd(cadd(cmul(gxy, ux), cmul(gyy, uy)), cmul(gyz, uz));
        v[2][m] = cadd(cadd(cmul(gxz, ux), cmul(gyz, uy)), cmul(gzz, uz));
        if (m + kRing < 8) wide_load_green<T>(G3, g, k1, a, m + kRing, Gm);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fft64<T, true>(v[c], w, a, X, f);         // v[c][b] = column value at y = a + 8 b
#pragma unroll
        for (int b = 0; b < 4; ++b) R[rpos(c, a + 8 * b, kx)] = v[c][b];
      }
    }
    __syncthreads();
    // ---- C: inverse x transforms of the row tasks of A, crop, store
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int ft = q + 64 * t;
      if (ft < 96 && (ft & 31) < n2) {
        const int c = ft >> 5, y = ft & 31;
        cx<T> v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = R[rpos(c, y, a + 8 * m)];
        fft64<T, true>(v, w, a, X, f);            // v[b] = row value at x = a + 8 b
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int x = a + 8 * b;
          if (x < n1) P[(c * n2 + y) * n1 + x] = v[b];
        }
      }
    }
    __syncthreads();
  }
}

// V = 0: full-plane variant; V = 1: x-frequency halves; V = 2: wide
template <typename T, int V>
__device__ __forceinline__ void xy64_planes(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
                                            const cx<T>* __restrict__ tw64, int kz_first, int nplanes, int kz_second,
                                            cx<T>* R) {
  if constexpr (V == 0) xy64_full<T>(U, goct, g, tw64, kz_first, nplanes, kz_second, R);
  else if constexpr (V == 1) xy64_half<T>(U, goct, g, tw64, kz_first, nplanes, kz_second, R);
  else xy64_wide<T>(U, goct, g, tw64, kz_first, nplanes, kz_second, R);
}

// threads per workgroup and occupancy hint of each variant (waves per SIMD).  The
// wide variant in FP32 takes 80 KiB of LDS, so two workgroups fit a CU when the
// compiler keeps to 128 registers (it spills a few; measured 39.8 -> 37.2 us for
// the FP32 32x32x512 xy pass, 68 -> 64.5 us per FP32 product back to back).
template <int V> constexpr int kXyThreads = V == 2 ? 512 : 256;
template <typename T, int V> constexpr int kXyWaves = V == 1 ? 2 : (V == 2 && sizeof(T) == 4 ? 4 : 1);

template <typename T, int V>
__device__ __forceinline__ void xy64_body(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
                                          const cx<T>* __restrict__ tw64, int pair, cx<T>* R) {
  int a, b;
  pair_planes(pair, g.M3, &a, &b);
  xy64_planes<T, V>(U, goct, g, tw64, a, g.M3 == 1 ? 1 : 2, b, R);
}

// One plane per workgroup.  The two planes of a pair read the same spectrum
// slab; they go to workgroups b and b + 8 (same XCD under round-robin
// dispatch, launched one after the other) so the second read hits L2.
template <typename T, int V>
__global__ __launch_bounds__(kXyThreads<V>, (kXyWaves<T, V>)) void k_xy64(cx<T>* __restrict__ U,
                                                                    const cx<T>* __restrict__ goct, Geom g,
                                                                    const cx<T>* __restrict__ tw64) {
  extern __shared__ unsigned char smem_raw[];
  xy64_planes<T, V>(U, goct, g, tw64, paired_plane(blockIdx.x, g.M3), 1, 0, reinterpret_cast<cx<T>*>(smem_raw));
}

template <typename T, int V>
__global__ __launch_bounds__(256, V == 1 ? 2 : 1) void k_xy64_batch(const PassDesc* __restrict__ d,
                                                                    const int* __restrict__ prefix, int nsys,
                                                                    int total) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* R = reinterpret_cast<cx<T>*>(smem_raw);
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const PassDesc& D = d[lo];
    if (D.active && *D.active == 0) continue;
    xy64_body<T, V>((cx<T>*)D.U, (const cx<T>*)D.goct, D.g, (const cx<T>*)D.twx, item - prefix[lo], R);
    __syncthreads();
  }
}

template <typename T, int V>
__global__ __launch_bounds__(kXyThreads<V>, (kXyWaves<T, V>)) void k_xy64_batch_single(cx<T>* __restrict__ U,
                                                                                 const cx<T>* __restrict__ goct,
                                                                                 Geom g,
                                                                                 const cx<T>* __restrict__ tw64) {
  extern __shared__ unsigned char smem_raw[];
  xy64_body<T, V>(U, goct, g, tw64, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

template <typename T>
size_t xy64_lds(int V) {
  return (size_t)(V == 1 ? kXyLdsVals : V == 2 ? kWideLdsVals : kFullLdsVals) * sizeof(cx<T>);
}

// Variant of the batched kernel: x-frequency halves in FP64 (register-bound
// planes gain from two workgroups per CU), full plane in FP32.
template <typename T>
constexpr int kBatchVariant = sizeof(T) == 8 ? 1 : 0;

template <typename T>
hipError_t launch_xy64_batch(const PassDesc* d, const int* prefix, int nsys, int total, hipStream_t s) {
  constexpr int V = kBatchVariant<T>;
  hipLaunchKernelGGL((k_xy64_batch<T, V>), dim3(total < 4096 ? total : 4096), dim3(256), xy64_lds<T>(V), s, d,
                     prefix, nsys, total);
  return hipGetLastError();
}
template hipError_t launch_xy64_batch<double>(const PassDesc*, const int*, int, int, hipStream_t);
template hipError_t launch_xy64_batch<float>(const PassDesc*, const int*, int, int, hipStream_t);

template <typename T>
hipError_t launch_xy64(const Geom& g, int V, void* U, const void* goct, const void* tw1, hipStream_t s) {
  const size_t lds = xy64_lds<T>(V);
  const dim3 block(V == 2 ? kXyThreads<2> : kXyThreads<0>);
  if (g.M3 % 16 != 0) {   // short z circulant: one workgroup per plane pair
    const dim3 grid(g.M3 == 1 ? 1 : g.M3 / 2);
#define VIE_XYS(VV)                                                                                           \
  if (V == VV) {                                                                                              \
    hipLaunchKernelGGL((k_xy64_batch_single<T, VV>), grid, block, lds, s, (cx<T>*)U, (const cx<T>*)goct, g,   \
                       (const cx<T>*)tw1);                                                                    \
    return hipGetLastError();                                                                                 \
  }
    VIE_XYS(0)
    VIE_XYS(1)
    VIE_XYS(2)
#undef VIE_XYS
    return hipErrorInvalidValue;
  }
#define VIE_XY(VV)                                                                                            \
  if (V == VV) {                                                                                              \
    hipLaunchKernelGGL((k_xy64<T, VV>), dim3(g.M3), block, lds, s, (cx<T>*)U, (const cx<T>*)goct, g,          \
                       (const cx<T>*)tw1);                                                                    \
    return hipGetLastError();                                                                                 \
  }
  VIE_XY(0)
  VIE_XY(1)
  VIE_XY(2)
#undef VIE_XY
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t allow_lds_xy64() {
  const auto attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_xy64<T, 0>, attr, (int)xy64_lds<T>(0)))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_xy64<T, 1>, attr, (int)xy64_lds<T>(1)))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_xy64_batch_single<T, 0>, attr, (int)xy64_lds<T>(0)))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_xy64_batch_single<T, 1>, attr, (int)xy64_lds<T>(1)))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_xy64<T, 2>, attr, (int)xy64_lds<T>(2)))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_xy64_batch_single<T, 2>, attr, (int)xy64_lds<T>(2)))) return e;
  return hipFuncSetAttribute((const void*)k_xy64_batch<T, kBatchVariant<T>>, attr,
                             (int)xy64_lds<T>(kBatchVariant<T>));
}

template hipError_t launch_xy64<double>(const Geom&, int, void*, const void*, const void*, hipStream_t);
template hipError_t launch_xy64<float>(const Geom&, int, void*, const void*, const void*, hipStream_t);
template hipError_t allow_lds_xy64<double>();
template hipError_t allow_lds_xy64<float>();

}  // namespace vie
