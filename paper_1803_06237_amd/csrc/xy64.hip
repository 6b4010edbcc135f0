// Pass 2 of the matvec for the 64 x 64 circulant cross-section (16 < n1, n2 <= 32):
// per kz plane, zero-padded 2-D FFT of the three current components, the 3x3
// symmetric product with the Green spectrum, inverse 2-D FFT and crop
// (Section III-A: N is block Toeplitz, its product a circular convolution).
//
// Each 64-point transform is a four-step radix-8 x 8 DFT done in registers:
// thread "a" (a = lane & 7) of an 8-thread group holds x[a + 8 b] (b = 0..7),
// takes an 8-point DFT over b, twiddles by W64^(a k), and one LDS exchange
// hands thread k the values k of all eight threads for the second 8-point DFT.
// Inputs are only 32 long (the upper half is the zero padding) and only the
// first 32 outputs of each inverse transform are kept (the crop).
//
// Stage A: rows (x) forward, thread (y, a), all 3 components.
// Stage B: columns (y) forward, Green product, columns inverse; thread (kx, a),
//          processed in two halves of kx so that the exchange of one half
//          (3 components x 32 columns x 64) fits where the rows were kept.
// Stage C: rows inverse, crop, store.
// Planes kz and M3 - kz use the same slab of the folded Green spectrum: the
// single-system kernel puts them on workgroups b and b + 8 (same XCD), the
// batched kernel transforms the pair in one workgroup.
// LDS: one region of 3 x 32 x 64 complex values (96 KiB FP64, 48 KiB FP32),
// element (c, y, kx) at (c*32 + y)*64 + (kx ^ (y & 7)) so the column accesses
// of 8 threads with consecutive y hit distinct banks.
#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "vie_internal.hpp"

namespace vie {

namespace {

template <typename T>
__device__ __forceinline__ int rpos(int c, int y, int kx) {
  return (c * 32 + y) * 64 + (kx ^ (y & 7));
}

// 8 x 8 exchange block for group g (64 complex values), element (i, j) stored
// rotated so 8 threads reading row i with j = 0..7 touch distinct banks.
__device__ __forceinline__ int xpos(int g, int i, int j) { return g * 64 + i * 8 + ((i + j) & 7); }

template <typename T, bool INV>
__device__ __forceinline__ void twiddle8(cx<T>* v, const cx<T>* w) {
#pragma unroll
  for (int k = 1; k < 8; ++k) v[k] = INV ? cmulc(v[k], w[k]) : cmul(v[k], w[k]);
}

}  // namespace

template <typename T>
__device__ __forceinline__ void xy64_planes(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
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
      for (int k = 0; k < 8; ++k) R[xpos(c * 32 + y, k, a)] = v[c][k];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[xpos(c * 32 + y, a, j)];
      dft8<T, false>(v[c]);    // v[c][m] = X[kx = a + 8 m]
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 8; ++m) R[rpos<T>(c, y, a + 8 * m)] = v[c][m];
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
      for (int b = 0; b < 4; ++b) in[h][c][b] = R[rpos<T>(c, a + 8 * b, kx)];
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
      for (int k = 0; k < 8; ++k) R[xpos(c * 32 + q, k, a)] = v[c][k];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[xpos(c * 32 + q, a, j)];
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
      for (int k = 0; k < 8; ++k) R[xpos(c * 32 + q, k, a)] = v[c][k];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[xpos(c * 32 + q, a, j)];
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
      for (int b = 0; b < 4; ++b) R[rpos<T>(c, a + 8 * b, kx)] = out[h][c][b];
  }
  __syncthreads();

  // ---------------- stage C: inverse FFT along x for row y = q, crop, store
  {
    const int y = q;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int m = 0; m < 8; ++m) v[c][m] = R[rpos<T>(c, y, a + 8 * m)];
      dft8<T, true>(v[c]);
      twiddle8<T, true>(v[c], w);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 8; ++k) R[xpos(c * 32 + y, k, a)] = v[c][k];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[c][j] = R[xpos(c * 32 + y, a, j)];
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

// plane pair p: (0, M3/2) for p = 0, (p, M3 - p) otherwise
__device__ __forceinline__ void pair_planes(int p, int M3, int* a, int* b) {
  *a = p == 0 ? 0 : p;
  *b = p == 0 ? M3 / 2 : M3 - p;
}

template <typename T>
__device__ __forceinline__ void xy64_body(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, const Geom& g,
                                          const cx<T>* __restrict__ tw64, int pair, cx<T>* R) {
  int a, b;
  pair_planes(pair, g.M3, &a, &b);
  xy64_planes<T>(U, goct, g, tw64, a, g.M3 == 1 ? 1 : 2, b, R);
}

// One plane per workgroup.  The two planes of a pair read the same spectrum
// slab; they go to workgroups b and b + 8 (same XCD under round-robin
// dispatch, launched one after the other) so the second read hits L2.
template <typename T>
__global__ __launch_bounds__(256) void k_xy64(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, Geom g,
                                              const cx<T>* __restrict__ tw64) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int base = (b / 16) * 16, r = b - base;
  int pa, pb;
  pair_planes(base / 2 + (r % 8), g.M3, &pa, &pb);
  xy64_planes<T>(U, goct, g, tw64, r < 8 ? pa : pb, 1, 0, reinterpret_cast<cx<T>*>(smem_raw));
}

template <typename T>
__global__ __launch_bounds__(256) void k_xy64_batch(const PassDesc* __restrict__ d, const int* __restrict__ prefix,
                                                    int nsys, int total) {
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
    xy64_body<T>((cx<T>*)D.U, (const cx<T>*)D.goct, D.g, (const cx<T>*)D.twx, item - prefix[lo], R);
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_xy64_batch_single(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct,
                                                           Geom g, const cx<T>* __restrict__ tw64) {
  extern __shared__ unsigned char smem_raw[];
  xy64_body<T>(U, goct, g, tw64, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

template <typename T>
hipError_t launch_xy64_batch(const PassDesc* d, const int* prefix, int nsys, int total, hipStream_t s) {
  const size_t lds = (size_t)3 * 32 * 64 * sizeof(cx<T>);
  hipLaunchKernelGGL((k_xy64_batch<T>), dim3(total < 4096 ? total : 4096), dim3(256), lds, s, d, prefix, nsys,
                     total);
  return hipGetLastError();
}
template hipError_t launch_xy64_batch<double>(const PassDesc*, const int*, int, int, hipStream_t);
template hipError_t launch_xy64_batch<float>(const PassDesc*, const int*, int, int, hipStream_t);

template <typename T>
hipError_t launch_xy64(const Geom& g, void* U, const void* goct, const void* tw1, hipStream_t s) {
  const size_t lds = (size_t)3 * 32 * 64 * sizeof(cx<T>);
  if (g.M3 % 16 != 0) {   // short z circulant: one workgroup per plane pair
    hipLaunchKernelGGL((k_xy64_batch_single<T>), dim3(g.M3 == 1 ? 1 : g.M3 / 2), dim3(256), lds, s, (cx<T>*)U,
                       (const cx<T>*)goct, g, (const cx<T>*)tw1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_xy64<T>), dim3(g.M3), dim3(256), lds, s, (cx<T>*)U, (const cx<T>*)goct, g,
                     (const cx<T>*)tw1);
  return hipGetLastError();
}

template <typename T>
hipError_t allow_lds_xy64() {
  hipError_t e = hipFuncSetAttribute((const void*)k_xy64<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)((size_t)3 * 32 * 64 * sizeof(cx<T>)));
  if (e) return e;
  e = hipFuncSetAttribute((const void*)k_xy64_batch_single<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)((size_t)3 * 32 * 64 * sizeof(cx<T>)));
  if (e) return e;
  return hipFuncSetAttribute((const void*)k_xy64_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)((size_t)3 * 32 * 64 * sizeof(cx<T>)));
}

template hipError_t launch_xy64<double>(const Geom&, void*, const void*, const void*, hipStream_t);
template hipError_t launch_xy64<float>(const Geom&, void*, const void*, const void*, hipStream_t);
template hipError_t allow_lds_xy64<double>();
template hipError_t allow_lds_xy64<float>();

}  // namespace vie
