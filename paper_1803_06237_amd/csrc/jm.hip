// The JM-VIE (Section III): the coupled product of electric and magnetic currents.
//
//   y = (I - M T~) x,   T~ = [[N, i kappa K], [-i kappa K, N]],
//
// x = (x_e, x_m) with six components, the magnetic unknowns in impedance units
// and exp(-i omega t); K = curl S is block Toeplitz like N, with three
// antisymmetric components (K^{ba} = -K^{ab}) odd along the axis other than a
// and b, so its spectrum is stored on one octant too.  The product reuses the
// z passes of the J-VIE once per half and adds three kernels over full
// cross-section spectra:
//   k_jm_xyfwd:   per (kz, component) plane: the n2 x n1 slice of the
//                 z-transformed intermediate, zero padded to M2 x M1, 2-D FFT
//                 in LDS, into S[component][kz][ky][kx]
//   k_jm_product: per spectral point: the 6 x 6 product with N^ and K^
//   k_jm_xyinv:   per plane: inverse 2-D FFT, crop to n2 x n1, back into U
// A plane is at most 64 x 64 values (n1, n2 <= 32), 64 KiB in FP64.
#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "vie_internal.hpp"

namespace vie {
namespace {

constexpr int kJmThreads = 256;
constexpr int kJmMaxV = 16;   // values per thread per FFT stage: 256 x 16 = 4096 = the largest plane

template <typename T>
__global__ __launch_bounds__(kJmThreads) void k_jm_xyfwd(const cx<T>* __restrict__ U, cx<T>* __restrict__ S, Geom g,
                                                          int c0, const cx<T>* __restrict__ tw1,
                                                          const cx<T>* __restrict__ tw2) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);     // [M2][M1]
  const int c = blockIdx.x % 3, kz = blockIdx.x / 3;
  const long plane = (long)g.n1 * g.n2;
  const cx<T>* src = U + ((long)kz * 3 + c) * plane;    // [i2][i1]
  // rows y < n2, columns x < n1; the transforms take every other slot as zero
  for (int t = threadIdx.x; t < g.n2 * g.n1; t += blockDim.x) {
    const int y = t / g.n1, x = t % g.n1;
    buf[y * g.M1 + x] = src[t];
  }
  __syncthreads();
  fft_lds<T, false, kJmMaxV>(buf, SeqMap{0, 0, g.M1, 1}, g.n2, g.L1, g.n1, tw1, 1);        // rows (x)
  fft_lds<T, false, kJmMaxV>(buf, SeqMap{g.L1, 1, 0, g.M1}, g.M1, g.L2, g.n2, tw2, 1);     // columns (y)
  __syncthreads();
  cx<T>* dst = S + ((long)(c0 + c) * g.M3 + kz) * g.M1 * g.M2;
  for (int t = threadIdx.x; t < g.M1 * g.M2; t += blockDim.x) dst[t] = buf[t];
}

template <typename T>
__global__ __launch_bounds__(kJmThreads) void k_jm_xyinv(const cx<T>* __restrict__ S, cx<T>* __restrict__ U, Geom g,
                                                          int c0, const cx<T>* __restrict__ tw1,
                                                          const cx<T>* __restrict__ tw2) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);     // [M2][M1]
  const int c = blockIdx.x % 3, kz = blockIdx.x / 3;
  const cx<T>* src = S + ((long)(c0 + c) * g.M3 + kz) * g.M1 * g.M2;
  for (int t = threadIdx.x; t < g.M1 * g.M2; t += blockDim.x) buf[t] = src[t];
  __syncthreads();
  fft_lds<T, true, kJmMaxV>(buf, SeqMap{g.L1, 1, 0, g.M1}, g.M1, g.L2, g.M2, tw2, 1);      // columns (y)
  fft_lds<T, true, kJmMaxV>(buf, SeqMap{0, 0, g.M1, 1}, g.n2, g.L1, g.M1, tw1, 1);         // rows y < n2 (x)
  __syncthreads();
  const long plane = (long)g.n1 * g.n2;
  cx<T>* dst = U + ((long)kz * 3 + c) * plane;
  for (int t = threadIdx.x; t < g.n2 * g.n1; t += blockDim.x) {
    const int y = t / g.n1, x = t % g.n1;
    dst[t] = buf[y * g.M1 + x];
  }
}

template <typename V>
__device__ __forceinline__ V cfma3(V a0, V b0, V a1, V b1, V a2, V b2) {
  return cadd(cadd(cmul(a0, b0), cmul(a1, b1)), cmul(a2, b2));
}

// i kappa z
template <typename T>
__device__ __forceinline__ cx<T> ikap(T kappa, cx<T> z) {
  return cx<T>{-kappa * z.y, kappa * z.x};
}

template <typename T>
__global__ void k_jm_product(cx<T>* __restrict__ S, const cx<T>* __restrict__ goct, const cx<T>* __restrict__ koct,
                             Geom g, T kappa) {
  const long P = (long)g.M1 * g.M2 * g.M3;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < P; i += (long)gridDim.x * blockDim.x) {
    const int kx = (int)(i % g.M1);
    const int ky = (int)((i / g.M1) % g.M2);
    const int kz = (int)(i / ((long)g.M1 * g.M2));
    // fold each axis to the stored octant; s_d = -1 where the frequency was negated
    const int k1 = kx <= g.M1 / 2 ? kx : g.M1 - kx;
    const int k2 = ky <= g.M2 / 2 ? ky : g.M2 - ky;
    const int k3 = kz <= g.M3 / 2 ? kz : g.M3 - kz;
    const T s1 = kx <= g.M1 / 2 ? (T)1 : (T)-1;
    const T s2 = ky <= g.M2 / 2 ? (T)1 : (T)-1;
    const T s3 = kz <= g.M3 / 2 ? (T)1 : (T)-1;
    const long o = ((long)k3 * g.H2 + k2) * g.H1 + k1;
    const cx<T>* G = goct + o * 6;
    const cx<T>* Kp = koct + o * 3;
    // N^{ab} is odd along d when exactly one of a, b is d; K^{ab} along the third axis
    const cx<T> gxx = G[0], gyy = G[3], gzz = G[5];
    const cx<T> gxy = cscale(G[1], s1 * s2), gxz = cscale(G[2], s1 * s3), gyz = cscale(G[4], s2 * s3);
    const cx<T> kxy = cscale(Kp[0], s3), kxz = cscale(Kp[1], s2), kyz = cscale(Kp[2], s1);
    cx<T> ue[3], um[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ue[a] = S[a * P + i];
      um[a] = S[(3 + a) * P + i];
    }
    const cx<T> zero{(T)0, (T)0};
    // (K u)_x = K^{xy} u_y + K^{xz} u_z, (K u)_y = -K^{xy} u_x + K^{yz} u_z, (K u)_z = -K^{xz} u_x - K^{yz} u_y
    auto Kmul = [&](const cx<T>* u, cx<T>* out) {
      out[0] = cadd(cmul(kxy, u[1]), cmul(kxz, u[2]));
      out[1] = csub(cmul(kyz, u[2]), cmul(kxy, u[0]));
      out[2] = csub(zero, cadd(cmul(kxz, u[0]), cmul(kyz, u[1])));
    };
    cx<T> kue[3], kum[3];
    Kmul(ue, kue);
    Kmul(um, kum);
    const cx<T> ne[3] = {cfma3(gxx, ue[0], gxy, ue[1], gxz, ue[2]), cfma3(gxy, ue[0], gyy, ue[1], gyz, ue[2]),
                         cfma3(gxz, ue[0], gyz, ue[1], gzz, ue[2])};
    const cx<T> nm[3] = {cfma3(gxx, um[0], gxy, um[1], gxz, um[2]), cfma3(gxy, um[0], gyy, um[1], gyz, um[2]),
                         cfma3(gxz, um[0], gyz, um[1], gzz, um[2])};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S[a * P + i] = cadd(ne[a], ikap(kappa, kum[a]));
      S[(3 + a) * P + i] = csub(nm[a], ikap(kappa, kue[a]));
    }
  }
}

}  // namespace

size_t jm_spectrum_values(const Geom& g) { return (size_t)6 * g.M1 * g.M2 * g.M3; }

template <typename T>
hipError_t allow_lds_jm() {
  const int bytes = 64 * 64 * (int)sizeof(cx<T>);
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_jm_xyfwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)))
    return e;
  return hipFuncSetAttribute((const void*)k_jm_xyinv<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T>
hipError_t launch_jm_matvec(const Geom& g, const Tune& t, const void* x, void* y, const void* b, int mode,
                            void* Ue, void* Um, void* S, const void* goct, const void* koct, const void* chi_e,
                            const void* chi_m, double kappa, const void* const tw[3], hipStream_t s) {
  using C = cx<T>;
  if (g.M1 * g.M2 > 64 * 64) return hipErrorInvalidValue;
  const long n3 = 3 * g.N;
  const C* xe = static_cast<const C*>(x);
  const C* xm = xe + n3;
  C* ye = static_cast<C*>(y);
  C* ym = ye + n3;
  const C* be = static_cast<const C*>(b);
  const C* bm = be ? be + n3 : nullptr;
  hipError_t e;
  if ((e = launch_pass<T>(0, g, t, xe, nullptr, nullptr, 0, Ue, goct, chi_e, tw, s))) return e;
  if ((e = launch_pass<T>(0, g, t, xm, nullptr, nullptr, 0, Um, goct, chi_m, tw, s))) return e;
  const size_t lds = (size_t)g.M1 * g.M2 * sizeof(C);
  const dim3 planes(3 * g.M3), block(kJmThreads);
  hipLaunchKernelGGL(k_jm_xyfwd<T>, planes, block, lds, s, (const C*)Ue, (C*)S, g, 0, (const C*)tw[0],
                     (const C*)tw[1]);
  hipLaunchKernelGGL(k_jm_xyfwd<T>, planes, block, lds, s, (const C*)Um, (C*)S, g, 3, (const C*)tw[0],
                     (const C*)tw[1]);
  if ((e = hipGetLastError())) return e;
  const long P = (long)g.M1 * g.M2 * g.M3;
  const long nb = (P + 255) / 256;
  hipLaunchKernelGGL(k_jm_product<T>, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(256), 0, s, (C*)S,
                     (const C*)goct, (const C*)koct, g, (T)kappa);
  hipLaunchKernelGGL(k_jm_xyinv<T>, planes, block, lds, s, (const C*)S, (C*)Ue, g, 0, (const C*)tw[0],
                     (const C*)tw[1]);
  hipLaunchKernelGGL(k_jm_xyinv<T>, planes, block, lds, s, (const C*)S, (C*)Um, g, 3, (const C*)tw[0],
                     (const C*)tw[1]);
  if ((e = hipGetLastError())) return e;
  if ((e = launch_pass<T>(2, g, t, xe, ye, be, mode, Ue, goct, chi_e, tw, s))) return e;
  return launch_pass<T>(2, g, t, xm, ym, bm, mode, Um, goct, chi_m, tw, s);
}

template hipError_t allow_lds_jm<double>();
template hipError_t allow_lds_jm<float>();
template hipError_t launch_jm_matvec<double>(const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                             void*, void*, const void*, const void*, const void*, const void*, double,
                                             const void* const[3], hipStream_t);
template hipError_t launch_jm_matvec<float>(const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                            void*, void*, const void*, const void*, const void*, const void*, double,
                                            const void* const[3], hipStream_t);

}  // namespace vie
