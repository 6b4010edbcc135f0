// The JM-VIE (Section III): the coupled product of electric and magnetic currents.
//
//   y = (I - M T~) x,   T~ = [[N, i kappa K], [-i kappa K, N]],
//
// x = (x_e, x_m) with six components, the magnetic unknowns in impedance units
// and exp(-i omega t); K = curl S is block Toeplitz like N, with three
// antisymmetric components (K^{ba} = -K^{ab}) odd along the axis other than a
// and b, so its spectrum is stored on one octant too.  The product reuses the
// z passes of the J-VIE once per half.  Between them, when the row-transformed
// plane of all six components fits in LDS (every FP32 grid; FP64 while
// 6 n2 M1 values leave room for the column chunk), one fused kernel per kz plane:
//   k_jm_xy:      rows along x, column chunks along y, the 6 x 6 product with
//                 N^ and K^, inverse columns and rows, crop: U_e, U_m in place.
// Otherwise three kernels over full cross-section spectra in HBM:
//   k_jm_xyfwd:   per (kz, component) plane: the n2 x n1 slice of the
//                 z-transformed intermediate, zero padded to M2 x M1, 2-D FFT
//                 in LDS, into S[component][kz][ky][kx]
//   k_jm_product: per spectral point: the 6 x 6 product
//   k_jm_xyinv:   per plane: inverse 2-D FFT, crop to n2 x n1, back into U
// A plane is at most 64 x 64 values (n1, n2 <= 32), 64 KiB in FP64.
#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "lds_fft.hpp"
#include "vie_internal.hpp"

namespace vie {
namespace {

constexpr int kJmThreads = 256;
constexpr int kJmMaxV = 16;   // values per thread per FFT stage: 256 x 16 = 4096 = the largest plane
constexpr size_t kJmFusedLds = 160 * 1024;   // the fused pass may take a CU's whole LDS

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

// N and K at one frequency of the full circulant, from the stored octant: the
// signs of the odd components follow the folded axes (N^{ab} odd along d when
// exactly one of a, b is d; K^{ab} odd along its third axis).
template <typename T>
struct JmCoef {
  cx<T> gxx, gxy, gxz, gyy, gyz, gzz, kxy, kxz, kyz;
};

template <typename T>
__device__ __forceinline__ JmCoef<T> jm_coef(const cx<T>* __restrict__ G, const cx<T>* __restrict__ Kp, T s1, T s2,
                                             T s3) {
  JmCoef<T> c;
  c.gxx = G[0];
  c.gyy = G[3];
  c.gzz = G[5];
  c.gxy = cscale(G[1], s1 * s2);
  c.gxz = cscale(G[2], s1 * s3);
  c.gyz = cscale(G[4], s2 * s3);
  c.kxy = cscale(Kp[0], s3);
  c.kxz = cscale(Kp[1], s2);
  c.kyz = cscale(Kp[2], s1);
  return c;
}

// out_e = N u_e + i kappa K u_m, out_m = N u_m - i kappa K u_e (K antisymmetric)
template <typename T>
__device__ __forceinline__ void jm_apply(const JmCoef<T>& c, T kappa, const cx<T> ue[3], const cx<T> um[3],
                                         cx<T> oe[3], cx<T> om[3]) {
  const cx<T> zero{(T)0, (T)0};
  const cx<T> kue[3] = {cadd(cmul(c.kxy, ue[1]), cmul(c.kxz, ue[2])), csub(cmul(c.kyz, ue[2]), cmul(c.kxy, ue[0])),
                        csub(zero, cadd(cmul(c.kxz, ue[0]), cmul(c.kyz, ue[1])))};
  const cx<T> kum[3] = {cadd(cmul(c.kxy, um[1]), cmul(c.kxz, um[2])), csub(cmul(c.kyz, um[2]), cmul(c.kxy, um[0])),
                        csub(zero, cadd(cmul(c.kxz, um[0]), cmul(c.kyz, um[1])))};
  const cx<T> ne[3] = {cfma3(c.gxx, ue[0], c.gxy, ue[1], c.gxz, ue[2]), cfma3(c.gxy, ue[0], c.gyy, ue[1], c.gyz, ue[2]),
                       cfma3(c.gxz, ue[0], c.gyz, ue[1], c.gzz, ue[2])};
  const cx<T> nm[3] = {cfma3(c.gxx, um[0], c.gxy, um[1], c.gxz, um[2]), cfma3(c.gxy, um[0], c.gyy, um[1], c.gyz, um[2]),
                       cfma3(c.gxz, um[0], c.gyz, um[1], c.gzz, um[2])};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    oe[a] = cadd(ne[a], ikap(kappa, kum[a]));
    om[a] = csub(nm[a], ikap(kappa, kue[a]));
  }
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
    const JmCoef<T> c = jm_coef<T>(goct + o * 6, koct + o * 3, s1, s2, s3);
    cx<T> ue[3], um[3], oe[3], om[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ue[a] = S[a * P + i];
      um[a] = S[(3 + a) * P + i];
    }
    jm_apply<T>(c, kappa, ue, um, oe, om);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S[a * P + i] = oe[a];
      S[(3 + a) * P + i] = om[a];
    }
  }
}

// Fused cross-section pass of the JM product on one kz plane (used when the
// plane's row transforms of all six components fit in LDS): row transforms
// along x of the n2 valid rows, then for each chunk of cc x-frequencies the
// column transforms along y, the coupled product with N and i kappa K, the
// inverse column transforms, and at the end the inverse row transforms and the
// crop.  Ue, Um are read and overwritten in place; the spectra stay in LDS.
//
// The transforms are the padded LDS stages of lds_fft.hpp (bank-conflict free
// rows and position-major column chunks); twiddles are staged in LDS.

// SPLIT = 2 (cross-sections whose full rows of six components do not fit in
// LDS): the x-frequencies in two halves.  With x_n = 0 for n >= M1/2, the
// M1-point transform splits into X[2m] = DFT_{M1/2}(x)[m] and
// X[2m + 1] = DFT_{M1/2}(x_n W^n)[m], W = exp(-2 pi i / M1); the inverse with
// the crop to n < M1/2 is y_n = IDFT(Y_even)_n + W^{-n} IDFT(Y_odd)_n.  The
// workgroup runs both halves in turn on half-length rows and keeps the first
// half's output in registers (kAcc values per thread).
template <int SPLIT>
constexpr int kJmXyThreads = SPLIT == 1 ? 1024 : 512;
constexpr int kJmAcc = 16;

template <typename T, int SPLIT>
__global__ __launch_bounds__(kJmXyThreads<SPLIT>) void k_jm_xy(cx<T>* __restrict__ Ue, cx<T>* __restrict__ Um,
                                                               const cx<T>* __restrict__ goct,
                                                               const cx<T>* __restrict__ koct, Geom g, int cc,
                                                               T kappa, const cx<T>* __restrict__ tw1,
                                                               const cx<T>* __restrict__ tw2) {
  extern __shared__ unsigned char smem_raw[];
  const int Mx = g.M1 / SPLIT;                          // row transform length
  const int Lx = g.L1 - (SPLIT == 2 ? 1 : 0);
  const int pitch = Mx + (Mx >> 3);
  const int M2p = g.M2 + (g.M2 >> 3);
  cx<T>* A = reinterpret_cast<cx<T>*>(smem_raw);       // [6 n2][pitch]: e components, then m
  cx<T>* C = A + 6 * g.n2 * pitch;                      // [6][M2p][cc]
  cx<T>* W2 = C + 6 * M2p * cc;                         // twiddles of M2
  cx<T>* W1 = W2 + g.M2;                                // twiddles of M1 (the twist W^n)
  cx<T>* Wx = SPLIT == 1 ? W1 : W1 + g.M1;              // twiddles of the row length
  const int kz = paired_plane(blockIdx.x, g.M3);
  const int plane = 3 * g.n1 * g.n2;
  cx<T>* Pe = Ue + (long)kz * plane;
  cx<T>* Pm = Um + (long)kz * plane;
  for (int t = threadIdx.x; t < g.M1; t += blockDim.x) W1[t] = tw1[t];
  for (int t = threadIdx.x; t < g.M2; t += blockDim.x) W2[t] = tw2[t];
  if (SPLIT == 2)
    for (int t = threadIdx.x; t < Mx; t += blockDim.x) Wx[t] = tw1[2 * t];
  // rows r < 6 n2, x < n1: lanes along x with a power-of-two row width (M1/2 >= n1)
  const int wlog = g.L1 > 0 ? g.L1 - 1 : 0;
  const int rows = 6 * g.n2;
  const int items = rows << wlog;
  cx<T> acc[SPLIT == 2 ? kJmAcc : 1];

  const int k3 = kz <= g.M3 / 2 ? kz : g.M3 - kz;
  const T s3 = kz <= g.M3 / 2 ? (T)1 : (T)-1;
  const cx<T>* G3 = goct + (long)k3 * g.H2 * g.H1 * 6;
  const cx<T>* K3 = koct + (long)k3 * g.H2 * g.H1 * 3;
  int cclog = 0;
  while ((1 << cclog) < cc) ++cclog;
  const int npts = g.M2 << cclog;
  for (int h = 0; h < SPLIT; ++h) {
    __syncthreads();   // the rows of the previous half have been read
    for (int t = threadIdx.x; t < items; t += blockDim.x) {
      const int x = t & ((1 << wlog) - 1), r = t >> wlog;
      if (x < g.n1) {
        cx<T> v = r < 3 * g.n2 ? Pe[r * g.n1 + x] : Pm[(r - 3 * g.n2) * g.n1 + x];
        if (SPLIT == 2 && h == 1) v = cmul(v, W1[x]);
        A[r * pitch + pad8(x)] = v;
      }
    }
    __syncthreads();
    // the electric rows, then the magnetic rows (half the plane per call)
    pad_rows<T, false>(A, 3 * g.n2, pitch, Lx, g.n1, Wx, opaque_tid());
    pad_rows<T, false>(A + 3 * g.n2 * pitch, 3 * g.n2, pitch, Lx, g.n1, Wx, opaque_tid());
    for (int c0 = 0; c0 < Mx; c0 += cc) {
      const PadCols m{6, cclog, M2p, g.n2, pitch, c0};
      // a fresh opaque thread index per chunk: otherwise every stage's per-lane
      // address terms are hoisted out of the chunk loop and held in registers
      const int tid = opaque_tid();
      pad_cols<T, false>(A, C, m, g.L2, W2, tid);
      // product points: col fastest, then ky
      for (int t = tid; t < npts; t += blockDim.x) {
        const int col = t & (cc - 1), ky = t >> cclog;
        const int kx = SPLIT * (c0 + col) + h;
        const int k1 = kx <= g.M1 / 2 ? kx : g.M1 - kx;
        const int k2 = ky <= g.M2 / 2 ? ky : g.M2 - ky;
        const long f = (long)k2 * g.H1 + k1;
        const JmCoef<T> c =
            jm_coef<T>(G3 + f * 6, K3 + f * 3, kx <= g.M1 / 2 ? (T)1 : (T)-1, ky <= g.M2 / 2 ? (T)1 : (T)-1, s3);
        const int o = ((pad8(ky)) << cclog) + col;
        const int cs = M2p << cclog;
        cx<T> ue[3], um[3], oe[3], om[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          ue[a] = C[a * cs + o];
          um[a] = C[(3 + a) * cs + o];
        }
        jm_apply<T>(c, kappa, ue, um, oe, om);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          C[a * cs + o] = oe[a];
          C[(3 + a) * cs + o] = om[a];
        }
      }
      __syncthreads();
      pad_cols<T, true>(A, C, m, g.L2, W2, tid);
    }
    pad_rows<T, true>(A, 3 * g.n2, pitch, Lx, Mx, Wx, opaque_tid());
    pad_rows<T, true>(A + 3 * g.n2 * pitch, 3 * g.n2, pitch, Lx, Mx, Wx, opaque_tid());
    if (SPLIT == 1) {
      for (int t = threadIdx.x; t < items; t += blockDim.x) {
        const int x = t & ((1 << wlog) - 1), r = t >> wlog;
        if (x < g.n1) {
          const cx<T> v = A[r * pitch + pad8(x)];
          if (r < 3 * g.n2) Pe[r * g.n1 + x] = v;
          else Pm[(r - 3 * g.n2) * g.n1 + x] = v;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < (SPLIT == 2 ? kJmAcc : 1); ++q) {
        const int t = threadIdx.x + q * blockDim.x;
        const int x = t & ((1 << wlog) - 1), r = t >> wlog;
        if (t < items && x < g.n1) {
          const cx<T> v = A[r * pitch + pad8(x)];
          if (h == 0) {
            acc[q] = v;
          } else {
            const cx<T> y = cadd(acc[q], cmulc(v, W1[x]));
            if (r < 3 * g.n2) Pe[r * g.n1 + x] = y;
            else Pm[(r - 3 * g.n2) * g.n1 + x] = y;
          }
        }
      }
    }
  }
}

}  // namespace

size_t jm_spectrum_values(const Geom& g) { return (size_t)6 * g.M1 * g.M2 * g.M3; }

template <typename T>
size_t jm_fused_lds(const Geom& g, int cc, int split) {
  const size_t Mx = g.M1 / split;
  const size_t pitch = Mx + (Mx >> 3), M2p = g.M2 + (g.M2 >> 3);
  return (6 * g.n2 * pitch + 6 * M2p * cc + g.M1 + g.M2 + (split == 2 ? Mx : 0)) * sizeof(cx<T>);
}

template <typename T>
bool jm_fused_shape(const Geom& g, int* cc_out, int* threads_out, int* split_out) {
  for (int split = 1; split <= 2; ++split) {
    if (split == 2 && g.M1 < 2) break;
    const int Mx = g.M1 / split;
    int cc = Mx < 16 ? Mx : 16;
    while (cc > 1 && jm_fused_lds<T>(g, cc, split) > kJmFusedLds) cc >>= 1;
    if (jm_fused_lds<T>(g, cc, split) > kJmFusedLds) continue;
    // every stage holds at most kPadMaxV values per thread (rows: one half of the
    // components at a time); the halves variant keeps kJmAcc outputs per thread
    const size_t rows = (size_t)3 * g.n2 * Mx, cols = (size_t)6 * g.M2 * cc;
    size_t need = ((rows > cols ? rows : cols) + kPadMaxV - 1) / kPadMaxV;
    if (split == 2) {
      const size_t items = (size_t)6 * g.n2 * (g.M1 / 2);
      const size_t acc = (items + kJmAcc - 1) / kJmAcc;
      if (acc > need) need = acc;
    }
    int threads = (int)((need + 63) / 64) * 64;
    if (threads < 256) threads = 256;
    // at least 512 threads: more waves hide the latency of the LDS stages (with
    // more, the FP32 strip's workgroups no longer fit two to a CU)
    if (threads < 512) threads = 512;
    if (threads > (split == 1 ? kJmXyThreads<1> : kJmXyThreads<2>)) continue;
    if (cc_out) *cc_out = cc;
    if (threads_out) *threads_out = threads;
    if (split_out) *split_out = split;
    return true;
  }
  return false;
}

template <typename T>
hipError_t allow_lds_jm() {
  const int bytes = 64 * 64 * (int)sizeof(cx<T>);
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_jm_xyfwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_jm_xy<T, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kJmFusedLds)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_jm_xy<T, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kJmFusedLds)))
    return e;
  return hipFuncSetAttribute((const void*)k_jm_xyinv<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T>
hipError_t launch_jm_matvec(const Geom& g, const Tune& t, const void* x, void* y, const void* b, int mode,
                            void* Ue, void* Um, void* S, const void* goct, const void* koct, const void* chi_e,
                            const void* chi_m, double kappa, bool fused, const void* const tw[3], hipStream_t s) {
  using C = cx<T>;
  if (g.M1 * g.M2 > 64 * 64) return hipErrorInvalidValue;
  int cc = 0, threads = 0, split = 1;
  if (fused && !jm_fused_shape<T>(g, &cc, &threads, &split)) return hipErrorInvalidValue;
  if (!fused && !S) return hipErrorInvalidValue;
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
  if (fused) {
    const size_t lds = jm_fused_lds<T>(g, cc, split);
    if (split == 1)
      hipLaunchKernelGGL((k_jm_xy<T, 1>), dim3(g.M3), dim3(threads), lds, s, (C*)Ue, (C*)Um, (const C*)goct,
                         (const C*)koct, g, cc, (T)kappa, (const C*)tw[0], (const C*)tw[1]);
    else
      hipLaunchKernelGGL((k_jm_xy<T, 2>), dim3(g.M3), dim3(threads), lds, s, (C*)Ue, (C*)Um, (const C*)goct,
                         (const C*)koct, g, cc, (T)kappa, (const C*)tw[0], (const C*)tw[1]);
    if ((e = hipGetLastError())) return e;
    if ((e = launch_pass<T>(2, g, t, xe, ye, be, mode, Ue, goct, chi_e, tw, s))) return e;
    return launch_pass<T>(2, g, t, xm, ym, bm, mode, Um, goct, chi_m, tw, s);
  }
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
template bool jm_fused_shape<double>(const Geom&, int*, int*, int*);
template bool jm_fused_shape<float>(const Geom&, int*, int*, int*);
template hipError_t launch_jm_matvec<double>(const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                             void*, void*, const void*, const void*, const void*, const void*, double,
                                             bool, const void* const[3], hipStream_t);
template hipError_t launch_jm_matvec<float>(const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                            void*, void*, const void*, const void*, const void*, const void*, double,
                                            bool, const void* const[3], hipStream_t);

}  // namespace vie
