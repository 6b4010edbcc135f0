// Matrix-vector product of the discrete J-VIE operator on gfx950, and the
// plan-time construction of the Green spectrum.
//
// y = (I - M_eps N) x (Section III-A / Section V-D).  N is block Toeplitz; its
// product is a circular convolution after embedding in a circulant of size
// M = (M1, M2, M3) >= 2n - 1 and zero padding x.  Three passes over HBM:
//
//   pass 1 (k_zfwd):  per z-pencil of one component: zero-pad n3 -> M3, forward
//                     FFT, write kz-plane-major  U[kz][c][i2][i1]
//   pass 2 (k_xyp):   per kz plane: forward FFT along i1 (pad n1 -> M1) and i2
//                     (pad n2 -> M2), 3x3 symmetric product with the Green
//                     spectrum, inverse FFT along i2 and i1, crop to n2 x n1
//   pass 3 (k_zinv):  per z-pencil: inverse FFT, crop to n3, and the contrast:
//                     y = x - chi * u   (or the residual b - y)
//
// The spectrum is stored on one octant only: negating frequency k_d multiplies
// G^{ab} by -1 exactly when one of a, b is d (the parity of the Toeplitz
// entries carries over to the DFT), and it already holds the 1/(M1 M2 M3)
// of the inverse transform.
#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "lds_fft.hpp"
#include "vie_internal.hpp"

namespace vie {

template <typename T>
hipError_t launch_xy64(const Geom& g, int V, void* U, const void* goct, const void* tw1, hipStream_t s);
template <typename T>
hipError_t allow_lds_xy64();
template <typename T>
hipError_t launch_xy6432(const Geom& g, int V, void* U, const void* goct, const void* tw1, const void* tw2,
                         hipStream_t s);
template <typename T>
hipError_t allow_lds_xy6432();
template <typename T>
hipError_t launch_z4(int which, const Geom& g, int P, const void* x, void* y, const void* b, int mode, void* U,
                     const void* chi, const void* twz, hipStream_t st);
template <typename T>
hipError_t allow_lds_z4();
template <typename T>
hipError_t launch_z4_batch(int which, int mode, const PassDesc* d, const int* prefix, int nsys, int total, int A,
                           int B, int P, int jx, int jy, hipStream_t st);
template <typename T>
hipError_t launch_xy64_batch(const PassDesc* d, const int* prefix, int nsys, int total, hipStream_t s);

constexpr int kMaxV = 16;   // complex values per thread per FFT stage

// ------------------------------------------------------------------ pass 1
template <typename T>
__global__ __launch_bounds__(1024) void k_zfwd(const cx<T>* __restrict__ x, cx<T>* __restrict__ U, Geom g,
                                                int tp, const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const PencilBlock pb = pencil_block(xcd_group8(blockIdx.x, gridDim.x), g.n1, g.n2, tp);
  const int i2 = pb.i2, c = pb.c, i1_0 = pb.i1_0, np = pb.np;
  const int ld = g.M3 + 1;
  for (int p = 0; p < np; ++p) {
    const cx<T>* src = x + (((long)c * g.n1 + i1_0 + p) * g.n2 + i2) * g.n3;
    for (int z = threadIdx.x; z < g.n3; z += blockDim.x) buf[p * ld + z] = src[z];
  }
  __syncthreads();
  fft_lds<T, false, kMaxV>(buf, SeqMap{0, 0, ld, 1}, np, g.L3, g.n3, tw, 1);
  const long plane = 3L * g.n1 * g.n2;
  cx<T>* dst = U + ((long)c * g.n2 + i2) * g.n1 + i1_0;
  for (int t = threadIdx.x; t < np * g.M3; t += blockDim.x) {
    const int p = t % np, kz = t / np;
    dst[kz * plane + p] = buf[p * ld + kz];
  }
}

// ------------------------------------------------------------------ pass 3
template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_zinv(const cx<T>* __restrict__ U, const cx<T>* __restrict__ x,
                                                cx<T>* __restrict__ y, const cx<T>* __restrict__ bvec,
                                                const cx<T>* __restrict__ chi, Geom g, int tp,
                                                const cx<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const PencilBlock pb = pencil_block(xcd_group8(blockIdx.x, gridDim.x), g.n1, g.n2, tp);
  const int i2 = pb.i2, c = pb.c, i1_0 = pb.i1_0, np = pb.np;
  const int ld = g.M3 + 1;
  const long plane = 3L * g.n1 * g.n2;
  const cx<T>* src = U + ((long)c * g.n2 + i2) * g.n1 + i1_0;
  for (int t = threadIdx.x; t < np * g.M3; t += blockDim.x) {
    const int p = t % np, kz = t / np;
    buf[p * ld + kz] = src[kz * plane + p];
  }
  __syncthreads();
  fft_lds<T, true, kMaxV>(buf, SeqMap{0, 0, ld, 1}, np, g.L3, g.M3, tw, 1);
  for (int p = 0; p < np; ++p) {
    const long vox = ((long)(i1_0 + p) * g.n2 + i2) * g.n3;
    const long off = (long)c * g.N + vox;
    for (int z = threadIdx.x; z < g.n3; z += blockDim.x) {
      const cx<T> u = buf[p * ld + z];
      const cx<T> xv = x[off + z];
      const cx<T> r = csub(xv, cmul(chi[vox + z], u));
      y[off + z] = MODE == 0 ? r : csub(bvec[off + z], r);
    }
  }
}

// ------------------------------------------------------------------ pass 2
// Cross-sections other than 64 x 64: one workgroup per kz plane.  x transforms
// of the 3 n2 valid rows, then for each chunk of cc x-frequencies the y
// transforms, the 3 x 3 Green product and the inverse y transforms, finally the
// inverse x transforms and the crop; U is read and overwritten in place.  The
// transforms are the padded LDS stages of lds_fft.hpp (bank-conflict-free rows
// and position-major column chunks); twiddles are staged in LDS.
template <typename T>
__global__ __launch_bounds__(1024) void k_xyp(cx<T>* __restrict__ U, const cx<T>* __restrict__ goct, Geom g, int cc,
                                              const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ tw2) {
  extern __shared__ unsigned char smem_raw[];
  const int pitch = g.M1 + (g.M1 >> 3);
  const int M2p = g.M2 + (g.M2 >> 3);
  cx<T>* A = reinterpret_cast<cx<T>*>(smem_raw);      // [3 n2][pitch]
  cx<T>* C = A + 3 * g.n2 * pitch;                     // [3][M2p][cc]
  cx<T>* W1 = C + 3 * M2p * cc;                        // twiddles of M1, then of M2
  cx<T>* W2 = W1 + g.M1;
  const int kz = paired_plane(blockIdx.x, g.M3);
  cx<T>* P = U + (long)kz * 3 * g.n1 * g.n2;
  // rows r < 3 n2, x < n1: lanes along x with a power-of-two row width
  const int wlog = g.L1 > 0 ? g.L1 - 1 : 0;
  const int rows = 3 * g.n2;
  for (int t = threadIdx.x; t < rows << wlog; t += blockDim.x) {
    const int x = t & ((1 << wlog) - 1), r = t >> wlog;
    if (x < g.n1) A[r * pitch + pad8(x)] = P[r * g.n1 + x];
  }
  for (int t = threadIdx.x; t < g.M1; t += blockDim.x) W1[t] = tw1[t];
  for (int t = threadIdx.x; t < g.M2; t += blockDim.x) W2[t] = tw2[t];
  __syncthreads();
  pad_rows<T, false>(A, rows, pitch, g.L1, g.n1, W1, opaque_tid());

  // plane frequency along z, folded to the stored octant
  const int k3 = kz <= g.M3 / 2 ? kz : g.M3 - kz;
  const T s3 = kz <= g.M3 / 2 ? (T)1 : (T)-1;
  const cx<T>* G3 = goct + (long)k3 * g.H2 * g.H1 * 6;
  int cclog = 0;
  while ((1 << cclog) < cc) ++cclog;
  const int npts = g.M2 << cclog;
  const int cs = M2p << cclog;
  for (int c0 = 0; c0 < g.M1; c0 += cc) {
    const PadCols m{3, cclog, M2p, g.n2, pitch, c0};
    // a fresh opaque thread index per chunk keeps the stages' per-lane address
    // terms from being hoisted out of the chunk loop
    const int tid = opaque_tid();
    pad_cols<T, false>(A, C, m, g.L2, W2, tid);
    for (int t = tid; t < npts; t += blockDim.x) {
      const int col = t & (cc - 1), ky = t >> cclog;
      const int kx = c0 + col;
      const int k1 = kx <= g.M1 / 2 ? kx : g.M1 - kx;
      const int k2 = ky <= g.M2 / 2 ? ky : g.M2 - ky;
      const T s1 = kx <= g.M1 / 2 ? (T)1 : (T)-1;
      const T s2 = ky <= g.M2 / 2 ? (T)1 : (T)-1;
      const cx<T>* Gp = G3 + ((long)k2 * g.H1 + k1) * 6;
      const cx<T> gxx = Gp[0], gyy = Gp[3], gzz = Gp[5];
      const cx<T> gxy = cscale(Gp[1], s1 * s2), gxz = cscale(Gp[2], s1 * s3), gyz = cscale(Gp[4], s2 * s3);
      const int o = (pad8(ky) << cclog) + col;
      const cx<T> ux = C[o], uy = C[cs + o], uz = C[2 * cs + o];
      C[o] = cadd(cadd(cmul(gxx, ux), cmul(gxy, uy)), cmul(gxz, uz));
      C[cs + o] = cadd(cadd(cmul(gxy, ux), cmul(gyy, uy)), cmul(gyz, uz));
      C[2 * cs + o] = cadd(cadd(cmul(gxz, ux), cmul(gyz, uy)), cmul(gzz, uz));
    }
    __syncthreads();
    pad_cols<T, true>(A, C, m, g.L2, W2, tid);
  }
  pad_rows<T, true>(A, rows, pitch, g.L1, g.M1, W1, opaque_tid());
  for (int t = threadIdx.x; t < rows << wlog; t += blockDim.x) {
    const int x = t & ((1 << wlog) - 1), r = t >> wlog;
    if (x < g.n1) P[r * g.n1 + x] = A[r * pitch + pad8(x)];
  }
}

template <typename T>
size_t z_lds_bytes(const Geom& g, int tp) { return (size_t)tp * (g.M3 + 1) * sizeof(cx<T>); }
template <typename T>
size_t xy_lds_bytes(const Geom& g, int cc) {
  const size_t pitch = g.M1 + (g.M1 >> 3), M2p = g.M2 + (g.M2 >> 3);
  return (3 * g.n2 * pitch + 3 * M2p * cc + g.M1 + g.M2) * sizeof(cx<T>);
}
template size_t xy_lds_bytes<double>(const Geom&, int);
template size_t xy_lds_bytes<float>(const Geom&, int);

template <typename T>
hipError_t launch_pass(int which, const Geom& g, const Tune& t, const void* x, void* y, const void* b, int mode,
                       void* U, const void* goct, const void* chi, const void* const tw[3], hipStream_t s) {
  using C = cx<T>;
  if (which != 1 && t.z4) return launch_z4<T>(which, g, t.zp, x, y, b, mode, U, chi, tw[2], s);
  const int nb1 = (g.n1 + t.tp - 1) / t.tp;
  const dim3 gz(3 * g.n2 * nb1);
  const size_t zl = z_lds_bytes<T>(g, t.tp);
  if (which == 0) {
    hipLaunchKernelGGL((k_zfwd<T>), gz, dim3(t.zthreads), zl, s, (const C*)x, (C*)U, g, t.tp, (const C*)tw[2]);
  } else if (which == 1 && g.M1 == 64 && g.M2 == 64) {
    return launch_xy64<T>(g, t.xyv, U, goct, tw[0], s);
  } else if (which == 1 && g.M1 == 64 && g.M2 == 32 && (t.xyv == 1 || t.xyv == 2)) {
    return launch_xy6432<T>(g, t.xyv, U, goct, tw[0], tw[1], s);
  } else if (which == 1) {
    hipLaunchKernelGGL((k_xyp<T>), dim3(g.M3), dim3(t.xythreads), xy_lds_bytes<T>(g, t.cc), s, (C*)U,
                       (const C*)goct, g, t.cc, (const C*)tw[0], (const C*)tw[1]);
  } else if (mode == 0) {
    hipLaunchKernelGGL((k_zinv<T, 0>), gz, dim3(t.zthreads), zl, s, (const C*)U, (const C*)x, (C*)y,
                       (const C*)nullptr, (const C*)chi, g, t.tp, (const C*)tw[2]);
  } else {
    hipLaunchKernelGGL((k_zinv<T, 1>), gz, dim3(t.zthreads), zl, s, (const C*)U, (const C*)x, (C*)y,
                       (const C*)b, (const C*)chi, g, t.tp, (const C*)tw[2]);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_matvec(const Geom& g, const Tune& t, const void* x, void* y, const void* b, int mode,
                         void* U, const void* goct, const void* chi, const void* const tw[3],
                         hipStream_t s) {
  hipError_t e;
  for (int which = 0; which < 3; ++which)
    if ((e = launch_pass<T>(which, g, t, x, y, b, mode, U, goct, chi, tw, s))) return e;
  return hipSuccess;
}

template <typename T>
hipError_t launch_pass_batch(int which, int mode, const PassDesc* d, const int* prefix, int nsys, int total, int A,
                             int B, int P, int jx, int jy, hipStream_t s) {
  if (which == 1) return launch_xy64_batch<T>(d, prefix, nsys, total, s);
  return launch_z4_batch<T>(which, mode, d, prefix, nsys, total, A, B, P, jx, jy, s);
}
template hipError_t launch_pass_batch<double>(int, int, const PassDesc*, const int*, int, int, int, int, int, int,
                                              int, hipStream_t);
template hipError_t launch_pass_batch<float>(int, int, const PassDesc*, const int*, int, int, int, int, int, int,
                                             int, hipStream_t);

template hipError_t launch_pass<double>(int, const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                        const void*, const void*, const void* const[3], hipStream_t);
template hipError_t launch_pass<float>(int, const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                       const void*, const void*, const void* const[3], hipStream_t);
template hipError_t launch_matvec<double>(const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                          const void*, const void*, const void* const[3], hipStream_t);
template hipError_t launch_matvec<float>(const Geom&, const Tune&, const void*, void*, const void*, int, void*,
                                         const void*, const void*, const void* const[3], hipStream_t);

// Kernel attribute set-up for large LDS allocations (called once per plan).
template <typename T>
hipError_t allow_lds(size_t bytes) {
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_zfwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_zinv<T, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_zinv<T, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)))
    return e;
  if ((e = allow_lds_xy64<T>())) return e;
  if ((e = allow_lds_xy6432<T>())) return e;
  if ((e = allow_lds_z4<T>())) return e;
  return hipFuncSetAttribute((const void*)k_xyp<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
template hipError_t allow_lds<double>(size_t);
template hipError_t allow_lds<float>(size_t);

// ------------------------------------------------------------------ spectrum (plan time)

// Circulant embedding of one tensor component: slot k_d < n_d holds offset k_d,
// slot k_d > M_d - n_d holds offset k_d - M_d (sign from the parity), others 0.
__global__ void k_embed(const double2* __restrict__ table, double2* __restrict__ F, Geom g, int comp,
                        int pa, int pb) {
  const long P = (long)g.M1 * g.M2 * g.M3;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < P; i += (long)gridDim.x * blockDim.x) {
    const int k3 = (int)(i % g.M3);
    const int k2 = (int)((i / g.M3) % g.M2);
    const int k1 = (int)(i / ((long)g.M3 * g.M2));
    const int k[3] = {k1, k2, k3};
    const int n[3] = {g.n1, g.n2, g.n3};
    const int M[3] = {g.M1, g.M2, g.M3};
    int o[3];
    double sign = 1.0;
    bool zero = false;
    for (int d = 0; d < 3; ++d) {
      if (k[d] < n[d]) {
        o[d] = k[d];
      } else if (k[d] > M[d] - n[d]) {
        o[d] = M[d] - k[d];
        if ((pa == d) != (pb == d)) sign = -sign;
      } else {
        zero = true;
        o[d] = 0;
      }
    }
    double2 v = {0.0, 0.0};
    if (!zero) {
      v = table[(((long)comp * g.n1 + o[0]) * g.n2 + o[1]) * g.n3 + o[2]];
      v.x *= sign;
      v.y *= sign;
    }
    F[i] = v;
  }
}

// In-place forward FFT of many lines of a full array in global memory.  A line s
// starts at (s / inner_cnt) * outer + (s % inner_cnt) * inner_stride, element k
// at + k * es.  Each workgroup stages gb lines in LDS as [k][g].
__global__ __launch_bounds__(1024) void k_fft_lines(double2* __restrict__ F, int Llog2, long es, long inner_cnt,
                                                    long inner_stride, long outer, long nlines, int gb,
                                                    const double2* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  double2* buf = reinterpret_cast<double2*>(smem_raw);
  const int L = 1 << Llog2;
  const long s0 = (long)blockIdx.x * gb;
  const int ng = (int)min((long)gb, nlines - s0);
  for (int t = threadIdx.x; t < ng * L; t += blockDim.x) {
    const int gi = t % ng, k = t / ng;
    const long s = s0 + gi;
    buf[k * gb + gi] = F[(s / inner_cnt) * outer + (s % inner_cnt) * inner_stride + k * es];
  }
  __syncthreads();
  int glog = 0;
  while ((1 << glog) < gb) ++glog;
  fft_lds<double, false, kMaxV>(buf, SeqMap{glog, 1, 0, gb}, ng, Llog2, L, tw, 1);
  for (int t = threadIdx.x; t < ng * L; t += blockDim.x) {
    const int gi = t % ng, k = t / ng;
    const long s = s0 + gi;
    F[(s / inner_cnt) * outer + (s % inner_cnt) * inner_stride + k * es] = buf[k * gb + gi];
  }
}

__global__ void k_octant(const double2* __restrict__ F, double2* __restrict__ g64, float2* __restrict__ g32,
                         Geom g, int comp, int ncomp, double invP) {
  const long H = (long)g.H1 * g.H2 * g.H3;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < H; i += (long)gridDim.x * blockDim.x) {
    const int k1 = (int)(i % g.H1);
    const int k2 = (int)((i / g.H1) % g.H2);
    const int k3 = (int)(i / ((long)g.H1 * g.H2));
    double2 v = F[((long)k1 * g.M2 + k2) * g.M3 + k3];
    v.x *= invP;
    v.y *= invP;
    g64[i * ncomp + comp] = v;
    if (g32) g32[i * ncomp + comp] = float2{(float)v.x, (float)v.y};
  }
}

static hipError_t fft_axis(double2* F, const Geom& g, int axis, const double2* tw, hipStream_t s) {
  const long M1 = g.M1, M2 = g.M2, M3 = g.M3;
  int Llog2, L;
  long es, inner_cnt, inner_stride, outer, nlines;
  if (axis == 2) {
    Llog2 = g.L3; es = 1; inner_cnt = 1; inner_stride = 0; outer = M3; nlines = M1 * M2;
  } else if (axis == 1) {
    Llog2 = g.L2; es = M3; inner_cnt = M3; inner_stride = 1; outer = M2 * M3; nlines = M1 * M3;
  } else {
    Llog2 = g.L1; es = M2 * M3; inner_cnt = M2 * M3; inner_stride = 1; outer = 0; nlines = M2 * M3;
  }
  L = 1 << Llog2;
  if (L == 1) return hipSuccess;
  int gb = 1;
  while (gb * 2 * L <= 4096 && gb * 2 <= 64) gb *= 2;      // <= 64 KiB of LDS
  const int threads = min(1024, max(64, (gb * L + kMaxV - 1) / kMaxV));
  const long blocks = (nlines + gb - 1) / gb;
  hipLaunchKernelGGL(k_fft_lines, dim3((unsigned)blocks), dim3(threads), (size_t)gb * L * sizeof(double2), s, F,
                     Llog2, es, inner_cnt, inner_stride, outer, nlines, gb, tw);
  return hipGetLastError();
}

hipError_t launch_spectrum(const Geom& g, const double2* table_dev, double2* full_tmp, double2* goct64,
                           float2* goct32, const double2* const tw64[3], hipStream_t s) {
  static const int comp_ab[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  const double invP = 1.0 / ((double)g.M1 * g.M2 * g.M3);
  hipError_t e;
  for (int c = 0; c < 6; ++c) {
    hipLaunchKernelGGL(k_embed, dim3(2048), dim3(256), 0, s, table_dev, full_tmp, g, c, comp_ab[c][0],
                       comp_ab[c][1]);
    if ((e = hipGetLastError())) return e;
    for (int axis = 2; axis >= 0; --axis)
      if ((e = fft_axis(full_tmp, g, axis, tw64[axis], s))) return e;
    hipLaunchKernelGGL(k_octant, dim3(1024), dim3(256), 0, s, full_tmp, goct64, goct32, g, c, 6, invP);
    if ((e = hipGetLastError())) return e;
  }
  return hipSuccess;
}

// The spectrum of K = curl S (JM-VIE) on the same octant: components (0,1), (0,2),
// (1,2), each odd along its third axis c (k_embed with parities (c, none)).
hipError_t launch_curl_spectrum(const Geom& g, const double2* ktable_dev, double2* full_tmp, double2* koct64,
                                float2* koct32, const double2* const tw64[3], hipStream_t s) {
  static const int odd_axis[3] = {2, 1, 0};
  const double invP = 1.0 / ((double)g.M1 * g.M2 * g.M3);
  hipError_t e;
  for (int c = 0; c < 3; ++c) {
    hipLaunchKernelGGL(k_embed, dim3(2048), dim3(256), 0, s, ktable_dev, full_tmp, g, c, odd_axis[c], -1);
    if ((e = hipGetLastError())) return e;
    for (int axis = 2; axis >= 0; --axis)
      if ((e = fft_axis(full_tmp, g, axis, tw64[axis], s))) return e;
    hipLaunchKernelGGL(k_octant, dim3(1024), dim3(256), 0, s, full_tmp, koct64, koct32, g, c, 3, invP);
    if ((e = hipGetLastError())) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ contrast and rhs

// chi = (eps_r - 1)/eps_r = 1 - eps_b/eps (Section III multiplier, background scaled to 1)
__global__ void k_contrast(const double2* __restrict__ eps, long N, double eps_b, double2* __restrict__ chi64,
                           float2* __restrict__ chi32, int* bad) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    const double2 e = eps[i];
    double2 c = {0.0, 0.0};
    const double m2 = e.x * e.x + e.y * e.y;
    if (!isfinite(e.x) || !isfinite(e.y) || m2 == 0.0) {
      atomicOr(bad, 1);
    } else if (!(e.x == eps_b && e.y == 0.0)) {
      // 1 - eps_b * conj(e) / |e|^2
      c.x = 1.0 - eps_b * e.x / m2;
      c.y = eps_b * e.y / m2;
    }
    chi64[i] = c;
    if (chi32) chi32[i] = float2{(float)c.x, (float)c.y};
  }
}

hipError_t launch_contrast(long N, const double2* eps, double eps_b, double2* chi64, float2* chi32, int* bad,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_contrast, dim3(1024), dim3(256), 0, s, eps, N, eps_b, chi64, chi32, bad);
  return hipGetLastError();
}

__global__ void k_rhs(long N, double scale, const double2* __restrict__ chi, const double2* einc,
                      double2* b) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < 3 * N; i += (long)gridDim.x * blockDim.x) {
    const double2 c = chi[i % N];
    const double2 e = einc[i];
    b[i] = double2{scale * (c.x * e.x - c.y * e.y), scale * (c.x * e.y + c.y * e.x)};
  }
}

hipError_t launch_rhs(long N, double scale, const double2* chi, const double2* einc, double2* b, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs, dim3(1024), dim3(256), 0, s, N, scale, chi, einc, b);
  return hipGetLastError();
}

}  // namespace vie
