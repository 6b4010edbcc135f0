// Device building blocks for power-of-two FFTs on gfx950: complex helpers,
// radix-2/4/8 butterflies and one Stockham (self-sorting) stage that works on
// a batch of sequences resident in LDS.
//
// Stage convention for a length-L transform built from radices R_1..R_S, with
// Ns the product of the radices already applied (Ns = 1 at the first stage):
// task j in [0, L/R) reads x[j + r L/R], r < R, multiplies element r by
// W^{r (j mod Ns)} with W = exp(-+2 pi i / (Ns R)), applies the R-point DFT and
// writes element r to (j / Ns) Ns R + (j mod Ns) + r Ns.  After the last stage
// the sequence is in natural order.  Every stage is in place: all reads happen
// before a barrier, all writes after it.
#pragma once
#include <hip/hip_runtime.h>

namespace vie {

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename T> using cx = typename cplx_of<T>::type;

// Pointer into global memory.  Device functions that batched kernels share take
// their arrays in this form: a pointer read from device memory (a batch
// descriptor) has no address space, so accesses through it would compile to flat
// loads and stores, which the compiler must also order against LDS traffic.
// (The host pass only type-checks device code, without address spaces.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename P> using gptr = __attribute__((address_space(1))) P*;
#else
template <typename P> using gptr = P*;
#endif

// The thread index as a value the compiler cannot see through.  Persistent
// kernels take it once per work item: otherwise every thread-dependent LDS and
// global address of the body is hoisted out of the item loop and held in
// registers across it (about a hundred VGPRs).
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// conj(a) * b
template <typename V> __device__ __forceinline__ V cconjmul(V a, V b) {
  return V{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(a.x) s) { return V{a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V> __device__ __forceinline__ V rot90(V a) {
  return INV ? V{-a.y, a.x} : V{a.y, -a.x};
}

template <typename T, bool INV> __device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  cx<T> t2 = cadd(v[1], v[3]), t3 = rot90<INV>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(cx<T>* v) {
  // even/odd split into two 4-point DFTs, then W8^k combination
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const T r = (T)0.70710678118654752440;
  // W8^1 = (1 -+ i)/sqrt2, W8^2 = -+i, W8^3 = (-1 -+ i)/sqrt2
  cx<T> o1 = INV ? cx<T>{(o[1].x - o[1].y) * r, (o[1].x + o[1].y) * r}
                 : cx<T>{(o[1].x + o[1].y) * r, (o[1].y - o[1].x) * r};
  cx<T> o2 = rot90<INV>(o[2]);
  cx<T> o3 = INV ? cx<T>{(-o[3].x - o[3].y) * r, (o[3].x - o[3].y) * r}
                 : cx<T>{(o[3].y - o[3].x) * r, (-o[3].x - o[3].y) * r};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else dft8<T, INV>(v);
}

// Addressing of a batch of sequences in LDS: sequence s starts at
// (s >> inner_log2) * outer + (s & (inner - 1)) * inner_stride, element k at + k * es.
struct SeqMap {
  int inner_log2;
  int inner_stride;
  int outer;
  int es;
  __device__ __forceinline__ int base(int s) const {
    return (s >> inner_log2) * outer + (s & ((1 << inner_log2) - 1)) * inner_stride;
  }
};

// One Stockham stage of radix R over nseq sequences of length L = 2^Llog2.
// valid: elements with index >= valid are taken as zero (zero-padded input).
// tw: forward twiddle table exp(-2 pi i k / Ltw), k < Ltw, Ltw = L * twstride.
// MAXV bounds the values each thread holds (nseq * L <= MAXV * blockDim.x).
template <typename T, int R, bool INV, int MAXV>
__device__ __forceinline__ void stockham_stage(cx<T>* buf, SeqMap map, int nseq, int Llog2, int Nslog2,
                                               int valid, const cx<T>* __restrict__ tw, int twstride) {
  constexpr int TPT = MAXV / R;
  constexpr int Rlog2 = R == 2 ? 1 : (R == 4 ? 2 : 3);
  const int perlog2 = Llog2 - Rlog2;      // tasks per sequence = L / R
  const int per = 1 << perlog2;
  const int total = nseq << perlog2;
  const int Ns = 1 << Nslog2;
  cx<T> v[TPT][R];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int t = threadIdx.x + q * blockDim.x;
    if (t < total) {
      const int s = t >> perlog2, j = t & (per - 1);
      const int b = map.base(s);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = j + r * per;
        v[q][r] = (k < valid) ? buf[b + k * map.es] : cx<T>{(T)0, (T)0};
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int t = threadIdx.x + q * blockDim.x;
    if (t < total) {
      const int s = t >> perlog2, j = t & (per - 1);
      const int b = map.base(s);
      const int jm = j & (Ns - 1);
      if (Ns > 1) {
        // W^{r jm} with W = exp(-+2 pi i/(Ns R)): table index r*jm*(L/(Ns R))*twstride
        const int step = (1 << (Llog2 - Nslog2 - Rlog2)) * twstride;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * jm * step];
          v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
        }
      }
      dft<T, R, INV>(v[q]);
      const int o = ((j >> Nslog2) << (Nslog2 + Rlog2)) + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[b + (o + (r << Nslog2)) * map.es] = v[q][r];
    }
  }
  __syncthreads();
}

// Full transform of length L = 2^Llog2 in LDS: radix-8 stages, then one radix-4
// or radix-2 stage for the remainder.  Only the first stage reads padded zeros.
template <typename T, bool INV, int MAXV>
__device__ __forceinline__ void fft_lds(cx<T>* buf, SeqMap map, int nseq, int Llog2, int valid,
                                        const cx<T>* __restrict__ tw, int twstride) {
  int Ns = 0;
  int rem = Llog2;
  bool first = true;
  while (rem >= 3) {
    stockham_stage<T, 8, INV, MAXV>(buf, map, nseq, Llog2, Ns, first ? valid : (1 << Llog2), tw, twstride);
    Ns += 3;
    rem -= 3;
    first = false;
  }
  if (rem == 2) stockham_stage<T, 4, INV, MAXV>(buf, map, nseq, Llog2, Ns, first ? valid : (1 << Llog2), tw, twstride);
  else if (rem == 1) stockham_stage<T, 2, INV, MAXV>(buf, map, nseq, Llog2, Ns, first ? valid : (1 << Llog2), tw, twstride);
}

}  // namespace vie
