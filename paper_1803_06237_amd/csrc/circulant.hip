// Block-circulant preconditioner of I - M_eps N along the guide axis
// (Section V-D; Chan and Olkin's construction for Toeplitz-block matrices).
//
// Restricted to the support of the contrast -- the voxel columns S where chi
// is non-zero on some slice (m = 3|S| unknowns per slice) and a window of P
// slices from z0 covering every slice where it is non-zero (P the smallest
// 2,3,5-smooth length >= that extent, at most n3) -- the operator has blocks
// A_{ij} = delta_ij I - D_i N_{i-j} between window slices i and j.  The block
// circulant nearest in the Frobenius norm averages each wrapped diagonal:
//
//   W_k = delta_k0 I - (1/P) [ U_k N_k + (U_0 - U_k) N_{k-P} ],
//   U_k = diag(sum_{i >= k} chi(p, z0 + i))  (suffix sums of the contrast),
//
// and the DFT along the window block-diagonalises it: W^ f = sum_k W_k w^{fk},
// w = exp(-2 pi i / P).  Every other voxel keeps the identity.
//
// Set-up (FP64): the blocks W_k as n3-long sequences per matrix entry, a
// mixed-radix Stockham FFT of every sequence, then a batched blocked
// Gauss-Jordan inversion with partial pivoting of the n3 dense m x m blocks
// (panel of nb columns factored in LDS, the rest of the matrix updated by a
// rank-nb product, columns unscrambled at the end).  The inverses are kept in
// FP64 or FP32.
//
// Apply (z = W^{-1} r): per support row a length-n3 FFT read straight from the
// voxel vector, one m x m matrix-vector product per frequency, the inverse FFT
// written straight back; voxels outside S are copied.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "fft_device.hpp"
#include "vie.h"
#include "vie_internal.hpp"

namespace vie {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxRadices = 24;
constexpr int kGemvRows = 64;

struct Radices {
  int n;
  int count;
  int r[kMaxRadices];
};

int smooth_length(int n) {
  for (int m = n < 1 ? 1 : n;; ++m) {
    int v = m;
    for (int p : {2, 3, 5})
      while (v % p == 0) v /= p;
    if (v == 1) return m;
  }
}

Radices factor(int n) {
  Radices rd{};
  rd.n = n;
  int v = n;
  for (int r : {8, 4, 2})
    while (v % r == 0 && v > 1) {
      rd.r[rd.count++] = r;
      v /= r;
    }
  for (int p = 3; v > 1; p += 2)
    while (v % p == 0) {
      rd.r[rd.count++] = p;
      v /= p;
    }
  return rd;
}

__device__ __forceinline__ int comp_index(int a, int b) {
  // xx, xy, xz, yy, yz, zz
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
}

// ---- W_k, stored as Wt[e][k] with e = col * m + row (k < P; table offsets < n3) ----
__global__ __launch_bounds__(kThreads) void k_circ_blocks(double2* __restrict__ Wt, const double2* __restrict__ table,
                                                          const int2* __restrict__ S, const double2* __restrict__ ucum,
                                                          int s, int n1, int n2, int n3, int P, long total) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int k = (int)(idx % P);
  const long e = idx / P;
  const int m = 3 * s;
  const int row = (int)(e % m), col = (int)(e / m);
  const int a = row / s, p = row % s, b = col / s, q = col % s;
  const int2 sp = S[p], sq = S[q];
  const int d1 = sp.x - sq.x, d2 = sp.y - sq.y;
  double sg = 1.0;
  if (d1 < 0 && ((a == 0) != (b == 0))) sg = -sg;   // parity of N^{ab} along axis 1
  if (d2 < 0 && ((a == 1) != (b == 1))) sg = -sg;   // along axis 2
  const long base = (((long)comp_index(a, b) * n1 + abs(d1)) * n2 + abs(d2)) * n3;
  const double2 up = ucum[(long)p * (P + 1) + k];
  double2 acc = cmul(up, table[base + k]);
  if (k > 0) {
    const double2 tot = ucum[(long)p * (P + 1)];
    const double s3 = ((a == 2) != (b == 2)) ? -1.0 : 1.0;   // offset k - P < 0 along axis 3
    acc = cadd(acc, cscale(cmul(csub(tot, up), table[base + P - k]), s3));
  }
  double2 w = cscale(acc, -sg / P);
  if (k == 0 && row == col) w.x += 1.0;
  Wt[idx] = w;
}

// ---- length-n FFT of one sequence per workgroup (mixed radix Stockham) -----
// Stage with radix R after Ns = product of earlier radices: output q of task
// j < n/R is sum_r x[j + r n/R] w^{r ((j mod Ns) n/(Ns R) + q n/R)}, written to
// (j / Ns) Ns R + (j mod Ns) + q Ns.  Natural order after the last stage.
// Window slices t < P of a support row start at z0 of a voxel column; the
// transform rows are [seq][P].
template <typename T>
struct IoVoxelIn {   // FP64 voxel vector (through the support map) -> rows[seq][t]
  const double2* r;
  cx<T>* rows;
  const int* col;
  int s;
  long n12;
  int n3, z0, P;
  __device__ cx<T> load(long seq, int t) const {
    const int a = (int)(seq / s), p = (int)(seq % s);
    const double2 v = r[((long)a * n12 + col[p]) * n3 + z0 + t];
    return cx<T>{(T)v.x, (T)v.y};
  }
  __device__ void store(long seq, int t, cx<T> v) const { rows[seq * P + t] = v; }
};

template <typename T>
struct IoVoxelOut {  // rows[seq][t] -> FP64 voxel vector (through the support map)
  const cx<T>* rows;
  double2* z;
  const int* col;
  int s;
  long n12;
  int n3, z0, P;
  __device__ cx<T> load(long seq, int t) const { return rows[seq * P + t]; }
  __device__ void store(long seq, int t, cx<T> v) const {
    const int a = (int)(seq / s), p = (int)(seq % s);
    z[((long)a * n12 + col[p]) * n3 + z0 + t] = double2{(double)v.x, (double)v.y};
  }
};

template <typename T>
struct IoRowsIn {    // FP64 support-compressed vector (rows of n3 slices) -> rows of T
  const double2* r;
  cx<T>* rows;
  int n3, z0, P;
  __device__ cx<T> load(long seq, int t) const {
    const double2 v = r[seq * n3 + z0 + t];
    return cx<T>{(T)v.x, (T)v.y};
  }
  __device__ void store(long seq, int t, cx<T> v) const { rows[seq * P + t] = v; }
};

template <typename T>
struct IoRowsOut {   // rows of T -> FP64 support-compressed vector
  const cx<T>* rows;
  double2* z;
  int n3, z0, P;
  __device__ cx<T> load(long seq, int t) const { return rows[seq * P + t]; }
  __device__ void store(long seq, int t, cx<T> v) const {
    z[seq * n3 + z0 + t] = double2{(double)v.x, (double)v.y};
  }
};

struct IoBlocks {    // Wt[e][k] -> What[f][e]
  const double2* Wt;
  double2* Wh;
  long m2;
  int P;
  __device__ double2 load(long seq, int t) const { return Wt[seq * P + t]; }
  __device__ void store(long seq, int t, double2 v) const { Wh[(long)t * m2 + seq] = v; }
};

template <typename T, bool INV, class IO>
__global__ __launch_bounds__(kThreads) void k_circ_fft(Radices rd, const double2* __restrict__ tw_g, IO io,
                                                       long count, T scale) {
  extern __shared__ unsigned char smem_raw[];
  using C = cx<T>;
  const long seq = blockIdx.x;
  if (seq >= count) return;
  const int n = rd.n;
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* src = tw + n;
  C* dst = src + n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const double2 w = tw_g[t];
    tw[t] = C{(T)w.x, (T)(INV ? -w.y : w.y)};
    src[t] = io.load(seq, t);
  }
  __syncthreads();
  int Ns = 1;
  for (int st = 0; st < rd.count; ++st) {
    const int R = rd.r[st];
    const int L = n / R;
    const int str = L / Ns;
    for (int item = threadIdx.x; item < n; item += blockDim.x) {
      const int j = item % L, q = item / L;
      const int jm = j % Ns;
      int step = jm * str + q * L;
      if (step >= n) step -= n;
      C acc{0, 0};
      int ti = 0;
      for (int r = 0; r < R; ++r) {
        acc = cadd(acc, cmul(src[j + r * L], tw[ti]));
        ti += step;
        if (ti >= n) ti -= n;
      }
      dst[(j / Ns) * Ns * R + jm + q * Ns] = acc;
    }
    __syncthreads();
    C* t_ = src;
    src = dst;
    dst = t_;
    Ns *= R;
  }
  for (int t = threadIdx.x; t < n; t += blockDim.x) io.store(seq, t, cscale(src[t], scale));
}

// ---- blocked Gauss-Jordan inversion, one m x m column-major matrix per f ----
// Panel: columns [j, j+nb) of all m rows in LDS.  Each step k = j + jj picks
// the largest |.| in column jj among rows >= k, swaps it to row k, and applies
// the in-place Gauss-Jordan step to the panel: the pivot row is divided by the
// pivot, every other row loses its multiple of it, and column jj receives the
// corresponding column of the accumulated transformation.
__global__ __launch_bounds__(kThreads) void k_gj_panel(double2* __restrict__ A, int m, int j, int nb,
                                                       int* __restrict__ piv, int* __restrict__ bad) {
  extern __shared__ unsigned char smem_raw[];
  double2* P = reinterpret_cast<double2*>(smem_raw);   // P[c * m + r]
  __shared__ double red_v[kThreads / 64];
  __shared__ int red_i[kThreads / 64];
  __shared__ int s_p;
  const long f = blockIdx.x;
  double2* Af = A + f * (long)m * m;
  const int w = min(nb, m - j);
  for (int i = threadIdx.x; i < w * m; i += blockDim.x) P[i] = Af[(long)j * m + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int jj = 0; jj < w; ++jj) {
    const int k = j + jj;
    // pivot: largest squared magnitude, lowest row on ties
    double bv = -1.0;
    int bi = m;
    for (int r = k + threadIdx.x; r < m; r += blockDim.x) {
      const double2 v = P[jj * m + r];
      const double a2 = v.x * v.x + v.y * v.y;
      if (a2 > bv) {
        bv = a2;
        bi = r;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[wave] = bv;
      red_i[wave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = red_v[0];
      int i = red_i[0];
      for (int q = 1; q < kThreads / 64; ++q)
        if (red_v[q] > v || (red_v[q] == v && red_i[q] < i)) {
          v = red_v[q];
          i = red_i[q];
        }
      if (!(v > 0.0)) {
        bad[0] = 1;     // singular block (or non-finite): reported by the host
        i = k;
      }
      s_p = i;
      piv[f * m + k] = i;
    }
    __syncthreads();
    const int p = s_p;
    if (p != k)
      for (int c = threadIdx.x; c < w; c += blockDim.x) {
        const double2 t = P[c * m + k];
        P[c * m + k] = P[c * m + p];
        P[c * m + p] = t;
      }
    __syncthreads();
    double2 d = P[jj * m + k];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 ck = dd > 0.0 ? double2{d.x / dd, -d.y / dd} : double2{1.0, 0.0};
    // rows r = threadIdx.x + t * kThreads owned by this thread (t compile-time, so
    // the cache stays in registers); pivot-column values read before the barrier
    constexpr int kMaxRows = 2048 / kThreads;
    double2 fr[kMaxRows];
#pragma unroll
    for (int t = 0; t < kMaxRows; ++t) {
      const int r = threadIdx.x + t * kThreads;
      fr[t] = r < m ? P[jj * m + r] : double2{0.0, 0.0};
    }
    __syncthreads();
    for (int c = 0; c < w; ++c) {
      const double2 rk = c == jj ? ck : cmul(P[c * m + k], ck);
#pragma unroll
      for (int t = 0; t < kMaxRows; ++t) {
        const int r = threadIdx.x + t * kThreads;
        if (r >= m || r == k) continue;
        const double2 fv = fr[t];
        if (c == jj)
          P[c * m + r] = double2{-(fv.x * ck.x - fv.y * ck.y), -(fv.x * ck.y + fv.y * ck.x)};
        else
          P[c * m + r] = csub(P[c * m + r], cmul(fv, rk));
      }
    }
    __syncthreads();
    // pivot row last (its old values fed every other row)
    if (threadIdx.x < w) {
      const int c = threadIdx.x;
      P[c * m + k] = c == jj ? ck : cmul(P[c * m + k], ck);
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < w * m; i += blockDim.x) Af[(long)j * m + i] = P[i];
}

// Columns c in [cb, ce) outside the panel [j, j + w), 64 per workgroup: apply the
// panel's row swaps, then A[:, c] = (rows of the panel zeroed) + T[:, panel] *
// A[panel rows, c], with T the panel's in-place Gauss-Jordan columns.
template <int NB>
__global__ __launch_bounds__(kThreads) void k_gj_update(double2* __restrict__ A, int m, int j,
                                                        const int* __restrict__ piv, int cb, int ce) {
  __shared__ double2 B[NB][64];
  __shared__ int s_piv[NB];
  const long f = blockIdx.y;
  double2* Af = A + f * (long)m * m;
  const int w = min(NB, m - j);
  const int c0 = cb + blockIdx.x * 64;
  if (threadIdx.x < w) s_piv[threadIdx.x] = piv[f * m + j + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int c = c0 + threadIdx.x;
    const bool own = c < ce && (c < j || c >= j + w);
    if (own) {
      double2* col = Af + (long)c * m;
      for (int jj = 0; jj < w; ++jj) {
        const int k = j + jj, p = s_piv[jj];
        if (p != k) {
          const double2 t = col[k];
          col[k] = col[p];
          col[p] = t;
        }
      }
      for (int jj = 0; jj < w; ++jj) B[jj][threadIdx.x] = col[j + jj];
    } else {
      for (int jj = 0; jj < w; ++jj) B[jj][threadIdx.x] = double2{0.0, 0.0};
    }
  }
  __syncthreads();
  const int ncol = min(64, ce - c0);
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    double2 tr[NB];
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) tr[jj] = jj < w ? Af[(long)(j + jj) * m + r] : double2{0.0, 0.0};
    const bool in_panel_row = r >= j && r < j + w;
    for (int t = 0; t < ncol; ++t) {
      const int c = c0 + t;
      if (c >= j && c < j + w) continue;
      double2 acc = in_panel_row ? double2{0.0, 0.0} : Af[(long)c * m + r];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const double2 b = B[jj][t];
        acc.x += tr[jj].x * b.x - tr[jj].y * b.y;
        acc.y += tr[jj].x * b.y + tr[jj].y * b.x;
      }
      Af[(long)c * m + r] = acc;
    }
  }
}

// Undo the row interchanges on the inverse: swap columns k and piv[k], k descending.
__global__ __launch_bounds__(kThreads) void k_gj_unscramble(double2* __restrict__ A, int m,
                                                            const int* __restrict__ piv) {
  const long f = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  double2* Af = A + f * (long)m * m;
  const int* pf = piv + f * m;
  for (int k = m - 1; k >= 0; --k) {
    const int p = pf[k];
    if (p != k) {
      const double2 t = Af[(long)k * m + r];
      Af[(long)k * m + r] = Af[(long)p * m + r];
      Af[(long)p * m + r] = t;
    }
  }
}

__global__ void k_to_c64(const double2* __restrict__ a, float2* __restrict__ b, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = float2{(float)a[i].x, (float)a[i].y};
}

// ---- apply: one m x m product per frequency ---------------------------------
// yhat[row][f] = sum_j inv[f][j][row] xhat[j][f]; a workgroup owns 64 rows of one
// frequency, its four waves split j and add their partial sums in LDS.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_circ_gemv(const cx<T>* __restrict__ inv, const cx<T>* __restrict__ xhat,
                                                        cx<T>* __restrict__ yhat, int m, int n3) {
  __shared__ cx<T> xs[2048];
  __shared__ cx<T> part[kThreads / 64][64];
  const int f = blockIdx.y;
  for (int j = threadIdx.x; j < m; j += blockDim.x) xs[j] = xhat[(long)j * n3 + f];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = blockIdx.x * kGemvRows + lane;
  const int per = (m + 3) / 4;
  const int j0 = wave * per, j1 = min(m, j0 + per);
  T ax = 0, ay = 0;
  if (row < m) {
    const cx<T>* col = inv + (long)f * m * m + row;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
      const cx<T> a = col[(long)j * m];
      const cx<T> x = xs[j];
      ax += a.x * x.x - a.y * x.y;
      ay += a.x * x.y + a.y * x.x;
    }
  }
  part[wave][lane] = cx<T>{ax, ay};
  __syncthreads();
  if (wave == 0 && row < m) {
    cx<T> acc = part[0][lane];
    for (int q = 1; q < kThreads / 64; ++q) acc = cadd(acc, part[q][lane]);
    yhat[(long)row * n3 + f] = acc;
  }
}

template <typename T, bool INV, class IO>
hipError_t launch_fft(const Radices& rd, const double2* tw, const IO& io, long count, double scale, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t lds = 3 * (size_t)rd.n * sizeof(cx<T>);
  hipLaunchKernelGGL((k_circ_fft<T, INV, IO>), dim3((unsigned)count), dim3(kThreads), lds, s, rd, tw, io, count,
                     (T)scale);
  return hipGetLastError();
}

template <int NB>
hipError_t launch_update(double2* A, int m, int j, const int* piv, int cb, int ce, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_update<NB>, dim3((ce - cb + 63) / 64, nblk), dim3(kThreads), 0, s, A, m, j, piv, cb, ce);
  return hipGetLastError();
}

hipError_t launch_update_w(int nbw, double2* A, int m, int j, const int* piv, int cb, int ce, int nblk,
                           hipStream_t s) {
  switch (nbw) {
    case 32: return launch_update<32>(A, m, j, piv, cb, ce, nblk, s);
    case 16: return launch_update<16>(A, m, j, piv, cb, ce, nblk, s);
    case 8: return launch_update<8>(A, m, j, piv, cb, ce, nblk, s);
    default: return launch_update<4>(A, m, j, piv, cb, ce, nblk, s);
  }
}

}  // namespace

struct Circ {
  int s = 0, m = 0, n1 = 0, n2 = 0, n3 = 0;
  int z0 = 0, P = 0;           // slice window of the circulant
  bool fp64 = false;
  int* col = nullptr;          // voxel column i1 * n2 + i2 of each support column
  double2* tw = nullptr;       // exp(-2 pi i t / P)
  double2* inv64 = nullptr;    // P blocks, column-major m x m
  float2* inv32 = nullptr;
  void* xhat = nullptr;        // m x P rows of the apply precision
  void* yhat = nullptr;
  Radices rd{};
  CircInfo info{};
};

void circ_destroy(Circ* c) {
  if (!c) return;
  for (void* q : {(void*)c->col, (void*)c->tw, (void*)c->inv64, (void*)c->inv32, c->xhat, c->yhat})
    if (q) (void)hipFree(q);
  delete c;
}

int circ_build(Circ** out, const Geom& g, const std::complex<double>* table, const double2* chi64, bool fp64,
               hipStream_t s, std::string& err, CircInfo* info) {
  const auto t0 = std::chrono::steady_clock::now();
  *out = nullptr;
  auto* c = new Circ();
  c->n1 = g.n1;
  c->n2 = g.n2;
  c->n3 = g.n3;
  c->fp64 = fp64;
  std::vector<void*> tmp;
  auto finish = [&](int code, const std::string& msg) {
    for (void* q : tmp)
      if (q) (void)hipFree(q);
    if (code != VIE_OK) {
      err = msg;
      circ_destroy(c);
    } else {
      *out = c;
    }
    return code;
  };
#define CTRY(...)                                                           \
  do {                                                                      \
    hipError_t _e = (__VA_ARGS__);                                                 \
    if (_e != hipSuccess) return finish(VIE_EDEVICE, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(_e)); \
  } while (0)
  const long n12 = (long)g.n1 * g.n2;
  const int n3 = g.n3;
  std::vector<double2> chi((size_t)g.N);
  CTRY(hipMemcpyAsync(chi.data(), chi64, sizeof(double2) * g.N, hipMemcpyDeviceToHost, s));
  CTRY(hipStreamSynchronize(s));
  std::vector<int2> S;
  std::vector<int> cols;
  for (int i1 = 0; i1 < g.n1; ++i1)
    for (int i2 = 0; i2 < g.n2; ++i2) {
      const double2* z = chi.data() + ((long)i1 * g.n2 + i2) * n3;
      bool any = false;
      for (int k = 0; k < n3 && !any; ++k) any = z[k].x != 0.0 || z[k].y != 0.0;
      if (any) {
        S.push_back(int2{i1, i2});
        cols.push_back(i1 * g.n2 + i2);
      }
    }
  c->s = (int)S.size();
  c->m = 3 * c->s;
  const int m = c->m;
  c->info.s = c->s;
  c->info.m = m;
  c->info.fp64 = fp64 ? 1 : 0;
  if (c->s == 0) {
    c->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = c->info;
    return finish(VIE_OK, "");
  }
  if (m > 2048) return finish(VIE_EINVAL, "contrast support wider than 682 voxel columns");
  // slice window: every slice where chi is non-zero on S, grown to a 2,3,5-smooth length
  int first = n3, last = -1;
  for (int p = 0; p < c->s; ++p) {
    const double2* z = chi.data() + (long)cols[p] * n3;
    for (int k = 0; k < n3; ++k)
      if (z[k].x != 0.0 || z[k].y != 0.0) {
        first = std::min(first, k);
        last = std::max(last, k);
      }
  }
  int P = smooth_length(last - first + 1);
  int z0 = std::min(first, n3 - P);
  if (P > n3) {
    P = n3;
    z0 = 0;
  }
  c->z0 = z0;
  c->P = P;
  c->info.z0 = z0;
  c->info.P = P;
  const long m2 = (long)m * m;
  const size_t blk = sizeof(double2) * (size_t)P * m2;
  size_t free_b = 0, total_b = 0;
  CTRY(hipMemGetInfo(&free_b, &total_b));
  const size_t need = 2 * blk + (fp64 ? 0 : blk / 2);
  if (need > free_b / 10 * 9) return finish(VIE_ENOMEM, "preconditioner blocks exceed free device memory");
  c->rd = factor(P);
  // suffix sums of the contrast over the window per support column: U_k, k = 0..P
  std::vector<double2> ucum((size_t)c->s * (P + 1));
  for (int p = 0; p < c->s; ++p) {
    const double2* z = chi.data() + (long)cols[p] * n3 + z0;
    double ax = 0, ay = 0;
    double2* u = ucum.data() + (size_t)p * (P + 1);
    u[P] = double2{0, 0};
    for (int k = P - 1; k >= 0; --k) {
      ax += z[k].x;
      ay += z[k].y;
      u[k] = double2{ax, ay};
    }
  }
  std::vector<double2> tw(P);
  for (int t = 0; t < P; ++t) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * t / P;
    tw[t] = double2{(double)std::cos(a), (double)std::sin(a)};
  }
  int2* S_d = nullptr;
  double2* ucum_d = nullptr;
  double2* table_d = nullptr;
  double2* Wt = nullptr;
  double2* Wh = nullptr;
  int* piv = nullptr;
  int* bad = nullptr;
  CTRY(dmalloc(&c->col, sizeof(int) * c->s));
  CTRY(dmalloc(&c->tw, sizeof(double2) * P));
  CTRY(dmalloc(&S_d, sizeof(int2) * c->s));
  tmp.push_back(S_d);
  CTRY(dmalloc(&ucum_d, sizeof(double2) * ucum.size()));
  tmp.push_back(ucum_d);
  CTRY(dmalloc(&table_d, sizeof(double2) * 6 * g.N));
  tmp.push_back(table_d);
  CTRY(dmalloc(&Wt, blk));
  tmp.push_back(Wt);
  CTRY(hipMemcpyAsync(c->col, cols.data(), sizeof(int) * c->s, hipMemcpyHostToDevice, s));
  CTRY(hipMemcpyAsync(c->tw, tw.data(), sizeof(double2) * P, hipMemcpyHostToDevice, s));
  CTRY(hipMemcpyAsync(S_d, S.data(), sizeof(int2) * c->s, hipMemcpyHostToDevice, s));
  CTRY(hipMemcpyAsync(ucum_d, ucum.data(), sizeof(double2) * ucum.size(), hipMemcpyHostToDevice, s));
  CTRY(hipMemcpyAsync(table_d, table, sizeof(double2) * 6 * g.N, hipMemcpyHostToDevice, s));
  const long total = (long)P * m2;
  hipLaunchKernelGGL(k_circ_blocks, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, Wt,
                     table_d, S_d, ucum_d, c->s, g.n1, g.n2, n3, P, total);
  CTRY(hipGetLastError());
  CTRY(dmalloc(&Wh, blk));
  tmp.push_back(Wh);
  const size_t wh_slot = tmp.size() - 1;
  CTRY(hipFuncSetAttribute((const void*)k_circ_fft<double, false, IoBlocks>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)(3 * (size_t)P * sizeof(double2))));
  CTRY(launch_fft<double, false>(c->rd, c->tw, IoBlocks{Wt, Wh, m2, P}, m2, 1.0, s));
  CTRY(hipStreamSynchronize(s));
  CTRY(hipFree(Wt));
  tmp[3] = nullptr;
  CTRY(hipFree(table_d));
  tmp[2] = nullptr;
  // Gauss-Jordan on every frequency block
  CTRY(dmalloc(&piv, sizeof(int) * (size_t)P * m));
  tmp.push_back(piv);
  CTRY(dmalloc(&bad, sizeof(int)));
  tmp.push_back(bad);
  CTRY(hipMemsetAsync(bad, 0, sizeof(int), s));
  const int nb = m <= 600 ? 16 : (m <= 1200 ? 8 : 4);
  const size_t panel_lds = sizeof(double2) * (size_t)m * nb;
  CTRY(hipFuncSetAttribute((const void*)k_gj_panel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)panel_lds));
  // two-level panels: 2 nb columns at a time; each nb-column sub-panel is factored in
  // LDS and applied to the other columns of the outer panel, then the outer panel's
  // composite transformation goes to the rest of the matrix in one rank-2nb pass
  const int nb2 = 2 * nb;
  for (int J = 0; J < m; J += nb2) {
    const int wJ = std::min(nb2, m - J);
    for (int j = J; j < J + wJ; j += nb) {
      hipLaunchKernelGGL(k_gj_panel, dim3(P), dim3(kThreads), panel_lds, s, Wh, m, j, nb, piv, bad);
      CTRY(hipGetLastError());
      if (wJ > nb) CTRY(launch_update_w(nb, Wh, m, j, piv, J, J + wJ, P, s));
    }
    CTRY(launch_update_w(nb2, Wh, m, J, piv, 0, m, P, s));
  }
  hipLaunchKernelGGL(k_gj_unscramble, dim3((m + kThreads - 1) / kThreads, P), dim3(kThreads), 0, s, Wh, m, piv);
  CTRY(hipGetLastError());
  int bad_h = 0;
  CTRY(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  CTRY(hipStreamSynchronize(s));
  if (bad_h) return finish(VIE_ENUMERIC, "a frequency block of the circulant preconditioner is singular");
  const size_t es = fp64 ? sizeof(double2) : sizeof(float2);
  if (fp64) {
    c->inv64 = Wh;
    tmp[wh_slot] = nullptr;
  } else {
    CTRY(dmalloc(&c->inv32, sizeof(float2) * (size_t)P * m2));
    hipLaunchKernelGGL(k_to_c64, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, Wh,
                       c->inv32, total);
    CTRY(hipGetLastError());
    CTRY(hipStreamSynchronize(s));
  }
  CTRY(dmalloc(&c->xhat, es * (size_t)m * P));
  CTRY(dmalloc(&c->yhat, es * (size_t)m * P));
  const int lds_need = (int)(3 * (size_t)P * es);
  const auto attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  if (fp64) {
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<double, false, IoVoxelIn<double>>, attr, lds_need));
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<double, true, IoVoxelOut<double>>, attr, lds_need));
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<double, false, IoRowsIn<double>>, attr, lds_need));
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<double, true, IoRowsOut<double>>, attr, lds_need));
  } else {
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<float, false, IoVoxelIn<float>>, attr, lds_need));
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<float, true, IoVoxelOut<float>>, attr, lds_need));
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<float, false, IoRowsIn<float>>, attr, lds_need));
    CTRY(hipFuncSetAttribute((const void*)k_circ_fft<float, true, IoRowsOut<float>>, attr, lds_need));
  }
  c->info.bytes = (fp64 ? sizeof(double2) : sizeof(float2)) * (size_t)P * m2;
  c->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = c->info;
  return finish(VIE_OK, "");
#undef CTRY
}

namespace {
// forward FFT of every support row, one product per frequency, inverse FFT
template <typename T, class IN, class OUT>
hipError_t apply_t(Circ* c, const cx<T>* inv, const IN& in, const OUT& out, hipStream_t s) {
  auto* xh = reinterpret_cast<cx<T>*>(c->xhat);
  auto* yh = reinterpret_cast<cx<T>*>(c->yhat);
  hipError_t e = launch_fft<T, false>(c->rd, c->tw, in, c->m, 1.0, s);
  if (e) return e;
  hipLaunchKernelGGL(k_circ_gemv<T>, dim3((c->m + kGemvRows - 1) / kGemvRows, c->P), dim3(kThreads), 0, s, inv, xh,
                     yh, c->m, c->P);
  if ((e = hipGetLastError())) return e;
  return launch_fft<T, true>(c->rd, c->tw, out, c->m, 1.0 / c->P, s);
}

template <typename T>
hipError_t apply_voxels(Circ* c, const cx<T>* inv, const double2* r, double2* z, hipStream_t s) {
  const long n12 = (long)c->n1 * c->n2;
  auto* xh = reinterpret_cast<cx<T>*>(c->xhat);
  auto* yh = reinterpret_cast<cx<T>*>(c->yhat);
  return apply_t<T>(c, inv, IoVoxelIn<T>{r, xh, c->col, c->s, n12, c->n3, c->z0, c->P},
                    IoVoxelOut<T>{yh, z, c->col, c->s, n12, c->n3, c->z0, c->P}, s);
}

template <typename T>
hipError_t apply_rows(Circ* c, const cx<T>* inv, const double2* r, double2* z, hipStream_t s) {
  auto* xh = reinterpret_cast<cx<T>*>(c->xhat);
  auto* yh = reinterpret_cast<cx<T>*>(c->yhat);
  return apply_t<T>(c, inv, IoRowsIn<T>{r, xh, c->n3, c->z0, c->P}, IoRowsOut<T>{yh, z, c->n3, c->z0, c->P}, s);
}
}  // namespace

hipError_t circ_apply(Circ* c, const double2* r, double2* z, hipStream_t s) {
  const long n = 3 * (long)c->n1 * c->n2 * c->n3;
  hipError_t e = hipMemcpyAsync(z, r, sizeof(double2) * n, hipMemcpyDeviceToDevice, s);
  if (e || c->s == 0) return e;
  return c->fp64 ? apply_voxels<double>(c, c->inv64, r, z, s) : apply_voxels<float>(c, c->inv32, r, z, s);
}

hipError_t circ_apply_rows(Circ* c, const double2* r, double2* z, hipStream_t s) {
  if (c->s == 0) return hipSuccess;
  if (c->P < c->n3) {   // slices outside the window keep the identity
    const hipError_t e = hipMemcpyAsync(z, r, sizeof(double2) * 3 * (size_t)c->s * c->n3, hipMemcpyDeviceToDevice, s);
    if (e) return e;
  }
  return c->fp64 ? apply_rows<double>(c, c->inv64, r, z, s) : apply_rows<float>(c, c->inv32, r, z, s);
}

const CircInfo& circ_info(const Circ* c) { return c->info; }

}  // namespace vie
