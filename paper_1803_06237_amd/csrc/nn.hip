// Learned preconditioner: a 4-level 3-D U-Net (channels 16/32/48/64, 3x3x3
// convolutions, bias-free ReLU) that maps a normalised residual r (and the
// contrast chi) to the correction A^{-1} r - r; the preconditioner is
// z = r + net(r).  It is used as the right
// preconditioner of flexible GMRES and as an initial guess, with plain GMRES as
// the fallback.  This part is this library's addition, not the paper's method.
//
// Activations are channels-last bfloat16 [V][C] (V = D H W voxels, W fastest,
// C a multiple of 16, channel stride / offset per view so concatenations are
// written in place).  Convolutions are implicit GEMMs on the matrix cores:
// v_mfma_f32_16x16x16bf16_1k, FP32 accumulation.  Forward: M = voxels, N = Cout,
// K = 27 Cin, operands loaded straight from global memory into MFMA fragments
// (a 16-voxel x 4-channel slab per lane group is one 8-byte load).  Input
// gradient: the same kernel with taps flipped and channels swapped, the ReLU
// mask of the forward input fused into the epilogue.  Weight gradient: split-K
// over voxel chunks with a fixed-order reduction.  Master weights, gradients and
// Adam moments are FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "krylov.hpp"
#include "vie_internal.hpp"

namespace vie {

typedef unsigned short bf16_t;
typedef short s4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16_t f2bf(float f) {   // round to nearest, ties to even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((unsigned)h) << 16); }

struct Vol {
  int D, H, W;
  __host__ __device__ long V() const { return (long)D * H * W; }
};

// ------------------------------------------------------------------ convolution
// Y[v, o] = act(sum_t sum_i W[t][o][i] X[v + t][i]); tap t = (dz+1)*9 + (dy+1)*3 + (dx+1).
// LDS-staged implicit GEMM on v_mfma_f32_16x16x32_bf16.  A workgroup of four waves
// computes a tile of TZ (D) x 4 (H) x 16 MT (W) output voxels for up to 64 output
// channels (grid.y picks the group of NT 16-channel N-tiles).  Wave w takes the
// TZ rows (z0 + (TZ == 2 ? w / 2 : 0), y0 + ...) assigned to it, i.e. TZ * MT / ...
// 16-voxel M-tiles: with TZ = 2, MT = 2 (the 2 x 4 x 32 tile of the large levels)
// four M-tiles per wave; with TZ = 1, MT = 1 (the 1 x 4 x 16 tile that keeps the
// small levels' launches wide) one.  The input is consumed in chunks of 16
// channels: the chunk's halo tile and its weights for all taps and the group's
// output channels are staged in LDS once and read by every K-step.  One MFMA
// K-step covers two taps of the chunk (K = 2 x 16): lanes 0-31 take tap t, lanes
// 32-63 tap t + 1 (the 28th tap is zero).  Halo layout [half][voxel][8 channels]
// (half = channels 0-7 or 8-15), so the 16 lanes of one fragment row read 256
// contiguous bytes; weight layout [tap pair][N-tile][lane] of 16-byte B fragments,
// so a wave reads 1 KiB contiguous.
constexpr int kCty = 4;                                  // output tile height (H)
constexpr int kPairs = 14;                               // tap pairs of a 3 x 3 x 3 kernel
template <int TZ, int MT> struct ConvTile {
  static constexpr int tx = 16 * MT, ty = kCty, tz = TZ;
  static constexpr int hx = tx + 2, hy = ty + 2, hz = tz + 2;
  static constexpr int hvox = hx * hy * hz;
  static constexpr int rows = TZ;                        // rows (z, y pairs) per wave: TZ
};

// dynamic LDS bytes of k_conv2 for nt N-tiles
template <int TZ, int MT>
static inline size_t conv2_lds(int taps, int nt) {
  return (size_t)2 * ConvTile<TZ, MT>::hvox * 8 * 2 + (size_t)(taps == 1 ? 1 : kPairs) * nt * 64 * 16;
}

template <int TAPS, int NT, int TZ, int MT>
__global__ __launch_bounds__(256) void k_conv2(const bf16_t* __restrict__ X, int xcs, int xco, int Cin,
                                               const bf16_t* __restrict__ Wt, int Cout, bf16_t* __restrict__ Y,
                                               int ycs, int yco, float* __restrict__ Yf, Vol vol, int relu,
                                               const bf16_t* __restrict__ mask, int mcs, int mco, int g0) {
  using Tl = ConvTile<TZ, MT>;
  constexpr int kHx = Tl::hx, kHy = Tl::hy, kHvox = Tl::hvox;
  constexpr int MI = TZ * MT;                  // M-tiles per wave
  extern __shared__ __attribute__((aligned(16))) unsigned char conv_smem[];
  bf16_t* tile = reinterpret_cast<bf16_t*>(conv_smem);
  u4v* wfrag = reinterpret_cast<u4v*>(conv_smem + (size_t)2 * kHvox * 8 * 2);
  constexpr int NPAIR = TAPS == 1 ? 1 : kPairs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntx = (vol.W + Tl::tx - 1) / Tl::tx, nty = (vol.H + Tl::ty - 1) / Tl::ty;
  int b = blockIdx.x;
  const int tx = b % ntx;
  b /= ntx;
  const int ty = b % nty;
  const int tz = b / nty;
  const int x0 = tx * Tl::tx, y0 = ty * Tl::ty, z0 = tz * Tl::tz;
  const int nt0 = (g0 + blockIdx.y) * 4;       // first N-tile of this workgroup's group
  const int m = lane & 15, kq = lane >> 4;     // fragment row / K-quarter
  const int half = kq & 1, second = kq >> 1;   // channel half, which tap of the pair
  // wave rows: TZ = 2: (wave / 2, 2 (wave % 2) + {0, 1}); TZ = 1: (0, wave)
  const int wz = TZ == 2 ? wave >> 1 : 0, wy = TZ == 2 ? 2 * (wave & 1) : wave;
  // this lane's halo row for tap offset 0 (the halo corner) of its first M-tile
  const int lds_lane = (half * kHvox + (wz * kHy + wy) * kHx + m) * 8;
  f4v acc[MI][NT];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[i][t] = f4v{0.f, 0.f, 0.f, 0.f};
  const int nchunk = Cin / 16;
  for (int ch = 0; ch < nchunk; ++ch) {
    __syncthreads();
    // halo tile: one 16-byte (8-channel) piece per step
    for (int e = threadIdx.x; e < 2 * kHvox; e += 256) {
      const int hv = e >> 1, hf = e & 1;
      const int hx = hv % kHx, hy = (hv / kHx) % kHy, hz = hv / (kHx * kHy);
      const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
      u4v val = u4v{0u, 0u, 0u, 0u};
      if (xx >= 0 && xx < vol.W && yy >= 0 && yy < vol.H && zz >= 0 && zz < vol.D) {
        const long v = ((long)zz * vol.H + yy) * vol.W + xx;
        val = *reinterpret_cast<const u4v*>(X + v * xcs + xco + ch * 16 + hf * 8);
      }
      *reinterpret_cast<u4v*>(tile + ((long)hf * kHvox + hv) * 8) = val;
    }
    // B fragments of the chunk: entry (pair, N-tile, lane) = W[tap][co][ci .. ci + 7]
    for (int e = threadIdx.x; e < NPAIR * NT * 64; e += 256) {
      const int l = e & 63, t = (e >> 6) % NT, tp = (e >> 6) / NT;
      const int lm = l & 15, lq = l >> 4;
      const int tap = TAPS == 1 ? 0 : 2 * tp + (lq >> 1);
      u4v val = u4v{0u, 0u, 0u, 0u};
      if (TAPS == 1 ? (lq >> 1) == 0 : tap < 27)
        val = *reinterpret_cast<const u4v*>(Wt + ((long)tap * Cout + (nt0 + t) * 16 + lm) * Cin + ch * 16 +
                                            (lq & 1) * 8);
      wfrag[e] = val;
    }
    __syncthreads();
#pragma unroll
    for (int tp = 0; tp < NPAIR; ++tp) {
      constexpr int kStep = kHx * kHy;
      const int t0 = 2 * tp, t1 = 2 * tp + 1;
      const int off0 = TAPS == 1 ? kStep + kHx + 1 : (t0 / 9) * kStep + ((t0 / 3) % 3) * kHx + t0 % 3;
      // the 28th tap (t1 = 27) does not exist: it reads tap t0's (finite) halo values,
      // and its B fragment is zero
      const int off1 = (TAPS == 1 || t1 >= 27) ? off0 : (t1 / 9) * kStep + ((t1 / 3) % 3) * kHx + t1 % 3;
      const int off = second ? off1 : off0;
      bf8v bfr[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) bfr[t] = __builtin_bit_cast(bf8v, wfrag[(tp * NT + t) * 64 + lane]);
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        // M-tile i: row (i / MT) of the wave, voxels 16 (i % MT) .. + 15
        const int ao = lds_lane + (off + (i / MT) * kHx + 16 * (i % MT)) * 8;
        const bf8v a = __builtin_bit_cast(bf8v, *reinterpret_cast<const u4v*>(tile + ao));
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[t], acc[i][t], 0, 0, 0);
      }
    }
  }
  // D[row = 4 kq + r][col = m]: voxel 16 (i % MT) + 4 kq + r of wave row i / MT
  const int zz = z0 + wz;
  if (zz >= vol.D) return;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int yy = y0 + wy + i / MT;
    if (yy >= vol.H) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = (nt0 + t) * 16 + m;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int xx = x0 + 16 * (i % MT) + 4 * kq + r;
        if (xx >= vol.W) continue;
        const long vo = ((long)zz * vol.H + yy) * vol.W + xx;
        float val = acc[i][t][r];
        if (relu) val = fmaxf(val, 0.f);
        if (mask) val = bf2f(mask[vo * mcs + mco + n]) > 0.f ? val : 0.f;
        if (Y) Y[vo * ycs + yco + n] = f2bf(val);
        if (Yf) Yf[vo * Cout + n] = val;
      }
    }
  }
}

// partial[chunk][tap][o][i] = sum over the chunk's voxels v of dY[v, o] X[v + tap, i]
template <int TAPS>
__global__ __launch_bounds__(256) void k_wgrad(const bf16_t* __restrict__ X, int xcs, int xco, int Cin,
                                               const bf16_t* __restrict__ dY, int ycs, int yco, int Cout,
                                               float* __restrict__ partial, Vol vol, int chunk) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int tap = blockIdx.y;
  const long V = vol.V();
  const long v0 = (long)blockIdx.x * chunk;
  const int dz = TAPS == 1 ? 0 : tap / 9 - 1, dy = TAPS == 1 ? 0 : (tap / 3) % 3 - 1,
            dx = TAPS == 1 ? 0 : tap % 3 - 1;
  const int to_n = Cout / 16, ti_n = Cin / 16;
  for (int tile = wave; tile < to_n * ti_n; tile += 4) {
    const int to = tile / ti_n, ti = tile % ti_n;
    f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
    for (long vb = v0; vb < v0 + chunk && vb < V; vb += 16) {
      s4v a, b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long v = vb + 4 * kq + i;
        short av = 0, bv = 0;
        if (v < V && v < v0 + chunk) {
          av = (short)dY[v * ycs + yco + to * 16 + m];
          const int x = (int)(v % vol.W), y = (int)((v / vol.W) % vol.H), z = (int)(v / ((long)vol.W * vol.H));
          const int zz = z + dz, yy = y + dy, xx = x + dx;
          if (zz >= 0 && zz < vol.D && yy >= 0 && yy < vol.H && xx >= 0 && xx < vol.W)
            bv = (short)X[(((long)zz * vol.H + yy) * vol.W + xx) * xcs + xco + ti * 16 + m];
        }
        a[i] = av;
        b[i] = bv;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      partial[(((long)blockIdx.x * TAPS + tap) * Cout + to * 16 + 4 * kq + r) * Cin + ti * 16 + m] = acc[r];
  }
}

// g (+)= sum over chunks of partial (fixed order)
__global__ void k_wreduce(const float* __restrict__ partial, int nchunk, long per, float* __restrict__ g,
                          int accumulate) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < per; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += partial[(long)c * per + i];
    g[i] = accumulate ? g[i] + s : s;
  }
}

// ------------------------------------------------------------------ pooling, upsampling
// Y (coarse) = mean of the 8 children of X (fine); one thread per 8 channels of a
// coarse voxel (C, strides and offsets are multiples of 8: 16-byte accesses)
__global__ void k_pool(const bf16_t* __restrict__ X, int xcs, int xco, bf16_t* __restrict__ Y, int ycs, int yco, int C,
                       Vol fine) {
  const Vol c{fine.D / 2, fine.H / 2, fine.W / 2};
  const int C8 = C / 8;
  const long n = c.V() * C8;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % C8) * 8;
    const long v = i / C8;
    const int x = (int)(v % c.W), y = (int)((v / c.W) % c.H), z = (int)(v / ((long)c.W * c.H));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int q = 0; q < 8; ++q) {
      const long fv = (((long)(2 * z + (q >> 2)) * fine.H + 2 * y + ((q >> 1) & 1)) * fine.W + 2 * x + (q & 1));
      const u4v raw = *reinterpret_cast<const u4v*>(X + fv * xcs + xco + ch);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s[2 * k] += __uint_as_float(raw[k] << 16);
        s[2 * k + 1] += __uint_as_float(raw[k] & 0xFFFF0000u);
      }
    }
    u4v o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = (unsigned)f2bf(s[2 * k] * 0.125f) | ((unsigned)f2bf(s[2 * k + 1] * 0.125f) << 16);
    *reinterpret_cast<u4v*>(Y + v * ycs + yco + ch) = o;
  }
}

// dX (fine) (+)= dY[parent] / 8, masked by mask > 0 (the ReLU before the pooling)
__global__ void k_pool_grad(const bf16_t* __restrict__ dY, int ycs, int yco, bf16_t* __restrict__ dX, int xcs, int xco,
                            int C, Vol fine, const bf16_t* __restrict__ mask, int mcs, int mco, int accumulate) {
  const long n = fine.V() * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % C);
    const long v = i / C;
    const int x = (int)(v % fine.W), y = (int)((v / fine.W) % fine.H), z = (int)(v / ((long)fine.W * fine.H));
    const long pv = ((long)(z / 2) * (fine.H / 2) + y / 2) * (fine.W / 2) + x / 2;
    float g = bf2f(dY[pv * ycs + yco + ch]) * 0.125f;
    if (mask && !(bf2f(mask[v * mcs + mco + ch]) > 0.f)) g = 0.f;
    const long o = v * xcs + xco + ch;
    dX[o] = f2bf(accumulate ? bf2f(dX[o]) + g : g);
  }
}

// Y (fine) = X[parent] (nearest neighbour); one thread per 8 channels of a fine voxel
__global__ void k_up(const bf16_t* __restrict__ X, int xcs, int xco, bf16_t* __restrict__ Y, int ycs, int yco, int C,
                     Vol fine) {
  const int C8 = C / 8;
  const long n = fine.V() * C8;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % C8) * 8;
    const long v = i / C8;
    const int x = (int)(v % fine.W), y = (int)((v / fine.W) % fine.H), z = (int)(v / ((long)fine.W * fine.H));
    const long pv = ((long)(z / 2) * (fine.H / 2) + y / 2) * (fine.W / 2) + x / 2;
    *reinterpret_cast<u4v*>(Y + v * ycs + yco + ch) = *reinterpret_cast<const u4v*>(X + pv * xcs + xco + ch);
  }
}

// dX (coarse) = sum of dY over the 8 children
__global__ void k_up_grad(const bf16_t* __restrict__ dY, int ycs, int yco, bf16_t* __restrict__ dX, int xcs, int xco,
                          int C, Vol fine) {
  const Vol c{fine.D / 2, fine.H / 2, fine.W / 2};
  const long n = c.V() * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % C);
    const long v = i / C;
    const int x = (int)(v % c.W), y = (int)((v / c.W) % c.H), z = (int)(v / ((long)c.W * c.H));
    float s = 0.f;
    for (int q = 0; q < 8; ++q) {
      const long fv = (((long)(2 * z + (q >> 2)) * fine.H + 2 * y + ((q >> 1) & 1)) * fine.W + 2 * x + (q & 1));
      s += bf2f(dY[fv * ycs + yco + ch]);
    }
    dX[v * xcs + xco + ch] = f2bf(s);
  }
}

// ------------------------------------------------------------------ data in / out, loss, Adam
// X0[v][0..15] = (Re/Im r_x, r_y, r_z) * s, Re/Im chi, (Re/Im w_x, w_y, w_z) * s or zeros
// when w is null, zeros;  s = sqrt(3N / ||r||^2)
__global__ void k_pack(const double2* __restrict__ r, const double2* __restrict__ w, const double2* __restrict__ chi,
                       const double2* __restrict__ sumsq, long N, bf16_t* __restrict__ X0) {
  const double s = sumsq->x > 0 ? sqrt(3.0 * (double)N / sumsq->x) : 0.0;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x) {
    bf16_t* o = X0 + v * 16;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 a = r[(long)c * N + v];
      o[2 * c] = f2bf((float)(a.x * s));
      o[2 * c + 1] = f2bf((float)(a.y * s));
    }
    const double2 k = chi[v];
    o[6] = f2bf((float)k.x);
    o[7] = f2bf((float)k.y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 a = w ? w[(long)c * N + v] : double2{0.0, 0.0};
      o[8 + 2 * c] = f2bf((float)(a.x * s));
      o[9 + 2 * c] = f2bf((float)(a.y * s));
    }
    o[14] = 0;
    o[15] = 0;
  }
}

// z[c][v] = base[c][v] + (out[v][2c] + i out[v][2c+1]) / s with base = w, or r when w
// is null: the network predicts the correction A^{-1} r - base, so an untrained
// (small) network leaves the base preconditioner (or the identity)
__global__ void k_unpack(const float* __restrict__ out, const double2* __restrict__ sumsq, long N,
                         const double2* __restrict__ base, double2* __restrict__ z) {
  const double s = sumsq->x > 0 ? sqrt(3.0 * (double)N / sumsq->x) : 0.0;
  const double is = s > 0 ? 1.0 / s : 0.0;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 rv = base[(long)c * N + v];
      z[(long)c * N + v] = double2{rv.x + out[v * 16 + 2 * c] * is, rv.y + out[v * 16 + 2 * c + 1] * is};
    }
}

// mean squared error of out against (target - base) * s over 6 channels; dOut = d(loss)/d(out)
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ out, const double2* __restrict__ target,
                                              const double2* __restrict__ base, const double2* __restrict__ sumsq,
                                              long N, bf16_t* __restrict__ dOut, float gscale,
                                              double* __restrict__ partial) {
  __shared__ double red[256];
  const double s = sumsq->x > 0 ? sqrt(3.0 * (double)N / sumsq->x) : 0.0;
  double acc = 0.0;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < N; v += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 t = target[(long)c * N + v], rv = base[(long)c * N + v];
      const float d0 = out[v * 16 + 2 * c] - (float)((t.x - rv.x) * s);
      const float d1 = out[v * 16 + 2 * c + 1] - (float)((t.y - rv.y) * s);
      acc += (double)d0 * d0 + (double)d1 * d1;
      dOut[v * 16 + 2 * c] = f2bf(gscale * d0);
      dOut[v * 16 + 2 * c + 1] = f2bf(gscale * d1);
    }
#pragma unroll
    for (int c = 6; c < 16; ++c) dOut[v * 16 + c] = 0;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// The constants come from the host, formed in FP64 and rounded once: k.omb1 = 1 - beta1,
// k.omb2 = 1 - beta2 and the bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t
// (1 - 0.999f in FP32 would carry a relative error of 1.3e-5).
struct AdamK {
  float lr, b1, omb1, b2, omb2, eps, c1, c2;
};

__global__ void k_adam(float* __restrict__ w, float* __restrict__ mo, float* __restrict__ ve,
                       const float* __restrict__ g, long n, AdamK k, int taps, int Cout, int Cin,
                       bf16_t* __restrict__ wbf, bf16_t* __restrict__ wtbf, int update) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float wi = w[i];
    if (update) {
      const float gi = g[i];
      const float m1 = k.b1 * mo[i] + k.omb1 * gi;
      const float v1 = k.b2 * ve[i] + k.omb2 * gi * gi;
      mo[i] = m1;
      ve[i] = v1;
      wi -= k.lr * (m1 / k.c1) / (sqrtf(v1 / k.c2) + k.eps);
      w[i] = wi;
    }
    const int ci = (int)(i % Cin);
    const int co = (int)((i / Cin) % Cout);
    const int t = (int)(i / ((long)Cin * Cout));
    const bf16_t h = f2bf(wi);
    wbf[i] = h;
    wtbf[((long)(taps - 1 - t) * Cin + ci) * Cout + co] = h;
  }
}

__global__ void k_f2bf(const float* a, bf16_t* b, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = f2bf(a[i]);
}

__global__ void k_bf2f(const bf16_t* a, float* b, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = bf2f(a[i]);
}

__global__ void k_fill_bf(bf16_t* p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0;
}

// Adam (Kingma & Ba) constants of step t and learning rate lr
static inline AdamK adam_constants(int t, float lr) {
  const double b1 = 0.9, b2 = 0.999;
  AdamK k;
  k.lr = lr;
  k.b1 = (float)b1;
  k.omb1 = (float)(1.0 - b1);
  k.b2 = (float)b2;
  k.omb2 = (float)(1.0 - b2);
  k.eps = 1e-8f;
  k.c1 = (float)(1.0 - std::pow(b1, (double)t));
  k.c2 = (float)(1.0 - std::pow(b2, (double)t));
  return k;
}

static inline int gblocks(long n) { return (int)std::min<long>(4096, (n + 255) / 256); }

// k_conv2 may use more than 64 KiB of dynamic LDS (83.5 KiB with four N-tiles)
template <int TAPS, int TZ, int MT>
static hipError_t allow_conv_lds_shape() {
  const auto a = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_conv2<TAPS, 1, TZ, MT>, a, (int)conv2_lds<TZ, MT>(TAPS, 1)))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_conv2<TAPS, 2, TZ, MT>, a, (int)conv2_lds<TZ, MT>(TAPS, 2)))) return e;
  if ((e = hipFuncSetAttribute((const void*)k_conv2<TAPS, 3, TZ, MT>, a, (int)conv2_lds<TZ, MT>(TAPS, 3)))) return e;
  return hipFuncSetAttribute((const void*)k_conv2<TAPS, 4, TZ, MT>, a, (int)conv2_lds<TZ, MT>(TAPS, 4));
}
static hipError_t allow_conv_lds() {
  hipError_t e;
  if ((e = allow_conv_lds_shape<27, 2, 2>())) return e;
  if ((e = allow_conv_lds_shape<1, 2, 2>())) return e;
  if ((e = allow_conv_lds_shape<27, 1, 1>())) return e;
  return allow_conv_lds_shape<1, 1, 1>();
}

template <int TAPS, int TZ, int MT>
static void conv2_launch_nt(int nt, dim3 grid, int g0, hipStream_t s, const bf16_t* X, int xcs, int xco, int Cin,
                            const bf16_t* W, int Cout, bf16_t* Y, int ycs, int yco, float* Yf, Vol vol, int relu,
                            const bf16_t* mask, int mcs, int mco) {
  const size_t lds = conv2_lds<TZ, MT>(TAPS, nt);
#define VIE_CONV2(NTV)                                                                                           \
  if (nt == NTV)                                                                                                 \
    hipLaunchKernelGGL((k_conv2<TAPS, NTV, TZ, MT>), grid, dim3(256), lds, s, X, xcs, xco, Cin, W, Cout, Y, ycs,  \
                       yco, Yf, vol, relu, mask, mcs, mco, g0);
  VIE_CONV2(1)
  VIE_CONV2(2)
  VIE_CONV2(3)
  VIE_CONV2(4)
#undef VIE_CONV2
}

// Output-channel groups of four N-tiles in one launch, a smaller last group in a
// second.  The 2 x 4 x 32 voxel tile where it gives at least 512 workgroups, else the
// 1 x 4 x 16 tile (the small levels of the network).
hipError_t conv_launch(int taps, const bf16_t* X, int xcs, int xco, int Cin, const bf16_t* W, int Cout, bf16_t* Y,
                       int ycs, int yco, float* Yf, Vol vol, int relu, const bf16_t* mask, int mcs, int mco,
                       hipStream_t s) {
  static const hipError_t lds_ok = allow_conv_lds();
  if (lds_ok) return lds_ok;
  const long big = (long)((vol.D + 1) / 2) * ((vol.H + kCty - 1) / kCty) * ((vol.W + 31) / 32);
  const long small = (long)vol.D * ((vol.H + kCty - 1) / kCty) * ((vol.W + 15) / 16);
  const bool use_big = big >= 512;
  const int ntiles = Cout / 16, full = ntiles / 4, rest = ntiles % 4;
  auto go = [&](int nt, int groups, int g0) {
    const dim3 grid((unsigned)(use_big ? big : small), (unsigned)groups);
    if (use_big) {
      if (taps == 27)
        conv2_launch_nt<27, 2, 2>(nt, grid, g0, s, X, xcs, xco, Cin, W, Cout, Y, ycs, yco, Yf, vol, relu, mask, mcs,
                                  mco);
      else
        conv2_launch_nt<1, 2, 2>(nt, grid, g0, s, X, xcs, xco, Cin, W, Cout, Y, ycs, yco, Yf, vol, relu, mask, mcs,
                                 mco);
    } else {
      if (taps == 27)
        conv2_launch_nt<27, 1, 1>(nt, grid, g0, s, X, xcs, xco, Cin, W, Cout, Y, ycs, yco, Yf, vol, relu, mask, mcs,
                                  mco);
      else
        conv2_launch_nt<1, 1, 1>(nt, grid, g0, s, X, xcs, xco, Cin, W, Cout, Y, ycs, yco, Yf, vol, relu, mask, mcs,
                                 mco);
    }
  };
  if (full) go(4, full, 0);
  if (rest) go(rest, 1, full);
  return hipGetLastError();
}

hipError_t wgrad_launch(int taps, const bf16_t* X, int xcs, int xco, int Cin, const bf16_t* dY, int ycs, int yco,
                        int Cout, float* partial, long partial_cap, float* g, int accumulate, Vol vol, hipStream_t s) {
  const long V = vol.V();
  const long per = (long)taps * Cout * Cin;
  int chunk = 2048;
  while ((V + chunk - 1) / chunk * per > partial_cap) chunk *= 2;
  const int nchunk = (int)((V + chunk - 1) / chunk);
  if (taps == 27)
    hipLaunchKernelGGL((k_wgrad<27>), dim3(nchunk, 27), dim3(256), 0, s, X, xcs, xco, Cin, dY, ycs, yco, Cout,
                       partial, vol, chunk);
  else
    hipLaunchKernelGGL((k_wgrad<1>), dim3(nchunk, 1), dim3(256), 0, s, X, xcs, xco, Cin, dY, ycs, yco, Cout,
                       partial, vol, chunk);
  hipLaunchKernelGGL(k_wreduce, dim3(gblocks(per)), dim3(256), 0, s, partial, nchunk, per, g, accumulate);
  return hipGetLastError();
}

}  // namespace vie

// =============================================================================
// the network object
// =============================================================================
using namespace vie;

namespace {

struct Conv {
  int taps, cin, cout;       // padded channel counts (multiples of 16)
  int cin_real;
  float *w, *m, *v, *g;
  bf16_t *wbf, *wtbf;
  long n() const { return (long)taps * cin * cout; }
};

struct View {
  bf16_t* p;
  int cs, co, c;   // channel stride, offset, count
};

}  // namespace

struct vie_net_s {
  int n[3];
  Vol lv[4];
  hipStream_t stream;
  Conv L[15];
  // activations and their gradients
  bf16_t *X0, *E1a, *D1cat, *Dd1a, *Dd1b, *P1, *E2a, *D2cat, *Dd2a, *Dd2b, *P2, *E3a, *D3cat, *Dd3a, *Dd3b, *P3, *E4a,
      *E4b;
  bf16_t *gE1a, *gD1cat, *gDd1a, *gDd1b, *gP1, *gE2a, *gD2cat, *gDd2a, *gDd2b, *gP2, *gE3a, *gD3cat, *gDd3a, *gDd3b,
      *gP3, *gE4a, *gE4b, *gOut;
  float* out;          // [V1][16] FP32 network output
  float* partial;      // wgrad split-K partials
  long partial_cap;
  double2* sumsq;      // ||r||^2 of the current input
  double2* red;        // reduction scratch
  double* lpart;       // loss partials
  double* lpart_h;
  int step = 0;
  std::vector<void*> allocs;
  std::string err;
};

namespace {

hipError_t nalloc(vie_net_s* n, void** p, size_t bytes) {
  hipError_t e = dmalloc(p, bytes);
  if (!e) n->allocs.push_back(*p);
  return e;
}

// forward pass from X0 to out; all activations kept for the backward pass
hipError_t net_forward(vie_net_s* N) {
  hipStream_t s = N->stream;
  const Vol *l = N->lv;
  hipError_t e;
#define CONV(i, X, xcs, xco, Y, ycs, yco, lev, relu)                                                           \
  if ((e = conv_launch(N->L[i].taps, X, xcs, xco, N->L[i].cin, N->L[i].wbf, N->L[i].cout, Y, ycs, yco, nullptr, \
                       l[lev], relu, nullptr, 0, 0, s)))                                                          \
    return e;
  CONV(0, N->X0, 16, 0, N->E1a, 16, 0, 0, 1)
  CONV(1, N->E1a, 16, 0, N->D1cat, 48, 32, 0, 1)
  hipLaunchKernelGGL(k_pool, dim3(gblocks(l[1].V() * 16)), dim3(256), 0, s, N->D1cat, 48, 32, N->P1, 16, 0, 16, l[0]);
  CONV(2, N->P1, 16, 0, N->E2a, 32, 0, 1, 1)
  CONV(3, N->E2a, 32, 0, N->D2cat, 80, 48, 1, 1)
  hipLaunchKernelGGL(k_pool, dim3(gblocks(l[2].V() * 32)), dim3(256), 0, s, N->D2cat, 80, 48, N->P2, 32, 0, 32, l[1]);
  CONV(4, N->P2, 32, 0, N->E3a, 48, 0, 2, 1)
  CONV(5, N->E3a, 48, 0, N->D3cat, 112, 64, 2, 1)
  hipLaunchKernelGGL(k_pool, dim3(gblocks(l[3].V() * 48)), dim3(256), 0, s, N->D3cat, 112, 64, N->P3, 48, 0, 48, l[2]);
  CONV(6, N->P3, 48, 0, N->E4a, 64, 0, 3, 1)
  CONV(7, N->E4a, 64, 0, N->E4b, 64, 0, 3, 1)
  hipLaunchKernelGGL(k_up, dim3(gblocks(l[2].V() * 64)), dim3(256), 0, s, N->E4b, 64, 0, N->D3cat, 112, 0, 64, l[2]);
  CONV(8, N->D3cat, 112, 0, N->Dd3a, 48, 0, 2, 1)
  CONV(9, N->Dd3a, 48, 0, N->Dd3b, 48, 0, 2, 1)
  hipLaunchKernelGGL(k_up, dim3(gblocks(l[1].V() * 48)), dim3(256), 0, s, N->Dd3b, 48, 0, N->D2cat, 80, 0, 48, l[1]);
  CONV(10, N->D2cat, 80, 0, N->Dd2a, 32, 0, 1, 1)
  CONV(11, N->Dd2a, 32, 0, N->Dd2b, 32, 0, 1, 1)
  hipLaunchKernelGGL(k_up, dim3(gblocks(l[0].V() * 32)), dim3(256), 0, s, N->Dd2b, 32, 0, N->D1cat, 48, 0, 32, l[0]);
  CONV(12, N->D1cat, 48, 0, N->Dd1a, 16, 0, 0, 1)
  CONV(13, N->Dd1a, 16, 0, N->Dd1b, 16, 0, 0, 1)
#undef CONV
  return conv_launch(1, N->Dd1b, 16, 0, 16, N->L[14].wbf, 16, nullptr, 0, 0, N->out, l[0], 0, nullptr, 0, 0, s);
}

// backward pass from gOut; accumulates weight gradients into L[i].g
hipError_t net_backward(vie_net_s* N, int accumulate) {
  hipStream_t s = N->stream;
  const Vol* l = N->lv;
  hipError_t e;
  const long cap = N->partial_cap;
  // dgrad of layer i: input gradient (cin channels) from output gradient dY (cout channels)
#define DGRAD(i, dY, ycs, yco, dX, xcs, xco, lev, mask, mcs, mco)                                                 \
  if ((e = conv_launch(N->L[i].taps, dY, ycs, yco, N->L[i].cout, N->L[i].wtbf, N->L[i].cin, dX, xcs, xco, nullptr, \
                       l[lev], 0, mask, mcs, mco, s)))                                                               \
    return e;
#define WGRAD(i, X, xcs, xco, dY, ycs, yco, lev)                                                                   \
  if ((e = wgrad_launch(N->L[i].taps, X, xcs, xco, N->L[i].cin, dY, ycs, yco, N->L[i].cout, N->partial, cap,      \
                        N->L[i].g, accumulate, l[lev], s)))                                                          \
    return e;
  // level 1 decoder
  WGRAD(14, N->Dd1b, 16, 0, N->gOut, 16, 0, 0)
  DGRAD(14, N->gOut, 16, 0, N->gDd1b, 16, 0, 0, N->Dd1b, 16, 0)
  WGRAD(13, N->Dd1a, 16, 0, N->gDd1b, 16, 0, 0)
  DGRAD(13, N->gDd1b, 16, 0, N->gDd1a, 16, 0, 0, N->Dd1a, 16, 0)
  WGRAD(12, N->D1cat, 48, 0, N->gDd1a, 16, 0, 0)
  DGRAD(12, N->gDd1a, 16, 0, N->gD1cat, 48, 0, 0, N->D1cat, 48, 0)
  hipLaunchKernelGGL(k_up_grad, dim3(gblocks(l[1].V() * 32)), dim3(256), 0, s, N->gD1cat, 48, 0, N->gDd2b, 32, 0, 32,
                     l[0]);
  // level 2 decoder
  WGRAD(11, N->Dd2a, 32, 0, N->gDd2b, 32, 0, 1)
  DGRAD(11, N->gDd2b, 32, 0, N->gDd2a, 32, 0, 1, N->Dd2a, 32, 0)
  WGRAD(10, N->D2cat, 80, 0, N->gDd2a, 32, 0, 1)
  DGRAD(10, N->gDd2a, 32, 0, N->gD2cat, 80, 0, 1, N->D2cat, 80, 0)
  hipLaunchKernelGGL(k_up_grad, dim3(gblocks(l[2].V() * 48)), dim3(256), 0, s, N->gD2cat, 80, 0, N->gDd3b, 48, 0, 48,
                     l[1]);
  // level 3 decoder
  WGRAD(9, N->Dd3a, 48, 0, N->gDd3b, 48, 0, 2)
  DGRAD(9, N->gDd3b, 48, 0, N->gDd3a, 48, 0, 2, N->Dd3a, 48, 0)
  WGRAD(8, N->D3cat, 112, 0, N->gDd3a, 48, 0, 2)
  DGRAD(8, N->gDd3a, 48, 0, N->gD3cat, 112, 0, 2, N->D3cat, 112, 0)
  hipLaunchKernelGGL(k_up_grad, dim3(gblocks(l[3].V() * 64)), dim3(256), 0, s, N->gD3cat, 112, 0, N->gE4b, 64, 0, 64,
                     l[2]);
  // bottom
  WGRAD(7, N->E4a, 64, 0, N->gE4b, 64, 0, 3)
  DGRAD(7, N->gE4b, 64, 0, N->gE4a, 64, 0, 3, N->E4a, 64, 0)
  WGRAD(6, N->P3, 48, 0, N->gE4a, 64, 0, 3)
  DGRAD(6, N->gE4a, 64, 0, N->gP3, 48, 0, 3, nullptr, 0, 0)
  // skip E3b = D3cat[64:112]: its gradient already holds the skip path; add the pooling path
  hipLaunchKernelGGL(k_pool_grad, dim3(gblocks(l[2].V() * 48)), dim3(256), 0, s, N->gP3, 48, 0, N->gD3cat, 112, 64, 48,
                     l[2], N->D3cat, 112, 64, 1);
  WGRAD(5, N->E3a, 48, 0, N->gD3cat, 112, 64, 2)
  DGRAD(5, N->gD3cat, 112, 64, N->gE3a, 48, 0, 2, N->E3a, 48, 0)
  WGRAD(4, N->P2, 32, 0, N->gE3a, 48, 0, 2)
  DGRAD(4, N->gE3a, 48, 0, N->gP2, 32, 0, 2, nullptr, 0, 0)
  hipLaunchKernelGGL(k_pool_grad, dim3(gblocks(l[1].V() * 32)), dim3(256), 0, s, N->gP2, 32, 0, N->gD2cat, 80, 48, 32,
                     l[1], N->D2cat, 80, 48, 1);
  WGRAD(3, N->E2a, 32, 0, N->gD2cat, 80, 48, 1)
  DGRAD(3, N->gD2cat, 80, 48, N->gE2a, 32, 0, 1, N->E2a, 32, 0)
  WGRAD(2, N->P1, 16, 0, N->gE2a, 32, 0, 1)
  DGRAD(2, N->gE2a, 32, 0, N->gP1, 16, 0, 1, nullptr, 0, 0)
  hipLaunchKernelGGL(k_pool_grad, dim3(gblocks(l[0].V() * 16)), dim3(256), 0, s, N->gP1, 16, 0, N->gD1cat, 48, 32, 16,
                     l[0], N->D1cat, 48, 32, 1);
  WGRAD(1, N->E1a, 16, 0, N->gD1cat, 48, 32, 0)
  DGRAD(1, N->gD1cat, 48, 32, N->gE1a, 16, 0, 0, N->E1a, 16, 0)
  WGRAD(0, N->X0, 16, 0, N->gE1a, 16, 0, 0)
#undef DGRAD
#undef WGRAD
  return hipGetLastError();
}

hipError_t refresh_weights(vie_net_s* N, int update, float lr) {
  if (update) N->step++;
  const AdamK k = adam_constants(std::max(1, N->step), lr);
  for (auto& L : N->L)
    hipLaunchKernelGGL(k_adam, dim3(gblocks(L.n())), dim3(256), 0, N->stream, L.w, L.m, L.v, L.g, L.n(), k, L.taps,
                       L.cout, L.cin, L.wbf, L.wtbf, update);
  return hipGetLastError();
}

int nfail(vie_net_s* n, int code, const std::string& m) {
  if (n) n->err = m;
  return code;
}

}  // namespace

namespace vie {
// used by the solver (vie_api.cpp): z = ||r|| net(r / ||r||, chi)
hipError_t net_apply(vie_net_s* N, const double2* r, const double2* w, const double2* chi, double2* z) {
  const long V = N->lv[0].V();
  hipError_t e;
  if ((e = KrylovOps<double>::nrm2sq(r, 3 * V, N->red, N->sumsq, N->stream))) return e;
  hipLaunchKernelGGL(k_pack, dim3(gblocks(V)), dim3(256), 0, N->stream, r, w, chi, N->sumsq, V, N->X0);
  if ((e = net_forward(N))) return e;
  hipLaunchKernelGGL(k_unpack, dim3(gblocks(V)), dim3(256), 0, N->stream, N->out, N->sumsq, V, w ? w : r, z);
  return hipGetLastError();
}
const int* net_grid(vie_net_s* N) { return N->n; }
void net_set_stream(vie_net_s* N, hipStream_t s) { N->stream = s; }
}  // namespace vie

extern "C" {

int vie_net_create(vie_net_t* out, const int grid[3], unsigned seed, void* hip_stream) {
  if (!out || !grid) return VIE_EINVAL;
  *out = nullptr;
  for (int d = 0; d < 3; ++d)
    if (grid[d] < 8 || grid[d] % 8 != 0 || grid[d] > 4096) return VIE_EINVAL;
  auto* N = new vie_net_s();
  std::memcpy(N->n, grid, sizeof(int) * 3);
  N->stream = reinterpret_cast<hipStream_t>(hip_stream);
  for (int l = 0; l < 4; ++l) N->lv[l] = Vol{grid[0] >> l, grid[1] >> l, grid[2] >> l};
  // (taps, cin, cout, cin_real): 16/32/48/64 U-Net, input 8 real channels, output 6
  const int spec[15][4] = {{27, 16, 16, 14},  {27, 16, 16, 16},  {27, 16, 32, 16},  {27, 32, 32, 32},
                           {27, 32, 48, 32},  {27, 48, 48, 48},  {27, 48, 64, 48},  {27, 64, 64, 64},
                           {27, 112, 48, 112}, {27, 48, 48, 48}, {27, 80, 32, 80},  {27, 32, 32, 32},
                           {27, 48, 16, 48},  {27, 16, 16, 16},  {1, 16, 16, 16}};
  auto bail = [&](int code) {
    vie_net_destroy(N);
    return code;
  };
  std::mt19937_64 rng(seed);
  for (int i = 0; i < 15; ++i) {
    Conv& C = N->L[i];
    C.taps = spec[i][0];
    C.cin = spec[i][1];
    C.cout = spec[i][2];
    C.cin_real = spec[i][3];
    const long n = C.n();
    for (float** p : {&C.w, &C.m, &C.v, &C.g})
      if (nalloc(N, (void**)p, sizeof(float) * n)) return bail(VIE_ENOMEM);
    if (nalloc(N, (void**)&C.wbf, sizeof(bf16_t) * n) || nalloc(N, (void**)&C.wtbf, sizeof(bf16_t) * n))
      return bail(VIE_ENOMEM);
    // He initialisation over the real fan-in; padded input channels and the
    // padded outputs of the last layer stay zero
    std::vector<float> w(n, 0.f);
    std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (C.taps * C.cin_real)) * (i == 14 ? 0.1 : 1.0));
    const int cout_real = i == 14 ? 6 : C.cout;
    for (int t = 0; t < C.taps; ++t)
      for (int o = 0; o < cout_real; ++o)
        for (int ci = 0; ci < C.cin_real; ++ci) w[((long)t * C.cout + o) * C.cin + ci] = (float)nd(rng);
    if (hipMemcpy(C.w, w.data(), sizeof(float) * n, hipMemcpyHostToDevice)) return bail(VIE_EDEVICE);
    if (hipMemset(C.m, 0, sizeof(float) * n) || hipMemset(C.v, 0, sizeof(float) * n) ||
        hipMemset(C.g, 0, sizeof(float) * n))
      return bail(VIE_EDEVICE);
  }
  const long V[4] = {N->lv[0].V(), N->lv[1].V(), N->lv[2].V(), N->lv[3].V()};
  struct B {
    bf16_t** p;
    long v;
    int c;
  } bufs[] = {{&N->X0, V[0], 16},    {&N->E1a, V[0], 16},   {&N->D1cat, V[0], 48}, {&N->Dd1a, V[0], 16},
              {&N->Dd1b, V[0], 16},  {&N->P1, V[1], 16},    {&N->E2a, V[1], 32},   {&N->D2cat, V[1], 80},
              {&N->Dd2a, V[1], 32},  {&N->Dd2b, V[1], 32},  {&N->P2, V[2], 32},    {&N->E3a, V[2], 48},
              {&N->D3cat, V[2], 112}, {&N->Dd3a, V[2], 48}, {&N->Dd3b, V[2], 48},  {&N->P3, V[3], 48},
              {&N->E4a, V[3], 64},   {&N->E4b, V[3], 64},   {&N->gE1a, V[0], 16},  {&N->gD1cat, V[0], 48},
              {&N->gDd1a, V[0], 16}, {&N->gDd1b, V[0], 16}, {&N->gP1, V[1], 16},   {&N->gE2a, V[1], 32},
              {&N->gD2cat, V[1], 80}, {&N->gDd2a, V[1], 32}, {&N->gDd2b, V[1], 32}, {&N->gP2, V[2], 32},
              {&N->gE3a, V[2], 48},  {&N->gD3cat, V[2], 112}, {&N->gDd3a, V[2], 48}, {&N->gDd3b, V[2], 48},
              {&N->gP3, V[3], 48},   {&N->gE4a, V[3], 64},  {&N->gE4b, V[3], 64},  {&N->gOut, V[0], 16}};
  for (auto& b : bufs) {
    if (nalloc(N, (void**)b.p, sizeof(bf16_t) * b.v * b.c)) return bail(VIE_ENOMEM);
    hipLaunchKernelGGL(k_fill_bf, dim3(gblocks(b.v * b.c)), dim3(256), 0, N->stream, *b.p, b.v * b.c);
  }
  if (nalloc(N, (void**)&N->out, sizeof(float) * V[0] * 16)) return bail(VIE_ENOMEM);
  N->partial_cap = 8L << 20;   // floats
  if (nalloc(N, (void**)&N->partial, sizeof(float) * N->partial_cap)) return bail(VIE_ENOMEM);
  if (nalloc(N, (void**)&N->sumsq, sizeof(double2) * 2)) return bail(VIE_ENOMEM);
  // partials of KrylovOps::nrm2sq over the 3V residual values
  if (nalloc(N, (void**)&N->red, sizeof(double2) * (partial_blocks(3 * V[0]) + 1))) return bail(VIE_ENOMEM);
  if (nalloc(N, (void**)&N->lpart, sizeof(double) * 4096)) return bail(VIE_ENOMEM);
  if (hipHostMalloc(&N->lpart_h, sizeof(double) * 4096, hipHostMallocDefault)) return bail(VIE_ENOMEM);
  if (refresh_weights(N, 0, 0.f) || hipStreamSynchronize(N->stream)) return bail(VIE_EDEVICE);
  *out = N;
  return VIE_OK;
}

void vie_net_destroy(vie_net_t N) {
  if (!N) return;
  for (void* p : N->allocs) (void)hipFree(p);
  if (N->lpart_h) (void)hipHostFree(N->lpart_h);
  delete N;
}

int vie_net_num_params(vie_net_t N, size_t* count) {
  if (!N || !count) return VIE_EINVAL;
  size_t c = 0;
  for (auto& L : N->L) c += L.n();
  *count = c;
  return VIE_OK;
}

int vie_net_get_params(vie_net_t N, float* host, size_t count) {
  size_t c = 0;
  if (!N || !host || vie_net_num_params(N, &c) || c != count) return VIE_EINVAL;
  size_t off = 0;
  for (auto& L : N->L) {
    if (hipMemcpy(host + off, L.w, sizeof(float) * L.n(), hipMemcpyDeviceToHost)) return VIE_EDEVICE;
    off += L.n();
  }
  return VIE_OK;
}

int vie_net_set_params(vie_net_t N, const float* host, size_t count) {
  size_t c = 0;
  if (!N || !host || vie_net_num_params(N, &c) || c != count) return VIE_EINVAL;
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(host[i])) return nfail(N, VIE_EINVAL, "weight " + std::to_string(i) + " is not finite");
  size_t off = 0;
  for (auto& L : N->L) {
    if (hipMemcpy(L.w, host + off, sizeof(float) * L.n(), hipMemcpyHostToDevice)) return VIE_EDEVICE;
    off += L.n();
  }
  if (refresh_weights(N, 0, 0.f) || hipStreamSynchronize(N->stream)) return VIE_EDEVICE;
  return VIE_OK;
}

int vie_net_get_state(vie_net_t N, float* host, size_t count, int* step) {
  size_t c = 0;
  if (!N || !host || !step || vie_net_num_params(N, &c) || c != count) return VIE_EINVAL;
  size_t off = 0;
  for (auto& L : N->L) {
    const size_t b = sizeof(float) * L.n();
    if (hipMemcpy(host + off, L.w, b, hipMemcpyDeviceToHost) ||
        hipMemcpy(host + count + off, L.m, b, hipMemcpyDeviceToHost) ||
        hipMemcpy(host + 2 * count + off, L.v, b, hipMemcpyDeviceToHost))
      return VIE_EDEVICE;
    off += L.n();
  }
  *step = N->step;
  return VIE_OK;
}

int vie_net_set_state(vie_net_t N, const float* host, size_t count, int step) {
  size_t c = 0;
  if (!N || !host || vie_net_num_params(N, &c) || c != count) return VIE_EINVAL;
  if (step < 0) return nfail(N, VIE_EINVAL, "negative Adam step");
  for (size_t i = 0; i < 3 * count; ++i)
    if (!std::isfinite(host[i])) return nfail(N, VIE_EINVAL, "state value " + std::to_string(i) + " is not finite");
  for (size_t i = 2 * count; i < 3 * count; ++i)
    if (host[i] < 0.f) return nfail(N, VIE_EINVAL, "negative second moment " + std::to_string(i - 2 * count));
  size_t off = 0;
  for (auto& L : N->L) {
    const size_t b = sizeof(float) * L.n();
    if (hipMemcpy(L.w, host + off, b, hipMemcpyHostToDevice) ||
        hipMemcpy(L.m, host + count + off, b, hipMemcpyHostToDevice) ||
        hipMemcpy(L.v, host + 2 * count + off, b, hipMemcpyHostToDevice))
      return VIE_EDEVICE;
    off += L.n();
  }
  N->step = step;
  if (refresh_weights(N, 0, 0.f) || hipStreamSynchronize(N->stream)) return VIE_EDEVICE;
  return VIE_OK;
}

int vie_net_apply(vie_net_t N, const vie_c128* r, const vie_c128* chi, vie_c128* z) {
  return vie_net_apply_base(N, r, nullptr, chi, z);
}

int vie_net_apply_base(vie_net_t N, const vie_c128* r, const vie_c128* w, const vie_c128* chi, vie_c128* z) {
  if (!N || !r || !chi || !z) return VIE_EINVAL;
  if (net_apply(N, reinterpret_cast<const double2*>(r), reinterpret_cast<const double2*>(w),
                reinterpret_cast<const double2*>(chi), reinterpret_cast<double2*>(z)))
    return VIE_EDEVICE;
  return VIE_OK;
}

int vie_net_train_step(vie_net_t N, int count, const vie_c128* const* r, const vie_c128* const* chi,
                       const vie_c128* const* target, float lr, double* loss) {
  return vie_net_train_step_base(N, count, r, nullptr, chi, target, lr, loss);
}

int vie_net_train_step_base(vie_net_t N, int count, const vie_c128* const* r, const vie_c128* const* w,
                            const vie_c128* const* chi, const vie_c128* const* target, float lr, double* loss) {
  if (!N || count < 1 || !r || !chi || !target || !(lr >= 0)) return VIE_EINVAL;
  const long V = N->lv[0].V();
  double total = 0.0;
  const int nb = gblocks(V);
  for (int i = 0; i < count; ++i) {
    if (!r[i] || !chi[i] || !target[i]) return VIE_EINVAL;
    const double2* ri = reinterpret_cast<const double2*>(r[i]);
    if (KrylovOps<double>::nrm2sq(ri, 3 * V, N->red, N->sumsq, N->stream)) return VIE_EDEVICE;
    const double2* wi = w ? reinterpret_cast<const double2*>(w[i]) : nullptr;
    hipLaunchKernelGGL(k_pack, dim3(gblocks(V)), dim3(256), 0, N->stream, ri, wi,
                       reinterpret_cast<const double2*>(chi[i]), N->sumsq, V, N->X0);
    if (net_forward(N)) return VIE_EDEVICE;
    const float gscale = 2.0f / (6.0f * (float)V * (float)count);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, N->stream, N->out, reinterpret_cast<const double2*>(target[i]),
                       wi ? wi : ri, N->sumsq, V, N->gOut, gscale, N->lpart);
    if (net_backward(N, i > 0 ? 1 : 0)) return VIE_EDEVICE;
    if (hipMemcpyAsync(N->lpart_h, N->lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, N->stream) ||
        hipStreamSynchronize(N->stream))
      return VIE_EDEVICE;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += N->lpart_h[b];
    total += s / (6.0 * (double)V);
  }
  if (refresh_weights(N, 1, lr) || hipStreamSynchronize(N->stream)) return VIE_EDEVICE;
  if (loss) *loss = total / count;
  return VIE_OK;
}

// Diagnostic single-layer operations on FP32 device buffers (converted to BF16
// on the way in, FP32 out) for parity tests: mode 0 forward (relu optional),
// 1 input gradient, 2 weight gradient.
int vie_nn_conv_test(int mode, const int dims[3], int taps, int cin, int cout, const float* x, const float* w,
                     float* out, int relu, void* hip_stream) {
  if (!dims || !x || !out || (taps != 1 && taps != 27) || cin % 16 || cout % 16 || cin < 16 || cout < 16)
    return VIE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const Vol vol{dims[0], dims[1], dims[2]};
  const long V = vol.V();
  const long nw = (long)taps * cin * cout;
  std::vector<void*> tmp;
  auto al = [&](size_t b) {
    void* p = nullptr;
    if (dmalloc(&p, b)) return (void*)nullptr;
    tmp.push_back(p);
    return p;
  };
  auto fin = [&](int c) {
    (void)hipStreamSynchronize(s);
    for (void* p : tmp) (void)hipFree(p);
    return c;
  };
  // convert inputs: x has (mode 0, 2: cin; mode 1: cout) channels per voxel
  const int xc = mode == 1 ? cout : cin;
  bf16_t* xb = (bf16_t*)al(sizeof(bf16_t) * V * xc);
  if (!xb) return fin(VIE_ENOMEM);
  hipLaunchKernelGGL(k_f2bf, dim3(gblocks(V * xc)), dim3(256), 0, s, x, xb, V * xc);
  if (mode == 2) {
    // w holds dY (cout channels per voxel)
    bf16_t* yb = (bf16_t*)al(sizeof(bf16_t) * V * cout);
    float* part = (float*)al(sizeof(float) * (8L << 20));
    if (!yb || !part) return fin(VIE_ENOMEM);
    hipLaunchKernelGGL(k_f2bf, dim3(gblocks(V * cout)), dim3(256), 0, s, w, yb, V * cout);
    if (wgrad_launch(taps, xb, cin, 0, cin, yb, cout, 0, cout, part, 8L << 20, out, 0, vol, s)) return fin(VIE_EDEVICE);
    return fin(VIE_OK);
  }
  // weights [taps][cout][cin] FP32 -> BF16 forward copy and flipped-transposed copy
  float* w32 = (float*)al(sizeof(float) * nw);
  float* dummy = (float*)al(sizeof(float) * nw);
  bf16_t* wbf = (bf16_t*)al(sizeof(bf16_t) * nw);
  bf16_t* wtbf = (bf16_t*)al(sizeof(bf16_t) * nw);
  if (!w32 || !dummy || !wbf || !wtbf) return fin(VIE_ENOMEM);
  if (hipMemcpyAsync(w32, w, sizeof(float) * nw, hipMemcpyDeviceToDevice, s)) return fin(VIE_EDEVICE);
  hipLaunchKernelGGL(k_adam, dim3(gblocks(nw)), dim3(256), 0, s, w32, dummy, dummy, dummy, nw, adam_constants(1, 0.f),
                     taps, cout, cin, wbf, wtbf, 0);
  hipError_t e;
  if (mode == 0)
    e = conv_launch(taps, xb, cin, 0, cin, wbf, cout, nullptr, 0, 0, out, vol, relu, nullptr, 0, 0, s);
  else
    e = conv_launch(taps, xb, cout, 0, cout, wtbf, cin, nullptr, 0, 0, out, vol, 0, nullptr, 0, 0, s);
  return fin(e ? VIE_EDEVICE : VIE_OK);
}

int vie_net_get_grads(vie_net_t N, float* host, size_t count) {
  size_t c = 0;
  if (!N || !host || vie_net_num_params(N, &c) || c != count) return VIE_EINVAL;
  if (hipStreamSynchronize(N->stream)) return VIE_EDEVICE;
  size_t off = 0;
  for (auto& L : N->L) {
    if (hipMemcpy(host + off, L.g, sizeof(float) * L.n(), hipMemcpyDeviceToHost)) return VIE_EDEVICE;
    off += L.n();
  }
  return VIE_OK;
}

// Diagnostic pooling / upsampling on FP32 device buffers (rounded to bfloat16 on
// entry, bfloat16 results widened to FP32), C channels per voxel, fine grid dims:
// op 0 pool x[fine] -> out[coarse]; 1 pool gradient x = dY[coarse] -> out[fine],
// masked by mask[fine] > 0 when mask != NULL and added to acc[fine] when acc != NULL;
// 2 upsampling x[coarse] -> out[fine]; 3 its gradient x = dY[fine] -> out[coarse].
int vie_nn_op_test(int op, const int dims[3], int C, const float* x, const float* mask, const float* acc,
                   float* out, void* hip_stream) {
  if (!dims || !x || !out || C < 8 || C % 8 || op < 0 || op > 3) return VIE_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (dims[d] < 2 || dims[d] % 2) return VIE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const Vol fine{dims[0], dims[1], dims[2]};
  const long Vf = fine.V(), Vc = Vf / 8;
  const long nin = (op == 0 || op == 3) ? Vf * C : Vc * C;
  const long nout = (op == 0 || op == 3) ? Vc * C : Vf * C;
  std::vector<void*> tmp;
  auto al = [&](size_t b) {
    void* p = nullptr;
    if (dmalloc(&p, b)) return (void*)nullptr;
    tmp.push_back(p);
    return p;
  };
  auto fin = [&](int c) {
    (void)hipStreamSynchronize(s);
    for (void* p : tmp) (void)hipFree(p);
    return c;
  };
  bf16_t* xb = (bf16_t*)al(sizeof(bf16_t) * nin);
  bf16_t* ob = (bf16_t*)al(sizeof(bf16_t) * nout);
  if (!xb || !ob) return fin(VIE_ENOMEM);
  hipLaunchKernelGGL(k_f2bf, dim3(gblocks(nin)), dim3(256), 0, s, x, xb, nin);
  bf16_t* mb = nullptr;
  if (op == 1 && mask) {
    if (!(mb = (bf16_t*)al(sizeof(bf16_t) * nout))) return fin(VIE_ENOMEM);
    hipLaunchKernelGGL(k_f2bf, dim3(gblocks(nout)), dim3(256), 0, s, mask, mb, nout);
  }
  if (op == 1 && acc) hipLaunchKernelGGL(k_f2bf, dim3(gblocks(nout)), dim3(256), 0, s, acc, ob, nout);
  if (op == 0)
    hipLaunchKernelGGL(k_pool, dim3(gblocks(nout)), dim3(256), 0, s, xb, C, 0, ob, C, 0, C, fine);
  else if (op == 1)
    hipLaunchKernelGGL(k_pool_grad, dim3(gblocks(nout)), dim3(256), 0, s, xb, C, 0, ob, C, 0, C, fine, mb, C, 0,
                       acc ? 1 : 0);
  else if (op == 2)
    hipLaunchKernelGGL(k_up, dim3(gblocks(nout)), dim3(256), 0, s, xb, C, 0, ob, C, 0, C, fine);
  else
    hipLaunchKernelGGL(k_up_grad, dim3(gblocks(nout)), dim3(256), 0, s, xb, C, 0, ob, C, 0, C, fine);
  hipLaunchKernelGGL(k_bf2f, dim3(gblocks(nout)), dim3(256), 0, s, ob, out, nout);
  return fin(hipGetLastError() ? VIE_EDEVICE : VIE_OK);
}

// Diagnostic Adam step t (t >= 1) on n FP32 device values in place: w, m, v updated
// with gradient g as the training step does.
int vie_nn_adam_test(long n, float* w, float* m, float* v, const float* g, int t, float lr, void* hip_stream) {
  if (n < 1 || !w || !m || !v || !g || t < 1 || !(lr >= 0)) return VIE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  bf16_t *wb = nullptr, *wtb = nullptr;
  if (dmalloc(&wb, sizeof(bf16_t) * n)) return VIE_ENOMEM;
  if (dmalloc(&wtb, sizeof(bf16_t) * n)) {
    (void)hipFree(wb);
    return VIE_ENOMEM;
  }
  hipLaunchKernelGGL(k_adam, dim3(gblocks(n)), dim3(256), 0, s, w, m, v, g, n, adam_constants(t, lr), 1, 1, (int)n,
                     wb, wtb, 1);
  const hipError_t e = hipGetLastError();
  (void)hipStreamSynchronize(s);
  (void)hipFree(wb);
  (void)hipFree(wtb);
  return e ? VIE_EDEVICE : VIE_OK;
}

const char* vie_net_last_error(vie_net_t N) { return N ? N->err.c_str() : ""; }

}  // extern "C"
