// Radix-8/4/2 Stockham transforms of LDS-resident cross-section data with
// bank-conflict-free layouts, shared by the generic J-VIE xy pass and the fused
// JM pass.
//
// Rows: sequence s (a row along x) lives at A + s pitch with element k at
// pad8(k) = k + k/8 (one spare slot per 8; pitch M1 + M1/8).  The radix-8
// stage writes element 8j + r from lane j: the spare slots spread those
// strides over all banks, for 16-byte (FP64) and 8-byte (FP32) values alike.
// Lanes run along j, then along rows.
//
// Column chunks: cc x-frequencies of nc components, stored position-major,
// C[comp][pad8(k)][col] (M2p = M2 + M2/8 positions), with consecutive lanes on
// consecutive columns.  The first forward stage reads the chunk straight from
// the rows (rows comp n2 + k, k < n2) and the last inverse stage writes the
// kept positions k < n2 straight back, so there is no separate gather or
// scatter pass; with fewer than two stages explicit copies do it.
//
// Every stage holds at most kPadMaxV values per thread (nseq L <= 8 blockDim);
// the callers size their workgroups for that.  tid is the caller's thread
// index (an opaque copy inside loops keeps per-lane address terms from being
// hoisted across iterations).
#pragma once

#include "block_maps.hpp"
#include "fft_device.hpp"

namespace vie {

__device__ __forceinline__ int pad8(int k) { return k + (k >> 3); }

constexpr int kPadMaxV = 8;   // values per thread per stage

// One radix-R stage over nseq row sequences of length 2^Llog2 at A + s pitch.
template <typename T, int R, bool INV>
__device__ __forceinline__ void pad_row_stage(cx<T>* A, int nseq, int pitch, int Llog2, int Nslog2, int valid,
                                             const cx<T>* tw, int tid) {
  constexpr int TPT = kPadMaxV / R;
  constexpr int Rlog2 = R == 2 ? 1 : (R == 4 ? 2 : 3);
  const int perlog2 = Llog2 - Rlog2;
  const int total = nseq << perlog2;
  cx<T> v[TPT][R];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int t = tid + q * blockDim.x;
    if (t < total) {
      const int s = t >> perlog2, j = t & ((1 << perlog2) - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = j + (r << perlog2);
        v[q][r] = k < valid ? A[s * pitch + pad8(k)] : cx<T>{(T)0, (T)0};
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int t = tid + q * blockDim.x;
    if (t < total) {
      const int s = t >> perlog2, j = t & ((1 << perlog2) - 1);
      const int jm = j & ((1 << Nslog2) - 1);
      if (Nslog2 > 0) {
        const int step = 1 << (Llog2 - Nslog2 - Rlog2);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w = tw[r * jm * step];
          v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
        }
      }
      dft<T, R, INV>(v[q]);
      const int o = ((j >> Nslog2) << (Nslog2 + Rlog2)) + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) A[s * pitch + pad8(o + (r << Nslog2))] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, bool INV>
__device__ __forceinline__ void pad_rows(cx<T>* A, int nseq, int pitch, int Llog2, int valid, const cx<T>* tw,
                                        int tid) {
  int ns = 0, rem = Llog2;
  bool first = true;
  while (rem >= 3) {
    pad_row_stage<T, 8, INV>(A, nseq, pitch, Llog2, ns, first ? valid : (1 << Llog2), tw, tid);
    ns += 3;
    rem -= 3;
    first = false;
  }
  if (rem == 2) pad_row_stage<T, 4, INV>(A, nseq, pitch, Llog2, ns, first ? valid : (1 << Llog2), tw, tid);
  else if (rem == 1) pad_row_stage<T, 2, INV>(A, nseq, pitch, Llog2, ns, first ? valid : (1 << Llog2), tw, tid);
}

// Where a column stage reads and writes: the chunk C, or (first forward stage /
// last inverse stage) the rows, element k of column (comp, col) being
// A[(comp n2 + k) pitch + pad8(c0 + col)], k < n2.
struct PadCols {
  int nc, cclog, M2p, n2, pitch, c0;   // nc components in the chunk
};

template <typename T, int R, bool INV, bool SRC_ROWS, bool DST_ROWS>
__device__ __forceinline__ void pad_col_stage(cx<T>* A, cx<T>* C, const PadCols& m, int Llog2, int Nslog2, int valid,
                                             const cx<T>* tw, int tid) {
  constexpr bool src_rows = SRC_ROWS, dst_rows = DST_ROWS;
  constexpr int TPT = kPadMaxV / R;
  constexpr int Rlog2 = R == 2 ? 1 : (R == 4 ? 2 : 3);
  const int perlog2 = Llog2 - Rlog2;
  const int total = (m.nc << m.cclog) << perlog2;
  const int ccm = (1 << m.cclog) - 1;
  cx<T> v[TPT][R];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int t = tid + q * blockDim.x;
    if (t < total) {
      const int col = t & ccm, j = (t >> m.cclog) & ((1 << perlog2) - 1), comp = t >> (m.cclog + perlog2);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = j + (r << perlog2);
        cx<T> x{(T)0, (T)0};
        if (k < valid)
          x = src_rows ? A[(comp * m.n2 + k) * m.pitch + pad8(m.c0 + col)]
                       : C[((comp * m.M2p + pad8(k)) << m.cclog) + col];
        v[q][r] = x;
      }
    }
  }
  if (src_rows == dst_rows) __syncthreads();   // in place: every read before any write
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int t = tid + q * blockDim.x;
    if (t < total) {
      const int col = t & ccm, j = (t >> m.cclog) & ((1 << perlog2) - 1), comp = t >> (m.cclog + perlog2);
      const int jm = j & ((1 << Nslog2) - 1);
      if (Nslog2 > 0) {
        const int step = 1 << (Llog2 - Nslog2 - Rlog2);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w = tw[r * jm * step];
          v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
        }
      }
      dft<T, R, INV>(v[q]);
      const int o = ((j >> Nslog2) << (Nslog2 + Rlog2)) + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = o + (r << Nslog2);
        if (dst_rows) {
          if (k < m.n2) A[(comp * m.n2 + k) * m.pitch + pad8(m.c0 + col)] = v[q][r];
        } else {
          C[((comp * m.M2p + pad8(k)) << m.cclog) + col] = v[q][r];
        }
      }
    }
  }
  __syncthreads();
}

// Column transform of the chunk: forward from the rows into C, or inverse from C
// back into the rows (the first / last stage does the hand-over).  Fewer than two
// stages: explicit copies around the stages.
template <typename T, bool INV>
__device__ __forceinline__ void pad_cols(cx<T>* A, cx<T>* C, const PadCols& m, int Llog2, const cx<T>* tw, int tid) {
  const int nst = Llog2 == 0 ? 0 : (Llog2 + 2) / 3;
  const int ccm = (1 << m.cclog) - 1;
  if (nst < 2 && !INV) {
    for (int t = tid; t < (m.nc * m.n2) << m.cclog; t += blockDim.x) {
      const int col = t & ccm, rc = t >> m.cclog;   // rc = comp * n2 + k
      const int comp = rc / m.n2, k = rc - comp * m.n2;
      C[((comp * m.M2p + pad8(k)) << m.cclog) + col] = A[rc * m.pitch + pad8(m.c0 + col)];
    }
    // positions n2 <= k < M2 stay unread: the transform takes them as zero
    __syncthreads();
  }
  int ns = 0, rem = Llog2, st = 0;
  while (rem > 0) {
    const int R = rem >= 3 ? 8 : (rem == 2 ? 4 : 2);
    const bool src_rows = !INV && st == 0 && nst >= 2;
    const bool dst_rows = INV && st == nst - 1 && nst >= 2;
    const int valid = (!INV && st == 0) ? m.n2 : (1 << Llog2);
    if (src_rows) {
      // first forward stage (INV false): radix 8, 4 or 2 from the rows
      if (R == 8) pad_col_stage<T, 8, INV, true, false>(A, C, m, Llog2, ns, valid, tw, tid);
      else if (R == 4) pad_col_stage<T, 4, INV, true, false>(A, C, m, Llog2, ns, valid, tw, tid);
      else pad_col_stage<T, 2, INV, true, false>(A, C, m, Llog2, ns, valid, tw, tid);
    } else if (dst_rows) {
      if (R == 8) pad_col_stage<T, 8, INV, false, true>(A, C, m, Llog2, ns, valid, tw, tid);
      else if (R == 4) pad_col_stage<T, 4, INV, false, true>(A, C, m, Llog2, ns, valid, tw, tid);
      else pad_col_stage<T, 2, INV, false, true>(A, C, m, Llog2, ns, valid, tw, tid);
    } else {
      if (R == 8) pad_col_stage<T, 8, INV, false, false>(A, C, m, Llog2, ns, valid, tw, tid);
      else if (R == 4) pad_col_stage<T, 4, INV, false, false>(A, C, m, Llog2, ns, valid, tw, tid);
      else pad_col_stage<T, 2, INV, false, false>(A, C, m, Llog2, ns, valid, tw, tid);
    }
    ns += R == 8 ? 3 : (R == 4 ? 2 : 1);
    rem -= R == 8 ? 3 : (R == 4 ? 2 : 1);
    ++st;
  }
  if (nst < 2 && INV) {
    for (int t = tid; t < (m.nc * m.n2) << m.cclog; t += blockDim.x) {
      const int col = t & ccm, rc = t >> m.cclog;
      const int comp = rc / m.n2, k = rc - comp * m.n2;
      A[rc * m.pitch + pad8(m.c0 + col)] = C[((comp * m.M2p + pad8(k)) << m.cclog) + col];
    }
    __syncthreads();
  }
}

}  // namespace vie
