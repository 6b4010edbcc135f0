// LDS maps of the 64 x 32 cross-section pass (xy6432.hip), shared with the host
// check (maps_check.cpp) that enumerates them for bijection, extents and LDS bank
// conflicts.
#pragma once
#include <hip/hip_runtime.h>

namespace vie {

constexpr int kXy32HandVals = 3 * 16 * 64;   // hand-off: 3 x 16 rows of 64 x-frequencies
constexpr int kXy32ColX = 32;                 // exchange values per column group (variant 1)

// hand-off element (c, y, kx): row (c, y), column kx ^ 10 (y & 3)
__host__ __device__ __forceinline__ int xy32_hand(int c, int y, int kx) {
  return (c * 16 + y) * 64 + (kx ^ ((y & 3) * 10));
}
// row exchange element (i, j) of row group q (f = q & 3), inside the row's 64 slots
__host__ __device__ __forceinline__ int xy32_rowx(int i, int j, int f) { return (i ^ f) * 8 + ((i + j) & 7); }
// column exchange element (a, k) of column group g (r = g & 3), inside its own area
__host__ __device__ __forceinline__ int xy32_colx(int a, int k, int r) {
  return ((k + r) & 7) * 4 + (a ^ ((k >> 1) & 3));
}
// column exchange element (a, k) of column kx inside the column's own hand-off
// entries of components 0 and 1 (the four lanes of a group always differ in y & 3)
__host__ __device__ __forceinline__ int xy32_cslot(int a, int k, int kx) {
  const int kh = k >> 1;
  return xy32_hand(k & 1, (kh << 2) | ((a + kh) & 3), kx);
}
// row task i (0, 1) of row group q (0..31): component and row; only q < 16 has task 1
__host__ __device__ __forceinline__ void xy32_row_task(int q, int i, int* c, int* y) {
  if (q < 16) {
    *c = i == 0 ? 0 : 2;
    *y = q;
  } else {
    *c = 1;
    *y = q - 16;
  }
}

}  // namespace vie
