// Workgroup-to-work maps of the product's pass kernels, compiled for host and
// device: the kernels call them, and vie_check_block_maps runs the same code on
// the host over every supported shape (each map a bijection onto its range,
// every write inside its buffer).
//
// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b on XCD b % 8);
// the maps below put workgroups that share cache lines or spectrum slabs on one
// XCD, dispatched close together.
#pragma once
#include <hip/hip_runtime.h>

namespace vie {

// Pencil block of the z passes: blk -> component c, row i2 and the pencils
// i1 = i1_0 .. i1_0 + np - 1 (P per block, fewer in the last block of a row).
// Blocks run over 3 n2 ceil(n1 / P).
struct PencilBlock {
  int c, i2, i1_0, np;
};
__host__ __device__ __forceinline__ PencilBlock pencil_block(int blk, int n1, int n2, int P) {
  const int nb1 = (n1 + P - 1) / P;
  const int ib1 = blk % nb1;
  blk /= nb1;
  PencilBlock r;
  r.i2 = blk % n2;
  r.c = blk / n2;
  r.i1_0 = ib1 * P;
  r.np = n1 - r.i1_0 < P ? n1 - r.i1_0 : P;
  return r;
}
__host__ __device__ __forceinline__ int pencil_blocks(int n1, int n2, int P) { return 3 * n2 * ((n1 + P - 1) / P); }

// Generic z passes (one pencil block per workgroup): eight consecutive pencil
// blocks, which read and write the same cache lines of the kz-plane-major
// intermediate, go to workgroups b, b + 8, ..., b + 56 (one XCD).  A bijection on
// every full group of 64 workgroups; identity on a tail shorter than 64.
__host__ __device__ __forceinline__ int xcd_group8(int b, int nblocks) {
  const int base = (b / 64) * 64;
  if (base + 64 > nblocks) return b;
  const int r = b - base;
  return base + (r % 8) * 8 + r / 8;
}

// Four-step z passes: the G = 128 / (P value bytes) blocks that share a 128-byte
// line of the intermediate (at least 2, at most 8) go to workgroups b, b + 8, ...,
// b + 8 (G - 1).  A bijection on every full group of 8 G workgroups; identity on
// a shorter tail.
__host__ __device__ __forceinline__ int xcd_group(int b, int nblocks, int P, int value_bytes) {
  int G = 128 / (P * value_bytes);
  G = G < 2 ? 2 : (G > 8 ? 8 : G);
  const int base = (b / (8 * G)) * (8 * G);
  if (base + 8 * G > nblocks) return b;
  const int r = b - base;
  return base + (r % 8) * G + r / 8;
}

// Plane pair p of the cross-section passes: (0, M3/2) for p = 0, (p, M3 - p)
// otherwise (p < M3 / 2; for M3 = 1 the single plane 0).
__host__ __device__ __forceinline__ void pair_planes(int p, int M3, int* a, int* b) {
  *a = p == 0 ? 0 : p;
  *b = p == 0 ? M3 / 2 : M3 - p;
}

// kz plane of workgroup b in the cross-section passes (one plane per workgroup,
// M3 workgroups).  Planes kz and M3 - kz read the same slab of the folded spectra,
// so pair p goes to workgroups 16 (p / 8) + p % 8 and that + 8: one XCD, one after
// the other.  Identity when M3 is not a multiple of 16.
__host__ __device__ __forceinline__ int paired_plane(int b, int M3) {
  if (M3 % 16 != 0) return b;
  const int base = (b / 16) * 16, r = b - base;
  int pa, pb;
  pair_planes(base / 2 + (r % 8), M3, &pa, &pb);
  return r < 8 ? pa : pb;
}

}  // namespace vie
