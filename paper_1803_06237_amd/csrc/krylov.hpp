// Krylov building blocks launched on a stream (implementations in krylov.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "fft_device.hpp"

namespace vie {

template <typename T>
struct KrylovOps {
  // out[0].x = ||w||^2 (FP64 accumulation); partial needs partial_blocks(n) entries
  // gate (device, optional): when *gate == 0 at run time the kernels do nothing
  static hipError_t nrm2sq(const cx<T>* w, long n, double2* partial, double2* out, hipStream_t s,
                           const int* gate = nullptr);
  // out[i] (+)= V_i^H w for i < nv; partial needs nv * partial_blocks(n) entries
  static hipError_t mdot(const cx<T>* V, long ldv, int nv, const cx<T>* w, long n, double2* partial,
                         double2* out, int accumulate, hipStream_t s, const int* gate = nullptr);
  // w += sign * sum_i coef[i] V_i
  template <typename TW>
  static hipError_t maxpy(const cx<T>* V, long ldv, int nv, const double2* coef, double sign, cx<TW>* w, long n,
                          hipStream_t s, const int* gate = nullptr);
  // *gate = 1 when ||w'||^2 = sumsq->x < ||h1||^2 (second sweep needed), else 0 and h2 = 0
  static hipError_t dgks(const double2* h1, int nv, const double2* sumsq, int* gate, double2* h2, hipStream_t s);
  // maxpy (nv <= 512) that also writes the block partial sums of |w|^2 to partial[0, maxpy_blocks(n))
  template <typename TW>
  static hipError_t maxpy_nrm(const cx<T>* V, long ldv, int nv, const double2* coef, double sign, cx<TW>* w, long n,
                              double2* partial, hipStream_t s, const int* gate = nullptr);
  // sumsq = sum of nblk partials, then the second-sweep decision of dgks in the same block
  static hipError_t reduce_dgks(const double2* partial, int nblk, double2* sumsq, const double2* h1, int nv,
                                int* gate, double2* h2, hipStream_t s);
  // out[0].x = sum of nblk partials
  static hipError_t reduce(const double2* partial, int nblk, double2* out, hipStream_t s, const int* gate = nullptr);
  // dst = src / sqrt(sumsq->x)
  static hipError_t scale(const cx<T>* src, cx<T>* dst, long n, const double2* sumsq, hipStream_t s);
  static hipError_t zero(cx<T>* dst, long n, hipStream_t s);
  static hipError_t arnoldi_update(const double2* h1, const double2* h2, const double2* sumsq, double2* H, int ldh, double* cs,
                                   double2* sn, double2* g, int j, double bnorm, double* state, hipStream_t s);
  static hipError_t trisolve(const double2* H, int ldh, const double2* g, int k, double2* y, hipStream_t s);
  static hipError_t set_g(double2* g, int m, const double2* sumsq, hipStream_t s);
};

template <typename TS, typename TD>
hipError_t convert(const cx<TS>* src, cx<TD>* dst, long n, hipStream_t s);

// The voxel columns (i1, i2) where the contrast is non-zero on some slice.  A
// maps vectors supported on these columns (all slices, all three components) to
// vectors supported there, so Krylov vectors can be stored compressed:
// comp[(a s + p) n3 + i3] = full[a][col[p]][i3] with col[p] = i1 n2 + i2.
struct Support {
  const int* col;   // device, s entries, increasing
  int s;
  long n12;         // n1 n2
  int n3;
  long size() const { return 3L * s * n3; }
};
// comp = full on the support (sub != nullptr: comp = sub - full on the support; may alias comp)
template <typename T>
hipError_t gather(const Support& u, const cx<T>* full, cx<T>* comp, const cx<T>* sub, hipStream_t s);
// full on the support = comp (other entries untouched)
template <typename T>
hipError_t scatter(const Support& u, const cx<T>* comp, cx<T>* full, hipStream_t s);
// full on the support = 0
template <typename T>
hipError_t zero_support(const Support& u, cx<T>* full, hipStream_t s);
// flags[c] = 1 if chi[c][i3] != 0 for some i3, else 0 (c < n12)
hipError_t column_flags(const double2* chi, long n12, int n3, int* flags, hipStream_t s);

int partial_blocks(long n);
// blocks (partial sums) of maxpy_nrm over n elements
int maxpy_blocks(long n);

}  // namespace vie
