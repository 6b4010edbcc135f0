// Internal declarations shared by the host side of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstddef>
#include <string>

namespace vie {

// Host FP64 Toeplitz table (green_table.cpp): out[6][n1][n2][n3].
int green_table(const int n[3], double kappa, std::complex<double>* out, int nthreads);
// Host FP64 table of K = curl S (green_table.cpp): out[3][n1][n2][n3], components
// (0,1), (0,2), (1,2) at h = 1.
int curl_table(const int n[3], double kappa, std::complex<double>* out, int nthreads);

// Geometry and launch shapes of one operator, passed to the kernel launchers.
struct Geom {
  int n1, n2, n3;           // voxel grid
  int M1, M2, M3;           // circulant sizes (powers of two)
  int L1, L2, L3;           // log2 of M
  int H1, H2, H3;           // octant extents M/2 + 1
  long N;                   // voxels
};

struct Tune {
  int tp;        // z-pencils per workgroup in the z passes
  int zthreads;  // threads per workgroup in the z passes
  int cc;        // column chunk in the xy pass
  int xythreads; // threads per workgroup in the xy pass
  int z4;        // 1: z passes use the register four-step kernels
  int xyv;       // xy pass variant; 64 x 64: 0 full plane, 1 x-frequency halves, 2 wide;
                 // 64 x 32: 0 generic padded LDS pass, 1 and 2 register transforms
                 // (1: column exchange areas of their own, 2: exchange in the hand-off)
  int zp;        // pencils per workgroup in the four-step z passes (0: the default for M3)
};

// Number of xy pass variants of a cross-section: 3 for 64 x 64 and 64 x 32, else 1.
inline int xy_variants(const Geom& g) { return g.M1 == 64 && (g.M2 == 64 || g.M2 == 32) ? 3 : 1; }

// Candidate pencil counts of the four-step z passes for M3 (empty when none exist);
// the first is the default.
template <typename T>
int z4_pencil_options(int M3, int* out, int cap);

template <typename T>
size_t z4_lds_bytes(int M3, int P = 0);   // 0 when no four-step instance exists for M3

// ---- matvec passes (kernels.hip) ----------------------------------------
// mode for the inverse z pass: 0 -> y = x - chi u ; 1 -> y = b - (x - chi u)
template <typename T>
hipError_t launch_matvec(const Geom& g, const Tune& t, const void* x, void* y, const void* b, int mode,
                         void* U, const void* goct, const void* chi, const void* const tw[3],
                         hipStream_t s);

// one of the three passes (0: forward z, 1: xy + Green, 2: inverse z + contrast)
template <typename T>
hipError_t launch_pass(int which, const Geom& g, const Tune& t, const void* x, void* y, const void* b, int mode,
                       void* U, const void* goct, const void* chi, const void* const tw[3], hipStream_t s);

// ---- plan-time spectrum -----------------------------------------------------
hipError_t launch_spectrum(const Geom& g, const double2* table_dev, double2* full_tmp, double2* goct64,
                           float2* goct32, const double2* const tw64[3], hipStream_t s);

hipError_t launch_curl_spectrum(const Geom& g, const double2* ktable_dev, double2* full_tmp, double2* koct64,
                                float2* koct32, const double2* const tw64[3], hipStream_t s);

// LDS bytes of the generic xy pass with column chunks of cc x-frequencies
template <typename T>
size_t xy_lds_bytes(const Geom& g, int cc);

// ---- JM-VIE product (jm.hip) --------------------------------------------------
// y = (I - M T~) x on 6N vectors (electric then magnetic, each [3][n1][n2][n3]);
// mode 1: y = b - (I - M T~) x.  Ue, Um: z-pass intermediates of each half.
// fused: one cross-section kernel with the spectra in LDS (requires
// jm_fused_shape); otherwise the spectra go through S, jm_spectrum_values(g)
// values.  M1 M2 <= 4096.
size_t jm_spectrum_values(const Geom& g);
template <typename T>
bool jm_fused_shape(const Geom& g, int* cc, int* threads, int* split = nullptr);
template <typename T>
hipError_t allow_lds_jm();
template <typename T>
hipError_t launch_jm_matvec(const Geom& g, const Tune& t, const void* x, void* y, const void* b, int mode,
                            void* Ue, void* Um, void* S, const void* goct, const void* koct, const void* chi_e,
                            const void* chi_m, double kappa, bool fused, const void* const tw[3], hipStream_t s);

// ---- contrast / rhs ---------------------------------------------------------
hipError_t launch_contrast(long N, const double2* eps, double eps_b, double2* chi64, float2* chi32,
                           int* bad_flag, hipStream_t s);
hipError_t launch_rhs(long N, double scale, const double2* chi, const double2* einc, double2* b,
                      hipStream_t s);

// ---- batched passes ---------------------------------------------------------
// One system of a batch as seen by the batched pass kernels.  The vector
// operands are xb + jx * xs and yb + jy * ys (elements), with (jx, jy) passed
// to the launch, so one descriptor serves every Krylov step of a cycle.
struct PassDesc {
  Geom g;
  const void* xb;
  long xs;
  void* yb;
  long ys;
  const void* b;        // residual mode: y = b - A x
  void* U;
  const void* goct;
  const void* chi;
  const void* twz;      // z twiddles, length M3
  const void* twx;      // x twiddles, length M1
  int P;                // pencils per workgroup in the z passes
  const int* active;    // device flag; 0 skips the system (nullptr: always on)
};

// which: 0 forward z, 1 xy + Green, 2 inverse z (+ contrast; mode 1: residual).
// items: prefix[s] = first item of system s (z passes: pencil blocks; xy pass:
// plane pairs), prefix[nsys] = total.  All systems share (A, B) for the z passes.
template <typename T>
hipError_t launch_pass_batch(int which, int mode, const PassDesc* d, const int* prefix, int nsys, int total, int A,
                             int B, int P, int jx, int jy, hipStream_t s);
template <typename T>
bool z4_shape(int M3, int* A, int* B, int* P);

// ---- Krylov building blocks (krylov.hip) -----------------------------------
template <typename T>
struct KrylovWork;

// ---- block-circulant preconditioner (circulant.hip) -------------------------
struct CircInfo {
  int s;          // support columns
  int m;          // block size 3 s
  int fp64;       // 1: inverse blocks kept in FP64
  size_t bytes;   // device bytes of the inverse blocks
  double seconds; // set-up wall time
  int z0, P;      // slice window of the circulant
};
struct Circ;
// Builds W^{-1} for the contrast chi64 (device, FP64) with the host Toeplitz table.
int circ_build(Circ** out, const Geom& g, const std::complex<double>* table, const double2* chi64, bool fp64,
               hipStream_t s, std::string& err, CircInfo* info);
// z = W^{-1} r on FP64 device vectors of 3N values (no overlap).
hipError_t circ_apply(Circ* c, const double2* r, double2* z, hipStream_t s);
// The same on support-compressed FP64 vectors (3 s n3 values, rows (a, p) of n3 slices,
// columns in increasing i1 n2 + i2 order, as the solver stores them).
hipError_t circ_apply_rows(Circ* c, const double2* r, double2* z, hipStream_t s);
void circ_destroy(Circ* c);
const CircInfo& circ_info(const Circ* c);

// Device allocation used throughout the library.  With VIE_DEBUG_NANFILL=1 in the
// environment every fresh allocation is filled with all-ones bytes (a NaN in FP32
// and FP64), so a kernel that reads memory nothing has written shows NaN in its
// results instead of stale zeros.
hipError_t dmalloc_bytes(void** p, size_t bytes);
template <typename P>
inline hipError_t dmalloc(P** p, size_t bytes) {
  return dmalloc_bytes(reinterpret_cast<void**>(p), bytes);
}

// LDS budget the kernels may use per workgroup (queried once per device)
size_t lds_budget(int device);

struct Tune;
}  // namespace vie
typedef struct vie_plan_s* vie_plan_t;
namespace vie {
// The parts of a plan the batched solver needs (vie_api.cpp).
int plan_export(vie_plan_t p, Geom* g, Tune* t64, Tune* t32, void** U64, void** U32, void** goct64, void** goct32,
                void** chi64, void** chi32, const void** tw64, const void** tw32, hipStream_t* stream,
                int* has_contrast);
// The plan's block-circulant preconditioner, or null when none is built.
Circ* plan_circ(vie_plan_t p);
// The plan's support columns (device, *ns increasing indices i1 n2 + i2 where the
// contrast is non-zero on some slice), valid while the contrast is unchanged.
int plan_support(vie_plan_t p, const int** col, int* ns);

}  // namespace vie
