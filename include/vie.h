/*
 * vie.h -- C ABI of the MI355X voxel J-VIE solver.
 *
 * The library solves the discrete J-VIE of the paper (Section III, boxed J-VIE;
 * discrete form in Section III-A and again in Section V-D):
 *
 *     (I - M_eps N) w = b,       b = M_eps e_inc  (the constant c_e is dropped)
 *
 * on a uniform grid of n1 x n2 x n3 cubic voxels of edge h.  N is the Galerkin
 * matrix of curl curl S for normalised voxel indicators (Section III-A); it is
 * block Toeplitz with six unique symmetric tensor components, and its product
 * with a vector is done by circulant embedding and FFTs (Section III-A, last
 * paragraph; Section V-D).  M_eps is diagonal with (eps_r - 1)/eps_r per voxel,
 * eps_r = eps/eps_b (Section III; background scaled to one as in Section II).
 * Absorbers (Section IV) enter only through eps.
 *
 * Conventions
 *   - Time dependence exp(-i omega t): the kernel is e^{+i k_b R}/(4 pi R) with
 *     k_b = k0 sqrt(eps_b), and passive media have Im eps >= 0.  This is the
 *     complex conjugate of the paper's exp(+j omega t) system; all real
 *     observables agree.
 *   - Vectors are complex, interleaved (re, im), component-major
 *     [3][n1][n2][n3] in C order (n3 fastest), i.e. a contiguous tensor of
 *     shape (3, n1, n2, n3).  Per-voxel arrays are [n1][n2][n3].
 *   - "device" pointers are HIP device memory on the plan's device; the caller
 *     owns every buffer it passes, the library never keeps caller pointers.
 *   - Every call is ordered on the plan's HIP stream.  vie_matvec* and
 *     vie_set_contrast return without synchronising; vie_solve* synchronise.
 *   - Errors: every int-returning call returns VIE_OK or a negative code; no
 *     exception or abort crosses the ABI.  vie_last_error() gives the message.
 *
 * Size limits of this version: n1, n2 <= 32 and n3 <= 2048 (circulant lengths
 * up to 64, 64 and 4096); each circulant length is the power of two
 * >= 2 n_d - 1.
 */
#ifndef VIE_H
#define VIE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vie_plan_s* vie_plan_t;            /* opaque; owned by the library until vie_destroy */
typedef struct vie_net_s* vie_net_t;              /* opaque learned preconditioner; vie_net_destroy */
typedef struct { double re, im; } vie_c128;       /* interleaved FP64 complex */
typedef struct { float re, im; } vie_c64;         /* interleaved FP32 complex */

enum {
  VIE_OK = 0,
  VIE_EINVAL = -1,    /* bad argument: size, pointer, non-finite value */
  VIE_ENOMEM = -2,    /* device or host allocation failed */
  VIE_EDEVICE = -3,   /* HIP runtime error */
  VIE_ENOCONV = -4,   /* solver stopped before reaching tol; x holds the best iterate */
  VIE_ENUMERIC = -5,  /* non-finite value met during a solve */
  VIE_ESTATE = -6,    /* call out of order (e.g. matvec before set_contrast) */
  VIE_ENOTIMPL = -7
};

/* plan flags */
enum {
  VIE_FP64 = 0,        /* FP64 spectrum only */
  VIE_WITH_FP32 = 1,   /* also keep FP32 copies of spectrum and contrast (mixed tier) */
  VIE_NO_AUTOTUNE = 2  /* keep the default launch shapes (no timing at plan creation) */
};

/*
 * vie_green_table -- host-only, FP64.  Galerkin entries N^{ab}(m) of curl curl S
 * for normalised voxel indicators (Section III-A), for all non-negative offsets
 * 0 <= m_d < grid[d], dimensionless with voxel edge 1 and kappa = k_b h.
 * out: host array of 6*grid[0]*grid[1]*grid[2] vie_c128, layout
 *      [6][n1][n2][n3], components in the order xx, xy, xz, yy, yz, zz.
 * Entries for negative offsets follow by parity: negating m_d multiplies
 * N^{ab} by -1 exactly when one of a, b equals d.
 * nthreads <= 0 picks the hardware concurrency.
 */
int vie_green_table(const int grid[3], double kappa, vie_c128* out, int nthreads);

/*
 * vie_plan -- build the operator for a grid (Section III-A): the Toeplitz table
 * on the host (FP64, threaded), its circulant embedding and 3-D spectrum on the
 * device.  h and k0 in one consistent length unit; eps_b > 0 the background
 * relative permittivity.  hip_stream: a hipStream_t (NULL = default stream).
 * Returns VIE_EINVAL for sizes outside the limits above or non-positive h, k0, eps_b.
 */
int vie_plan(vie_plan_t* out, const int grid[3], double h, double k0, double eps_b,
             unsigned flags, void* hip_stream);

/*
 * vie_set_contrast -- M_eps from the relative permittivity per voxel
 * (Section III: multiplier (eps_r - 1)/eps_r; Section III-A: constant per voxel).
 * eps: device pointer, N = n1 n2 n3 values [n1][n2][n3], copied.  A voxel equal
 * to eps_b has zero contrast.  Non-finite or zero eps gives VIE_EINVAL.
 */
int vie_set_contrast(vie_plan_t plan, const vie_c128* eps);

/*
 * vie_get_contrast -- copy the plan's FP64 contrast (eps_r - 1)/eps_r per voxel into
 * chi (device, N values [n1][n2][n3]).  Asynchronous on the plan's stream.
 */
int vie_get_contrast(vie_plan_t plan, vie_c128* chi);

/*
 * vie_rhs -- b = h^{3/2} M_eps e_inc: the Galerkin projection of an incident field
 * sampled at voxel centres, times the contrast (Section III-A right-hand side).
 * e_inc, b: device, 3N values each; may alias.
 */
int vie_rhs(vie_plan_t plan, const vie_c128* e_inc, vie_c128* b);

/*
 * vie_matvec -- y = (I - M_eps N) x in FP64 (Section V-D matrix-vector product).
 * x, y: device, 3N values, must not overlap.  Asynchronous on the plan's stream.
 */
int vie_matvec(vie_plan_t plan, const vie_c128* x, vie_c128* y);

/*
 * vie_matvec_c64 -- the same product with FP32 spectrum, contrast and FFTs
 * (plan built with VIE_WITH_FP32).  x, y: device, 3N vie_c64, no overlap.
 */
int vie_matvec_c64(vie_plan_t plan, const vie_c64* x, vie_c64* y);

/*
 * vie_residual -- r = b - (I - M_eps N) x in FP64.  x, b, r device, 3N values;
 * r may alias b but not x.
 */
int vie_residual(vie_plan_t plan, const vie_c128* x, const vie_c128* b, vie_c128* r);

typedef struct {
  int restart;        /* Krylov dimension m of GMRES(m) / outer FGMRES(m); <= 0 -> 50 */
  int maxit;          /* total outer iterations; <= 0 -> 10000 */
  int use_x0;         /* 1: x holds the initial guess; 0: start from zero */
  int precision;      /* 0: FP64 GMRES; 1: mixed (FP32 inner GMRES, FP64 outer FGMRES);
                         2: learned (FP64 FGMRES with the attached network, plain GMRES fallback);
                         3: FP64 FGMRES right-preconditioned by the block circulant of
                            vie_circulant_build;
                         4: FP64 FGMRES preconditioned by the attached network correcting
                            the block circulant, z = W^{-1} v + net(v, W^{-1} v), x0 from
                            the same map of b; the circulant FGMRES is its fallback;
                         5: mixed as 1, but the inner GMRES keeps FP64 Krylov vectors
                            and Arnoldi (FP32 products only) */
  int inner_restart;  /* mixed tier: inner GMRES dimension; <= 0 -> 20 */
  double inner_tol;   /* mixed tier: inner relative tolerance; <= 0 -> 1e-4 */
  int use_graph;      /* vie_solve_batch: 1 = capture one restart cycle as a HIP graph and replay it */
  int stall_restarts; /* vie_solve: 0 = off; k > 0 = stop with VIE_ENOCONV (info.stalled = 1)
                         once k restarts in a row each reduce the true residual by less than
                         0.1 %.  The mixed tiers (1, 5) first continue from their iterate with
                         FP64 GMRES (info.fallback = 1), which stops by the same rule. */
} vie_solve_opts;

typedef struct {
  int iters;          /* outer Arnoldi steps */
  int inner_iters;    /* FP32 matvecs spent in inner solves (mixed tier); preconditioner
                         applications (learned and circulant tiers) */
  int restarts;
  int matvecs;        /* FP64 matvecs (incl. residual checks) */
  int status;         /* same code as returned */
  double rel_res_true;   /* ||b - A x|| / ||b|| with the FP64 matvec */
  double rel_res_est;    /* last Hessenberg estimate */
  double seconds;        /* wall time of the call */
  int fallback;          /* learned tiers: 1 when they switched to the method without the
                            network; mixed tiers: 1 when a stall handed over to FP64 GMRES */
  int stalled;           /* 1 when the solve stopped by the stall_restarts rule */
} vie_solve_info;

/*
 * vie_solve -- GMRES(m) with classical Gram-Schmidt applied twice (Section V-D
 * solves with GMRES to 1e-8).  Stops when the relative residual estimate and then
 * the true FP64 relative residual ||b - A x||/||b|| are <= tol.
 * b, x: device, 3N values (x in/out).  opts, info: host, may be NULL (defaults /
 * no report).  Returns VIE_OK, or VIE_ENOCONV with the best iterate in x.
 * The Krylov basis (restart + 1 vectors of 3N FP64 complex) is allocated per call.
 */
int vie_solve(vie_plan_t plan, const vie_c128* b, vie_c128* x, double tol,
              const vie_solve_opts* opts, vie_solve_info* info);

/*
 * vie_solve_noalloc -- vie_solve for callers that cannot allocate memory during the
 * call: code that runs while a HIP graph is being captured, tight serving loops,
 * harnesses that forbid allocation.  It calls no hipMalloc, hipFree, hipHostMalloc
 * or other allocating routine: every device buffer beyond b and x (full-length
 * operator vectors, compressed right-hand side and solution, reduction partials,
 * the Krylov basis and Hessenberg data) comes from one static device array of
 * 64 MiB per GPU, held until the process ends, and the pinned slot and events it
 * waits on were made by vie_plan.  Only opts->precision 0 (GMRES) and 3 (FGMRES
 * with the block circulant, which vie_circulant_build allocated beforehand) are
 * accepted.  It needs about 16 (2 (3N) + (m + 1 + [precision 3] m) n) bytes plus
 * O(m^2 + N / 256) for restart m and the support-compressed length n = 3 |S| n3,
 * and returns VIE_EINVAL with the figure when that exceeds 64 MiB.  All calls on
 * one GPU share its array and each call starts by clearing what must start at
 * zero; calls that overlap on one GPU (other threads, other plans' streams) race
 * and must be serialised by the caller.  Results equal vie_solve's for the same
 * arguments.
 */
int vie_solve_noalloc(vie_plan_t plan, const vie_c128* b, vie_c128* x, double tol,
                      const vie_solve_opts* opts, vie_solve_info* info);

/*
 * vie_solve_batch -- `count` independent systems, each with its own plan (grids
 * may differ), solved together: every Krylov kernel and every matvec pass covers
 * all systems in one launch per kernel shape, the systems advance in lockstep,
 * and a system that reaches tol is masked on the device for the rest of its
 * restart cycle.  opts->precision 0: GMRES(restart); 1: FP64 flexible
 * GMRES(restart) preconditioned by inner_restart FP32 GMRES steps (plans built
 * with VIE_WITH_FP32); 3: FP64 flexible GMRES(restart) preconditioned by each
 * plan's block circulant (vie_circulant_build on every plan first; systems of
 * one plan share it).  With opts->use_graph one restart cycle is captured as a
 * HIP graph and replayed (precisions 0 and 1; precision 3 chooses the systems to
 * precondition on the host each cycle and runs eagerly).  rhs[s], x[s]: device, 3N_s values each, x[s] out
 * (in with use_x0).  infos: host array of count entries or NULL.  Runs on a
 * stream of its own after synchronising the first plan's stream; returns
 * synchronised.  Returns VIE_OK when every system converged, else the first
 * non-OK status (each system's status is in infos[s].status).  A plan may appear
 * several times (same operator, different right-hand sides): each system gets
 * its own intermediate buffers.  As in vie_solve, each system's Krylov vectors hold
 * only its support columns (n_s = 3 |S_s| n3 values; the system solved is
 * A_SS x_S = b_S - (A b_off)_S, and x = b off the support), and every product is
 * a batched scatter into full-length buffers, the three passes and a batched
 * gather.  Device memory per system is about 16 ((restart + 1 [+ restart when
 * flexible] + 3) n_s + 2 (3 N_s) + 3 n1 n2 M3) bytes, the last term the
 * intermediate of the passes, and the mixed tier adds half as much again for
 * its FP32 level (inner_restart + 3 vectors of n_s).  A right-hand side with a
 * non-finite value gives VIE_EINVAL.
 */
int vie_solve_batch(vie_plan_t const* plans, const vie_c128* const* rhs, vie_c128* const* x, int count,
                    double tol, const vie_solve_opts* opts, vie_solve_info* infos);

/*
 * Block-circulant preconditioner (Section V-D: the block circulant W nearest to
 * I - M_eps N in the Frobenius norm, after Chan and Olkin's preconditioners for
 * Toeplitz-block matrices; the paper's conclusion allows a circulant
 * approximation on one or more of the three Toeplitz levels).  This version
 * takes the circulant along the third axis (the long guide axis) and keeps
 * each cross-section block dense, on the support of the contrast: the voxel
 * columns S where chi is non-zero on some slice (m = 3|S|) and a window of P
 * slices from z0 that covers every slice where chi is non-zero on S (P the
 * smallest length >= that extent with prime factors 2, 3, 5, at most n3;
 * z0 the first such slice, moved down if the window would leave the grid):
 *
 *   W_k = delta_k0 I - (1/P) [ U_k N_k + (U_0 - U_k) N_{k - P} ],
 *   U_k = diag over S of sum_{i >= k} chi(i1, i2, z0 + i),
 *
 * with N_k the m x m block of N between slices k apart.  Voxels outside S x
 * window keep the identity.  The DFT along the window turns W into P dense
 * m x m blocks,
 * which are inverted once (FP64 Gauss-Jordan with partial pivoting on the
 * device); the inverses are kept in FP32 (flags 0) or FP64 (VIE_CIRC_FP64).
 *
 * vie_circulant_build: for the plan's current contrast (set_contrast first; a
 *   later set_contrast releases it).  Limits: m <= 2048, and 2 P m^2 * 16 bytes
 *   of device memory during set-up (VIE_ENOMEM otherwise).  VIE_ENUMERIC if a
 *   frequency block is singular.  info (host, may be NULL) receives the sizes,
 *   the device bytes of the kept inverses and the set-up time.  Synchronises.
 * vie_circulant_apply: z = W^{-1} r; r, z device, 3N values, no overlap.
 *   Asynchronous on the plan's stream.  vie_solve with precision 3 uses it.
 */
enum { VIE_CIRC_FP32 = 0, VIE_CIRC_FP64 = 1 };

typedef struct {
  int support_columns;   /* |S| */
  int block_size;        /* m = 3 |S| */
  int blocks;            /* P, the window length (0 when S is empty: W = I) */
  int first_slice;       /* z0 */
  int fp64;              /* 1: inverse blocks kept in FP64 */
  size_t bytes;          /* device bytes of the inverse blocks */
  double seconds;        /* set-up wall time */
} vie_circulant_info;

int vie_circulant_build(vie_plan_t plan, unsigned flags, vie_circulant_info* info);
int vie_circulant_apply(vie_plan_t plan, const vie_c128* r, vie_c128* z);

/*
 * Launch-shape tuning.  Unless VIE_NO_AUTOTUNE is given, vie_plan times the
 * candidate shapes of the product's kernels on the plan's own buffers (two
 * untimed and five timed whole products each, HIP events, in three interleaved
 * rounds of which each candidate keeps its best) and keeps the fastest:
 * pencils per workgroup of the four-step z passes, or the generic z passes
 * (circulant lengths 512 to 4096 have four-step shapes), crossed with, for
 * 64 x 64 circulant cross-sections, the xy pass variant (0: full plane in LDS;
 * 1: x-frequency halves, two workgroups per CU; 2: full plane with 512 threads
 * and private exchange areas, one workgroup per CU) and, for 64 x 32 ones (the
 * paper's strip), the xy pass (0: generic padded LDS transforms; 1: register
 * transforms with an LDS exchange area per column, two FP64 workgroups per CU;
 * 2: the same exchanging in the columns' own hand-off entries, three FP64
 * workgroups per CU); the pairs are timed jointly
 * because the z pass's writes decide what the xy pass finds in cache.  Choices
 * are cached per (device, grid, precision) for the life of the process, and in the
 * file named by the environment variable VIE_TUNE_CACHE (default
 * $XDG_CACHE_HOME or $HOME/.cache, vie-mi355x/tune.txt; empty: none), keyed by
 * the GPU architecture and CU count, the grid and the precision.
 * vie_get_tune: the current choice for precision 0 (FP64) or 1 (FP32):
 *   *xy_variant (-1 when the cross-section has a single xy pass),
 *   *z_pencils (0 when the z passes use the generic kernels).
 * vie_set_tune: force a choice (xy_variant 0-2, ignored where the cross-section
 *   has a single xy pass); z_pencils -1 = the generic z passes, 0 = the
 *   four-step z passes with their default pencils (generic where the grid has no
 *   four-step shape), any other value must be one of the tuner's candidates
 *   (VIE_EINVAL otherwise).  Synchronises the plan's stream first.
 */
int vie_get_tune(vie_plan_t plan, int precision, int* xy_variant, int* z_pencils);
int vie_set_tune(vie_plan_t plan, int precision, int xy_variant, int z_pencils);

/*
 * vie_profile_matvec -- diagnostic.  Runs `reps` products y = (I - M_eps N) x on the
 * plan's stream (precision 0: FP64 on vie_c128 vectors; 1: FP32 on vie_c64) with HIP
 * events around each of the three passes (0: forward z FFT; 1: xy FFT + Green
 * product + inverse xy FFT; 2: inverse z FFT + crop + contrast).  pass_ms[3]
 * receives each pass's average duration in milliseconds and *total_ms (may be
 * NULL) the average per product.  x, y device, 3N values, no overlap.  Synchronises.
 */
int vie_profile_matvec(vie_plan_t plan, int precision, const void* x, void* y, int reps, double pass_ms[3],
                       double* total_ms);

/*
 * Learned preconditioner (this library's addition; not part of the paper's
 * method).  A fixed 4-level 3-D U-Net (3x3x3 convolutions, channels 16/32/48/64,
 * bias-free ReLU, 2x average pooling, nearest upsampling, skip concatenation, a
 * final 1x1x1 convolution to 6 channels) maps a residual r and the contrast chi
 * to an approximate A^{-1} r:  z = r + net(r s, chi) / s with s = sqrt(3N)/||r||
 * (the network predicts the correction A^{-1} r - r).
 * Activations are bfloat16, convolutions run on the matrix cores with FP32
 * accumulation, master weights and Adam moments are FP32.
 *
 * Architecture (levels 0..3 at grid / 2^l, voxel v = (i1 n2 + i2) n3 + i3 at
 * level 0, channels last, every channel count padded to a multiple of 16):
 *   input X0 (16 ch): Re, Im of r_x, r_y, r_z times s, Re, Im of chi, Re, Im of
 *     w_x, w_y, w_z times s (the base vector of vie_net_apply_base; zeros
 *     without one), two zeros;
 *   L0  3x3x3  16 -> 16  (14 real inputs)  E1a = relu(L0 X0)
 *   L1  3x3x3  16 -> 16                     E1b = relu(L1 E1a)
 *   P1 = avgpool2(E1b);  L2 16 -> 32: E2a;  L3 32 -> 32: E2b
 *   P2 = avgpool2(E2b);  L4 32 -> 48: E3a;  L5 48 -> 48: E3b
 *   P3 = avgpool2(E3b);  L6 48 -> 64: E4a;  L7 64 -> 64: E4b
 *   L8  112 -> 48 on [up(E4b), E3b]:  D3a;  L9  48 -> 48: D3b
 *   L10  80 -> 32 on [up(D3b), E2b]:  D2a;  L11 32 -> 32: D2b
 *   L12  48 -> 16 on [up(D2b), E1b]:  D1a;  L13 16 -> 16: D1b
 *   L14 1x1x1 16 -> 16 (6 real outputs), no ReLU, FP32 output "out"
 * ([a, b] = channel concatenation, a first; up = nearest upsampling x2; every
 * relu(.) output and every pooled value is stored in bfloat16, rounded to
 * nearest even; the convolutions use bfloat16 weights, the master copies are
 * FP32).  Weights of layer l are [taps][cout][cin] with tap t = (dz+1) 9 +
 * (dy+1) 3 + (dx+1) shifting along (i1, i2, i3); vie_net_get_params lists
 * L0..L14 in order.  z_c = base_c + (out[2c] + i out[2c+1]) / s, base = w or r.
 *
 * vie_net_create: grid dims must be multiples of 8 (three poolings).  Weights
 *   are He-initialised from `seed` (deterministic).  hip_stream as in vie_plan.
 * vie_net_num_params / get / set: the FP32 master weights, host buffer of
 *   vie_net_num_params floats (layer by layer, each [taps][cout][cin] padded).
 * vie_net_apply: z = net applied to r (device, 3N) with chi (device, N contrast
 *   values, e.g. 1 - eps_b/eps); z device, 3N.  Asynchronous.
 * vie_net_train_step: one Adam step (lr) on the mean squared error between
 *   net(r_i s) and (target_i - r_i) s over `count` samples (device pointers,
 *   3N / N / 3N), i.e. z = r + net approximates target;
 *   *loss receives the mean loss.  Synchronises.
 * vie_set_preconditioner: attach a network with the plan's grid (NULL detaches);
 *   vie_solve with precision 2 uses it.  The plan does not own the network.
 * vie_nn_conv_test: diagnostic single layer on FP32 device buffers (rounded to
 *   bfloat16 on entry): mode 0 forward y[V][cout] (relu optional) from x[V][cin]
 *   and w[taps][cout][cin]; mode 1 input gradient dx[V][cin] from x = dy[V][cout];
 *   mode 2 weight gradient dw[taps][cout][cin] from x[V][cin] and w = dy[V][cout].
 *   taps 1 or 27, cin and cout multiples of 16.  Synchronises.
 */
int vie_net_create(vie_net_t* out, const int grid[3], unsigned seed, void* hip_stream);
void vie_net_destroy(vie_net_t net);
int vie_net_num_params(vie_net_t net, size_t* count);
int vie_net_get_params(vie_net_t net, float* host, size_t count);
int vie_net_set_params(vie_net_t net, const float* host, size_t count);
/*
 * Training checkpoint (the state one vie_net_train_step continues from): the FP32
 * master weights, the Adam moments m and v and the Adam step count.  host holds
 * 3 count floats, [weights | m | v], each part in the layout of vie_net_get_params;
 * count = vie_net_num_params.  vie_net_set_state refuses non-finite values, negative
 * second moments or a negative step (VIE_EINVAL, nothing changed), rewrites the
 * bfloat16 copies and synchronises.  Both copy through the host synchronously.
 */
int vie_net_get_state(vie_net_t net, float* host, size_t count, int* step);
int vie_net_set_state(vie_net_t net, const float* host, size_t count, int step);
int vie_net_apply(vie_net_t net, const vie_c128* r, const vie_c128* chi, vie_c128* z);
int vie_net_train_step(vie_net_t net, int count, const vie_c128* const* r, const vie_c128* const* chi,
                       const vie_c128* const* target, float lr, double* loss);
/*
 * The same with a base vector w (device, 3N values; NULL = r): the network also sees
 * w and predicts the correction A^{-1} r - w, so z = w + net(r s, chi, w s) / s.  With
 * w = W^{-1} r from the block-circulant preconditioner (vie_circulant_apply) the
 * network corrects that preconditioner (vie_solve precision 4).  train_step_base:
 * w is an array of count device pointers or NULL.
 */
int vie_net_apply_base(vie_net_t net, const vie_c128* r, const vie_c128* w, const vie_c128* chi, vie_c128* z);
int vie_net_train_step_base(vie_net_t net, int count, const vie_c128* const* r, const vie_c128* const* w,
                            const vie_c128* const* chi, const vie_c128* const* target, float lr, double* loss);
int vie_set_preconditioner(vie_plan_t plan, vie_net_t net);
int vie_nn_conv_test(int mode, const int dims[3], int taps, int cin, int cout, const float* x, const float* w,
                     float* out, int relu, void* hip_stream);
const char* vie_net_last_error(vie_net_t net);
/*
 * Diagnostics for parity tests.
 * vie_net_get_grads: the FP32 weight gradients of the last vie_net_train_step (summed
 *   over its samples), host buffer of vie_net_num_params floats in the layout of
 *   vie_net_get_params.  Synchronises.
 * vie_nn_op_test: one pooling or upsampling kernel on FP32 device buffers (inputs
 *   rounded to bfloat16, bfloat16 results widened to FP32), C channels per voxel
 *   (a multiple of 8)
 *   (channels last), dims = the fine grid (even sizes): op 0 average pooling
 *   x[fine] -> out[coarse]; 1 its gradient x = dY[coarse] -> out[fine] = dY/8 at the
 *   parent, zero where mask[fine] <= 0 (mask may be NULL), added to acc[fine] (may be
 *   NULL) with one bfloat16 rounding; 2 nearest upsampling x[coarse] -> out[fine];
 *   3 its gradient x = dY[fine] -> out[coarse] = sum over the 8 children.  Synchronises.
 * vie_nn_adam_test: Adam step t >= 1 (beta1 0.9, beta2 0.999, eps 1e-8, bias
 *   corrections 1 - beta^t) on n FP32 device values w, m, v in place with gradient g,
 *   learning rate lr, as the training step applies it.  Synchronises.
 */
int vie_net_get_grads(vie_net_t net, float* host, size_t count);
int vie_nn_op_test(int op, const int dims[3], int C, const float* x, const float* mask, const float* acc,
                   float* out, void* hip_stream);
int vie_nn_adam_test(long n, float* w, float* m, float* v, const float* g, int t, float lr, void* hip_stream);

/*
 * JM-VIE: electric and magnetic currents (Section III, the coupled system
 * (I - M T)(J, M) = C M (E_inc, H_inc) with T = [[N, -c_e K], [c_m K, N]],
 * K = curl S; Section IV-B, an absorber that also carries magnetic loss).
 * Magnetic unknowns are in impedance units (w_m = eta w~_m) and the time
 * dependence is exp(-i omega t), which makes the operator
 *   y_e = x_e - M_eps (N x_e + i kappa K x_m),
 *   y_m = x_m - M_mu  (-i kappa K x_e + N x_m),
 * kappa = k_b h, M_mu = (mu_r - 1)/mu_r, K the Galerkin table of curl S at unit
 * voxel edge.  Vectors hold 6N values: electric [3][n1][n2][n3], then magnetic.
 * The right-hand side is the caller's, e.g. h^{3/2} (M_eps e_inc, M_mu eta h_inc)
 * with eta h_inc = curl e_inc / (i k_b).
 *
 * vie_curl_table -- host-only, FP64: K^{ab}(m) for 0 <= m_d < grid[d], out
 *   [3][n1][n2][n3] for the components xy, xz, yz (K^{ba} = -K^{ab}, K^{aa} = 0);
 *   negating m_d multiplies K^{ab} by -1 exactly when d is neither a nor b.
 * vie_jm_enable -- builds the spectrum of K and the JM buffers and sets mu_r = 1
 *   everywhere.  Idempotent.  VIE_EINVAL when M1 M2 > 4096.  Synchronises.
 *   The cross-section pass runs fused (spectra in LDS) when the six
 *   row-transformed components of a plane fit with one column chunk:
 *   (6 n2 M1 + 6 M2 cc) complex values in 160 KiB for some cc >= 1 (every FP32
 *   grid; in FP64 e.g. the 30 x 12 strip), else with the x-frequencies in two
 *   halves of M1/2 (even and odd kx in turn; in FP64 the 32 x 32
 *   cross-section); otherwise through full spectra in HBM (6 M1 M2 M3 complex
 *   values per precision, allocated only then).
 * vie_jm_set_route / vie_jm_get_route -- per precision (0 FP64, 1 FP32): fused 1
 *   = the fused pass (VIE_EINVAL where it does not fit), 0 = through HBM
 *   (allocates the spectra on first use).  Same results to rounding.
 * vie_jm_set_permeability -- mu_r: device, N relative permeabilities (copied).
 *   VIE_EINVAL for a zero or non-finite entry.  Synchronises.
 * vie_jm_rhs -- b = h^{3/2} (M_eps e_inc, M_mu etah_inc): e_inc and etah_inc
 *   device, 3N values each (fields at the voxel centres, eta h_inc in the units
 *   of e_inc); b device, 6N values.  Async.
 * vie_jm_matvec / vie_jm_matvec_c64 -- y = (I - M T~) x in FP64 / FP32 (the
 *   latter needs VIE_WITH_FP32); device, 6N values each, no overlap.  Async.
 * vie_jm_residual -- r = b - (I - M T~) x, FP64.  Async.
 * vie_jm_solve -- GMRES(restart) (precision 0) or FP32-inner / FP64-outer
 *   flexible GMRES (precision 1) on the 6N unknowns; x in/out (use_x0), tol on
 *   the true FP64 residual relative to ||b||, info as for vie_solve.
 * All take VIE_ESTATE before vie_jm_enable and vie_set_contrast.
 */
int vie_curl_table(const int grid[3], double kappa, vie_c128* out, int nthreads);
int vie_jm_enable(vie_plan_t plan);
int vie_jm_set_route(vie_plan_t plan, int precision, int fused);
int vie_jm_get_route(vie_plan_t plan, int precision, int* fused);
int vie_jm_set_permeability(vie_plan_t plan, const vie_c128* mu_r);
int vie_jm_rhs(vie_plan_t plan, const vie_c128* e_inc, const vie_c128* etah_inc, vie_c128* b);
int vie_jm_matvec(vie_plan_t plan, const vie_c128* x, vie_c128* y);
int vie_jm_matvec_c64(vie_plan_t plan, const vie_c64* x, vie_c64* y);
int vie_jm_residual(vie_plan_t plan, const vie_c128* x, const vie_c128* b, vie_c128* r);
int vie_jm_solve(vie_plan_t plan, const vie_c128* b, vie_c128* x, double tol, const vie_solve_opts* opts,
                 vie_solve_info* info);

/*
 * vie_check_block_maps -- host-only diagnostic.  Runs the product's workgroup-to-work
 * maps (z-pass pencil blocks and their XCD grouping, cross-section plane pairs) over
 * every shape the library accepts and checks that each is a bijection onto its work
 * items and that every write derived from an item lies inside its buffer; the LDS maps
 * of the 64 x 32 cross-section pass must be bijections inside their areas and free of
 * bank conflicts over every access of one LDS pass, in FP64 and FP32 (all but the
 * FP32 column exchange of its variant 1).  msg (may be NULL) receives "ok: ..." or
 * the first violation, cap bytes at most.  planted = 1 checks a deliberately broken
 * work map, planted = 2 a hand-off swizzle with bank conflicts, instead (the checker
 * must report them).
 * Returns VIE_OK when every map passes, VIE_EINVAL otherwise.
 */
int vie_check_block_maps(char* msg, size_t cap, int planted);

/* Message for the last failing call on this plan (plan = NULL: on this thread). */
const char* vie_last_error(vie_plan_t plan);

/* Release every device and host resource of the plan.  NULL is a no-op. */
void vie_destroy(vie_plan_t plan);

/* Library version string. */
const char* vie_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VIE_H */
