/*
 * bem.h - C ABI of the MI355X non-singular boundary-integral / Fourier
 * space-time solver (Klaseboer, Sepehrirahnama & Chan, "Space-time domain
 * solutions of the wave equation by a non-singular boundary integral method
 * and Fourier transform").
 *
 * Conventions for every call
 *   - Sound speed c = 1, time dependence e^{-i w t} with w = k (Sec. III,
 *     Eq. inverseFourier); scattered fields radiate as e^{ikr}.
 *   - Complex numbers are interleaved (re, im): "c64" = 2 x float,
 *     "c128" = 2 x double.
 *   - Surface normals point OUT OF THE BODY, into the fluid.
 *   - Every pointer marked [dev] is a device pointer on the context's device;
 *     [host] pointers are host memory.  All buffers are allocated and owned by
 *     the caller; the library keeps no pointer after a call returns.
 *   - Work is enqueued on the context's stream.  Calls that return values in
 *     host memory synchronise that stream before returning; the others are
 *     asynchronous with respect to the host.
 *   - Argument checks happen on the host before any launch and return
 *     BEM_EINVAL with a message available from bem_last_error().
 */
#ifndef BEM_H
#define BEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BEM_OK = 0,
  BEM_EINVAL = -1,        /* bad argument (NULL, size <= 0, non-finite k, ...) */
  BEM_ENOMEM = -2,        /* device workspace could not be allocated */
  BEM_EHIP = -3,          /* a HIP runtime call failed */
  BEM_ESINGULAR = -4,     /* an exactly zero pivot was met in a factorisation */
  BEM_ENOCONV = -5,       /* iterative refinement did not converge (fallback off) */
  BEM_EUNSUPPORTED = -6   /* option not supported by this build */
} bem_status;

typedef enum { BEM_C64 = 0, BEM_C128 = 1 } bem_prec;

/* Boundary condition flag per node (Sec. IV A). */
enum { BEM_BC_HARD = 0,   /* dP/dn known (sound-hard): P is the unknown      */
       BEM_BC_SOFT = 1 }; /* P known (sound-soft): dP/dn is the unknown      */

typedef struct bem_ctx bem_ctx;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t, NULL = the null stream).  The context owns the solver
 * workspace and the tuning cache; it is not thread-safe (one context per host
 * thread).  Returns BEM_EHIP if the device cannot be selected or the device
 * address of the library's fixed field scratch cannot be taken. */
bem_status bem_ctx_create(int device, void* hip_stream, bem_ctx** out);
void bem_ctx_destroy(bem_ctx* ctx);
/* Message of the last failed call on this context ("" if none). */
const char* bem_last_error(const bem_ctx* ctx);
/* Upper bound (bytes) of device workspace bem_solve_batched may hold; 0 = 75%
 * of the free device memory at the time of the call.  A nonzero limit also caps
 * the packing buffer of BEM_GEMM_BF16X3 factorisations at a quarter of it. */
bem_status bem_ctx_set_workspace_limit(bem_ctx* ctx, uint64_t bytes);

/* Per-kernel accounting for roofline reports.  With profiling on, each launch
 * of a counted kernel is bracketed by HIP events on the stream it runs on and
 * credited with its algorithmic work; bem_ctx_kernel_stats returns the sums
 * (flops, bytes, milliseconds of device time, launch count) since profiling
 * was last switched (set_profiling resets them).  Kernel names: "gemm_c32" and
 * "gemm_3m" (float32 4M / 3M updates of at least 65 columns), "gemm_c32_narrow" and
 * "gemm_3m_narrow" (17 to 64 columns), "gemm_c32_unaligned" and "gemm_3m_unaligned"
 * (operands not 16-byte aligned), "gemm_b3", "gemm_b3_narrow", "gemm_b3_packed",
 * "gemm_small", "pack", "gemm_c64", "panel", "laswp", "trsm", "assemble", "residual",
 * "getrs", "field", "synth".
 * For "assemble"/"residual" the flop slot counts node pairs and for "field"
 * kernel terms (point x frequency x node).  Unknown names report zeros.
 * Profiling turns the hipGraph replay of bem_solve_batched off.
 * Synchronises the stream.
 * bem_ctx_set_profiling_filter: count only the named kernels (a
 * comma-separated list; NULL or "" = all), so that timing one kernel adds no
 * events to the others; takes effect at the next set_profiling. */
bem_status bem_ctx_set_profiling(bem_ctx* ctx, int32_t on);
bem_status bem_ctx_set_profiling_filter(bem_ctx* ctx, const char* names);
bem_status bem_ctx_kernel_stats(bem_ctx* ctx, const char* kernel, double* flops, double* bytes,
                                double* ms, int64_t* launches);

/* Discretised scatterer surface(s): n nodes with positions x[n][3], unit
 * normals nrm[n][3] (out of the body), quadrature weights w[n] > 0 and flags
 * bc[n] in {BEM_BC_HARD, BEM_BC_SOFT}; all [dev], float64/uint8.  The surface
 * of several bodies is the concatenation of their nodes (Sec. III: S is the
 * union of the scatterer surfaces). */
typedef struct {
  int32_t n;
  const double* x;
  const double* nrm;
  const double* w;
  const uint8_t* bc;
} bem_surface;

/* ---------------------------------------------------------------- geometry
 * Icosphere surface of one body (the nodal discretisation of Sec. IV A's
 * element meshes): `level` midpoint subdivisions of the icosahedron, mapped
 * to center + (radius*u0, radius*u1, radius*aspect*u2); analytic normals;
 * weights = 1/3 of the adjacent flat-triangle areas, rescaled to the analytic
 * area if rescale_area != 0.  All outputs [host], caller-allocated with
 * bem_mesh_counts() entries: x[V][3], nrm[V][3], w[V], faces[F][3].
 * Arithmetic is done in a fixed order (no fused multiply-add), so results are
 * reproducible bit for bit.  Returns BEM_EINVAL for level outside 0..7,
 * radius <= 0 or aspect < 1. */
bem_status bem_mesh_counts(int32_t level, int32_t* n_vertices, int32_t* n_faces);
bem_status bem_mesh_icosphere(int32_t level, double radius, double aspect,
                              const double center[3], int32_t rescale_area,
                              double* x, double* nrm, double* w, int32_t* faces);

/* The axisymmetric acoustic bowl of Sec. IV C (Eq. dish): the closed meridian
 * curve xi = a sin(theta), eta = a (0.2 cos(theta) - 0.6 sin^2(theta)),
 * 0 <= theta <= pi, rotated about the eta axis -- a thin curved shell whose
 * faces meet at a sharp rim.  Nodes: the pole theta = 0, rings
 * theta_i = pi i / n_theta (0 < i < n_theta) of n_phi nodes at
 * phi_j = 2 pi j / n_phi, the pole theta = pi; local frame
 * (xi cos phi, xi sin phi, eta), then the eta axis turned by `tilt` about x
 * (y' = y cos t - z sin t, z' = y sin t + z cos t) and shifted by `center`.
 * Normals are analytic (outward normal of the meridian curve); weights are one
 * third of the adjacent flat-triangle areas.  Outputs [host], caller-allocated
 * with bem_mesh_bowl_counts() entries (x[V][3], nrm[V][3], w[V], faces[F][3]
 * or NULL); fixed evaluation order, reproducible bit for bit.  EINVAL for
 * n_theta < 2, n_phi < 3 or radius <= 0. */
bem_status bem_mesh_bowl_counts(int32_t n_theta, int32_t n_phi, int32_t* n_vertices,
                                int32_t* n_faces);
bem_status bem_mesh_bowl(int32_t n_theta, int32_t n_phi, double radius, double tilt,
                         const double center[3], double* x, double* nrm, double* w,
                         int32_t* faces);

/* ---------------------------------------------------------------- incident
 * Known surface data of the scattered field for the incident plane wave
 * e^{ik d.x} (Sec. IV A): y = -dP_inc/dn = -ik (d.n) e^{ik d.x} on hard nodes,
 * y = -e^{ik d.x} on soft nodes.  k[n_k] [dev] float64, dir[3] [host] unit
 * vector, y[n_k][n] c128 [dev]. */
bem_status bem_incident(bem_ctx* ctx, const bem_surface* s, int32_t n_k, const double* k,
                        const double dir[3], void* y);

/* ---------------------------------------------------------------- assembly
 * Dense system of the discrete non-singular boundary integral equation
 * (Eq. BRIEF with f, g of Appendix A, S_inf integrals of Appendix B), nodal
 * quadrature with collocation at the nodes:
 *   (M_phi)_ij = -w_j H_ij,  (M_phi)_ii = 4 pi - sum_{j!=i} w_j (g'_ij G_ij - g_ij H_ij)
 *   (M_psi)_ij =  w_j G_ij,  (M_psi)_ii =      - sum_{j!=i} w_j (f'_ij G_ij - f_ij H_ij)
 * Column j of A is column j of M_phi (hard node) or M_psi (soft node); B holds
 * the other columns; b = -B y for each right-hand side.
 *   k[n_k]                 [dev] wavenumbers (> 0)
 *   y[n_k][n_rhs][n]       [dev] c128 known data
 *   A[n_k][n][ld]          [dev] ROW-MAJOR (element (i,j) at i*ld + j), c64 or
 *                          c128 per `prec`; ld >= n
 *   b[n_k][n_rhs][n]       [dev] c128
 *   diag64[n_k][n][2]      [dev] c128 (M_phi)_ii, (M_psi)_ii, or NULL
 * Every pair term is evaluated in float64; A is rounded to `prec` on store.
 * A may be NULL (ld ignored): then only diag64 and b are produced. */
bem_status bem_assemble(bem_ctx* ctx, const bem_surface* s, int32_t n_k, const double* k,
                        int32_t n_rhs, const void* y, bem_prec prec, void* A, int32_t ld,
                        void* b, void* diag64);

/* r = b - A x for the float64 operator regenerated on the fly (matrix-free):
 *   k[n_k] [dev] (> 0, checked: BEM_EINVAL otherwise),
 *   x[n_k][n_rhs][n] c128 unknowns [dev], y as for bem_assemble,
 *   diag64 from bem_assemble [dev], r[n_k][n_rhs][n] c128 [dev] (output). */
bem_status bem_residual(bem_ctx* ctx, const bem_surface* s, int32_t n_k, const double* k,
                        int32_t n_rhs, const void* y, const void* x, const void* diag64,
                        void* r);

/* Relative residual of given unknowns: rel[q] = ||b - A x||_2 / ||b||_2 per
 * (wavenumber, rhs) with the float64 operator (the acceptance test of
 * predicted solutions).  k [dev] (> 0, checked); x, y [dev] c128
 * [n_k][n_rhs][n]; rel [host] double[n_k*n_rhs].  Synchronises the stream. */
bem_status bem_residual_check(bem_ctx* ctx, const bem_surface* s, int32_t n_k, const double* k,
                              int32_t n_rhs, const void* y, const void* x, double* rel);

/* ---------------------------------------------------------------- solve
 * One linear system per wavenumber (Sec. IV A: direct solve).  Modes:
 *   BEM_FP64_DIRECT : c128 assembly + float64 LU (MFMA f64) + triangular solves
 *   BEM_FP32_IR_4M  : c64 LU (complex GEMM as 4 real products on MFMA f32,
 *                     float32 accumulation) + iterative refinement with the
 *                     float64 matrix-free residual, until ||dx||/||x|| <= tol_step
 *   BEM_FP32_IR_3M  : as 4M with the 3-product complex GEMM
 *   BEM_FP32_IR_B3  : as 4M with every real product of the GEMM taken as three
 *                     bfloat16 MFMA products of the split operands
 *                     (x = hi + lo; hi hi + hi lo + lo hi, float32 accumulation)
 * The refinement makes all three float32 modes reach the same float64-residual
 * accuracy; they differ in speed and in the number of sweeps.
 * Items that do not converge within max_iter are re-solved with the FP64
 * direct path when fallback != 0 (flagged in info), else BEM_ENOCONV. */
typedef enum {
  BEM_FP64_DIRECT = 0,
  BEM_FP32_IR_4M = 1,
  BEM_FP32_IR_3M = 2,
  BEM_FP32_IR_B3 = 3
} bem_mode;

/* complex GEMM form of a c64 factorisation (last argument of bem_getrf_batched).
 * BEM_GEMM_BF16X3 runs the updates of at least 512 x 512 (the trailing update
 * of each block column among them) on operands split once into bf16 words by
 * a packing pass (the context keeps a packing
 * buffer of at most 4 GiB and packs larger batches in slices; if it cannot be
 * allocated the unpacked kernel runs).  BEM_GEMM_BF16X3_UNPACKED is the same
 * arithmetic, bit for bit, with the split done inside every GEMM tile and no
 * packing buffer. */
typedef enum {
  BEM_GEMM_4M = 0,
  BEM_GEMM_3M = 1,
  BEM_GEMM_BF16X3 = 2,
  BEM_GEMM_BF16X3_UNPACKED = 3
} bem_gemm_kind;

typedef struct {
  const bem_surface* s;   /* [host] struct holding [dev] arrays */
  int32_t n_k;
  const double* k;        /* [dev] n_k wavenumbers */
  int32_t n_rhs;
  const void* y;          /* [dev] c128 [n_k][n_rhs][n] known data */
} bem_problem;

typedef struct {
  int32_t mode;           /* bem_mode */
  double tol_step;        /* stop an item when ||dx||_2/||x||_2 <= tol_step (x is then kept
                             without dx), or when the ratio rho < 1/2 of the last two
                             correction norms bounds the error left after applying dx by
                             rho/(1-rho) ||dx||_2/||x+dx||_2 <= tol_step (default 1e-8) */
  int32_t max_iter;       /* refinement sweeps (default 10) */
  int32_t fallback;       /* 1: re-solve non-converged items in FP64 */
  int32_t use_graph;      /* 1 (default): replay the factorisation as a hipGraph captured
                             on first use of a given set of matrices and sizes (kept by
                             the context, dropped when its workspace moves); ignored
                             while profiling is on */
  int32_t nb;             /* block width of the factorisation; 0 = the width measured by
                             bem_autotune_lu for this size class, else the default */
} bem_solve_opts;

typedef struct {
  int32_t iters;          /* refinement sweeps done (0 for FP64_DIRECT) */
  int32_t used_fp64;      /* 1 if the FP64 fallback produced the result */
  int32_t singular;       /* 1 if a zero pivot was met */
  int32_t converged;      /* 1 if the step tolerance was reached (or FP64 direct) */
  double rel_resid;       /* ||b - A x||_2 / ||b||_2, float64 operator */
  double rel_step;        /* last ||dx||_2/||x||_2 */
} bem_solve_info;

/* Defaults: mode BEM_FP32_IR_3M, tol_step 1e-8, max_iter 10, fallback 1,
 * use_graph 1, nb 0. */
void bem_solve_opts_default(bem_solve_opts* opts);

/* probs[n_probs] [host]; x_out[p] [dev] c128 [n_k][n_rhs][n] unknowns of
 * problem p (P on hard nodes, dP/dn on soft nodes); info [host]
 * [sum_p n_k*n_rhs] in problem order, or NULL.  Problems may have different
 * n (uneven batch); all are scheduled together.  Synchronises the stream. */
bem_status bem_solve_batched(bem_ctx* ctx, const bem_problem* probs, int32_t n_probs,
                             const bem_solve_opts* opts, void* const* x_out,
                             bem_solve_info* info);

/* Remedy for fictitious resonances (Sec. IV A avoids the wavenumbers where
 * the interior of a body resonates; there the surface equation is nearly
 * singular and its solution carries a spurious interior mode).  Green's second
 * identity on the exterior domain gives, for the radiating scattered field
 * and a point x_c strictly inside a body (normals out of the body),
 *   sum_j w_j (phi_j H_cj - psi_j G_cj) = 0,  d = x_j - x_c,
 *   G = e^{ikr}/r,  H = e^{ikr}(ikr - 1)(d.n_j)/r^3,
 * one more row C x = d per point (split by the boundary conditions as the
 * surface rows).  The surface rows A x = b and the n_c interior rows are
 * solved in the least-squares sense, float64 throughout: the normal equations
 * (A^H A + C^H C) x = A^H b + C^H d are formed by complex GEMMs (rocBLAS) and
 * factored by the library's LU.  Away from resonances the interior rows hold
 * to the discretisation error and the result moves by that much.
 * xc [dev] [n_c][3] float64: points strictly inside the bodies, off the nodal
 * surfaces of the interior eigenfunctions (random points are); k [dev] n_k
 * wavenumbers; y [dev] c128 [n_k][n_rhs][n] known data; x_out [dev] c128
 * [n_k][n_rhs][n] unknowns; info [host] [n_k*n_rhs] or NULL (rel_resid: the
 * stacked system's least-squares residual, ||[A;C] x - [b;d]|| / ||[b;d]||).
 * Holds about (2 n + n_c) (n + n_rhs) 16 bytes per wavenumber of workspace;
 * ESINGULAR if the normal equations have a zero pivot; synchronises the
 * stream. */
bem_status bem_solve_chief(bem_ctx* ctx, const bem_surface* s, int32_t n_k, const double* k,
                           int32_t n_rhs, const void* y, int32_t n_c, const double* xc,
                           void* x_out, bem_solve_info* info);

/* Building blocks of the direct solve (Sec. IV A), exposed for testing and for
 * callers that keep the factors to re-use them for other right-hand sides
 * (Sec. V notes that the factorised system of a frequency can be kept and
 * re-used).
 * bem_getrf_batched: in-place LU with partial pivoting (P A = L U, unit L) of
 *   `batch` row-major n x n matrices A + b*stride (elements of `prec`, leading
 *   dimension ld >= n, stride >= n*ld elements) [dev].  piv[batch][n] [dev]
 *   int32: row i was interchanged with row piv[i] (absolute, 0-based).
 *   info[batch] [dev] int32: 0, or 1 + index of the first exactly-zero pivot.
 *   nb = block width (0 = the width measured by bem_autotune_lu for this size
 *   class, else 512 for n >= 4096 and 256 below; at most 1024 is used), gemm_kind
 *   (bem_gemm_kind) the complex GEMM form of the trailing updates for c64
 *   (ignored for c128).  n * ld must stay below 2^31.
 * bem_getrs_batched: X = A^{-1} B for n_rhs vectors per matrix:
 *   B, X [dev] [batch][n_rhs][n] (vector stride n, matrix stride bstride
 *   elements), same precision as the factors; B and X must not overlap. */
bem_status bem_getrf_batched(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t ld, int64_t stride,
                             int32_t batch, void* A, int32_t* piv, int32_t* info, int32_t nb,
                             int32_t gemm_kind);
bem_status bem_getrs_batched(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t ld, int64_t stride,
                             int32_t batch, const void* LU, const int32_t* piv, int32_t n_rhs,
                             const void* B, void* X, int64_t bstride);

/* Plan of the factorisation measured on this device: factors `batch`
 * pseudo-random n x n matrices (diagonally dominant, deterministic) of the
 * given precision and GEMM form once per candidate block width (a
 * 0-terminated list [host], or NULL for 256, 384, 512, 768, 1024) and, for
 * the float32 MFMA forms (BEM_GEMM_4M, BEM_GEMM_3M), per GEMM shape: 128 x 64
 * tiles for updates of up to 64 or up to 128 columns (128 x 128 above), and
 * one workgroup per tile or persistent workgroups drawing tiles from per-XCD
 * counters; best of two runs each.  The fastest plan is kept in the context
 * for every later factorisation of that precision, GEMM form and size class
 * (n rounded up to 512) whose caller passes nb = 0 (the GEMM shape applies
 * whatever nb the caller passes).  best_nb, best_ms [host] may be NULL.
 * Allocates batch * n * ld elements for the duration of the call (BEM_ENOMEM
 * if they do not fit); synchronises the stream. */
bem_status bem_autotune_lu(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t batch,
                           int32_t gemm_kind, const int32_t* candidates, int32_t* best_nb,
                           double* best_ms);

/* Every plan tried by the context's last bem_autotune_lu call, in the order
 * tried: block width, GEMM tile threshold (columns), persistent launches
 * (0/1) and time (ms); the first max entries are written to the [host]
 * arrays (each may be NULL).  Returns the number of plans tried. */
int32_t bem_autotune_lu_results(bem_ctx* ctx, int32_t max, int32_t* nb, int32_t* narrow_max,
                                int32_t* persistent, double* ms);
/* Sets the plan of a size class by hand (as bem_autotune_lu would keep it):
 * block width nb > 0, 128 x 64 GEMM tiles up to narrow_max columns (64 ..
 * 1024), persistent GEMM launches 0/1.  Drops the context's captured
 * factorisations. */
bem_status bem_lu_set_plan(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t gemm_kind, int32_t nb,
                           int32_t narrow_max, int32_t persistent);
/* The plan bem_autotune_lu (or bem_lu_set_plan) kept for (prec, gemm_kind,
 * size class of n); EINVAL if none.  Outputs [host] may be NULL. */
bem_status bem_lu_tuned_plan(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t gemm_kind,
                             int32_t* nb, int32_t* narrow_max, int32_t* persistent);

/* Iterative refinement of given unknowns with stored float32 factors of
 * other (nearby) wavenumbers: x <- x + LU_f^{-1} (b - A(k) x), residual in
 * float64 with the exact operator of each k, until ||dx||/||x|| <= tol_step or
 * max_iter sweeps (converged = 0 in info then).  Used to re-use the factors of
 * neighbouring frequencies (Sec. V: the solution matrix can be stored) for a
 * dense frequency grid, starting from a predicted solution.
 *   LU [dev] c64 factors from bem_getrf_batched, n_fac sets of [n][ld] with
 *   stride; piv [dev] [n_fac][n]; fac_index [dev] int32[n_k] factor set used
 *   for each wavenumber; k [dev] (> 0, checked); x [dev] c128
 *   [n_k][n_rhs][n] initial guess, refined in place; info [host] [n_k*n_rhs]
 *   or NULL.  Synchronises the stream. */
bem_status bem_refine_batched(bem_ctx* ctx, const bem_surface* s, int32_t n_k, const double* k,
                              int32_t n_rhs, const void* y, const void* LU, int32_t ld,
                              int64_t stride, const int32_t* piv, int32_t n_fac,
                              const int32_t* fac_index, double tol_step, int32_t max_iter,
                              void* x, bem_solve_info* info);

/* phi = (hard ? x : y), psi = (hard ? y : x): full surface data from the
 * unknowns and the known data; all [dev] c128 [n_k][n_rhs][n]. */
bem_status bem_split_unknowns(bem_ctx* ctx, const bem_surface* s, int32_t n_k, int32_t n_rhs,
                              const void* x, const void* y, void* phi, void* psi);

/* ---------------------------------------------------------------- field
 * Scattered field at observation points by the non-singular representation
 * (Eq. BRIEFdmn, S_inf part evaluated):
 *   4 pi P(x_p) = 4 pi phi_i0 + sum_{j!=i0} w_j [u_j (H^p_j - H_i0j) - u'_j (G^p_j - G_i0j)]
 * where i0 is the surface node closest to x_p (float64 squared distance
 * (dx*dx+dy*dy)+dz*dz without fused multiply-add, ties to the lowest index)
 * and u, u' are the surface data minus their f/g expansion about x_i0.
 * Points with n_i0.(x_p - x_i0) < 0 are inside a body: U = 0, inside = 1.
 *   k[n_k] [dev]; phi, psi [dev] c128 [n_k][n_rhs][n]; xp[m][3] [dev] float64
 *   i0[m] [dev] int32: output, or input when i0_given != 0
 *   inside[m] [dev] uint8 output
 *   U [dev] [n_rhs][m][n_k], c64 (float32 kernel) or c128 (float64 kernel)
 * Both kernels take the per-node sums S(x_i0) in float64.  The float32
 * kernel sorts the outside points by i0 (counting sort), takes the node sums
 * of the nodes that are some point's i0 only, forms the brackets
 * w_j u_j, w_j u'_j once per node i0 and node tile (float64, rounded to
 * float32) and sums each point's terms in float32 in sixteen interleaved
 * partial sums; P is assembled in float64. */
bem_status bem_field_eval(bem_ctx* ctx, const bem_surface* s, int32_t n_k, const double* k,
                          int32_t n_rhs, const void* phi, const void* psi, int32_t m,
                          const double* xp, int32_t* i0, int32_t i0_given, uint8_t* inside,
                          bem_prec prec, void* U);

/* The same evaluation with no allocation: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts that
 * forbid hipMalloc).  It calls no hipMalloc / hipFree and creates no profiling
 * events; the scratch that bem_field_eval takes from the context's workspace
 * comes from a fixed 32 MiB device array of the library instead: the float64
 * per-node sums S(x_a) (n_rhs * n_k * n * 16 bytes) and, for BEM_C64, the
 * grouping of the points by closest node (about 4.5 m + 40 n bytes); calls
 * needing more than 32 MiB return BEM_EINVAL before any launch (e.g. n = 5124
 * nodes, one right-hand side, 4096 points: 409 frequencies for BEM_C128, 406 for
 * BEM_C64).  Arguments, results and ordering are those of
 * bem_field_eval (same kernels, same results bit for bit).  Every context on a device shares
 * that device's array, which keeps the last call's contents (nothing in it
 * needs to start at zero): calls that overlap on one device (different
 * streams or threads) race and give undefined results.  Returns BEM_EHIP if
 * the context has no address for the array. */
bem_status bem_field_eval_noalloc(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                  const double* k, int32_t n_rhs, const void* phi,
                                  const void* psi, int32_t m, const double* xp, int32_t* i0,
                                  int32_t i0_given, uint8_t* inside, bem_prec prec, void* U);

/* ---------------------------------------------------------------- synthesis
 * Space-time field by inverse DFT over frequency (Sec. III last paragraph,
 * Sec. IV: Fourier components of a periodic pulse train):
 *   p_q(x, t_n) = sum_{m=1}^{n_k} alpha_m Re[ c_q,m X_m(x) e^{-2 pi i m n / T} ]
 * with alpha_m = 2 (m < T/2), 1 (m = T/2), X_m = U_m(x) (+ e^{i m dk z} when
 * add_incident != 0), t_n = n * 2 pi / (dk T).
 *   U[m][n_k] [dev] c64; c[n_pulse][n_k] [dev] c128; xp[m][3] [dev] (read
 *   only when add_incident); p[n_pulse][m][T] [dev] float32 (output).
 *   T: power of two, 64 <= T <= 8192, T >= 2 n_k. */
bem_status pulse_synthesize(bem_ctx* ctx, int32_t m, int32_t n_k, const void* U,
                            int32_t n_pulse, const double* c, int32_t T, int32_t add_incident,
                            const double* xp, double dk, float* p);

/* The same synthesis over a subset of the frequencies (Sec. IV, discussion of
 * Fig. RMSerror and Table 1: the space-time field rebuilt from the solutions at
 * only the wavenumbers whose incident amplitudes |c_m| are largest; every other
 * bin is zero):
 *   p_q(x, t_n) = sum_j alpha_{m_j} Re[ c_q,j X_j(x) e^{-2 pi i m_j n / T} ]
 * with X_j = U_j(x) (+ e^{i m_j dk z} when add_incident != 0).
 *   m_index[n_sel] [host] int32: 1-based frequency indices, strictly
 *   increasing, at most T/2 (copied to device memory of the context; the call
 *   waits for the context stream's earlier work so the host list may be
 *   reused when it returns);
 *   U[m][n_sel] [dev] c64; c[n_pulse][n_sel] [dev] c128; xp, dk, T, p as for
 *   pulse_synthesize.  EINVAL for an index list that breaks these rules. */
bem_status pulse_synthesize_sparse(bem_ctx* ctx, int32_t m, int32_t n_sel,
                                   const int32_t* m_index, const void* U, int32_t n_pulse,
                                   const double* c, int32_t T, int32_t add_incident,
                                   const double* xp, double dk, float* p);

/* Fourier coefficients of a periodic incident pulse train F(z - t - z_shift)
 * sampled at T left-closed points s_n = -L/2 + n L/T, L = 2 pi/dk:
 *   c_m = (1/T) sum_n F(s_n) e^{-i k_m s_n} e^{-i k_m z_shift},  k_m = m dk,
 * m = 1..n_k (Sec. IV, Eq. pulse and the phase factor e^{i beta}).
 * kind / params:
 *   0 paper  {N_c, alpha, w}: sin(tau) e^{-alpha|tau|} on |tau| < 2 pi N_c, tau = (8 pi N_c / w) s
 *   1 gauss  {sigma}: e^{-s^2/2sigma^2}      2 ricker {sigma}: (1 - s^2/sigma^2) e^{-s^2/2sigma^2}
 *   3 nwave  {sigma}: s/sigma on |s|<=sigma  4 chirp {ka, kb, D}: sin(ka s + (kb-ka) s^2/(2D)) e^{-s^2/2D^2}
 *   5 gsine  {k0, sigma}: sin(k0 s) e^{-s^2/2sigma^2}
 *   6 gaussk {k0, width}: spectrum exp(-(k-k0)^2/(2 width^2)) given directly
 * c_out[n_k] [host] c128. */
bem_status bem_pulse_coeffs(int32_t kind, const double* params, int32_t n_params, double dk,
                            int32_t n_k, int32_t T, double z_shift, double* c_out);

/* The n_keep frequencies of largest incident amplitude (Sec. IV, Table 1:
 * 5, 10 or 20 of the largest |P~(w_m)| kept).  Ranking by |c_m| (hypot of
 * the float64 parts) descending, equal magnitudes by lower m; the selection
 * is returned as 1-based indices m in increasing order.
 *   c[n_k] [host] c128; m_index[n_keep] [host] int32 (output);
 *   0 < n_keep <= n_k, else EINVAL. */
bem_status bem_pulse_dominant(const double* c, int32_t n_k, int32_t n_keep, int32_t* m_index);

/* ---------------------------------------------------------------- quadratic elements
 * Surface of six-node quadratic elements (Sec. III: quadratic interpolants
 * within each element, integrals free of singularities evaluated by Gauss
 * quadrature; Sec. IV A: the sphere as 500 quadratic elements and 1002
 * nodes): nodes x[n][3] with unit normals nrm[n][3] (out of the body; used at
 * the collocation nodes) and BC flags bc[n]; elements elem[n_elem][6] =
 * (v0, v1, v2, m01, m12, m20), the corners counter-clockwise seen from
 * outside, then the nodes on the edges (v0 v1), (v1 v2), (v2 v0).  All [dev].
 * A node may belong to at most 12 elements (EINVAL otherwise). */
typedef struct {
  int32_t n;
  const double* x;
  const double* nrm;
  const uint8_t* bc;
  int32_t n_elem;
  const int32_t* elem;
} bem_quad_surface;

/* Frequency-nu geodesic sphere of six-node elements [host]: every icosahedron
 * face cut into nu^2 triangles on its barycentric grid, points projected onto
 * the sphere and mapped to center + (radius u0, radius u1, radius aspect u2);
 * the edge midpoints are the projected chord midpoints; analytic normals.
 * 40 nu^2 + 2 nodes (the vertices first) and 20 nu^2 elements (nu = 5: 1002
 * and 500, the paper's sizes).  Fixed evaluation order (no fused
 * multiply-add): reproducible bit for bit.  x[n][3], nrm[n][3],
 * elems[n_elem][6] caller-allocated; EINVAL for nu outside 1..64, radius <= 0
 * or aspect < 1. */
bem_status bem_mesh_quadratic_counts(int32_t nu, int32_t* n_nodes, int32_t* n_elems);
bem_status bem_mesh_quadratic(int32_t nu, double radius, double aspect, const double center[3],
                              double* x, double* nrm, int32_t* elems);

/* System of the quadratic-element equation, collocated at the nodes:
 *   4 pi phi_i + int [psi - phi_i g' - psi_i f'] G dS = int [phi - phi_i g - psi_i f] H dS
 * with phi, psi and the geometry interpolated by each element's six shape
 * functions, f, g of Appendix A about x_i, H = dG/dn with the element normal,
 * every element integrated by the 7-point degree-5 triangle rule (Radon's):
 *   (M_psi)_ij =  sum N_a(q) wJ_q G_q,  (M_phi)_ij = -sum N_a(q) wJ_q H_q  (node a of e = j)
 *   (M_phi)_ii += 4 pi - sum_q (g' G - g H) wJ_q,  (M_psi)_ii += -sum_q (f' G - f H) wJ_q
 * in float64.  Arguments and outputs (A row-major, b = -B y, diag64) as for
 * bem_assemble. */
bem_status bem_assemble_quadratic(bem_ctx* ctx, const bem_quad_surface* s, int32_t n_k,
                                  const double* k, int32_t n_rhs, const void* y, bem_prec prec,
                                  void* A, int32_t ld, void* b, void* diag64);

/* Direct solve of the quadratic-element system per wavenumber (Sec. IV A).
 * BEM_FP64_DIRECT: float64 LU.  The float32 modes: the float32 LU of the
 * rounded matrix (4M / 3M / bf16x3 updates) refined against the stored float64
 * operator until ||dx||_2/||x||_2 <= tol_step; items that do not converge in
 * max_iter sweeps are re-solved in float64 when fallback != 0 (else ENOCONV).
 * k[n_k], y[n_k][n_rhs][n] c128 [dev]; x_out[n_k][n_rhs][n] c128 [dev];
 * info [host] [n_k*n_rhs] or NULL (rel_resid is that of the stored float64
 * operator).  Synchronises the stream. */
bem_status bem_solve_quadratic(bem_ctx* ctx, const bem_quad_surface* s, int32_t n_k,
                               const double* k, int32_t n_rhs, const void* y,
                               const bem_solve_opts* opts, void* x_out, bem_solve_info* info);

/* Field at observation points by Eq. BRIEFdmn with the element quadrature
 * (x0 the closest node a; the Gauss quadrature of the paper's Sec. III):
 *   4 pi P(x_p) = 4 pi phi_a + int [u (H^p - H^a) - u' (G^p - G^a)] dS,
 *   u = phi - phi_a g - psi_a f,  u' = psi - phi_a g' - psi_a f'
 * in float64; closest node and inside flags as for bem_field_eval.
 * phi, psi [dev] c128 [n_k][n_rhs][n]; xp[m][3], i0[m] (output), inside[m]
 * (output) [dev]; U [dev] c128 [n_rhs][m][n_k]. */
bem_status bem_field_eval_quadratic(bem_ctx* ctx, const bem_quad_surface* s, int32_t n_k,
                                    const double* k, int32_t n_rhs, const void* phi,
                                    const void* psi, int32_t m, const double* xp, int32_t* i0,
                                    uint8_t* inside, void* U);

/* ---------------------------------------------------------------- surrogate
 * A small network mapping a wavenumber to the surface unknowns of a fixed
 * geometry (not part of the paper; its predictions are only used after
 * bem_residual_check accepts them, else the direct solve is used).
 * All arrays [dev] float32 row-major unless stated; W is [in][out].
 * bem_mlp_features: x[B][2 n_oct] = sin / cos(2^l pi k_b / kscale), l < n_oct
 *   (k [dev] float64[B]).
 * bem_mlp_dense_fwd: y = act(x W + b) for x[B][in]; act 0 identity, 1 SiLU
 *   (then z[B][out] receives the pre-activation x W + b).
 * bem_mlp_dense_bwd: given dy[B][out]: dW = x^T dz, db = column sums of dz,
 *   dx = dz W^T (dx may be NULL), dz = dy * silu'(z) (act 1; dz is caller
 *   scratch [B][out]) or dy (act 0).
 * bem_mlp_mse_grad: dy = 2 (y - t) / count and loss_partial[n_partial] [dev]
 *   float64 partial sums of (y - t)^2 over `count` elements.
 * bem_mlp_adam: one Adam step (Kingma & Ba 2015, Algorithm 1) on n params.
 * bem_mlp_pack: t[B][2n] = (Re x, Im x) / scale_j from c128 x[B][n]; with
 *   compute_scale the per-node RMS of |x| over the batch is first stored in
 *   scale[n] [dev] float64.  bem_mlp_unpack is the inverse. */
bem_status bem_mlp_features(bem_ctx* ctx, int32_t B, const double* k, int32_t n_oct,
                            double kscale, float* x);
bem_status bem_mlp_dense_fwd(bem_ctx* ctx, int32_t B, int32_t in, int32_t out, const float* x,
                             const float* W, const float* b, int32_t act, float* z, float* y);
bem_status bem_mlp_dense_bwd(bem_ctx* ctx, int32_t B, int32_t in, int32_t out, const float* x,
                             const float* W, const float* z, int32_t act, const float* dy,
                             float* dW, float* db, float* dx, float* dz);
bem_status bem_mlp_mse_grad(bem_ctx* ctx, int64_t count, const float* y, const float* t,
                            float* dy, double* loss_partial, int32_t n_partial);
bem_status bem_mlp_adam(bem_ctx* ctx, int64_t n, float* p, const float* g, float* m, float* v,
                        int32_t step, float lr, float b1, float b2, float eps);
bem_status bem_mlp_pack(bem_ctx* ctx, int32_t B, int32_t n, const void* x, double* scale,
                        int32_t compute_scale, float* t);
bem_status bem_mlp_unpack(bem_ctx* ctx, int32_t B, int32_t n, const float* t,
                          const double* scale, void* x);

#ifdef __cplusplus
}
#endif
#endif /* BEM_H */
