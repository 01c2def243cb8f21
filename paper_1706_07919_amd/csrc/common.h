// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/bem.h"

// Per-kernel accounting filled when profiling is on: every launch of a
// counted kernel is bracketed by two events on the context stream and carries
// its algorithmic flop and byte counts.
struct KernelStat {
  double flops = 0.0, bytes = 0.0, ms = 0.0;
  int64_t launches = 0;
  std::vector<hipEvent_t> ev;       // pending (start, stop) pairs
  std::vector<double> ev_flops, ev_bytes;
};

struct bem_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  uint64_t ws_limit = 0;
  // cached device workspace (grown on demand, freed with the context)
  void* ws = nullptr;
  size_t ws_size = 0;
  // small pinned host staging buffer for norms / flags
  void* pinned = nullptr;
  size_t pinned_size = 0;
  // measured plans of the factorisation keyed by (precision * 16 + GEMM form,
  // n rounded up to 512): block width, the column count up to which the
  // 128 x 64 GEMM tile is used, persistent GEMM launches
  struct TunedPlan {
    int nb, narrow_max, persistent;
  };
  std::map<std::pair<int, int>, TunedPlan> tuned;
  // every candidate of the last bem_autotune_lu call and its time (ms)
  std::vector<std::pair<TunedPlan, double>> tune_log;
  int num_cus = 256;
  bool profiling = false;
  std::string prof_filter;   // ",name,name," of the counted kernels, or empty = all
  std::map<std::string, KernelStat> stats;
  std::vector<hipEvent_t> event_pool;
  // captured factorisations, keyed by every argument of the launch sequence
  // (matrix pointers, sizes, plan, GEMM form); dropped when the workspace moves
  struct LuGraph {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<LuGraph> lu_graphs;
  hipStream_t capture_stream = nullptr;
  // operands of the trailing updates split into bf16 words (grown on demand)
  void* pack = nullptr;
  size_t pack_size = 0;
  // frequency indices of a sparse synthesis (grown on demand)
  int32_t* midx = nullptr;
  size_t midx_cap = 0;
  // device address of the field evaluation's fixed scratch on this context's
  // device (taken once, when the context is created) and its size
  void* field_scratch = nullptr;
  size_t field_scratch_bytes = 0;
  // rocBLAS handle of the interior-point least-squares solve (created on first use)
  void* blas = nullptr;
  // tile counters of the persistent GEMM launches (8 ranges x {next, done},
  // zeroed at creation; every launch leaves them zero)
  void* gemm_queue = nullptr;
};

namespace bem {

bem_status fail(bem_ctx* ctx, bem_status st, const char* fmt, ...);

#define BEM_HIP_TRY(ctx, call)                                                       \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::bem::fail((ctx), BEM_EHIP, "%s failed: %s (%s:%d)", #call,            \
                         hipGetErrorString(e_), __FILE__, __LINE__);                 \
  } while (0)

#define BEM_CHECK_LAUNCH(ctx) BEM_HIP_TRY(ctx, hipGetLastError())

// Profiling brackets: prof_begin returns an index (or -1 when off); prof_end
// records the stop event with the launch's algorithmic work.
int prof_begin(bem_ctx* ctx, const char* kernel);
void prof_end(bem_ctx* ctx, const char* kernel, int idx, double flops, double bytes);

// grow-only device workspace owned by the context
bem_status workspace(bem_ctx* ctx, size_t bytes, void** out);
bem_status pinned(bem_ctx* ctx, size_t bytes, void** out);

// ------------------------------------------------------------------ operator
bem_status launch_incident(bem_ctx*, const bem_surface*, int n_k, const double* k,
                           double dx, double dy, double dz, void* y);
bem_status launch_assemble(bem_ctx*, const bem_surface*, int n_k, const double* k, int n_rhs,
                           const void* y, bem_prec prec, void* A, int64_t ld,
                           int64_t a_stride, void* b, void* diag64);
// kidx (optional, device): evaluate only the n_sel wavenumbers listed (indices
// into k, y, x, diag64, r), leaving the other rows of r untouched.
bem_status launch_residual(bem_ctx*, const bem_surface*, int n_k, const double* k, int n_rhs,
                           const void* y, const void* x, const void* diag64, void* r,
                           const int32_t* kidx = nullptr, int n_sel = 0);
// The same residual from the float64 right-hand side b of the assembly
// (r = b - A x) for wavenumbers on the even grid k_q = k_0 + q dk (dk > 0, as
// even_grid_step reports); y is used only by the fallback (dk <= 0 or surfaces
// under 1024 nodes).  parts: device staging of residual_parts_bytes bytes.
size_t residual_parts_bytes(int n, int n_k, int n_rhs);
bem_status launch_residual_b(bem_ctx*, const bem_surface*, int n_k, const double* k, double dk,
                             int n_rhs, const void* y, const void* b, const void* x,
                             const void* diag64, void* r, void* parts);
// dk of an even grid k_q = k_0 + q dk (to 4e-16 relative per entry, host
// values), else 0
double even_grid_step(const double* k_host, int n_k);
bem_status launch_split(bem_ctx*, const bem_surface*, int n_k, int n_rhs, const void* x,
                        const void* y, void* phi, void* psi);

// ------------------------------------------------------------------ dense LA
// Batched LU with partial pivoting of row-major matrices A_b = A + b*stride
// (n x n, leading dimension ld).  piv_b = piv + b*n (absolute row indices).
// info_b = info + b: 0, or 1 + first zero pivot column.
// complex GEMM forms of the c64 factorisation (the last argument of
// bem_getrf_batched)
enum { kGemm4M = 0, kGemm3M = 1, kGemmBf16x3 = 2, kGemmBf16x3Unpacked = 3 };

struct LuPlan {
  int nb = 0;          // top-level panel width (0 = recursive halving)
  int base = 8;        // width of the register-held base panel
  // float32 MFMA updates: the 128 x 64 tile for updates of at most this many
  // columns (128 x 128 above), and the launch form (0: a workgroup per tile,
  // 1: persistent workgroups drawing tiles from a per-XCD counter)
  int gemm_narrow_max = 64;
  int gemm_persistent = 0;
};
bem_status lu_factor(bem_ctx*, bem_prec, int n, int64_t ld, int64_t stride, int batch, void* A,
                     int32_t* piv, int32_t* info, const LuPlan& plan, int gemm_kind);
// Uneven batches: up to 8 sets of equal-size matrices factored together, one
// launch per recursion step covering every set that still has columns left.
struct LuMatrixSet {
  void* A;
  int32_t* piv;
  int32_t* info;
  int64_t ld, stride;
  int n, count;
};
bem_status lu_factor_groups(bem_ctx*, bem_prec, const std::vector<LuMatrixSet>& sets,
                            const LuPlan& plan, int gemm_kind);
// The same factorisation replayed from a captured hipGraph (captured on first
// use of a given argument set, launched on ctx->stream).
bem_status lu_factor_groups_graph(bem_ctx*, bem_prec, const std::vector<LuMatrixSet>& sets,
                                  const LuPlan& plan, int gemm_kind);
void drop_graphs(bem_ctx* ctx);
// Solve A_b X = B_b in place for B_b = B + b*bstride (n_rhs vectors of length n, stride n).
bem_status lu_solve(bem_ctx*, bem_prec, int n, int64_t ld, int64_t stride, int batch,
                    const void* LU, const int32_t* piv, int n_rhs, void* B, int64_t bstride);
int lu_default_nb(bem_prec prec, int n);
// block width for a factorisation: the measured one of this context when
// bem_autotune_lu has run for the size class, else the default
int lu_plan_nb(bem_ctx* ctx, bem_prec prec, int gemm_kind, int n);
// a factorisation's plan: block width nb (> 0) or the measured / default one,
// and the measured GEMM tile threshold and launch form when the context has
// them for this size class
LuPlan lu_plan_for(bem_ctx* ctx, bem_prec prec, int gemm_kind, int n, int nb);
bem_status lu_autotune(bem_ctx* ctx, bem_prec prec, int n, int batch, int gemm_kind,
                       const int32_t* candidates, int32_t* best_nb, double* best_ms);

// ------------------------------------------------------------------ iterative refinement
bem_status launch_ir_scale(bem_ctx*, int nvec, int n, const void* r, void* r32, double* scale);
bem_status launch_ir_update(bem_ctx*, int nvec, int n, const void* d32, const double* scale,
                            const uint8_t* active, void* x, double* dnorm2, double* xnorm2,
                            int apply = 1);
bem_status launch_norm2(bem_ctx*, int nvec, int n, const void* v, double* out);
bem_status launch_c128_to_c64(bem_ctx*, int64_t count, const void* in, void* out);
bem_status fill_zero(bem_ctx*, void* p, size_t bytes);

// ------------------------------------------------------------------ interior-point rows
bem_status launch_aug_b(bem_ctx*, int n, int n_k, int n_rhs, const void* b, void* A, int64_t ld,
                        int64_t stride);
bem_status launch_interior_rows(bem_ctx*, const bem_surface*, int n_k, const double* k, int n_rhs,
                                const void* y, int n_c, const double* xc, void* C, int64_t ld,
                                int64_t stride);
bem_status gram_c128(bem_ctx*, int len, int m_cols, const void* R, int64_t ld, int64_t r_stride,
                     void* M, int64_t ldm, int64_t m_stride, int batch, bool accumulate);
bem_status launch_extract_rhs(bem_ctx*, int n, int n_k, int n_rhs, const void* M, int64_t ld,
                              int64_t stride, void* r);
bem_status launch_aug_resid(bem_ctx*, int n, int n_k, int n_rhs, const void* R, int64_t ld,
                            int64_t stride, int rows, const void* x, double* rs, int rs_rows,
                            int rs_off);
void blas_destroy(bem_ctx*);
bem_status launch_copy_active(bem_ctx*, int nvec, int n, const uint8_t* active, const void* src,
                              void* dst);

// ------------------------------------------------------------------ field / synthesis
bem_status launch_closest(bem_ctx*, const bem_surface*, int m, const double* xp, int32_t* i0,
                          uint8_t* inside);
bem_status launch_inside(bem_ctx*, const bem_surface*, int m, const double* xp,
                         const int32_t* i0, uint8_t* inside);
// fixed_scratch: node sums in the fixed per-device scratch (no workspace, no
// profiling events), EINVAL when they do not fit
bem_status launch_field(bem_ctx*, const bem_surface*, int n_k, const double* k, int n_rhs,
                        const void* phi, const void* psi, int m, const double* xp,
                        const int32_t* i0, const uint8_t* inside, bem_prec prec, void* U,
                        bool fixed_scratch = false);
// take the device address of the field scratch for ctx (its device current)
bem_status field_scratch_init(bem_ctx* ctx);
// device bytes of the float32 field's node sums and point grouping
size_t field_group_bytes(int n, int m, int n_k, int n_rhs);
// m_index (device, or NULL for the dense grid m = 1..n_k): frequency index of
// each column of U and c
bem_status launch_synth(bem_ctx*, int m, int n_k, const void* U, const int32_t* m_index,
                        int n_pulse, const double* c, int T, int add_incident, const double* xp,
                        double dk, float* p);

// ------------------------------------------------------------------ quadratic elements
// workspace of quad_setup (quadrature points and node incidences)
size_t quad_setup_bytes(int n, int n_elem);
bem_status quad_setup(bem_ctx*, const bem_quad_surface*, void* ws, double** qp, int32_t** inc);
bem_status launch_quad_assemble(bem_ctx*, const bem_quad_surface*, const double* qp,
                                const int32_t* inc, int n_k, const double* k, int n_rhs,
                                const void* y, bem_prec prec, void* A, int64_t ld,
                                int64_t a_stride, void* b, void* diag64);
// r = b - A64 x over n_k matrices (stride elements apart) and n_rhs vectors each
bem_status launch_quad_residual(bem_ctx*, int n, const void* A64, int64_t ld, int64_t stride,
                                int n_k, int n_rhs, const void* b, const void* x, void* r);
// phq, psq: [n_k * n_rhs][n_elem * 7] c128 scratch
bem_status launch_quad_field(bem_ctx*, const bem_quad_surface*, const double* qp, int n_k,
                             const double* k, int n_rhs, const void* phi, const void* psi,
                             void* phq, void* psq, int m, const double* xp, const int32_t* i0,
                             const uint8_t* inside, void* U);

}  // namespace bem
