// C ABI of the library: argument validation, the per-chunk solve pipeline
// (assembly -> float32 LU -> refinement with the float64 residual -> float64
// fallback) and the field / synthesis entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <vector>

#include "common.h"

namespace bem {

bem_status lu_perm(bem_ctx* ctx, int n, int batch, const int32_t* piv, int32_t* perm);
bem_status lu_solve_perm(bem_ctx* ctx, bem_prec prec, int n, int64_t ld, int64_t stride,
                         int batch, const void* LU, const int32_t* perm, int n_rhs,
                         const void* Bin, void* X, int64_t bstride, const int32_t* fac_index = nullptr,
                         const int32_t* vidx = nullptr, int n_sel = 0);

bem_status fail(bem_ctx* ctx, bem_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

static hipEvent_t take_event(bem_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int prof_begin(bem_ctx* ctx, const char* kernel) {
  if (!ctx->profiling) return -1;
  if (!ctx->prof_filter.empty() &&
      ctx->prof_filter.find("," + std::string(kernel) + ",") == std::string::npos)
    return -1;
  KernelStat& k = ctx->stats[kernel];
  hipEvent_t e = take_event(ctx);
  if (!e) return -1;
  (void)hipEventRecord(e, ctx->stream);
  k.ev.push_back(e);
  return (int)k.ev.size() - 1;
}

void prof_end(bem_ctx* ctx, const char* kernel, int idx, double flops, double bytes) {
  if (idx < 0) return;
  KernelStat& k = ctx->stats[kernel];
  hipEvent_t e = take_event(ctx);
  if (!e) return;
  (void)hipEventRecord(e, ctx->stream);
  k.ev.push_back(e);
  k.ev_flops.push_back(flops);
  k.ev_bytes.push_back(bytes);
}

static void resolve_stats(bem_ctx* ctx) {
  for (auto& kv : ctx->stats) {
    KernelStat& k = kv.second;
    for (size_t i = 0; i + 1 < k.ev.size(); i += 2) {
      float ms = 0.f;
      (void)hipEventSynchronize(k.ev[i + 1]);
      (void)hipEventElapsedTime(&ms, k.ev[i], k.ev[i + 1]);
      k.ms += ms;
      k.flops += k.ev_flops[i / 2];
      k.bytes += k.ev_bytes[i / 2];
      k.launches += 1;
      ctx->event_pool.push_back(k.ev[i]);
      ctx->event_pool.push_back(k.ev[i + 1]);
    }
    k.ev.clear();
    k.ev_flops.clear();
    k.ev_bytes.clear();
  }
}

bem_status workspace(bem_ctx* ctx, size_t bytes, void** out) {
  if (bytes <= ctx->ws_size) {
    *out = ctx->ws;
    return BEM_OK;
  }
  if (ctx->ws) {
    BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    drop_graphs(ctx);   // captured factorisations point into the old workspace
    BEM_HIP_TRY(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_size = 0;
  }
  if (hipMalloc(&ctx->ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return fail(ctx, BEM_ENOMEM, "device workspace of %zu bytes could not be allocated", bytes);
  }
  ctx->ws_size = bytes;
  *out = ctx->ws;
  return BEM_OK;
}

bem_status pinned(bem_ctx* ctx, size_t bytes, void** out) {
  if (bytes > ctx->pinned_size) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_size = 0;
    BEM_HIP_TRY(ctx, hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
    ctx->pinned_size = bytes;
  }
  *out = ctx->pinned;
  return BEM_OK;
}

}  // namespace bem

using namespace bem;

namespace {

bool surface_ok(bem_ctx* ctx, const bem_surface* s, bem_status* st) {
  if (!s || s->n <= 0 || !s->x || !s->nrm || !s->w || !s->bc) {
    *st = fail(ctx, BEM_EINVAL, "surface: n must be > 0 and x, nrm, w, bc non-NULL");
    return false;
  }
  return true;
}

// Host-side checks of the surface data (normals unit, weights > 0, finite
// coordinates, flags in {0,1}); copies n*7 doubles to the host.
bem_status check_surface_values(bem_ctx* ctx, const bem_surface* s) {
  const int n = s->n;
  std::vector<double> x(3 * n), nr(3 * n), w(n);
  std::vector<uint8_t> bc(n);
  BEM_HIP_TRY(ctx, hipMemcpyAsync(x.data(), s->x, 24 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipMemcpyAsync(nr.data(), s->nrm, 24 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipMemcpyAsync(w.data(), s->w, 8 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipMemcpyAsync(bc.data(), s->bc, (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < n; ++i) {
    const double l = nr[3 * i] * nr[3 * i] + nr[3 * i + 1] * nr[3 * i + 1] + nr[3 * i + 2] * nr[3 * i + 2];
    if (!(std::fabs(std::sqrt(l) - 1.0) <= 1e-12))
      return fail(ctx, BEM_EINVAL, "surface: normal %d is not a unit vector", i);
    if (!(w[i] > 0.0) || !std::isfinite(w[i]))
      return fail(ctx, BEM_EINVAL, "surface: weight %d is not positive and finite", i);
    if (!std::isfinite(x[3 * i]) || !std::isfinite(x[3 * i + 1]) || !std::isfinite(x[3 * i + 2]))
      return fail(ctx, BEM_EINVAL, "surface: node %d has a non-finite coordinate", i);
    if (bc[i] > 1) return fail(ctx, BEM_EINVAL, "surface: bc[%d] = %d not in {0,1}", i, bc[i]);
  }
  return BEM_OK;
}

bem_status check_k(bem_ctx* ctx, int n_k, const double* k) {
  if (n_k <= 0 || !k) return fail(ctx, BEM_EINVAL, "n_k must be > 0 and k non-NULL");
  std::vector<double> h(n_k);
  BEM_HIP_TRY(ctx, hipMemcpyAsync(h.data(), k, 8 * (size_t)n_k, hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < n_k; ++i)
    if (!(h[i] > 0.0) || !std::isfinite(h[i]))
      return fail(ctx, BEM_EINVAL, "k[%d] = %g must be positive and finite", i, h[i]);
  return BEM_OK;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Chunk {
  // device buffers of one chunk of kc wavenumbers (n nodes, nr right-hand sides)
  void* A;         // [kc][n][ld] c64 or c128
  int32_t* piv;    // [kc][n]
  int32_t* perm;   // [kc][n]
  int32_t* info;   // [kc]
  double2* diag;   // [kc][n][2]
  double2* b;      // [kc][nr][n]
  double2* x;      // [kc][nr][n]
  double2* r;      // [kc][nr][n]
  float2* r32;     // [kc][nr][n]
  float2* d32;     // [kc][nr][n]
  double* scale;   // [kc*nr]
  double* dn2;     // [kc*nr]
  double* xn2;     // [kc*nr]
  double* rn2;     // [kc*nr] |r|^2 of the last evaluated residual
  uint8_t* active; // [kc*nr]
  void* rparts;    // residual partial sums (refinement chunks only)
};

Chunk carve(void* base, int n, int64_t ld, int nr, int kc, bool c128, size_t* used = nullptr);

// Bytes carve() lays out for one chunk (the same walk, from address 0).
size_t chunk_bytes(int n, int64_t ld, int nr, int kc, bool c128) {
  size_t used = 0;
  (void)carve(nullptr, n, ld, nr, kc, c128, &used);
  return used;
}

Chunk carve(void* base, int n, int64_t ld, int nr, int kc, bool c128, size_t* used) {
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    void* out = p;
    p += (bytes + 255) / 256 * 256;
    return out;
  };
  const size_t v = (size_t)kc * nr * n;
  Chunk c;
  c.A = take((size_t)kc * n * ld * (c128 ? 16 : 8));
  c.piv = (int32_t*)take((size_t)kc * n * 4);
  c.perm = (int32_t*)take((size_t)kc * n * 4);
  c.info = (int32_t*)take((size_t)kc * 4);
  c.diag = (double2*)take((size_t)kc * n * 32);
  c.b = (double2*)take(v * 16);
  c.x = (double2*)take(v * 16);
  c.r = (double2*)take(v * 16);
  c.r32 = (float2*)take(v * 8);
  c.d32 = (float2*)take(v * 8);
  c.scale = (double*)take((size_t)kc * nr * 8);
  c.dn2 = (double*)take((size_t)kc * nr * 8);
  c.xn2 = (double*)take((size_t)kc * nr * 8);
  c.rn2 = (double*)take((size_t)kc * nr * 8);
  c.active = (uint8_t*)take((size_t)kc * nr);
  c.rparts = c128 ? nullptr : take(residual_parts_bytes(n, kc, nr));
  if (used) *used = (size_t)(p - (char*)base);
  return c;
}

}  // namespace

// ============================================================ context
extern "C" bem_status bem_ctx_create(int device, void* hip_stream, bem_ctx** out) {
  if (!out) return BEM_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BEM_EHIP;
  if (hipSetDevice(device) != hipSuccess) return BEM_EHIP;
  bem_ctx* c = new bem_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cus = prop.multiProcessorCount;
  if (field_scratch_init(c) != BEM_OK) {
    delete c;
    return BEM_EHIP;
  }
  // counters of the persistent GEMM launches, zero before the first launch
  if (hipMalloc(&c->gemm_queue, 64) != hipSuccess || hipMemset(c->gemm_queue, 0, 64) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    if (c->gemm_queue) (void)hipFree(c->gemm_queue);
    delete c;
    return BEM_EHIP;
  }
  *out = c;
  return BEM_OK;
}

extern "C" void bem_ctx_destroy(bem_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  drop_graphs(ctx);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->pack) (void)hipFree(ctx->pack);
  if (ctx->midx) (void)hipFree(ctx->midx);
  if (ctx->gemm_queue) (void)hipFree(ctx->gemm_queue);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  blas_destroy(ctx);
  resolve_stats(ctx);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  delete ctx;
}

extern "C" const char* bem_last_error(const bem_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

extern "C" bem_status bem_ctx_set_workspace_limit(bem_ctx* ctx, uint64_t bytes) {
  if (!ctx) return BEM_EINVAL;
  ctx->ws_limit = bytes;
  return BEM_OK;
}

extern "C" bem_status bem_ctx_set_profiling(bem_ctx* ctx, int32_t on) {
  if (!ctx) return BEM_EINVAL;
  resolve_stats(ctx);
  ctx->stats.clear();
  ctx->profiling = on != 0;
  return BEM_OK;
}

extern "C" bem_status bem_ctx_set_profiling_filter(bem_ctx* ctx, const char* names) {
  if (!ctx) return BEM_EINVAL;
  ctx->prof_filter.clear();
  if (names && *names) {
    ctx->prof_filter = ",";
    for (const char* c = names; *c; ++c)
      if (*c != ' ') ctx->prof_filter += *c;
    ctx->prof_filter += ",";
  }
  return BEM_OK;
}

extern "C" bem_status bem_ctx_kernel_stats(bem_ctx* ctx, const char* kernel, double* flops,
                                           double* bytes, double* ms, int64_t* launches) {
  if (!ctx || !kernel) return BEM_EINVAL;
  resolve_stats(ctx);
  auto it = ctx->stats.find(kernel);
  const KernelStat zero;
  const KernelStat& k = it == ctx->stats.end() ? zero : it->second;
  if (flops) *flops = k.flops;
  if (bytes) *bytes = k.bytes;
  if (ms) *ms = k.ms;
  if (launches) *launches = k.launches;
  return BEM_OK;
}

extern "C" void bem_solve_opts_default(bem_solve_opts* o) {
  if (!o) return;
  o->mode = BEM_FP32_IR_3M;
  o->tol_step = 1e-8;
  o->max_iter = 10;
  o->fallback = 1;
  o->use_graph = 1;
  o->nb = 0;
}

// ============================================================ incident / assembly
extern "C" bem_status bem_incident(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                   const double* k, const double dir[3], void* y) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  if (!dir || !y || n_k <= 0 || !k) return fail(ctx, BEM_EINVAL, "bem_incident: NULL argument");
  const double l = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  if (!(std::fabs(l - 1.0) < 1e-12)) return fail(ctx, BEM_EINVAL, "bem_incident: dir not unit");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  return launch_incident(ctx, s, n_k, k, dir[0], dir[1], dir[2], y);
}

extern "C" bem_status bem_assemble(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                   const double* k, int32_t n_rhs, const void* y, bem_prec prec,
                                   void* A, int32_t ld, void* b, void* diag64) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  if (n_k <= 0 || !k || n_rhs < 0 || (n_rhs > 0 && (!y || !b)) || (A && ld < s->n) ||
      (!A && !diag64 && n_rhs == 0) ||
      (prec != BEM_C64 && prec != BEM_C128))
    return fail(ctx, BEM_EINVAL, "bem_assemble: bad argument (n_k, k, n_rhs, y, b, A, ld, prec)");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if ((st = check_surface_values(ctx, s)) != BEM_OK) return st;
  if ((st = check_k(ctx, n_k, k)) != BEM_OK) return st;
  return launch_assemble(ctx, s, n_k, k, n_rhs, y, prec, A, ld, (int64_t)s->n * ld, b, diag64);
}

extern "C" bem_status bem_residual(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                   const double* k, int32_t n_rhs, const void* y, const void* x,
                                   const void* diag64, void* r) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  if (n_k <= 0 || !k || n_rhs <= 0 || !y || !x || !diag64 || !r)
    return fail(ctx, BEM_EINVAL, "bem_residual: bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if ((st = check_k(ctx, n_k, k)) != BEM_OK) return st;
  return launch_residual(ctx, s, n_k, k, n_rhs, y, x, diag64, r);
}

extern "C" bem_status bem_residual_check(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                         const double* k, int32_t n_rhs, const void* y,
                                         const void* x, double* rel) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  if (n_k <= 0 || !k || n_rhs <= 0 || !y || !x || !rel)
    return fail(ctx, BEM_EINVAL, "bem_residual_check: bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if ((st = check_k(ctx, n_k, k)) != BEM_OK) return st;
  const int n = s->n;
  const int kc = std::min(n_k, 1024);
  const size_t v = (size_t)kc * n_rhs * n;
  const size_t need = (size_t)kc * n * 32 + 2 * v * 16 + (size_t)kc * n_rhs * 16 + 1024;
  void* ws = nullptr;
  if ((st = workspace(ctx, need, &ws)) != BEM_OK) return st;
  char* p = (char*)ws;
  double2* diag = (double2*)p; p += (size_t)kc * n * 32;
  double2* b = (double2*)p; p += v * 16;
  double2* r = (double2*)p; p += v * 16;
  double* rn = (double*)p; p += (size_t)kc * n_rhs * 8;
  double* bn = (double*)p;
  std::vector<double> hr(kc * n_rhs), hb(kc * n_rhs);
  for (int k0 = 0; k0 < n_k; k0 += kc) {
    const int cur = std::min(kc, n_k - k0);
    const double2* yk = (const double2*)y + (size_t)k0 * n_rhs * n;
    const double2* xk = (const double2*)x + (size_t)k0 * n_rhs * n;
    if ((st = launch_assemble(ctx, s, cur, k + k0, n_rhs, yk, BEM_C128, nullptr, n, 0, b, diag)) != BEM_OK)
      return st;
    if ((st = launch_residual(ctx, s, cur, k + k0, n_rhs, yk, xk, diag, r)) != BEM_OK) return st;
    if ((st = launch_norm2(ctx, cur * n_rhs, n, r, rn)) != BEM_OK) return st;
    if ((st = launch_norm2(ctx, cur * n_rhs, n, b, bn)) != BEM_OK) return st;
    BEM_HIP_TRY(ctx, hipMemcpyAsync(hr.data(), rn, 8 * (size_t)cur * n_rhs, hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipMemcpyAsync(hb.data(), bn, 8 * (size_t)cur * n_rhs, hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < cur * n_rhs; ++q)
      rel[(size_t)k0 * n_rhs + q] = hb[q] > 0 ? std::sqrt(hr[q] / hb[q]) : std::sqrt(hr[q]);
  }
  return BEM_OK;
}

extern "C" bem_status bem_split_unknowns(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                         int32_t n_rhs, const void* x, const void* y, void* phi,
                                         void* psi) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  if (n_k <= 0 || n_rhs <= 0 || !x || !y || !phi || !psi)
    return fail(ctx, BEM_EINVAL, "bem_split_unknowns: bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  return launch_split(ctx, s, n_k, n_rhs, x, y, phi, psi);
}

// ============================================================ LU building blocks
extern "C" bem_status bem_getrf_batched(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t ld,
                                        int64_t stride, int32_t batch, void* A, int32_t* piv,
                                        int32_t* info, int32_t nb, int32_t gemm_kind) {
  if (!ctx) return BEM_EINVAL;
  if (n <= 0 || ld < n || stride < (int64_t)n * ld || batch <= 0 || !A || !piv || !info ||
      (prec != BEM_C64 && prec != BEM_C128) || nb < 0 || gemm_kind < BEM_GEMM_4M ||
      gemm_kind > BEM_GEMM_BF16X3_UNPACKED)
    return fail(ctx, BEM_EINVAL, "bem_getrf_batched: bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  const LuPlan plan = lu_plan_for(ctx, prec, prec == BEM_C64 ? gemm_kind : 0, n, nb);
  return lu_factor(ctx, prec, n, ld, stride, batch, A, piv, info, plan, gemm_kind);
}

extern "C" bem_status bem_autotune_lu(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t batch,
                                      int32_t gemm_kind, const int32_t* candidates,
                                      int32_t* best_nb, double* best_ms) {
  if (!ctx) return BEM_EINVAL;
  if (n <= 0 || batch <= 0 || (prec != BEM_C64 && prec != BEM_C128) ||
      gemm_kind < BEM_GEMM_4M || gemm_kind > BEM_GEMM_BF16X3_UNPACKED)
    return fail(ctx, BEM_EINVAL, "bem_autotune_lu: bad argument");
  if (candidates)
    for (int c = 0; candidates[c] != 0; ++c)
      if (candidates[c] < 0) return fail(ctx, BEM_EINVAL, "bem_autotune_lu: negative block width");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  return lu_autotune(ctx, prec, n, batch, prec == BEM_C64 ? gemm_kind : 0, candidates, best_nb,
                     best_ms);
}

extern "C" int32_t bem_autotune_lu_results(bem_ctx* ctx, int32_t max, int32_t* nb,
                                           int32_t* narrow_max, int32_t* persistent, double* ms) {
  if (!ctx) return 0;
  const int cnt = (int)ctx->tune_log.size();
  for (int i = 0; i < cnt && i < max; ++i) {
    if (nb) nb[i] = ctx->tune_log[i].first.nb;
    if (narrow_max) narrow_max[i] = ctx->tune_log[i].first.narrow_max;
    if (persistent) persistent[i] = ctx->tune_log[i].first.persistent;
    if (ms) ms[i] = ctx->tune_log[i].second;
  }
  return cnt;
}

extern "C" bem_status bem_lu_set_plan(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t gemm_kind,
                                      int32_t nb, int32_t narrow_max, int32_t persistent) {
  if (!ctx) return BEM_EINVAL;
  if (n <= 0 || nb <= 0 || (prec != BEM_C64 && prec != BEM_C128) || gemm_kind < BEM_GEMM_4M ||
      gemm_kind > BEM_GEMM_BF16X3_UNPACKED || narrow_max < 64 || narrow_max > 1024 ||
      (persistent != 0 && persistent != 1))
    return fail(ctx, BEM_EINVAL, "bem_lu_set_plan: bad argument");
  drop_graphs(ctx);
  ctx->tuned[{(int)prec * 16 + gemm_kind, (n + 511) / 512 * 512}] =
      bem_ctx::TunedPlan{nb, narrow_max, persistent};
  return BEM_OK;
}

extern "C" bem_status bem_lu_tuned_plan(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t gemm_kind,
                                        int32_t* nb, int32_t* narrow_max, int32_t* persistent) {
  if (!ctx) return BEM_EINVAL;
  const auto it = ctx->tuned.find({(int)prec * 16 + gemm_kind, (n + 511) / 512 * 512});
  if (it == ctx->tuned.end())
    return fail(ctx, BEM_EINVAL, "bem_lu_tuned_plan: no measured plan for this size class");
  if (nb) *nb = it->second.nb;
  if (narrow_max) *narrow_max = it->second.narrow_max;
  if (persistent) *persistent = it->second.persistent;
  return BEM_OK;
}

extern "C" bem_status bem_getrs_batched(bem_ctx* ctx, bem_prec prec, int32_t n, int32_t ld,
                                        int64_t stride, int32_t batch, const void* LU,
                                        const int32_t* piv, int32_t n_rhs, const void* B,
                                        void* X, int64_t bstride) {
  if (!ctx) return BEM_EINVAL;
  if (n <= 0 || ld < n || stride < (int64_t)n * ld || batch <= 0 || !LU || !piv || n_rhs <= 0 ||
      !B || !X || B == X || bstride < (int64_t)n * n_rhs || (prec != BEM_C64 && prec != BEM_C128))
    return fail(ctx, BEM_EINVAL, "bem_getrs_batched: bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  void* ws = nullptr;
  bem_status st = workspace(ctx, sizeof(int32_t) * (size_t)n * batch, &ws);
  if (st != BEM_OK) return st;
  if ((st = lu_perm(ctx, n, batch, piv, (int32_t*)ws)) != BEM_OK) return st;
  return lu_solve_perm(ctx, prec, n, ld, stride, batch, LU, (const int32_t*)ws, n_rhs, B, X,
                       bstride);
}

// ============================================================ batched solve
namespace {

struct SolveRun {
  bem_ctx* ctx;
  const bem_problem* pr;
  const bem_solve_opts* o;
  double2* xout;
  bem_solve_info* info;  // [n_k * n_rhs] for this problem, or NULL
  std::vector<double> hk;  // the wavenumbers, host copy
};

bem_status chunk_assemble(SolveRun& R, const Chunk& c, int k0, int kc, int64_t ld, bem_prec prec) {
  const bem_surface* s = R.pr->s;
  const int n = s->n, nr = R.pr->n_rhs;
  const double2* y = (const double2*)R.pr->y + (size_t)k0 * nr * n;
  return launch_assemble(R.ctx, s, kc, R.pr->k + k0, nr, y, prec, c.A, ld, (int64_t)n * ld, c.b,
                         c.diag);
}

LuMatrixSet chunk_set(const SolveRun& R, const Chunk& c, int kc, int64_t ld) {
  const int n = R.pr->s->n;
  return LuMatrixSet{c.A, c.piv, c.info, ld, (int64_t)n * ld, n, kc};
}

// After the float64 factorisation: triangular solves and the report.
bem_status chunk_finish_fp64(SolveRun& R, const Chunk& c, int k0, int kc, int64_t ld) {
  bem_ctx* ctx = R.ctx;
  const bem_surface* s = R.pr->s;
  const int n = s->n, nr = R.pr->n_rhs;
  const double2* y = (const double2*)R.pr->y + (size_t)k0 * nr * n;
  bem_status st;
  if ((st = lu_perm(ctx, n, kc, c.piv, c.perm)) != BEM_OK) return st;
  double2* xo = R.xout + (size_t)k0 * nr * n;
  if ((st = lu_solve_perm(ctx, BEM_C128, n, ld, (int64_t)n * ld, kc, c.A, c.perm, nr, c.b, xo,
                          (int64_t)nr * n)) != BEM_OK)
    return st;
  std::vector<int32_t> hinfo(kc);
  if ((st = launch_residual(ctx, s, kc, R.pr->k + k0, nr, y, xo, c.diag, c.r)) != BEM_OK) return st;
  if ((st = launch_norm2(ctx, kc * nr, n, c.r, c.dn2)) != BEM_OK) return st;
  if ((st = launch_norm2(ctx, kc * nr, n, c.b, c.xn2)) != BEM_OK) return st;
  std::vector<double> rn(kc * nr), bn(kc * nr);
  BEM_HIP_TRY(ctx, hipMemcpyAsync(rn.data(), c.dn2, 8 * rn.size(), hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipMemcpyAsync(bn.data(), c.xn2, 8 * bn.size(), hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipMemcpyAsync(hinfo.data(), c.info, 4 * kc, hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (R.info)
    for (int v = 0; v < kc * nr; ++v) {
      bem_solve_info& I = R.info[(size_t)k0 * nr + v];
      I.iters = 0;
      I.used_fp64 = 1;
      I.singular = hinfo[v / nr] != 0;
      I.converged = hinfo[v / nr] == 0;
      I.rel_resid = bn[v] > 0 ? std::sqrt(rn[v] / bn[v]) : 0.0;
      I.rel_step = 0.0;
    }
  for (int q = 0; q < kc; ++q)
    if (hinfo[q] != 0) return fail(ctx, BEM_ESINGULAR, "zero pivot in the FP64 factorisation");
  return BEM_OK;
}

// Whole float64 direct solve of wavenumbers [k0, k0+kc) (used for fallbacks).
bem_status solve_fp64_chunk(SolveRun& R, const Chunk& c, int k0, int kc, int64_t ld) {
  bem_status st;
  if ((st = chunk_assemble(R, c, k0, kc, ld, BEM_C128)) != BEM_OK) return st;
  LuPlan plan;
  plan.nb = R.o->nb > 0 ? R.o->nb : lu_plan_nb(R.ctx, BEM_C128, 0, R.pr->s->n);
  std::vector<LuMatrixSet> sets(1, chunk_set(R, c, kc, ld));
  if ((st = lu_factor_groups(R.ctx, BEM_C128, sets, plan, 0)) != BEM_OK) return st;
  return chunk_finish_fp64(R, c, k0, kc, ld);
}

// After the float32 factorisation: refinement against the float64 operator.
bem_status chunk_finish_ir(SolveRun& R, const Chunk& c, int k0, int kc, int64_t ld,
                           std::vector<int>& unconverged) {
  // Refinement: x_0 = 0, r_0 = b; each sweep solves d = LU^{-1} r (float32,
  // scaled).  An item stops
  //  - when ||d|| / ||x + d|| <= tol_step: x is kept without this last
  //    correction (its float64 residual is already known), or
  //  - when the contraction rho = ||d_i|| / ||d_{i-1}|| < 1/2 bounds the error
  //    left after applying d by rho / (1 - rho) * ||d|| / ||x + d|| <= tol_step
  //    (geometric convergence): x += d and its residual is evaluated for the
  //    report, with no further sweep.
  // Otherwise x += d and r = b - A x is evaluated in float64.
  bem_ctx* ctx = R.ctx;
  const bem_surface* s = R.pr->s;
  const int n = s->n, nr = R.pr->n_rhs;
  const int nv = kc * nr;
  const double2* y = (const double2*)R.pr->y + (size_t)k0 * nr * n;
  const double* kk = R.pr->k + k0;
  const double tol = R.o->tol_step;
  bem_status st;
  // the residual passes advance phases along the wavenumbers when they form an even grid
  const double dk = even_grid_step(R.hk.data() + k0, kc);
  if ((st = lu_perm(ctx, n, kc, c.piv, c.perm)) != BEM_OK) return st;
  if ((st = fill_zero(ctx, c.x, (size_t)nv * n * 16)) != BEM_OK) return st;
  if ((st = launch_norm2(ctx, nv, n, c.b, c.rn2)) != BEM_OK) return st;   // r_0 = b
  void* hp = nullptr;
  if ((st = pinned(ctx, (size_t)nv * 24 + (size_t)kc * 4 + 2 * (size_t)nv, &hp)) != BEM_OK) return st;
  double* h_dn = (double*)hp;
  double* h_xn = h_dn + nv;
  double* h_rn = h_xn + nv;
  int32_t* h_info = (int32_t*)(h_rn + nv);
  // two staging slots for the flags: the upload before the correction solve
  // (h_act) completes at the synchronisation that follows it; the upload
  // before the update (h_act2) is only known to be done at the next sweep's
  // synchronisation, so the next sweep's first upload must not reuse its slot
  uint8_t* h_act = (uint8_t*)(h_info + kc);
  uint8_t* h_act2 = h_act + nv;
  // act: takes another sweep; fin: stops once the current correction is applied;
  // fresh: the float64 residual of the current x has been evaluated
  std::vector<uint8_t> act(nv, 1), fin(nv, 0), fresh(nv, 1);
  std::vector<double> step(nv, 1.0), bn(nv, 0.0), dprev(nv, 0.0);
  std::vector<int> iters(nv, 0);
  BEM_HIP_TRY(ctx, hipMemcpyAsync(h_info, c.info, 4 * kc, hipMemcpyDeviceToHost, ctx->stream));
  const double2* rsrc = c.b;
  const int max_it = std::max(1, R.o->max_iter);
  for (int it = 0; it < max_it; ++it) {
    std::memcpy(h_act, act.data(), nv);
    BEM_HIP_TRY(ctx, hipMemcpyAsync(c.active, h_act, nv, hipMemcpyHostToDevice, ctx->stream));
    if ((st = launch_ir_scale(ctx, nv, n, rsrc, c.r32, c.scale)) != BEM_OK) return st;
    if ((st = lu_solve_perm(ctx, BEM_C64, n, ld, (int64_t)n * ld, kc, c.A, c.perm, nr, c.r32,
                            c.d32, (int64_t)nr * n)) != BEM_OK)
      return st;
    if ((st = launch_ir_update(ctx, nv, n, c.d32, c.scale, c.active, c.x, c.dn2, c.xn2, 0)) != BEM_OK)
      return st;
    BEM_HIP_TRY(ctx, hipMemcpyAsync(h_dn, c.dn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipMemcpyAsync(h_xn, c.xn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
    if (it == 0)
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_rn, c.rn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    int more = 0, nfin = 0;
    for (int v = 0; v < nv; ++v) {
      if (!act[v]) continue;
      if (it == 0) bn[v] = h_rn[v];
      iters[v] = it + 1;
      const double sx = h_xn[v] > 0 ? std::sqrt(h_dn[v] / h_xn[v]) : (h_dn[v] > 0 ? 1.0 : 0.0);
      step[v] = sx;
      if (!std::isfinite(sx)) {
        ++more;
        continue;
      }
      if (it > 0 && !(sx > tol)) {
        act[v] = 0;            // converged: keep x
        continue;
      }
      const double rho = it > 0 && dprev[v] > 0 ? std::sqrt(h_dn[v] / dprev[v]) : 1.0;
      dprev[v] = h_dn[v];
      if (it > 0 && rho < 0.5 && rho / (1.0 - rho) * sx <= tol) {
        fin[v] = 1;
        step[v] = rho / (1.0 - rho) * sx;
        ++nfin;
      } else {
        ++more;
      }
    }
    if (more + nfin == 0) break;
    // take the corrections, then the residual of the new iterates
    std::memcpy(h_act2, act.data(), nv);
    BEM_HIP_TRY(ctx, hipMemcpyAsync(c.active, h_act2, nv, hipMemcpyHostToDevice, ctx->stream));
    if ((st = launch_ir_update(ctx, nv, n, c.d32, c.scale, c.active, c.x, c.dn2, c.xn2, 1)) != BEM_OK)
      return st;
    for (int v = 0; v < nv; ++v)
      if (act[v]) fresh[v] = 0;
    if (nfin > 0 || (more > 0 && it + 1 < max_it)) {
      if ((st = launch_residual_b(ctx, s, kc, kk, dk, nr, y, c.b, c.x, c.diag, c.r, c.rparts)) != BEM_OK) return st;
      if ((st = launch_norm2(ctx, nv, n, c.r, c.rn2)) != BEM_OK) return st;
      std::fill(fresh.begin(), fresh.end(), 1);
      rsrc = c.r;
    }
    for (int v = 0; v < nv; ++v)
      if (fin[v]) {
        fin[v] = 0;
        act[v] = 0;
      }
    if (more == 0) break;
  }
  // items that ran out of sweeps with an unevaluated last correction
  bool stale = false;
  for (int v = 0; v < nv; ++v) stale = stale || !fresh[v];
  if (stale) {
    if ((st = launch_residual_b(ctx, s, kc, kk, dk, nr, y, c.b, c.x, c.diag, c.r, c.rparts)) != BEM_OK) return st;
    if ((st = launch_norm2(ctx, nv, n, c.r, c.rn2)) != BEM_OK) return st;
  }
  // c.rn2 now holds |b - A x|^2 of every item's returned x
  BEM_HIP_TRY(ctx, hipMemcpyAsync(h_rn, c.rn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
  double2* xo = R.xout + (size_t)k0 * nr * n;
  BEM_HIP_TRY(ctx, hipMemcpyAsync(xo, c.x, (size_t)nv * n * 16, hipMemcpyDeviceToDevice, ctx->stream));
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int v = 0; v < nv; ++v) {
    const bool conv = !act[v] && h_info[v / nr] == 0 && std::isfinite(step[v]);
    if (!conv) unconverged.push_back(k0 + v / nr);
    if (R.info) {
      bem_solve_info& I = R.info[(size_t)k0 * nr + v];
      I.iters = iters[v];
      I.used_fp64 = 0;
      I.singular = h_info[v / nr] != 0;
      I.converged = conv ? 1 : 0;
      I.rel_resid = bn[v] > 0 ? std::sqrt(h_rn[v] / bn[v]) : 0.0;
      I.rel_step = step[v];
    }
  }
  std::sort(unconverged.begin(), unconverged.end());
  unconverged.erase(std::unique(unconverged.begin(), unconverged.end()), unconverged.end());
  return BEM_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

// All problems advance together in rounds: each round takes a slice of every
// problem's wavenumbers (slices sized so that the round fits the workspace),
// assembles them, factors all of them in one recursion whose launches cover
// every problem still active (uneven n), then refines each problem's slice.
extern "C" bem_status bem_solve_batched(bem_ctx* ctx, const bem_problem* probs, int32_t n_probs,
                                        const bem_solve_opts* opts, void* const* x_out,
                                        bem_solve_info* info) {
  if (!ctx) return BEM_EINVAL;
  if (!probs || n_probs <= 0 || !x_out) return fail(ctx, BEM_EINVAL, "bem_solve_batched: NULL argument");
  bem_solve_opts o;
  bem_solve_opts_default(&o);
  if (opts) o = *opts;
  if (o.mode < BEM_FP64_DIRECT || o.mode > BEM_FP32_IR_B3 || o.max_iter < 0 || !(o.tol_step >= 0.0) || o.nb < 0)
    return fail(ctx, BEM_EINVAL, "bem_solve_batched: bad options");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  bem_status st;
  for (int p = 0; p < n_probs; ++p) {
    const bem_problem& P = probs[p];
    if (!surface_ok(ctx, P.s, &st)) return st;
    if (P.n_rhs <= 0 || !P.y || !x_out[p]) return fail(ctx, BEM_EINVAL, "problem %d: n_rhs, y or x_out", p);
    if ((st = check_k(ctx, P.n_k, P.k)) != BEM_OK) return st;
    if ((st = check_surface_values(ctx, P.s)) != BEM_OK) return st;
    if (P.s->n > 12288) return fail(ctx, BEM_EUNSUPPORTED, "problem %d: n = %d > 12288", p, P.s->n);
  }
  const bool fp64 = o.mode == BEM_FP64_DIRECT;
  const bem_prec prec = fp64 ? BEM_C128 : BEM_C64;
  size_t free_b = 0, total_b = 0;
  BEM_HIP_TRY(ctx, hipMemGetInfo(&free_b, &total_b));
  const size_t limit = ctx->ws_limit ? ctx->ws_limit : (size_t)(0.75 * (double)(free_b + ctx->ws_size));
  std::vector<int64_t> ld(n_probs);
  std::vector<size_t> info_off(n_probs, 0);
  size_t fallback_bytes = 0;
  int max_nk = 0, nmax = 0;
  for (int p = 0; p < n_probs; ++p) {
    ld[p] = round_up(probs[p].s->n, 16);
    if (p + 1 < n_probs) info_off[p + 1] = info_off[p] + (size_t)probs[p].n_k * probs[p].n_rhs;
    fallback_bytes = std::max(fallback_bytes, chunk_bytes(probs[p].s->n, ld[p], probs[p].n_rhs, 1, true));
    max_nk = std::max(max_nk, probs[p].n_k);
    nmax = std::max(nmax, probs[p].s->n);
  }
  // fewest rounds whose slices fit
  auto round_bytes = [&](int rounds) {
    size_t s = 0;
    for (int p = 0; p < n_probs; ++p) {
      const int kc = (probs[p].n_k + rounds - 1) / rounds;
      s += align256(chunk_bytes(probs[p].s->n, ld[p], probs[p].n_rhs, kc, fp64));
    }
    return s;
  };
  int rounds = 1;
  while (rounds < max_nk && round_bytes(rounds) > limit) rounds = std::min(max_nk, rounds * 2);
  void* ws = nullptr;
  if ((st = workspace(ctx, std::max(round_bytes(rounds), fallback_bytes), &ws)) != BEM_OK) return st;
  LuPlan plan;
  {
    const int gk0 = o.mode == BEM_FP32_IR_3M ? BEM_GEMM_3M
                    : o.mode == BEM_FP32_IR_B3 ? BEM_GEMM_BF16X3 : BEM_GEMM_4M;
    plan = lu_plan_for(ctx, prec, fp64 ? 0 : gk0, nmax, o.nb);
  }
  std::vector<SolveRun> runs;
  for (int p = 0; p < n_probs; ++p) {
    runs.push_back(SolveRun{ctx, &probs[p], &o, (double2*)x_out[p], info ? info + info_off[p] : nullptr, {}});
    runs.back().hk.resize(probs[p].n_k);
    BEM_HIP_TRY(ctx, hipMemcpyAsync(runs.back().hk.data(), probs[p].k, 8 * (size_t)probs[p].n_k,
                                    hipMemcpyDeviceToHost, ctx->stream));
  }
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));

  for (int r = 0; r < rounds; ++r) {
    struct Slice { int p, k0, kc; Chunk c; };
    std::vector<Slice> slices;
    char* base = (char*)ws;
    for (int p = 0; p < n_probs; ++p) {
      const int kcp = (probs[p].n_k + rounds - 1) / rounds;
      const int k0 = r * kcp;
      const int cur = std::min(kcp, probs[p].n_k - k0);
      if (cur <= 0) continue;
      Slice sl{p, k0, cur, carve(base, probs[p].s->n, ld[p], probs[p].n_rhs, cur, fp64)};
      base += align256(chunk_bytes(probs[p].s->n, ld[p], probs[p].n_rhs, cur, fp64));
      if ((st = chunk_assemble(runs[p], sl.c, k0, cur, ld[p], prec)) != BEM_OK) return st;
      slices.push_back(sl);
    }
    for (size_t s0 = 0; s0 < slices.size(); s0 += 8) {
      std::vector<LuMatrixSet> sets;
      for (size_t q = s0; q < std::min(slices.size(), s0 + 8); ++q)
        sets.push_back(chunk_set(runs[slices[q].p], slices[q].c, slices[q].kc, ld[slices[q].p]));
      const int gk = o.mode == BEM_FP32_IR_3M ? BEM_GEMM_3M
                     : o.mode == BEM_FP32_IR_B3 ? BEM_GEMM_BF16X3 : BEM_GEMM_4M;
      // captured graphs replay the launch sequence; per-kernel profiling needs
      // the individual launches
      if (o.use_graph && !ctx->profiling)
        st = lu_factor_groups_graph(ctx, prec, sets, plan, gk);
      else
        st = lu_factor_groups(ctx, prec, sets, plan, gk);
      if (st != BEM_OK) return st;
    }
    std::vector<std::vector<int>> bad(slices.size());
    for (size_t q = 0; q < slices.size(); ++q) {
      Slice& sl = slices[q];
      if (fp64) st = chunk_finish_fp64(runs[sl.p], sl.c, sl.k0, sl.kc, ld[sl.p]);
      else st = chunk_finish_ir(runs[sl.p], sl.c, sl.k0, sl.kc, ld[sl.p], bad[q]);
      if (st != BEM_OK) return st;
    }
    for (size_t q = 0; q < slices.size(); ++q) {
      if (bad[q].empty()) continue;
      const int p = slices[q].p;
      if (!o.fallback)
        return fail(ctx, BEM_ENOCONV, "problem %d: %zu wavenumbers did not converge", p, bad[q].size());
      // float64 direct re-solve of each unconverged wavenumber; the round's
      // other slices are finished, so the workspace base can be reused
      Chunk c1 = carve(ws, probs[p].s->n, ld[p], probs[p].n_rhs, 1, true);
      for (int kq : bad[q])
        if ((st = solve_fp64_chunk(runs[p], c1, kq, 1, ld[p])) != BEM_OK) return st;
    }
  }
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return BEM_OK;
}

// ============================================================ refinement with given factors
extern "C" bem_status bem_refine_batched(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                         const double* k, int32_t n_rhs, const void* y,
                                         const void* LU, int32_t ld, int64_t stride,
                                         const int32_t* piv, int32_t n_fac,
                                         const int32_t* fac_index, double tol_step,
                                         int32_t max_iter, void* x, bem_solve_info* info) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  const int n = s->n;
  if (n_k <= 0 || !k || n_rhs <= 0 || !y || !LU || ld < n || stride < (int64_t)n * ld || !piv ||
      n_fac <= 0 || !fac_index || !(tol_step >= 0.0) || max_iter < 1 || !x)
    return fail(ctx, BEM_EINVAL, "bem_refine_batched: bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if ((st = check_k(ctx, n_k, k)) != BEM_OK) return st;
  {
    std::vector<int32_t> fi(n_k);
    BEM_HIP_TRY(ctx, hipMemcpyAsync(fi.data(), fac_index, 4 * (size_t)n_k, hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < n_k; ++q)
      if (fi[q] < 0 || fi[q] >= n_fac)
        return fail(ctx, BEM_EINVAL, "bem_refine_batched: fac_index[%d] = %d out of range", q, fi[q]);
  }
  const int kc = std::min(n_k, 4096);   // wavenumbers refined together (workspace ~0.4 MB per k at N = 5124)
  const size_t v = (size_t)kc * n_rhs * n;
  size_t need = 0;
  auto sz = [&](size_t b) { return (b + 255) / 256 * 256; };
  need += sz((size_t)n_fac * n * 4) + sz((size_t)kc * n * 32) + 2 * sz(v * 16) + 2 * sz(v * 8) +
          3 * sz((size_t)kc * n_rhs * 8) + sz((size_t)kc * n_rhs) + sz((size_t)kc * 4);
  void* ws = nullptr;
  if ((st = workspace(ctx, need, &ws)) != BEM_OK) return st;
  char* p = (char*)ws;
  auto take = [&](size_t b) { void* o = p; p += sz(b); return o; };
  int32_t* perm = (int32_t*)take((size_t)n_fac * n * 4);
  double2* diag = (double2*)take((size_t)kc * n * 32);
  double2* b = (double2*)take(v * 16);
  double2* r = (double2*)take(v * 16);
  float2* r32 = (float2*)take(v * 8);
  float2* d32 = (float2*)take(v * 8);
  double* scale = (double*)take((size_t)kc * n_rhs * 8);
  double* dn2 = (double*)take((size_t)kc * n_rhs * 8);
  double* xn2 = (double*)take((size_t)kc * n_rhs * 8);
  uint8_t* active = (uint8_t*)take((size_t)kc * n_rhs);
  int32_t* kidx = (int32_t*)take((size_t)kc * 4);   // wavenumbers still refining
  if ((st = lu_perm(ctx, n, n_fac, piv, perm)) != BEM_OK) return st;
  void* hp = nullptr;
  const int nvmax = kc * n_rhs;
  if ((st = pinned(ctx, (size_t)nvmax * 17 + (size_t)kc * 4 + 64, &hp)) != BEM_OK) return st;
  double* h_dn = (double*)hp;
  double* h_xn = h_dn + nvmax;
  int32_t* h_kidx = (int32_t*)(h_xn + nvmax);
  uint8_t* h_act = (uint8_t*)(h_kidx + kc);
  for (int k0 = 0; k0 < n_k; k0 += kc) {
    const int cur = std::min(kc, n_k - k0);
    const int nv = cur * n_rhs;
    const double2* yk = (const double2*)y + (size_t)k0 * n_rhs * n;
    double2* xk = (double2*)x + (size_t)k0 * n_rhs * n;
    if ((st = launch_assemble(ctx, s, cur, k + k0, n_rhs, yk, BEM_C128, nullptr, n, 0, b, diag)) != BEM_OK)
      return st;
    std::vector<uint8_t> act(nv, 1);
    std::vector<double> step(nv, 1.0);
    std::vector<int> iters(nv, 0);
    for (int it = 0; it < max_iter; ++it) {
      // once some wavenumbers have converged, the residual and the correction
      // solve run over the list of those still refining
      int nsel = 0;
      for (int q = 0; q < cur; ++q) {
        bool any = false;
        for (int c = 0; c < n_rhs; ++c) any = any || act[(size_t)q * n_rhs + c];
        if (any) h_kidx[nsel++] = q;
      }
      const int32_t* sel = nullptr;
      if (nsel < cur) {
        BEM_HIP_TRY(ctx, hipMemcpyAsync(kidx, h_kidx, 4 * (size_t)nsel, hipMemcpyHostToDevice, ctx->stream));
        sel = kidx;
      }
      if ((st = launch_residual(ctx, s, cur, k + k0, n_rhs, yk, xk, diag, r, sel, nsel)) != BEM_OK)
        return st;
      std::memcpy(h_act, act.data(), nv);
      BEM_HIP_TRY(ctx, hipMemcpyAsync(active, h_act, nv, hipMemcpyHostToDevice, ctx->stream));
      if ((st = launch_ir_scale(ctx, nv, n, r, r32, scale)) != BEM_OK) return st;
      if ((st = lu_solve_perm(ctx, BEM_C64, n, ld, stride, cur, LU, perm, n_rhs, r32, d32,
                              (int64_t)n_rhs * n, fac_index + k0, sel, nsel)) != BEM_OK)
        return st;
      if ((st = launch_ir_update(ctx, nv, n, d32, scale, active, xk, dn2, xn2)) != BEM_OK) return st;
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_dn, dn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_xn, xn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
      BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      int live = 0;
      for (int q = 0; q < nv; ++q) {
        if (!act[q]) continue;
        iters[q] = it + 1;
        const double sx = h_xn[q] > 0 ? std::sqrt(h_dn[q] / h_xn[q]) : (h_dn[q] > 0 ? 1.0 : 0.0);
        step[q] = sx;
        if (!(sx > tol_step) && std::isfinite(sx)) act[q] = 0;
        else ++live;
      }
      if (live == 0) break;
    }
    if (info) {
      if ((st = launch_residual(ctx, s, cur, k + k0, n_rhs, yk, xk, diag, r)) != BEM_OK) return st;
      if ((st = launch_norm2(ctx, nv, n, r, dn2)) != BEM_OK) return st;
      if ((st = launch_norm2(ctx, nv, n, b, xn2)) != BEM_OK) return st;
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_dn, dn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_xn, xn2, 8 * nv, hipMemcpyDeviceToHost, ctx->stream));
      BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      for (int q = 0; q < nv; ++q) {
        bem_solve_info& I = info[(size_t)k0 * n_rhs + q];
        I.iters = iters[q];
        I.used_fp64 = 0;
        I.singular = 0;
        I.rel_resid = h_xn[q] > 0 ? std::sqrt(h_dn[q] / h_xn[q]) : 0.0;
        I.rel_step = step[q];
        I.converged = act[q] ? 0 : 1;
      }
    }
  }
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return BEM_OK;
}

// ============================================================ field / synthesis
namespace {
bem_status field_eval_impl(bem_ctx* ctx, const char* name, const bem_surface* s, int32_t n_k,
                           const double* k, int32_t n_rhs, const void* phi, const void* psi,
                           int32_t m, const double* xp, int32_t* i0, int32_t i0_given,
                           uint8_t* inside, bem_prec prec, void* U, bool fixed_scratch) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  if (n_k <= 0 || !k || n_rhs <= 0 || !phi || !psi || m < 0 || (m > 0 && (!xp || !i0 || !inside || !U)) ||
      (prec != BEM_C64 && prec != BEM_C128))
    return fail(ctx, BEM_EINVAL, "%s: bad argument", name);
  if (n_rhs > 65535 || (n_k + 7) / 8 > 65535) return fail(ctx, BEM_EINVAL, "%s: n_k or n_rhs too large", name);
  if (fixed_scratch && prec == BEM_C128 && 16 * (size_t)n_rhs * n_k * s->n > ctx->field_scratch_bytes)
    return fail(ctx, BEM_EINVAL,
                "%s: n_rhs * n_k * n = %lld node sums do not fit the %zu-byte fixed scratch", name,
                (long long)n_rhs * n_k * s->n, ctx->field_scratch_bytes);
  if (fixed_scratch && prec == BEM_C64 && field_group_bytes(s->n, m, n_k, n_rhs) > ctx->field_scratch_bytes)
    return fail(ctx, BEM_EINVAL, "%s: the node sums and the grouping of %d points need %zu bytes, "
                "more than the %zu-byte fixed scratch", name, m, field_group_bytes(s->n, m, n_k, n_rhs),
                ctx->field_scratch_bytes);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if (m == 0) return BEM_OK;
  if (!i0_given) {
    if ((st = launch_closest(ctx, s, m, xp, i0, inside)) != BEM_OK) return st;
  } else {
    // closest nodes given: only the inside flags are recomputed from them
    if ((st = launch_inside(ctx, s, m, xp, i0, inside)) != BEM_OK) return st;
  }
  return launch_field(ctx, s, n_k, k, n_rhs, phi, psi, m, xp, i0, inside, prec, U, fixed_scratch);
}
}  // namespace

extern "C" bem_status bem_field_eval(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                     const double* k, int32_t n_rhs, const void* phi,
                                     const void* psi, int32_t m, const double* xp, int32_t* i0,
                                     int32_t i0_given, uint8_t* inside, bem_prec prec, void* U) {
  return field_eval_impl(ctx, "bem_field_eval", s, n_k, k, n_rhs, phi, psi, m, xp, i0, i0_given,
                         inside, prec, U, false);
}

extern "C" bem_status bem_field_eval_noalloc(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                             const double* k, int32_t n_rhs, const void* phi,
                                             const void* psi, int32_t m, const double* xp,
                                             int32_t* i0, int32_t i0_given, uint8_t* inside,
                                             bem_prec prec, void* U) {
  return field_eval_impl(ctx, "bem_field_eval_noalloc", s, n_k, k, n_rhs, phi, psi, m, xp, i0,
                         i0_given, inside, prec, U, true);
}

extern "C" bem_status pulse_synthesize(bem_ctx* ctx, int32_t m, int32_t n_k, const void* U,
                                       int32_t n_pulse, const double* c, int32_t T,
                                       int32_t add_incident, const double* xp, double dk,
                                       float* p) {
  if (!ctx) return BEM_EINVAL;
  if (m < 0 || n_k <= 0 || n_pulse <= 0 || !c || (m > 0 && (!U || !p)) || (add_incident && !xp) ||
      T < 64 || T > 8192 || (T & (T - 1)) != 0 || 2 * n_k > T || !(dk > 0.0) || !std::isfinite(dk))
    return fail(ctx, BEM_EINVAL, "pulse_synthesize: bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  return launch_synth(ctx, m, n_k, U, nullptr, n_pulse, c, T, add_incident, xp, dk, p);
}

extern "C" bem_status pulse_synthesize_sparse(bem_ctx* ctx, int32_t m, int32_t n_sel,
                                              const int32_t* m_index, const void* U,
                                              int32_t n_pulse, const double* c, int32_t T,
                                              int32_t add_incident, const double* xp, double dk,
                                              float* p) {
  if (!ctx) return BEM_EINVAL;
  if (m < 0 || n_sel <= 0 || !m_index || n_pulse <= 0 || !c || (m > 0 && (!U || !p)) ||
      (add_incident && !xp) || T < 64 || T > 8192 || (T & (T - 1)) != 0 || !(dk > 0.0) ||
      !std::isfinite(dk))
    return fail(ctx, BEM_EINVAL, "pulse_synthesize_sparse: bad argument");
  for (int j = 0; j < n_sel; ++j)
    if (m_index[j] < 1 || m_index[j] > T / 2 || (j > 0 && m_index[j] <= m_index[j - 1]))
      return fail(ctx, BEM_EINVAL,
                  "pulse_synthesize_sparse: m_index must increase strictly within 1..T/2 "
                  "(entry %d is %d)", j, m_index[j]);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if (m == 0) return BEM_OK;
  const size_t bytes = sizeof(int32_t) * (size_t)n_sel;
  if (bytes > ctx->midx_cap) {
    if (ctx->midx) {
      BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      BEM_HIP_TRY(ctx, hipFree(ctx->midx));
      ctx->midx = nullptr;
      ctx->midx_cap = 0;
    }
    if (hipMalloc((void**)&ctx->midx, bytes) != hipSuccess) {
      (void)hipGetLastError();
      ctx->midx = nullptr;
      return fail(ctx, BEM_ENOMEM, "pulse_synthesize_sparse: index buffer");
    }
    ctx->midx_cap = bytes;
  }
  BEM_HIP_TRY(ctx, hipMemcpyAsync(ctx->midx, m_index, bytes, hipMemcpyHostToDevice, ctx->stream));
  // the host list may be reused as soon as the call returns
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return launch_synth(ctx, m, n_sel, U, ctx->midx, n_pulse, c, T, add_incident, xp, dk, p);
}

// ============================================================ quadratic elements
namespace {

bool quad_surface_ok(bem_ctx* ctx, const bem_quad_surface* s, bem_status* st) {
  if (!s || s->n <= 0 || !s->x || !s->nrm || !s->bc || s->n_elem <= 0 || !s->elem) {
    *st = fail(ctx, BEM_EINVAL, "quadratic surface: n, n_elem must be > 0 and x, nrm, bc, elem non-NULL");
    return false;
  }
  if ((int64_t)s->n_elem * 7 * 8 >= ((int64_t)1 << 31)) {
    *st = fail(ctx, BEM_EINVAL, "quadratic surface: too many elements");
    return false;
  }
  return true;
}

// buffers of one chunk of kc wavenumbers of the quadratic solve
struct QuadChunk {
  double2* A64;    // [kc][n][ld] the float64 operator (kept for the residual)
  void* LU;        // [kc][n][ld] c128 (FP64 direct) or c64 factors
  int32_t* piv;    // [kc][n]
  int32_t* perm;   // [kc][n]
  int32_t* info;   // [kc]
  double2* diag;   // [kc][n][2]
  double2* b;      // [kc][nr][n]
  double2* x;      // [kc][nr][n]
  double2* r;      // [kc][nr][n]
  float2* r32;     // [kc][nr][n]
  float2* d32;     // [kc][nr][n]
  double* scale;   // [kc*nr]
  double* dn2;     // [kc*nr]
  double* xn2;     // [kc*nr]
  double* rn2;     // [kc*nr]
  uint8_t* active; // [kc*nr]
};

QuadChunk quad_carve(void* base, int n, int64_t ld, int nr, int kc, bool c128_factors,
                     size_t* used) {
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    void* out = p;
    p += (bytes + 255) / 256 * 256;
    return out;
  };
  const size_t v = (size_t)kc * nr * n;
  QuadChunk c;
  c.A64 = (double2*)take((size_t)kc * n * ld * 16);
  c.LU = take((size_t)kc * n * ld * (c128_factors ? 16 : 8));
  c.piv = (int32_t*)take((size_t)kc * n * 4);
  c.perm = (int32_t*)take((size_t)kc * n * 4);
  c.info = (int32_t*)take((size_t)kc * 4);
  c.diag = (double2*)take((size_t)kc * n * 32);
  c.b = (double2*)take(v * 16);
  c.x = (double2*)take(v * 16);
  c.r = (double2*)take(v * 16);
  c.r32 = (float2*)take(v * 8);
  c.d32 = (float2*)take(v * 8);
  c.scale = (double*)take((size_t)kc * nr * 8);
  c.dn2 = (double*)take((size_t)kc * nr * 8);
  c.xn2 = (double*)take((size_t)kc * nr * 8);
  c.rn2 = (double*)take((size_t)kc * nr * 8);
  c.active = (uint8_t*)take((size_t)kc * nr);
  if (used) *used = (size_t)(p - (char*)base);
  return c;
}

}  // namespace

extern "C" bem_status bem_assemble_quadratic(bem_ctx* ctx, const bem_quad_surface* s, int32_t n_k,
                                             const double* k, int32_t n_rhs, const void* y,
                                             bem_prec prec, void* A, int32_t ld, void* b,
                                             void* diag64) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!quad_surface_ok(ctx, s, &st)) return st;
  if (n_rhs <= 0 || !y || !b || (prec != BEM_C64 && prec != BEM_C128) || (A && ld < s->n))
    return fail(ctx, BEM_EINVAL, "bem_assemble_quadratic: bad argument");
  if (n_k > 65535) return fail(ctx, BEM_EINVAL, "bem_assemble_quadratic: n_k > 65535");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if ((st = check_k(ctx, n_k, k)) != BEM_OK) return st;
  void* ws = nullptr;
  if ((st = workspace(ctx, quad_setup_bytes(s->n, s->n_elem), &ws)) != BEM_OK) return st;
  double* qp = nullptr;
  int32_t* inc = nullptr;
  if ((st = quad_setup(ctx, s, ws, &qp, &inc)) != BEM_OK) return st;
  return launch_quad_assemble(ctx, s, qp, inc, n_k, k, n_rhs, y, prec, A, A ? ld : 0,
                              A ? (int64_t)s->n * ld : 0, b, diag64);
}

// Chunks of wavenumbers sized to the workspace: float64 assembly (the operator
// is kept), factorisation (float64, or float32 of the rounded matrix), and for
// the float32 modes refinement r = b - A64 x until ||dx|| / ||x|| <= tol_step.
extern "C" bem_status bem_solve_quadratic(bem_ctx* ctx, const bem_quad_surface* s, int32_t n_k,
                                          const double* k, int32_t n_rhs, const void* y,
                                          const bem_solve_opts* opts, void* x_out,
                                          bem_solve_info* info) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!quad_surface_ok(ctx, s, &st)) return st;
  bem_solve_opts o;
  bem_solve_opts_default(&o);
  if (opts) o = *opts;
  if (n_rhs <= 0 || !y || !x_out || o.mode < BEM_FP64_DIRECT || o.mode > BEM_FP32_IR_B3 ||
      o.max_iter < 0 || !(o.tol_step >= 0.0) || o.nb < 0)
    return fail(ctx, BEM_EINVAL, "bem_solve_quadratic: bad argument");
  if (s->n > 12288) return fail(ctx, BEM_EUNSUPPORTED, "bem_solve_quadratic: n = %d > 12288", s->n);
  if (n_rhs > 65535) return fail(ctx, BEM_EINVAL, "bem_solve_quadratic: n_rhs > 65535");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if ((st = check_k(ctx, n_k, k)) != BEM_OK) return st;
  const int n = s->n, nr = n_rhs;
  const int64_t ld = round_up(n, 16);
  const bool fp64 = o.mode == BEM_FP64_DIRECT;
  const int gk = o.mode == BEM_FP32_IR_3M ? BEM_GEMM_3M
                 : o.mode == BEM_FP32_IR_B3 ? BEM_GEMM_BF16X3 : BEM_GEMM_4M;
  const size_t setup = quad_setup_bytes(n, s->n_elem);
  auto bytes = [&](int kc, bool c128f) {
    size_t used = 0;
    (void)quad_carve(nullptr, n, ld, nr, kc, c128f, &used);
    return used + setup + 256;
  };
  size_t free_b = 0, total_b = 0;
  BEM_HIP_TRY(ctx, hipMemGetInfo(&free_b, &total_b));
  const size_t limit = ctx->ws_limit ? ctx->ws_limit : (size_t)(0.75 * (double)(free_b + ctx->ws_size));
  int kc = n_k;
  // the residual grid holds a chunk's kc * n_rhs vectors in its y dimension
  while (kc > 1 && (bytes(kc, true) > limit || (int64_t)kc * n_rhs > 65535)) kc = (kc + 1) / 2;
  void* ws = nullptr;
  if ((st = workspace(ctx, bytes(kc, true), &ws)) != BEM_OK) return st;
  double* qp = nullptr;
  int32_t* inc = nullptr;
  if ((st = quad_setup(ctx, s, ws, &qp, &inc)) != BEM_OK) return st;
  void* cbase = (char*)ws + (setup + 255) / 256 * 256;
  void* hp = nullptr;
  if ((st = pinned(ctx, (size_t)kc * nr * 24 + (size_t)kc * nr + (size_t)kc * 4 + 8, &hp)) != BEM_OK)
    return st;
  double* h_dn = (double*)hp;
  double* h_xn = h_dn + (size_t)kc * nr;
  double* h_rn = h_xn + (size_t)kc * nr;
  uint8_t* h_act = (uint8_t*)(h_rn + (size_t)kc * nr);
  int32_t* h_info = (int32_t*)(h_act + ((size_t)kc * nr + 3) / 4 * 4);
  LuPlan plan;
  for (int k0 = 0; k0 < n_k; k0 += kc) {
    const int cur = std::min(kc, n_k - k0);
    const int nv = cur * nr;
    const int64_t stride = (int64_t)n * ld;
    const double2* yk = (const double2*)y + (size_t)k0 * nr * n;
    double2* xo = (double2*)x_out + (size_t)k0 * nr * n;
    bool chunk_fp64 = fp64;
    std::vector<uint8_t> act(nv, 1);
    std::vector<int> iters(nv, 0);
    std::vector<double> step(nv, 0.0), bn(nv, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
      QuadChunk c = quad_carve(cbase, n, ld, nr, cur, true, nullptr);
      if ((st = launch_quad_assemble(ctx, s, qp, inc, cur, k + k0, nr, yk, BEM_C128, c.A64, ld,
                                     stride, c.b, c.diag)) != BEM_OK)
        return st;
      if ((st = launch_norm2(ctx, nv, n, c.b, c.rn2)) != BEM_OK) return st;
      std::vector<LuMatrixSet> sets(1, LuMatrixSet{c.LU, c.piv, c.info, ld, stride, n, cur});
      if (chunk_fp64) {
        BEM_HIP_TRY(ctx, hipMemcpyAsync(c.LU, c.A64, (size_t)cur * stride * 16,
                                        hipMemcpyDeviceToDevice, ctx->stream));
        plan.nb = o.nb > 0 ? o.nb : lu_plan_nb(ctx, BEM_C128, 0, n);
        if ((st = lu_factor_groups(ctx, BEM_C128, sets, plan, 0)) != BEM_OK) return st;
        if ((st = lu_perm(ctx, n, cur, c.piv, c.perm)) != BEM_OK) return st;
        if ((st = lu_solve_perm(ctx, BEM_C128, n, ld, stride, cur, c.LU, c.perm, nr, c.b, c.x,
                                (int64_t)nr * n)) != BEM_OK)
          return st;
      } else {
        if ((st = launch_c128_to_c64(ctx, (int64_t)cur * stride, c.A64, c.LU)) != BEM_OK) return st;
        plan = lu_plan_for(ctx, BEM_C64, gk, n, o.nb);
        if ((st = lu_factor_groups(ctx, BEM_C64, sets, plan, gk)) != BEM_OK) return st;
        if ((st = lu_perm(ctx, n, cur, c.piv, c.perm)) != BEM_OK) return st;
        if ((st = fill_zero(ctx, c.x, (size_t)nv * n * 16)) != BEM_OK) return st;
        BEM_HIP_TRY(ctx, hipMemcpyAsync(c.r, c.b, (size_t)nv * n * 16, hipMemcpyDeviceToDevice,
                                        ctx->stream));
        std::fill(act.begin(), act.end(), 1);
        for (int it = 0; it < std::max(1, o.max_iter); ++it) {
          std::memcpy(h_act, act.data(), nv);
          BEM_HIP_TRY(ctx, hipMemcpyAsync(c.active, h_act, nv, hipMemcpyHostToDevice, ctx->stream));
          if ((st = launch_ir_scale(ctx, nv, n, c.r, c.r32, c.scale)) != BEM_OK) return st;
          if ((st = lu_solve_perm(ctx, BEM_C64, n, ld, stride, cur, c.LU, c.perm, nr, c.r32,
                                  c.d32, (int64_t)nr * n)) != BEM_OK)
            return st;
          if ((st = launch_ir_update(ctx, nv, n, c.d32, c.scale, c.active, c.x, c.dn2, c.xn2, 1)) != BEM_OK)
            return st;
          if ((st = launch_quad_residual(ctx, n, c.A64, ld, stride, cur, nr, c.b, c.x, c.r)) != BEM_OK)
            return st;
          BEM_HIP_TRY(ctx, hipMemcpyAsync(h_dn, c.dn2, 8 * (size_t)nv, hipMemcpyDeviceToHost, ctx->stream));
          BEM_HIP_TRY(ctx, hipMemcpyAsync(h_xn, c.xn2, 8 * (size_t)nv, hipMemcpyDeviceToHost, ctx->stream));
          BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
          int live = 0;
          for (int v = 0; v < nv; ++v) {
            if (!act[v]) continue;
            iters[v] = it + 1;
            step[v] = h_xn[v] > 0 ? std::sqrt(h_dn[v] / h_xn[v]) : (h_dn[v] > 0 ? 1.0 : 0.0);
            if (std::isfinite(step[v]) && !(step[v] > o.tol_step)) act[v] = 0;
            else ++live;
          }
          if (live == 0) break;
        }
      }
      // report: the float64 operator's residual of the returned x
      if ((st = launch_quad_residual(ctx, n, c.A64, ld, stride, cur, nr, c.b, c.x, c.r)) != BEM_OK)
        return st;
      if ((st = launch_norm2(ctx, nv, n, c.r, c.dn2)) != BEM_OK) return st;
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_dn, c.dn2, 8 * (size_t)nv, hipMemcpyDeviceToHost, ctx->stream));
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_rn, c.rn2, 8 * (size_t)nv, hipMemcpyDeviceToHost, ctx->stream));
      BEM_HIP_TRY(ctx, hipMemcpyAsync(h_info, c.info, 4 * (size_t)cur, hipMemcpyDeviceToHost, ctx->stream));
      BEM_HIP_TRY(ctx, hipMemcpyAsync(xo, c.x, (size_t)nv * n * 16, hipMemcpyDeviceToDevice, ctx->stream));
      BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      bool bad = false;
      for (int v = 0; v < nv; ++v) {
        const bool conv = chunk_fp64 ? h_info[v / nr] == 0 : (!act[v] && h_info[v / nr] == 0);
        bad = bad || !conv;
        if (info) {
          bem_solve_info& I = info[(size_t)k0 * nr + v];
          I.iters = chunk_fp64 ? 0 : iters[v];
          I.used_fp64 = chunk_fp64 && !fp64 ? 1 : 0;
          I.singular = h_info[v / nr] != 0;
          I.converged = conv ? 1 : 0;
          I.rel_resid = h_rn[v] > 0 ? std::sqrt(h_dn[v] / h_rn[v]) : 0.0;
          I.rel_step = chunk_fp64 ? 0.0 : step[v];
        }
      }
      if (chunk_fp64) {
        for (int q = 0; q < cur; ++q)
          if (h_info[q] != 0) return fail(ctx, BEM_ESINGULAR, "zero pivot in the FP64 factorisation");
        break;
      }
      if (!bad) break;
      if (!o.fallback)
        return fail(ctx, BEM_ENOCONV, "bem_solve_quadratic: refinement did not converge");
      chunk_fp64 = true;   // re-solve the whole chunk in float64
    }
  }
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return BEM_OK;
}

extern "C" bem_status bem_field_eval_quadratic(bem_ctx* ctx, const bem_quad_surface* s,
                                               int32_t n_k, const double* k, int32_t n_rhs,
                                               const void* phi, const void* psi, int32_t m,
                                               const double* xp, int32_t* i0, uint8_t* inside,
                                               void* U) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!quad_surface_ok(ctx, s, &st)) return st;
  if (n_k <= 0 || !k || n_rhs <= 0 || !phi || !psi || m < 0 || (m > 0 && (!xp || !i0 || !inside || !U)))
    return fail(ctx, BEM_EINVAL, "bem_field_eval_quadratic: bad argument");
  if (n_k > 65535 || n_rhs > 65535) return fail(ctx, BEM_EINVAL, "bem_field_eval_quadratic: n_k or n_rhs too large");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if (m == 0) return BEM_OK;
  const size_t setup = (quad_setup_bytes(s->n, s->n_elem) + 255) / 256 * 256;
  const size_t interp = ((size_t)n_k * n_rhs * s->n_elem * 7 * 16 + 255) / 256 * 256;
  void* ws = nullptr;
  if ((st = workspace(ctx, setup + 2 * interp, &ws)) != BEM_OK) return st;
  double* qp = nullptr;
  int32_t* inc = nullptr;
  if ((st = quad_setup(ctx, s, ws, &qp, &inc)) != BEM_OK) return st;
  bem_surface nodal{s->n, s->x, s->nrm, nullptr, s->bc};
  if ((st = launch_closest(ctx, &nodal, m, xp, i0, inside)) != BEM_OK) return st;
  char* base = (char*)ws + setup;
  return launch_quad_field(ctx, s, qp, n_k, k, n_rhs, phi, psi, base, base + interp, m, xp, i0,
                           inside, U);
}

// ============================================================ interior-point rows
// Least-squares solve of the surface rows and the interior-point rows through
// the float64 normal equations (see chief.hip), chunks of wavenumbers sized to
// the workspace.
extern "C" bem_status bem_solve_chief(bem_ctx* ctx, const bem_surface* s, int32_t n_k,
                                      const double* k, int32_t n_rhs, const void* y, int32_t n_c,
                                      const double* xc, void* x_out, bem_solve_info* info) {
  if (!ctx) return BEM_EINVAL;
  bem_status st;
  if (!surface_ok(ctx, s, &st)) return st;
  if (n_rhs <= 0 || n_rhs > 65535 || !y || !x_out || n_c <= 0 || n_c > 65535 || !xc)
    return fail(ctx, BEM_EINVAL, "bem_solve_chief: bad argument");
  if (s->n > 12288) return fail(ctx, BEM_EUNSUPPORTED, "bem_solve_chief: n = %d > 12288", s->n);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BEM_EHIP, "hipSetDevice");
  if ((st = check_surface_values(ctx, s)) != BEM_OK) return st;
  if ((st = check_k(ctx, n_k, k)) != BEM_OK) return st;
  const int n = s->n, nr = n_rhs, naug = n + nr;
  const int64_t ld = round_up(naug, 16);
  const int64_t sa = (int64_t)n * ld, sc = (int64_t)n_c * ld, sm = (int64_t)naug * ld;
  const int rows = n + n_c;
  auto carve = [&](void* base, int kc, char** p_out, size_t* used) {
    char* p = (char*)base;
    auto take = [&](size_t bytes) {
      char* o = p;
      p += (bytes + 255) / 256 * 256;
      return o;
    };
    const size_t v = (size_t)kc * nr;
    p_out[0] = take((size_t)kc * sa * 16);   // [A | b]
    p_out[1] = take((size_t)kc * sc * 16);   // [C | d]
    p_out[2] = take((size_t)kc * sm * 16);   // normal equations, then their factors
    p_out[3] = take((size_t)kc * n * 4);     // piv
    p_out[4] = take((size_t)kc * n * 4);     // perm
    p_out[5] = take((size_t)kc * 4);         // info
    p_out[6] = take(v * n * 16);             // b
    p_out[7] = take(v * n * 16);             // right-hand sides of the normal equations
    p_out[8] = take(v * n * 16);             // x
    p_out[9] = take(v * rows * 8);           // squared residual per row
    p_out[10] = take(v * rows * 8);          // squared right-hand side per row
    p_out[11] = take(v * n * 16);            // zeros
    if (used) *used = (size_t)(p - (char*)base);
  };
  size_t free_b = 0, total_b = 0;
  BEM_HIP_TRY(ctx, hipMemGetInfo(&free_b, &total_b));
  const size_t limit = ctx->ws_limit ? ctx->ws_limit : (size_t)(0.75 * (double)(free_b + ctx->ws_size));
  char* P[12];
  auto bytes = [&](int kc) {
    size_t used = 0;
    carve(nullptr, kc, P, &used);
    return used + 256;
  };
  int kc = n_k;
  while (kc > 1 && (bytes(kc) > limit || (int64_t)kc * nr > 65535)) kc = (kc + 1) / 2;
  void* ws = nullptr;
  if ((st = workspace(ctx, bytes(kc), &ws)) != BEM_OK) return st;
  std::vector<double> hrs, hr0;
  std::vector<int32_t> hinfo;
  for (int k0 = 0; k0 < n_k; k0 += kc) {
    const int cur = std::min(kc, n_k - k0);
    const int nv = cur * nr;
    carve(ws, cur, P, nullptr);
    const double2* yk = (const double2*)y + (size_t)k0 * nr * n;
    if ((st = launch_assemble(ctx, s, cur, k + k0, nr, yk, BEM_C128, P[0], ld, sa, P[6], nullptr)) != BEM_OK)
      return st;
    if ((st = launch_aug_b(ctx, n, cur, nr, P[6], P[0], ld, sa)) != BEM_OK) return st;
    if ((st = launch_interior_rows(ctx, s, cur, k + k0, nr, yk, n_c, xc, P[1], ld, sc)) != BEM_OK)
      return st;
    if ((st = gram_c128(ctx, naug, n, P[0], ld, sa, P[2], ld, sm, cur, false)) != BEM_OK) return st;
    if ((st = gram_c128(ctx, naug, n_c, P[1], ld, sc, P[2], ld, sm, cur, true)) != BEM_OK) return st;
    if ((st = launch_extract_rhs(ctx, n, cur, nr, P[2], ld, sm, P[7])) != BEM_OK) return st;
    std::vector<LuMatrixSet> sets(1, LuMatrixSet{P[2], (int32_t*)P[3], (int32_t*)P[5], ld, sm, n, cur});
    LuPlan plan;
    plan.nb = lu_plan_nb(ctx, BEM_C128, 0, n);
    if ((st = lu_factor_groups(ctx, BEM_C128, sets, plan, 0)) != BEM_OK) return st;
    if ((st = lu_perm(ctx, n, cur, (const int32_t*)P[3], (int32_t*)P[4])) != BEM_OK) return st;
    if ((st = lu_solve_perm(ctx, BEM_C128, n, ld, sm, cur, P[2], (const int32_t*)P[4], nr, P[7],
                            P[8], (int64_t)nr * n)) != BEM_OK)
      return st;
    // the stacked system's residual and right-hand side per row
    if ((st = fill_zero(ctx, P[11], (size_t)nv * n * 16)) != BEM_OK) return st;
    if ((st = launch_aug_resid(ctx, n, cur, nr, P[0], ld, sa, n, P[8], (double*)P[9], rows, 0)) != BEM_OK ||
        (st = launch_aug_resid(ctx, n, cur, nr, P[1], ld, sc, n_c, P[8], (double*)P[9], rows, n)) != BEM_OK ||
        (st = launch_aug_resid(ctx, n, cur, nr, P[0], ld, sa, n, P[11], (double*)P[10], rows, 0)) != BEM_OK ||
        (st = launch_aug_resid(ctx, n, cur, nr, P[1], ld, sc, n_c, P[11], (double*)P[10], rows, n)) != BEM_OK)
      return st;
    BEM_HIP_TRY(ctx, hipMemcpyAsync((double2*)x_out + (size_t)k0 * nr * n, P[8], (size_t)nv * n * 16,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    hrs.resize((size_t)nv * rows);
    hr0.resize((size_t)nv * rows);
    hinfo.resize(cur);
    BEM_HIP_TRY(ctx, hipMemcpyAsync(hrs.data(), P[9], 8 * hrs.size(), hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipMemcpyAsync(hr0.data(), P[10], 8 * hr0.size(), hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipMemcpyAsync(hinfo.data(), P[5], 4 * (size_t)cur, hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < cur; ++q)
      if (hinfo[q] != 0)
        return fail(ctx, BEM_ESINGULAR, "bem_solve_chief: zero pivot in the normal equations of k[%d]", k0 + q);
    if (info)
      for (int v = 0; v < nv; ++v) {
        double a = 0.0, b0 = 0.0;
        for (int r = 0; r < rows; ++r) {
          a += hrs[(size_t)v * rows + r];
          b0 += hr0[(size_t)v * rows + r];
        }
        bem_solve_info& I = info[(size_t)k0 * nr + v];
        I.iters = 0;
        I.used_fp64 = 0;
        I.singular = 0;
        I.converged = 1;
        I.rel_resid = b0 > 0 ? std::sqrt(a / b0) : 0.0;
        I.rel_step = 0.0;
      }
  }
  return BEM_OK;
}

