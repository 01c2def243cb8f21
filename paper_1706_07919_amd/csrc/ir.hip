// Vector kernels of the mixed-precision iterative refinement: the float64
// residual is scaled into float32 for the correction solve, the float32
// correction is added back in float64, and per-vector norms decide
// convergence.  One workgroup per vector.
#include "common.h"

namespace bem {
namespace {

constexpr int kT = 256;

__device__ inline double block_reduce(double v, double* sh, bool is_max) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off, 64);
    v = is_max ? fmax(v, o) : v + o;
  }
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int q = 1; q < kT / 64; ++q) s = is_max ? fmax(s, sh[q]) : s + sh[q];
    sh[0] = s;
  }
  __syncthreads();
  const double out = sh[0];
  __syncthreads();
  return out;
}

__global__ __launch_bounds__(kT) void ir_scale_kernel(int n, const double2* __restrict__ r,
                                                      float2* __restrict__ r32,
                                                      double* __restrict__ scale) {
  __shared__ double sh[kT / 64];
  const int64_t off = (int64_t)blockIdx.x * n;
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) {
    const double2 v = r[off + i];
    m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
  }
  m = block_reduce(m, sh, true);
  const double s = m > 0.0 ? m : 1.0;
  const double inv = 1.0 / s;
  for (int i = threadIdx.x; i < n; i += kT) {
    const double2 v = r[off + i];
    r32[off + i] = make_float2((float)(v.x * inv), (float)(v.y * inv));
  }
  if (threadIdx.x == 0) scale[blockIdx.x] = s;
}

// d = scale * d32; dn2 = |d|^2, xn2 = |x + d|^2; x += d only when apply != 0
// (apply == 0 sizes the correction before deciding whether to take it).
__global__ __launch_bounds__(kT) void ir_update_kernel(int n, const float2* __restrict__ d32,
                                                       const double* __restrict__ scale,
                                                       const uint8_t* __restrict__ active,
                                                       double2* __restrict__ x,
                                                       double* __restrict__ dn2,
                                                       double* __restrict__ xn2, int apply) {
  __shared__ double sh[kT / 64];
  const int v = blockIdx.x;
  if (active && !active[v]) return;
  const int64_t off = (int64_t)v * n;
  const double s = scale[v];
  double dd = 0.0, xx = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) {
    const float2 d = d32[off + i];
    const double dr = s * (double)d.x, di = s * (double)d.y;
    double2 xv = x[off + i];
    xv.x += dr;
    xv.y += di;
    if (apply) x[off + i] = xv;
    dd += dr * dr + di * di;
    xx += xv.x * xv.x + xv.y * xv.y;
  }
  dd = block_reduce(dd, sh, false);
  xx = block_reduce(xx, sh, false);
  if (threadIdx.x == 0) {
    dn2[v] = dd;
    xn2[v] = xx;
  }
}

__global__ __launch_bounds__(kT) void norm2_kernel(int n, const double2* __restrict__ v,
                                                   double* __restrict__ out) {
  __shared__ double sh[kT / 64];
  const int64_t off = (int64_t)blockIdx.x * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) {
    const double2 a = v[off + i];
    s += a.x * a.x + a.y * a.y;
  }
  s = block_reduce(s, sh, false);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void c128_to_c64_kernel(int64_t count, const double2* __restrict__ in,
                                   float2* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = make_float2((float)in[t].x, (float)in[t].y);
}

__global__ void fill_zero_kernel(int64_t count, uint32_t* __restrict__ p) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0u;
}

__global__ void copy_active_kernel(int n, const uint8_t* __restrict__ active,
                                   const double2* __restrict__ src, double2* __restrict__ dst) {
  const int v = blockIdx.y;
  if (!active[v]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[(int64_t)v * n + i] = src[(int64_t)v * n + i];
}

}  // namespace

bem_status launch_ir_scale(bem_ctx* ctx, int nvec, int n, const void* r, void* r32,
                           double* scale) {
  if (nvec <= 0) return BEM_OK;
  hipLaunchKernelGGL(ir_scale_kernel, dim3(nvec), dim3(kT), 0, ctx->stream, n,
                     (const double2*)r, (float2*)r32, scale);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_ir_update(bem_ctx* ctx, int nvec, int n, const void* d32, const double* scale,
                            const uint8_t* active, void* x, double* dnorm2, double* xnorm2,
                            int apply) {
  if (nvec <= 0) return BEM_OK;
  hipLaunchKernelGGL(ir_update_kernel, dim3(nvec), dim3(kT), 0, ctx->stream, n,
                     (const float2*)d32, scale, active, (double2*)x, dnorm2, xnorm2, apply);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_norm2(bem_ctx* ctx, int nvec, int n, const void* v, double* out) {
  if (nvec <= 0) return BEM_OK;
  hipLaunchKernelGGL(norm2_kernel, dim3(nvec), dim3(kT), 0, ctx->stream, n, (const double2*)v,
                     out);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_c128_to_c64(bem_ctx* ctx, int64_t count, const void* in, void* out) {
  if (count <= 0) return BEM_OK;
  hipLaunchKernelGGL(c128_to_c64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     ctx->stream, count, (const double2*)in, (float2*)out);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

// Zero-fill with a kernel (kept out of hipMemsetAsync so that the sequence can
// be captured into a graph and replayed).
bem_status fill_zero(bem_ctx* ctx, void* p, size_t bytes) {
  const int64_t words = (int64_t)(bytes / 4);
  if (words <= 0) return BEM_OK;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0,
                     ctx->stream, words, (uint32_t*)p);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_copy_active(bem_ctx* ctx, int nvec, int n, const uint8_t* active,
                              const void* src, void* dst) {
  if (nvec <= 0) return BEM_OK;
  hipLaunchKernelGGL(copy_active_kernel, dim3((n + 255) / 256, nvec), dim3(256), 0, ctx->stream,
                     n, active, (const double2*)src, (double2*)dst);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

}  // namespace bem
