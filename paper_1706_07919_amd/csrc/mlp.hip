// Kernels of the frequency surrogate (a learned map k -> surface unknowns of a
// fixed geometry, trained on solutions of the direct method and accepted only
// where the float64 residual of the discrete equation is below tolerance).
// Dense layers y = act(x W + b) with W stored [in][out] row-major; the three
// products of a layer (forward x W, backward x^T dZ and dZ W^T) share one real
// float32 GEMM on MFMA 32x32x2 with transposable operands.
#include "common.h"

namespace bem {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int MB = 64, NB = 64, KB = 16;

// C[M x N] = op(A) op(B) (+ bias[n]) with optional SiLU epilogue.
// op(A)(m,k) = TA ? A[k*lda + m] : A[m*lda + k];  op(B)(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n].
// EPI: 0 store C; 1 store Z = C + bias and Y = silu(Z); 2 store C + bias.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_r32_kernel(int M, int N, int K, const float* A,
                                                       int lda, const float* B, int ldb,
                                                       const float* bias, float* C, int ldc,
                                                       float* Y) {
  __shared__ float As[KB][MB + 4];
  __shared__ float Bs[KB][NB + 4];
  const int m0 = blockIdx.y * MB, n0 = blockIdx.x * NB;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int h = lane >> 5, l32 = lane & 31;
  floatx16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = 0; k0 < K; k0 += KB) {
    // stage op(A) tile [KB][MB] and op(B) tile [KB][NB]: 1024 elements each
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int mm, kk;
      if (TA) { kk = e >> 6; mm = e & 63; } else { mm = e >> 4; kk = e & 15; }
      const int gm = m0 + mm, gk = k0 + kk;
      float va = 0.f;
      if (gm < M && gk < K) va = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[kk][mm] = va;
      int nn, kb;
      if (TB) { nn = e >> 4; kb = e & 15; } else { kb = e >> 6; nn = e & 63; }
      const int gn = n0 + nn, gkb = k0 + kb;
      float vb = 0.f;
      if (gn < N && gkb < K) vb = TB ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn];
      Bs[kb][nn] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KB; k += 2) {
      const float a = As[k + h][wm * 32 + l32];
      const float b = Bs[k + h][wn * 32 + l32];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = n0 + wn * 32 + l32;
  if (col >= N) return;
  const float bv = (EPI != 0 && bias) ? bias[col] : 0.f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = m0 + wm * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
    if (row >= M) continue;
    const float z = acc[v] + bv;
    C[(int64_t)row * ldc + col] = z;
    if (EPI == 1) Y[(int64_t)row * ldc + col] = z / (1.f + __expf(-z));
  }
}

__global__ void silu_bwd_kernel(int64_t count, const float* __restrict__ z,
                                const float* __restrict__ dy, float* __restrict__ dz) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const float zz = z[t];
  const float s = 1.f / (1.f + __expf(-zz));
  dz[t] = dy[t] * s * (1.f + zz * (1.f - s));
}

// db[n] = sum_b dz[b][n]: one thread per column, coalesced over n.
__global__ void colsum_kernel(int B, int N, const float* __restrict__ dz, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dz[(int64_t)b * N + n];
  db[n] = s;
}

__global__ void features_kernel(int B, const double* __restrict__ k, int n_oct, double kscale,
                                float* __restrict__ x) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  for (int l = 0; l < n_oct; ++l) {
    double s, c;
    sincospi(ldexp(1.0, l) * k[b] / kscale, &s, &c);
    x[(int64_t)b * 2 * n_oct + l] = (float)s;
    x[(int64_t)b * 2 * n_oct + n_oct + l] = (float)c;
  }
}

__global__ void mse_grad_kernel(int64_t count, float scale, const float* __restrict__ y,
                                const float* __restrict__ t, float* __restrict__ dy,
                                double* __restrict__ partial) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d * scale;
    acc += (double)d * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Surface unknowns (c128 [B][n]) <-> scaled real targets (float [B][2n]):
// t[b][2j] = Re x_bj / s_j, t[b][2j+1] = Im x_bj / s_j, with s_j the RMS of
// |x_.j| over the batch (computed by rms_kernel).
__global__ void rms_kernel(int B, int n, const double2* __restrict__ x, double* __restrict__ s) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double a = 0.0;
  for (int b = 0; b < B; ++b) {
    const double2 v = x[(int64_t)b * n + j];
    a += v.x * v.x + v.y * v.y;
  }
  a = sqrt(a / B);
  s[j] = a > 0.0 ? a : 1.0;
}

__global__ void pack_kernel(int64_t total, int n, const double2* __restrict__ x,
                            const double* __restrict__ s, float* __restrict__ t) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int j = (int)(e % n);
  const double inv = 1.0 / s[j];
  t[2 * e] = (float)(x[e].x * inv);
  t[2 * e + 1] = (float)(x[e].y * inv);
}

__global__ void unpack_kernel(int64_t total, int n, const float* __restrict__ t,
                              const double* __restrict__ s, double2* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int j = (int)(e % n);
  x[e] = make_double2((double)t[2 * e] * s[j], (double)t[2 * e + 1] * s[j]);
}

template <bool TA, bool TB, int EPI>
void gemm_go(bem_ctx* ctx, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
             const float* bias, float* C, int ldc, float* Y) {
  dim3 grid((N + NB - 1) / NB, (M + MB - 1) / MB);
  hipLaunchKernelGGL((gemm_r32_kernel<TA, TB, EPI>), grid, dim3(256), 0, ctx->stream, M, N, K, A,
                     lda, B, ldb, bias, C, ldc, Y);
}

}  // namespace
}  // namespace bem

using namespace bem;

extern "C" bem_status bem_mlp_features(bem_ctx* ctx, int32_t B, const double* k, int32_t n_oct,
                                       double kscale, float* x) {
  if (!ctx || B <= 0 || !k || n_oct <= 0 || n_oct > 30 || !(kscale > 0.0) || !x)
    return BEM_EINVAL;
  hipLaunchKernelGGL(features_kernel, dim3((B + 255) / 256), dim3(256), 0, ctx->stream, B, k,
                     n_oct, kscale, x);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

extern "C" bem_status bem_mlp_dense_fwd(bem_ctx* ctx, int32_t B, int32_t in, int32_t out,
                                        const float* x, const float* W, const float* b,
                                        int32_t act, float* z, float* y) {
  if (!ctx) return BEM_EINVAL;
  if (B <= 0 || in <= 0 || out <= 0 || !x || !W || !b || !y || (act && !z) || act < 0 || act > 1)
    return fail(ctx, BEM_EINVAL, "bem_mlp_dense_fwd: bad argument");
  const int pi = prof_begin(ctx, "mlp");
  if (act)
    gemm_go<false, false, 1>(ctx, B, out, in, x, in, W, out, b, z, out, y);
  else
    gemm_go<false, false, 2>(ctx, B, out, in, x, in, W, out, b, y, out, nullptr);
  prof_end(ctx, "mlp", pi, 2.0 * B * in * out, 4.0 * ((double)B * in + (double)in * out + B * out));
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

extern "C" bem_status bem_mlp_dense_bwd(bem_ctx* ctx, int32_t B, int32_t in, int32_t out,
                                        const float* x, const float* W, const float* z,
                                        int32_t act, const float* dy, float* dW, float* db,
                                        float* dx, float* dz) {
  if (!ctx) return BEM_EINVAL;
  if (B <= 0 || in <= 0 || out <= 0 || !x || !W || !dy || !dW || !db || (act && (!z || !dz)) ||
      act < 0 || act > 1)
    return fail(ctx, BEM_EINVAL, "bem_mlp_dense_bwd: bad argument");
  const int pi = prof_begin(ctx, "mlp");
  const float* g = dy;
  if (act) {
    const int64_t cnt = (int64_t)B * out;
    hipLaunchKernelGGL(silu_bwd_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       ctx->stream, cnt, z, dy, dz);
    g = dz;
  }
  // dW[in][out] = x^T g ; db = colsum(g) ; dx[B][in] = g W^T
  gemm_go<true, false, 0>(ctx, in, out, B, x, in, g, out, nullptr, dW, out, nullptr);
  hipLaunchKernelGGL(colsum_kernel, dim3((out + 255) / 256), dim3(256), 0, ctx->stream, B, out, g,
                     db);
  if (dx) gemm_go<false, true, 0>(ctx, B, in, out, g, out, W, out, nullptr, dx, in, nullptr);
  prof_end(ctx, "mlp", pi, 2.0 * B * in * out * (dx ? 2.0 : 1.0),
           4.0 * ((double)B * in + (double)in * out + 2.0 * B * out));
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

extern "C" bem_status bem_mlp_mse_grad(bem_ctx* ctx, int64_t count, const float* y,
                                       const float* t, float* dy, double* loss_partial,
                                       int32_t n_partial) {
  if (!ctx || count <= 0 || !y || !t || !dy || !loss_partial || n_partial <= 0)
    return BEM_EINVAL;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(n_partial), dim3(256), 0, ctx->stream, count,
                     (float)(1.0 / (double)count), y, t, dy, loss_partial);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

extern "C" bem_status bem_mlp_adam(bem_ctx* ctx, int64_t n, float* p, const float* g, float* m,
                                   float* v, int32_t step, float lr, float b1, float b2,
                                   float eps) {
  if (!ctx || n <= 0 || !p || !g || !m || !v || step <= 0) return BEM_EINVAL;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, n,
                     p, g, m, v, lr, b1, b2, eps, c1, c2);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

extern "C" bem_status bem_mlp_pack(bem_ctx* ctx, int32_t B, int32_t n, const void* x,
                                   double* scale, int32_t compute_scale, float* t) {
  if (!ctx || B <= 0 || n <= 0 || !x || !scale || !t) return BEM_EINVAL;
  if (compute_scale)
    hipLaunchKernelGGL(rms_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, B, n,
                       (const double2*)x, scale);
  const int64_t total = (int64_t)B * n;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, ctx->stream,
                     total, n, (const double2*)x, scale, t);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

extern "C" bem_status bem_mlp_unpack(bem_ctx* ctx, int32_t B, int32_t n, const float* t,
                                     const double* scale, void* x) {
  if (!ctx || B <= 0 || n <= 0 || !t || !scale || !x) return BEM_EINVAL;
  const int64_t total = (int64_t)B * n;
  hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     ctx->stream, total, n, t, scale, (double2*)x);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}
