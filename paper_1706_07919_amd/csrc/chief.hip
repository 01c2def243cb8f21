// Interior-point conditions against fictitious resonances.  At wavenumbers
// where a body's interior resonates, the surface equation (Eq. BRIEF) is
// nearly singular and its solution carries a spurious interior mode; Sec. IV A
// side-steps those wavenumbers.  Green's second identity on the exterior
// domain, with normals out of the body, gives for the radiating scattered
// field
//   0 = int_S (P dG/dn - G dP/dn) dS      (x_c strictly inside a body),
// which, in the nodal quadrature of the surface equation, is one more row per
// interior point:  sum_j w_j (phi_j H_cj - psi_j G_cj) = 0 with d = x_j - x_c,
// G = e^{ikr}/r, H = e^{ikr}(ikr - 1)(d.n_j)/r^3.  Split by the boundary
// conditions (hard node: unknown phi, soft node: unknown psi), the interior
// rows are C x = d.  The surface rows A x = b and the interior rows are solved
// together in the least-squares sense through the normal equations
//   (A^H A + C^H C) x = A^H b + C^H d
// in float64.  Both products come from one complex GEMM each on the
// augmented rows [A | b] and [C | d]: with the row-major buffers read as
// column-major matrices X (rows of [A | b] as columns), X X^H is
// [A | b]^H [A | b] read back row-major, whose leading block is A^H A and
// whose last columns are A^H b.
#include <rocblas/rocblas.h>

#include "common.h"

namespace bem {
namespace {

constexpr int kCT = 256;
constexpr int kCRhs = 4;   // right-hand sides per pass of the interior-row kernel

__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kCT / 64; ++w) s += sh[w];
  return s;
}

// A_aug[kq][i][n + q] = b[kq][q][i]
__global__ void aug_b_kernel(int n, int n_k, int n_rhs, const double2* __restrict__ b,
                             double2* __restrict__ A, int64_t ld, int64_t stride) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_k * n_rhs * n) return;
  const int i = (int)(t % n);
  const int64_t v = t / n;
  const int q = (int)(v % n_rhs), kq = (int)(v / n_rhs);
  A[kq * stride + (int64_t)i * ld + n + q] = b[t];
}

// Interior rows of wavenumber blockIdx.y, point blockIdx.x:
//   C[kq][c][j] = w_j H_cj (hard j) or -w_j G_cj (soft j),
//   C[kq][c][n + q] = d_q = -sum_j (known coefficient) y_q[j]
__global__ __launch_bounds__(kCT) void interior_rows_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const uint8_t* __restrict__ bc, const double* __restrict__ kv,
    int n_rhs, const double2* __restrict__ y, const double* __restrict__ xc,
    double2* __restrict__ C, int64_t ld, int64_t stride, int n_c) {
  __shared__ double sh[kCT / 64];
  const int c = blockIdx.x, kq = blockIdx.y;
  const double k = kv[kq];
  const double cx = xc[3 * c], cy = xc[3 * c + 1], cz = xc[3 * c + 2];
  double2* row = C + kq * stride + (int64_t)c * ld;
  for (int r0 = 0; r0 < n_rhs; r0 += kCRhs) {
    double dr[kCRhs], di[kCRhs];
#pragma unroll
    for (int r = 0; r < kCRhs; ++r) dr[r] = di[r] = 0.0;
    for (int j = threadIdx.x; j < n; j += kCT) {
      const double d0 = x[3 * j] - cx, d1 = x[3 * j + 1] - cy, d2 = x[3 * j + 2] - cz;
      const double r = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
      double s, co;
      sincos(k * r, &s, &co);
      const double ri = 1.0 / r;
      const double wj = w[j];
      const double dn = ((d0 * nrm[3 * j] + d1 * nrm[3 * j + 1]) + d2 * nrm[3 * j + 2]) * ri * ri * ri;
      const double kr = k * r;
      // w G and w H
      const double gr = wj * co * ri, gi = wj * s * ri;
      const double hr = wj * (-co - kr * s) * dn, hi = wj * (-s + kr * co) * dn;
      const bool hard = bc[j] == BEM_BC_HARD;
      // unknown coefficient and known coefficient of node j
      const double ur = hard ? hr : -gr, ui = hard ? hi : -gi;
      const double kr_ = hard ? -gr : hr, ki_ = hard ? -gi : hi;
      if (r0 == 0) row[j] = make_double2(ur, ui);
#pragma unroll
      for (int q = 0; q < kCRhs; ++q)
        if (r0 + q < n_rhs) {
          const double2 yv = y[((int64_t)kq * n_rhs + r0 + q) * n + j];
          dr[q] -= kr_ * yv.x - ki_ * yv.y;
          di[q] -= kr_ * yv.y + ki_ * yv.x;
        }
    }
#pragma unroll
    for (int q = 0; q < kCRhs; ++q) {
      if (r0 + q >= n_rhs) break;   // uniform
      const double sr = block_sum(dr[q], sh), si = block_sum(di[q], sh);
      if (threadIdx.x == 0) row[n + r0 + q] = make_double2(sr, si);
    }
  }
}

// r[kq][q][i] = M[kq][i][n + q]
__global__ void extract_rhs_kernel(int n, int n_k, int n_rhs, const double2* __restrict__ M,
                                   int64_t ld, int64_t stride, double2* __restrict__ r) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_k * n_rhs * n) return;
  const int i = (int)(t % n);
  const int64_t v = t / n;
  const int q = (int)(v % n_rhs), kq = (int)(v / n_rhs);
  r[t] = M[kq * stride + (int64_t)i * ld + n + q];
}

// rs[kq][q][row] = |R_row x_q - R_row[n + q]|^2 for the rows of R (the
// augmented surface rows or interior rows of each wavenumber)
__global__ __launch_bounds__(kCT) void aug_resid_kernel(int n, int n_rhs, const double2* __restrict__ R,
                                                        int64_t ld, int64_t stride, int rows,
                                                        const double2* __restrict__ xv,
                                                        double* __restrict__ rs, int rs_rows,
                                                        int rs_off) {
  __shared__ double sh[kCT / 64];
  const int row = blockIdx.x, vq = blockIdx.y, kq = vq / n_rhs, q = vq % n_rhs;
  const double2* Rr = R + kq * stride + (int64_t)row * ld;
  const double2* x = xv + (int64_t)vq * n;
  double sr = 0.0, si = 0.0;
  for (int j = threadIdx.x; j < n; j += kCT) {
    const double2 a = Rr[j], v = x[j];
    sr += a.x * v.x - a.y * v.y;
    si += a.x * v.y + a.y * v.x;
  }
  sr = block_sum(sr, sh);
  si = block_sum(si, sh);
  if (threadIdx.x == 0) {
    const double2 bb = Rr[n + q];
    const double er = sr - bb.x, ei = si - bb.y;
    rs[(int64_t)vq * rs_rows + rs_off + row] = er * er + ei * ei;
    (void)rows;
  }
}

rocblas_handle handle_of(bem_ctx* ctx, bem_status* st) {
  if (!ctx->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
      *st = fail(ctx, BEM_EHIP, "rocblas_create_handle failed");
      return nullptr;
    }
    ctx->blas = h;
  }
  rocblas_handle h = (rocblas_handle)ctx->blas;
  if (rocblas_set_stream(h, ctx->stream) != rocblas_status_success) {
    *st = fail(ctx, BEM_EHIP, "rocblas_set_stream failed");
    return nullptr;
  }
  *st = BEM_OK;
  return h;
}

}  // namespace

bem_status launch_aug_b(bem_ctx* ctx, int n, int n_k, int n_rhs, const void* b, void* A,
                        int64_t ld, int64_t stride) {
  const int64_t tot = (int64_t)n_k * n_rhs * n;
  hipLaunchKernelGGL(aug_b_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream,
                     n, n_k, n_rhs, (const double2*)b, (double2*)A, ld, stride);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_interior_rows(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k,
                                int n_rhs, const void* y, int n_c, const double* xc, void* C,
                                int64_t ld, int64_t stride) {
  hipLaunchKernelGGL(interior_rows_kernel, dim3(n_c, n_k), dim3(kCT), 0, ctx->stream, s->n, s->x,
                     s->nrm, s->w, s->bc, k, n_rhs, (const double2*)y, xc, (double2*)C, ld, stride,
                     n_c);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

// M[kq] = X X^H (+ M[kq] when accumulate) for the column-major X of m_cols
// columns of length len (ld), i.e. the row-major R[kq] (m_cols rows of len
// entries): M = R^H R, len x len, read row-major.
bem_status gram_c128(bem_ctx* ctx, int len, int m_cols, const void* R, int64_t ld,
                     int64_t r_stride, void* M, int64_t ldm, int64_t m_stride, int batch,
                     bool accumulate) {
  bem_status st;
  rocblas_handle h = handle_of(ctx, &st);
  if (!h) return st;
  const rocblas_double_complex one = {1.0, 0.0};
  const rocblas_double_complex beta = {accumulate ? 1.0 : 0.0, 0.0};
  const rocblas_status rs = rocblas_zgemm_strided_batched(
      h, rocblas_operation_none, rocblas_operation_conjugate_transpose, len, len, m_cols, &one,
      (const rocblas_double_complex*)R, (rocblas_int)ld, r_stride, (const rocblas_double_complex*)R,
      (rocblas_int)ld, r_stride, &beta, (rocblas_double_complex*)M, (rocblas_int)ldm, m_stride,
      batch);
  if (rs != rocblas_status_success)
    return fail(ctx, BEM_EHIP, "rocblas_zgemm_strided_batched failed (%d)", (int)rs);
  return BEM_OK;
}

bem_status launch_extract_rhs(bem_ctx* ctx, int n, int n_k, int n_rhs, const void* M, int64_t ld,
                              int64_t stride, void* r) {
  const int64_t tot = (int64_t)n_k * n_rhs * n;
  hipLaunchKernelGGL(extract_rhs_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, n, n_k, n_rhs, (const double2*)M, ld, stride, (double2*)r);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_aug_resid(bem_ctx* ctx, int n, int n_k, int n_rhs, const void* R, int64_t ld,
                            int64_t stride, int rows, const void* x, double* rs, int rs_rows,
                            int rs_off) {
  if (rows <= 0) return BEM_OK;
  hipLaunchKernelGGL(aug_resid_kernel, dim3(rows, n_k * n_rhs), dim3(kCT), 0, ctx->stream, n,
                     n_rhs, (const double2*)R, ld, stride, rows, (const double2*)x, rs, rs_rows,
                     rs_off);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

void blas_destroy(bem_ctx* ctx) {
  if (ctx->blas) (void)rocblas_destroy_handle((rocblas_handle)ctx->blas);
  ctx->blas = nullptr;
}

}  // namespace bem
