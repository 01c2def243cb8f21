// Float64 operator of the discrete non-singular boundary integral equation
// (Eq. BRIEF with the f, g of Appendix A; the S_inf integrals of Appendix B
// leave 4 pi on the diagonal of M_phi).  For a collocation node i and a node
// j != i, with d = x_j - x_i, r = |d|, E = e^{ikr}:
//   G = E/r,  H = E (ikr - 1)(d.n_j)/r^3,  s = k n_i.d,
//   g = cos s, f = sin(s)/k, g' = -k sin(s) (n_i.n_j), f' = cos(s) (n_i.n_j)
//   (M_phi)_ij = -w_j H,  (M_psi)_ij = w_j G,
//   (M_phi)_ii = 4 pi - sum_j w_j (g' G - g H),  (M_psi)_ii = -sum_j w_j (f' G - f H).
// One workgroup owns one (wavenumber, row) pair and sweeps j with coalesced
// loads of the node arrays and coalesced stores of the row-major matrix row.
#include "common.h"

namespace bem {
namespace {

constexpr int kThreads = 256;
constexpr int kRhsChunk = 4;
constexpr double kFourPi = 12.566370614359172953850573533118;

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-wide sum of `cnt` doubles held per thread; result valid in thread 0.
template <int CNT>
__device__ inline void block_sum(double (&v)[CNT]) {
  __shared__ double red[kThreads / 64][CNT];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < CNT; ++c) v[c] = wave_sum(v[c]);
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < CNT; ++c) red[wid][c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
      double s = 0.0;
      for (int q = 0; q < kThreads / 64; ++q) s += red[q][c];
      v[c] = s;
    }
  }
}

struct PairGH {
  double2 G, H;
};

// G, H of the pair (i -> j) and the in-plane quantities used by f, g.
__device__ inline PairGH pair_gh(double k, double dx, double dy, double dz, double njx,
                                 double njy, double njz, double& r) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  r = sqrt(r2);
  const double rinv = 1.0 / r;
  double sn, cs;
  sincos(k * r, &sn, &cs);
  PairGH o;
  o.G = make_double2(cs * rinv, sn * rinv);
  const double q = (dx * njx + dy * njy + dz * njz) * (rinv * rinv * rinv);
  const double kr = k * r;
  // E (ikr - 1) q
  o.H = make_double2(q * (-cs - kr * sn), q * (kr * cs - sn));
  return o;
}

template <bool OUT128, bool WRITE_A>
__global__ __launch_bounds__(kThreads) void assemble_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const uint8_t* __restrict__ bc, const double* __restrict__ kv,
    int n_rhs, int rhs0, const double2* __restrict__ y, void* __restrict__ A, int64_t ld,
    int64_t a_stride, double2* __restrict__ b, double2* __restrict__ diag64) {
  const int i = blockIdx.x;
  const int kq = blockIdx.y;
  const double k = kv[kq];
  const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
  const double nix = nrm[3 * i], niy = nrm[3 * i + 1], niz = nrm[3 * i + 2];
  const int nr = min(kRhsChunk, n_rhs - rhs0);
  const double2* yk = y + (int64_t)kq * n_rhs * n;

  // acc: Dphi(re,im), Dpsi(re,im), then b partial sums (re,im) per rhs
  double acc[4 + 2 * kRhsChunk];
#pragma unroll
  for (int c = 0; c < 4 + 2 * kRhsChunk; ++c) acc[c] = 0.0;

  float2* A32 = reinterpret_cast<float2*>(A) + (int64_t)kq * a_stride + (int64_t)i * ld;
  double2* A64 = reinterpret_cast<double2*>(A) + (int64_t)kq * a_stride + (int64_t)i * ld;
  const double kinv = 1.0 / k;

  for (int j = threadIdx.x; j < n; j += kThreads) {
    if (j == i) continue;
    const double dx = x[3 * j] - xi, dy = x[3 * j + 1] - yi, dz = x[3 * j + 2] - zi;
    const double njx = nrm[3 * j], njy = nrm[3 * j + 1], njz = nrm[3 * j + 2];
    double r;
    const PairGH p = pair_gh(k, dx, dy, dz, njx, njy, njz, r);
    double ss, cs;
    sincos(k * (nix * dx + niy * dy + niz * dz), &ss, &cs);
    const double nn = nix * njx + niy * njy + niz * njz;
    const double g = cs, f = ss * kinv, gp = -k * ss * nn, fp = cs * nn;
    const double wj = w[j];
    acc[0] += wj * (gp * p.G.x - g * p.H.x);
    acc[1] += wj * (gp * p.G.y - g * p.H.y);
    acc[2] += wj * (fp * p.G.x - f * p.H.x);
    acc[3] += wj * (fp * p.G.y - f * p.H.y);
    const bool hard = bc[j] == BEM_BC_HARD;
    const double2 mphi = make_double2(-wj * p.H.x, -wj * p.H.y);
    const double2 mpsi = make_double2(wj * p.G.x, wj * p.G.y);
    const double2 a = hard ? mphi : mpsi;
    const double2 bb = hard ? mpsi : mphi;
    if (WRITE_A && A) {
      if (OUT128)
        A64[j] = a;
      else
        A32[j] = make_float2((float)a.x, (float)a.y);
    }
#pragma unroll
    for (int q = 0; q < kRhsChunk; ++q) {
      if (q < nr) {
        const double2 yy = yk[(int64_t)(rhs0 + q) * n + j];
        acc[4 + 2 * q] += bb.x * yy.x - bb.y * yy.y;
        acc[5 + 2 * q] += bb.x * yy.y + bb.y * yy.x;
      }
    }
  }
  block_sum(acc);
  if (threadIdx.x == 0) {
    const double2 mphi = make_double2(kFourPi - acc[0], -acc[1]);
    const double2 mpsi = make_double2(-acc[2], -acc[3]);
    const bool hard = bc[i] == BEM_BC_HARD;
    const double2 a = hard ? mphi : mpsi;
    const double2 bb = hard ? mpsi : mphi;
    if (WRITE_A) {
      if (A) {
        if (OUT128)
          A64[i] = a;
        else
          A32[i] = make_float2((float)a.x, (float)a.y);
      }
      if (diag64) {
        diag64[((int64_t)kq * n + i) * 2] = mphi;
        diag64[((int64_t)kq * n + i) * 2 + 1] = mpsi;
      }
    }
    for (int q = 0; q < nr; ++q) {
      const double2 yy = yk[(int64_t)(rhs0 + q) * n + i];
      const double2 t = cmul(bb, yy);
      b[((int64_t)kq * n_rhs + rhs0 + q) * n + i] =
          make_double2(-(acc[4 + 2 * q] + t.x), -(acc[5 + 2 * q] + t.y));
    }
  }
}

// r = -(M_phi phi + M_psi psi) with (phi, psi) from the unknowns x and data y.
__global__ __launch_bounds__(kThreads) void residual_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const uint8_t* __restrict__ bc, const double* __restrict__ kv,
    int n_rhs, int rhs0, const double2* __restrict__ y, const double2* __restrict__ xs,
    const double2* __restrict__ diag64, double2* __restrict__ r_out) {
  const int i = blockIdx.x;
  const int kq = blockIdx.y;
  const double k = kv[kq];
  const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
  const int nr = min(kRhsChunk, n_rhs - rhs0);
  const int64_t base = (int64_t)kq * n_rhs * n;
  double acc[2 * kRhsChunk];
#pragma unroll
  for (int c = 0; c < 2 * kRhsChunk; ++c) acc[c] = 0.0;
  for (int j = threadIdx.x; j < n; j += kThreads) {
    if (j == i) continue;
    const double dx = x[3 * j] - xi, dy = x[3 * j + 1] - yi, dz = x[3 * j + 2] - zi;
    double r;
    const PairGH p = pair_gh(k, dx, dy, dz, nrm[3 * j], nrm[3 * j + 1], nrm[3 * j + 2], r);
    const double wj = w[j];
    const bool hard = bc[j] == BEM_BC_HARD;
#pragma unroll
    for (int q = 0; q < kRhsChunk; ++q) {
      if (q < nr) {
        const int64_t o = base + (int64_t)(rhs0 + q) * n + j;
        const double2 u = xs[o], v = y[o];
        const double2 phi = hard ? u : v, psi = hard ? v : u;
        // -w H phi + w G psi
        acc[2 * q] += wj * ((p.G.x * psi.x - p.G.y * psi.y) - (p.H.x * phi.x - p.H.y * phi.y));
        acc[2 * q + 1] += wj * ((p.G.x * psi.y + p.G.y * psi.x) - (p.H.x * phi.y + p.H.y * phi.x));
      }
    }
  }
  block_sum(acc);
  if (threadIdx.x == 0) {
    const double2 dphi = diag64[((int64_t)kq * n + i) * 2];
    const double2 dpsi = diag64[((int64_t)kq * n + i) * 2 + 1];
    const bool hard = bc[i] == BEM_BC_HARD;
    for (int q = 0; q < nr; ++q) {
      const int64_t o = base + (int64_t)(rhs0 + q) * n + i;
      const double2 u = xs[o], v = y[o];
      const double2 phi = hard ? u : v, psi = hard ? v : u;
      const double2 t1 = cmul(dphi, phi), t2 = cmul(dpsi, psi);
      r_out[o] = make_double2(-(acc[2 * q] + t1.x + t2.x), -(acc[2 * q + 1] + t1.y + t2.y));
    }
  }
}

__global__ void incident_kernel(int n, const double* __restrict__ x, const double* __restrict__ nrm,
                                const uint8_t* __restrict__ bc, const double* __restrict__ kv,
                                double dx, double dy, double dz, double2* __restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int kq = blockIdx.y;
  if (j >= n) return;
  const double k = kv[kq];
  const double ph = k * (x[3 * j] * dx + x[3 * j + 1] * dy + x[3 * j + 2] * dz);
  double sn, cs;
  sincos(ph, &sn, &cs);
  double2 out;
  if (bc[j] == BEM_BC_HARD) {
    const double kd = k * (nrm[3 * j] * dx + nrm[3 * j + 1] * dy + nrm[3 * j + 2] * dz);
    out = make_double2(kd * sn, -kd * cs);  // -(i kd)(cs + i sn)
  } else {
    out = make_double2(-cs, -sn);
  }
  y[(int64_t)kq * n + j] = out;
}

__global__ void split_kernel(int n, int64_t total, const uint8_t* __restrict__ bc,
                             const double2* __restrict__ xs, const double2* __restrict__ y,
                             double2* __restrict__ phi, double2* __restrict__ psi) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const bool hard = bc[t % n] == BEM_BC_HARD;
  const double2 u = xs[t], v = y[t];
  phi[t] = hard ? u : v;
  psi[t] = hard ? v : u;
}

}  // namespace

bem_status launch_incident(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k,
                           double dx, double dy, double dz, void* y) {
  dim3 grid((s->n + 255) / 256, n_k);
  hipLaunchKernelGGL(incident_kernel, grid, dim3(256), 0, ctx->stream, s->n, s->x, s->nrm, s->bc,
                     k, dx, dy, dz, reinterpret_cast<double2*>(y));
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_assemble(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k,
                           int n_rhs, const void* y, bem_prec prec, void* A, int64_t ld,
                           int64_t a_stride, void* b, void* diag64) {
  for (int k0 = 0; k0 < n_k; k0 += 65535) {
    const int nk = std::min(65535, n_k - k0);
    dim3 grid(s->n, nk);
    for (int r0 = 0; r0 < std::max(n_rhs, 1); r0 += kRhsChunk) {
      const bool first = r0 == 0;
      const int pi = prof_begin(ctx, "assemble");
      const double2* yk = reinterpret_cast<const double2*>(y) + (int64_t)k0 * n_rhs * s->n;
      double2* bk = reinterpret_cast<double2*>(b) + (int64_t)k0 * n_rhs * s->n;
      double2* dk = diag64 ? reinterpret_cast<double2*>(diag64) + (int64_t)k0 * s->n * 2 : nullptr;
      const size_t esz = prec == BEM_C128 ? 16 : 8;
      void* Ak = A ? reinterpret_cast<char*>(A) + (int64_t)k0 * a_stride * esz : nullptr;
      if (prec == BEM_C128) {
        if (first)
          hipLaunchKernelGGL((assemble_kernel<true, true>), grid, dim3(kThreads), 0, ctx->stream,
                             s->n, s->x, s->nrm, s->w, s->bc, k + k0, n_rhs, r0, yk, Ak, ld,
                             a_stride, bk, dk);
        else
          hipLaunchKernelGGL((assemble_kernel<true, false>), grid, dim3(kThreads), 0, ctx->stream,
                             s->n, s->x, s->nrm, s->w, s->bc, k + k0, n_rhs, r0, yk, Ak, ld,
                             a_stride, bk, dk);
      } else {
        if (first)
          hipLaunchKernelGGL((assemble_kernel<false, true>), grid, dim3(kThreads), 0, ctx->stream,
                             s->n, s->x, s->nrm, s->w, s->bc, k + k0, n_rhs, r0, yk, Ak, ld,
                             a_stride, bk, dk);
        else
          hipLaunchKernelGGL((assemble_kernel<false, false>), grid, dim3(kThreads), 0,
                             ctx->stream, s->n, s->x, s->nrm, s->w, s->bc, k + k0, n_rhs, r0, yk,
                             Ak, ld, a_stride, bk, dk);
      }
      // node pairs evaluated; bytes: matrix written (first pass) + b written
      const double pairs = (double)s->n * s->n * nk;
      prof_end(ctx, "assemble", pi, pairs,
               (first ? (double)(prec == BEM_C128 ? 16 : 8) * s->n * s->n * nk : 0.0) +
                   16.0 * s->n * std::min(kRhsChunk, std::max(n_rhs - r0, 0)) * nk);
      BEM_CHECK_LAUNCH(ctx);
    }
  }
  return BEM_OK;
}

bem_status launch_residual(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k,
                           int n_rhs, const void* y, const void* x, const void* diag64, void* r) {
  for (int k0 = 0; k0 < n_k; k0 += 65535) {
    const int nk = std::min(65535, n_k - k0);
    dim3 grid(s->n, nk);
    const int64_t off = (int64_t)k0 * n_rhs * s->n;
    for (int r0 = 0; r0 < n_rhs; r0 += kRhsChunk) {
      const int pi = prof_begin(ctx, "residual");
      hipLaunchKernelGGL(residual_kernel, grid, dim3(kThreads), 0, ctx->stream, s->n, s->x,
                         s->nrm, s->w, s->bc, k + k0, n_rhs, r0,
                         reinterpret_cast<const double2*>(y) + off,
                         reinterpret_cast<const double2*>(x) + off,
                         reinterpret_cast<const double2*>(diag64) + (int64_t)k0 * s->n * 2,
                         reinterpret_cast<double2*>(r) + off);
      prof_end(ctx, "residual", pi, (double)s->n * s->n * nk,
               48.0 * s->n * std::min(kRhsChunk, n_rhs - r0) * nk);
      BEM_CHECK_LAUNCH(ctx);
    }
  }
  return BEM_OK;
}

bem_status launch_split(bem_ctx* ctx, const bem_surface* s, int n_k, int n_rhs, const void* x,
                        const void* y, void* phi, void* psi) {
  const int64_t total = (int64_t)n_k * n_rhs * s->n;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, s->n, total,
                     s->bc, reinterpret_cast<const double2*>(x),
                     reinterpret_cast<const double2*>(y), reinterpret_cast<double2*>(phi),
                     reinterpret_cast<double2*>(psi));
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

}  // namespace bem
