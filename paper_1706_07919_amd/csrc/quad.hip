// Quadratic-element discretisation of the non-singular boundary integral
// equation (Sec. III: quadratic interpolants within each element, integrals
// free of singularities evaluated by standard Gauss quadrature; Sec. IV A:
// 500 six-node elements and 1002 nodes on the sphere), collocated at the
// nodes:
//   4 pi phi_i + int [psi - phi_i g' - psi_i f'] G dS = int [phi - phi_i g - psi_i f] H dS
// with phi, psi and the geometry interpolated by the six shape functions of
// each element (nodes v0 v1 v2 m01 m12 m20; L_a (2 L_a - 1) at the vertices,
// 4 L_a L_b at the midpoints), f, g of Appendix A about x_i with its normal,
// and H = dG/dn with the element's normal at the quadrature point.  The
// integrands are regular at x_i, so every element takes the same rule: the
// symmetric 7-point rule of degree 5 on triangles (Radon's).  Collecting terms:
//   (M_psi)_ij =  sum_{e,q : node a of e is j} N_a(q) wJ_q G_q
//   (M_phi)_ij = -sum ...                      N_a(q) wJ_q H_q
//   (M_phi)_ii += 4 pi - sum_{all q} (g'_q G_q - g_q H_q) wJ_q
//   (M_psi)_ii += -sum_{all q} (f'_q G_q - f_q H_q) wJ_q
// All in float64.  Column j of A is column j of M_phi (hard node) or M_psi
// (soft node), b = -B y.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace bem {

namespace {

constexpr int kQ = 7;          // points of the triangle rule
constexpr int kMaxInc = 12;    // element incidences kept per node
constexpr int kQT = 256;       // threads of the row kernels
constexpr int kRhsChunk = 4;   // right-hand sides per assembly launch
constexpr double kFourPiQ = 12.566370614359172953850573533118;

// The rule's points and weights (weights summing to the reference area 1/2)
// and the six shape functions with their derivatives at the points.
struct QuadRule {
  double N[kQ][6], dxi[kQ][6], deta[kQ][6], w[kQ];
};

QuadRule make_rule() {
  QuadRule R;
  const double s15 = std::sqrt(15.0);
  double bx[kQ], by[kQ], bz[kQ];
  bx[0] = by[0] = bz[0] = 1.0 / 3.0;
  R.w[0] = 0.5 * (9.0 / 40.0);
  const double as[2] = {(6.0 - s15) / 21.0, (6.0 + s15) / 21.0};
  const double ws[2] = {(155.0 - s15) / 1200.0, (155.0 + s15) / 1200.0};
  for (int g = 0; g < 2; ++g) {
    const double a = as[g], c = 1.0 - 2.0 * a;
    const double pts[3][3] = {{c, a, a}, {a, c, a}, {a, a, c}};
    for (int t = 0; t < 3; ++t) {
      const int q = 1 + 3 * g + t;
      bx[q] = pts[t][0];
      by[q] = pts[t][1];
      bz[q] = pts[t][2];
      R.w[q] = 0.5 * ws[g];
    }
  }
  for (int q = 0; q < kQ; ++q) {
    // barycentric (L0, L1, L2) with L1 = xi, L2 = eta
    const double L0 = bx[q], L1 = by[q], L2 = bz[q];
    const double N[6] = {L0 * (2 * L0 - 1), L1 * (2 * L1 - 1), L2 * (2 * L2 - 1),
                         4 * L0 * L1, 4 * L1 * L2, 4 * L2 * L0};
    // d/dxi: dL0 = -1, dL1 = +1; d/deta: dL0 = -1, dL2 = +1
    const double dx[6] = {-(4 * L0 - 1), 4 * L1 - 1, 0.0, 4 * (L0 - L1), 4 * L2, -4 * L2};
    const double de[6] = {-(4 * L0 - 1), 0.0, 4 * L2 - 1, -4 * L1, 4 * L1, 4 * (L0 - L2)};
    for (int a = 0; a < 6; ++a) {
      R.N[q][a] = N[a];
      R.dxi[q][a] = dx[a];
      R.deta[q][a] = de[a];
    }
  }
  return R;
}

// quadrature points of every element: [F*7][8] = x, y, z, nx, ny, nz (unit
// normal of the element surface), wJ (weight times area Jacobian), 0
__global__ void quad_points_kernel(int F, const double* __restrict__ x,
                                   const int32_t* __restrict__ elem, QuadRule R,
                                   double* __restrict__ qp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= F * kQ) return;
  const int e = t / kQ, q = t % kQ;
  double p[3] = {0, 0, 0}, t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
  for (int a = 0; a < 6; ++a) {
    const int v = elem[6 * e + a];
    for (int d = 0; d < 3; ++d) {
      const double c = x[3 * v + d];
      p[d] += R.N[q][a] * c;
      t1[d] += R.dxi[q][a] * c;
      t2[d] += R.deta[q][a] * c;
    }
  }
  const double c0 = t1[1] * t2[2] - t1[2] * t2[1];
  const double c1 = t1[2] * t2[0] - t1[0] * t2[2];
  const double c2 = t1[0] * t2[1] - t1[1] * t2[0];
  const double J = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  double* o = qp + 8 * (int64_t)t;
  o[0] = p[0];
  o[1] = p[1];
  o[2] = p[2];
  o[3] = c0 / J;
  o[4] = c1 / J;
  o[5] = c2 / J;
  o[6] = R.w[q] * J;
  o[7] = 0.0;
}

// inc[j][c] = 6 e + a for the c-th (element e, local node a) holding node j,
// in element order; -1 past the last; *overflow set when a node has more
// than kMaxInc incidences or an element refers to a node outside [0, n)
__global__ void quad_incidence_kernel(int n, int F, const int32_t* __restrict__ elem,
                                      int32_t* __restrict__ inc, int32_t* __restrict__ overflow) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int c = 0;
  for (int t = 0; t < 6 * F; ++t) {
    const int v = elem[t];
    if (j == 0 && (v < 0 || v >= n)) overflow[0] = 1;
    if (v == j) {
      if (c < kMaxInc) inc[(int64_t)j * kMaxInc + c] = t;
      ++c;
    }
  }
  if (c > kMaxInc) overflow[0] = 1;
  for (int s = c; s < kMaxInc; ++s) inc[(int64_t)j * kMaxInc + s] = -1;
}

__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kQT / 64; ++w) s += sh[w];
  return s;
}

// G = e^{ikr}/r and H = dG/dn_q = e^{ikr}(ikr - 1)(d.n_q)/r^3, d = x_q - x_i
__device__ inline void green(double k, double dx, double dy, double dz, double nx, double ny,
                             double nz, double2& G, double2& H) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double s, c;
  sincos(k * r, &s, &c);
  const double ri = 1.0 / r;
  G = make_double2(c * ri, s * ri);
  const double dn = (dx * nx + dy * ny + dz * nz) * ri * ri * ri;
  const double kr = k * r;
  H = make_double2((-c - kr * s) * dn, (-s + kr * c) * dn);
}

// One workgroup per (row i, wavenumber): the row's diagonal integrals over
// every quadrature point, then each column's entries gathered from the
// elements that hold its node (deterministic order, no atomics).
template <typename OUT>
__global__ __launch_bounds__(kQT) void quad_assemble_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const uint8_t* __restrict__ bc, int npts, const double* __restrict__ qp,
    const int32_t* __restrict__ inc, QuadRule R, const double* __restrict__ kv, int n_rhs, int r0,
    int nr, const double2* __restrict__ y, OUT* __restrict__ A, int64_t ld, int64_t a_stride,
    double2* __restrict__ b, double2* __restrict__ diag64) {
  __shared__ double sh[kQT / 64];
  const int i = blockIdx.x, kq = blockIdx.y;
  const double k = kv[kq];
  const double xi0 = x[3 * i], xi1 = x[3 * i + 1], xi2 = x[3 * i + 2];
  const double ni0 = nrm[3 * i], ni1 = nrm[3 * i + 1], ni2 = nrm[3 * i + 2];
  double d1r = 0, d1i = 0, d2r = 0, d2i = 0;
  for (int p = threadIdx.x; p < npts; p += kQT) {
    const double* o = qp + 8 * (int64_t)p;
    const double dx = o[0] - xi0, dy = o[1] - xi1, dz = o[2] - xi2;
    double2 G, H;
    green(k, dx, dy, dz, o[3], o[4], o[5], G, H);
    double ss, cs;
    sincos(k * (ni0 * dx + ni1 * dy + ni2 * dz), &ss, &cs);
    const double nn = ni0 * o[3] + ni1 * o[4] + ni2 * o[5];
    const double g = cs, f = ss / k, gp = -k * ss * nn, fp = cs * nn, wJ = o[6];
    d1r += (gp * G.x - g * H.x) * wJ;
    d1i += (gp * G.y - g * H.y) * wJ;
    d2r += (fp * G.x - f * H.x) * wJ;
    d2i += (fp * G.y - f * H.y) * wJ;
  }
  d1r = block_sum(d1r, sh);
  d1i = block_sum(d1i, sh);
  d2r = block_sum(d2r, sh);
  d2i = block_sum(d2i, sh);
  double bac[kRhsChunk][2];
#pragma unroll
  for (int r = 0; r < kRhsChunk; ++r) bac[r][0] = bac[r][1] = 0.0;
  for (int j = threadIdx.x; j < n; j += kQT) {
    double mpr = 0, mpi = 0, mhr = 0, mhi = 0;   // M_psi and M_phi entries
    for (int c = 0; c < kMaxInc; ++c) {
      const int v = inc[(int64_t)j * kMaxInc + c];
      if (v < 0) break;
      const int e = v / 6, a = v % 6;
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const double* o = qp + 8 * ((int64_t)e * kQ + q);
        double2 G, H;
        green(k, o[0] - xi0, o[1] - xi1, o[2] - xi2, o[3], o[4], o[5], G, H);
        const double wn = R.N[q][a] * o[6];
        mpr += wn * G.x;
        mpi += wn * G.y;
        mhr -= wn * H.x;
        mhi -= wn * H.y;
      }
    }
    if (j == i) {
      mhr += kFourPiQ - d1r;
      mhi += -d1i;
      mpr += -d2r;
      mpi += -d2i;
      if (r0 == 0 && diag64) {
        diag64[2 * ((int64_t)kq * n + i)] = make_double2(mhr, mhi);
        diag64[2 * ((int64_t)kq * n + i) + 1] = make_double2(mpr, mpi);
      }
    }
    const bool hard = bc[j] == BEM_BC_HARD;
    const double ar = hard ? mhr : mpr, ai = hard ? mhi : mpi;
    const double br = hard ? mpr : mhr, bi = hard ? mpi : mhi;
    if (r0 == 0 && A) {
      OUT* Ap = A + kq * a_stride + (int64_t)i * ld + j;
      Ap->x = ar;
      Ap->y = ai;
    }
#pragma unroll
    for (int r = 0; r < kRhsChunk; ++r)
      if (r < nr) {
        const double2 yv = y[((int64_t)kq * n_rhs + r0 + r) * n + j];
        bac[r][0] -= br * yv.x - bi * yv.y;
        bac[r][1] -= br * yv.y + bi * yv.x;
      }
  }
#pragma unroll
  for (int r = 0; r < kRhsChunk; ++r) {
    if (r >= nr) break;   // uniform
    const double sr = block_sum(bac[r][0], sh);
    const double si = block_sum(bac[r][1], sh);
    if (threadIdx.x == 0) b[((int64_t)kq * n_rhs + r0 + r) * n + i] = make_double2(sr, si);
  }
}

// r = b - A x for the stored float64 operator: one workgroup per (row, vector)
__global__ __launch_bounds__(kQT) void quad_residual_kernel(int n, const double2* __restrict__ A,
                                                            int64_t ld, int64_t stride, int nr,
                                                            const double2* __restrict__ b,
                                                            const double2* __restrict__ xv,
                                                            double2* __restrict__ r) {
  __shared__ double sh[kQT / 64];
  const int i = blockIdx.x, q = blockIdx.y, kq = q / nr;
  const double2* Ar = A + kq * stride + (int64_t)i * ld;
  const double2* xq = xv + (int64_t)q * n;
  double sr = 0, si = 0;
  for (int j = threadIdx.x; j < n; j += kQT) {
    const double2 a = Ar[j], v = xq[j];
    sr += a.x * v.x - a.y * v.y;
    si += a.x * v.y + a.y * v.x;
  }
  sr = block_sum(sr, sh);
  si = block_sum(si, sh);
  if (threadIdx.x == 0) {
    const double2 bb = b[(int64_t)q * n + i];
    r[(int64_t)q * n + i] = make_double2(bb.x - sr, bb.y - si);
  }
}

// surface data at the quadrature points: out[v][p] = sum_a N_a(q) data[v][node a of e]
__global__ void quad_interp_kernel(int n, int F, int nvec, const int32_t* __restrict__ elem,
                                   QuadRule R, const double2* __restrict__ data,
                                   double2* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npts = (int64_t)F * kQ;
  if (t >= npts * nvec) return;
  const int v = (int)(t / npts);
  const int p = (int)(t % npts), e = p / kQ, q = p % kQ;
  double sr = 0, si = 0;
  for (int a = 0; a < 6; ++a) {
    const double2 d = data[(int64_t)v * n + elem[6 * e + a]];
    sr += R.N[q][a] * d.x;
    si += R.N[q][a] * d.y;
  }
  out[t] = make_double2(sr, si);
}

// Scattered field by Eq. BRIEFdmn with the element quadrature, x0 the closest
// node a:  4 pi P(x_p) = 4 pi phi_a + int [u (H^p - H^a) - u' (G^p - G^a)] dS,
// u = phi - phi_a g - psi_a f, u' = psi - phi_a g' - psi_a f' (f, g about x_a).
// One thread per (point, wavenumber, rhs); float64.
__global__ __launch_bounds__(kQT) void quad_field_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm, int npts,
    const double* __restrict__ qp, const double* __restrict__ kv, int n_k, int n_rhs,
    const double2* __restrict__ phi, const double2* __restrict__ psi,
    const double2* __restrict__ phq, const double2* __restrict__ psq, int m,
    const double* __restrict__ xp, const int32_t* __restrict__ i0,
    const uint8_t* __restrict__ inside, double2* __restrict__ U) {
  const int p = blockIdx.x * kQT + threadIdx.x;
  const int kq = blockIdx.y, rhs = blockIdx.z;
  if (p >= m) return;
  double2* out = U + ((int64_t)rhs * m + p) * n_k + kq;
  if (inside[p]) {
    *out = make_double2(0.0, 0.0);
    return;
  }
  const double k = kv[kq];
  const int a = i0[p];
  const int64_t vec = (int64_t)kq * n_rhs + rhs;
  const double2 pa = phi[vec * n + a], qa = psi[vec * n + a];
  const double ax = x[3 * a], ay = x[3 * a + 1], az = x[3 * a + 2];
  const double anx = nrm[3 * a], any = nrm[3 * a + 1], anz = nrm[3 * a + 2];
  const double px = xp[3 * p], py = xp[3 * p + 1], pz = xp[3 * p + 2];
  if (px == ax && py == ay && pz == az) {   // x_p = x0: the integrand vanishes identically
    *out = pa;
    return;
  }
  double sr = 0, si = 0;
  for (int t = 0; t < npts; ++t) {
    const double* o = qp + 8 * (int64_t)t;
    const double dax = o[0] - ax, day = o[1] - ay, daz = o[2] - az;
    double2 Ga, Ha, Gp, Hp;
    green(k, dax, day, daz, o[3], o[4], o[5], Ga, Ha);
    green(k, o[0] - px, o[1] - py, o[2] - pz, o[3], o[4], o[5], Gp, Hp);
    double ss, cs;
    sincos(k * (anx * dax + any * day + anz * daz), &ss, &cs);
    const double nn = anx * o[3] + any * o[4] + anz * o[5];
    const double g = cs, f = ss / k, gp = -k * ss * nn, fp = cs * nn;
    const double2 ph = phq[vec * npts + t], ps = psq[vec * npts + t];
    // u = phi - phi_a g - psi_a f ;  u' = psi - phi_a g' - psi_a f'
    const double ur = ph.x - pa.x * g - qa.x * f, ui = ph.y - pa.y * g - qa.y * f;
    const double vr = ps.x - pa.x * gp - qa.x * fp, vi = ps.y - pa.y * gp - qa.y * fp;
    const double hr = Hp.x - Ha.x, hi = Hp.y - Ha.y, gr = Gp.x - Ga.x, gi = Gp.y - Ga.y;
    const double wJ = o[6];
    sr += ((ur * hr - ui * hi) - (vr * gr - vi * gi)) * wJ;
    si += ((ur * hi + ui * hr) - (vr * gi + vi * gr)) * wJ;
  }
  *out = make_double2(pa.x + sr / kFourPiQ, pa.y + si / kFourPiQ);
}

}  // namespace

size_t quad_setup_bytes(int n, int F) {
  return ((size_t)F * kQ * 8 * 8 + 255) / 256 * 256 + ((size_t)n * kMaxInc * 4 + 255) / 256 * 256 + 256;
}

// Quadrature points and node incidences of the surface into ws (at least
// quad_setup_bytes); *qp and *inc point into it.  Synchronises the stream (the
// incidence check is read back).
bem_status quad_setup(bem_ctx* ctx, const bem_quad_surface* s, void* ws, double** qp,
                      int32_t** inc) {
  char* p = (char*)ws;
  *qp = (double*)p;
  p += ((size_t)s->n_elem * kQ * 8 * 8 + 255) / 256 * 256;
  *inc = (int32_t*)p;
  p += ((size_t)s->n * kMaxInc * 4 + 255) / 256 * 256;
  int32_t* flag = (int32_t*)p;
  const QuadRule R = make_rule();
  bem_status st = fill_zero(ctx, flag, 4);
  if (st != BEM_OK) return st;
  const int npts = s->n_elem * kQ;
  hipLaunchKernelGGL(quad_points_kernel, dim3((npts + 255) / 256), dim3(256), 0, ctx->stream,
                     s->n_elem, s->x, s->elem, R, *qp);
  hipLaunchKernelGGL(quad_incidence_kernel, dim3((s->n + 255) / 256), dim3(256), 0, ctx->stream,
                     s->n, s->n_elem, s->elem, *inc, flag);
  BEM_CHECK_LAUNCH(ctx);
  int32_t hflag = 0;
  BEM_HIP_TRY(ctx, hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, ctx->stream));
  BEM_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (hflag)
    return fail(ctx, BEM_EINVAL,
                "quadratic surface: an element refers to a node outside [0, n) or a node belongs "
                "to more than %d elements",
                kMaxInc);
  return BEM_OK;
}

bem_status launch_quad_assemble(bem_ctx* ctx, const bem_quad_surface* s, const double* qp,
                                const int32_t* inc, int n_k, const double* k, int n_rhs,
                                const void* y, bem_prec prec, void* A, int64_t ld,
                                int64_t a_stride, void* b, void* diag64) {
  const QuadRule R = make_rule();
  const int npts = s->n_elem * kQ;
  const int pi = prof_begin(ctx, "assemble_quad");
  for (int r0 = 0; r0 < n_rhs; r0 += kRhsChunk) {
    const int nr = std::min(kRhsChunk, n_rhs - r0);
    dim3 grid(s->n, n_k);
    if (prec == BEM_C128)
      hipLaunchKernelGGL(quad_assemble_kernel<double2>, grid, dim3(kQT), 0, ctx->stream, s->n,
                         s->x, s->nrm, s->bc, npts, qp, inc, R, k, n_rhs, r0, nr,
                         (const double2*)y, (double2*)A, ld, a_stride, (double2*)b,
                         (double2*)diag64);
    else
      hipLaunchKernelGGL(quad_assemble_kernel<float2>, grid, dim3(kQT), 0, ctx->stream, s->n,
                         s->x, s->nrm, s->bc, npts, qp, inc, R, k, n_rhs, r0, nr,
                         (const double2*)y, (float2*)A, ld, a_stride, (double2*)b,
                         (double2*)diag64);
    BEM_CHECK_LAUNCH(ctx);
  }
  // node-pair work: every (row, quadrature point) kernel value once for the
  // diagonal integrals plus once per element node holding the column
  prof_end(ctx, "assemble_quad", pi, (double)s->n * n_k * (npts + 6.0 * npts), 0.0);
  return BEM_OK;
}

bem_status launch_quad_residual(bem_ctx* ctx, int n, const void* A64, int64_t ld, int64_t stride,
                                int n_k, int n_rhs, const void* b, const void* x, void* r) {
  hipLaunchKernelGGL(quad_residual_kernel, dim3(n, n_k * n_rhs), dim3(kQT), 0, ctx->stream, n,
                     (const double2*)A64, ld, stride, n_rhs, (const double2*)b,
                     (const double2*)x, (double2*)r);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_quad_field(bem_ctx* ctx, const bem_quad_surface* s, const double* qp,
                             int n_k, const double* k, int n_rhs, const void* phi,
                             const void* psi, void* phq, void* psq, int m, const double* xp,
                             const int32_t* i0, const uint8_t* inside, void* U) {
  const QuadRule R = make_rule();
  const int npts = s->n_elem * kQ;
  const int64_t tot = (int64_t)npts * n_k * n_rhs;
  hipLaunchKernelGGL(quad_interp_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, s->n, s->n_elem, n_k * n_rhs, s->elem, R,
                     (const double2*)phi, (double2*)phq);
  hipLaunchKernelGGL(quad_interp_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, s->n, s->n_elem, n_k * n_rhs, s->elem, R,
                     (const double2*)psi, (double2*)psq);
  const int pi = prof_begin(ctx, "field_quad");
  hipLaunchKernelGGL(quad_field_kernel, dim3((m + kQT - 1) / kQT, n_k, n_rhs), dim3(kQT), 0,
                     ctx->stream, s->n, s->x, s->nrm, npts, qp, k, n_k, n_rhs,
                     (const double2*)phi, (const double2*)psi, (const double2*)phq,
                     (const double2*)psq, m, xp, i0, inside, (double2*)U);
  prof_end(ctx, "field_quad", pi, (double)m * n_k * n_rhs * npts, 0.0);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

}  // namespace bem
