// Surface-to-field evaluation by the non-singular representation (Sec. III,
// Eq. BRIEFdmn; its S_inf integrals evaluated, which leaves 4 pi P(x0) as the
// constant term when the integrals run over S only):
//   4 pi P(x_p) = 4 pi phi_a + sum_{j!=a} w_j [u_j (H^p_j - H^a_j) - u'_j (G^p_j - G^a_j)]
// with a the surface node closest to x_p, u_j = phi_j - phi_a g_aj - psi_a f_aj,
// u'_j = psi_j - phi_a g'_aj - psi_a f'_aj (f, g of Appendix A about x_a).
// The sum splits into S(x_p) - S(x_a) with
//   S(x) = A1 - phi_a A2 - psi_a A3,
//   A1 = sum w_j (phi_j H^x_j - psi_j G^x_j), A2 = sum w_j (g_aj H^x_j - g'_aj G^x_j),
//   A3 = sum w_j (f_aj H^x_j - f'_aj G^x_j)   (j != a).
// S(x_a) is computed once per node by the same kernel, so the per-point work
// is one sweep over the nodes.  A2 and A3 do not depend on the right-hand
// side: a workgroup takes NR right-hand sides at once and applies every
// generated kernel value (w G, w H for one node, point and frequency) to all
// of them, so NR right-hand sides cost one kernel generation and NR complex
// multiply-adds per term instead of NR generations.  Float32 kernels take every phase k*r and k*s
// in float64, reduce it to [-1/2, 1/2) revolutions, and evaluate the
// trigonometric functions in float32 on the reduced argument.  Each point's
// sweep is split over kParts lanes (lane q takes every kParts-th node), whose
// partial sums are combined by a butterfly at the end: the float32 sums then
// run over n / kParts terms each, which bounds their rounding error kParts
// times tighter than one chain over all n nodes.
#include <type_traits>

#include "common.h"

namespace bem {
namespace {

// ---------------------------------------------------------------- fixed scratch
// The node sums S(x_a) of bem_field_eval_noalloc live in this file-scope
// array (one copy per device, held until the process ends) instead of the
// context's workspace.  Host code never passes the array's name as an address
// (in host code it is only a stand-in for the device symbol): field_scratch_init
// takes the device address once per context, with the context's device
// current, and the kernels receive that pointer.
constexpr size_t kFieldScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kFieldScratchBytes];

constexpr double kInv2Pi = 0.15915494309189533576888376337251;
constexpr double kFourPi = 12.566370614359172953850573533118;

// --------------------------------------------------------------- closest node
// i0[p] = argmin_j (dx*dx + dy*dy) + dz*dz, float64 without contraction,
// ties to the lowest j; inside[p] = n_a.(x_p - x_a) < 0.
constexpr int kCT = 256, kCChunk = 1024;

__global__ __launch_bounds__(kCT) void closest_kernel(int n, const double* __restrict__ x,
                                                      const double* __restrict__ nrm, int m,
                                                      const double* __restrict__ xp,
                                                      int32_t* __restrict__ i0,
                                                      uint8_t* __restrict__ inside) {
  __shared__ double sx[kCChunk], sy[kCChunk], sz[kCChunk];
  const int p = blockIdx.x * kCT + threadIdx.x;
  const bool valid = p < m;
  const double px = valid ? xp[3 * p] : 0.0, py = valid ? xp[3 * p + 1] : 0.0,
               pz = valid ? xp[3 * p + 2] : 0.0;
  double best = __builtin_inf();
  int bi = 0;
  for (int j0 = 0; j0 < n; j0 += kCChunk) {
    const int cnt = min(kCChunk, n - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += kCT) {
      sx[e] = x[3 * (j0 + e)];
      sy[e] = x[3 * (j0 + e) + 1];
      sz[e] = x[3 * (j0 + e) + 2];
    }
    __syncthreads();
    for (int e = 0; e < cnt; ++e) {
      const double d0 = __dsub_rn(px, sx[e]);
      const double d1 = __dsub_rn(py, sy[e]);
      const double d2 = __dsub_rn(pz, sz[e]);
      const double dist = __dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)), __dmul_rn(d2, d2));
      if (dist < best) { best = dist; bi = j0 + e; }
    }
  }
  if (!valid) return;
  i0[p] = bi;
  const double d0 = __dsub_rn(px, x[3 * bi]), d1 = __dsub_rn(py, x[3 * bi + 1]),
               d2 = __dsub_rn(pz, x[3 * bi + 2]);
  const double nd = __dadd_rn(__dadd_rn(__dmul_rn(nrm[3 * bi], d0), __dmul_rn(nrm[3 * bi + 1], d1)),
                              __dmul_rn(nrm[3 * bi + 2], d2));
  inside[p] = nd < 0.0 ? 1 : 0;
}

__global__ void inside_kernel(const double* __restrict__ x, const double* __restrict__ nrm, int m,
                              const double* __restrict__ xp, const int32_t* __restrict__ i0,
                              uint8_t* __restrict__ inside) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const int bi = i0[p];
  const double d0 = __dsub_rn(xp[3 * p], x[3 * bi]), d1 = __dsub_rn(xp[3 * p + 1], x[3 * bi + 1]),
               d2 = __dsub_rn(xp[3 * p + 2], x[3 * bi + 2]);
  const double nd = __dadd_rn(__dadd_rn(__dmul_rn(nrm[3 * bi], d0), __dmul_rn(nrm[3 * bi + 1], d1)),
                              __dmul_rn(nrm[3 * bi + 2], d2));
  inside[p] = nd < 0.0 ? 1 : 0;
}

// --------------------------------------------------------------- field sums
template <typename R> struct CX;
template <> struct CX<float> { using T = float2; };
template <> struct CX<double> { using T = double2; };

template <typename R>
__device__ inline void phase(double theta, R& s, R& c);
template <>
__device__ inline void phase<float>(double theta, float& s, float& c) {
  double t = theta * kInv2Pi;
  t -= rint(t);
  const float tf = (float)t;
  s = __builtin_amdgcn_sinf(tf);   // argument in revolutions
  c = __builtin_amdgcn_cosf(tf);
}
// the same from the phase in revolutions (t = theta / 2 pi)
__device__ inline void phase_rev(double t, float& s, float& c) {
  t -= rint(t);
  const float tf = (float)t;
  s = __builtin_amdgcn_sinf(tf);
  c = __builtin_amdgcn_cosf(tf);
}
template <>
__device__ inline void phase<double>(double theta, double& s, double& c) {
  sincos(theta, &s, &c);
}

constexpr int kFT = 256, kNJ = 128, kParts = 8, kPW = kFT / kParts;   // kPW points per workgroup

// sum over the kParts consecutive lanes of one point (butterfly: every lane
// ends with the total)
template <typename R>
__device__ inline R part_sum(R v) {
#pragma unroll
  for (int o = 1; o < kParts; o <<= 1) v += __shfl_xor(v, o, kParts);
  return v;
}

// MODE 0: write S(x_p) for points = nodes (raw, [rhs][n_k][n]); with a node
// list (nlist, its length at *ncount), point p is node nlist[p] and only the
// listed nodes are written.
// MODE 1: write P(x_p) = phi_a + (S(x_p) - S(x_a)) / (4 pi) into U[rhs][m][n_k].
// Right-hand sides blockIdx.z * NR + r, r < min(NR, n_rhs - blockIdx.z * NR).
template <typename R, int FCH, int MODE, int NR>
__global__ __launch_bounds__(kFT, sizeof(R) == 4 ? 3 : 1) void field_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const double* __restrict__ kv, int n_k, int n_rhs,
    const double2* __restrict__ phi, const double2* __restrict__ psi, int m,
    const double* __restrict__ xp, const int32_t* __restrict__ i0,
    const uint8_t* __restrict__ inside, typename CX<R>::T* __restrict__ Snode,
    typename CX<R>::T* __restrict__ U, const int32_t* __restrict__ nlist = nullptr,
    const int32_t* __restrict__ ncount = nullptr) {
  using C = typename CX<R>::T;
  if (MODE == 0 && nlist) {
    m = *ncount;
    if ((int)blockIdx.x * kPW >= m) return;   // the whole workgroup
  }
  __shared__ double sx[kNJ][3];
  __shared__ double sn[kNJ][3];
  __shared__ R sw[kNJ];
  __shared__ C sphi[NR][FCH][kNJ];
  __shared__ C spsi[NR][FCH][kNJ];
  const int p = blockIdx.x * kPW + threadIdx.x / kParts;
  const int part = threadIdx.x % kParts;
  const int m0 = blockIdx.y * FCH;
  const int r0 = blockIdx.z * NR;
  const int nrh = min(NR, n_rhs - r0);
  const int nf = min(FCH, n_k - m0);
  const bool valid = p < m && (MODE == 0 || !inside[p]);
  const int a = p < m ? (MODE == 0 ? (nlist ? nlist[p] : p) : i0[p]) : 0;
  const int pc = MODE == 0 ? a : p;   // the point's coordinates
  const double px = p < m ? xp[3 * pc] : 0.0, py = p < m ? xp[3 * pc + 1] : 0.0,
               pz = p < m ? xp[3 * pc + 2] : 0.0;
  const double ax = x[3 * a], ay = x[3 * a + 1], az = x[3 * a + 2];
  const double anx = nrm[3 * a], any = nrm[3 * a + 1], anz = nrm[3 * a + 2];
  double kk[FCH];
#pragma unroll
  for (int f = 0; f < FCH; ++f) kk[f] = f < nf ? kv[m0 + f] : kv[m0];
  R kinv[FCH];
#pragma unroll
  for (int f = 0; f < FCH; ++f) kinv[f] = (R)(1.0 / kk[f]);
  // float32 kernels on an evenly spaced chunk of wavenumbers advance both
  // phases by a rotation (e^{i k_f t} = e^{i k_0 t} (e^{i dk t})^f): two phase
  // evaluations per node instead of 2 FCH; about one float32 rounding per step
  // (a few 1e-7 over a chunk of 8)
  const double dkk = nf > 1 ? (kk[nf - 1] - kk[0]) / (nf - 1) : 0.0;
  bool uni = sizeof(R) == 4 && nf > 1;
#pragma unroll
  for (int f = 1; f < FCH; ++f)
    if (f < nf && !(fabs(kk[f] - (kk[0] + f * dkk)) <= 4e-16 * fabs(kk[f]))) uni = false;
  C A1[NR][FCH], A2[FCH], A3[FCH];
#pragma unroll
  for (int f = 0; f < FCH; ++f) {
#pragma unroll
    for (int r = 0; r < NR; ++r) A1[r][f].x = A1[r][f].y = R(0);
    A2[f].x = A2[f].y = R(0);
    A3[f].x = A3[f].y = R(0);
  }
  for (int j0 = 0; j0 < n; j0 += kNJ) {
    const int cnt = min(kNJ, n - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * 3; e += kFT) {
      sx[e / 3][e % 3] = x[3 * j0 + e];
      sn[e / 3][e % 3] = nrm[3 * j0 + e];
    }
    for (int e = threadIdx.x; e < cnt; e += kFT) sw[e] = (R)w[j0 + e];
    for (int e = threadIdx.x; e < NR * FCH * kNJ; e += kFT) {
      const int r = e / (FCH * kNJ), f = (e / kNJ) % FCH, jj = e % kNJ;
      if (r < nrh && f < nf && jj < cnt) {
        const int64_t o = ((int64_t)(m0 + f) * n_rhs + r0 + r) * n + j0 + jj;
        const double2 u = phi[o], v = psi[o];
        sphi[r][f][jj].x = (R)u.x; sphi[r][f][jj].y = (R)u.y;
        spsi[r][f][jj].x = (R)v.x; spsi[r][f][jj].y = (R)v.y;
      } else {
        sphi[r][f][jj].x = sphi[r][f][jj].y = R(0);
        spsi[r][f][jj].x = spsi[r][f][jj].y = R(0);
      }
    }
    __syncthreads();
    if (!valid) continue;
    for (int jj = part; jj < cnt; jj += kParts) {
      if (j0 + jj == a) continue;
      const double dx = sx[jj][0] - px, dy = sx[jj][1] - py, dz = sx[jj][2] - pz;
      // r and the phase argument n_a.(x_j - x_a) stay in float64 (they enter
      // k r and k s); magnitudes (1/r, d.n, n_a.n_j) only need the kernel's
      // precision: float32 reciprocal and dot products in the float32 kernel
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      R rinv, dn, nn;
      if (sizeof(R) == 4) {
        rinv = (R)__builtin_amdgcn_rcpf((float)r);
        const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
        dn = (R)((fdx * (float)sn[jj][0] + fdy * (float)sn[jj][1] + fdz * (float)sn[jj][2]) *
                 ((float)rinv * (float)rinv));
        nn = (R)((float)anx * (float)sn[jj][0] + (float)any * (float)sn[jj][1] +
                 (float)anz * (float)sn[jj][2]);
      } else {
        const double ri = 1.0 / r;
        rinv = (R)ri;
        dn = (R)((dx * sn[jj][0] + dy * sn[jj][1] + dz * sn[jj][2]) * ri * ri);
        nn = (R)(anx * sn[jj][0] + any * sn[jj][1] + anz * sn[jj][2]);
      }
      const R wj = sw[jj];
      const R wg = wj * rinv;               // w/r
      const R wh2 = -wj * (dn * rinv);      // -w (d.n)/r^3
      const R wh1 = wj * dn;                // w (d.n)/r^2 (times k)
      const double sa = anx * (sx[jj][0] - ax) + any * (sx[jj][1] - ay) + anz * (sx[jj][2] - az);
      R es, ec, ss, cs, des = R(0), dec = R(1), dss = R(0), dcs = R(1);
      phase<R>(kk[0] * r, es, ec);
      phase<R>(kk[0] * sa, ss, cs);
      if (uni) {
        phase<R>(dkk * r, des, dec);
        phase<R>(dkk * sa, dss, dcs);
      }
#pragma unroll
      for (int f = 0; f < FCH; ++f) {
        const R k = (R)kk[f];
        if (f > 0) {
          if (uni) {
            const R e1 = ec * des + es * dec, e0 = ec * dec - es * des;
            es = e1;
            ec = e0;
            const R s1 = cs * dss + ss * dcs, s0 = cs * dcs - ss * dss;
            ss = s1;
            cs = s0;
          } else {
            phase<R>(kk[f] * r, es, ec);
            phase<R>(kk[f] * sa, ss, cs);
          }
        }
        // wG = (w/r) E ; wH = E (-w dn/r^3 + i k w dn/r^2)
        const R gr = wg * ec, gi = wg * es;
        const R hb = k * wh1;
        const R hr = ec * wh2 - es * hb, hi = ec * hb + es * wh2;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (NR > 1 && r >= nrh) break;   // uniform (one right-hand side: nrh = 1)
          const C ph = sphi[r][f][jj], ps = spsi[r][f][jj];
          A1[r][f].x += (ph.x * hr - ph.y * hi) - (ps.x * gr - ps.y * gi);
          A1[r][f].y += (ph.x * hi + ph.y * hr) - (ps.x * gi + ps.y * gr);
        }
        const R g = cs, gp = -k * ss * nn;
        const R fv = ss * kinv[f], fp = cs * nn;
        A2[f].x += g * hr - gp * gr;
        A2[f].y += g * hi - gp * gi;
        A3[f].x += fv * hr - fp * gr;
        A3[f].y += fv * hi - fp * gi;
      }
    }
  }
#pragma unroll
  for (int f = 0; f < FCH; ++f) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      A1[r][f].x = part_sum(A1[r][f].x);
      A1[r][f].y = part_sum(A1[r][f].y);
    }
    A2[f].x = part_sum(A2[f].x);
    A2[f].y = part_sum(A2[f].y);
    A3[f].x = part_sum(A3[f].x);
    A3[f].y = part_sum(A3[f].y);
  }
  if (p >= m) return;
  // the point's NR * FCH outputs (r, f) are shared out over its kParts lanes
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int f = 0; f < FCH; ++f) {
      if ((r * FCH + f) % kParts != part || r >= nrh || f >= nf) continue;
      const int rhs = r0 + r;
      const int64_t oa = ((int64_t)(m0 + f) * n_rhs + rhs) * n + a;
      const double2 pa = phi[oa], qa = psi[oa];
      const R par = (R)pa.x, pai = (R)pa.y, qar = (R)qa.x, qai = (R)qa.y;
      C S;
      S.x = A1[r][f].x - (par * A2[f].x - pai * A2[f].y) - (qar * A3[f].x - qai * A3[f].y);
      S.y = A1[r][f].y - (par * A2[f].y + pai * A2[f].x) - (qar * A3[f].y + qai * A3[f].x);
      if (MODE == 0) {
        Snode[((int64_t)rhs * n_k + m0 + f) * n + a] = S;
      } else {
        C out;
        if (!valid) {
          out.x = out.y = R(0);
        } else {
          const C s0 = Snode[((int64_t)rhs * n_k + m0 + f) * n + a];
          const R inv4pi = (R)(1.0 / kFourPi);
          out.x = par + (S.x - s0.x) * inv4pi;
          out.y = pai + (S.y - s0.y) * inv4pi;
        }
        U[((int64_t)rhs * m + p) * n_k + m0 + f] = out;
      }
    }
  }
}

// ---------------------------------------------------------------- grouped field
// The float32 field of points grouped by their closest node a.  For one
// node, Eq. BRIEFdmn's brackets
//   u_j = w_j (phi_j - phi_a g_aj - psi_a f_aj),  v_j = w_j (psi_j - phi_a g'_aj - psi_a f'_aj)
// depend on (a, j, k) only, so a workgroup holding points of one node forms
// them once per node tile and frequency chunk (float64, rounded to float32)
// and every point's sum becomes S(x) = sum_{j != a} (u_j H^x_j - v_j G^x_j):
// one phase and two complex multiply-adds per term.  The node sums S(x_a)
// come from the float64 node pass (they are of the size of the surface data,
// while far from the bodies S(x_p) and the field are much smaller), and
//   P(x_p) = phi_a + (S(x_p) - S(x_a)) / (4 pi)
// is formed in float64.  Points are sorted by closest node with a counting
// sort; each node's points are cut into chunks of kGP = kPW (one workgroup
// each).  Inside points are in no chunk and get 0.
constexpr int kGP = kPW;

// cnt[a] = number of outside points whose closest node is a (cnt zeroed)
__global__ void group_count_kernel(int m, const int32_t* __restrict__ i0,
                                   const uint8_t* __restrict__ inside, int32_t* __restrict__ cnt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < m && !inside[p]) atomicAdd(&cnt[i0[p]], 1);
}

// one workgroup of 1024 threads: off = exclusive scan of cnt, choff =
// exclusive scan of ceil(cnt / kGP), uoff = exclusive scan of (cnt > 0), all
// with their totals at [n]
__global__ __launch_bounds__(1024) void group_scan_kernel(int n, const int32_t* __restrict__ cnt,
                                                          int32_t* __restrict__ off,
                                                          int32_t* __restrict__ choff,
                                                          int32_t* __restrict__ uoff) {
  __shared__ int32_t sa[1024], sb[1024], sc[1024];
  __shared__ int32_t carry[3];
  if (threadIdx.x == 0) carry[0] = carry[1] = carry[2] = 0;
  __syncthreads();
  for (int b0 = 0; b0 < n; b0 += 1024) {
    const int i = b0 + threadIdx.x;
    const int c = i < n ? cnt[i] : 0;
    const int u = c > 0;
    sa[threadIdx.x] = c;
    sb[threadIdx.x] = (c + kGP - 1) / kGP;
    sc[threadIdx.x] = u;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive scans (Hillis-Steele)
      const int va = threadIdx.x >= o ? sa[threadIdx.x - o] : 0;
      const int vb = threadIdx.x >= o ? sb[threadIdx.x - o] : 0;
      const int vc = threadIdx.x >= o ? sc[threadIdx.x - o] : 0;
      __syncthreads();
      sa[threadIdx.x] += va;
      sb[threadIdx.x] += vb;
      sc[threadIdx.x] += vc;
      __syncthreads();
    }
    if (i < n) {
      off[i] = carry[0] + sa[threadIdx.x] - c;
      choff[i] = carry[1] + sb[threadIdx.x] - (c + kGP - 1) / kGP;
      uoff[i] = carry[2] + sc[threadIdx.x] - u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      carry[0] += sa[1023];
      carry[1] += sb[1023];
      carry[2] += sc[1023];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    off[n] = carry[0];
    choff[n] = carry[1];
    uoff[n] = carry[2];
  }
}

// perm: the outside points ordered by closest node (fill zeroed); the order
// inside a node's range does not matter
__global__ void group_scatter_kernel(int m, const int32_t* __restrict__ i0,
                                     const uint8_t* __restrict__ inside,
                                     const int32_t* __restrict__ off, int32_t* __restrict__ fill,
                                     int32_t* __restrict__ perm) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m || inside[p]) return;
  const int a = i0[p];
  perm[off[a] + atomicAdd(&fill[a], 1)] = p;
}

// chunks[c] = (node, first index into perm, points), kGP points at most;
// used[uoff[a]] = a for the nodes that are some point's closest node
__global__ void group_chunks_kernel(int n, const int32_t* __restrict__ cnt,
                                    const int32_t* __restrict__ off,
                                    const int32_t* __restrict__ choff, int4* __restrict__ chunks,
                                    const int32_t* __restrict__ uoff, int32_t* __restrict__ used) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  if (cnt[a] > 0) used[uoff[a]] = a;
  const int c0 = choff[a], nc = choff[a + 1] - c0;
  for (int c = 0; c < nc; ++c)
    chunks[c0 + c] = make_int4(a, off[a] + c * kGP, min(kGP, cnt[a] - c * kGP), 0);
}

// U = 0 for inside points
__global__ void zero_inside_kernel(int m, int n_k, int n_rhs, const uint8_t* __restrict__ inside,
                                   float2* __restrict__ U) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * n_k * n_rhs) return;
  const int p = (int)((t / n_k) % m);
  if (inside[p]) U[t] = make_float2(0.f, 0.f);
}

template <int FCH, int NR>
__global__ __launch_bounds__(kFT, 3) void field_grouped_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const double* __restrict__ kv, int n_k, int n_rhs,
    const double2* __restrict__ phi, const double2* __restrict__ psi, int m,
    const double* __restrict__ xp, const int4* __restrict__ chunks,
    const int32_t* __restrict__ nchunks, const int32_t* __restrict__ perm,
    const double2* __restrict__ Snode, float2* __restrict__ U) {
  __shared__ double sx[kNJ][3];
  __shared__ float2 su[NR][FCH][kNJ], sv[NR][FCH][kNJ];
  __shared__ float snrm[kNJ][3];
  // per chunk frequency f: k, 1/k, and phi, psi of node a per right-hand side
  // (looked up by the bracket loop, whose f varies per thread)
  __shared__ double skk[FCH], skinv[FCH];
  __shared__ double2 spa[NR][FCH], sqa[NR][FCH];
  if ((int)blockIdx.x >= *nchunks) return;   // uniform
  const int4 ch = chunks[blockIdx.x];
  const int a = ch.x, start = ch.y, len = ch.z;
  const int gi = threadIdx.x / kParts, part = threadIdx.x % kParts;
  const bool valid = gi < len;
  const int p = valid ? perm[start + gi] : -1;
  const double ax = x[3 * a], ay = x[3 * a + 1], az = x[3 * a + 2];
  const double anx = nrm[3 * a], any = nrm[3 * a + 1], anz = nrm[3 * a + 2];
  const double px = p >= 0 ? xp[3 * p] : ax, py = p >= 0 ? xp[3 * p + 1] : ay,
               pz = p >= 0 ? xp[3 * p + 2] : az;
  const int m0 = blockIdx.y * FCH;
  const int r0 = blockIdx.z * NR;
  const int nrh = min(NR, n_rhs - r0);
  const int nf = min(FCH, n_k - m0);
  double kk[FCH];
#pragma unroll
  for (int f = 0; f < FCH; ++f) kk[f] = f < nf ? kv[m0 + f] : kv[m0];
  const double dkk = nf > 1 ? (kk[nf - 1] - kk[0]) / (nf - 1) : 0.0;
  bool uni = nf > 1;
#pragma unroll
  for (int f = 1; f < FCH; ++f)
    if (f < nf && !(fabs(kk[f] - (kk[0] + f * dkk)) <= 4e-16 * fabs(kk[f]))) uni = false;
  if (threadIdx.x < FCH) {
    const double kf0 = kv[m0 + min((int)threadIdx.x, nf - 1)];
    skk[threadIdx.x] = kf0;
    skinv[threadIdx.x] = 1.0 / kf0;
  }
  if (threadIdx.x < NR * FCH) {
    const int r = threadIdx.x / FCH, f = threadIdx.x % FCH;
    double2 pa = make_double2(0.0, 0.0), qa = pa;
    if (r < nrh && f < nf) {
      const int64_t va = ((int64_t)(m0 + f) * n_rhs + r0 + r) * n;
      pa = phi[va + a];
      qa = psi[va + a];
    }
    spa[r][f] = pa;
    sqa[r][f] = qa;
  }
  // (the node loop's first barrier publishes these tables)
  const double k0rev = kk[0] * kInv2Pi, dkrev = dkk * kInv2Pi;
  float2 S[NR][FCH], S1[NR][FCH];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int f = 0; f < FCH; ++f) S[r][f] = S1[r][f] = make_float2(0.f, 0.f);
  for (int j0 = 0; j0 < n; j0 += kNJ) {
    const int cnt = min(kNJ, n - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * 3; e += kFT) {
      sx[e / 3][e % 3] = x[3 * j0 + e];
      snrm[e / 3][e % 3] = (float)nrm[3 * j0 + e];
    }
    // the brackets u, v of the tile's nodes for the workgroup's node a
    for (int e = threadIdx.x; e < NR * FCH * kNJ; e += kFT) {
      const int r = e / (FCH * kNJ), f = (e / kNJ) % FCH, jj = e % kNJ;
      float2 uu = make_float2(0.f, 0.f), vv = uu;
      const int j = j0 + jj;
      if (r < nrh && f < nf && jj < cnt && j != a) {
        const double k = skk[f];
        const double njx = nrm[3 * j], njy = nrm[3 * j + 1], njz = nrm[3 * j + 2];
        const double sa = anx * (x[3 * j] - ax) + any * (x[3 * j + 1] - ay) + anz * (x[3 * j + 2] - az);
        const double nn = anx * njx + any * njy + anz * njz;
        // the phase reduced in float64, its sine and cosine in float32 (the
        // brackets are rounded to float32)
        float fsn, fcs;
        phase<float>(k * sa, fsn, fcs);
        const double sn = fsn, cs = fcs;
        const double g = cs, fv = sn * skinv[f], gp = -k * sn * nn, fp = cs * nn;
        const int64_t va = ((int64_t)(m0 + f) * n_rhs + r0 + r) * n;
        const double2 pa = spa[r][f], qa = sqa[r][f], pj = phi[va + j], qj = psi[va + j];
        const double wj = w[j];
        uu = make_float2((float)(wj * (pj.x - pa.x * g - qa.x * fv)),
                         (float)(wj * (pj.y - pa.y * g - qa.y * fv)));
        vv = make_float2((float)(wj * (qj.x - pa.x * gp - qa.x * fp)),
                         (float)(wj * (qj.y - pa.y * gp - qa.y * fp)));
      }
      su[r][f][jj] = uu;
      sv[r][f][jj] = vv;
    }
    __syncthreads();
    if (!valid) continue;
    // the lane's nodes alternate between two partial sums (halving the
    // length of each float32 chain)
    // uni_c: std::true_type / std::false_type (the test folded away) or a
    // runtime bool
    auto term = [&](int jj, float2 (&Sh)[NR][FCH], auto uni_c) {
      const bool UNI = static_cast<bool>(uni_c);
      if (j0 + jj == a) return;   // its brackets vanish (and r = 0 for a point on the node)
      const double dx = sx[jj][0] - px, dy = sx[jj][1] - py, dz = sx[jj][2] - pz;
      // r from the float32 reciprocal square root of r^2 and one Newton step in
      // float64 (relative error ~1e-14, ample for the float64 phase k r);
      // that reciprocal is also the kernel's float32 1/r
      const double r2 = dx * dx + dy * dy + dz * dz;
      const float rinv = __builtin_amdgcn_rsqf((float)r2);
      double r = r2 * (double)rinv;
      r = fma(fma(-r, r, r2), 0.5 * (double)rinv, r);
      // u H - v G = E' t with E' = -E / r (rotated like E) and
      // t = c u (1 - ikr) + v, c = (d.n_j)/r^2
      const float c = ((float)dx * snrm[jj][0] + (float)dy * snrm[jj][1] + (float)dz * snrm[jj][2]) *
                      (rinv * rinv);
      float es, ec, des = 0.f, dec = 1.f;
      // (the wavenumbers carry the 1 / 2 pi of the reduction)
      phase_rev(k0rev * r, es, ec);
      if (UNI) phase_rev(dkrev * r, des, dec);
      const float cr = c * (float)r;
      es *= -rinv;
      ec *= -rinv;
      // on an even chunk the phase advances by the three-term recurrence
      // E'_{f+1} = 2 cos(dk r) E'_f - E'_{f-1} (two multiply-adds a step; a
      // rounding at step f grows at most f-fold over the chunk)
      const float tc = 2.f * dec;
      float esp = 0.f, ecp = 0.f;
#pragma unroll
      for (int f = 0; f < FCH; ++f) {
        if (f > 0) {
          if (UNI) {
            float e1, e0;
            if (f == 1) {
              e1 = ec * des + es * dec;
              e0 = ec * dec - es * des;
            } else {
              e1 = fmaf(tc, es, -esp);
              e0 = fmaf(tc, ec, -ecp);
            }
            esp = es;
            ecp = ec;
            es = e1;
            ec = e0;
          } else {
            phase<float>(kk[f] * r, es, ec);
            es *= -rinv;
            ec *= -rinv;
          }
        }
        const float cq = (float)kk[f] * cr;   // c k r
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
          if (NR > 1 && rr >= nrh) break;   // uniform (one right-hand side: nrh = 1)
          const float2 u = su[rr][f][jj], v = sv[rr][f][jj];
          const float tx = fmaf(c, u.x, fmaf(cq, u.y, v.x));
          const float ty = fmaf(c, u.y, fmaf(-cq, u.x, v.y));
          Sh[rr][f].x = fmaf(ec, tx, fmaf(-es, ty, Sh[rr][f].x));
          Sh[rr][f].y = fmaf(ec, ty, fmaf(es, tx, Sh[rr][f].y));
        }
      }
    };
    auto nodes = [&](auto uni_c) {
      for (int jj = part; jj < cnt; jj += 2 * kParts) {
        term(jj, S, uni_c);
        if (jj + kParts < cnt) term(jj + kParts, S1, uni_c);
      }
    };
    // one right-hand side: the even-chunk test is hoisted out of the node loop
    // (no per-frequency branch inside it); with several, the two loop bodies
    // would not fit the register budget, so the test stays inside
    if constexpr (NR == 1) {
      if (uni)
        nodes(std::true_type{});
      else
        nodes(std::false_type{});
    } else {
      nodes(uni);
    }
  }
#pragma unroll
  for (int rr = 0; rr < NR; ++rr)
#pragma unroll
    for (int f = 0; f < FCH; ++f) {
      S[rr][f].x += S1[rr][f].x;
      S[rr][f].y += S1[rr][f].y;
    }
#pragma unroll
  for (int rr = 0; rr < NR; ++rr)
#pragma unroll
    for (int f = 0; f < FCH; ++f) {
      S[rr][f].x = part_sum(S[rr][f].x);
      S[rr][f].y = part_sum(S[rr][f].y);
    }
  if (p < 0) return;
  const double inv4pi = 1.0 / kFourPi;
#pragma unroll
  for (int rr = 0; rr < NR; ++rr)
#pragma unroll
    for (int f = 0; f < FCH; ++f) {
      if ((rr * FCH + f) % kParts != part || rr >= nrh || f >= nf) continue;
      const double2 pa = phi[((int64_t)(m0 + f) * n_rhs + r0 + rr) * n + a];
      const double2 sa = Snode[((int64_t)(r0 + rr) * n_k + m0 + f) * n + a];
      U[((int64_t)(r0 + rr) * m + p) * n_k + m0 + f] =
          make_float2((float)(pa.x + ((double)S[rr][f].x - sa.x) * inv4pi),
                      (float)(pa.y + ((double)S[rr][f].y - sa.y) * inv4pi));
    }
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// fixed: the fixed scratch (bem_field_eval_noalloc: no workspace, no
// profiling events), else NULL
template <int FCH, int NR>
bem_status field_grouped(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k, int n_rhs,
                         const void* phi, const void* psi, int m, const double* xp,
                         const int32_t* i0, const uint8_t* inside, void* U, void* fixed) {
  const int n = s->n;
  auto al = al256;
  const size_t max_chunks = (size_t)(m + kGP - 1) / kGP + n;
  const size_t bytes = field_group_bytes(n, m, n_k, n_rhs);
  void* ws = fixed;
  bem_status st = BEM_OK;
  if (!ws && (st = workspace(ctx, bytes, &ws)) != BEM_OK) return st;
  char* q = (char*)ws;
  double2* Snode = (double2*)q; q += al(16 * (size_t)n_rhs * n_k * n);
  int32_t* cnt = (int32_t*)q;   q += al(4 * (size_t)n);
  int32_t* fill = (int32_t*)q;  q += al(4 * (size_t)n);
  int32_t* off = (int32_t*)q;   q += al(4 * (size_t)(n + 1));
  int32_t* choff = (int32_t*)q; q += al(4 * (size_t)(n + 1));
  int32_t* uoff = (int32_t*)q;  q += al(4 * (size_t)(n + 1));
  int32_t* used = (int32_t*)q;  q += al(4 * (size_t)n);
  int32_t* perm = (int32_t*)q;  q += al(4 * (size_t)m);
  int4* chunks = (int4*)q;
  if ((st = fill_zero(ctx, cnt, 2 * al(4 * (size_t)n))) != BEM_OK) return st;   // cnt and fill
  const int pi = fixed ? -1 : prof_begin(ctx, "field");
  hipLaunchKernelGGL(group_count_kernel, dim3((m + 255) / 256), dim3(256), 0, ctx->stream, m, i0,
                     inside, cnt);
  hipLaunchKernelGGL(group_scan_kernel, dim3(1), dim3(1024), 0, ctx->stream, n, cnt, off, choff,
                     uoff);
  hipLaunchKernelGGL(group_chunks_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, cnt,
                     off, choff, chunks, uoff, used);
  // float64 node sums S(x_a) of the nodes that are some point's closest node
  // (their count uoff[n] stays on the device: the grid covers all n nodes and
  // the workgroups past the count return at once)
  {
    const int nz = (n_rhs + NR - 1) / NR;
    if (NR == 1)
      hipLaunchKernelGGL((field_kernel<double, 8, 0, 1>),
                         dim3((n + kPW - 1) / kPW, (n_k + 7) / 8, nz), dim3(kFT), 0, ctx->stream,
                         n, s->x, s->nrm, s->w, k, n_k, n_rhs, (const double2*)phi,
                         (const double2*)psi, n, s->x, (const int32_t*)nullptr,
                         (const uint8_t*)nullptr, Snode, (double2*)nullptr, used, uoff + n);
    else
      hipLaunchKernelGGL((field_kernel<double, 4, 0, 4>),
                         dim3((n + kPW - 1) / kPW, (n_k + 3) / 4, nz), dim3(kFT), 0, ctx->stream,
                         n, s->x, s->nrm, s->w, k, n_k, n_rhs, (const double2*)phi,
                         (const double2*)psi, n, s->x, (const int32_t*)nullptr,
                         (const uint8_t*)nullptr, Snode, (double2*)nullptr, used, uoff + n);
  }
  hipLaunchKernelGGL(group_scatter_kernel, dim3((m + 255) / 256), dim3(256), 0, ctx->stream, m, i0,
                     inside, off, fill, perm);
  const int64_t tot = (int64_t)m * n_k * n_rhs;
  hipLaunchKernelGGL(zero_inside_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     ctx->stream, m, n_k, n_rhs, inside, (float2*)U);
  dim3 grid((unsigned)max_chunks, (n_k + FCH - 1) / FCH, (n_rhs + NR - 1) / NR);
  hipLaunchKernelGGL((field_grouped_kernel<FCH, NR>), grid, dim3(kFT), 0, ctx->stream, n, s->x,
                     s->nrm, s->w, k, n_k, n_rhs, (const double2*)phi, (const double2*)psi, m, xp,
                     chunks, choff + n, perm, Snode, (float2*)U);
  // kernel terms: one per (point, frequency, node, rhs); the node pass adds
  // as many per node used as some point's closest node
  if (!fixed)
    prof_end(ctx, "field", pi, (double)m * n_k * n * n_rhs, 8.0 * (double)m * n_k * n_rhs);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

// Snode_fixed: the fixed scratch (bem_field_eval_noalloc: no workspace, no
// profiling events), or NULL for the context's workspace.
template <typename R, int FCH, int NR>
void field_pass(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k, int n_rhs,
                const void* phi, const void* psi, int m, const double* xp, const int32_t* i0,
                const uint8_t* inside, void* Snode, void* U) {
  using C = typename CX<R>::T;
  const int fch = (n_k + FCH - 1) / FCH;
  const int nz = (n_rhs + NR - 1) / NR;
  dim3 gnode((s->n + kPW - 1) / kPW, fch, nz);
  hipLaunchKernelGGL((field_kernel<R, FCH, 0, NR>), gnode, dim3(kFT), 0, ctx->stream, s->n, s->x,
                     s->nrm, s->w, k, n_k, n_rhs, (const double2*)phi, (const double2*)psi, s->n,
                     s->x, (const int32_t*)nullptr, (const uint8_t*)nullptr, (C*)Snode, (C*)nullptr);
  dim3 gpts((m + kPW - 1) / kPW, fch, nz);
  hipLaunchKernelGGL((field_kernel<R, FCH, 1, NR>), gpts, dim3(kFT), 0, ctx->stream, s->n, s->x,
                     s->nrm, s->w, k, n_k, n_rhs, (const double2*)phi, (const double2*)psi, m, xp,
                     i0, inside, (C*)Snode, (C*)U);
}

template <typename R>
bem_status field_go(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k, int n_rhs,
                    const void* phi, const void* psi, int m, const double* xp,
                    const int32_t* i0, const uint8_t* inside, void* U, void* Snode_fixed) {
  using C = typename CX<R>::T;
  void* ws = Snode_fixed;
  if (!ws) {
    const size_t need = sizeof(C) * (size_t)n_rhs * n_k * s->n;
    bem_status st = workspace(ctx, need, &ws);
    if (st != BEM_OK) return st;
  }
  // the profiling bracket covers both passes: the field at the nodes (the
  // expansion centres) and at the points
  const int pi = Snode_fixed ? -1 : prof_begin(ctx, "field");
  // one right-hand side: 8 frequencies per thread; more: 4 frequencies and up
  // to 4 right-hand sides per workgroup (8 frequencies with 2 right-hand
  // sides already exceed the 168-register budget of three workgroups per CU)
  if (n_rhs == 1)
    field_pass<R, 8, 1>(ctx, s, n_k, k, n_rhs, phi, psi, m, xp, i0, inside, ws, U);
  else
    field_pass<R, 4, 4>(ctx, s, n_k, k, n_rhs, phi, psi, m, xp, i0, inside, ws, U);
  // kernel terms: one per (point or node, frequency, node, rhs)
  if (!Snode_fixed)
    prof_end(ctx, "field", pi, ((double)m + s->n) * n_k * s->n * n_rhs,
             (double)sizeof(C) * ((double)m + s->n) * n_k * n_rhs);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

}  // namespace

bem_status launch_closest(bem_ctx* ctx, const bem_surface* s, int m, const double* xp,
                          int32_t* i0, uint8_t* inside) {
  if (m <= 0) return BEM_OK;
  hipLaunchKernelGGL(closest_kernel, dim3((m + kCT - 1) / kCT), dim3(kCT), 0, ctx->stream, s->n,
                     s->x, s->nrm, m, xp, i0, inside);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_inside(bem_ctx* ctx, const bem_surface* s, int m, const double* xp,
                         const int32_t* i0, uint8_t* inside) {
  if (m <= 0) return BEM_OK;
  hipLaunchKernelGGL(inside_kernel, dim3((m + 255) / 256), dim3(256), 0, ctx->stream, s->x, s->nrm,
                     m, xp, i0, inside);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status launch_field(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k, int n_rhs,
                        const void* phi, const void* psi, int m, const double* xp,
                        const int32_t* i0, const uint8_t* inside, bem_prec prec, void* U,
                        bool fixed_scratch) {
  if (m <= 0) return BEM_OK;
  void* fixed = nullptr;
  if (fixed_scratch && prec == BEM_C128) {
    const size_t need = 16 * (size_t)n_rhs * n_k * s->n;
    if (!ctx->field_scratch)
      return fail(ctx, BEM_EHIP, "bem_field_eval_noalloc: no device address for the fixed scratch");
    if (need > ctx->field_scratch_bytes)
      return fail(ctx, BEM_EINVAL,
                  "bem_field_eval_noalloc: n_rhs * n_k * n = %lld node sums need %zu bytes, more "
                  "than the %zu-byte fixed scratch",
                  (long long)n_rhs * n_k * s->n, need, ctx->field_scratch_bytes);
    fixed = ctx->field_scratch;
  }
  if (prec == BEM_C128)
    return field_go<double>(ctx, s, n_k, k, n_rhs, phi, psi, m, xp, i0, inside, U, fixed);
  // float32: points grouped by closest node (the bookkeeping in the fixed
  // scratch for bem_field_eval_noalloc, whose caller checked its size)
  void* gfixed = fixed_scratch ? ctx->field_scratch : nullptr;
  if (fixed_scratch && field_group_bytes(s->n, m, n_k, n_rhs) > ctx->field_scratch_bytes)
    return fail(ctx, BEM_EINVAL, "bem_field_eval_noalloc: point grouping does not fit the fixed scratch");
  if (n_rhs == 1)
    return field_grouped<8, 1>(ctx, s, n_k, k, n_rhs, phi, psi, m, xp, i0, inside, U, gfixed);
  return field_grouped<4, 4>(ctx, s, n_k, k, n_rhs, phi, psi, m, xp, i0, inside, U, gfixed);
}

bem_status field_scratch_init(bem_ctx* ctx) {
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    ctx->field_scratch = nullptr;
    ctx->field_scratch_bytes = 0;
    return fail(ctx, BEM_EHIP, "hipGetSymbolAddress of the field scratch failed: %s",
                hipGetErrorString(e));
  }
  ctx->field_scratch = ptr;
  ctx->field_scratch_bytes = kFieldScratchBytes;
  return BEM_OK;
}

size_t field_group_bytes(int n, int m, int n_k, int n_rhs) {
  const size_t max_chunks = (size_t)(m + kGP - 1) / kGP + n;
  return al256(16 * (size_t)n_rhs * n_k * n) + 3 * al256(4 * (size_t)n) +
         3 * al256(4 * (size_t)(n + 1)) + al256(4 * (size_t)m) + al256(16 * max_chunks);
}

}  // namespace bem
