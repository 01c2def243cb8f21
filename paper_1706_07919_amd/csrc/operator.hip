// Float64 operator of the discrete non-singular boundary integral equation
// (Eq. BRIEF with the f, g of Appendix A; the S_inf integrals of Appendix B
// leave 4 pi on the diagonal of M_phi).  For a collocation node i and a node
// j != i, with d = x_j - x_i, r = |d|, E = e^{ikr}:
//   G = E/r,  H = E (ikr - 1)(d.n_j)/r^3,  s = k n_i.d,
//   g = cos s, f = sin(s)/k, g' = -k sin(s) (n_i.n_j), f' = cos(s) (n_i.n_j)
//   (M_phi)_ij = -w_j H,  (M_psi)_ij = w_j G,
//   (M_phi)_ii = 4 pi - sum_j w_j (g' G - g H),  (M_psi)_ii = -sum_j w_j (f' G - f H).
// One workgroup owns one row and a chunk of wavenumbers and sweeps j with
// coalesced loads of the node arrays and coalesced stores of the row-major
// matrix rows.
#include "common.h"
#include "phase.h"

#include <cmath>

namespace bem {
namespace {

constexpr int kThreads = 256;
constexpr double kFourPi = 12.566370614359172953850573533118;

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// r and 1/r from r^2 > 0 in float64: the float32 reciprocal square root
// refined by two Newton steps y <- y (3 - r^2 y^2) / 2 (each squares the
// relative error: ~1e-7, ~1e-14, then float64 rounding), without the
// library's square root and division sequences
__device__ inline void dist_and_inverse(double r2, double& r, double& rinv) {
  double y = (double)__builtin_amdgcn_rsqf((float)r2);
  y *= fma(-0.5 * r2, y * y, 1.5);
  y *= fma(-0.5 * r2, y * y, 1.5);
  rinv = y;
  r = r2 * y;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Wave sums of 8 values by recursive halving: lanes l and l ^ 32 trade halves
// of the values (each keeps the half picked by bit 5 of its lane), then
// quarters across 16 and pairs across 8, then the single value left is summed
// across lanes l ^ 4, l ^ 2, l ^ 1.  Afterwards every lane whose bits 3..5
// spell q holds the wave sum of value q (10 shuffles instead of 48).
__device__ inline double wave_reduce8(const double (&v)[8]) {
  const int lane = threadIdx.x & 63;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  double h4[4], h2[2];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double keep = b5 ? v[4 + m] : v[m], give = b5 ? v[m] : v[4 + m];
    h4[m] = keep + __shfl_xor(give, 32, 64);
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const double keep = b4 ? h4[2 + m] : h4[m], give = b4 ? h4[m] : h4[2 + m];
    h2[m] = keep + __shfl_xor(give, 16, 64);
  }
  double h = (b3 ? h2[1] : h2[0]) + __shfl_xor(b3 ? h2[0] : h2[1], 8, 64);
  h += __shfl_xor(h, 4, 64);
  h += __shfl_xor(h, 2, 64);
  h += __shfl_xor(h, 1, 64);
  return h;
}

// Block-wide sum of a [R][C] array held per thread; result valid in thread 0.
template <int R, int C>
__device__ inline void block_sum_2d(double (&v)[R][C]) {
  __shared__ double red[kThreads / 64][R][C];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int c = 0; c < C; ++c) v[a][c] = wave_sum(v[a][c]);
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int c = 0; c < C; ++c) red[wid][a][c] = v[a][c];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double t = 0.0;
        for (int q = 0; q < kThreads / 64; ++q) t += red[q][a][c];
        v[a][c] = t;
      }
  }
}

// ---------------------------------------------------------------- wavenumber chunks
// A workgroup owns one row i and a chunk of consecutive
// wavenumbers.  The pair geometry (d, r, 1/r, d.n_j, n_i.d, n_i.n_j) is formed
// once per pair and shared by the chunk.  When the chunk's wavenumbers are
// evenly spaced (k_q = k_0 + q dk to a few ulp, the uniform grids of the
// frequency sweep), the phases are advanced by multiplication:
// e^{i k_q r} = e^{i k_0 r} (e^{i dk r})^q, and likewise e^{i k_q n_i.d}, so a
// chunk costs two sincos per pair and phase instead of one per wavenumber; otherwise each
// wavenumber takes its own sincos.  The recurrence adds about one rounding
// per step (relative error below 1e-15 over a chunk).
constexpr int kKcResidual = 8;   // wavenumbers per workgroup, residual
constexpr int kKcAssemble = 8;   // wavenumbers per workgroup, assembly

template <int KC>
struct KChunk {
  double k[KC];
  double dk;
  int kc;
  bool uniform;
};

// kidx (optional): slot t of the launch -> wavenumber index kidx[t]; the
// chunk is formed over slots, so a sparse list of wavenumbers is evaluated
// with a sincos per wavenumber unless its values still form an even grid.
template <int KC>
__device__ inline KChunk<KC> load_chunk(const double* __restrict__ kv, int nk,
                                        const int32_t* __restrict__ kidx) {
  KChunk<KC> c;
  const int q0 = blockIdx.y * KC;
  c.kc = min(KC, nk - q0);
#pragma unroll
  for (int q = 0; q < KC; ++q) c.k[q] = q < c.kc ? kv[kidx ? kidx[q0 + q] : q0 + q] : 0.0;
  c.uniform = c.kc > 1;
  // (the last wavenumber read again from memory: no dynamic index into c.k,
  // which would put the array in scratch memory)
  const int ql = q0 + c.kc - 1;
  c.dk = c.kc > 1 ? (kv[kidx ? kidx[ql] : ql] - c.k[0]) / (c.kc - 1) : 0.0;
#pragma unroll
  for (int q = 1; q < KC; ++q)
    if (q < c.kc && !(fabs(c.k[q] - (c.k[0] + q * c.dk)) <= 4e-16 * fabs(c.k[q]))) c.uniform = false;
  return c;
}

// Phase e^{i k_q t} stepped along the chunk: start() gives q = 0, next(q)
// advances to wavenumber q (by the recurrence, or a fresh sincos).
struct Phase {
  double2 e, d;
  template <int KC>
  __device__ inline void start(const KChunk<KC>& c, double t) {
    double s, co;
    phase_sincos(c.k[0] * t, &s, &co);
    e = make_double2(co, s);
    if (c.uniform) {
      phase_sincos(c.dk * t, &s, &co);
      d = make_double2(co, s);
    }
  }
  template <int KC>
  __device__ inline void next(const KChunk<KC>& c, int q, double t) {
    if (c.uniform) {
      e = make_double2(e.x * d.x - e.y * d.y, e.x * d.y + e.y * d.x);
    } else {
      double s, co;
      phase_sincos(c.k[q] * t, &s, &co);
      e = make_double2(co, s);
    }
  }
};

// ---------------------------------------------------------------- assembly
// One workgroup owns row i and a chunk of kKcAssemble wavenumbers, for one
// right-hand side (column rhs of y).  Thread t takes the columns
// j = t + 256 m; per pair it forms the geometry and the starting phases once
// and then, for each wavenumber of the chunk, the two kernels w G and w H,
// their contributions to the two diagonal sums and to b, and the matrix entry
// (first pass over the right-hand sides; later passes only form b).  The pair
// loop is instantiated per phase form: the recurrence on an even grid or a
// sincos per wavenumber, both with the branch-free reduction valid below
// 2^20 rad, and the library sincos for a row whose phases reach beyond (taken
// only when a pair of the row needs it: the whole row is then redone, one
// wavenumber at a time).  The per-thread sums are reduced across the
// workgroup once, at the end.
enum { kPhRec = 0, kPhNear = 1, kPhWide = 2 };

// A wave-uniform double moved to scalar registers.
__device__ inline double uniform_d(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

struct AsmRow {
  int n, n_rhs, rhs, i, q0;
  const double2* y;
  void* A;
  int64_t ld, a_stride;
};

template <int PH>
__device__ inline double2 phase_e(double x) {
  double sn, cs;
  if (PH == kPhWide)
    sincos(x, &sn, &cs);
  else
    phase_sincos_near(x, &sn, &cs);
  return make_double2(cs, sn);
}

// Terms of pair (i, j) for the chunk's wavenumbers.  wr = w_j / r,
// wq = w_j (d.n_j) / r^3, s0 = n_i.d, nn = n_i.n_j;
// acc[q] = {Dphi re, im, Dpsi re, im, b re, im}.
template <int KC, bool OUT128, bool WRITE_A, bool RHS, int PH>
__device__ __forceinline__ void pair_terms(const AsmRow& p, const KChunk<KC>& kc,
                                           int j, bool hard, double r,
                                           double s0, double wr, double wq, double nn,
                                           double (&acc)[KC][6]) {
  double2 E = phase_e<PH>(kc.k[0] * r), F = phase_e<PH>(kc.k[0] * s0), dE, dF, Ep, Fp;
  double tE = 0.0, tF = 0.0;
  // row bases of A and y for wavenumber q0 and their steps per wavenumber,
  // made opaque here so that the per-wavenumber addresses are formed in the
  // loop rather than held in scalar registers across it
  int64_t abase = (int64_t)p.q0 * p.a_stride + (int64_t)p.i * p.ld, astep = p.a_stride;
  int64_t ybase = ((int64_t)p.q0 * p.n_rhs + p.rhs) * p.n, ystep = (int64_t)p.n_rhs * p.n;
  asm volatile("" : "+s"(abase), "+s"(astep), "+s"(ybase), "+s"(ystep));
  // the known data of column j for the chunk, loaded before any store of the
  // row (the stores to A could otherwise alias them and hold each load back
  // until its use) so that the loads are in flight during the phases
  double2 yv[KC];
  if (RHS && PH == kPhRec) {
#pragma unroll
    for (int q = 0; q < KC; ++q) yv[q] = p.y[ybase + q * ystep + j];
  }
  double kr_s = 0.0, kn_s = 0.0, dkr = 0.0, dkn = 0.0;
  if (PH == kPhRec) {
    kr_s = kc.k[0] * r;
    kn_s = kc.k[0] * nn;
    dkr = kc.dk * r;
    dkn = kc.dk * nn;
  }
  if (PH == kPhRec) {
    // the three-term recurrence e^{i(q+1)t} = 2 cos(t) e^{iqt} - e^{i(q-1)t}
    // after the first step (a rounding at step q grows at most q-fold)
    dE = phase_e<PH>(kc.dk * r);
    dF = phase_e<PH>(kc.dk * s0);
    tE = 2.0 * dE.x;
    tF = 2.0 * dF.x;
  }
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    // workgroup-uniform; the recurrence runs on whole chunks only, so its
    // loop has no exits
    if (PH != kPhRec && q >= kc.kc) break;
    const double k = kc.k[q];
    if (PH == kPhRec) {
      // k r and k (n_i.n_j) stepped along the chunk (the wavenumbers are then
      // not held across the pair loop)
      if (q > 0) {
        kr_s += dkr;
        kn_s += dkn;
      }
    }
    if (q > 0) {
      if (PH == kPhRec) {
        double2 En, Fn;
        if (q == 1) {
          En = cmul(E, dE);
          Fn = cmul(F, dF);
        } else {
          En = make_double2(fma(tE, E.x, -Ep.x), fma(tE, E.y, -Ep.y));
          Fn = make_double2(fma(tF, F.x, -Fp.x), fma(tF, F.y, -Fp.y));
        }
        Ep = E;
        Fp = F;
        E = En;
        F = Fn;
      } else {
        E = phase_e<PH>(k * r);
        F = phase_e<PH>(k * s0);
      }
    }
    const double kr = PH == kPhRec ? kr_s : k * r;
    // w G = w E / r,  w H = w E (ikr - 1)(d.n_j) / r^3
    const double2 wG = make_double2(wr * E.x, wr * E.y);
    const double2 wH = make_double2(wq * fma(-kr, E.y, -E.x), wq * fma(kr, E.x, -E.y));
    // g = cos(k s0), f = sin(k s0)/k, g' = -k sin(k s0) nn, f' = cos(k s0) nn;
    // the psi sums are accumulated times k (k f' wG - k f wH, divided by k at
    // the end)
    const double kn = PH == kPhRec ? kn_s : k * nn;
    const double g = F.x, gp = -kn * F.y, kfp = kn * F.x;
    acc[q][0] = fma(gp, wG.x, fma(-g, wH.x, acc[q][0]));
    acc[q][1] = fma(gp, wG.y, fma(-g, wH.y, acc[q][1]));
    acc[q][2] = fma(kfp, wG.x, fma(-F.y, wH.x, acc[q][2]));
    acc[q][3] = fma(kfp, wG.y, fma(-F.y, wH.y, acc[q][3]));
    // unknown coefficient a (M_phi = -w H for a hard node, M_psi = w G for a
    // soft one) and known coefficient bb (the other)
    const double2 mwH = make_double2(-wH.x, -wH.y);
    const double2 a = hard ? mwH : wG, bb = hard ? wG : mwH;
    if (WRITE_A) {
      if (OUT128)
        reinterpret_cast<double2*>(p.A)[abase + q * astep + j] = a;
      else
        reinterpret_cast<float2*>(p.A)[abase + q * astep + j] = make_float2((float)a.x, (float)a.y);
    }
    if (RHS) {
      const double2 yy = PH == kPhRec ? yv[q] : p.y[ybase + q * ystep + j];
      acc[q][4] = fma(bb.x, yy.x, fma(-bb.y, yy.y, acc[q][4]));
      acc[q][5] = fma(bb.x, yy.y, fma(bb.y, yy.x, acc[q][5]));
    }
  }
}

// The thread's columns of row p.i; returns whether a phase of one of its
// pairs reaches 2^20 rad (the near forms are then invalid for the row).
template <int KC, bool OUT128, bool WRITE_A, bool RHS, int PH>
__device__ __forceinline__ bool row_terms(const AsmRow& p, const KChunk<KC>& kc,
                                          double kmax,
                                          const double* __restrict__ x,
                                          const double* __restrict__ nrm,
                                          const double* __restrict__ w,
                                          const uint8_t* __restrict__ bc, double (&acc)[KC][6]) {
  const int i = p.i;
  const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
  const double nix = nrm[3 * i], niy = nrm[3 * i + 1], niz = nrm[3 * i + 2];
  bool wide = false;
  // the node data of the thread's next column is loaded one column ahead (the
  // index clamped to the last node), so its latency falls on the current pair
  struct Node {
    double x0, x1, x2, n0, n1, n2, w;
    uint8_t bc;
  };
  auto node = [&](int j) {
    Node d;
    d.x0 = x[3 * j];
    d.x1 = x[3 * j + 1];
    d.x2 = x[3 * j + 2];
    d.n0 = nrm[3 * j];
    d.n1 = nrm[3 * j + 1];
    d.n2 = nrm[3 * j + 2];
    d.w = w[j];
    d.bc = bc[j];
    return d;
  };
  Node nx = node(min((int)threadIdx.x, p.n - 1));
  for (int j = threadIdx.x; j < p.n; j += kThreads) {
    const Node c = nx;
    nx = node(min(j + kThreads, p.n - 1));
    if (j == i) continue;
    const double dx = c.x0 - xi, dy = c.x1 - yi, dz = c.x2 - zi;
    const double njx = c.n0, njy = c.n1, njz = c.n2;
    double r, rinv;
    dist_and_inverse(dx * dx + dy * dy + dz * dz, r, rinv);
    const double wj = c.w;
    const double wq = wj * ((dx * njx + dy * njy + dz * njz) * (rinv * rinv * rinv));
    const double wr = wj * rinv;
    const double s0 = nix * dx + niy * dy + niz * dz;
    const double nn = nix * njx + niy * njy + niz * njz;
    const bool hard = c.bc == BEM_BC_HARD;
    if (PH != kPhWide) wide |= !(kmax * fmax(r, fabs(s0)) < kPhaseNear);
    pair_terms<KC, OUT128, WRITE_A, RHS, PH>(p, kc, j, hard, r, s0, wr, wq, nn, acc);
  }
  return wide;
}

// FIRST: the first pass over the right-hand sides (writes the diagonal and,
// STORE_A, the matrix row); later passes only form b.  RHS: b is formed
// (false only for a call without right-hand sides).
template <bool OUT128, bool FIRST, bool STORE_A, bool RHS>
__global__ __launch_bounds__(kThreads, 2) void assemble_kc_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const uint8_t* __restrict__ bc, const double* __restrict__ kv,
    int nk, int n_rhs, int rhs, const double2* __restrict__ y, void* __restrict__ A, int64_t ld,
    int64_t a_stride, double2* __restrict__ b, double2* __restrict__ diag64) {
  constexpr int KC = kKcAssemble, NW = kThreads / 64;
  static_assert(KC == 8, "the reduction sums 8 wavenumbers per wave");
  __shared__ double red[NW][6][KC];
  const int i = blockIdx.x;
  KChunk<KC> kc = load_chunk<KC>(kv, nk, nullptr);
  kc.dk = uniform_d(kc.dk);
  double kmax = 0.0;
#pragma unroll
  for (int q = 0; q < KC; ++q) kmax = fmax(kmax, fabs(kc.k[q]));
  const AsmRow p{n, n_rhs, rhs, i, (int)blockIdx.y * KC, y, A, ld, a_stride};
  double acc[KC][6];
#pragma unroll
  for (int q = 0; q < KC; ++q)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[q][c] = 0.0;
  constexpr bool WA = FIRST && STORE_A;
  bool wide;
  if (kc.uniform && kc.kc == KC)
    wide = row_terms<KC, OUT128, WA, RHS, kPhRec>(p, kc, kmax, x, nrm, w, bc, acc);
  else
    wide = row_terms<KC, OUT128, WA, RHS, kPhNear>(p, kc, kmax, x, nrm, w, bc, acc);
  // workgroup sums: per component c, the wave sums of the 8 wavenumbers by
  // recursive halving (lanes 8q..8q+7 end with wavenumber q), then the waves
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double v8[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) v8[q] = acc[q][c];
    const double v = wave_reduce8(v8);
    if ((lane & 7) == 0) red[wid][c][lane >> 3] = v;
  }
  if (__syncthreads_or(wide)) {
    // a phase of the row reaches past the near range: the row again, one
    // wavenumber at a time with the library sincos; its entries and sums
    // replace the first pass's
    for (int q = 0; q < kc.kc; ++q) {
      double a1[1][6] = {{0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
      KChunk<1> k1;
      k1.k[0] = kc.k[q];
      k1.dk = 0.0;
      k1.kc = 1;
      k1.uniform = false;
      AsmRow p1 = p;
      p1.q0 = p.q0 + q;
      (void)row_terms<1, OUT128, WA, RHS, kPhWide>(p1, k1, kmax, x, nrm, w, bc, a1);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double v = wave_sum(a1[0][c]);
        if (lane == 0) red[wid][c][q] = v;
      }
    }
  }
  __syncthreads();
  const int q = threadIdx.x;
  if (q < kc.kc) {
    double s[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      s[c] = 0.0;
#pragma unroll
      for (int v = 0; v < NW; ++v) s[c] += red[v][c][q];
    }
    const bool hard = bc[i] == BEM_BC_HARD;
    const int64_t kq = p.q0 + q;
    const double kval = kv[kq];   // (the psi sums were accumulated times k)
    const double2 mphi = make_double2(kFourPi - s[0], -s[1]);
    const double2 mpsi = make_double2(-s[2] / kval, -s[3] / kval);
    const double2 a = hard ? mphi : mpsi;
    const double2 bb = hard ? mpsi : mphi;
    if (FIRST) {
      if (STORE_A) {
        if (OUT128)
          reinterpret_cast<double2*>(A)[kq * a_stride + (int64_t)i * ld + i] = a;
        else
          reinterpret_cast<float2*>(A)[kq * a_stride + (int64_t)i * ld + i] =
              make_float2((float)a.x, (float)a.y);
      }
      if (diag64) {
        diag64[(kq * n + i) * 2] = mphi;
        diag64[(kq * n + i) * 2 + 1] = mpsi;
      }
    }
    if (RHS) {
      const double2 yy = y[(kq * n_rhs + rhs) * n + i];
      const double2 t = cmul(bb, yy);
      b[(kq * n_rhs + rhs) * n + i] = make_double2(-(s[4] + t.x), -(s[5] + t.y));
    }
  }
}

// r = -(M_phi phi + M_psi psi) for one row, a chunk of wavenumbers and one
// right-hand side, with (phi, psi) from the unknowns xs and data y.
__global__ __launch_bounds__(kThreads) void residual_kc_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const uint8_t* __restrict__ bc, const double* __restrict__ kv,
    int nk, int n_rhs, int rhs, const double2* __restrict__ y, const double2* __restrict__ xs,
    const double2* __restrict__ diag64, double2* __restrict__ r_out,
    const int32_t* __restrict__ kidx) {
  const int i = blockIdx.x;
  const KChunk<kKcResidual> kc = load_chunk<kKcResidual>(kv, nk, kidx);
  const int q0 = blockIdx.y * kKcResidual;
  int64_t kq_of[kKcResidual];
#pragma unroll
  for (int q = 0; q < kKcResidual; ++q) kq_of[q] = q < kc.kc ? (kidx ? kidx[q0 + q] : q0 + q) : 0;
  const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
  double acc[kKcResidual][2];
#pragma unroll
  for (int q = 0; q < kKcResidual; ++q) { acc[q][0] = 0.0; acc[q][1] = 0.0; }
  for (int j = threadIdx.x; j < n; j += kThreads) {
    if (j == i) continue;
    const double dx = x[3 * j] - xi, dy = x[3 * j + 1] - yi, dz = x[3 * j + 2] - zi;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double rinv = 1.0 / r;
    const double qn = (dx * nrm[3 * j] + dy * nrm[3 * j + 1] + dz * nrm[3 * j + 2]) * (rinv * rinv * rinv);
    const double wj = w[j];
    const bool hard = bc[j] == BEM_BC_HARD;
    Phase E;
    E.start(kc, r);
#pragma unroll
    for (int q = 0; q < kKcResidual; ++q) {
      if (q < kc.kc) {
        if (q > 0) E.next(kc, q, r);
        const double kr = kc.k[q] * r;
        const double2 G = make_double2(E.e.x * rinv, E.e.y * rinv);
        const double2 H = make_double2(qn * (-E.e.x - kr * E.e.y), qn * (kr * E.e.x - E.e.y));
        const int64_t o = (kq_of[q] * n_rhs + rhs) * n + j;
        const double2 u = xs[o], v = y[o];
        const double2 phi = hard ? u : v, psi = hard ? v : u;
        // -w H phi + w G psi
        acc[q][0] += wj * ((G.x * psi.x - G.y * psi.y) - (H.x * phi.x - H.y * phi.y));
        acc[q][1] += wj * ((G.x * psi.y + G.y * psi.x) - (H.x * phi.y + H.y * phi.x));
      }
    }
  }
  block_sum_2d(acc);
  if (threadIdx.x == 0) {
    const bool hard = bc[i] == BEM_BC_HARD;
#pragma unroll
    for (int q = 0; q < kKcResidual; ++q) {
      if (q >= kc.kc) break;
      const int64_t kq = kq_of[q];
      const double2 dphi = diag64[(kq * n + i) * 2];
      const double2 dpsi = diag64[(kq * n + i) * 2 + 1];
      const int64_t o = (kq * n_rhs + rhs) * n + i;
      const double2 u = xs[o], v = y[o];
      const double2 phi = hard ? u : v, psi = hard ? v : u;
      const double2 t1 = cmul(dphi, phi), t2 = cmul(dpsi, psi);
      r_out[o] = make_double2(-(acc[q][0] + t1.x + t2.x), -(acc[q][1] + t1.y + t2.y));
    }
  }
}

// ---------------------------------------------------------------- residual sweep
// r = b - A x with the float64 right-hand side b of the assembly, for one row
// i and every wavenumber of the launch per workgroup, for wavenumbers on an
// even grid k_q = k_0 + q dk (checked on the host).  Thread t holds the pairs
// (i, j) of its columns and carries e^{i k r_ij} and the step e^{i dk r_ij}
// in registers from one chunk of kSweepKc wavenumbers to the next; every
// kReanchor wavenumbers the phases start afresh from the stored k with
// sincos, which bounds the recurrence's rounding drift (about one rounding
// per step).  Only the coefficient of the unknown is formed (-w H for a hard
// node, w G for a soft one).  Chunk partial sums are reduced across the
// workgroup through a parity-double-buffered LDS array, one barrier per chunk.
constexpr int kSweepThreads = 256;
constexpr int kSweepKc = 4;
constexpr int kReanchor = 64;
constexpr int kSweepSlots = 6;   // columns per thread and part

// Part p = blockIdx.y covers the columns j = t + kSweepThreads (p JPT + s)
// and writes its sums to part_out[p]; residual_parts_kernel then forms
// r = b - a_ii x_i - (the sum of the parts).
template <int JPT>
__global__ __launch_bounds__(kSweepThreads) void residual_sweep_kernel(
    int n, const double* __restrict__ x, const double* __restrict__ nrm,
    const double* __restrict__ w, const uint8_t* __restrict__ bc, const double* __restrict__ kv,
    double dk, int nk, int n_rhs, int rhs, const double2* __restrict__ xs,
    double2* __restrict__ part_out) {
  constexpr int KC = kSweepKc, NW = kSweepThreads / 64;
  __shared__ double red[2][NW][KC][2];
  const int i = blockIdx.x, part = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int64_t plane = (int64_t)nk * n_rhs * n;
  // per slot: r, the coefficient of the unknown as E (ca + i k cb) (a soft node:
  // ca = w/r, cb = 0; a hard one: -w H = E (ca + i k cb) with ca = w (d.n)/r^3,
  // cb = -w (d.n)/r^2; all 0 for j = i and j >= n), the clamped column, and the
  // phase state
  double rr[JPT], ca[JPT], cb[JPT];
  int jj[JPT];
  double2 e[JPT], d[JPT];
  {
    const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
#pragma unroll
    for (int sl = 0; sl < JPT; ++sl) {
      const int j = t + (part * JPT + sl) * kSweepThreads;
      jj[sl] = min(j, n - 1);
      rr[sl] = 0.0;
      ca[sl] = 0.0;
      cb[sl] = 0.0;
      if (j < n && j != i) {
        const double dx = x[3 * j] - xi, dy = x[3 * j + 1] - yi, dz = x[3 * j + 2] - zi;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double rinv = 1.0 / r;
        rr[sl] = r;
        if (bc[j] == BEM_BC_HARD) {
          const double cf = -w[j] * (dx * nrm[3 * j] + dy * nrm[3 * j + 1] + dz * nrm[3 * j + 2]) *
                            (rinv * rinv * rinv);
          ca[sl] = -cf;
          cb[sl] = cf * r;
        } else {
          ca[sl] = w[j] * rinv;
        }
      }
    }
  }
  for (int c0 = 0, chunk = 0; c0 < nk; c0 += KC, ++chunk) {
    const int kc = min(KC, nk - c0);
    double kk[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) kk[q] = q < kc ? kv[c0 + q] : 0.0;
    const bool go_on = c0 % kReanchor != 0;
    double acc[KC][2];
#pragma unroll
    for (int q = 0; q < KC; ++q) { acc[q][0] = 0.0; acc[q][1] = 0.0; }
    {
      if (!go_on) {
        // fresh phases (grid start, a break of the grid, or re-anchoring)
#pragma clang loop unroll(full)
        for (int sl = 0; sl < JPT; ++sl) {
          double sn, cs;
          sincos(kk[0] * rr[sl], &sn, &cs);
          e[sl] = make_double2(cs, sn);
          sincos(dk * rr[sl], &sn, &cs);
          d[sl] = make_double2(cs, sn);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma clang loop unroll(full)
      for (int sl = 0; sl < JPT; ++sl) {
        double2 u[KC];
#pragma unroll
        for (int q = 0; q < KC; ++q)
          u[q] = xs[((int64_t)(q < kc ? c0 + q : c0) * n_rhs + rhs) * n + jj[sl]];
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          const double2 E = e[sl];
          e[sl] = cmul(e[sl], d[sl]);
          // the coefficient E (ca + i k cb): no select between the node kinds
          const double bk = cb[sl] * kk[q];
          const double ax = fma(E.x, ca[sl], -E.y * bk), ay = fma(E.x, bk, E.y * ca[sl]);
          acc[q][0] += ax * u[q].x - ay * u[q].y;
          acc[q][1] += ax * u[q].y + ay * u[q].x;
        }
        // keep the loads of one slot together (bounds the live registers)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    const int buf = chunk & 1;
    static_assert(KC * 2 == 8, "the chunk reduction sums 8 values per thread");
    {
      double v8[8];
#pragma unroll
      for (int q = 0; q < KC; ++q) { v8[2 * q] = acc[q][0]; v8[2 * q + 1] = acc[q][1]; }
      const double v = wave_reduce8(v8);
      if ((lane & 7) == 0) {
        const int idx = lane >> 3;   // value index q * 2 + c
        red[buf][wid][idx >> 1][idx & 1] = v;
      }
    }
    __syncthreads();
    // lane q stores wavenumber q's sum (stores only: no wave waits on memory
    // here); residual_parts_kernel forms r from the parts
    if (t < kc) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int v = 0; v < NW; ++v) { s0 += red[buf][v][t][0]; s1 += red[buf][v][t][1]; }
      const int64_t o = ((int64_t)(c0 + t) * n_rhs + rhs) * n + i;
      part_out[part * plane + o] = make_double2(s0, s1);
    }
  }
}

// r = b - a_ii x_i - (the sums of the parts), entry o = (k n_rhs + rhs) n + i
__global__ void residual_parts_kernel(int64_t plane, int nparts, int n, int n_rhs,
                                      const uint8_t* __restrict__ bc,
                                      const double2* __restrict__ diag64,
                                      const double2* __restrict__ xs,
                                      const double2* __restrict__ bvec,
                                      const double2* __restrict__ part_out,
                                      double2* __restrict__ r_out) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= plane) return;
  const int i = (int)(o % n);
  const int64_t kq = o / ((int64_t)n * n_rhs);
  const double2 aii = diag64[(kq * n + i) * 2 + (bc[i] == BEM_BC_HARD ? 0 : 1)];
  const double2 au = cmul(aii, xs[o]), bb = bvec[o];
  double sx = 0.0, sy = 0.0;
  for (int p = 0; p < nparts; ++p) {
    const double2 s = part_out[(int64_t)p * plane + o];
    sx += s.x;
    sy += s.y;
  }
  r_out[o] = make_double2(bb.x - (sx + au.x), bb.y - (sy + au.y));
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
  phase_sincos(ph, &sn, &cs);
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
  const int kmax = 65535 * kKcAssemble;
  for (int k0 = 0; k0 < n_k; k0 += kmax) {
    const int nk = std::min(kmax, n_k - k0);
    dim3 grid(s->n, (nk + kKcAssemble - 1) / kKcAssemble);
    const double2* yk = reinterpret_cast<const double2*>(y) + (int64_t)k0 * n_rhs * s->n;
    double2* bk = reinterpret_cast<double2*>(b) + (int64_t)k0 * n_rhs * s->n;
    double2* dk = diag64 ? reinterpret_cast<double2*>(diag64) + (int64_t)k0 * s->n * 2 : nullptr;
    const size_t esz = prec == BEM_C128 ? 16 : 8;
    void* Ak = A ? reinterpret_cast<char*>(A) + (int64_t)k0 * a_stride * esz : nullptr;
    for (int r = 0; r < std::max(n_rhs, 1); ++r) {
      const bool first = r == 0;
      const int pi = prof_begin(ctx, "assemble");
#define BEM_ASM(O, F, S, R)                                                                       \
  hipLaunchKernelGGL((assemble_kc_kernel<O, F, S, R>), grid, dim3(kThreads), 0, ctx->stream,      \
                     s->n, s->x, s->nrm, s->w, s->bc, k + k0, nk, n_rhs, r, yk, Ak, ld, a_stride, \
                     bk, dk)
      const bool c128 = prec == BEM_C128;
      if (!first) {
        if (c128) BEM_ASM(true, false, false, true); else BEM_ASM(false, false, false, true);
      } else if (n_rhs == 0) {
        // no right-hand side: the diagonal (and the matrix) only
        if (Ak) {
          if (c128) BEM_ASM(true, true, true, false); else BEM_ASM(false, true, true, false);
        } else {
          if (c128) BEM_ASM(true, true, false, false); else BEM_ASM(false, true, false, false);
        }
      } else if (Ak) {
        if (c128) BEM_ASM(true, true, true, true); else BEM_ASM(false, true, true, true);
      } else {
        if (c128) BEM_ASM(true, true, false, true); else BEM_ASM(false, true, false, true);
      }
#undef BEM_ASM
      // node pairs evaluated; bytes: matrix written (first pass) + b written
      const double pairs = (double)s->n * s->n * nk;
      prof_end(ctx, "assemble", pi, pairs,
               (first && A ? (double)esz * s->n * s->n * nk : 0.0) + (n_rhs ? 16.0 * s->n * nk : 0.0));
      BEM_CHECK_LAUNCH(ctx);
    }
  }
  return BEM_OK;
}

bem_status launch_residual(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k,
                           int n_rhs, const void* y, const void* x, const void* diag64, void* r,
                           const int32_t* kidx, int n_sel) {
  if (kidx) {
    // a selected subset of the n_k wavenumbers, evaluated in place
    if (n_sel <= 0) return BEM_OK;
    if (n_sel > 65535 * kKcResidual)
      return fail(ctx, BEM_EUNSUPPORTED, "residual: %d selected wavenumbers in one call", n_sel);
    dim3 grid(s->n, (n_sel + kKcResidual - 1) / kKcResidual);
    for (int rh = 0; rh < n_rhs; ++rh) {
      const int pi = prof_begin(ctx, "residual");
      hipLaunchKernelGGL(residual_kc_kernel, grid, dim3(kThreads), 0, ctx->stream, s->n, s->x,
                         s->nrm, s->w, s->bc, k, n_sel, n_rhs, rh,
                         reinterpret_cast<const double2*>(y), reinterpret_cast<const double2*>(x),
                         reinterpret_cast<const double2*>(diag64), reinterpret_cast<double2*>(r),
                         kidx);
      prof_end(ctx, "residual", pi, (double)s->n * s->n * n_sel, 48.0 * s->n * n_sel);
      BEM_CHECK_LAUNCH(ctx);
    }
    return BEM_OK;
  }
  const int kmax = 65535 * kKcResidual;
  for (int k0 = 0; k0 < n_k; k0 += kmax) {
    const int nk = std::min(kmax, n_k - k0);
    dim3 grid(s->n, (nk + kKcResidual - 1) / kKcResidual);
    const int64_t off = (int64_t)k0 * n_rhs * s->n;
    for (int rh = 0; rh < n_rhs; ++rh) {
      const int pi = prof_begin(ctx, "residual");
      hipLaunchKernelGGL(residual_kc_kernel, grid, dim3(kThreads), 0, ctx->stream, s->n, s->x,
                         s->nrm, s->w, s->bc, k + k0, nk, n_rhs, rh,
                         reinterpret_cast<const double2*>(y) + off,
                         reinterpret_cast<const double2*>(x) + off,
                         reinterpret_cast<const double2*>(diag64) + (int64_t)k0 * s->n * 2,
                         reinterpret_cast<double2*>(r) + off, nullptr);
      prof_end(ctx, "residual", pi, (double)s->n * s->n * nk, 48.0 * s->n * nk);
      BEM_CHECK_LAUNCH(ctx);
    }
  }
  return BEM_OK;
}

double even_grid_step(const double* k, int n_k) {
  if (n_k < 2) return 0.0;
  const double dk = (k[n_k - 1] - k[0]) / (n_k - 1);
  if (!(dk > 0.0)) return 0.0;
  for (int q = 0; q < n_k; ++q)
    if (!(std::fabs(k[q] - (k[0] + q * dk)) <= 4e-16 * std::fabs(k[q]))) return 0.0;
  return dk;
}

// r = b - A x through the sweep kernel: ceil(N / 1536) parts per row, the
// partial sums of parts past the first staged in `parts` (residual_parts_bytes);
// surfaces under 1024 nodes and wavenumbers off an even grid (dk <= 0) take
// residual_kc_kernel with the known data y.
int residual_parts(int n) { return (n + kSweepSlots * kSweepThreads - 1) / (kSweepSlots * kSweepThreads); }

size_t residual_parts_bytes(int n, int n_k, int n_rhs) {
  if (n < 1024) return 0;
  return (size_t)residual_parts(n) * n_k * n_rhs * n * 16;
}

bem_status launch_residual_b(bem_ctx* ctx, const bem_surface* s, int n_k, const double* k,
                             double dk, int n_rhs, const void* y, const void* b, const void* x,
                             const void* diag64, void* r, void* parts) {
  if (s->n < 1024 || !(dk > 0.0)) return launch_residual(ctx, s, n_k, k, n_rhs, y, x, diag64, r);
  const int np = residual_parts(s->n);
  if (np > 65535 || !parts)
    return fail(ctx, BEM_EINVAL, "residual: %d parts need a staging buffer", np);
  const int64_t plane = (int64_t)n_k * n_rhs * s->n;
  const int pi = prof_begin(ctx, "residual");
  for (int rh = 0; rh < n_rhs; ++rh)
    hipLaunchKernelGGL((residual_sweep_kernel<kSweepSlots>), dim3(s->n, np), dim3(kSweepThreads), 0,
                       ctx->stream, s->n, s->x, s->nrm, s->w, s->bc, k, dk, n_k, n_rhs, rh,
                       reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(parts));
  hipLaunchKernelGGL(residual_parts_kernel, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0,
                     ctx->stream, plane, np, s->n, n_rhs, s->bc,
                     reinterpret_cast<const double2*>(diag64), reinterpret_cast<const double2*>(x),
                     reinterpret_cast<const double2*>(b), reinterpret_cast<const double2*>(parts),
                     reinterpret_cast<double2*>(r));
  // one complex multiply-add per pair; x read once per pair from L2
  prof_end(ctx, "residual", pi, 8.0 * s->n * s->n * (double)n_k * n_rhs,
           16.0 * s->n * s->n * (double)n_k * n_rhs);
  BEM_CHECK_LAUNCH(ctx);
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
