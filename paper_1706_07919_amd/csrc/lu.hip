// Batched dense complex LU with partial pivoting and triangular solves for the
// direct solve of the discrete system at each wavenumber (Sec. IV A).
// Matrices are row-major (element (i,j) at
// i*ld + j), so row interchanges touch contiguous memory.
//
// Factorisation = recursion over column ranges (left half, swaps, triangular
// solve, trailing complex GEMM, right half); the leaves are panels of a few
// columns held in registers by one workgroup per matrix.  The trailing updates
// carry all O(n^3) work and run on MFMA: float32 complex products as real
// products of the interleaved operands (4M) accumulated in float32, float64
// complex products on the f64 MFMA.
#include <algorithm>
#include <climits>

#include <type_traits>

#include "common.h"

namespace bem {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Pointers into the matrices are qualified with the global address space so
// that loads and stores compile to global (not flat) memory instructions: flat
// accesses also count against the LDS wait counter and would make every LDS
// wait in the GEMM loop wait for the global prefetch as well.  (The qualifier
// only exists in the device pass; the host pass sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL __attribute__((address_space(1)))
#define LDS_AS __attribute__((address_space(3)))
#else
#define GLOBAL
#define LDS_AS
#endif

template <typename R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

template <typename C> __device__ inline C cmk(decltype(C::x) a, decltype(C::x) b) {
  C c; c.x = a; c.y = b; return c;
}
template <typename C> __device__ inline C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ inline C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
// s - a b as four fused multiply-adds (one rounding per real product-sum
// instead of a rounded product then a subtraction)
template <typename C> __device__ inline C cfms(C s, C a, C b) {
  return cmk<C>(fma(-a.x, b.x, fma(a.y, b.y, s.x)), fma(-a.x, b.y, fma(-a.y, b.x, s.y)));
}
template <typename C> __device__ inline C crecip(C a) {
  // 1/a with scaling to avoid overflow (Smith's method)
  using R = decltype(C::x);
  if (fabs(a.x) >= fabs(a.y)) {
    R t = a.y / a.x, d = a.x + a.y * t;
    return cmk<C>(R(1) / d, -t / d);
  } else {
    R t = a.x / a.y, d = a.y + a.x * t;
    return cmk<C>(t / d, R(-1) / d);
  }
}

// ============================================================== matrix groups
// The matrices of one launch come in up to kMaxGroups size classes (uneven
// batches: bodies of different node counts, each with many wavenumbers).  The
// table travels by value in the kernel arguments; the flattened matrix index
// of a workgroup selects its group, and every range is clipped to the group's
// own n, so one recursion over the largest n factors every matrix.
constexpr int kMaxGroups = 8;
struct LuGroup {
  void* A;          // matrix 0 of the group (row-major, element type of the launch)
  int32_t* piv;     // [count][n]
  int32_t* info;    // [count]
  int64_t ld;       // leading dimension (elements)
  int64_t stride;   // elements between consecutive matrices
  int n;
  int count;
};
struct LuGroups {
  LuGroup g[kMaxGroups];
  int ng;
};

// q: flattened matrix index -> its group (copied out) and index li inside it.
// Both loops run over constant indices and copy field by field, so the table
// is read with uniform loads from the kernel arguments (a dynamic index or a
// whole-struct copy would place the table in scratch memory).
__device__ inline bool locate(const LuGroups& G, int q, LuGroup& out, int& li) {
  int sel = -1;
#pragma unroll
  for (int i = 0; i < kMaxGroups; ++i) {
    if (sel < 0 && i < G.ng) {
      if (q < G.g[i].count) { sel = i; li = q; }
      else q -= G.g[i].count;
    }
  }
  if (sel < 0) return false;
#pragma unroll
  for (int i = 0; i < kMaxGroups; ++i)
    if (i == sel) {
      out.A = G.g[i].A;
      out.piv = G.g[i].piv;
      out.info = G.g[i].info;
      out.ld = G.g[i].ld;
      out.stride = G.g[i].stride;
      out.n = G.g[i].n;
      out.count = G.g[i].count;
    }
  return true;
}

// matrix b of a group, as a global pointer
template <typename C> __device__ inline GLOBAL C* gmat(const LuGroup& g, int b) {
  return (GLOBAL C*)g.A + (int64_t)b * g.stride;
}

// ============================================================== base panel
// Factor columns [c0, c0+w) of rows [c0, n) in place; w <= W.  Thread t owns
// rows c0 + t + q*NT (q < RPT).  Pivot = max |re|+|im| (lowest row on ties).
constexpr int kPanelThreads = 512;

template <typename R, int W, int RPT>
__global__ __launch_bounds__(kPanelThreads) void panel_kernel(LuGroups G, int c0, int w_all) {
  using C = typename Cx<R>::T;
  constexpr int NT = kPanelThreads, NW = NT / 64;
  // pivot and top rows are double-buffered by column parity, so one column's
  // readers never race the next column's writers; two barriers per column
  __shared__ C pivrow[2][W];
  __shared__ C toprow[2][W];
  __shared__ R rv[NW];
  __shared__ int ri[NW];
  LuGroup grp;
  int b = 0;
  if (!locate(G, blockIdx.x, grp, b)) return;
  const int n = grp.n;
  const int64_t ld = grp.ld;
  if (c0 >= n) return;
  const int w = min(w_all, n - c0);
  GLOBAL C* Ab = gmat<C>(grp, b);
  GLOBAL int32_t* piv = (GLOBAL int32_t*)grp.piv;
  GLOBAL int32_t* info = (GLOBAL int32_t*)grp.info;
  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  C a[RPT][W];
  // full-width panels with 16-byte aligned rows move whole rows as 16-byte
  // words; rows past n are read clamped and zeroed, never stored
  const bool vec = w == W && (sizeof(C) == 16 || ((ld | c0) & 1) == 0);
  if (vec) {
    constexpr int PER = 16 / sizeof(C);   // complex values per 16-byte word
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + t + q * NT;
      const GLOBAL uint4* src = (const GLOBAL uint4*)(Ab + (int64_t)min(r, n - 1) * ld + c0);
      uint4 v[W / PER];
#pragma unroll
      for (int m = 0; m < W / PER; ++m) v[m] = src[m];
#pragma unroll
      for (int m = 0; m < W / PER; ++m) {
        C e[PER];
        __builtin_memcpy(e, &v[m], 16);
#pragma unroll
        for (int u = 0; u < PER; ++u) a[q][m * PER + u] = r < n ? e[u] : cmk<C>(R(0), R(0));
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + t + q * NT;
#pragma unroll
      for (int c = 0; c < W; ++c)
        a[q][c] = (r < n && c < w) ? Ab[(int64_t)r * ld + c0 + c] : cmk<C>(R(0), R(0));
    }
  }
  // The column loop is unrolled so that every register index is static.  Row
  // c0 + c is held by thread c in slot 0; a row r > c0 + c is below the
  // diagonal unless it sits in slot 0 of a thread t <= c.
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (c >= w) break;
    const int pr = c0 + c;
    const int buf = c & 1;
    // candidate of this thread, then of its wave
    R best = R(-1);
    int bidx = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + t + q * NT;
      const R m = fabs(a[q][c].x) + fabs(a[q][c].y);
      if ((q > 0 || t >= c) && r < n && m > best) { best = m; bidx = r; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const R ob = __shfl_down(best, off, 64);
      const int oi = __shfl_down(bidx, off, 64);
      if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
    }
    if (lane == 0) { rv[wid] = best; ri[wid] = bidx; }
    __syncthreads();
    // every thread reduces the wave partials (same order, same result)
    R bb = rv[0];
    int bi = ri[0];
#pragma unroll
    for (int q = 1; q < NW; ++q)
      if (rv[q] > bb || (rv[q] == bb && ri[q] < bi)) { bb = rv[q]; bi = ri[q]; }
    const bool singular = !(bb > R(0));   // exactly zero (or NaN) column: no interchange
    const int p = singular ? pr : bi;
    if (t == 0) {
      if (singular && info[b] == 0) info[b] = pr + 1;
      piv[(int64_t)b * n + pr] = p;
    }
    // the owners of rows p and pr publish them
    const int op = (p - c0) % NT, qp = (p - c0) / NT;
    if (t == op) {
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (q == qp)
#pragma unroll
          for (int cc = 0; cc < W; ++cc) pivrow[buf][cc] = a[q][cc];
    }
    if (t == c && p != pr)
#pragma unroll
      for (int cc = 0; cc < W; ++cc) toprow[buf][cc] = a[0][cc];
    __syncthreads();
    if (p != pr) {
      if (t == op) {
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (q == qp)
#pragma unroll
            for (int cc = 0; cc < W; ++cc) a[q][cc] = toprow[buf][cc];
      }
      if (t == c)
#pragma unroll
        for (int cc = 0; cc < W; ++cc) a[0][cc] = pivrow[buf][cc];
    }
    if (!singular) {
      C u[W];
#pragma unroll
      for (int cc = c; cc < W; ++cc) u[cc] = pivrow[buf][cc];
      const C inv = crecip(u[c]);
      // rows past n hold zeros and are never stored
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (q == 0 && t <= c) continue;
        const C l = cmul(a[q][c], inv);
        a[q][c] = l;
#pragma unroll
        for (int cc = c + 1; cc < W; ++cc) a[q][cc] = cfms(a[q][cc], l, u[cc]);
      }
    }
  }
  if (vec) {
    constexpr int PER = 16 / sizeof(C);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + t + q * NT;
      if (r < n) {
        GLOBAL uint4* dst = (GLOBAL uint4*)(Ab + (int64_t)r * ld + c0);
#pragma unroll
        for (int m = 0; m < W / PER; ++m) {
          uint4 v;
          __builtin_memcpy(&v, &a[q][m * PER], 16);
          dst[m] = v;
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + t + q * NT;
      if (r < n)
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c < w) Ab[(int64_t)r * ld + c0 + c] = a[q][c];
    }
  }
}

// ============================================================== row swaps
// Interchanges t <-> piv[t] for t in [r0, r1) (r1 - r0 <= kSwapRows), applied
// in order to the columns [ca0, ca1) and [cb0, cb1), all clipped to each
// matrix's n.  One workgroup per (matrix, strip of LW columns).
//
// The composition is formed on row indices in parallel.  Since piv[t] >= t,
// position t is final after step t, and its content just before step t is
// c(t) = c(u) for the last earlier step u with piv[u] = t, else row t itself;
// c follows by pointer jumping over those parent links.  The final content of
// position t is then c(t) if piv[t] = t, else the content of piv[t] before
// step t: c(q) for the last earlier step q with the same target, else row
// piv[t].  A row below r1 ends holding c(u) of the last step u that targets
// it.  The touched rows are then gathered into LDS and scattered back.
constexpr int kSwapRows = 256;

template <typename C, int LW>
__global__ __launch_bounds__(256) void laswp_kernel(LuGroups G, int r0, int r1_all, int ca0,
                                                    int ca1_all, int cb0, int cb1_all) {
  __shared__ int P[kSwapRows];
  __shared__ int root[kSwapRows];
  __shared__ int dst[2 * kSwapRows], src[2 * kSwapRows];
  __shared__ int npair, any;
  __shared__ C buf[2 * kSwapRows][LW];
  LuGroup grp;
  int b = 0;
  if (!locate(G, blockIdx.y, grp, b)) return;
  const int n = grp.n;
  const int64_t ld = grp.ld;
  const int r1 = min(r1_all, n);
  if (r1 <= r0) return;
  const int ca1 = min(ca1_all, n), cb1 = min(cb1_all, n);
  const int na = max(0, ca1 - ca0), nbc = max(0, cb1 - cb0);
  const int s0 = blockIdx.x * LW;
  if (s0 >= na + nbc) return;
  const int L = r1 - r0;
  const int tid = threadIdx.x;
  GLOBAL C* Ab = gmat<C>(grp, b);
  const GLOBAL int32_t* pb = (const GLOBAL int32_t*)grp.piv + (int64_t)b * n;
  if (tid == 0) { npair = 0; any = 0; }
  __syncthreads();
  int p = 0;
  if (tid < L) {
    p = pb[r0 + tid];
    P[tid] = p;
    root[tid] = -1;
    if (p != r0 + tid) any = 1;
  }
  __syncthreads();
  if (!any) return;
  // parent links: the last earlier step whose target is this position
  if (tid < L && p != r0 + tid && p < r1) atomicMax(&root[p - r0], tid);
  __syncthreads();
  if (tid < L && root[tid] < 0) root[tid] = tid;
  __syncthreads();
  // pointer jumping to the chain roots (root[i] == i marks a root)
  for (int it = 0; it < 9; ++it) {
    int rr = 0;
    if (tid < L) rr = root[root[tid]];
    __syncthreads();
    if (tid < L) root[tid] = rr;
    __syncthreads();
  }
  if (tid < L) {
    const int i = tid;
    int q = -1;
    bool last = true;
    for (int u = 0; u < L; ++u) {
      const int pu = P[u];
      if (pu == p && u != i) {
        if (u < i) q = u;
        else last = false;
      }
    }
    const int s = p == r0 + i ? r0 + root[i] : (q >= 0 ? r0 + root[q] : p);
    if (s != r0 + i) {
      const int k = atomicAdd(&npair, 1);
      dst[k] = r0 + i;
      src[k] = s;
    }
    if (p >= r1 && last) {
      const int k = atomicAdd(&npair, 1);
      dst[k] = p;
      src[k] = r0 + root[i];
    }
  }
  __syncthreads();
  const int m = npair;
  // gather the source rows of this strip, then scatter them to their destinations
  for (int e = tid; e < m * LW; e += 256) {
    const int k = e / LW, j = e % LW, v = s0 + j;
    if (v < na + nbc) {
      const int col = v < na ? ca0 + v : cb0 + (v - na);
      buf[k][j] = Ab[(int64_t)src[k] * ld + col];
    }
  }
  __syncthreads();
  for (int e = tid; e < m * LW; e += 256) {
    const int k = e / LW, j = e % LW, v = s0 + j;
    if (v < na + nbc) {
      const int col = v < na ? ca0 + v : cb0 + (v - na);
      Ab[(int64_t)dst[k] * ld + col] = buf[k][j];
    }
  }
}

// ============================================================== small TRSM
// X = L^{-1} B, L = unit lower triangle of rows/cols [r0, r0+m1) (m1 <= 32),
// B = rows [r0, r0+m1) x cols [col0, col0+ncol); one column per thread.
template <typename C>
__global__ __launch_bounds__(256) void trsm_kernel(LuGroups G, int r0, int m1_all, int col0,
                                                   int col1) {
  __shared__ C L[32][33];
  LuGroup grp;
  int b = 0;
  if (!locate(G, blockIdx.y, grp, b)) return;
  const int n = grp.n;
  const int64_t ld = grp.ld;
  const int m1 = min(m1_all, n - r0);
  if (m1 <= 1) return;
  GLOBAL C* Ab = gmat<C>(grp, b);
  for (int e = threadIdx.x; e < m1 * m1; e += blockDim.x) {
    const int i = e / m1, j = e % m1;
    L[i][j] = Ab[(int64_t)(r0 + i) * ld + r0 + j];
  }
  __syncthreads();
  const int col = col0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= min(col1, n)) return;
  C x[32];
  // rows past m1 are read clamped and never stored, so the loads and stores
  // carry no per-row branches
#pragma unroll
  for (int i = 0; i < 32; ++i) x[i] = Ab[(int64_t)(r0 + min(i, m1 - 1)) * ld + col];
#pragma unroll
  for (int i = 1; i < 32; ++i) {
    if (i < m1) {
      C s = x[i];
#pragma unroll
      for (int j = 0; j < 32; ++j)
        if (j < i) s = cfms(s, L[i][j], x[j]);
      x[i] = s;
    }
  }
  if (m1 == 32) {
#pragma unroll
    for (int i = 1; i < 32; ++i) Ab[(int64_t)(r0 + i) * ld + col] = x[i];
  } else {
#pragma unroll
    for (int i = 1; i < 32; ++i)
      if (i < m1) Ab[(int64_t)(r0 + i) * ld + col] = x[i];
  }
}

// ============================================================== GEMM f32 (4M)
// C[M x N] -= A[M x K] B[K x N] for complex float, each operand a row-major
// block of the same matrix.  128 x 128 tile per workgroup of 4 waves (2 x 2),
// each wave 64 x 64 as 2 x 2 MFMA 32x32x2 blocks with separate real and
// imaginary accumulators.  With the interleaved A row viewed as a real row of
// length 2K, Re C = A_real . [Re B; -Im B], Im C = A_real . [Im B; Re B].
constexpr int G32_BM = 128, G32_BN = 128, G32_BK = 8;
constexpr int G32_APAD = 8;

// Operands of one workgroup's matrix: C = rows [rowC, min(rowEnd, n)) x cols
// [colC, min(colEnd, n)), A = same rows x cols [colA, colA+K), B = rows
// [rowB, rowB+K) x C's cols.
template <typename C>
struct GemmView {
  const GLOBAL C* A;
  const GLOBAL C* B;
  GLOBAL C* Cm;
  int64_t ld;
  int M, N;
};

template <typename C>
__device__ inline bool gemm_view(const LuGroups& G, int rowC, int colC, int colA, int rowB,
                                 int rowEnd, int colEnd, GemmView<C>& v) {
  LuGroup grp;
  int b = 0;
  if (!locate(G, blockIdx.y, grp, b)) return false;
  v.ld = grp.ld;
  v.M = min(rowEnd, grp.n) - rowC;
  v.N = min(colEnd, grp.n) - colC;
  GLOBAL C* base = gmat<C>(grp, b);
  v.A = base + (int64_t)rowC * v.ld + colA;
  v.B = base + (int64_t)rowB * v.ld + colC;
  v.Cm = base + (int64_t)rowC * v.ld + colC;
  return v.M > 0 && v.N > 0;
}

__global__ __launch_bounds__(256, 2) void gemm_c32_kernel(LuGroups G, int rowC, int colC, int colA,
                                                       int rowB, int rowEnd, int colEnd, int K,
                                                       int tiles_n) {
  __shared__ float As[2][G32_BK][2 * G32_BM + G32_APAD];
  __shared__ float Bs1[2][G32_BK][2 * G32_BN];
  __shared__ float Bs2[2][G32_BK][2 * G32_BN];
  GemmView<float2> gv;
  if (!gemm_view(G, rowC, colC, colA, rowB, rowEnd, colEnd, gv)) return;
  const int tile = blockIdx.x;
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  const int m0 = tm * G32_BM, n0 = tn * G32_BN;
  const int M = gv.M, N = gv.N;
  if (m0 >= M || n0 >= N) return;
  const int64_t ld = gv.ld;
  const GLOBAL float2* A = gv.A;
  const GLOBAL float2* B = gv.B;
  GLOBAL float2* C = gv.Cm;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int h = lane >> 5, l32 = lane & 31;

  floatx16 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) { acc_re[i][j][v] = 0.f; acc_im[i][j][v] = 0.f; }

  float2 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int row = e >> 3, kk = e & 7;
      const int gr = m0 + row, gk = k0 + kk;
      const bool oka = gr < M && gk < K;
      const float2 va = A[oka ? (int64_t)gr * ld + gk : 0];
      ra[q] = oka ? va : make_float2(0.f, 0.f);
      const int brow = e >> 7, bcol = e & 127;
      const int gbk = k0 + brow, gbc = n0 + bcol;
      const bool okb = gbk < K && gbc < N;
      const float2 vb = B[okb ? (int64_t)gbk * ld + gbc : 0];
      rb[q] = okb ? vb : make_float2(0.f, 0.f);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int row = e >> 3, kk = e & 7;
      As[buf][kk][row] = ra[q].x;
      As[buf][kk][G32_BM + row] = ra[q].y;
      const int brow = e >> 7, bcol = e & 127;
      Bs1[buf][brow][bcol] = rb[q].x;
      Bs1[buf][brow][G32_BN + bcol] = -rb[q].y;
      Bs2[buf][brow][bcol] = rb[q].y;
      Bs2[buf][brow][G32_BN + bcol] = rb[q].x;
    }
  };

  const int nk = (K + G32_BK - 1) / G32_BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * G32_BK);
#pragma unroll
    for (int k = 0; k < G32_BK; ++k) {
      float a[2], b1[2], b2[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[cur][k][h * G32_BM + wm * 64 + i * 32 + l32];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        b1[j] = Bs1[cur][k][h * G32_BN + wn * 64 + j * 32 + l32];
        b2[j] = Bs2[cur][k][h * G32_BN + wn * 64 + j * 32 + l32];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b1[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b2[j], acc_im[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + l32;
      if (col >= N) continue;
      // all loads of the block first (one wait), then the stores
      float2 c[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        c[v] = C[(int64_t)min(row, M - 1) * ld + col];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < M)
          C[(int64_t)row * ld + col] = make_float2(c[v].x - acc_re[i][j][v], c[v].y - acc_im[i][j][v]);
      }
    }
}

// ============================================================== GEMM f32 (3M)
// The same update with three real products per complex product:
//   T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi);  Re C -= T1 - T2,
//   Im C -= T3 - T1 - T2.
// Each MFMA 32x32x2 covers two complex k of one product, so a complex k costs
// 1.5 MFMA per 32x32 block instead of 2 (4M).  The operand sums are formed
// once while staging the tiles in LDS.
__global__ __launch_bounds__(256) void gemm_c32_3m_kernel(LuGroups G, int rowC, int colC,
                                                          int colA, int rowB, int rowEnd,
                                                          int colEnd, int K, int tiles_n) {
  __shared__ float As[2][3][G32_BK][G32_BM + 4];
  __shared__ float Bs[2][3][G32_BK][G32_BN + 4];
  GemmView<float2> gv;
  if (!gemm_view(G, rowC, colC, colA, rowB, rowEnd, colEnd, gv)) return;
  const int tile = blockIdx.x;
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  const int m0 = tm * G32_BM, n0 = tn * G32_BN;
  const int M = gv.M, N = gv.N;
  if (m0 >= M || n0 >= N) return;
  const int64_t ld = gv.ld;
  const GLOBAL float2* A = gv.A;
  const GLOBAL float2* B = gv.B;
  GLOBAL float2* C = gv.Cm;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int h = lane >> 5, l32 = lane & 31;

  floatx16 acc[3][2][2];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[p][i][j][v] = 0.f;

  float2 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int row = e >> 3, kk = e & 7;
      const int gr = m0 + row, gk = k0 + kk;
      const bool oka = gr < M && gk < K;
      const float2 va = A[oka ? (int64_t)gr * ld + gk : 0];
      ra[q] = oka ? va : make_float2(0.f, 0.f);
      const int brow = e >> 7, bcol = e & 127;
      const int gbk = k0 + brow, gbc = n0 + bcol;
      const bool okb = gbk < K && gbc < N;
      const float2 vb = B[okb ? (int64_t)gbk * ld + gbc : 0];
      rb[q] = okb ? vb : make_float2(0.f, 0.f);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int row = e >> 3, kk = e & 7;
      As[buf][0][kk][row] = ra[q].x;
      As[buf][1][kk][row] = ra[q].y;
      As[buf][2][kk][row] = ra[q].x + ra[q].y;
      const int brow = e >> 7, bcol = e & 127;
      Bs[buf][0][brow][bcol] = rb[q].x;
      Bs[buf][1][brow][bcol] = rb[q].y;
      Bs[buf][2][brow][bcol] = rb[q].x + rb[q].y;
    }
  };

  const int nk = (K + G32_BK - 1) / G32_BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * G32_BK);
#pragma unroll
    for (int k = 0; k < G32_BK; k += 2) {
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[cur][p][k + h][wm * 64 + i * 32 + l32];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[cur][p][k + h][wn * 64 + j * 32 + l32];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[p][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[p][i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + l32;
      if (col >= N) continue;
      float2 c[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        c[v] = C[(int64_t)min(row, M - 1) * ld + col];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const float t1 = acc[0][i][j][v], t2 = acc[1][i][j][v], t3 = acc[2][i][j][v];
        if (row < M)
          C[(int64_t)row * ld + col] = make_float2(c[v].x - (t1 - t2), c[v].y - (t3 - t1 - t2));
      }
    }
}

// ============================================================== GEMM f32, operands streamed into LDS
// The complex update C -= A B on MFMA 32x32x2 f32 for the float32
// factorisation, as three real products (3M: T1 = Ar Br, T2 = Ai Bi,
// T3 = (Ar + Ai)(Br + Bi); Re C -= T1 - T2, Im C -= T3 - T1 - T2) or four (4M:
// the interleaved real row of A against [Re B; -Im B] and [Im B; Re B]).
//
// * Operands go from global memory straight into LDS (global_load_lds, one
//   16-byte word per lane, no staging registers), 16 complex k per stage, one
//   stage in flight while the previous one is multiplied.  A keeps its
//   row-major interleaved layout: 128 bytes per tile row and stage, the eight
//   16-byte words of row r stored at positions permuted by r mod 8 so that
//   the 32 rows an MFMA block reads hit distinct banks.  B rows are stored as
//   they are (consecutive lanes read consecutive columns).
// * Edges: rows past M and columns past N load clamped addresses and are never
//   stored, and a wave skips the MFMAs of its 32 x 32 blocks that lie wholly
//   past the edge (the partial tile row and column of an update whose size is
//   not a multiple of 128: at n = 5124 every trailing update has a 4-wide
//   one); depth past K (the last stage when K is not a multiple of 16) is
//   zeroed on the way from LDS to the MFMA operands.
// * Work list: every (matrix, tile) pair of the launch, over all size classes
//   (each with its own tile counts), in matrix order, cut into eight
//   contiguous ranges; range x runs on XCD x (workgroup w is dispatched to
//   XCD w mod 8).  Tiles sharing an A or a B panel therefore read it through
//   one XCD's L2, and in a large batch every matrix stays on one XCD.  Inside
//   a matrix, tiles are walked in strips of GL_GM tile rows, column by column,
//   odd strips from the last column back.  With 64 tiles in flight per XCD a
//   strip of 4 rows keeps its four A panels (2 MB at K = 512) in the 4 MB L2
//   while the B panels stream past, each read once per strip: measured L2
//   fetches 1.48x the algorithmic bytes against 1.68x for strips of 8 (whose
//   A panels do not survive) and 1.98x for 16.
// * Tile 128 x BN (BN = 64 WJ) per workgroup of 4 waves (2 x 2), each wave
//   64 x 32 WJ as 2 x WJ MFMA blocks.
// * Launch forms: one workgroup per tile, or (queue != NULL) a persistent
//   grid of the resident workgroups in which the workgroups of range x take
//   its tiles in turn from range x's counter in `queue` (an atomic ticket per
//   tile); the last workgroup of a range to find it empty resets the range's
//   counters for the next launch.
constexpr int GL_BM = 128, GL_BK = 16, GL_GM = 4;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Work list of one launch: group g owns items [start[g], start[g + 1]), each
// item one tile of one of its matrices (tm[g] x tn[g] tiles per matrix).
struct GemmList {
  int64_t start[kMaxGroups + 1];
  int tm[kMaxGroups], tn[kMaxGroups];
};

// One 16-byte word per lane from global memory straight into LDS at
// lds_wave + 16 * lane (lds_wave wave-uniform, in M0).  The compiler does not
// order these loads against later LDS reads; the kernels using it wait on the
// load counter themselves before each barrier.
__device__ inline void lds_dma16(const GLOBAL u32x4* src, unsigned lds_wave) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off"
               :: "v"(src), "s"(lds_wave) : "memory", "m0");
}

// One tile (work item `item` < the list's total) of the update.
template <bool M3, int WJ>
__device__ __forceinline__ void gemm_lds_tile(const LuGroups& G, const GemmList& W, int64_t item,
                                              int rowC, int colC, int colA, int rowB, int rowEnd,
                                              int colEnd, int K, u32x4 (*As)[GL_BM * GL_BK / 2],
                                              u32x4 (*Bs)[GL_BK * 64 * WJ / 2]) {
  constexpr int BN = 64 * WJ;
  constexpr int BW = GL_BK * BN / 2;            // 16-byte words of a B stage
  // ---- work item -> (group, matrix, tile)
  int gsel = 0;
#pragma unroll
  for (int i = 1; i < kMaxGroups; ++i)
    if (i < G.ng && item >= W.start[i]) gsel = i;
  int64_t first_item = 0, ld = 0, stride = 0;
  const void* Abase = nullptr;
  int n = 0, tiles_m = 1, tiles_n = 1;
#pragma unroll
  for (int i = 0; i < kMaxGroups; ++i)
    if (i == gsel) {
      first_item = W.start[i];
      Abase = G.g[i].A;
      ld = G.g[i].ld;
      stride = G.g[i].stride;
      n = G.g[i].n;
      tiles_m = W.tm[i];
      tiles_n = W.tn[i];
    }
  const int64_t local = item - first_item;
  const int tiles = tiles_m * tiles_n;
  const int64_t b = local / tiles;
  const int t = (int)(local - b * tiles);
  const int strip = GL_GM * tiles_n;
  const int first = (t / strip) * GL_GM;
  const int gsz = min(tiles_m - first, GL_GM);
  // odd strips walk the columns backwards, so a strip starts on the B
  // columns the previous one ended on (still in L2)
  const int tcol = (t % strip) / gsz;
  const int tm = first + (t % strip) % gsz, tn = ((t / strip) & 1) ? tiles_n - 1 - tcol : tcol;
  const int M = min(rowEnd, n) - rowC, N = min(colEnd, n) - colC;
  const int m0 = tm * GL_BM, n0 = tn * BN;
  const GLOBAL float2* Mat = (const GLOBAL float2*)Abase + b * stride;
  const GLOBAL float2* A = Mat + (int64_t)rowC * ld + colA;
  const GLOBAL float2* B = Mat + (int64_t)rowB * ld + colC;
  GLOBAL float2* C = (GLOBAL float2*)Mat + (int64_t)rowC * ld + colC;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wid >> 1, wn = wid & 1;
  const int h = lane >> 5, l32 = lane & 31;

  // ---- loads of one stage: A slots q*256 + tid (row q*32 + tid/8, 16-byte
  // word (tid % 8) ^ (row % 8)), B slots q*256 + tid (k row (q*256 + tid) /
  // (BN/2), word tid % (BN/2)).  The addresses are recomputed per stage from
  // the thread index (kept opaque to the compiler) so that none of them stays
  // live across the MFMA loop, whose accumulators fill the register budget.
  constexpr int BQ = BW / 256;
  const int ldi = (int)ld;   // n * ld < 2^31 is checked on the host
  const unsigned a_lds = (unsigned)(uintptr_t)(LDS_AS void*)&As[0][0] + wid * 1024;
  const unsigned b_lds = (unsigned)(uintptr_t)(LDS_AS void*)&Bs[0][0] + wid * 1024;
  const int S = (K + GL_BK - 1) / GL_BK;
  auto load_stage = [&](int s) {
    int tt = tid;
    asm volatile("" : "+v"(tt));
    const int k0 = s * GL_BK;
    const unsigned abuf = (unsigned)(s & 1) * (GL_BM * GL_BK / 2 * 16);
    const unsigned bbuf = (unsigned)(s & 1) * (BW * 16);
    const int ka = min(k0 + 2 * ((tt & 7) ^ ((tt >> 3) & 7)), K - 2);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = min(m0 + q * 32 + (tt >> 3), M - 1);
      lds_dma16((const GLOBAL u32x4*)(A + (row * ldi + ka)),
                __builtin_amdgcn_readfirstlane(a_lds + abuf + q * 4096));
    }
    const int bc = min(n0 + 2 * (tt & (BN / 2 - 1)), ldi - colC - 2);
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int kr = min(k0 + (q * 256 + tt) / (BN / 2), K - 1);
      lds_dma16((const GLOBAL u32x4*)(B + (kr * ldi + bc)),
                __builtin_amdgcn_readfirstlane(b_lds + bbuf + q * 4096));
    }
  };

  constexpr int NACC = M3 ? 3 : 2;
  floatx16 acc[NACC][2][WJ];
#pragma unroll
  for (int p = 0; p < NACC; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < WJ; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[p][i][j][v] = 0.f;

  const int arow0 = wm * 64 + l32;                   // + 32 i
  const int bcol0 = wn * 32 * WJ + l32;              // + 32 j
  // MFMA blocks whose rows or columns all lie past the edge are skipped
  // (wave-uniform: partial edge tiles do only the blocks they need)
  bool live_i[2], live_j[WJ];
#pragma unroll
  for (int i = 0; i < 2; ++i) live_i[i] = m0 + wm * 64 + 32 * i < M;
#pragma unroll
  for (int j = 0; j < WJ; ++j) live_j[j] = n0 + wn * 32 * WJ + 32 * j < N;
  const int sw = l32 & 7;
  // Operands of one group of 4 complex k (q4) in registers.  3M: lane half h
  // holds k = 4 q4 + 2h + p for MFMA p (A as one 16-byte word per block).
  // 4M: both halves take the same k, re (h = 0) or im (h = 1) of A, and the
  // matching entries of the two B patterns.
  constexpr int AW = M3 ? 1 : 2;   // 16-byte A words per block and group
  constexpr int BK = M3 ? 2 : 4;   // B entries per block and group
  struct Ops {
    float4 a[2][AW];
    float2 b[WJ][BK];
  };
  auto read_ops = [&](const u32x4* Ab, const float2* Bf, int q4, Ops& o) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int w = 0; w < AW; ++w) {
        const int c = M3 ? 2 * q4 + h : 2 * q4 + w;
        o.a[i][w] = __builtin_bit_cast(float4, Ab[(arow0 + 32 * i) * 8 + (c ^ sw)]);
      }
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int e = 0; e < BK; ++e) {
        const int kk = M3 ? 4 * q4 + 2 * h + e : 4 * q4 + e;
        o.b[j][e] = Bf[kk * BN + bcol0 + 32 * j];
      }
  };
  // ALL: every MFMA block of the wave is live (interior tiles), so the
  // block loop carries no per-block branch
  auto mma = [&](const Ops& o, auto all_live) {
    constexpr bool ALL = decltype(all_live)::value;
    if constexpr (M3) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        float ar[2], ai[2], as[2], br[WJ], bi[WJ], bs[WJ];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          ar[i] = p ? o.a[i][0].z : o.a[i][0].x;
          ai[i] = p ? o.a[i][0].w : o.a[i][0].y;
          as[i] = ar[i] + ai[i];
        }
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
          br[j] = o.b[j][p].x;
          bi[j] = o.b[j][p].y;
          bs[j] = br[j] + bi[j];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < WJ; ++j) {
            if (ALL || (live_i[i] && live_j[j])) {
              acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], br[j], acc[0][i][j], 0, 0, 0);
              acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i], bi[j], acc[1][i][j], 0, 0, 0);
              acc[2][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[i], bs[j], acc[2][i][j], 0, 0, 0);
            }
          }
      }
    } else {
#pragma unroll
      for (int e4 = 0; e4 < 4; ++e4) {
        const int w = e4 >> 1, e = e4 & 1;
        float a[2], bre[WJ], bim[WJ];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float re = e ? o.a[i][w].z : o.a[i][w].x, im = e ? o.a[i][w].w : o.a[i][w].y;
          a[i] = h ? im : re;
        }
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
          const float2 v = o.b[j][e4];
          bre[j] = h ? -v.y : v.x;
          bim[j] = h ? v.x : v.y;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < WJ; ++j) {
            if (ALL || (live_i[i] && live_j[j])) {
              acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], bre[j], acc[0][i][j], 0, 0, 0);
              acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], bim[j], acc[1][i][j], 0, 0, 0);
            }
          }
      }
    }
  };
  // A partial last stage (K not a multiple of 16; K is even, so every A word
  // is all in or all out): each thread zeroes the LDS words of its own loads
  // that lie at or past K, after its loads have landed.
  auto zero_tail = [&](int cur, int kvalid) {
    const int tt = tid;
    const u32x4 z = {0u, 0u, 0u, 0u};
    const int c = (tt & 7) ^ ((tt >> 3) & 7);
    if (2 * c >= kvalid)
#pragma unroll
      for (int q = 0; q < 4; ++q) As[cur][q * 256 + tt] = z;
#pragma unroll
    for (int q = 0; q < BQ; ++q)
      if ((q * 256 + tt) / (BN / 2) >= kvalid) Bs[cur][q * 256 + tt] = z;
  };

  auto kloop = [&](auto all_live) {
    load_stage(0);
    for (int s = 0; s < S; ++s) {
      // stage s has landed, and every wave is past its reads of stage s - 1,
      // whose buffer the next load reuses
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
      const int cur = s & 1;
      const int kvalid = K - s * GL_BK;
      if (kvalid < GL_BK) {
        zero_tail(cur, kvalid);
        __syncthreads();
      }
      if (s + 1 < S) load_stage(s + 1);
      // the next group's operands are read while the current group's MFMAs run
      const u32x4* Ab = &As[cur][0];
      const float2* Bf = (const float2*)&Bs[cur][0];
      Ops o[2];
      read_ops(Ab, Bf, 0, o[0]);
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        if (q4 + 1 < 4) read_ops(Ab, Bf, q4 + 1, o[(q4 + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        mma(o[q4 & 1], all_live);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  bool all = true;
#pragma unroll
  for (int i = 0; i < 2; ++i) all = all && live_i[i];
#pragma unroll
  for (int j = 0; j < WJ; ++j) all = all && live_j[j];
  if (all)
    kloop(std::true_type{});
  else
    kloop(std::false_type{});
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const int col = n0 + bcol0 + 32 * j;
      if (col >= N) continue;
      float2 c[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        c[v] = C[min(row, M - 1) * ldi + col];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        float dr, di;
        if constexpr (M3) {
          const float t1 = acc[0][i][j][v], t2 = acc[1][i][j][v], t3 = acc[2][i][j][v];
          dr = t1 - t2;
          di = t3 - t1 - t2;
        } else {
          dr = acc[0][i][j][v];
          di = acc[1][i][j][v];
        }
        if (row < M) C[row * ldi + col] = make_float2(c[v].x - dr, c[v].y - di);
      }
    }
}

template <bool M3, int WJ, bool PERSIST>
__global__ __launch_bounds__(256, 2) void gemm_c32_lds_kernel(LuGroups G, GemmList W, int rowC,
                                                              int colC, int colA, int rowB,
                                                              int rowEnd, int colEnd, int K,
                                                              uint32_t* queue) {
  __shared__ u32x4 As[2][GL_BM * GL_BK / 2], Bs[2][GL_BK * 64 * WJ / 2];
  const int64_t total = W.start[G.ng];
  const int64_t per = (total + 7) >> 3;
  const int x = blockIdx.x & 7;
  if constexpr (!PERSIST) {
    const int64_t item = (int64_t)x * per + (blockIdx.x >> 3);
    if (item < total)
      gemm_lds_tile<M3, WJ>(G, W, item, rowC, colC, colA, rowB, rowEnd, colEnd, K, As, Bs);
    return;
  }
  __shared__ uint32_t ticket;
  const int64_t lo = (int64_t)x * per, hi = min(total, lo + per);
  for (;;) {
    if (threadIdx.x == 0) ticket = atomicAdd(&queue[2 * x], 1u);
    __syncthreads();
    const int64_t item = lo + ticket;
    // every thread has its ticket, and the previous tile's LDS reads are done
    __syncthreads();
    if (item >= hi) break;
    gemm_lds_tile<M3, WJ>(G, W, item, rowC, colC, colA, rowB, rowEnd, colEnd, K, As, Bs);
  }
  if (threadIdx.x == 0) {
    // all of range x's tickets are drawn once its gridDim.x / 8 workgroups
    // have each drawn one past the end
    if (atomicAdd(&queue[2 * x + 1], 1u) == (gridDim.x >> 3) - 1) {
      atomicExch(&queue[2 * x], 0u);
      atomicExch(&queue[2 * x + 1], 0u);
    }
  }
}

// ============================================================== GEMM f32 via bf16 split
// The same 4M update with every real product taken as three bfloat16 MFMA
// products: each float32 operand x is split into hi = bf16(x) and
// lo = bf16(x - hi), and x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y (the dropped
// lo_x lo_y and the rounding of lo leave about 17 significant bits per
// operand), accumulated in float32 by MFMA 32x32x16 bf16.
//
// 128 x 128 tile per workgroup of 4 waves, each 64 x 64 as 2 x 2 MFMA blocks;
// 16 complex k per LDS stage (four k groups of 8 interleaved real k), double
// buffered.  The split is done while staging: A as hi/lo of (Re A, Im A)
// pairs, B as hi/lo of the real-part pattern (Re B, -Im B); the
// imaginary-part pattern (Im B, Re B) is derived from it in registers (swap
// the halves of each 32-bit pair, flip one sign bit).  Bounds are applied as
// masks at staging time, so the global loads of the next stage stay in flight
// across the MFMA loop.
//
// Tile order: the grid is padded to a multiple of 8 so that workgroup x runs
// on XCD x % 8; each XCD takes a contiguous range of tiles walked in groups of
// GB_GM tile rows, so the workgroups resident on one XCD share A and B panels
// in that XCD's L2.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
union Pack8 {
  uint4 u;
  bf16x8 v;
};

__device__ inline void split8(const float* x, uint4& hi, uint4& lo) {
  unsigned hw[4], lw[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const f2v v = {x[2 * p], x[2 * p + 1]};
    const unsigned hu = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf2v));
    const f2v r = {x[2 * p] - __uint_as_float(hu << 16), x[2 * p + 1] - __uint_as_float(hu & 0xffff0000u)};
    hw[p] = hu;
    lw[p] = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf2v));
  }
  hi = make_uint4(hw[0], hw[1], hw[2], hw[3]);
  lo = make_uint4(lw[0], lw[1], lw[2], lw[3]);
}

// (a, b) pairs of the real-part pattern -> (-b, a) of the imaginary-part pattern
__device__ inline uint4 re_to_im(uint4 r) {
  uint4 o;
  o.x = ((r.x >> 16) | (r.x << 16)) ^ 0x8000u;
  o.y = ((r.y >> 16) | (r.y << 16)) ^ 0x8000u;
  o.z = ((r.z >> 16) | (r.z << 16)) ^ 0x8000u;
  o.w = ((r.w >> 16) | (r.w << 16)) ^ 0x8000u;
  return o;
}

constexpr int GB_BM = 128, GB_BN = 128, GB_KB = 16, GB_KG = GB_KB / 4, GB_GM = 8;

__global__ __launch_bounds__(256, 2) void gemm_c32_b3_kernel(LuGroups G, int rowC, int colC,
                                                             int colA, int rowB, int rowEnd,
                                                             int colEnd, int K, int tiles_m,
                                                             int tiles_n) {
  __shared__ uint4 Ah[2][GB_KG][GB_BM], Al[2][GB_KG][GB_BM];
  __shared__ uint4 Brh[2][GB_KG][GB_BN], Brl[2][GB_KG][GB_BN];
  // XCD-aware grouped tile order (launch-level tile counts; tiles outside a
  // smaller matrix exit below)
  const int per = gridDim.x / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= tiles_m * tiles_n) return;
  const int grp = t / (GB_GM * tiles_n), first = grp * GB_GM;
  const int gsz = min(tiles_m - first, GB_GM);
  const int tm = first + (t % (GB_GM * tiles_n)) % gsz;
  const int tn = (t % (GB_GM * tiles_n)) / gsz;
  GemmView<float2> gv;
  if (!gemm_view(G, rowC, colC, colA, rowB, rowEnd, colEnd, gv)) return;
  const int m0 = tm * GB_BM, n0 = tn * GB_BN;
  const int M = gv.M, N = gv.N;
  if (m0 >= M || n0 >= N) return;
  const int ld = (int)gv.ld;   // n * ld < 2^31 is checked on the host
  const GLOBAL float2* A = gv.A;
  const GLOBAL float2* B = gv.B;
  GLOBAL float2* C = gv.Cm;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int h = lane >> 5, l32 = lane & 31;
  floatx16 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) { acc_re[i][j][v] = 0.f; acc_im[i][j][v] = 0.f; }

  // staging: chunk e = tid + 256 c; A chunk = (row e / 4, k group e % 4),
  // B chunk = (col e % 128, k group e / 128); 4 complex each
  constexpr int NC = GB_BM * GB_KG / 256;
  float2 ra[NC][4], rb[NC][4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int e = tid + 256 * c;
      const int row = e / GB_KG, akg = e % GB_KG;
      const GLOBAL float2* Ap = A + min(m0 + row, M - 1) * ld;
#pragma unroll
      for (int q = 0; q < 4; ++q) ra[c][q] = Ap[min(k0 + 4 * akg + q, K - 1)];
      const int col = e % GB_BN, bkg = e / GB_BN;
      const GLOBAL float2* Bp = B + min(n0 + col, N - 1);
#pragma unroll
      for (int q = 0; q < 4; ++q) rb[c][q] = Bp[min(k0 + 4 * bkg + q, K - 1) * ld];
    }
  };
  auto sstore = [&](int buf, int k0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int e = tid + 256 * c;
      const int row = e / GB_KG, akg = e % GB_KG;
      const int col = e % GB_BN, bkg = e / GB_BN;
      const bool rok = m0 + row < M, cok = n0 + col < N;
      float xa[8], xr[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const unsigned ma = (rok && k0 + 4 * akg + q < K) ? 0xffffffffu : 0u;
        xa[2 * q] = __uint_as_float(__float_as_uint(ra[c][q].x) & ma);
        xa[2 * q + 1] = __uint_as_float(__float_as_uint(ra[c][q].y) & ma);
        const unsigned mb = (cok && k0 + 4 * bkg + q < K) ? 0xffffffffu : 0u;
        xr[2 * q] = __uint_as_float(__float_as_uint(rb[c][q].x) & mb);
        xr[2 * q + 1] = __uint_as_float(__float_as_uint(-rb[c][q].y) & mb);
      }
      uint4 hi, lo;
      split8(xa, hi, lo);
      Ah[buf][akg][row] = hi;
      Al[buf][akg][row] = lo;
      split8(xr, hi, lo);
      Brh[buf][bkg][col] = hi;
      Brl[buf][bkg][col] = lo;
    }
  };

  const int nk = (K + GB_KB - 1) / GB_KB;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * GB_KB);
#pragma unroll
    for (int s2 = 0; s2 < GB_KG / 2; ++s2) {
      // lanes 0-31 take k group 2 s2, lanes 32-63 k group 2 s2 + 1
      const int g = 2 * s2 + h;
      Pack8 ah[2], al[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ah[i].u = Ah[cur][g][wm * 64 + i * 32 + l32];
        al[i].u = Al[cur][g][wm * 64 + i * 32 + l32];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        brh[j].u = Brh[cur][g][wn * 64 + j * 32 + l32];
        brl[j].u = Brl[cur][g][wn * 64 + j * 32 + l32];
        bih[j].u = re_to_im(brh[j].u);
        bil[j].u = re_to_im(brl[j].u);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i].v, brh[j].v, acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i].v, brl[j].v, acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i].v, brh[j].v, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i].v, bih[j].v, acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i].v, bil[j].v, acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i].v, bih[j].v, acc_im[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) sstore(cur ^ 1, (kt + 1) * GB_KB);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + l32;
      if (col >= N) continue;
      float2 c[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        c[v] = C[min(row, M - 1) * ld + col];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < M) C[row * ld + col] = make_float2(c[v].x - acc_re[i][j][v], c[v].y - acc_im[i][j][v]);
      }
    }
}

// ============================================================== GEMM f32 via bf16 split, narrow
// Narrow updates (N <= 64, the tall panels inside a block): 128 x 32 tile per
// workgroup of 4 waves (one 32 x 32 MFMA block each), so narrow matrices do
// not pay for 128-wide tiles and four workgroups fit per CU.  C is loaded into
// the accumulators at the start together with the first operand stage (A is
// staged negated: acc = C - A B), which overlaps the C read with the k loop.
constexpr int GT_BM = 128, GT_BN = 32;

__global__ __launch_bounds__(256, 4) void gemm_c32_tsb_kernel(LuGroups G, int rowC, int colC,
                                                              int colA, int rowB, int rowEnd,
                                                              int colEnd, int K, int tiles_n) {
  __shared__ uint4 Ah[2][GB_KG][GT_BM], Al[2][GB_KG][GT_BM];
  __shared__ uint4 Brh[2][GB_KG][GT_BN], Brl[2][GB_KG][GT_BN];
  GemmView<float2> gv;
  if (!gemm_view(G, rowC, colC, colA, rowB, rowEnd, colEnd, gv)) return;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int m0 = tm * GT_BM, n0 = tn * GT_BN;
  const int M = gv.M, N = gv.N;
  if (m0 >= M || n0 >= N) return;
  const int ld = (int)gv.ld;   // n * ld < 2^31 is checked on the host
  const GLOBAL float2* A = gv.A;
  const GLOBAL float2* B = gv.B;
  GLOBAL float2* C = gv.Cm;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  // this wave's C block: rows m0 + 32 wid + 8 (v/4) + 4 h + v%4, column n0 + l32
  floatx16 acc_re, acc_im;
  const int ccol = n0 + l32;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = m0 + 32 * wid + 8 * (v >> 2) + 4 * h + (v & 3);
    const float2 c = C[min(row, M - 1) * ld + min(ccol, N - 1)];
    acc_re[v] = c.x;
    acc_im[v] = c.y;
  }
  // staging: two A chunks (row e / 4, k group e % 4) per thread, one B chunk
  // (col tid % 32, k group tid / 32) for the first 128 threads; 4 complex each
  float2 ra[2][4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int e = tid + 256 * c, row = e / GB_KG, akg = e % GB_KG;
      const GLOBAL float2* Ap = A + min(m0 + row, M - 1) * ld;
#pragma unroll
      for (int q = 0; q < 4; ++q) ra[c][q] = Ap[min(k0 + 4 * akg + q, K - 1)];
    }
    if (tid < GT_BN * GB_KG) {
      const int col = tid % GT_BN, bkg = tid / GT_BN;
      const GLOBAL float2* Bp = B + min(n0 + col, N - 1);
#pragma unroll
      for (int q = 0; q < 4; ++q) rb[q] = Bp[min(k0 + 4 * bkg + q, K - 1) * ld];
    }
  };
  auto sstore = [&](int buf, int k0) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int e = tid + 256 * c, row = e / GB_KG, akg = e % GB_KG;
      const bool rok = m0 + row < M;
      float xa[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const unsigned ma = (rok && k0 + 4 * akg + q < K) ? 0xffffffffu : 0u;
        xa[2 * q] = __uint_as_float(__float_as_uint(-ra[c][q].x) & ma);
        xa[2 * q + 1] = __uint_as_float(__float_as_uint(-ra[c][q].y) & ma);
      }
      uint4 hi, lo;
      split8(xa, hi, lo);
      Ah[buf][akg][row] = hi;
      Al[buf][akg][row] = lo;
    }
    if (tid < GT_BN * GB_KG) {
      const int col = tid % GT_BN, bkg = tid / GT_BN;
      const bool cok = n0 + col < N;
      float xr[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const unsigned mb = (cok && k0 + 4 * bkg + q < K) ? 0xffffffffu : 0u;
        xr[2 * q] = __uint_as_float(__float_as_uint(rb[q].x) & mb);
        xr[2 * q + 1] = __uint_as_float(__float_as_uint(-rb[q].y) & mb);
      }
      uint4 hi, lo;
      split8(xr, hi, lo);
      Brh[buf][bkg][col] = hi;
      Brl[buf][bkg][col] = lo;
    }
  };
  const int nk = (K + GB_KB - 1) / GB_KB;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * GB_KB);
#pragma unroll
    for (int s2 = 0; s2 < GB_KG / 2; ++s2) {
      const int g = 2 * s2 + h;
      Pack8 ah, al, bh, bl, bih, bil;
      ah.u = Ah[cur][g][32 * wid + l32];
      al.u = Al[cur][g][32 * wid + l32];
      bh.u = Brh[cur][g][l32];
      bl.u = Brl[cur][g][l32];
      bih.u = re_to_im(bh.u);
      bil.u = re_to_im(bl.u);
      acc_re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.v, bh.v, acc_re, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.v, bih.v, acc_im, 0, 0, 0);
      acc_re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.v, bl.v, acc_re, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.v, bil.v, acc_im, 0, 0, 0);
      acc_re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.v, bh.v, acc_re, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.v, bih.v, acc_im, 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(cur ^ 1, (kt + 1) * GB_KB);
    __syncthreads();
  }
  if (ccol < N) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = m0 + 32 * wid + 8 * (v >> 2) + 4 * h + (v & 3);
      if (row < M) C[row * ld + ccol] = make_float2(acc_re[v], acc_im[v]);
    }
  }
}

// ============================================================== GEMM f32, small width and depth
// The smallest updates inside the panels (N, K <= 16: the pairs of 8-column
// panels and of 16-column halves) are bound by moving C.  NK/2 adjacent lanes
// share a row, each holding two columns of A and of C (one 16-byte word when
// aligned), so a wave reads whole row segments; the lanes of a row exchange
// their A values by shuffles and take B (K x N, zero-padded) from LDS.
// float32 FMA.
template <int NK>
__global__ __launch_bounds__(256) void gemm_c32_small_kernel(LuGroups G, int rowC, int colC,
                                                             int colA, int rowB, int rowEnd,
                                                             int colEnd, int K) {
  constexpr int LPR = NK / 2;           // lanes per row
  constexpr int RPB = 256 / LPR;        // rows per workgroup
  __shared__ __align__(16) float2 Bs[NK][NK];
  LuGroup grp;
  int b = 0;
  if (!locate(G, blockIdx.y, grp, b)) return;
  const int M = min(rowEnd, grp.n) - rowC, N = min(colEnd, grp.n) - colC;
  if (M <= 0 || N <= 0 || (int)(blockIdx.x * RPB) >= M) return;
  const int64_t ld = grp.ld;
  GLOBAL float2* base = gmat<float2>(grp, b);
  const int t = threadIdx.x;
  const int l = t % LPR;                // this lane's columns: 2l, 2l + 1
  const int row = blockIdx.x * RPB + t / LPR;
  // rows past the end load the last row and store nothing; every lane stays
  // in the shuffles and the barrier
  const bool live = row < M;
  const int rr = min(row, M - 1);
  const GLOBAL float2* Ar = base + (int64_t)(rowC + rr) * ld + colA;
  GLOBAL float2* Cr = base + (int64_t)(rowC + rr) * ld + colC;
  const bool vec = ((ld | colA | colC) & 1) == 0;
  float2 a0, a1, c0, c1;
  if (vec && K == NK && N == NK) {
    const float4 va = ((const GLOBAL float4*)Ar)[l], vc = ((const GLOBAL float4*)Cr)[l];
    a0 = make_float2(va.x, va.y);
    a1 = make_float2(va.z, va.w);
    c0 = make_float2(vc.x, vc.y);
    c1 = make_float2(vc.z, vc.w);
  } else {
    const int k0 = 2 * l, k1 = 2 * l + 1;
    a0 = Ar[min(k0, K - 1)];
    a1 = Ar[min(k1, K - 1)];
    if (k0 >= K) a0 = make_float2(0.f, 0.f);
    if (k1 >= K) a1 = make_float2(0.f, 0.f);
    c0 = Cr[min(k0, N - 1)];
    c1 = Cr[min(k1, N - 1)];
  }
  // B after this thread's row loads, so the two loads overlap
  for (int e = t; e < NK * NK; e += 256) {
    const int kk = e / NK, j = e % NK;
    Bs[kk][j] = (kk < K && j < N) ? base[(int64_t)(rowB + kk) * ld + colC + j] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int g0 = (t % 64) - l;          // first lane of this row within the wave
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    const float2 own = (kk & 1) ? a1 : a0;
    const float ar = __shfl(own.x, g0 + kk / 2, 64), ai = __shfl(own.y, g0 + kk / 2, 64);
    const float4 bv = *reinterpret_cast<const float4*>(&Bs[kk][2 * l]);
    c0.x -= ar * bv.x - ai * bv.y;
    c0.y -= ar * bv.y + ai * bv.x;
    c1.x -= ar * bv.z - ai * bv.w;
    c1.y -= ar * bv.w + ai * bv.z;
  }
  if (!live) return;
  if (vec && N == NK) {
    ((GLOBAL float4*)Cr)[l] = make_float4(c0.x, c0.y, c1.x, c1.y);
  } else {
    if (2 * l < N) Cr[2 * l] = c0;
    if (2 * l + 1 < N) Cr[2 * l + 1] = c1;
  }
}

// ============================================================== GEMM f32 via bf16 split, packed operands
// Updates of at least 512 x 512 take their operands split once: a packing
// pass converts A (a block column of L, e.g. below the block just factored)
// and B (a block row of U, in the real-part pattern (Re, -Im)) into bf16
// hi/lo words laid out as the GEMM's LDS stage buffers -- per 128-row (or
// -column) tile and 8-k block, [k group of 4][hi/lo][row] 16-byte words,
// zero-padded past the edges -- so each element is split once rather than
// once per tile reading it.  The GEMM streams 16-k stages (two 8-k blocks,
// contiguous) straight from global memory into LDS with global_load_lds
// (no register staging), one stage ahead into the other of two LDS buffers,
// with an explicit wait on the load counter and a barrier per stage.  The
// products and their order are those of gemm_c32_b3_kernel, so the update
// is bit-identical to it.
constexpr int GP_BLK = 2 * 2 * GB_BM;   // 16-byte words per tile and 8-k block
// largest packing buffer a context holds; bigger batches are packed in slices
constexpr size_t kPackLimit = (size_t)4 << 30;

// 16-byte words of the packed A and B of one matrix for an M x N update of depth K
inline int64_t pack_words(int M, int N, int K) {
  const int64_t S8 = (K + 7) / 8;
  return ((int64_t)(M + GB_BM - 1) / GB_BM + (N + GB_BN - 1) / GB_BN) * S8 * GP_BLK;
}

// A = rows [rowC, min(rowEnd, n)) x cols [colA, colA + K) -> out + y * ms.
// One thread per (tile, 8-k block, row): the row's 8 values are read with
// clamped addresses (16-byte words when aligned) and zeroed past the edges.
__global__ __launch_bounds__(256) void pack_a_kernel(LuGroups G, int rowC, int colA, int rowEnd,
                                                     int K, int tiles_m, int64_t ms,
                                                     uint4* __restrict__ out) {
  LuGroup grp;
  int b = 0;
  if (!locate(G, blockIdx.y, grp, b)) return;
  const int M = min(rowEnd, grp.n) - rowC;
  if (M <= 0) return;
  const int S8 = (K + 7) / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (tile, block, row)
  if (idx >= (int64_t)tiles_m * S8 * GB_BM) return;
  const int row = (int)(idx % GB_BM);
  const int64_t tb = idx / GB_BM;                                 // tile * S8 + block
  const int s8 = (int)(tb % S8);
  const int gr = (int)(tb / S8) * GB_BM + row, k0 = s8 * 8;
  const GLOBAL float2* A = gmat<float2>(grp, b) + (int64_t)(rowC + min(gr, M - 1)) * grp.ld + colA;
  float x[16];
  if (k0 + 8 <= K && ((grp.ld | colA) & 1) == 0) {
    const GLOBAL float4* p4 = (const GLOBAL float4*)(A + k0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float4 v = p4[m];
      x[4 * m] = v.x;
      x[4 * m + 1] = v.y;
      x[4 * m + 2] = v.z;
      x[4 * m + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float2 v = A[min(k0 + q, K - 1)];
      x[2 * q] = v.x;
      x[2 * q + 1] = v.y;
    }
  }
  const bool rok = gr < M;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const bool ok = rok && k0 + q < K;
    x[2 * q] = ok ? x[2 * q] : 0.f;
    x[2 * q + 1] = ok ? x[2 * q + 1] : 0.f;
  }
  uint4* o = out + blockIdx.y * ms + tb * GP_BLK;
#pragma unroll
  for (int kg = 0; kg < 2; ++kg) {
    uint4 hi, lo;
    split8(x + 8 * kg, hi, lo);
    o[kg * 2 * GB_BM + row] = hi;
    o[kg * 2 * GB_BM + GB_BM + row] = lo;
  }
}

// B = rows [rowB, rowB + K) x cols [colC, min(colEnd, n)) -> out + y * ms.
// One thread per (tile, 8-k block, k group, column); clamped loads, zeroed
// past the edges.
__global__ __launch_bounds__(256) void pack_b_kernel(LuGroups G, int rowB, int colC, int colEnd,
                                                     int K, int tiles_n, int64_t ms,
                                                     uint4* __restrict__ out) {
  LuGroup grp;
  int b = 0;
  if (!locate(G, blockIdx.y, grp, b)) return;
  const int N = min(colEnd, grp.n) - colC;
  if (N <= 0) return;
  const int S8 = (K + 7) / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (tile, block, k group, col)
  if (idx >= (int64_t)tiles_n * S8 * (GP_BLK / 2)) return;
  const int col = (int)(idx % GB_BN), kg = (int)((idx / GB_BN) % 2);
  const int64_t tb = idx / (2 * GB_BN);
  const int s8 = (int)(tb % S8);
  const int gc = (int)(tb / S8) * GB_BN + col, k0 = s8 * 8 + 4 * kg;
  const GLOBAL float2* B = gmat<float2>(grp, b) + (int64_t)rowB * grp.ld + colC + min(gc, N - 1);
  float x[8];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float2 v = B[(int64_t)min(k0 + q, K - 1) * grp.ld];
    const bool ok = gc < N && k0 + q < K;
    x[2 * q] = ok ? v.x : 0.f;
    x[2 * q + 1] = ok ? -v.y : 0.f;
  }
  uint4 hi, lo;
  split8(x, hi, lo);
  uint4* o = out + blockIdx.y * ms + tb * GP_BLK + kg * 2 * GB_BN;
  o[col] = hi;
  o[GB_BN + col] = lo;
}

__device__ inline bf16x8 re_to_im8(bf16x8 b) {
  const u32x4 r = __builtin_bit_cast(u32x4, b);
  return __builtin_bit_cast(bf16x8, ((r >> 16) | (r << 16)) ^ 0x8000u);
}

__global__ __launch_bounds__(256, 2) void gemm_c32_b3p_kernel(LuGroups G, int rowC, int colC,
                                                              int rowEnd, int colEnd, int K,
                                                              int tiles_m, int tiles_n,
                                                              const uint4* __restrict__ Ap,
                                                              int64_t a_ms,
                                                              const uint4* __restrict__ Bp,
                                                              int64_t b_ms) {
  __shared__ u32x4 As[2][2 * GP_BLK], Bs[2][2 * GP_BLK];
  const int per = gridDim.x / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= tiles_m * tiles_n) return;
  const int grp = t / (GB_GM * tiles_n), first = grp * GB_GM;
  const int gsz = min(tiles_m - first, GB_GM);
  const int tm = first + (t % (GB_GM * tiles_n)) % gsz;
  const int tn = (t % (GB_GM * tiles_n)) / gsz;
  GemmView<float2> gv;
  if (!gemm_view(G, rowC, colC, 0, 0, rowEnd, colEnd, gv)) return;
  const int m0 = tm * GB_BM, n0 = tn * GB_BN;
  const int M = gv.M, N = gv.N;
  if (m0 >= M || n0 >= N) return;
  const int ld = (int)gv.ld;   // n * ld < 2^31 is checked on the host
  GLOBAL float2* C = gv.Cm;
  const int S8 = (K + 7) / 8, S = (S8 + 1) / 2;
  const GLOBAL u32x4* Ag = (const GLOBAL u32x4*)Ap + blockIdx.y * a_ms + (int64_t)tm * S8 * GP_BLK;
  const GLOBAL u32x4* Bg = (const GLOBAL u32x4*)Bp + blockIdx.y * b_ms + (int64_t)tn * S8 * GP_BLK;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int h = lane >> 5, l32 = lane & 31;
  floatx16 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) { acc_re[i][j][v] = 0.f; acc_im[i][j][v] = 0.f; }
  // LDS byte offsets of this wave's 64 words in buffer 0
  const unsigned a_lds = (unsigned)(uintptr_t)(LDS_AS void*)&As[0][tid & ~63];
  const unsigned b_lds = (unsigned)(uintptr_t)(LDS_AS void*)&Bs[0][tid & ~63];
  // stage s = 8-k blocks 2s and 2s + 1 (only the first when S8 is odd and s is last)
  auto load_stage = [&](int s) {
    const unsigned boff = (unsigned)(s & 1) * (2 * GP_BLK * 16);
    const int nw = 2 * s + 1 < S8 ? 4 : 2;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nw) {
        lds_dma16(Ag + (int64_t)s * 2 * GP_BLK + tid + 256 * q,
                  __builtin_amdgcn_readfirstlane(a_lds + boff + q * 4096));
        lds_dma16(Bg + (int64_t)s * 2 * GP_BLK + tid + 256 * q,
                  __builtin_amdgcn_readfirstlane(b_lds + boff + q * 4096));
      }
  };
  load_stage(0);
  for (int s = 0; s < S; ++s) {
    // stage s has landed, and every wave is past its reads of stage s - 1,
    // whose buffer the next load reuses
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    if (s + 1 < S) load_stage(s + 1);
    const int cur = s & 1;
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      if (2 * s + s2 >= S8) break;
      const int base = s2 * GP_BLK + h * 2 * GB_BM;   // lanes 32-63 take the second k group
      bf16x8 ah[2], al[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ah[i] = __builtin_bit_cast(bf16x8, As[cur][base + wm * 64 + i * 32 + l32]);
        al[i] = __builtin_bit_cast(bf16x8, As[cur][base + GB_BM + wm * 64 + i * 32 + l32]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        brh[j] = __builtin_bit_cast(bf16x8, Bs[cur][base + wn * 64 + j * 32 + l32]);
        brl[j] = __builtin_bit_cast(bf16x8, Bs[cur][base + GB_BN + wn * 64 + j * 32 + l32]);
        bih[j] = re_to_im8(brh[j]);
        bil[j] = re_to_im8(brl[j]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], brh[j], acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], brl[j], acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], brh[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bih[j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bil[j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bih[j], acc_im[i][j], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + l32;
      if (col >= N) continue;
      float2 c[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        c[v] = C[min(row, M - 1) * ld + col];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row < M) C[row * ld + col] = make_float2(c[v].x - acc_re[i][j][v], c[v].y - acc_im[i][j][v]);
      }
    }
}

// ============================================================== GEMM f64
// Same contraction in float64 on MFMA 16x16x4 f64: one MFMA covers two
// complex k (four interleaved real k).  64 x 64 tile, 4 waves of 32 x 32.
constexpr int G64_BM = 64, G64_BN = 64, G64_BK = 8;

__global__ __launch_bounds__(256) void gemm_c64_kernel(LuGroups G, int rowC, int colC, int colA,
                                                       int rowB, int rowEnd, int colEnd, int K,
                                                       int tiles_n) {
  __shared__ double As[2][G64_BK][2 * G64_BM + 4];
  __shared__ double Bs1[2][G64_BK][2 * G64_BN];
  __shared__ double Bs2[2][G64_BK][2 * G64_BN];
  GemmView<double2> gv;
  if (!gemm_view(G, rowC, colC, colA, rowB, rowEnd, colEnd, gv)) return;
  const int tile = blockIdx.x;
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  const int m0 = tm * G64_BM, n0 = tn * G64_BN;
  const int M = gv.M, N = gv.N;
  if (m0 >= M || n0 >= N) return;
  const int64_t ld = gv.ld;
  const GLOBAL double2* A = gv.A;
  const GLOBAL double2* B = gv.B;
  GLOBAL double2* C = gv.Cm;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int l16 = lane & 15, kq = lane >> 4;   // kq: real k index 0..3
  const int kc = kq >> 1, part = kq & 1;       // complex k offset, re/im

  doublex4 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) { acc_re[i][j][v] = 0.0; acc_im[i][j][v] = 0.0; }

  double2 ra[2], rb[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      const int row = e >> 3, kk = e & 7;
      const int gr = m0 + row, gk = k0 + kk;
      const bool oka = gr < M && gk < K;
      const double2 va = A[oka ? (int64_t)gr * ld + gk : 0];
      ra[q] = oka ? va : make_double2(0.0, 0.0);
      const int brow = e >> 6, bcol = e & 63;
      const int gbk = k0 + brow, gbc = n0 + bcol;
      const bool okb = gbk < K && gbc < N;
      const double2 vb = B[okb ? (int64_t)gbk * ld + gbc : 0];
      rb[q] = okb ? vb : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      const int row = e >> 3, kk = e & 7;
      As[buf][kk][row] = ra[q].x;
      As[buf][kk][G64_BM + row] = ra[q].y;
      const int brow = e >> 6, bcol = e & 63;
      Bs1[buf][brow][bcol] = rb[q].x;
      Bs1[buf][brow][G64_BN + bcol] = -rb[q].y;
      Bs2[buf][brow][bcol] = rb[q].y;
      Bs2[buf][brow][G64_BN + bcol] = rb[q].x;
    }
  };
  const int nk = (K + G64_BK - 1) / G64_BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * G64_BK);
#pragma unroll
    for (int k = 0; k < G64_BK; k += 2) {
      double a[2], b1[2], b2[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[cur][k + kc][part * G64_BM + wm * 32 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        b1[j] = Bs1[cur][k + kc][part * G64_BN + wn * 32 + j * 16 + l16];
        b2[j] = Bs2[cur][k + kc][part * G64_BN + wn * 32 + j * 16 + l16];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b1[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b2[j], acc_im[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + j * 16 + l16;
      if (col >= N) continue;
      // f64 16x16x4 result layout: lane l, item v holds row l/16 + 4v, column l%16
      double2 c[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + kq + 4 * v;
        c[v] = C[(int64_t)min(row, M - 1) * ld + col];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + kq + 4 * v;
        if (row < M)
          C[(int64_t)row * ld + col] = make_double2(c[v].x - acc_re[i][j][v], c[v].y - acc_im[i][j][v]);
      }
    }
}

// ============================================================== pivots -> permutation
// perm[i] = original row that ends in position i after the interchanges; the
// sequential composition runs in LDS (one workgroup per matrix).
__global__ void perm_kernel(int n, const int32_t* piv, int32_t* perm) {
  extern __shared__ int32_t q[];
  const int32_t* pb = piv + (int64_t)blockIdx.x * n;
  int32_t* qb = perm + (int64_t)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] = i;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) {
      const int p = pb[i];
      if (p != i) { const int32_t t = q[i]; q[i] = q[p]; q[p] = t; }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) qb[i] = q[i];
}

__global__ void fill_i32_kernel(int64_t count, int32_t* p, int32_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}

// ============================================================== triangular solves
// One workgroup (8 waves) per (matrix, right-hand side): X = U^{-1} L^{-1} P B,
// processed in blocks of 64 rows.  For each block, the 64 x 64 diagonal block
// is staged in LDS while the waves form the off-diagonal dot products (row-major
// rows against the solved part of x, coalesced), then one wave substitutes
// through the diagonal block from LDS.  x lives in LDS when it fits (XLDS),
// otherwise in global memory.
constexpr int TS_B = 64;
constexpr int TS_T = 512;

template <typename R, bool XLDS>
__global__ __launch_bounds__(TS_T) void getrs_kernel(int n, int64_t ld, int64_t stride,
                                                     const typename Cx<R>::T* LU,
                                                     const int32_t* perm, int n_rhs,
                                                     const typename Cx<R>::T* Bin,
                                                     typename Cx<R>::T* X, int64_t bstride,
                                                     const int32_t* fac_index,
                                                     const int32_t* vidx) {
  using C = typename Cx<R>::T;
  extern __shared__ unsigned char smem[];
  C* D = reinterpret_cast<C*>(smem);                 // [TS_B][TS_B + 1]
  C* part = D + TS_B * (TS_B + 1);                   // [TS_B]
  C* xs = part + TS_B;                               // [n] when XLDS
  // vector group: blockIdx / n_rhs, or the vidx entry when a subset is solved
  const int mat = vidx ? vidx[blockIdx.x / n_rhs] : blockIdx.x / n_rhs;
  const int rhs = blockIdx.x % n_rhs;
  // vector group `mat` is solved with factor set fac_index[mat] (identity if NULL)
  const int fac = fac_index ? fac_index[mat] : mat;
  const C* Lb = LU + (int64_t)fac * stride;
  const int32_t* pb = perm + (int64_t)fac * n;
  const C* bin = Bin + (int64_t)mat * bstride + (int64_t)rhs * n;
  C* xg = X + (int64_t)mat * bstride + (int64_t)rhs * n;
  C* x = XLDS ? xs : xg;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int NW = TS_T / 64;
  for (int i = tid; i < n; i += TS_T) x[i] = bin[pb[i]];
  __threadfence_block();
  __syncthreads();
  const int nb = (n + TS_B - 1) / TS_B;
  // every off-diagonal range starts at an even column (0, or a multiple of 64)
  const bool vec2 = sizeof(C) == 8 && ((ld | stride) & 1) == 0 && ((uintptr_t)LU & 15) == 0;
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = pass == 0;
    for (int step = 0; step < nb; ++step) {
      const int I = fwd ? step : nb - 1 - step;
      const int i0 = I * TS_B, rows = min(TS_B, n - i0);
      // stage the diagonal block
      for (int e = tid; e < rows * TS_B; e += TS_T) {
        const int r = e / TS_B, c = e % TS_B;
        if (c < rows) D[r * (TS_B + 1) + c] = Lb[(int64_t)(i0 + r) * ld + i0 + c];
      }
      // off-diagonal dot products: forward uses columns [0, i0), backward [i0+rows, n)
      const int jlo = fwd ? 0 : i0 + rows, jhi = fwd ? i0 : n;
      for (int rr = wid; rr < rows; rr += NW) {
        const C* Li = Lb + (int64_t)(i0 + rr) * ld;
        R sr = 0, si = 0, sr2 = 0, si2 = 0;
        if (vec2) {
          // complex float rows with even ld and start: each lane takes pairs of
          // elements as 16-byte words, two pairs per iteration
          int j = jlo + 2 * lane;
          for (; j + 129 < jhi; j += 256) {
            const float4 la = *reinterpret_cast<const float4*>(Li + j);
            const float4 lb = *reinterpret_cast<const float4*>(Li + j + 128);
            const C a0 = x[j], a1 = x[j + 1], b0 = x[j + 128], b1 = x[j + 129];
            sr += (la.x * a0.x - la.y * a0.y) + (la.z * a1.x - la.w * a1.y);
            si += (la.x * a0.y + la.y * a0.x) + (la.z * a1.y + la.w * a1.x);
            sr2 += (lb.x * b0.x - lb.y * b0.y) + (lb.z * b1.x - lb.w * b1.y);
            si2 += (lb.x * b0.y + lb.y * b0.x) + (lb.z * b1.y + lb.w * b1.x);
          }
          for (; j + 1 < jhi; j += 128) {
            const float4 la = *reinterpret_cast<const float4*>(Li + j);
            const C a0 = x[j], a1 = x[j + 1];
            sr += (la.x * a0.x - la.y * a0.y) + (la.z * a1.x - la.w * a1.y);
            si += (la.x * a0.y + la.y * a0.x) + (la.z * a1.y + la.w * a1.x);
          }
          if (j < jhi) {
            const C l0 = Li[j], v0 = x[j];
            sr += l0.x * v0.x - l0.y * v0.y;
            si += l0.x * v0.y + l0.y * v0.x;
          }
        } else {
          int j = jlo + lane;
          for (; j + 64 < jhi; j += 128) {
            const C l0 = Li[j], v0 = x[j], l1 = Li[j + 64], v1 = x[j + 64];
            sr += l0.x * v0.x - l0.y * v0.y;
            si += l0.x * v0.y + l0.y * v0.x;
            sr2 += l1.x * v1.x - l1.y * v1.y;
            si2 += l1.x * v1.y + l1.y * v1.x;
          }
          if (j < jhi) {
            const C l0 = Li[j], v0 = x[j];
            sr += l0.x * v0.x - l0.y * v0.y;
            si += l0.x * v0.y + l0.y * v0.x;
          }
        }
        sr += sr2;
        si += si2;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          sr += __shfl_down(sr, off, 64);
          si += __shfl_down(si, off, 64);
        }
        if (lane == 0) part[rr] = cmk<C>(sr, si);
      }
      __syncthreads();
      if (wid == 0) {
        C v = cmk<C>(R(0), R(0));
        if (lane < rows) v = csub(x[i0 + lane], part[lane]);
        if (fwd) {
          for (int c = 0; c < rows; ++c) {
            const R xr = __shfl(v.x, c, 64), xi = __shfl(v.y, c, 64);
            if (lane > c && lane < rows) v = csub(v, cmul(D[lane * (TS_B + 1) + c], cmk<C>(xr, xi)));
          }
        } else {
          const C dinv = lane < rows ? crecip(D[lane * (TS_B + 1) + lane]) : cmk<C>(R(1), R(0));
          for (int c = rows - 1; c >= 0; --c) {
            if (lane == c) v = cmul(v, dinv);
            const R xr = __shfl(v.x, c, 64), xi = __shfl(v.y, c, 64);
            if (lane < c) v = csub(v, cmul(D[lane * (TS_B + 1) + c], cmk<C>(xr, xi)));
          }
        }
        if (lane < rows) x[i0 + lane] = v;
      }
      __threadfence_block();
      __syncthreads();
    }
  }
  if (XLDS)
    for (int i = tid; i < n; i += TS_T) xg[i] = x[i];
}

// ============================================================== host driver
// One recursion over the columns of the largest matrix; every launch covers
// all groups whose n exceeds the launch's first column, with each range
// clipped per group inside the kernels.
struct Fac {
  bem_ctx* ctx;
  bem_prec prec;
  std::vector<LuGroup> groups;   // sorted by n, descending
  LuPlan plan;
  int base = 8;
  int gkind = kGemm4M;           // complex GEMM form for c64 (bem_gemm_kind)
  int nmax = 0;
  bool use_pack = false;         // trailing updates through the packed bf16x3 GEMM
  void* pack = nullptr;          // packing buffer (context-owned) and its size
  size_t pack_bytes = 0;

  size_t esz() const { return prec == BEM_C128 ? 16 : 8; }

  // groups with n > c, and their matrix count / largest n
  LuGroups active(int c, int* total, int* maxn) const {
    LuGroups G{};
    G.ng = 0;
    *total = 0;
    *maxn = 0;
    for (const LuGroup& g : groups)
      if (g.n > c && g.count > 0) {
        G.g[G.ng++] = g;
        *total += g.count;
        *maxn = std::max(*maxn, g.n);
      }
    return G;
  }
  // sum over active groups of f(n_g) * count_g
  template <typename F>
  double work(int c, F f) const {
    double s = 0.0;
    for (const LuGroup& g : groups)
      if (g.n > c) s += f(g.n) * g.count;
    return s;
  }

  template <typename R, int W, int RPT>
  void panel_go(const LuGroups& G, int total, int c0, int w) {
    hipLaunchKernelGGL((panel_kernel<R, W, RPT>), dim3(total), dim3(kPanelThreads), 0,
                       ctx->stream, G, c0, w);
  }
  template <typename R, int W>
  void panel_w(const LuGroups& G, int total, int rows, int c0, int w) {
    const int rpt = (rows + kPanelThreads - 1) / kPanelThreads;
    if (rpt <= 1) panel_go<R, W, 1>(G, total, c0, w);
    else if (rpt <= 2) panel_go<R, W, 2>(G, total, c0, w);
    else if (rpt <= 4) panel_go<R, W, 4>(G, total, c0, w);
    else if (rpt <= 6) panel_go<R, W, 6>(G, total, c0, w);
    else if (rpt <= 8) panel_go<R, W, 8>(G, total, c0, w);
    else if (rpt <= 10) panel_go<R, W, 10>(G, total, c0, w);
    else if (rpt <= 11) panel_go<R, W, 11>(G, total, c0, w);
    else if (rpt <= 12) panel_go<R, W, 12>(G, total, c0, w);
    else if (W <= 4 && sizeof(R) == 4) panel_go<R, (W <= 4 ? W : 4), 24>(G, total, c0, w);
    else panel_go<R, (W <= 2 ? W : 2), 24>(G, total, c0, w);
  }
  void panel(int c0, int w) {
    int total, maxn;
    const LuGroups G = active(c0, &total, &maxn);
    if (total == 0) return;
    const int pi = prof_begin(ctx, "panel");
    const int rows = maxn - c0;
    if (prec == BEM_C128) {
      if (base >= 4) panel_w<double, 4>(G, total, rows, c0, w);
      else panel_w<double, 2>(G, total, rows, c0, w);
    } else {
      if (base >= 8) panel_w<float, 8>(G, total, rows, c0, w);
      else panel_w<float, 4>(G, total, rows, c0, w);
    }
    // a panel of w columns over m rows: ~ 8 m w^2 / 2 flops, m w elements read and written
    const double es = (double)esz();
    prof_end(ctx, "panel", pi,
             work(c0, [&](int n) { const double m = n - c0, ww = std::min(w, n - c0); return 4.0 * m * ww * ww; }),
             work(c0, [&](int n) { const double m = n - c0, ww = std::min(w, n - c0); return 2.0 * es * m * ww; }));
  }
  // interchanges of rows [r0, r1) applied to columns [ca0, ca1) and [cb0, cb1)
  void laswp(int r0, int r1, int ca0, int ca1, int cb0 = 0, int cb1 = 0) {
    for (int q0 = r0; q0 < r1; q0 += kSwapRows) {
      const int q1 = std::min(r1, q0 + kSwapRows);
      int total, maxn;
      const LuGroups G = active(q0, &total, &maxn);
      if (total == 0) return;
      const int na = std::max(0, std::min(ca1, maxn) - ca0);
      const int nbc = std::max(0, std::min(cb1, maxn) - cb0);
      if (na + nbc == 0) return;
      const int pi = prof_begin(ctx, "laswp");
      if (prec == BEM_C128) {
        constexpr int LW = 8;
        hipLaunchKernelGGL((laswp_kernel<double2, LW>), dim3((na + nbc + LW - 1) / LW, total),
                           dim3(256), 0, ctx->stream, G, q0, q1, ca0, ca1, cb0, cb1);
      } else {
        constexpr int LW = 16;
        hipLaunchKernelGGL((laswp_kernel<float2, LW>), dim3((na + nbc + LW - 1) / LW, total),
                           dim3(256), 0, ctx->stream, G, q0, q1, ca0, ca1, cb0, cb1);
      }
      // at most every row of the range moves once (read and write)
      prof_end(ctx, "laswp", pi, 0.0, 2.0 * esz() * (double)(q1 - q0) * (na + nbc) * total);
    }
  }
  // C = rows [rowC, rowEnd) x cols [colC, colEnd) -= A(rows, [colA, colA+K)) B([rowB, rowB+K), cols)
  // float32 3M / 4M update through gemm_c32_lds_kernel; false (nothing
  // launched) when an operand is not 16-byte aligned (odd ld, column offset or
  // depth)
  bool gemm_lds(const LuGroups& G, int rowC, int colC, int colA, int rowB, int rowEnd, int colEnd,
                int K, int N) {
    if ((colA | colC | K) & 1) return false;
    for (int i = 0; i < G.ng; ++i)
      if (G.g[i].ld & 1) return false;
    const bool narrow = N <= std::max(64, plan.gemm_narrow_max);
    const int BN = narrow ? 64 : 128;
    GemmList W{};
    W.start[0] = 0;
    for (int i = 0; i < G.ng; ++i) {
      const int m = std::max(0, std::min(rowEnd, G.g[i].n) - rowC);
      const int nn = std::max(0, std::min(colEnd, G.g[i].n) - colC);
      W.tm[i] = std::max(1, (m + GL_BM - 1) / GL_BM);
      W.tn[i] = std::max(1, (nn + BN - 1) / BN);
      W.start[i + 1] = W.start[i] + (m > 0 && nn > 0 ? (int64_t)G.g[i].count * W.tm[i] * W.tn[i] : 0);
    }
    for (int i = G.ng + 1; i <= kMaxGroups; ++i) W.start[i] = W.start[G.ng];
    const int64_t total = W.start[G.ng];
    if (total <= 0) return true;
    // persistent form: the resident workgroups (two per CU) when the launch
    // has more tiles than that
    const int64_t resident = (int64_t)ctx->num_cus * 2 / 8 * 8;
    const bool persist = plan.gemm_persistent && ctx->gemm_queue && total > resident;
    const int64_t grid = persist ? resident : (total + 7) / 8 * 8;
    uint32_t* queue = persist ? (uint32_t*)ctx->gemm_queue : nullptr;
    const bool m3 = gkind == kGemm3M;
    const char* kname = m3 ? (narrow ? "gemm_3m_narrow" : "gemm_3m")
                           : (narrow ? "gemm_c32_narrow" : "gemm_c32");
    const int pi = prof_begin(ctx, kname);
    const dim3 gd((unsigned)grid), bd(256);
#define BEM_GEMM_LDS(M3_, WJ_)                                                                   \
  if (persist)                                                                                   \
    hipLaunchKernelGGL((gemm_c32_lds_kernel<M3_, WJ_, true>), gd, bd, 0, ctx->stream, G, W, rowC, \
                       colC, colA, rowB, rowEnd, colEnd, K, queue);                               \
  else                                                                                           \
    hipLaunchKernelGGL((gemm_c32_lds_kernel<M3_, WJ_, false>), gd, bd, 0, ctx->stream, G, W,      \
                       rowC, colC, colA, rowB, rowEnd, colEnd, K, queue);
    if (m3 && narrow) {
      BEM_GEMM_LDS(true, 1)
    } else if (m3) {
      BEM_GEMM_LDS(true, 2)
    } else if (narrow) {
      BEM_GEMM_LDS(false, 1)
    } else {
      BEM_GEMM_LDS(false, 2)
    }
#undef BEM_GEMM_LDS
    gemm_prof(kname, pi, rowC, colC, rowEnd, colEnd, K);
    return true;
  }
  // algorithmic work of C -= A B: 8 M N K flops (complex multiply-adds of the
  // 4M form), A, B read and C read and written once
  void gemm_prof(const char* kname, int pi, int rowC, int colC, int rowEnd, int colEnd, int K) {
    const double es = (double)esz();
    auto mn = [&](int n, double& m, double& nn) {
      m = std::max(0, std::min(rowEnd, n) - rowC);
      nn = std::max(0, std::min(colEnd, n) - colC);
    };
    prof_end(ctx, kname, pi,
             work(std::max(rowC, colC), [&](int n) { double m, nn; mn(n, m, nn); return 8.0 * m * nn * K; }),
             work(std::max(rowC, colC), [&](int n) {
               double m, nn; mn(n, m, nn);
               return es * (m * K + (double)K * nn + 2.0 * m * nn);
             }));
  }
  void gemm(int rowC, int colC, int colA, int rowB, int rowEnd, int colEnd, int K) {
    if (K <= 0) return;
    if (use_pack && gemm_packed(rowC, colC, colA, rowB, rowEnd, colEnd, K)) return;
    int total, maxn;
    const LuGroups G = active(std::max(rowC, colC), &total, &maxn);
    if (total == 0) return;
    const int M = std::min(rowEnd, maxn) - rowC, N = std::min(colEnd, maxn) - colC;
    if (M <= 0 || N <= 0) return;
    if (prec == BEM_C64 && (gkind == kGemm3M || gkind == kGemm4M) && !(N <= 16 && K <= 16) &&
        gemm_lds(G, rowC, colC, colA, rowB, rowEnd, colEnd, K, N))
      return;
    const char* kname = prec == BEM_C128 ? "gemm_c64"
                        : N <= 16 && K <= 16 ? "gemm_small"
                        : gkind == kGemmBf16x3 ? (N <= 64 ? "gemm_b3_narrow" : "gemm_b3")
                        : gkind == kGemm3M ? "gemm_3m_unaligned" : "gemm_c32_unaligned";
    const int pi = prof_begin(ctx, kname);
    if (prec == BEM_C128) {
      const int tn = (N + G64_BN - 1) / G64_BN, tm = (M + G64_BM - 1) / G64_BM;
      hipLaunchKernelGGL(gemm_c64_kernel, dim3(tm * tn, total), dim3(256), 0, ctx->stream, G, rowC,
                         colC, colA, rowB, rowEnd, colEnd, K, tn);
    } else {
      const int tn = (N + G32_BN - 1) / G32_BN, tm = (M + G32_BM - 1) / G32_BM;
      if (N <= 16 && K <= 16) {
        if (N <= 8 && K <= 8)
          hipLaunchKernelGGL(gemm_c32_small_kernel<8>, dim3((unsigned)((M + 63) / 64), total),
                             dim3(256), 0, ctx->stream, G, rowC, colC, colA, rowB, rowEnd, colEnd,
                             K);
        else
          hipLaunchKernelGGL(gemm_c32_small_kernel<16>, dim3((unsigned)((M + 31) / 32), total),
                             dim3(256), 0, ctx->stream, G, rowC, colC, colA, rowB, rowEnd, colEnd,
                             K);
      } else if (gkind == kGemmBf16x3 && N <= 64) {
        const int tmt = (M + GT_BM - 1) / GT_BM, tnt = (N + GT_BN - 1) / GT_BN;
        hipLaunchKernelGGL(gemm_c32_tsb_kernel, dim3(tmt * tnt, total), dim3(256), 0, ctx->stream,
                           G, rowC, colC, colA, rowB, rowEnd, colEnd, K, tnt);
      } else if (gkind == kGemmBf16x3) {
        const int tmb = (M + GB_BM - 1) / GB_BM, tnb = (N + GB_BN - 1) / GB_BN;
        const int gx = (tmb * tnb + 7) / 8 * 8;
        hipLaunchKernelGGL(gemm_c32_b3_kernel, dim3(gx, total), dim3(256), 0, ctx->stream, G,
                           rowC, colC, colA, rowB, rowEnd, colEnd, K, tmb, tnb);
      }
      else if (gkind == kGemm3M)
        hipLaunchKernelGGL(gemm_c32_3m_kernel, dim3(tm * tn, total), dim3(256), 0, ctx->stream, G,
                           rowC, colC, colA, rowB, rowEnd, colEnd, K, tn);
      else
        hipLaunchKernelGGL(gemm_c32_kernel, dim3(tm * tn, total), dim3(256), 0, ctx->stream, G,
                           rowC, colC, colA, rowB, rowEnd, colEnd, K, tn);
    }
    gemm_prof(kname, pi, rowC, colC, rowEnd, colEnd, K);
  }
  // matrices [b0, b1) of the concatenation of G's groups
  static LuGroups slice(const LuGroups& G, int b0, int b1, size_t es) {
    LuGroups S{};
    S.ng = 0;
    int base = 0;
    for (int i = 0; i < G.ng; ++i) {
      const LuGroup& g = G.g[i];
      const int lo = std::max(b0, base), hi = std::min(b1, base + g.count);
      if (lo < hi) {
        LuGroup t = g;
        const int off = lo - base;
        t.A = (char*)g.A + (size_t)off * g.stride * es;
        t.piv = g.piv + (size_t)off * g.n;
        t.info = g.info + off;
        t.count = hi - lo;
        S.g[S.ng++] = t;
      }
      base += g.count;
    }
    return S;
  }
  // packing buffer bytes that would let every trailing update run in one slice
  size_t pack_need(int nb) const {
    size_t need = 0;
    for (int c = 0; c < nmax; c = block_end(c, nb)) {
      const int e = block_end(c, nb);
      int total, maxn;
      active(e, &total, &maxn);
      if (total == 0) continue;
      need = std::max(need, (size_t)pack_words(maxn - e, maxn - e, e - c) * 16 * total);
    }
    return need;
  }
  // C -= A B through the pre-split operands, in slices of the batch that fit
  // the packing buffer; false (nothing launched) when not even one matrix
  // fits or the update is too small for packing to pay
  bool gemm_packed(int rowC, int colC, int colA, int rowB, int rowEnd, int colEnd, int K) {
    if (K <= 0) return true;
    int total, maxn;
    const LuGroups G = active(std::max(rowC, colC), &total, &maxn);
    if (total == 0) return true;
    const int M = std::min(rowEnd, maxn) - rowC, N = std::min(colEnd, maxn) - colC;
    if (M <= 0 || N <= 0) return true;
    // each packed operand must be read by at least four tiles to repay its
    // pass (measured: at two or three, the pass costs more than it saves)
    if (M < 4 * GB_BM || N < 4 * GB_BN) return false;
    const size_t per = (size_t)pack_words(M, N, K) * 16;
    const int fit = (int)std::min<size_t>((size_t)total, pack ? pack_bytes / per : 0);
    if (fit <= 0) return false;
    const int tiles_m = (M + GB_BM - 1) / GB_BM, tiles_n = (N + GB_BN - 1) / GB_BN;
    const int S8 = (K + 7) / 8;
    const int64_t a_ms = (int64_t)tiles_m * S8 * GP_BLK, b_ms = (int64_t)tiles_n * S8 * GP_BLK;
    uint4* Ap = (uint4*)pack;
    uint4* Bp = Ap + a_ms * fit;
    const int64_t ta = (int64_t)tiles_m * S8 * GB_BM, tb = (int64_t)tiles_n * S8 * (GP_BLK / 2);
    const int gx = (tiles_m * tiles_n + 7) / 8 * 8;
    for (int b0 = 0; b0 < total; b0 += fit) {
      const int nbat = std::min(fit, total - b0);
      const LuGroups Gs = slice(G, b0, b0 + nbat, esz());
      double mk = 0.0, kn = 0.0, mn = 0.0;
      for (int i = 0; i < Gs.ng; ++i) {
        const double m = std::max(0, std::min(rowEnd, Gs.g[i].n) - rowC);
        const double nn = std::max(0, std::min(colEnd, Gs.g[i].n) - colC);
        mk += m * K * Gs.g[i].count;
        kn += nn * K * Gs.g[i].count;
        mn += m * nn * Gs.g[i].count;
      }
      int pi = prof_begin(ctx, "pack");
      hipLaunchKernelGGL(pack_a_kernel, dim3((unsigned)((ta + 255) / 256), nbat), dim3(256), 0,
                         ctx->stream, Gs, rowC, colA, rowEnd, K, tiles_m, a_ms, Ap);
      hipLaunchKernelGGL(pack_b_kernel, dim3((unsigned)((tb + 255) / 256), nbat), dim3(256), 0,
                         ctx->stream, Gs, rowB, colC, colEnd, K, tiles_n, b_ms, Bp);
      // float32 operands read, split words written (8 bytes per complex element each way)
      prof_end(ctx, "pack", pi, 0.0, 16.0 * (mk + kn));
      pi = prof_begin(ctx, "gemm_b3_packed");
      hipLaunchKernelGGL(gemm_c32_b3p_kernel, dim3(gx, nbat), dim3(256), 0, ctx->stream, Gs, rowC,
                         colC, rowEnd, colEnd, K, tiles_m, tiles_n, Ap, a_ms, Bp, b_ms);
      prof_end(ctx, "gemm_b3_packed", pi, 8.0 * mn * K, 8.0 * (mk + kn + 2.0 * mn));
    }
    return true;
  }
  // X = L^{-1} X for rows [r0, r0+m1) and columns [col0, col1)
  void trsm(int r0, int m1, int col0, int col1) {
    if (col1 <= col0 || m1 <= 1) return;
    if (m1 <= 32) {
      int total, maxn;
      const LuGroups G = active(r0 + 1, &total, &maxn);
      if (total == 0) return;
      const int ncol = std::min(col1, maxn) - col0;
      if (ncol <= 0) return;
      dim3 grid((ncol + 255) / 256, total);
      const int pi = prof_begin(ctx, "trsm");
      if (prec == BEM_C128)
        hipLaunchKernelGGL(trsm_kernel<double2>, grid, dim3(256), 0, ctx->stream, G, r0, m1, col0, col1);
      else
        hipLaunchKernelGGL(trsm_kernel<float2>, grid, dim3(256), 0, ctx->stream, G, r0, m1, col0, col1);
      prof_end(ctx, "trsm", pi, 4.0 * m1 * m1 * (double)ncol * total,
               2.0 * esz() * m1 * (double)ncol * total);
      return;
    }
    int h1 = ((m1 / 2) + 31) / 32 * 32;
    if (h1 >= m1) h1 = m1 - 32;
    trsm(r0, h1, col0, col1);
    gemm(r0 + h1, col0, r0, r0, r0 + m1, col1, h1);
    trsm(r0 + h1, m1 - h1, col0, col1);
  }
  int split(int w) const {
    int h = (w / 2 + base - 1) / base * base;
    if (h >= w) h = w - base;
    return h;
  }
  void rec(int c0, int c1) {
    const int w = c1 - c0;
    if (w <= base) { panel(c0, w); return; }
    const int h = split(w);
    rec(c0, c0 + h);
    laswp(c0, c0 + h, c0 + h, c1);
    trsm(c0, h, c0 + h, c1);
    gemm(c0 + h, c0 + h, c0, c0, INT32_MAX, c1, h);
    rec(c0 + h, c1);
    laswp(c0 + h, c1, c0, c0 + h);
  }
  // Right-looking blocked top level: factor a block of nb columns (recursively),
  // apply its interchanges to every column left and right of it in one pass,
  // then the block row of U and the trailing update.
  // end of the block of nb columns starting at column c
  int block_end(int c, int nb) const { return std::min(nmax, c + nb); }
  void blocked(int nb) {
    for (int c = 0; c < nmax; c = block_end(c, nb)) {
      const int e = block_end(c, nb);
      rec(c, e);
      laswp(c, e, 0, c, e, nmax);
      trsm(c, e - c, e, nmax);
      gemm(e, e, c, c, INT32_MAX, nmax, e - c);
    }
  }
};

}  // namespace

int lu_default_nb(bem_prec prec, int n) {
  (void)prec;
  // wide blocks cut the trailing-update traffic of large matrices (measured:
  // 512 beats 256 by 5 % at n = 5124 in a batch of 512)
  return n >= 4096 ? 2 * kSwapRows : kSwapRows;
}

int lu_plan_nb(bem_ctx* ctx, bem_prec prec, int gemm_kind, int n) {
  const auto it = ctx->tuned.find({(int)prec * 16 + gemm_kind, (n + 511) / 512 * 512});
  return it != ctx->tuned.end() ? it->second.nb : lu_default_nb(prec, n);
}

LuPlan lu_plan_for(bem_ctx* ctx, bem_prec prec, int gemm_kind, int n, int nb) {
  LuPlan plan;
  plan.nb = nb > 0 ? nb : lu_plan_nb(ctx, prec, gemm_kind, n);
  const auto it = ctx->tuned.find({(int)prec * 16 + gemm_kind, (n + 511) / 512 * 512});
  if (it != ctx->tuned.end()) {
    plan.gemm_narrow_max = it->second.narrow_max;
    plan.gemm_persistent = it->second.persistent;
  }
  return plan;
}

// Validate the sets and set up the driver: groups sorted by size, base panel
// width and top-level block width.
static bem_status build_fac(bem_ctx* ctx, bem_prec prec, const std::vector<LuMatrixSet>& sets,
                            const LuPlan& plan, int gemm_kind, Fac& f, int& nb) {
  f.ctx = ctx;
  f.prec = prec;
  f.plan = plan;
  f.gkind = prec == BEM_C64 ? (gemm_kind == kGemmBf16x3Unpacked ? kGemmBf16x3 : gemm_kind) : kGemm4M;
  f.use_pack = prec == BEM_C64 && gemm_kind == kGemmBf16x3;
  for (const LuMatrixSet& s : sets) {
    if (s.count <= 0 || s.n <= 0) continue;
    if (s.n > 24 * kPanelThreads)
      return fail(ctx, BEM_EUNSUPPORTED, "lu_factor: n=%d above the supported %d", s.n,
                  24 * kPanelThreads);
    if ((int64_t)s.n * s.ld >= ((int64_t)1 << 31))
      return fail(ctx, BEM_EUNSUPPORTED, "lu_factor: n*ld = %lld must stay below 2^31",
                  (long long)s.n * s.ld);
    LuGroup g{};
    g.A = s.A;
    g.piv = s.piv;
    g.info = s.info;
    g.ld = s.ld;
    g.stride = s.stride;
    g.n = s.n;
    g.count = s.count;
    f.groups.push_back(g);
  }
  if (f.groups.empty()) return BEM_OK;
  if ((int)f.groups.size() > kMaxGroups)
    return fail(ctx, BEM_EUNSUPPORTED, "lu_factor: more than %d matrix sizes in one batch", kMaxGroups);
  std::sort(f.groups.begin(), f.groups.end(), [](const LuGroup& a, const LuGroup& b) { return a.n > b.n; });
  f.nmax = f.groups[0].n;
  const int rows_per_thread = (f.nmax + kPanelThreads - 1) / kPanelThreads;
  if (prec == BEM_C128) f.base = rows_per_thread <= 10 ? 4 : 2;
  else f.base = rows_per_thread <= 11 ? 8 : 4;
  if (plan.base > 0 && plan.base < f.base) f.base = plan.base;
  // block width (the interchange passes are split into ranges of kSwapRows rows)
  nb = plan.nb > 0 ? std::min(plan.nb, 4 * kSwapRows) : kSwapRows;
  return BEM_OK;
}

// Grow the context's packing buffer towards what the factorisation would use
// (at most pack_cap); on allocation failure the buffer stays empty and the
// trailing updates take the unpacked kernel.
static size_t pack_cap(const bem_ctx* ctx) {
  return ctx->ws_limit ? std::min<size_t>(kPackLimit, ctx->ws_limit / 4) : kPackLimit;
}
static void reserve_pack(bem_ctx* ctx, const Fac& f, int nb) {
  const size_t want = std::min(f.pack_need(nb), pack_cap(ctx));
  if (want <= ctx->pack_size) return;
  (void)hipStreamSynchronize(ctx->stream);
  drop_graphs(ctx);   // captured factorisations point into the old buffer
  if (ctx->pack) (void)hipFree(ctx->pack);
  ctx->pack = nullptr;
  ctx->pack_size = 0;
  if (hipMalloc(&ctx->pack, want) != hipSuccess) {
    (void)hipGetLastError();
    ctx->pack = nullptr;
    return;
  }
  ctx->pack_size = want;
}

static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

bem_status lu_factor_groups(bem_ctx* ctx, bem_prec prec, const std::vector<LuMatrixSet>& sets,
                            const LuPlan& plan, int gemm_kind) {
  Fac f;
  int nb = 0;
  bem_status st = build_fac(ctx, prec, sets, plan, gemm_kind, f, nb);
  if (st != BEM_OK || f.groups.empty()) return st;
  for (const LuGroup& g : f.groups)
    hipLaunchKernelGGL(fill_i32_kernel, dim3((g.count + 255) / 256), dim3(256), 0, ctx->stream,
                       (int64_t)g.count, g.info, 0);
  if (f.use_pack) {
    // under capture the buffer was reserved before the capture began
    if (!capturing(ctx->stream)) reserve_pack(ctx, f, nb);
    f.pack = ctx->pack;
    f.pack_bytes = std::min(ctx->pack_size, pack_cap(ctx));
  }
  f.blocked(nb);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

// Deterministic pseudo-random matrices for timing: entries uniform in the unit
// square (a splitmix-style hash of the index), diagonal raised by n/2.
template <typename C>
__global__ void tune_fill_kernel(int n, int64_t ld, int64_t stride, int batch, C* A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)batch * stride) return;
  const int64_t in = t % stride;
  const int64_t i = in / ld, j = in % ld;
  uint64_t z = (uint64_t)t * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  double re = (double)(z & 0xFFFFFF) / 16777216.0 - 0.5;
  const double im = (double)((z >> 24) & 0xFFFFFF) / 16777216.0 - 0.5;
  if (i == j) re += 0.5 * n;
  C v;
  v.x = (decltype(v.x))(j < n ? re : 0.0);
  v.y = (decltype(v.y))(j < n ? im : 0.0);
  A[t] = v;
}

bem_status lu_autotune(bem_ctx* ctx, bem_prec prec, int n, int batch, int gemm_kind,
                       const int32_t* candidates, int32_t* best_nb, double* best_ms) {
  static const int32_t kDefault[] = {256, 384, 512, 768, 1024, 0};
  const int32_t* cand = candidates ? candidates : kDefault;
  const int64_t ld = (n + 15) / 16 * 16, stride = (int64_t)n * ld;
  const size_t esz = prec == BEM_C128 ? 16 : 8;
  void* A = nullptr;
  int32_t* piv = nullptr;
  if (hipMalloc(&A, esz * (size_t)stride * batch + (size_t)batch * (n + 1) * 4) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, BEM_ENOMEM, "autotune: %d matrices of n = %d do not fit", batch, n);
  }
  piv = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(A) + esz * (size_t)stride * batch);
  int32_t* info = piv + (size_t)batch * n;
  hipEvent_t e0, e1;
  BEM_HIP_TRY(ctx, hipEventCreate(&e0));
  BEM_HIP_TRY(ctx, hipEventCreate(&e1));
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  // GEMM shapes tried with every block width: the float32 MFMA forms (4M,
  // 3M) also try 128 x 64 tiles up to 128 columns and persistent launches
  const bool lds_forms = prec == BEM_C64 && (gemm_kind == kGemm4M || gemm_kind == kGemm3M);
  static const int kShapes[3][2] = {{64, 0}, {128, 0}, {64, 1}};
  const int n_shapes = lds_forms ? 3 : 1;
  int best = 0, best_narrow = 64, best_persist = 0;
  float bms = 0.f;
  bem_status st = BEM_OK;
  ctx->tune_log.clear();
  for (int c = 0; cand[c] > 0 && st == BEM_OK; ++c)
  for (int sh = 0; sh < n_shapes && st == BEM_OK; ++sh) {
    LuPlan plan;
    plan.nb = cand[c];
    plan.gemm_narrow_max = kShapes[sh][0];
    plan.gemm_persistent = kShapes[sh][1];
    float ms_min = 0.f;
    for (int rep = 0; rep < 2 && st == BEM_OK; ++rep) {
      const int64_t total = (int64_t)batch * stride;
      if (prec == BEM_C128)
        hipLaunchKernelGGL(tune_fill_kernel<double2>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                           ctx->stream, n, ld, stride, batch, (double2*)A);
      else
        hipLaunchKernelGGL(tune_fill_kernel<float2>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                           ctx->stream, n, ld, stride, batch, (float2*)A);
      (void)hipEventRecord(e0, ctx->stream);
      st = lu_factor(ctx, prec, n, ld, stride, batch, A, piv, info, plan, gemm_kind);
      (void)hipEventRecord(e1, ctx->stream);
      if (hipEventSynchronize(e1) != hipSuccess) st = fail(ctx, BEM_EHIP, "autotune: event");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep == 0 || ms < ms_min) ms_min = ms;
    }
    if (st == BEM_OK)
      ctx->tune_log.push_back({bem_ctx::TunedPlan{cand[c], kShapes[sh][0], kShapes[sh][1]}, ms_min});
    if (st == BEM_OK && (best == 0 || ms_min < bms)) {
      best = cand[c];
      best_narrow = kShapes[sh][0];
      best_persist = kShapes[sh][1];
      bms = ms_min;
    }
  }
  ctx->profiling = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(A);
  if (st != BEM_OK) return st;
  if (best == 0) return fail(ctx, BEM_EINVAL, "autotune: no candidate block width");
  ctx->tuned[{(int)prec * 16 + gemm_kind, (n + 511) / 512 * 512}] =
      bem_ctx::TunedPlan{best, best_narrow, best_persist};
  if (best_nb) *best_nb = best;
  if (best_ms) *best_ms = bms;
  return BEM_OK;
}

void drop_graphs(bem_ctx* ctx) {
  for (auto& g : ctx->lu_graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  ctx->lu_graphs.clear();
}

bem_status lu_factor_groups_graph(bem_ctx* ctx, bem_prec prec, const std::vector<LuMatrixSet>& sets,
                                  const LuPlan& plan, int gemm_kind) {
  std::vector<int64_t> key{(int64_t)prec, plan.nb, plan.base, plan.gemm_narrow_max,
                           plan.gemm_persistent, gemm_kind, (int64_t)sets.size()};
  for (const LuMatrixSet& m : sets) {
    key.push_back((int64_t)(intptr_t)m.A);
    key.push_back((int64_t)(intptr_t)m.piv);
    key.push_back((int64_t)(intptr_t)m.info);
    key.push_back(m.ld);
    key.push_back(m.stride);
    key.push_back(m.n);
    key.push_back(m.count);
  }
  for (auto& g : ctx->lu_graphs)
    if (g.key == key) {
      BEM_HIP_TRY(ctx, hipGraphLaunch(g.exec, ctx->stream));
      return BEM_OK;
    }
  {
    // the packing buffer must exist before capture (no allocation while capturing)
    Fac f;
    int nb = 0;
    const bem_status st = build_fac(ctx, prec, sets, plan, gemm_kind, f, nb);
    if (st != BEM_OK) return st;
    if (!f.groups.empty() && f.use_pack) reserve_pack(ctx, f, nb);
  }
  if (!ctx->capture_stream)
    BEM_HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
  // record the launch sequence on the side stream (nothing executes), then
  // launch the instantiated graph on the context stream
  hipStream_t saved = ctx->stream;
  ctx->stream = ctx->capture_stream;
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  BEM_HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
  const bem_status st = lu_factor_groups(ctx, prec, sets, plan, gemm_kind);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(ctx->capture_stream, &graph);
  ctx->stream = saved;
  ctx->profiling = prof;
  if (st != BEM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess)
    return fail(ctx, BEM_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess)
    return fail(ctx, BEM_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
  if (ctx->lu_graphs.size() >= 8) {
    (void)hipGraphExecDestroy(ctx->lu_graphs.front().exec);
    ctx->lu_graphs.erase(ctx->lu_graphs.begin());
  }
  ctx->lu_graphs.push_back(bem_ctx::LuGraph{key, exec});
  BEM_HIP_TRY(ctx, hipGraphLaunch(exec, ctx->stream));
  return BEM_OK;
}

bem_status lu_factor(bem_ctx* ctx, bem_prec prec, int n, int64_t ld, int64_t stride, int batch,
                     void* A, int32_t* piv, int32_t* info, const LuPlan& plan, int gemm_kind) {
  if (batch <= 0 || n <= 0) return BEM_OK;
  std::vector<LuMatrixSet> sets(1);
  sets[0] = LuMatrixSet{A, piv, info, ld, stride, n, batch};
  return lu_factor_groups(ctx, prec, sets, plan, gemm_kind);
}

bem_status lu_perm(bem_ctx* ctx, int n, int batch, const int32_t* piv, int32_t* perm) {
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)perm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(perm_kernel, dim3(batch), dim3(256), sizeof(int32_t) * n, ctx->stream, n,
                     piv, perm);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

bem_status lu_solve_perm(bem_ctx* ctx, bem_prec prec, int n, int64_t ld, int64_t stride,
                         int batch, const void* LU, const int32_t* perm, int n_rhs,
                         const void* Bin, void* X, int64_t bstride, const int32_t* fac_index,
                         const int32_t* vidx, int n_sel) {
  if (vidx) batch = n_sel;
  if (batch <= 0 || n_rhs <= 0) return BEM_OK;
  dim3 grid(batch * n_rhs);
  const size_t esz = prec == BEM_C128 ? 16 : 8;
  const size_t base_lds = esz * (size_t)(TS_B * (TS_B + 1) + TS_B);
  const bool xlds = base_lds + esz * (size_t)n <= 150 * 1024;
  const size_t lds = base_lds + (xlds ? esz * (size_t)n : 0);
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)getrs_kernel<double, true>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipFuncSetAttribute((const void*)getrs_kernel<float, true>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipFuncSetAttribute((const void*)getrs_kernel<double, false>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipFuncSetAttribute((const void*)getrs_kernel<float, false>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const int pi = prof_begin(ctx, "getrs");
  if (prec == BEM_C128) {
    if (xlds)
      hipLaunchKernelGGL((getrs_kernel<double, true>), grid, dim3(TS_T), lds, ctx->stream, n, ld,
                         stride, (const double2*)LU, perm, n_rhs, (const double2*)Bin,
                         (double2*)X, bstride, fac_index, vidx);
    else
      hipLaunchKernelGGL((getrs_kernel<double, false>), grid, dim3(TS_T), lds, ctx->stream, n, ld,
                         stride, (const double2*)LU, perm, n_rhs, (const double2*)Bin,
                         (double2*)X, bstride, fac_index, vidx);
  } else {
    if (xlds)
      hipLaunchKernelGGL((getrs_kernel<float, true>), grid, dim3(TS_T), lds, ctx->stream, n, ld,
                         stride, (const float2*)LU, perm, n_rhs, (const float2*)Bin, (float2*)X,
                         bstride, fac_index, vidx);
    else
      hipLaunchKernelGGL((getrs_kernel<float, false>), grid, dim3(TS_T), lds, ctx->stream, n, ld,
                         stride, (const float2*)LU, perm, n_rhs, (const float2*)Bin, (float2*)X,
                         bstride, fac_index, vidx);
  }
  prof_end(ctx, "getrs", pi, 8.0 * (double)n * n * n_rhs * batch,
           (double)esz * ((double)n * n + 3.0 * n * n_rhs) * batch);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

}  // namespace bem
