// Space-time synthesis: inverse DFT over the solved frequencies (Sec. III,
// last paragraph: the inverse Fourier transform of the frequency-domain
// solution by FFT; Sec. IV: the incident pulse train enters as its Fourier
// coefficients c_m).  For each pulse q and point x,
//   p_q(x, t_n) = sum_{m=1}^{F} alpha_m Re[c_qm X_m(x) e^{-2 pi i m n/T}],
// alpha_m = 2 (m < T/2), 1 (m = T/2).  With Y_m = conj(c_qm X_m) this is the
// unnormalised inverse real DFT of the half spectrum Y, computed as one
// complex FFT of length H = T/2 on the packed sequence
//   W_m = (Y_m + conj Y_{H-m}) + i e^{2 pi i m/T} (Y_m - conj Y_{H-m}),
// whose output z_n gives p_{2n} = Re z_n, p_{2n+1} = Im z_n.
//
// Layout of the work: a workgroup takes groups of G = max(2048, H) / H points
// in turn (its twiddle table e^{2 pi i j/T}, j < H/2, built once: the other
// quarter turn is i times it), reads their
// rows of U once into registers, and for every pulse packs W in pairs (m, H - m),
// runs the FFT in place in one LDS buffer of G H values, and writes the pulse
// as T contiguous floats per point.  The FFT is a Stockham autosort
// transform with radix-8 stages (a last radix-4 or radix-2 stage when log2 H
// is not a multiple of 3): every thread loads its butterflies' values into
// registers, the workgroup synchronises, and the twiddled 8-point transforms
// are written back, so a length-2048 transform takes 4 passes over LDS
// instead of the 11 of a radix-2 transform; the last stage's outputs go
// straight to HBM (its output positions are consecutive across lanes).  The
// buffer holds one padding slot after every 8 values, which keeps the strided
// stores of the first stages free of LDS bank conflicts.  HBM traffic: 8 F
// bytes read per point, 4 T bytes written per point and pulse; the float32
// copy of the coefficients is read from L2.
//
// Sparse form (Sec. IV: the space-time field rebuilt from only the frequencies
// of largest incident amplitude): U and c hold n_sel columns whose frequency
// indices m_j are listed; every other bin of the half spectrum is zero.  An LDS
// map from bin to column replaces the dense indexing, the FFT is unchanged.
#include <algorithm>

#include "common.h"

namespace bem {
namespace {

constexpr int kST = 256;

__device__ inline float2 cm(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// i a
__device__ inline float2 ci(float2 a) { return make_float2(-a.y, a.x); }

// inverse (e^{+2 pi i r k / R}) DFTs of length 2, 4, 8 in registers
__device__ inline void idft2(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ inline void idft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  const float2 s02 = cadd(v0, v2), d02 = csub(v0, v2);
  const float2 s13 = cadd(v1, v3), d13 = ci(csub(v1, v3));
  v0 = cadd(s02, s13);
  v2 = csub(s02, s13);
  v1 = cadd(d02, d13);
  v3 = csub(d02, d13);
}
__device__ inline void idft4(float2* v) { idft4(v[0], v[1], v[2], v[3]); }
__device__ inline void idft8(float2* v) {
  // even and odd halves, then X_k = E_k + w^k O_k, X_{k+4} = E_k - w^k O_k,
  // w = e^{i pi/4}
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  idft4(e0, e1, e2, e3);
  idft4(o0, o1, o2, o3);
  const float h = 0.70710678118654752f;
  const float2 w1 = make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y));   // (1 + i)/sqrt2 o1
  const float2 w2 = ci(o2);                                               // i o2
  const float2 w3 = make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y));  // (-1 + i)/sqrt2 o3
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1);
  v[5] = csub(e1, w1);
  v[2] = cadd(e2, w2);
  v[6] = csub(e2, w2);
  v[3] = cadd(e3, w3);
  v[7] = csub(e3, w3);
}
template <int R>
__device__ inline void idft(float2* v) {
  if (R == 8) idft8(v);
  else if (R == 4) idft4(v);
  else idft2(v);
}

// position of value i in the padded buffer
__device__ inline int pad(int i) { return i + (i >> 3); }

// One Stockham stage of radix R over the SLOTS values of buf (SLOTS / H
// transforms of length H = 2^LOGH, each contiguous, stored padded); Ns =
// 2^LOGNS is the length of the sub-transforms already combined.  In place:
// all loads, a barrier, then all stores and a barrier.  The last stage
// (Ns R = H) stores transform g's output n as float2 n of outq + (p0 + g) T
// instead, for the points below m.  Every stride is a compile-time constant,
// so the LDS accesses of a butterfly share one address and differ by
// immediate offsets.
template <int R, int SLOTS, int LOGH, int LOGNS, bool LAST>
__device__ inline void fft_stage(float2* buf, const float2* tw, float* __restrict__ outq, int p0,
                                 int m) {
  constexpr int LR = R == 8 ? 3 : (R == 4 ? 2 : 1);
  constexpr int H = 1 << LOGH, T = 2 * H, LOGT = LOGH + 1;
  constexpr int PER = SLOTS / kST / R;   // butterflies per thread
  constexpr int LOGNB = LOGH - LR;       // butterflies per transform: H / R
  constexpr int NB = 1 << LOGNB, NS = 1 << LOGNS;
  // the thread index is made opaque so that no index of this stage is
  // computed once and kept in registers across the enclosing loops
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  float2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bt = tid + i * kST;
    const int g = bt >> LOGNB, j = bt & (NB - 1);
    const int s0 = (g << LOGH) + j;
    if constexpr (NB % 8 == 0) {
      // pad(s0 + r NB) = pad(s0) + r (NB + NB / 8)
      const float2* src = buf + pad(s0);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * (NB + NB / 8)];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[pad(s0 + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bt = tid + i * kST;
    const int g = bt >> LOGNB, j = bt & (NB - 1);
    const int jm = j & (NS - 1);
    if constexpr (LOGNS > 0) {
      // twiddles w^r, w = e^{2 pi i jm / (Ns R)} = e^{2 pi i (jm 2^{LOGT - LOGNS - LR}) / T}:
      // w from the table (its index is below T / R <= H), its powers by products
      float2 w1;
      if constexpr (R == 2) {
        // index below H: the second quarter turn is i times the first
        const int ix = jm << (LOGT - LOGNS - LR);
        const float2 tq = tw[ix & (H / 2 - 1)];
        w1 = (ix & (H / 2)) ? ci(tq) : tq;
      } else {
        w1 = tw[jm << (LOGT - LOGNS - LR)];   // index below T / 4 = H / 2
      }
      v[i][1] = cm(v[i][1], w1);
      if constexpr (R >= 4) {
        const float2 w2 = cm(w1, w1), w3 = cm(w2, w1);
        v[i][2] = cm(v[i][2], w2);
        v[i][3] = cm(v[i][3], w3);
        if constexpr (R == 8) {
          const float2 w4 = cm(w2, w2);
          v[i][4] = cm(v[i][4], w4);
          v[i][5] = cm(v[i][5], cm(w4, w1));
          v[i][6] = cm(v[i][6], cm(w4, w2));
          v[i][7] = cm(v[i][7], cm(w4, w3));
        }
      }
    }
    idft<R>(v[i]);
    if constexpr (LAST) {
      // j < Ns here, so the outputs sit at j + r Ns
      if (p0 + g < m) {
        float2* o = reinterpret_cast<float2*>(outq + (int64_t)(p0 + g) * T) + j;
#pragma unroll
        for (int r = 0; r < R; ++r) o[r * NS] = v[i][r];
      }
    } else {
      // destination (j / Ns) Ns R + jm + r Ns: with Ns = 1 the R values are
      // consecutive from a multiple of 8, else Ns is a multiple of 8; either
      // way pad(d + r Ns) = pad(d) + r pad(Ns)
      const int d = (g << LOGH) + ((j >> LOGNS) << (LOGNS + LR)) + jm;
      float2* dst = buf + pad(d);
      constexpr int DS = NS == 1 ? 1 : NS + NS / 8;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * DS] = v[i][r];
    }
  }
  if constexpr (!LAST) __syncthreads();
}

// the stages of a length-H transform from sub-transform length 2^LOGNS on:
// radix 8 while more than 3 doublings remain, then a last radix-8, -4 or -2
template <int SLOTS, int LOGH, int LOGNS>
__device__ inline void fft_run(float2* buf, const float2* tw, float* __restrict__ outq, int p0,
                               int m) {
  constexpr int REM = LOGH - LOGNS;
  if constexpr (REM > 3) {
    fft_stage<8, SLOTS, LOGH, LOGNS, false>(buf, tw, outq, p0, m);
    fft_run<SLOTS, LOGH, LOGNS + 3>(buf, tw, outq, p0, m);
  } else if constexpr (REM == 3) {
    fft_stage<8, SLOTS, LOGH, LOGNS, true>(buf, tw, outq, p0, m);
  } else if constexpr (REM == 2) {
    fft_stage<4, SLOTS, LOGH, LOGNS, true>(buf, tw, outq, p0, m);
  } else {
    fft_stage<2, SLOTS, LOGH, LOGNS, true>(buf, tw, outq, p0, m);
  }
}

// W_m and W_{H-m} of one pair from Y_m, Y_{H-m}
__device__ inline float2 wpack(float2 ya, float2 yb, float2 t) {
  const float2 e = make_float2(ya.x + yb.x, ya.y - yb.y);   // ya + conj yb
  const float2 o = make_float2(ya.x - yb.x, ya.y + yb.y);   // ya - conj yb
  return cadd(e, cm(ci(t), o));                             // + i t o
}

// LDS: tw[H / 2] (a quarter turn); buf[SLOTS + SLOTS / 8] (padded); (sparse) col[H + 1]: column
// of bin m, or -1.  Thread item i (i < NW) of a group is the pair of bins
// (mm, H - mm), mm = (tid + i * 256) mod H/2, of point p0 + (tid + i * 256) /
// (H/2), with (H, H/2) in place of (0, H): the thread loads exactly the two
// columns of U it packs, so U needs no LDS copy.  cbin[q][j] (j = 0..H) holds
// pulse q's coefficient of bin j, 0 where no frequency was solved: a bin
// without a column then gives Y_j = 0 from any finite X, and no load or
// product needs a condition.
template <bool Sparse, int LOGH>
__global__ __launch_bounds__(kST, LOGH < 12 ? 5 : 1) void synth_kernel(
    int m, int n_k, const float2* __restrict__ U, const int32_t* __restrict__ midx, int n_pulse,
    const float2* __restrict__ cbin, int add_incident, const double* __restrict__ xp, double dk,
    float* __restrict__ out) {
  extern __shared__ float2 lds[];
  constexpr int H = 1 << LOGH, T = 2 * H;
  constexpr int SLOTS = H > 2048 ? H : 2048;
  constexpr int G = SLOTS / H;   // points per group
  constexpr int halfH = H >> 1;
  constexpr int NW = SLOTS / 2 / kST;   // pair items per thread
  float2* tw = lds;   // e^{2 pi i j / T}, j < H / 2 (a quarter turn)
  float2* buf = tw + halfH;
  int* col = reinterpret_cast<int*>(buf + SLOTS + SLOTS / 8);
  int tid = threadIdx.x;
  for (int j = tid; j < halfH; j += kST) {
    float s, co;
    sincospif(2.0f * (float)j / (float)T, &s, &co);
    tw[j] = make_float2(co, s);
  }
  if (Sparse) {
    for (int j = tid; j <= H; j += kST) col[j] = -1;
    __syncthreads();
    for (int j = tid; j < n_k; j += kST) col[midx[j]] = j;
  }
  __syncthreads();   // tw and col are complete
  const int ngroups = (m + G - 1) / G;
  // a valid column for bin j: its own, or (no frequency solved there, its
  // coefficient 0) column 0 or n_k - 1
  auto colof = [&](int j) -> int {
    return Sparse ? max(col[j], 0) : min(j, n_k) - 1;
  };
  auto bin_a = [&](int i) { const int mm = (tid + i * kST) & (halfH - 1); return mm ? mm : H; };
  auto bin_b = [&](int i) { const int mm = (tid + i * kST) & (halfH - 1); return mm ? H - mm : halfH; };
  // Registers: the next group's U values of this thread's bins (loaded while
  // the current group's transforms run) and the current pulse's coefficients
  // of the same bins (the next pulse's loaded during the current FFT).
  float2 ua[NW], ub[NW], xa[NW], xb[NW], ca[NW], cb[NW];
  auto load_u = [&](int grp) {
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      // points past m read the last point (their outputs are not stored)
      const int p = min(grp * G + ((tid + i * kST) >> (LOGH - 1)), m - 1);
      ua[i] = U[(int64_t)p * n_k + colof(bin_a(i))];
      ub[i] = U[(int64_t)p * n_k + colof(bin_b(i))];
    }
  };
  auto load_c = [&](int q) {
    const float2* cq = cbin + (int64_t)q * (H + 1);
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      ca[i] = cq[bin_a(i)];
      cb[i] = cq[bin_b(i)];
    }
  };
  // e^{i k_j z} of bin j (k_j = j dk), phase reduced in float64
  auto incident = [&](int j, double z) -> float2 {
    double t = (double)j * dk * z * 0.15915494309189533576888376337251;
    t -= rint(t);
    float sn, co;
    sincospif(2.0f * (float)t, &sn, &co);
    return make_float2(co, sn);
  };
  load_u(blockIdx.x);
  load_c(0);
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int p0 = grp * G;
    asm volatile("" : "+v"(tid));
    // the group's field at the thread's bins (scattered + incident)
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      xa[i] = ua[i];
      xb[i] = ub[i];
      if (add_incident) {
        const double z = xp[3 * min(p0 + ((tid + i * kST) >> (LOGH - 1)), m - 1) + 2];
        xa[i] = cadd(xa[i], incident(bin_a(i), z));
        xb[i] = cadd(xb[i], incident(bin_b(i), z));
      }
    }
    load_u(grp + gridDim.x < ngroups ? grp + gridDim.x : grp);
    for (int q = 0; q < n_pulse; ++q) {
      // indices are recomputed per pulse from an opaque thread index (kept
      // out of registers across the FFT)
      asm volatile("" : "+v"(tid));
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const int e = tid + i * kST;
        const int w = (e >> (LOGH - 1)) << LOGH, mm = e & (halfH - 1);
        // Y = conj(c X) of the pair's bins
        const float2 ya = make_float2(ca[i].x * xa[i].x - ca[i].y * xa[i].y,
                                      -(ca[i].x * xa[i].y + ca[i].y * xa[i].x));
        const float2 yb = make_float2(cb[i].x * xb[i].x - cb[i].y * xb[i].y,
                                      -(cb[i].x * xb[i].y + cb[i].y * xb[i].x));
        // mm > 0: W_mm = P(Y_mm, Y_{H-mm}) and W_{H-mm} = P(Y_{H-mm}, Y_mm).
        // mm = 0 (ya = the Nyquist bin H, yb = bin H/2): W_0 = P(Y_0 = 0, Re
        // Y_H) and W_{H/2} = P(Y_{H/2}, Y_{H/2}).
        const bool z0 = mm == 0;
        const float2 f1 = z0 ? make_float2(0.f, 0.f) : ya;
        const float2 f2 = z0 ? make_float2(ya.x, 0.f) : yb;
        const int pos2 = z0 ? halfH : H - mm;
        // twiddles of bins mm (< H/2, in the table) and H - mm (-conj of
        // mm's) or H/2 (i)
        const float2 t1 = tw[mm];
        const float2 t2 = z0 ? make_float2(0.f, 1.f) : make_float2(-t1.x, t1.y);
        buf[pad(w + mm)] = wpack(f1, f2, t1);
        buf[pad(w + pos2)] = wpack(yb, z0 ? yb : ya, t2);
      }
      // the next pulse's coefficients (the same for every point: with one
      // pulse they stay)
      if (n_pulse > 1) load_c(q + 1 < n_pulse ? q + 1 : 0);
      __syncthreads();
      // z_n -> p_{2n}, p_{2n+1}: the last stage writes one float2 per n
      fft_run<SLOTS, LOGH, 0>(buf, tw, out + (int64_t)q * m * T, p0, m);
      // the last stage's loads are behind its barrier: buf may be rewritten
    }
  }
}

// cbin[q][j], j = 0..H: pulse q's coefficient of bin j (column j - 1, or the
// listed column of bin j), 0 where no frequency was solved
__global__ void coeff_bins_kernel(int n_pulse, int n_k, int H, const double2* __restrict__ c,
                                  const int32_t* __restrict__ midx, float2* __restrict__ cbin) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_pulse * (H + 1)) return;
  const int q = (int)(t / (H + 1)), j = (int)(t % (H + 1));
  float2 v = make_float2(0.f, 0.f);
  if (midx) {
    // the listed indices increase strictly: binary search for bin j
    int lo = 0, hi = n_k - 1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int b = midx[mid];
      if (b == j) {
        const double2 cc = c[(int64_t)q * n_k + mid];
        v = make_float2((float)cc.x, (float)cc.y);
        break;
      }
      if (b < j) lo = mid + 1;
      else hi = mid - 1;
    }
  } else if (j >= 1 && j <= n_k) {
    const double2 cc = c[(int64_t)q * n_k + j - 1];
    v = make_float2((float)cc.x, (float)cc.y);
  }
  cbin[t] = v;
}


// launch of one instantiation (its dynamic LDS limit raised on first use)
template <bool Sparse, int LOGH>
bem_status synth_go(bem_ctx* ctx, dim3 grid, size_t lds, int m, int n_k, const float2* U,
                    const int32_t* midx, int n_pulse, const float2* cbin, int add_incident,
                    const double* xp, double dk, float* p) {
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)synth_kernel<Sparse, LOGH>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, BEM_EHIP, "pulse synthesis: cannot raise the kernel's LDS limit");
    }
    attr_set = true;
  }
  hipLaunchKernelGGL((synth_kernel<Sparse, LOGH>), grid, dim3(kST), lds, ctx->stream, m, n_k, U,
                     midx, n_pulse, cbin, add_incident, xp, dk, p);
  return BEM_OK;
}

}  // namespace

bem_status launch_synth(bem_ctx* ctx, int m, int n_k, const void* U, const int32_t* m_index,
                        int n_pulse, const double* c, int T, int add_incident, const double* xp,
                        double dk, float* p) {
  if (m <= 0 || n_pulse <= 0) return BEM_OK;
  int logH = 0;
  while ((1 << logH) < T / 2) ++logH;
  const int H = T / 2;
  if (logH < 5 || logH > 12 || (1 << logH) != H)
    return fail(ctx, BEM_EINVAL, "pulse synthesis: T = %d must be a power of two in 64..8192", T);
  const bool sparse = m_index != nullptr;
  const int slots = H > 2048 ? H : 2048;
  const int G = slots / H;
  const size_t lds = sizeof(float2) * (size_t)(H / 2 + slots + slots / 8) +
                     (sparse ? sizeof(int) * (size_t)(H + 1) : 0);
  if (lds > 160 * 1024)
    return fail(ctx, BEM_EUNSUPPORTED, "pulse synthesis: T = %d with %d frequencies needs %zu B of LDS",
                T, n_k, lds);
  // float32 coefficients per bin (read from L2 by every point)
  void* ws = nullptr;
  const int64_t nc = (int64_t)n_pulse * (H + 1);
  bem_status st = workspace(ctx, (size_t)nc * sizeof(float2), &ws);
  if (st != BEM_OK) return st;
  hipLaunchKernelGGL(coeff_bins_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0,
                     ctx->stream, n_pulse, n_k, H, (const double2*)c, m_index, (float2*)ws);
  // whole rounds of resident workgroups (LDS-limited; at most 5 of 256
  // threads per CU, which the registers allow), each taking groups in turn
  const int ngroups = (m + G - 1) / G;
  const int per_cu = std::max(1, std::min(5, (int)((160 * 1024) / lds)));
  const int resident = ctx->num_cus * per_cu;
  const dim3 grid(ngroups < 4 * resident ? ngroups : 4 * resident);
  const float2* cbin = (const float2*)ws;
  const float2* Uf = (const float2*)U;
  const int pi = prof_begin(ctx, "synth");
  bem_status lst = BEM_OK;
  switch (logH) {
#define BEM_SYNTH_CASE(L)                                                                     \
  case L:                                                                                     \
    lst = sparse ? synth_go<true, L>(ctx, grid, lds, m, n_k, Uf, m_index, n_pulse, cbin,      \
                                     add_incident, xp, dk, p)                                 \
                 : synth_go<false, L>(ctx, grid, lds, m, n_k, Uf, nullptr, n_pulse, cbin,     \
                                      add_incident, xp, dk, p);                               \
    break;
    BEM_SYNTH_CASE(5)
    BEM_SYNTH_CASE(6)
    BEM_SYNTH_CASE(7)
    BEM_SYNTH_CASE(8)
    BEM_SYNTH_CASE(9)
    BEM_SYNTH_CASE(10)
    BEM_SYNTH_CASE(11)
    BEM_SYNTH_CASE(12)
#undef BEM_SYNTH_CASE
    default:
      break;
  }
  if (lst != BEM_OK) return lst;
  // algorithmic HBM traffic: U read once, every pulse written once
  prof_end(ctx, "synth", pi, 0.0, 8.0 * m * n_k + 4.0 * (double)n_pulse * m * T);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

}  // namespace bem
