// Space-time synthesis: inverse DFT over the solved frequencies (Sec. III,
// last paragraph: the inverse Fourier transform of the frequency-domain
// solution by FFT; Sec. IV: the incident pulse train enters as its Fourier
// coefficients c_m).  For each pulse q and point x,
//   p_q(x, t_n) = sum_{m=1}^{F} alpha_m Re[c_qm X_m(x) e^{-2 pi i m n/T}],
// alpha_m = 2 (m < T/2), 1 (m = T/2).  With Y_m = conj(c_qm X_m) this is the
// unnormalised inverse real DFT of the half spectrum Y, computed as one
// complex FFT of length T/2 on the packed sequence
//   W_m = (Y_m + conj Y_{T/2-m}) + i e^{2 pi i m/T} (Y_m - conj Y_{T/2-m}),
// whose output z_n gives p_{2n} = Re z_n, p_{2n+1} = Im z_n.
// One workgroup per point: U is read once, every pulse is written as T
// contiguous floats.  HBM traffic: 8F bytes read + 4 T n_pulse written per point.
//
// Sparse form (Sec. IV: the space-time field rebuilt from only the frequencies
// of largest incident amplitude): U and c hold n_sel columns whose frequency
// indices m_j are listed; every other bin of the half spectrum is zero.  An LDS
// map from bin to column replaces the dense indexing, the FFT is unchanged.
#include "common.h"

namespace bem {
namespace {

constexpr int kST = 256;

__device__ inline float2 cm(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// LDS: tw[T/2] = e^{2 pi i j/T}; buf0/buf1 ping-pong of length T/2; U row;
// (sparse) col[T/2 + 1]: column of bin m, or -1.
template <bool Sparse>
__global__ __launch_bounds__(kST) void synth_kernel(int m, int n_k, const float2* __restrict__ U,
                                                    const int32_t* __restrict__ midx,
                                                    int n_pulse, const double2* __restrict__ c,
                                                    int T, int logH, int add_incident,
                                                    const double* __restrict__ xp, double dk,
                                                    float* __restrict__ out) {
  extern __shared__ float2 lds[];
  const int H = T >> 1;
  float2* tw = lds;
  float2* b0 = lds + H;
  float2* b1 = b0 + H;
  float2* X = b1 + H;  // [n_k] field of this point (scattered + incident)
  int* col = reinterpret_cast<int*>(X + n_k);
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  for (int j = tid; j < H; j += kST) {
    float s, co;
    sincospif(2.0f * (float)j / (float)T, &s, &co);
    tw[j] = make_float2(co, s);
  }
  if (Sparse) {
    for (int j = tid; j <= H; j += kST) col[j] = -1;
    __syncthreads();
    for (int j = tid; j < n_k; j += kST) col[midx[j]] = j;
  }
  const double z = add_incident ? xp[3 * p + 2] : 0.0;
  for (int mm = tid; mm < n_k; mm += kST) {
    float2 u = U[(int64_t)p * n_k + mm];
    if (add_incident) {
      // e^{i k_m z}, k_m = m dk (m = mm + 1, or the listed index); phase
      // reduced in float64
      const int mf = Sparse ? midx[mm] : mm + 1;
      double t = (double)mf * dk * z * 0.15915494309189533576888376337251;
      t -= rint(t);
      float s, co;
      sincospif(2.0f * (float)t, &s, &co);
      u.x += co;
      u.y += s;
    }
    X[mm] = u;
  }
  __syncthreads();
  for (int q = 0; q < n_pulse; ++q) {
    const double2* cq = c + (int64_t)q * n_k;
    // W_m for m = 0..H-1 from Y_m = conj(c_m X_m) (Y_0 = 0, Y_m = 0 for m > n_k)
    for (int mm = tid; mm < H; mm += kST) {
      float2 ya = make_float2(0.f, 0.f), yb = make_float2(0.f, 0.f);
      const int ja = Sparse ? (mm >= 1 ? col[mm] : -1) : (mm >= 1 && mm <= n_k ? mm - 1 : -1);
      if (ja >= 0) {
        const double2 cc = cq[ja];
        const float2 v = cm(make_float2((float)cc.x, (float)cc.y), X[ja]);
        ya = make_float2(v.x, -v.y);
      }
      const int mb = H - mm;  // Y_{H-m}; for m = 0 this is the Nyquist bin (real part only)
      const int jb = Sparse ? (mb >= 1 ? col[mb] : -1) : (mb >= 1 && mb <= n_k ? mb - 1 : -1);
      if (jb >= 0) {
        const double2 cc = cq[jb];
        const float2 v = cm(make_float2((float)cc.x, (float)cc.y), X[jb]);
        yb = mm == 0 ? make_float2(v.x, 0.f) : make_float2(v.x, -v.y);
      }
      // conj(yb)
      const float2 e = make_float2(ya.x + yb.x, ya.y - yb.y);
      const float2 o = make_float2(ya.x - yb.x, ya.y + yb.y);
      const float2 io = cm(make_float2(-tw[mm].y, tw[mm].x), o);  // i e^{2 pi i m/T} o
      b0[mm] = make_float2(e.x + io.x, e.y + io.y);
    }
    __syncthreads();
    // Stockham radix-2 inverse FFT of length H (twiddles e^{+2 pi i ...})
    float2* src = b0;
    float2* dst = b1;
    int len = 1;  // size of already-combined sub-transforms
    for (int s = 0; s < logH; ++s) {
      const int half = H >> 1;
      for (int t = tid; t < half; t += kST) {
        const int j = t % len;           // position inside sub-transform
        const int g = t / len;           // sub-transform index
        const float2 a = src[g * len + j];
        const float2 b = src[g * len + j + half];
        const float2 wv = tw[j * (H / len) ];  // e^{2 pi i j/(2 len)} = tw[j * T/(2 len)]
        const float2 bw = cm(b, wv);
        dst[2 * g * len + j] = make_float2(a.x + bw.x, a.y + bw.y);
        dst[2 * g * len + j + len] = make_float2(a.x - bw.x, a.y - bw.y);
      }
      __syncthreads();
      float2* tmp = src; src = dst; dst = tmp;
      len <<= 1;
    }
    float* o = out + ((int64_t)q * m + p) * T;
    for (int nn = tid; nn < H; nn += kST) {
      const float2 v = src[nn];
      o[2 * nn] = v.x;
      o[2 * nn + 1] = v.y;
    }
    __syncthreads();
  }
}

}  // namespace

bem_status launch_synth(bem_ctx* ctx, int m, int n_k, const void* U, const int32_t* m_index,
                        int n_pulse, const double* c, int T, int add_incident, const double* xp,
                        double dk, float* p) {
  if (m <= 0 || n_pulse <= 0) return BEM_OK;
  int logH = 0;
  while ((1 << logH) < T / 2) ++logH;
  const bool sparse = m_index != nullptr;
  const size_t lds = sizeof(float2) * (size_t)(3 * (T / 2) + n_k) +
                     (sparse ? sizeof(int) * (size_t)(T / 2 + 1) : 0);
  static bool attr_set[2] = {false, false};
  const void* fn = sparse ? (const void*)synth_kernel<true> : (const void*)synth_kernel<false>;
  if (!attr_set[sparse]) {
    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set[sparse] = true;
  }
  const int pi = prof_begin(ctx, "synth");
  if (sparse)
    hipLaunchKernelGGL(synth_kernel<true>, dim3(m), dim3(kST), lds, ctx->stream, m, n_k,
                       (const float2*)U, m_index, n_pulse, (const double2*)c, T, logH,
                       add_incident, xp, dk, p);
  else
    hipLaunchKernelGGL(synth_kernel<false>, dim3(m), dim3(kST), lds, ctx->stream, m, n_k,
                       (const float2*)U, nullptr, n_pulse, (const double2*)c, T, logH,
                       add_incident, xp, dk, p);
  // algorithmic HBM traffic: U read once, every pulse written once
  prof_end(ctx, "synth", pi, 0.0, 8.0 * m * n_k + 4.0 * (double)n_pulse * m * T);
  BEM_CHECK_LAUNCH(ctx);
  return BEM_OK;
}

}  // namespace bem
