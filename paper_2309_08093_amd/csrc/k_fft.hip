// Interface sketch SH_k = S_{-k}(G_{>k}^T (x) G_{<k}) via Theorems 1-2 (Sec. 3):
//   1. C_i = G_i x_2 S_i  (CountSketch of core i along its mode-2 index),
//   2. FFT of C_i along the bucket axis, w = exp(-2 pi i / J)  (Sec. 3, DFT
//      matrix F),
//   3. per frequency s: prefix P_<(s) = Chat_0(s) ... Chat_{k-1}(s) (1 x R_k)
//      and suffix P_>(s) = Chat_{k+1}(s) ... Chat_{d-1}(s) (R_{k+1} x 1), the
//      slice-wise products of Theorem 2,
//   4. face-splitting product, column a + b R_k = P_<(s)[a] P_>(s)[b]
//      (Theorem 1), inverse FFT, real part.
//
// The length-J transforms run in LDS, one workgroup per column, as a
// mixed-radix (4, 2, 3, 5, 7) Stockham autosort FFT with two ping-pong
// buffers, so no digit-reversal pass is needed.
#include "tt_internal.h"

namespace {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
// multiply by -i (fwd) or +i (inv): sg = -1 forward, +1 inverse
template <typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a, T sg) { return {-sg * a.y, sg * a.x}; }

__device__ __forceinline__ void sincos_2pi_frac(int e, int den, float* s, float* c) {
  sincospif(2.0f * (float)e / (float)den, s, c);
}
__device__ __forceinline__ void sincos_2pi_frac(int e, int den, double* s, double* c) {
  sincospi(2.0 * (double)e / (double)den, s, c);
}

// In-register R-point DFT, y_m = sum_r x_r exp(sg 2 pi i m r / R).
template <typename T>
__device__ __forceinline__ void dft_small(cplx<T>* v, int R, T sg) {
  if (R == 2) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 4) {
    const cplx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const cplx<T> s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    const cplx<T> t = mul_i(d13, sg);   // sg*i*(x1 - x3)
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, t);
    v[3] = csub(d02, t);
  } else if (R == 3) {
    const T c1 = (T)-0.5, s1 = (T)0.86602540378443864676;
    const cplx<T> a = cadd(v[1], v[2]), b = csub(v[1], v[2]);
    const cplx<T> m = {v[0].x + c1 * a.x, v[0].y + c1 * a.y};
    const cplx<T> t = mul_i(cplx<T>{s1 * b.x, s1 * b.y}, sg);
    v[0] = cadd(v[0], a);
    v[1] = cadd(m, t);
    v[2] = csub(m, t);
  } else if (R == 5) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    const cplx<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const cplx<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const cplx<T> m1 = {v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    const cplx<T> m2 = {v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    const cplx<T> t1 = mul_i(cplx<T>{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y}, sg);
    const cplx<T> t2 = mul_i(cplx<T>{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y}, sg);
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(m1, t1);
    v[4] = csub(m1, t1);
    v[2] = cadd(m2, t2);
    v[3] = csub(m2, t2);
  } else {  // R == 7, direct sum
    cplx<T> out[7];
    for (int m = 0; m < R; ++m) {
      cplx<T> acc = v[0];
      for (int r = 1; r < R; ++r) {
        T s, c;
        sincos_2pi_frac((m * r) % R, R, &s, &c);
        acc = cadd(acc, cmul(v[r], cplx<T>{c, sg * s}));
      }
      out[m] = acc;
    }
    for (int m = 0; m < R; ++m) v[m] = out[m];
  }
}

struct FftPlan {
  int rad[32];
  int nrad;
};

// Stockham autosort FFT of length N held in LDS buffer a (b is scratch);
// returns the buffer that holds the result.  sg = -1 forward, +1 inverse
// (unnormalised).  Must be called by the whole block.
template <typename T>
__device__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, int N, const FftPlan& fp, T sg) {
  int Ns = 1;
  for (int st = 0; st < fp.nrad; ++st) {
    const int R = fp.rad[st];
    const int NR = N / R;
    for (int j = threadIdx.x; j < NR; j += blockDim.x) {
      const int kk = j % Ns;
      cplx<T> v[8];
      for (int r = 0; r < R; ++r) v[r] = a[j + r * NR];
      if (Ns > 1) {
        for (int r = 1; r < R; ++r) {
          T s, c;
          sincos_2pi_frac(kk * r, Ns * R, &s, &c);
          v[r] = cmul(v[r], cplx<T>{c, sg * s});
        }
      }
      dft_small(v, R, sg);
      const int base = (j / Ns) * Ns * R + kk;
      for (int r = 0; r < R; ++r) b[base + r * Ns] = v[r];
    }
    __syncthreads();
    cplx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// One workgroup per (core i, column a + R_i c): CountSketch of the column
// over mode 2 into LDS, forward FFT, store to chat.
template <typename T>
__global__ __launch_bounds__(256) void k_core_fft(CoreDesc cd, const uint32_t* __restrict__ tab, cplx<T>* chat,
                                                  int32_t J, FftPlan fp, int32_t lo, int32_t hi, int32_t skip,
                                                  int64_t col_base) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b = a + J;
  // locate core i and its column q
  int64_t q = blockIdx.x + col_base;
  int i = lo;
  for (; i <= hi; ++i) {
    if (i == skip) continue;
    const int64_t cols = (int64_t)cd.r0[i] * cd.r1[i];
    if (q < cols) break;
    q -= cols;
  }
  const int r0 = cd.r0[i], ni = cd.n[i];
  const int aa = (int)(q % r0), cc = (int)(q / r0);
  // CountSketch of the column into J FP64 buckets (the FFT scratch buffer holds
  // J doubles), so the result hardly depends on the order of the atomic adds
  double* acc = reinterpret_cast<double*>(b);
  for (int s = threadIdx.x; s < J; s += blockDim.x) acc[s] = 0.0;
  __syncthreads();
  const double* G = cd.G[i];
  const uint32_t* t = tab + cd.tab_off[i];
  for (int j = threadIdx.x; j < ni; j += blockDim.x) {
    const uint32_t key = t[j];
    double val = G[aa + (int64_t)r0 * (j + (int64_t)ni * cc)];
    if (key & TT_KEY_SIGN) val = -val;
    atomicAdd(&acc[key & TT_KEY_MASK], val);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < J; s += blockDim.x) a[s] = cplx<T>{(T)acc[s], (T)0};
  __syncthreads();
  cplx<T>* res = fft_lds<T>(a, b, J, fp, (T)-1);
  cplx<T>* out = chat + (cd.chat_off[i] + q) * (int64_t)J;
  for (int s = threadIdx.x; s < J; s += blockDim.x) out[s] = res[s];
}

// Per frequency s: prefix (1 x R_k) and suffix (R_{k+1} x 1) slice-wise products.
template <typename T>
__global__ void k_chain(CoreDesc cd, const cplx<T>* __restrict__ chat, cplx<T>* __restrict__ pre,
                        cplx<T>* __restrict__ suf, int32_t J, int32_t k) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= J) return;
  cplx<T> v[TT_MAX_RANK], nv[TT_MAX_RANK];
#pragma unroll
  for (int a = 0; a < TT_MAX_RANK; ++a) v[a] = cplx<T>{(T)(a == 0), (T)0};
  for (int i = 0; i < k; ++i) {
    const int r0 = cd.r0[i], r1 = cd.r1[i];
    const cplx<T>* C = chat + cd.chat_off[i] * (int64_t)J + s;
#pragma unroll
    for (int c = 0; c < TT_MAX_RANK; ++c) {
      cplx<T> acc{(T)0, (T)0};
      if (c < r1) {
#pragma unroll
        for (int a = 0; a < TT_MAX_RANK; ++a)
          if (a < r0) acc = cadd(acc, cmul(v[a], C[(int64_t)(a + r0 * c) * J]));
      }
      nv[c] = acc;
    }
#pragma unroll
    for (int c = 0; c < TT_MAX_RANK; ++c) v[c] = nv[c];
  }
  const int rk = cd.r0[k];
#pragma unroll
  for (int a = 0; a < TT_MAX_RANK; ++a)
    if (a < rk) pre[(int64_t)a * J + s] = v[a];

#pragma unroll
  for (int a = 0; a < TT_MAX_RANK; ++a) v[a] = cplx<T>{(T)(a == 0), (T)0};
  for (int i = cd.d - 1; i > k; --i) {
    const int r0 = cd.r0[i], r1 = cd.r1[i];
    const cplx<T>* C = chat + cd.chat_off[i] * (int64_t)J + s;
#pragma unroll
    for (int a = 0; a < TT_MAX_RANK; ++a) {
      cplx<T> acc{(T)0, (T)0};
      if (a < r0) {
#pragma unroll
        for (int c = 0; c < TT_MAX_RANK; ++c)
          if (c < r1) acc = cadd(acc, cmul(C[(int64_t)(a + r0 * c) * J], v[c]));
      }
      nv[a] = acc;
    }
#pragma unroll
    for (int a = 0; a < TT_MAX_RANK; ++a) v[a] = nv[a];
  }
  const int rk1 = cd.r1[k];
#pragma unroll
  for (int b = 0; b < TT_MAX_RANK; ++b)
    if (b < rk1) suf[(int64_t)b * J + s] = v[b];
}

// One workgroup per output column q = a + R_k b: face-split product, inverse
// FFT, real part / J.
template <typename T>
__global__ __launch_bounds__(256) void k_facesplit_ifft(const cplx<T>* __restrict__ pre, const cplx<T>* __restrict__ suf,
                                                        T* __restrict__ SH, int32_t J, int32_t rk, FftPlan fp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b = a + J;
  const int q = blockIdx.x;
  const int al = q % rk, be = q / rk;
  const cplx<T>* P = pre + (int64_t)al * J;
  const cplx<T>* Q = suf + (int64_t)be * J;
  for (int s = threadIdx.x; s < J; s += blockDim.x) a[s] = cmul(P[s], Q[s]);
  __syncthreads();
  cplx<T>* res = fft_lds<T>(a, b, J, fp, (T)1);
  const T inv = (T)1 / (T)J;
  T* out = SH + (int64_t)q * J;
  for (int s = threadIdx.x; s < J; s += blockDim.x) out[s] = res[s].x * inv;
}

FftPlan make_fft_plan(const tt_plan_s* p) {
  FftPlan fp{};
  fp.nrad = p->fft_nrad;
  for (int i = 0; i < p->fft_nrad; ++i) fp.rad[i] = p->fft_radix[i];
  return fp;
}

template <typename T>
hipError_t core_fft_t(const tt_plan_s* p, const CoreDesc& cd, int lo, int hi, int skip) {
  int64_t cols = 0;
  for (int i = lo; i <= hi; ++i)
    if (i != skip) cols += (int64_t)cd.r0[i] * cd.r1[i];
  if (cols == 0) return hipSuccess;
  const size_t lds = 2 * (size_t)p->J * sizeof(cplx<T>);
  const FftPlan fp = make_fft_plan(p);
  hipError_t e = tt_allow_lds(k_core_fft<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_core_fft<T>, dim3((unsigned)cols), dim3(256), lds, p->stream, cd, p->at<uint32_t>(p->o_tab),
                     p->at<cplx<T>>(p->o_chat), (int32_t)p->J, fp, lo, hi, skip, (int64_t)0);
  return hipGetLastError();
}

template <typename T>
hipError_t interface_t(const tt_plan_s* p, const CoreDesc& cd, int k, void* SH) {
  cplx<T>* pre = p->at<cplx<T>>(p->o_pre);
  cplx<T>* suf = p->at<cplx<T>>(p->o_suf);
  hipLaunchKernelGGL(k_chain<T>, dim3((unsigned)((p->J + 127) / 128)), dim3(128), 0, p->stream, cd,
                     p->at<cplx<T>>(p->o_chat), pre, suf, (int32_t)p->J, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t s = p->r[k] * p->r[k + 1];
  const size_t lds = 2 * (size_t)p->J * sizeof(cplx<T>);
  if ((e = tt_allow_lds(k_facesplit_ifft<T>, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_facesplit_ifft<T>, dim3((unsigned)s), dim3(256), lds, p->stream, pre, suf,
                     static_cast<T*>(SH), (int32_t)p->J, (int32_t)p->r[k], make_fft_plan(p));
  return hipGetLastError();
}

}  // namespace

bool tt_factor_fft(int64_t J, int* radix, int* nrad) {
  int n = 0;
  while (J % 4 == 0 && n < 32) { radix[n++] = 4; J /= 4; }
  while (J % 2 == 0 && n < 32) { radix[n++] = 2; J /= 2; }
  for (int pr : {3, 5, 7})
    while (J % pr == 0 && n < 32) { radix[n++] = pr; J /= pr; }
  *nrad = n;
  return J == 1;
}

hipError_t launch_core_fft(const tt_plan_s* p, const CoreDesc& cd, int lo, int hi, int skip) {
  return p->wdt == TT_F64 ? core_fft_t<double>(p, cd, lo, hi, skip) : core_fft_t<float>(p, cd, lo, hi, skip);
}

hipError_t launch_interface_from_chat(const tt_plan_s* p, const CoreDesc& cd, int k, void* SH) {
  return p->wdt == TT_F64 ? interface_t<double>(p, cd, k, SH) : interface_t<float>(p, cd, k, SH);
}
