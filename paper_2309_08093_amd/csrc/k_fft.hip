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
// buffers, so no digit-reversal pass is needed.  Each stage is compiled for
// its radix (butterfly values in registers), and the twiddles come from a
// table of the J-th roots of unity computed once per J in FP64 (the plan's
// workspace), not from a sine/cosine per butterfly.
//
// The slice-wise products of step 3 give each frequency s one thread per
// output index (64 frequencies x up to 16 indices per workgroup), with the
// running row / column vector exchanged through LDS after each core.
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

// w^e for the J-th roots w = exp(-2 pi i / J) in the table (sg = -1), or its
// conjugate (sg = +1).
template <typename T>
__device__ __forceinline__ cplx<T> root(const cplx<T>* __restrict__ tw, int e, T sg) {
  const cplx<T> t = tw[e];
  return {t.x, -sg * t.y};
}

// In-register R-point DFT, y_m = sum_r x_r exp(sg 2 pi i m r / R).  The
// 7-point one is a direct sum with its roots from the table (J divisible by 7).
template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T> (&v)[R], T sg, const cplx<T>* __restrict__ tw, int J) {
  if constexpr (R == 2) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const cplx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const cplx<T> s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    const cplx<T> t = mul_i(d13, sg);   // sg*i*(x1 - x3)
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, t);
    v[3] = csub(d02, t);
  } else if constexpr (R == 3) {
    const T c1 = (T)-0.5, s1 = (T)0.86602540378443864676;
    const cplx<T> a = cadd(v[1], v[2]), b = csub(v[1], v[2]);
    const cplx<T> m = {v[0].x + c1 * a.x, v[0].y + c1 * a.y};
    const cplx<T> t = mul_i(cplx<T>{s1 * b.x, s1 * b.y}, sg);
    v[0] = cadd(v[0], a);
    v[1] = cadd(m, t);
    v[2] = csub(m, t);
  } else if constexpr (R == 5) {
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
  } else {
    static_assert(R == 7, "radix 2, 3, 4, 5 or 7");
    const int step = J / 7;
    cplx<T> out[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      cplx<T> acc = v[0];
#pragma unroll
      for (int r = 1; r < 7; ++r) acc = cadd(acc, cmul(v[r], root(tw, ((m * r) % 7) * step, sg)));
      out[m] = acc;
    }
#pragma unroll
    for (int m = 0; m < 7; ++m) v[m] = out[m];
  }
}

// Radices of the length-J transform, 4 bits each, first stage lowest.
struct FftPlan {
  uint64_t code;
  int nrad;
};

// One Stockham stage of radix R: b <- stage(a), Ns = product of the earlier radices.
template <typename T, int R>
__device__ __forceinline__ void fft_stage(const cplx<T>* __restrict__ a, cplx<T>* __restrict__ b, int N, int Ns,
                                          const cplx<T>* __restrict__ tw, T sg) {
  const int NR = N / R;
  const int tstep = N / (Ns * R);   // exp(sg 2 pi i kk r / (Ns R)) = root(kk r tstep)
  for (int j = threadIdx.x; j < NR; j += blockDim.x) {
    const int kk = j % Ns;
    cplx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[j + r * NR];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], root(tw, kk * r * tstep, sg));
    }
    dft_small<T, R>(v, sg, tw, N);
    const int base = (j - kk) * R + kk;
#pragma unroll
    for (int r = 0; r < R; ++r) b[base + r * Ns] = v[r];
  }
}

// Stockham autosort FFT of length N = J held in LDS buffer a (b is scratch);
// returns the buffer that holds the result.  sg = -1 forward, +1 inverse
// (unnormalised).  Must be called by the whole block.
template <typename T>
__device__ __forceinline__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, int N, FftPlan fp, const cplx<T>* __restrict__ tw, T sg) {
  int Ns = 1;
  for (int st = 0; st < fp.nrad; ++st) {
    const int R = (int)((fp.code >> (4 * st)) & 15u);
    switch (R) {
      case 4: fft_stage<T, 4>(a, b, N, Ns, tw, sg); break;
      case 2: fft_stage<T, 2>(a, b, N, Ns, tw, sg); break;
      case 3: fft_stage<T, 3>(a, b, N, Ns, tw, sg); break;
      case 5: fft_stage<T, 5>(a, b, N, Ns, tw, sg); break;
      default: fft_stage<T, 7>(a, b, N, Ns, tw, sg); break;
    }
    __syncthreads();
    cplx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// tw[e] = exp(-2 pi i e / J), computed in FP64.
template <typename T>
__global__ void k_fill_twiddles(cplx<T>* __restrict__ tw, int32_t J) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J) return;
  double sn, cs;
  sincospi(2.0 * (double)e / (double)J, &sn, &cs);
  tw[e] = cplx<T>{(T)cs, (T)-sn};
}

constexpr int kFftThreads = 512;

// One workgroup per (core i, column a + R_i c): CountSketch of the column
// over mode 2 into LDS, forward FFT, store to chat.
template <typename T>
__device__ __forceinline__ void core_fft_body(const CoreDesc& cd, const uint32_t* __restrict__ tab, cplx<T>* chat,
                                              int32_t J, FftPlan fp, const cplx<T>* __restrict__ tw, int32_t lo,
                                              int32_t hi, int32_t skip, int64_t q) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b = a + J;
  // locate core i and its column q
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
  cplx<T>* res = fft_lds<T>(a, b, J, fp, tw, (T)-1);
  cplx<T>* out = chat + (cd.chat_off[i] + q) * (int64_t)J;
  for (int s = threadIdx.x; s < J; s += blockDim.x) out[s] = res[s];
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_core_fft(CoreDesc cd, const uint32_t* __restrict__ tab, cplx<T>* chat,
                                                          int32_t J, FftPlan fp, const cplx<T>* __restrict__ tw,
                                                          int32_t lo, int32_t hi, int32_t skip, int64_t col_base) {
  core_fft_body<T>(cd, tab, chat, J, fp, tw, lo, hi, skip, blockIdx.x + col_base);
}

// Per frequency s: prefix P_<(s) (1 x R_k) and suffix P_>(s) (R_{k+1} x 1),
// the slice-wise products.  Workgroup: 64 consecutive frequencies (lane sl)
// x up to 16 output indices (wave c); after each core the running vector
// goes through LDS.  Entry c of the new vector sums over the old one in index
// order, as a plain matrix-vector product would.
template <typename T>
__device__ __forceinline__ void chain_body(const CoreDesc& cd, const cplx<T>* __restrict__ chat,
                                           cplx<T>* __restrict__ pre, cplx<T>* __restrict__ suf, int32_t J,
                                           int32_t k) {
  __shared__ cplx<T> vb[2][TT_MAX_RANK][64];
  const int sl = threadIdx.x & 63, c = threadIdx.x >> 6;
  const int s = blockIdx.x * 64 + sl;
  const bool ok = s < J;
  int buf = 0;
  cplx<T> v{(T)(c == 0), (T)0};
  for (int i = 0; i < k; ++i) {   // row vector times Chat_i(s) (R_i x R_{i+1})
    vb[buf][c][sl] = v;
    __syncthreads();
    const int r0 = cd.r0[i], r1 = cd.r1[i];
    cplx<T> acc{(T)0, (T)0};
    if (ok && c < r1) {
      const cplx<T>* C = chat + cd.chat_off[i] * (int64_t)J + s;
      for (int a = 0; a < r0; ++a) acc = cadd(acc, cmul(vb[buf][a][sl], C[(int64_t)(a + r0 * c) * J]));
    }
    v = acc;
    buf ^= 1;
  }
  if (ok && c < cd.r0[k]) pre[(int64_t)c * J + s] = v;
  v = cplx<T>{(T)(c == 0), (T)0};
  for (int i = cd.d - 1; i > k; --i) {   // Chat_i(s) times column vector
    vb[buf][c][sl] = v;
    __syncthreads();
    const int r0 = cd.r0[i], r1 = cd.r1[i];
    cplx<T> acc{(T)0, (T)0};
    if (ok && c < r0) {
      const cplx<T>* C = chat + cd.chat_off[i] * (int64_t)J + s;
      for (int b = 0; b < r1; ++b) acc = cadd(acc, cmul(C[(int64_t)(c + r0 * b) * J], vb[buf][b][sl]));
    }
    v = acc;
    buf ^= 1;
  }
  if (ok && c < cd.r1[k]) suf[(int64_t)c * J + s] = v;
}

template <typename T>
__global__ __launch_bounds__(64 * TT_MAX_RANK) void k_chain(CoreDesc cd, const cplx<T>* __restrict__ chat,
                                                           cplx<T>* __restrict__ pre, cplx<T>* __restrict__ suf,
                                                           int32_t J, int32_t k) {
  chain_body<T>(cd, chat, pre, suf, J, k);
}

// One workgroup per output column q = a + R_k b: face-split product, inverse
// FFT, real part / J.
template <typename T>
__device__ __forceinline__ void facesplit_body(const cplx<T>* __restrict__ pre, const cplx<T>* __restrict__ suf,
                                               T* __restrict__ SH, int32_t J, int32_t rk, FftPlan fp,
                                               const cplx<T>* __restrict__ tw, int q) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b = a + J;
  const int al = q % rk, be = q / rk;
  const cplx<T>* P = pre + (int64_t)al * J;
  const cplx<T>* Q = suf + (int64_t)be * J;
  for (int s = threadIdx.x; s < J; s += blockDim.x) a[s] = cmul(P[s], Q[s]);
  __syncthreads();
  cplx<T>* res = fft_lds<T>(a, b, J, fp, tw, (T)1);
  const T inv = (T)1 / (T)J;
  T* out = SH + (int64_t)q * J;
  for (int s = threadIdx.x; s < J; s += blockDim.x) out[s] = res[s].x * inv;
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_facesplit_ifft(const cplx<T>* __restrict__ pre,
                                                                const cplx<T>* __restrict__ suf, T* __restrict__ SH,
                                                                int32_t J, int32_t rk, FftPlan fp,
                                                                const cplx<T>* __restrict__ tw) {
  facesplit_body<T>(pre, suf, SH, J, rk, fp, tw, blockIdx.x);
}

// Batched (FP32): descriptor blockIdx.y; workgroups past a problem's count
// return at once.
__global__ __launch_bounds__(kFftThreads) void kb_core_fft(const BIface* __restrict__ d) {
  const BIface& u = d[blockIdx.y];
  if ((int32_t)blockIdx.x >= u.cols) return;
  core_fft_body<float>(u.cd, u.tab, static_cast<cplx<float>*>(u.chat), u.J, FftPlan{u.fft_code, u.fft_nrad},
                       static_cast<const cplx<float>*>(u.tw), u.k - 1, u.k - 1, -1, blockIdx.x);
}

// Batched (FP32), at the start of a sweep: the transforms of cores 1..d-1
// of problem blockIdx.y (the descriptors of step 0); columns past the
// problem's count return at once.
__global__ __launch_bounds__(kFftThreads) void kb_core_fft_all(const BIface* __restrict__ d) {
  const BIface& u = d[blockIdx.y];
  int64_t cols = 0;
  for (int i = 1; i < u.cd.d; ++i) cols += (int64_t)u.cd.r0[i] * u.cd.r1[i];
  if ((int64_t)blockIdx.x >= cols) return;
  core_fft_body<float>(u.cd, u.tab, static_cast<cplx<float>*>(u.chat), u.J, FftPlan{u.fft_code, u.fft_nrad},
                       static_cast<const cplx<float>*>(u.tw), 1, u.cd.d - 1, -1, blockIdx.x);
}

// grid.x covers the largest J; frequencies past a problem's J only take part
// in the workgroup's barriers
__global__ __launch_bounds__(64 * TT_MAX_RANK) void kb_chain(const BIface* __restrict__ d) {
  const BIface& u = d[blockIdx.y];
  chain_body<float>(u.cd, static_cast<const cplx<float>*>(u.chat), static_cast<cplx<float>*>(u.pre),
                    static_cast<cplx<float>*>(u.suf), u.J, u.k);
}

__global__ __launch_bounds__(kFftThreads) void kb_facesplit_ifft(const BIface* __restrict__ d) {
  const BIface& u = d[blockIdx.y];
  if ((int32_t)blockIdx.x >= u.s) return;
  facesplit_body<float>(static_cast<const cplx<float>*>(u.pre), static_cast<const cplx<float>*>(u.suf),
                        static_cast<float*>(u.SH), u.J, u.cd.r0[u.k], FftPlan{u.fft_code, u.fft_nrad},
                        static_cast<const cplx<float>*>(u.tw), blockIdx.x);
}

FftPlan make_fft_plan(const tt_plan_s* p) {
  FftPlan fp{};
  fp.nrad = p->fft_nrad;
  for (int i = 0; i < p->fft_nrad; ++i) fp.code |= (uint64_t)p->fft_radix[i] << (4 * i);
  return fp;
}

// Waves of one chain workgroup: the next power of two >= the largest rank.
int chain_waves(const tt_plan_s* p) {
  int64_t rm = 1;
  for (int i = 0; i <= p->d; ++i) rm = p->r[i] > rm ? p->r[i] : rm;
  int cw = 1;
  while (cw < rm) cw <<= 1;
  return cw;
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
  hipLaunchKernelGGL(k_core_fft<T>, dim3((unsigned)cols), dim3(kFftThreads), lds, p->stream, cd,
                     p->at<uint32_t>(p->o_tab), p->at<cplx<T>>(p->o_chat), (int32_t)p->J, fp,
                     p->at<cplx<T>>(p->o_tw), lo, hi, skip, (int64_t)0);
  return hipGetLastError();
}

template <typename T>
hipError_t interface_t(const tt_plan_s* p, const CoreDesc& cd, int k, void* SH) {
  cplx<T>* pre = p->at<cplx<T>>(p->o_pre);
  cplx<T>* suf = p->at<cplx<T>>(p->o_suf);
  hipLaunchKernelGGL(k_chain<T>, dim3((unsigned)((p->J + 63) / 64)), dim3(64 * chain_waves(p)), 0, p->stream, cd,
                     p->at<cplx<T>>(p->o_chat), pre, suf, (int32_t)p->J, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t s = p->r[k] * p->r[k + 1];
  const size_t lds = 2 * (size_t)p->J * sizeof(cplx<T>);
  if ((e = tt_allow_lds(k_facesplit_ifft<T>, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_facesplit_ifft<T>, dim3((unsigned)s), dim3(kFftThreads), lds, p->stream, pre, suf,
                     static_cast<T*>(SH), (int32_t)p->J, (int32_t)p->r[k], make_fft_plan(p), p->at<cplx<T>>(p->o_tw));
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

// Batched interface of step k for nprob problems (FP32), each with its own J
// and FFT radices: for k >= 1 the transform of core k - 1 (max_cols
// workgroups per problem), then the chains and the face-split inverse FFTs
// (max_s per problem).  Jmax: the largest J; cw: waves of a chain workgroup.
hipError_t launch_interface_batched(const void* desc, int32_t nprob, int32_t k, int32_t Jmax, int32_t max_cols,
                                    int32_t max_s, int32_t cw, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  const BIface* d = static_cast<const BIface*>(desc);
  const size_t lds = 2 * (size_t)Jmax * sizeof(cplx<float>);
  hipError_t e;
  if (k >= 1 && max_cols > 0) {
    if ((e = tt_allow_lds(kb_core_fft, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(kb_core_fft, dim3((unsigned)max_cols, (unsigned)nprob), dim3(kFftThreads), lds, st, d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kb_chain, dim3((unsigned)((Jmax + 63) / 64), (unsigned)nprob), dim3(64 * cw), 0, st, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = tt_allow_lds(kb_facesplit_ifft, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(kb_facesplit_ifft, dim3((unsigned)max_s, (unsigned)nprob), dim3(kFftThreads), lds, st, d);
  return hipGetLastError();
}

hipError_t launch_fill_twiddles(const tt_plan_s* p) {
  const unsigned g = (unsigned)((p->J + 255) / 256);
  if (p->wdt == TT_F64)
    hipLaunchKernelGGL(k_fill_twiddles<double>, dim3(g), dim3(256), 0, p->stream, p->at<cplx<double>>(p->o_tw),
                       (int32_t)p->J);
  else
    hipLaunchKernelGGL(k_fill_twiddles<float>, dim3(g), dim3(256), 0, p->stream, p->at<cplx<float>>(p->o_tw),
                       (int32_t)p->J);
  return hipGetLastError();
}

hipError_t launch_core_fft_batched(const void* desc, int32_t nprob, int32_t Jmax, int32_t max_cols, hipStream_t st) {
  if (nprob <= 0 || max_cols <= 0) return hipSuccess;
  const size_t lds = 2 * (size_t)Jmax * sizeof(cplx<float>);
  hipError_t e;
  if ((e = tt_allow_lds(kb_core_fft_all, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(kb_core_fft_all, dim3((unsigned)max_cols, (unsigned)nprob), dim3(kFftThreads), lds, st,
                     static_cast<const BIface*>(desc));
  return hipGetLastError();
}
