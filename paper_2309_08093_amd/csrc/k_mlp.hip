// Learned sketch-size policy: a small multilayer perceptron
// (8 -> 64 -> 64 -> 64 -> 2, ReLU, FP32) with its own forward, backward and
// Adam kernels, the Corollary 3 bound (Sec. 4) used as its fallback, and the
// per-core features it reads.
//
// The network is tiny (9026 parameters), so every kernel stages the weights
// in LDS and works on chunks of 64 samples.  The gradient kernel runs in one
// workgroup: each thread owns a fixed set of parameters and accumulates their
// gradients in FP64 over the chunks in sample order, so the result does not
// depend on scheduling.
#include <math.h>

#include "tt_internal.h"

namespace {

constexpr int F = TT_JPOLICY_FEATURES;
constexpr int H = TT_JPOLICY_HIDDEN;
constexpr int O = TT_JPOLICY_OUTPUTS;
constexpr int P = TT_JPOLICY_PARAMS;
constexpr int CH = 64;        // samples per chunk
constexpr int LS = H + 1;     // padded LDS row stride of 64-wide rows
constexpr int LF = F + 1;     // padded LDS row stride of feature rows

// offsets of W_l (fan_out x fan_in, row-major) and b_l in the parameter array
constexpr int oW1 = 0, ob1 = oW1 + H * F;
constexpr int oW2 = ob1 + H, ob2 = oW2 + H * H;
constexpr int oW3 = ob2 + H, ob3 = oW3 + H * H;
constexpr int oW4 = ob3 + H, ob4 = oW4 + O * H;
static_assert(ob4 + O == P, "parameter layout");

constexpr int GRAD_THREADS = 1024;
constexpr int NQ = (P + GRAD_THREADS - 1) / GRAD_THREADS;   // parameters owned per thread

struct Weights {
  float W1[H * LF];
  float W2[H * LS];
  float W3[H * LS];
  float W4[O * LS];
  float b1[H], b2[H], b3[H], b4[O];
};

struct FwdLds {
  Weights w;
  float x[CH * LF];
  float hA[CH * LS];
  float hB[CH * LS];
};

struct GradLds {
  Weights w;
  float x[CH * LF];
  float h1[CH * LS], h2[CH * LS], h3[CH * LS];
  float y[CH * O];
  float dA[CH * LS], dB[CH * LS];
};

__device__ void load_weights(Weights& w, const float* __restrict__ p, int tid, int nthr) {
  for (int e = tid; e < H * F; e += nthr) w.W1[(e / F) * LF + e % F] = p[oW1 + e];
  for (int e = tid; e < H * H; e += nthr) {
    w.W2[(e / H) * LS + e % H] = p[oW2 + e];
    w.W3[(e / H) * LS + e % H] = p[oW3 + e];
  }
  for (int e = tid; e < O * H; e += nthr) w.W4[(e / H) * LS + e % H] = p[oW4 + e];
  for (int e = tid; e < H; e += nthr) {
    w.b1[e] = p[ob1 + e];
    w.b2[e] = p[ob2 + e];
    w.b3[e] = p[ob3 + e];
  }
  for (int e = tid; e < O; e += nthr) w.b4[e] = p[ob4 + e];
}

// out[b][j] = act(bias[j] + sum_i W[j][i] in[b][i]) for the 64 rows of a chunk
template <int IN, bool RELU>
__device__ void dense(const float* W, int wls, const float* bias, const float* in, int ils, float* out, int ols, int nout,
                      int tid, int nthr) {
  for (int e = tid; e < CH * nout; e += nthr) {
    const int b = e / nout, j = e - b * nout;
    float z = bias[j];
#pragma unroll 8
    for (int i = 0; i < IN; ++i) z = fmaf(W[j * wls + i], in[b * ils + i], z);
    out[b * ols + j] = RELU ? fmaxf(z, 0.0f) : z;
  }
}

__device__ void load_rows(float* dst, int dls, const float* __restrict__ src, int width, int b0, int nb, int tid,
                          int nthr) {
  for (int e = tid; e < CH * width; e += nthr) {
    const int b = e / width, f = e - b * width;
    dst[b * dls + f] = b < nb ? src[(int64_t)(b0 + b) * width + f] : 0.0f;
  }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                     int32_t B, float* __restrict__ Y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  FwdLds& s = *reinterpret_cast<FwdLds*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int b0 = blockIdx.x * CH;
  const int nb = (B - b0) < CH ? (B - b0) : CH;
  load_weights(s.w, params, tid, nthr);
  load_rows(s.x, LF, X, F, b0, nb, tid, nthr);
  __syncthreads();
  dense<F, true>(s.w.W1, LF, s.w.b1, s.x, LF, s.hA, LS, H, tid, nthr);
  __syncthreads();
  dense<H, true>(s.w.W2, LS, s.w.b2, s.hA, LS, s.hB, LS, H, tid, nthr);
  __syncthreads();
  dense<H, true>(s.w.W3, LS, s.w.b3, s.hB, LS, s.hA, LS, H, tid, nthr);
  __syncthreads();
  for (int e = tid; e < CH * O; e += nthr) {
    const int b = e / O, o = e - b * O;
    if (b >= nb) continue;
    float z = s.w.b4[o];
    for (int i = 0; i < H; ++i) z = fmaf(s.w.W4[o * LS + i], s.hA[b * LS + i], z);
    Y[(int64_t)(b0 + b) * O + o] = z;
  }
}

// acc[q] += dL/dp for the owned parameters p = tid + q * nthr of one layer
// (weights at oW, fan-in IN, fan-out OUT, bias right after): the delta rows
// dl (stride dls) times the layer's input rows in (stride ins) over nb rows.
__device__ void accumulate(double* acc, int tid, int oW, int IN, int OUT, const float* dl, int dls, const float* in,
                           int ins, int nb) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = tid + q * GRAD_THREADS;
    const int r = p - oW;
    if (r < 0 || r >= IN * OUT + OUT) continue;
    double a = 0.0;
    if (r < IN * OUT) {
      const int j = r / IN, i = r - j * IN;
      for (int b = 0; b < nb; ++b) a += (double)dl[b * dls + j] * (double)in[b * ins + i];
    } else {
      const int j = r - IN * OUT;
      for (int b = 0; b < nb; ++b) a += (double)dl[b * dls + j];
    }
    acc[q] += a;
  }
}

// dprev[b][i] = (sum_j d[b][j] W[j][i]) * [h[b][i] > 0]
__device__ void backprop(const float* d, int dls, int nout, const float* W, const float* h, float* dprev, int tid,
                         int nthr) {
  for (int e = tid; e < CH * H; e += nthr) {
    const int b = e / H, i = e - b * H;
    float v = 0.0f;
    for (int j = 0; j < nout; ++j) v = fmaf(d[b * dls + j], W[j * LS + i], v);
    dprev[b * LS + i] = h[b * LS + i] > 0.0f ? v : 0.0f;
  }
}

__global__ __launch_bounds__(GRAD_THREADS) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ X,
                                                           const float* __restrict__ T, int32_t B,
                                                           float* __restrict__ grad, float* __restrict__ loss) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  GradLds& s = *reinterpret_cast<GradLds*>(smem_raw);
  __shared__ double red[GRAD_THREADS / 64];
  const int tid = threadIdx.x, nthr = GRAD_THREADS;
  load_weights(s.w, params, tid, nthr);
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  double lsum = 0.0;
  const float scale = 2.0f / ((float)B * (float)O);
  for (int b0 = 0; b0 < B; b0 += CH) {
    const int nb = (B - b0) < CH ? (B - b0) : CH;
    load_rows(s.x, LF, X, F, b0, nb, tid, nthr);
    __syncthreads();
    dense<F, true>(s.w.W1, LF, s.w.b1, s.x, LF, s.h1, LS, H, tid, nthr);
    __syncthreads();
    dense<H, true>(s.w.W2, LS, s.w.b2, s.h1, LS, s.h2, LS, H, tid, nthr);
    __syncthreads();
    dense<H, true>(s.w.W3, LS, s.w.b3, s.h2, LS, s.h3, LS, H, tid, nthr);
    __syncthreads();
    // output layer and dL/dy = 2 (y - t) / (B O), zero on padding rows
    for (int e = tid; e < CH * O; e += nthr) {
      const int b = e / O, o = e - b * O;
      float dy = 0.0f;
      if (b < nb) {
        float z = s.w.b4[o];
        for (int i = 0; i < H; ++i) z = fmaf(s.w.W4[o * LS + i], s.h3[b * LS + i], z);
        const float diff = z - T[(int64_t)(b0 + b) * O + o];
        lsum += (double)diff * (double)diff;
        dy = scale * diff;
      }
      s.y[b * O + o] = dy;
    }
    __syncthreads();
    accumulate(acc, tid, oW4, H, O, s.y, O, s.h3, LS, nb);
    backprop(s.y, O, O, s.w.W4, s.h3, s.dA, tid, nthr);
    __syncthreads();
    accumulate(acc, tid, oW3, H, H, s.dA, LS, s.h2, LS, nb);
    backprop(s.dA, LS, H, s.w.W3, s.h2, s.dB, tid, nthr);
    __syncthreads();
    accumulate(acc, tid, oW2, H, H, s.dB, LS, s.h1, LS, nb);
    backprop(s.dB, LS, H, s.w.W2, s.h1, s.dA, tid, nthr);
    __syncthreads();
    accumulate(acc, tid, oW1, F, H, s.dA, LS, s.x, LF, nb);
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = tid + q * GRAD_THREADS;
    if (p < P) grad[p] = (float)acc[q];
  }
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = lsum;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < GRAD_THREADS / 64; ++w) t += red[w];
    loss[0] = (float)(t / ((double)B * (double)O));
  }
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       int64_t count, float lr, float beta1, float beta2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

bool smooth(int64_t x) {
  if (x < 1) return false;
  for (int q : {2, 3, 5, 7})
    while (x % q == 0) x /= q;
  return x == 1;
}

}  // namespace

hipError_t launch_mlp_forward(const float* params, const float* feats, int32_t B, float* out, hipStream_t stream) {
  hipError_t e = tt_allow_lds(reinterpret_cast<const void*>(&k_mlp_forward), sizeof(FwdLds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((B + CH - 1) / CH)), dim3(256), sizeof(FwdLds), stream, params,
                     feats, B, out);
  return hipGetLastError();
}

// nearest product of 2, 3, 5, 7 to x within [lo, hi] (ties go down); hi is
// itself such a product
int64_t tt_round_smooth(double x, int64_t lo, int64_t hi) {
  if (!(x == x) || x < (double)lo) x = (double)lo;
  if (x > (double)hi) x = (double)hi;
  int64_t down = (int64_t)floor(x), up = (int64_t)ceil(x);
  while (down > lo && !smooth(down)) --down;
  while (up < hi && !smooth(up)) ++up;
  if (!smooth(down)) down = up;
  if (!smooth(up)) up = down;
  return (x - (double)down <= (double)up - x) ? down : up;
}

int64_t tt_floor_smooth(int64_t x) {
  while (x > 1 && !smooth(x)) --x;
  return x < 1 ? 1 : x;
}

extern "C" {

tt_status tt_jpolicy_forward(const float* params, const float* feats, int32_t B, float* out, void* stream) {
  if (!params || !feats || !out) return tt_fail(TT_ERR_ARG, "null argument");
  if (B < 1 || B > TT_JPOLICY_MAX_BATCH) return tt_fail(TT_ERR_ARG, "batch %d outside [1, %d]", B, TT_JPOLICY_MAX_BATCH);
  TT_HIP_TRY(launch_mlp_forward(params, feats, B, out, static_cast<hipStream_t>(stream)));
  return TT_OK;
}

tt_status tt_jpolicy_loss_grad(const float* params, const float* feats, const float* targets, int32_t B, float* grad,
                               float* loss, void* stream) {
  if (!params || !feats || !targets || !grad || !loss) return tt_fail(TT_ERR_ARG, "null argument");
  if (B < 1 || B > 4096) return tt_fail(TT_ERR_ARG, "batch %d outside [1, 4096]", B);
  TT_HIP_TRY(tt_allow_lds(reinterpret_cast<const void*>(&k_mlp_grad), sizeof(GradLds)));
  hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(GRAD_THREADS), sizeof(GradLds), static_cast<hipStream_t>(stream), params,
                     feats, targets, B, grad, loss);
  TT_HIP_TRY(hipGetLastError());
  return TT_OK;
}

tt_status tt_jpolicy_adam(float* params, float* m, float* v, const float* grad, int64_t count, int64_t step, float lr,
                          float beta1, float beta2, float eps, void* stream) {
  if (!params || !m || !v || !grad) return tt_fail(TT_ERR_ARG, "null argument");
  if (count < 1 || step < 1) return tt_fail(TT_ERR_ARG, "count and step must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !(lr >= 0.0f))
    return tt_fail(TT_ERR_ARG, "bad Adam hyper-parameters");
  const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     params, m, v, grad, count, lr, beta1, beta2, eps, c1, c2);
  TT_HIP_TRY(hipGetLastError());
  return TT_OK;
}

tt_status tt_sketch_size_bound(int64_t s, int32_t q, double eps, double delta, double* m) {
  if (!m) return tt_fail(TT_ERR_ARG, "null output");
  if (s < 1 || q < 1 || q > 60 || !(eps > 0.0) || !(delta > 0.0 && delta < 1.0))
    return tt_fail(TT_ERR_ARG, "need s >= 1, 1 <= q <= 60, eps > 0, 0 < delta < 1");
  const double c = 2.0 + pow(3.0, (double)q);
  const double a = 8.0 * (double)s * (double)s * c / delta;
  const double b = 8.0 * (double)s * c / (eps * delta);
  *m = a > b ? a : b;
  return TT_OK;
}

}  // extern "C"
