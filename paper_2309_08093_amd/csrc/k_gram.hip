// Gram and right-hand-side contractions of the closed-form update (Sec. 3,
// (ite)): [SH^T SH | SH^T Y] = SH^T [SH | Y], an s x (s + n_k) product
// over the J sketch rows.  Split-K: each 16 x 16 output tile and each K chunk
// of 256 rows is one wave running 16x16 MFMAs; partial tiles go to a buffer
// that the FP64 solve sums in chunk order.
//   FP64 and FP32 work: v_mfma_f64_16x16x4f64 (FP32 operands widened: the
//                products are exact and the sums FP64, so the solve sees the
//                Gram of the stored FP32 values up to FP64 rounding; the
//                kernel is bound by latency, not by the MFMA rate)
//   BF16 mode:   operands rounded to BF16 (RNE), v_mfma_f32_16x16x16bf16_1k,
//                FP32 accumulation
// MFMA 16x16 layouts (64 lanes, l = lane): A[row = l%16][k = K0*(l/16)+..],
// B[k = K0*(l/16)+..][col = l%16]; result register r of lane l holds
// D[row = 4*(l/16) + r][col = l%16] for the FP32-accumulating forms and
// D[row = 4*r + l/16][col = l%16] for the FP64 form (checked on gfx950).
#include "tt_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = 256;

__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// One wave: output tile (blk * 4 + wave) of [SH^T SH | SH^T Y], K chunk `chunk`,
// on the FP64 MFMA.
template <typename T>
__device__ __forceinline__ void gram_body(const T* __restrict__ SH, const T* __restrict__ Y, double* __restrict__ gpart,
                                          int32_t J, int32_t s, int32_t nk, int32_t tiles_c, int32_t ntiles, int blk,
                                          int chunk, int klen) {
  const int lane = threadIdx.x & 63;
  const int tile = blk * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;
  const int tr = tile / tiles_c, tc = tile - tr * tiles_c;
  const int k0 = chunk * klen;
  const int k1 = min(J, k0 + klen);
  const int ncol = s + nk;
  const int arow = tr * 16 + (lane & 15);   // row of SH^T = column of SH
  const int bcol = tc * 16 + (lane & 15);
  const int kq = lane >> 4;
  const bool a_ok = arow < s, b_ok = bcol < ncol;
  const T* Acol = SH + (int64_t)J * (a_ok ? arow : 0);
  const T* Bcol = bcol < s ? SH + (int64_t)J * bcol : Y + (int64_t)J * (b_ok ? bcol - s : 0);
  doublex4 acc = {0, 0, 0, 0};
  for (int k = k0; k < k1; k += 4) {
    const int kk = k + kq;
    const double a = (a_ok && kk < k1) ? (double)Acol[kk] : 0.0;
    const double b = (b_ok && kk < k1) ? (double)Bcol[kk] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  for (int r = 0; r < 4; ++r) {
    const int row = tr * 16 + 4 * r + kq;   // FP64 16x16 result rows interleave by lane group
    if (row < s && b_ok) gpart[((int64_t)chunk * s + row) * ncol + bcol] = acc[r];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gram(const T* __restrict__ SH, const T* __restrict__ Y, double* __restrict__ gpart,
                                             int32_t J, int32_t s, int32_t nk, int32_t tiles_c, int32_t ntiles) {
  gram_body<T>(SH, Y, gpart, J, s, nk, tiles_c, ntiles, blockIdx.x, blockIdx.y, kChunk);
}

// Batched: problem blockIdx.y; blockIdx.x runs over (tile block, chunk).
__global__ __launch_bounds__(256) void kb_gram(const BUpd* __restrict__ d) {
  const BUpd u = d[blockIdx.y];
  const int tiles_r = (u.s + 15) / 16, tiles_c = (u.s + u.nk + 15) / 16;
  const int ntiles = tiles_r * tiles_c;
  const int tb = (ntiles + 3) / 4;
  const int chunk = blockIdx.x / tb;
  if (chunk >= u.chunks) return;
  gram_body<float>(u.SH, u.Y, u.gpart, u.J, u.s, u.nk, tiles_c, ntiles, blockIdx.x - chunk * tb, chunk, u.kchunk);
}

// BF16 operands, FP32 accumulation; K step 16 (4 per lane).
__global__ __launch_bounds__(256) void k_gram_bf16(const float* __restrict__ SH, const float* __restrict__ Y,
                                                  float* __restrict__ gpart, int32_t J, int32_t s, int32_t nk,
                                                  int32_t tiles_c, int32_t ntiles) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;
  const int tr = tile / tiles_c, tc = tile - tr * tiles_c;
  const int chunk = blockIdx.y;
  const int k0 = chunk * kChunk;
  const int k1 = min(J, k0 + kChunk);
  const int ncol = s + nk;
  const int arow = tr * 16 + (lane & 15);
  const int bcol = tc * 16 + (lane & 15);
  const int kq = lane >> 4;
  const bool a_ok = arow < s, b_ok = bcol < ncol;
  const float* Acol = SH + (int64_t)J * (a_ok ? arow : 0);
  const float* Bcol = bcol < s ? SH + (int64_t)J * bcol : Y + (int64_t)J * (b_ok ? bcol - s : 0);
  floatx4 acc = {0, 0, 0, 0};
  for (int k = k0; k < k1; k += 16) {
    shortx4 a, b;
    for (int e = 0; e < 4; ++e) {
      const int kk = k + 4 * kq + e;
      a[e] = to_bf16((a_ok && kk < k1) ? Acol[kk] : 0.f);
      b[e] = to_bf16((b_ok && kk < k1) ? Bcol[kk] : 0.f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  for (int r = 0; r < 4; ++r) {
    const int row = tr * 16 + 4 * kq + r;
    if (row < s && b_ok) gpart[((int64_t)chunk * s + row) * ncol + bcol] = acc[r];
  }
}

}  // namespace

int64_t tt_gram_chunks(int64_t J) { return (J + kChunk - 1) / kChunk; }
int32_t tt_gram_chunk_min() { return kChunk; }

hipError_t launch_gram(const tt_plan_s* p, int k, const void* SH, const void* Y) {
  const int s = (int)(p->r[k] * p->r[k + 1]);
  const int nk = (int)p->n[k];
  const int tiles_r = (s + 15) / 16, tiles_c = (s + nk + 15) / 16;
  const int ntiles = tiles_r * tiles_c;
  const dim3 grid((unsigned)((ntiles + 3) / 4), (unsigned)tt_gram_chunks(p->J));
  if (p->wdt == TT_F64) {
    hipLaunchKernelGGL(k_gram<double>, grid, dim3(256), 0, p->stream, static_cast<const double*>(SH),
                       static_cast<const double*>(Y), p->at<double>(p->o_gram), (int32_t)p->J, s, nk, tiles_c, ntiles);
  } else if (p->gram_mode == TT_GRAM_BF16) {
    hipLaunchKernelGGL(k_gram_bf16, grid, dim3(256), 0, p->stream, static_cast<const float*>(SH),
                       static_cast<const float*>(Y), p->at<float>(p->o_gram), (int32_t)p->J, s, nk, tiles_c, ntiles);
  } else {
    hipLaunchKernelGGL(k_gram<float>, grid, dim3(256), 0, p->stream, static_cast<const float*>(SH),
                       static_cast<const float*>(Y), p->at<double>(p->o_gram), (int32_t)p->J, s, nk, tiles_c, ntiles);
  }
  return hipGetLastError();
}

hipError_t launch_gram_batched(const BUpd* d, int32_t nprob, int32_t gx, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_gram, dim3((unsigned)gx, (unsigned)nprob), dim3(256), 0, st, d);
  return hipGetLastError();
}
