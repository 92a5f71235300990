// FP64 proximal solve (Sec. 3, eq. (3.5)).
//
// Solve: the split-K Gram partials of [SH^T SH | SH^T Y] are summed in FP64;
// M = SH^T SH + lambda I is factored M = L L^T (blocked right-looking
// Cholesky, packed lower triangle in LDS, one workgroup); a second kernel
// forms B = SH^T Y + lambda G_(2)^T for a block of columns and solves
// L L^T Z = B by blocked forward and back substitution in LDS, one workgroup
// per block of columns.
// lambda > 0 makes M positive definite (Sec. 3, remark after eq. (3.5)); a
// non-positive pivot records TT_ERR_NOT_SPD in the status word.
#include "tt_internal.h"

namespace {

// Column-major packed lower triangle: column c holds rows c..s-1.
__device__ __forceinline__ int coff(int c, int s) { return c * s - (c * (c - 1)) / 2; }
__device__ __forceinline__ int lidx(int i, int c, int s) { return coff(c, s) + (i - c); }   // i >= c

// Blocked right-looking Cholesky, blocks of 16 columns: the first wave
// factors the 16 x 16 diagonal block (LDS, wave-ordered), one thread per row
// solves the panel below it with the row's 16 values in registers, and all
// threads apply the trailing update in 4 x 4 register tiles: three barriers
// per block of 16 pivots.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename AT>
__device__ __forceinline__ void chol_blk_body(const AT* __restrict__ gpart, int32_t chunks, int32_t s, int32_t ldg, double lambda,
                              double* __restrict__ Lout, int32_t* __restrict__ status, double* L, int& bad) {
  const int tid = threadIdx.x, T = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, NW = T >> 6;
  const int np = s * (s + 1) / 2;
  __shared__ double rdiag[16];   // reciprocal pivots of the current diagonal block
  if (tid == 0) bad = 0;
  // row i of M is contiguous in c: a wave per row, lanes along it
  for (int i = wv; i < s; i += NW)
    for (int c = lane; c <= i; c += 64) {
      double acc = 0.0;
      for (int q = 0; q < chunks; ++q) acc += (double)gpart[((int64_t)q * s + i) * ldg + c];
      L[lidx(i, c, s)] = acc + (i == c ? lambda : 0.0);
    }
  __syncthreads();
  constexpr int B = 16;
  const int nb = (s + B - 1) / B;
  for (int ib = 0; ib < nb; ++ib) {
    const int j0 = ib * B, j1 = min(s, j0 + B);
    // (a) diagonal block, unblocked, by wave 0
    if (wv == 0) {
      int fail = 0;
      for (int j = j0; j < j1; ++j) {
        const double djj = L[lidx(j, j, s)];
        if (!(djj > 0.0) || !isfinite(djj)) {
          fail = 1;
          break;
        }
        const double dj = sqrt(djj), inv = 1.0 / dj;
        wave_sync();
        const int oj = coff(j, s) - j;
        if (lane == 0) {
          L[oj + j] = dj;
          rdiag[j - j0] = inv;
        }
        if (j + 1 + lane < j1) L[oj + j + 1 + lane] *= inv;
        wave_sync();
        // trailing part of the block, j < c <= i < j1: lane -> row
        // i = j + 1 + (lane & 15), columns c = j + 1 + (lane >> 4) + 4 k
        {
          const int i = j + 1 + (lane & 15);
          if (i < j1) {
            const double li = L[oj + i];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int c = j + 1 + (lane >> 4) + 4 * k;
              if (c <= i) L[lidx(i, c, s)] -= li * L[oj + c];
            }
          }
        }
        wave_sync();
      }
      if (lane == 0 && fail) bad = 1;
    }
    __syncthreads();
    if (bad) break;
    // (b) panel rows i >= j1: L[i][j0:j1] <- M[i][j0:j1] L_blk^-T
    for (int i = j1 + tid; i < s; i += T) {
      double x[B];
#pragma unroll
      for (int u = 0; u < B; ++u) x[u] = (j0 + u < j1) ? L[lidx(i, j0 + u, s)] : 0.0;
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (j0 + u < j1) {
          double t = x[u];
#pragma unroll
          for (int v = 0; v < u; ++v) t -= L[lidx(j0 + u, j0 + v, s)] * x[v];
          x[u] = t * rdiag[u];
        }
      }
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (j0 + u < j1) L[lidx(i, j0 + u, s)] = x[u];
    }
    __syncthreads();
    // (c) trailing update of the lower triangle beyond j1 in 4 x 4 tiles
    const int R = s - j1;
    if (R > 0) {
      const int nt = (R + 3) / 4;
      for (int t = tid; t < nt * nt; t += T) {
        const int ti = t / nt, tc = t % nt;
        if (ti < tc) continue;
        const int i0 = j1 + 4 * ti, c0 = j1 + 4 * tc;
        double acc[4][4] = {};
        for (int u = j0; u < j1; ++u) {
          const int ou = coff(u, s) - u;
          double li[4], lc[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            li[a] = (i0 + a < s) ? L[ou + i0 + a] : 0.0;
            lc[a] = (c0 + a < s) ? L[ou + c0 + a] : 0.0;
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += li[a] * lc[b];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int i = i0 + a, c = c0 + b;
            if (i < s && c < s && i >= c) L[lidx(i, c, s)] -= acc[a][b];
          }
      }
    }
    __syncthreads();
  }
  if (bad) {
    for (int e = tid; e < np; e += T) Lout[e] = __longlong_as_double(0x7ff8000000000000ll);
    if (tid == 0) atomicOr(status, 1);
    return;
  }
  for (int e = tid; e < np; e += T) Lout[e] = L[e];
}

template <typename AT>
__global__ __launch_bounds__(256) void k_chol_blk(const AT* __restrict__ gpart, int32_t chunks, int32_t s, int32_t ldg,
                                                 double lambda, double* __restrict__ Lout,
                                                 int32_t* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int bad;
  chol_blk_body<AT>(gpart, chunks, s, ldg, lambda, Lout, status, reinterpret_cast<double*>(smem_raw), bad);
}

// Blocked variant of the substitution: rows in blocks of 16.  Per block, one
// thread per right-hand-side column solves the 16 x 16 diagonal triangle with
// the column's 16 values in registers, then all threads update the rows the
// block feeds in 4 x 4 register tiles: two barriers per block instead of one
// per pivot.
constexpr int kTB = 16;

template <typename AT>
__device__ __forceinline__ void trsm_blk_body(const AT* __restrict__ gpart, int32_t chunks, int32_t s, int32_t ldg, double lambda,
                              const double* __restrict__ Lg, const double* G_old, double* G_new, int32_t rk, int32_t nk,
                              int32_t CB, int bx, double* L) {
  const int np = s * (s + 1) / 2;
  double* Bs = L + np;                 // s x CB, column block index fastest
  double* invd = Bs + (size_t)s * CB;  // s
  const int c0 = bx * CB;
  const int tid = threadIdx.x, T = blockDim.x;
  for (int e = tid; e < np; e += T) L[e] = Lg[e];
  for (int e = tid; e < s * CB; e += T) {
    const int j = e / CB, cl = e - j * CB;
    const int col = c0 + cl;
    double acc = 0.0;
    if (col < nk) {
      for (int q = 0; q < chunks; ++q) acc += (double)gpart[((int64_t)q * s + j) * ldg + s + col];
      const int a = j % rk, b = j / rk;
      acc += lambda * G_old[a + (int64_t)rk * (col + (int64_t)nk * b)];
    }
    Bs[e] = acc;
  }
  __syncthreads();   // every read of G_old for these columns precedes the writes below
  for (int j = tid; j < s; j += T) invd[j] = 1.0 / L[lidx(j, j, s)];
  __syncthreads();
  const int nb = (s + kTB - 1) / kTB;
  const int ctiles = (CB + 3) / 4;
  // forward: L y = B
  for (int ib = 0; ib < nb; ++ib) {
    const int j0 = ib * kTB, j1 = min(s, j0 + kTB);
    if (tid < CB) {
      double x[kTB];
#pragma unroll
      for (int u = 0; u < kTB; ++u) x[u] = (j0 + u < j1) ? Bs[(j0 + u) * CB + tid] : 0.0;
#pragma unroll
      for (int u = 0; u < kTB; ++u) {
        if (j0 + u < j1) {
          x[u] *= invd[j0 + u];
          const int oj = coff(j0 + u, s) - (j0 + u);
#pragma unroll
          for (int v = u + 1; v < kTB; ++v)
            if (j0 + v < j1) x[v] -= L[oj + j0 + v] * x[u];
        }
      }
#pragma unroll
      for (int u = 0; u < kTB; ++u)
        if (j0 + u < j1) Bs[(j0 + u) * CB + tid] = x[u];
    }
    __syncthreads();
    const int rows = s - j1;
    if (rows > 0) {
      const int rtiles = (rows + 3) / 4;
      for (int t = tid; t < rtiles * ctiles; t += T) {
        const int i0 = j1 + (t / ctiles) * 4, cc = (t % ctiles) * 4;
        double acc[4][4] = {};
        for (int j = j0; j < j1; ++j) {
          const int oj = coff(j, s) - j;
          double lv[4], yv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) lv[a] = (i0 + a < s) ? L[oj + i0 + a] : 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b) yv[b] = (cc + b < CB) ? Bs[j * CB + cc + b] : 0.0;
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += lv[a] * yv[b];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (i0 + a < s && cc + b < CB) Bs[(i0 + a) * CB + cc + b] -= acc[a][b];
      }
    }
    __syncthreads();
  }
  // backward: L^T z = y
  for (int ib = nb - 1; ib >= 0; --ib) {
    const int j0 = ib * kTB, j1 = min(s, j0 + kTB);
    if (tid < CB) {
      double x[kTB];
#pragma unroll
      for (int u = 0; u < kTB; ++u) x[u] = (j0 + u < j1) ? Bs[(j0 + u) * CB + tid] : 0.0;
#pragma unroll
      for (int u = kTB - 1; u >= 0; --u) {
        if (j0 + u < j1) {
          x[u] *= invd[j0 + u];
#pragma unroll
          for (int v = 0; v < u; ++v) x[v] -= L[lidx(j0 + u, j0 + v, s)] * x[u];
        }
      }
#pragma unroll
      for (int u = 0; u < kTB; ++u)
        if (j0 + u < j1) Bs[(j0 + u) * CB + tid] = x[u];
    }
    __syncthreads();
    const int rows = j0;
    if (rows > 0) {
      const int rtiles = (rows + 3) / 4;
      for (int t = tid; t < rtiles * ctiles; t += T) {
        const int i0 = (t / ctiles) * 4, cc = (t % ctiles) * 4;
        double acc[4][4] = {};
        for (int j = j0; j < j1; ++j) {
          double lv[4], zv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) lv[a] = (i0 + a < rows) ? L[lidx(j, i0 + a, s)] : 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b) zv[b] = (cc + b < CB) ? Bs[j * CB + cc + b] : 0.0;
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += lv[a] * zv[b];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (i0 + a < rows && cc + b < CB) Bs[(i0 + a) * CB + cc + b] -= acc[a][b];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < s * CB; e += T) {
    const int q = e / CB, cl = e - q * CB;
    const int col = c0 + cl;
    if (col < nk) {
      const int a = q % rk, b = q / rk;
      G_new[a + (int64_t)rk * (col + (int64_t)nk * b)] = Bs[e];
    }
  }
}

template <typename AT>
__global__ __launch_bounds__(256) void k_prox_trsm_blk(const AT* __restrict__ gpart, int32_t chunks, int32_t s,
                                                      int32_t ldg, double lambda, const double* __restrict__ Lg,
                                                      const double* G_old, double* G_new, int32_t rk, int32_t nk,
                                                      int32_t CB) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  trsm_blk_body<AT>(gpart, chunks, s, ldg, lambda, Lg, G_old, G_new, rk, nk, CB, blockIdx.x,
                    reinterpret_cast<double*>(smem_raw));
}

// Batched forms (problem blockIdx.y, or blockIdx.x for the one-workgroup
// factorisation): the same bodies with each problem's sizes and buffers.
__global__ void kb_gram_sum(const BUpd* __restrict__ d) {
  const BUpd u = d[blockIdx.y];
  const int64_t count = (int64_t)u.s * (u.s + u.nk);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double acc = 0.0;
  for (int q = 0; q < u.chunks; ++q) acc += (double)u.gpart[(int64_t)q * count + e];
  u.gsum[e] = acc;
}

__global__ __launch_bounds__(256) void kb_chol(const BUpd* __restrict__ d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int bad;
  const BUpd u = d[blockIdx.x];
  chol_blk_body<double>(u.gsum, 1, u.s, u.s + u.nk, u.lambda, u.Lg, u.status, reinterpret_cast<double*>(smem_raw), bad);
}

__global__ __launch_bounds__(256) void kb_trsm(const BUpd* __restrict__ d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BUpd u = d[blockIdx.y];
  if ((int)blockIdx.x * u.CB >= u.nk) return;
  trsm_blk_body<double>(u.gsum, 1, u.s, u.s + u.nk, u.lambda, u.Lg, u.G, u.G, u.rk, u.nk, u.CB, blockIdx.x,
                        reinterpret_cast<double*>(smem_raw));
}

// out[e] = sum over the split-K chunks of the Gram / right-hand-side partials
// (chunk q at q * count), in FP64 and in chunk order; one thread per entry.
template <typename AT>
__global__ void k_gram_sum(const AT* __restrict__ gpart, int32_t chunks, int64_t count, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double acc = 0.0;
  for (int q = 0; q < chunks; ++q) acc += (double)gpart[(int64_t)q * count + e];
  out[e] = acc;
}

__global__ void k_copy_f64(double* dst, const double* src, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename AT>
hipError_t prox_t(const tt_plan_s* p, int k, const double* G_old, double* G_new) {
  const int s = (int)(p->r[k] * p->r[k + 1]);
  const int nk = (int)p->n[k];
  const int ldg = s + nk;
  const int chunks = (int)tt_gram_chunks(p->J);
  double* Lg = p->at<double>(p->o_minv);
  int32_t* status = p->at<int32_t>(p->o_status);
  // the split-K partials summed once, every entry in parallel; the solve
  // kernels then read one FP64 copy
  double* gsum = p->at<double>(p->o_gsum);
  const int64_t count = (int64_t)s * ldg;
  hipLaunchKernelGGL(k_gram_sum<AT>, dim3(nblk(count, 256)), dim3(256), 0, p->stream, p->at<AT>(p->o_gram), chunks,
                     count, gsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t np = (size_t)s * (s + 1) / 2;
  const size_t lds1 = np * sizeof(double);
  if ((e = tt_allow_lds(k_chol_blk<double>, lds1)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_blk<double>, dim3(1), dim3(256), lds1, p->stream, gsum, 1, s, ldg, p->lambda, Lg,
                     status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // right-hand-side block: as wide as fits next to L in 150 KB of LDS, at
  // most 64 columns (one thread per column solves the diagonal blocks)
  int CB = 64;
  while (CB > 1 && (np + (size_t)s * CB + s) * sizeof(double) > 150 * 1024) CB >>= 1;
  const size_t lds2 = (np + (size_t)s * CB + s) * sizeof(double);
  if ((e = tt_allow_lds(k_prox_trsm_blk<double>, lds2)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prox_trsm_blk<double>, dim3(nblk(nk, CB)), dim3(256), lds2, p->stream, gsum, 1, s, ldg,
                     p->lambda, Lg, G_old, G_new, (int32_t)p->r[k], nk, CB);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_prox_from_gram(const tt_plan_s* p, int k, const double* G_old, double* G_new) {
  return p->wdt == TT_F64 ? prox_t<double>(p, k, G_old, G_new) : prox_t<float>(p, k, G_old, G_new);
}

hipError_t launch_copy_f64(const tt_plan_s* p, double* dst, const double* src, int64_t count) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f64, dim3(nblk(count, 256)), dim3(256), 0, p->stream, dst, src, count);
  return hipGetLastError();
}

hipError_t launch_solve_batched(const BUpd* d, int32_t nprob, int32_t max_s, int32_t max_count, int32_t max_cb_blocks,
                                size_t lds_chol, size_t lds_trsm, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  (void)max_s;
  hipLaunchKernelGGL(kb_gram_sum, dim3(nblk(max_count, 256), (unsigned)nprob), dim3(256), 0, st, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = tt_allow_lds(kb_chol, lds_chol)) != hipSuccess) return e;
  hipLaunchKernelGGL(kb_chol, dim3((unsigned)nprob), dim3(256), lds_chol, st, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = tt_allow_lds(kb_trsm, lds_trsm)) != hipSuccess) return e;
  hipLaunchKernelGGL(kb_trsm, dim3((unsigned)max_cb_blocks, (unsigned)nprob), dim3(256), lds_trsm, st, d);
  return hipGetLastError();
}
